"""Seeded synthetic inputs for the batched branch-and-bound node-bound path.

This module only *draws data*: design matrices, responses, true coefficient
vectors and random node fixings.  It holds none of the method's arithmetic
(no losses, no relaxation, no proximal operator).  Both the GPU path (through
its tests and the benchmark) and the CPU oracle take their inputs from here.

Data model (paper, Appendix "Synthetic Data Generation Process"):
  * rows of X are i.i.d. centred Gaussian with Toeplitz covariance
    Sigma_jl = rho^|j-l|; each row is drawn as an AR(1) sequence
    x_0 = g_0, x_j = rho x_{j-1} + sqrt(1-rho^2) g_j, which has exactly that
    covariance;
  * the true coefficient vector has k nonzeros at evenly spaced indices;
  * squared loss: y = X beta* + eps with ||X beta*|| / ||eps|| = SNR (SNR 5);
  * logistic loss: y_i in {-1, +1}, P(y_i = 1) = 1 / (1 + exp(-x_i^T beta*)).

The instance is the matrix *after* rounding to its storage dtype: the float64
array returned in ``X`` holds the exact values of the stored float32 / bfloat16
entries, so every consumer sees the same numbers.

Readings where the paper leaves room (each listed in the design notes):
  * beta* positions: 0-based j_r = r * floor(p / k), r = 0..k-1;
  * beta* signs alternate +1, -1, +1, ... (or are random where stated);
  * the noise is scaled so that the norm ratio ||X beta*|| / ||eps|| equals SNR;
  * synthetic X is not column-normalised.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SQUARED = 0
LOGISTIC = 1

F64 = "f64"
F32 = "f32"
BF16 = "bf16"


@dataclass
class Instance:
    """One synthetic sparse-GLM instance.

    X        float64 (n, p): exact values of the stored entries (row-major)
    X_store  the stored array: float64, float32, or uint16 bfloat16 bit patterns
    dtype    "f64" | "f32" | "bf16"
    y        float64 (n,)
    """
    name: str
    X: np.ndarray
    X_store: np.ndarray
    dtype: str
    y: np.ndarray
    k: int
    loss: int
    lambda2: float
    M: float
    beta_true: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.X.shape[0]

    @property
    def p(self) -> int:
        return self.X.shape[1]


def bf16_bits_from_f32(a32: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest, ties to even).

    Returns the 16-bit patterns as uint16.  Pure bit manipulation of the
    storage format; NaN never occurs in these generators.
    """
    u = np.ascontiguousarray(a32, dtype=np.float32).view(np.uint32)
    lsb = (u >> np.uint32(16)) & np.uint32(1)
    rounded = u + np.uint32(0x7FFF) + lsb
    return (rounded >> np.uint32(16)).astype(np.uint16)


def f64_from_bf16_bits(b: np.ndarray) -> np.ndarray:
    """Exact float64 values of bfloat16 bit patterns."""
    u = b.astype(np.uint32) << np.uint32(16)
    return u.view(np.float32).astype(np.float64)


def ar1_design(n: int, p: int, rho: float, rng: np.random.Generator,
               chunk_rows: int = 8192) -> np.ndarray:
    """Gaussian rows with Toeplitz covariance rho^|j-l| (AR(1) recursion).

    Rows are drawn in blocks of chunk_rows standard normals (row-major order);
    within a block the recursion x_j = rho x_{j-1} + sqrt(1 - rho^2) g_j runs
    over the columns of the block's transpose, so each step reads and writes
    contiguous memory (the values do not depend on the layout)."""
    X = np.empty((n, p), dtype=np.float64)
    c = math.sqrt(1.0 - rho * rho)
    for r0 in range(0, n, chunk_rows):
        r1 = min(n, r0 + chunk_rows)
        gt = np.ascontiguousarray(rng.standard_normal((r1 - r0, p)).T)
        bt = np.empty_like(gt)
        bt[0] = gt[0]
        for j in range(1, p):
            np.multiply(bt[j - 1], rho, out=bt[j])
            bt[j] += c * gt[j]
        X[r0:r1] = bt.T
    return X


def _store(X64: np.ndarray, dtype: str):
    if dtype == F64:
        return X64.copy(), X64.copy()
    if dtype == F32:
        x32 = X64.astype(np.float32)
        return x32.astype(np.float64), x32
    if dtype == BF16:
        bits = bf16_bits_from_f32(X64.astype(np.float32))
        return f64_from_bf16_bits(bits), bits
    raise ValueError(dtype)


def evenly_spaced_support(p: int, k: int) -> np.ndarray:
    step = p // k
    return np.arange(k, dtype=np.int64) * step


def alternating_signs(k: int) -> np.ndarray:
    return np.where(np.arange(k) % 2 == 0, 1.0, -1.0)


def make_instance(name: str, n: int, p: int, rho: float, k: int, loss: int,
                  lambda2: float, M: float, dtype: str = F64, seed: int = 0,
                  snr: float = 5.0, beta_values: np.ndarray | None = None,
                  support: np.ndarray | None = None) -> Instance:
    """Draw one instance.  RNG order: X normals, then noise / label uniforms."""
    rng = np.random.Generator(np.random.PCG64(seed))
    X64 = ar1_design(n, p, rho, rng)
    X, X_store = _store(X64, dtype)
    supp = evenly_spaced_support(p, k) if support is None else np.asarray(support)
    vals = alternating_signs(len(supp)) if beta_values is None else np.asarray(beta_values, float)
    beta = np.zeros(p)
    beta[supp] = vals
    lin = X @ beta
    if loss == SQUARED:
        e = rng.standard_normal(n)
        e *= np.linalg.norm(lin) / (snr * np.linalg.norm(e))
        y = lin + e
    elif loss == LOGISTIC:
        u = rng.random(n)
        prob = 1.0 / (1.0 + np.exp(-lin))
        y = np.where(u < prob, 1.0, -1.0)
    else:
        raise ValueError(loss)
    return Instance(name=name, X=X, X_store=X_store, dtype=dtype, y=y, k=k,
                    loss=loss, lambda2=lambda2, M=M, beta_true=beta,
                    meta=dict(rho=rho, seed=seed, snr=snr))


# ---------------------------------------------------------------------------
# The named workloads.
# ---------------------------------------------------------------------------

def plain_bnb_squared_500x30(seed: int = 0) -> Instance:
    """500 x 30 float64, rho 0.5, k 5, squared loss, SNR 5, lambda2 1e-3, M 2."""
    return make_instance("squared_500x30", 500, 30, 0.5, 5, SQUARED, 1e-3, 2.0,
                         F64, seed)


def node_bounds_logistic_5000x200(seed: int = 0) -> Instance:
    """5000 x 200 float32, rho 0.5, k 10, logistic, lambda2 1, M 2."""
    return make_instance("logistic_5000x200", 5000, 200, 0.5, 10, LOGISTIC, 1.0,
                         2.0, F32, seed)


def bnb_squared_10000x1000_bf16(seed: int = 0) -> Instance:
    """10000 x 1000 bfloat16, rho 0.9, k 10, squared, SNR 5, lambda2 1e-3, M 2."""
    return make_instance("squared_10000x1000_bf16", 10000, 1000, 0.9, 10, SQUARED,
                         1e-3, 2.0, BF16, seed)


def large_logistic_100000x5000_bf16(seed: int = 0) -> Instance:
    """100000 x 5000 bfloat16, rho 0.7, k 15, logistic, lambda2 1, M 4.

    |beta*_j| ~ U[0.5, 2] with random signs at indices r * 333.
    """
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    k = 15
    mags = rng.uniform(0.5, 2.0, k)
    signs = np.where(rng.random(k) < 0.5, -1.0, 1.0)
    supp = np.arange(k) * 333
    return make_instance("logistic_100000x5000_bf16", 100000, 5000, 0.7, k, LOGISTIC,
                         1.0, 4.0, BF16, seed, beta_values=mags * signs, support=supp)


def small_instance(n: int, p: int, k: int, loss: int, seed: int = 0, rho: float = 0.5,
                   lambda2: float | None = None, M: float = 2.0,
                   dtype: str = F64) -> Instance:
    """Reduced-size instance with the same recipe (tests)."""
    if lambda2 is None:
        lambda2 = 1e-3 if loss == SQUARED else 1.0
    return make_instance(f"small_{n}x{p}", n, p, rho, k, loss, lambda2, M, dtype, seed)


def serving_mix_problems(count: int = 32, seed: int = 0, scale: float = 1.0):
    """Problem parameters for the multi-problem serving mix.

    n ~ U{1000..20000}, p ~ U{100..3000}, k ~ U{5..20}, loss 50/50,
    rho in {0.3, 0.6, 0.9}; float32 X.  ``scale`` shrinks n and p for tests.
    Returns a list of dicts (instances are drawn lazily with ``make_instance``).
    """
    rng = np.random.Generator(np.random.PCG64(seed + 424242))
    out = []
    for i in range(count):
        n = int(rng.integers(1000, 20001) * scale)
        p = int(rng.integers(100, 3001) * scale)
        k = int(rng.integers(5, 21))
        k = max(1, min(k, p // 4))
        loss = int(rng.integers(0, 2))
        rho = float(rng.choice([0.3, 0.6, 0.9]))
        out.append(dict(name=f"mix{i}", n=max(n, 8), p=max(p, 4), rho=rho, k=k, loss=loss,
                        lambda2=1e-3 if loss == SQUARED else 1.0, M=2.0, dtype=F32,
                        seed=seed + 1000 + i))
    return out


# ---------------------------------------------------------------------------
# Random branch-and-bound nodes.
# ---------------------------------------------------------------------------

@dataclass
class Node:
    """Fixed-in (J1) and fixed-out (J0) index sets, sorted int32 arrays."""
    fixed_in: np.ndarray
    fixed_out: np.ndarray


def random_nodes(p: int, count: int, max_in: int, max_out: int, seed: int) -> list[Node]:
    """|J1| ~ U{0..max_in}, |J0| ~ U{0..max_out}, disjoint uniform subsets of [p]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nodes = []
    for _ in range(count):
        n1 = int(rng.integers(0, max_in + 1))
        n0 = int(rng.integers(0, max_out + 1))
        n0 = min(n0, p - n1)
        perm = rng.permutation(p)
        nodes.append(Node(np.sort(perm[:n1]).astype(np.int32),
                          np.sort(perm[n1:n1 + n0]).astype(np.int32)))
    return nodes


def launch_nodes_5000x200(launch: int, count: int = 256) -> list[Node]:
    """Node batch `launch` of the 5000x200 logistic workload (seed 1000+launch)."""
    return random_nodes(200, count, 5, 60, 1000 + launch)


def node_state(p: int, node: Node) -> np.ndarray:
    """int8 coordinate states: 0 free, 1 fixed in, -1 fixed out."""
    st = np.zeros(p, dtype=np.int8)
    st[node.fixed_in] = 1
    st[node.fixed_out] = -1
    return st
