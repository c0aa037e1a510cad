"""The oracle: a plain, sequential float64 CPU reference (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The GPU library never calls it,
and it shares no code with the GPU library: it is ``kbnb_oracle.c`` (plain C,
gcc, no BLAS) behind ctypes.

Parity status of each routine (what pins it; see tests/test_oracle_pins.py):
  loss, dloss, loss_conj   Fenchel-Young equalities; finite differences
  huber, prox_huber        closed forms; scalar minimisation
  g                        direct minimisation over z (scipy) on small cases;
                           Fenchel-Young equality with g*
  gstar                    brute force over subsets of size kbar
  prox                     generic convex solve of the prox problem
  primal, dual             weak duality; ridge closed form when k = p
  node_bound               duality bracket; ridge closed form; brute force
  support_value            box-constrained least squares (scipy bvls)
  bnb                      brute force over all k-subsets; orthogonal design
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kbnb_oracle.c")
_LIB = os.path.join(_HERE, "libkbnb_oracle.so")

SQUARED = 0
LOGISTIC = 1
CONVERGED, PRUNED, MAXITER, INVALID = 0, 1, 2, -1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, IEEE semantics kept)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
               "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


class _Problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("p", ctypes.c_int), ("k", ctypes.c_int),
                ("loss", ctypes.c_int), ("lambda2", ctypes.c_double),
                ("M", ctypes.c_double), ("X", ctypes.c_void_p), ("y", ctypes.c_void_p)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        d, i, vp = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
        P = ctypes.POINTER(_Problem)
        sig = {
            "orc_loss": (d, [i, d, d]),
            "orc_dloss": (d, [i, d, d]),
            "orc_loss_conj": (d, [i, d, d]),
            "orc_huber": (d, [d, d]),
            "orc_prox_huber": (d, [d, d, d]),
            "orc_kbar": (i, [P, vp]),
            "orc_g": (d, [P, vp, vp]),
            "orc_gstar": (d, [P, vp, vp]),
            "orc_prox": (None, [P, vp, d, vp, vp]),
            "orc_primal": (d, [P, vp, vp]),
            "orc_dual": (d, [P, vp, vp]),
            "orc_dual_point": (None, [P, vp, vp]),
            "orc_lipschitz": (d, [P]),
            "orc_node_bound": (i, [P, vp, d, vp, d, i, d, d, vp, vp]),
            "orc_round_branch": (None, [P, vp, vp, vp, vp, vp]),
            "orc_support_value": (d, [P, vp, i, d, d, i, vp]),
            "orc_bnb": (i, [P, d, i, d, d, ctypes.c_long, vp, vp, vp]),
            "orc_rashomon": (ctypes.c_long, [P, d, ctypes.c_long, d, i, ctypes.c_long,
                                             ctypes.c_long, vp, vp, vp]),
            "orc_reliance": (None, [P, vp, vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Problem:
    """Holds float64 copies of X (row-major) and y for the C routines."""

    def __init__(self, X, y, k, loss, lambda2, M):
        self.X = np.ascontiguousarray(X, dtype=np.float64)
        self.y = np.ascontiguousarray(y, dtype=np.float64)
        self.n, self.p = self.X.shape
        self.k, self.loss = int(k), int(loss)
        self.lambda2, self.M = float(lambda2), float(M)
        self._c = _Problem(self.n, self.p, self.k, self.loss, self.lambda2, self.M,
                           self.X.ctypes.data, self.y.ctypes.data)
        self._L = None

    @classmethod
    def from_instance(cls, inst):
        return cls(inst.X, inst.y, inst.k, inst.loss, inst.lambda2, inst.M)

    @property
    def ref(self):
        return ctypes.byref(self._c)

    def _state(self, state):
        st = np.ascontiguousarray(state, dtype=np.int8)
        assert st.shape == (self.p,)
        return st

    # -- node functions -----------------------------------------------------
    def kbar(self, state):
        st = self._state(state)
        return _load().orc_kbar(self.ref, _ptr(st))

    def g(self, state, beta):
        st = self._state(state)
        b = np.ascontiguousarray(beta, dtype=np.float64)
        return _load().orc_g(self.ref, _ptr(st), _ptr(b))

    def gstar(self, state, q):
        st = self._state(state)
        qq = np.ascontiguousarray(q, dtype=np.float64)
        return _load().orc_gstar(self.ref, _ptr(st), _ptr(qq))

    def prox(self, state, eta, u):
        st = self._state(state)
        uu = np.ascontiguousarray(u, dtype=np.float64)
        out = np.empty(self.p)
        _load().orc_prox(self.ref, _ptr(st), float(eta), _ptr(uu), _ptr(out))
        return out

    def primal(self, state, beta):
        st = self._state(state)
        b = np.ascontiguousarray(beta, dtype=np.float64)
        return _load().orc_primal(self.ref, _ptr(st), _ptr(b))

    def dual(self, state, zeta):
        st = self._state(state)
        z = np.ascontiguousarray(zeta, dtype=np.float64)
        return _load().orc_dual(self.ref, _ptr(st), _ptr(z))

    def dual_point(self, beta):
        b = np.ascontiguousarray(beta, dtype=np.float64)
        out = np.empty(self.n)
        _load().orc_dual_point(self.ref, _ptr(b), _ptr(out))
        return out

    def lipschitz(self):
        if self._L is None:
            self._L = _load().orc_lipschitz(self.ref)
        return self._L

    def node_bound(self, state, warm=None, tol=1e-6, max_iter=20000, ub=np.inf,
                   prune_rel=1e-6, L=None):
        """Returns dict(lb, phi, gap, iterations, status, beta)."""
        st = self._state(state)
        L = self.lipschitz() if L is None else L
        beta = np.empty(self.p)
        info = np.empty(5)
        w = None if warm is None else np.ascontiguousarray(warm, dtype=np.float64)
        _load().orc_node_bound(self.ref, _ptr(st), float(L),
                               None if w is None else _ptr(w), float(tol), int(max_iter),
                               float(ub), float(prune_rel), _ptr(beta), _ptr(info))
        return dict(lb=info[0], phi=info[1], gap=info[2], iterations=int(info[3]),
                    status=int(info[4]), beta=beta)

    def round_branch(self, state, beta):
        st = self._state(state)
        b = np.ascontiguousarray(beta, dtype=np.float64)
        supp = np.full(self.p + 1, -1, dtype=np.int32)
        ln = ctypes.c_int(0)
        br = ctypes.c_int(-1)
        _load().orc_round_branch(self.ref, _ptr(st), _ptr(b), _ptr(supp),
                                 ctypes.byref(ln), ctypes.byref(br))
        return supp[:ln.value].copy(), br.value

    def support_value(self, support, tol=1e-13, max_iter=50000):
        s = np.ascontiguousarray(support, dtype=np.int32)
        beta = np.empty(self.p)
        v = _load().orc_support_value(self.ref, _ptr(s), len(s), float(self.lipschitz()),
                                      float(tol), int(max_iter), _ptr(beta))
        return v, beta

    def bnb(self, node_tol=1e-6, node_max_iter=20000, gap_tol=1e-6, prune_rel=1e-6,
            max_nodes=1_000_000):
        supp = np.full(self.k, -1, dtype=np.int32)
        beta = np.empty(self.p)
        info = np.empty(6)
        _load().orc_bnb(self.ref, float(node_tol), int(node_max_iter), float(gap_tol),
                        float(prune_rel), int(max_nodes), _ptr(supp), _ptr(beta), _ptr(info))
        return dict(objective=info[0], lower_bound=info[1], rel_gap=info[2],
                    nodes=int(info[3]), status=int(info[4]), updates=int(info[5]),
                    support=supp[supp >= 0].copy(), beta=beta)


    def rashomon(self, eps, cap=0, node_tol=1e-9, node_max_iter=100000, max_nodes=1_000_000,
                 max_out=100000):
        """Support-level Rashomon set: list of (support tuple, value) by value."""
        supp = np.full((max_out, self.k), -1, dtype=np.int32)
        vals = np.empty(max_out)
        info = np.empty(4)
        cnt = _load().orc_rashomon(self.ref, float(eps), int(cap), float(node_tol),
                                   int(node_max_iter), int(max_nodes), int(max_out),
                                   _ptr(supp), _ptr(vals), _ptr(info))
        out = [(tuple(int(j) for j in supp[r] if j >= 0), float(vals[r]))
               for r in range(min(cnt, max_out))]
        return dict(set=out, count=int(cnt), optimum=info[0], threshold=info[1],
                    nodes=int(info[2]), status=int(info[3]))


    def reliance(self, beta):
        """Fixed-model reliance R[j] of model beta (p entries; 0 where beta_j = 0)."""
        b = np.ascontiguousarray(beta, dtype=np.float64)
        assert b.shape == (self.p,)
        out = np.empty(self.p)
        _load().orc_reliance(self.ref, _ptr(b), _ptr(out))
        return out


# scalar helpers ------------------------------------------------------------

def loss(kind, s, y):
    return _load().orc_loss(int(kind), float(s), float(y))


def dloss(kind, s, y):
    return _load().orc_dloss(int(kind), float(s), float(y))


def loss_conj(kind, v, y):
    return _load().orc_loss_conj(int(kind), float(v), float(y))


def huber(q, M):
    return _load().orc_huber(float(q), float(M))


def prox_huber(x, c, M):
    return _load().orc_prox_huber(float(x), float(c), float(M))
