"""Pins for the oracle: each test checks it against something other than itself.

The references used here are independent of the oracle's C code: scipy solvers
(scalar minimisation, SLSQP, L-BFGS-B, bounded least squares), brute-force
enumeration, closed forms (ridge, orthogonal design), duality identities and
the worked example of the paper's Fig. 2.  Each test is chosen so that a
plausible slip in the oracle (a dropped term, a wrong sign, index or scaling)
fails it.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
from scipy import optimize

import oracle
import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=not os.path.exists(oracle._LIB))


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------------------
# Scalar losses: Fenchel-Young equality, derivative, conjugate as a supremum.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kind", [oracle.SQUARED, oracle.LOGISTIC])
def test_loss_derivative_and_fenchel_young(kind):
    r = rng(1)
    for _ in range(200):
        s = r.normal() * 3
        y = r.choice([-1.0, 1.0]) if kind == oracle.LOGISTIC else r.normal()
        h = 1e-5
        fd = (oracle.loss(kind, s + h, y) - oracle.loss(kind, s - h, y)) / (2 * h)
        d = oracle.dloss(kind, s, y)
        assert abs(fd - d) < 1e-7 * max(1.0, abs(d))
        # l(s) + l*(l'(s)) = s l'(s)
        lhs = oracle.loss(kind, s, y) + oracle.loss_conj(kind, d, y)
        assert abs(lhs - s * d) < 1e-12 * max(1.0, abs(s * d), oracle.loss(kind, s, y))


@pytest.mark.parametrize("kind", [oracle.SQUARED, oracle.LOGISTIC])
def test_loss_conjugate_is_supremum(kind):
    r = rng(2)
    for _ in range(60):
        y = r.choice([-1.0, 1.0]) if kind == oracle.LOGISTIC else r.normal()
        if kind == oracle.LOGISTIC:
            t = r.uniform(0.02, 0.98)
            v = -t * y
        else:
            v = r.normal() * 2
        res = optimize.minimize_scalar(lambda s: -(v * s - oracle.loss(kind, s, y)),
                                       bounds=(-60, 60), method="bounded",
                                       options={"xatol": 1e-11})
        assert abs(-res.fun - oracle.loss_conj(kind, v, y)) < 1e-8


def test_logistic_conjugate_domain():
    assert math.isinf(oracle.loss_conj(oracle.LOGISTIC, 0.5, 1.0))   # t = -0.5
    assert math.isinf(oracle.loss_conj(oracle.LOGISTIC, -1.5, 1.0))  # t = 1.5
    assert oracle.loss_conj(oracle.LOGISTIC, 0.0, 1.0) == 0.0
    assert oracle.loss_conj(oracle.LOGISTIC, -1.0, 1.0) == 0.0


def test_huber_and_prox():
    M = 1.7
    for q in [0.0, 0.3, -1.2, 1.7, -1.7, 2.5, -9.0]:
        exp = 0.5 * q * q if abs(q) <= M else M * abs(q) - 0.5 * M * M
        assert oracle.huber(q, M) == pytest.approx(exp, rel=1e-15, abs=0)
    r = rng(3)
    for _ in range(100):
        x, c = r.normal() * 5, r.uniform(0, 4)
        res = optimize.minimize_scalar(lambda v: 0.5 * (v - x) ** 2 + c * oracle.huber(v, M),
                                       bounds=(-abs(x) - 1, abs(x) + 1), method="bounded",
                                       options={"xatol": 1e-12})
        assert abs(res.x - oracle.prox_huber(x, c, M)) < 1e-7


# ---------------------------------------------------------------------------
# Node functions g_N and g*_N.
# ---------------------------------------------------------------------------

def tiny_problem(n=12, p=8, k=3, loss=oracle.SQUARED, seed=0, M=2.0, lambda2=0.7):
    r = rng(seed)
    X = r.normal(size=(n, p))
    y = r.choice([-1.0, 1.0], size=n) if loss == oracle.LOGISTIC else r.normal(size=n)
    return oracle.Problem(X, y, k, loss, lambda2, M)


def random_state(r, p, k):
    st = np.zeros(p, np.int8)
    perm = r.permutation(p)
    n1 = int(r.integers(0, k + 1))
    n0 = int(r.integers(0, p - n1 + 1))
    st[perm[:n1]] = 1
    st[perm[n1:n1 + n0]] = -1
    return st


def g_by_direct_z_minimisation(beta, st, k, M):
    """min_z 1/2 sum beta_j^2 / z_j over the node's z-polytope, by SLSQP."""
    J1 = np.where(st == 1)[0]
    Jf = np.where(st == 0)[0]
    kbar = k - len(J1)
    val = 0.5 * float(np.sum(beta[J1] ** 2))
    bf = beta[Jf]
    nz = np.abs(bf) > 0
    a = np.abs(bf[nz])
    if len(a) == 0:
        return val
    lo = a / M
    x0 = np.clip(np.full(len(a), min(1.0, kbar / len(a))), lo, 1.0)
    res = optimize.minimize(lambda z: 0.5 * np.sum(a * a / z), x0,
                            jac=lambda z: -0.5 * a * a / (z * z),
                            bounds=list(zip(lo, np.ones(len(a)))),
                            constraints=[{"type": "ineq", "fun": lambda z: kbar - z.sum(),
                                          "jac": lambda z: -np.ones(len(z))}],
                            method="SLSQP", options={"ftol": 1e-15, "maxiter": 1000})
    return val + res.fun


def g_by_sorted_threshold(beta, st, k):
    """Thm. 4.1's sorted form: find s with |b_(s)| >= tau >= |b_(s+1)|."""
    J1 = np.where(st == 1)[0]
    Jf = np.where(st == 0)[0]
    kbar = k - len(J1)
    val = 0.5 * float(np.sum(beta[J1] ** 2))
    a = np.sort(np.abs(beta[Jf]))[::-1]
    if np.count_nonzero(a) <= kbar:
        return val + 0.5 * float(np.sum(a * a))
    for s in range(kbar):
        tail = float(np.sum(a[s:]))
        tau = tail / (kbar - s)
        upper = math.inf if s == 0 else a[s - 1]
        if upper >= tau * (1 - 1e-12) and tau >= a[s] * (1 - 1e-12):
            return val + 0.5 * float(np.sum(a[:s] ** 2)) + 0.5 * tail * tau
    raise AssertionError("no threshold")


def feasible_beta(r, st, k, M):
    """A random point of dom g_N (scaled so that the free budget holds)."""
    p = len(st)
    b = r.normal(size=p) * r.uniform(0.1, 1.5)
    b[st == -1] = 0
    b = np.clip(b, -M, M)
    kbar = k - int(np.sum(st == 1))
    f = st == 0
    if kbar <= 0:
        b[f] = 0
    else:
        tot = np.sum(np.abs(b[f]))
        if tot > M * kbar:
            b[f] *= 0.999 * M * kbar / tot
    # sprinkle exact zeros
    b[f & (r.random(p) < 0.2)] = 0.0
    return b


def test_g_matches_direct_minimisation_and_sorted_form():
    r = rng(4)
    for trial in range(150):
        P = tiny_problem(p=9, k=4, seed=trial)
        st = random_state(r, 9, 4)
        b = feasible_beta(r, st, 4, P.M)
        g_or = P.g(st, b)
        g_thm = g_by_sorted_threshold(b, st, 4)
        assert g_or == pytest.approx(g_thm, rel=1e-12, abs=1e-14)
        g_dir = g_by_direct_z_minimisation(b, st, 4, P.M)
        assert g_or == pytest.approx(g_dir, rel=2e-6, abs=1e-9)


def test_g_domain_and_special_cases():
    P = tiny_problem(p=6, k=2)
    st = np.array([0, 0, 0, 1, -1, 0], np.int8)
    b = np.array([0.5, 0.0, 0.0, 1.0, 0.0, 0.0])
    assert P.g(st, b) == pytest.approx(0.5 * (0.25 + 1.0))       # nonbinding
    b2 = b.copy(); b2[4] = 1e-3
    assert math.isinf(P.g(st, b2))                                # beta on J0
    b3 = b.copy(); b3[0] = P.M * 1.01
    assert math.isinf(P.g(st, b3))                                # box
    st2 = np.array([1, 1, 0, 0, 0, 0], np.int8)                   # kbar = 0
    b4 = np.array([0.3, 0.2, 0.1, 0, 0, 0])
    assert math.isinf(P.g(st2, b4))
    b4[2] = 0
    assert P.g(st2, b4) == pytest.approx(0.5 * (0.09 + 0.04))
    # binding with budget exceeded: sum |free| > M kbar
    st3 = np.zeros(6, np.int8)
    b5 = np.array([1.9, 1.9, 0.5, 0, 0, 0])
    assert math.isinf(P.g(st3, b5))


def test_gstar_brute_force_subsets():
    r = rng(5)
    for trial in range(100):
        P = tiny_problem(p=8, k=3, seed=trial, M=1.3)
        st = random_state(r, 8, 3)
        q = r.normal(size=8) * 2
        H = np.where(np.abs(q) <= P.M, 0.5 * q * q, P.M * np.abs(q) - 0.5 * P.M ** 2)
        J1 = np.where(st == 1)[0]
        Jf = np.where(st == 0)[0]
        kbar = 3 - len(J1)
        best = max((sum(H[list(c)]) for c in itertools.combinations(Jf, min(kbar, len(Jf)))),
                   default=0.0)
        assert P.gstar(st, q) == pytest.approx(H[J1].sum() + best, rel=1e-13, abs=1e-14)


def test_g_gstar_fenchel_young():
    """g(b) + g*(q) >= q.b always, with equality at the q built from Thm. 4.1's z."""
    r = rng(6)
    for trial in range(200):
        P = tiny_problem(p=10, k=4, seed=trial, M=1.5)
        st = random_state(r, 10, 4)
        b = feasible_beta(r, st, 4, P.M)
        g = P.g(st, b)
        for _ in range(5):
            q = r.normal(size=10) * 2
            assert g + P.gstar(st, q) >= q @ b - 1e-12
        # equality point
        J1 = st == 1
        Jf = st == 0
        kbar = 4 - int(J1.sum())
        q = np.zeros(10)
        q[J1] = b[J1]
        a = np.abs(b[Jf])
        if np.count_nonzero(a) <= kbar:
            q[Jf] = b[Jf]
        else:
            srt = np.sort(a)[::-1]
            tau = None
            for s in range(kbar):
                tail = srt[s:].sum()
                t = tail / (kbar - s)
                if (s == 0 or srt[s - 1] >= t * (1 - 1e-12)) and t >= srt[s] * (1 - 1e-12):
                    tau = t
                    break
            bf = b[Jf]
            q[Jf] = np.where(np.abs(bf) >= tau, bf, tau * np.sign(bf))
        assert g + P.gstar(st, q) == pytest.approx(q @ b, rel=1e-11, abs=1e-12)


# ---------------------------------------------------------------------------
# The prox, against a generic convex solve of its definition.
# ---------------------------------------------------------------------------

def prox_by_generic_solve(u, st, k, rho, M):
    """beta = u - alpha/rho with alpha = argmin 1/2||a - rho u||^2 + rho g*(a).

    TopSum_kbar(h) = min_t kbar t + sum_j (h_j - t)_+ (kbar < #free), so the
    free part is the minimum over t of separable 1-D convex problems.  Each
    1-D problem is solved by bisection on the sign of its subgradient (exact to
    rounding); the convex outer function of t is minimised by golden section.
    J1 entries take the 1-D problem with weight rho and no threshold, J0
    entries are unpenalised.
    """
    w = rho * np.abs(u)

    def H(a):
        a = np.abs(a)
        return np.where(a <= M, 0.5 * a * a, M * a - 0.5 * M * M)

    def dH(a):
        return np.minimum(np.abs(a), M)

    def inner(wv, t):
        """argmin over a in [0, w] of 1/2 (a - w)^2 + rho (H(a) - t)_+ (t=-inf: rho H(a))."""
        lo = np.zeros_like(wv)
        hi = wv.copy()
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            Hm = H(mid)
            left = (mid - wv) + np.where(Hm > t, rho * dH(mid), 0.0)
            right = (mid - wv) + np.where(Hm >= t, rho * dH(mid), 0.0)
            go_up = right < 0
            go_down = left > 0
            lo = np.where(go_up, mid, lo)
            hi = np.where(go_down, mid, hi)
            stay = ~(go_up | go_down)
            lo = np.where(stay, mid, lo)
            hi = np.where(stay, mid, hi)
        return 0.5 * (lo + hi)

    def cost(a, wv, t):
        return 0.5 * (a - wv) ** 2 + rho * np.maximum(H(a) - t, 0.0)

    p = len(u)
    alpha = np.zeros(p)
    kbar = k - int(np.sum(st == 1))
    J0 = st == -1
    J1 = st == 1
    alpha[J0] = w[J0]
    if J1.any():
        alpha[J1] = inner(w[J1], -np.inf)
    free = st == 0
    if free.any():
        wf = w[free]
        if kbar <= 0:
            alpha[free] = wf
        elif kbar >= wf.size:
            alpha[free] = inner(wf, -np.inf)
        else:
            def outer(t):
                a = inner(wf, t)
                return kbar * rho * t + float(np.sum(cost(a, wf, t)))
            a, b = 0.0, float(np.max(H(wf)))
            g = (math.sqrt(5) - 1) / 2
            c, d = b - g * (b - a), a + g * (b - a)
            fc, fd = outer(c), outer(d)
            for _ in range(160):
                if fc <= fd:
                    b, d, fd = d, c, fc
                    c = b - g * (b - a)
                    fc = outer(c)
                else:
                    a, c, fc = c, d, fd
                    d = a + g * (b - a)
                    fd = outer(d)
            alpha[free] = inner(wf, 0.5 * (a + b))
    return np.sign(u) * (np.abs(u) - alpha / rho)


def test_prox_matches_generic_convex_solve():
    r = rng(7)
    for trial in range(40):
        p, k = 7, 3
        P = tiny_problem(p=p, k=k, seed=trial, M=1.2, lambda2=r.uniform(0.2, 2.0))
        st = random_state(r, p, k)
        u = r.normal(size=p) * r.uniform(0.3, 3.0)
        eta = r.uniform(0.05, 1.0)
        rho = 1.0 / (2 * eta * P.lambda2)
        got = P.prox(st, eta, u)
        ref = prox_by_generic_solve(u, st, k, rho, P.M)
        assert np.max(np.abs(got - ref)) < 1e-7, (trial, got, ref)


def test_prox_is_minimiser_of_primal_prox_problem():
    """prox_{eta G}(u) minimises 1/2||b - u||^2 + 2 eta lambda2 g(b): no random
    feasible perturbation improves it."""
    r = rng(8)
    for trial in range(60):
        p, k = 10, 4
        P = tiny_problem(p=p, k=k, seed=trial, M=1.0, lambda2=0.5)
        st = random_state(r, p, k)
        u = r.normal(size=p) * 1.5
        eta = 0.3
        b = P.prox(st, eta, u)
        obj = lambda x: 0.5 * np.sum((x - u) ** 2) + 2 * eta * P.lambda2 * P.g(st, x)
        f0 = obj(b)
        assert np.isfinite(f0)
        for _ in range(40):
            d = r.normal(size=p) * 10 ** r.uniform(-6, -1)
            d[st == -1] = 0
            assert obj(b + d) >= f0 - 1e-12


def test_prox_edge_budgets():
    P = tiny_problem(p=6, k=3, M=2.0, lambda2=1.0)
    u = np.array([3.0, -0.2, 0.7, -1.1, 0.05, 5.0])
    eta = 0.5
    # kbar = 0: every free coefficient is zero
    st = np.array([1, 1, 1, 0, 0, 0], np.int8)
    b = P.prox(st, eta, u)
    assert np.all(b[3:] == 0.0)
    # J1 coordinates: ridge shrink u / (1 + 2 eta lambda2), then clip at M
    assert b[0] == pytest.approx(min(3.0 / 2.0, 2.0))
    assert b[1] == pytest.approx(-0.1)
    # all free with kbar >= pf: plain ridge + box on every coordinate
    st = np.zeros(6, np.int8)
    P6 = tiny_problem(p=6, k=6, M=2.0, lambda2=1.0)
    b = P6.prox(st, eta, u)
    assert np.allclose(b, np.clip(u / 2.0, -2.0, 2.0), rtol=1e-15, atol=0)
    # J0 is zeroed
    st = np.array([-1, 0, 0, -1, 0, 0], np.int8)
    b = P.prox(st, eta, u)
    assert b[0] == 0.0 and b[3] == 0.0


def test_prox_ties():
    """Equal magnitudes straddling the budget boundary are pooled symmetrically."""
    P = tiny_problem(p=6, k=2, M=5.0, lambda2=1.0)
    st = np.zeros(6, np.int8)
    u = np.array([1.0, -1.0, 1.0, 0.2, -1.0, 0.1])
    b = P.prox(st, 0.25, u)
    ref = prox_by_generic_solve(u, st, 2, 2.0, 5.0)
    assert np.max(np.abs(b - ref)) < 1e-7
    mags = np.abs(b[[0, 1, 2, 4]])
    assert np.ptp(mags) < 1e-14


# ---------------------------------------------------------------------------
# Primal/dual objectives and node bounds.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kind", [oracle.SQUARED, oracle.LOGISTIC])
def test_weak_duality_random_pairs(kind):
    r = rng(9)
    viol = 0
    for trial in range(300):
        P = tiny_problem(n=15, p=8, k=3, loss=kind, seed=trial, M=1.5, lambda2=0.6)
        st = random_state(r, 8, 3)
        b = feasible_beta(r, st, 3, P.M)
        if kind == oracle.LOGISTIC:
            zeta = P.y * r.uniform(0, 1, size=P.n)
        else:
            zeta = r.normal(size=P.n) * 2
        if P.dual(st, zeta) > P.primal(st, b) + 1e-10:
            viol += 1
    assert viol == 0


@pytest.mark.parametrize("kind", [oracle.SQUARED, oracle.LOGISTIC])
def test_node_bound_bracket_and_brute_force(kind):
    """LB <= node value <= every feasible support's value inside the node."""
    r = rng(10)
    P = tiny_problem(n=40, p=8, k=3, loss=kind, seed=11, M=2.0,
                     lambda2=0.05 if kind == oracle.SQUARED else 0.5)
    supp_val = {}
    for S in itertools.chain.from_iterable(itertools.combinations(range(8), s) for s in range(4)):
        supp_val[S] = support_value_scipy(P, list(S))
    for trial in range(25):
        st = random_state(r, 8, 3)
        res = P.node_bound(st, tol=1e-10)
        assert res["status"] == oracle.CONVERGED
        assert res["lb"] <= res["phi"] + 1e-12 * abs(res["phi"])
        assert res["gap"] <= 1e-10
        J1 = set(np.where(st == 1)[0]); J0 = set(np.where(st == -1)[0])
        inside = [v for S, v in supp_val.items() if J1 <= set(S) and not (J0 & set(S))]
        assert res["lb"] <= min(inside) * (1 + 1e-9)


def test_ridge_closed_form_when_k_equals_p():
    inst = W.small_instance(200, 12, 12, W.SQUARED, seed=3, M=100.0, lambda2=0.5)
    P = oracle.Problem.from_instance(inst)
    st = np.zeros(12, np.int8)
    res = P.node_bound(st, tol=1e-12, max_iter=100000)
    X, y = inst.X, inst.y
    br = np.linalg.solve(X.T @ X + 0.5 * np.eye(12), X.T @ y)
    vr = np.sum((y - X @ br) ** 2) + 0.5 * np.sum(br ** 2)
    assert res["lb"] == pytest.approx(vr, rel=1e-11)
    assert res["phi"] == pytest.approx(vr, rel=1e-11)
    assert np.max(np.abs(res["beta"] - br)) < 1e-6


def test_node_bound_prunes_against_upper_bound():
    inst = W.small_instance(300, 20, 4, W.SQUARED, seed=5)
    P = oracle.Problem.from_instance(inst)
    st = np.zeros(20, np.int8)
    full = P.node_bound(st, tol=1e-10)
    cut = P.node_bound(st, tol=1e-10, ub=full["lb"] * 0.9)
    assert cut["status"] == oracle.PRUNED
    assert cut["iterations"] <= full["iterations"]


def test_round_branch_fig2_example():
    fx = json.load(open(os.path.join(HERE, "golden", "fig2_padding_example.json")))
    p, k = fx["p"], fx["k"]
    P = tiny_problem(p=p, k=k)
    for i, nd in enumerate(fx["nodes"]):
        st = np.zeros(p, np.int8)
        st[[j - 1 for j in nd["J1"]]] = 1
        st[[j - 1 for j in nd["J0"]]] = -1
        assert int(np.sum(st == 0)) == fx["free_counts"][i]
        assert P.kbar(st) == fx["reduced_budgets"][i]
        order = fx["sorted_free_order"][i]
        beta = np.zeros(p)
        for rank, j in enumerate(order):           # magnitudes in the printed order
            beta[j - 1] = (len(order) - rank) * (-1) ** rank * 0.1
        for j in nd["J1"]:
            beta[j - 1] = 0.05
        supp, br = P.round_branch(st, beta)
        kb = fx["reduced_budgets"][i]
        assert br == order[0] - 1
        exp = sorted([j - 1 for j in nd["J1"]] + [j - 1 for j in order[:kb]])
        assert list(supp) == exp
        assert p - fx["free_counts"][i] == fx["padding_rows_after_sort"][i]


def test_round_branch_ties_go_to_lowest_index():
    P = tiny_problem(p=6, k=3)
    st = np.array([0, 0, 0, 0, 0, 1], np.int8)
    beta = np.array([0.0, 2.0, 0.5, 2.0, 0.5, 1.0])
    supp, br = P.round_branch(st, beta)
    assert br == 1
    assert list(supp) == [1, 3, 5]
    beta = np.array([0.0, 2.0, 0.5, 2.0, 0.5, 1.0]); beta[3] = 0.5; beta[1] = 0.5
    supp, br = P.round_branch(st, beta)
    assert br == 1 and list(supp) == [1, 2, 5]


# ---------------------------------------------------------------------------
# Support values and branch and bound, against brute force and closed forms.
# ---------------------------------------------------------------------------

def support_value_scipy(P, S):
    """v(S) by a library solver: bvls for squared loss, L-BFGS-B for logistic."""
    S = list(S)
    if len(S) == 0:
        if P.loss == oracle.SQUARED:
            return float(np.sum(P.y ** 2))
        return float(P.n * math.log(2.0))
    XS = P.X[:, S]
    if P.loss == oracle.SQUARED:
        A = np.vstack([XS, math.sqrt(P.lambda2) * np.eye(len(S))])
        b = np.concatenate([P.y, np.zeros(len(S))])
        res = optimize.lsq_linear(A, b, bounds=(-P.M, P.M), method="bvls", tol=1e-14)
        beta = res.x
        return float(np.sum((P.y - XS @ beta) ** 2) + P.lambda2 * np.sum(beta ** 2))

    def f(bb):
        s = XS @ bb
        z = -P.y * s
        val = np.sum(np.logaddexp(0.0, z)) + P.lambda2 * bb @ bb
        sig = 1.0 / (1.0 + np.exp(-z))
        grad = XS.T @ (-P.y * sig) + 2 * P.lambda2 * bb
        return val, grad
    res = optimize.minimize(f, np.zeros(len(S)), jac=True, method="L-BFGS-B",
                            bounds=[(-P.M, P.M)] * len(S),
                            options={"ftol": 1e-15, "gtol": 1e-12, "maxiter": 5000})
    return float(res.fun)


def test_support_value_matches_library_solvers():
    r = rng(12)
    for kind in (oracle.SQUARED, oracle.LOGISTIC):
        P = tiny_problem(n=60, p=10, k=4, loss=kind, seed=13, M=0.8, lambda2=0.3)
        for _ in range(10):
            S = sorted(r.choice(10, size=int(r.integers(1, 5)), replace=False))
            v, beta = P.support_value(S)
            assert v == pytest.approx(support_value_scipy(P, S), rel=1e-9)
            off = np.setdiff1d(np.arange(10), S)
            assert np.all(beta[off] == 0.0) and np.all(np.abs(beta) <= P.M)


def brute_force_squared(X, y, k, lambda2, M):
    """All C(p, k) supports: batched ridge solves, bvls where the box binds."""
    n, p = X.shape
    G = X.T @ X
    c = X.T @ y
    yy = float(y @ y)
    combos = np.array(list(itertools.combinations(range(p), k)), dtype=np.int64)
    A = G[combos[:, :, None], combos[:, None, :]] + lambda2 * np.eye(k)
    b = c[combos]
    beta = np.linalg.solve(A, b[..., None])[..., 0]
    vals = yy - 2 * np.einsum("ij,ij->i", b, beta) + np.einsum("ij,ijk,ik->i", beta, A, beta)
    boxed = np.where(np.max(np.abs(beta), axis=1) > M)[0]
    for i in boxed:
        S = combos[i]
        Aa = np.vstack([X[:, S], math.sqrt(lambda2) * np.eye(k)])
        bb = np.concatenate([y, np.zeros(k)])
        res = optimize.lsq_linear(Aa, bb, bounds=(-M, M), method="bvls", tol=1e-14)
        vals[i] = np.sum((y - X[:, S] @ res.x) ** 2) + lambda2 * np.sum(res.x ** 2)
    order = np.argsort(vals)
    # recompute the two best from residuals (no Gram cancellation)
    out = []
    for i in order[:2]:
        S = combos[i]
        Aa = np.vstack([X[:, S], math.sqrt(lambda2) * np.eye(k)])
        bb = np.concatenate([y, np.zeros(k)])
        res = optimize.lsq_linear(Aa, bb, bounds=(-M, M), method="bvls", tol=1e-14)
        out.append((float(np.sum((y - X[:, S] @ res.x) ** 2) + lambda2 * np.sum(res.x ** 2)),
                    list(S)))
    return out, len(combos)


def test_bnb_plain_squared_500x30_matches_brute_force():
    inst = W.plain_bnb_squared_500x30()
    P = oracle.Problem.from_instance(inst)
    res = P.bnb()
    assert res["status"] == 0 and res["rel_gap"] <= 1e-6
    (best, second), count = brute_force_squared(inst.X, inst.y, inst.k, inst.lambda2, inst.M)
    assert count == math.comb(30, 5)
    margin = (second[0] - best[0]) / best[0]
    assert margin > 1e-6
    assert list(res["support"]) == best[1]
    assert res["objective"] == pytest.approx(best[0], rel=1e-9)


def test_bnb_orthogonal_design_closed_form():
    """X^T X diagonal: v(S) separates, the optimum is the top-k per-coordinate gains."""
    r = rng(14)
    n, p, k, lam, M = 300, 60, 5, 0.2, 1.5
    Q, _ = np.linalg.qr(r.normal(size=(n, p)))
    d = r.uniform(2.0, 6.0, size=p)
    X = Q * d
    beta_true = np.zeros(p)
    beta_true[r.choice(p, 8, replace=False)] = r.uniform(0.5, 1.3, 8) * r.choice([-1, 1], 8)
    y = X @ beta_true + 0.3 * r.normal(size=n)
    P = oracle.Problem(X, y, k, oracle.SQUARED, lam, M)
    res = P.bnb()
    c = X.T @ y
    a = d * d + lam
    bstar = np.clip(c / a, -M, M)
    gain = -(a * bstar ** 2 - 2 * c * bstar)
    top = np.argsort(-gain, kind="stable")[:k]
    assert sorted(gain)[-k] - sorted(gain)[-k - 1] > 1e-6
    assert list(res["support"]) == sorted(top.tolist())
    assert res["objective"] == pytest.approx(float(y @ y) - gain[top].sum(), rel=1e-9)


def test_bnb_logistic_tiny_matches_brute_force():
    inst = W.small_instance(200, 12, 3, W.LOGISTIC, seed=21, M=2.0, lambda2=1.0)
    P = oracle.Problem.from_instance(inst)
    res = P.bnb()
    vals = sorted((support_value_scipy(P, S), list(S))
                  for S in itertools.combinations(range(12), 3))
    assert (vals[1][0] - vals[0][0]) / vals[0][0] > 1e-6
    assert list(res["support"]) == vals[0][1]
    assert res["objective"] == pytest.approx(vals[0][0], rel=1e-8)
    assert res["lower_bound"] <= vals[0][0] * (1 + 1e-9)


def test_bnb_root_bound_below_optimum():
    inst = W.plain_bnb_squared_500x30()
    P = oracle.Problem.from_instance(inst)
    root = P.node_bound(np.zeros(30, np.int8), tol=1e-10)
    res = P.bnb()
    assert root["lb"] <= res["objective"] * (1 + 1e-12)


# ---------------------------------------------------------------------------
# Rashomon-set collection (Sec. 4.5): brute force over every support with
# |S| <= k.  The set's definition is v(S) <= (1 + eps) Phi*, with v computed
# by the (separately pinned) support_value; a cap N keeps the N best.
# ---------------------------------------------------------------------------
def _brute_rashomon(P, p, k, eps, cap=0):
    vals = {}
    for size in range(0, k + 1):
        for S in itertools.combinations(range(p), size):
            vals[S] = P.support_value(list(S))[0]
    phi = min(vals.values())
    tau = (1 + eps) * phi
    inside = sorted(((v, S) for S, v in vals.items() if v <= tau), key=lambda t: (t[0], t[1]))
    if cap:
        inside = inside[:cap]
    return phi, tau, [(S, v) for v, S in inside]


RASHOMON_CASES = [  # loss, n, p, k, seed, eps, cap
    (0, 60, 10, 3, 50, 0.05, 0), (0, 60, 10, 3, 50, 0.3, 0), (1, 80, 9, 3, 50, 0.05, 0),
    (1, 80, 9, 3, 50, 0.15, 0), (1, 40, 8, 3, 7, 0.05, 0), (1, 40, 8, 3, 7, 0.2, 12),
    (0, 60, 10, 3, 51, 0.5, 5)]


@pytest.mark.parametrize("loss,n,p,k,seed,eps,cap", RASHOMON_CASES)
def test_rashomon_matches_brute_force(loss, n, p, k, seed, eps, cap):
    inst = W.small_instance(n, p, k, loss, seed=seed, rho=0.5)
    P = oracle.Problem.from_instance(inst)
    phi, tau, want = _brute_rashomon(P, p, k, eps, cap)
    got = P.rashomon(eps, cap=cap)
    assert got["status"] == 0
    assert got["optimum"] == pytest.approx(phi, rel=1e-12)
    assert [S for S, _ in got["set"]] == [S for S, _ in want]
    for (_, v1), (_, v2) in zip(got["set"], want):
        assert v1 == pytest.approx(v2, rel=1e-12)


def test_rashomon_brute_force_cases_include_smaller_supports():
    """The pin above is only meaningful if some set holds supports of size
    < k (a leaf rule stopping at #free <= kbar would miss them) and some cap
    cuts a set short."""
    inst = W.small_instance(80, 9, 3, 1, seed=50, rho=0.5)
    P = oracle.Problem.from_instance(inst)
    _, _, want = _brute_rashomon(P, 9, 3, 0.15)
    assert any(len(S) < 3 for S, _ in want) and any(len(S) == 3 for S, _ in want)
    inst = W.small_instance(40, 8, 3, 1, seed=7, rho=0.5)
    P = oracle.Problem.from_instance(inst)
    assert len(_brute_rashomon(P, 8, 3, 0.2)[2]) > 12


def weak_logistic_120x20():
    """Weak signal (|beta*_j| = 0.3, SNR-free labels): many near-optimal supports."""
    return W.make_instance("weak_logistic_120x20", 120, 20, 0.5, 4, W.LOGISTIC, 1.0, 2.0, W.F64, 3,
                           snr=1.0, beta_values=np.full(4, 0.3))


def test_rashomon_matches_brute_force_p20():
    """6196 supports (|S| <= 4 of 20); the set has supports of sizes 3 and 4."""
    inst = weak_logistic_120x20()
    P = oracle.Problem.from_instance(inst)
    phi, tau, want = _brute_rashomon(P, 20, 4, 0.02)
    got = P.rashomon(0.02)
    assert got["optimum"] == pytest.approx(phi, rel=1e-12)
    assert [S for S, _ in got["set"]] == [S for S, _ in want]
    assert len(want) > 100


# ---------------------------------------------------------------------------
# Fixed-model reliance (appendix on variable importance over the Rashomon
# set): zero off the support, the squared-loss closed form, and for the
# logistic loss the first-order expansion in the removed coefficient.
# ---------------------------------------------------------------------------

def test_reliance_zero_off_support_and_squared_closed_form():
    inst = W.small_instance(90, 12, 4, oracle.SQUARED, seed=21)
    P = oracle.Problem.from_instance(inst)
    beta = np.zeros(12)
    beta[[1, 5, 9]] = [0.7, -1.3, 0.25]
    R = P.reliance(beta)
    assert np.all(R[[0, 2, 3, 4, 6, 7, 8, 10, 11]] == 0.0)
    # (r + x_j b_j)^2 - r^2 = 2 r x_j b_j + x_j^2 b_j^2 with r = y - X beta
    X, y, n = P.X, P.y, P.n
    r = y - X @ beta
    for j in (1, 5, 9):
        want = (2.0 * beta[j] * (X[:, j] @ r) + beta[j] ** 2 * (X[:, j] @ X[:, j])) / n
        assert R[j] == pytest.approx(want, rel=1e-12, abs=1e-14)


def test_reliance_logistic_first_order_in_the_removed_coefficient():
    inst = W.small_instance(150, 10, 4, oracle.LOGISTIC, seed=22)
    P = oracle.Problem.from_instance(inst)
    X, y, n = P.X, P.y, P.n
    base = np.zeros(10)
    base[[0, 3, 7]] = [0.9, -0.6, 0.4]
    for h in (1e-3, 1e-4):
        beta = base.copy()
        beta[5] = h
        R = P.reliance(beta)
        eta = X @ beta
        # d/dt mean l(eta - t x_5) at t = 0 is -(1/n) sum x_i5 l'(eta_i),
        # l'(s) = -y / (1 + exp(y s)); the remainder is O(h^2)
        dl = -y / (1.0 + np.exp(y * eta))
        first = -h * (X[:, 5] @ dl) / n
        assert abs(R[5] - first) <= 2.0 * h * h * (X[:, 5] ** 2).mean()
