"""GPU Rashomon-set collection against the oracle's (pinned by brute force).

Values on the GPU are certified to the support re-optimisation tolerance
(1e-7 relative), the oracle's to 1e-13, so a support whose value lies within
2e-6 of the threshold may fall on either side: outside that band the sets
must agree, values to 1e-6, and every returned iterate must attain its value
(the oracle's primal value at it, on its support)."""
import numpy as np
import pytest

import oracle
import paper_2605_22188_amd as K
import workloads as W
from test_oracle_pins import RASHOMON_CASES, weak_logistic_120x20

pytestmark = pytest.mark.gpu


def _compare(inst, eps, cap, batch_width=64):
    P = oracle.Problem.from_instance(inst)
    ref = P.rashomon(eps, cap=cap, node_tol=1e-9)
    h = K.create_from_instance(inst, batch_width=batch_width)
    out = K.branch_and_bound(h, rashomon_eps=eps, rashomon_n=cap)
    K.destroy_problem(h)
    assert out["status"] == 0
    assert out["objective"] == pytest.approx(ref["optimum"], rel=1e-6)
    # the whole tree was decided: its bound meets the optimum
    assert out["rel_gap"] <= 1e-6 and out["lower_bound"] <= out["objective"]
    got = {S: (v, b) for S, v, b in out["rashomon"]}
    want = dict(ref["set"])
    vals = [v for _, v, _ in out["rashomon"]]
    assert vals == sorted(vals)
    # the threshold of the comparison: the oracle's, and with a cap its N-th value
    tau = ref["threshold"]
    band = 2e-6 * abs(tau)
    for S, v in want.items():
        if v < tau - band:
            assert S in got, (S, v, tau)
            assert got[S][0] == pytest.approx(v, rel=1e-6)
    for S, (v, b) in got.items():
        assert S in want or abs(v - tau) <= band, (S, v, tau)
        st = np.full(inst.p, -1, np.int8)
        st[list(S)] = 1
        assert np.all(b[np.setdiff1d(np.arange(inst.p), list(S))] == 0.0)
        assert P.primal(st, b) == pytest.approx(v, rel=1e-9)
    return out, ref


@pytest.mark.parametrize("loss,n,p,k,seed,eps,cap", RASHOMON_CASES)
def test_rashomon_small_cases(loss, n, p, k, seed, eps, cap):
    print(f"[gpu-test] rashomon loss={loss} {n}x{p} k={k} eps={eps} cap={cap}", flush=True)
    inst = W.small_instance(n, p, k, loss, seed=seed, rho=0.5)
    _compare(inst, eps, cap)


@pytest.mark.parametrize("eps,cap", [(0.02, 0), (0.05, 40)])
def test_rashomon_weak_logistic_120x20(eps, cap):
    print(f"[gpu-test] rashomon weak logistic 120x20 eps={eps} cap={cap}", flush=True)
    inst = weak_logistic_120x20()
    out, ref = _compare(inst, eps, cap)
    assert len(out["rashomon"]) >= (40 if cap else 150)
    # the same set through the compact pool: ascending sequences, coefficients
    # in path order, and prefixes shared
    h = K.create_from_instance(inst, batch_width=64)
    out2 = K.branch_and_bound(h, rashomon_eps=eps, rashomon_n=cap)
    pool = K.Pool.from_problem(h)
    K.destroy_problem(h)
    N, T, C = pool.info()
    assert N == len(out2["rashomon"]) and C == sum(len(S) for S, _, _ in out2["rashomon"])
    assert T - 1 < C
    for m, (S, v, b) in enumerate(out2["rashomon"]):
        seq, coef, val = pool.record(m)
        assert seq == S and val == v
        np.testing.assert_array_equal(coef, b[list(S)])
    pool.close()


def test_rashomon_entry_errors_and_plain_bnb_unchanged():
    print("[gpu-test] rashomon entry errors", flush=True)
    inst = W.plain_bnb_squared_500x30()
    h = K.create_from_instance(inst, batch_width=64)
    with pytest.raises(K.KbnbError):
        K.rashomon_entry(h, 0)            # nothing collected yet
    with pytest.raises(K.KbnbError):
        K.Pool.from_problem(h)
    out = K.branch_and_bound(h, rashomon_eps=0.05)
    assert [S for S, _, _ in out["rashomon"]] == [(0, 6, 12, 18, 24)]
    with pytest.raises(K.KbnbError):
        K.rashomon_entry(h, 1)
    plain = K.branch_and_bound(h)
    assert list(plain["support"]) == [0, 6, 12, 18, 24] and "rashomon" not in plain
    K.destroy_problem(h)


def _reliance_vs_oracle(inst, eps, cap):
    h = K.create_from_instance(inst, batch_width=64)
    out = K.branch_and_bound(h, rashomon_eps=eps, rashomon_n=cap)
    pool = K.Pool.from_problem(h)
    rel = K.rashomon_reliance(h, pool)
    K.destroy_problem(h)
    P = oracle.Problem.from_instance(inst)
    mean_loss = None
    N, _, C = pool.info()
    assert N == len(out["rashomon"]) and rel.shape == (C,)
    o = 0
    for m in range(N):
        seq, coef, _ = pool.record(m)
        beta = np.zeros(inst.p)
        beta[list(seq)] = coef
        want = P.reliance(beta)
        if mean_loss is None:
            mean_loss = abs(P.primal(np.where(beta != 0, 1, -1).astype(np.int8), beta)) / inst.n
        # float64 sums of n terms in another order
        for r, j in enumerate(seq):
            assert abs(rel[o + r] - want[j]) <= 1e-11 * (mean_loss + abs(want[j])), (m, j)
        o += len(seq)
    s = K.pool_summary(pool, inst.p, rel)
    pool.close()
    return out, s


def test_reliance_matches_oracle_logistic_pool():
    print("[gpu-test] reliance on the weak logistic 120x20 pool", flush=True)
    out, s = _reliance_vs_oracle(weak_logistic_120x20(), 0.05, 40)
    assert len(out["rashomon"]) == 40
    # every record holds its own support: frequencies sum to the mean support size
    assert s["freq"].sum() == pytest.approx(np.mean([len(S) for S, _, _ in out["rashomon"]]))


def test_reliance_matches_oracle_squared_pool():
    print("[gpu-test] reliance on a squared-loss pool (float32 X)", flush=True)
    inst = W.small_instance(300, 16, 4, 0, seed=31, rho=0.7, dtype="f32")
    _reliance_vs_oracle(inst, 0.2, 25)


def test_reliance_errors():
    print("[gpu-test] reliance errors", flush=True)
    inst = W.small_instance(60, 10, 3, 0, seed=50)
    h = K.create_from_instance(inst, batch_width=64)
    pool = K.Pool()
    pool.add([1, 12], [0.5, 0.5], 1.0)  # feature 12 outside [0, 10)
    with pytest.raises(K.KbnbError):
        K.rashomon_reliance(h, pool)
    empty = K.Pool()
    assert K.rashomon_reliance(h, empty).shape == (0,)
    K.destroy_problem(h)
    pool.close()
    empty.close()
