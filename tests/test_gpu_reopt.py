"""Batched support re-optimisation on the GPU (evaluate_supports) against the
oracle's support value (pinned against scipy's bounded least squares and
L-BFGS-B).

The kernel stops at a relative duality gap of 1e-9 and reports the value at
its returned coefficients and a dual bound, so: value within 1e-8 of the
oracle's v(S) (solved to 1e-13), lower bound below it, and the oracle's own
objective at the returned coefficients equal to the reported value.

Tall instances split each support's rows over several workgroups (one grid
barrier per step, the partial sums added in a fixed order): the same checks
hold there, with the split forced on small cases (including workgroups with
no rows and supports that finish while others still iterate) and chosen
automatically on tall ones, where it must also agree with one workgroup per
support."""
import numpy as np
import pytest

import oracle
import paper_2605_22188_amd as K
import workloads as W

pytestmark = pytest.mark.gpu


def _check(inst, supports, rel=1e-8, **kw):
    P = oracle.Problem.from_instance(inst)
    h = K.create_from_instance(inst, batch_width=64, **kw)
    r = K.evaluate_supports(h, supports)
    K.destroy_problem(h)
    for i, S in enumerate(supports):
        S = list(S)
        v = P.support_value(S, tol=1e-12)[0] if S else P.primal(np.full(inst.p, -1, np.int8), np.zeros(inst.p))
        assert r["status"][i] == 0, (S, r["iterations"][i])
        assert r["value"][i] == pytest.approx(v, rel=rel), S
        assert r["lower_bound"][i] <= v * (1 + 1e-12) + 1e-12
        assert r["lower_bound"][i] <= r["value"][i]
        b = r["beta"][i]
        off = np.setdiff1d(np.arange(inst.p), S)
        assert np.all(b[off] == 0.0) and np.all(np.abs(b) <= inst.M)
        st = np.full(inst.p, -1, np.int8)
        st[S] = 1
        assert P.primal(st, b) == pytest.approx(r["value"][i], rel=1e-10)
    return r


def _random_supports(p, sizes, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    return [tuple(sorted(g.choice(p, size=s, replace=False).tolist())) for s in sizes]


@pytest.mark.parametrize("loss,dtype", [(0, "f64"), (1, "f32"), (0, "bf16"), (1, "bf16")])
def test_supports_small(loss, dtype):
    print(f"[gpu-test] evaluate_supports loss={loss} dtype={dtype}", flush=True)
    inst = W.small_instance(700, 50, 20, loss, seed=61, rho=0.6, dtype=dtype)
    sups = _random_supports(50, [1, 3, 5, 8, 12, 16, 17, 20], seed=62) + [()]
    _check(inst, sups)


def test_supports_template_edges_and_wide():
    print("[gpu-test] evaluate_supports 16/32/33/64 features", flush=True)
    inst = W.small_instance(900, 90, 64, 1, seed=63, rho=0.3, dtype="f32")
    sups = _random_supports(90, [32, 33, 48, 64], seed=64)
    _check(inst, sups, rel=1e-7)


def test_supports_many_rows():
    print("[gpu-test] evaluate_supports 20000 x 40 logistic", flush=True)
    inst = W.small_instance(20000, 40, 15, 1, seed=65, rho=0.7, dtype="f32")
    sups = _random_supports(40, [5, 10, 15], seed=66)
    sups.append(tuple(int(j) for j in np.flatnonzero(inst.beta_true)))
    _check(inst, sups)


def test_supports_errors():
    print("[gpu-test] evaluate_supports errors", flush=True)
    inst = W.small_instance(100, 20, 5, 0, seed=67)
    h = K.create_from_instance(inst, batch_width=64)
    with pytest.raises(K.KbnbError):
        K.evaluate_supports(h, [(1, 1)])
    with pytest.raises(K.KbnbError):
        K.evaluate_supports(h, [(3, 25)])
    assert K.evaluate_supports(h, [])["value"].shape == (0,)
    K.destroy_problem(h)


@pytest.mark.parametrize("groups,loss,dtype", [(2, 0, "f64"), (3, 1, "f32"), (7, 1, "bf16"), (16, 0, "f32")])
def test_supports_split_rows_forced(groups, loss, dtype):
    print(f"[gpu-test] evaluate_supports split over {groups} workgroups loss={loss} dtype={dtype}",
          flush=True)
    inst = W.small_instance(700, 50, 20, loss, seed=68, rho=0.6, dtype=dtype)
    sups = _random_supports(50, [1, 3, 5, 8, 12, 16, 17, 20], seed=69) + [()]
    _check(inst, sups, reopt_groups=groups)


def test_supports_split_rows_empty_groups():
    """More workgroups than the rows divide into: the last ones own no rows."""
    print("[gpu-test] evaluate_supports 5 rows over 4 workgroups", flush=True)
    inst = W.small_instance(5, 12, 3, 0, seed=70, dtype="f64")
    _check(inst, [(0,), (1, 4), (2, 5, 9)], reopt_groups=4)


def test_supports_split_rows_iteration_limit():
    """At the step limit every workgroup of a support stops at the same step."""
    print("[gpu-test] evaluate_supports split rows at the step limit", flush=True)
    inst = W.small_instance(3000, 60, 40, 1, seed=71, rho=0.9, dtype="f32")
    sups = _random_supports(60, [20, 20, 40], seed=72)
    for g in (1, 5):
        h = K.create_from_instance(inst, batch_width=64, reopt_groups=g)
        r = K.evaluate_supports(h, sups, rel_tol=1e-15, max_iters=35)
        K.destroy_problem(h)
        assert np.all(r["status"] == 2) and np.all(r["iterations"] == 35), (g, r["iterations"])
        assert np.all(r["lower_bound"] <= r["value"])


def test_supports_tall_automatic_split():
    """100000 rows (the tall logistic shape): the automatic split against the
    oracle and against one workgroup per support."""
    print("[gpu-test] evaluate_supports 100000 x 60 logistic, automatic split", flush=True)
    inst = W.small_instance(100000, 60, 40, 1, seed=73, rho=0.7, dtype="bf16")
    sups = _random_supports(60, [1, 5, 10, 15, 15, 24, 40], seed=74)
    sups.append(tuple(int(j) for j in np.flatnonzero(inst.beta_true)))
    r = _check(inst, sups)
    h = K.create_from_instance(inst, batch_width=64, reopt_groups=1)
    one = K.evaluate_supports(h, sups)
    K.destroy_problem(h)
    assert np.all(one["status"] == 0)
    np.testing.assert_allclose(r["value"], one["value"], rtol=2e-9)
    assert np.all(r["lower_bound"] <= one["value"] * (1 + 1e-12))
    assert np.all(one["lower_bound"] <= r["value"] * (1 + 1e-12))
