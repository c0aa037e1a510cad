"""Parity at the full benchmark sizes, in the launch configurations bench.py
times, on sampled outputs the oracle can check one by one:

  * 100000 x 5000 bfloat16 logistic (rho 0.7, k 15): sampled nodes of a
    256-node launch (anchored bfloat16 iteration, certificate every 32
    steps) satisfy the duality bracket at the returned iterate,
    LB <= Phi_oracle(beta) and Phi_oracle(beta) - LB <= 1e-6 |Phi_oracle|,
    with the rounding support and branching index bit-exact at beta; the
    branch and bound with eps = 0.01 returns an objective the oracle
    reproduces at its coefficients and a gap within 1e-6;
  * 10000 x 1000 bfloat16 squared (rho 0.9, k 10): the full branch and bound
    at zero gap, with the incumbent's objective reproduced by the oracle at
    the returned coefficients and its bound below it.

Both searches run in audit mode: every discarded subtree comes back with the
certificate of its bound, and the oracle replays each certificate's dual
value in float64 from the exact instance (tests/audit_replay.py), so every
pruning decision and the reported global bound are checked independently of
the device arithmetic.

The oracle's own node solves are too slow at these sizes; its certificate
arithmetic is compared element by element elsewhere."""
import numpy as np
import pytest

import audit_replay
import oracle
import paper_2605_22188_amd as K
import workloads as W

pytestmark = pytest.mark.gpu


def _state_of_support(p, S):
    st = np.full(p, -1, np.int8)
    st[list(S)] = 1
    return st


def test_large_logistic_100000x5000_sampled_nodes_and_rashomon():
    print("[gpu-test] 100000x5000 bf16 logistic: drawing", flush=True)
    torch = pytest.importorskip("torch")
    inst = W.large_logistic_100000x5000_bf16()
    X = torch.from_numpy(inst.X_store).cuda()
    y = torch.from_numpy(inst.y).cuda()
    h = K.create_problem(X, y, inst.k, inst.loss, inst.lambda2, inst.M, dtype=inst.dtype,
                         batch_width=256, cert_period=32)
    del X, y
    P = oracle.Problem.from_instance(inst)
    nodes = W.random_nodes(inst.p, 256, 7, 500, seed=3000)
    print("[gpu-test] 100000x5000: one 256-node launch", flush=True)
    res = K.bound_nodes(h, nodes, rel_tol=1e-6)
    assert all(g["status"] == K.CONVERGED for g in res)
    for i in (0, 37, 101, 255):
        st = W.node_state(inst.p, nodes[i])
        g = res[i]
        phi_o = P.primal(st, g["beta"])
        assert g["lower_bound"] <= phi_o + 1e-12 * abs(phi_o), i
        assert phi_o - g["lower_bound"] <= (1e-6 + 1e-9) * abs(phi_o), i
        s_o, br_o = P.round_branch(st, g["beta"])
        assert list(g["support"]) == list(s_o), i
        assert g["branch_index"] == br_o, i
    print("[gpu-test] 100000x5000: branch and bound, eps 0.01", flush=True)
    out = K.branch_and_bound(h, time_limit_s=150, rashomon_eps=0.01, audit=True)
    K.destroy_problem(h)
    assert out["status"] == 0 and out["rel_gap"] <= 1e-6
    S = [int(j) for j in out["support"]]
    assert P.primal(_state_of_support(inst.p, S), out["beta"]) == pytest.approx(out["objective"], rel=1e-9)
    assert [tuple(S)] == [T for T, _, _ in out["rashomon"]]
    print(f"[gpu-test] 100000x5000: replaying {len(out['leaves'])} leaf certificates", flush=True)
    summary = audit_replay.replay(P, out, rashomon_eps=0.01)
    print(f"[gpu-test] 100000x5000 audit: {summary}", flush=True)


def test_bnb_squared_10000x1000_bf16_zero_gap():
    print("[gpu-test] 10000x1000 bf16 squared: branch and bound", flush=True)
    inst = W.bnb_squared_10000x1000_bf16()
    P = oracle.Problem.from_instance(inst)
    h = K.create_from_instance(inst, batch_width=1024, cert_period=16)
    out = K.branch_and_bound(h, time_limit_s=120, audit=True)
    K.destroy_problem(h)
    assert out["status"] == 0 and out["rel_gap"] <= 1e-6
    S = [int(j) for j in out["support"]]
    assert len(S) <= inst.k
    phi = P.primal(_state_of_support(inst.p, S), out["beta"])
    assert phi == pytest.approx(out["objective"], rel=1e-9)
    assert out["lower_bound"] <= phi * (1 + 1e-12)
    summary = audit_replay.replay(P, out)
    print(f"[gpu-test] 10000x1000 audit: {summary}", flush=True)
    # the replayed bounds alone certify the optimum to the gap tolerance
    assert summary["min_replayed"] >= out["objective"] * (1 - 1e-6) - 1e-9 * abs(out["objective"])
