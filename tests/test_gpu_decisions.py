"""GPU parity of pruning decisions close to the pruning threshold, and the
handle's state after a search that stops early.

A node is pruned when its certified bound reaches UB - 1e-6 |UB| (the prune
rule of Sec. 3, "Safe Lower Bound and Pruning", with the relative slack the
driver uses).  The oracle's node value v (solved to a 1e-10 gap, so v is
known to far better than the band) decides what the right decision is; the
GPU must agree on every node whose v lies outside the band
|v - (UB - 1e-6 |UB|)| <= 2e-6 |UB|, and the band nodes are counted.
"""
import numpy as np
import pytest

import audit_replay
import oracle
import paper_2605_22188_amd as K
import workloads as W

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[gpu-test] {msg}", flush=True)


# relative offsets of UB from the node value: the band is +-2e-6, the node
# tolerance 1e-6, so +-5e-6 sits just outside the band
OFFSETS = (-1e-4, -1e-5, -5e-6, 5e-6, 1e-5, 1e-4)


def _setup(count, seed):
    inst = W.small_instance(2000, 80, 8, W.LOGISTIC, seed=12)
    P = oracle.Problem.from_instance(inst)
    nodes = W.random_nodes(80, count, 4, 20, seed=seed)
    refs = [P.node_bound(W.node_state(80, nd), tol=1e-10, max_iter=100000) for nd in nodes]
    r = np.random.Generator(np.random.PCG64(seed + 1))
    offs = np.array([OFFSETS[i % len(OFFSETS)] for i in range(count)])
    r.shuffle(offs)
    ubs = np.array([0.5 * (rf["lb"] + rf["phi"]) * (1 + o) for rf, o in zip(refs, offs)])
    return inst, P, nodes, refs, ubs, offs


def test_prune_decisions_near_the_band():
    announce("prune decisions logistic 2000x80, UB at v(1 +- 5e-6 / 1e-5 / 1e-4)")
    inst, P, nodes, refs, ubs, offs = _setup(60, 31)
    h = K.create_from_instance(inst, batch_width=64, cert_period=4)
    warm = [rf["beta"] if i % 2 else None for i, rf in enumerate(refs)]
    res = K.bound_nodes(h, nodes, upper_bound=ubs, rel_tol=1e-6, warm_starts=warm)
    band = 0
    for rf, ub, g in zip(refs, ubs, res):
        v = rf["lb"]
        thr = ub - 1e-6 * abs(ub)
        assert g["lower_bound"] <= rf["phi"] * (1 + 1e-12)
        if abs(v - thr) <= 2e-6 * abs(ub):
            band += 1
            continue
        assert (g["status"] == K.PRUNED) == (v >= thr), (v, ub, g["status"], g["lower_bound"])
    print(f"[gpu-test] band nodes: {band}", flush=True)
    assert band == 0
    K.destroy_problem(h)


def test_stop_unprunable_near_the_band():
    """With stop_unprunable: below the threshold by more than the band the
    node stops as UNPRUNABLE (primal value under the threshold) or converges;
    above it, it is PRUNED."""
    announce("stop_unprunable decisions logistic 2000x80, UB at v(1 +- 5e-6 / 1e-5 / 1e-4)")
    inst, P, nodes, refs, ubs, offs = _setup(48, 41)
    h = K.create_from_instance(inst, batch_width=64, cert_period=4)
    res = K.bound_nodes(h, nodes, upper_bound=ubs, rel_tol=1e-6, stop_unprunable=1)
    for rf, ub, g in zip(refs, ubs, res):
        v = rf["lb"]
        thr = ub - 1e-6 * abs(ub)
        assert abs(v - thr) > 2e-6 * abs(ub)
        assert g["lower_bound"] <= rf["phi"] * (1 + 1e-12)
        if v >= thr:
            assert g["status"] == K.PRUNED, (v, ub, g)
        else:
            assert g["status"] in (K.UNPRUNABLE, K.CONVERGED), (v, ub, g)
            if g["status"] == K.UNPRUNABLE:
                assert g["primal_value"] < thr
                assert g["primal_value"] >= rf["lb"] * (1 - 1e-12)
    K.destroy_problem(h)


def test_cancel_and_reuse_after_time_limit():
    """A branch and bound stopped by its time limit leaves the handle idle
    (no stale result of its nodes reaches a later call), and the same handle
    then bounds nodes that match the oracle and finishes a full search."""
    announce("bnb time limit, cancel, handle reuse: logistic 1000x60")
    inst = W.small_instance(1000, 60, 6, W.LOGISTIC, seed=61, rho=0.9)
    P = oracle.Problem.from_instance(inst)
    h = K.create_from_instance(inst, batch_width=128, cert_period=8)
    out = K.branch_and_bound(h, max_nodes=25)
    assert out["status"] == 2, out["status"]
    # nothing is left: an immediate poll finds no result
    res, rc = K.poll_bounds(h, cap=16, timeout_us=0)
    assert res == [] and rc == K.TIMEOUT
    nodes = W.random_nodes(60, 20, 3, 10, seed=62)
    got = K.bound_nodes(h, nodes, rel_tol=1e-6)
    for nd, g in zip(nodes, got):
        rf = P.node_bound(W.node_state(60, nd), tol=1e-10, max_iter=100000)
        assert g["status"] == K.CONVERGED
        assert g["lower_bound"] <= rf["phi"] * (1 + 1e-12)
        assert g["lower_bound"] >= rf["lb"] - 1e-6 * abs(rf["lb"])
    # submitted and cancelled before polling: nothing comes back, the handle is idle
    K.submit_nodes(h, nodes, tags=list(range(1000, 1020)))
    K.cancel_nodes(h)
    res, rc = K.poll_bounds(h, cap=32, timeout_us=0)
    assert res == [] and rc == K.TIMEOUT
    # a search that does not start from an idle handle is refused
    K.submit_nodes(h, nodes[:2])
    with pytest.raises(K.KbnbError):
        K.branch_and_bound(h)
    K.cancel_nodes(h)
    full = K.branch_and_bound(h)
    assert full["status"] == 0 and full["rel_gap"] <= 1e-6
    v_o, _ = P.support_value(full["support"])
    assert full["objective"] == pytest.approx(v_o, rel=1e-6)
    K.destroy_problem(h)


@pytest.mark.parametrize("order", [0, 1])
def test_audit_plain_squared_500x30(order):
    """Every discarded subtree of the 500x30 search carries a certificate the
    oracle replays; the replayed bounds certify the brute-force optimum."""
    announce(f"audited branch_and_bound squared 500x30, node order {order}")
    inst = W.plain_bnb_squared_500x30()
    P = oracle.Problem.from_instance(inst)
    ref = P.bnb()
    h = K.create_from_instance(inst, batch_width=64)
    out = K.branch_and_bound(h, node_order=order, audit=True)
    K.destroy_problem(h)
    assert out["status"] == 0
    assert list(out["support"]) == list(ref["support"])
    summary = audit_replay.replay(P, out)
    print(f"[gpu-test] audit: {summary}", flush=True)
    assert summary["min_replayed"] >= ref["objective"] * (1 - 1e-6) - 1e-9 * abs(ref["objective"])


def test_audit_rashomon_logistic_80x9():
    """Rashomon mode: pruned leaves replay above the final threshold, and
    the support leaves carry the re-optimisation kernel's dual certificate."""
    announce("audited Rashomon collection logistic 80x9, eps 0.15")
    inst = W.small_instance(80, 9, 3, W.LOGISTIC, seed=50, rho=0.5)
    P = oracle.Problem.from_instance(inst)
    h = K.create_from_instance(inst, batch_width=64)
    out = K.branch_and_bound(h, rashomon_eps=0.15, audit=True)
    K.destroy_problem(h)
    assert out["status"] == 0
    summary = audit_replay.replay(P, out, rashomon_eps=0.15)
    print(f"[gpu-test] audit: {summary}", flush=True)
    assert summary["kinds"][2] > 0


def test_audit_stopped_search():
    """A search stopped by its node limit while nodes are in flight:
    unexplored subtrees keep their parents' certified bounds, and the
    reported bound is below every replay."""
    announce("audited node-limited branch_and_bound logistic 1000x60")
    inst = W.small_instance(1000, 60, 6, W.LOGISTIC, seed=61, rho=0.9)
    P = oracle.Problem.from_instance(inst)
    h = K.create_from_instance(inst, batch_width=128, cert_period=8)
    out = K.branch_and_bound(h, max_nodes=25, audit=True)
    K.destroy_problem(h)
    assert out["status"] == 2
    summary = audit_replay.replay(P, out)
    print(f"[gpu-test] audit: status {out['status']} {summary}", flush=True)
    assert summary["kinds"][3] > 0
