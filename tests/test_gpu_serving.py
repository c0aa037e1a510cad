"""Serving behaviour: continuous batching over several concurrent problems.

Each node's result must not depend on what else is in flight: the same node
bounded alone, and in a mix with other nodes of its problem while another
problem runs on the device at the same time, gives the same bound within the
node tolerance.  The rounds of a problem are launched over the narrowest
column range that covers its occupied slots, with split-K counts chosen for
that width, so the float32 summation order of the gradient (and hence the
exact iterates) depends on the mix; the certified results do not: both
bounds lie in [v - tol |Phi|, v] for the node value v, so they differ by at
most tol |Phi|, and the rounding support and branching index agree.
"""
import threading

import numpy as np
import pytest

import paper_2605_22188_amd as K
import workloads as W

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[gpu-test] {msg}", flush=True)


def test_alone_vs_mix_and_concurrent_problems():
    announce("serving: alone vs mix, two concurrent problems")
    inst_a = W.small_instance(3000, 150, 8, W.LOGISTIC, seed=31)
    inst_b = W.small_instance(2500, 120, 6, W.SQUARED, seed=32)
    nodes_a = W.random_nodes(150, 200, 4, 40, seed=33)
    nodes_b = W.random_nodes(120, 150, 3, 30, seed=34)
    probe = [0, 7, 19, 55, 101, 199]

    # alone: each probe node on its own, nothing else in flight
    ha = K.create_from_instance(inst_a, batch_width=64, cert_period=8)
    alone = {i: K.bound_nodes(ha, [nodes_a[i]], rel_tol=1e-6)[0] for i in probe}

    # mix: all nodes of problem a (more than the 64 slots, so slots refill while
    # others iterate), while problem b runs on its own engine concurrently
    hb = K.create_from_instance(inst_b, batch_width=64, cert_period=8)
    out_b = {}

    def run_b():
        out_b["res"] = K.bound_nodes(hb, nodes_b, rel_tol=1e-6)

    t = threading.Thread(target=run_b)
    t.start()
    mix = K.bound_nodes(ha, nodes_a, rel_tol=1e-6)
    t.join()
    assert len(out_b["res"]) == len(nodes_b)
    assert all(r["status"] == K.CONVERGED for r in out_b["res"])
    for i in probe:
        a, m = alone[i], mix[i]
        assert m["status"] == a["status"] == K.CONVERGED
        scale = max(abs(a["primal_value"]), abs(m["primal_value"]))
        assert abs(m["lower_bound"] - a["lower_bound"]) <= 1e-6 * scale, (i, a, m)
        # each primal value is above the other's certified bound
        assert m["primal_value"] >= a["lower_bound"] - 1e-12 * scale
        assert a["primal_value"] >= m["lower_bound"] - 1e-12 * scale
        assert np.array_equal(m["support"], a["support"])
        assert m["branch_index"] == a["branch_index"]
    K.destroy_problem(ha)
    K.destroy_problem(hb)


def test_budget_sizes_the_batch_and_rejects_what_cannot_fit():
    announce("serving: device-memory budget")
    inst = W.small_instance(2000, 100, 5, W.LOGISTIC, seed=35)
    small = K.create_from_instance(inst, hbm_budget_bytes=40 << 20)
    big = K.create_from_instance(inst, hbm_budget_bytes=2 << 30)
    wa, wb = K.problem_info(small)["batch_width"], K.problem_info(big)["batch_width"]
    assert 1 <= wa < wb
    assert K.problem_info(small)["device_bytes"] <= 40 << 20
    res = K.bound_nodes(small, W.random_nodes(100, 3 * wa, 2, 20, seed=36), rel_tol=1e-6)
    assert all(r["status"] == K.CONVERGED for r in res)
    with pytest.raises(K.KbnbError) as e:
        K.create_from_instance(inst, hbm_budget_bytes=1 << 20)
    assert e.value.code == -3
    K.destroy_problem(small)
    K.destroy_problem(big)


def test_mix_requests_match_the_oracle():
    """Requests of four concurrent problems (scaled-down serving-mix shapes,
    both losses) submitted at once from four threads: a sample of every
    problem's results against the oracle solved to a 1e-10 gap (validity
    LB <= Phi_oracle, accuracy LB >= Psi_oracle - 1e-6 |Psi_oracle|), and each
    result carries its split of latency into queueing and solving."""
    import oracle
    announce("serving: mix requests of 4 problems against the oracle")
    specs = [(1500, 120, 6, W.LOGISTIC, 0.3, 41), (3000, 200, 8, W.SQUARED, 0.6, 42),
             (2200, 90, 5, W.SQUARED, 0.9, 43), (1200, 150, 10, W.LOGISTIC, 0.6, 44)]
    insts = [W.small_instance(n, p, k, loss, seed=sd, rho=rho, dtype="f32")
             for n, p, k, loss, rho, sd in specs]
    handles = [K.create_from_instance(inst, batch_width=32, cert_period=8) for inst in insts]
    reqs = [W.random_nodes(inst.p, 80, inst.k // 2, int(0.3 * inst.p), seed=50 + i)
            for i, inst in enumerate(insts)]
    out = [None] * len(insts)

    def run(i):
        out[i] = K.bound_nodes(handles[i], reqs[i], rel_tol=1e-6)
    th = [threading.Thread(target=run, args=(i,)) for i in range(len(insts))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for i, inst in enumerate(insts):
        P = oracle.Problem.from_instance(inst)
        res = out[i]
        assert len(res) == len(reqs[i])
        # 80 requests on 32 slots: later ones waited for a slot
        assert max(r["queue_seconds"] for r in res) > 0
        assert all(r["solve_seconds"] > 0 and r["queue_seconds"] >= 0 for r in res)
        for j in (0, 13, 41, 79):
            st = W.node_state(inst.p, reqs[i][j])
            rf = P.node_bound(st, tol=1e-10, max_iter=100000)
            g = res[j]
            assert g["status"] == K.CONVERGED, (i, j, g["status"])
            assert g["lower_bound"] <= rf["phi"] * (1 + 1e-12) + 1e-12, (i, j)
            assert g["lower_bound"] >= rf["lb"] - 1e-6 * abs(rf["lb"]), (i, j, g["lower_bound"], rf["lb"])
    for h in handles:
        K.destroy_problem(h)


def test_process_wide_budget_admits_defers_and_refuses():
    """The device budget shared by all problems: an automatic width shrinks to
    what is left, a problem that cannot fit is refused at once without a wait
    and admitted when another problem releases its memory within its wait."""
    announce("serving: process-wide device budget")
    inst = W.small_instance(2000, 100, 5, W.LOGISTIC, seed=35, dtype="f32")
    used0 = K.device_budget(-1)  # problems still alive in this process
    try:
        a = K.create_from_instance(inst, batch_width=256)
        need_a = K.problem_info(a)["device_bytes"]
        assert K.device_budget(-1) == used0 + need_a
        # room for A and half as much again: B's automatic width shrinks to fit
        K.device_budget(used0 + int(need_a * 1.5))
        b = K.create_from_instance(inst, hbm_budget_bytes=1 << 30)
        wb = K.problem_info(b)["batch_width"]
        assert 1 <= wb < 256
        assert K.device_budget(-1) <= used0 + int(need_a * 1.5)
        # a fixed width that cannot fit now: refused at once
        with pytest.raises(K.KbnbError) as e:
            K.create_from_instance(inst, batch_width=256)
        assert e.value.code == -3
        # ... and admitted after A is destroyed while it waits
        got = {}

        def late():
            got["h"] = K.create_from_instance(inst, batch_width=256, admit_timeout_ms=20000)
        t = threading.Thread(target=late)
        t.start()
        t.join(0.3)
        assert t.is_alive()  # waiting for memory
        K.destroy_problem(a)
        t.join(30)
        assert not t.is_alive() and "h" in got
        c = got["h"]
        assert K.problem_info(c)["batch_width"] == 256
        res = K.bound_nodes(c, W.random_nodes(100, 40, 2, 20, seed=37), rel_tol=1e-6)
        assert all(r["status"] == K.CONVERGED for r in res)
        K.destroy_problem(b)
        K.destroy_problem(c)
        assert K.device_budget(-1) == used0
    finally:
        K.device_budget(0)


def test_shared_stream_pool():
    """Problems sharing two streams give the same certified results as ones
    with their own streams."""
    announce("serving: shared stream pool")
    inst = W.small_instance(1800, 90, 5, W.LOGISTIC, seed=38, dtype="f32")
    nodes = W.random_nodes(90, 40, 2, 20, seed=39)
    own = K.create_from_instance(inst, batch_width=32)
    ref = K.bound_nodes(own, nodes, rel_tol=1e-6)
    K.destroy_problem(own)
    try:
        K.engine_streams(2)
        hs = [K.create_from_instance(inst, batch_width=32) for _ in range(3)]
        out = [None] * 3

        def run(i):
            out[i] = K.bound_nodes(hs[i], nodes, rel_tol=1e-6)
        th = [threading.Thread(target=run, args=(i,)) for i in range(3)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        for res in out:
            for a, g in zip(ref, res):
                assert g["status"] == K.CONVERGED
                scale = max(abs(a["primal_value"]), abs(g["primal_value"]))
                assert abs(g["lower_bound"] - a["lower_bound"]) <= 1e-6 * scale
        for h in hs:
            K.destroy_problem(h)
    finally:
        K.engine_streams(0)
