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
