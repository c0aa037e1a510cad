"""Autotuner: every candidate is measured on the same node sample, and the
choice follows the stated rule (smallest width whose best rate is within the
tie fraction of the overall best, at that width's fastest period)."""
import numpy as np
import pytest

import paper_2605_22188_amd as K
import workloads as W

pytestmark = pytest.mark.gpu


def test_autotune_choice_follows_the_rule():
    print("[gpu-test] autotune 2000x150 logistic, widths 16/64/256, periods 4/8", flush=True)
    inst = W.small_instance(2000, 150, 8, W.LOGISTIC, seed=51)
    widths, periods = [16, 64, 256], [4, 8]
    out = K.autotune(inst.X_store, inst.y, inst.k, inst.loss, inst.lambda2, inst.M,
                     dtype=inst.dtype, widths=widths, periods=periods, max_iters=400,
                     sample_nodes=256, tie_frac=0.03, seed=7)
    rates = out["rates"]
    assert rates.shape == (3, 2) and np.all(rates > 0)
    assert out["trials"] == 6 and out["sample_nodes"] == 256
    best = rates.max()
    ok_w = [w for w, row in zip(widths, rates) if row.max() >= 0.97 * best]
    assert out["batch_width"] == min(ok_w)
    row = rates[widths.index(out["batch_width"])]
    assert out["cert_period"] == periods[int(np.argmax(row))]
    assert out["rate"] == pytest.approx(row.max())


def test_autotune_with_given_nodes_and_budget():
    print("[gpu-test] autotune with caller nodes and a small budget", flush=True)
    inst = W.small_instance(1500, 100, 5, W.SQUARED, seed=52)
    nodes = W.random_nodes(100, 64, 2, 10, seed=53)
    out = K.autotune(inst.X_store, inst.y, inst.k, inst.loss, inst.lambda2, inst.M,
                     dtype=inst.dtype, nodes=nodes, widths=[32, 4096], periods=[8],
                     max_iters=300, hbm_budget_bytes=64 << 20)
    # the 4096-wide candidate cannot fit 64 MiB: skipped with rate 0
    assert out["rates"][1, 0] == 0.0 and out["rates"][0, 0] > 0
    assert out["batch_width"] == 32 and out["sample_nodes"] == 64


def test_iteration_precision_resolution():
    print("[gpu-test] iteration precision: auto resolution", flush=True)
    cases = [((300, 20, W.SQUARED, "f64"), 0, "f64"),
             ((300, 20, W.SQUARED, "f32"), 0, "anchored"),
             ((300, 20, W.SQUARED, "bf16"), 0, "anchored"),
             ((300, 20, W.SQUARED, "f32"), "f64", "f64"),
             ((300, 20, W.LOGISTIC, "f32"), 0, "f32"),
             ((300, 20, W.LOGISTIC, "bf16"), 0, "f32"),
             ((12000, 20, W.LOGISTIC, "f32"), 0, "anchored"),
             ((300, 20, W.LOGISTIC, "bf16"), "anchored", "anchored"),
             ((300, 20, W.SQUARED, "f32"), "f32", "f32")]
    for (n, p, loss, dt), it, want in cases:
        inst = W.small_instance(n, p, 4, loss, seed=3, dtype=dt)
        h = K.create_from_instance(inst, batch_width=8, iter_dtype=it)
        assert K.problem_info(h)["iteration"] == want, (n, p, loss, dt, it)
        K.destroy_problem(h)
    inst = W.small_instance(300, 20, 4, W.LOGISTIC, seed=3, dtype="f64")
    for it in ("f32", "anchored"):
        with pytest.raises(K.KbnbError) as e:
            K.create_from_instance(inst, iter_dtype=it)
        assert e.value.code == -1


def test_autotune_tile_height_split_depth_and_cache():
    """Second stage: tile height and split depth at the chosen width and
    period; a candidate replaces the launch-size rule only when it is faster by
    more than the tie margin.  The choice is cached per shape bucket and
    returned without measuring; refresh measures again."""
    print("[gpu-test] autotune tiles and split depth, cache", flush=True)
    inst = W.small_instance(2000, 150, 6, W.LOGISTIC, seed=60, dtype="f32")
    kw = dict(widths=[64, 256], periods=[8], max_iters=300, seed=3, tie_frac=0.03)
    out = K.autotune(inst.X_store, inst.y, inst.k, inst.loss, inst.lambda2, inst.M, dtype="f32",
                     tune_tiles=True, refresh=True, **kw)
    assert not out["cached"] and out["tile_trials"] > 0
    assert out["tile_rows"] in (0, 32, 64)
    cw = out["widths"].index(out["batch_width"])
    rule_rate = out["rates"][cw, 0]
    if out["tile_rows"] or out["split_rows"]:
        assert out["rate"] > rule_rate * 1.03
    else:
        assert out["rate"] == rule_rate
    again = K.autotune(inst.X_store, inst.y, inst.k, inst.loss, inst.lambda2, inst.M, dtype="f32",
                       tune_tiles=True, **kw)
    assert again["cached"] and again["seconds"] == 0.0
    for key in ("batch_width", "cert_period", "tile_rows", "split_rows"):
        assert again[key] == out[key]
    # the choice applied, and the explicit controls give valid bounds
    nodes = W.random_nodes(150, 30, 3, 15, seed=61)
    h0 = K.create_from_instance(inst, batch_width=64)
    ref = K.bound_nodes(h0, nodes, rel_tol=1e-6)
    K.destroy_problem(h0)
    for tr, sr in ((out["tile_rows"], out["split_rows"]), (64, 128), (32, 1024)):
        h = K.create_from_instance(inst, batch_width=64, tile_rows=tr, split_rows=sr)
        info = K.problem_info(h)
        if tr:
            assert info["tile_rows"] == tr
        if sr:
            assert info["split_rows"] >= sr
        res = K.bound_nodes(h, nodes, rel_tol=1e-6)
        for a, g in zip(ref, res):
            assert g["status"] == K.CONVERGED
            scale = max(abs(a["primal_value"]), abs(g["primal_value"]))
            assert abs(g["lower_bound"] - a["lower_bound"]) <= 1e-6 * scale
        K.destroy_problem(h)


def test_tile_rows_apply_to_their_kernel_only():
    print("[gpu-test] tile_rows validation", flush=True)
    f32 = W.small_instance(300, 20, 4, W.LOGISTIC, seed=3, dtype="f32")
    bf = W.small_instance(300, 20, 4, W.LOGISTIC, seed=3, dtype="bf16")
    for inst, bad in ((f32, 128), (bf, 32), (f32, 48)):
        with pytest.raises(K.KbnbError) as e:
            K.create_from_instance(inst, batch_width=8, tile_rows=bad)
        assert e.value.code == -1
    # the streaming kernel takes 64-, 128- and 256-row tiles; its rule picks
    # the tallest that still gives a launch 256 workgroups, here the shortest
    for tr, want in ((128, 128), (64, 64), (0, 64)):
        h = K.create_from_instance(bf, batch_width=8, tile_rows=tr)
        assert K.problem_info(h)["tile_rows"] == want
        res = K.bound_nodes(h, W.random_nodes(20, 8, 2, 5, seed=4), rel_tol=1e-6)
        assert all(r["status"] == K.CONVERGED for r in res)
        K.destroy_problem(h)


def test_split_count_is_a_multiple_of_eight():
    """Split s of a split-K launch runs on XCD s % 8, so the plain contractions
    round the split count to a multiple of 8.  At 12000 x 1000 float64 and
    width 1024 the launch-size rule asks for 3 splits (at most 4096 rows
    each), which would leave five XCDs idle; the count is 8.  600 nodes at
    full width give the same certified bounds as a problem forced to 3 splits
    (split depth 4096 rows)."""
    print("[gpu-test] split count 12000x1000 f64 at width 1024, 600 nodes, against 3 splits", flush=True)
    inst = W.small_instance(12000, 1000, 10, W.SQUARED, seed=21, dtype="f64")
    nodes = W.random_nodes(1000, 600, 3, 20, seed=22)
    out = []
    for sr, want in ((0, 8), (4096, 3)):
        h = K.create_from_instance(inst, batch_width=1024, cert_period=8, split_rows=sr)
        info = K.problem_info(h)
        assert info["gsplit"] == want, info
        out.append(K.bound_nodes(h, nodes, rel_tol=1e-6))
        K.destroy_problem(h)
    for a, g in zip(*out):
        assert a["status"] == K.CONVERGED and g["status"] == K.CONVERGED
        scale = max(abs(a["primal_value"]), abs(g["primal_value"]))
        assert abs(g["lower_bound"] - a["lower_bound"]) <= 2e-6 * scale
