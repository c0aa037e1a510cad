"""The compact support pool (host-only calls of the C-ABI library) against
the paper's worked example of its storage format, plus the structural
invariants of the trie on random pools (each checked against a plain
per-record list, which is what the trie must reproduce)."""
import json
import os

import numpy as np
import pytest

import paper_2605_22188_amd as K

HERE = os.path.dirname(os.path.abspath(__file__))


def _example():
    with open(os.path.join(HERE, "golden", "rashomon_trie_example.json")) as f:
        return json.load(f)


def _paths(ex):
    """Every record's labels, walking the exported parent links up from its end node."""
    out = []
    for v in ex["end_node"]:
        s = []
        while v > 0:
            s.append(int(ex["label"][v]))
            v = ex["parent"][v]
        out.append(tuple(reversed(s)))
    return out


def test_pool_paper_worked_example():
    g = _example()
    pool = K.Pool()
    for seq, coef in zip(g["insertion_sequences"], g["coefficients"]):
        pool.add(seq, coef, value=float(len(seq)))
    ex = pool.export()
    assert ex["offsets"].tolist() == g["offsets"]
    assert ex["coef"].tolist() == g["c"]
    # 11 labels in the four sequences, 3 of them shared: 8 nodes below the root
    assert pool.info() == (4, 9, 11)
    assert ex["parent"][0] == -1 and ex["label"][0] == -1
    paths = _paths(ex)
    assert paths == [tuple(s) for s in g["insertion_sequences"]]
    assert [sorted(s) for s in paths] == g["supports"]
    # shared prefix nodes: (18, 2) by the first two records, (18) by the first three
    def prefix_nodes(v):
        chain = []
        while v > 0:
            chain.append(v)
            v = ex["parent"][v]
        return chain[::-1]
    c1, c2, c3, c4 = (prefix_nodes(v) for v in ex["end_node"])
    assert c1[:2] == c2[:2] and c1[2] != c2[2]
    assert c1[0] == c3[0] and c1[1] != c3[1]
    assert c4[0] != c1[0]
    # the second record: entries 4..6 (1-based) of c, path (18, 2, 11)
    seq, coef, v = pool.record(1)
    lo, hi = g["second_record"]["c_entries_1based"]
    assert seq == tuple(g["second_record"]["path"])
    assert coef.tolist() == g["c"][lo - 1:hi]
    assert sorted(seq) == g["second_record"]["support"] and v == 3.0
    pool.close()


def test_pool_random_against_plain_list():
    rng = np.random.default_rng(7)
    pool = K.Pool()
    plain = []
    for m in range(300):
        L = int(rng.integers(0, 6))
        seq = rng.choice(12, size=L, replace=False).astype(np.int32)
        coef = rng.standard_normal(L)
        val = float(rng.standard_normal())
        pool.add(seq, coef, val)
        plain.append((tuple(int(j) for j in seq), coef, val))
    ex = pool.export()
    N, T, C = pool.info()
    assert N == 300 and C == sum(len(s) for s, _, _ in plain)
    # one trie node per distinct nonempty prefix, plus the root
    prefixes = {s[:r] for s, _, _ in plain for r in range(1, len(s) + 1)}
    assert T == len(prefixes) + 1
    assert _paths(ex) == [s for s, _, _ in plain]
    assert np.all(np.diff(ex["offsets"]) == [len(s) for s, _, _ in plain])
    for m, (s, c, v) in enumerate(plain):
        seq, coef, val = pool.record(m)
        assert seq == s and val == v
        np.testing.assert_array_equal(coef, c)
        np.testing.assert_array_equal(ex["coef"][ex["offsets"][m]:ex["offsets"][m + 1]], c)
    # children of one node carry distinct labels (prefixes are shared, never duplicated)
    kids = {}
    for v in range(1, T):
        key = (int(ex["parent"][v]), int(ex["label"][v]))
        assert key not in kids
        kids[key] = v
        assert 0 <= ex["parent"][v] < v
    pool.close()


def test_pool_errors():
    pool = K.Pool()
    with pytest.raises(K.KbnbError):
        pool.add([3, 5, 3], [1.0, 2.0, 3.0])
    with pytest.raises(K.KbnbError):
        pool.add([-1], [1.0])
    with pytest.raises(K.KbnbError):
        pool.record(0)
    pool.add([], None, 5.0)  # the empty support ends at the root
    assert pool.info() == (1, 1, 0) and pool.record(0) == ((), pytest.approx(np.zeros(0)), 5.0)
    pool.add([4, 1], None, 1.0)
    assert pool.record(1)[1].tolist() == [0.0, 0.0]
    pool.close()


def test_pool_summary_on_the_worked_example():
    """Summaries over the four records of the paper's storage example, worked
    by hand: feature 18 is in three records with coefficients 0.4, 0.5, 0.2
    and absent (0) from the fourth; feature 2 has -1.2 and -1.0 in two."""
    g = _example()
    pool = K.Pool()
    for seq, coef in zip(g["insertion_sequences"], g["coefficients"]):
        pool.add(seq, coef, value=1.0)
    rel = np.arange(1, 12, dtype=np.float64) / 10.0  # laid out like c
    s = K.pool_summary(pool, 20, rel)
    assert s["freq"][18] == 0.75 and s["freq"][2] == 0.5 and s["freq"][4] == 0.25
    assert s["freq"][0] == 0.0 and s["freq"].sum() == 11 / 4
    assert s["mean"][18] == pytest.approx(0.275) and s["abs_mean"][18] == pytest.approx(0.275)
    assert s["mean"][2] == pytest.approx(-0.55) and s["abs_mean"][2] == pytest.approx(0.55)
    assert s["pos_frac"][18] == 0.75 and s["pos_frac"][2] == 0.0 and s["pos_frac"][4] == 0.25
    assert (s["coef_min"][18], s["coef_max"][18]) == (0.0, 0.5)
    assert (s["coef_min"][2], s["coef_max"][2]) == (-1.2, 0.0)
    # reliance of 18: entries 1, 4, 7 of c (0.1, 0.4, 0.7), and 0 in record 4
    assert (s["reliance_min"][18], s["reliance_max"][18]) == (0.0, 0.7)
    assert s["reliance_mean"][18] == pytest.approx(0.3)
    # feature 12: only record 4 (entry 10 of c: 1.0)
    assert (s["reliance_min"][12], s["reliance_max"][12], s["reliance_mean"][12]) == (0.0, 1.0, 0.25)
    s0 = K.pool_summary(pool, 20)
    assert not s0["reliance_max"].any()
    with pytest.raises(K.KbnbError):
        K.pool_summary(pool, 18)  # feature 18 outside [0, 18)
    empty = K.Pool()
    assert not K.pool_summary(empty, 5)["freq"].any()
    pool.close()
    empty.close()
