"""GPU parity: the HIP path (through the C ABI) against the oracle.

Every test prints its case before the first GPU call, so a failing GPU run
names it.  Tolerances:
  * prox, primal and dual values at the same input: both sides compute the
    same float64 formulas in different orders; relative 1e-11 (values are
    sums of up to n terms of magnitude ~1, so rounding stays near 1e-13);
  * node bounds: validity LB_gpu <= Phi_oracle (the oracle's primal value is
    an upper bound on the node optimum, at 1e-12 relative slack for
    rounding) and accuracy LB_gpu >= Psi_oracle - 1e-6 |Psi_oracle|, where
    the oracle is run to a 1e-10 relative gap;
  * rounding supports and branching indices at the same beta: bit-exact.
"""
import math

import numpy as np
import pytest

import oracle
import paper_2605_22188_amd as K
import workloads as W

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[gpu-test] {msg}", flush=True)


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def edge_states(r, p, k, m):
    """Random node states plus the degenerate budgets: kbar 0, 1, #free-1,
    #free, > #free, and no free coordinate at all."""
    states = []
    for b in range(m):
        st = np.zeros(p, np.int8)
        perm = r.permutation(p)
        kind = b % 8
        if kind == 0:      # kbar = 0
            n1, n0 = k, int(r.integers(0, p - k + 1))
        elif kind == 1:    # kbar = 1
            n1, n0 = k - 1, int(r.integers(0, p - k + 1))
        elif kind == 2:    # #free = kbar + 1
            n1 = int(r.integers(0, k))
            n0 = p - n1 - (k - n1) - 1
        elif kind == 3:    # #free = kbar
            n1 = int(r.integers(0, k))
            n0 = p - n1 - (k - n1)
        elif kind == 4:    # #free < kbar
            n1 = 0
            n0 = p - max(1, k // 2)
        elif kind == 5:    # nothing free
            n1 = min(k, p)
            n0 = p - n1
        else:
            n1 = int(r.integers(0, k + 1))
            n0 = int(r.integers(0, p - n1 + 1))
        n0 = max(0, min(n0, p - n1))
        st[perm[:n1]] = 1
        st[perm[n1:n1 + n0]] = -1
        states.append(st)
    return np.array(states)


@pytest.mark.parametrize("p,k", [(30, 5), (200, 10), (257, 12), (1000, 10), (2048, 40),
                                 (3000, 20), (5000, 15), (8192, 64)])
def test_prox_batch_matches_oracle(p, k):
    announce(f"prox_batch p={p} k={k}")
    r = rng(100 + p)
    inst = W.small_instance(64, p, k, W.SQUARED, seed=p, M=1.5, lambda2=0.8)
    h = K.create_from_instance(inst, batch_width=64)
    P = oracle.Problem.from_instance(inst)
    m = 48
    states = edge_states(r, p, k, m)
    u = r.normal(size=(m, p)) * r.uniform(0.2, 3.0, size=(m, 1))
    u[::3] = np.round(u[::3], 1)  # many exact ties
    for eta in (0.05, 0.7, 4e-4):
        got = K.prox_batch(h, states, u, eta)
        for b in range(m):
            ref = P.prox(states[b], eta, u[b])
            scale = max(1.0, np.max(np.abs(u[b])))
            err = np.max(np.abs(got[b] - ref))
            assert err <= 1e-12 * scale, (b, eta, err)
            # exact zeros agree, except for an entry on the pooled block's edge
            # whose value is zero up to rounding on the other side
            differ = (got[b] == 0.0) != (ref == 0.0)
            assert np.all(np.abs(got[b][differ]) + np.abs(ref[differ]) <= 1e-12 * scale), (b, eta)
    K.destroy_problem(h)


def _certify_case(inst, m, seed):
    r = rng(seed)
    h = K.create_from_instance(inst, batch_width=64)
    P = oracle.Problem.from_instance(inst)
    p, k = inst.p, inst.k
    states = edge_states(r, p, k, m)
    betas = np.empty((m, p))
    for b in range(m):
        u = r.normal(size=p) * r.uniform(0.05, 1.0)
        betas[b] = P.prox(states[b], r.uniform(0.05, 2.0) / 10, u)
    betas[::4] = np.round(betas[::4], 2)   # ties in |beta|
    for b in range(0, m, 4):               # keep them in dom g
        betas[b] = P.prox(states[b], 1e-9, betas[b])
    phi, psi, sup, br = K.certify_batch(h, states, betas)
    for b in range(m):
        phi_o = P.primal(states[b], betas[b])
        psi_o = P.dual(states[b], P.dual_point(betas[b]))
        assert phi[b] == pytest.approx(phi_o, rel=1e-11), b
        assert psi[b] == pytest.approx(psi_o, rel=1e-11), b
        s_o, br_o = P.round_branch(states[b], betas[b])
        assert list(sup[b][:len(s_o)]) == list(s_o), b
        assert np.all(sup[b][len(s_o):] == -1), b
        assert br[b] == br_o, b
    K.destroy_problem(h)


def test_certify_batch_logistic_5000x200():
    announce("certify_batch logistic 5000x200 f32")
    _certify_case(W.node_bounds_logistic_5000x200(), 64, 7)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_certify_batch_ragged_dtypes(dtype):
    announce(f"certify_batch squared 777x61 {dtype}")
    inst = W.small_instance(777, 61, 7, W.SQUARED, seed=3, dtype=dtype)
    _certify_case(inst, 40, 11)


@pytest.mark.parametrize("n,p,k,loss", [(700, 3000, 20, W.LOGISTIC), (600, 5000, 15, W.SQUARED)])
def test_certify_batch_wide_nodes(n, p, k, loss):
    """p above 2048: one multi-wave workgroup per node."""
    announce(f"certify_batch {n}x{p} k={k} loss={loss}")
    _certify_case(W.small_instance(n, p, k, loss, seed=p, lambda2=1.0), 24, 13)


def _threshold_betas(r, states, k, M):
    """Iterates whose free magnitudes put Thm. 4.1's threshold tau exactly on
    an entry (several s satisfy the threshold condition), or many equal
    entries, or a large head with a tail thousands of times smaller (where a
    tail formed as total minus head would lose its digits)."""
    m, p = states.shape
    betas = np.zeros((m, p))
    for b in range(m):
        st = states[b]
        fin = np.flatnonzero(st == 1)
        free = r.permutation(np.flatnonzero(st == 0))
        kbar = k - len(fin)
        betas[b, fin] = r.uniform(-M, M, size=len(fin))
        kind = b % 3
        if kbar < 2 or len(free) < 3:
            continue
        if kind == 2:   # q > kbar equal entries: tau = q c / kbar
            q = min(len(free), kbar + 1 + int(r.integers(0, kbar + 1)))
            c = M * kbar / q * r.uniform(0.3, 1.0)
            a = np.full(q, c)
        else:
            s0 = int(r.integers(0, kbar - 1))          # kbar - s0 >= 2
            q = min(3 * (kbar - s0), len(free) - s0 - 1)
            head = np.sort(M * r.uniform(0.6, 1.0, size=s0))[::-1]
            x = (0.3 if kind == 0 else 1e-3) * (head[-1] if s0 else M)
            # tail sum (kbar - s0) x: tau = x exactly, a tie between s0 and s0 + 1
            y = np.full(q, (kbar - s0 - 1) * x / q)
            a = np.concatenate([head, [x], y])
        sg = r.choice([-1.0, 1.0], size=len(a))
        betas[b, free[:len(a)]] = sg * a
    return betas


def test_certify_batch_threshold_ties():
    """The primal value where the threshold of Thm. 4.1 ties with an entry,
    where many entries are equal, and where the tail is tiny next to the
    head: Phi against the oracle, which solves the budget equation by
    bisection.  A large lambda2 makes 2 lambda2 g(beta) dominate Phi."""
    announce("certify_batch threshold ties squared 300x64")
    inst = W.small_instance(300, 64, 12, W.SQUARED, seed=21, lambda2=1e3, M=2.0)
    h = K.create_from_instance(inst, batch_width=64)
    P = oracle.Problem.from_instance(inst)
    r = rng(22)
    m = 60
    states = np.zeros((m, 64), np.int8)
    for b in range(m):
        perm = r.permutation(64)
        n1, n0 = int(r.integers(0, 4)), int(r.integers(0, 11))
        states[b, perm[:n1]] = 1
        states[b, perm[n1:n1 + n0]] = -1
    betas = _threshold_betas(r, states, 12, 2.0)
    phi, psi, sup, br = K.certify_batch(h, states, betas)
    for b in range(m):
        g_o = P.g(states[b], betas[b])
        assert np.isfinite(g_o), b
        phi_o = P.primal(states[b], betas[b])
        assert phi[b] == pytest.approx(phi_o, rel=1e-11), (b, phi[b], phi_o)
        assert psi[b] == pytest.approx(P.dual(states[b], P.dual_point(betas[b])), rel=1e-11), b
        s_o, br_o = P.round_branch(states[b], betas[b])
        assert list(sup[b][:len(s_o)]) == list(s_o), b
        assert br[b] == br_o, b
    K.destroy_problem(h)


def _bound_parity(inst, nodes, batch_width, cert_period, warm=None, sample=None, iter_dtype=0):
    h = K.create_from_instance(inst, batch_width=batch_width, cert_period=cert_period,
                               iter_dtype=iter_dtype)
    P = oracle.Problem.from_instance(inst)
    res = K.bound_nodes(h, nodes, rel_tol=1e-6, warm_starts=warm)
    idx = range(len(nodes)) if sample is None else sample
    for i in idx:
        st = W.node_state(inst.p, nodes[i])
        ref = P.node_bound(st, tol=1e-10, max_iter=100000)
        g = res[i]
        assert g["status"] == K.CONVERGED, (i, g)
        assert g["rel_gap"] <= 1e-6
        assert g["lower_bound"] <= ref["phi"] + 1e-12 * abs(ref["phi"]), (i, g["lower_bound"], ref)
        assert g["lower_bound"] >= ref["lb"] - 1e-6 * abs(ref["lb"]), (i, g["lower_bound"], ref)
        # the returned rounding support is the top-kbar of the returned beta
        s_o, br_o = P.round_branch(st, g["beta"])
        assert list(g["support"]) == list(s_o)
        assert g["branch_index"] == br_o
    K.destroy_problem(h)
    return res


@pytest.mark.parametrize("loss,dtype,it", [(W.SQUARED, "f64", 0), (W.LOGISTIC, "f64", 0),
                                            (W.SQUARED, "f32", 0), (W.LOGISTIC, "f32", 0),
                                            (W.SQUARED, "bf16", 0), (W.LOGISTIC, "bf16", 0),
                                            (W.LOGISTIC, "f32", "f64"),
                                            (W.SQUARED, "f32", "f64"),
                                            (W.SQUARED, "bf16", "f64"),
                                            (W.SQUARED, "f32", "anchored"),
                                            (W.LOGISTIC, "f32", "anchored"),
                                            (W.SQUARED, "bf16", "anchored"),
                                            (W.LOGISTIC, "bf16", "anchored")])
def test_node_bounds_small_all_nodes(loss, dtype, it):
    """Iteration precision "auto" (0): float64 for float64 X; anchored for the
    squared loss on float32 / bfloat16 X; float32 for the logistic loss on
    float32 / bfloat16 X (bfloat16 X: the products stream a tiled copy of X
    on bfloat16 MFMA against three bfloat16 planes of the float32 operand).
    "f64": float64 iteration forced on float32 / bfloat16 X.  "anchored":
    float32 / bfloat16 products of the change since each node's last float64
    certificate (two planes on bfloat16 X)."""
    announce(f"node bounds 700x50 loss={loss} X {dtype} iteration {it}, 100 nodes on 64 slots")
    inst = W.small_instance(700, 50, 6, loss, seed=5 + loss, rho=0.6, dtype=dtype)
    nodes = W.random_nodes(50, 100, 3, 15, seed=77)
    _bound_parity(inst, nodes, batch_width=64, cert_period=4, iter_dtype=it)


@pytest.mark.parametrize("loss", [W.SQUARED, W.LOGISTIC])
def test_node_bounds_bf16_anchored_three_column_tiles(loss):
    """Two-plane streaming products over three 64-column tiles (150 nodes on
    192 slots): the split-K X^T R runs with one A register set and the column
    tiles of a row block side by side; every node against the oracle."""
    announce(f"node bounds 700x50 loss={loss} X bf16 anchored, 150 nodes on 192 slots")
    inst = W.small_instance(700, 50, 6, loss, seed=11 + loss, rho=0.6, dtype="bf16")
    nodes = W.random_nodes(50, 150, 3, 15, seed=78)
    _bound_parity(inst, nodes, batch_width=192, cert_period=4, iter_dtype="anchored")


def test_node_bounds_logistic_5000x200_launch():
    announce("node bounds logistic 5000x200, one 256-node launch, 16 sampled")
    inst = W.node_bounds_logistic_5000x200()
    nodes = W.launch_nodes_5000x200(0)
    sample = list(range(0, 256, 16))
    res = _bound_parity(inst, nodes, batch_width=256, cert_period=8, sample=sample)
    assert all(r["status"] == K.CONVERGED for r in res)


def test_node_bounds_logistic_5000x200_bench_settings():
    """The benchmark's launch exactly as timed: 256 nodes of launch 0, batch
    width 256, certificate every 16 steps, float32 iteration; 64 of the 256
    nodes (every fourth) against the oracle solved to a 1e-10 gap."""
    from concurrent.futures import ThreadPoolExecutor
    announce("node bounds logistic 5000x200 at the benchmark settings, 64 of 256 sampled")
    inst = W.node_bounds_logistic_5000x200()
    nodes = W.launch_nodes_5000x200(0)
    h = K.create_from_instance(inst, batch_width=256, cert_period=16)
    res = K.bound_nodes(h, nodes, rel_tol=1e-6)
    K.destroy_problem(h)
    assert all(g["status"] == K.CONVERGED for g in res)
    P = oracle.Problem.from_instance(inst)
    sample = list(range(0, 256, 4))

    def ref(i):
        return P.node_bound(W.node_state(inst.p, nodes[i]), tol=1e-10, max_iter=100000)
    with ThreadPoolExecutor(16) as ex:
        refs = list(ex.map(ref, sample))
    worst = 0.0
    for i, rf in zip(sample, refs):
        g = res[i]
        assert g["lower_bound"] <= rf["phi"] + 1e-12 * abs(rf["phi"]), (i, g["lower_bound"], rf)
        assert g["lower_bound"] >= rf["lb"] - 1e-6 * abs(rf["lb"]), (i, g["lower_bound"], rf)
        worst = max(worst, abs(g["lower_bound"] - rf["lb"]) / abs(rf["lb"]))
        s_o, br_o = P.round_branch(W.node_state(inst.p, nodes[i]), g["beta"])
        assert list(g["support"]) == list(s_o) and g["branch_index"] == br_o, i
    print(f"[gpu-test] worst |LB_gpu - LB_oracle| / |LB_oracle| = {worst:.3e}", flush=True)


def test_node_bounds_float64_instance():
    announce("node bounds squared 500x30 f64")
    inst = W.plain_bnb_squared_500x30()
    nodes = W.random_nodes(30, 40, 4, 10, seed=9)
    _bound_parity(inst, nodes, batch_width=64, cert_period=8)


def test_batch_width_one():
    announce("node bounds batch width 1")
    inst = W.small_instance(300, 20, 4, W.LOGISTIC, seed=2)
    nodes = W.random_nodes(20, 5, 2, 5, seed=3)
    _bound_parity(inst, nodes, batch_width=1, cert_period=8)


def test_warm_start_and_prune_decisions():
    announce("prune decisions logistic 2000x80")
    inst = W.small_instance(2000, 80, 8, W.LOGISTIC, seed=12)
    P = oracle.Problem.from_instance(inst)
    nodes = W.random_nodes(80, 60, 4, 20, seed=13)
    refs = [P.node_bound(W.node_state(80, nd), tol=1e-10) for nd in nodes]
    r = rng(14)
    ubs = np.array([ref["phi"] * (1 + r.choice([-0.02, 0.02])) for ref in refs])
    h = K.create_from_instance(inst, batch_width=64, cert_period=4)
    warm = [ref["beta"] if i % 2 else None for i, ref in enumerate(refs)]
    res = K.bound_nodes(h, nodes, upper_bound=ubs, rel_tol=1e-6, warm_starts=warm)
    band = 0
    for ref, ub, g in zip(refs, ubs, res):
        v = ref["lb"]
        thr = ub - 1e-6 * abs(ub)
        if abs(v - thr) <= 2e-6 * abs(ub):
            band += 1
            continue
        assert (g["status"] == K.PRUNED) == (v >= thr), (v, ub, g)
        assert g["lower_bound"] <= ref["phi"] * (1 + 1e-12)
    assert band == 0
    K.destroy_problem(h)


def test_stop_unprunable_decisions():
    """With stop_unprunable, a node whose value lies 2% below its upper bound
    stops as UNPRUNABLE (its certified primal value is below the pruning
    threshold, so its value is too, and its bound is still valid); 2% above,
    it is PRUNED as before; with no upper bound it converges."""
    announce("stop_unprunable decisions logistic 2000x80")
    inst = W.small_instance(2000, 80, 8, W.LOGISTIC, seed=12)
    P = oracle.Problem.from_instance(inst)
    nodes = W.random_nodes(80, 40, 4, 20, seed=15)
    refs = [P.node_bound(W.node_state(80, nd), tol=1e-10) for nd in nodes]
    r = rng(16)
    side = r.choice([-1, 1], size=len(nodes))
    ubs = np.array([ref["phi"] * (1 + 0.02 * s_) for ref, s_ in zip(refs, side)])
    h = K.create_from_instance(inst, batch_width=64, cert_period=4)
    res = K.bound_nodes(h, nodes, upper_bound=ubs, rel_tol=1e-6, stop_unprunable=1)
    for ref, ub, s_, g in zip(refs, ubs, side, res):
        assert g["lower_bound"] <= ref["phi"] * (1 + 1e-12)
        if s_ > 0:  # value well below the threshold
            assert g["status"] == K.UNPRUNABLE, g
            assert g["primal_value"] < ub - 1e-6 * abs(ub)
            assert g["primal_value"] >= ref["lb"] * (1 - 1e-12)
        else:
            assert g["status"] == K.PRUNED, g
    res = K.bound_nodes(h, nodes[:8], rel_tol=1e-6, stop_unprunable=1)
    assert all(g["status"] == K.CONVERGED for g in res)
    K.destroy_problem(h)


def test_invalid_nodes_are_rejected_atomically():
    announce("invalid submissions")
    inst = W.small_instance(100, 10, 3, W.SQUARED, seed=1)
    h = K.create_from_instance(inst, batch_width=8)
    good = ([0], [1, 2])
    for bad in [([10], []), ([0, 0], []), ([0], [0]), ([0, 1, 2, 3], []), ([-1], [])]:
        with pytest.raises(K.KbnbError):
            K.submit_nodes(h, [good, bad])
    K.submit_nodes(h, [])
    res, rc = K.poll_bounds(h, cap=4, timeout_us=0)
    assert res == [] and rc == K.TIMEOUT
    out = K.bound_nodes(h, [good])
    assert out[0]["status"] == K.CONVERGED
    K.destroy_problem(h)


@pytest.mark.parametrize("order", [0, 1])
def test_bnb_plain_squared_500x30_on_gpu(order):
    announce(f"branch_and_bound squared 500x30 f64, node order {order}")
    inst = W.plain_bnb_squared_500x30()
    P = oracle.Problem.from_instance(inst)
    ref = P.bnb()
    h = K.create_from_instance(inst, batch_width=64)
    out = K.branch_and_bound(h, node_order=order)
    assert out["status"] == 0
    assert list(out["support"]) == list(ref["support"])
    assert out["objective"] == pytest.approx(ref["objective"], rel=1e-6)
    assert out["lower_bound"] <= ref["objective"] * (1 + 1e-9)
    assert out["rel_gap"] <= 1e-6
    with pytest.raises(K.KbnbError):
        K.branch_and_bound(h, node_order=2)
    K.destroy_problem(h)


def test_bnb_depth_first_logistic_and_rashomon():
    announce("branch_and_bound depth first: logistic 80x9 and its Rashomon set")
    inst = W.small_instance(80, 9, 3, W.LOGISTIC, seed=50, rho=0.5)
    P = oracle.Problem.from_instance(inst)
    ref = P.rashomon(0.15, node_tol=1e-9)
    h = K.create_from_instance(inst, batch_width=64)
    best = K.branch_and_bound(h)
    dfs = K.branch_and_bound(h, node_order=1)
    assert dfs["status"] == 0 and dfs["rel_gap"] <= 1e-6
    assert list(dfs["support"]) == list(best["support"])
    assert dfs["objective"] == pytest.approx(ref["optimum"], rel=1e-6)
    rs = K.branch_and_bound(h, node_order=1, rashomon_eps=0.15)
    K.destroy_problem(h)
    band = 2e-6 * abs(ref["threshold"])
    got = {S for S, _, _ in rs["rashomon"]}
    for S, v in ref["set"]:
        if v < ref["threshold"] - band:
            assert S in got, S


@pytest.mark.parametrize("n,p,k,loss,dtype,it", [(1500, 3000, 10, W.LOGISTIC, "bf16", 0),
                                                  (2500, 5000, 15, W.SQUARED, "bf16", 0),
                                                  (2500, 5000, 15, W.SQUARED, "bf16", "anchored"),
                                                  (3000, 4000, 12, W.LOGISTIC, "f32", "anchored")])
def test_node_bounds_wide_nodes(n, p, k, loss, dtype, it):
    """Node bounds at p above 2048, checked by the duality bracket the oracle
    evaluates at the returned iterate: the certified bound LB must satisfy
    LB <= Phi_oracle(beta) (validity, up to 1e-12 rounding) and
    Phi_oracle(beta) - LB <= 1e-6 |Phi_oracle(beta)| (so LB is within the
    tolerance of the node value, which lies in between).  The oracle's own
    solve to 1e-10 is too slow at these sizes; its certificate arithmetic at
    the same sizes is compared element by element in the certify_batch test."""
    announce(f"node bounds {n}x{p} k={k} loss={loss} X {dtype} iteration {it}")
    inst = W.small_instance(n, p, k, loss, seed=p + 1, lambda2=1.0, dtype=dtype)
    P = oracle.Problem.from_instance(inst)
    nodes = W.random_nodes(p, 12, k // 2, p // 10, seed=p + 2)
    h = K.create_from_instance(inst, batch_width=8, cert_period=8, iter_dtype=it)
    res = K.bound_nodes(h, nodes, rel_tol=1e-6)
    for i, (nd, g) in enumerate(zip(nodes, res)):
        st = W.node_state(p, nd)
        assert g["status"] == K.CONVERGED, (i, g["status"], g["rel_gap"])
        phi_o = P.primal(st, g["beta"])
        assert g["lower_bound"] <= phi_o + 1e-12 * abs(phi_o), (i, g["lower_bound"], phi_o)
        assert phi_o - g["lower_bound"] <= (1e-6 + 1e-9) * abs(phi_o), (i, g["lower_bound"], phi_o)
        s_o, br_o = P.round_branch(st, g["beta"])
        assert list(g["support"]) == list(s_o)
        assert g["branch_index"] == br_o
    K.destroy_problem(h)


@pytest.mark.parametrize("n,p,rho,loss,dtype", [(700, 50, 0.5, W.SQUARED, "f64"),
                                                (3000, 400, 0.9, W.LOGISTIC, "bf16")])
def test_step_constant_is_the_largest_eigenvalue(n, p, rho, loss, dtype):
    """L = 1.02 c_l lambda_max(X^T X) (c_l = 2 squared, 1/4 logistic), with
    lambda_max from the device's Lanczos iteration on the stored X, against
    numpy's symmetric eigensolver in float64 (rho 0.9: a correlated design
    with a large, well separated top eigenvalue)."""
    announce(f"step constant {n}x{p} rho {rho} {dtype}")
    inst = W.small_instance(n, p, 5, loss, seed=90, rho=rho, dtype=dtype)
    h = K.create_from_instance(inst, batch_width=8)
    L = K.problem_info(h)["L"]
    K.destroy_problem(h)
    lam = np.linalg.eigvalsh(inst.X.T @ inst.X)[-1]
    c = 2.0 if loss == W.SQUARED else 0.25
    assert L == pytest.approx(1.02 * c * lam, rel=1e-9)


def test_sparse_warm_starts_match_dense():
    """A warm start given sparsely (indices and values) is the dense one
    with zeros elsewhere: the same nodes give bit-identical results either
    way, entries on J0 are ignored as in the dense form, and malformed
    sparse entries are rejected."""
    announce("sparse warm starts, logistic 1500x90")
    inst = W.small_instance(1500, 90, 6, W.LOGISTIC, seed=15, dtype="f32")
    nodes = W.random_nodes(90, 40, 3, 20, seed=16)
    r = rng(17)
    dense, sparse = [], []
    for nd in nodes:
        w = np.zeros(90)
        idx = np.sort(r.choice(90, size=12, replace=False)).astype(np.int32)
        w[idx] = r.normal(0, 0.5, size=12)
        dense.append(w)
        sparse.append((idx, w[idx]))  # some indices fall on J0: ignored by both
    h = K.create_from_instance(inst, batch_width=64, cert_period=8)
    a = K.bound_nodes(h, nodes, rel_tol=1e-6, warm_starts=dense)
    b = K.bound_nodes(h, nodes, rel_tol=1e-6, warm_starts=sparse)
    for x, y in zip(a, b):
        assert x["status"] == y["status"] == K.CONVERGED
        assert x["lower_bound"] == y["lower_bound"] and x["primal_value"] == y["primal_value"]
        assert x["iterations"] == y["iterations"] and np.array_equal(x["beta"], y["beta"])
    for bad in ((np.array([3, 90], np.int32), np.array([0.1, 0.2])),
                (np.array([3, -1], np.int32), np.array([0.1, 0.2])),
                (np.array([3, 4], np.int32), np.array([0.1, np.nan]))):
        with pytest.raises(K.KbnbError):
            K.bound_nodes(h, nodes[:1], rel_tol=1e-6, warm_starts=[bad])
    K.destroy_problem(h)


def test_bnb_support_paths_and_reopt_controls():
    """The three ways of re-optimising rounding supports (automatic, the
    re-optimisation kernel, the node engine; rows split over forced
    workgroups too) reach the oracle's optimum of the 500x30 search; invalid
    values of the controls are rejected."""
    announce("branch_and_bound 500x30 over support paths and reopt_groups")
    inst = W.plain_bnb_squared_500x30()
    P = oracle.Problem.from_instance(inst)
    ref = P.bnb()
    for groups in (0, 1, 3):
        h = K.create_from_instance(inst, batch_width=64, reopt_groups=groups)
        for path in (0, 1, 2):
            out = K.branch_and_bound(h, support_path=path)
            assert out["status"] == 0 and out["rel_gap"] <= 1e-6, (groups, path)
            assert list(out["support"]) == list(ref["support"]), (groups, path)
            assert out["objective"] == pytest.approx(ref["objective"], rel=1e-6)
            assert out["lower_bound"] <= ref["objective"] * (1 + 1e-9)
        if groups == 0:
            with pytest.raises(K.KbnbError):
                K.branch_and_bound(h, support_path=3)
        K.destroy_problem(h)
    for bad in (-1, 1025):
        with pytest.raises(K.KbnbError):
            K.create_from_instance(inst, batch_width=64, reopt_groups=bad)
