"""The allocation-free certificate entry point against certify_batch.

certify_batch_noalloc runs the same float64 certificate kernels as
certify_batch, with its intermediate buffers in the library's fixed device
array instead of allocations, on device inputs and outputs.  Both must give
the same primal and dual values (relative 1e-11: the same kernels and split
counts, so in practice identical) and bit-identical rounding supports and
branching indices, over two calls in a row on one handle, the second with
fewer nodes (the array keeps the first call's contents)."""
import numpy as np
import pytest

import oracle
import paper_2605_22188_amd as K
import workloads as W

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _batch(P, inst, m, seed):
    r = np.random.Generator(np.random.PCG64(seed))
    p, k = inst.p, inst.k
    states = np.zeros((m, p), np.int8)
    betas = np.zeros((m, p))
    for b in range(m):
        perm = r.permutation(p)
        n1 = int(r.integers(0, k + 1))
        n0 = int(r.integers(0, p - n1 + 1))
        states[b, perm[:n1]] = 1
        states[b, perm[n1:n1 + n0]] = -1
        u = r.normal(size=p) * r.uniform(0.05, 1.0)
        betas[b] = P.prox(states[b], r.uniform(0.005, 0.2), u)
    return states, betas


def _noalloc(h, states, betas, stream=None):
    import torch
    m, p = states.shape
    dst = torch.from_numpy(states).cuda()
    dbe = torch.from_numpy(betas).cuda()
    phi = torch.full((m,), -1.0, dtype=torch.float64, device="cuda")
    psi = torch.full((m,), -1.0, dtype=torch.float64, device="cuda")
    sup = torch.full((m, h.k), -7, dtype=torch.int32, device="cuda")
    br = torch.full((m,), -7, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    K.certify_batch_noalloc(h, dst, dbe, phi, psi, sup, br, stream=stream)
    torch.cuda.synchronize()
    return phi.cpu().numpy(), psi.cpu().numpy(), sup.cpu().numpy(), br.cpu().numpy()


@pytest.mark.parametrize("name", ["squared_777x61_f32", "logistic_5000x200_f32"])
def test_noalloc_matches_certify_batch_twice(name):
    pytest.importorskip("torch")
    if name == "squared_777x61_f32":
        inst = W.small_instance(777, 61, 7, W.SQUARED, seed=3, dtype="f32")
    else:
        inst = W.node_bounds_logistic_5000x200()
    h = K.create_from_instance(inst, batch_width=64)
    P = oracle.Problem.from_instance(inst)
    for call, m in enumerate((150, 37)):
        announce(f"certify_batch_noalloc {name}: call {call + 1}, m={m}")
        states, betas = _batch(P, inst, m, 100 + call)
        phi, psi, sup, br = K.certify_batch(h, states, betas)
        phi2, psi2, sup2, br2 = _noalloc(h, states, betas)
        np.testing.assert_allclose(phi2, phi, rtol=1e-11, atol=0)
        np.testing.assert_allclose(psi2, psi, rtol=1e-11, atol=0)
        assert np.array_equal(sup2, sup)
        assert np.array_equal(br2, br)
    K.destroy_problem(h)


def test_noalloc_stream_invalid_nodes_and_limit():
    torch = pytest.importorskip("torch")
    announce("certify_batch_noalloc on a caller stream, invalid nodes, size limit")
    inst = W.small_instance(500, 40, 5, W.LOGISTIC, seed=8, dtype="f32")
    h = K.create_from_instance(inst, batch_width=64)
    P = oracle.Problem.from_instance(inst)
    states, betas = _batch(P, inst, 20, 7)
    states[3, :] = 1        # more than k fixed in
    states[5, 2] = 4        # not a state value
    phi, psi, sup, br = K.certify_batch(h, _valid(states), betas)
    s = torch.cuda.Stream()
    phi2, psi2, sup2, br2 = _noalloc(h, states, betas, stream=s)
    for b in range(20):
        if b in (3, 5):
            assert np.isnan(phi2[b]) and np.isnan(psi2[b]) and br2[b] == -1 and np.all(sup2[b] == -1)
        else:
            assert phi2[b] == pytest.approx(phi[b], rel=1e-11)
            assert psi2[b] == pytest.approx(psi[b], rel=1e-11)
            assert np.array_equal(sup2[b], sup[b]) and br2[b] == br[b]
    big = 100000  # 8 (n + ...) bytes per node: far beyond the array
    st = torch.zeros((big, inst.p), dtype=torch.int8, device="cuda")
    be = torch.zeros((big, inst.p), dtype=torch.float64, device="cuda")
    out = torch.zeros(big, dtype=torch.float64, device="cuda")
    with pytest.raises(K.KbnbError):
        K.certify_batch_noalloc(h, st, be, out, out)
    K.destroy_problem(h)


def _valid(states):
    """The nodes certify_batch accepts: invalid rows (3 and 5 above) replaced
    by the all-free node, whose results the comparison skips."""
    v = states.copy()
    v[3, :] = 0
    v[5, :] = 0
    return v
