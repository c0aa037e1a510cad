"""Independent audit of a finished branch and bound (helper of the GPU tests).

branch_and_bound(audit=True) returns every discarded subtree (leaf) with the
bound the search used for it and that bound's certificate: a node containing
the leaf and the iterate whose dual point gave the bound.  The oracle
recomputes each certificate in float64 from the exact instance (dual point
zeta = -l'(X beta), dual value Psi of the certifying node; Sec. 3, "Safe Lower
Bound and Pruning"), so a pruning decision or the reported global bound is
checked without trusting any device arithmetic: weak duality makes every
replayed Psi a lower bound of its node, hence of the leaf it contains.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np


def _contains(cert_state, leaf_state):
    """The certifying node contains the leaf: its fixed-in and fixed-out sets
    are subsets of the leaf's."""
    return (np.all(leaf_state[cert_state == 1] == 1) and np.all(leaf_state[cert_state == -1] == -1))


def replay(P, out, threads=16, rashomon_eps=None):
    """Checks, for the search result `out` (with "leaves"):
      * every leaf with a finite bound has a certificate whose node contains it;
      * the oracle's Psi at the certificate equals the device's to 1e-10 and is
        at least the leaf's bound (up to that rounding);
      * pruned leaves: Psi_oracle >= UB - 1e-6 |UB| (optimal-support mode), or
        Psi_oracle > tau_final = (1 + eps) UB (Rashomon mode, uncapped);
      * the reported global bound is at most every replayed Psi and at most
        the objective.
    Returns a summary dict."""
    leaves = out["leaves"]
    UB = out["objective"]
    assert len(leaves) > 0

    def psi(lf):
        if not np.isfinite(lf["bound"]):
            return -np.inf
        return P.dual(lf["cert_state"], P.dual_point(lf["cert_beta"]))

    with ThreadPoolExecutor(threads) as ex:
        psis = list(ex.map(psi, leaves))
    worst_dev = 0.0
    kinds = [0, 0, 0, 0]
    for lf, ps in zip(leaves, psis):
        kinds[lf["kind"]] += 1
        b = lf["bound"]
        if not np.isfinite(b):
            assert lf["kind"] == 3, lf["kind"]  # only an unexplored root can lack a bound
            continue
        assert _contains(lf["cert_state"], lf["state"]), lf["kind"]
        scale = max(abs(ps), 1e-12)
        dev = abs(ps - lf["cert_bound"]) / scale
        worst_dev = max(worst_dev, dev)
        assert dev <= 1e-10, (lf["kind"], ps, lf["cert_bound"])
        assert b <= ps + 1e-10 * scale, (lf["kind"], b, ps)
        if lf["kind"] == 0:
            if rashomon_eps is None:
                assert ps >= UB - 1e-6 * abs(UB) - 1e-10 * abs(UB), (ps, UB)
            else:
                tau = (1.0 + rashomon_eps) * UB
                assert ps > tau - 1e-10 * abs(tau), (ps, tau)
        assert out["lower_bound"] <= ps + 1e-10 * scale, (out["lower_bound"], ps)
    assert out["lower_bound"] <= UB
    return dict(leaves=len(leaves), kinds=kinds, worst_rel_dev=worst_dev,
                min_replayed=float(min(psis)))
