"""Labels of the learned impedance model regenerated with the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: the library never imports this module.  It restates
the labelling rule of the learned impedances (an addition to the paper's
impedance matching of Section 7.1: the multiplier over the diagonal rule
Z = 1/a_vv that the method's own probe sweeps favour) and runs it with the
oracle's Jacobi VTM of (5.6)-(5.8), so that the GPU labeller can be checked
against it:

  1. global probe: for alpha in {2^(j/2): j = 0..16}, K sweeps from zero waves
     with Z = alpha / a_vv; alpha* = the alpha with the lowest relative residual
     of the merged potentials after K sweeps (Table 1 step 6's test);
  2. per-interface refinement: the pairs of subgraphs joined by VTLs are edge-
     coloured greedily (pairs in ascending (k, k') order, each takes the
     smallest colour used by neither of its subgraphs); for every colour and
     every beta in {2^(j/2): j = -4..4}, that colour's VTLs get
     beta alpha* / a_vv, the others alpha* / a_vv, K sweeps run, and each pair of
     the colour keeps the beta with the smallest RMS twin mismatch
     |u_p - u_twin(p)| over the ports of its VTLs (u_p the local potential at
     the port after K sweeps);
  3. label of a VTL = ln(alpha* beta*) of its pair.
"""
from __future__ import annotations

import numpy as np

from . import oracle as O

ALPHAS = 2.0 ** (np.arange(17) / 2.0)
BETAS = 2.0 ** (np.arange(-4, 5) / 2.0)


def pair_colours(vtl_k, vtl_k2):
    """Pair id of every VTL and the greedy colour of every pair (pairs in ascending (k, k') order)."""
    pairs = sorted(set(zip(vtl_k.tolist(), vtl_k2.tolist())))
    index = {pq: i for i, pq in enumerate(pairs)}
    taken: dict[int, set] = {}
    colour = []
    for a, b in pairs:
        used = taken.setdefault(a, set()) | taken.setdefault(b, set())
        c = 0
        while c in used:
            c += 1
        colour.append(c)
        taken[a].add(c)
        taken[b].add(c)
    pid = np.array([index[(a, b)] for a, b in zip(vtl_k.tolist(), vtl_k2.tolist())], dtype=np.int64)
    return pid, np.array(colour, dtype=np.int64)


def port_potentials(part, solver, b, k):
    """Potential of every port after k sweeps from zero waves (local solution at its vertex)."""
    xl, _ = solver.run_local(b, k)
    return xl[part.loc_ptr[np.repeat(np.arange(part.nsub), np.diff(part.port_ptr))] + _port_lidx(part)]


def _port_lidx(part):
    """Local index of every port's vertex in its subgraph's sorted vertex list."""
    out = np.empty(part.nports, dtype=np.int64)
    for k in range(part.nsub):
        lv = part.loc_vtx[part.loc_ptr[k]:part.loc_ptr[k + 1]]
        sl = slice(part.port_ptr[k], part.port_ptr[k + 1])
        out[sl] = np.searchsorted(lv, part.port_v[sl])
    return out


def make_labels(A, spec, b, k_probe=200):
    """(alpha*, per-VTL labels, per-pair scores [colour runs x pairs]) for one system, first RHS."""
    part = O.Partition(A, spec)
    b = np.ascontiguousarray(np.atleast_2d(b)[0])
    z0 = part.zdiag
    res = []
    for a in ALPHAS:
        r = O.Solver(part, a * z0).run(b, k_probe, k_probe, 0.0)
        res.append(float(r["relres"][0, 0]))
    a_star = float(ALPHAS[int(np.argmin(res))])
    pid, colour = pair_colours(part.vtl_k, part.vtl_k2)
    npair = len(colour)
    pair_of_port = pid[part.port_vtl]
    scores = np.full((len(BETAS), npair), np.inf)
    for c in range(int(colour.max()) + 1 if npair else 0):
        sel = colour[pid] == c
        for ib, beta in enumerate(BETAS):
            z = a_star * z0
            z[sel] *= beta
            u = port_potentials(part, O.Solver(part, z), b, k_probe)
            mis = np.abs(u - u[part.port_twin])
            ss = np.bincount(pair_of_port, weights=mis * mis, minlength=npair)
            cnt = np.maximum(np.bincount(pair_of_port, minlength=npair), 1)
            score = np.sqrt(ss / cnt)
            in_c = colour == c
            scores[ib, in_c] = score[in_c]
    beta_best = BETAS[np.argmin(scores, axis=0)] if npair else np.ones(0)
    labels = np.log(a_star * beta_best[pid])
    return a_star, labels, dict(alpha_residuals=np.array(res), scores=scores, pid=pid, colour=colour)
