"""Learned impedance: labels from probe sweeps, training, evaluation.

The paper picks characteristic impedances by impedance matching (Section 7.1)
and notes that the convergence speed depends strongly on them.  Here a small
MLP predicts delta = ln(Z a_vv) per VTL from scale-free features
(``vtm_zfeatures``); its labels come from the method itself:

1. global probe: Z = alpha / a_vv for alpha in {2^(j/2): j = 0..16}; run
   K_probe sweeps from zero waves and keep the alpha* with the lowest relative
   residual (measured on the device by vtm_solve with max_sweeps = K_probe).
   K_probe must reach the asymptotic regime: short probes reward the decay of
   the first transient and pick much too small multipliers;
2. per-interface refinement: colour the subgraph-pair graph so that no two
   pairs of a colour share a subgraph; for each colour and each
   beta in {2^(j/2): j = -4..4}, scale that colour's VTLs by beta, run K_probe
   sweeps and keep, per pair, the beta with the smallest RMS twin mismatch
   |u_p - u_twin(p)| over the pair's ports (port potentials from the waves:
   u_p = (o_p + a_p) / 2);
3. label = ln(alpha* beta*).

All sweeps, residuals and the network's forward/backward passes run in
libvtm's kernels; this module only orchestrates them.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import binding as B

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "zmodel_weights.json")

ALPHAS = 2.0 ** (np.arange(17) / 2.0)
BETAS = 2.0 ** (np.arange(-4, 5) / 2.0)


def pair_colouring(k1: np.ndarray, k2: np.ndarray):
    """Greedy edge colouring of the subgraph-pair graph; returns (pair id per VTL, colour per pair)."""
    keys = k1.astype(np.int64) * (1 << 32) + k2.astype(np.int64)
    uniq, pid = np.unique(keys, return_inverse=True)
    pa, pb = (uniq >> 32).astype(np.int64), (uniq & 0xFFFFFFFF).astype(np.int64)
    used: dict[int, set] = {}
    colour = np.zeros(len(uniq), np.int32)
    for i in range(len(uniq)):
        busy = used.setdefault(int(pa[i]), set()) | used.setdefault(int(pb[i]), set())
        c = 0
        while c in busy:
            c += 1
        colour[i] = c
        used[int(pa[i])].add(c)
        used[int(pb[i])].add(c)
    return pid, colour


def port_vtl(part: dict, nsub: int) -> np.ndarray:
    """VTL of every port: a port of subgraph k at vertex v with other end k2 lies on VTL (v, min, max)."""
    k_of_port = np.repeat(np.arange(nsub), np.diff(part["port_ptr"]))
    lo = np.minimum(k_of_port, part["port_other"]).astype(np.int64)
    hi = np.maximum(k_of_port, part["port_other"]).astype(np.int64)
    key_l = np.stack([part["vtl_v"], part["vtl_k"].astype(np.int64), part["vtl_k2"].astype(np.int64)])
    order = np.lexsort(key_l[::-1])
    ks = key_l[:, order]
    # position of (v, lo, hi) among the sorted VTL keys
    idx = np.lexsort((np.concatenate([ks[2], hi]), np.concatenate([ks[1], lo]), np.concatenate([ks[0], part["port_v"]])))
    nv = ks.shape[1]
    out = np.empty(len(lo), np.int64)
    last = -1
    for j in idx:  # sorted merge: every port follows its VTL key
        if j < nv:
            last = j
        else:
            out[j - nv] = order[last]
    return out


class Prober:
    """Probe runs of K sweeps on one partitioned system."""

    def __init__(self, A, spec, b, k_probe=200, device=0, nsys=1, sys_ptr=None):
        # substitution sweeps: the probes change Z every few hundred sweeps, so the port Green's
        # functions would cost more than they save
        self.h = B.VTM(device=device, check_every=k_probe, max_sweeps=k_probe, sweep_mode=1)
        self.info = self.h.evs_partition(A, spec, nsys=nsys, sys_ptr=sys_ptr)
        self.part = self.h.get_partition()
        self.b = np.atleast_2d(b)
        self.k = k_probe
        self.z0 = self.part["zdiag"]
        self.twin = self.part["port_twin"]
        self.port_vtl = port_vtl(self.part, self.info["nsub"])

    def residual(self, z) -> float:
        self.h.setup(B.VTM_Z_USER, z)
        r = self.h.solve(self.b, 1e-300)
        return float(np.max(r["relres"]))

    def port_mismatch(self, z) -> np.ndarray:
        """|u_p - u_twin(p)| after K sweeps, per port."""
        self.h.setup(B.VTM_Z_USER, z)
        self.h.run_sweeps(self.b, self.k - 1)
        a_k = self.h.get_waves(1)[0]          # incoming waves of sweep K
        self.h.run_sweeps(self.b, 1)
        a_k1 = self.h.get_waves(1)[0]         # incoming of sweep K+1 = outgoing of sweep K at the twin
        o_k = a_k1[self.twin]
        u = 0.5 * (o_k + a_k)
        return np.abs(u - u[self.twin])

    def close(self):
        self.h.close()


def make_labels(A, spec, b, k_probe=200, device=0, log=None, nsys=1, sys_ptr=None):
    pr = Prober(A, spec, b[:1], k_probe, device, nsys, sys_ptr)
    try:
        res = np.array([pr.residual(a * pr.z0) for a in ALPHAS])
        a_star = float(ALPHAS[int(np.argmin(res))])
        part = pr.part
        pid, colour = pair_colouring(part["vtl_k"], part["vtl_k2"])
        npair = int(pid.max()) + 1 if len(pid) else 0
        best = np.full(npair, np.inf)
        beta_best = np.ones(npair)
        pair_of_port = pid[pr.port_vtl]
        for c in range(int(colour.max()) + 1 if npair else 0):
            sel = colour[pid] == c
            for beta in BETAS:
                z = a_star * pr.z0
                z[sel] *= beta
                mis = pr.port_mismatch(z)
                ss = np.bincount(pair_of_port, weights=mis * mis, minlength=npair)
                cnt = np.maximum(np.bincount(pair_of_port, minlength=npair), 1)
                score = np.sqrt(ss / cnt)
                in_c = colour == c
                better = in_c & (score < best)
                best[better] = score[better]
                beta_best[better] = beta
        labels = np.log(a_star * beta_best[pid])
        feats = pr.h.zfeatures()
        if log:
            log(f"    alpha*={a_star:g} (residual after {k_probe} sweeps {res.min():.2e}), "
                f"{npair} pairs, {int(colour.max()) + 1 if npair else 0} colours")
        return feats, labels.astype(np.float32), a_star
    finally:
        pr.close()


def init_params(X, seed=0):
    """He-initialised weights, input standardisation from the training features."""
    rng = np.random.default_rng(seed)
    X = np.asarray(X, dtype=np.float64)
    nf, nh = B.NUM_FEATURES, 64
    mu = X.mean(0)
    sd = np.maximum(X.std(0), 1e-3)
    W1 = rng.standard_normal((nh, nf)) * np.sqrt(2.0 / nf)
    W2 = rng.standard_normal((nh, nh)) * np.sqrt(2.0 / nh)
    w3 = rng.standard_normal(nh) * np.sqrt(1.0 / nh)
    return np.concatenate([mu, sd, W1.ravel(), np.zeros(nh), W2.ravel(), np.zeros(nh), w3, [0.0]]).astype(np.float32)


def fit(feats, labels, epochs=30, batch=512, lr=2e-3, seed=0, device=0, log=None):
    """Train on the device (BF16 MFMA forward/backward, Adam); returns the parameter blob and loss history."""
    P = init_params(feats, seed)
    P[-1] = float(np.mean(labels))  # start at the mean label
    tr = B.Trainer(P, device=device)
    tr.set_data(feats, labels)
    hist = []
    for ep in range(epochs):
        loss = tr.epoch(batch, lr * (0.5 ** (ep // max(1, epochs // 3))), seed * 1000 + ep)
        hist.append(loss)
        if log and (ep % 5 == 0 or ep == epochs - 1):
            log(f"    epoch {ep}: loss {loss:.4f}")
    P = tr.get_params()
    tr.close()
    return P, hist


def save(P, path=DEFAULT_WEIGHTS, meta=None):
    with open(path, "w") as f:
        json.dump(dict(params=[float(v) for v in P], meta=meta or {}), f)


def load(path=DEFAULT_WEIGHTS) -> np.ndarray:
    with open(path) as f:
        return np.array(json.load(f)["params"], dtype=np.float32)


def solve_iters(A, spec, b, tol, z_rule, z=None, params=None, precision=B.VTM_FP64, check_every=10, device=0,
                nsys=1, sys_ptr=None, sweep_mode=0):
    """Sweeps and time to tolerance for one impedance choice.  The comparisons use a fixed test cadence
    and report the first passing test (sweeps), so the counts depend on the iteration alone."""
    h = B.VTM(device=device, precision=precision, check_every=check_every, max_sweeps=200000, sweep_mode=sweep_mode)
    h.evs_partition(A, spec, nsys=nsys, sys_ptr=sys_ptr)
    if params is not None:
        h.zmodel_load(params)
    t0 = time.perf_counter()
    h.setup(z_rule, z)
    r = h.solve(b, tol)
    dt = time.perf_counter() - t0
    st = h.get_stats()
    passed = r["status"] == B.VTM_OK
    out = dict(sweeps=int(np.max(r["iters"])) if passed else None, sweeps_run=int(st["sweeps"]), time_s=dt,
               relres=float(np.max(r["relres"])), status=int(r["status"]), setup_ms=st["setup_ms"],
               solve_ms=st["solve_ms"], check_every=check_every)
    h.close()
    return out
