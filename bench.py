#!/usr/bin/env python3
"""Benchmark: VTM on the batch of 64 random-geometric-graph systems (7.4M unknowns, 4 RHS each).

One step = the whole hot path on one batch of synthetic input, with the EVS
partition (host) done once beforehand and timed on its own: vtm_setup (the
learned impedance model's inference on the GPU, port augmentation, device
factorisation of all 14,380 local matrices, port Green's functions) +
vtm_solve to relative residual 1e-8 in every system and right-hand side
(FP32 sweeps, exchanges, FP64 residual tests, refinement; a system that has
converged stops sweeping).  Inputs are resident in HBM (torch tensors) before
the timed region.

Prints ONE JSON line.  value = unknown-updates per second of the headline:
sum over systems of n_s * nrhs * (sweeps system s ran) / step time.  Beside it:
time to tolerance with and without the host partition, sweeps, the residual
re-checked on the host in FP64, the element-wise error against the FP64 oracle
after a fixed number of sweeps, plain FP64 VTM on the same workload (the
speed-up), the 3D Poisson and 1024^2 workloads on the same path, the roofline
of the dominant kernel (the port-reduced sweep k_schur: algorithmic bytes of the
sweeps of the timed steps over their event-timed duration), the set-up's
matrix-core use and the CPU oracle timed on this host.  Measured HBM traffic and
matrix-core counts come from the rocprofv3 summaries under profiles/ while the
kernels' source is the one they were taken with.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    "c5": "64 random geometric graph Laplacians + 1e-2 I, n ~ U[20k, 200k] (7,362,043 unknowns), graph EVS (tree VTLs) into "
          "14,380 subgraphs, 4 RHS per system",
    "c3": "3D 7-point Poisson 128^3 (2,097,152 unknowns), seeded RCB into 4096 subgraphs, 8 RHS",
    "c2": "2D random-conductance Laplacian lognormal(0,1) + 1e-3 I on 1024^2, 1024 subgraphs of 33x33, 1 RHS",
    "c4": "2D GRF diffusion 512^2, 256 subgraphs, 1 RHS",
    "c1": "2D Dirichlet Laplacian 64^2, 16 subgraphs, 1 RHS",
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse_variant(B, Zm, v, A, spec):
    """{ir,fp64}_{lrn,match,diag,aNN}[_sub|_port] -> (precision, z_rule, z, params, sweep_mode)."""
    parts = v.split("_")
    prec_s, zr = parts[0], parts[1]
    mode = {"sub": 1, "port": 2}.get(parts[2], 0) if len(parts) > 2 else 0
    precision = B.VTM_FP32_IR if prec_s == "ir" else B.VTM_FP64
    params = None
    if zr == "diag":
        z_rule, z = B.VTM_Z_DIAG, None
    elif zr == "lrn":
        z_rule, z, params = B.VTM_Z_LEARNED, None, Zm.load()
    elif zr == "match":
        z_rule, z = B.VTM_Z_MATCHED, None
    else:  # uniform multiplier alpha on the diagonal rule, e.g. a64
        hh = B.VTM(device=-1)
        hh.evs_partition(A, spec)
        z_rule, z = B.VTM_Z_USER, float(zr[1:]) * hh.get_partition()["zdiag"]
        hh.close()
    return precision, z_rule, z, params, mode


def run_variant(B, Zm, torch, cfg, variant, steps, warmup, check_every=0, max_sweeps=200000):
    """Partition once (timed), then warmup + steps of setup + solve; returns timings, stats and x."""
    import numpy as np

    A, spec = cfg["A"], cfg["spec"]
    precision, z_rule, z, params, mode = parse_variant(B, Zm, variant, A, spec)
    h = B.VTM(device=0, precision=precision, check_every=check_every, max_sweeps=max_sweeps, sweep_mode=mode)
    t0 = time.perf_counter()
    info = h.evs_partition(A, spec, nsys=cfg["nsys"], sys_ptr=cfg["sys_ptr"])
    part_s = time.perf_counter() - t0
    if params is not None:
        h.zmodel_load(params)
    b_dev = torch.tensor(cfg["b"], dtype=torch.float64, device="cuda")
    x_dev = torch.empty_like(b_dev)
    times, res = [], None
    for i in range(warmup + steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.setup(z_rule, z)
        res = h.solve(b_dev, cfg["tol"], x_dev)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if i >= warmup:
            times.append(dt)
        log(f"  {variant} step {i} ({'warmup' if i < warmup else 'timed'}): {dt * 1e3:.2f} ms, status {res['status']}, "
            f"sweeps {h.get_stats()['sweeps']}, relres {float(res['relres'].max()):.2e}")
    st = h.get_stats()
    n_s = np.diff(cfg["sys_ptr"])
    stop = np.where(res["iters"] > 0, res["iters"], st["sweeps"]).max(axis=0)  # sweeps each system ran
    updates = float((n_s * stop).sum()) * cfg["b"].shape[0]
    out = dict(partition_s=part_s, info=info, step_s=sum(times) / len(times), stats=st, iters=res["iters"],
               relres=float(res["relres"].max()), status=int(res["status"]), x=x_dev.cpu().numpy(), z=h.get_z(),
               updates=updates, sys_sweeps=stop)
    h.close()
    del b_dev, x_dev
    return out


def host_residual(cfg, x):
    """max over (rhs, system) of ||b - A x|| / ||b|| in FP64 on the host (SciPy)."""
    import numpy as np

    As = cfg["A"].to_scipy()
    b, sp = cfg["b"], cfg["sys_ptr"]
    worst = 0.0
    for c in range(b.shape[0]):
        r = b[c] - As @ x[c]
        for s in range(cfg["nsys"]):
            lo, hi = sp[s], sp[s + 1]
            worst = max(worst, float(np.linalg.norm(r[lo:hi]) / np.linalg.norm(b[c, lo:hi])))
    return worst


def oracle_error_fixed_sweeps(B, Zm, torch, cfg, variant, z, nsweeps=20):
    """Element-wise error of the GPU iterate after nsweeps against the FP64 oracle's with the same
    impedances (first right-hand side): max |x_gpu - x_oracle| / max |x_oracle|, for the variant's
    precision and for FP64 sweeps."""
    import numpy as np

    from oracle import oracle as O

    A, spec = cfg["A"], cfg["spec"]
    b = cfg["b"][:1]
    P = O.Partition(A, spec)
    xo = O.Solver(P, z).run(b, nsweeps, 0, 0.0, sys_ptr=cfg["sys_ptr"])["x"][0]
    out = {}
    prec_head = B.VTM_FP32_IR if variant.startswith("ir") else B.VTM_FP64
    for label, prec in (("headline_precision", prec_head), ("fp64", B.VTM_FP64)):
        h = B.VTM(device=0, precision=prec)
        h.evs_partition(A, spec, nsys=cfg["nsys"], sys_ptr=cfg["sys_ptr"])
        h.setup(B.VTM_Z_USER, z)
        xg = h.run_sweeps(b, nsweeps)[0]
        h.close()
        out[label] = float(np.max(np.abs(xg - xo)) / np.max(np.abs(xo)))
    return dict(sweeps=nsweeps, rhs=1, max_abs_err_over_max_abs_x=out)


def _profile_fields(name, keys):
    """Fields of a committed counter summary under profiles/, or None when the kernels' source has
    changed since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.split(":", 1)[0].strip() in keys + ("kernels-source-sha256",):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    src = os.path.join(ROOT, "paper_0807_1949_amd", "csrc", "kernels.hip")
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != fields.get("kernels-source-sha256"):
        return None
    if any(k not in fields for k in keys):
        return None
    return fields


def measured_traffic(kernel, summary):
    """HBM bytes per launch of a kernel (FETCH_SIZE + WRITE_SIZE, copy-calibrated) from a committed
    counter summary, or None."""
    key = kernel + "-traffic-bytes-per-launch"
    f = _profile_fields(summary, (key,))
    return None if f is None else float(f[key])


def setup_mfma(workload):
    """Matrix-core use of the set-up kernels (factorisation and Gram) from their counters: FP64 MFMA
    FLOPs of one set-up over the two launches' durations, or None when the kernels have changed since."""
    keys = ("setup-mfma-flops-per-launch", "setup-duration-us")
    f = _profile_fields(f"setup_mfma_{workload.replace('^', '')}.md", keys)
    if f is None:
        return None
    flops, us = float(f[keys[0]]), float(f[keys[1]])
    achieved = flops / (us * 1e-6) / 1e12
    return dict(kernel="k_factor + k_gram", workload=workload, bound="latency", mfma_dtype="f64",
                flops_per_launch=flops, avg_launch_us=us, achieved=achieved, peak=78.6, unit="TFLOP/s",
                frac=achieved / 78.6)


def host_cpu():
    """CPU model, logical CPUs available to this process and physical cores of the machine."""
    model, cores, cur = None, set(), {}
    try:
        for line in open("/proc/cpuinfo"):
            if ":" not in line:
                if cur:
                    cores.add((cur.get("physical id"), cur.get("core id")))
                cur = {}
                continue
            k, v = (t.strip() for t in line.split(":", 1))
            cur[k] = v
            if k == "model name" and model is None:
                model = v
        if cur:
            cores.add((cur.get("physical id"), cur.get("core id")))
    except OSError:
        pass
    return dict(cpu_model=model, nproc=len(os.sched_getaffinity(0)), physical_cores=len(cores),
                logical_cpus=os.cpu_count())


def cpu_baseline(O, cfg, z, target_s=15.0):
    """The oracle (plain FP64 C, OpenMP over subgraphs) on a bounded sample of the headline workload:
    sweeps of the same system, partition and impedances on the first right-hand side, sized to about
    target_s seconds (its partition and factorisation excluded); unknown-updates/s = n * sweeps / t."""
    A, spec = cfg["A"], cfg["spec"]
    P = O.Partition(A, spec)
    t0 = time.perf_counter()
    s = O.Solver(P, z)
    t_setup = time.perf_counter() - t0
    b = cfg["b"][:1]
    sp = cfg["sys_ptr"]
    s.run(b, 2, 0, 0.0, sys_ptr=sp)  # first touch of the factors
    t0 = time.perf_counter()
    s.run(b, 5, 0, 0.0, sys_ptr=sp)
    t5 = time.perf_counter() - t0
    nsw = int(max(2, min(50000, target_s / max(t5 / 5, 1e-6))))
    t0 = time.perf_counter()
    s.run(b, nsw, 0, 0.0, sys_ptr=sp)
    dt = time.perf_counter() - t0
    out = dict(value=A.n * nsw / dt, unit="unknown-updates/s", cores=O.num_threads(), kind="oracle",
               sample=f"{nsw} FP64 sweeps of {cfg['name']} (all {cfg['nsys']} systems, first right-hand side, "
                      f"same partition and learned impedances; partition and factorisation excluded), {dt:.1f} s",
               time_per_sweep_s=dt / nsw, factorisation_s=t_setup)
    out.update(host_cpu())
    return out


def roofline_of(st, workload):
    """Roofline of the sweep kernel of a solve from its own statistics: algorithmic bytes of the sweeps
    it ran over their event-timed duration (HIP events on the library's stream around the sweep
    launches; in per-sweep launches one sweep is one launch of the kernel)."""
    kernel = ("k_schur_persist" if st["persistent"] else "k_schur") if st["sweep_mode"] == 2 else "k_sweep"
    sweep_s = st["sweep_ms"] / 1e3
    achieved = st["sweep_bytes"] / max(sweep_s, 1e-12) / 1e9
    summary = f"sweep_traffic_{workload.replace('^', '')}.md"
    r = dict(kernel=kernel, bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
             frac=achieved / HBM_PEAK_GBS, traffic=measured_traffic(kernel, summary),
             bytes_per_launch=st["sweep_bytes"] / max(st["sweeps"], 1), avg_launch_us=sweep_s * 1e6 / max(st["sweeps"], 1),
             sweeps=int(st["sweeps"]), bytes_per_full_launch=st["bytes_per_sweep"],
             traffic_note="traffic: HBM bytes (copy-calibrated FETCH_SIZE + WRITE_SIZE) of the launches that cover "
                          "every subgraph, to compare with bytes_per_full_launch (algorithmic bytes of such a "
                          "launch); bytes_per_launch averages the solve's launches, fewer once systems converge")
    if st["persistent"]:
        r["bound"] = "latency"
        r["note"] = ("one persistent launch per batch of sweeps: G_k read once per launch; the time per sweep is "
                     "set by the latency of the wave exchange, so the HBM fraction is not its bound")
    return r


def run_configs(names, B, Zm, torch, out_path=None, sweep_mode=0):
    """Every named workload at full size: learned-Z FP32+IR VTM on the GPU to its tolerance (timed:
    setup + solve after one warm-up), its relative residual re-checked on the host in FP64, and its
    error against the FP64 oracle with the same impedances, both solved to 1e-12 (at 1e-8 the error
    is bounded only by the condition number times the residual)."""
    import numpy as np

    import gen
    from oracle import oracle as O

    rows = []
    for name in names:
        cfg = gen.make_config(name)
        A, spec, b, tol = cfg["A"], cfg["spec"], cfg["b"], cfg["tol"]
        oracle_rhs = 1 if A.n > 1_500_000 else b.shape[0]  # the FP64 oracle runs one RHS at a time
        As = A.to_scipy()
        log(f"config {cfg['name']}: n {A.n}, nrhs {b.shape[0]}, systems {cfg['nsys']}")
        h = B.VTM(device=0, precision=B.VTM_FP32_IR, check_every=0, sweep_mode=sweep_mode)
        info = h.evs_partition(A, spec, nsys=cfg["nsys"], sys_ptr=cfg["sys_ptr"])
        h.zmodel_load(Zm.load())
        b_dev = torch.tensor(b, dtype=torch.float64, device="cuda")
        x_dev = torch.empty_like(b_dev)
        times = []
        for i in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h.setup(B.VTM_Z_LEARNED)
            res = h.solve(b_dev, tol, x_dev)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        st = h.get_stats()
        log(f"  GPU: {times[-1] * 1e3:.2f} ms to {tol:g}, {st['sweeps']} sweeps, {st['checks']} tests, "
            f"mode {st['sweep_mode']}, persistent {st['persistent']}")
        x = x_dev.cpu().numpy()
        sp = cfg["sys_ptr"]
        host_rel = 0.0
        for c in range(b.shape[0]):
            r = b[c] - As @ x[c]
            for k in range(cfg["nsys"]):
                lo, hi = sp[k], sp[k + 1]
                host_rel = max(host_rel, float(np.linalg.norm(r[lo:hi]) / np.linalg.norm(b[c, lo:hi])))
        log(f"  host residual {host_rel:.3e}")
        z = h.get_z()
        h.reset_waves()
        tight = h.solve(b_dev, 1e-12, x_dev)
        xt = x_dev.cpu().numpy()
        log(f"  GPU at 1e-12: {int(np.max(tight['iters']))} sweeps; oracle on {oracle_rhs} right-hand side(s)")
        P = O.Partition(A, spec)
        t0 = time.perf_counter()
        ro = O.Solver(P, z).run(b[:oracle_rhs], 10 ** 6, 10, 1e-12, sys_ptr=sp)
        t_oracle = time.perf_counter() - t0
        err = max(float(np.linalg.norm(xt[c] - ro["x"][c]) / np.linalg.norm(ro["x"][c])) for c in range(oracle_rhs))
        row = dict(config=cfg["name"], n=int(A.n), nsub=int(info["nsub"]), nrhs=int(b.shape[0]), systems=int(cfg["nsys"]),
                   tol=tol, time_to_tol_s=times[-1], setup_ms=st["setup_ms"], sweeps=int(st["sweeps"]),
                   outer_steps=int(st["outer_steps"]), tests=int(st["checks"]), sweep_mode=int(st["sweep_mode"]),
                   persistent=int(st["persistent"]), relres_lib=float(np.max(res["relres"])), relres_host=host_rel,
                   err_vs_oracle_at_1e12=err, oracle_rhs=oracle_rhs, sweeps_1e12=int(np.max(tight["iters"])),
                   oracle_sweeps_1e12=int(np.max(ro["iters"])), oracle_s_1e12=t_oracle, oracle_threads=O.num_threads())
        log("  " + json.dumps(row))
        rows.append(row)
        h.close()
    if out_path:
        with open(out_path, "w") as f:
            json.dump(rows, f, indent=1)
    return rows


def paper_shape(B, Zm, out_path=None):
    """Section 9's experiments in shape (the paper's figures are absent, so there is no number to
    compare with): a 5-point Dirichlet Laplacian, (i) 65 x 65 (n = 4225) on p = 4 ... 128 tiles,
    (ii) p = 64 tiles for n = 17^2 ... 121^2.  The exact solution x* is seeded uniform[-1, 1] and
    b = A x*; plain FP64 VTM (substitution sweeps) with the diagonal rule, impedance matching
    and the learned rule; K = sweeps until the RMS error against x* falls below 1e-12 RMS(x*) (tested every
    5 sweeps; the double-precision floor of this iteration lies near 1e-14)."""
    import numpy as np

    from gen import systems as S

    tiles = {4: (2, 2), 8: (4, 2), 16: (4, 4), 32: (8, 4), 64: (8, 8), 128: (16, 8)}
    cases = [("p", p, 65) for p in (4, 8, 16, 32, 64, 128)] + [("n", 64, nx) for nx in (17, 33, 49, 65, 97, 121)]
    rows = []
    for kind, p, nx in cases:
        A = S.laplace2d_dirichlet(nx)
        xs = np.random.default_rng([9, nx]).uniform(-1.0, 1.0, A.n)
        b = (A.to_scipy() @ xs)[None, :]
        px, py = tiles[p]
        spec = dict(kind="grid", dims=(nx, nx, 1), parts=(px, py, 1))
        row = dict(series=kind, p=p, n=A.n)
        for rule, label in ((B.VTM_Z_DIAG, "diag"), (B.VTM_Z_MATCHED, "matched"), (B.VTM_Z_LEARNED, "learned")):
            h = B.VTM(device=0, precision=B.VTM_FP64, sweep_mode=1)
            h.evs_partition(A, spec)
            if rule == B.VTM_Z_LEARNED:
                h.zmodel_load(Zm.load())
            h.setup(rule)
            k, err, floor = 0, 1.0, 1.0
            while k < 40000:
                x = h.run_sweeps(b, 5)[0]
                k += 5
                err = float(np.sqrt(np.mean((x - xs) ** 2)) / np.sqrt(np.mean(xs ** 2)))
                floor = min(floor, err)
                if err <= 1e-12:
                    break
            row[label] = k if err <= 1e-12 else None
            h.close()
        rows.append(row)
        log(f"  {kind}: p {p:3d} n {A.n:6d}  K(diag) {row['diag']}  K(matched) {row['matched']}  K(learned) {row['learned']}")
    if out_path:
        with open(out_path, "w") as f:
            json.dump(rows, f, indent=1)
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c5", help="headline workload (c1..c5)")
    ap.add_argument("--variants", default="ir_lrn,fp64_diag_sub",
                    help="comma list of {ir,fp64}_{lrn,match,diag,aNN}[_sub|_port]: precision, impedance rule "
                         "(learned network, impedance matching, diagonal, or NN times the diagonal), sweep mode (substitution, "
                         "port-reduced, default chosen by the library); the first is the headline, the others are "
                         "timed beside it (one step each)")
    ap.add_argument("--extra", default="c3,c2", help="further workloads timed on the headline variant (one step each; "
                    "c2 also with plain FP64 VTM)")
    ap.add_argument("--no-extra-plain", action="store_true", help="skip plain FP64 VTM on the extra 1024^2 workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle-error", action="store_true", help="skip the fixed-sweep comparison with the oracle")
    ap.add_argument("--check-every", type=int, default=0, help="0 = adaptive test placement")
    ap.add_argument("--configs", default="", help="instead of the benchmark line: check these workloads at full "
                    "size (comma list of c1..c5) against the oracle")
    ap.add_argument("--configs-out", default="", help="write the --configs results as JSON to this path")
    ap.add_argument("--configs-mode", type=int, default=0, help="sweep mode for --configs (0 library choice, 1, 2)")
    ap.add_argument("--paper-shape", default="", help="instead of the benchmark line: Section 9's K(p), K(n) "
                    "experiments; write the table as JSON to this path")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="copy this many MiB with a plain device copy first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design, not a build).", file=sys.stderr)
        sys.exit(2)

    import torch

    import gen
    from paper_0807_1949_amd import binding as B
    from paper_0807_1949_amd import zmodel as Zm

    if args.paper_shape:
        paper_shape(B, Zm, args.paper_shape)
        return
    if args.configs:
        run_configs(args.configs.split(","), B, Zm, torch, args.configs_out or None, args.configs_mode)
        return
    if args.calib_copy_mib > 0:
        src = torch.empty(args.calib_copy_mib << 18, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calib_copy_mib} MiB read + {args.calib_copy_mib} MiB written")
        del src, dst
    variants = args.variants.split(",")
    log(f"workload {args.workload}")
    cfg = gen.make_config(args.workload)
    head = run_variant(B, Zm, torch, cfg, variants[0], args.steps, args.warmup, args.check_every)
    st = head["stats"]
    others = {v: run_variant(B, Zm, torch, cfg, v, 1, 1, args.check_every) for v in variants[1:]}
    nrhs = int(cfg["b"].shape[0])
    ms_step = head["step_s"] * 1e3

    def summary(r, cfg_):
        s_ = r["stats"]
        return dict(time_to_tol_s=r["step_s"], time_to_tol_with_partition_s=r["step_s"] + r["partition_s"],
                    partition_s=r["partition_s"], setup_ms=s_["setup_ms"], solve_ms=s_["solve_ms"],
                    sweeps=int(s_["sweeps"]), sweeps_per_system_max=int(r["sys_sweeps"].max()),
                    sweeps_per_system_min=int(r["sys_sweeps"].min()), outer_steps=s_["outer_steps"],
                    tests=s_["checks"], relres=r["relres"], status=r["status"], sweep_mode=s_["sweep_mode"],
                    persistent=s_["persistent"], unknown_updates_per_s=r["updates"] / r["step_s"],
                    sweep_us=s_["sweep_ms"] * 1e3 / max(s_["sweeps"], 1))

    line = dict(
        metric="time to rel. residual 1e-8 (s) & unknown-updates/s; learned-Z vs plain VTM",
        value=head["updates"] / head["step_s"], unit="unknown-updates/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=ms_step, higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f32+f64" if variants[0].startswith("ir") else "f64", data="synthetic",
        config=dict(workload=cfg["name"] + " (" + WORKLOADS[args.workload] + ")", n=int(cfg["A"].n),
                    nsub=head["info"]["nsub"], nsys=int(cfg["nsys"]), nrhs=nrhs, tol=cfg["tol"], variant=variants[0],
                    parallelism="1 GPU, all subgraphs of all systems on one device"),
        time_to_tol_s=head["step_s"], time_to_tol_with_partition_s=head["step_s"] + head["partition_s"],
        partition_s=head["partition_s"], sweeps=int(st["sweeps"]), setup_ms=st["setup_ms"], solve_ms=st["solve_ms"],
        relres=head["relres"],
        value_note="unknown-updates = sum over systems of n_s x nrhs x the sweeps system s ran (it stops at its "
                   "converged test); port-reduced sweeps update the port unknowns, whose iterates equal those "
                   "of full local solves, so the count is of equivalent updates; time = setup + solve",
    )
    line["host_relres"] = host_residual(cfg, head["x"])
    line["variants"] = {variants[0]: summary(head, cfg)}
    for v, r in others.items():
        line["variants"][v] = summary(r, cfg)
        line["speedup_vs_" + v] = r["step_s"] / head["step_s"]
        line["speedup_vs_" + v + "_with_partition"] = (r["step_s"] + r["partition_s"]) / (head["step_s"] + head["partition_s"])
    line["roofline"] = roofline_of(st, cfg["name"])
    if not args.no_oracle_error:
        log("fixed-sweep error against the oracle")
        line["oracle_error_20_sweeps"] = oracle_error_fixed_sweeps(B, Zm, torch, cfg, variants[0], head["z"])
    extra = {}
    for w in [e for e in args.extra.split(",") if e]:
        log(f"extra workload {w}")
        c = gen.make_config(w)
        r = run_variant(B, Zm, torch, c, variants[0], 1, 1, args.check_every)
        e = summary(r, c)
        e.update(workload=c["name"] + " (" + WORKLOADS[w] + ")", host_relres=host_residual(c, r["x"]),
                 roofline=roofline_of(r["stats"], c["name"]))
        if not args.no_oracle_error:
            e["oracle_error_20_sweeps"] = oracle_error_fixed_sweeps(B, Zm, torch, c, variants[0], r["z"])
        if w == "c2" and not args.no_extra_plain:
            p = run_variant(B, Zm, torch, c, "fp64_diag_sub", 1, 1, args.check_every)
            e["fp64_diag_sub"] = summary(p, c)
            e["speedup_vs_fp64_diag_sub"] = p["step_s"] / r["step_s"]
        extra[w] = e
    line["extra_workloads"] = extra
    line["setup_mfma"] = setup_mfma(cfg["name"])
    if not args.no_cpu_baseline:
        from oracle import oracle as O

        log("cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(O, cfg, head["z"])
    torch.cuda.synchronize()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
