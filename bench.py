#!/usr/bin/env python3
"""Benchmark: VTM on the 1024^2 lognormal-conductance system (32x32 subgraphs).

One step = the whole hot path on one batch of synthetic input, with the
partition (host) done once beforehand: vtm_setup (impedances -- for the
learned rule the network's inference on the GPU --, port augmentation, device
factorisation of all 1024 local matrices, port Green's functions) + vtm_solve
to relative residual 1e-8 (sweeps, exchanges, FP64 residual tests,
refinement).  Inputs are resident in HBM (torch tensors) before the timed
region.  The per-VTL features of the learned rule depend only on the matrix
and the partition and are computed with it, in the warm-up step.

Prints ONE JSON line.  value = unknown-updates per second of the headline
variant (n * nrhs * sweeps / step time).  Also reported: time to tolerance of
every variant and the speedup of the headline over plain FP64 VTM, the sweep
kernel's roofline (algorithmic bytes per sweep over the event-timed sweep
duration), the roofline of the streaming port-reduced sweep where G comes
from HBM every sweep (3D Poisson 128^3, 8 RHS), the set-up's matrix-core use
and the CPU oracle timed on this host.  Measured HBM traffic and matrix-core
counts come from the rocprofv3 summaries under profiles/ while the kernels'
source is the one they were taken with.
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


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_variant(B, torch, A, spec, b_dev, tol, precision, z_rule, z, steps, warmup, check_every, max_sweeps,
                mode=0, params=None, leaf_size=0):
    h = B.VTM(device=0, precision=precision, check_every=check_every, max_sweeps=max_sweeps, sweep_mode=mode,
              leaf_size=leaf_size)
    t0 = time.perf_counter()
    info = h.evs_partition(A, spec)
    part_s = time.perf_counter() - t0
    if params is not None:
        h.zmodel_load(params)
    x_dev = torch.empty_like(b_dev)
    times, res = [], None
    for i in range(warmup + steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.setup(z_rule, z)
        res = h.solve(b_dev, tol, x_dev)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if i >= warmup:
            times.append(dt)
        log(f"  step {i} ({'warmup' if i < warmup else 'timed'}): {dt * 1e3:.2f} ms, status {res['status']}, "
            f"sweeps {h.get_stats()['sweeps']}, relres {float(res['relres'].max()):.2e}")
    st = h.get_stats()
    out = dict(partition_s=part_s, info=info, step_s=sum(times) / len(times), stats=st,
               relres=float(res["relres"].max()), status=int(res["status"]), x=x_dev.clone(), z=h.get_z())
    h.close()
    return out


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


def measured_traffic(kernel, summary="sweep_traffic_c2_lognormal_1024.md"):
    """HBM bytes per sweep of the sweep kernel (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None."""
    key = kernel + "-traffic-bytes-per-sweep"
    f = _profile_fields(summary, (key,))
    return None if f is None else float(f[key])


def streaming_sweep_roofline(B, Zm, torch, nsweeps=48):
    """The port-reduced sweep where it streams G from HBM: the 3D Poisson 128^3 workload (4096 RCB
    subgraphs, 8 RHS, FP32 sweeps, learned impedances), one kernel launch per sweep.  Algorithmic
    bytes per sweep (every packed G_k once, the port constants, the incoming and outgoing waves) over
    the event-timed duration of the sweep launches."""
    import gen

    cfg = gen.make_config("c3")
    h = B.VTM(device=0, precision=B.VTM_FP32_IR, check_every=nsweeps, max_sweeps=nsweeps, sweep_mode=2, persistent=1)
    info = h.evs_partition(cfg["A"], cfg["spec"])
    h.zmodel_load(Zm.load())
    h.setup(B.VTM_Z_LEARNED)
    b_dev = torch.tensor(cfg["b"], dtype=torch.float64, device="cuda")
    x_dev = torch.empty_like(b_dev)
    for _ in range(2):  # the first solve warms up (graph capture)
        h.reset_waves()
        h.solve(b_dev, 1e-30, x_dev, raise_on=())
    st = h.get_stats()
    h.close()
    sweep_s = st["sweep_ms"] / 1e3 / max(st["sweeps"], 1)
    achieved = st["bytes_per_sweep"] / sweep_s / 1e9
    return dict(kernel="k_schur", workload=cfg["name"] + " (3D 7-point Poisson 128^3, 4096 RCB subgraphs, 8 RHS, FP32)",
                bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                traffic=measured_traffic("k_schur", "sweep_traffic_c3_poisson_128.md"),
                bytes_per_sweep=st["bytes_per_sweep"], avg_sweep_us=sweep_s * 1e6, sweeps_timed=int(st["sweeps"]),
                nsub=int(info["nsub"]))


def setup_mfma():
    """Matrix-core use of the factorisation kernel from its counters (FP64 MFMA FLOPs per launch over
    the launch's duration), or None when the kernels have changed since."""
    keys = ("k_factor-mfma-flops-per-launch", "k_factor-duration-us")
    f = _profile_fields("setup_mfma_c2_lognormal_1024.md", keys)
    if f is None:
        return None
    flops, us = float(f[keys[0]]), float(f[keys[1]])
    achieved = flops / (us * 1e-6) / 1e12
    return dict(kernel="k_factor", bound="latency", mfma_dtype="f64", flops_per_launch=flops, avg_launch_us=us,
                achieved=achieved, peak=78.6, unit="TFLOP/s", frac=achieved / 78.6)


def cpu_baseline(O, A, spec, b, z):
    """Oracle (plain FP64 C, OpenMP) on a bounded sample: a few sweeps of the same system."""
    P = O.Partition(A, spec)
    s = O.Solver(P, z)
    s.run(b[:1], 2, 0, 0.0)  # first touch of the factors
    t0 = time.perf_counter()
    s.run(b[:1], 20, 0, 0.0)
    t20 = time.perf_counter() - t0
    nsw = int(max(2, min(50000, 15.0 / max(t20 / 20, 1e-6))))  # about 15 s of oracle work
    t0 = time.perf_counter()
    s.run(b[:1], nsw, 0, 0.0)
    dt = time.perf_counter() - t0
    return dict(value=A.n * nsw / dt, unit="unknown-updates/s", cores=O.num_threads(), kind="oracle",
                sample=f"{nsw} FP64 sweeps of the same system and partition (factorisation excluded), "
                       f"{dt:.1f} s", time_per_sweep_s=dt / nsw)


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
    ap.add_argument("--small", action="store_true", help="128^2 version of the workload (quick check)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-streaming-roofline", action="store_true",
                    help="skip the port-reduced sweep's HBM roofline on the 3D Poisson workload")
    ap.add_argument("--variants", default="ir_lrn,fp64_diag_sub,ir_diag",
                    help="comma list of {ir,fp64}_{lrn,match,diag,aNN}[_sub|_port]: precision, impedance rule "
                         "(learned network, impedance matching, diagonal, or NN times the diagonal), sweep mode (substitution, "
                         "port-reduced, default chosen by the library); the first is the headline, the "
                         "second its comparison")
    ap.add_argument("--check-every", type=int, default=0, help="0 = adaptive test placement")
    ap.add_argument("--leaf-size", type=int, default=0, help="nested-dissection leaf size (0 = library default)")
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
    cfg = gen.make_config("c2", small=args.small)
    A, spec, tol = cfg["A"], cfg["spec"], cfg["tol"]
    b_dev = torch.tensor(cfg["b"], dtype=torch.float64, device="cuda")
    results = {}
    variants = args.variants.split(",")
    zinfo = {}
    for v in variants:
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
            alpha = float(zr[1:])
            hh = B.VTM(device=-1)
            hh.evs_partition(A, spec)
            z_rule, z = B.VTM_Z_USER, alpha * hh.get_partition()["zdiag"]
            hh.close()
        log(f"variant {v}")
        results[v] = run_variant(B, torch, A, spec, b_dev, tol, precision, z_rule, z, args.steps, args.warmup,
                                 args.check_every, 200000, mode, params, args.leaf_size)
        zinfo[v] = results[v]["z"]
    head = results[variants[0]]
    st = head["stats"]
    sweeps = st["sweeps"]
    nrhs = 1
    ms_step = head["step_s"] * 1e3
    value = A.n * nrhs * sweeps / head["step_s"]
    sweep_s = st["sweep_ms"] / 1e3 / max(sweeps, 1)
    achieved = st["bytes_per_sweep"] / sweep_s / 1e9
    kernel = ("k_schur_persist" if st["persistent"] else "k_schur") if st["sweep_mode"] == 2 else "k_sweep"
    line = dict(
        metric="time to rel. residual 1e-8 (s) & unknown-updates/s; learned-Z vs plain VTM",
        value=value, unit="unknown-updates/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=ms_step, higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f32+f64" if variants[0].startswith("ir") else "f64", data="synthetic",
        config=dict(workload=cfg["name"] + " (2D random-conductance Laplacian lognormal(0,1) + 1e-3 I, "
                    "1024 subgraphs of 33x33, single RHS)", n=A.n, nsub=head["info"]["nsub"], nrhs=nrhs, tol=tol,
                    variant=variants[0], parallelism="1 GPU, all subgraphs on one device"),
        time_to_tol_s=head["step_s"], sweeps=sweeps, setup_ms=st["setup_ms"], solve_ms=st["solve_ms"],
        relres=head["relres"], partition_s=head["partition_s"],
        variants={v: dict(time_to_tol_s=r["step_s"], sweeps=r["stats"]["sweeps"], setup_ms=r["stats"]["setup_ms"],
                          sweep_us=r["stats"]["sweep_ms"] * 1e3 / max(r["stats"]["sweeps"], 1),
                          outer_steps=r["stats"]["outer_steps"], checks=r["stats"]["checks"],
                          relres=r["relres"], status=r["status"], persistent=r["stats"]["persistent"],
                          sweep_mode=r["stats"]["sweep_mode"])
                  for v, r in results.items()},
        roofline=dict(kernel=kernel, bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=achieved / HBM_PEAK_GBS, traffic=measured_traffic(kernel),
                      bytes_per_sweep=st["bytes_per_sweep"], avg_sweep_us=sweep_s * 1e6,
                      note=("one persistent launch per batch of sweeps: G_k read once per launch, the per-sweep "
                            "time is set by the latency of the wave exchange between neighbouring workgroups, "
                            "not by bandwidth; achieved and traffic are per sweep") if st["persistent"] else
                           "one launch per sweep; achieved and traffic are per launch"),
    )
    if len(variants) > 1:
        line["speedup_vs_" + variants[1]] = results[variants[1]]["step_s"] / head["step_s"]
    line["setup_mfma"] = setup_mfma()
    if not args.no_streaming_roofline:
        log("streaming sweep roofline (3D Poisson 128^3, 8 RHS)")
        line["streaming_sweep_roofline"] = streaming_sweep_roofline(B, Zm, torch)
    if not args.no_cpu_baseline:
        from oracle import oracle as O

        z = zinfo[variants[0]]
        log("cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(O, A, spec, cfg["b"], z)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
