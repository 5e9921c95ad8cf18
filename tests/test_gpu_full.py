"""GPU parity at full workload sizes, the batch entry point, and the error paths, through the C ABI.

Full sizes: a fixed number of sweeps from zero waves (the oracle needs seconds per sweep batch at these
sizes, so the test compares iterates, not converged solves), element by element against the FP64
oracle with the same impedances: FP64 sweeps to rounding (1e-10), FP32 sweeps to FP32 accuracy.
"""
import numpy as np
import pytest

import gen
from oracle import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0807_1949_amd import binding

    binding.lib()
    return binding


def _close(a, b, tol, what=""):
    a, b = np.asarray(a), np.asarray(b)
    emax = float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
    rel = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    print(f"    {what}: max element error {emax:.2e}, relative 2-norm {rel:.2e} (tol {tol:g})", flush=True)
    assert emax <= tol and rel <= tol, (what, emax, rel, tol)


@pytest.mark.parametrize("name", ["c3", "c5"])
def test_full_size_fp64_iterates(B, name):
    """3D Poisson 128^3 (4096 RCB boxes) and the 64-system graph batch (7.4M unknowns): 20 FP64
    sweeps with the library's own mode choice, first right-hand side, against the oracle."""
    print(f"[full] {name} fp64 20 sweeps", flush=True)
    cfg = gen.make_config(name)
    b = cfg["b"][:1]
    h = B.VTM(device=0, check_every=10)
    h.evs_partition(cfg["A"], cfg["spec"], nsys=cfg["nsys"], sys_ptr=cfg["sys_ptr"])
    P = O.Partition(cfg["A"], cfg["spec"])
    z = 16.0 * P.zdiag
    h.setup(B.VTM_Z_USER, z)
    xg = h.run_sweeps(b, 20)
    mode = h.get_stats()["sweep_mode"]
    h.close()
    xo = O.Solver(P, z).run(b, 20, 0, 0.0, sys_ptr=cfg["sys_ptr"])["x"]
    _close(xg[0], xo[0], 1e-10, f"{name} mode {mode}")


def test_full_size_headline_path_c2(B):
    """The 1024^2 workload on the benchmark's path: learned impedances (BF16 network), FP32 factors,
    FP32 port-reduced sweeps in one persistent launch; 20 sweeps against the FP64 oracle with the
    same impedances."""
    from paper_0807_1949_amd import zmodel as Zm

    print("[full] c2 headline path", flush=True)
    cfg = gen.make_config("c2")
    h = B.VTM(device=0, precision=B.VTM_FP32_IR, check_every=10)
    h.evs_partition(cfg["A"], cfg["spec"])
    h.zmodel_load(Zm.load())
    h.setup(B.VTM_Z_LEARNED)
    xg = h.run_sweeps(cfg["b"], 20)
    st = h.get_stats()
    z = h.get_z()
    h.close()
    assert st["sweep_mode"] == 2 and st["persistent"] == 1
    P = O.Partition(cfg["A"], cfg["spec"])
    xo = O.Solver(P, z).run(cfg["b"], 20, 0, 0.0)["x"]
    _close(xg[0], xo[0], 2e-5, "c2 fp32 persistent learned")


def test_full_size_fp32_batch_c5(B):
    """The graph batch on the benchmark's path (learned impedances, FP32 port-reduced sweeps, four
    right-hand sides), 20 sweeps, every right-hand side against the FP64 oracle."""
    from paper_0807_1949_amd import zmodel as Zm

    print("[full] c5 fp32 learned 20 sweeps", flush=True)
    cfg = gen.make_config("c5")
    h = B.VTM(device=0, precision=B.VTM_FP32_IR, check_every=10)
    h.evs_partition(cfg["A"], cfg["spec"], nsys=cfg["nsys"], sys_ptr=cfg["sys_ptr"])
    h.zmodel_load(Zm.load())
    h.setup(B.VTM_Z_LEARNED)
    xg = h.run_sweeps(cfg["b"], 20)
    z = h.get_z()
    h.close()
    P = O.Partition(cfg["A"], cfg["spec"])
    xo = O.Solver(P, z).run(cfg["b"], 20, 0, 0.0, sys_ptr=cfg["sys_ptr"])["x"]
    for c in range(cfg["b"].shape[0]):
        _close(xg[c], xo[c], 2e-5, f"c5 fp32 rhs {c}")


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_solve_independent_handles(B, precision):
    """vtm_batch_solve over three independently partitioned and set-up handles (a 2D grid, a 3D RCB
    box system, a graph system with two RHS each): one launch per sweep for all, each handle's
    systems tested on their own.  FP64: every handle's iters equal the oracle's first passing sweep
    and x its iterate there; FP32 with refinement: the true residual of every x meets tol.  A second
    call reuses the batch and gives the same result; a re-set-up member rebuilds it."""
    print(f"[batch] precision {precision}", flush=True)
    cfgs = [gen.make_config("c2", small=True), gen.make_config("c3", small=True), gen.make_config("c5", small=True)]
    hs, Ps, zs, bs = [], [], [], []
    for i, cfg in enumerate(cfgs):
        h = B.VTM(device=0, precision=precision, check_every=10)
        h.evs_partition(cfg["A"], cfg["spec"], nsys=cfg["nsys"], sys_ptr=cfg["sys_ptr"])
        P = O.Partition(cfg["A"], cfg["spec"])
        z = (8.0 + 4.0 * i) * P.zdiag
        h.setup(B.VTM_Z_USER, z)
        b = np.random.default_rng(100 + i).uniform(-1.0, 1.0, (2, cfg["A"].n))
        hs.append(h), Ps.append(P), zs.append(z), bs.append(b)
    tol = 1e-8
    out = B.batch_solve(hs, bs, tol)
    again = B.batch_solve(hs, bs, tol)
    for i, cfg in enumerate(cfgs):
        assert out[i]["status"] == 0 and (out[i]["relres"] <= tol).all()
        assert np.array_equal(out[i]["x"], again[i]["x"]) and np.array_equal(out[i]["iters"], again[i]["iters"])
        A = cfg["A"].to_scipy()
        sp = cfg["sys_ptr"]
        for c in range(2):
            res = bs[i][c] - A @ out[i]["x"][c]
            for s in range(cfg["nsys"]):
                lo, hi = sp[s], sp[s + 1]
                rel = np.linalg.norm(res[lo:hi]) / np.linalg.norm(bs[i][c, lo:hi])
                assert rel <= tol * 1.001 and abs(rel - out[i]["relres"][c, s]) <= 1e-6 * rel, (i, c, s, rel)
        if precision == 0:
            ro = O.Solver(Ps[i], zs[i]).run(bs[i], 100000, 10, tol, sys_ptr=sp)
            assert np.array_equal(out[i]["iters"], ro["iters"]), (i, out[i]["iters"], ro["iters"])
            for s in range(cfg["nsys"]):
                stop = int(out[i]["iters"][:, s].max())
                xo = O.Solver(Ps[i], zs[i]).run(bs[i], stop, 0, 0.0, sys_ptr=sp)["x"]
                lo, hi = sp[s], sp[s + 1]
                for c in range(2):
                    _close(out[i]["x"][c, lo:hi], xo[c, lo:hi], 1e-10, f"batch member {i} system {s} rhs {c}")
    # a member set up again (other impedances): the batch is rebuilt with them
    hs[1].setup(B.VTM_Z_USER, 2.0 * zs[1])
    third = B.batch_solve(hs, bs, tol)
    assert third[1]["status"] == 0 and (third[1]["relres"] <= tol).all()
    if precision == 0:
        ro = O.Solver(Ps[1], 2.0 * zs[1]).run(bs[1], 100000, 10, tol, sys_ptr=cfgs[1]["sys_ptr"])
        assert np.array_equal(third[1]["iters"], ro["iters"])
        assert np.array_equal(third[0]["x"], out[0]["x"])  # the other members are unchanged
    for h in hs:
        h.close()


def test_batch_solve_rejects_mixed_precision(B):
    cfg = gen.make_config("c1")
    hs = []
    for prec in (0, 1):
        h = B.VTM(device=0, precision=prec)
        h.evs_partition(cfg["A"], cfg["spec"])
        h.setup(B.VTM_Z_DIAG)
        hs.append(h)
    with pytest.raises(B.VTMError) as e:
        B.batch_solve(hs, [cfg["b"], cfg["b"]], 1e-8)
    assert e.value.code == B.VTM_ERR_INVALID


@pytest.mark.parametrize("precision", [0, 1])
def test_not_converged_returns_consistent_x_and_relres(B, precision):
    """max_sweeps reached: VTM_ERR_NOT_CONVERGED, x written, and the reported relative residual is the
    one of the returned x (recomputed on the host)."""
    cfg = gen.make_config("c2", small=True)
    P = O.Partition(cfg["A"], cfg["spec"])
    h = B.VTM(device=0, precision=precision, check_every=7, max_sweeps=60)
    h.evs_partition(cfg["A"], cfg["spec"])
    h.setup(B.VTM_Z_USER, 8.0 * P.zdiag)
    r = h.solve(cfg["b"], 1e-14)
    assert r["status"] == B.VTM_ERR_NOT_CONVERGED
    assert h.get_stats()["sweeps"] == 60 and (r["iters"] == -1).all()
    A = cfg["A"].to_scipy()
    rel = np.linalg.norm(cfg["b"][0] - A @ r["x"][0]) / np.linalg.norm(cfg["b"][0])
    assert abs(rel - r["relres"][0, 0]) <= 1e-6 * rel, (rel, r["relres"][0, 0])
    if precision == 0:
        xo = O.Solver(P, 8.0 * P.zdiag).run(cfg["b"], 60, 0, 0.0)["x"]
        _close(r["x"][0], xo[0], 1e-10, "not converged: iterate after max_sweeps")


def test_non_finite_right_side_reports_diverged(B):
    """A non-finite value in b makes the residual non-finite at the first test: VTM_ERR_DIVERGED, with
    the call returning normally."""
    cfg = gen.make_config("c1")
    h = B.VTM(device=0, check_every=5)
    h.evs_partition(cfg["A"], cfg["spec"])
    h.setup(B.VTM_Z_DIAG)
    b = cfg["b"].copy()
    b[0, 100] = np.nan
    r = h.solve(b, 1e-8, raise_on=())
    assert r["status"] == B.VTM_ERR_DIVERGED and h.get_stats()["sweeps"] == 5
    # the handle stays usable
    r2 = h.solve(cfg["b"], 1e-6)
    assert r2["status"] == 0


@pytest.mark.parametrize("mode", [0, 2])
def test_single_subgraph_is_one_cholesky_solve(B, mode):
    """One subgraph and no ports (Section 4 with N = 1): the first sweep is the exact solve."""
    A = gen.laplace2d_dirichlet(40)
    b = np.random.default_rng(5).uniform(-1.0, 1.0, (1, A.n))
    h = B.VTM(device=0, check_every=1, sweep_mode=mode)
    info = h.evs_partition(A, dict(kind="grid", dims=(40, 40, 1), parts=(1, 1, 1)))
    assert info["nsub"] == 1 and info["nports"] == 0
    h.setup(B.VTM_Z_DIAG)
    r = h.solve(b, 1e-12)
    import scipy.sparse.linalg as spl

    xs = spl.spsolve(A.to_scipy().tocsc(), b[0])
    assert r["status"] == 0 and int(r["iters"][0, 0]) == 1
    _close(r["x"][0], xs, 1e-12, "single subgraph")


def test_portless_subgraph_in_a_batch(B):
    """A batch whose first system is one subgraph without ports beside a 3-subgraph system: iterates
    equal the oracle's, and the portless system converges at the first test."""
    A1 = gen.random_geometric_graph(600, 11)
    A2 = gen.random_geometric_graph(1800, 12)
    A = gen.block_diag([A1, A2])
    coords = np.concatenate([A1.coords, A2.coords])
    spec = dict(kind="graph", coords=coords, blocks=[(0, A1.n, 1), (A1.n, A2.n, 3)])
    sp = np.array([0, A1.n, A1.n + A2.n], np.int64)
    b = np.random.default_rng(9).uniform(-1.0, 1.0, (1, A.n))
    h = B.VTM(device=0, check_every=1)
    h.evs_partition(A, spec, nsys=2, sys_ptr=sp)
    P = O.Partition(A, spec)
    assert P.port_ptr[1] == P.port_ptr[0]  # subgraph 0 has no ports
    z = 8.0 * P.zdiag
    h.setup(B.VTM_Z_USER, z)
    xg = h.run_sweeps(b, 15)
    xo = O.Solver(P, z).run(b, 15, 0, 0.0, sys_ptr=sp)["x"]
    _close(xg[0], xo[0], 1e-10, "portless batch iterates")
    r = h.solve(b, 1e-10)
    assert r["status"] == 0 and int(r["iters"][0, 0]) == 1


def test_oversized_subgraphs_are_refused_at_setup(B):
    """A subgraph whose local solve cannot keep its vectors in one CU's LDS (here 73 x 73 tiles of a
    145^2 Laplacian: 5329 local unknowns) is refused by vtm_setup with VTM_ERR_INVALID and a message
    naming the limit; the handle stays usable for a partition with more subgraphs."""
    A = gen.systems.laplace2d_dirichlet(145)
    h = B.VTM(device=0)
    h.evs_partition(A, dict(kind="grid", dims=(145, 145, 1), parts=(2, 2, 1)))
    with pytest.raises(B.VTMError) as e:
        h.setup(B.VTM_Z_DIAG)
    assert e.value.code == B.VTM_ERR_INVALID and "subgraphs too large" in str(e.value)
    h.evs_partition(A, dict(kind="grid", dims=(145, 145, 1), parts=(8, 8, 1)))
    h.setup(B.VTM_Z_DIAG)
    b = np.random.default_rng(1).uniform(-1, 1, A.n)
    r = h.solve(b, 1e-8)
    assert r["status"] == 0
