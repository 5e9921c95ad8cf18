"""GPU parity: libvtm (HIP, gfx950) against the CPU oracle, through the C ABI.

Tolerances.  Both sides run the same iteration in FP64 from the same split:
iterates at a fixed sweep count differ only by rounding order (factor
ordering, inverted diagonal blocks), which grows at most linearly with the
sweep count for a nonexpansive iteration (Appendix 3), so 1e-10 relative is a
generous bound for <= a few hundred sweeps.  Converged solutions are compared
at the same stopping rule; FP32 sweeps with FP64 refinement are compared with
the FP64 oracle's converged solution.
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


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _close(a, b, tol, what=""):
    """Element by element, max |a - b| <= tol * max |b|, and the relative 2-norm <= tol."""
    a, b = np.asarray(a), np.asarray(b)
    emax = float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
    assert emax <= tol, (what, "element-wise", emax, tol)
    assert _rel(a, b) <= tol, (what, "norm", _rel(a, b), tol)


def _setup(B, cfg, precision=0, check_every=1, z_scale=1.0, **kw):
    h = B.VTM(device=0, precision=precision, check_every=check_every, **kw)
    h.evs_partition(cfg["A"], cfg["spec"], nsys=cfg["nsys"], sys_ptr=cfg["sys_ptr"])
    P = O.Partition(cfg["A"], cfg["spec"])
    z = z_scale * P.zdiag
    h.setup(B.VTM_Z_USER, z)
    return h, P, z


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c4", "c5"])
def test_iterates_match_oracle(B, name):
    """Merged potentials after 1, 3 and 40 sweeps from zero waves, every config (small sizes)."""
    cfg = gen.make_config(name, small=True)
    print(f"[parity] iterates {name}", flush=True)
    h, P, z = _setup(B, cfg, z_scale=8.0)
    s = O.Solver(P, z)
    b = cfg["b"][:2] if name in ("c3", "c5") else cfg["b"][:1]
    for k in (1, 3, 40):
        h.reset_waves()
        xg = h.run_sweeps(b, k)
        xo = s.run(b, k, 0, 0.0, sys_ptr=cfg["sys_ptr"])["x"]
        for r in range(b.shape[0]):
            _close(xg[r], xo[r], 1e-10, (name, k, r, _rel(xg[r], xo[r])))


def test_c1_converged_matches_oracle(B):
    """C1 as specified: diagonal-rule Z, tol 1e-10; same sweep count and x within 1e-8 of the oracle."""
    cfg = gen.make_config("c1")
    h = B.VTM(device=0, check_every=1)
    h.evs_partition(cfg["A"], cfg["spec"])
    h.setup(B.VTM_Z_DIAG)
    r = h.solve(cfg["b"], 1e-10)
    P = O.Partition(cfg["A"], cfg["spec"])
    ro = O.Solver(P, P.zdiag).run(cfg["b"], 100000, 1, 1e-10)
    assert r["status"] == 0
    assert abs(int(r["iters"][0, 0]) - int(ro["iters"][0, 0])) <= 1
    _close(r["x"][0], ro["x"][0], 1e-8)
    assert r["relres"][0, 0] <= 1e-10


@pytest.mark.parametrize("precision", [0, 1])
def test_c2_small_converged(B, precision):
    """Lognormal conductances, 4x4 tiles of 33: FP64 and FP32+IR reach 1e-8 and match the oracle."""
    cfg = gen.make_config("c2", small=True)
    h, P, z = _setup(B, cfg, precision=precision, check_every=10, z_scale=32.0)
    r = h.solve(cfg["b"], 1e-8)
    assert r["status"] == 0 and r["relres"][0, 0] <= 1e-8
    ro = O.Solver(P, z).run(cfg["b"], 100000, 10, 1e-12)
    assert ro["relres"][0, 0] <= 1e-12
    x_exact = ro["x"][0]
    # the residual bounds the error by the condition number; measure against a tight oracle solve
    A = cfg["A"].to_scipy()
    err = _rel(r["x"][0], x_exact)
    res = np.linalg.norm(cfg["b"][0] - A @ r["x"][0]) / np.linalg.norm(cfg["b"][0])
    assert res <= 1e-8
    assert err <= 1e-5, err
    if precision == 0:
        ro8 = O.Solver(P, z).run(cfg["b"], 100000, 10, 1e-8)
        _close(r["x"][0], ro8["x"][0], 1e-8)
        assert int(r["iters"][0, 0]) == int(ro8["iters"][0, 0])


@pytest.mark.parametrize("mode", [1, 2])
def test_multi_rhs_and_batch(B, mode):
    """C5 small: a batch of 4 independent systems x 4 RHS, per-system convergence with the done mask:
    each system stops sweeping at the test where all its right-hand sides pass, so its x is the
    oracle's iterate after that system's own sweep count (substitution and port-reduced sweeps)."""
    cfg = gen.make_config("c5", small=True)
    h, P, z = _setup(B, cfg, check_every=10, z_scale=8.0, sweep_mode=mode)
    r = h.solve(cfg["b"], 1e-8)
    assert r["status"] == 0 and h.get_stats()["sweep_mode"] == mode
    assert r["iters"].shape == (4, cfg["nsys"]) and (r["iters"] > 0).all()
    ro = O.Solver(P, z).run(cfg["b"], 100000, 10, 1e-8, sys_ptr=cfg["sys_ptr"])
    assert (r["relres"] <= 1e-8).all()
    assert np.array_equal(r["iters"], ro["iters"])
    sp = cfg["sys_ptr"]
    stop = r["iters"].max(axis=0)  # per system
    assert len(set(stop.tolist())) > 1  # the systems stop at different sweeps
    A = cfg["A"].to_scipy()
    for s in range(cfg["nsys"]):
        xo = O.Solver(P, z).run(cfg["b"], int(stop[s]), 0, 0.0, sys_ptr=sp)["x"]
        lo, hi = sp[s], sp[s + 1]
        for c in range(4):
            _close(r["x"][c, lo:hi], xo[c, lo:hi], 1e-10, (s, c))
            res = np.linalg.norm(cfg["b"][c, lo:hi] - (A @ r["x"][c])[lo:hi]) / np.linalg.norm(cfg["b"][c, lo:hi])
            assert abs(res - r["relres"][c, s]) <= 1e-6 * res, (s, c, res, r["relres"][c, s])


def test_checkpoint_resume_bitwise(B):
    """k1 sweeps, export the waves, import into a fresh handle, k2 sweeps == k1 + k2 uninterrupted."""
    cfg = gen.make_config("c2", small=True)
    h1, P, z = _setup(B, cfg, z_scale=16.0)
    full = h1.run_sweeps(cfg["b"], 30)
    h1.reset_waves()
    h1.run_sweeps(cfg["b"], 12)
    a = h1.get_waves(1)
    h2, _, _ = _setup(B, cfg, z_scale=16.0)
    h2.set_waves(a)
    resumed = h2.run_sweeps(cfg["b"], 18)
    assert np.array_equal(resumed, full)


def test_device_pointers(B):
    """b and x as device (torch) tensors give the same result as host arrays."""
    import torch

    cfg = gen.make_config("c1")
    h, P, z = _setup(B, cfg, check_every=5, z_scale=16.0)
    rh = h.solve(cfg["b"], 1e-10)
    bd = torch.tensor(cfg["b"], dtype=torch.float64, device="cuda")
    rd = h.solve(bd, 1e-10)
    assert np.array_equal(rd["x"].cpu().numpy(), rh["x"])


def test_not_spd_detected(B):
    """A non-conformal split (EQUAL rule on lognormal weights) with tiny port terms is rejected."""
    A = gen.lognormal_conductance_2d(65, seed=2)
    spec = dict(kind="grid", dims=(65, 65, 1), parts=(2, 2, 1))
    h = B.VTM(device=0)
    info = h.evs_partition(A, spec, split="equal")
    with pytest.raises(B.VTMError) as e:
        h.setup(B.VTM_Z_USER, np.full(info["nvtl"], 1e12))
    assert e.value.code == B.VTM_ERR_NOT_SPD


def test_invalid_inputs(B):
    cfg = gen.make_config("c1")
    h = B.VTM(device=0)
    with pytest.raises(B.VTMError) as e:
        h.solve(cfg["b"], 1e-8)  # before partition/setup
    assert e.value.code == B.VTM_ERR_STATE
    info = h.evs_partition(cfg["A"], cfg["spec"])
    with pytest.raises(B.VTMError) as e:
        h.setup(B.VTM_Z_USER, np.full(info["nvtl"], -1.0))
    assert e.value.code == B.VTM_ERR_INVALID


def test_c2_full_iterates(B):
    """C2 at full size (1024^2, 32x32 tiles), the benchmark's FP64 launch: 20 sweeps vs the oracle."""
    cfg = gen.make_config("c2")
    print("[parity] c2 full", flush=True)
    h, P, z = _setup(B, cfg, z_scale=64.0)
    xg = h.run_sweeps(cfg["b"], 20)
    xo = O.Solver(P, z).run(cfg["b"], 20, 0, 0.0)["x"]
    _close(xg[0], xo[0], 1e-10)


def test_graph_replay_matches_eager(B):
    """Sweep batches replayed from captured HIP graphs (19 sweeps per test: two 8-sweep graph replays
    plus 3 direct launches, so both starting wave buffers are captured; several replays with host
    synchronisation between them) give bitwise the eager result."""
    cfg = gen.make_config("c2", small=True)
    out = []
    for gm in (0, 1):
        h, P, z = _setup(B, cfg, check_every=19, z_scale=16.0, graph_mode=gm)
        r1 = h.solve(cfg["b"], 1e-8)
        r2 = h.solve(cfg["b"], 1e-8)
        out.append((r1["x"], r2["x"], r1["iters"].copy()))
        h.close()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    assert np.array_equal(out[0][0], out[0][1]) and np.array_equal(out[0][2], out[1][2])


def test_autotune_then_solve(B):
    """The autotuner picks a launch shape; the solve with it still matches the oracle (3D, 8 RHS)."""
    cfg = gen.make_config("c3", small=True)
    h, P, z = _setup(B, cfg, check_every=10, z_scale=8.0)
    ch = h.autotune(8)
    assert ch["rhs_per_block"] in (1, 2, 4, 8) and ch["sweep_threads"] in (128, 256, 512) and ch["sweep_mode"] in (1, 2)
    r = h.solve(cfg["b"], 1e-8)
    assert r["status"] == 0
    ro = O.Solver(P, z).run(cfg["b"], 100000, 10, 1e-8)
    # every RHS passes the test at the oracle's sweep; the solve runs until the last one passes,
    # so x is compared with the oracle's iterate after that many sweeps
    last = int(r["iters"].max())
    xo = O.Solver(P, z).run(cfg["b"], last, 0, 0.0)["x"]
    for c in range(8):
        assert int(r["iters"][c, 0]) == int(ro["iters"][c, 0])
        _close(r["x"][c], xo[c], 1e-10)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("name", ["c2", "c3", "c5"])
def test_sweep_variants_match_oracle(B, variant, name, precision):
    """The substitution sweep's own loop (sweep_mode 1: local forward/back solve every sweep), both
    forward-substitution variants, gives the oracle's iterates: FP64 to rounding, FP32 to FP32
    accuracy (2 RHS)."""
    cfg = gen.make_config(name, small=True)
    h, P, z = _setup(B, cfg, z_scale=8.0, sweep_variant=variant, sweep_mode=1, precision=precision)
    b = cfg["b"][:2] if cfg["b"].shape[0] > 1 else np.vstack([cfg["b"], cfg["b"][:, ::-1]])
    xg = h.run_sweeps(b, 25)
    assert h.get_stats()["sweep_mode"] == 1
    xo = O.Solver(P, z).run(b, 25, 0, 0.0, sys_ptr=cfg["sys_ptr"])["x"]
    if precision == 1:
        for r in range(2):
            _close(xg[r], xo[r], 2e-5, (name, variant, r))
        return
    for r in range(2):
        _close(xg[r], xo[r], 1e-10)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name", ["c1", "c2", "c4", "c5"])
def test_port_reduced_sweeps_match_substitution(B, name, precision):
    """Port-reduced sweeps (u = c + G Z^-1 a) give the oracle's iterates and the same converged
    solution and sweep count as substitution sweeps."""
    cfg = gen.make_config(name, small=True)
    b = cfg["b"][:2] if cfg["b"].shape[0] > 1 else cfg["b"]
    hs, P, z = _setup(B, cfg, z_scale=8.0, sweep_mode=2, precision=precision, check_every=10)
    if precision == 0:
        xg = hs.run_sweeps(b, 30)
        xo = O.Solver(P, z).run(b, 30, 0, 0.0, sys_ptr=cfg["sys_ptr"])["x"]
        for r in range(b.shape[0]):
            _close(xg[r], xo[r], 1e-10)
    hs.reset_waves()
    rs = hs.solve(b, 1e-8)
    assert hs.get_stats()["sweep_mode"] == 2
    ht, _, _ = _setup(B, cfg, z_scale=8.0, sweep_mode=1, precision=precision, check_every=10)
    rt = ht.solve(b, 1e-8)
    assert ht.get_stats()["sweep_mode"] == 1
    assert rs["status"] == 0 and rt["status"] == 0
    assert np.array_equal(rs["iters"], rt["iters"]) or precision == 1
    for r in range(b.shape[0]):
        _close(rs["x"][r], rt["x"][r], 1e-10 if precision == 0 else 1e-6)


@pytest.mark.parametrize("W", [1, 2])
@pytest.mark.parametrize("R", [1, 2, 4, 8])
@pytest.mark.parametrize("name", ["c3", "c5"])
def test_port_reduced_multi_rhs_match_oracle(B, name, R, W):
    """Port-reduced sweeps with 8 right-hand sides in groups of R per wave (matrix-core y_I += B x_J,
    vector-unit y_J += B^T x_I), one or two waves per subgraph: FP64 iterates equal the oracle's to
    rounding for every RHS; FP32 iterates to FP32 accuracy."""
    cfg = gen.make_config(name, small=True)
    rng = np.random.default_rng(77)
    b = rng.uniform(-1.0, 1.0, (8, cfg["A"].n))
    print(f"[parity] port-reduced multi-RHS {name} R={R} W={W}", flush=True)
    P = O.Partition(cfg["A"], cfg["spec"])
    z = 8.0 * P.zdiag
    xo = O.Solver(P, z).run(b, 23, 0, 0.0, sys_ptr=cfg["sys_ptr"])["x"]
    for precision, tol in ((0, 1e-10), (1, 2e-5)):
        h = B.VTM(device=0, precision=precision, check_every=10, sweep_mode=2, rhs_per_block=R, sweep_waves=W)
        h.evs_partition(cfg["A"], cfg["spec"], nsys=cfg["nsys"], sys_ptr=cfg["sys_ptr"])
        h.setup(B.VTM_Z_USER, z)
        xg = h.run_sweeps(b, 23)
        assert h.get_stats()["sweep_mode"] == 2
        for c in range(8):
            _close(xg[c], xo[c], tol, (name, R, precision, c))
        h.close()


@pytest.mark.parametrize("W", [1, 2])
def test_port_reduced_sweeps_bitwise_repeatable(B, W):
    """Two runs of the same port-reduced sweeps (FP32 and FP64, 8 RHS, one or two waves per subgraph)
    give bitwise equal results: every sum of the kernel has a fixed order."""
    cfg = gen.make_config("c3", small=True)
    b = cfg["b"]
    P = O.Partition(cfg["A"], cfg["spec"])
    for precision in (0, 1):
        outs = []
        for rep in range(2):
            h = B.VTM(device=0, precision=precision, check_every=10, sweep_mode=2, persistent=1, sweep_waves=W)
            h.evs_partition(cfg["A"], cfg["spec"])
            h.setup(B.VTM_Z_USER, 8.0 * P.zdiag)
            outs.append((h.run_sweeps(b, 17), h.get_waves(b.shape[0])))
            h.close()
        assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_adaptive_check_cadence(B):
    """check_every = 0 places the tests by the observed contraction rate: same solution quality, and the
    reported sweep count is one where the tolerance holds."""
    cfg = gen.make_config("c2", small=True)
    h, P, z = _setup(B, cfg, check_every=0, z_scale=32.0)
    r = h.solve(cfg["b"], 1e-8)
    assert r["status"] == 0 and r["relres"][0, 0] <= 1e-8
    st = h.get_stats()
    ro = O.Solver(P, z).run(cfg["b"], int(st["sweeps"]), 0, 0.0)
    assert ro["relres"][0, 0] <= 1e-8
    _close(r["x"][0], ro["x"][0], 1e-10)
    ro1 = O.Solver(P, z).run(cfg["b"], 100000, 1, 1e-8)
    assert st["sweeps"] <= 1.25 * int(ro1["iters"][0, 0]) + 10


@pytest.mark.parametrize("name,nrhs", [("c2", 1), ("c2", 2), ("c5", 1)])
def test_persistent_sweeps_match_per_sweep_launches(B, name, nrhs):
    """FP32 port-reduced sweeps in one persistent launch (G_k rows on chip, tagged wave words) give
    the oracle's iterates to FP32 accuracy, the per-sweep kernel's waves to rounding, and the same
    converged solve."""
    cfg = gen.make_config(name, small=True)
    b = np.vstack([cfg["b"][:1]] * nrhs) if nrhs > 1 else cfg["b"][:1].copy()
    if nrhs > 1:
        b[1] = b[1][::-1]
    print(f"[parity] persistent {name} nrhs={nrhs}", flush=True)
    out = {}
    for pers in (0, 1):
        # fixed test cadence: the adaptive one depends on measured timings
        h, P, z = _setup(B, cfg, precision=1, z_scale=8.0, sweep_mode=2, persistent=pers, check_every=10)
        x = h.run_sweeps(b, 37)
        ran_persistent = h.get_stats()["persistent"]
        w = h.get_waves(nrhs)
        h.reset_waves()
        r = h.solve(b, 1e-8)
        out[pers] = (x, w, r, h.get_stats())
        h.close()
        assert ran_persistent == (1 if pers == 0 else 0)
    (x0, w0, r0, s0), (x1, w1, r1, s1) = out[0], out[1]
    assert s0["sweep_mode"] == 2 and s1["sweep_mode"] == 2 and s0["persistent"] == 1 and s1["persistent"] == 0
    xo = O.Solver(P, z).run(b, 37, 0, 0.0, sys_ptr=cfg["sys_ptr"])["x"]
    for c in range(nrhs):
        _close(x0[c], xo[c], 2e-5, (c, _rel(x0[c], xo[c])))
        _close(x0[c], x1[c], 2e-5)
        _close(w0[c], w1[c], 2e-5)
    assert r0["status"] == 0 and r1["status"] == 0
    assert np.all(np.abs(r0["iters"] - r1["iters"]) <= 10)
    for c in range(nrhs):
        _close(r0["x"][c], r1["x"][c], 1e-6)


@pytest.mark.parametrize("call", ["solve", "run_sweeps"])
def test_persistent_wait_timeout_is_reported_and_recoverable(B, call):
    """A persistent launch whose wave-word waits give up after one re-read (spin_limit=1) ends
    normally (every other wait gives up too), the call reports VTM_ERR_HIP, and the device flag is
    cleared: the same handle then fails the same way again, not from a stale flag alone, and a
    handle with the default limit solves the system."""
    cfg = gen.make_config("c2", small=True)
    b = cfg["b"][:1].copy()
    print(f"[parity] persistent timeout via {call}", flush=True)
    h, P, z = _setup(B, cfg, precision=1, z_scale=8.0, sweep_mode=2, check_every=10, spin_limit=1)
    for _ in range(2):
        with pytest.raises(B.VTMError) as e:
            if call == "solve":
                h.solve(b, 1e-8)
            else:
                h.run_sweeps(b, 200)
        assert e.value.code == B.VTM_ERR_HIP and "timed out" in str(e.value), str(e.value)
        assert h.get_stats()["persistent"] == 1
        h.reset_waves()
    h.close()
    h, P, z = _setup(B, cfg, precision=1, z_scale=8.0, sweep_mode=2, check_every=10)
    r = h.solve(b, 1e-8)
    st = h.get_stats()
    h.close()
    assert r["status"] == 0 and st["persistent"] == 1
    A = cfg["A"].to_scipy()
    assert np.linalg.norm(b[0] - A @ r["x"][0]) <= 1e-8 * np.linalg.norm(b[0]) * 1.01


@pytest.mark.parametrize("name,precision", [("c2", 0), ("c1", 0), ("c3", 0), ("c2", 1), ("c3", 1), ("c4", 1), ("c5", 1)])
def test_test_solve_from_green_columns_matches_substitution(B, name, precision):
    """The convergence test's local solve from the stored Green's columns (y_b + Y w, then the
    backward substitution) gives the iterate of the substitution solve: FP64 solve == run_sweeps
    over the same sweep count (to rounding) == the oracle's iterate at that count; FP32 sweeps with
    refinement: the returned x has the requested true residual."""
    cfg = gen.make_config(name, small=True)
    print(f"[parity] green-column test solve {name} precision {precision}", flush=True)
    h, P, z = _setup(B, cfg, precision=precision, z_scale=8.0, sweep_mode=2, check_every=10)
    b = cfg["b"][:2] if name == "c3" else cfg["b"][:1]
    tol = 1e-6
    r = h.solve(b, tol)
    assert r["status"] == 0 and h.get_stats()["sweep_mode"] == 2
    if precision == 0:
        n = int(r["iters"].max())
        h.reset_waves()
        xs = h.run_sweeps(b, n)
        xo = O.Solver(P, z).run(b, n, 0, 0.0, sys_ptr=cfg["sys_ptr"])["x"]
        for q in range(b.shape[0]):
            _close(r["x"][q], xs[q], 1e-12, (q, _rel(r["x"][q], xs[q])))
            _close(r["x"][q], xo[q], 1e-10, (q, _rel(r["x"][q], xo[q])))
    else:
        A = cfg["A"].to_scipy()
        for q in range(b.shape[0]):
            res = np.linalg.norm(b[q] - A @ r["x"][q]) / np.linalg.norm(b[q])
            assert res <= 2 * tol, (q, res)
