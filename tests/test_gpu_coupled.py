"""Coupled VTLs (Section 7.2, Theorem 7.1) on the GPU against the oracle, through the C ABI.

The coupling is SPD and tridiagonal along every interface (consecutive VTLs, by vertex, between the same
two subgraphs), so each Z_j^{-1} block is dense: the local matrices gain entries and the sweep's right
side gathers the incoming waves of coupled ports.  FP64 iterates to rounding (1e-10), FP32 to FP32
accuracy.
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
    assert emax <= tol and rel <= tol, (what, emax, rel, tol)


def _coupling(P, z, beta):
    key = P.vtl_k.astype(np.int64) * P.nsub + P.vtl_k2
    order = np.lexsort((P.vtl_v, key))
    l1, l2 = [], []
    for a, b in zip(order[:-1], order[1:]):
        if key[a] == key[b]:
            l1.append(a), l2.append(b)
    l1, l2 = np.array(l1, np.int64), np.array(l2, np.int64)
    return l1, l2, beta * np.sqrt(z[l1] * z[l2])


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name,beta", [("c2", 0.3), ("c2", -0.3), ("c3", 0.3), ("c5", 0.3)])
def test_coupled_iterates_match_oracle(B, name, beta, precision):
    cfg = gen.make_config(name, small=True)
    print(f"[coupled] {name} beta {beta} precision {precision}", flush=True)
    P = O.Partition(cfg["A"], cfg["spec"])
    z = 8.0 * P.zdiag
    cpl = _coupling(P, z, beta)
    assert len(cpl[0]) > 0
    b = cfg["b"][:2] if cfg["b"].shape[0] > 1 else cfg["b"]
    h = B.VTM(device=0, precision=precision, check_every=5)
    h.evs_partition(cfg["A"], cfg["spec"], nsys=cfg["nsys"], sys_ptr=cfg["sys_ptr"])
    h.setup_coupled(z, *cpl)
    s = O.Solver(P, z, coupling=cpl)
    for k in (1, 4, 30):
        h.reset_waves()
        xg = h.run_sweeps(b, k)
        assert h.get_stats()["sweep_mode"] == 1
        xo = s.run(b, k, 0, 0.0, sys_ptr=cfg["sys_ptr"])["x"]
        for c in range(b.shape[0]):
            _close(xg[c], xo[c], 1e-10 if precision == 0 else 2e-5, (name, k, c))
    h.close()


def test_coupled_solve_converges_like_the_oracle(B):
    """Converged coupled solve (FP64, test every 5 sweeps): same first passing sweep as the oracle and
    its iterate there; the pieces returned by vtm_get_partition are still the EVS pieces."""
    cfg = gen.make_config("c2", small=True)
    P = O.Partition(cfg["A"], cfg["spec"])
    z = 16.0 * P.zdiag
    cpl = _coupling(P, z, 0.4)
    h = B.VTM(device=0, check_every=5)
    h.evs_partition(cfg["A"], cfg["spec"])
    h.setup_coupled(z, *cpl)
    r = h.solve(cfg["b"], 1e-8)
    ro = O.Solver(P, z, coupling=cpl).run(cfg["b"], 100000, 5, 1e-8)
    assert r["status"] == 0 and int(r["iters"][0, 0]) == int(ro["iters"][0, 0])
    _close(r["x"][0], ro["x"][0], 1e-10, "coupled converged")
    lp = h.get_partition()
    assert np.array_equal(lp["lval"].view(np.uint64), P.lval.view(np.uint64))
    # uncoupled set-up on the same handle afterwards: the plain iteration again
    h.setup(B.VTM_Z_USER, z)
    r2 = h.solve(cfg["b"], 1e-8)
    ro2 = O.Solver(P, z).run(cfg["b"], 100000, 5, 1e-8)
    assert int(r2["iters"][0, 0]) == int(ro2["iters"][0, 0])
    _close(r2["x"][0], ro2["x"][0], 1e-10, "uncoupled after coupled")


def test_coupled_rejects_invalid_couplings(B):
    cfg = gen.make_config("c2", small=True)
    h = B.VTM(device=0)
    info = h.evs_partition(cfg["A"], cfg["spec"])
    P = O.Partition(cfg["A"], cfg["spec"])
    z = 8.0 * P.zdiag
    # two VTLs between different pairs of subgraphs
    key = P.vtl_k.astype(np.int64) * P.nsub + P.vtl_k2
    a = 0
    b = int(np.nonzero(key != key[0])[0][0])
    with pytest.raises(B.VTMError) as e:
        h.setup_coupled(z, [a], [b], [0.1 * z[a]])
    assert e.value.code == B.VTM_ERR_INVALID
    # a block that is not positive definite
    l1, l2, zc = _coupling(P, z, 0.3)
    with pytest.raises(B.VTMError) as e:
        h.setup_coupled(z, l1[:1], l2[:1], [2.0 * np.sqrt(z[l1[0]] * z[l2[0]])])
    assert e.value.code == B.VTM_ERR_INVALID
    with pytest.raises(B.VTMError) as e:
        h.setup_coupled(z, [0], [info["nvtl"]], [0.0])
    assert e.value.code == B.VTM_ERR_INVALID
