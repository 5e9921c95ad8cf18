"""Impedance matching (Section 7.1) on the GPU: input impedances of the ports (Definition 7.1) and
the matched-Z rule, against dense computations from the oracle's split pieces and against the
oracle's iteration with the same impedances."""
import numpy as np
import pytest

import gen
from oracle import oracle as O
from oracle import tiny

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0807_1949_amd import binding

    binding.lib()
    return binding


def _augmented(P, k, z, skip_port=None):
    """Dense K_k = A~_k + sum over the subgraph's ports of Z^-1 e e^T (optionally without one port)."""
    K = P.local_dense(k)
    g = P.loc_vtx[P.loc_ptr[k]:P.loc_ptr[k + 1]]
    for p in range(P.port_ptr[k], P.port_ptr[k + 1]):
        if p != skip_port:
            i = int(np.searchsorted(g, P.port_v[p]))
            K[i, i] += 1.0 / z[P.port_vtl[p]]
    return K, g


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_input_impedance_matches_definition(B, name):
    """r_in of each port = potential for a unit inflow current at that port with the other ports
    terminated by their Z (Definition 7.1 on the dense augmented piece)."""
    cfg = gen.make_config(name, small=True)
    h = B.VTM(device=0, sweep_mode=2)
    h.evs_partition(cfg["A"], cfg["spec"])
    P = O.Partition(cfg["A"], cfg["spec"])
    z = 2.0 * P.zdiag
    h.setup(B.VTM_Z_USER, z)
    r = h.input_impedance()
    rng = np.random.default_rng(0)
    for k in rng.choice(P.nsub, size=min(P.nsub, 4), replace=False):
        for p in range(P.port_ptr[k], P.port_ptr[k + 1], 7):
            K, g = _augmented(P, k, z, skip_port=p)
            want = tiny.input_impedance(K, int(np.searchsorted(g, P.port_v[p])))
            assert abs(r[p] - want) <= 1e-10 * abs(want), (k, p, r[p], want)


def test_input_impedance_open_ports_limit(B):
    """With very large Z the other ports are effectively open and r_in tends to Definition 7.1's
    value on the bare piece (subgraphs whose piece is SPD, i.e. touching the Dirichlet boundary)."""
    cfg = gen.make_config("c1")
    h = B.VTM(device=0, sweep_mode=2)
    h.evs_partition(cfg["A"], cfg["spec"])
    P = O.Partition(cfg["A"], cfg["spec"])
    z = 1e8 * P.zdiag
    h.setup(B.VTM_Z_USER, z)
    r = h.input_impedance()
    checked = 0
    for k in range(P.nsub):
        A = P.local_dense(k)
        if np.linalg.eigvalsh(A)[0] < 1e-6:
            continue  # floating piece: the open-port input impedance is infinite
        g = P.loc_vtx[P.loc_ptr[k]:P.loc_ptr[k + 1]]
        for p in range(P.port_ptr[k], P.port_ptr[k + 1], 5):
            want = tiny.input_impedance(A, int(np.searchsorted(g, P.port_v[p])))
            assert abs(r[p] - want) <= 1e-5 * abs(want), (k, p, r[p], want)
            checked += 1
    assert checked > 10


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_matched_z_beats_diagonal_rule_and_matches_oracle(B, name):
    """VTM_Z_MATCHED: every Z lies between the clamps, the solve needs fewer sweeps than the diagonal
    rule, and its iterates are the oracle's with the same impedances."""
    cfg = gen.make_config(name, small=True)
    P = O.Partition(cfg["A"], cfg["spec"])
    sweeps = {}
    for rule in (B.VTM_Z_DIAG, B.VTM_Z_MATCHED):
        h = B.VTM(device=0, check_every=10)
        h.evs_partition(cfg["A"], cfg["spec"])
        h.setup(rule)
        r = h.solve(cfg["b"], cfg["tol"])
        assert r["status"] == 0
        sweeps[rule] = int(r["iters"].max())
        if rule == B.VTM_Z_MATCHED:
            z = h.get_z()
            assert np.all(z >= 0.25 * P.zdiag * (1 - 1e-12)) and np.all(z <= 4096 * P.zdiag * (1 + 1e-12))
            h.reset_waves()
            xg = h.run_sweeps(cfg["b"], 30)
            xo = O.Solver(P, z).run(cfg["b"], 30, 0, 0.0)["x"]
            assert np.linalg.norm(xg[0] - xo[0]) <= 1e-10 * np.linalg.norm(xo[0])
        h.close()
    assert sweeps[B.VTM_Z_MATCHED] < sweeps[B.VTM_Z_DIAG], sweeps
