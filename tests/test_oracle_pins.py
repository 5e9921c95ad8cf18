"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these tests compares the oracle with itself: each checks a value the
paper prints, an identity that holds exactly (Theorem 4.1's sum-back), a
closed form, or a brute-force dense solve.
"""
import numpy as np
import pytest

import gen
from oracle import oracle as O
from oracle import tiny as T

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# ------------------------------------------------------------------ paper examples

def test_example_41_split_sums_back(golden):
    """Example 4.1: the printed pieces (4.1), (4.2) scatter back to (3.2) exactly (Theorem 4.1)."""
    S = T.SplitSystem(6, [dict(glob=golden["split_4_1"]["glob"], A=np.array(golden["split_4_1"]["A"], float),
                               b=np.array(golden["split_4_1"]["b"], float)),
                          dict(glob=golden["split_4_2"]["glob"], A=np.array(golden["split_4_2"]["A"], float),
                               b=np.array(golden["split_4_2"]["b"], float))], [(0, 2, 1, 0), (0, 3, 1, 1)])
    A, b = S.scatter_back()
    assert np.array_equal(A, np.array(golden["system_3_2"]["A"], float))
    assert np.array_equal(b, np.array(golden["system_3_2"]["b"], float))
    # each piece is SPD, as Theorem 4.2 allows for this split
    for pc in S.pieces:
        assert np.linalg.eigvalsh(pc["A"]).min() > 0


def test_example_51_port_augmentation(golden):
    """Example 5.1: adding Z^-1 at the ports gives exactly (5.4) and (5.5)."""
    S = T.example_41()
    K1, K2 = S.augmented(golden["example_5_1"]["Z"])
    assert np.array_equal(K1, np.array(golden["example_5_1"]["K1_5_4"], float))
    assert np.array_equal(K2, np.array(golden["example_5_1"]["K2_5_5"], float))


def test_example_51_converges_to_solution(golden):
    """Example 5.1 reaches the solution of (3.2); twins agree and currents cancel (Appendix 3 end)."""
    A = np.array(golden["system_3_2"]["A"], float)
    b = np.array(golden["system_3_2"]["b"], float)
    xs = np.linalg.solve(A, b)
    S = T.example_41()
    hist, u, w, _ = S.vtm(golden["example_5_1"]["Z"], 80)
    assert np.abs(hist[-1] - xs).max() < 1e-13
    assert np.abs(u[:, 0] - u[:, 1]).max() < 1e-13
    assert np.abs(w[:, 0] + w[:, 1]).max() < 1e-13
    # the first sweep from zero boundary variables solves (5.4) with right side (1, 2, 1.6, 1.8)
    hist1, u1, _, xs1 = S.vtm(golden["example_5_1"]["Z"], 1)
    K1 = np.array(golden["example_5_1"]["K1_5_4"], float)
    assert np.allclose(xs1[0], np.linalg.solve(K1, [1, 2, 1.6, 1.8]), rtol=0, atol=1e-15)


def test_example_71_input_impedances(golden):
    """Definition 7.1 / Example 7.1: the four printed input impedances, to 4 digits."""
    S = T.example_41()
    g = golden["example_7_1"]
    got = [T.input_impedance(S.pieces[0]["A"], 2), T.input_impedance(S.pieces[0]["A"], 3),
           T.input_impedance(S.pieces[1]["A"], 0), T.input_impedance(S.pieces[1]["A"], 1)]
    want = [g["r_in_3a"], g["r_in_4a"], g["r_in_3b"], g["r_in_4b"]]
    assert np.allclose(np.round(got, 4), want, atol=0, rtol=0)


def test_impedance_matching_effect(golden):
    """Section 7.1 / Fig. 11: after 20 iterations, Z near r_in beats Z = (1, 0.5) of Example 5.1."""
    A = np.array(golden["system_3_2"]["A"], float)
    xs = np.linalg.solve(A, np.array(golden["system_3_2"]["b"], float))
    S = T.example_41()
    rms = lambda z: np.sqrt(np.mean((S.vtm(z, 20)[0][-1] - xs) ** 2))
    matched = rms([0.2598, 0.3190])
    plain = rms([1.0, 0.5])
    assert matched < 1e-3 * plain


# --------------------------------------------------------------- the C oracle

def _tiny_random_system(n, seed, nparts):
    """Random sparse SPD M-matrix (graph Laplacian + shift) and a USER membership."""
    rng = np.random.default_rng(seed)
    A = np.zeros((n, n))
    for i in range(n):
        for j in rng.choice(n, size=3, replace=False):
            if j != i:
                w = rng.uniform(0.1, 1.0)
                A[i, j] = A[j, i] = -w
    np.fill_diagonal(A, -A.sum(1) + rng.uniform(0.01, 0.5, n))
    owner = rng.integers(0, nparts, n)
    owner[:nparts] = np.arange(nparts)  # no empty part
    S = []
    for v in range(n):
        s = {int(owner[v])}
        for u in np.nonzero(A[v])[0]:
            if u != v and owner[u] > owner[v]:
                s.add(int(owner[u]))
        S.append(sorted(s))
    s_ptr = np.concatenate([[0], np.cumsum([len(s) for s in S])]).astype(np.int64)
    s_idx = np.concatenate([np.array(s, np.int32) for s in S])
    r, c = np.nonzero(A)
    csr = gen.systems._from_coo(n, r, c, A[r, c])
    spec = dict(kind="user", s_ptr=s_ptr, s_idx=s_idx, nsub=nparts)
    return A, csr, spec


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_oracle_matches_dense_cholesky(seed):
    """Brute force: converged VTM equals a dense Cholesky solve on tiny random SPD systems."""
    n = 30 + 7 * seed
    A, csr, spec = _tiny_random_system(n, seed, 3 + seed % 3)
    b = np.random.default_rng(100 + seed).uniform(-1, 1, n)
    P = O.Partition(csr, spec)
    x_ref = T.dense_cholesky_solve(A, b)
    for topo in ("face", "complete"):
        P = O.Partition(csr, spec, topology=topo)
        s = O.Solver(P, 4.0 * P.zdiag)
        r = s.run(b, 20000, 1, 1e-14)
        assert r["iters"][0, 0] > 0
        assert np.abs(r["x"][0] - x_ref).max() <= 1e-12 * np.abs(x_ref).max()


@pytest.mark.parametrize("seed", [0, 1])
def test_oracle_sweeps_match_dense_split_system(seed):
    """The C oracle's sweeps equal the dense (5.8) iteration on the same split, sweep by sweep."""
    A, csr, spec = _tiny_random_system(24, 10 + seed, 3)
    b = np.random.default_rng(7 + seed).uniform(-1, 1, 24)
    P = O.Partition(csr, spec)
    z = 2.0 * P.zdiag
    S = T.from_oracle_partition(P, b)
    hist, _, _, _ = S.vtm(z, 12)
    s = O.Solver(P, z)
    for k in (1, 2, 5, 12):
        r = s.run(b, k, 0, 0.0)
        assert np.allclose(r["x"][0], hist[k - 1], rtol=0, atol=1e-13)


def test_single_subdomain_is_one_cholesky_solve():
    """One subdomain, no ports: a single sweep is the exact solve."""
    cfg = gen.make_config("c1")
    spec = dict(kind="grid", dims=(64, 64, 1), parts=(1, 1, 1))
    P = O.Partition(cfg["A"], spec)
    assert P.nvtl == 0 and P.nsub == 1
    s = O.Solver(P, P.zdiag)
    r = s.run(cfg["b"], 1, 1, 0.0)
    x = np.linalg.solve(cfg["A"].to_dense(), cfg["b"][0])
    assert np.abs(r["x"][0] - x).max() < 1e-12
    assert r["relres"][0, 0] < 1e-14


def _chain_split(n=9, diag=2.5):
    """Path graph split at its middle vertex into two subdomains with one VTL."""
    A = np.diag(np.full(n, diag)) - np.diag(np.ones(n - 1), 1) - np.diag(np.ones(n - 1), -1)
    m = n // 2
    S = [[0] if v < m else ([0, 1] if v == m else [1]) for v in range(n)]
    s_ptr = np.concatenate([[0], np.cumsum([len(s) for s in S])]).astype(np.int64)
    s_idx = np.concatenate([np.array(s, np.int32) for s in S])
    r, c = np.nonzero(A)
    csr = gen.systems._from_coo(n, r, c, A[r, c])
    return A, csr, dict(kind="user", s_ptr=s_ptr, s_idx=s_idx, nsub=2), m


def test_single_vtl_closed_form():
    """Two subdomains, one VTL.  With s = 1/r_in (Definition 7.1), a pass through side a maps the
    incoming wave by (1 - Z s_a)/(1 + Z s_a); two sweeps multiply the wave error by the product of
    both sides' factors, and Z = r_in,a makes u_b exact at sweep 2 and u_a exact at sweep 3."""
    A, csr, spec, m = _chain_split()
    b = np.linspace(-1.0, 1.0, A.shape[0])
    xs = np.linalg.solve(A, b)
    P = O.Partition(csr, spec)
    assert P.nvtl == 1
    ra = T.input_impedance(P.local_dense(0), m)          # port is the last local vertex of subdomain 0
    rb = T.input_impedance(P.local_dense(1), 0)          # and the first of subdomain 1
    # matched impedance: exactness after 2 / 3 sweeps
    s = O.Solver(P, np.array([ra]))
    xl2, _ = s.run_local(b, 2)
    xl3, _ = s.run_local(b, 3)
    nb0 = P.loc_ptr[1]
    assert abs(xl2[nb0 + 0] - xs[m]) < 1e-14
    assert abs(xl3[m] - xs[m]) < 1e-14
    # generic impedance: two-sweep contraction of the wave error
    z = 0.7
    s = O.Solver(P, np.array([z]))
    a_star = s.run(b, 400, 0, 0.0)["waves"][0]
    ga = (1 - z / ra) / (1 + z / ra)
    gb = (1 - z / rb) / (1 + z / rb)
    _, a4 = s.run_local(b, 4)
    _, a6 = s.run_local(b, 6)
    ratio = (a6 - a_star) / (a4 - a_star)
    assert np.allclose(ratio, ga * gb, rtol=1e-8)


@pytest.mark.parametrize("cfgname,alpha", [("c1", 16.0), ("c2s", 32.0)])
def test_scaled_wave_error_is_nonexpansive(cfgname, alpha):
    """Appendix 3: with Z^{-1/2}-scaled waves, one sweep maps the wave error by J(2W - I) with
    0 <= W <= I for a conformal split, so the scaled error never grows."""
    if cfgname == "c1":
        cfg = gen.make_config("c1")
        A, spec = cfg["A"], cfg["spec"]
    else:
        A = gen.lognormal_conductance_2d(65, seed=9)
        spec = dict(kind="grid", dims=(65, 65, 1), parts=(4, 4, 1))
    b = gen.random_rhs(A.n, 1, 5)[0]
    P = O.Partition(A, spec)
    z = alpha * P.zdiag
    s = O.Solver(P, z)
    a_star = s.run(b, 3000, 0, 0.0)["waves"][0]
    zp = z[P.port_vtl]
    a = np.zeros(P.nports)
    prev = np.linalg.norm((a - a_star) / np.sqrt(zp))
    for _ in range(150):
        _, a = s.run_local(b, 1, a)
        cur = np.linalg.norm((a - a_star) / np.sqrt(zp))
        assert cur <= prev * (1 + 1e-12) + 1e-13
        prev = cur


# ------------------------------------------------------------ partition rules

def _scatter(P):
    import scipy.sparse as sp

    rows, cols = [], []
    for k in range(P.nsub):
        b = P.loc_ptr[k]
        lv = P.loc_vtx[b:P.loc_ptr[k + 1]]
        for i in range(len(lv)):
            s, e = P.lrp[b + i], P.lrp[b + i + 1]
            rows.append(np.full(e - s, lv[i]))
            cols.append(lv[P.lcol[s:e]])
    return sp.coo_matrix((P.lval, (np.concatenate(rows), np.concatenate(cols))), shape=(P.n, P.n)).tocsr()


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c4", "c5"])
def test_split_sums_back_and_pieces_are_snnd(name):
    """Theorem 4.1 ((A2.3) sums C_se + C_ju = C, E_se + E_ju = E) and Corollary 4.1 (SNND pieces)."""
    cfg = gen.make_config(name, small=True)
    A = cfg["A"]
    P = O.Partition(A, cfg["spec"])
    M = _scatter(P)
    D = (M - A.to_scipy()).tocoo()
    scale = np.abs(A.val).max()
    assert np.abs(D.data).max(initial=0.0) <= 4e-16 * scale
    if name == "c1":  # multiplicities 2 and 4 only: the split is exact
        assert np.abs(D.data).max(initial=0.0) == 0.0
    # weak diagonal dominance with non-positive off-diagonals => SNND (Gershgorin)
    for k in range(P.nsub):
        b = P.loc_ptr[k]
        for i in range(P.loc_ptr[k + 1] - b):
            s, e = P.lrp[b + i], P.lrp[b + i + 1]
            c, v = P.lcol[s:e], P.lval[s:e]
            d = v[c == i][0]
            off = v[c != i]
            assert (off <= 0).all()
            assert d >= np.abs(off).sum() - 1e-12 * abs(d)


def test_equal_split_can_be_indefinite():
    """Negative case: splitting vertex weights equally on lognormal conductances is not conformal."""
    A = gen.lognormal_conductance_2d(65, seed=2)
    spec = dict(kind="grid", dims=(65, 65, 1), parts=(2, 2, 1))
    P = O.Partition(A, spec, split="equal")
    lam = min(np.linalg.eigvalsh(P.local_dense(k)).min() for k in range(P.nsub))
    assert lam < 0
    Pb = O.Partition(A, spec, split="branch")
    lam_b = min(np.linalg.eigvalsh(Pb.local_dense(k)).min() for k in range(Pb.nsub))
    assert lam_b > -1e-12


def test_grid_geometry_c1_c2():
    """Shared-separator tiling: 64 = 16*4 gives tiles of 17,17,17,16 vertices per axis."""
    cfg = gen.make_config("c1")
    P = O.Partition(cfg["A"], cfg["spec"])
    sizes = np.diff(P.loc_ptr)
    assert P.nsub == 16 and sizes.sum() == 4489 and P.nvtl == 402 and P.nports == 804
    assert sorted(set(sizes)) == [16 * 16, 16 * 17, 17 * 17]
    # level-two splitting at the 9 interior cross points: 4 children, 2 ports each (Fig. 7C)
    mult = P.multiplicity()
    assert (mult == 4).sum() == 9
    pv, cnt = np.unique(P.port_v, return_counts=True)
    assert (cnt[mult[pv] == 4] == 8).all()
    A2 = gen.lognormal_conductance_2d(1024, seed=2)
    P2 = O.Partition(A2, dict(kind="grid", dims=(1024, 1024, 1), parts=(32, 32, 1)))
    assert P2.nsub == 1024 and P2.nsplit == 1113025 and P2.nvtl == 65410


def test_splitmix64_reference_values():
    """splitmix64 (Steele, Lea & Flood 2014), published outputs for seed 0."""
    assert O.splitmix64_seq(0, 3) == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_rcb_boxes_cover_grid():
    cfg = gen.make_config("c3", small=True)
    P = O.Partition(cfg["A"], cfg["spec"])
    assert P.nsub == 64
    mult = P.multiplicity()
    assert mult.min() >= 1
    # every box is a full box of the grid and boxes overlap only on cut planes
    nx = cfg["spec"]["dims"][0]
    owned = np.zeros(P.nsub)
    for k in range(P.nsub):
        lv = P.loc_vtx[P.loc_ptr[k]:P.loc_ptr[k + 1]]
        x, y, z = lv % nx, (lv // nx) % nx, lv // (nx * nx)
        ext = [(a.max() - a.min() + 1) for a in (x, y, z)]
        assert np.prod(ext) == len(lv)
        owned[k] = (1.0 / mult[lv]).sum()
    assert abs(owned.sum() - cfg["A"].n) < 1e-6


def test_graph_partition_covers_edges():
    cfg = gen.make_config("c5", small=True)
    P = O.Partition(cfg["A"], cfg["spec"])
    A = cfg["A"]
    assert P.nsub == sum(b[2] for b in cfg["spec"]["blocks"])
    # subdomains never mix systems of the batch
    sp = cfg["sys_ptr"]
    for k in range(P.nsub):
        lv = P.loc_vtx[P.loc_ptr[k]:P.loc_ptr[k + 1]]
        assert np.searchsorted(sp, lv.min(), "right") == np.searchsorted(sp, lv.max(), "right")
