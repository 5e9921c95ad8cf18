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


@pytest.mark.parametrize("name", ["c2", "c5"])
def test_oracle_relres_is_the_true_residual(name):
    """The relative residual that the oracle reports (Table 1 step 6, per system) equals
    ||b - A x||_2 / ||b||_2 recomputed from its returned x with SciPy's sparse product."""
    cfg = gen.make_config(name, small=True)
    P = O.Partition(cfg["A"], cfg["spec"])
    sp = cfg["sys_ptr"]
    A = cfg["A"].to_scipy()
    for sweeps in (1, 17):
        r = O.Solver(P, 8.0 * P.zdiag).run(cfg["b"][:2], sweeps, 0, 0.0, sys_ptr=sp)
        for c in range(r["x"].shape[0]):
            res = cfg["b"][c] - A @ r["x"][c]
            for s in range(cfg["nsys"]):
                lo, hi = sp[s], sp[s + 1]
                want = np.linalg.norm(res[lo:hi]) / np.linalg.norm(cfg["b"][c, lo:hi])
                assert abs(r["relres"][c, s] - want) <= 1e-12 * want, (c, s, r["relres"][c, s], want)


def test_face_pairing_3d_eight_way_point():
    """Fig. 7 in 3D: a 9^3 grid in 2 x 2 x 2 tiles.  The centre vertex has 8 children joined as the edges
    of a cube (12 VTLs, 3 ports per child, only tiles that differ in one tile index); vertices on a
    tile edge have 4 children with 2 ports each; face vertices 2 children with 1 port each."""
    A = gen.poisson3d_dirichlet(9)
    P = O.Partition(A, dict(kind="grid", dims=(9, 9, 9), parts=(2, 2, 2)))
    mult = P.multiplicity()
    centre = (4 * 9 + 4) * 9 + 4
    assert mult[centre] == 8 and (mult == 8).sum() == 1
    at = P.vtl_v == centre
    assert at.sum() == 12
    for k, k2 in zip(P.vtl_k[at], P.vtl_k2[at]):
        ti = np.array([k % 2, (k // 2) % 2, k // 4])
        tj = np.array([k2 % 2, (k2 // 2) % 2, k2 // 4])
        assert np.abs(ti - tj).sum() == 1
    kp = np.repeat(np.arange(P.nsub), np.diff(P.port_ptr))
    for want_mult, ports_per_child in ((8, 3), (4, 2), (2, 1)):
        vs = np.nonzero(mult == want_mult)[0]
        assert len(vs) > 0
        sel = np.isin(P.port_v, vs)
        _, cnt = np.unique(P.port_v[sel] * P.nsub + kp[sel], return_counts=True)
        assert (cnt == ports_per_child).all(), want_mult
    # the twin of a twin is the port itself, and twins sit at the same vertex in the other tile
    assert np.array_equal(P.port_twin[P.port_twin], np.arange(P.nports))
    assert np.array_equal(P.port_v[P.port_twin], P.port_v)
    assert np.array_equal(P.port_other, kp[P.port_twin])


def test_rcb_owned_sizes_within_bounds_3d_workload():
    """The 3D workload's RCB: 4096 boxes, every owned size sum 1/|S(v)| in [300, 700] (recomputed here
    from the membership), the sizes summing to n, and the seed actually used reported."""
    cfg = gen.make_config("c3")
    P = O.Partition(cfg["A"], cfg["spec"])
    assert P.nsub == 4096 and P.rcb_seed >= cfg["spec"]["seed"]
    inv = 1.0 / P.multiplicity()
    own = np.add.reduceat(inv[P.loc_vtx], P.loc_ptr[:-1])
    assert own.min() >= 300.0 and own.max() <= 700.0, (own.min(), own.max())
    assert abs(own.sum() - cfg["A"].n) <= 1e-6 * cfg["A"].n


# ------------------------------------------------------------ coupled VTLs (Section 7.2)

def _interface_coupling(P, z, beta):
    """Tridiagonal coupling along every interface: consecutive VTLs (by vertex) that join the same two
    subgraphs get Z_lm = beta sqrt(Z_l Z_m); with |beta| < 1/2 every block is SPD."""
    key = P.vtl_k.astype(np.int64) * P.nsub + P.vtl_k2
    order = np.lexsort((P.vtl_v, key))
    l1, l2 = [], []
    for a, b in zip(order[:-1], order[1:]):
        if key[a] == key[b]:
            l1.append(a), l2.append(b)
    l1, l2 = np.array(l1, np.int64), np.array(l2, np.int64)
    return l1, l2, beta * np.sqrt(z[l1] * z[l2])


def _z_matrix(nvtl, z, coupling):
    Z = np.diag(z)
    l1, l2, zc = coupling
    Z[l1, l2] = zc
    Z[l2, l1] = zc
    return Z


def test_coupled_example_51_theorem_71(golden):
    """Example 5.1 with T3 and T4 coupled by an SPD 2 x 2 Z, iterated through (5.7) itself: it converges
    to the solution of (3.2) (Theorem 7.1), twins agree and their currents cancel; with the coupling
    set to zero the (5.7) iterates equal those of (5.8) with Z = (1, 0.5)."""
    A = np.array(golden["system_3_2"]["A"], float)
    xs = np.linalg.solve(A, np.array(golden["system_3_2"]["b"], float))
    S = T.example_41()
    hist, u, w = S.vtm_coupled(np.array([[1.0, 0.3], [0.3, 0.5]]), 120)
    assert np.abs(hist[-1] - xs).max() < 1e-13
    assert np.abs(u[:, 0] - u[:, 1]).max() < 1e-13 and np.abs(w[:, 0] + w[:, 1]).max() < 1e-13
    h57, _, _ = S.vtm_coupled(np.diag(golden["example_5_1"]["Z"]), 10)
    h58 = S.vtm(golden["example_5_1"]["Z"], 10)[0]
    assert np.abs(h57 - h58).max() < 1e-14


@pytest.mark.parametrize("seed,nparts", [(0, 2), (1, 3), (2, 4)])
def test_coupled_oracle_matches_dense_57(seed, nparts):
    """The C oracle with coupled VTLs (Z_j^{-1} in the port block of (5.8), w = Z_j^{-1}(a - u),
    o = u - Z_j w) equals the unreduced (5.7) iteration sweep by sweep, on tiny random systems with a
    random dense SPD block per pair of subgraphs."""
    A, csr, spec = _tiny_random_system(26 + 4 * seed, 20 + seed, nparts)
    b = np.random.default_rng(30 + seed).uniform(-1, 1, A.shape[0])
    P = O.Partition(csr, spec)
    rng = np.random.default_rng(40 + seed)
    z = rng.uniform(0.5, 2.0, P.nvtl) * P.zdiag
    key = P.vtl_k.astype(np.int64) * P.nsub + P.vtl_k2
    l1, l2, zc = [], [], []
    for kk in np.unique(key):
        ls = np.nonzero(key == kk)[0]
        m = len(ls)
        if m < 2:
            continue
        M = rng.standard_normal((m, m))
        C = M @ M.T / m * np.sqrt(np.outer(z[ls], z[ls])) * 0.3
        for i in range(m):
            for j in range(i + 1, m):
                l1.append(ls[i]), l2.append(ls[j]), zc.append(C[i, j])
        z[ls] += np.diag(C)
    cpl = (np.array(l1, np.int64), np.array(l2, np.int64), np.array(zc))
    assert len(cpl[0]) > 0
    Zv = _z_matrix(P.nvtl, z, cpl)
    assert np.linalg.eigvalsh(Zv).min() > 0
    hist, _, _ = T.from_oracle_partition(P, b).vtm_coupled(Zv, 15)
    s = O.Solver(P, z, coupling=cpl)
    for k in (1, 2, 6, 15):
        r = s.run(b, k, 0, 0.0)
        assert np.abs(r["x"][0] - hist[k - 1]).max() <= 1e-13 * np.abs(hist[k - 1]).max(), k


def test_coupled_diagonal_reproduces_uncoupled():
    """A coupled set-up with no off-diagonal entries reproduces the diagonal-Z iterates (to rounding:
    the diagonal block is inverted through its Cholesky factor)."""
    cfg = gen.make_config("c2", small=True)
    P = O.Partition(cfg["A"], cfg["spec"])
    z = 8.0 * P.zdiag
    e = np.zeros(0, np.int64)
    x0 = O.Solver(P, z).run(cfg["b"], 30, 0, 0.0)["x"][0]
    x1 = O.Solver(P, z, coupling=(e, e, np.zeros(0))).run(cfg["b"], 30, 0, 0.0)["x"][0]
    assert np.abs(x1 - x0).max() <= 1e-13 * np.abs(x0).max()


@pytest.mark.parametrize("beta", [-0.3, 0.3])
def test_coupled_converges_and_is_nonexpansive(beta):
    """Theorem 7.1 on a 2D grid in 3 x 3 tiles with SPD tridiagonal coupling along every interface: the
    iteration reaches the dense Cholesky solution, and the wave error measured in the norm
    e^T Zhat^{-1} e (Zhat: the block-diagonal port impedance, twin-symmetric) never grows (the
    argument of Appendix 3 with Z_j a matrix: one sweep maps the scaled error by J(2W - I))."""
    A = gen.lognormal_conductance_2d(25, seed=7, shift=1e-2)
    spec = dict(kind="grid", dims=(25, 25, 1), parts=(3, 3, 1))
    P = O.Partition(A, spec)
    z = 8.0 * P.zdiag
    cpl = _interface_coupling(P, z, beta)
    b = np.random.default_rng(3).uniform(-1, 1, A.n)
    s = O.Solver(P, z, coupling=cpl)
    r = s.run(b, 50000, 1, 1e-13)
    xref = T.dense_cholesky_solve(A.to_dense(), b)
    assert r["iters"][0, 0] > 0 and np.abs(r["x"][0] - xref).max() <= 1e-10 * np.abs(xref).max()
    # the port-level inverse impedance: Zhat^{-1} restricted to each subgraph's ports of one group
    Zv = _z_matrix(P.nvtl, z, cpl)
    Y = np.linalg.inv(Zv)  # block diagonal like Zv
    kp = np.repeat(np.arange(P.nsub), np.diff(P.port_ptr))
    same = kp[:, None] == kp[None, :]
    Yp = Y[np.ix_(P.port_vtl, P.port_vtl)] * same
    assert np.allclose(Yp[np.ix_(P.port_twin, P.port_twin)], Yp, rtol=0, atol=1e-14 * np.abs(Yp).max())
    a_star = s.run(b, 6000, 0, 0.0)["waves"][0]
    prev = np.inf
    for k in range(1, 60):
        e = s.run(b, k, 0, 0.0)["waves"][0] - a_star
        nrm = float(e @ Yp @ e)
        assert nrm <= prev * (1 + 1e-9) + 1e-28, (k, nrm, prev)
        prev = nrm


def test_tree_topology_is_a_spanning_tree_of_the_face_pairs():
    """TREE (repeated binary splitting): at every split vertex the VTLs are |S(v)| - 1 pairs of the FACE
    topology that connect all children of v, so no cycle of VTLs meets at one vertex.  Checked on a 3D
    RCB partition, whose corner vertices have up to eight children and FACE cycles."""
    import gen
    from oracle import oracle as O
    cfg = gen.make_config("c3", small=True)
    face = O.Partition(cfg["A"], cfg["spec"], topology="face")
    tree = O.Partition(cfg["A"], cfg["spec"], topology="tree")
    assert np.array_equal(face.s_ptr, tree.s_ptr) and np.array_equal(face.s_idx, tree.s_idx)
    fset = set(zip(face.vtl_v.tolist(), face.vtl_k.tolist(), face.vtl_k2.tolist()))
    tv = tree.vtl_v
    mult = np.diff(tree.s_ptr)
    assert np.array_equal(np.bincount(tv, minlength=tree.n), np.maximum(mult - 1, 0))
    cycles = 0
    for v in np.nonzero(mult >= 3)[0]:
        sel = tv == v
        kids = tree.s_idx[tree.s_ptr[v]:tree.s_ptr[v + 1]].tolist()
        par = {k: k for k in kids}

        def root(k):
            while par[k] != k:
                k = par[k]
            return k
        for k1, k2 in zip(tree.vtl_k[sel].tolist(), tree.vtl_k2[sel].tolist()):
            assert (int(v), k1, k2) in fset
            assert root(k1) != root(k2)  # adding it closes no cycle
            par[root(k1)] = root(k2)
        assert len({root(k) for k in kids}) == 1
        cycles += int((face.vtl_v == v).sum()) - (len(kids) - 1)
    assert cycles > 0  # FACE had cycles here that the tree drops
    # ports and twins follow the VTLs: two ports per VTL, each the other's twin
    assert len(tree.port_v) == 2 * tree.nvtl and np.array_equal(tree.port_twin[tree.port_twin], np.arange(2 * tree.nvtl))


def _hand_graph(n, edges, xs):
    """Laplacian of the listed unit-weight edges plus I, with x coordinates xs (y = 0)."""
    from gen import systems as S
    u = np.array([a for a, b in edges], dtype=np.int64)
    v = np.array([b for a, b in edges], dtype=np.int64)
    w = np.ones(len(edges))
    diag = np.ones(n)
    np.add.at(diag, u, w)
    np.add.at(diag, v, w)
    coords = np.stack([np.asarray(xs, dtype=np.float64), np.zeros(n)], axis=1)
    return S._assemble_weighted(n, u, v, w, diag, coords=coords)


def test_graph_parts_are_made_connected_worked_example():
    """A coordinate cut leaves vertex 2 in the left part although its edges all lead right; it moves
    to the part it shares most edges with.  Worked by hand: left part {0, 1}, right {2, .., 5}; the
    cut edge 1-3 makes vertex 1 the only split vertex (children in both parts).  Then a tie: vertex 3
    of the middle part touches the left and the right part by one edge each and goes to the left
    (smaller id)."""
    from oracle import oracle as O
    A = _hand_graph(6, [(0, 1), (1, 3), (2, 4), (2, 5), (3, 4), (4, 5)], [0, 1, 2, 3, 4, 5])
    P = O.Partition(A, dict(kind="graph", coords=A.coords, blocks=[(0, 6, 2)]))
    assert P.s_ptr.tolist() == [0, 1, 3, 4, 5, 6, 7]
    assert P.s_idx.tolist() == [0, 0, 1, 1, 1, 1, 1]
    # three parts of two vertices: {0, 1}, {2, 3}, {4, 5}; 2 - 3 is no edge, so the middle part falls
    # into {2} (kept: smaller vertex at equal size) and {3}, which has one edge left (1 - 3) and one
    # right (3 - 4): it goes left.  Vertex 1 (part 0) has a neighbour in part 1 (vertex 2): split.
    B = _hand_graph(6, [(0, 1), (1, 2), (1, 3), (2, 4), (3, 4), (4, 5)], [0, 1, 2, 3, 4, 5])
    Q = O.Partition(B, dict(kind="graph", coords=B.coords, blocks=[(0, 6, 3)]))
    owner = Q.s_idx[Q.s_ptr[:-1]]
    assert owner.tolist() == [0, 0, 1, 0, 2, 2]
    assert Q.s_idx[Q.s_ptr[1]:Q.s_ptr[2]].tolist() == [0, 1]  # vertex 1: its own part and vertex 2's
    assert Q.s_idx[Q.s_ptr[3]:Q.s_ptr[4]].tolist() == [0, 2]  # vertex 3: moved to 0, split into 2


def test_graph_parts_are_connected():
    """After the coordinate cut every part's owned vertices form one connected piece, up to
    components of A lying wholly inside the part (which have no ports); every part keeps vertices."""
    import scipy.sparse as sp
    import gen
    from oracle import oracle as O
    cfg = gen.make_config("c5", small=True)
    A = cfg["A"]
    P = O.Partition(A, cfg["spec"])
    M = A.to_scipy()
    owner = P.s_idx[P.s_ptr[:-1]]
    assert np.array_equal(np.unique(owner), np.arange(P.nsub))
    for k in range(P.nsub):
        vs = np.nonzero(owner == k)[0]
        nc, lab = sp.csgraph.connected_components(M[vs][:, vs], directed=False)
        keep = np.argmax(np.bincount(lab))
        for c in range(nc):
            if c != keep:
                C = vs[lab == c]
                assert (owner[M[C].indices] == k).all()  # a component of A, no edge leaves the part
