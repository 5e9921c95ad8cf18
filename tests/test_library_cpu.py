"""Host-side checks of libvtm that need no GPU.

* the shared library loads and exports every entry point the headers declare;
* the library's EVS partition equals the oracle's bit for bit (membership,
  local vertex lists, split values, VTLs, ports, twins, diagonal-rule Z);
* the symbolic analysis is a valid multifrontal elimination: re-running it in
  NumPy from the exported class data reproduces K = L L^T of eq. (5.8)'s local
  matrix exactly up to rounding.
"""
import os
import re

import numpy as np
import pytest

import gen
from oracle import oracle as O

from paper_0807_1949_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_declared_symbols():
    L = B.lib()
    names = set()
    for h in ("vtm.h", "vtm_debug.h"):
        src = open(os.path.join(ROOT, "include", h)).read()
        names |= set(re.findall(r"\b(vtm_[a-z_]+)\s*\(", src))
    assert names == set(B.EXPORTS)
    for nm in names:
        assert hasattr(L, nm), nm


def _host_handle():
    return B.VTM(device=-1)


def _assert_partition_equal(lp, op):
    for key in ("s_ptr", "s_idx", "loc_ptr", "loc_vtx", "lrp", "lcol", "vtl_v", "vtl_k", "vtl_k2", "port_ptr",
                "port_v", "port_other", "port_twin"):
        a, b = lp[key], getattr(op, key)
        assert a.shape == b.shape and np.array_equal(a, b.astype(a.dtype)), key
    for key in ("lval", "zdiag"):
        assert np.array_equal(lp[key].view(np.uint64), getattr(op, key).view(np.uint64)), key


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c4", "c5"])
def test_partition_bit_exact_small(name):
    cfg = gen.make_config(name, small=True)
    h = _host_handle()
    h.evs_partition(cfg["A"], cfg["spec"], nsys=cfg["nsys"], sys_ptr=cfg["sys_ptr"])
    _assert_partition_equal(h.get_partition(), O.Partition(cfg["A"], cfg["spec"]))


@pytest.mark.parametrize("split,topo", [("equal", "face"), ("branch", "complete"), ("branch", "tree")])
def test_partition_bit_exact_rules(split, topo):
    cfg = gen.make_config("c3", small=True)
    h = _host_handle()
    h.evs_partition(cfg["A"], cfg["spec"], split=split, topology=topo)
    _assert_partition_equal(h.get_partition(), O.Partition(cfg["A"], cfg["spec"], split=split, topology=topo))


def test_partition_bit_exact_graph_parts_made_connected():
    """GRAPH parts that the coordinate cut leaves in pieces: the stray pieces move to the part they
    share most edges with, in the library as in the oracle (hand-made graphs with a move and a tie)."""
    from gen import systems as S
    for edges, parts in (([(0, 1), (1, 3), (2, 4), (2, 5), (3, 4), (4, 5)], 2),
                         ([(0, 1), (1, 2), (1, 3), (2, 4), (3, 4), (4, 5)], 3)):
        u = np.array([a for a, b in edges], dtype=np.int64)
        v = np.array([b for a, b in edges], dtype=np.int64)
        diag = np.ones(6)
        np.add.at(diag, u, 1.0)
        np.add.at(diag, v, 1.0)
        coords = np.stack([np.arange(6, dtype=np.float64), np.zeros(6)], axis=1)
        A = S._assemble_weighted(6, u, v, np.ones(len(edges)), diag, coords=coords)
        spec = dict(kind="graph", coords=coords, blocks=[(0, 6, parts)])
        h = _host_handle()
        h.evs_partition(A, spec)
        _assert_partition_equal(h.get_partition(), O.Partition(A, spec))


@pytest.mark.parametrize("name", ["c1", "c2", "c4", "c3", "c5"])
def test_partition_bit_exact_full(name):
    """Every workload at full size, including the 3D RCB (4096 boxes) and the 64-system graph batch."""
    cfg = gen.make_config(name)
    h = _host_handle()
    info = h.evs_partition(cfg["A"], cfg["spec"], nsys=cfg["nsys"], sys_ptr=cfg["sys_ptr"])
    op = O.Partition(cfg["A"], cfg["spec"])
    _assert_partition_equal(h.get_partition(), op)
    if name == "c2":
        assert info["nsub"] == 1024 and info["n_split"] == 1113025 and info["nvtl"] == 65410
    if name == "c3":
        assert info["nsub"] == 4096 and info["rcb_seed"] == op.rcb_seed
    if name == "c5":
        assert info["nsys"] == 64 and info["nsub"] == sum(b[2] for b in cfg["spec"]["blocks"])


def test_partition_errors():
    A = gen.laplace2d_dirichlet(8)
    h = _host_handle()
    with pytest.raises(B.VTMError) as e:
        h.evs_partition(A, dict(kind="grid", dims=(8, 7, 1), parts=(2, 2, 1)))
    assert e.value.code == B.VTM_ERR_INVALID
    # an edge whose endpoints share no subgraph
    s_ptr = np.arange(65, dtype=np.int64)
    s_idx = (np.arange(64) >= 32).astype(np.int32)
    with pytest.raises(B.VTMError) as e:
        h.evs_partition(A, dict(kind="user", s_ptr=s_ptr, s_idx=s_idx, nsub=2))
    assert e.value.code == B.VTM_ERR_PARTITION
    # non-symmetric values
    A2 = gen.laplace2d_dirichlet(8)
    A2.val = A2.val.copy()
    A2.val[1] = -0.5
    with pytest.raises(B.VTMError) as e:
        h.evs_partition(A2, dict(kind="grid", dims=(8, 8, 1), parts=(2, 2, 1)))
    assert e.value.code == B.VTM_ERR_INVALID
    # setup on a host-only handle is a state error
    h.evs_partition(A, dict(kind="grid", dims=(8, 8, 1), parts=(2, 2, 1)))
    with pytest.raises(B.VTMError) as e:
        h.setup()
    assert e.value.code == B.VTM_ERR_STATE


def test_option_errors():
    """Options outside their documented range are rejected at vtm_create, before any device use."""
    for bad in (dict(sweep_waves=3), dict(sweep_waves=-1), dict(precision=7), dict(spin_limit=-1)):
        with pytest.raises(B.VTMError) as e:
            B.VTM(device=-1, **bad)
        assert e.value.code == B.VTM_ERR_INVALID


def _emulate_multifrontal(d, lval, dplus):
    """Re-run the device factorisation in NumPy from the class data: assemble every front from the
    scatter pairs (local CSR values) and the port diagonal, extend-add the children's update
    matrices through the relative indices, eliminate the pivot columns.  Returns L (factor order)."""
    nk, sn = d["nk"], d["sn"]
    L = np.zeros((nk, nk))
    U, fronts = {}, {}
    for s in range(d["nsn"]):
        c0, nc, m, _, ro, _, _, _, sc0, sc1 = sn[s]
        f = nc + m
        idx = np.concatenate([np.arange(c0, c0 + nc), d["ridx"][ro:ro + m].astype(np.int64)])
        fronts[s] = idx
        F = np.zeros(f * f)
        F[d["sc"][sc0:sc1, 1]] = lval[d["sc"][sc0:sc1, 0]]
        F = F.reshape(f, f)
        F[np.arange(nc), np.arange(nc)] += dplus[c0:c0 + nc]
        for c in np.nonzero(sn[:, 5] == s)[0]:
            mc = sn[c, 2]
            rel = d["rel"][sn[c, 4]:sn[c, 4] + mc].astype(np.int64)
            assert np.array_equal(idx[rel], fronts[c][sn[c, 1]:])
            F[np.ix_(rel, rel)] += np.tril(U[c])
        for kk in range(nc):
            F[kk, kk] = np.sqrt(F[kk, kk])
            F[kk + 1:, kk] /= F[kk, kk]
            F[kk + 1:, kk + 1:] -= np.tril(np.outer(F[kk + 1:, kk], F[kk + 1:, kk]))
        L[np.ix_(idx, np.arange(c0, c0 + nc))] = np.tril(F[:, :nc])
        U[s] = F[nc:, nc:]
    return L


@pytest.mark.parametrize("name,k", [("c1", 5), ("c2", 0), ("c3", 7), ("c4", 3), ("c5", 2)])
def test_symbolic_analysis_factorises(name, k):
    cfg = gen.make_config(name, small=True)
    h = _host_handle()
    h.evs_partition(cfg["A"], cfg["spec"], nsys=cfg["nsys"], sys_ptr=cfg["sys_ptr"])
    p = h.get_partition()
    d = h.debug_class(k)
    b, e = p["loc_ptr"][k], p["loc_ptr"][k + 1]
    nk = e - b
    assert nk == d["nk"]
    K = np.zeros((nk, nk))
    for i in range(nk):
        s, t = p["lrp"][b + i], p["lrp"][b + i + 1]
        K[i, p["lcol"][s:t]] = p["lval"][s:t]
    # port augmentation Z^{-1} with some positive impedances
    zadd = np.random.default_rng(0).uniform(0.5, 2.0, p["port_ptr"][k + 1] - p["port_ptr"][k])
    perm = d["perm"]
    ipos = np.argsort(perm)
    dplus = np.zeros(nk)
    for q in range(p["port_ptr"][k], p["port_ptr"][k + 1]):
        li = np.searchsorted(p["loc_vtx"][b:e], p["port_v"][q])
        dplus[ipos[li]] += zadd[q - p["port_ptr"][k]]
    L = _emulate_multifrontal(d, p["lval"][p["lrp"][b]:p["lrp"][e]], dplus)
    Kp = K[np.ix_(perm, perm)] + np.diag(dplus)
    assert np.allclose(L @ L.T, Kp, rtol=0, atol=1e-12 * np.abs(Kp).max())
    # levels: contiguous column ranges, children strictly below parents
    sn = d["sn"]
    for s in range(d["nsn"]):
        lev = sn[s, 6]
        assert d["lev_c0"][lev] <= sn[s, 0] < d["lev_c0"][lev + 1]
        if sn[s, 5] >= 0:
            assert sn[sn[s, 5], 6] > lev
    # assembly scatter covers every lower entry of K exactly once
    assert d["sc"].shape[0] == (np.count_nonzero(K) + nk) // 2


def _emulate_green_forward(d, L, port_pos):
    """Port Green's functions as the device computes them in the port-reduced setup: ports sorted by
    the postorder of their supernode, one multifrontal forward substitution carrying only the ports
    below each supernode (a contiguous column range), update blocks pushed into the parent's front
    through the relative indices, and G = sum over supernodes of Y_s^T Y_s."""
    sn, nsn = d["sn"], d["nsn"]
    par = sn[:, 5]
    col_sn = np.empty(d["nk"], np.int64)
    for s in range(nsn):
        col_sn[sn[s, 0]:sn[s, 0] + sn[s, 1]] = s
    children = [[] for _ in range(nsn)]
    for s in range(nsn):
        if par[s] >= 0:
            children[par[s]].append(s)
    post, first, cnt = np.zeros(nsn, np.int64), np.zeros(nsn, np.int64), 0
    for r in [r for r in range(nsn) if par[r] < 0]:  # iterative postorder of every tree
        st = [[r, 0]]
        first[r] = cnt
        while st:
            s, i = st[-1]
            if i < len(children[s]):
                st[-1][1] += 1
                q = children[s][i]
                first[q] = cnt
                st.append([q, 0])
            else:
                post[s] = cnt
                cnt += 1
                st.pop()
    key = post[col_sn[port_pos]]
    order = np.argsort(key, kind="stable")
    ks = key[order]
    lo = np.searchsorted(ks, first, "left")
    hi = np.searchsorted(ks, post, "right")
    p = len(port_pos)
    F = {}
    for s in range(nsn):
        nc, m = sn[s, 1], sn[s, 2]
        F[s] = np.zeros((nc + m, hi[s] - lo[s]))
    for a in range(p):
        s = col_sn[port_pos[order[a]]]
        F[s][port_pos[order[a]] - sn[s, 0], a - lo[s]] = 1.0
    G = np.zeros((p, p))
    for s in range(nsn):  # supernodes are sorted by level: children first
        c0, nc, m, ro = sn[s, 0], sn[s, 1], sn[s, 2], sn[s, 4]
        if hi[s] == lo[s]:
            continue
        L11 = L[c0:c0 + nc, c0:c0 + nc]
        rows = d["ridx"][ro:ro + m].astype(np.int64)
        Linv = np.linalg.inv(L11)
        W = L[rows][:, c0:c0 + nc] @ Linv
        T = F[s][:nc]
        Y = Linv @ T
        if m:
            U = F[s][nc:] - W @ T
            q = par[s]
            rel = d["rel"][ro:ro + m].astype(np.int64)
            F[q][np.ix_(rel, np.arange(lo[s], hi[s]) - lo[q])] = U
        js = order[lo[s]:hi[s]]
        G[np.ix_(js, js)] += Y.T @ Y
    return G


@pytest.mark.parametrize("name,k", [("c1", 5), ("c2", 0), ("c3", 7), ("c4", 3), ("c5", 2)])
def test_green_by_port_forward_substitution(name, k):
    cfg = gen.make_config(name, small=True)
    h = _host_handle()
    h.evs_partition(cfg["A"], cfg["spec"], nsys=cfg["nsys"], sys_ptr=cfg["sys_ptr"])
    p = h.get_partition()
    d = h.debug_class(k)
    b, e = p["loc_ptr"][k], p["loc_ptr"][k + 1]
    nk = e - b
    K = np.zeros((nk, nk))
    for i in range(nk):
        s, t = p["lrp"][b + i], p["lrp"][b + i + 1]
        K[i, p["lcol"][s:t]] = p["lval"][s:t]
    zadd = np.random.default_rng(1).uniform(0.5, 2.0, p["port_ptr"][k + 1] - p["port_ptr"][k])
    perm = d["perm"]
    ipos = np.argsort(perm)
    dplus = np.zeros(nk)
    for q in range(p["port_ptr"][k], p["port_ptr"][k + 1]):
        li = np.searchsorted(p["loc_vtx"][b:e], p["port_v"][q])
        dplus[ipos[li]] += zadd[q - p["port_ptr"][k]]
    L = _emulate_multifrontal(d, p["lval"][p["lrp"][b]:p["lrp"][e]], dplus)
    pv = np.unique(p["port_v"][p["port_ptr"][k]:p["port_ptr"][k + 1]])  # port vertices, ascending = group order
    port_pos = ipos[np.searchsorted(p["loc_vtx"][b:e], pv)]
    G = _emulate_green_forward(d, L, port_pos)
    Kp = K[np.ix_(perm, perm)] + np.diag(dplus)
    Gref = np.linalg.inv(Kp)[np.ix_(port_pos, port_pos)]
    assert np.allclose(G, Gref, rtol=0, atol=1e-11 * np.abs(Gref).max())
