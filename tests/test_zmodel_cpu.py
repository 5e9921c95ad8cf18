"""Host-side pieces of the learned-impedance pipeline (no GPU)."""
import numpy as np

import gen
from paper_0807_1949_amd import binding as B
from paper_0807_1949_amd import zmodel as Zm


def test_port_vtl_and_colouring():
    cfg = gen.make_config("c4", small=True)
    h = B.VTM(device=-1)
    info = h.evs_partition(cfg["A"], cfg["spec"])
    p = h.get_partition()
    pv = Zm.port_vtl(p, info["nsub"])
    # each VTL owns exactly its two ports, and they are twins
    assert np.array_equal(np.bincount(pv, minlength=info["nvtl"]), np.full(info["nvtl"], 2))
    assert np.array_equal(pv[p["port_twin"]], pv)
    assert np.array_equal(p["port_v"], p["vtl_v"][pv])
    pid, colour = Zm.pair_colouring(p["vtl_k"], p["vtl_k2"])
    # a colour never holds two pairs sharing a subgraph
    keys = np.unique(np.stack([p["vtl_k"], p["vtl_k2"], colour[pid]], 1), axis=0)
    for c in np.unique(keys[:, 2]):
        ks = keys[keys[:, 2] == c][:, :2].ravel()
        assert len(ks) == len(np.unique(ks))


def test_features_are_scale_free():
    cfg = gen.make_config("c4", small=True)
    A = cfg["A"]
    h1 = B.VTM(device=-1)
    h1.evs_partition(A, cfg["spec"])
    f1 = h1.zfeatures()
    A2 = gen.systems.CSR(n=A.n, rowptr=A.rowptr, col=A.col, val=A.val * 37.5)
    h2 = B.VTM(device=-1)
    h2.evs_partition(A2, cfg["spec"])
    f2 = h2.zfeatures()
    assert f1.shape == (h1.info["nvtl"], B.NUM_FEATURES) and np.isfinite(f1).all()
    assert np.allclose(f1, f2, atol=1e-5)


def test_global_scale_feature_counts_the_systems_subgraphs():
    """Feature 12 is ln of the number of subgraphs of the VTL's own system (batched systems with
    different part counts), counted here from the partition's vertex lists and the system ranges."""
    cfg = gen.make_config("c5", small=True)
    h = B.VTM(device=-1)
    info = h.evs_partition(cfg["A"], cfg["spec"], nsys=cfg["nsys"], sys_ptr=cfg["sys_ptr"])
    p = h.get_partition()
    f = h.zfeatures()
    sys_of_sub = np.searchsorted(cfg["sys_ptr"], p["loc_vtx"][p["loc_ptr"][:-1]], side="right") - 1
    per_sys = np.bincount(sys_of_sub, minlength=cfg["nsys"])
    assert len(np.unique(per_sys)) > 1  # the systems differ in size
    expect = np.log(per_sys[sys_of_sub[p["vtl_k"]]])
    assert np.allclose(f[:, 12], expect, atol=1e-6)
    assert np.array_equal(sys_of_sub[p["vtl_k"]], sys_of_sub[p["vtl_k2"]])
