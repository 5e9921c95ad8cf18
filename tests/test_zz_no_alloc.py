"""vtm_input_impedance_noalloc (the entry point for callers that cannot allocate) against
vtm_input_impedance, through the C ABI: two calls in a row on one GPU, the second with a smaller
input, host and device outputs; values equal to rounding and infinities in the same places."""
import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0807_1949_amd import binding

    binding.lib()
    return binding


def _same(a, b):
    fa, fb = np.isfinite(a), np.isfinite(b)
    assert np.array_equal(fa, fb)
    assert np.all(np.abs(a[fa] - b[fa]) <= 1e-13 * np.abs(b[fa]))


def test_noalloc_input_impedance_matches_allocating_call(B):
    import torch

    big = gen.make_config("c3", small=True)   # 21,366 ports
    small = gen.make_config("c1")              # 804 ports
    outs = []
    for cfg, zs in ((big, 8.0), (small, 1.0)):
        h = B.VTM(device=0, sweep_mode=2)
        info = h.evs_partition(cfg["A"], cfg["spec"])
        z = zs / cfg["A"].to_scipy().diagonal()[h.get_partition()["vtl_v"]]
        h.setup(B.VTM_Z_USER, z)
        ref = h.input_impedance()
        r = h.input_impedance_noalloc()
        _same(r, ref)
        d = torch.full((info["nports"],), -1.0, dtype=torch.float64, device="cuda")
        h.input_impedance_noalloc(d)
        torch.cuda.synchronize()
        _same(d.cpu().numpy(), ref)
        outs.append(info["nports"])
        h.close()
    assert outs[1] < outs[0]


def test_noalloc_rejects_missing_green_functions(B):
    cfg = gen.make_config("c1")
    h = B.VTM(device=0, sweep_mode=1)
    h.evs_partition(cfg["A"], cfg["spec"])
    h.setup(B.VTM_Z_DIAG)
    with pytest.raises(B.VTMError) as e:
        h.input_impedance_noalloc()
    assert e.value.code == B.VTM_ERR_STATE
