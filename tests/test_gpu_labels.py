"""The learned-impedance labels (probe sweeps of the method itself) from the GPU labeller against the
same rule run by the FP64 CPU oracle (oracle/labels.py), on two small training systems.

alpha* and every pair's beta* are argmins over a grid of FP64 probe results, taken in FP64 on both
sides; where the two differ, the oracle's own scores of both choices must tie to rounding (several
choices are then correct).
"""
import numpy as np
import pytest

from gen import systems as GS
from oracle import labels as OL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Zm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0807_1949_amd import binding, zmodel

    binding.lib()
    return zmodel


def _systems():
    A1 = GS.lognormal_conductance_2d(64, seed=101, shift=1e-3)
    yield "lognormal 64^2, 4x4 tiles", A1, dict(kind="grid", dims=(64, 64, 1), parts=(4, 4, 1)), GS.random_rhs(A1.n, 1, 101)
    A2 = GS.poisson3d_dirichlet(32)
    yield ("Poisson 32^3, RCB 64 boxes", A2, dict(kind="rcb", dims=(32, 32, 32), levels=6, seed=301, min_size=0.0,
                                                    max_size=1e30), GS.random_rhs(A2.n, 1, 301))


@pytest.mark.parametrize("which", [0, 1])
def test_labels_match_oracle(Zm, which):
    name, A, spec, b = list(_systems())[which]
    print(f"[labels] {name}", flush=True)
    _, lab_gpu, a_gpu = Zm.make_labels(A, spec, b, k_probe=200)
    a_or, lab_or, info = OL.make_labels(A, spec, b, k_probe=200)
    res = info["alpha_residuals"]
    if a_gpu != a_or:
        i, j = list(OL.ALPHAS).index(a_gpu), list(OL.ALPHAS).index(a_or)
        floor = 1e-13  # residuals at the FP64 floor of the iteration are ties
        assert abs(res[i] - res[j]) <= 1e-9 * res[j] or max(res[i], res[j]) <= floor, (a_gpu, a_or, res[i], res[j])
        pytest.skip("alpha* tie: the refinement differs from its start")
    pid, sc = info["pid"], info["scores"]
    diff = np.nonzero(np.abs(lab_gpu - lab_or) > 1e-6)[0]
    for l in diff:  # a differing beta must be a tie in the oracle's scores
        p = pid[l]
        bg = int(np.argmin(np.abs(OL.BETAS - np.exp(lab_gpu[l]) / a_or)))
        assert abs(sc[bg, p] - sc[:, p].min()) <= 1e-6 * sc[:, p].min(), (l, sc[:, p], bg)
    print(f"    alpha* {a_or:g}; {len(lab_or)} VTL labels, {len(diff)} on ties; label values "
          f"{sorted(set(np.round(lab_or, 3)))}", flush=True)
