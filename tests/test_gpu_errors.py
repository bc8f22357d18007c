"""Failure handling on the GPU, forced from the host so every kernel still
exits normally: a Newton cap too small for the foot solves, training pairs
naming curves outside the set."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_newton_cap_reports_failure(torch_mod):
    from paper_2010_03901_amd import fc2d
    case = W.cfg_star(320)
    grid = fc2d.make_grid(case.x0, case.y0, case.h, case.n, case.n)
    curve = fc2d.make_curve(*case.curve)
    with pytest.raises(fc2d.Fc2dError) as ei:
        fc2d.Plan(curve, grid, d=case.d, C_=case.C, B=case.B, k1=case.k1, M=case.M, newton_maxit=1)
    assert ei.value.status == fc2d.FC2D_E_NEWTON
    # the same plan with the default cap builds
    pl = fc2d.Plan(curve, grid, d=case.d, C_=case.C, B=case.B, k1=case.k1, M=case.M)
    assert pl.info.n_strip > 0


def test_training_pairs_flag_unknown_curves(torch_mod):
    from paper_2010_03901_amd import fc2d
    torch = torch_mod
    curves, cidx, th, eta = W.mlp_training_draws(0, 4, 8, 0.01)
    cidx = cidx.copy()
    cidx[3] = 7          # not a curve of the set
    cidx[5] = -1
    n = cidx.size
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    X = torch.zeros((n, 8), dtype=torch.float32, device="cuda:0")
    Y = torch.zeros((n, 2), dtype=torch.float32, device="cuda:0")
    its = torch.zeros(n, dtype=torch.int32, device="cuda:0")
    fc2d.fc2d_mlp_make_data(dev(curves), dev(cidx), dev(th), dev(eta), 0.01, X, Y, None, its)
    torch.cuda.synchronize()
    it = its.cpu().numpy()
    assert it[3] == -1 and it[5] == -1
    assert np.all(np.delete(it, [3, 5]) >= 1)
