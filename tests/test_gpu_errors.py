"""Failure handling on the GPU, forced from the host so every kernel still
exits normally: a Newton cap too small for the foot solves, training pairs
naming curves outside the set, empty and negative field counts."""
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


def test_zero_fields_write_nothing(torch_mod):
    """nf = 0 is an empty call on every per-field entry point of a plan: status 0
    and no output touched (outputs sized for one field and filled with a
    sentinel); a negative count is refused with FC2D_E_ARG."""
    import ctypes as C
    from paper_2010_03901_amd import fc2d
    torch = torch_mod
    case = W.cfg_disc128()
    grid = fc2d.make_grid(case.x0, case.y0, case.h, case.n, case.n)
    pl = fc2d.Plan(fc2d.make_curve(*case.curve), grid, d=case.d, C_=case.C, B=case.B, k1=case.k1, M=case.M)
    inf = pl.info
    n, B, d = case.n, inf.B, inf.d
    lib = fc2d._lib()
    S = -7.25
    f64 = dict(dtype=torch.float64, device="cuda:0")
    fg = torch.full((1, n, n), S, **f64)
    fb = torch.full((1, inf.n_bdry), S, **f64)
    outs = {"fD": torch.full((1, B, d), S, **f64), "F": torch.full((1, inf.Cr + 1, B), S, **f64),
            "ext": torch.full((1, n, n), S, **f64), "work": torch.full((1, n, n), S, **f64),
            "bv": torch.full((1, inf.n_bdry), S, **f64),
            "spec": torch.full((1, n, n // 2 + 1), S, dtype=torch.complex128, device="cuda:0")}
    p = lambda t: C.c_void_p(t.data_ptr())
    h = pl.handle
    calls = {
        "fc2d_matching": lambda nf: lib.fc2d_matching(h, p(fg), p(fb), p(outs["fD"]), nf, None),
        "fc2d_blend": lambda nf: lib.fc2d_blend(h, p(fg), p(fb), p(outs["F"]), nf, None),
        "fc2d_extend": lambda nf: lib.fc2d_extend(h, p(fg), p(fb), p(outs["ext"]), nf, None),
        "fc2d_boundary_values": lambda nf: lib.fc2d_boundary_values(h, p(fg), p(outs["bv"]), nf, None),
        "fc2d_extend_fft": lambda nf: lib.fc2d_extend_fft(h, p(fg), p(fb), p(outs["work"]), p(outs["spec"]), nf,
                                                          None),
        "fc2d_extend_fft_ld": lambda nf: lib.fc2d_extend_fft_ld(h, p(fg), p(fb), p(outs["work"]), p(outs["spec"]),
                                                                n // 2 + 1, nf, None),
        "fc2d_extend_fft_noalloc": lambda nf: lib.fc2d_extend_fft_noalloc(h, p(fg), p(fb), p(outs["work"]),
                                                                          p(outs["spec"]), nf, None),
    }
    for name, call in calls.items():
        assert call(0) == 0, name
        assert call(-1) == fc2d.FC2D_E_ARG, name
    torch.cuda.synchronize()
    for k, t in outs.items():
        assert bool((t == S).all()), k
    assert bool((fg == S).all()) and bool((fb == S).all())
