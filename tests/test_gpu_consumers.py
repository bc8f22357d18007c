"""GPU parity of the 2D FFT over all supported sizes and of the spectral
consumers (Poisson particular solution, Sec. 4.1; Fourier-Forwarding
propagation, Sec. 4.2) against the oracle, through the C ABI."""
import numpy as np
import pytest

import workloads as W
from gpu_common import fields, gpu_plan, oracle_plan, rel_err
from oracle import extend as OE
from oracle import plan as OP
from oracle import spectral as OS

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.mark.parametrize("nx,ny,nf", [(16, 16, 3), (32, 64, 3), (64, 16, 3), (128, 128, 3), (256, 512, 3),
                                      (512, 512, 3), (1024, 1024, 3), (2048, 256, 3), (256, 2048, 3), (4096, 64, 3),
                                      (64, 8192, 3), (16, 4096, 3), (512, 256, 8), (1024, 128, 16)])
def test_fft_sizes(torch_mod, nx, ny, nf):
    """nf a multiple of 8 takes the whole-fields-per-XCD column mapping."""
    from paper_2010_03901_amd import fc2d
    torch = torch_mod
    print("\n[fft] %dx%d nf=%d" % (nx, ny, nf), flush=True)
    rng = np.random.default_rng(nx * 7 + ny)
    u = rng.standard_normal((nf, nx, ny))
    grid = fc2d.make_grid(0.0, 0.0, 0.01, nx, ny)
    du = _dev(torch, u)
    spec = torch.zeros((nf, nx, ny // 2 + 1), dtype=torch.complex128, device="cuda:0")
    fc2d.fc2d_fft(grid, du, spec, fc2d.FC2D_FORWARD)
    back = torch.zeros_like(du)
    fc2d.fc2d_fft(grid, spec.clone(), back, fc2d.FC2D_INVERSE)
    torch.cuda.synchronize()
    s = spec.cpu().numpy()
    for k in range(nf):
        assert rel_err(s[k], np.fft.rfft2(u[k])) < 1e-13
    assert rel_err(back.cpu().numpy(), u) < 1e-13


def test_fft_inverse_matches_irfft2_on_hermitian_spectra(torch_mod):
    from paper_2010_03901_amd import fc2d
    torch = torch_mod
    nx, ny = 128, 256
    rng = np.random.default_rng(11)
    U = np.fft.rfft2(rng.standard_normal((2, nx, ny)))
    grid = fc2d.make_grid(0.0, 0.0, 0.01, nx, ny)
    out = torch.zeros((2, nx, ny), dtype=torch.float64, device="cuda:0")
    fc2d.fc2d_fft(grid, _dev(torch, U), out, fc2d.FC2D_INVERSE)
    torch.cuda.synchronize()
    assert rel_err(out.cpu().numpy(), np.fft.irfft2(U, s=(nx, ny))) < 1e-13


@pytest.mark.parametrize("op", ["lap", "dx", "dy"])
def test_spectral_ops(torch_mod, op):
    from paper_2010_03901_amd import fc2d
    torch = torch_mod
    nx, ny, h = 64, 128, 0.03
    rng = np.random.default_rng(5)
    U = np.fft.rfft2(rng.standard_normal((2, nx, ny)))
    grid = fc2d.make_grid(0.0, 0.0, h, nx, ny)
    code = {"lap": fc2d.FC2D_LAPLACE_INV, "dx": fc2d.FC2D_DX, "dy": fc2d.FC2D_DY}[op]
    dU = _dev(torch, U)
    out = torch.zeros_like(dU)
    fc2d.fc2d_spectral_apply(grid, code, dU, out)
    fc2d.fc2d_spectral_apply(grid, code, dU, dU)      # in place
    torch.cuda.synchronize()
    for k in range(2):
        if op == "lap":
            ref = OS.laplace_inverse(U[k], nx, ny, h)
        else:
            ref = OS.derivative(U[k], nx, ny, h, 0 if op == "dx" else 1)
        assert rel_err(out[k].cpu().numpy(), ref) < 1e-14
    assert np.array_equal(out.cpu().numpy(), dU.cpu().numpy())


def test_ff_propagate_against_oracle(torch_mod):
    from paper_2010_03901_amd import fc2d
    torch = torch_mod
    nx, ny, h, c, t = 128, 64, 0.02, 1.0, 0.37
    rng = np.random.default_rng(6)
    U0 = np.fft.rfft2(rng.standard_normal((2, nx, ny)))
    U1 = np.fft.rfft2(rng.standard_normal((2, nx, ny)))
    grid = fc2d.make_grid(0.0, 0.0, h, nx, ny)
    a = torch.zeros((2, nx, ny // 2 + 1), dtype=torch.complex128, device="cuda:0")
    at = torch.zeros_like(a)
    fc2d.ff_propagate(grid, c, t, _dev(torch, U0), _dev(torch, U1), a, at)
    torch.cuda.synchronize()
    for k in range(2):
        ra, rat = OS.ff_propagate(U0[k], U1[k], nx, ny, h, c, t)
        assert rel_err(a[k].cpu().numpy(), ra) < 1e-13
        assert rel_err(at[k].cpu().numpy(), rat) < 1e-13


@pytest.mark.parametrize("n", [256, 2048])
def test_poisson_chain_kite(torch_mod, n):
    """Extension -> R2C -> division by -|k|^2 -> C2R on the kite (the Poisson
    particular-solution consumer), compared with the oracle chain; n = 2048 is
    the full Poisson workload (fitted box, B = 4096, about 169k STRIP points)."""
    from paper_2010_03901_amd import fc2d
    torch = torch_mod
    print("\n[poisson] kite%d" % n, flush=True)
    case, opl = oracle_plan("kite%d" % n, W.cfg_kite, n)
    gpl = gpu_plan(case)
    f = W.poisson_rhs(0)
    fg, fbo = fields(case, [f], OP.boundary_points(opl))
    _, fbg = fields(case, [f], fc2d.fc2d_boundary_points(gpl))
    grid = fc2d.make_grid(case.x0, case.y0, case.h, case.n, case.n)
    ext = torch.zeros((1, case.n, case.n), dtype=torch.float64, device="cuda:0")
    fc2d.fc2d_extend(gpl, _dev(torch, fg), _dev(torch, fbg), ext)
    spec = torch.zeros((1, case.n, case.n // 2 + 1), dtype=torch.complex128, device="cuda:0")
    fc2d.fc2d_fft(grid, ext, spec, fc2d.FC2D_FORWARD)
    fc2d.fc2d_spectral_apply(grid, fc2d.FC2D_LAPLACE_INV, spec, spec)
    up = torch.zeros_like(ext)
    fc2d.fc2d_fft(grid, spec, up, fc2d.FC2D_INVERSE)
    torch.cuda.synchronize()
    e = OE.extend(opl, fg[0], fbo[0])
    ref = OS.fft2_inverse(OS.laplace_inverse(OS.fft2_forward(e), case.n, case.n, case.h), case.n)
    err_all = rel_err(up[0].cpu().numpy(), ref)
    inm = opl.cls == OP.IN
    err_in = rel_err(up[0].cpu().numpy()[inm], ref[inm])
    print("[poisson] kite%d rel err all %.3e interior %.3e" % (n, err_all, err_in))
    assert err_all < 1e-11 and err_in < 1e-11


def test_ff_chain_disc(torch_mod):
    """One Fourier-Forwarding step of a Gaussian pulse on the disc:
    extend u0 -> R2C, u1 = 0, propagate by t, C2R, against the oracle."""
    from paper_2010_03901_amd import fc2d
    torch = torch_mod
    case, opl = oracle_plan("disc256", W.cfg_disc, 256)
    gpl = gpu_plan(case)
    f, _ = W.gaussian_pulse(W.disc(), 3)
    fg, fbo = fields(case, [f], OP.boundary_points(opl))
    _, fbg = fields(case, [f], fc2d.fc2d_boundary_points(gpl))
    grid = fc2d.make_grid(case.x0, case.y0, case.h, case.n, case.n)
    ext = torch.zeros((1, case.n, case.n), dtype=torch.float64, device="cuda:0")
    fc2d.fc2d_extend(gpl, _dev(torch, fg), _dev(torch, fbg), ext)
    u0 = torch.zeros((1, case.n, case.n // 2 + 1), dtype=torch.complex128, device="cuda:0")
    fc2d.fc2d_fft(grid, ext, u0, fc2d.FC2D_FORWARD)
    u1 = torch.zeros_like(u0)
    a = torch.zeros_like(u0)
    at = torch.zeros_like(u0)
    fc2d.ff_propagate(grid, 1.0, 0.25, u0, u1, a, at)
    u = torch.zeros_like(ext)
    fc2d.fc2d_fft(grid, a, u, fc2d.FC2D_INVERSE)
    torch.cuda.synchronize()
    e = OE.extend(opl, fg[0], fbo[0])
    ra, _ = OS.ff_propagate(OS.fft2_forward(e), np.zeros_like(OS.fft2_forward(e)), case.n, case.n, case.h, 1.0, 0.25)
    ref = OS.fft2_inverse(ra, case.n)
    assert rel_err(u[0].cpu().numpy(), ref) < 1e-11


def test_empty_batch_is_a_no_op(torch_mod):
    from paper_2010_03901_amd import fc2d
    import ctypes as C
    lib = fc2d._lib()
    g = fc2d.make_grid(0, 0, 0.1, 64, 64)
    assert lib.fc2d_fft(C.byref(g), C.c_void_p(8), C.c_void_p(16), fc2d.FC2D_FORWARD, 0, None) == 0
    assert lib.ff_propagate(C.byref(g), 1.0, 1.0, None, None, None, None, 0, None) == 0
