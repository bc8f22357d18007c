"""The HIP extension against the paper's own printed accuracy (Sec. 3.6):
Table 1 (unit disc, Example 3.1; M = d + 3) and Table 2 (kite, Example 3.2;
M = d + 1, d + 2, d + 3), k1 = h.  The GPU extension of the closed-form f is interpolated to the grid of
step h/2 by zero padding its DFT (numpy, on the host: a measuring instrument,
not part of the path) and compared with f there inside the domain.  Bars: the
error within a factor 2 (Table 1, measured 0.82 - 1.07) or 3 (Table 2, every
M column and the rows h = 1e-2, 5e-3, 2.5e-3, measured 0.48 - 2.5) of the printed value, and the convergence order
of the last halving above d - 0.7 (Table 1)."""
import numpy as np
import pytest

import workloads as W
from conftest import load_golden
from oracle import plan as OP
from oracle import spectral as OS
from oracle.curves import Curve

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _gpu_extension(torch, curve, x0, y0, h, nx, ny, B, d, f, M=None):
    from paper_2010_03901_amd import fc2d
    grid = fc2d.make_grid(x0, y0, h, nx, ny)
    pl = fc2d.Plan(fc2d.make_curve(*curve), grid, d=d, C_=27, B=B, k1=h, M=M or d + 3)
    bp = fc2d.fc2d_boundary_points(pl)
    X, Y = np.meshgrid(x0 + np.arange(nx) * h, y0 + np.arange(ny) * h, indexing="ij")
    fg = torch.from_numpy(f(X, Y)[None]).to("cuda:0")
    fb = torch.from_numpy(f(bp[:, 0], bp[:, 1])[None]).to("cuda:0")
    out = torch.empty_like(fg)
    fc2d.fc2d_extend(pl, fg, fb, out)
    torch.cuda.synchronize()
    return out[0].cpu().numpy()


@pytest.mark.parametrize("d", [4, 5])
def test_table1_disc(torch_mod, d):
    rows = [r for r in load_golden("paper_table1_disc.txt") if int(r[0]) == d]
    errs = []
    for _, h, _, B, ref in rows:
        n = int(round(3.2 / h))
        ext = _gpu_extension(torch_mod, W.disc(), -1.6, -1.6, h, n, n, int(B), d, W.f_paper_disc)
        up = OS.upsample_h2(ext)
        x = -1.6 + np.arange(2 * n) * h / 2
        X, Y = np.meshgrid(x, x, indexing="ij")
        ins = X ** 2 + Y ** 2 < 1
        ex = W.f_paper_disc(X, Y)
        e = np.abs(up - ex)[ins].max() / np.abs(ex[ins]).max()
        print("[paper] Table 1 d=%d h=%g: GPU %.2e printed %.2e (x%.2f)" % (d, h, e, ref, e / ref))
        assert ref / 2 < e < 2 * ref, (d, h, e, ref)
        errs.append(e)
    order = np.log2(errs[-2] / errs[-1])
    assert order > d - 0.7, (d, errs)


def test_table1_disc_d10(torch_mod):
    """Table 1's d = 10 rows (M = 13): within 10x at h = 2e-2 and 3x at h = 1e-2
    (measured 7.4x and 1.9x)."""
    rows = [r for r in load_golden("paper_table1_disc.txt") if int(r[0]) == 10]
    for (_, h, _, B, ref), bar in zip(rows, (10.0, 3.0)):
        n = int(round(3.2 / h))
        ext = _gpu_extension(torch_mod, W.disc(), -1.6, -1.6, h, n, n, int(B), 10, W.f_paper_disc)
        up = OS.upsample_h2(ext)
        x = -1.6 + np.arange(2 * n) * h / 2
        X, Y = np.meshgrid(x, x, indexing="ij")
        ins = X ** 2 + Y ** 2 < 1
        ex = W.f_paper_disc(X, Y)
        e = np.abs(up - ex)[ins].max() / np.abs(ex[ins]).max()
        print("[paper] Table 1 d=10 h=%g: GPU %.2e printed %.2e (x%.2f)" % (h, e, ref, e / ref))
        assert ref / bar < e < bar * ref, (h, e, ref)


@pytest.mark.parametrize("d", [4, 5])
def test_table2_kite(torch_mod, d):
    rows = [r for r in load_golden("paper_table2_kite.txt") if int(r[0]) == d]
    curve = W.kite(0.35, 0.7)
    xmin, xmax, ymin, ymax = W.bbox(curve)
    for _, h, nx, ny, *refs in rows:
        nx, ny = int(nx), int(ny)
        x0 = 0.5 * (xmin + xmax) - 0.5 * nx * h
        y0 = 0.5 * (ymin + ymax) - 0.5 * ny * h
        for M, ref in zip((d + 1, d + 2, d + 3), refs):
            ext = _gpu_extension(torch_mod, curve, x0, y0, h, nx, ny, int(round(2 * np.pi / h)), d,
                                 W.f_paper_kite, M)
            U = np.fft.fft2(ext)
            P2 = np.zeros((2 * nx, 2 * ny), dtype=complex)
            hx, hy = nx // 2, ny // 2
            P2[:hx + 1, :hy + 1] = U[:hx + 1, :hy + 1]
            P2[-hx:, :hy + 1] = U[-hx:, :hy + 1]
            P2[:hx + 1, -hy:] = U[:hx + 1, -hy:]
            P2[-hx:, -hy:] = U[-hx:, -hy:]
            up = np.real(np.fft.ifft2(P2)) * 4
            X2, Y2 = np.meshgrid(x0 + np.arange(2 * nx) * h / 2, y0 + np.arange(2 * ny) * h / 2, indexing="ij")
            ins = OP.column_parity_inside(Curve(*curve), OP.Grid(x0, y0, h / 2, 2 * nx, 2 * ny), 16384)
            e = np.abs(up - W.f_paper_kite(X2, Y2))[ins].max()
            print("[paper] Table 2 d=%d M=%d h=%g (%dx%d): GPU %.2e printed %.2e (x%.2f)"
                  % (d, M, h, nx, ny, e, ref, e / ref))
            assert ref / 3 < e < 3 * ref, (d, M, h, e, ref)
