"""fc2d_extend_fft_noalloc (Gram records in the library's fixed scratch, no
allocation) against fc2d_extend_fft (per-call work space), through the C ABI:
bitwise equal on two calls in a row, the second one smaller (fewer fields on a
smaller plan), and oversized requests refused before any launch."""
import ctypes as C

import pytest

import workloads as W
from gpu_common import fields, gpu_plan

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _run_pair(torch, case, funcs):
    from paper_2010_03901_amd import fc2d
    gpl = gpu_plan(case)
    fg, fb = fields(case, funcs, fc2d.fc2d_boundary_points(gpl))
    dfg = torch.from_numpy(fg).to("cuda:0")
    dfb = torch.from_numpy(fb).to("cuda:0")
    nf, n = len(funcs), case.n
    ref = torch.empty((nf, n, n // 2 + 1), dtype=torch.complex128, device="cuda:0")
    fc2d.fc2d_extend_fft(gpl, dfg, dfb, torch.empty_like(dfg), ref)
    out = torch.full_like(ref, float("nan"))
    work = torch.empty_like(dfg)
    lib = fc2d._lib()
    st = lib.fc2d_extend_fft_noalloc(gpl.handle, C.c_void_p(dfg.data_ptr()), C.c_void_p(dfb.data_ptr()),
                                     C.c_void_p(work.data_ptr()), C.c_void_p(out.data_ptr()), nf,
                                     C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, lib.fc2d_last_error()
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    return gpl


def test_noalloc_matches_extend_fft_twice(torch_mod):
    torch = torch_mod
    print("\n[noalloc] star512, 9 fields", flush=True)
    _run_pair(torch, W.cfg_star(512), [W.f_star(s) for s in range(9)])
    print("[noalloc] disc128, 2 fields (smaller, after the larger call)", flush=True)
    _run_pair(torch, W.cfg_disc128(), [W.f_cfg1, W.f_paper_disc])


def test_noalloc_refuses_more_fields_than_the_scratch_holds(torch_mod):
    from paper_2010_03901_amd import fc2d
    torch = torch_mod
    case = W.cfg_disc128()
    gpl = gpu_plan(case)
    info = gpl.info
    per_field = info.B * ((info.d + 2) & ~1) * 8
    nf = (16 << 20) // per_field + 1
    n = case.n
    lib = fc2d._lib()
    print("\n[noalloc] refusal check, nf", nf, flush=True)
    # host-side size check: refused before any pointer is touched
    st = lib.fc2d_extend_fft_noalloc(gpl.handle, C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), C.c_void_p(8), nf,
                                     C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == fc2d.FC2D_E_ARG
    assert b"fixed scratch" in lib.fc2d_last_error()
    assert n > 0
