"""A plan is read-only after creation: extension calls sharing one plan on two
streams, queued without any host synchronisation between them, give bitwise
the results of the same calls made one at a time on one stream (each call
takes its Gram-record work space on its own stream)."""
import numpy as np
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


def _inputs(torch, case, gpl, seeds):
    from paper_2010_03901_amd import fc2d
    funcs = [W.f_star(s) for s in seeds]
    fg, fb = fields(case, funcs, fc2d.fc2d_boundary_points(gpl))
    return (torch.from_numpy(fg).to("cuda:0"), torch.from_numpy(fb).to("cuda:0"))


def test_extend_fft_two_streams_one_plan(torch_mod):
    from paper_2010_03901_amd import fc2d
    torch = torch_mod
    case = W.cfg_star(512)
    print("\n[streams] star512 extend_fft, two streams, 12 + 5 fields", flush=True)
    gpl = gpu_plan(case)
    n = case.n
    (fa, ba), (fb_, bb) = _inputs(torch, case, gpl, range(12)), _inputs(torch, case, gpl, range(20, 25))
    # reference: one call at a time on the default stream
    ref_a = torch.empty((12, n, n // 2 + 1), dtype=torch.complex128, device="cuda:0")
    ref_b = torch.empty((5, n, n // 2 + 1), dtype=torch.complex128, device="cuda:0")
    fc2d.fc2d_extend_fft(gpl, fa, ba, torch.empty_like(fa), ref_a)
    torch.cuda.synchronize()
    fc2d.fc2d_extend_fft(gpl, fb_, bb, torch.empty_like(fb_), ref_b)
    torch.cuda.synchronize()
    # concurrent: alternating calls on two streams, no host synchronisation in between
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs_a = [torch.full_like(ref_a, float("nan")) for _ in range(3)]
    outs_b = [torch.full_like(ref_b, float("nan")) for _ in range(3)]
    wa = [torch.empty_like(fa) for _ in range(3)]
    wb = [torch.empty_like(fb_) for _ in range(3)]
    torch.cuda.synchronize()
    for k in range(3):
        fc2d.fc2d_extend_fft(gpl, fa, ba, wa[k], outs_a[k], stream=s1.cuda_stream)
        fc2d.fc2d_extend_fft(gpl, fb_, bb, wb[k], outs_b[k], stream=s2.cuda_stream)
    torch.cuda.synchronize()
    for k in range(3):
        assert torch.equal(outs_a[k], ref_a), k
        assert torch.equal(outs_b[k], ref_b), k


def test_extend_two_streams_one_plan(torch_mod):
    from paper_2010_03901_amd import fc2d
    torch = torch_mod
    case = W.cfg_star(512)
    print("\n[streams] star512 extend, two streams, 7 + 3 fields", flush=True)
    gpl = gpu_plan(case)
    (fa, ba), (fb_, bb) = _inputs(torch, case, gpl, range(7)), _inputs(torch, case, gpl, range(30, 33))
    ref_a, ref_b = torch.empty_like(fa), torch.empty_like(fb_)
    fc2d.fc2d_extend(gpl, fa, ba, ref_a)
    torch.cuda.synchronize()
    fc2d.fc2d_extend(gpl, fb_, bb, ref_b)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    oa = [torch.full_like(fa, float("nan")) for _ in range(3)]
    ob = [torch.full_like(fb_, float("nan")) for _ in range(3)]
    torch.cuda.synchronize()
    for k in range(3):
        fc2d.fc2d_extend(gpl, fa, ba, oa[k], stream=s1.cuda_stream)
        fc2d.fc2d_extend(gpl, fb_, bb, ob[k], stream=s2.cuda_stream)
    torch.cuda.synchronize()
    for k in range(3):
        assert torch.equal(oa[k], ref_a), k
        assert torch.equal(ob[k], ref_b), k
    assert np.isfinite(ref_a.cpu().numpy()).all()
