"""GPU parity of the batched Fourier-Forwarding path: boundary values read off
the full-box field, one step per (plan, field) against the oracle's step from
the same state, and HIP-graph replays against eager steps."""
import numpy as np
import pytest

import workloads as W
from gpu_common import gpu_plan, oracle_ff_step_worker, oracle_plan, oracle_pool_map, pulse_field, rel_err
from oracle import ff as OF
from oracle import plan as OP

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def test_boundary_values(torch_mod):
    from paper_2010_03901_amd import fc2d
    torch = torch_mod
    case, opl = oracle_plan("star256ff", W.cfg_ff, "star5", 256)
    gpl = gpu_plan(case)
    X, Y = np.meshgrid(opl.grid.xs(), opl.grid.ys(), indexing="ij")
    u = np.stack([np.sin(3 * X + 1) * np.cos(2 * Y), np.exp(-(X * X + Y * Y))])
    fb = torch.zeros((2, gpl.info.n_bdry), dtype=torch.float64, device="cuda:0")
    fc2d.fc2d_boundary_values(gpl, _dev(torch, u), fb)
    torch.cuda.synchronize()
    bpo = OP.boundary_points(opl)
    for k in range(2):
        assert rel_err(fb[k].cpu().numpy(), OF.boundary_interp(u[k], opl.grid, bpo, opl.M)) < 1e-12


def _pulses(case, seeds):
    x = case.x0 + np.arange(case.n) * case.h
    X, Y = np.meshgrid(x, x, indexing="ij")
    out = []
    for s in seeds:
        f, _ = W.gaussian_pulse(case.curve, s)
        out.append(f(X, Y))
    return np.stack(out)


@pytest.fixture(scope="module")
def batch_setup(torch_mod):
    from paper_2010_03901_amd import fc2d
    specs = [("disc", 256), ("star5", 256), ("kite", 256), ("ellipse", 512)]
    cases, oplans, gplans = [], [], []
    for dom, n in specs:
        case, opl = oracle_plan("%s%dff" % (dom, n), W.cfg_ff, dom, n)
        print("\n[batch] plan", dom, n, flush=True)
        cases.append(case)
        oplans.append(opl)
        gplans.append(gpu_plan(case))
    nf = [2, 2, 1, 2]
    batch = fc2d.Batch(gplans, nf, autotune=True)
    u0 = [_pulses(c, range(10 * k, 10 * k + m)) for k, (c, m) in enumerate(zip(cases, nf))]
    return batch, cases, oplans, gplans, nf, u0


def _load_state(batch, u0):
    for k, u in enumerate(u0):
        du, dut = batch.state(k)
        du.copy_(__import__("torch").from_numpy(u))
        dut.zero_()


def test_batch_one_step_matches_oracle(batch_setup, torch_mod):
    torch = torch_mod
    batch, cases, oplans, gplans, nf, u0 = batch_setup
    pts, nl, sf = batch.info()
    print("[batch] points/step", pts, "launches/step", nl, "strip fields/thread", sf)
    _load_state(batch, u0)
    dt = 0.02
    batch.run_ff(1.0, dt, 1, use_graph=False)
    torch.cuda.synchronize()
    for k, (opl, m) in enumerate(zip(oplans, nf)):
        du, dut = batch.state(k)
        for f in range(m):
            ou, out_ = OF.ff_step(opl, u0[k][f], np.zeros_like(u0[k][f]), dt)
            eu = rel_err(du[f].cpu().numpy(), ou)
            et = rel_err(dut[f].cpu().numpy(), out_)
            print("[batch] plan %d field %d: u %.2e u_t %.2e" % (k, f, eu, et))
            assert eu < 1e-11 and et < 1e-11


def test_batch_graph_replays_match_eager(batch_setup, torch_mod):
    torch = torch_mod
    batch, cases, oplans, gplans, nf, u0 = batch_setup
    dt = 0.01
    _load_state(batch, u0)
    eager = []
    for _ in range(3):
        batch.run_ff(1.0, dt, 1, use_graph=False)
        torch.cuda.synchronize()
        eager.append([tuple(t.cpu().numpy().copy() for t in batch.state(k)) for k in range(len(nf))])
    _load_state(batch, u0)
    for step in range(3):
        batch.run_ff(1.0, dt, 1, use_graph=True)
        torch.cuda.synchronize()
        _ = torch.ones(1, device="cuda:0").sum().item()       # unrelated eager work between replays
        for k in range(len(nf)):
            du, dut = batch.state(k)
            assert np.array_equal(du.cpu().numpy(), eager[step][k][0]), (step, k)
            assert np.array_equal(dut.cpu().numpy(), eager[step][k][1]), (step, k)


def test_fused_spectral_step_matches_separate(batch_setup, torch_mod):
    """The fused column-pass + propagation kernel against the separate passes
    and against the oracle's step, on the same plans and initial data."""
    from paper_2010_03901_amd import fc2d
    torch = torch_mod
    _, cases, oplans, gplans, nf, u0 = batch_setup
    dt = 0.02
    res = []
    for fused in (False, True):
        b = fc2d.Batch(gplans, nf, fused_ff=fused)
        _load_state(b, u0)
        b.run_ff(1.0, dt, 1, use_graph=False)
        torch.cuda.synchronize()
        res.append([tuple(t.cpu().numpy().copy() for t in b.state(k)) for k in range(len(nf))])
        b.close()
    for k, (opl, m) in enumerate(zip(oplans, nf)):
        for f in range(m):
            ou, out_ = OF.ff_step(opl, u0[k][f], np.zeros_like(u0[k][f]), dt)
            for j, ref in ((0, ou), (1, out_)):
                assert rel_err(res[1][k][j][f], res[0][k][j][f]) < 1e-13
                assert rel_err(res[1][k][j][f], ref) < 1e-11


def test_batch_three_steps_match_oracle(batch_setup, torch_mod):
    """Three Fourier-Forwarding steps in a row (graph replays) against the
    oracle's three steps, for the first field of the two 256^2 plans.

    Without the paper's near-boundary solver the iterated step is not a PDE
    solver: each step's continuation amplifies the previous step's rounding
    (by about 3-4x per step here).  The bar is therefore derived from the
    oracle itself: ten times the change of its own three-step result under a
    relative perturbation of 1e-16 of the initial field, and at least the
    single-step bar 1e-11."""
    torch = torch_mod
    batch, cases, oplans, gplans, nf, u0 = batch_setup
    dt = 0.02
    _load_state(batch, u0)
    batch.run_ff(1.0, dt, 3, use_graph=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(42)

    def oracle_run(opl, u):
        ut = np.zeros_like(u)
        for _ in range(3):
            u, ut = OF.ff_step(opl, u, ut, dt)
        return u, ut

    for k in (0, 2):
        ou, out_ = oracle_run(oplans[k], u0[k][0])
        pu, put = oracle_run(oplans[k], u0[k][0] * (1.0 + 1e-16 * rng.standard_normal(u0[k][0].shape)))
        bar_u = max(1e-11, 10 * rel_err(pu, ou))
        bar_t = max(1e-11, 10 * rel_err(put, out_))
        du, dut = batch.state(k)
        eu = rel_err(du[0].cpu().numpy(), ou)
        et = rel_err(dut[0].cpu().numpy(), out_)
        print("[batch] three steps plan %d: u %.2e (bar %.2e) u_t %.2e (bar %.2e)" % (k, eu, bar_u, et, bar_t))
        assert eu < bar_u and et < bar_t


def test_fused_spectral_step_eight_fields(torch_mod):
    """Eight fields on one plan (the whole-fields-per-XCD mapping of the column
    kernels): fused against separate spectral steps, and a field against the
    oracle's step."""
    from paper_2010_03901_amd import fc2d
    torch = torch_mod
    case, opl = oracle_plan("disc256ff", W.cfg_ff, "disc", 256)
    gpl = gpu_plan(case)
    u0 = _pulses(case, range(50, 58))
    dt = 0.02
    res = []
    for fused in (False, True):
        b = fc2d.Batch([gpl], [8], fused_ff=fused)
        _load_state(b, [u0])
        b.run_ff(1.0, dt, 1, use_graph=False)
        torch.cuda.synchronize()
        res.append(tuple(t.cpu().numpy().copy() for t in b.state(0)))
        b.close()
    assert rel_err(res[1][0], res[0][0]) < 1e-13 and rel_err(res[1][1], res[0][1]) < 1e-13
    ou, out_ = OF.ff_step(opl, u0[5], np.zeros_like(u0[5]), dt)
    assert rel_err(res[1][0][5], ou) < 1e-11 and rel_err(res[1][1][5], out_) < 1e-11


@pytest.mark.parametrize("nf8", [False, True], ids=["mixed", "eight_fields"])
def test_transposed_spectra_bitwise(batch_setup, torch_mod, nf8):
    """Transposed spectra ([field][column][row]) change only where the
    spectrum sits in memory: the step equals the row-major fused step bit for
    bit, on the mixed batch and on eight fields of one plan (the
    whole-fields-per-XCD mapping), and matches the oracle's step."""
    from paper_2010_03901_amd import fc2d
    torch = torch_mod
    _, cases, oplans, gplans, nf, u0 = batch_setup
    if nf8:
        case, opl = oracle_plan("disc256ff", W.cfg_ff, "disc", 256)
        gplans, oplans, nf = [gpu_plan(case)], [opl], [8]
        u0 = [_pulses(case, range(50, 58))]
    dt = 0.02
    res = []
    for trans in (False, True):
        b = fc2d.Batch(gplans, nf, fused_ff=True, transposed=trans)
        _load_state(b, u0)
        b.run_ff(1.0, dt, 2, use_graph=False)
        torch.cuda.synchronize()
        res.append([tuple(t.cpu().numpy().copy() for t in b.state(k)) for k in range(len(nf))])
        b.close()
    for k in range(len(nf)):
        assert np.array_equal(res[0][k][0], res[1][k][0]) and np.array_equal(res[0][k][1], res[1][k][1]), k
    # one step against the oracle
    b = fc2d.Batch(gplans, nf, transposed=True)
    _load_state(b, u0)
    b.run_ff(1.0, dt, 1, use_graph=True)
    torch.cuda.synchronize()
    for k, (opl, m) in enumerate(zip(oplans, nf)):
        du, dut = b.state(k)
        f = m - 1
        ou, out_ = OF.ff_step(opl, u0[k][f], np.zeros_like(u0[k][f]), dt)
        assert rel_err(du[f].cpu().numpy(), ou) < 1e-11 and rel_err(dut[f].cpu().numpy(), out_) < 1e-11
    b.close()


def test_batch_interior_only_plan(torch_mod):
    """A batch mixing a plan built from interior data only (Remark 3.1 II; its
    matching reads no boundary values) with an ordinary one: one step per field
    against the oracle's step on the same plans (1e-11)."""
    from paper_2010_03901_amd import fc2d
    from oracle import fcgram
    from oracle.curves import Curve
    torch = torch_mod
    case_io = W.cfg_ff("disc", 256)
    g = OP.Grid(case_io.x0, case_io.y0, case_io.h, case_io.n, case_io.n)
    opl_io = OP.make_plan(Curve(*case_io.curve), g, fcgram.load_tables(case_io.d), case_io.B, k1=case_io.k1,
                          M=case_io.M, interior_only=True)
    gpl_io = fc2d.Plan(fc2d.make_curve(*case_io.curve),
                       fc2d.make_grid(case_io.x0, case_io.y0, case_io.h, case_io.n, case_io.n),
                       d=case_io.d, C_=case_io.C, B=case_io.B, k1=case_io.k1, M=case_io.M, interior_only=True)
    case_k, opl_k = oracle_plan("kite256ff", W.cfg_ff, "kite", 256)
    gpl_k = gpu_plan(case_k)
    nf = [2, 1]
    batch = fc2d.Batch([gpl_io, gpl_k], nf, autotune=False)
    u0 = [_pulses(case_io, [3, 4]), _pulses(case_k, [5])]
    _load_state(batch, u0)
    dt = 0.02
    batch.run_ff(1.0, dt, 1, use_graph=False)
    torch.cuda.synchronize()
    for k, (opl, m) in enumerate(zip([opl_io, opl_k], nf)):
        du, dut = batch.state(k)
        for f in range(m):
            ou, out_ = OF.ff_step(opl, u0[k][f], np.zeros_like(u0[k][f]), dt)
            eu = rel_err(du[f].cpu().numpy(), ou)
            et = rel_err(dut[f].cpu().numpy(), out_)
            print("\n[batch] interior-only mix plan %d field %d: u %.2e u_t %.2e" % (k, f, eu, et), end="")
            assert eu < 1e-11 and et < 1e-11


@pytest.mark.gpu
@pytest.mark.parametrize("n,nfl", [(1024, 2), (2048, 2), (4096, 2), (1024, 8), (2048, 8)])
def test_every_fused_shape_matches_separate(torch_mod, n, nfl):
    """Every compiled shape of the fused column-pass + propagation kernel for
    length n (the two-spectra blocks and the paired one-column blocks that
    propagate in registers; at 4096 the paired kernel holds 64 KiB of LDS),
    with row-major and transposed spectra, against the separate column passes
    and propagation on the same kite plan and data (one step of nfl fields):
    1e-13.  Two fields take the column-tile-per-XCD mapping, eight fields the
    whole-fields-per-XCD mapping."""
    from paper_2010_03901_amd import fc2d
    torch = torch_mod
    case = W.cfg_ff("kite", n)
    gpl = gpu_plan(case)
    u0 = [_pulses(case, range(nfl))]

    def run(fused, trans):
        b = fc2d.Batch([gpl], [nfl], fused_ff=fused, transposed=trans)
        _load_state(b, u0)
        b.run_ff(1.0, 0.02, 1, use_graph=False)
        torch.cuda.synchronize()
        r = [t.cpu().numpy().copy() for t in b.state(0)]
        b.close()
        return r

    ref = run(False, False)
    keep = fc2d.fc2d_tune_get(fc2d.FC2D_TUNE_FF_SHAPE, n)
    nshape = 0
    try:
        while True:
            try:
                fc2d.fc2d_tune_set(fc2d.FC2D_TUNE_FF_SHAPE, n, nshape)
            except Exception:
                break
            for trans in (False, True):
                print("\n[batch] n=%d fields %d fused shape %d transposed %d" % (n, nfl, nshape, trans), end="",
                      flush=True)
                got = run(True, trans)
                for j in (0, 1):
                    assert rel_err(got[j], ref[j]) < 1e-13
            nshape += 1
    finally:
        fc2d.fc2d_tune_set(fc2d.FC2D_TUNE_FF_SHAPE, n, keep)
    assert nshape == {1024: 6, 2048: 6, 4096: 2}[n]


def test_bench_shaped_batch_step_matches_oracle(torch_mod):
    """The batch the way the benchmark builds it, at its two largest sizes: four
    domains x {1024^2, 2048^2}, 32 fields per plan (128 per grid size, so each
    XCD takes whole fields), launch shapes from the autotuner (transposed spectra
    and the paired column kernel wherever they win), one HIP-graph step of
    dt = 0.01.  One field per (domain, size) against the oracle's step from the
    same state: 1e-11.  The oracle steps run in spawned CPU-only processes."""
    from paper_2010_03901_amd import fc2d
    torch = torch_mod
    doms = list(W.FF_DOMAINS)
    specs = [(dom, n) for n in (1024, 2048) for dom in doms]
    nfp, dt = 32, 0.01
    check = [(5 * k + 3) % nfp for k in range(len(specs))]      # the field compared per plan
    seeds = [1000 * k + f for k, f in enumerate(check)]
    print("\n[batch] oracle steps of %d (domain, size) pairs in spawned workers" % len(specs), flush=True)
    ref = oracle_pool_map(oracle_ff_step_worker, [(dom, n, s, dt) for (dom, n), s in zip(specs, seeds)])
    print("[batch] oracle done; building the GPU batch", flush=True)
    cases = [W.cfg_ff(dom, n) for dom, n in specs]
    gplans = [gpu_plan(c) for c in cases]
    batch = fc2d.Batch(gplans, [nfp] * len(specs), autotune=True)
    print("[batch] autotuned fused-kernel shapes %s, column (E, T) %s" % (
        {n: fc2d.fc2d_tune_get(fc2d.FC2D_TUNE_FF_SHAPE, n) for n in (1024, 2048)},
        {n: (fc2d.fc2d_tune_get(fc2d.FC2D_TUNE_COL_ELEMS, n), fc2d.fc2d_tune_get(fc2d.FC2D_TUNE_COL_TILE, n))
         for n in (1024, 2048)}), flush=True)
    for k, case in enumerate(cases):
        u, ut = batch.state(k)
        x = case.x0 + torch.arange(case.n, device="cuda:0", dtype=torch.float64) * case.h
        for f in range(nfp):
            _, (xc, yc, sig) = W.gaussian_pulse(case.curve, 1000 * k + f)
            u[f].copy_(torch.exp(-((x[:, None] - xc) ** 2 + (x[None, :] - yc) ** 2) / sig ** 2))
        u[check[k]].copy_(torch.from_numpy(pulse_field(case, seeds[k])))   # the oracle's own initial field
        ut.zero_()
    batch.run_ff(1.0, dt, 1, use_graph=True)
    torch.cuda.synchronize()
    try:
        for k, ((dom, n), (ou, out_)) in enumerate(zip(specs, ref)):
            u, ut = batch.state(k)
            f = check[k]
            eu = rel_err(u[f].cpu().numpy(), ou)
            et = rel_err(ut[f].cpu().numpy(), out_)
            print("[batch] %s %d^2 field %d: u %.2e u_t %.2e" % (dom, n, f, eu, et), flush=True)
            assert eu < 1e-11 and et < 1e-11, (dom, n, eu, et)
    finally:
        batch.close()
