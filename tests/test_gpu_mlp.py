"""GPU checks of the learned foot seed: training pairs against the oracle's
foot solve and features, the FP32 forward pass and gradient against the
float64 oracle network, Adam steps, training progress, and plans seeded by the
polar angle or by the trained network against the proximity-seeded plan and
the oracle (same classes, STRIP list and feet), including forced fallbacks."""
import math

import numpy as np
import pytest

import workloads as W
from gpu_common import fields, oracle_plan, rel_err
from oracle import curves as OC
from oracle import extend as OE
from oracle import mlp as OM
from oracle import plan as OP

pytestmark = pytest.mark.gpu

WIDTH = 27 * W.mlp_k1()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _dev(torch, a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def _make_data(torch, ncurves, npts, seed=0):
    from paper_2010_03901_amd import fc2d
    curves, cidx, th, eta = W.mlp_training_draws(seed, ncurves, npts, WIDTH)
    n = cidx.size
    X = torch.zeros((n, 8), dtype=torch.float32, device="cuda:0")
    Y = torch.zeros((n, 2), dtype=torch.float32, device="cuda:0")
    foot = torch.zeros((n, 2), dtype=torch.float64, device="cuda:0")
    its = torch.zeros(n, dtype=torch.int32, device="cuda:0")
    fc2d.fc2d_mlp_make_data(_dev(torch, curves), _dev(torch, cidx), _dev(torch, th), _dev(torch, eta), WIDTH,
                            X, Y, foot, its)
    torch.cuda.synchronize()
    return (curves, cidx, th, eta), X, Y, foot, its


def test_training_pairs_against_oracle(torch_mod):
    torch = torch_mod
    print("\n[mlp] training pairs 12 curves x 40 points", flush=True)
    (curves, cidx, th_s, eta_s), X, Y, foot, its = _make_data(torch, 12, 40)
    its = its.cpu().numpy()
    assert its.min() >= 1
    foot = foot.cpu().numpy()
    X = X.cpu().numpy()
    Y = Y.cpu().numpy()
    for c in range(curves.shape[0]):
        sel = cidx == c
        cv = OC.Curve("polar", curves[c])
        bd = OC.boundary_grid(cv, 4096)
        x, y, x1, y1, _, _ = cv.eval_vec(th_s[sel])
        sp = np.hypot(x1, y1)
        Qx = x + eta_s[sel] * y1 / sp
        Qy = y - eta_s[sel] * x1 / sp
        p = np.rint(np.mod(np.arctan2(Qy, Qx), 2 * math.pi) / bd["k2"]).astype(np.int64) % 4096
        th_o, eta_o, _ = OP.foot_solve(cv, bd, Qx, Qy, p, 8)
        dth = np.abs(np.mod(foot[sel, 0] - th_o + math.pi, 2 * math.pi) - math.pi)
        assert dth.max() < 1e-13
        assert np.abs(foot[sel, 1] - eta_o).max() < 1e-14
        # the points were placed at distance eta_s along the normal of theta_s
        assert np.abs(np.mod(th_o - th_s[sel] + math.pi, 2 * math.pi) - math.pi).max() < 1e-12
        assert np.abs(eta_o - eta_s[sel]).max() < 1e-13
        F = OM.features(Qx, Qy, curves[c], WIDTH)
        assert np.abs(X[sel] - F).max() <= 2e-6 * max(1.0, np.abs(F).max())
        T = OM.targets(Qx, Qy, th_o, eta_o, WIDTH, F)
        assert np.abs(Y[sel] - T).max() <= 1e-5 + 1e-6 * np.abs(T).max()


def _weights(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    w = OM.init_weights(seed) * scale
    w[np.r_[OM.LAYERS[0][0] * 64:OM.LAYERS[0][0] * 64 + 64]] = rng.normal(0, 0.1, 64)   # non-zero first bias
    return w.astype(np.float32)


@pytest.mark.parametrize("n", [1, 64, 1000])
def test_forward_and_gradient_against_oracle(torch_mod, n):
    from paper_2010_03901_amd import fc2d
    torch = torch_mod
    print("\n[mlp] forward / gradient n =", n, flush=True)
    rng = np.random.default_rng(n)
    w = _weights(3)
    Xh = rng.normal(0, 1, (n, 8)).astype(np.float32)
    Yh = rng.normal(0, 0.5, (n, 2)).astype(np.float32)
    dw, dX, dY = _dev(torch, w), _dev(torch, Xh), _dev(torch, Yh)
    out = torch.zeros((n, 2), dtype=torch.float32, device="cuda:0")
    fc2d.fc2d_mlp_forward(dw, dX, out)
    grad = torch.zeros(OM.NW, dtype=torch.float32, device="cuda:0")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda:0")
    fc2d.fc2d_mlp_loss_grad(dw, dX, dY, grad, loss)
    torch.cuda.synchronize()
    w64 = w.astype(np.float64)
    ref_out, _ = OM.forward(w64, Xh.astype(np.float64))
    assert rel_err(out.cpu().numpy(), ref_out) < 1e-5
    ref_loss, ref_grad = OM.loss_and_grad(w64, Xh.astype(np.float64), Yh.astype(np.float64))
    g = grad.cpu().numpy()
    e = np.abs(g - ref_grad).max() / np.abs(ref_grad).max()
    print("[mlp] gradient rel err %.2e, loss %.6e vs %.6e" % (e, float(loss.item()), ref_loss))
    assert e < 1e-4
    assert abs(loss.item() - ref_loss) <= 1e-5 * ref_loss


def test_adam_steps_against_oracle(torch_mod):
    from paper_2010_03901_amd import fc2d
    torch = torch_mod
    print("\n[mlp] two Adam steps", flush=True)
    rng = np.random.default_rng(8)
    n = 300
    w = _weights(4)
    Xh = rng.normal(0, 1, (n, 8)).astype(np.float32)
    Yh = rng.normal(0, 0.5, (n, 2)).astype(np.float32)
    dw = _dev(torch, w)
    m = torch.zeros_like(dw)
    v = torch.zeros_like(dw)
    hist = torch.zeros(2, dtype=torch.float32, device="cuda:0")
    lr = 1e-3
    # batch = n: every step sees every sample once
    fc2d.fc2d_mlp_train(dw, m, v, _dev(torch, Xh), _dev(torch, Yh), n, 2, 0, lr, lr, 2, hist)
    torch.cuda.synchronize()
    wr = w.astype(np.float64)
    mr = np.zeros_like(wr)
    vr = np.zeros_like(wr)
    gabs = None
    losses = []
    for t in (1, 2):
        L, g = OM.loss_and_grad(wr, Xh.astype(np.float64), Yh.astype(np.float64))
        losses.append(L)
        gabs = np.abs(g) if gabs is None else np.minimum(gabs, np.abs(g))
        OM.adam_step(wr, g, mr, vr, t, lr)
    big = gabs > 1e-3 * gabs.max()          # entries whose step direction is not decided by rounding
    assert big.mean() > 0.5
    wg = dw.cpu().numpy().astype(np.float64)
    assert np.abs(wg - wr)[big].max() < 2e-3 * lr
    assert np.allclose(hist.cpu().numpy(), losses, rtol=1e-5)


@pytest.fixture(scope="module")
def trained(torch_mod):
    """A network trained on 200 curves x 1000 points (the bench trains on 1000 x 1000)."""
    from paper_2010_03901_amd import fc2d
    torch = torch_mod
    print("\n[mlp] training 200 x 1000 pairs", flush=True)
    _, X, Y, _, its = _make_data(torch, 200, 1000)
    assert int(its.min().item()) >= 1
    w = _dev(torch, OM.init_weights(0).astype(np.float32))
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    steps = 6000
    hist = torch.zeros(steps, dtype=torch.float32, device="cuda:0")
    fc2d.fc2d_mlp_train(w, m, v, X, Y, 4096, steps, 0, 3e-3, 1e-5, steps, hist)
    h = hist.cpu().numpy()
    print("[mlp] loss first %.3e last %.3e" % (h[:50].mean(), h[-50:].mean()))
    return w.cpu().numpy(), h


def test_training_reduces_loss(trained):
    _, h = trained
    assert np.all(np.isfinite(h))
    assert h[-100:].mean() < 0.05 * h[:20].mean()


def _plan(case, **kw):
    from paper_2010_03901_amd import fc2d
    grid = fc2d.make_grid(case.x0, case.y0, case.h, case.n, case.n)
    return fc2d.Plan(fc2d.make_curve(*case.curve), grid, d=case.d, C_=case.C, B=case.B, k1=case.k1, M=case.M, **kw)


def _same_plan(a, b):
    from paper_2010_03901_amd import fc2d
    assert np.array_equal(fc2d.fc2d_plan_classes(a), fc2d.fc2d_plan_classes(b))
    ia, tha, ea, _ = fc2d.fc2d_plan_strip(a)
    ib, thb, eb, sb = fc2d.fc2d_plan_strip(b)
    assert np.array_equal(ia, ib)
    assert np.abs(np.mod(tha - thb + math.pi, 2 * math.pi) - math.pi).max() < 1e-13
    assert np.abs(ea - eb).max() < 1e-14
    dp = np.abs(((sb - thb / b.info.k2) + b.info.B / 2) % b.info.B - b.info.B / 2)
    assert dp.max() <= 0.5 + 1e-9


@pytest.fixture(scope="module")
def rnd1024(torch_mod):
    case, opl = oracle_plan("rnd1024", W.cfg_mlp, 1024)
    print("\n[mlp] plans rnd1024", flush=True)
    return case, opl, _plan(case)


def test_polar_seed_plan_matches(rnd1024):
    from paper_2010_03901_amd import fc2d
    case, opl, prox = rnd1024
    pol = _plan(case, seed=fc2d.FC2D_SEED_POLAR)
    _same_plan(prox, pol)
    assert np.array_equal(fc2d.fc2d_plan_classes(pol), opl.cls)
    assert pol.info.n_fallback == 0


def _classify_kernel_ms(case, reps=3, **kw):
    """Smallest total time of the plan's classification kernels (HIP events of
    the library's tracer) over reps plan builds."""
    from paper_2010_03901_amd import fc2d
    best = None
    for _ in range(reps):
        fc2d.fc2d_trace_begin()
        p = _plan(case, **kw)
        tr = fc2d.fc2d_trace_end()
        p.close()
        t = sum(v for k, v in tr if k.startswith("k_"))
        best = t if best is None else min(best, t)
    return best


def test_mlp_seed_plan_matches_and_saves_newton_steps(rnd1024, trained):
    """The MLP-seeded plan equals the proximity-seeded plan and the oracle; the
    trained seed lets most points finish after two Newton steps, fewer than the
    polar-angle seed it replaces.  Against the paper's seed (proximity map +
    T(tau), the default) the gain is in the classification kernels: the
    learned seed needs no proximity scatter, so its kernels take less time."""
    from paper_2010_03901_amd import fc2d
    case, opl, prox = rnd1024
    w, _ = trained
    pol = _plan(case, seed=fc2d.FC2D_SEED_POLAR)
    mlp = _plan(case, seed=fc2d.FC2D_SEED_MLP, mlp_weights=w)
    _same_plan(prox, mlp)
    assert np.array_equal(fc2d.fc2d_plan_classes(mlp), opl.cls)
    assert np.array_equal(fc2d.fc2d_plan_strip(mlp)[0], opl.strip_idx)
    ip, im = pol.info, mlp.info
    assert ip.n_solved == im.n_solved
    rate = im.n_fallback / im.n_solved
    it_pol = ip.newton_iters / ip.n_solved
    it_mlp = im.newton_iters / im.n_solved
    it_prox = prox.info.newton_iters / prox.info.n_solved
    print("[mlp] rnd1024 solved %d, fallback %.4f, Newton steps/point: proximity+T(tau) %.2f, polar %.2f, MLP %.2f"
          % (im.n_solved, rate, it_prox, it_pol, it_mlp))
    assert rate < 0.05
    assert it_mlp < it_pol
    t_prox = _classify_kernel_ms(case)
    t_mlp = _classify_kernel_ms(case, seed=fc2d.FC2D_SEED_MLP, mlp_weights=w)
    print("[mlp] rnd1024 classification kernels: proximity+T(tau) %.3f ms, MLP %.3f ms (%.2fx)"
          % (t_prox, t_mlp, t_prox / t_mlp))
    assert t_mlp < t_prox


def test_mlp_seed_plan_extension_parity(rnd1024, trained, torch_mod):
    from paper_2010_03901_amd import fc2d
    torch = torch_mod
    case, opl, _ = rnd1024
    w, _ = trained
    mlp = _plan(case, seed=fc2d.FC2D_SEED_MLP, mlp_weights=w)
    funcs = [W.f_cfg1, W.f_star(1)]
    fg, fbo = fields(case, funcs, OP.boundary_points(opl))
    _, fbg = fields(case, funcs, fc2d.fc2d_boundary_points(mlp))
    out = torch.zeros((2, case.n, case.n), dtype=torch.float64, device="cuda:0")
    fc2d.fc2d_extend(mlp, _dev(torch, fg), _dev(torch, fbg), out)
    torch.cuda.synchronize()
    for k in range(2):
        e = rel_err(out[k].cpu().numpy(), OE.extend(opl, fg[k], fbo[k]))
        print("[mlp] extension parity field %d rel err %.2e" % (k, e))
        assert e < 1e-11


@pytest.mark.parametrize("how", ["nan_weights", "negative_tol"])
def test_forced_fallback_keeps_results(rnd1024, trained, how):
    from paper_2010_03901_amd import fc2d
    case, _, prox = rnd1024
    w, _ = trained
    if how == "nan_weights":
        bad = np.full_like(w, np.nan)
        pl = _plan(case, seed=fc2d.FC2D_SEED_MLP, mlp_weights=bad)
    else:
        pl = _plan(case, seed=fc2d.FC2D_SEED_MLP, mlp_weights=w, mlp_tol=-1.0)
    assert pl.info.n_fallback == pl.info.n_solved
    _same_plan(prox, pl)


def test_mlp_plan_full_size_parity(trained, torch_mod):
    """The learned-seed workload at full size (held-out curve, 4096^2, B = 8192),
    in the launch configuration the benchmark times: classes and STRIP list
    against the oracle plan, and the fused extension + FFT of one field
    against numpy's FFT of the oracle's extension."""
    from paper_2010_03901_amd import fc2d
    torch = torch_mod
    w, _ = trained
    print("\n[mlp] rnd4096 oracle plan", flush=True)
    case, opl = oracle_plan("rnd4096", W.cfg_mlp, 4096)
    mlp = _plan(case, seed=fc2d.FC2D_SEED_MLP, mlp_weights=w)
    assert np.array_equal(fc2d.fc2d_plan_classes(mlp), opl.cls)
    idx, th, eta, _ = fc2d.fc2d_plan_strip(mlp)
    assert np.array_equal(idx, opl.strip_idx)
    assert np.abs(np.mod(th - opl.strip_theta + math.pi, 2 * math.pi) - math.pi).max() < 1e-13
    assert np.abs(eta - opl.strip_eta).max() < 1e-14
    f = W.f_star(2)
    fg, fbo = fields(case, [f], OP.boundary_points(opl))
    _, fbg = fields(case, [f], fc2d.fc2d_boundary_points(mlp))
    dfg = _dev(torch, fg)
    spec = torch.zeros((1, case.n, case.n // 2 + 1), dtype=torch.complex128, device="cuda:0")
    fc2d.fc2d_extend_fft(mlp, dfg, _dev(torch, fbg), dfg, spec)
    torch.cuda.synchronize()
    ref = np.fft.rfft2(OE.extend(opl, fg[0], fbo[0]))
    e = rel_err(spec[0].cpu().numpy(), ref)
    print("[mlp] rnd4096 fallback %.4f, extend_fft rel err %.2e" % (mlp.info.n_fallback / mlp.info.n_solved, e))
    assert e < 1e-11
