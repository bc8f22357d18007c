"""The plan's lists built on the device (row runs, pair classes, STRIP lists
and their order by theta; the red stars' line scans and crossings) through what
the C ABI shows of them, and the per-phase plan timers.  The classes, STRIP
lists, feet and squares themselves are held to the oracle in
test_gpu_parity.py; here: the structure the kernels rely on."""
import time

import numpy as np
import pytest

import workloads as W
from gpu_common import gpu_plan

pytestmark = pytest.mark.gpu

CASES = {"disc128": (W.cfg_disc128,), "star320": (W.cfg_star, 320), "kite256": (W.cfg_kite, 256),
         "mlp1024": (W.cfg_mlp, 1024)}


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("name", list(CASES))
def test_strip_list_and_counts(torch_mod, name):
    """Row-major STRIP list: strictly increasing, exactly the STRIP-class points,
    feet in [0, 2 pi), 0 < eta <= C k1; the class counts add up."""
    from paper_2010_03901_amd import fc2d
    case = CASES[name][0](*CASES[name][1:])
    pl = gpu_plan(case)
    cls = fc2d.fc2d_plan_classes(pl)
    idx, th, eta, seed = fc2d.fc2d_plan_strip(pl)
    inf = pl.info
    assert idx.size == inf.n_strip
    assert np.all(np.diff(idx) > 0)
    assert np.array_equal(np.flatnonzero(cls.ravel() == 2), idx)
    assert inf.n_in == int((cls == 1).sum()) and inf.n_far == int((cls == 0).sum())
    assert inf.n_in + inf.n_far + inf.n_strip == cls.size
    assert th.min() >= 0.0 and th.max() <= 2 * np.pi   # a foot a rounding below 0 wraps to 2 pi
    assert eta.min() > 0.0 and eta.max() <= inf.C * inf.k1 * (1 + 1e-12)
    assert seed.min() >= 0 and seed.max() < inf.B
    pl.close()


def test_plan_phase_timers(torch_mod):
    """fc2d_plan_info.t_ms: one non-negative host wall time per phase, together
    within the wall time around fc2d_plan_create."""
    from paper_2010_03901_amd import fc2d
    case = W.cfg_star(320)
    gpu_plan(case).close()                       # tables and code objects warm
    torch_mod.cuda.synchronize()
    t0 = time.perf_counter()
    pl = gpu_plan(case)
    wall_ms = (time.perf_counter() - t0) * 1e3
    t = [pl.info.t_ms[k] for k in range(len(fc2d.PLAN_PHASES))]
    print("\n[plan] phases %s, wall %.2f ms" % (dict(zip(fc2d.PLAN_PHASES, [round(x, 3) for x in t])), wall_ms))
    assert all(x >= 0.0 for x in t) and sum(t) > 0.0
    assert sum(t) <= wall_ms * 1.01 + 0.1
    pl.close()
