"""Host-side checks of the C-ABI library: it loads, exports every entry point
that include/fc2d.h declares, and rejects bad arguments before touching a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fc2d.h")
LIB = os.path.join(ROOT, "paper_2010_03901_amd", "libfc2d.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libfc2d.so not built (run __graft_entry__.build())")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*\b([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n.startswith(("fc2d_", "ff_"))))


def test_header_declares_the_path():
    names = declared_functions()
    for must in ("fc2d_plan_create", "fc2d_extend", "fc2d_fft", "ff_propagate", "fc2d_spectral_apply"):
        assert must in names


def test_every_declared_symbol_is_exported():
    lib = C.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_version_and_strerror():
    from paper_2010_03901_amd import fc2d
    lib = fc2d._lib()
    assert lib.fc2d_version() == 100
    assert lib.fc2d_strerror(fc2d.FC2D_E_GEOMETRY) == b"inadmissible geometry"


def test_argument_errors_without_gpu():
    from paper_2010_03901_amd import fc2d
    lib = fc2d._lib()
    g = fc2d.make_grid(0, 0, 0.1, 100, 64)          # 100 is not a power of two
    assert lib.fc2d_fft(C.byref(g), C.c_void_p(8), C.c_void_p(16), fc2d.FC2D_FORWARD, 1, None) == fc2d.FC2D_E_ARG
    assert b"power of two" in lib.fc2d_last_error()
    g2 = fc2d.make_grid(0, 0, 0.1, 64, 64)
    assert lib.fc2d_fft(C.byref(g2), C.c_void_p(8), C.c_void_p(8), fc2d.FC2D_FORWARD, 1, None) == fc2d.FC2D_E_ARG
    assert lib.fc2d_fft(C.byref(g2), C.c_void_p(8), C.c_void_p(16), 7, 1, None) == fc2d.FC2D_E_ARG
    assert lib.fc2d_fft(C.byref(g2), None, None, fc2d.FC2D_FORWARD, 0, None) == fc2d.FC2D_OK   # empty batch
    h = C.c_void_p()
    assert lib.fc2d_plan_create(None, C.byref(g2), 5, 27, None, None, C.byref(h)) == fc2d.FC2D_E_ARG
    cv = fc2d.make_curve("polar", [1.0])
    assert lib.fc2d_plan_create(C.byref(cv), C.byref(g2), 5, 27, None, None, None) == fc2d.FC2D_E_ARG
    o = fc2d.fc2d_opts()
    lib.fc2d_opts_default(C.byref(g2), C.byref(o))
    o.M = 20                                           # beyond the supported interpolation size
    assert lib.fc2d_plan_create(C.byref(cv), C.byref(g2), 5, 27, C.byref(o), None, C.byref(h)) == fc2d.FC2D_E_ARG
    assert lib.fc2d_spectral_apply(C.byref(g2), 99, C.c_void_p(8), C.c_void_p(8), 1, None) == fc2d.FC2D_E_ARG


def test_opts_default_follows_the_paper():
    from paper_2010_03901_amd import fc2d
    lib = fc2d._lib()
    g = fc2d.make_grid(-1.5, -1.5, 3.0 / 128, 128, 128)
    o = fc2d.fc2d_opts()
    lib.fc2d_opts_default(C.byref(g), C.byref(o))
    assert (o.n_r, o.Z, o.n_os, o.mf) == (6, 12, 20, 20)
    assert o.k1 == g.h and o.B == 256
    assert o.seed == fc2d.FC2D_SEED_PROXIMITY and o.mlp_tol == 1e-13 and not o.mlp_weights


def test_seed_options_rejected_without_gpu():
    from paper_2010_03901_amd import fc2d
    lib = fc2d._lib()
    g = fc2d.make_grid(-1.5, -1.5, 3.0 / 128, 128, 128)
    h = C.c_void_p()
    o = fc2d.fc2d_opts()
    lib.fc2d_opts_default(C.byref(g), C.byref(o))
    polar = fc2d.make_curve("polar", [1.0])
    kite = fc2d.make_curve("cartesian", ([-0.65, 1.0, 0.0, 0.65], [0.0, 0.0, 1.5]))
    o.seed = fc2d.FC2D_SEED_MLP                       # no weights
    assert lib.fc2d_plan_create(C.byref(polar), C.byref(g), 5, 27, C.byref(o), None, C.byref(h)) == fc2d.FC2D_E_ARG
    o.seed = fc2d.FC2D_SEED_POLAR                     # not a polar curve
    assert lib.fc2d_plan_create(C.byref(kite), C.byref(g), 5, 27, C.byref(o), None, C.byref(h)) == fc2d.FC2D_E_ARG
    o.seed = 7
    assert lib.fc2d_plan_create(C.byref(polar), C.byref(g), 5, 27, C.byref(o), None, C.byref(h)) == fc2d.FC2D_E_ARG
    assert b"seed" in lib.fc2d_last_error()


def test_mlp_argument_errors_without_gpu():
    from paper_2010_03901_amd import fc2d
    lib = fc2d._lib()
    p = C.c_void_p(256)
    assert lib.fc2d_mlp_forward(p, p, -1, p, None) == fc2d.FC2D_E_ARG
    assert lib.fc2d_mlp_forward(None, None, 0, None, None) == fc2d.FC2D_OK          # nothing to do
    assert lib.fc2d_mlp_loss_grad(p, p, p, 0, p, p, None) == fc2d.FC2D_E_ARG
    assert lib.fc2d_mlp_train(p, p, p, p, p, 10, 0, 1, 0, 1e-3, 1e-5, 1, None, None) == fc2d.FC2D_E_ARG   # batch 0
    assert lib.fc2d_mlp_train(p, p, p, p, p, 10, 4, 0, 0, 1e-3, 1e-5, 1, None, None) == fc2d.FC2D_OK     # no steps
    assert lib.fc2d_mlp_make_data(p, 1, 8, p, p, p, 5, 0.0, p, p, None, None, None) == fc2d.FC2D_E_ARG   # width 0


def test_geometry_rejected_before_any_device_work():
    """Admissibility (Sec. 3.1): C k1 above 0.9 x the exterior reach, or a box
    that does not hold Omega u V+, fail with FC2D_E_GEOMETRY on the host."""
    from paper_2010_03901_amd import fc2d
    import workloads as W
    lib = fc2d._lib()
    star = fc2d.make_curve(*W.star5())
    g = fc2d.make_grid(-1.6, -1.6, 3.2 / 256, 256, 256)
    h = C.c_void_p()
    o = fc2d.fc2d_opts()
    lib.fc2d_opts_default(C.byref(g), C.byref(o))
    o.k1 = 0.01                                       # C k1 = 0.27 > 0.9 x reach 0.072
    assert lib.fc2d_plan_create(C.byref(star), C.byref(g), 5, 27, C.byref(o), None, C.byref(h)) == fc2d.FC2D_E_GEOMETRY
    assert b"reach" in lib.fc2d_last_error()
    small = fc2d.make_grid(-1.2, -1.2, 2.4 / 256, 256, 256)   # the star reaches 1.3
    lib.fc2d_opts_default(C.byref(small), C.byref(o))
    o.k1 = 0.002
    assert lib.fc2d_plan_create(C.byref(star), C.byref(small), 5, 27, C.byref(o), None, C.byref(h)) == fc2d.FC2D_E_GEOMETRY
    assert b"box" in lib.fc2d_last_error()


def test_tuning_knobs_host_side():
    """The launch-shape knobs are host state: set, read back and restored
    without a GPU; invalid settings are refused."""
    from paper_2010_03901_amd import fc2d
    lib = fc2d._lib()
    v = C.c_int()
    for knob, good, bad in ((fc2d.FC2D_TUNE_STRIP_FIELDS, 4, -1), (fc2d.FC2D_TUNE_STRIP_WINDOW, 16, -3)):
        assert lib.fc2d_tune_get(knob, 0, C.byref(v)) == fc2d.FC2D_OK
        old = v.value
        assert lib.fc2d_tune_set(knob, 0, good) == fc2d.FC2D_OK
        assert lib.fc2d_tune_get(knob, 0, C.byref(v)) == fc2d.FC2D_OK and v.value == good
        assert lib.fc2d_tune_set(knob, 0, bad) == fc2d.FC2D_E_ARG
        assert lib.fc2d_tune_set(knob, 0, old) == fc2d.FC2D_OK
    # column shapes: only compiled (E, T) pairs
    assert lib.fc2d_tune_set(fc2d.FC2D_TUNE_COL_TILE, 1024, 3) == fc2d.FC2D_E_ARG
    assert lib.fc2d_tune_set(99, 0, 1) == fc2d.FC2D_E_ARG


def test_poisson_argument_errors_without_gpu():
    from paper_2010_03901_amd import fc2d
    lib = fc2d._lib()
    assert lib.fc2d_poisson_solve(None, None, None, None, 64, None, 1, None, None) == fc2d.FC2D_E_ARG
    assert lib.fc2d_poisson_nodes(None, 64, None) == fc2d.FC2D_E_ARG


def test_spectrum_pitch_below_half_width_refused():
    from paper_2010_03901_amd import fc2d
    lib = fc2d._lib()
    g = fc2d.make_grid(0.0, 0.0, 0.01, 64, 64)
    assert lib.fc2d_fft_ld(C.byref(g), C.c_void_p(8), C.c_void_p(16), fc2d.FC2D_FORWARD, 32, 1, None) == fc2d.FC2D_E_ARG
    assert b"spec_ld" in lib.fc2d_last_error()
