"""Throughput of the 2D-FC hot path on one MI355X: extension + forward 2D FFT.

Workload (the star domain of the paper-derived benchmark): r(t) = 1 + 0.3 cos 5t,
B = 2048 boundary points, box [-1.6, 1.6]^2 on a 1024 x 1024 float64 grid, d = 5,
C = 27, M = 8, normal step k1 = 0.0024 (0.9 x exterior reach / C).  A step
extends nf fields f = sin(k1 x) cos(k2 y) + x^3 y ((k1, k2) drawn by seed) and
takes their forward 2D FFT; inputs are resident in HBM before timing.

Prints one JSON line (metric, value = extended grid points per second, roofline
of the dominant kernel from HIP-event kernel times, cpu_baseline = the oracle
timed on a bounded sample on the host; the same leg compares sampled outputs
of the timed runs with the oracle: max_rel_err_vs_oracle).  Further legs: the
batched Fourier-Forwarding step against its plain per-plan form on identical
work, the learned foot seed, and the full Poisson solve.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COUNTERS = os.path.join(ROOT, "profiles", "star1024_extend_fft_counters.json")


# sources of the extension and FFT kernels whose HBM counters are committed
KERNEL_SOURCES = ["kernels_extend.hip", "kernels_fft.hip", "dd.h", "geom.h", "internal.h", "lagrange_dev.h"]


def source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2010_03901_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per dispatch from the committed rocprofv3 counter runs, or None
    when they are missing or the kernels changed since they were taken.  kernel
    is a tracer name; the timed path's instantiation is picked by its template
    arguments: the masked, row-major row pass, and the forward column pass on
    128-byte-aligned rows (non-temporal form)."""
    try:
        with open(COUNTERS) as fh:
            c = json.load(fh)
    except (OSError, ValueError):
        return None
    if c.get("source_hash") != source_hash():
        return None
    base = kernel.replace("_ext", "")
    for name, v in c["kernels"].items():
        if name.split("<")[0] != base:
            continue
        targs = [a.strip() for a in name[name.find("<") + 1: name.rfind(">")].split(",")] if "<" in name else []
        if base == "k_rows_r2c" and (len(targs) < 5 or targs[3] != ("true" if kernel.endswith("_ext") else "false")
                                     or targs[4] != "false"):
            continue
        if base == "k_cols" and (len(targs) < 5 or targs[3] != "false" or targs[4] != "true"):
            continue
        return v["traffic_bytes"]
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--nf", type=int, default=128, help="fields per step")
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the cpu_baseline leg (the oracle timing and the oracle checks of sampled outputs)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched Fourier-Forwarding measurement")
    ap.add_argument("--ff-fields", type=int, default=128, help="fields per (grid size) in the batched run")
    ap.add_argument("--ff-steps", type=int, default=100)
    ap.add_argument("--cpu-sample-fields", type=int, default=96)
    ap.add_argument("--col-tile", type=int, default=0, help="columns per block of the column FFT pass (0 = default)")
    ap.add_argument("--col-elems", type=int, default=0, help="elements per thread of the column FFT pass (0 = default)")
    ap.add_argument("--strip-fields", type=int, default=-1, help="fields per thread of the strip kernel (-1 = default)")
    ap.add_argument("--no-mlp", action="store_true", help="skip the learned-seed measurement")
    ap.add_argument("--mlp-curves", type=int, default=1000)
    ap.add_argument("--mlp-steps", type=int, default=20000)
    ap.add_argument("--mlp-batch", type=int, default=4096)
    ap.add_argument("--mlp-fields", type=int, default=8)
    ap.add_argument("--no-poisson", action="store_true", help="skip the full Poisson solve measurement")
    ap.add_argument("--no-ff-solver", action="store_true", help="skip the Fourier Forwarding solver measurement")
    ap.add_argument("--ff-solver-n", type=int, default=1024, help="grid of the Fourier Forwarding solver run")
    ap.add_argument("--poisson-n", type=int, default=2048, help="grid of the full Poisson solve")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 1 GiB device copy first (known-size kernel for counter calibration)")
    return ap.parse_args()


def algorithmic_bytes(name, n, nf, info):
    """Bytes a kernel must move per launch (float64 / complex128 arrays)."""
    npts = n * n
    half = n * (n // 2 + 1)
    if name == "k_rows_r2c":
        return nf * (8 * npts + 16 * half)
    if name == "k_rows_r2c_ext":     # read f at IN points and the STRIP values, write the half spectrum
        return nf * (8 * info.n_in + 8 * info.n_strip + 16 * half)
    if name == "k_cols":
        return nf * 32 * half
    if name == "k_mask":            # out of place: read IN, write IN and FAR
        return nf * (8 * info.n_in + 8 * (info.n_in + info.n_far))
    if name == "k_strip":           # write the STRIP values, read (index, theta, eta)
        return nf * 8 * info.n_strip + 20 * info.n_strip
    if name == "k_match":
        return nf * 8 * (info.B * 8 * 8 + info.B * info.d)
    return 0


def cpu_baseline(case, nf_sample, checks, ff_check):
    """The oracle (plain NumPy, one thread) on nf_sample fields of the same
    workload, timed; the same leg compares sampled outputs of the timed GPU
    runs with the oracle's: checks maps a field seed to {name: GPU array} with
    the fused path's half spectrum ("spectrum") and the plain path's extension
    ("extension") of that field; ff_check holds one field of the batched
    Fourier-Forwarding step and of its plain form with the initial state."""
    from threadpoolctl import threadpool_limits
    import numpy as np
    import workloads as W
    from oracle import extend as OE, fcgram, ff as OF, plan as OP, spectral as OS
    from oracle.curves import Curve
    rel = lambda a, b: float(np.abs(a - b).max() / np.abs(b).max())
    res = {}
    with threadpool_limits(limits=1):
        pl = OP.make_plan(Curve(*case.curve), OP.Grid(case.x0, case.y0, case.h, case.n, case.n),
                          fcgram.load_tables(case.d), case.B, k1=case.k1, M=case.M)
        bp = OP.boundary_points(pl)
        fields = []
        for s in range(nf_sample):
            f = W.f_star(s)
            fields.append((W.grid_values(case, f), f(bp[:, 0], bp[:, 1])))
        kept = {}
        t0 = time.perf_counter()
        for s, (fg, fb) in enumerate(fields):
            ext = OE.extend(pl, fg, fb)
            spec = OS.fft2_forward(ext)
            if s in checks:
                kept[s] = (ext, spec)
        dt = time.perf_counter() - t0
        errs = {"spectrum": [], "extension": []}
        in_bitwise = True
        ins = pl.cls == OP.IN
        for s, gpu in checks.items():
            ext, spec = kept[s]
            errs["spectrum"].append(rel(gpu["spectrum"], spec))
            errs["extension"].append(rel(gpu["extension"], ext))
            in_bitwise &= bool(np.array_equal(gpu["extension"][ins], ext[ins]))
        res["checks"] = {"fields": sorted(checks), "fused_spectrum_max_rel_err": max(errs["spectrum"]),
                         "plain_extension_max_rel_err": max(errs["extension"]), "in_points_bitwise": in_bitwise}
        if ff_check is not None:
            fc = ff_check
            c = fc["case"]
            fpl = OP.make_plan(Curve(*c.curve), OP.Grid(c.x0, c.y0, c.h, c.n, c.n), fcgram.load_tables(c.d), c.B,
                               k1=c.k1, M=c.M)
            ou, out_ = OF.ff_step(fpl, fc["u0"], np.zeros_like(fc["u0"]), fc["dt"])
            res["ff_check"] = {"field": fc["name"], "batched_u": rel(fc["batched"][0], ou),
                               "batched_ut": rel(fc["batched"][1], out_)}
            if "plain" in fc:
                res["ff_check"].update(plain_u=rel(fc["plain"][0], ou), plain_ut=rel(fc["plain"][1], out_))
    res["baseline"] = {"value": nf_sample * case.n * case.n / dt, "unit": "points/s", "cores": 1, "kind": "oracle",
                       "sample": "%d fields of the %dx%d star workload (plan excluded), extend + rfft2, one thread"
                                 % (nf_sample, case.n, case.n)}
    return res


def run_ff(args):
    """Batched Fourier Forwarding: 4 domains x 4 grid sizes, ff_fields fields per
    size (domains round-robin), Gaussian pulses, dt = 0.01, c = 1.  The same
    step is timed two ways on identical plans, fields and initial data:
      plain    one plan at a time through the per-plan entry points
               (boundary values, fused extension + FFT of u and u_t,
               propagation, inverse FFTs), no graph, default launch shapes;
      batched  the batch: persistent multi-plan kernels, the fused column +
               propagation kernel, one HIP-graph replay per step, launch
               shapes from the autotuner.
    The first step of one 2048^2 field of each is kept for the oracle check."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2010_03901_amd import fc2d
    sizes = [256, 512, 1024, 2048]
    doms = list(W.FF_DOMAINS)
    plans, nf, cases = [], [], []
    t0 = time.perf_counter()
    for n in sizes:
        for k, dom in enumerate(doms):
            m = args.ff_fields // len(doms) + (1 if k < args.ff_fields % len(doms) else 0)
            case = W.cfg_ff(dom, n)
            grid = fc2d.make_grid(case.x0, case.y0, case.h, case.n, case.n)
            plans.append(fc2d.Plan(fc2d.make_curve(*case.curve), grid, d=case.d, C_=case.C, B=case.B, k1=case.k1,
                                   M=case.M))
            nf.append(m)
            cases.append(case)
    plan_s = time.perf_counter() - t0
    dt, c = 0.01, 1.0
    kc = len(cases) - 2                      # the checked field: first field of the 2048^2 kite plan
    x_c = cases[kc].x0 + np.arange(cases[kc].n) * cases[kc].h
    f_c, _ = W.gaussian_pulse(cases[kc].curve, 1000 * kc)
    u0_c = f_c(*np.meshgrid(x_c, x_c, indexing="ij"))

    def load(k, u, ut):
        """Seeded Gaussian pulses inside the domain (built on the device), u_t = 0."""
        case = cases[k]
        x = case.x0 + torch.arange(case.n, device="cuda:0", dtype=torch.float64) * case.h
        for f in range(nf[k]):
            _, (xc, yc, sig) = W.gaussian_pulse(case.curve, 1000 * k + f)
            u[f].copy_(torch.exp(-((x[:, None] - xc) ** 2 + (x[None, :] - yc) ** 2) / sig ** 2))
        if k == kc:
            u[0].copy_(torch.from_numpy(u0_c))
        ut.zero_()

    def timed(step, steps):
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        step(steps)
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / steps

    # ---- plain: per-plan entry points, default launch shapes, no graph ----
    state = []
    for k, (case, m) in enumerate(zip(cases, nf)):
        u = torch.empty((m, case.n, case.n), dtype=torch.float64, device="cuda:0")
        ut = torch.empty_like(u)
        load(k, u, ut)
        fbu = torch.empty((m, plans[k].info.n_bdry), dtype=torch.float64, device="cuda:0")
        state.append((u, ut, fbu, torch.empty_like(fbu)))
    smax = max(m * cs.n * (cs.n // 2 + 1) for m, cs in zip(nf, cases))
    sbuf = torch.empty(2 * smax, dtype=torch.complex128, device="cuda:0")

    def plain_steps(steps):
        for _ in range(steps):
            for k, (case, m) in enumerate(zip(cases, nf)):
                u, ut, fbu, fbt = state[k]
                g = plans[k].grid
                su = sbuf[: m * case.n * (case.n // 2 + 1)].view(m, case.n, case.n // 2 + 1)
                st = sbuf[smax: smax + m * case.n * (case.n // 2 + 1)].view(m, case.n, case.n // 2 + 1)
                fc2d.fc2d_boundary_values(plans[k], u, fbu)
                fc2d.fc2d_boundary_values(plans[k], ut, fbt)
                fc2d.fc2d_extend_fft(plans[k], u, fbu, u, su)
                fc2d.fc2d_extend_fft(plans[k], ut, fbt, ut, st)
                fc2d.ff_propagate(g, c, dt, su, st, su, st)
                fc2d.fc2d_fft(g, su, u, fc2d.FC2D_INVERSE)
                fc2d.fc2d_fft(g, st, ut, fc2d.FC2D_INVERSE)

    plain_steps(1)                                     # first step: kept for the oracle check
    torch.cuda.synchronize()
    plain_first = (state[kc][0][0].cpu().numpy(), state[kc][1][0].cpu().numpy())
    plain_n = min(args.ff_steps, 20)
    ms_plain = timed(plain_steps, plain_n)
    pts = 2 * sum(m * cs.n * cs.n for m, cs in zip(nf, cases))
    del state, sbuf
    torch.cuda.empty_cache()

    # ---- batched: persistent kernels, fused spectral step, graph, autotuned shapes ----
    t0 = time.perf_counter()
    batch = fc2d.Batch(plans, nf, autotune=True)
    tune_s = time.perf_counter() - t0
    for k in range(len(cases)):
        load(k, *batch.state(k))
    torch.cuda.synchronize()
    pts_b, _, sf = batch.info()
    assert pts_b == pts
    batch.run_ff(c, dt, 1, use_graph=True)          # capture + first step: kept for the oracle check
    torch.cuda.synchronize()
    bu, but = batch.state(kc)
    batched_first = (bu[0].cpu().numpy(), but[0].cpu().numpy())
    ms = timed(lambda steps: batch.run_ff(c, dt, steps, use_graph=True), args.ff_steps)
    _, nl, _ = batch.info()
    tiles = {n: (fc2d.fc2d_tune_get(fc2d.FC2D_TUNE_COL_ELEMS, n), fc2d.fc2d_tune_get(fc2d.FC2D_TUNE_COL_TILE, n))
             for n in sizes}
    ffs = {n: fc2d.fc2d_tune_get(fc2d.FC2D_TUNE_FF_SHAPE, n) for n in sizes}
    batch.close()
    for p in plans:
        p.close()
    ff_check = {"case": cases[kc], "name": "%s field 0" % cases[kc].name, "u0": u0_c, "dt": dt,
                "batched": batched_first, "plain": plain_first}
    return {"points_per_s": pts / (ms * 1e-3), "ms_per_step": ms, "points_per_step": pts,
            "plain_points_per_s": pts / (ms_plain * 1e-3), "plain_ms_per_step": ms_plain, "plain_steps": plain_n,
            "speedup_batched_vs_plain": ms_plain / ms,
            "fields": int(sum(nf)), "steps": args.ff_steps, "dt": dt, "launches_per_step": nl, "graph": True,
            "autotuned": {"col_elems_tile": tiles, "ff_shape": ffs, "strip_fields_per_thread": sf},
            "plan_s": plan_s, "batch_create_and_tune_s": tune_s,
            "workload": "disc, star5, kite(0.65,1.5), ellipse(1,0.5) on [-2,2]^2 at 256^2..2048^2, "
                        "Gaussian pulses, u and u_t extended each step",
            "note": "throughput of the step; each step matches the oracle's step from the same state; the "
                    "iterated state takes its later boundary values from the full-box field (the near-boundary "
                    "solver of Sec. 4.2 is the separate fc2d_ff_* entry point, timed in ff_solver)"}, ff_check


def run_poisson(args):
    """Full Poisson solve (Sec. 4.1) on the Poisson workload: kite(0.65, 1.5) in
    its fitted box (poisson_n^2, d = 5, M = 8, B by the workload's rule), one
    field, manufactured solution u = sin(2 pi x) sin(2 pi y) / (8 pi^2) (so
    f = -sin(2 pi x) sin(2 pi y), g = u on Gamma), nb = N Nystrom nodes as in
    the paper.  Reports the wall time of a solve (it synchronises), the GMRES
    iterations, per-kernel times (HIP events) and the relative l2 / l_inf error
    over the IN points against the exact solution."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2010_03901_amd import fc2d
    case = W.cfg_kite(args.poisson_n)
    grid = fc2d.make_grid(case.x0, case.y0, case.h, case.n, case.n)
    t0 = time.perf_counter()
    plan = fc2d.Plan(fc2d.make_curve(*case.curve), grid, d=case.d, C_=case.C, B=case.B, k1=case.k1, M=case.M)
    plan_s = time.perf_counter() - t0
    nb = case.n
    ue = lambda x, y: np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y) / (8 * np.pi ** 2)
    f = lambda x, y: -np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y)
    x = case.x0 + np.arange(case.n) * case.h
    y = case.y0 + np.arange(case.n) * case.h
    X, Y = np.meshgrid(x, y, indexing="ij")
    bp = fc2d.fc2d_boundary_points(plan)
    q = fc2d.fc2d_poisson_nodes(plan, nb)
    fg = torch.from_numpy(f(X, Y)[None]).to("cuda:0")
    fb = torch.from_numpy(f(bp[:, 0], bp[:, 1])[None]).to("cuda:0")
    gn = torch.from_numpy(ue(q[:, 0], q[:, 1])[None]).to("cuda:0")
    u = torch.empty_like(fg)
    fc2d.fc2d_poisson_solve(plan, fg, fb, gn, u)            # warm-up
    reps = 3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        it = fc2d.fc2d_poisson_solve(plan, fg, fb, gn, u)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    fc2d.fc2d_trace_begin()
    fc2d.fc2d_poisson_solve(plan, fg, fb, gn, u)
    tr = fc2d.fc2d_trace_end()
    per = {}
    for name, t in tr:
        if name != "begin":
            per[name] = per.get(name, 0.0) + t
    # four fields in one call (their double-layer sums share the geometry work)
    u4 = torch.empty((4,) + tuple(fg.shape[1:]), dtype=fg.dtype, device=fg.device)
    fg4, fb4, gn4 = fg.repeat(4, 1, 1), fb.repeat(4, 1), gn.repeat(4, 1)
    fc2d.fc2d_poisson_solve(plan, fg4, fb4, gn4, u4)             # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fc2d.fc2d_poisson_solve(plan, fg4, fb4, gn4, u4)
    torch.cuda.synchronize()
    ms4 = (time.perf_counter() - t0) * 1e3
    same4 = float((u4 - u[0]).abs().max().item() / u[0].abs().max().item())
    ins = fc2d.fc2d_plan_classes(plan) == 1
    err = u[0].cpu().numpy()[ins] - ue(X, Y)[ins]
    ex = ue(X, Y)[ins]
    return {"workload": "kite(0.65,1.5) fitted %d^2, d=%d, M=%d, B=%d, nb=%d, u=sin(2 pi x)sin(2 pi y)/(8 pi^2)"
                        % (case.n, case.d, case.M, case.B, nb, ),
            "ms_per_solve": ms, "ms_per_field_4_fields": ms4 / 4, "four_fields_vs_one": same4,
            "gmres_iters": it, "plan_s": plan_s, "in_points": int(ins.sum()),
            "rel_l2_err": float(np.linalg.norm(err) / np.linalg.norm(ex)),
            "rel_linf_err": float(np.abs(err).max() / np.abs(ex).max()),
            "kernels_ms": {k: round(v, 4) for k, v in sorted(per.items(), key=lambda kv: -kv[1])}}


def run_ff_solver(args):
    """Fourier Forwarding solver (Sec. 4.2; fc2d_ff_advance): Ex. 4.4's
    manufactured plane wave u = cos(2 kappa (x + t) / 3) + cos(kappa (y + t)),
    kappa = 10, on the unit disc in the box [-1.6, 1.6]^2 at ff_solver_n^2
    (d = 5, n_c = 6, CFL 0.125), Dirichlet data from the exact solution.
    Reports the time of a large step (48 small steps; HIP events, the data
    arrays resident) and the largest error over Omega after two large steps."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2010_03901_amd import fc2d
    kap = 10.0
    ue = lambda x, y, t: np.cos(2 * kap * (x + t) / 3) + np.cos(kap * (y + t))
    ute = lambda x, y, t: -(2 * kap / 3) * np.sin(2 * kap * (x + t) / 3) - kap * np.sin(kap * (y + t))
    n = args.ff_solver_n
    case = W.cfg_disc(n)
    t0 = time.perf_counter()
    plan = fc2d.Plan(fc2d.make_curve(*case.curve), fc2d.make_grid(case.x0, case.y0, case.h, n, n), d=case.d,
                     C_=case.C, B=case.B, k1=case.k1, M=case.M)
    ff = fc2d.FF(plan)
    setup_s = time.perf_counter() - t0
    inf = ff.info
    inside = ff.regions() > 0
    x = case.x0 + np.arange(n) * case.h
    X, Y = np.meshgrid(x, x, indexing="ij")
    bp = fc2d.fc2d_boundary_points(plan)
    cx = ff.crossings()
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    nlarge = 2
    data = []
    for j in range(nlarge):
        T = j * inf.dT
        ts = T + np.arange(inf.K + 1) * inf.dt
        data.append((dev(ue(bp[:, 0], bp[:, 1], T)), dev(ute(bp[:, 0], bp[:, 1], T)),
                     dev(np.stack([ue(cx[:, 0], cx[:, 1], t) for t in ts])),
                     dev(np.stack([ute(cx[:, 0], cx[:, 1], t) for t in ts]))))
    u0 = dev(np.where(inside, ue(X, Y, 0.0), 0.0))
    v0 = dev(np.where(inside, ute(X, Y, 0.0), 0.0))
    u, v = u0.clone(), v0.clone()
    ff.advance(u, v, *data[0])                  # warm-up
    torch.cuda.synchronize()
    u.copy_(u0)
    v.copy_(v0)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(nlarge + 1)]
    ev[0].record()
    for j in range(nlarge):
        ff.advance(u, v, *data[j])
        ev[j + 1].record()
    torch.cuda.synchronize()
    ms = [ev[j].elapsed_time(ev[j + 1]) for j in range(nlarge)]
    t_end = nlarge * inf.dT
    err = float(np.abs(u.cpu().numpy() - ue(X, Y, t_end))[inside].max())
    ff.close()
    plan.close()
    return {"workload": "Ex. 4.4 plane wave (kappa = 10) on the unit disc, [-1.6,1.6]^2 at %d^2, d=5, n_c=6, CFL 0.125"
                        % n,
            "ms_per_large_step": float(np.mean(ms)), "small_steps_per_large_step": inf.K,
            "ms_per_small_step": float(np.mean(ms)) / inf.K, "stepped_points": int(inf.n_stepped),
            "boundary_points": int(inf.n_bnd), "segments": int(inf.n_segments), "setup_s": setup_s,
            "t_end": t_end, "max_err_vs_exact": err}


def run_mlp(args):
    """Learned foot seed: training pairs (the method's own foot solves on
    mlp_curves random curves x 1000 points in the exterior strip) and training on
    the GPU, then the plan of the held-out random curve (seed 1) on 4096^2 with
    B = 8192 built with the proximity, polar-angle and learned seeds.  Reports
    plan wall time, classification-kernel time (HIP events), Newton steps per
    solved point and the fallback rate, and the extend + FFT throughput of the
    learned-seed plan."""
    import math
    import numpy as np
    import torch
    import workloads as W
    from paper_2010_03901_amd import fc2d
    width = 27 * W.mlp_k1()
    curves, cidx, th, eta = W.mlp_training_draws(0, args.mlp_curves, 1000, width)
    n = cidx.size
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    X = torch.empty((n, 8), dtype=torch.float32, device="cuda:0")
    Y = torch.empty((n, 2), dtype=torch.float32, device="cuda:0")
    its = torch.empty(n, dtype=torch.int32, device="cuda:0")
    dc, di, dth, deta = dev(curves), dev(cidx), dev(th), dev(eta)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fc2d.fc2d_mlp_make_data(dc, di, dth, deta, width, X, Y, None, its)
    torch.cuda.synchronize()
    data_s = time.perf_counter() - t0
    if int(its.min().item()) < 1:
        raise RuntimeError("training pairs: foot solve failed")
    label_steps = float(its.double().mean().item())
    # Glorot-uniform initial weights, zero biases
    rng = np.random.default_rng(0)
    parts = []
    for fi, fo in [(8, 64), (64, 64), (64, 64), (64, 2)]:
        lim = math.sqrt(6.0 / (fi + fo))
        parts += [rng.uniform(-lim, lim, fi * fo), np.zeros(fo)]
    w = dev(np.concatenate(parts).astype(np.float32))
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    steps = args.mlp_steps
    hist = torch.zeros(steps, dtype=torch.float32, device="cuda:0")
    t0 = time.perf_counter()
    fc2d.fc2d_mlp_train(w, m, v, X, Y, args.mlp_batch, steps, 0, 3e-3, 1e-5, steps, hist)
    train_s = time.perf_counter() - t0
    h = hist.cpu().numpy()
    weights = w.cpu().numpy()
    print("[bench] mlp: data %.2fs, %d steps in %.2fs, loss %.3e -> %.3e" % (data_s, steps, train_s, h[:20].mean(),
                                                                        h[-100:].mean()), file=sys.stderr, flush=True)
    del X, Y, its
    torch.cuda.empty_cache()

    case = W.cfg_mlp(4096)
    grid = fc2d.make_grid(case.x0, case.y0, case.h, case.n, case.n)
    curve = fc2d.make_curve(*case.curve)

    def build(**kw):
        return fc2d.Plan(curve, grid, d=case.d, C_=case.C, B=case.B, k1=case.k1, M=case.M, **kw)

    build().close()                                       # tables and code objects warm
    modes = {"proximity": {}, "polar": {"seed": fc2d.FC2D_SEED_POLAR},
             "mlp": {"seed": fc2d.FC2D_SEED_MLP, "mlp_weights": weights}}
    res, plans = {}, {}
    for name, kw in modes.items():
        best = None
        for _ in range(9):   # the fastest of nine builds: host timings vary from build to build
            torch.cuda.synchronize()
            fc2d.fc2d_trace_begin()
            t0 = time.perf_counter()
            pl = build(**kw)
            wall = time.perf_counter() - t0
            tr = fc2d.fc2d_trace_end()
            kms = sum(t for k, t in tr if k.startswith("k_"))
            if best is None or wall < best["plan_s"]:
                inf = pl.info
                best = {"plan_s": wall, "classify_kernel_ms": kms,
                        "phases_ms": {k: inf.t_ms[i] for i, k in enumerate(fc2d.PLAN_PHASES)},
                        "kernels_ms": {k: t for k, t in tr if k.startswith("k_")},
                        "solved": inf.n_solved, "strip": inf.n_strip,
                        "newton_steps_per_point": inf.newton_iters / max(inf.n_solved, 1),
                        "fallback_rate": inf.n_fallback / max(inf.n_solved, 1)}
                plans[name] = pl
        res[name] = best
        print("[bench] mlp plan %-9s %s" % (name, json.dumps(best)), file=sys.stderr, flush=True)
    same = all(np.array_equal(fc2d.fc2d_plan_classes(plans["proximity"]), fc2d.fc2d_plan_classes(plans[k]))
               for k in ("polar", "mlp"))
    # extend + FFT on the learned-seed plan: nf fields built on the device
    nf = args.mlp_fields
    pl = plans["mlp"]
    bp = torch.from_numpy(fc2d.fc2d_boundary_points(pl)).to("cuda:0")
    x = case.x0 + torch.arange(case.n, device="cuda:0", dtype=torch.float64) * case.h
    fg = torch.empty((nf, case.n, case.n), dtype=torch.float64, device="cuda:0")
    fb = torch.empty((nf, bp.shape[0]), dtype=torch.float64, device="cuda:0")
    for s in range(nf):
        k1, k2 = W.star_wavenumbers(s)
        fg[s] = torch.sin(k1 * x)[:, None] * torch.cos(k2 * x)[None, :] + (x ** 3)[:, None] * x[None, :]
        fb[s] = torch.sin(k1 * bp[:, 0]) * torch.cos(k2 * bp[:, 1]) + bp[:, 0] ** 3 * bp[:, 1]
    spec = torch.empty((nf, case.n, case.n // 2 + 1), dtype=torch.complex128, device="cuda:0")
    for _ in range(2):
        fc2d.fc2d_extend_fft(pl, fg, fb, fg, spec)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    reps = 10
    ev0.record()
    for _ in range(reps):
        fc2d.fc2d_extend_fft(pl, fg, fb, fg, spec)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    for p in plans.values():
        p.close()
    sp = lambda a, b: res[a]["classify_kernel_ms"] / res[b]["classify_kernel_ms"]
    return {"workload": "held-out random curve (seed 1), fitted box 4096^2, B=8192, k1=%.4g" % case.k1,
            "training": {"pairs": int(n), "curves": int(args.mlp_curves), "data_s": data_s,
                         "label_newton_steps": label_steps, "steps": steps, "batch": args.mlp_batch,
                         "train_s": train_s, "loss_first": float(h[:20].mean()), "loss_last": float(h[-100:].mean())},
            "plans": res, "identical_classes": bool(same),
            "classify_speedup_mlp_vs_proximity": sp("proximity", "mlp"),
            "classify_speedup_mlp_vs_polar": sp("polar", "mlp"),
            "plan_speedup_mlp_vs_proximity": res["proximity"]["plan_s"] / res["mlp"]["plan_s"],
            "plan_speedup_mlp_vs_polar": res["polar"]["plan_s"] / res["mlp"]["plan_s"],
            "extend_fft": {"fields": nf, "ms": ms, "points_per_s": nf * case.n * case.n / (ms * 1e-3)}}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import workloads as W
    from paper_2010_03901_amd import fc2d

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    case = W.cfg_star(args.n)
    nf = args.nf
    print("[bench] workload star%d nf=%d steps=%d warmup=%d" % (case.n, nf, args.steps, args.warmup),
          file=sys.stderr, flush=True)
    grid = fc2d.make_grid(case.x0, case.y0, case.h, case.n, case.n)
    if args.col_elems:
        fc2d.fc2d_tune_set(fc2d.FC2D_TUNE_COL_ELEMS, case.n, args.col_elems)
    if args.col_tile:
        fc2d.fc2d_tune_set(fc2d.FC2D_TUNE_COL_TILE, case.n, args.col_tile)
    if args.strip_fields >= 0:
        fc2d.fc2d_tune_set(fc2d.FC2D_TUNE_STRIP_FIELDS, 0, args.strip_fields)
    t0 = time.perf_counter()
    plan = fc2d.Plan(fc2d.make_curve(*case.curve), grid, d=case.d, C_=case.C, B=case.B, k1=case.k1, M=case.M)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    info = plan.info
    bp = fc2d.fc2d_boundary_points(plan)
    # inputs: nf seeded fields, built on the host once and copied to HBM
    x = case.x0 + np.arange(case.n) * case.h
    fg = torch.empty((nf, case.n, case.n), dtype=torch.float64, device="cuda:0")
    fb = torch.empty((nf, bp.shape[0]), dtype=torch.float64, device="cuda:0")
    X, Y = np.meshgrid(x, x, indexing="ij")
    for s in range(nf):
        f = W.f_star(s)
        fg[s].copy_(torch.from_numpy(f(X, Y)))
        fb[s].copy_(torch.from_numpy(f(bp[:, 0], bp[:, 1])))
    ext = torch.empty_like(fg)
    if args.calib_copy:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    # the timed fused step writes the half spectrum with 128-byte-aligned rows (row pitch
    # ld = ny/2 + 1 rounded up to a multiple of 8 complex; fc2d_extend_fft_ld); the same
    # step into the numpy layout (ld = ny/2 + 1, fc2d_extend_fft) is timed beside it
    half = case.n // 2 + 1
    ld = (half + 7) // 8 * 8
    spec = torch.empty((nf, case.n, ld), dtype=torch.complex128, device="cuda:0")
    spec_np = torch.empty((nf, case.n, half), dtype=torch.complex128, device="cuda:0")
    torch.cuda.synchronize()
    print("[bench] plan %.2fs, inputs ready" % plan_s, file=sys.stderr, flush=True)

    def step_plain():
        fc2d.fc2d_extend(plan, fg, fb, ext)
        fc2d.fc2d_fft(grid, ext, spec_np, fc2d.FC2D_FORWARD)

    def step_fused():
        fc2d.fc2d_extend_fft_ld(plan, fg, fb, ext, spec)

    def step_fused_numpy_layout():
        fc2d.fc2d_extend_fft(plan, fg, fb, ext, spec_np)

    def timed(step):
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(args.steps):
            step()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / args.steps

    ms_plain = timed(step_plain)
    # sampled outputs of the timed runs (the last step's), for the oracle check of the cpu_baseline leg
    check_seeds = sorted({0, min(nf, args.cpu_sample_fields) - 1})
    checks = {s: {"extension": ext[s].cpu().numpy()} for s in check_seeds}
    ms_np = timed(step_fused_numpy_layout)
    ms = timed(step_fused)
    for s in check_seeds:
        checks[s]["spectrum"] = spec[s, :, :half].cpu().numpy()
    value = nf * case.n * case.n / (ms * 1e-3)
    value_plain = nf * case.n * case.n / (ms_plain * 1e-3)
    value_np = nf * case.n * case.n / (ms_np * 1e-3)
    print("[bench] plain %.3f ms/step (%.3e points/s); fused, numpy layout %.3f ms/step (%.3e points/s); fused, "
          "aligned rows %.3f ms/step (%.3e points/s)" % (ms_plain, value_plain, ms_np, value_np, ms, value),
          file=sys.stderr, flush=True)

    # side-by-side reference (not the library's path): torch.fft.rfft2 on ROCm
    # (rocFFT through hipFFT), float64, the same fields, already extended
    fc2d.fc2d_extend(plan, fg, fb, ext)
    torch.cuda.synchronize()
    ref_spec = torch.fft.rfft2(ext)
    err_vs_rocfft = float(((spec_np - ref_spec).abs().max() / ref_spec.abs().max()).item())
    del ref_spec
    ms_rocfft = timed(lambda: torch.fft.rfft2(ext))
    ms_fft_only = timed(lambda: fc2d.fc2d_fft(grid, ext, spec_np, fc2d.FC2D_FORWARD))
    print("[bench] 2D R2C of the extended fields: library %.3f ms, rocFFT (torch.fft.rfft2) %.3f ms, spectra agree "
          "to %.1e" % (ms_fft_only, ms_rocfft, err_vs_rocfft), file=sys.stderr, flush=True)

    # per-kernel times from HIP events on the launch stream (library tracer)
    fc2d.fc2d_trace_begin()
    for _ in range(args.steps):
        step_fused()
    tr = fc2d.fc2d_trace_end()
    per = {}
    for name, t in tr:
        if name == "begin":
            continue
        per.setdefault(name, []).append(t)
    # the fused path may split the fields into chunks: bytes per launch = bytes per step / launches per step
    kernels = {k: {"avg_ms": float(np.mean(v)), "launches": len(v),
                   "alg_bytes": algorithmic_bytes(k, case.n, nf, info) * args.steps / len(v)} for k, v in per.items()}
    for k, v in kernels.items():
        v["GBs"] = v["alg_bytes"] / (v["avg_ms"] * 1e-3) / 1e9 if v["avg_ms"] > 0 else None
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"] * kernels[k]["launches"])
    dk = kernels[dom]
    roofline = {"bound": "hbm", "kernel": dom, "achieved": dk["GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": dk["GBs"] / HBM_PEAK_GBS, "traffic": measured_traffic(dom),
                "alg_bytes_per_launch": dk["alg_bytes"], "avg_ms": dk["avg_ms"]}
    print("[bench] kernels " + json.dumps(kernels), file=sys.stderr, flush=True)

    batched, ff_check = None, None
    if not args.no_batched:
        print("[bench] Fourier Forwarding, plain and batched ...", file=sys.stderr, flush=True)
        del fg, fb, ext, spec, spec_np
        torch.cuda.empty_cache()
        batched, ff_check = run_ff(args)
        print("[bench] FF step: plain %.3f ms (%.3e points/s), batched %.3f ms (%.3e points/s)"
              % (batched["plain_ms_per_step"], batched["plain_points_per_s"], batched["ms_per_step"],
                 batched["points_per_s"]), file=sys.stderr, flush=True)

    learned = None
    if not args.no_mlp:
        print("[bench] learned foot seed ...", file=sys.stderr, flush=True)
        if batched is None:
            del fg, fb, ext, spec, spec_np
            torch.cuda.empty_cache()
        learned = run_mlp(args)
        print("[bench] learned seed: " + json.dumps(learned), file=sys.stderr, flush=True)

    poisson = None
    if not args.no_poisson:
        print("[bench] full Poisson solve ...", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        poisson = run_poisson(args)
        print("[bench] poisson: " + json.dumps(poisson), file=sys.stderr, flush=True)

    ff_solver = None
    if not args.no_ff_solver:
        print("[bench] Fourier Forwarding solver ...", file=sys.stderr, flush=True)
        ff_solver = run_ff_solver(args)
        print("[bench] ff solver: " + json.dumps(ff_solver), file=sys.stderr, flush=True)

    cpu, oracle_checks = None, None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline and oracle checks ...", file=sys.stderr, flush=True)
        leg = cpu_baseline(case, args.cpu_sample_fields, checks, ff_check)
        cpu = leg["baseline"]
        oracle_checks = {k: v for k, v in leg.items() if k != "baseline"}
        print("[bench] oracle checks: " + json.dumps(oracle_checks), file=sys.stderr, flush=True)
        if batched is not None and "ff_check" in oracle_checks:
            batched["max_rel_err_vs_oracle"] = max(v for k, v in oracle_checks["ff_check"].items() if k != "field")

    out = {
        "metric": "2D-FC extended grid points/s at <=1e-11 err vs oracle; plain vs batched+MLP",
        "value": value, "unit": "points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "star r=1+0.3cos5t, B=%d, [-1.6,1.6]^2 on %dx%d, d=5, C=27, M=8, k1=%g; "
                               "extend + forward FFT of %d fields per step" % (case.B, case.n, case.n, case.k1, nf),
                   "fields_per_step": nf, "grid": case.n,
                   "path": "fused extend+FFT into a half spectrum with 128-byte-aligned rows (fc2d_extend_fft_ld, "
                           "row pitch %d complex)" % ld,
                   "numpy_layout_points_per_s": value_np, "numpy_layout_ms_per_step": ms_np,
                   "plain_points_per_s": value_plain, "plain_ms_per_step": ms_plain,
                   "fft_only_ms": ms_fft_only, "rocfft_reference_ms": ms_rocfft,
                   "rocfft_reference": "torch.fft.rfft2 (rocFFT via hipFFT), float64, same extended fields",
                   "spectrum_rel_diff_vs_rocfft": err_vs_rocfft},
        "max_rel_err_vs_oracle": oracle_checks["checks"]["fused_spectrum_max_rel_err"] if oracle_checks else None,
        "oracle_checks": oracle_checks,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "batched_ff": batched,
        "learned_seed": learned,
        "poisson_full": poisson,
        "ff_solver": ff_solver,
        "plan_s": plan_s,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
