"""Shared set-up for GPU parity tests: builds the oracle plan and the HIP plan
of the same workload case (each side on its own) and moves data to the device."""
import functools

import numpy as np

import workloads as W
from oracle import fcgram
from oracle import plan as OP
from oracle.curves import Curve


def torch_dev():
    import torch
    return torch.device("cuda:0")


@functools.lru_cache(maxsize=None)
def oracle_plan(case_name, builder, *args):
    case = builder(*args)
    tab = fcgram.load_tables(case.d)
    g = OP.Grid(case.x0, case.y0, case.h, case.n, case.n)
    return case, OP.make_plan(Curve(*case.curve), g, tab, case.B, k1=case.k1, M=case.M)


def gpu_plan(case):
    from paper_2010_03901_amd import fc2d
    grid = fc2d.make_grid(case.x0, case.y0, case.h, case.n, case.n)
    curve = fc2d.make_curve(*case.curve)
    return fc2d.Plan(curve, grid, d=case.d, C_=case.C, B=case.B, k1=case.k1, M=case.M)


def fields(case, funcs, bpts):
    """Grid values [nf, n, n] and boundary values [nf, nb] for closed-form f's."""
    fg = np.stack([W.grid_values(case, f) for f in funcs])
    fb = np.stack([f(bpts[:, 0], bpts[:, 1]) for f in funcs])
    return fg, fb


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def pulse_field(case, seed):
    """Seeded Gaussian pulse of the batched Fourier-Forwarding workload on the case's grid."""
    x = case.x0 + np.arange(case.n) * case.h
    X, Y = np.meshgrid(x, x, indexing="ij")
    f, _ = W.gaussian_pulse(case.curve, seed)
    return f(X, Y)


def oracle_ff_step_worker(domain, n, seed, dt):
    """The oracle's Fourier-Forwarding step of one pulse (u_t = 0) on the batched
    workload's (domain, n) plan.  Runs in a separate process that never touches
    the GPU (spawned), so several can run beside a GPU test."""
    from oracle import ff as OF
    case = W.cfg_ff(domain, n)
    tab = fcgram.load_tables(case.d)
    g = OP.Grid(case.x0, case.y0, case.h, case.n, case.n)
    pl = OP.make_plan(Curve(*case.curve), g, tab, case.B, k1=case.k1, M=case.M)
    u0 = pulse_field(case, seed)
    return OF.ff_step(pl, u0, np.zeros_like(u0), dt)


def oracle_pool_map(fn, argsets, procs=8):
    """Run fn(*args) for every args in spawned CPU-only worker processes."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    with ctx.Pool(min(procs, len(argsets))) as pool:
        return pool.starmap(fn, argsets)
