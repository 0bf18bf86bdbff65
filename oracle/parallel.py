"""Process-pool evaluation of the per-point oracle solves.

Test infrastructure (see ``oracle/__init__.py``).  The solves are independent per IB
point (section "Reconciliation with the Interior Numerical Discretization": each
stencil centre has its own extrapolation), so they map over a pool unchanged.
"""
from __future__ import annotations

import multiprocessing as mp
import os
import sys

import numpy as np

_MODEL = None


def _init_worker(model):
    global _MODEL
    _MODEL = model


def _solve_one(p):
    s = _MODEL.solve_point(p)
    return (tuple(int(v) for v in p), s)


def _solve_task(task):
    fam, g = task
    s = _MODEL.solve_p_point(g) if fam < 0 else _MODEL.solve_v_point(fam, g)
    return (fam, tuple(int(v) for v in g), s)


class _Threads1:
    """Single-threaded BLAS in the spawned workers (restored on exit)."""

    def __enter__(self):
        self.saved = {k: os.environ.get(k) for k in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS", "MKL_NUM_THREADS")}
        for k in self.saved:
            os.environ[k] = "1"

    def __exit__(self, *exc):
        for k, v in self.saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def solve_staggered(model, procs=None):
    """Modified rows of a staggered p-v model, in parallel: ([{node: solution} per v_n],
    {node: solution} of the divergence rows), the same result as ``staggered.solve_all``."""
    tasks = [(n, g) for n in range(model.d) for g in model.ib_v(n)] + [(-1, g) for g in model.ib_p()]
    if procs is None:
        procs = min(16, os.cpu_count() or 1)
    if len(tasks) < 64 or procs <= 1:
        res = [_solve_task_with(model, t) for t in tasks]
    else:
        with _Threads1():
            ctx = mp.get_context("spawn")
            res = []
            with ctx.Pool(procs, initializer=_init_worker, initargs=(model,)) as pool:
                it = pool.imap(_solve_task, tasks, chunksize=max(1, len(tasks) // (procs * 16)))
                for k, r in enumerate(it):
                    res.append(r)
                    if (k + 1) % 200 == 0:
                        print(f"  [oracle] {k + 1}/{len(tasks)} staggered rows solved", file=sys.stderr, flush=True)
    vsol = [dict() for _ in range(model.d)]
    psol = {}
    for fam, g, s in res:
        (psol if fam < 0 else vsol[fam])[g] = s
    return vsol, psol


def _solve_task_with(model, task):
    fam, g = task
    s = model.solve_p_point(g) if fam < 0 else model.solve_v_point(fam, g)
    return (fam, tuple(int(v) for v in g), s)


def solve_points(model, points=None, procs=None):
    """{node tuple: solution}.  A spawned process pool (fresh interpreters with
    single-threaded BLAS: forking after the parent started BLAS or HIP threads can
    deadlock the children) solves the points in parallel."""
    pts = model.ib_points() if points is None else np.asarray(points)
    if procs is None:
        procs = min(16, os.cpu_count() or 1)
    if len(pts) < 64 or procs <= 1:
        return {tuple(int(v) for v in p): model.solve_point(p) for p in pts}
    saved = {k: os.environ.get(k) for k in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"
    try:
        ctx = mp.get_context("spawn")
        res = []
        with ctx.Pool(procs, initializer=_init_worker, initargs=(model,)) as pool:
            it = pool.imap(_solve_one, list(pts), chunksize=max(1, len(pts) // (procs * 16)))
            for k, r in enumerate(it):
                res.append(r)
                if (k + 1) % 200 == 0:
                    print(f"  [oracle] {k + 1}/{len(pts)} IB points solved", file=sys.stderr, flush=True)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    return dict(res)


