"""Test helpers: build oracle results for a workload (CPU, FP64), in parallel."""
import numpy as np

from oracle import stepper
from oracle.parallel import solve_points, solve_staggered  # noqa: F401
from oracle.weights import IBModel

def model_for(wl, **kw):
    return IBModel(wl.heights, wl.h, wl.shape, M=wl.M, surface=wl.surface, eta=wl.eta, **kw)


def simulation(wl, model, sols):
    L = stepper.assemble_laplacian(model, sols)
    return stepper.Simulation(model, L, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width,
                              damp_R=wl.damp_R), L


def rel_l2_per_trace(d, ref, floor=1e-3):
    """Per-trace ||d - ref|| / max(||ref||, floor * max_r ||ref||) over axis 0 = time."""
    num = np.linalg.norm(d - ref, axis=0)
    den = np.linalg.norm(ref, axis=0)
    den = np.maximum(den, floor * den.max())
    return num / den


# ---- full-size sampling ---------------------------------------------------------------
# The method is local: a node's class, its boundary point, the exclusion mask and the
# support of an IB point depend only on the surface within a few cells.  An IB point of a
# large 3D grid is therefore checked against the oracle built on a lateral window of the
# heightfield centred on it (WIN columns; supports reach at most 7.5 cells, the
# closest-point search and the cubic surface patches two more, so the window's periodic
# seam stays far from everything the point uses).
WIN = 40


def window_task(args):
    """(solution, full Laplacian row {full-grid memory index: weight}) of one IB point."""
    H, h, nz, M, surface, eta, point = args
    ny, nx = H.shape
    px, py, pz = (int(v) for v in point)
    c = WIN // 2
    jj = (np.arange(WIN) + py - c) % ny
    ii = (np.arange(WIN) + px - c) % nx
    m = IBModel(H[np.ix_(jj, ii)], h, (WIN, WIN, nz), M=M, surface=surface, eta=eta)
    g = np.array([c, c, pz])
    s = m.solve_point(g)
    full = {}
    for (x, y, z), w in m.laplacian_row(g, s).items():
        q = (z * ny + (y - c + py) % ny) * nx + (x - c + px) % nx
        full[q] = full.get(q, 0.0) + w
    return s, full


def pool_map(fn, tasks, procs=None):
    """Map over a spawned process pool with single-threaded BLAS (see oracle.parallel)."""
    import multiprocessing as mp
    import os
    procs = procs or min(16, os.cpu_count() or 1)
    saved = {k: os.environ.get(k) for k in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"
    try:
        with mp.get_context("spawn").Pool(procs) as pool:
            return pool.map(fn, tasks, chunksize=1)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
