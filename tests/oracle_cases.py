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
