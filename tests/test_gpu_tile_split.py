"""IB patch tiles that overflow the per-tile point limit: a steep periodic surface (slope
up to 3.1, within the range of the fractal workloads) puts more than 512 IB points into
some 8 x 8 x 16 tiles, which the host splits.  GPU traces through the C ABI against the
FP64 oracle."""
import math
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from oracle_cases import model_for, rel_l2_per_trace, simulation, solve_points  # noqa: E402

from paper_2309_03600_amd import workloads as W  # noqa: E402

TILE_X, TILE_Y, TILE_Z, TILE_MAX = 8, 8, 16, 512
_cache = {}


def steep_case():
    if not _cache:
        import paper_2309_03600_amd as ib
        n, nz, h = 32, 64, 10.0
        x = np.arange(n) * h
        X, Y = np.meshgrid(x, x)
        H = 30 * h + 8 * h * np.sin(2 * math.pi * X / (16 * h)) + 2.4 * h * np.cos(2 * math.pi * Y / (n * h))
        vel = W.gradient_velocity((nz, n, n), h, 1500.0, 3500.0, 0.05, 4.0, W.rng(95, 1))
        src = np.array([[16 * h + 3.0, 16 * h + 4.0, H[16, 16] + 60.0]])
        rec = W._rec_on_surface(H, h, 3, 15.0, n, n)
        wl = W.Workload("steep3d", 3, (n, n, nz), h, 8, "free", H, vel, 0.616e-3, 60, 15.0, src, rec, damp_width=8)
        print(f"[tile split] shape={wl.shape}", flush=True)
        w = ib.ib_build_weights(wl.heights, wl.h, wl.shape, space_order=wl.M, surface=wl.surface, eta=wl.eta)
        m = model_for(wl)
        _cache.update(wl=wl, w=w, ex=w.export(), m=m, sols=solve_points(m))
    return _cache


def test_some_tiles_overflow_the_point_limit():
    # the host's tiling rule, replayed: the smallest supports (radius 4.5) are tiled by
    # lateral 8 x 8 column, each tile opening at its first point in depth
    c = steep_case()
    ex, (nx, ny, nz) = c["ex"], c["wl"].shape
    tiled = ex["ib_meta"][:, 0] == 0
    z, r = np.divmod(ex["ib_nodes"][tiled], nx * ny)
    y, x = np.divmod(r, nx)
    col = (y // TILE_Y) * nx + x // TILE_X
    order = np.lexsort((z, col))
    col, z = col[order], z[order]
    starts = np.flatnonzero(np.r_[True, col[1:] != col[:-1]])
    sizes = []
    for a, b in zip(starts, np.r_[starts[1:], len(col)]):
        zc, k = z[a:b], 0
        while k < len(zc):
            m = int(np.searchsorted(zc, zc[k] + TILE_Z, side="left"))
            sizes.append(m - k)
            k = m
    assert max(sizes) > TILE_MAX, max(sizes)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_split_tiles_match_oracle(prec):
    import torch

    import paper_2309_03600_amd as ib
    c = steep_case()
    wl, w = c["wl"], c["w"]
    sim, _ = simulation(wl, c["m"], c["sols"])
    ref = sim.run(wl.wavelets(np.float64), wl.nt)
    tdt = torch.float64 if prec == "f64" else torch.float32
    st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision=prec)
    tr = st.step(wl.nt, torch.tensor(wl.wavelets(np.float64), dtype=tdt, device="cuda"), use_graph=True)
    e = rel_l2_per_trace(tr.double().cpu().numpy()[0], ref)
    print(f"[tile split {prec}] per-trace rel-L2: max {e.max():.2e} median {np.median(e):.2e}", flush=True)
    assert e.max() < (1e-9 if prec == "f64" else 1e-4)
