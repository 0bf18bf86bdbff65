"""The windowed oracle used for full-size sampling reproduces the full-grid oracle."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from oracle_cases import WIN, model_for, window_task  # noqa: E402

from paper_2309_03600_amd import workloads as W  # noqa: E402


def test_window_solution_equals_full_grid_solution():
    wl = W.small3d(n=64, nz=60, relief=120.0, cfg=99, z_top_cells=14)
    assert wl.shape[0] > WIN
    m = model_for(wl)
    ib = m.ib_points()
    rng = np.random.default_rng([2309, 99, 7])
    nx, ny, nz = wl.shape
    for p in ib[rng.choice(len(ib), 6, replace=False)]:
        s_full = m.solve_point(p)
        row_full = m.laplacian_row(p, s_full)
        s_win, row_win = window_task((wl.heights, wl.h, nz, wl.M, wl.surface, wl.eta, p))
        assert (s_win["order"], s_win["radius_step"]) == (s_full["order"], s_full["radius_step"])
        assert np.array_equal(s_win["offsets"], s_full["offsets"])
        assert np.allclose(s_win["weights"], s_full["weights"], rtol=0, atol=1e-12 * max(1, np.abs(s_full["weights"]).max()))
        full = {(z * ny + y) * nx + x: w for (x, y, z), w in row_full.items()}
        assert set(full) == set(row_win)
        assert max(abs(full[k] - row_win[k]) for k in full) < 1e-12 * max(1, max(abs(v) for v in full.values()))
