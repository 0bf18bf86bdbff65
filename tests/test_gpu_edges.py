"""Edge cases and error paths of the GPU library (through the C ABI): degenerate surfaces
against the oracle, empty acquisition, zero-length calls and rejected inputs."""
import math
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from oracle_cases import model_for, rel_l2_per_trace, simulation, solve_points, solve_staggered  # noqa: E402

from paper_2309_03600_amd import workloads as W  # noqa: E402


def flat2d(depth_cells, M=8, surface="free", nt=200, nx=64, nz=64, h=5.0):
    """Flat surface at ``depth_cells`` (grid units): through a node row when integer, on the
    half-open hosting boundary when it ends in .5."""
    H = W.flat_surface(nx, depth_cells * h)
    vel = np.full((nz, nx), 2000.0)
    dt = 0.5 * 2 * h / (2000.0 * math.sqrt(2) * 2.572619047619048)
    src = np.array([[nx * h / 2 + 1.0, (depth_cells + 12) * h]])
    rec = np.array([[i * h, (math.floor(depth_cells) + 2) * h] for i in range(0, nx, 4)])
    return W.Workload(f"flat2d-{depth_cells}", 2, (nx, nz), h, M, surface, H, vel, dt, nt, 25.0, src, rec,
                      damp_width=8)


@pytest.mark.parametrize("depth", [20.0, 20.5, 20.25])
@pytest.mark.parametrize("surface", ["free", "rigid"])
def test_flat_surface_degenerate_positions(depth, surface):
    """Surface through a node row (nodes on it are exterior, boundary points coincide with
    nodes) and on the half-cell tie of the hosting rule."""
    import torch

    import paper_2309_03600_amd as ib
    wl = flat2d(depth, surface=surface)
    w = ib.ib_build_weights(wl.heights, wl.h, wl.shape, space_order=wl.M, surface=wl.surface, eta=wl.eta)
    ex = w.export()
    m = model_for(wl)
    assert np.array_equal((ex["node_class"] & 1).astype(bool), m.geom.interior_grid().ravel())
    assert ex["bpoints"].shape[0] == len(m.bp_host)
    st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision="f64")
    tr = st.step(wl.nt, torch.tensor(wl.wavelets(np.float64), device="cuda")).cpu().numpy()[0]
    sim, _ = simulation(wl, m, solve_points(m))
    ref = sim.run(wl.wavelets(np.float64), wl.nt)
    e = rel_l2_per_trace(tr, ref)
    print(f"[flat {depth} {surface}] rel-L2 vs oracle max {e.max():.2e}")
    assert e.max() < 1e-9


@pytest.mark.parametrize("depth", [20.0, 20.5])
def test_flat_surface_degenerate_positions_first_order(depth):
    import torch

    import paper_2309_03600_amd as ib
    from oracle import staggered as S
    wl = flat2d(depth)
    w = ib.ib_build_weights(wl.heights, wl.h, wl.shape, space_order=wl.M, surface=wl.surface, eta=wl.eta,
                            form="pv1")
    st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision="f64")
    tr = st.step(wl.nt, torch.tensor(wl.wavelets(np.float64), device="cuda")).cpu().numpy()[0]
    m = S.StaggeredModel(wl.heights, wl.h, wl.shape, M=wl.M, surface=wl.surface, eta_p=wl.eta, eta_v=0.0)
    G, D = S.assemble(m, *solve_staggered(m))
    sim = S.StaggeredSimulation(m, G, D, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width,
                                damp_R=wl.damp_R)
    ref = sim.run(wl.wavelets(np.float64), wl.nt)
    e = rel_l2_per_trace(tr, ref)
    print(f"[flat pv1 {depth}] rel-L2 vs oracle max {e.max():.2e}")
    assert e.max() < 1e-9


def test_no_receivers_and_zero_steps():
    import torch

    import paper_2309_03600_amd as ib
    wl = W.small3d(n=16, nz=40, relief=40.0, nt=20)
    w = ib.ib_build_weights(wl.heights, wl.h, wl.shape, space_order=wl.M, surface=wl.surface, eta=wl.eta)
    st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, np.zeros((0, 3)), precision="f32")
    wav = torch.tensor(wl.wavelets(np.float32), device="cuda")
    assert st.step(0, wav) is None or st.step_count == 0
    assert st.step_count == 0
    st.step(5, wav, use_graph=True)
    assert st.step_count == 5
    p = st.field(0, 0)
    assert torch.isfinite(p).all() and float(p.abs().max()) > 0


def test_rejected_inputs():
    import torch

    import paper_2309_03600_amd as ib
    wl = W.small3d(n=16, nz=40, relief=40.0, nt=20)
    w = ib.ib_build_weights(wl.heights, wl.h, wl.shape, space_order=wl.M, surface=wl.surface, eta=wl.eta)
    wav = torch.tensor(wl.wavelets(np.float32), device="cuda")
    st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, precision="f32")
    with pytest.raises(RuntimeError, match="wavelet"):
        st.step(wl.nt + 1, wav)
    above = wl.src.copy()
    above[0, 2] = 5.0                                  # in the air, above the surface
    with pytest.raises(RuntimeError, match="exterior"):
        ib.ib_state_create(w, wl.vel, wl.dt, above, wl.rec, precision="f32")
    outside = wl.src.copy()
    outside[0, 2] = 1e6
    with pytest.raises(RuntimeError):
        ib.ib_state_create(w, wl.vel, wl.dt, outside, wl.rec, precision="f32")
    with pytest.raises(RuntimeError):
        ib.ib_build_weights(wl.heights, wl.h, wl.shape, space_order=7)        # odd order
    high = np.full_like(wl.heights, 2.0 * wl.h)     # surface 2 cells below the top: supports leave the box
    with pytest.raises(RuntimeError):
        ib.ib_build_weights(high, wl.h, wl.shape, space_order=8)
