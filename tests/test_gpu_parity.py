"""GPU (HIP, through the C ABI) against the FP64 CPU oracle on seeded synthetic inputs."""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from oracle_cases import model_for, rel_l2_per_trace, simulation, solve_points  # noqa: E402

from paper_2309_03600_amd import workloads as W  # noqa: E402

CASES = {
    "2d-m8-free": lambda: W.small2d(M=8, surface="free", nt=300),
    "2d-m8-rigid": lambda: W.small2d(M=8, surface="rigid", nt=300),
    "2d-m4-free": lambda: W.small2d(M=4, surface="free", nt=300, cfg=92),
    "3d-m8-free": lambda: W.small3d(n=16, nz=40, relief=40.0, surface="free", nt=120),
    "3d-m8-rigid": lambda: W.small3d(n=16, nz=40, relief=40.0, surface="rigid", nt=120, cfg=93),
}

_cache = {}


def case(name):
    if name not in _cache:
        import torch

        import paper_2309_03600_amd as ib
        wl = CASES[name]()
        print(f"[case {name}] shape={wl.shape} M={wl.M} surface={wl.surface}", flush=True)
        w = ib.ib_build_weights(wl.heights, wl.h, wl.shape, space_order=wl.M, surface=wl.surface, eta=wl.eta)
        torch.cuda.synchronize()
        m = model_for(wl)
        sols = solve_points(m)
        _cache[name] = (wl, w, w.export(), m, sols)
    return _cache[name]


def _grid_to_memory(a):
    return np.asarray(a).ravel()


@pytest.mark.parametrize("name", list(CASES))
def test_geometry_sets_identical(name):
    wl, w, ex, m, sols = case(name)
    cls = ex["node_class"]
    inter = m.geom.interior_grid().ravel()
    assert np.array_equal((cls & 1).astype(bool), inter)
    # boundary points: identical host sets, positions to rounding
    bp = ex["bpoints"]
    d = m.d
    gh = bp[:, :3].astype(np.int64)
    gx = bp[:, 3:6]
    if d == 2:
        gh = gh[:, [0, 2]]
        gx = gx[:, [0, 2]]
    key_g = {tuple(h): x for h, x in zip(gh.tolist(), gx)}
    key_o = {tuple(h): x for h, x in zip(m.bp_host.tolist(), m.bp_xb)}
    assert set(key_g) == set(key_o)
    for k in key_o:
        assert np.max(np.abs(key_g[k] - key_o[k])) < 1e-11
    # exclusion only matters (and is only recorded by the library) at interior nodes
    excl = m.excl_grid.ravel() & inter
    assert np.array_equal(((cls >> 1) & 1).astype(bool), excl)
    # IB points in memory order
    ib_o = m.ib_points()
    if d == 2:
        lin = ib_o[:, 1] * wl.shape[0] + ib_o[:, 0]
    else:
        lin = (ib_o[:, 2] * wl.shape[1] + ib_o[:, 1]) * wl.shape[0] + ib_o[:, 0]
    assert np.array_equal(ex["ib_nodes"], lin)


@pytest.mark.parametrize("name", list(CASES))
def test_weights_match_oracle(name):
    wl, w, ex, m, sols = case(name)
    ib_o = m.ib_points()
    meta = ex["ib_meta"]
    W64 = ex["weights"]
    worst = 0.0
    for j, p in enumerate(ib_o):
        s = sols[tuple(int(v) for v in p)]
        k, Mb, nw, off = meta[j]
        assert (k, Mb) == (s["radius_step"], s["order"]), (p, meta[j], s["radius_step"], s["order"])
        assert nw == len(s["weights"])
        yg = W64[off:off + nw]
        yo = s["weights"]
        scale = max(1.0, np.abs(yo).max())
        # boundary points from the two independent closest-point solvers agree to
        # ~1e-14; rows of A move by ~1e-13 relative, and y = (A^+)^T c by up to cond(A)
        # times that; both solvers add O(m cond eps).  Bound: cond * 1e-12.
        tol = max(1e-11, s["cond"] * 1e-12)
        err = np.abs(yg - yo).max() / scale
        worst = max(worst, err / tol)
        assert err <= tol, (p, err, tol, s["cond"])
    print(f"[{name}] worst weight error / tolerance = {worst:.3f}")


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_one_step_matches_oracle(name, prec):
    import torch

    import paper_2309_03600_amd as ib
    wl, w, ex, m, sols = case(name)
    sim, L = simulation(wl, m, sols)
    st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision=prec)
    rng = np.random.default_rng(7)
    inter = m.geom.interior_grid()
    shape = inter.shape
    u = np.where(inter, rng.standard_normal(shape), 0.0)
    um = np.where(inter, rng.standard_normal(shape), 0.0)
    dt = torch.float64 if prec == "f64" else torch.float32
    st.field(0, 0, torch.tensor(u, dtype=dt))
    st.field(1, 0, torch.tensor(um, dtype=dt))
    wav = torch.zeros((1, 4), dtype=dt, device="cuda")
    st.step(1, wav)
    got = st.field(0, 0).double().cpu().numpy().ravel()
    ur = np.asarray(torch.tensor(u, dtype=dt).double()).ravel()
    umr = np.asarray(torch.tensor(um, dtype=dt).double()).ravel()
    ref = (2 * ur - (1 - sim.s) * umr + sim.K * (L @ ur)) / (1 + sim.s)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    # FP64: weight differences (cond * 1e-12, cond <~ 1e4) times K <~ 0.1; FP32: rounding
    tol = 1e-11 if prec == "f64" else 2e-6
    print(f"[{name} {prec}] one-step max error {err:.2e}")
    assert err < tol


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_traces_match_oracle(name, prec):
    import torch

    import paper_2309_03600_amd as ib
    wl, w, ex, m, sols = case(name)
    sim, _ = simulation(wl, m, sols)
    ref = sim.run(wl.wavelets(np.float64), wl.nt)
    st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision=prec)
    dt = torch.float64 if prec == "f64" else torch.float32
    wav = torch.tensor(wl.wavelets(np.float64), dtype=dt, device="cuda")
    tr = st.step(wl.nt, wav).double().cpu().numpy()[0]
    e = rel_l2_per_trace(tr, ref)
    print(f"[{name} {prec}] per-trace rel-L2: max {e.max():.2e} median {np.median(e):.2e}")
    assert e.max() < (1e-9 if prec == "f64" else 1e-4)


@pytest.mark.parametrize("name", ["3d-m8-free", "2d-m8-free"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_source_at_an_ib_point_matches_oracle(prec, name):
    """A source whose interpolation corners include an IB point.  In 3D its injection cannot
    ride in the column-run patch launch (it would race with that point's patch row) and runs
    as a launch of its own; traces against the oracle, eager and graph-replayed."""
    import dataclasses

    import torch

    import paper_2309_03600_amd as ib
    wl0, w, ex, m, sols = case(name)
    shape = wl0.shape[::-1]                       # (nz, [ny,] nx)
    cls = ex["node_class"].reshape(shape)
    inter, ibp = (cls & 1).astype(bool), (cls & 4).astype(bool)
    pick = None
    for idx in np.ndindex(*[n - 1 for n in shape]):
        if any(i < 3 or i >= n - 4 for i, n in zip(idx[1:], shape[1:])):
            continue                              # away from the lateral edges
        cell = tuple(slice(i, i + 2) for i in idx)
        if inter[cell].all() and ibp[cell].any():
            pick = idx
            break
    assert pick is not None
    pos = [(i + 0.5) * wl0.h for i in pick[::-1]]   # (x, [y,] z)
    wl = dataclasses.replace(wl0, src=np.array([pos]))
    print(f"[source at IB {name} {prec}] cell {pick[::-1]}", flush=True)
    sim, _ = simulation(wl, m, sols)
    ref = sim.run(wl.wavelets(np.float64), wl.nt)
    dt = torch.float64 if prec == "f64" else torch.float32
    wav = torch.tensor(wl.wavelets(np.float64), dtype=dt, device="cuda")
    for graph in (False, True):
        st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision=prec)
        tr = st.step(wl.nt, wav, use_graph=graph).double().cpu().numpy()[0]
        e = rel_l2_per_trace(tr, ref)
        print(f"[source at IB {name} {prec} graph={graph}] per-trace rel-L2: max {e.max():.2e}", flush=True)
        assert e.max() < (1e-9 if prec == "f64" else 1e-4)


@pytest.mark.parametrize("name", ["3d-m8-free", "2d-m8-free"])
def test_split_calls_match_one_call(name):
    """The step counter, the sources and the receivers ride in the patch launch, and a
    call's last step is sampled at its end: a run split into calls of 1 to 33 steps, eager
    and graph-replayed, gives the traces of one call, bit for bit."""
    import torch

    import paper_2309_03600_amd as ib
    wl, w, ex, m, sols = case(name)
    wav = torch.tensor(wl.wavelets(np.float32), dtype=torch.float32, device="cuda")
    chunks = [1, 2, 3, 16, 17, 1, 33, 47]
    n = sum(chunks)
    st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision="f32")
    one = st.step(n, wav, use_graph=True).cpu().numpy()
    for graph in (False, True):
        st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision="f32")
        parts = [st.step(c, wav, use_graph=graph) for c in chunks]
        split = torch.cat(parts, dim=1).cpu().numpy()
        print(f"[split calls {name} graph={graph}] steps {st.step_count}", flush=True)
        assert st.step_count == n
        assert np.abs(one).max() > 0
        assert np.array_equal(split, one)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_graph_replay_matches_eager(prec):
    import torch

    import paper_2309_03600_amd as ib
    wl, w, ex, m, sols = case("3d-m8-free")
    dt = torch.float64 if prec == "f64" else torch.float32
    wav = torch.tensor(wl.wavelets(np.float64), dtype=dt, device="cuda")
    outs = []
    for graph in (False, True):
        st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision=prec)
        parts = [st.step(40, wav, use_graph=graph), st.step(41, wav, use_graph=graph), st.step(39, wav, use_graph=graph)]
        torch.cuda.synchronize()
        outs.append(torch.cat(parts, dim=1).cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


def test_config1_matches_oracle_fp64():
    import torch

    import paper_2309_03600_amd as ib
    wl = W.config1(nt=600)
    w = ib.ib_build_weights(wl.heights, wl.h, wl.shape, space_order=wl.M, surface=wl.surface, eta=wl.eta)
    st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, precision="f64")
    tr = st.step(wl.nt, torch.tensor(wl.wavelets(np.float64), device="cuda")).cpu().numpy()[0]
    m = model_for(wl)
    sols = solve_points(m)
    sim, _ = simulation(wl, m, sols)
    ref = sim.run(wl.wavelets(np.float64), wl.nt)
    e = rel_l2_per_trace(tr, ref)
    print(f"[config1 f64] per-trace rel-L2 vs oracle: max {e.max():.2e}")
    assert e.max() < 1e-10
