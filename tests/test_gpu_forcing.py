"""Non-zero boundary values (inhomogeneous conditions): GPU through the C ABI against the FP64
oracle (condition-value weights, forced traces) and against a manufactured standing wave."""
import math
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from manufactured import standing_wave, undulating_surface  # noqa: E402
from oracle_cases import model_for, rel_l2_per_trace, solve_points  # noqa: E402

from oracle import fd, forcing, stepper  # noqa: E402
from paper_2309_03600_amd import workloads as W  # noqa: E402

CASES = {
    "2d-m8-free": lambda: W.small2d(M=8, surface="free", nt=300),
    "2d-m8-rigid": lambda: W.small2d(M=8, surface="rigid", nt=300),
    "2d-m4-free": lambda: W.small2d(M=4, surface="free", nt=300, cfg=92),
    "3d-m8-free": lambda: W.small3d(n=16, nz=40, relief=40.0, surface="free", nt=120),
    "3d-m4-rigid": lambda: W.small3d(n=16, nz=36, relief=30.0, surface="rigid", nt=120, cfg=93, z_top_cells=12),
}

_cache = {}


def case(name):
    if name not in _cache:
        import dataclasses

        import torch

        import paper_2309_03600_amd as ib
        wl = CASES[name]()
        if name == "3d-m4-rigid":
            wl = dataclasses.replace(wl, M=4)
        print(f"[forcing case {name}] shape={wl.shape} M={wl.M} surface={wl.surface}", flush=True)
        w = ib.ib_build_weights(wl.heights, wl.h, wl.shape, space_order=wl.M, surface=wl.surface, eta=wl.eta,
                                keep_bc_weights=True)
        torch.cuda.synchronize()
        m = model_for(wl)
        sols = solve_points(m)
        ex = w.export()
        # boundary point of the table -> the oracle's, by host node
        gh = ex["bpoints"][:, :3].astype(np.int64)
        if m.d == 2:
            gh = gh[:, [0, 2]]
        omap = {tuple(h): k for k, h in enumerate(m.bp_host.tolist())}
        g2o = np.array([omap[tuple(h)] for h in gh.tolist()], dtype=np.int64)
        _cache[name] = (wl, w, ex, m, sols, g2o)
    return _cache[name]


@pytest.mark.parametrize("name", list(CASES))
def test_condition_value_weights_match_oracle(name):
    wl, w, ex, m, sols, g2o = case(name)
    cnt, ent = ex["bc_counts"], ex["bc_entries"]
    starts = np.concatenate([[0], np.cumsum(cnt)])
    worst = 0.0
    for j, p in enumerate(m.ib_points()):
        s = sols[tuple(int(v) for v in p)]
        ref = {(int(b), q): v for b, q, v in forcing.forcing_row(s)}
        e = ent[starts[j]:starts[j + 1]]
        got = {(int(g2o[int(b)]), int(q)): v for b, q, v in e}
        assert set(got) == set(ref), (tuple(p), sorted(set(got) ^ set(ref))[:4])
        scale = max(1.0, max(abs(v) for v in ref.values()))
        tol = max(1e-11, s["cond"] * 1e-12)
        err = max(abs(got[k] - ref[k]) for k in ref) / scale
        worst = max(worst, err / tol)
        assert err <= tol, (tuple(p), err, tol)
    print(f"[forcing {name}] {int(cnt.sum())} condition-value weights, worst error / tolerance = {worst:.3f}")


def _forcing_inputs(wl, m, nq):
    rng = np.random.default_rng(41)
    nb = len(m.bp_xb)
    g_o = rng.standard_normal((nb, nq)) / np.array([wl.h ** forcing.order_of(wl.surface, q) for q in range(nq)])
    t = np.arange(wl.nt + 5) * wl.dt
    s = np.stack([np.sin(2 * math.pi * (8.0 + 3 * q) * t) * np.exp(-((t - 0.05) / 0.04) ** 2)
                  for q in range(nq)])
    return g_o, s


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_forced_traces_match_oracle(name, prec):
    import torch

    import paper_2309_03600_amd as ib
    wl, w, ex, m, sols, g2o = case(name)
    nq = forcing.n_conditions(wl.surface, wl.M)
    g_o, s = _forcing_inputs(wl, m, nq)
    B = forcing.forcing_vectors(m, sols, g_o)
    L = stepper.assemble_laplacian(m, sols)
    sim = stepper.Simulation(m, L, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, damp_R=wl.damp_R,
                             forcing=(B, s))
    ref = sim.run(wl.wavelets(np.float64), wl.nt)
    st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision=prec)
    st.set_forcing(g_o[g2o], s)
    tdt = torch.float64 if prec == "f64" else torch.float32
    tr = st.step(wl.nt, torch.tensor(wl.wavelets(np.float64), dtype=tdt, device="cuda"), use_graph=True)
    e = rel_l2_per_trace(tr.double().cpu().numpy()[0], ref)
    print(f"[forcing {name} {prec}] per-trace rel-L2: max {e.max():.2e} median {np.median(e):.2e}")
    assert e.max() < (1e-9 if prec == "f64" else 1e-4)


def test_forcing_graph_and_eager_agree_and_clearing_restores_homogeneous():
    import torch

    import paper_2309_03600_amd as ib
    wl, w, ex, m, sols, g2o = case("2d-m8-free")
    nq = forcing.n_conditions("free", 8)
    g_o, s = _forcing_inputs(wl, m, nq)
    wav = torch.tensor(wl.wavelets(np.float64), device="cuda")
    runs = []
    for graph, forced in ((True, True), (False, True), (True, False)):
        st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision="f64")
        st.set_forcing(g_o[g2o], s)
        if not forced:
            st.set_forcing(None, None)
        runs.append(st.step(120, wav, use_graph=graph).cpu().numpy())
    plain = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision="f64")
    ref_plain = plain.step(120, wav, use_graph=True).cpu().numpy()
    assert np.array_equal(runs[0], runs[1])
    assert np.array_equal(runs[2], ref_plain)
    assert np.abs(runs[0] - ref_plain).max() > 1e-3 * np.abs(ref_plain).max()


def test_forcing_argument_and_state_errors():
    import torch

    import paper_2309_03600_amd as ib
    wl, w, ex, m, sols, g2o = case("2d-m4-free")
    nq = forcing.n_conditions("free", 4)
    g_o, s = _forcing_inputs(wl, m, nq)
    st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, precision="f64")
    with pytest.raises(RuntimeError, match="nq"):
        st.set_forcing(np.zeros((len(g2o), nq + 1)), np.zeros((nq + 1, 10)))
    st.set_forcing(g_o[g2o], s[:, :20])
    wav = torch.zeros((1, 100), dtype=torch.float64, device="cuda")
    with pytest.raises(RuntimeError, match="time functions"):
        st.step(30, wav)
    with pytest.raises(RuntimeError, match="boundary values"):
        st.forward(10, wav)
    plain = ib.ib_build_weights(wl.heights, wl.h, wl.shape, space_order=4, surface="free", eta=wl.eta)
    st2 = ib.ib_state_create(plain, wl.vel, wl.dt, wl.src, wl.rec, precision="f64")
    with pytest.raises(RuntimeError, match="keep_bc_weights"):
        st2.set_forcing(g_o[g2o], s)
    with pytest.raises(RuntimeError, match="N-D method"):
        ib.ib_build_weights(wl.heights, wl.h, wl.shape, space_order=4, surface="free", method="1d",
                            keep_bc_weights=True)


def _manufactured_error_gpu(h, M=4, T=0.04, c=1500.0, forced=True, prec="f64"):
    """GPU version of the oracle's manufactured standing-wave check (same set-up)."""
    import torch

    import paper_2309_03600_amd as ib
    nx, nz = int(round(240.0 / h)), int(round(500.0 / h))
    x = np.arange(nx) * h
    H = undulating_surface(x, nx * h)
    w = ib.ib_build_weights(H, h, (nx, nz), space_order=M, surface="free", eta=0.5, keep_bc_weights=True)
    ex = w.export()
    inter = (ex["node_class"] & 1).astype(bool).reshape(nz, nx)
    dt = 0.1 * fd.critical_dt(h, c, M, 2)
    nt = int(round(T / dt))
    p, g, om = standing_wave(nx, h, c)
    xb = ex["bpoints"][:, [3, 5]] * h
    nq = forcing.n_conditions("free", M)
    G = np.stack([g(xb, q) for q in range(nq)], axis=1)
    s = np.cos(om * np.arange(nt + 1) * dt)[None, :].repeat(nq, axis=0)
    st = ib.ib_state_create(w, np.full((nz, nx), c), dt, [[0.5 * nx * h, 300.0]], [], precision=prec)
    if forced:
        st.set_forcing(G, s)
    X, Z = np.meshgrid(x, np.arange(nz) * h)
    tdt = torch.float64 if prec == "f64" else torch.float32
    st.field(0, 0, torch.tensor(np.where(inter, p(X, Z, 0.0), 0.0), dtype=tdt))
    st.field(1, 0, torch.tensor(np.where(inter, p(X, Z, -dt), 0.0), dtype=tdt))
    st.step(nt, torch.zeros((1, nt), dtype=tdt, device="cuda"), use_graph=True)
    got = st.field(0, 0).double().cpu().numpy()
    exact = np.where(inter, p(X, Z, nt * dt), 0.0)
    sel = inter & (Z < 340.0)
    return np.abs(got - exact)[sel].max()


def test_manufactured_standing_wave_gpu():
    e10, e5 = _manufactured_error_gpu(10.0), _manufactured_error_gpu(5.0)
    e5_plain = _manufactured_error_gpu(5.0, forced=False)
    e5_f32 = _manufactured_error_gpu(5.0, prec="f32")
    print(f"[forcing manufactured] max error h=10: {e10:.3e}, h=5: {e5:.3e} (order {np.log2(e10 / e5):.2f}); "
          f"FP32 h=5: {e5_f32:.3e}; without the boundary values: {e5_plain:.3e}")
    assert e5 < 1e-3 and np.log2(e10 / e5) > 2.5
    assert e5_plain > 30 * e5
    assert e5_f32 < 2 * e5 + 1e-4
