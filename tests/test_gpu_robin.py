"""Mixed surface p + a(x_b) dp/dn = 0 with a laterally varying coefficient: GPU through the C
ABI against the FP64 oracle (coefficients at the boundary points, weights, condition-value
weights, traces with and without boundary values) and against a flat-surface standing wave."""
import math
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from manufactured import robin_coefficient, robin_standing_wave  # noqa: E402
from oracle_cases import rel_l2_per_trace, solve_points  # noqa: E402

from oracle import fd, forcing, stepper  # noqa: E402
from oracle.weights import IBModel  # noqa: E402
from paper_2309_03600_amd import workloads as W  # noqa: E402


def _robin_2d(wl):
    return robin_coefficient(np.arange(wl.shape[0]) * wl.h, wl.shape[0] * wl.h)


def _robin_3d(wl):
    nx, ny = wl.shape[0], wl.shape[1]
    x = np.arange(nx) * wl.h
    y = np.arange(ny) * wl.h
    return robin_coefficient(x[None, :], nx * wl.h) * (1.0 + 0.3 * np.sin(2 * math.pi * y[:, None] / (ny * wl.h)))


CASES = {
    "2d-m8": lambda: (W.small2d(M=8, surface="robin", nt=300), _robin_2d),
    "2d-m4": lambda: (W.small2d(M=4, surface="robin", nt=300, cfg=92), _robin_2d),
    "3d-m8": lambda: (W.small3d(n=16, nz=40, relief=40.0, surface="robin", nt=120), _robin_3d),
}

_cache = {}


def case(name):
    if name not in _cache:
        import torch

        import paper_2309_03600_amd as ib
        wl, mk = CASES[name]()
        a = mk(wl)
        print(f"[robin case {name}] shape={wl.shape} M={wl.M} a in [{a.min():.1f}, {a.max():.1f}] m", flush=True)
        w = ib.ib_build_weights(wl.heights, wl.h, wl.shape, space_order=wl.M, surface="robin", eta=wl.eta,
                                keep_bc_weights=True, robin=a)
        torch.cuda.synchronize()
        m = IBModel(wl.heights, wl.h, wl.shape, M=wl.M, surface="robin", eta=wl.eta, robin=a)
        sols = solve_points(m)
        ex = w.export()
        gh = ex["bpoints"][:, :3].astype(np.int64)
        if m.d == 2:
            gh = gh[:, [0, 2]]
        omap = {tuple(h): k for k, h in enumerate(m.bp_host.tolist())}
        g2o = np.array([omap[tuple(h)] for h in gh.tolist()], dtype=np.int64)
        _cache[name] = (wl, a, w, ex, m, sols, g2o)
    return _cache[name]


@pytest.mark.parametrize("name", list(CASES))
def test_coefficients_at_boundary_points(name):
    wl, a, w, ex, m, sols, g2o = case(name)
    got = ex["bpoints"][:, 6]
    ref = m.bp_robin[g2o] * wl.h
    assert np.abs(got - ref).max() < 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("name", list(CASES))
def test_weights_match_oracle(name):
    wl, a, w, ex, m, sols, g2o = case(name)
    meta, W64 = ex["ib_meta"], ex["weights"]
    cnt, ent = ex["bc_counts"], ex["bc_entries"]
    starts = np.concatenate([[0], np.cumsum(cnt)])
    worst = 0.0
    for j, p in enumerate(m.ib_points()):
        s = sols[tuple(int(v) for v in p)]
        k, Mb, nw, off = meta[j]
        assert (k, Mb, nw) == (s["radius_step"], s["order"], len(s["weights"])), (tuple(p), meta[j])
        tol = max(1e-11, s["cond"] * 1e-12)
        scale = max(1.0, np.abs(s["weights"]).max())
        err = np.abs(W64[off:off + nw] - s["weights"]).max() / scale
        ref = {(int(b), q): v for b, q, v in forcing.forcing_row(s)}
        got = {(int(g2o[int(b)]), int(q)): v for b, q, v in ent[starts[j]:starts[j + 1]]}
        assert set(got) == set(ref), tuple(p)
        fscale = max(1.0, max(abs(v) for v in ref.values()))
        ferr = max(abs(got[key] - ref[key]) for key in ref) / fscale
        worst = max(worst, err / tol, ferr / tol)
        assert err <= tol and ferr <= tol, (tuple(p), err, ferr, tol)
    print(f"[robin {name}] worst weight error / tolerance = {worst:.3f}")


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("forced", [False, True])
def test_traces_match_oracle(name, prec, forced):
    import torch

    import paper_2309_03600_amd as ib
    wl, a, w, ex, m, sols, g2o = case(name)
    L = stepper.assemble_laplacian(m, sols)
    st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision=prec)
    fo = None
    if forced:
        nq = forcing.n_conditions("robin", wl.M)
        rng = np.random.default_rng(43)
        g_o = rng.standard_normal((len(m.bp_xb), nq)) / np.array([wl.h ** (2 * q) for q in range(nq)])
        t = np.arange(wl.nt + 2) * wl.dt
        s = np.stack([np.cos(2 * math.pi * (10.0 + 2 * q) * t) * np.exp(-((t - 0.04) / 0.03) ** 2)
                      for q in range(nq)])
        fo = (forcing.forcing_vectors(m, sols, g_o), s)
        st.set_forcing(g_o[g2o], s)
    sim = stepper.Simulation(m, L, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, damp_R=wl.damp_R,
                             forcing=fo)
    ref = sim.run(wl.wavelets(np.float64), wl.nt)
    tdt = torch.float64 if prec == "f64" else torch.float32
    tr = st.step(wl.nt, torch.tensor(wl.wavelets(np.float64), dtype=tdt, device="cuda"), use_graph=True)
    e = rel_l2_per_trace(tr.double().cpu().numpy()[0], ref)
    print(f"[robin {name} {prec} forced={forced}] per-trace rel-L2: max {e.max():.2e} median {np.median(e):.2e}")
    assert e.max() < (1e-9 if prec == "f64" else 1e-4)


def _flat_error_gpu(h, a=15.0, M=4, T=0.04, c=1500.0):
    import torch

    import paper_2309_03600_amd as ib
    nx, nz = int(round(240.0 / h)), int(round(500.0 / h))
    zs = 200.3
    w = ib.ib_build_weights(np.full(nx, zs), h, (nx, nz), space_order=M, surface="robin", eta=0.5,
                            robin=np.full(nx, a))
    inter = (w.export()["node_class"] & 1).astype(bool).reshape(nz, nx)
    dt = 0.1 * fd.critical_dt(h, c, M, 2)
    nt = int(round(T / dt))
    p, om = robin_standing_wave(nx * h, zs, a, c)
    st = ib.ib_state_create(w, np.full((nz, nx), c), dt, [[0.5 * nx * h, 300.0]], [], precision="f64")
    X, Z = np.meshgrid(np.arange(nx) * h, np.arange(nz) * h)
    st.field(0, 0, torch.tensor(np.where(inter, p(X, Z, 0.0), 0.0)))
    st.field(1, 0, torch.tensor(np.where(inter, p(X, Z, -dt), 0.0)))
    st.step(nt, torch.zeros((1, nt), dtype=torch.float64, device="cuda"), use_graph=True)
    got = st.field(0, 0).cpu().numpy()
    exact = np.where(inter, p(X, Z, nt * dt), 0.0)
    sel = inter & (Z < 340.0)
    return np.abs(got - exact)[sel].max()


def test_flat_robin_standing_wave_gpu():
    e10, e5 = _flat_error_gpu(10.0), _flat_error_gpu(5.0)
    print(f"[robin standing wave] max error h=10: {e10:.3e}, h=5: {e5:.3e} (order {np.log2(e10 / e5):.2f})")
    assert e5 < 2e-3 and np.log2(e10 / e5) > 2.5


def test_robin_argument_errors():
    import paper_2309_03600_amd as ib
    wl = W.small2d(M=4, nt=10)
    with pytest.raises(RuntimeError, match="robin_dev"):
        ib.ib_build_weights(wl.heights, wl.h, wl.shape, space_order=4, surface="robin")
    with pytest.raises(RuntimeError, match="robin_dev"):
        ib.ib_build_weights(wl.heights, wl.h, wl.shape, space_order=4, surface="free", robin=_robin_2d(wl))
    with pytest.raises(RuntimeError, match="free surface only|second-order form"):
        ib.ib_build_weights(wl.heights, wl.h, wl.shape, space_order=4, surface="robin", robin=_robin_2d(wl),
                            form="pv1")
