"""First-order p-v form: GPU (HIP, through the C ABI) against the FP64 staggered oracle."""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from oracle_cases import rel_l2_per_trace, solve_staggered  # noqa: E402

from paper_2309_03600_amd import workloads as W  # noqa: E402

CASES = {
    "2d-m8-free": lambda: W.small2d(M=8, surface="free", nt=300),
    "2d-m4-free": lambda: W.small2d(M=4, surface="free", nt=300, cfg=92),
    "2d-m6-free": lambda: W.small2d(M=6, surface="free", nt=300, cfg=94, hill=90.0),
}

_cache = {}


def case(name):
    if name not in _cache:
        import torch

        import paper_2309_03600_amd as ib
        from oracle import staggered as S
        wl = CASES[name]()
        print(f"[pv case {name}] shape={wl.shape} M={wl.M} surface={wl.surface}", flush=True)
        w = ib.ib_build_weights(wl.heights, wl.h, wl.shape, space_order=wl.M, surface=wl.surface, eta=wl.eta,
                                form="pv1", eta_v=0.0)
        torch.cuda.synchronize()
        m = S.StaggeredModel(wl.heights, wl.h, wl.shape, M=wl.M, surface=wl.surface, eta_p=wl.eta, eta_v=0.0)
        vsol, psol = solve_staggered(m)
        G, D = S.assemble(m, vsol, psol)
        _cache[name] = (wl, w, w.export(), m, vsol, psol, G, D)
    return _cache[name]


def _lin(g, shape):
    return int(g[1]) * shape[0] + int(g[0] % shape[0])


def _node_weights(offsets, weights, g, shape):
    out = {}
    for o, wv in zip(offsets, weights):
        q = (int(g[0] + o[0]) % shape[0], int(g[1] + o[1]))
        out[_lin(q, shape)] = out.get(_lin(q, shape), 0.0) + float(wv)
    return out


@pytest.mark.parametrize("name", list(CASES))
def test_classes_identical(name):
    wl, w, ex, m, *_ = case(name)
    cls = ex["node_class"]
    ip = m.inter["p"].ravel()
    assert np.array_equal((cls & 1).astype(bool), ip)
    assert np.array_equal(((cls >> 1) & 1).astype(bool), m.excl["p"].ravel() & ip)
    for n in range(m.d):
        vc = ex["vclass"][n]
        iv = m.inter[n].ravel()
        assert np.array_equal((vc & 1).astype(bool), iv), n
        assert not np.any((vc >> 1) & 1)          # eta_v = 0: no velocity node is excluded


@pytest.mark.parametrize("name", list(CASES))
def test_rows_match_oracle(name):
    wl, w, ex, m, vsol, psol, G, D = case(name)
    rows, ent = ex["rows"], ex["entries"]
    d = m.d
    starts = np.concatenate([[0], np.cumsum(rows[:, 2])])
    # row sets per family, memory order
    for fam in range(d + 1):
        sel = np.nonzero(rows[:, 0] == fam)[0]
        pts = m.ib_v(fam) if fam < d else m.ib_p()
        lin = [_lin(g, wl.shape) for g in pts]
        assert list(rows[sel, 1]) == lin, fam
    worst = 0.0
    for r in range(len(rows)):
        fam, node = int(rows[r, 0]), int(rows[r, 1])
        g = (node % wl.shape[0], node // wl.shape[0])
        e = ent[starts[r]:starts[r + 1]]
        if fam < d:
            s = vsol[fam][g]
            assert np.all(e[:, 0] == -1)
            ref = {(-1, k): v for k, v in _node_weights(s["offsets"], s["weights"], g, wl.shape).items()}
        else:
            s = psol[g]
            ref = {}
            for n, (offs, wts) in enumerate(s["fields"]):
                for k, v in _node_weights(offs, wts, g, wl.shape).items():
                    ref[(n, k)] = v
        got = {}
        for fld, nd, wv in e:
            got[(int(fld), int(nd))] = got.get((int(fld), int(nd)), 0.0) + wv
        assert set(got) == set(ref), (fam, g)
        scale = max(1.0, max(abs(v) for v in ref.values()))
        err = max(abs(got[k] - ref[k]) for k in ref) / scale
        # same bound as the second-order form: boundary points agree to ~1e-14, y moves by
        # up to cond(A) times the relative row perturbation
        tol = max(1e-11, s["cond"] * 1e-12)
        worst = max(worst, err / tol)
        assert err <= tol, (fam, g, err, tol)
    print(f"[pv {name}] rows {len(rows)} worst weight error / tolerance = {worst:.3f}")


def _oracle_sim(wl, m, G, D):
    from oracle import staggered as S
    return S.StaggeredSimulation(m, G, D, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width,
                                 damp_R=wl.damp_R)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_one_step_matches_oracle(name, prec):
    import torch

    import paper_2309_03600_amd as ib
    wl, w, ex, m, vsol, psol, G, D = case(name)
    sim = _oracle_sim(wl, m, G, D)
    st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision=prec)
    rng = np.random.default_rng(11)
    tdt = torch.float64 if prec == "f64" else torch.float32
    p = np.where(m.inter["p"], rng.standard_normal(m.inter["p"].shape), 0.0)
    st.field(0, 0, torch.tensor(p, dtype=tdt))
    sim.p = torch.tensor(p, dtype=tdt).double().numpy().ravel()
    for n in range(m.d):
        v = np.where(m.inter[n], rng.standard_normal(m.inter[n].shape), 0.0)
        st.field(2 + n, 0, torch.tensor(v, dtype=tdt))
        sim.v[n] = torch.tensor(v, dtype=tdt).double().numpy().ravel()
    st.step(1, torch.zeros((1, 4), dtype=tdt, device="cuda"))
    sim.step([0.0])
    tol = 1e-11 if prec == "f64" else 2e-6
    errs = []
    for which, ref in [(0, sim.p)] + [(2 + n, sim.v[n]) for n in range(m.d)]:
        got = st.field(which, 0).double().cpu().numpy().ravel()
        errs.append(np.abs(got - ref).max() / np.abs(ref).max())
    print(f"[pv {name} {prec}] one-step max errors p/v: {['%.2e' % e for e in errs]}")
    assert max(errs) < tol


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_traces_match_oracle(name, prec):
    import torch

    import paper_2309_03600_amd as ib
    wl, w, ex, m, vsol, psol, G, D = case(name)
    sim = _oracle_sim(wl, m, G, D)
    ref = sim.run(wl.wavelets(np.float64), wl.nt)
    st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision=prec)
    tdt = torch.float64 if prec == "f64" else torch.float32
    wav = torch.tensor(wl.wavelets(np.float64), dtype=tdt, device="cuda")
    tr = st.step(wl.nt, wav).double().cpu().numpy()[0]
    e = rel_l2_per_trace(tr, ref)
    print(f"[pv {name} {prec}] per-trace rel-L2: max {e.max():.2e} median {np.median(e):.2e}")
    assert e.max() < (1e-9 if prec == "f64" else 1e-4)


def test_split_calls_match_one_call():
    """The rows launches carry the sources (divergence rows) and the receivers of the step
    before (gradient rows), and a call's last step is sampled at its end: a run split into
    calls of 1 to 47 steps, eager and graph-replayed, gives the traces of one call, bit for
    bit."""
    import torch

    import paper_2309_03600_amd as ib
    wl, w, *_ = case("2d-m8-free")
    wav = torch.tensor(wl.wavelets(np.float32), dtype=torch.float32, device="cuda")
    chunks = [1, 2, 3, 16, 17, 1, 33, 47]
    n = sum(chunks)
    st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision="f32")
    one = st.step(n, wav, use_graph=True).cpu().numpy()
    for graph in (False, True):
        st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision="f32")
        split = torch.cat([st.step(c, wav, use_graph=graph) for c in chunks], dim=1).cpu().numpy()
        print(f"[pv split calls graph={graph}] steps {st.step_count}", flush=True)
        assert st.step_count == n
        assert np.abs(one).max() > 0
        assert np.array_equal(split, one)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_source_at_a_modified_row_matches_oracle(prec):
    """A source whose interpolation corners include a p node just under the surface (a
    modified divergence row): its injection would race with the row's update inside the
    rows launch, so it runs as a launch of its own; traces against the oracle."""
    import dataclasses

    import torch

    import paper_2309_03600_amd as ib
    wl0, w, ex, m, vsol, psol, G, D = case("2d-m8-free")
    nx, nz = wl0.shape
    inter = np.asarray(m.inter["p"]).reshape(nz, nx).astype(bool)
    pick = None
    for z in range(nz - 1):
        for x in range(3, nx - 4):
            cell = inter[z:z + 2, x:x + 2]
            depth = z * wl0.h - wl0.heights[x]
            if pick is None and cell.all() and 0.0 < depth < wl0.h:
                pick = (x, z)
    assert pick is not None
    x, z = pick
    wl = dataclasses.replace(wl0, src=np.array([[(x + 0.5) * wl0.h, (z + 0.5) * wl0.h]]))
    print(f"[pv source at a row {prec}] cell {pick}", flush=True)
    sim = _oracle_sim(wl, m, G, D)
    ref = sim.run(wl.wavelets(np.float64), wl.nt)
    tdt = torch.float64 if prec == "f64" else torch.float32
    wav = torch.tensor(wl.wavelets(np.float64), dtype=tdt, device="cuda")
    st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision=prec)
    tr = st.step(wl.nt, wav, use_graph=True).double().cpu().numpy()[0]
    e = rel_l2_per_trace(tr, ref)
    print(f"[pv source at a row {prec}] per-trace rel-L2: max {e.max():.2e}", flush=True)
    assert e.max() < (1e-9 if prec == "f64" else 1e-4)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_graph_replay_matches_eager(prec):
    import torch

    import paper_2309_03600_amd as ib
    wl, w, *_ = case("2d-m8-free")
    tdt = torch.float64 if prec == "f64" else torch.float32
    wav = torch.tensor(wl.wavelets(np.float64), dtype=tdt, device="cuda")
    outs = []
    for graph in (False, True):
        st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision=prec)
        parts = []
        for n in (40, 41, 39):
            parts.append(st.step(n, wav, use_graph=graph))
            torch.cuda.synchronize()
        outs.append(torch.cat(parts, dim=1).cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


def test_first_order_rigid_rejected():
    import paper_2309_03600_amd as ib
    wl = W.small2d(M=8, surface="rigid", nt=10)
    with pytest.raises(RuntimeError, match="free surface"):
        ib.ib_build_weights(wl.heights, wl.h, wl.shape, space_order=8, surface="rigid", form="pv1")


def test_first_order_state_rejects_adjoint_calls():
    import torch

    import paper_2309_03600_amd as ib
    wl, w, *_ = case("2d-m8-free")
    st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision="f64")
    wav = torch.tensor(wl.wavelets(np.float64), device="cuda")
    with pytest.raises(RuntimeError):
        st.forward(10, wav, ckpt_every=5)
    with pytest.raises(RuntimeError):
        st.run_kernel(0, 1)
    with pytest.raises(RuntimeError):
        st.field(1, 0)
