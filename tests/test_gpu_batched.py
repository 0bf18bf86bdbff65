"""Batched shots (one launch per kernel per step over all shots, optionally replayed from
a HIP graph) reproduce the single-shot runs exactly."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2309_03600_amd import workloads as W  # noqa: E402


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("graph", [False, True])
def test_batched_equals_single_shots(prec, graph):
    import torch

    import paper_2309_03600_amd as ib
    wl = W.small3d(n=32, nz=48, relief=50.0, nt=90, nshots=5, cfg=99)
    w = ib.ib_build_weights(wl.heights, wl.h, wl.shape, space_order=wl.M, surface=wl.surface, eta=wl.eta)
    dt = torch.float32 if prec == "f32" else torch.float64
    rng = np.random.default_rng(3)
    # different wavelets per shot (frequency and amplitude)
    wav = np.stack([W.ricker(wl.nt, wl.dt, 10.0 + 2 * s) * (1 + 0.1 * s) for s in range(wl.src.shape[0])])
    wav_t = torch.tensor(wav, dtype=dt, device="cuda")
    st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision=prec)
    tb = torch.cat([st.step(45, wav_t, use_graph=graph), st.step(45, wav_t, use_graph=graph)], dim=1).cpu().numpy()
    for s in range(wl.src.shape[0]):
        s1 = ib.ib_state_create(w, wl.vel, wl.dt, wl.src[s:s + 1], wl.rec, damp_width=wl.damp_width, precision=prec)
        t1 = s1.step(wl.nt, wav_t[s:s + 1].contiguous()).cpu().numpy()[0]
        assert np.array_equal(tb[s], t1), (s, np.abs(tb[s] - t1).max())
    assert np.abs(tb).max() > 0


def test_batched_graph_replays_are_repeatable():
    import torch

    import paper_2309_03600_amd as ib
    wl = W.small3d(n=32, nz=48, relief=50.0, nt=64, nshots=4, cfg=99)
    w = ib.ib_build_weights(wl.heights, wl.h, wl.shape, space_order=wl.M, surface=wl.surface, eta=wl.eta)
    wav = torch.tensor(wl.wavelets(np.float64), dtype=torch.float32, device="cuda")
    outs = []
    for _ in range(3):
        st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision="f32")
        parts = []
        for k in range(4):
            parts.append(st.step(16, wav, use_graph=True))
            torch.cuda.synchronize()
        outs.append(torch.cat(parts, dim=1).cpu().numpy())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[1], outs[2])


_oracle = {}


def _multishot_case():
    """Three shots at distinct positions with distinct wavelets (frequency, delay, sign and
    amplitude), on a 3D grid large enough for several patch tiles; the oracle's traces of
    each shot, run on its own."""
    if not _oracle:
        import os
        import sys
        sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
        from oracle_cases import model_for, simulation, solve_points

        import paper_2309_03600_amd as ib
        wl = W.small3d(n=32, nz=48, relief=50.0, nt=160, nshots=3, cfg=121)
        assert len({tuple(p) for p in wl.src}) == 3
        wav = np.stack([W.ricker(wl.nt, wl.dt, 35.0 + 10 * s, t0=(1.2 + 0.2 * s) / (35.0 + 10 * s)) * (1 - 0.8 * s)
                        for s in range(3)])
        print(f"[multishot] {wl.shape}, sources {wl.src.tolist()}", flush=True)
        w = ib.ib_build_weights(wl.heights, wl.h, wl.shape, space_order=wl.M, surface=wl.surface, eta=wl.eta)
        m = model_for(wl)
        sols = solve_points(m)
        sim, L = simulation(wl, m, sols)
        refs = []
        for s in range(3):
            ss = type(sim)(m, L, wl.vel, wl.dt, wl.src[s:s + 1], wl.rec, damp_width=wl.damp_width, damp_R=wl.damp_R)
            refs.append(ss.run(wav[s:s + 1], wl.nt))
        _oracle.update(wl=wl, w=w, wav=wav, refs=refs)
    return _oracle


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("graph", [False, True])
def test_multishot_traces_match_oracle(prec, graph):
    # every shot of one batched state (for FP32 with the column-run patch taking two shots
    # per pass, variant 9) against the oracle's run of that shot alone, per trace
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from oracle_cases import rel_l2_per_trace

    import torch

    import paper_2309_03600_amd as ib
    c = _multishot_case()
    wl, w, wav, refs = c["wl"], c["w"], c["wav"], c["refs"]
    dt = torch.float32 if prec == "f32" else torch.float64
    st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision=prec)
    st.set_tuning(1, 0, 9)
    wav_t = torch.tensor(wav, dtype=dt, device="cuda")
    tr = torch.cat([st.step(61, wav_t, use_graph=graph), st.step(99, wav_t, use_graph=graph)], dim=1)
    tr = tr.double().cpu().numpy()
    for s in range(3):
        e = rel_l2_per_trace(tr[s], refs[s])
        print(f"[multishot {prec} graph={graph}] shot {s}: per-trace rel-L2 max {e.max():.2e} "
              f"median {np.median(e):.2e}", flush=True)
        assert np.abs(refs[s]).max() > 0
        assert e.max() < (1e-9 if prec == "f64" else 1e-4), s
