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
