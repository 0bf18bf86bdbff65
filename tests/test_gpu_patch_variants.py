"""The tiled IB patch kernels (dense-range records with point records read per wavefront or
staged in LDS, compact records, and column-run records with one or two shots per pass) on
one 3D case with many tiles: the variants that share a summation order give bit-identical
traces, the others agree to rounding."""
import numpy as np
import pytest

from paper_2309_03600_amd import workloads as W

pytestmark = pytest.mark.gpu

SAME_ORDER = [4, 5, 6]
OTHER_ORDER = [0, 1, 2, 3, 7, 8, 9]

_weights = {}


def _case():
    if "w" not in _weights:
        import paper_2309_03600_amd as ib
        wl = W.small3d(n=48, nz=56, relief=60.0, nshots=3, nt=60)
        print(f"[patch variants] shape={wl.shape} M={wl.M}", flush=True)
        _weights["w"] = (wl, ib.ib_build_weights(wl.heights, wl.h, wl.shape, space_order=wl.M, surface=wl.surface,
                                                 eta=wl.eta))
    return _weights["w"]


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("nshots", [1, 3])
def test_patch_variants_agree(prec, nshots):
    import torch

    import paper_2309_03600_amd as ib
    wl, w = _case()
    tdt = torch.float64 if prec == "f64" else torch.float32
    wav = torch.tensor(wl.wavelets(np.float64)[:nshots], dtype=tdt, device="cuda")
    out = {}
    for v in SAME_ORDER + OTHER_ORDER:
        print(f"[patch variants] {prec} shots={nshots} variant {v}", flush=True)
        st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src[:nshots], wl.rec, damp_width=wl.damp_width, precision=prec)
        st.set_tuning(1, 0, v)
        out[v] = st.step(wl.nt, wav, use_graph=True).double().cpu().numpy()
    ref = out[4]
    assert np.isfinite(ref).all() and np.abs(ref).max() > 0
    for v in SAME_ORDER:
        rel = np.abs(out[v] - ref).max() / np.abs(ref).max()
        assert np.array_equal(out[v], ref), (v, rel)
    # the column-run kernel sums the same way with one or two shots per pass
    assert np.array_equal(out[8], out[9])
    tol = 1e-12 if prec == "f64" else 1e-5
    for v in OTHER_ORDER:
        rel = np.abs(out[v] - ref).max() / np.abs(ref).max()
        assert rel < tol, (v, rel)
