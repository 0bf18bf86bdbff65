"""State-level calls of the C ABI: the watchdog (IB_ERR_NONFINITE on a growing run, no
effect on a stable one), caller-held checkpoint handles (ib_forward_ckpt /
ib_adjoint_ckpt / ib_checkpoints_free) against the state's own checkpoints, and the
clearing of exterior values written through ib_state_field."""
import numpy as np
import pytest

from paper_2309_03600_amd import workloads as W

pytestmark = pytest.mark.gpu

_cache = {}


def _case():
    if "w" not in _cache:
        import paper_2309_03600_amd as ib
        wl = W.small2d(nx=64, nz=56, M=8, surface="free", nt=240, hill=30.0, cfg=111)
        _cache["w"] = (wl, ib.ib_build_weights(wl.heights, wl.h, wl.shape, space_order=wl.M, surface=wl.surface,
                                               eta=wl.eta))
    return _cache["w"]


def _wav(wl, prec, n=None, scale=1.0):
    import torch
    dt = torch.float64 if prec == "f64" else torch.float32
    w = wl.wavelets(np.float64) * scale
    if n is not None:
        w = np.repeat(w, n, axis=0)
    return torch.tensor(w, dtype=dt, device="cuda")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_watchdog_trips_on_a_growing_run(prec):
    import paper_2309_03600_amd as ib
    wl, w = _case()
    # three times the stable step: the leapfrog's high wavenumbers grow by a large factor
    # per step until they overflow
    st = ib.ib_state_create(w, wl.vel, 3.0 * wl.dt, wl.src, wl.rec, damp_width=0, precision=prec)
    st.set_watchdog(every=20)
    wav = _wav(wl, prec)
    print(f"[watchdog {prec}] growing run", flush=True)
    st.step(200, wav, use_graph=True)
    with pytest.raises(ib.NonFiniteError, match="after step"):
        st.status(wait=True)
    # every later step call is refused, nothing is enqueued, the step counter stays
    t = st.step_count
    with pytest.raises(ib.NonFiniteError):
        st.step(2, wav, use_graph=True)
    assert st.step_count == t
    # re-arming clears it
    st.set_watchdog(every=20)
    st.status(wait=True)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_watchdog_leaves_a_stable_run_alone(prec):
    import paper_2309_03600_amd as ib
    wl, w = _case()
    wav = _wav(wl, prec)
    out = {}
    for every in (0, 20, 7):
        st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision=prec)
        st.set_watchdog(every=every)
        a = st.step(101, wav, use_graph=True)
        st.status(wait=True)
        out[every] = a.double().cpu().numpy()
    assert np.isfinite(out[0]).all() and np.abs(out[0]).max() > 0
    # the scans read the wavefield only: identical traces with and without them
    assert np.array_equal(out[20], out[0])
    assert np.array_equal(out[7], out[0])


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_watchdog_limit_and_off_switch(prec):
    import paper_2309_03600_amd as ib
    wl, w = _case()
    wav = _wav(wl, prec)
    # a limit below the wave's amplitude trips on a stable run
    st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision=prec)
    st.set_watchdog(every=10, limit=1e-30)
    st.step(60, wav, use_graph=False)
    with pytest.raises(ib.NonFiniteError):
        st.status(wait=True)
    # scans off: the growing run is not flagged (its traces blow up)
    st = ib.ib_state_create(w, wl.vel, 3.0 * wl.dt, wl.src, wl.rec, damp_width=0, precision=prec)
    st.set_watchdog(every=0)
    tr = st.step(200, wav, use_graph=True).double().cpu().numpy()
    st.status(wait=True)
    assert not np.isfinite(tr).all() or np.abs(tr).max() > 1e30
    with pytest.raises(RuntimeError):
        st.set_watchdog(every=-1)
    with pytest.raises(RuntimeError):
        st.set_watchdog(every=10, limit=0.0)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_checkpoint_handles_match_the_state_checkpoints(prec):
    import torch

    import paper_2309_03600_amd as ib
    wl, w = _case()
    nt = 150
    wa = _wav(wl, prec)
    wb = _wav(wl, prec, scale=-0.5)
    st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision=prec)
    g = torch.Generator(device="cpu").manual_seed(7)
    # two forward runs kept side by side
    da, ca = st.forward_ckpt(nt, wa, ckpt_every=40)
    db, cb = st.forward_ckpt(nt, wb, ckpt_every=40)
    ra = (da + 0.05 * torch.randn(da.shape, generator=g, dtype=torch.float64).to(da)).contiguous()
    rb = (db + 0.05 * torch.randn(db.shape, generator=g, dtype=torch.float64).to(db)).contiguous()
    ga = st.adjoint(ra, wa, checkpoints=ca).cpu().numpy()
    gb = st.adjoint(rb, wb, checkpoints=cb).cpu().numpy()
    # the state's own checkpoints (ib_forward / ib_adjoint) give the same bits
    for wav, res, d, gr in ((wa, ra, da, ga), (wb, rb, db, gb)):
        d2 = st.forward(nt, wav, ckpt_every=40)
        assert torch.equal(d, d2)
        assert np.array_equal(st.adjoint(res, wav).cpu().numpy(), gr)
    assert np.abs(ga).max() > 0 and not np.array_equal(ga, gb)
    # a handle is tied to the state that wrote it
    other = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision=prec)
    other.forward(nt, wa, ckpt_every=40)
    with pytest.raises(RuntimeError, match="another state"):
        other.adjoint(ra, wa, checkpoints=ca)
    # reuse keeps the handle
    h = ca._h
    _, ca2 = st.forward_ckpt(nt, wa, ckpt_every=40, checkpoints=ca)
    assert ca2 is ca and ca._h == h
    assert np.array_equal(st.adjoint(ra, wa, checkpoints=ca).cpu().numpy(), ga)
    ca.close()
    cb.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_field_write_clears_exterior_nodes(prec):
    import torch

    import paper_2309_03600_amd as ib
    wl, w = _case()
    cls = w.export()["node_class"].reshape(wl.shape[1], wl.shape[0])
    interior = (cls & 1).astype(bool)
    st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, precision=prec)
    dt = torch.float64 if prec == "f64" else torch.float32
    ones = torch.ones((wl.shape[1], wl.shape[0]), dtype=dt, device="cuda")
    st.field(0, 0, ones)
    st.field(1, 0, 0.5 * ones)
    p = st.field(0, 0).double().cpu().numpy()
    pm = st.field(1, 0).double().cpu().numpy()
    assert (p[interior] == 1.0).all() and (p[~interior] == 0.0).all()
    assert (pm[interior] == 0.5).all() and (pm[~interior] == 0.0).all()
