"""Convergence under refinement (the paper's convergence-testing set-up: fourth-order space
discretisation, time step 10 % of critical), GPU path against the method-of-images
solution of a flat free or rigid surface placed between grid rows, for both forms.

The surface sits off-grid (107 m, or 147 m at M = 8) at every spacing used; a Ricker source
103 m below it and four receivers (offsets 0 and 200 m, 3 m and 53 m below the surface).  The lateral
period is 1000 m (images of the periodic copies are included up to +-2), the window
0.45 s ends before the bottom reflection returns.  FP64 wavefields."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from oracle import analytic, fd  # noqa: E402
from paper_2309_03600_amd import workloads as W  # noqa: E402

C, F0, T, LX = 1500.0, 15.0, 0.45, 1000.0


def _run(h, kind, M, form, ZS):
    import torch

    import paper_2309_03600_amd as ib
    SRC = (500.0, ZS + 103.0)
    RECS = [(500.0 + dx, ZS + dz) for dx in (0.0, 200.0) for dz in (3.0, 53.0)]
    nx, nz = int(round(LX / h)), int(round(900.0 / h))
    if form == "p2":
        crit = fd.critical_dt(h, C, M, 2)
    else:
        crit = 2 * h / (C * math.sqrt(2) * np.abs(fd.staggered_first_derivative_weights(M)).sum())
    dt = 0.1 * crit
    nt = int(T / dt)
    wl = W.Workload("images", 2, (nx, nz), h, M, kind, W.flat_surface(nx, ZS), np.full((nz, nx), C), dt, nt, F0,
                    np.array([SRC]), np.array(RECS))
    w = ib.ib_build_weights(wl.heights, h, wl.shape, space_order=M, surface=kind, eta=0.5, form=form)
    st = ib.ib_state_create(w, wl.vel, dt, wl.src, wl.rec, precision="f64")
    wav = torch.tensor(analytic.ricker(np.arange(nt) * dt, F0)[None, :], device="cuda")
    tr = st.step(nt, wav, use_graph=True).cpu().numpy()[0]
    tt = (np.arange(nt) + 1) * dt
    if form == "p2":
        s = lambda tau: analytic.ricker(tau, F0)
    else:
        t0 = 1.5 / F0

        def s(tau):
            # the first-order form's pressure answers the time derivative of the source,
            # applied half a step later by the staggered update
            tau = tau - dt / 2 - t0
            a = (math.pi * F0 * tau) ** 2
            return -2 * math.pi ** 2 * F0 ** 2 * tau * (3 - 2 * a) * np.exp(-a)
    errs = []
    for k, r in enumerate(RECS):
        a = analytic.image_trace(SRC, r, ZS, tt, C, s, kind, period=(LX,), nper=2)
        errs.append(np.linalg.norm(tr[:, k] - a) / np.linalg.norm(a))
    return np.array(errs)


# M = 4 as in the paper's convergence study, M = 8 as in its examples; the first-order form
# is built for the free surface.  Expected orders: close to M for the second-order form
# (the paper reports near fourth order at M = 4); for M = 8 the time error of the
# second-order leapfrog (dt = 10 % of critical) limits the finest levels.
# surface depth: 107 m, or 147 m for M = 8 (its supports need more room above the surface)
CASES = [("p2", "free", 4, 107.0), ("p2", "rigid", 4, 107.0), ("pv1", "free", 4, 107.0), ("p2", "free", 8, 147.0)]


@pytest.mark.parametrize("form,kind,M,ZS", CASES)
def test_convergence_against_method_of_images(form, kind, M, ZS):
    levels = (10.0, 5.0, 2.5)
    errs = [_run(h, kind, M, form, ZS) for h in levels]
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(len(levels) - 1)]
    print(f"[convergence {form} {kind} M={M}] h={levels}: max errors "
          f"{['%.3e' % e.max() for e in errs]}, orders (per receiver, per halving) "
          f"{[np.round(o, 2).tolist() for o in orders]}", flush=True)
    assert errs[-1].max() < errs[0].max()
    assert np.median(orders[0]) > (3.5 if M == 4 else 4.0)
    # at M = 8 the second halving meets the leapfrog's second-order time error (dt stays at
    # 10 % of critical, so it shrinks with h): the order drops to about 2 there
    assert np.all(np.concatenate(orders) > (2.0 if M == 4 else 1.5))
