"""Seeded synthetic inputs (topographies, velocity models, wavelets, acquisition).

Serves both the HIP path and the oracle in tests and benchmarks; holds none of the
method's arithmetic.  The paper's own workloads (a Mount St Helens elevation model and
the exact-solution setup of its convergence tests) are not available, so these
synthetic surfaces stand in for them: a flat off-grid surface, a Gaussian hill and
periodic fractal topography.  Seeds: numpy.random.default_rng([2309, config, purpose]).

All lengths in metres, depth positive downward; heightfields are indexed [y][x]
(3D) or [x] (2D); velocity arrays [z][y][x] or [z][x].
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def rng(cfg: int, purpose: int):
    return np.random.default_rng([2309, cfg, purpose])


def ricker(nt: int, dt: float, f0: float, t0: float | None = None):
    """Ricker source time function sampled at t_n = n dt (n = 0..nt-1)."""
    if t0 is None:
        t0 = 1.5 / f0
    t = np.arange(nt) * dt - t0
    a = (math.pi * f0 * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def flat_surface(nlat, depth):
    return np.full(nlat, float(depth))


def gaussian_hill(nx, h, z_base, height, sigma, xc=None):
    x = np.arange(nx) * h
    if xc is None:
        xc = 0.5 * (nx - 1) * h
    return z_base - height * np.exp(-((x - xc) ** 2) / (2.0 * sigma ** 2))


def fractal_surface(nx, ny, h, relief, z_top, seed_rng, exponent=-2.0, kc_cells=8.0):
    """Periodic random surface: 2D power spectrum ~ |k|^exponent, zero beyond
    k_c = 2 pi / (kc_cells h), random phases, scaled to ``relief`` peak to peak and
    placed with its shallowest point at depth z_top."""
    kx = np.fft.fftfreq(nx, d=h) * 2 * math.pi
    ky = np.fft.fftfreq(ny, d=h) * 2 * math.pi
    KX, KY = np.meshgrid(kx, ky, indexing="xy")
    k = np.sqrt(KX ** 2 + KY ** 2)
    kc = 2 * math.pi / (kc_cells * h)
    amp = np.zeros_like(k)
    live = (k > 0) & (k <= kc)
    amp[live] = k[live] ** (exponent / 2.0)
    phase = np.exp(2j * math.pi * seed_rng.random(k.shape))
    surf = np.real(np.fft.ifft2(amp * phase))
    surf -= surf.min()
    surf *= relief / surf.max()
    return z_top + surf


def smooth_noise(shape, corr_cells, seed_rng):
    """Periodic white noise filtered by a Gaussian of ``corr_cells`` cells, scaled so
    that max |xi| = 1 (float32 FFTs keep the 3D case light)."""
    x = seed_rng.standard_normal(shape).astype(np.float32)
    F = np.fft.rfftn(x)
    ks = [np.fft.fftfreq(n) for n in shape[:-1]] + [np.fft.rfftfreq(shape[-1])]
    g = np.ones(F.shape, dtype=np.float32)
    for ax, kk in enumerate(ks):
        sh = [1] * len(shape)
        sh[ax] = len(kk)
        g = g * np.exp(-0.5 * (2 * math.pi * kk * corr_cells) ** 2).reshape(sh).astype(np.float32)
    y = np.fft.irfftn(F * g, s=shape, axes=tuple(range(len(shape)))).astype(np.float32)
    return y / np.abs(y).max()


def gradient_velocity(shape_zyx, h, v_top, v_bottom, pert, corr_cells, seed_rng):
    """v = v_top + (v_bottom - v_top) z / z_max times (1 + pert * xi)."""
    nz = shape_zyx[0]
    z = np.arange(nz) * h
    base = v_top + (v_bottom - v_top) * z / z[-1]
    base = base.reshape((nz,) + (1,) * (len(shape_zyx) - 1))
    if pert == 0.0:
        return np.broadcast_to(base, shape_zyx).astype(np.float64).copy()
    xi = smooth_noise(shape_zyx, corr_cells, seed_rng)
    return (base * (1.0 + pert * xi)).astype(np.float64)


@dataclass
class Workload:
    name: str
    ndim: int
    shape: tuple            # (nx, [ny,] nz)
    h: float
    M: int
    surface: str            # 'free' | 'rigid'
    heights: np.ndarray
    vel: np.ndarray         # [z][y][x]
    dt: float
    nt: int
    f0: float
    src: np.ndarray         # (nshots, ndim) metres
    rec: np.ndarray         # (nrec, ndim) metres
    damp_width: int = 0
    damp_R: float = 1e-3
    eta: float = 0.5
    extra: dict = field(default_factory=dict)

    def wavelets(self, dtype=np.float64):
        w = ricker(self.nt, self.dt, self.f0)
        return np.tile(w, (self.src.shape[0], 1)).astype(dtype)


def config1(nt=600):
    """2D, 201x201, 10 m, v = 1500 m/s, M = 4, flat free surface 0.3 dx above node row
    40, Ricker 15 Hz 100 m below it, dt = 0.5 dt_crit, 101 receivers 3 m below the
    surface (the first wet node row)."""
    nx = nz = 201
    h = 10.0
    zs = 397.0
    vel = np.full((nz, nx), 1500.0)
    dt = 2.0412414523193153e-3      # 0.5 * 2 h / (c sqrt(2 * 16/3))
    src = np.array([[100 * h, 50 * h]])
    rec = np.array([[x * h, 40 * h] for x in range(50, 151)], dtype=float)
    return Workload("config1-2d-m4-flat-free", 2, (nx, nz), h, 4, "free", flat_surface(nx, zs),
                    vel, dt, nt, 15.0, src, rec, extra=dict(z_surface=zs))


def config2(surface="free", nt=2000):
    """2D, 801x401, 5 m, M = 8: Gaussian hill (150 m high, sigma 400 m) on a base at
    120 dx; v from 1500 to 3500 m/s with depth times (1 + 0.05 xi); Ricker 15 Hz 100 m
    below the surface at x_c - 600 m; 161 receivers (every 5th column) 1.5 dx below the
    surface; 40-cell damping; dt = 0.5 dt_crit for c_max = 3675 m/s."""
    nx, nz, h = 801, 401, 5.0
    H = gaussian_hill(nx, h, 120 * h, 150.0, 400.0)
    vel = gradient_velocity((nz, nx), h, 1500.0, 3500.0, 0.05, 10.0, rng(2, 1))
    # 0.5 x the staggered-form limit 2 h / (c sqrt(2) sum|w|), sum|w| = 2.572619... for the
    # eighth-order staggered first derivative (the stricter of the two forms)
    dt = 0.5 * 2 * h / (3675.0 * math.sqrt(2) * 2.572619047619048)
    xc = 0.5 * (nx - 1) * h
    xs = xc - 600.0
    zs_src = float(np.interp(xs, np.arange(nx) * h, H)) + 100.0
    rec = []
    for i in range(0, nx, 5):
        rec.append([i * h, H[i] + 1.5 * h])
    return Workload(f"config2-2d-m8-hill-{surface}", 2, (nx, nz), h, 8, surface, H, vel, dt, nt, 15.0,
                    np.array([[xs, zs_src]]), np.array(rec), damp_width=40)


def _fractal3d(nx, ny, nz, h, cfg, relief=300.0, z_top_cells=20):
    return fractal_surface(nx, ny, h, relief, z_top_cells * h, rng(cfg, 0))


def _rec_on_surface(H, h, stride, depth_below, nx, ny, count=None):
    rec = []
    for j in range(0, ny, stride):
        for i in range(0, nx, stride):
            rec.append([i * h, j * h, H[j, i] + depth_below])
    return np.array(rec)


def config3(nt=3000, lateral=401, depth=301, with_velocity=True):
    """3D, 401x401x301, 10 m, M = 8, fractal free surface (spectral exponent -2, 300 m
    relief between 20 dx and 50 dx deep), v 1500 -> 3500 m/s with depth x (1 + 0.05 xi),
    40-cell damping, Ricker 10 Hz at the centre column 100 m below the surface,
    201x201 receivers at columns (2i, 2j) 15 m below the surface, dt = 0.616 ms, exclusion
    cutoff eta = 1.0.

    The cutoff is chosen empirically, as the paper chooses its own: with eta = 0.5 (and
    0.4, 0.25, 0.6, 0.75) a mode localized at one spot of this surface grows, in FP64 as in
    FP32; with eta = 1.0 the field decays over 6000 steps."""
    nx = ny = lateral
    nz = depth
    h = 10.0
    H = _fractal3d(nx, ny, nz, h, 3)
    if with_velocity:
        vel = gradient_velocity((nz, ny, nx), h, 1500.0, 3500.0, 0.05, 10.0, rng(3, 1))
    else:
        vel = None
    cx, cy = nx // 2, ny // 2
    src = np.array([[cx * h, cy * h, H[cy, cx] + 100.0]])
    rec = _rec_on_surface(H, h, 2, 15.0, nx, ny)
    dt = 0.616e-3
    return Workload(f"config3-3d-m8-fractal-free-{nx}x{ny}x{nz}", 3, (nx, ny, nz), h, 8, "free", H, vel,
                    dt, nt, 10.0, src, rec, damp_width=40, eta=1.0)


def config4(nt=2000, nshots=64, lateral=301, depth=201):
    """3D, 301x301x201, 10 m, M = 8, its own fractal free surface, 64 sources at seeded
    (x, y) outside the damping layer 50 m below the surface, 151x151 receivers."""
    nx = ny = lateral
    nz = depth
    h = 10.0
    H = _fractal3d(nx, ny, nz, h, 4)
    vel = gradient_velocity((nz, ny, nx), h, 1500.0, 3500.0, 0.05, 10.0, rng(4, 1))
    r = rng(4, 2)
    xy = r.uniform(45 * h, (nx - 46) * h, size=(nshots, 2))
    src = []
    for x, y in xy:
        i, j = int(round(x / h)), int(round(y / h))
        src.append([x, y, H[j % ny, i % nx] + 50.0 + 10.0])
    rec = _rec_on_surface(H, h, 2, 15.0, nx, ny)
    return Workload(f"config4-3d-m8-batched-{nshots}shots", 3, (nx, ny, nz), h, 8, "free", H, vel,
                    0.616e-3, nt, 10.0, np.array(src), rec, damp_width=40)


def config5(nt=1500, nshots=16, n=256, damp_width=20):
    """3D, 256^3, 10 m, M = 8, rigid fractal surface (physical side below it), velocity a
    linear depth gradient v0 = 1500 -> 3500 m/s; the observed data come from
    v_true = v0 (1 + 0.03 G), G a Gaussian blob (sigma 10 dx, peak 1) centred 90 dx deep;
    16 sources in a 4x4 pattern 50 m below the surface, 64x64 receivers (every 4th column)
    15 m below the surface, dt = 0.616 ms, 20-cell damping, exclusion cutoff eta = 0.25.

    The cutoff is chosen empirically, as the paper chooses its own.  With eta = 0.5 this
    rigid surface has a growing mode at one spot under a steep slope: the modified
    operator there has a complex eigenvalue whose leapfrog amplification is 1.019 per
    step.  With eta <= 0.4, 6000 steps show no growth."""
    nx = ny = nz = n
    h = 10.0
    H = _fractal3d(nx, ny, nz, h, 5)
    vel = gradient_velocity((nz, ny, nx), h, 1500.0, 3500.0, 0.0, 10.0, rng(5, 1))
    idx = np.indices((nz, ny, nx)).astype(np.float64)
    cz, cy, cx = 90.0, ny / 2.0, nx / 2.0
    G = np.exp(-((idx[0] - cz) ** 2 + (idx[1] - cy) ** 2 + (idx[2] - cx) ** 2) / (2 * 10.0 ** 2))
    v_true = vel * (1.0 + 0.03 * G)
    k = 4
    lo, hi = damp_width + 8, n - damp_width - 9
    pos = np.linspace(lo, hi, k)
    src = []
    for j in range(k):
        for i in range(k):
            xi, yj = int(round(pos[i])), int(round(pos[j]))
            src.append([xi * h, yj * h, H[yj, xi] + 50.0])
    src = np.array(src[:nshots])
    rec = _rec_on_surface(H, h, max(1, n // 64), 15.0, nx, ny)
    return Workload(f"config5-3d-m8-rigid-adjoint-{n}^3-{nshots}shots", 3, (nx, ny, nz), h, 8, "rigid", H, vel,
                    0.616e-3, nt, 10.0, src, rec, damp_width=damp_width, extra=dict(v_true=v_true), eta=0.25)


def small3d(cfg=90, n=24, nz=44, relief=50.0, surface="free", nt=100, h=10.0, nshots=1, z_top_cells=16):
    """Small 3D fractal case for parity tests (same recipe, scaled down)."""
    H = fractal_surface(n, n, h, relief, z_top_cells * h, rng(cfg, 0))
    vel = gradient_velocity((nz, n, n), h, 1500.0, 3500.0, 0.05, 4.0, rng(cfg, 1))
    r = rng(cfg, 2)
    src = []
    for s in range(nshots):
        i, j = r.integers(n // 4, 3 * n // 4, size=2)
        src.append([i * h + 3.0, j * h + 4.0, H[j, i] + 60.0])
    rec = _rec_on_surface(H, h, 3, 15.0, n, n)
    return Workload(f"small3d-{n}x{n}x{nz}-{surface}", 3, (n, n, nz), h, 8, surface, H, vel,
                    0.616e-3, nt, 15.0, np.array(src), rec, damp_width=8)


def small2d(cfg=91, nx=120, nz=80, M=8, surface="free", nt=200, h=5.0, hill=60.0):
    """Small 2D Gaussian-hill case for parity tests."""
    H = gaussian_hill(nx, h, 36 * h, hill, 80.0)
    vel = gradient_velocity((nz, nx), h, 1500.0, 3500.0, 0.05, 4.0, rng(cfg, 1))
    dt = 0.5 * 2 * h / (3675.0 * math.sqrt(2 * 6.501587301587301))
    xs = 0.3 * nx * h
    src = np.array([[xs + 1.0, float(np.interp(xs, np.arange(nx) * h, H)) + 60.0]])
    rec = np.array([[i * h, H[i] + 1.5 * h] for i in range(0, nx, 3)])
    return Workload(f"small2d-{nx}x{nz}-m{M}-{surface}", 2, (nx, nz), h, M, surface, H, vel, dt, nt, 20.0,
                    src, rec, damp_width=10)
