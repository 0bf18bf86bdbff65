"""MI355X-native immersed-boundary acoustic finite differences (arXiv 2309.03600).

Python binding of the C ABI in ``include/ib.h``: every call marshals torch tensors
(device memory) and streams into the HIP library ``libibwave.so``; every step of the
method runs in that library's kernels.  There is no CPU fallback: without the built
library (``paper_2309_03600_amd.build.build()``) every call raises.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import IB_F32, IB_F64, IB_SURF_FREE, IB_SURF_RIGID, IB_SURF_ROBIN, NonFiniteError  # noqa: F401

__all__ = ["IBWeights", "IBState", "Checkpoints", "NonFiniteError", "ib_build_weights", "ib_state_create", "ib_step",
           "modelling", "abi_version"]


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("a HIP device is required")
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def abi_version():
    return _lib.load().ib_abi_version()


class IBWeights:
    """Handle of a built stencil table (library-owned device memory)."""

    def __init__(self, handle, ndim, shape, form="p2", keep_bc_weights=False):
        self._h = handle
        self.ndim = ndim
        self.shape = shape
        self.form = form
        self.keep_bc_weights = keep_bc_weights

    def stats(self):
        st = _lib.ib_stats()
        _lib.check(_lib.load().ib_weights_stats(self._h, C.byref(st)))
        out = {k: getattr(st, k) for k, _ in _lib.ib_stats._fields_}
        out["radius_hist"] = list(st.radius_hist)
        out["order_hist"] = list(st.order_hist)
        return out

    def copy(self, field, dtype, count):
        a = np.zeros(count, dtype=dtype)
        _lib.check(_lib.load().ib_weights_copy(self._h, field, a.ctypes.data_as(C.c_void_p), a.nbytes))
        return a

    def export(self):
        """Host copies of the table: node classes, boundary points, IB nodes, meta, weights."""
        s = self.stats()
        N, nb, nib, sw = s["n_nodes"], s["n_boundary_points"], s["n_ib"], s["sum_nw"]
        if self.form == "pv1":
            return dict(
                node_class=self.copy(_lib.FIELD_NODE_CLASS, np.uint8, N),
                bpoints=self.copy(_lib.FIELD_BPOINTS, np.float64, nb * 7).reshape(nb, 7),
                rows=self.copy(_lib.FIELD_PV_ROWS, np.int64, nib * 3).reshape(nib, 3),
                entries=self.copy(_lib.FIELD_PV_ENTRIES, np.float64, sw * 3).reshape(sw, 3),
                vclass=self.copy(_lib.FIELD_VCLASS, np.uint8, self.ndim * N).reshape(self.ndim, N),
                stats=s,
            )
        out = dict(
            node_class=self.copy(_lib.FIELD_NODE_CLASS, np.uint8, N),
            bpoints=self.copy(_lib.FIELD_BPOINTS, np.float64, nb * 7).reshape(nb, 7),
            ib_nodes=self.copy(_lib.FIELD_IB_NODES, np.int64, nib),
            ib_meta=self.copy(_lib.FIELD_IB_META, np.int32, nib * 4).reshape(nib, 4),
            weights=self.copy(_lib.FIELD_WEIGHTS_F64, np.float64, sw),
            sigma=self.copy(_lib.FIELD_SIGMA, np.float64, nib),
            stats=s,
        )
        if self.keep_bc_weights:
            cnt = self.copy(_lib.FIELD_BC_COUNTS, np.int32, nib)
            out["bc_counts"] = cnt
            out["bc_entries"] = self.copy(_lib.FIELD_BC_ENTRIES, np.float64, int(cnt.sum()) * 3).reshape(-1, 3)
        return out

    def close(self):
        if self._h:
            _lib.load().ib_weights_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ib_build_weights(heights, h, shape, space_order=8, surface="free", eta=0.5, max_radius_steps=3,
                     min_basis_order=None, physical_below=True, rank_rtol=0.0, form="p2", eta_v=0.0, method="nd",
                     keep_bc_weights=False, robin=None, stream=None):
    """Build the IB stencils for a heightfield (torch float64 device tensor or array, metres).

    ``form`` "p2" is the second-order pressure form, "pv1" the first-order pressure-velocity
    form on a staggered grid.  ``method`` "nd" builds the N-D extrapolants of the paper,
    "1d" the per-axis 1D extrapolations of its reduction to 1D (second-order form, free
    surface).  ``keep_bc_weights`` also keeps the weights of the boundary-condition values
    (needed by ``IBState.set_forcing``; second-order form, N-D method).  ``surface`` is
    "free", "rigid" or "robin": p + a dp/dn = 0 with the outward normal and a (metres) given
    by ``robin``, per-column samples shaped like ``heights``.
    """
    if form not in ("p2", "pv1"):
        raise ValueError("form must be 'p2' or 'pv1'")
    if method not in ("nd", "1d"):
        raise ValueError("method must be 'nd' or '1d'")
    torch = _torch()
    ndim = len(shape)
    Ht = torch.as_tensor(np.ascontiguousarray(heights, dtype=np.float64) if not torch.is_tensor(heights) else heights,
                         dtype=torch.float64, device="cuda").contiguous()
    g = _lib.ib_grid()
    g.ndim = ndim
    for i, n in enumerate(shape):
        g.n[i] = int(n)
    g.h = float(h)
    p = _lib.ib_params()
    p.form = _lib.IB_FORM_P2 if form == "p2" else _lib.IB_FORM_PV1
    p.eta_v = float(eta_v)
    p.method = _lib.IB_METHOD_ND if method == "nd" else _lib.IB_METHOD_1D
    if surface not in ("free", "rigid", "robin"):
        raise ValueError("surface must be 'free', 'rigid' or 'robin'")
    p.surface = {"free": IB_SURF_FREE, "rigid": IB_SURF_RIGID, "robin": IB_SURF_ROBIN}[surface]
    Rt = None
    if robin is not None:
        Rt = torch.as_tensor(np.ascontiguousarray(robin, dtype=np.float64) if not torch.is_tensor(robin) else robin,
                             dtype=torch.float64, device="cuda").contiguous()
        assert tuple(Rt.shape) == tuple(Ht.shape)
        p.robin_dev = Rt.data_ptr()
    p.space_order = int(space_order)
    p.max_radius_steps = int(max_radius_steps)
    p.min_basis_order = int(min_basis_order if min_basis_order is not None else max(2, space_order // 2))
    p.physical_below = 1 if physical_below else 0
    p.eta = float(eta)
    p.rank_rtol = float(rank_rtol)
    p.keep_bc_weights = 1 if keep_bc_weights else 0
    out = C.c_void_p()
    _lib.check(_lib.load().ib_build_weights(C.byref(g), C.c_void_p(Ht.data_ptr()), C.byref(p), _stream(stream),
                                            C.byref(out)))
    return IBWeights(out, ndim, tuple(int(v) for v in shape), form, bool(keep_bc_weights))


class Checkpoints:
    """Caller-held time checkpoints of one forward run (ib_checkpoints); freed on close()
    or garbage collection."""

    def __init__(self):
        self._h = None

    def close(self):
        if self._h:
            _torch().cuda.synchronize()
            _lib.load().ib_checkpoints_free(C.c_void_p(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class IBState:
    """Wavefields and acquisition of ``nshots`` shots (library-owned device memory)."""

    def __init__(self, handle, weights, prec, nshots, nrec):
        self._h = handle
        self.weights = weights
        self.prec = prec
        self.nshots = nshots
        self.nrec = nrec

    @property
    def dtype(self):
        torch = _torch()
        return torch.float32 if self.prec == IB_F32 else torch.float64

    def step(self, nsteps, wavelet, traces=None, use_graph=False, stream=None):
        """Advance ``nsteps`` steps; wavelet [nshots][nt] and traces [nshots][nsteps][nrec] tensors."""
        torch = _torch()
        assert wavelet.dtype == self.dtype and wavelet.is_cuda and wavelet.is_contiguous()
        assert wavelet.shape[0] == self.nshots
        if traces is None and self.nrec > 0:
            traces = torch.zeros((self.nshots, nsteps, self.nrec), dtype=self.dtype, device="cuda")
        if traces is not None:
            assert traces.dtype == self.dtype and traces.is_contiguous()
            assert tuple(traces.shape) == (self.nshots, nsteps, self.nrec)
        tp = C.c_void_p(traces.data_ptr()) if traces is not None else C.c_void_p()
        _lib.check(_lib.load().ib_step(self._h, int(nsteps), C.c_void_p(wavelet.data_ptr()), int(wavelet.shape[1]),
                                       tp, 1 if use_graph else 0, _stream(stream)))
        return traces

    def field(self, which=0, shot=0, value=None, stream=None):
        """Get (value None) or set p^n (which=0) / p^{n-1} (which=1) of one shot.

        First-order form: which=0 is p^n and which=2+k the velocity v_k^{n-1/2}."""
        torch = _torch()
        shape = tuple(reversed(self.weights.shape))
        if value is None:
            out = torch.empty(shape, dtype=self.dtype, device="cuda")
            _lib.check(_lib.load().ib_state_field(self._h, which, shot, C.c_void_p(out.data_ptr()), 0,
                                                  _stream(stream)))
            return out
        v = value.to(device="cuda", dtype=self.dtype).contiguous()
        assert tuple(v.shape) == shape
        _lib.check(_lib.load().ib_state_field(self._h, which, shot, C.c_void_p(v.data_ptr()), 1, _stream(stream)))
        torch.cuda.current_stream().synchronize()
        return None

    def forward(self, nt, wavelet, ckpt_every=50, traces=None, stream=None):
        """Restart from rest and run ``nt`` steps keeping checkpoints for ``adjoint``."""
        torch = _torch()
        assert wavelet.dtype == self.dtype and wavelet.is_cuda and wavelet.is_contiguous()
        if traces is None:
            traces = torch.zeros((self.nshots, nt, self.nrec), dtype=self.dtype, device="cuda")
        tp = C.c_void_p(traces.data_ptr()) if self.nrec > 0 else C.c_void_p()
        _lib.check(_lib.load().ib_forward(self._h, int(nt), C.c_void_p(wavelet.data_ptr()), int(wavelet.shape[1]),
                                          tp, int(ckpt_every), _stream(stream)))
        return traces

    def forward_ckpt(self, nt, wavelet, ckpt_every=50, traces=None, checkpoints=None, stream=None):
        """``forward`` into a caller-held ``Checkpoints`` object (ib_forward_ckpt); returns
        (traces, checkpoints).  Passing an earlier object reuses its memory."""
        torch = _torch()
        assert wavelet.dtype == self.dtype and wavelet.is_cuda and wavelet.is_contiguous()
        if traces is None:
            traces = torch.zeros((self.nshots, nt, self.nrec), dtype=self.dtype, device="cuda")
        if checkpoints is None:
            checkpoints = Checkpoints()
        h = C.c_void_p(checkpoints._h)
        tp = C.c_void_p(traces.data_ptr()) if self.nrec > 0 else C.c_void_p()
        _lib.check(_lib.load().ib_forward_ckpt(self._h, int(nt), C.c_void_p(wavelet.data_ptr()), int(wavelet.shape[1]),
                                               tp, int(ckpt_every), C.byref(h), _stream(stream)))
        checkpoints._h = h.value
        return traces, checkpoints

    def adjoint(self, residual, wavelet, stream=None, grad=None, noalloc=False, checkpoints=None):
        """dJ/dc (float64 grid tensor) for residual = dJ/dtraces of the last ``forward`` (or
        of the ``forward_ckpt`` run that wrote ``checkpoints``).  ``noalloc`` calls
        ib_adjoint_noalloc (the library allocates nothing and does not wait for the stream);
        ``grad`` may be a preallocated float64 grid tensor to overwrite."""
        torch = _torch()
        res = residual.to(device="cuda", dtype=self.dtype).contiguous()
        shape = tuple(reversed(self.weights.shape))
        if grad is None:
            grad = torch.zeros(shape, dtype=torch.float64, device="cuda")
        assert grad.dtype == torch.float64 and grad.is_cuda and grad.is_contiguous() and tuple(grad.shape) == shape
        args = (C.c_void_p(res.data_ptr()), C.c_void_p(wavelet.data_ptr()), int(wavelet.shape[1]),
                C.c_void_p(grad.data_ptr()), _stream(stream))
        lib = _lib.load()
        if checkpoints is not None:
            assert not noalloc
            _lib.check(lib.ib_adjoint_ckpt(self._h, C.c_void_p(checkpoints._h), *args))
        else:
            _lib.check((lib.ib_adjoint_noalloc if noalloc else lib.ib_adjoint)(self._h, *args))
        return grad

    def set_watchdog(self, every=100, limit=1e30, stream=None):
        """Scan p^n after every ``every`` steps (0: off) for NaN/Inf or |p| > limit; clears a
        tripped watchdog."""
        _lib.check(_lib.load().ib_state_set_watchdog(self._h, int(every), float(limit), _stream(stream)))

    def status(self, wait=True):
        """Raises NonFiniteError if a watchdog scan has tripped (``wait``: for the last scan)."""
        _lib.check(_lib.load().ib_state_status(self._h, 1 if wait else 0))

    def set_forcing(self, g, s, stream=None):
        """Non-zero boundary values g_q(x_b) s_q(t): g [n_boundary_points][nq] (float64, physical
        units, boundary points in the table's order), s [nq][len] host array of time functions;
        ``g=None`` restores homogeneous conditions."""
        torch = _torch()
        if g is None:
            _lib.check(_lib.load().ib_state_set_forcing(self._h, C.c_void_p(), 0, C.c_void_p(), 0, _stream(stream)))
            return
        gt = torch.as_tensor(np.ascontiguousarray(g, dtype=np.float64) if not torch.is_tensor(g) else g,
                             dtype=torch.float64, device="cuda").contiguous()
        sh = np.ascontiguousarray(np.atleast_2d(s), dtype=np.float64)
        assert gt.dim() == 2 and sh.shape[0] == gt.shape[1]
        _lib.check(_lib.load().ib_state_set_forcing(self._h, C.c_void_p(gt.data_ptr()), int(gt.shape[1]),
                                                    sh.ctypes.data_as(C.c_void_p), int(sh.shape[1]),
                                                    _stream(stream)))

    def run_kernel(self, which, count, stream=None):
        """Enqueue ``count`` launches of one step kernel (0 interior, 1 patch) for timing."""
        _lib.check(_lib.load().ib_state_run_kernel(self._h, int(which), int(count), _stream(stream)))

    def set_tuning(self, variant, zchunk, patch_variant=-1):
        """Interior-kernel variant (0-4), depth planes per workgroup (0: the tuned value) and
        IB-patch variant (-1: keep)."""
        _lib.check(_lib.load().ib_state_set_tuning(self._h, int(variant), int(zchunk), int(patch_variant)))

    @property
    def step_count(self):
        return _lib.load().ib_state_step_count(self._h)

    def close(self):
        if self._h:
            _lib.load().ib_state_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ib_state_create(weights, vel, dt, src_pos, rec_pos, damp_width=0, damp_R=1e-3, precision="f32",
                    stream=None):
    torch = _torch()
    vel_t = torch.as_tensor(np.ascontiguousarray(vel, dtype=np.float64) if not torch.is_tensor(vel) else vel,
                            dtype=torch.float64, device="cuda").contiguous()
    src = np.ascontiguousarray(np.atleast_2d(src_pos), dtype=np.float64)
    rec = np.ascontiguousarray(np.asarray(rec_pos, dtype=np.float64).reshape(-1, weights.ndim))
    prec = IB_F32 if precision in ("f32", "float32") else IB_F64
    out = C.c_void_p()
    _lib.check(_lib.load().ib_state_create(weights._h, C.c_void_p(vel_t.data_ptr()), float(dt), int(damp_width),
                                           float(damp_R), prec, int(src.shape[0]), src.ctypes.data_as(C.c_void_p),
                                           int(rec.shape[0]), rec.ctypes.data_as(C.c_void_p), _stream(stream),
                                           C.byref(out)))
    torch.cuda.current_stream().synchronize()
    return IBState(out, weights, prec, int(src.shape[0]), int(rec.shape[0]))


def ib_step(state, nsteps, wavelet, traces=None, use_graph=False, stream=None):
    return state.step(nsteps, wavelet, traces, use_graph, stream)


def _autograd():
    import torch

    class IBModelling(torch.autograd.Function):
        """traces = F(velocity); backward = the library's discrete adjoint (ib_adjoint)."""

        @staticmethod
        def forward(ctx, vel, weights, wavelet, src, rec, dt, nt, damp_width, precision, ckpt_every):
            st = ib_state_create(weights, vel.detach().to(torch.float64), dt, src, rec, damp_width=damp_width,
                                 precision=precision)
            wav = wavelet.to(device="cuda", dtype=st.dtype).contiguous()
            tr = st.forward(nt, wav, ckpt_every=ckpt_every)
            ctx.st = st
            ctx.wav = wav
            ctx.vdtype = vel.dtype
            return tr

        @staticmethod
        def backward(ctx, grad_traces):
            g = ctx.st.adjoint(grad_traces, ctx.wav)
            ctx.st.close()
            return g.to(ctx.vdtype), None, None, None, None, None, None, None, None, None

    return IBModelling


def modelling(vel, weights, wavelet, src, rec, dt, nt, damp_width=0, precision="f32", ckpt_every=50):
    """Differentiable forward modelling: traces [nshots][nt][nrec] as a function of the
    velocity tensor (torch.autograd), gradients from the hand-written adjoint."""
    return _autograd().apply(vel, weights, wavelet, src, rec, dt, nt, damp_width, precision, ckpt_every)
