"""Python binding of libq2d (the C ABI in include/q2d.h).

Quasi-2D long-range electrostatics on an AMD MI355X: the SOE Ewald2D sum
(arXiv:2403.01521, Sec. 3) and its random-batch form (Sec. 4).  This module
only marshals arguments: every step of the computation runs in the HIP
kernels of libq2d.so.  PyTorch supplies device memory and the stream.

    import paper_2403_01521_amd as q2d
    w, s, err = q2d.soe_fit(16)
    plan = q2d.Plan(box=(600, 600, 10), alpha=0.1, w=w, s=s, precision="fp32",
                    n_max=10**6, p_max=100)
    phi, F, E, modes = plan.rbm_step(pos, q, P=100, seed=1, step=0)

There is no CPU fallback: importing works without a GPU (for symbol checks),
but every compute call needs the built library and a HIP device.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libq2d.so")

STATUS = {
    0: "Q2D_OK", 1: "Q2D_EINVAL", 2: "Q2D_ENONNEUTRAL", 3: "Q2D_EOUTOFBOX", 4: "Q2D_ENOMEM",
    5: "Q2D_ECAPACITY", 6: "Q2D_EDEVICE", 7: "Q2D_ESAMPLER", 8: "Q2D_EUNSUPPORTED",
    9: "Q2D_EDTYPE",
}
Q2D_EINVAL, Q2D_ENONNEUTRAL, Q2D_EOUTOFBOX, Q2D_ECAPACITY, Q2D_EUNSUPPORTED, Q2D_EDTYPE = (
    1, 2, 3, 5, 8, 9)
SAMPLERS = {"metropolis": 0, "iid": 1}
FP64, FP32 = 0, 1
TIMER_SWEEP, TIMER_AGG, TIMER_SORT, TIMER_K0, TIMER_CALL = 0, 1, 2, 3, 4
TIMING_ALL = 31

EXPORTS = ("q2d_plan_create", "q2d_plan_destroy", "q2d_plan_set_stream", "q2d_plan_info",
           "q2d_long_range", "q2d_rbm_step", "q2d_rbm_step_noalloc", "q2d_long_range_vjp",
           "q2d_rbm_step_vjp",
           "q2d_modes_eval", "q2d_short_range", "q2d_batch_create", "q2d_batch_destroy",
           "q2d_batch_set_stream", "q2d_batch_set_segment", "q2d_batch_set_config",
           "q2d_batch_get_config", "q2d_batch_info",
           "q2d_batch_rbm_step", "q2d_batch_tune", "q2d_batch_capture", "q2d_batch_replay",
           "q2d_batch_check",
           "q2d_plan_check",
           "q2d_slab", "q2d_langevin_step",
           "q2d_soe_fit", "q2d_soe_fit_reduced", "q2d_soe_fit_eps",
           "q2d_plan_timing_enable", "q2d_plan_timing_read",
           "q2d_plan_timing_stride",
           "q2d_status_string")


class Q2DError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__("%s failed: %s (%s)" % (where, STATUS.get(code, code), _status_str(code)))


class _Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("thin", ctypes.c_int32),
                ("n_max", ctypes.c_int64), ("p_max", ctypes.c_int32),
                ("validate", ctypes.c_int32), ("sampler", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("n_modes_exact", ctypes.c_int64), ("M", ctypes.c_int32), ("H", ctypes.c_double),
                ("diag_exact", ctypes.c_double), ("diag_rb", ctypes.c_double),
                ("soe_k0_self", ctypes.c_double)]


_lib = None


def load_library(path=None):
    """Load libq2d.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError("libq2d.so not built: run __graft_entry__.build() or "
                           "python -m paper_2403_01521_amd.build")
    lib = ctypes.CDLL(path)
    vp, i32, i64, u64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    dp = ctypes.POINTER(ctypes.c_double)
    lib.q2d_plan_create.argtypes = [dbl, dbl, dbl, dbl, dbl, dbl, i32, dp, dp,
                                    ctypes.POINTER(_Opts), vp, ctypes.POINTER(vp)]
    lib.q2d_plan_destroy.argtypes = [vp]
    lib.q2d_plan_set_stream.argtypes = [vp, vp]
    lib.q2d_plan_info.argtypes = [vp, ctypes.POINTER(_Info)]
    lib.q2d_long_range.argtypes = [vp, vp, vp, i64, vp, vp, vp]
    lib.q2d_rbm_step.argtypes = [vp, vp, vp, i64, i32, u64, u64, vp, vp, vp, vp]
    lib.q2d_rbm_step_noalloc.argtypes = [vp, vp, vp, i64, i32, u64, u64, vp, vp, vp, vp]
    lib.q2d_long_range_vjp.argtypes = [vp, vp, vp, vp, i64, vp, vp]
    lib.q2d_rbm_step_vjp.argtypes = [vp, vp, vp, vp, i64, i32, u64, u64, vp, vp]
    lib.q2d_modes_eval.argtypes = [vp, vp, vp, i64, vp, vp, i64, vp, vp, vp]
    lib.q2d_short_range.argtypes = [vp, vp, vp, i64, vp, vp, vp]
    lib.q2d_plan_check.argtypes = [vp]
    lib.q2d_slab.argtypes = [vp, vp, vp, i64, i32, vp, vp, vp, dbl, dbl, vp, vp, vp]
    lib.q2d_langevin_step.argtypes = [vp, vp, vp, vp, i64, vp, vp, vp, dbl, dbl, dbl, u64, u64,
                                      i32]
    lib.q2d_soe_fit.argtypes = [i32, dp, dp, dp]
    lib.q2d_soe_fit_reduced.argtypes = [i32, dp, dp, dp]
    lib.q2d_soe_fit_eps.argtypes = [dbl, i32, ctypes.POINTER(ctypes.c_int32), dp, dp, dp]
    lib.q2d_plan_timing_enable.argtypes = [vp, i32]
    lib.q2d_plan_timing_read.argtypes = [vp, i32, dp, ctypes.POINTER(ctypes.c_int64)]
    lib.q2d_plan_timing_stride.argtypes = [vp, i32]
    i64p = ctypes.POINTER(ctypes.c_int64)
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.q2d_batch_create.argtypes = [i32, dp, i64p, dbl, i32, dp, dp, ctypes.POINTER(_Opts), vp,
                                     ctypes.POINTER(vp)]
    lib.q2d_batch_destroy.argtypes = [vp]
    lib.q2d_batch_set_stream.argtypes = [vp, vp]
    lib.q2d_batch_set_segment.argtypes = [vp, i32]
    lib.q2d_batch_set_config.argtypes = [vp, i32, i32, i32]
    lib.q2d_batch_get_config.argtypes = [vp, i32p, i32p, i32p]
    lib.q2d_batch_info.argtypes = [vp, i32p, i64p, dp, dp]
    lib.q2d_batch_rbm_step.argtypes = [vp, vp, vp, i32, u64, u64, vp, vp, vp, vp]
    lib.q2d_batch_tune.argtypes = [vp, vp, vp, i32, u64, vp, vp, vp, i32p]
    lib.q2d_batch_capture.argtypes = [vp, vp, vp, i32, u64, u64, vp, vp, vp]
    lib.q2d_batch_replay.argtypes = [vp, i32]
    lib.q2d_batch_check.argtypes = [vp]
    lib.q2d_status_string.argtypes = [ctypes.c_int]
    lib.q2d_status_string.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name != "q2d_status_string":
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _status_str(code):
    try:
        return load_library().q2d_status_string(int(code)).decode()
    except Exception:  # noqa: BLE001 - diagnostic only
        return "?"


def _check(code, where):
    if code != 0:
        raise Q2DError(code, where)


def soe_fit(M):
    """Host SOE of exp(-x^2) with M terms: (w, s, sup_err), complex numpy arrays."""
    lib = load_library()
    w = np.zeros(2 * M)
    s = np.zeros(2 * M)
    err = ctypes.c_double(0.0)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(lib.q2d_soe_fit(M, w.ctypes.data_as(dp), s.ctypes.data_as(dp), ctypes.byref(err)),
           "q2d_soe_fit")
    return w[0::2] + 1j * w[1::2], s[0::2] + 1j * s[1::2], err.value


def soe_fit_reduced(M):
    """Host model-reduced SOE of exp(-x^2) with M terms (balanced truncation of
    a 48-term Talbot table, then a minimax polish): (w, s, sup_err)."""
    lib = load_library()
    w = np.zeros(2 * M)
    s = np.zeros(2 * M)
    err = ctypes.c_double(0.0)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(lib.q2d_soe_fit_reduced(M, w.ctypes.data_as(dp), s.ctypes.data_as(dp),
                                   ctypes.byref(err)), "q2d_soe_fit_reduced")
    return w[0::2] + 1j * w[1::2], s[0::2] + 1j * s[1::2], err.value


def soe_fit_eps(eps, M_max=64):
    """Fewest-term host SOE with sup error <= eps: (w, s, M, sup_err); raises
    Q2DError(Q2D_ECAPACITY) if M_max terms do not reach eps."""
    lib = load_library()
    w = np.zeros(2 * M_max)
    s = np.zeros(2 * M_max)
    M = ctypes.c_int32(0)
    err = ctypes.c_double(0.0)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(lib.q2d_soe_fit_eps(float(eps), int(M_max), ctypes.byref(M), w.ctypes.data_as(dp),
                               s.ctypes.data_as(dp), ctypes.byref(err)), "q2d_soe_fit_eps")
    m = M.value
    return w[0:2 * m:2] + 1j * w[1:2 * m:2], s[0:2 * m:2] + 1j * s[1:2 * m:2], m, err.value


def _interleave(z):
    z = np.asarray(z, dtype=np.complex128)
    out = np.empty(2 * len(z))
    out[0::2] = z.real
    out[1::2] = z.imag
    return out


class Plan:
    """A solver for one box, Ewald parameter and SOE table (q2d_plan_create)."""

    def __init__(self, box, alpha, w, s, *, rc=0.0, kc=0.0, precision="fp64", n_max,
                 p_max=0, thin=1, validate=False, sampler="metropolis", stream=None):
        import torch
        self._torch = torch
        lib = load_library()
        self.box = tuple(float(v) for v in box)
        self.alpha = float(alpha)
        self.precision = precision
        self.dtype = torch.float32 if precision == "fp32" else torch.float64
        w = _interleave(w)
        s = _interleave(s)
        opts = _Opts(FP32 if precision == "fp32" else FP64, int(thin), int(n_max), int(p_max),
                     1 if validate else 0, SAMPLERS[sampler])
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self._stream = stream
        h = ctypes.c_void_p()
        dp = ctypes.POINTER(ctypes.c_double)
        _check(lib.q2d_plan_create(self.box[0], self.box[1], self.box[2], self.alpha, float(rc),
                                   float(kc), len(w) // 2, w.ctypes.data_as(dp),
                                   s.ctypes.data_as(dp), ctypes.byref(opts),
                                   ctypes.c_void_p(stream), ctypes.byref(h)), "q2d_plan_create")
        self._h = h
        self._lib = lib

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.q2d_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    def info(self):
        inf = _Info()
        _check(self._lib.q2d_plan_info(self._h, ctypes.byref(inf)), "q2d_plan_info")
        return dict(n_modes_exact=inf.n_modes_exact, M=inf.M, H=inf.H, diag_exact=inf.diag_exact,
                    diag_rb=inf.diag_rb, soe_k0_self=inf.soe_k0_self)

    def _sync_stream(self):
        s = self._torch.cuda.current_stream().cuda_stream
        if s != self._stream:
            _check(self._lib.q2d_plan_set_stream(self._h, ctypes.c_void_p(s)), "q2d_plan_set_stream")
            self._stream = s

    def _prep(self, pos, q):
        t = self._torch
        if not (pos.is_cuda and q.is_cuda):
            raise ValueError("pos and q must be device tensors")
        if pos.dtype != self.dtype or q.dtype != self.dtype:
            raise Q2DError(Q2D_EDTYPE, "dtype %s/%s for a %s plan" % (pos.dtype, q.dtype,
                                                                       self.dtype))
        pos = pos.contiguous()
        q = q.contiguous()
        if pos.dim() != 2 or pos.shape[1] != 3 or q.shape != (pos.shape[0],):
            raise ValueError("pos must be (N, 3) and q (N,)")
        n = pos.shape[0]
        phi = t.empty(n, dtype=self.dtype, device=pos.device)
        F = t.empty((n, 3), dtype=self.dtype, device=pos.device)
        E = t.empty(1, dtype=t.float64, device=pos.device)
        return pos, q, n, phi, F, E

    def long_range(self, pos, q):
        """Exact-k SOE long-range sum: (phi, F, E) device tensors."""
        self._sync_stream()
        pos, q, n, phi, F, E = self._prep(pos, q)
        _check(self._lib.q2d_long_range(self._h, pos.data_ptr(), q.data_ptr(), n,
                                        phi.data_ptr(), F.data_ptr(), E.data_ptr()),
               "q2d_long_range")
        return phi, F, E

    def rbm_step(self, pos, q, P, seed, step):
        """Random-batch step: (phi, F, E, modes[P, 2] int32) device tensors."""
        self._sync_stream()
        pos, q, n, phi, F, E = self._prep(pos, q)
        modes = self._torch.empty((P, 2), dtype=self._torch.int32, device=pos.device)
        _check(self._lib.q2d_rbm_step(self._h, pos.data_ptr(), q.data_ptr(), n, int(P),
                                      ctypes.c_uint64(seed), ctypes.c_uint64(step),
                                      phi.data_ptr(), F.data_ptr(), E.data_ptr(),
                                      modes.data_ptr()), "q2d_rbm_step")
        return phi, F, E, modes

    def rbm_step_noalloc(self, pos, q, P, seed, step, out=None):
        """The random-batch step through q2d_rbm_step_noalloc, whose scratch is the
        library's static per-device array (the C call allocates no device memory).
        out: optional preallocated (phi, F, E, modes) device tensors of the shapes
        rbm_step returns; they are written and returned."""
        self._sync_stream()
        t = self._torch
        if out is None:
            pos, q, n, phi, F, E = self._prep(pos, q)
            modes = t.empty((P, 2), dtype=t.int32, device=pos.device)
        else:
            if not (pos.is_cuda and q.is_cuda):
                raise ValueError("pos and q must be device tensors")
            if pos.dtype != self.dtype or q.dtype != self.dtype:
                raise Q2DError(Q2D_EDTYPE, "dtype %s/%s for a %s plan" % (pos.dtype, q.dtype,
                                                                           self.dtype))
            if not (pos.is_contiguous() and q.is_contiguous()):
                raise ValueError("pos and q must be contiguous")
            n = pos.shape[0]
            if pos.dim() != 2 or pos.shape[1] != 3 or q.shape != (n,):
                raise ValueError("pos must be (N, 3) and q (N,)")
            phi, F, E, modes = out
            if (phi.shape != (n,) or F.shape != (n, 3) or E.numel() < 1 or
                    modes.shape != (P, 2) or phi.dtype != self.dtype or F.dtype != self.dtype or
                    E.dtype != t.float64 or modes.dtype != t.int32 or
                    not all(x.is_contiguous() for x in (phi, F, E, modes))):
                raise ValueError("out tensors do not match (N,), (N, 3), (1,) f64, (P, 2) i32")
        _check(self._lib.q2d_rbm_step_noalloc(self._h, pos.data_ptr(), q.data_ptr(), n, int(P),
                                              ctypes.c_uint64(seed), ctypes.c_uint64(step),
                                              phi.data_ptr(), F.data_ptr(), E.data_ptr(),
                                              modes.data_ptr()), "q2d_rbm_step_noalloc")
        return phi, F, E, modes

    def _prep_vjp(self, pos, q, g):
        pos, q, n, _, _, _ = self._prep(pos, q)
        if not g.is_cuda or g.dtype != self.dtype or g.shape != (n,):
            raise ValueError("g must be a device tensor of shape (N,) and the plan's dtype")
        g = g.contiguous()
        t = self._torch
        dq = t.empty(n, dtype=self.dtype, device=pos.device)
        dpos = t.empty((n, 3), dtype=self.dtype, device=pos.device)
        return pos, q, g, n, dq, dpos

    def long_range_vjp(self, pos, q, g):
        """Adjoint of long_range's potential for weights g: (dq, dpos) device tensors."""
        self._sync_stream()
        pos, q, g, n, dq, dpos = self._prep_vjp(pos, q, g)
        _check(self._lib.q2d_long_range_vjp(self._h, pos.data_ptr(), q.data_ptr(), g.data_ptr(),
                                            n, dq.data_ptr(), dpos.data_ptr()),
               "q2d_long_range_vjp")
        return dq, dpos

    def rbm_step_vjp(self, pos, q, g, P, seed, step):
        """Adjoint of rbm_step's potential (same modes for the same seed, step)."""
        self._sync_stream()
        pos, q, g, n, dq, dpos = self._prep_vjp(pos, q, g)
        _check(self._lib.q2d_rbm_step_vjp(self._h, pos.data_ptr(), q.data_ptr(), g.data_ptr(), n,
                                          int(P), ctypes.c_uint64(seed), ctypes.c_uint64(step),
                                          dq.data_ptr(), dpos.data_ptr()),
               "q2d_rbm_step_vjp")
        return dq, dpos

    def modes_eval(self, pos, q, modes, weights):
        """k != 0 sum over the given modes ((n, 2) int32 device tensor) with the
        given weights ((n,) float64 device tensor): (phi, F, E) device tensors."""
        self._sync_stream()
        pos, q, n, phi, F, E = self._prep(pos, q)
        t = self._torch
        if not (modes.is_cuda and weights.is_cuda):
            raise ValueError("modes and weights must be device tensors")
        modes = modes.to(t.int32).contiguous()
        weights = weights.to(t.float64).contiguous()
        if modes.dim() != 2 or modes.shape[1] != 2 or weights.shape != (modes.shape[0],):
            raise ValueError("modes must be (n, 2) and weights (n,)")
        _check(self._lib.q2d_modes_eval(self._h, pos.data_ptr(), q.data_ptr(), n,
                                        modes.data_ptr(), weights.data_ptr(), modes.shape[0],
                                        phi.data_ptr(), F.data_ptr(), E.data_ptr()),
               "q2d_modes_eval")
        return phi, F, E

    def short_range(self, pos, q):
        """Real-space erfc sum with cutoff rc: (phi, F, E) device tensors."""
        self._sync_stream()
        pos, q, n, phi, F, E = self._prep(pos, q)
        _check(self._lib.q2d_short_range(self._h, pos.data_ptr(), q.data_ptr(), n,
                                         phi.data_ptr(), F.data_ptr(), E.data_ptr()),
               "q2d_short_range")
        return phi, F, E

    def slab(self, pos, q, sig0_bot=0.0, sig0_top=0.0, modes=None, sig_bot=None, sig_top=None):
        """Particle-slab term of charged walls (q2d_slab): (phi, F, E) device tensors.
        sig0_*: charge per cell of each wall (sigma A for a uniform wall);
        modes ((n, 2) int32), sig_bot, sig_top ((n,) complex128): device tensors
        of the walls' Fourier coefficients over one cell, or None."""
        self._sync_stream()
        pos, q, n, phi, F, E = self._prep(pos, q)
        t = self._torch
        nm, mp, bp, tp = 0, None, None, None
        if modes is not None:
            modes = modes.to(t.int32).contiguous()
            sb = t.view_as_real(sig_bot.to(t.complex128).contiguous()).contiguous()
            st = t.view_as_real(sig_top.to(t.complex128).contiguous()).contiguous()
            if modes.dim() != 2 or modes.shape[1] != 2 or sb.shape != (modes.shape[0], 2) or \
                    st.shape != (modes.shape[0], 2):
                raise ValueError("modes (n, 2), sig_bot and sig_top (n,) complex")
            nm, mp, bp, tp = modes.shape[0], modes.data_ptr(), sb.data_ptr(), st.data_ptr()
            self._keep = (modes, sb, st)
        _check(self._lib.q2d_slab(self._h, pos.data_ptr(), q.data_ptr(), n, nm, mp, bp, tp,
                                  float(sig0_bot), float(sig0_top), phi.data_ptr(),
                                  F.data_ptr(), E.data_ptr()), "q2d_slab")
        return phi, F, E

    def langevin_step(self, pos, mom, forces, dt, gamma, kT, seed, step, stage, mass=None):
        """One BAOAB stage (q2d_langevin_step) in place on pos (stage 0) and mom.
        forces: up to three (N, 3) device tensors summed."""
        self._sync_stream()
        for tt in [pos, mom] + list(forces) + ([mass] if mass is not None else []):
            if tt.dtype != self.dtype:
                raise Q2DError(Q2D_EDTYPE, "langevin_step")
            if not tt.is_contiguous():
                raise ValueError("tensors must be contiguous")
        fs = [f.data_ptr() for f in forces] + [None] * (3 - len(forces))
        _check(self._lib.q2d_langevin_step(self._h, pos.data_ptr(), mom.data_ptr(),
                                           mass.data_ptr() if mass is not None else None,
                                           mom.shape[0], fs[0], fs[1], fs[2], float(dt),
                                           float(gamma), float(kT), ctypes.c_uint64(seed),
                                           ctypes.c_uint64(step), int(stage)),
               "q2d_langevin_step")

    def check(self):
        """Wait for the stream; return the device-side data status code (0 = ok)."""
        return int(self._lib.q2d_plan_check(self._h))

    def timing_enable(self, mask=TIMING_ALL):
        """Select timed kernel families (bit TIMER_x); True = all, False/0 = none."""
        if mask is True:
            mask = TIMING_ALL
        _check(self._lib.q2d_plan_timing_enable(self._h, int(mask)), "timing_enable")

    def timing_stride(self, n):
        """Record the timed kernel families on every n-th call only (n >= 1)."""
        _check(self._lib.q2d_plan_timing_stride(self._h, int(n)), "timing_stride")

    def timing_read(self, which):
        ms = ctypes.c_double(0.0)
        cnt = ctypes.c_int64(0)
        _check(self._lib.q2d_plan_timing_read(self._h, int(which), ctypes.byref(ms),
                                              ctypes.byref(cnt)), "timing_read")
        return ms.value, cnt.value


REPLICA_SEED_STEP = 0x9E3779B97F4A7C15


def replica_seed(seed, r):
    """Philox key with which replica r of a batch draws its modes."""
    return (int(seed) + int(r) * REPLICA_SEED_STEP) % (1 << 64)


class Batch:
    """R independent systems advanced together (q2d_batch_create).

    boxes: R x 3 (Lx, Ly, Lz); counts: R particle counts.  Positions and charges
    are passed concatenated by replica; outputs come back in the same layout,
    with one energy per replica."""

    def __init__(self, boxes, counts, alpha, w, s, *, precision="fp32", p_max, thin=1,
                 validate=False, stream=None):
        import torch
        self._torch = torch
        lib = load_library()
        self.boxes = np.ascontiguousarray(np.asarray(boxes, dtype=np.float64).reshape(-1, 3))
        self.counts = np.ascontiguousarray(np.asarray(counts, dtype=np.int64))
        self.R = len(self.counts)
        if self.boxes.shape[0] != self.R:
            raise ValueError("one box per replica")
        self.N = int(self.counts.sum())
        self.precision = precision
        self.dtype = torch.float32 if precision == "fp32" else torch.float64
        w = _interleave(w)
        s = _interleave(s)
        opts = _Opts(FP32 if precision == "fp32" else FP64, int(thin), max(self.N, 1),
                     int(p_max), 1 if validate else 0, 0)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self._stream = stream
        h = ctypes.c_void_p()
        dp = ctypes.POINTER(ctypes.c_double)
        _check(lib.q2d_batch_create(self.R, self.boxes.ctypes.data_as(dp),
                                    self.counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                    float(alpha), len(w) // 2, w.ctypes.data_as(dp),
                                    s.ctypes.data_as(dp), ctypes.byref(opts),
                                    ctypes.c_void_p(stream), ctypes.byref(h)), "q2d_batch_create")
        self._h = h
        self._lib = lib
        self._captured = None

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.q2d_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    def _sync_stream(self):
        st = self._torch.cuda.current_stream().cuda_stream
        if st != self._stream:
            _check(self._lib.q2d_batch_set_stream(self._h, ctypes.c_void_p(st)),
                   "q2d_batch_set_stream")
            self._stream = st

    def _io(self, pos, q):
        t = self._torch
        if not (pos.is_cuda and q.is_cuda):
            raise ValueError("pos, q must be device tensors")
        if pos.dtype != self.dtype or q.dtype != self.dtype:
            raise Q2DError(Q2D_EDTYPE, "dtype %s/%s for a %s batch" % (pos.dtype, q.dtype,
                                                                        self.dtype))
        pos = pos.contiguous()
        q = q.contiguous()
        if pos.shape != (self.N, 3) or q.shape != (self.N,):
            raise ValueError("pos must be (sum n_r, 3) and q (sum n_r,)")
        phi = t.empty(self.N, dtype=self.dtype, device=pos.device)
        F = t.empty((self.N, 3), dtype=self.dtype, device=pos.device)
        E = t.empty(self.R, dtype=t.float64, device=pos.device)
        return pos, q, phi, F, E

    def info(self):
        seg = ctypes.c_int32(0)
        npad = ctypes.c_int64(0)
        H = np.zeros(self.R)
        D = np.zeros(self.R)
        dp = ctypes.POINTER(ctypes.c_double)
        _check(self._lib.q2d_batch_info(self._h, ctypes.byref(seg), ctypes.byref(npad),
                                        H.ctypes.data_as(dp), D.ctypes.data_as(dp)),
               "q2d_batch_info")
        return dict(segment=seg.value, n_padded=npad.value, H=H, diag_rb=D)

    def rbm_step(self, pos, q, P, seed, step):
        """(phi, F, E[R], modes[R, P, 2]) device tensors."""
        self._sync_stream()
        pos, q, phi, F, E = self._io(pos, q)
        modes = self._torch.empty((self.R, P, 2), dtype=self._torch.int32, device=pos.device)
        _check(self._lib.q2d_batch_rbm_step(self._h, pos.data_ptr(), q.data_ptr(), int(P),
                                            ctypes.c_uint64(seed), ctypes.c_uint64(step),
                                            phi.data_ptr(), F.data_ptr(), E.data_ptr(),
                                            modes.data_ptr()), "q2d_batch_rbm_step")
        return phi, F, E, modes

    def set_segment(self, S):
        _check(self._lib.q2d_batch_set_segment(self._h, int(S)), "q2d_batch_set_segment")

    def set_config(self, S, split, agg_cpw):
        """Launch shapes: segment length S, split (1: one work-group per sweep
        direction, 2: both in one), agg_cpw (16-mode chunks per wave, 1/2/4)."""
        _check(self._lib.q2d_batch_set_config(self._h, int(S), int(split), int(agg_cpw)),
               "q2d_batch_set_config")

    def config(self):
        S, sp, cw = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
        _check(self._lib.q2d_batch_get_config(self._h, ctypes.byref(S), ctypes.byref(sp),
                                              ctypes.byref(cw)), "q2d_batch_get_config")
        return dict(segment=S.value, split=sp.value, agg_cpw=cw.value)

    def tune(self, pos, q, P, seed=0):
        """Tune the launch shapes on these inputs (segment length, sweep split,
        aggregate chunks per wave); keeps the fastest and returns its segment
        length (the whole choice: config())."""
        self._sync_stream()
        pos, q, phi, F, E = self._io(pos, q)
        seg = ctypes.c_int32(0)
        _check(self._lib.q2d_batch_tune(self._h, pos.data_ptr(), q.data_ptr(), int(P),
                                        ctypes.c_uint64(seed), phi.data_ptr(), F.data_ptr(),
                                        E.data_ptr(), ctypes.byref(seg)), "q2d_batch_tune")
        return seg.value

    def capture(self, pos, q, P, seed, step0):
        """Capture one step as a graph; returns the (phi, F, E) tensors every
        replay writes.  pos and q are read at replay time (update in place)."""
        self._sync_stream()
        pos, q, phi, F, E = self._io(pos, q)
        _check(self._lib.q2d_batch_capture(self._h, pos.data_ptr(), q.data_ptr(), int(P),
                                           ctypes.c_uint64(seed), ctypes.c_uint64(step0),
                                           phi.data_ptr(), F.data_ptr(), E.data_ptr()),
               "q2d_batch_capture")
        self._captured = (pos, q, phi, F, E)
        return phi, F, E

    def replay(self, n=1):
        self._sync_stream()
        _check(self._lib.q2d_batch_replay(self._h, int(n)), "q2d_batch_replay")

    def check(self):
        return int(self._lib.q2d_batch_check(self._h))

