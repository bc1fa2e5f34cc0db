"""Thin ctypes binding of libtufrg.so (the C ABI of include/tufrg.h).

Argument marshalling only: every step of the right-hand side runs in the HIP
library.  Device arrays are torch tensors of dtype complex128 on a ROCm device
(contiguous, [Nq][B][B] unless stated); the library reads their data pointers.
If the library has not been built, importing this module raises.
"""

import ctypes
import os

import numpy as np
import torch  # noqa: F401  (torch's HIP runtime is loaded before the library's: the order the library is tested in)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtufrg.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`"
    )

_lib = ctypes.CDLL(LIB_PATH)

TUFRG_OK = 0
STATUS = {0: "OK", 1: "E_INVAL", 2: "E_NOMEM", 3: "E_HIP", 4: "E_NONFINITE", 5: "E_STEPSIZE",
          6: "E_UNSUPPORTED"}
CUT_TEMPERATURE, CUT_OMEGA, CUT_SHELL = 0, 1, 2
CUTOFFS = {"temperature": CUT_TEMPERATURE, "omega": CUT_OMEGA, "shell": CUT_SHELL}
BASIS_ORBITAL, BASIS_BAND = 0, 1
BASES = {"orbital": BASIS_ORBITAL, "band": BASIS_BAND}
FP64, FP32, BF16X3 = 0, 1, 2
PP, PH = 0, 1

SYMBOLS = ["tufrg_create", "tufrg_destroy", "tufrg_last_error", "tufrg_dims", "tufrg_band_data",
           "tufrg_bubble", "tufrg_project", "tufrg_rhs", "tufrg_flow", "tufrg_timing",
           "tufrg_timing_read", "tufrg_loops_compact", "tufrg_dR", "tufrg_mlp_create",
           "tufrg_mlp_destroy", "tufrg_mlp_last_error", "tufrg_mlp_n_params", "tufrg_mlp_params",
           "tufrg_mlp_set_params", "tufrg_mlp_forward", "tufrg_mlp_loss_grad", "tufrg_mlp_adam_step",
           "tufrg_mlp_train", "tufrg_sur_features", "tufrg_sur_targets", "tufrg_sur_attach",
           "tufrg_sur_loops", "tufrg_batch_create", "tufrg_batch_destroy", "tufrg_batch_last_error",
           "tufrg_batch_dims", "tufrg_batch_flow", "tufrg_set_initial_c", "tufrg_basis_matrix",
           "tufrg_basis_apply", "tufrg_set_initial_p", "tufrg_ff_symmetrize", "tufrg_ff_apply",
           "tufrg_project_static", "tufrg_channel_d", "tufrg_autotune", "tufrg_su2_rhs", "tufrg_su2_flow",
           "tufrg_pair_bands"]
TIMER_LOOP, TIMER_PROJECT, TIMER_BUNDLE, TIMER_SURROGATE = 0, 1, 2, 3


class TuneResult(ctypes.Structure):
    _fields_ = [("tunable", ctypes.c_int32), ("from_cache", ctypes.c_int32), ("loop_kx_chunks", ctypes.c_int32),
                ("mfma_kx_rows", ctypes.c_int32), ("n_candidates", ctypes.c_int32), ("loop_ms", ctypes.c_double),
                ("default_ms", ctypes.c_double)]


class c64(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class Model(ctypes.Structure):
    _fields_ = [("n_orb", ctypes.c_int32), ("n_hop", ctypes.c_int32),
                ("hop_R", ctypes.POINTER(ctypes.c_int32)), ("hop_t", ctypes.POINTER(c64)),
                ("mu", ctypes.c_double), ("V0", ctypes.POINTER(c64))]


class Setup(ctypes.Structure):
    _fields_ = [("n_ff", ctypes.c_int32), ("ff_R", ctypes.POINTER(ctypes.c_int32)),
                ("Lq", ctypes.c_int32), ("n_ref", ctypes.c_int32), ("cutoff", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("temperature", ctypes.c_double), ("basis", ctypes.c_int32)]


STEP_CB = ctypes.CFUNCTYPE(ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_double,
                           ctypes.c_double)


class FlowOpts(ctypes.Structure):
    _fields_ = [("lambda0", ctypes.c_double), ("lambda_end", ctypes.c_double),
                ("n_steps", ctypes.c_int32), ("rtol", ctypes.c_double), ("atol", ctypes.c_double),
                ("h0", ctypes.c_double), ("v_max", ctypes.c_double),
                ("channel_mask", ctypes.c_uint32), ("max_steps", ctypes.c_int32),
                ("on_step", STEP_CB), ("user", ctypes.c_void_p),
                ("surrogate", ctypes.c_int32), ("sample_frac", ctypes.c_double),
                ("sur_tol", ctypes.c_double), ("plain_above", ctypes.c_double),
                ("sample_seed", ctypes.c_uint64), ("graph_steps", ctypes.c_int32),
                ("fused_loops", ctypes.c_int32)]


class FlowResult(ctypes.Structure):
    _fields_ = [("lambda_stop", ctypes.c_double), ("lambda_c", ctypes.c_double),
                ("max_coupling", ctypes.c_double), ("diverged", ctypes.c_int32),
                ("n_steps", ctypes.c_int32), ("n_rhs", ctypes.c_int32),
                ("n_reject", ctypes.c_int32), ("stopped_by_callback", ctypes.c_int32),
                ("n_plain", ctypes.c_int32), ("n_surrogate", ctypes.c_int32),
                ("n_fallback", ctypes.c_int32), ("max_sample_err", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp = ctypes.c_void_p
_lib.tufrg_create.argtypes = [ctypes.POINTER(Model), ctypes.POINTER(Setup), _vp, ctypes.POINTER(_vp)]
_lib.tufrg_destroy.argtypes = [_vp]
_lib.tufrg_last_error.argtypes = [_vp]
_lib.tufrg_last_error.restype = ctypes.c_char_p
_lib.tufrg_dims.argtypes = [_vp] + [ctypes.POINTER(ctypes.c_int32)] * 4
_lib.tufrg_band_data.argtypes = [_vp, _vp, _vp]
_lib.tufrg_bubble.argtypes = [_vp, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, _vp]
_lib.tufrg_project.argtypes = [_vp, _vp, _vp, _vp, _vp]
_lib.tufrg_project_static.argtypes = [_vp, _vp, _vp, _vp, _vp]
_lib.tufrg_channel_d.argtypes = [_vp, _vp, _vp]
_lib.tufrg_su2_rhs.argtypes = [_vp, ctypes.c_double] + [_vp] * 6
_lib.tufrg_autotune.argtypes = [_vp, ctypes.c_double, ctypes.c_char_p, ctypes.POINTER(TuneResult)]
_lib.tufrg_pair_bands.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
_lib.tufrg_basis_matrix.argtypes = [_vp, ctypes.c_int32, _vp, _vp]
_lib.tufrg_basis_apply.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int32]
_lib.tufrg_ff_symmetrize.argtypes = [ctypes.c_int32, _vp, _vp, _vp]
_lib.tufrg_ff_apply.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_int32]
_lib.tufrg_rhs.argtypes = [_vp, ctypes.c_double, _vp, _vp, _vp, _vp]
_lib.tufrg_flow.argtypes = [_vp, ctypes.POINTER(FlowOpts), _vp, _vp, ctypes.POINTER(FlowResult)]
_lib.tufrg_su2_flow.argtypes = [_vp, ctypes.POINTER(FlowOpts), _vp, _vp, _vp, ctypes.POINTER(FlowResult)]
_lib.tufrg_timing.argtypes = [_vp, ctypes.c_int32]
_lib.tufrg_timing_read.argtypes = [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_int32)]
_i32p = ctypes.POINTER(ctypes.c_int32)
_lib.tufrg_loops_compact.argtypes = [_vp, ctypes.c_double, ctypes.c_int32, _vp]
_lib.tufrg_dR.argtypes = [_vp, _i32p]
_lib.tufrg_mlp_create.argtypes = [ctypes.c_int32, _i32p, _vp, _vp, ctypes.POINTER(_vp)]
_lib.tufrg_mlp_destroy.argtypes = [_vp]
_lib.tufrg_mlp_last_error.argtypes = [_vp]
_lib.tufrg_mlp_last_error.restype = ctypes.c_char_p
_lib.tufrg_mlp_n_params.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64)]
_lib.tufrg_mlp_params.argtypes = [_vp, _vp]
_lib.tufrg_mlp_set_params.argtypes = [_vp, _vp]
_lib.tufrg_mlp_forward.argtypes = [_vp, ctypes.c_int64, _vp, _vp]
_lib.tufrg_mlp_loss_grad.argtypes = [_vp, ctypes.c_int32, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_double)]
_lib.tufrg_mlp_adam_step.argtypes = [_vp, _vp, ctypes.c_float]
_lib.tufrg_mlp_train.argtypes = [_vp, ctypes.c_int64, _vp, _vp, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_float, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)]
_lib.tufrg_sur_features.argtypes = [_vp, ctypes.c_int64, _vp, _vp, _vp, ctypes.c_double, _vp]
_lib.tufrg_sur_targets.argtypes = [_vp, ctypes.c_int64, _vp, _vp, _vp, ctypes.c_double, _vp, _vp,
                                   ctypes.POINTER(ctypes.c_double)]
_f64p = ctypes.POINTER(ctypes.c_double)
_lib.tufrg_sur_attach.argtypes = [_vp, _vp, ctypes.c_int32, _f64p, _f64p]
_lib.tufrg_sur_loops.argtypes = [_vp, ctypes.c_double, _vp]
_lib.tufrg_batch_create.argtypes = [ctypes.c_int32, ctypes.POINTER(Model), ctypes.POINTER(Setup), ctypes.c_int32,
                                    ctypes.POINTER(_vp)]
_lib.tufrg_batch_destroy.argtypes = [_vp]
_lib.tufrg_batch_last_error.argtypes = [_vp]
_lib.tufrg_batch_last_error.restype = ctypes.c_char_p
_lib.tufrg_batch_dims.argtypes = [_vp, ctypes.c_int32] + [ctypes.POINTER(ctypes.c_int32)] * 4
_lib.tufrg_batch_flow.argtypes = [_vp, ctypes.POINTER(FlowOpts), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                  ctypes.POINTER(FlowResult)]
for _f in ("tufrg_create", "tufrg_destroy", "tufrg_dims", "tufrg_band_data", "tufrg_bubble",
           "tufrg_project", "tufrg_rhs", "tufrg_flow", "tufrg_timing", "tufrg_timing_read",
           "tufrg_loops_compact", "tufrg_dR", "tufrg_mlp_create", "tufrg_mlp_destroy",
           "tufrg_mlp_n_params", "tufrg_mlp_params", "tufrg_mlp_set_params", "tufrg_mlp_forward",
           "tufrg_mlp_loss_grad", "tufrg_mlp_adam_step", "tufrg_mlp_train", "tufrg_sur_features",
           "tufrg_sur_targets", "tufrg_sur_attach", "tufrg_sur_loops", "tufrg_batch_create",
           "tufrg_batch_destroy", "tufrg_batch_dims", "tufrg_batch_flow"):
    getattr(_lib, _f).restype = ctypes.c_int


class TufrgError(RuntimeError):
    """A status other than TUFRG_OK, with the library's message."""

    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _check(status, ctx=None):
    if status != TUFRG_OK:
        msg = _lib.tufrg_last_error(ctx).decode(errors="replace")
        raise TufrgError(status, msg)


def _ptr(t):
    """Data pointer of a device tensor (the library checks it is device memory)."""
    if hasattr(t, "data_ptr"):
        if not t.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return ctypes.c_void_p(t.data_ptr())
    return ctypes.c_void_p(int(t))


_DTYPES = {"c128": torch.complex128, "f64": torch.float64, "f32": torch.float32, "i32": torch.int32}


def _arr(t, dt, n, name):
    """Pointer of a tensor that a kernel reads or writes n elements of, checked
    for dtype and size first (the library itself sees only an address).  A raw
    address given as an int is passed on unchecked."""
    if hasattr(t, "data_ptr"):
        if t.dtype != _DTYPES[dt]:
            raise TypeError(f"{name} must have dtype {_DTYPES[dt]}, not {t.dtype}")
        if t.numel() < n:
            raise ValueError(f"{name} holds {t.numel()} elements, the call needs {n}")
    return _ptr(t)


def _compact(ctx, t, name="Lc"):
    """Pointer of a compact loop table [2][Nq][n_dR][n_o^4] complex128."""
    return _arr(t, "c128", 2 * ctx.Nq * ctx.n_dR * ctx.n_o ** 4, name)


def _state(ctx, t, name):
    """Pointer of a [Nq][B][B] complex128 device array of the context."""
    return _arr(t, "c128", ctx.Nq * ctx.B * ctx.B, name)


def _model_arrays(hop_R, hop_t, V0):
    hop_R = np.ascontiguousarray(hop_R, dtype=np.int32).reshape(-1, 2)
    hop_t = np.ascontiguousarray(hop_t, dtype=np.complex128)
    V0 = np.ascontiguousarray(V0, dtype=np.complex128)
    if hop_t.ndim != 3 or hop_t.shape[0] != hop_R.shape[0] or hop_t.shape[1] != hop_t.shape[2]:
        raise ValueError(f"hop_t must be [n_hop={hop_R.shape[0]}][n_o][n_o], got {hop_t.shape}")
    if V0.size != hop_t.shape[1] ** 4:
        raise ValueError(f"V0 must hold n_o^4 = {hop_t.shape[1] ** 4} entries, got {V0.size}")
    return hop_R, hop_t, V0


def _stream_handle(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


class Context:
    """Owns a tufrg_ctx.  ``model``/``setup`` are host-side numpy inputs."""

    def __init__(self, hop_R, hop_t, mu, V0, ff, Lq, n_ref, cutoff, precision, stream=None, temperature=None,
                 basis="orbital"):
        hop_R, hop_t, V0 = _model_arrays(hop_R, hop_t, V0)
        ff = np.ascontiguousarray(ff, dtype=np.int32).reshape(-1, 2)
        n_o = hop_t.shape[1]
        self._keep = (hop_R, hop_t, V0, ff)
        m = Model(n_o, hop_R.shape[0], hop_R.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                  hop_t.ctypes.data_as(ctypes.POINTER(c64)), float(mu),
                  V0.ctypes.data_as(ctypes.POINTER(c64)))
        cut = CUTOFFS.get(cutoff, cutoff)
        prec = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3}.get(precision, precision)
        s = Setup(ff.shape[0], ff.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(Lq), int(n_ref),
                  int(cut), int(prec), float(temperature or 0.0), int(BASES.get(basis, basis)))
        h = ctypes.c_void_p()
        _check(_lib.tufrg_create(ctypes.byref(m), ctypes.byref(s), _stream_handle(stream),
                                 ctypes.byref(h)))
        self.handle = h
        B, Nq, Nf, nD = (ctypes.c_int32() for _ in range(4))
        _check(_lib.tufrg_dims(h, ctypes.byref(B), ctypes.byref(Nq), ctypes.byref(Nf),
                               ctypes.byref(nD)), h)
        self.B, self.Nq, self.Nf, self.n_dR = B.value, Nq.value, Nf.value, nD.value
        self.n_o, self.n_ff = n_o, ff.shape[0]

    @classmethod
    def from_workload(cls, w, precision=None, stream=None, **over):
        kw = dict(hop_R=w["hop_R"], hop_t=w["hop_t"], mu=w["mu"], V0=w["V0"], ff=w["ff"],
                  Lq=w["Lq"], n_ref=w["n_ref"], cutoff=w["cutoff"], temperature=w.get("temperature"),
                  precision=precision if precision is not None else w["prec"])
        kw.update(over)
        return cls(stream=stream, **kw)

    def close(self):
        if self.handle is not None and self.handle.value:
            _lib.tufrg_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tufrg_band_data(ctx, e, Pi):
    """Band energies e [n_o][Nf] (float64) and projectors Pi [n_o][Nf][n_o][n_o] (complex128), device."""
    _check(_lib.tufrg_band_data(ctx.handle, _arr(e, "f64", ctx.n_o * ctx.Nf, "e"),
                                 _arr(Pi, "c128", ctx.n_o ** 3 * ctx.Nf, "Pi")), ctx.handle)


def tufrg_bubble(ctx, channel, lam, deriv, L):
    """Loop (deriv) or bubble matrices L [Nq][B][B] of channel PP or PH at scale lam, device."""
    _check(_lib.tufrg_bubble(ctx.handle, int(channel), float(lam), int(deriv), _state(ctx, L, "L")), ctx.handle)


def tufrg_project(ctx, P, C, VP, VC):
    """Projected vertices VP, VC [Nq][B][B] of the state P, C, all on the device."""
    _check(_lib.tufrg_project(ctx.handle, _state(ctx, P, "P"), _state(ctx, C, "C"), _state(ctx, VP, "VP"),
                              _state(ctx, VC, "VC")), ctx.handle)


def tufrg_pair_bands(ctx, enable=True):
    """Use (enable) or bypass the Kramers-paired BF16X3 loops; returns whether
    the pairs are in use (they are only where the bands were found paired)."""
    act = ctypes.c_int32()
    _check(_lib.tufrg_pair_bands(ctx.handle, int(bool(enable)), ctypes.byref(act)), ctx.handle)
    return bool(act.value)


def tufrg_autotune(ctx, lam, cache_path=None):
    """Time the loop kernels' candidate launch shapes at scale lam and keep the
    fastest (or take it from the JSON cache file); returns the result fields."""
    r = TuneResult()
    path = None if cache_path is None else os.fsencode(cache_path)
    _check(_lib.tufrg_autotune(ctx.handle, float(lam), path, ctypes.byref(r)), ctx.handle)
    return {k: getattr(r, k) for k, _ in TuneResult._fields_}


def tufrg_channel_d(ctx, C, D):
    """The third channel D [Nq][B][B] (layout of C) of the state C, on the
    device: D_{n1n2n3n4} = -C_{n1n2n4n3}."""
    _check(_lib.tufrg_channel_d(ctx.handle, _state(ctx, C, "C"), _state(ctx, D, "D")), ctx.handle)


def tufrg_project_static(ctx, P, C, VP, VC):
    """tufrg_project without any device allocation: its rho-space buffers live
    in the library's static per-GPU scratch (calls on one GPU must not overlap)."""
    _check(_lib.tufrg_project_static(ctx.handle, _state(ctx, P, "P"), _state(ctx, C, "C"), _state(ctx, VP, "VP"),
                                     _state(ctx, VC, "VC")),
           ctx.handle)


def tufrg_set_initial_c(ctx, C0):
    """Static C-channel term of a non-local initial interaction ([Nq][B][B] on
    the device, C layout), or None to remove it."""
    _check(_lib.tufrg_set_initial_c(ctx.handle, None if C0 is None else _state(ctx, C0, "C0")), ctx.handle)


def tufrg_basis_matrix(ctx, channel, U, M):
    """Basis matrix M [Nq][B][B] of channel PP (U matrix) or PH (X matrix) from
    the unitaries U [Nf][n_o][n_o] (orbital rows, band columns), all on the device."""
    _check(_lib.tufrg_basis_matrix(ctx.handle, int(channel), _arr(U, "c128", ctx.Nf * ctx.n_o ** 2, "U"),
                                   _state(ctx, M, "M")), ctx.handle)


def tufrg_basis_apply(ctx, M, X, Y, to_orbital=False):
    """Y = M^H X M per q (orbital -> band), or M X M^H (to_orbital)."""
    _check(_lib.tufrg_basis_apply(ctx.handle, _state(ctx, M, "M"), _state(ctx, X, "X"), _state(ctx, Y, "Y"),
                                  int(bool(to_orbital))), ctx.handle)


def tufrg_ff_symmetrize(ff):
    """Symmetrised form factors of the set ff [n_ff][2]: (W [n_ff][n_ff], labels)."""
    ff = np.ascontiguousarray(ff, dtype=np.int32).reshape(-1, 2)
    n = ff.shape[0]
    W = np.zeros((n, n), dtype=np.complex128)
    lab = np.zeros(n, dtype=np.int32)
    _check(_lib.tufrg_ff_symmetrize(n, ff.ctypes.data, W.ctypes.data, lab.ctypes.data))
    return W, lab


def tufrg_ff_apply(ctx, W, X, Y, to_plane_waves=False):
    """Y = W X W^H in the form-factor index (or the converse), [Nq][B][B] on the device."""
    W = np.ascontiguousarray(W, dtype=np.complex128)
    if W.shape != (ctx.n_ff, ctx.n_ff):
        raise ValueError(f"W must be [{ctx.n_ff}][{ctx.n_ff}], got {W.shape}")
    _check(_lib.tufrg_ff_apply(ctx.handle, W.ctypes.data, _state(ctx, X, "X"), _state(ctx, Y, "Y"),
                               int(bool(to_plane_waves))),
           ctx.handle)


def tufrg_set_initial_p(ctx, P0):
    """Static P-channel term of the bare vertex ([Nq][B][B] on the device, P
    layout), or None to remove it."""
    _check(_lib.tufrg_set_initial_p(ctx.handle, None if P0 is None else _state(ctx, P0, "P0")), ctx.handle)


def tufrg_rhs(ctx, lam, P, C, dP, dC):
    """Right-hand side dP, dC [Nq][B][B] at scale lam; outputs must not overlap P, C."""
    _check(_lib.tufrg_rhs(ctx.handle, float(lam), _state(ctx, P, "P"), _state(ctx, C, "C"),
                          _state(ctx, dP, "dP"), _state(ctx, dC, "dC")), ctx.handle)


def tufrg_flow(ctx, P, C, lambda0, lambda_end, n_steps=0, rtol=1e-6, atol=1e-6, h0=0.05,
               v_max=50.0, channel_mask=3, max_steps=0, on_step=None, surrogate=False,
               sample_frac=0.05, sur_tol=1e-3, plain_above=20.0, sample_seed=3, graph_steps=0):
    """Integrates P, C in place; returns the result as a dict."""
    cb = STEP_CB(on_step) if on_step is not None else STEP_CB()
    o = FlowOpts(float(lambda0), float(lambda_end), int(n_steps), float(rtol), float(atol),
                 float(h0), float(v_max), int(channel_mask), int(max_steps), cb, None,
                 int(bool(surrogate)), float(sample_frac), float(sur_tol), float(plain_above),
                 int(sample_seed), int(graph_steps))
    r = FlowResult()
    _check(_lib.tufrg_flow(ctx.handle, ctypes.byref(o), _state(ctx, P, "P"), _state(ctx, C, "C"),
                           ctypes.byref(r)),
           ctx.handle)
    return r.as_dict()


def tufrg_su2_rhs(ctx, lam, p, c, d, dp, dc, dd):
    """SU(2)-reduced right-hand side of a one-orbital context: (dp, dc, dd) of
    the state (p, c, d), all complex128 [Nq][n_ff][n_ff] on the device."""
    _check(_lib.tufrg_su2_rhs(ctx.handle, float(lam), *[_state(ctx, x, n) for x, n in
                                                         ((p, "p"), (c, "c"), (d, "d"), (dp, "dp"), (dc, "dc"),
                                                          (dd, "dd"))]), ctx.handle)


def tufrg_su2_flow(ctx, p, c, d, lambda0, lambda_end, n_steps, v_max=50.0, max_steps=0, on_step=None):
    """Euler flow of the SU(2)-reduced state (p, c, d) in place; the result as a dict."""
    cb = STEP_CB(on_step) if on_step is not None else STEP_CB()
    o = FlowOpts(float(lambda0), float(lambda_end), int(n_steps), 1e-6, 1e-6, 0.05, float(v_max), 3,
                 int(max_steps), cb, None, 0, 0.05, 1e-3, 20.0, 3, 0)
    r = FlowResult()
    _check(_lib.tufrg_su2_flow(ctx.handle, ctypes.byref(o), _state(ctx, p, "p"), _state(ctx, c, "c"),
                               _state(ctx, d, "d"), ctypes.byref(r)), ctx.handle)
    return r.as_dict()


def tufrg_timing(ctx, enable):
    """Switch the per-stage event timers of the context on or off."""
    _check(_lib.tufrg_timing(ctx.handle, int(bool(enable))), ctx.handle)


def tufrg_timing_read(ctx, timer):
    """(total milliseconds, number of timed intervals) of one timer."""
    ms = ctypes.c_double()
    n = ctypes.c_int32()
    _check(_lib.tufrg_timing_read(ctx.handle, int(timer), ctypes.byref(ms), ctypes.byref(n)),
           ctx.handle)
    return ms.value, n.value


def tufrg_loops_compact(ctx, lam, deriv, Lc):
    """Compact loops of both channels, Lc: complex128 [2][Nq][n_dR][n_o^4]."""
    _check(_lib.tufrg_loops_compact(ctx.handle, float(lam), int(deriv), _compact(ctx, Lc)), ctx.handle)


def tufrg_dR(ctx):
    """Difference vectors of the compact loop blocks, int32 [n_dR][2]."""
    out = np.zeros((ctx.n_dR, 2), dtype=np.int32)
    _check(_lib.tufrg_dR(ctx.handle, out.ctypes.data_as(_i32p)), ctx.handle)
    return out


class Mlp:
    """Owns a tufrg_mlp (the loop surrogate network)."""

    def __init__(self, sizes, params=None, stream=None):
        sz = np.ascontiguousarray(sizes, dtype=np.int32)
        p = None if params is None else np.ascontiguousarray(params, dtype=np.float32)
        h = ctypes.c_void_p()
        st = _lib.tufrg_mlp_create(len(sz), sz.ctypes.data_as(_i32p),
                                   None if p is None else p.ctypes.data_as(ctypes.c_void_p),
                                   _stream_handle(stream), ctypes.byref(h))
        if st != TUFRG_OK:
            raise TufrgError(st, _lib.tufrg_mlp_last_error(None).decode(errors="replace"))
        self.handle = h
        self.sizes = [int(x) for x in sz]
        n = ctypes.c_int64()
        self._check(_lib.tufrg_mlp_n_params(h, ctypes.byref(n)))
        self.n_params = n.value

    def _check(self, status):
        if status != TUFRG_OK:
            raise TufrgError(status, _lib.tufrg_mlp_last_error(self.handle).decode(errors="replace"))

    def close(self):
        if self.handle is not None and self.handle.value:
            _lib.tufrg_mlp_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tufrg_mlp_params(net, out):
    """Copy the flat parameter vector (float32, device) into out."""
    net._check(_lib.tufrg_mlp_params(net.handle, _arr(out, "f32", net.n_params, "out")))


def tufrg_mlp_set_params(net, params):
    """Set the flat parameter vector (float32, device); resets the Adam moments."""
    net._check(_lib.tufrg_mlp_set_params(net.handle, _arr(params, "f32", net.n_params, "params")))


def tufrg_mlp_forward(net, X, Y):
    """Y [n][n_out] = net(X [n][n_in]), float32 device arrays."""
    n = int(X.shape[0])
    net._check(_lib.tufrg_mlp_forward(net.handle, n, _arr(X, "f32", n * net.sizes[0], "X"),
                                      _arr(Y, "f32", n * net.sizes[-1], "Y")))


def tufrg_mlp_loss_grad(net, X, T, grad=None):
    """Mean squared error of the batch (returned) and its gradient into grad."""
    loss = ctypes.c_double()
    n = int(X.shape[0])
    net._check(_lib.tufrg_mlp_loss_grad(net.handle, n, _arr(X, "f32", n * net.sizes[0], "X"),
                                        _arr(T, "f32", n * net.sizes[-1], "T"),
                                        None if grad is None else _arr(grad, "f32", net.n_params, "grad"),
                                        ctypes.byref(loss)))
    return loss.value


def tufrg_mlp_adam_step(net, grad, lr):
    """One Adam update with gradient grad (device; None: the last computed one) and rate lr."""
    g = None if grad is None else _arr(grad, "f32", net.n_params, "grad")
    net._check(_lib.tufrg_mlp_adam_step(net.handle, g, float(lr)))


def tufrg_mlp_train(net, X, T, batch, epochs, lr, seed=0):
    """Minibatch Adam epochs; returns the mean batch loss of the last epoch."""
    loss = ctypes.c_double()
    n = int(X.shape[0])
    net._check(_lib.tufrg_mlp_train(net.handle, n, _arr(X, "f32", n * net.sizes[0], "X"),
                                    _arr(T, "f32", n * net.sizes[-1], "T"), int(batch),
                                    int(epochs), float(lr), int(seed), ctypes.byref(loss)))
    return loss.value


def _opt(t, n, name):
    return None if t is None else _arr(t, "i32", n, name)


def tufrg_sur_features(ctx, n, lam, X, q=None, ch=None, iD=None):
    """Feature rows X [n][11 + n_dR] (float32, device) of n loop blocks at scale
    lam; q, ch, iD: int32 device lists of the blocks, or None for the first n of
    all 2 Nq n_dR blocks in compact order."""
    n = int(n)
    _check(_lib.tufrg_sur_features(ctx.handle, n, _opt(q, n, "q"), _opt(ch, n, "ch"), _opt(iD, n, "iD"),
                                   float(lam), _arr(X, "f32", n * (11 + ctx.n_dR), "X")), ctx.handle)


def tufrg_sur_targets(ctx, n, scale, Lc, T, q=None, ch=None, iD=None):
    """Writes the targets Lc / scale; returns max |Lc| over the blocks."""
    mx = ctypes.c_double()
    n = int(n)
    _check(_lib.tufrg_sur_targets(ctx.handle, n, _opt(q, n, "q"), _opt(ch, n, "ch"), _opt(iD, n, "iD"),
                                  float(scale), _compact(ctx, Lc), _arr(T, "f32", n * 2 * ctx.n_o ** 4, "T"),
                                  ctypes.byref(mx)), ctx.handle)
    return mx.value


def tufrg_sur_attach(ctx, net, lambdas=(1.0,), scales=(1.0,)):
    """Attach net with its target scale table (None detaches)."""
    lam = np.ascontiguousarray(lambdas, dtype=np.float64)
    sc = np.ascontiguousarray(scales, dtype=np.float64)
    if lam.shape != sc.shape:
        raise ValueError("scale table arrays differ in length")
    _check(_lib.tufrg_sur_attach(ctx.handle, None if net is None else net.handle, len(lam),
                                 lam.ctypes.data_as(_f64p), sc.ctypes.data_as(_f64p)), ctx.handle)


def tufrg_sur_loops(ctx, lam, Lc):
    """Compact loops Lc [2][Nq][n_dR][n_o^4] (device) from the attached network."""
    _check(_lib.tufrg_sur_loops(ctx.handle, float(lam), _compact(ctx, Lc)), ctx.handle)


class Batch:
    """Owns a tufrg_batch of independent instances given as workload dicts
    (keys as in synth.workloads) and a common arithmetic precision."""

    def __init__(self, workloads, precision="fp32", n_streams=4):
        n = len(workloads)
        models, setups = (Model * n)(), (Setup * n)()
        self._keep = []
        for i, w in enumerate(workloads):
            hop_R, hop_t, V0 = _model_arrays(w["hop_R"], w["hop_t"], w["V0"])
            ff = np.ascontiguousarray(w["ff"], dtype=np.int32).reshape(-1, 2)
            self._keep.append((hop_R, hop_t, V0, ff))
            models[i] = Model(hop_t.shape[1], hop_R.shape[0], hop_R.ctypes.data_as(_i32p),
                              hop_t.ctypes.data_as(ctypes.POINTER(c64)), float(w["mu"]),
                              V0.ctypes.data_as(ctypes.POINTER(c64)))
            cut = CUTOFFS.get(w["cutoff"], w["cutoff"])
            prec = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3}.get(precision, precision)
            setups[i] = Setup(ff.shape[0], ff.ctypes.data_as(_i32p), int(w["Lq"]), int(w["n_ref"]), int(cut),
                              int(prec), float(w.get("temperature") or 0.0),
                              int(BASES.get(w.get("basis", "orbital"), w.get("basis", "orbital"))))
        h = ctypes.c_void_p()
        st = _lib.tufrg_batch_create(n, models, setups, int(n_streams), ctypes.byref(h))
        if st != TUFRG_OK:
            raise TufrgError(st, _lib.tufrg_batch_last_error(None).decode(errors="replace"))
        self.handle = h
        self.n = n
        self.dims = []
        for i in range(n):
            B, Nq, Nf, nD = (ctypes.c_int32() for _ in range(4))
            self._check(_lib.tufrg_batch_dims(h, i, ctypes.byref(B), ctypes.byref(Nq), ctypes.byref(Nf),
                                              ctypes.byref(nD)))
            self.dims.append(dict(B=B.value, Nq=Nq.value, Nf=Nf.value, n_dR=nD.value))

    def _check(self, status):
        if status != TUFRG_OK:
            raise TufrgError(status, _lib.tufrg_batch_last_error(self.handle).decode(errors="replace"))

    def close(self):
        if self.handle is not None and self.handle.value:
            _lib.tufrg_batch_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tufrg_batch_flow(batch, Ps, Cs, lambda0, lambda_end, n_steps, v_max=50.0, channel_mask=3, max_steps=0,
                     graph_steps=0, fused_loops=False):
    """Lockstep Euler flow of every instance (P, C in place); list of result
    dicts.  graph_steps > 1: that many lockstep steps of all instances per HIP
    graph.  fused_loops: the loop kernels of all (two-orbital) instances in one
    launch per kernel shape instead of one per instance."""
    n = batch.n
    if len(Ps) != n or len(Cs) != n:
        raise ValueError(f"one P and one C per instance ({n})")
    sizes = [d["Nq"] * d["B"] * d["B"] for d in batch.dims]
    pp = (_vp * n)(*[_arr(x, "c128", m, f"P[{i}]") for i, (x, m) in enumerate(zip(Ps, sizes))])
    cp = (_vp * n)(*[_arr(x, "c128", m, f"C[{i}]") for i, (x, m) in enumerate(zip(Cs, sizes))])
    o = FlowOpts(float(lambda0), float(lambda_end), int(n_steps), 0.0, 0.0, 0.0, float(v_max),
                 int(channel_mask), int(max_steps), STEP_CB(), None, 0, 0.0, 0.0, 0.0, 0, int(graph_steps),
                 int(bool(fused_loops)))
    res = (FlowResult * n)()
    batch._check(_lib.tufrg_batch_flow(batch.handle, ctypes.byref(o), pp, cp, res))
    return [r.as_dict() for r in res]
