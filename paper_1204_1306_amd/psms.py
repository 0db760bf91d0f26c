"""Thin ctypes binding of libpsms (C-ABI in include/psms.h).

Argument marshalling only: every step of the hot path runs in the HIP library.
Fields are complex128 arrays in the boundary layout ``[nrhs, V, 4, 3]`` (or
``[V, 4, 3]`` for one field): numpy arrays (host memory, staged by the library)
or torch tensors on the GPU (used in place, no copy). Results come back in the
same kind of container as the input.

The library must have been built (``python -m paper_1204_1306_amd.build``);
importing this module on a machine without it raises immediately.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpsms.so")

F64, MIXED = 0, 1
OP_FULL, OP_SCHUR = 0, 1
PC_NONE, PC_SAP, PC_NET = 0, 1, 2
SPINOR_F32, SPINOR_BF16 = 0, 1

STATUS = {0: "ok", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENOTCONV", -5: "ENOTSU3", -6: "ENAN"}


class PsmsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Geom(C.Structure):
    _fields_ = [("L", C.c_int * 4), ("b", C.c_int * 4), ("antiperiodic_t", C.c_int), ("kappa", C.c_double),
                ("sap_b", C.c_int * 4), ("outer_b", C.c_int * 4)]


class SolveParams(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int), ("restart", C.c_int), ("prec", C.c_int),
                ("pc", C.c_int), ("sap_cycles", C.c_int), ("block_iters", C.c_int), ("inner_tol", C.c_double),
                ("inner_storage", C.c_int), ("net_fallback", C.c_int), ("rhs_chunk", C.c_int)]


class SolveStats(C.Structure):
    _fields_ = [("converged", C.c_int), ("outer_iters", C.c_int), ("inner_iters", C.c_int),
                ("used_fallback", C.c_int), ("true_rel_residual", C.c_double), ("seconds", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class GfParams(C.Structure):
    _fields_ = [("alpha", C.c_double), ("alpha_min", C.c_double), ("theta_tol", C.c_double), ("max_iter", C.c_int)]


class GfStats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("functional_start", C.c_double), ("functional_end", C.c_double),
                ("theta_end", C.c_double), ("alpha_end", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FilterParams(C.Structure):
    _fields_ = [("beta", C.c_double * 3), ("solve", SolveParams), ("work_slot", C.c_int * 2), ("slot_out", C.c_int)]


class FilterResult(C.Structure):
    _fields_ = [("delta1", C.c_void_p), ("accept1", C.c_void_p), ("delta2", C.c_void_p), ("accept2", C.c_void_p),
                ("delta3", C.c_double), ("accept3", C.c_int), ("inner_iters", C.c_int)]


class TrainParams(C.Structure):
    _fields_ = [("npairs", C.c_int), ("batch", C.c_int), ("epochs", C.c_int), ("chunk", C.c_int), ("lr", C.c_double),
                ("solve_tol", C.c_double), ("seed", C.c_ulonglong), ("ckpt_path", C.c_char_p), ("ckpt_every", C.c_int)]


class TrainStats(C.Structure):
    _fields_ = [("first_loss", C.c_double), ("final_loss", C.c_double), ("steps", C.c_int),
                ("seconds_data", C.c_double), ("seconds_train", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None

_SIGS = {
    "psms_default_params": (None, [C.c_void_p]),
    "psms_create": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "psms_destroy": (None, [C.c_void_p]),
    "psms_last_error": (C.c_char_p, [C.c_void_p]),
    "psms_status_string": (C.c_char_p, [C.c_int]),
    "psms_device_bytes": (C.c_ulonglong, [C.c_void_p]),
    "psms_gauge_load": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p]),
    "psms_apply_dw": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_int]),
    "psms_apply_dw_lowp": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int]),
    "psms_apply_dw_noalloc": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_int]),
    "psms_apply_dhat_ee": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int]),
    "psms_apply_block": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_int]),
    "psms_apply_hop_bw": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_int]),
    "psms_apply_proj": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "psms_solve": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "psms_solve_block": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p,
                                   C.c_void_p]),
    "psms_apply_schur": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "psms_apply_schur_inv": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p,
                                       C.c_void_p]),
    "psms_logdet_ratio": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_int, C.c_int,
                                    C.c_void_p, C.c_void_p, C.c_void_p]),
    "psms_log_ratio_estimate": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p]),
    "psms_block_logdet": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    "psms_default_gf_params": (None, [C.c_void_p]),
    "psms_default_filter_params": (None, [C.c_void_p]),
    "psms_filter_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p]),
    "psms_relative_gauge_fix": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_int, C.c_void_p,
                                          C.c_void_p]),
    "psms_logdet_ratio_blocks": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_int, C.c_void_p,
                                           C.c_void_p, C.c_void_p]),
    "psms_net_init": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_ulonglong, C.c_double]),
    "psms_net_num_weights": (C.c_longlong, [C.c_void_p]),
    "psms_net_set_weights": (C.c_int, [C.c_void_p, C.c_void_p, C.c_longlong]),
    "psms_net_get_weights": (C.c_int, [C.c_void_p, C.c_void_p, C.c_longlong]),
    "psms_net_apply": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int]),
    "psms_net_loss_grad": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "psms_default_train_params": (None, [C.c_void_p]),
    "psms_net_train": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "psms_net_save": (C.c_int, [C.c_void_p, C.c_char_p]),
    "psms_net_load": (C.c_int, [C.c_void_p, C.c_char_p]),
    "psms_set_tuning": (C.c_int, [C.c_void_p, C.c_char_p, C.c_int]),
    "psms_get_tuning": (C.c_int, [C.c_void_p, C.c_char_p, C.c_void_p]),
    "psms_autotune": (C.c_int, [C.c_void_p, C.c_int, C.c_char_p]),
    "psms_profile": (C.c_int, [C.c_void_p, C.c_int]),
    "psms_profile_read": (C.c_int, [C.c_void_p, C.c_char_p, C.c_void_p, C.c_void_p, C.c_void_p]),
}


def load_library():
    """Open libpsms.so and declare every exported symbol's signature.

    PyTorch is imported first when it is installed: its wheel carries its own HIP
    runtime under the same soname as the system one, and the library must bind to the
    runtime already in the process (a second HIP/HSA runtime in one process cannot open
    the GPU that the first one holds)."""
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1204_1306_amd.build`")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def default_params(**kw) -> SolveParams:
    p = SolveParams()
    load_library().psms_default_params(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def log_ratio_estimate(delta) -> np.ndarray:
    """ln mean_j exp(-delta[p, j]) per proposal p (psms_log_ratio_estimate)."""
    d = np.ascontiguousarray(np.asarray(delta, np.float64))
    if d.ndim == 1:
        d = d[None, :]
    out = np.empty(d.shape[0], np.float64)
    s = load_library().psms_log_ratio_estimate(C.c_void_p(d.ctypes.data), d.shape[0], d.shape[1],
                                               C.c_void_p(out.ctypes.data))
    if s != 0:
        raise PsmsError(s, "psms_log_ratio_estimate: null, empty or non-finite input")
    return out


def filter_step(inner: "Context", outer: "Context", slot_U: int, slot_Up: int, uniforms, noise, beta=(1.0, 0.0, 0.0),
                solve: SolveParams | None = None, work_slots=(62, 63), slot_out: int = -1) -> dict:
    """psms_filter_step: the three filters of one recursion level; returns the exponents
    and decisions of every step."""
    lib = load_library()
    p = FilterParams()
    lib.psms_default_filter_params(C.byref(p))
    p.beta[:] = list(beta)
    if solve is not None:
        p.solve = solve
    p.work_slot[:] = list(work_slots)
    p.slot_out = slot_out
    nsmall = int(np.prod(np.asarray(inner.L) // np.asarray(inner.b)))
    nouter = int(np.prod(np.asarray(outer.L) // np.asarray(outer.b)))
    u = np.ascontiguousarray(np.asarray(uniforms, np.float64))
    if u.size != nsmall + nouter + 1:
        raise ValueError(f"uniforms must hold {nsmall} + {nouter} + 1 values")
    d1, a1 = np.empty(nsmall), np.empty(nsmall, np.int32)
    d2, a2 = np.empty(nouter), np.empty(nouter, np.int32)
    r = FilterResult()
    r.delta1, r.accept1 = d1.ctypes.data, a1.ctypes.data
    r.delta2, r.accept2 = d2.ctypes.data, a2.ctypes.data
    s = lib.psms_filter_step(inner._h, outer._h, slot_U, slot_Up, C.byref(p), C.c_void_p(u.ctypes.data), _ptr(noise),
                             C.byref(r))
    if s != 0:
        raise PsmsError(s, lib.psms_last_error(outer._h).decode())
    return {"delta1": d1, "accept1": a1.astype(bool), "delta2": d2, "accept2": a2.astype(bool), "delta3": r.delta3,
            "accept3": bool(r.accept3), "inner_iters": r.inner_iters}


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


def _ptr(a):
    if _is_torch(a):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return C.c_void_p(a.data_ptr())
    if not (a.flags["C_CONTIGUOUS"] and a.dtype == np.complex128):
        raise ValueError("numpy arrays must be C-contiguous complex128")
    return C.c_void_p(a.ctypes.data)


def _empty_like(a):
    if _is_torch(a):
        import torch

        return torch.empty_like(a)
    return np.empty_like(a)


class Context:
    """One libpsms context (geometry, device, stream)."""

    def __init__(self, L, b, kappa: float, antiperiodic: bool = True, device: int = 0, stream=None, sap_b=None,
                 outer_b=None):
        lib = load_library()
        g = Geom()
        g.L[:] = list(L)
        g.b[:] = list(b)
        g.antiperiodic_t = 1 if antiperiodic else 0
        g.kappa = float(kappa)
        g.sap_b[:] = list(sap_b) if sap_b is not None else [0, 0, 0, 0]
        g.outer_b[:] = list(outer_b) if outer_b is not None else [0, 0, 0, 0]
        self.L, self.b, self.kappa = tuple(L), tuple(b), float(kappa)
        self.outer_b = tuple(outer_b) if outer_b is not None else None
        self.V = int(np.prod(L))
        h = C.c_void_p()
        st = C.c_void_p(stream) if stream is not None else None
        s = lib.psms_create(C.byref(g), int(device), st, C.byref(h))
        if s != 0:
            raise PsmsError(s, "psms_create failed (see stderr)")
        self._h = h
        self._lib = lib

    def close(self):
        if getattr(self, "_h", None):
            self._lib.psms_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, s: int):
        if s != 0:
            raise PsmsError(s, self._lib.psms_last_error(self._h).decode())

    def _nrhs(self, a) -> int:
        n = int(np.prod(a.shape)) // (self.V * 12)
        if n * self.V * 12 != int(np.prod(a.shape)):
            raise ValueError("field size is not a multiple of 12 V")
        return n

    @property
    def device_bytes(self) -> int:
        return int(self._lib.psms_device_bytes(self._h))

    # ---------------------------------------------------------------- gauge
    def gauge_load(self, slot: int, U, allow_non_su3: bool = False):
        s = self._lib.psms_gauge_load(self._h, int(slot), _ptr(U))
        if s == -5 and allow_non_su3:
            return False
        self._check(s)
        return True

    # ---------------------------------------------------------------- operators
    def apply_dw(self, slot: int, psi, prec: int = F64):
        out = _empty_like(psi)
        self._check(self._lib.psms_apply_dw(self._h, slot, _ptr(psi), _ptr(out), self._nrhs(psi), prec))
        return out

    def apply_dw_lowp(self, slot: int, psi, in_storage: int = SPINOR_BF16, out_storage: int = SPINOR_BF16):
        out = _empty_like(psi)
        self._check(self._lib.psms_apply_dw_lowp(self._h, slot, _ptr(psi), _ptr(out), self._nrhs(psi), in_storage,
                                                 out_storage))
        return out

    def apply_dw_noalloc(self, slot: int, psi, out, prec: int = F64, check: bool = True) -> int:
        """psms_apply_dw_noalloc into the caller's `out` (device tensors only); returns the status."""
        s = self._lib.psms_apply_dw_noalloc(self._h, slot, _ptr(psi), _ptr(out), self._nrhs(psi), prec)
        if check:
            self._check(s)
        return s

    def apply_dhat_ee(self, slot: int, psi):
        out = _empty_like(psi)
        self._check(self._lib.psms_apply_dhat_ee(self._h, slot, _ptr(psi), _ptr(out), self._nrhs(psi)))
        return out

    def apply_block(self, slot: int, colour: int, psi):
        out = _empty_like(psi)
        self._check(self._lib.psms_apply_block(self._h, slot, colour, _ptr(psi), _ptr(out), self._nrhs(psi)))
        return out

    def apply_hop_bw(self, slot: int, from_colour: int, psi):
        out = _empty_like(psi)
        self._check(self._lib.psms_apply_hop_bw(self._h, slot, from_colour, _ptr(psi), _ptr(out), self._nrhs(psi)))
        return out

    def apply_proj(self, psi):
        out = _empty_like(psi)
        self._check(self._lib.psms_apply_proj(self._h, _ptr(psi), _ptr(out), self._nrhs(psi)))
        return out

    # ---------------------------------------------------------------- solves
    def solve(self, slot: int, b, params: SolveParams | None = None, check: bool = True):
        p = params or default_params()
        x = _empty_like(b)
        st = SolveStats()
        s = self._lib.psms_solve(self._h, slot, _ptr(b), _ptr(x), self._nrhs(b), C.byref(p), C.byref(st))
        if check:
            self._check(s)
        return x, st.as_dict()

    def solve_block(self, slot: int, colour: int, b, params: SolveParams | None = None, check: bool = True):
        p = params or default_params()
        x = _empty_like(b)
        st = SolveStats()
        s = self._lib.psms_solve_block(self._h, slot, colour, _ptr(b), _ptr(x), self._nrhs(b), C.byref(p),
                                       C.byref(st))
        if check:
            self._check(s)
        return x, st.as_dict()

    def apply_schur(self, slot: int, xi, params: SolveParams | None = None):
        p = params or default_params()
        out = _empty_like(xi)
        st = SolveStats()
        self._check(self._lib.psms_apply_schur(self._h, slot, _ptr(xi), _ptr(out), self._nrhs(xi), C.byref(p),
                                               C.byref(st)))
        return out, st.as_dict()

    def apply_schur_inv(self, slot: int, phi, params: SolveParams | None = None):
        p = params or default_params()
        out = _empty_like(phi)
        st = SolveStats()
        self._check(self._lib.psms_apply_schur_inv(self._h, slot, _ptr(phi), _ptr(out), self._nrhs(phi), C.byref(p),
                                                   C.byref(st)))
        return out, st.as_dict()

    def logdet_ratio(self, op: int, slot_U: int, slots_Up, noise, params: SolveParams | None = None, delta=None,
                     check: bool = True, n_interp: int = 1):
        """Delta[p, j] for proposals slots_Up and noise fields; returns (delta, stats).
        With n_interp > 1 the noise holds n_interp groups of nnoise fields, group i for
        interpolation factor i."""
        p = params or default_params()
        nprop = len(slots_Up)
        nfield = self._nrhs(noise)
        if n_interp < 1 or nfield % n_interp:
            raise ValueError("the noise must hold n_interp groups of equally many fields")
        nnoise = nfield // n_interp
        slots = (C.c_int * nprop)(*slots_Up)
        if delta is None:
            delta = np.empty((nprop, nnoise), np.float64)
        dptr = C.c_void_p(delta.data_ptr()) if _is_torch(delta) else C.c_void_p(delta.ctypes.data)
        st = SolveStats()
        s = self._lib.psms_logdet_ratio(self._h, op, slot_U, slots, nprop, _ptr(noise), nnoise, int(n_interp), C.byref(p),
                                        dptr, C.byref(st))
        if check:
            self._check(s)
        return delta, st.as_dict()

    def relative_gauge_fix(self, slot_U: int, slot_Up: int, slot_gU: int, slot_gUp: int, want_g: bool = False, **kw):
        """psms_relative_gauge_fix; returns (g [V,3,3] complex or None, stats)."""
        p = GfParams()
        self._lib.psms_default_gf_params(C.byref(p))
        for k, v in kw.items():
            setattr(p, k, v)
        g = np.empty((self.V, 3, 3), np.complex128) if want_g else None
        st = GfStats()
        self._check(self._lib.psms_relative_gauge_fix(self._h, slot_U, slot_Up, C.byref(p), slot_gU, slot_gUp,
                                                      C.c_void_p(g.ctypes.data) if want_g else None, C.byref(st)))
        return g, st.as_dict()

    def n_outer(self) -> int:
        return int(np.prod(np.asarray(self.L) // np.asarray(self.outer_b))) if self.outer_b else 0

    def logdet_ratio_blocks(self, slot_U: int, slots_Up, noise, params: SolveParams | None = None, delta=None,
                            check: bool = True):
        """Delta[p, j, B] per outer block B (a context made with outer_b); returns (delta, stats)."""
        p = params or default_params()
        nprop = len(slots_Up)
        nnoise = self._nrhs(noise)
        slots = (C.c_int * nprop)(*slots_Up)
        if delta is None:
            delta = np.empty((nprop, nnoise, self.n_outer()), np.float64)
        dptr = C.c_void_p(delta.data_ptr()) if _is_torch(delta) else C.c_void_p(delta.ctypes.data)
        st = SolveStats()
        s = self._lib.psms_logdet_ratio_blocks(self._h, slot_U, slots, nprop, _ptr(noise), nnoise, C.byref(p), dptr,
                                               C.byref(st))
        if check:
            self._check(s)
        return delta, st.as_dict()

    def block_logdet(self, slots) -> np.ndarray:
        """ln det D_b per gauge slot and block (lexicographic block order) as complex
        (ln|det|, i arg det): shape [len(slots), nblk]."""
        arr = (C.c_int * len(slots))(*slots)
        nblk = int(np.prod(np.asarray(self.L) // np.asarray(self.b)))
        out = np.empty((len(slots), nblk, 2), np.float64)
        self._check(self._lib.psms_block_logdet(self._h, arr, len(slots), C.c_void_p(out.ctypes.data)))
        return out[..., 0] + 1j * out[..., 1]

    # ---------------------------------------------------------------- learned preconditioner
    def net_init(self, channels=(1, 8, 8, 8, 1), seed: int = 1, scale: float = 0.1):
        ch = (C.c_int * len(channels))(*channels)
        self._check(self._lib.psms_net_init(self._h, ch, len(channels) - 1, int(seed), float(scale)))

    def net_num_weights(self) -> int:
        return int(self._lib.psms_net_num_weights(self._h))

    def net_get_weights(self) -> np.ndarray:
        n = self.net_num_weights()
        w = np.empty(n, np.complex128)
        self._check(self._lib.psms_net_get_weights(self._h, C.c_void_p(w.ctypes.data), n))
        return w

    def net_set_weights(self, w):
        w = np.ascontiguousarray(np.asarray(w, np.complex128).ravel())
        self._check(self._lib.psms_net_set_weights(self._h, C.c_void_p(w.ctypes.data), w.size))

    def net_apply(self, slot: int, psi):
        out = _empty_like(psi)
        self._check(self._lib.psms_net_apply(self._h, slot, _ptr(psi), _ptr(out), self._nrhs(psi)))
        return out

    def net_loss_grad(self, slot: int, r, e):
        loss = C.c_double()
        g = np.empty(self.net_num_weights(), np.complex128)
        self._check(self._lib.psms_net_loss_grad(self._h, slot, _ptr(r), _ptr(e), self._nrhs(r), C.byref(loss),
                                                 C.c_void_p(g.ctypes.data)))
        return loss.value, g

    def net_train(self, slots, **kw):
        tp = TrainParams()
        self._lib.psms_default_train_params(C.byref(tp))
        keep = None
        for k, v in kw.items():
            if k == "ckpt_path" and v is not None:
                keep = v.encode()
                v = keep
            setattr(tp, k, v)
        arr = (C.c_int * len(slots))(*slots)
        ts = TrainStats()
        self._check(self._lib.psms_net_train(self._h, arr, len(slots), C.byref(tp), C.byref(ts)))
        return ts.as_dict()

    def net_save(self, path: str):
        self._check(self._lib.psms_net_save(self._h, path.encode()))

    def net_load(self, path: str):
        self._check(self._lib.psms_net_load(self._h, path.encode()))

    # ---------------------------------------------------------------- tuning
    TUNING_KEYS = ("dslash_variant_f64", "dslash_variant_f32", "dslash_variant_bf16", "nr_f64", "nr_low", "xcd_map",
                   "net_mfma", "block_solver", "block_lanes", "block_eo", "block_eo_lanes",
                   "block_tol_prec", "sap_bf16", "block_xcd", "sap_link16")

    def set_tuning(self, key: str, value: int):
        self._check(self._lib.psms_set_tuning(self._h, key.encode(), int(value)))

    def get_tuning(self, key: str) -> int:
        v = C.c_int()
        self._check(self._lib.psms_get_tuning(self._h, key.encode(), C.byref(v)))
        return v.value

    def tuning(self) -> dict:
        return {k: self.get_tuning(k) for k in self.TUNING_KEYS}

    def autotune(self, slot: int = 0, cache_path: str | None = None) -> dict:
        self._check(self._lib.psms_autotune(self._h, int(slot), cache_path.encode() if cache_path else None))
        return self.tuning()

    # ---------------------------------------------------------------- profiling
    def profile(self, enable: bool):
        self._check(self._lib.psms_profile(self._h, 1 if enable else 0))

    def profile_read(self, family: str):
        ms, n, by = C.c_double(), C.c_longlong(), C.c_double()
        self._check(self._lib.psms_profile_read(self._h, family.encode(), C.byref(ms), C.byref(n), C.byref(by)))
        return {"ms": ms.value, "launches": n.value, "bytes": by.value}
