"""ctypes binding of the C ABI declared in include/kgf.h.

Argument marshalling only.  Tensors must be torch.complex128, contiguous,
on the context's device; they are passed as raw device pointers and the
library runs on torch's current stream of that device.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_NAME = "libkgf.so"
ABI_VERSION = 2   # KGF_ABI_VERSION of include/kgf.h that the signatures below follow

DIRECTION_FORWARD = -1      # exp(-i H dt)
DIRECTION_BACKWARD = +1     # exp(+i H dt)
DIRECTION_IMAGINARY = 0     # exp(-(H - shift) dt)

KGF_OK = 0
_CODES = {-1: "KGF_EINVAL", -2: "KGF_ENOMEM", -3: "KGF_EHIP", -4: "KGF_ENOCONV", -5: "KGF_EUNSUPPORTED",
          -6: "KGF_EDEGENERATE"}


class KgfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code


class _C128(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class _ModelDesc(C.Structure):
    _fields_ = [("L", C.c_int), ("n_bonds", C.c_int),
                ("bond_i", C.POINTER(C.c_int32)), ("bond_j", C.POINTER(C.c_int32)),
                ("t_bond", C.POINTER(C.c_double)), ("eps_up", C.POINTER(C.c_double)),
                ("eps_dn", C.POINTER(C.c_double)), ("U", C.POINTER(C.c_double))]


class _ContourFn(C.Structure):
    """kgf_contour_fn: device pointers of the components of a contour function."""
    _fields_ = [("lesser", C.c_void_p), ("greater", C.c_void_p), ("mixed", C.c_void_p), ("mixed_left", C.c_void_p),
                ("vert_greater", C.c_void_p), ("vert_lesser", C.c_void_p)]


CONTOUR_KEYS = ("lesser", "greater", "mixed", "mixed_left", "vert_greater", "vert_lesser")


class _GsOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int), ("check_every", C.c_int), ("reorth", C.c_int),
                ("unique_check", C.c_int), ("unique_tol", C.c_double), ("unique_seed", C.c_uint64)]


class _GsInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("converged", C.c_int), ("residual", C.c_double), ("fidelity2", C.c_double)]


def _gs(tol, max_iter, check_every, reorth, unique_check=False, unique_tol=0.0, unique_seed=8):
    """kgf_gs_opts; unique_check runs the second-start uniqueness test."""
    return _GsOpts(float(tol), int(max_iter), int(check_every), int(reorth), int(bool(unique_check)),
                   float(unique_tol), int(unique_seed))


class _PropOpts(C.Structure):
    _fields_ = [("krylov_dim", C.c_int), ("reorth", C.c_int), ("dt", C.c_double),
                ("direction", C.c_int), ("shift", C.c_double), ("breakdown_tol", C.c_double)]


class _RunInfo(C.Structure):
    _fields_ = [("intervals", C.c_int), ("width", C.c_int), ("done", C.c_int), ("next_width", C.c_int),
                ("next_mesh_index", C.c_int), ("chunk_width", C.c_int), ("branch", C.c_int),
                ("vector_steps", C.c_int64), ("total_vector_steps", C.c_int64), ("chunk_start", C.c_int)]


class _KStat(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("sampled", C.c_int64),
                ("sampled_ms", C.c_double), ("sampled_bytes", C.c_double)]


_PROGRESS_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_char_p, C.c_int64, C.c_int64)

_lib = None


def lib_path() -> str:
    return os.path.join(_HERE, _LIB_NAME)


def load_library():
    """Load libkgf.so from the package directory (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1109_1205_amd.build` "
                          "(there is no CPU fallback)")
    L = C.CDLL(path)
    P, I, I64, D = C.c_void_p, C.c_int, C.c_int64, C.c_double
    sig = {
        "kgf_create": (I, [C.POINTER(P), I, P]),
        "kgf_destroy": (None, [P]),
        "kgf_set_stream": (I, [P, P]),
        "kgf_last_error": (C.c_char_p, []),
        "kgf_version": (I, []),
        "kgf_model_create": (I, [P, C.POINTER(_ModelDesc), C.POINTER(P)]),
        "kgf_model_destroy": (None, [P]),
        "kgf_model_set_params": (I, [P, C.POINTER(_ModelDesc)]),
        "kgf_propagate_driven": (I, [P, P, P, P, I, I64, I, I, P, P, C.POINTER(_PropOpts)]),
        "kgf_greens2_neq": (I, [P, P, P, P, C.POINTER(_GsOpts), P, P, I, I, I, C.POINTER(_PropOpts), I, P,
                                C.POINTER(D)]),
        "kgf_bath_chain": (I, [P, I, D, D, I, D, P, P]),
        "kgf_necpt": (I, [P, I, I, I, D, D, P, P, P, P, P, P]),
        "kgf_bath_chain_contour": (I, [P, I, D, D, I, D, I, D, C.POINTER(_ContourFn)]),
        "kgf_necpt_contour": (I, [P, I, I, I, I, D, D, D, C.POINTER(_ContourFn), C.POINTER(_ContourFn), P, P, P,
                                  P]),
        "kgf_cluster_contour": (I, [P, I, I, I, P, P, P, P, P, P, I, I, C.POINTER(_ContourFn)]),
        "kgf_greens_neq_driven": (I, [P, P, P, P, C.POINTER(_GsOpts), P, P, I, I, I, C.POINTER(_PropOpts), I, I,
                                      P, P, P, P, C.POINTER(D)]),
        "kgf_sector_create": (I, [P, I, I, I, C.POINTER(P)]),
        "kgf_sector_destroy": (None, [P]),
        "kgf_sector_dims": (I, [P, C.POINTER(I64), C.POINTER(I64)]),
        "kgf_sector_states": (I, [P, P, I, P]),
        "kgf_sector_rank": (I, [P, P, I, P, I64, P]),
        "kgf_hop_table": (I, [P, P, I, P, P, C.POINTER(I)]),
        "kgf_apply_h": (I, [P, P, P, P, P, I, I64]),
        "kgf_apply_c": (I, [P, P, P, I, I, P, P, I, I64, I64]),
        "kgf_ground_state": (I, [P, P, P, C.POINTER(_GsOpts), P, P, C.POINTER(D), C.POINTER(_GsInfo)]),
        "kgf_propagate": (I, [P, P, P, P, I, I64, I, C.POINTER(_PropOpts), C.POINTER(D), C.POINTER(D)]),
        "kgf_propagate_noalloc": (I, [P, P, P, P, I, I64, I, C.POINTER(_PropOpts), C.POINTER(D)]),
        "kgf_model_get_params": (I, [P, P, P, P, P]),
        "kgf_greens_eq": (I, [P, P, P, P, D, P, I, I, I, C.POINTER(_PropOpts), I, P, P]),
        "kgf_greens_neq": (I, [P, P, P, P, C.POINTER(_GsOpts), P, P, I, I, I, C.POINTER(_PropOpts), I, I,
                               I, I, D, P, P, P, P, P, C.POINTER(D), P]),
        "kgf_neq_run_create": (I, [P, P, P, P, C.POINTER(_GsOpts), P, P, I, I, I, C.POINTER(_PropOpts), I,
                                   C.POINTER(P), C.POINTER(D)]),
        "kgf_neq_run_advance": (I, [P, I, C.POINTER(_RunInfo)]),
        "kgf_neq_run_result": (I, [P, P, P]),
        "kgf_neq_run_destroy": (None, [P]),
        "kgf_neq_run_checkpoint": (I, [P, P, C.c_size_t, C.POINTER(C.c_size_t)]),
        "kgf_neq_run_restore": (I, [P, P, C.c_size_t]),
        "kgf_set_progress": (I, [P, _PROGRESS_FN, P]),
        "kgf_set_option": (I, [P, I, I]),
        "kgf_greens_omega": (I, [P, P, P, P, D, I, I, I, P, I, D, P, P, P]),
        "kgf_greens_eq_fine": (I, [P, P, P, P, D, I, I, I, I, C.POINTER(_PropOpts), P]),
        "kgf_fourier": (I, [P, P, I, D, D, P, I, P]),
        "kgf_greens_neq_vjp_multi": (I, [P, I, P, P, P, C.POINTER(_GsOpts), P, P, I, I, I, C.POINTER(_PropOpts), P, P,
                                         I, D, P, P, P, P]),
        "kgf_greens_neq_multi": (I, [P, I, P, P, P, P, C.POINTER(_GsOpts), P, I, I, I, C.POINTER(_PropOpts), I, P, P,
                                     P]),
        "kgf_n_theta": (I, [P]),
        "kgf_dH_expect": (I, [P, P, P, P, P, I, I64, P, P]),
        "kgf_propagate_vjp": (I, [P, P, P, P, P, I, C.POINTER(_PropOpts), I, P]),
        "kgf_greens_neq_vjp": (I, [P, P, P, P, C.POINTER(_GsOpts), P, P, I, I, I, C.POINTER(_PropOpts), P, P, I, D,
                                   P, P, P, P, C.POINTER(D), C.POINTER(I)]),
        "kgf_profile_begin": (I, [P, I]),
        "kgf_profile_end": (I, [P, C.POINTER(_KStat), I]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    if L.kgf_version() != ABI_VERSION:
        raise ImportError(f"{path} has ABI version {L.kgf_version()}, this binding expects {ABI_VERSION}: "
                          "rebuild it with `python -m paper_1109_1205_amd.build`")
    _lib = L
    return L


def exported_symbols() -> Sequence[str]:
    return ["kgf_create", "kgf_destroy", "kgf_set_stream", "kgf_last_error", "kgf_version",
            "kgf_model_create", "kgf_model_destroy", "kgf_sector_create", "kgf_sector_destroy",
            "kgf_sector_dims", "kgf_sector_states", "kgf_sector_rank", "kgf_hop_table",
            "kgf_apply_h", "kgf_apply_c", "kgf_ground_state", "kgf_propagate", "kgf_greens_eq",
            "kgf_greens_neq", "kgf_set_progress", "kgf_n_theta", "kgf_dH_expect", "kgf_propagate_vjp",
            "kgf_greens_neq_vjp", "kgf_set_option", "kgf_greens_neq_multi", "kgf_greens_neq_vjp_multi", "kgf_greens_omega", "kgf_greens_eq_fine", "kgf_fourier", "kgf_model_set_params",
            "kgf_propagate_driven", "kgf_greens_neq_driven", "kgf_bath_chain", "kgf_necpt", "kgf_bath_chain_contour", "kgf_necpt_contour", "kgf_cluster_contour", "kgf_greens2_neq",
            "kgf_neq_run_create", "kgf_neq_run_advance", "kgf_neq_run_result", "kgf_neq_run_destroy",
            "kgf_neq_run_checkpoint", "kgf_neq_run_restore",
            "kgf_propagate_noalloc", "kgf_model_get_params",
            "kgf_profile_begin",
            "kgf_profile_end"]


def _check(rc: int):
    if rc < 0:
        msg = _lib.kgf_last_error()
        raise KgfError(rc, msg.decode() if msg else "")
    return rc


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _host_c128(shape):
    return np.zeros(shape, dtype=np.complex128)


def _np_ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Model:
    """Handle of the model parameters (see include/kgf.h)."""

    def __init__(self, ctx: "Context", L: int, bonds, t, eps_up, eps_dn, U):
        self.ctx = ctx
        self.L = int(L)
        b = np.ascontiguousarray(np.asarray(bonds, dtype=np.int32).reshape(-1, 2))
        self._bi = np.ascontiguousarray(b[:, 0])
        self._bj = np.ascontiguousarray(b[:, 1])
        self._t = np.ascontiguousarray(np.asarray(t, dtype=np.float64).reshape(-1))
        self._eu = np.ascontiguousarray(np.asarray(eps_up, dtype=np.float64).reshape(-1))
        self._ed = np.ascontiguousarray(np.asarray(eps_dn, dtype=np.float64).reshape(-1))
        self._U = np.ascontiguousarray(np.asarray(U, dtype=np.float64).reshape(-1))
        if not (len(self._eu) == len(self._ed) == len(self._U) == self.L) or len(self._t) != len(self._bi):
            raise ValueError("model arrays have inconsistent sizes")
        d = _ModelDesc(self.L, len(self._bi),
                       self._bi.ctypes.data_as(C.POINTER(C.c_int32)), self._bj.ctypes.data_as(C.POINTER(C.c_int32)),
                       self._t.ctypes.data_as(C.POINTER(C.c_double)), self._eu.ctypes.data_as(C.POINTER(C.c_double)),
                       self._ed.ctypes.data_as(C.POINTER(C.c_double)), self._U.ctypes.data_as(C.POINTER(C.c_double)))
        h = C.c_void_p()
        _check(_lib.kgf_model_create(ctx.handle, C.byref(d), C.byref(h)))
        self.handle = h

    def _desc(self):
        return _ModelDesc(self.L, len(self._bi),
                          self._bi.ctypes.data_as(C.POINTER(C.c_int32)), self._bj.ctypes.data_as(C.POINTER(C.c_int32)),
                          self._t.ctypes.data_as(C.POINTER(C.c_double)), self._eu.ctypes.data_as(C.POINTER(C.c_double)),
                          self._ed.ctypes.data_as(C.POINTER(C.c_double)), self._U.ctypes.data_as(C.POINTER(C.c_double)))

    @property
    def theta(self) -> np.ndarray:
        """The parameter vector (t_b, eps_up, eps_dn, U)."""
        return np.concatenate([self._t, self._eu, self._ed, self._U])

    def set_params(self, t, eps_up, eps_dn, U) -> None:
        """kgf_model_set_params: new parameters on the same sites and bonds."""
        arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1)) for a in (t, eps_up, eps_dn, U)]
        if len(arrs[0]) != len(self._bi) or any(len(a) != self.L for a in arrs[1:]):
            raise ValueError("set_params: arrays do not match the model's bonds and sites")
        old = (self._t, self._eu, self._ed, self._U)
        self._t, self._eu, self._ed, self._U = arrs
        try:
            _check(_lib.kgf_model_set_params(self.handle, C.byref(self._desc())))
        except Exception:
            self._t, self._eu, self._ed, self._U = old
            raise

    def device_params(self):
        """kgf_model_get_params: the parameters the library holds (t, eps_up,
        eps_dn, U) -- after a driven propagation, the last stage's."""
        nb = len(self._bi)
        t, eu, ed, U = (np.zeros(max(n, 1)) for n in (nb, self.L, self.L, self.L))
        _check(_lib.kgf_model_get_params(self.handle, _np_ptr(t), _np_ptr(eu), _np_ptr(ed), _np_ptr(U)))
        return t[:nb], eu, ed, U

    def _sync_params(self):
        # mirror the library's copy after calls that replace the parameters in place
        self._t, self._eu, self._ed, self._U = (np.ascontiguousarray(a.copy()) for a in self.device_params())

    @classmethod
    def from_spec(cls, ctx: "Context", spec) -> "Model":
        """From any object with L, bonds, t, eps_up, eps_dn, U attributes."""
        return cls(ctx, spec.L, spec.bonds if len(spec.bonds) else np.zeros((0, 2)), spec.t,
                   spec.eps_up, spec.eps_dn, spec.U)

    def close(self):
        # The native destroy synchronises on the context's stream, so it must
        # run while the context exists; at interpreter shutdown (or when a
        # traceback keeps handles in a reference cycle) finalisers may run in
        # any order, and a handle whose context is gone is left to the process.
        if getattr(self, "handle", None):
            if getattr(self.ctx, "handle", None):
                _lib.kgf_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Sector:
    """Handle of a (L, N_up, N_dn) sector basis built on the device."""

    def __init__(self, ctx: "Context", L: int, n_up: int, n_dn: int):
        self.ctx = ctx
        self.L, self.n_up, self.n_dn = int(L), int(n_up), int(n_dn)
        h = C.c_void_p()
        _check(_lib.kgf_sector_create(ctx.handle, self.L, self.n_up, self.n_dn, C.byref(h)))
        self.handle = h
        du, dd = C.c_int64(), C.c_int64()
        _check(_lib.kgf_sector_dims(h, C.byref(du), C.byref(dd)))
        self.d_up, self.d_dn = du.value, dd.value

    @property
    def dim(self) -> int:
        return self.d_up * self.d_dn

    def states(self, spin: int) -> np.ndarray:
        n = self.d_up if spin == 0 else self.d_dn
        out = np.zeros(max(n, 1), dtype=np.uint32)
        _check(_lib.kgf_sector_states(self.ctx.handle, self.handle, int(spin), _np_ptr(out)))
        return out[:n]

    def rank(self, spin: int, masks) -> "object":
        """Combinatorial rank of device uint32 masks (torch.int32 tensor
        reinterpreted) into a device int64 tensor."""
        import torch
        out = torch.empty(masks.numel(), dtype=torch.int64, device=masks.device)
        _check(_lib.kgf_sector_rank(self.ctx.handle, self.handle, int(spin), _ptr(masks), masks.numel(), _ptr(out)))
        return out

    def close(self):
        # see Model.close: only while the context exists
        if getattr(self, "handle", None):
            if getattr(self.ctx, "handle", None):
                _lib.kgf_sector_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class NeqRun:
    """Handle of a step-wise four-step run (kgf_neq_run_*): steps (i), (ii) at
    creation, steps (iii), (iv) one mesh interval per advance()."""

    def __init__(self, ctx: "Context", handle, E0: float, nt: int, n_orb: int):
        self.ctx, self.handle, self.E0, self.nt, self.n_orb = ctx, handle, E0, nt, n_orb

    def advance(self, n_intervals: int = 1) -> dict:
        info = _RunInfo()
        _check(_lib.kgf_neq_run_advance(self.handle, int(n_intervals), C.byref(info)))
        return {k: getattr(info, k) for k, _ in _RunInfo._fields_}

    def result(self):
        shape = (self.nt, self.nt, self.n_orb, self.n_orb)
        Gl, Gg = _host_c128(shape), _host_c128(shape)
        _check(_lib.kgf_neq_run_result(self.handle, _np_ptr(Gl), _np_ptr(Gg)))
        return {"G_lesser": Gl, "G_greater": Gg, "E0": self.E0}

    def checkpoint(self) -> bytes:
        """kgf_neq_run_checkpoint: the run's progress as bytes (between chunks)."""
        need = C.c_size_t(0)
        _check(_lib.kgf_neq_run_checkpoint(self.handle, None, 0, C.byref(need)))
        buf = C.create_string_buffer(need.value)
        _check(_lib.kgf_neq_run_checkpoint(self.handle, buf, need.value, C.byref(need)))
        return buf.raw[:need.value]

    def restore(self, image: bytes) -> None:
        """kgf_neq_run_restore: continue a saved run (on a run just created
        from the same inputs)."""
        buf = C.create_string_buffer(bytes(image), len(image))
        _check(_lib.kgf_neq_run_restore(self.handle, buf, len(image)))

    def close(self):
        # see Model.close: only while the context exists
        if getattr(self, "handle", None):
            if getattr(self.ctx, "handle", None):
                _lib.kgf_neq_run_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _prop(krylov_dim, reorth, dt, direction, shift, breakdown_tol):
    return _PropOpts(int(krylov_dim), int(reorth), float(dt), int(direction), float(shift), float(breakdown_tol))


class Context:
    """A libkgf context bound to one HIP device and torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        load_library()
        self.device = int(device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self._stream = stream
        h = C.c_void_p()
        _check(_lib.kgf_create(C.byref(h), self.device, C.c_void_p(stream.cuda_stream)))
        self.handle = h

    # -- handles ---------------------------------------------------------
    def model(self, spec=None, **kw) -> Model:
        return Model.from_spec(self, spec) if spec is not None else Model(self, **kw)

    def sector(self, L: int, n_up: int, n_dn: int) -> Sector:
        return Sector(self, L, n_up, n_dn)

    def close(self):
        if getattr(self, "handle", None):
            _lib.kgf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- tensors ---------------------------------------------------------
    def _chk(self, t, n: int, name: str):
        import torch
        if t.dtype != torch.complex128 or not t.is_cuda or t.device.index != self.device:
            raise ValueError(f"{name} must be a complex128 tensor on cuda:{self.device}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.numel() % n:
            raise ValueError(f"{name} has {t.numel()} elements, not a multiple of {n}")
        return t.numel() // n

    def empty(self, *shape):
        import torch
        return torch.empty(*shape, dtype=torch.complex128, device=f"cuda:{self.device}")

    # -- calls -------------------------------------------------------------
    def hop_table(self, model: Model, n: int):
        from math import comb
        D = comb(model.L, n)
        width = C.c_int()
        cnt = np.zeros(max(D, 1), dtype=np.int32)
        ent = np.zeros(max(D * max(len(model._bi), 1), 1), dtype=np.uint32)
        _check(_lib.kgf_hop_table(self.handle, model.handle, int(n), _np_ptr(cnt), _np_ptr(ent), C.byref(width)))
        w = width.value
        return cnt[:D], ent[:D * w].reshape(w, D), w

    def apply_h(self, model: Model, sec: Sector, v, out=None):
        nvec = self._chk(v, sec.dim, "v")
        out = self.empty(*v.shape) if out is None else out
        self._chk(out, sec.dim, "out")
        _check(_lib.kgf_apply_h(self.handle, model.handle, sec.handle, _ptr(v), _ptr(out), nvec, sec.dim))
        return out

    def apply_c(self, src: Sector, dst: Sector, site: int, spin: int, dagger: bool, v, out=None):
        nvec = self._chk(v, src.dim, "v") if src.dim else (v.shape[0] if v.dim() > 1 else 1)
        shape = (nvec, dst.dim) if v.dim() > 1 else (dst.dim,)
        out = self.empty(*shape) if out is None else out
        self._chk(out, dst.dim, "out")
        _check(_lib.kgf_apply_c(self.handle, src.handle, dst.handle, 2 * int(site) + int(spin), int(bool(dagger)),
                                _ptr(v), _ptr(out), nvec, max(src.dim, 1), dst.dim))
        return out

    def ground_state(self, model: Model, sec: Sector, v0, tol=1e-12, max_iter=300, check_every=1, reorth=2,
                     out=None, allow_unconverged=False, unique_check=False, unique_tol=0.0, unique_seed=8):
        """kgf_ground_state; with unique_check a second start (SplitMix64,
        unique_seed) tests the uniqueness of |0> (KgfError KGF_EDEGENERATE
        when the two Ritz vectors differ)."""
        self._chk(v0, sec.dim, "v0")
        out = self.empty(sec.dim) if out is None else out
        E0 = C.c_double()
        info = _GsInfo()
        rc = _lib.kgf_ground_state(self.handle, model.handle, sec.handle,
                                   C.byref(_gs(tol, max_iter, check_every, reorth, unique_check, unique_tol,
                                               unique_seed)),
                                   _ptr(v0), _ptr(out), C.byref(E0), C.byref(info))
        if rc == -4 and allow_unconverged:
            pass
        else:
            _check(rc)
        return E0.value, out, {"iters": info.iters, "converged": bool(info.converged), "residual": info.residual,
                               "fidelity2": info.fidelity2}

    def propagate(self, model: Model, sec: Sector, psi, nsteps: int, dt: float, krylov_dim: int = 15,
                  direction: int = DIRECTION_FORWARD, shift: float = 0.0, reorth: int = 0,
                  breakdown_tol: float = 1e-13, return_err: bool = False, return_drift: bool = False):
        """kgf_propagate; with return_err also the largest per-step a-posteriori
        error estimate, with return_drift the largest per-step norm drift
        | ||psi after|| / ||psi before|| - 1 | (returns (psi, err), (psi, drift)
        or (psi, err, drift))."""
        nvec = self._chk(psi, sec.dim, "psi")
        o = _prop(krylov_dim, reorth, dt, direction, shift, breakdown_tol)
        err = C.c_double()
        drift = C.c_double()
        _check(_lib.kgf_propagate(self.handle, model.handle, sec.handle, _ptr(psi), nvec, sec.dim, int(nsteps),
                                  C.byref(o), C.byref(err) if return_err else None,
                                  C.byref(drift) if return_drift else None))
        extra = ([err.value] if return_err else []) + ([drift.value] if return_drift else [])
        return (psi, *extra) if extra else psi

    def propagate_noalloc(self, model: Model, sec: Sector, psi, nsteps: int, dt: float, krylov_dim: int = 15,
                          direction: int = DIRECTION_FORWARD, shift: float = 0.0, reorth: int = 0,
                          breakdown_tol: float = 1e-13):
        """kgf_propagate_noalloc: propagate() with every device buffer in the
        library's fixed per-GPU scratch (no allocation)."""
        nvec = self._chk(psi, sec.dim, "psi")
        o = _prop(krylov_dim, reorth, dt, direction, shift, breakdown_tol)
        _check(_lib.kgf_propagate_noalloc(self.handle, model.handle, sec.handle, _ptr(psi), nvec, sec.dim,
                                          int(nsteps), C.byref(o), None))
        return psi

    # Gauss-Legendre nodes of the driven integrator, as fractions of a step
    DRIVE_NODES = (0.5 - np.sqrt(3.0) / 6.0, 0.5 + np.sqrt(3.0) / 6.0)

    def propagate_driven(self, work: Model, sec: Sector, psi, thetas, f, nsteps: int, dt: float, t0: float = 0.0,
                         krylov_dim: int = 15, reorth: int = 0, breakdown_tol: float = 1e-13):
        """kgf_propagate_driven: psi (device, [nvec, D] or [D]) advanced under
        H(t) = sum_j f(t)[j] H(thetas[j]) from t0 in nsteps steps of dt (fourth-
        order commutator-free integrator).  thetas: [n_terms, n_theta] parameter
        vectors on the bonds of `work`; f(t) returns the n_terms drive values;
        `work` holds the last stage's parameters afterwards."""
        nvec = self._chk(psi, sec.dim, "psi")
        th, fv = self._drive_table(work, thetas, f, nsteps, dt, t0)
        o = _prop(krylov_dim, reorth, dt, DIRECTION_FORWARD, 0.0, breakdown_tol)
        _check(_lib.kgf_propagate_driven(self.handle, work.handle, sec.handle, _ptr(psi), nvec, sec.dim, int(nsteps),
                                         th.shape[0], _np_ptr(th), _np_ptr(fv), C.byref(o)))
        work._sync_params()
        return psi

    def _drive_table(self, work: Model, thetas, f, nsteps: int, dt: float, t0: float):
        """[n_terms, n_theta] parameter vectors and the drive values at the
        two Gauss nodes of each step, [nsteps, 2, n_terms]."""
        th = np.ascontiguousarray(np.asarray(thetas, dtype=np.float64))
        if th.ndim == 1:
            th = th.reshape(1, -1)
        n_terms = th.shape[0]
        if th.shape[1] != len(work._bi) + 3 * work.L:
            raise ValueError("driven: thetas must have n_bonds + 3 L columns")
        fv = np.empty((max(int(nsteps), 1), 2, n_terms))
        for n in range(int(nsteps)):
            for q, c in enumerate(self.DRIVE_NODES):
                fv[n, q] = np.asarray(f(t0 + (n + c) * dt), dtype=np.float64).reshape(n_terms)
        if nsteps <= 0:
            fv[:] = 0.0
        return th, np.ascontiguousarray(fv)

    def greens_neq_driven(self, H_ini: Model, work: Model, sec: Sector, v0, orbitals: Sequence[Tuple[int, int]],
                          thetas, f, nt: int, steps_per_grid: int, dt: float, krylov_dim: int = 15, reorth: int = 0,
                          batch: int = 0, gs_tol: float = 1e-12, gs_max_iter: int = 300, gs_check_every: int = 1,
                          gs_reorth: int = 2, gs_unique_check: bool = False, breakdown_tol: float = 1e-13):
        """kgf_greens_neq_driven: four-step G^<, G^> [nt, nt, n_orb, n_orb] after
        the ground state of H_ini, under H(t) = sum_j f(t)[j] H(thetas[j]) from
        t = 0 (steps of dt, steps_per_grid per mesh interval).  `work` (not
        H_ini) holds the last stage's parameters afterwards."""
        self._chk(v0, sec.dim, "v0")
        if work is H_ini:
            raise ValueError("greens_neq_driven: work must not be H_ini")
        nsteps = (int(nt) - 1) * int(steps_per_grid)
        th, fv = self._drive_table(work, thetas, f, nsteps, dt, 0.0)
        orbs = np.ascontiguousarray([2 * s + sp for s, sp in orbitals], dtype=np.int32)
        no = len(orbs)
        Gl = _host_c128((nt, nt, no, no))
        Gg = _host_c128((nt, nt, no, no))
        E0 = C.c_double()
        o = _prop(krylov_dim, reorth, dt, DIRECTION_FORWARD, 0.0, breakdown_tol)
        g = _gs(gs_tol, gs_max_iter, gs_check_every, gs_reorth, gs_unique_check)
        _check(_lib.kgf_greens_neq_driven(self.handle, H_ini.handle, work.handle, sec.handle, C.byref(g), _ptr(v0),
                                          _np_ptr(orbs), no, int(nt), int(steps_per_grid), C.byref(o), int(batch),
                                          th.shape[0], _np_ptr(th), _np_ptr(fv), _np_ptr(Gl), _np_ptr(Gg),
                                          C.byref(E0)))
        work._sync_params()
        return {"G_lesser": Gl, "G_greater": Gg, "E0": E0.value}

    def greens_eq(self, model: Model, sec: Sector, psi0, E0: float, orbitals: Sequence[Tuple[int, int]],
                  nt: int, steps_per_grid: int, dt: float, krylov_dim: int = 15, reorth: int = 0,
                  batch: int = 0, breakdown_tol: float = 1e-13):
        self._chk(psi0, sec.dim, "psi0")
        orbs = np.ascontiguousarray([2 * s + sp for s, sp in orbitals], dtype=np.int32)
        no = len(orbs)
        Gg = _host_c128((nt, no, no))
        Gl = _host_c128((nt, no, no))
        o = _prop(krylov_dim, reorth, dt, DIRECTION_FORWARD, 0.0, breakdown_tol)
        _check(_lib.kgf_greens_eq(self.handle, model.handle, sec.handle, _ptr(psi0), float(E0), _np_ptr(orbs), no,
                                  int(nt), int(steps_per_grid), C.byref(o), int(batch), _np_ptr(Gg), _np_ptr(Gl)))
        return Gg, Gl

    def greens_neq(self, H_ini: Model, H: Model, sec: Sector, v0, orbitals: Sequence[Tuple[int, int]], nt: int,
                   steps_per_grid: int, dt: float, krylov_dim: int = 15, reorth: int = 0, schedule: int = 1,
                   batch: int = 0, ntau: int = 0, tau_steps_per_grid: int = 1, dtau: float = 0.0,
                   gs_tol: float = 1e-12, gs_max_iter: int = 300, gs_check_every: int = 1, gs_reorth: int = 2, gs_unique_check: bool = False,
                   breakdown_tol: float = 1e-13, psi0_out=None):
        self._chk(v0, sec.dim, "v0")
        if psi0_out is not None:
            self._chk(psi0_out, sec.dim, "psi0_out")
        orbs = np.ascontiguousarray([2 * s + sp for s, sp in orbitals], dtype=np.int32)
        no = len(orbs)
        Gl = _host_c128((nt, nt, no, no))
        Gg = _host_c128((nt, nt, no, no))
        GM = _host_c128((2, ntau, no, no)) if ntau > 0 else None
        Gx = _host_c128((nt, ntau, no, no)) if ntau > 0 else None
        Gxl = _host_c128((ntau, nt, no, no)) if ntau > 0 else None
        E0 = C.c_double()
        o = _prop(krylov_dim, reorth, dt, DIRECTION_FORWARD, 0.0, breakdown_tol)
        g = _gs(gs_tol, gs_max_iter, gs_check_every, gs_reorth, gs_unique_check)
        _check(_lib.kgf_greens_neq(self.handle, H_ini.handle, H.handle, sec.handle, C.byref(g), _ptr(v0),
                                   _np_ptr(orbs), no, int(nt), int(steps_per_grid), C.byref(o), int(schedule),
                                   int(batch), int(ntau), int(tau_steps_per_grid), float(dtau), _np_ptr(Gl),
                                   _np_ptr(Gg), _np_ptr(GM), _np_ptr(Gx), _np_ptr(Gxl), C.byref(E0),
                                   _ptr(psi0_out)))
        out = {"G_lesser": Gl, "G_greater": Gg, "E0": E0.value}
        if ntau > 0:
            out["G_matsubara"] = GM
            out["G_mixed"] = Gx
            out["G_mixed_left"] = Gxl
        return out

    def neq_run(self, H_ini: Model, H: Model, sec: Sector, v0, orbitals: Sequence[Tuple[int, int]], nt: int,
                steps_per_grid: int, dt: float, krylov_dim: int = 15, reorth: int = 0, batch: int = 0,
                gs_tol: float = 1e-12, gs_max_iter: int = 300, gs_check_every: int = 1, gs_reorth: int = 2, gs_unique_check: bool = False,
                breakdown_tol: float = 1e-13) -> NeqRun:
        """kgf_neq_run_create: ground state and forward mesh of the four-step
        procedure; the returned run advances the backward sweeps."""
        self._chk(v0, sec.dim, "v0")
        orbs = np.ascontiguousarray([2 * s + sp for s, sp in orbitals], dtype=np.int32)
        E0 = C.c_double()
        h = C.c_void_p()
        o = _prop(krylov_dim, reorth, dt, DIRECTION_FORWARD, 0.0, breakdown_tol)
        g = _gs(gs_tol, gs_max_iter, gs_check_every, gs_reorth, gs_unique_check)
        _check(_lib.kgf_neq_run_create(self.handle, H_ini.handle, H.handle, sec.handle, C.byref(g), _ptr(v0),
                                       _np_ptr(orbs), len(orbs), int(nt), int(steps_per_grid), C.byref(o), int(batch),
                                       C.byref(h), C.byref(E0)))
        return NeqRun(self, h, E0.value, int(nt), len(orbs))

    def greens_neq_multi(self, H_ini: Sequence[Model], H: Sequence[Model], secs: Sequence[Sector], v0s,
                         orbitals: Sequence[Tuple[int, int]], nt: int, steps_per_grid: int, dt: float,
                         krylov_dim: int = 15, reorth: int = 0, batch: int = 0, gs_tol: float = 1e-12,
                         gs_max_iter: int = 300, gs_check_every: int = 1, gs_reorth: int = 2, gs_unique_check: bool = False,
                         breakdown_tol: float = 1e-13):
        """kgf_greens_neq_multi: four-step G^<, G^> of many instances in one call
        (same-sector, same-topology instances batched).  Returns G_lesser,
        G_greater [n][nt][nt][n_orb][n_orb] and E0 [n]."""
        n = len(H)
        assert len(H_ini) == n and len(secs) == n and len(v0s) == n
        for v, s_ in zip(v0s, secs):
            self._chk(v, s_.dim, "v0")
        orbs = np.ascontiguousarray([2 * s_ + sp for s_, sp in orbitals], dtype=np.int32)
        no = len(orbs)
        Gl = _host_c128((n, nt, nt, no, no))
        Gg = _host_c128((n, nt, nt, no, no))
        E0 = np.zeros(n)
        def arr(xs):
            return (C.c_void_p * n)(*[(x.value if isinstance(x, C.c_void_p) else int(x)) for x in xs])
        o = _prop(krylov_dim, reorth, dt, DIRECTION_FORWARD, 0.0, breakdown_tol)
        g = _gs(gs_tol, gs_max_iter, gs_check_every, gs_reorth, gs_unique_check)
        _check(_lib.kgf_greens_neq_multi(self.handle, n, arr(m.handle for m in H_ini), arr(m.handle for m in H),
                                         arr(s_.handle for s_ in secs), arr(_ptr(v) for v in v0s), C.byref(g),
                                         _np_ptr(orbs), no, int(nt), int(steps_per_grid), C.byref(o), int(batch),
                                         _np_ptr(Gl), _np_ptr(Gg), _np_ptr(E0)))
        return {"G_lesser": Gl, "G_greater": Gg, "E0": E0}

    def greens2_neq(self, H_ini: Model, H: Model, sec: Sector, v0, orbitals: Sequence[Tuple[int, int]], nt: int,
                    steps_per_grid: int, dt: float, pattern=(1, 1, 0, 0), krylov_dim: int = 15, reorth: int = 0,
                    gs_tol: float = 1e-12, gs_max_iter: int = 300, gs_check_every: int = 1, gs_reorth: int = 2, gs_unique_check: bool = False,
                    breakdown_tol: float = 1e-13):
        """kgf_greens2_neq: chi[k1, k2, k3, k4, a, b, c, d] =
        <0| O1_a(t_k1) O2_b(t_k2) O3_c(t_k3) O4_d(t_k4) |0> after the ground
        state of H_ini, t_k = k * steps_per_grid * dt, O_m = c+ where
        pattern[m] else c (default c+ c+ c c).  Returns chi and E0."""
        self._chk(v0, sec.dim, "v0")
        bits = sum(int(bool(q)) << (3 - m) for m, q in enumerate(pattern))
        orbs = np.ascontiguousarray([2 * s + sp for s, sp in orbitals], dtype=np.int32)
        no = len(orbs)
        chi = _host_c128((nt, nt, nt, nt, no, no, no, no))
        E0 = C.c_double()
        o = _prop(krylov_dim, reorth, dt, DIRECTION_FORWARD, 0.0, breakdown_tol)
        g = _gs(gs_tol, gs_max_iter, gs_check_every, gs_reorth, gs_unique_check)
        _check(_lib.kgf_greens2_neq(self.handle, H_ini.handle, H.handle, sec.handle, C.byref(g), _ptr(v0),
                                    _np_ptr(orbs), no, int(nt), int(steps_per_grid), C.byref(o), bits,
                                    _np_ptr(chi), C.byref(E0)))
        return {"chi": chi, "E0": E0.value}

    # -- nonequilibrium cluster-perturbation theory ---------------------------
    def bath_chain(self, L_b: int, T_b: float, nt: int, dt: float, beta: float = float("inf")):
        """kgf_bath_chain: (G^<, G^>) [nt, nt] device tensors of the first site
        of an L_b-site chain with hopping -T_b (Eqs. (gb1), (gb2))."""
        import torch
        Gl = torch.empty((nt, nt), dtype=torch.complex128, device=f"cuda:{self.device}")
        Gg = torch.empty_like(Gl)
        _check(_lib.kgf_bath_chain(self.handle, int(L_b), float(T_b), float(beta), int(nt), float(dt), _ptr(Gl),
                                   _ptr(Gg)))
        return Gl, Gg

    def necpt(self, Gc_lesser, Gc_greater, Gb_lesser, Gb_greater, boundary: int, V: float, dt: float):
        """kgf_necpt: cluster block (G^<, G^>) [nt, nt, n_c, n_c] of the CPT
        equation on the Keldysh contour; inputs are contiguous complex128
        device tensors (cluster [nt, nt, n_c, n_c], bath [nt, nt])."""
        import torch
        nt, n_c = int(Gc_lesser.shape[0]), int(Gc_lesser.shape[2])
        for x, shp in ((Gc_lesser, (nt, nt, n_c, n_c)), (Gc_greater, (nt, nt, n_c, n_c)), (Gb_lesser, (nt, nt)),
                       (Gb_greater, (nt, nt))):
            if (tuple(x.shape) != shp or x.dtype != torch.complex128 or not x.is_cuda or not x.is_contiguous()
                    or x.device.index != self.device):
                raise ValueError(f"necpt: expected a contiguous complex128 tensor of shape {shp} on cuda:{self.device}")
        Gl = torch.empty_like(Gc_lesser)
        Gg = torch.empty_like(Gc_lesser)
        _check(_lib.kgf_necpt(self.handle, nt, n_c, int(boundary), float(dt), float(V), _ptr(Gc_lesser),
                              _ptr(Gc_greater), _ptr(Gb_lesser), _ptr(Gb_greater), _ptr(Gl), _ptr(Gg)))
        return Gl, Gg

    def _contour_fn(self, fn: dict, nt: int, ntau: int, n: int):
        import torch
        shapes = {"lesser": (nt, nt), "greater": (nt, nt), "mixed": (nt, ntau), "mixed_left": (ntau, nt),
                  "vert_greater": (ntau,), "vert_lesser": (ntau,)}
        for k in CONTOUR_KEYS:
            x = fn[k]
            shp = shapes[k] + ((n, n) if n > 1 else ())
            if (tuple(x.shape) != shp or x.dtype != torch.complex128 or not x.is_cuda or not x.is_contiguous()
                    or x.device.index != self.device):
                raise ValueError(f"contour function: {k} must be a contiguous complex128 tensor of shape {shp} "
                                 f"on cuda:{self.device}")
        return _ContourFn(*[_ptr(fn[k]) for k in CONTOUR_KEYS])

    def bath_chain_contour(self, L_b: int, T_b: float, nt: int, dt: float, ntau: int, dtau: float,
                           beta: float = float("inf")):
        """kgf_bath_chain_contour: the components (device tensors; keys
        CONTOUR_KEYS) of the first site of an L_b-site chain on the contour with
        an imaginary branch of ntau points dtau apart."""
        import torch
        dev = f"cuda:{self.device}"
        out = {"lesser": torch.empty((nt, nt), dtype=torch.complex128, device=dev),
               "greater": torch.empty((nt, nt), dtype=torch.complex128, device=dev),
               "mixed": torch.empty((nt, ntau), dtype=torch.complex128, device=dev),
               "mixed_left": torch.empty((ntau, nt), dtype=torch.complex128, device=dev),
               "vert_greater": torch.empty((ntau,), dtype=torch.complex128, device=dev),
               "vert_lesser": torch.empty((ntau,), dtype=torch.complex128, device=dev)}
        f = self._contour_fn(out, nt, ntau, 1)
        _check(_lib.kgf_bath_chain_contour(self.handle, int(L_b), float(T_b), float(beta), int(nt), float(dt),
                                           int(ntau), float(dtau), C.byref(f)))
        return out

    def cluster_contour(self, four_step: dict, orbitals=None, kms: bool = True):
        """kgf_cluster_contour: a cluster's contour components (device tensors;
        keys CONTOUR_KEYS) from the output of greens_neq with ntau >= 2, for the
        orbital indices `orbitals` (positions in its orbital list; None: all);
        kms completes them for the imaginary branch of finite length."""
        import torch
        Gl = np.ascontiguousarray(four_step["G_lesser"], dtype=np.complex128)
        nt, n_orb = int(Gl.shape[0]), int(Gl.shape[2])
        GM = np.ascontiguousarray(four_step["G_matsubara"], dtype=np.complex128)
        ntau = int(GM.shape[1])
        arrs = [Gl, np.ascontiguousarray(four_step["G_greater"], dtype=np.complex128), GM,
                np.ascontiguousarray(four_step["G_mixed"], dtype=np.complex128),
                np.ascontiguousarray(four_step["G_mixed_left"], dtype=np.complex128)]
        shapes = [(nt, nt, n_orb, n_orb), (nt, nt, n_orb, n_orb), (2, ntau, n_orb, n_orb), (nt, ntau, n_orb, n_orb),
                  (ntau, nt, n_orb, n_orb)]
        for x, shp in zip(arrs, shapes):
            if tuple(x.shape) != shp:
                raise ValueError(f"cluster_contour: expected four-step components of shape {shp}")
        sel = np.ascontiguousarray(range(n_orb) if orbitals is None else orbitals, dtype=np.int32)
        n_c = int(sel.shape[0])
        dev = f"cuda:{self.device}"
        shp = {"lesser": (nt, nt), "greater": (nt, nt), "mixed": (nt, ntau), "mixed_left": (ntau, nt),
               "vert_greater": (ntau,), "vert_lesser": (ntau,)}
        out = {k: torch.empty(shp[k] + (n_c, n_c), dtype=torch.complex128, device=dev) for k in CONTOUR_KEYS}
        f = self._contour_fn(out, nt, ntau, n_c) if n_c > 1 else _ContourFn(*[_ptr(out[k]) for k in CONTOUR_KEYS])
        _check(_lib.kgf_cluster_contour(self.handle, nt, ntau, n_orb, *[_np_ptr(x) for x in arrs], _np_ptr(sel), n_c,
                                        1 if kms else 0, C.byref(f)))
        return out

    def necpt_contour(self, Gc: dict, Gb: dict, boundary: int, V: float, dt: float, dtau: float):
        """kgf_necpt_contour: cluster block of the CPT equation on the contour
        with its imaginary branch; Gc, Gb: components (CONTOUR_KEYS) as
        contiguous complex128 device tensors (cluster [..., n_c, n_c], bath
        site 1 [...]).  Returns G_lesser, G_greater, G_mixed, G_mixed_left."""
        import torch
        nt, n_c = int(Gc["lesser"].shape[0]), int(Gc["lesser"].shape[2])
        ntau = int(Gc["vert_greater"].shape[0])
        fc = self._contour_fn(Gc, nt, ntau, n_c)
        fb = self._contour_fn(Gb, nt, ntau, 1)
        dev = Gc["lesser"].device
        out = {"G_lesser": torch.empty_like(Gc["lesser"]), "G_greater": torch.empty_like(Gc["lesser"]),
               "G_mixed": torch.empty((nt, ntau, n_c, n_c), dtype=torch.complex128, device=dev),
               "G_mixed_left": torch.empty((ntau, nt, n_c, n_c), dtype=torch.complex128, device=dev)}
        _check(_lib.kgf_necpt_contour(self.handle, nt, ntau, n_c, int(boundary), float(dt), float(dtau), float(V),
                                      C.byref(fc), C.byref(fb), _ptr(out["G_lesser"]), _ptr(out["G_greater"]),
                                      _ptr(out["G_mixed"]), _ptr(out["G_mixed_left"])))
        return out

    # -- equilibrium spectra --------------------------------------------------
    def greens_omega(self, model: Model, sec: Sector, psi0, E0: float, orbital: Tuple[int, int], n_lanczos: int,
                     omega, eta: float, reorth: int = 2):
        """Conventional Lanczos G^(L)(omega) (kgf_greens_omega): particle and hole
        parts; the retarded G is their sum."""
        self._chk(psi0, sec.dim, "psi0")
        w = np.ascontiguousarray(np.asarray(omega, dtype=np.float64).reshape(-1))
        Gg, Gl = _host_c128(w.shape), _host_c128(w.shape)
        steps = np.zeros(2, dtype=np.int32)
        _check(_lib.kgf_greens_omega(self.handle, model.handle, sec.handle, _ptr(psi0), float(E0),
                                     2 * orbital[0] + orbital[1], int(n_lanczos), int(reorth), _np_ptr(w), len(w),
                                     float(eta), _np_ptr(Gg), _np_ptr(Gl), _np_ptr(steps)))
        return {"G_greater": Gg, "G_lesser": Gl, "steps": steps}

    def greens_eq_fine(self, model: Model, sec: Sector, psi0, E0: float, orbital: Tuple[int, int], dagger: int,
                       nsteps: int, nfine: int, dt: float, krylov_dim: int = 15, reorth: int = 0,
                       breakdown_tol: float = 1e-13):
        """Time-dependent Lanczos G^> (dagger=1) or G^< (dagger=0) on t_j = j dt / nfine."""
        self._chk(psi0, sec.dim, "psi0")
        G = _host_c128(nsteps * nfine + 1)
        o = _prop(krylov_dim, reorth, dt, DIRECTION_FORWARD, 0.0, breakdown_tol)
        _check(_lib.kgf_greens_eq_fine(self.handle, model.handle, sec.handle, _ptr(psi0), float(E0),
                                       2 * orbital[0] + orbital[1], int(dagger), int(nsteps), int(nfine), C.byref(o),
                                       _np_ptr(G)))
        return G

    def fourier(self, G, dt: float, eta: float, omega):
        """kgf_fourier: int_0^T dt e^{i omega t - eta t} G(t), trapezoid rule."""
        g = np.ascontiguousarray(np.asarray(G, dtype=np.complex128).reshape(-1))
        w = np.ascontiguousarray(np.asarray(omega, dtype=np.float64).reshape(-1))
        out = _host_c128(w.shape)
        _check(_lib.kgf_fourier(self.handle, _np_ptr(g), len(g), float(dt), float(eta), _np_ptr(w), len(w),
                                _np_ptr(out)))
        return out

    (HV_PASSES, HV_STRIP, GS_MAX_BASIS, PHI_EVERY, ADJ_EVERY, HV_TUNE, CG_MAX_ITER, GRAPHS, LOCKSTEP, HV_FUSE,
     HV_SEG, HV_UP_THREADS) = range(1, 13)

    def set_option(self, option: int, value: int) -> None:
        """kgf_set_option: HV_PASSES 0..4, HV_STRIP 0/8/16/32/64/128, GS_MAX_BASIS 0 or >= 8, PHI_EVERY >= 0,
        ADJ_EVERY >= 0, HV_TUNE 0/1, CG_MAX_ITER >= 0, GRAPHS 0/1, LOCKSTEP 0/1, HV_FUSE 0/1,
        HV_SEG 0/1, HV_UP_THREADS 256/512/1024."""
        _check(_lib.kgf_set_option(self.handle, int(option), int(value)))

    def set_progress(self, fn=None):
        """fn(phase: str, done: int, total: int) called from the library's
        drivers as mesh times complete; None disables."""
        if fn is None:
            self._progress_cb = None
            _check(_lib.kgf_set_progress(self.handle, _PROGRESS_FN(), None))
            return
        def cb(user, phase, done, total):
            try:
                fn(phase.decode(), int(done), int(total))
            except Exception:
                pass
        self._progress_cb = _PROGRESS_FN(cb)
        _check(_lib.kgf_set_progress(self.handle, self._progress_cb, None))

    # -- parameter derivatives / adjoint ------------------------------------
    def n_theta(self, model: Model) -> int:
        return _check(_lib.kgf_n_theta(model.handle))

    def dH_expect(self, model: Model, sec: Sector, lam, psi, weights):
        """sum_p Re(w_p <lam_p| dH/dtheta |psi_p>) for theta = (t_b, eps_up, eps_dn, U)."""
        npair = self._chk(lam, sec.dim, "lam")
        if self._chk(psi, sec.dim, "psi") != npair:
            raise ValueError("lam and psi hold different numbers of vectors")
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.complex128).reshape(-1))
        if len(w) != npair:
            raise ValueError("one weight per vector pair")
        g = np.zeros(self.n_theta(model), dtype=np.float64)
        _check(_lib.kgf_dH_expect(self.handle, model.handle, sec.handle, _ptr(lam), _ptr(psi), npair, sec.dim,
                                  _np_ptr(w), _np_ptr(g)))
        return g

    def propagate_vjp(self, model: Model, sec: Sector, psi0, lam, nsteps: int, dt: float, krylov_dim: int = 15,
                      direction: int = DIRECTION_FORWARD, reorth: int = 0, quad_nodes: int = 12,
                      breakdown_tol: float = 1e-13):
        """Adjoint of propagate(): lam (cotangent of the final state) is
        replaced in place by the cotangent of psi0; returns dL/dtheta."""
        self._chk(psi0, sec.dim, "psi0")
        self._chk(lam, sec.dim, "lam")
        g = np.zeros(self.n_theta(model), dtype=np.float64)
        o = _prop(krylov_dim, reorth, dt, direction, 0.0, breakdown_tol)
        _check(_lib.kgf_propagate_vjp(self.handle, model.handle, sec.handle, _ptr(psi0), _ptr(lam), int(nsteps),
                                      C.byref(o), int(quad_nodes), _np_ptr(g)))
        return g

    def greens_neq_vjp(self, H_ini: Model, H: Model, sec: Sector, v0, orbitals, nt: int, steps_per_grid: int,
                       dt: float, W_lesser=None, W_greater=None, krylov_dim: int = 15, reorth: int = 0,
                       quad_nodes: int = 12, cg_tol: float = 1e-12, gs_tol: float = 1e-12, gs_max_iter: int = 300,
                       gs_check_every: int = 1, gs_reorth: int = 2, gs_unique_check: bool = False, breakdown_tol: float = 1e-13):
        """dL/dtheta_ini and dL/dtheta for L = Re sum conj(W^<) G^< + Re sum conj(W^>) G^>."""
        self._chk(v0, sec.dim, "v0")
        orbs = np.ascontiguousarray([2 * s + sp for s, sp in orbitals], dtype=np.int32)
        no = len(orbs)
        shape = (nt, nt, no, no)
        Wl = None if W_lesser is None else np.ascontiguousarray(np.asarray(W_lesser, dtype=np.complex128).reshape(shape))
        Wg = None if W_greater is None else np.ascontiguousarray(np.asarray(W_greater, dtype=np.complex128).reshape(shape))
        gi = np.zeros(self.n_theta(H_ini), dtype=np.float64)
        g = np.zeros(self.n_theta(H), dtype=np.float64)
        Gl = _host_c128(shape)
        Gg = _host_c128(shape)
        E0 = C.c_double()
        cgi = C.c_int()
        o = _prop(krylov_dim, reorth, dt, DIRECTION_FORWARD, 0.0, breakdown_tol)
        gso = _gs(gs_tol, gs_max_iter, gs_check_every, gs_reorth, gs_unique_check)
        _check(_lib.kgf_greens_neq_vjp(self.handle, H_ini.handle, H.handle, sec.handle, C.byref(gso), _ptr(v0),
                                       _np_ptr(orbs), no, int(nt), int(steps_per_grid), C.byref(o), _np_ptr(Wl),
                                       _np_ptr(Wg), int(quad_nodes), float(cg_tol), _np_ptr(gi), _np_ptr(g),
                                       _np_ptr(Gl), _np_ptr(Gg), C.byref(E0), C.byref(cgi)))
        return {"grad_ini": gi, "grad": g, "G_lesser": Gl, "G_greater": Gg, "E0": E0.value,
                "cg_iters": cgi.value}

    def greens_neq_vjp_multi(self, H_ini: Sequence[Model], H: Sequence[Model], secs: Sequence[Sector], v0s, orbitals,
                             nt: int, steps_per_grid: int, dt: float, W_lesser=None, W_greater=None,
                             krylov_dim: int = 15, reorth: int = 0, quad_nodes: int = 12, cg_tol: float = 1e-12,
                             gs_tol: float = 1e-12, gs_max_iter: int = 300, gs_check_every: int = 1,
                             gs_reorth: int = 2, gs_unique_check: bool = False, breakdown_tol: float = 1e-13):
        """kgf_greens_neq_vjp_multi: gradients of n instances (same-sector,
        same-topology instances batched).  W_lesser / W_greater: sequences of
        [nt][nt][n_orb][n_orb] arrays (or None).  Returns a list of dicts."""
        n = len(H)
        for v, s_ in zip(v0s, secs):
            self._chk(v, s_.dim, "v0")
        orbs = np.ascontiguousarray([2 * s_ + sp for s_, sp in orbitals], dtype=np.int32)
        no = len(orbs)
        shape = (nt, nt, no, no)

        def arrs(W):
            if W is None:
                return None, []
            keep = [None if w is None else np.ascontiguousarray(np.asarray(w, dtype=np.complex128).reshape(shape))
                    for w in W]
            return (C.c_void_p * n)(*[(0 if w is None else w.ctypes.data) for w in keep]), keep
        Wl, keep_l = arrs(W_lesser)
        Wg, keep_g = arrs(W_greater)
        gi = [np.zeros(self.n_theta(m), dtype=np.float64) for m in H_ini]
        g = [np.zeros(self.n_theta(m), dtype=np.float64) for m in H]
        E0 = np.zeros(n)
        cgi = np.zeros(n, dtype=np.int32)

        def hv(xs):
            return (C.c_void_p * n)(*[(x.value if isinstance(x, C.c_void_p) else int(x)) for x in xs])
        o = _prop(krylov_dim, reorth, dt, DIRECTION_FORWARD, 0.0, breakdown_tol)
        gso = _gs(gs_tol, gs_max_iter, gs_check_every, gs_reorth, gs_unique_check)
        _check(_lib.kgf_greens_neq_vjp_multi(self.handle, n, hv(m.handle for m in H_ini), hv(m.handle for m in H),
                                             hv(s_.handle for s_ in secs), C.byref(gso), hv(_ptr(v) for v in v0s),
                                             _np_ptr(orbs), no, int(nt), int(steps_per_grid), C.byref(o), Wl, Wg,
                                             int(quad_nodes), float(cg_tol), hv(a.ctypes.data for a in gi),
                                             hv(a.ctypes.data for a in g), _np_ptr(E0), _np_ptr(cgi)))
        return [{"grad_ini": gi[i], "grad": g[i], "E0": float(E0[i]), "cg_iters": int(cgi[i])} for i in range(n)]

    def profile_begin(self, sample_every: int = 1):
        _check(_lib.kgf_profile_begin(self.handle, int(sample_every)))

    def profile_end(self):
        arr = (_KStat * 64)()
        n = _check(_lib.kgf_profile_end(self.handle, arr, 64))
        return {arr[i].name.decode(): {"launches": arr[i].launches, "sampled": arr[i].sampled,
                                       "sampled_ms": arr[i].sampled_ms, "sampled_bytes": arr[i].sampled_bytes}
                for i in range(n)}
