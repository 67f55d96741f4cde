"""ctypes binding of include/dg.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os
import threading
from math import comb

import numpy as np

DG_FP64 = 0
DG_FP32 = 1
DG_MIXED = 2
DG_BF16X3 = 3


class BatchItem(ctypes.Structure):
    """dg_batch_item of include/dg.h."""
    _fields_ = [("degree", ctypes.c_int), ("E", ctypes.c_int64), ("dt", ctypes.c_double),
                ("Q", ctypes.c_void_p), ("I", ctypes.c_void_p), ("traces", ctypes.c_void_p),
                ("star_packed", ctypes.c_void_p), ("Aplus", ctypes.c_void_p), ("Aminus", ctypes.c_void_p),
                ("neigh", ctypes.c_void_p), ("face_rot", ctypes.c_void_p), ("n_quant", ctypes.c_int),
                ("omega", ctypes.c_double * 3)]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBNAME = "libdg_mi355x.so"
_lock = threading.Lock()
_lib = None


class DGError(RuntimeError):
    pass


def library_path() -> str:
    return os.path.join(_HERE, _LIBNAME)


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        path = library_path()
        if not os.path.exists(path):
            raise DGError("HIP library %s is not built (run paper_1903_11521_amd/build.py); "
                          "there is no CPU fallback" % path)
        lib = ctypes.CDLL(path)
        vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
        dp = ctypes.POINTER(ctypes.c_double)
        lib.dg_last_error.restype = ctypes.c_char_p
        lib.dg_reference_blob_size.restype = i64
        lib.dg_reference_blob_size.argtypes = [i32]
        lib.dg_reference_matrices.argtypes = [i32, dp]
        lib.dg_element_data_host.argtypes = [i64, dp, dp, ctypes.POINTER(ctypes.c_int32), dp, dp, dp]
        lib.dg_visco_element_data_host.argtypes = [i64, dp, dp, dp, dp, dp, ctypes.POINTER(ctypes.c_int32), dp, dp,
                                                   dp]
        lib.dg_plan_create.argtypes = [i32, i32, ctypes.POINTER(vp)]
        lib.dg_plan_destroy.argtypes = [vp]
        lib.dg_plan_sizes.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        lib.dg_pack_star.argtypes = [vp, i64, vp, vp, vp]
        lib.dg_predictor.argtypes = [vp, i64, dbl, vp, vp, vp, vp]
        lib.dg_time_integral.argtypes = [vp, i64, dbl, vp, vp, vp]
        lib.dg_volume.argtypes = [vp, i64, vp, vp, vp, vp]
        lib.dg_local_flux.argtypes = [vp, i64, vp, vp, vp, vp]
        lib.dg_neighbour_flux.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp, vp]
        lib.dg_step.argtypes = [vp, i64, dbl, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.dg_step_fused.argtypes = [vp, i64, dbl, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.dg_step_noalloc.argtypes = [vp, i64, dbl, i32, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.dg_fused_step.argtypes = [vp, i64, dbl, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.dg_mra_apply.argtypes = [i32, i64, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.dg_plan_fuses_steps.argtypes = [vp]
        lib.dg_plan_tune.argtypes = [vp, i64, vp]
        lib.dg_plan_set_fusion.argtypes = [vp, i32]
        lib.dg_set_debug_checks.argtypes = [i32]
        lib.dg_step_predict.argtypes = [vp, i64, dbl, vp, vp, vp, vp, vp]
        lib.dg_step_correct.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.dg_sync.argtypes = [vp]
        lib.dg_batch_create.argtypes = [i32, ctypes.POINTER(BatchItem), i32, ctypes.POINTER(vp)]
        lib.dg_batch_step.argtypes = [vp, i32, vp]
        lib.dg_batch_update.argtypes = [vp, ctypes.POINTER(BatchItem), i32]
        lib.dg_batch_destroy.argtypes = [vp]
        lib.dg_lts_create.argtypes = [vp, i64, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), dbl,
                                      ctypes.POINTER(vp)]
        lib.dg_lts_clusters.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i64)]
        lib.dg_lts_advance.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp]
        lib.dg_lts_destroy.argtypes = [vp]
        lib.dg_lina_blob_size.restype = i64
        lib.dg_lina_blob_size.argtypes = [i32]
        lib.dg_lina_coefficients.argtypes = [i32, dbl, dbl, dbl, dp]
        lib.dg_lina_step.argtypes = [i32, i32, i64, i32, dbl, vp, vp, vp, vp, vp]
        lib.dg_visco_step.argtypes = [i32, i64, dbl, i32, vp, vp, vp, vp, vp, vp, dp, vp, vp, vp, vp]
        lib.dg_visco_tune.argtypes = [i32, i64, vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        lib.dg_visco_set_shape.argtypes = [i32, i32, i32]
        lib.dg_visco_get_shape.argtypes = [i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        _lib = lib
        return lib


def _check(rc):
    if rc != 0:
        raise DGError("dg error %d: %s" % (rc, _load().dg_last_error().decode(errors="replace")))


def set_debug_checks(enable: bool) -> bool:
    """Process-wide synchronous validation of neighbour tables (see
    dg_set_debug_checks in include/dg.h); returns the previous setting."""
    return bool(_load().dg_set_debug_checks(1 if enable else 0))


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ---------------------------------------------------------------------------
# host helpers
# ---------------------------------------------------------------------------
def reference_blob(degree: int) -> np.ndarray:
    """The packed reference-matrix blob of dg_reference_matrices (FP64), as
    the step kernels take it on the device."""
    lib = _load()
    n = lib.dg_reference_blob_size(degree)
    if n <= 0:
        raise DGError("unsupported degree %d" % degree)
    buf = np.zeros(n)
    _check(lib.dg_reference_matrices(degree, _dptr(buf)))
    return buf


def reference_matrices(degree: int) -> dict:
    lib = _load()
    n = lib.dg_reference_blob_size(degree)
    if n <= 0:
        raise DGError("unsupported degree %d" % degree)
    buf = np.zeros(n)
    _check(lib.dg_reference_matrices(degree, _dptr(buf)))
    B, Bf = comb(degree + 3, 3), comb(degree + 2, 2)
    out, o = {}, 0
    for name, shape in (("Khat", (3, B, B)), ("Ktilde", (3, B, B)), ("R", (4, B, Bf)), ("Rhat", (4, B, Bf)),
                        ("f", (3, Bf, Bf)), ("mass", (B,)), ("face_mass", (Bf,))):
        sz = int(np.prod(shape))
        out[name] = buf[o:o + sz].reshape(shape).copy()
        o += sz
    return out


def element_data(X, materials, neigh):
    """Star matrices (E,3,9,9) and flux solvers A+, A- (E,4,9,9) on the host."""
    lib = _load()
    X = np.ascontiguousarray(X, dtype=np.float64)
    mats = np.ascontiguousarray(materials, dtype=np.float64)
    nb = np.ascontiguousarray(neigh, dtype=np.int32)
    E = X.shape[0]
    if X.shape != (E, 4, 3) or mats.shape != (E, 3) or nb.shape != (E, 4):
        raise ValueError("element_data: expected X (E,4,3), materials (E,3), neigh (E,4)")
    star = np.empty((E, 3, 9, 9))
    Ap = np.empty((E, 4, 9, 9))
    Am = np.empty((E, 4, 9, 9))
    _check(lib.dg_element_data_host(E, _dptr(X), _dptr(mats), nb.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                    _dptr(star), _dptr(Ap), _dptr(Am)))
    return star, Ap, Am


def visco_element_data(X, materials, omega, Ylam, Ymu, neigh):
    """Viscoelastic star matrices (E,3,27,9) and flux solvers A+, A- (E,4,27,9)
    on the host (27 rows: elastic, then 3 mechanisms x 6 memory variables;
    the 9 elastic columns)."""
    lib = _load()
    X = np.ascontiguousarray(X, dtype=np.float64)
    mats = np.ascontiguousarray(materials, dtype=np.float64)
    om = np.ascontiguousarray(omega, dtype=np.float64)
    yl = np.ascontiguousarray(Ylam, dtype=np.float64)
    ym = np.ascontiguousarray(Ymu, dtype=np.float64)
    nb = np.ascontiguousarray(neigh, dtype=np.int32)
    E = X.shape[0]
    if (X.shape != (E, 4, 3) or mats.shape != (E, 3) or om.shape != (3,) or yl.shape != (E, 3)
            or ym.shape != (E, 3) or nb.shape != (E, 4)):
        raise ValueError("visco_element_data: expected X (E,4,3), materials (E,3), omega (3,), Ylam, Ymu (E,3), "
                         "neigh (E,4)")
    star = np.empty((E, 3, 27, 9))
    Ap = np.empty((E, 4, 27, 9))
    Am = np.empty((E, 4, 27, 9))
    _check(lib.dg_visco_element_data_host(E, _dptr(X), _dptr(mats), _dptr(om), _dptr(yl), _dptr(ym),
                                          nb.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dptr(star),
                                          _dptr(Ap), _dptr(Am)))
    return star, Ap, Am


def _nnz_models(degree):
    M = reference_matrices(degree)
    N = degree
    bd = [comb(N - d + 3, 3) for d in range(N + 1)]
    Bv = comb(N + 2, 3)
    nk = sum(int(np.count_nonzero(M["Ktilde"][:, :, :bd[d]])) for d in range(N))
    return M, bd, Bv, nk


def flop_model(degree: int, orient_counts=None) -> dict:
    """Non-zero flops per element of the kernels of one time step (the
    paper's counting: one multiply and one add per structural non-zero
    product, Sec. 4.3), for the algorithm this library runs.
    orient_counts: fraction of faces with orientation h=0,1,2 (default uniform)."""
    M, bd, Bv, nk = _nnz_models(degree)
    N = degree
    B = bd[0]
    Bf = comb(N + 2, 2)
    w = np.full(3, 1 / 3) if orient_counts is None else np.asarray(orient_counts, float)
    star_nnz = 24
    ck = sum(2 * 3 * star_nnz * bd[d] for d in range(N)) + 2 * 9 * nk
    ti = sum(2 * 9 * bd[d] for d in range(N + 1))
    traces = 2 * 9 * sum(int(np.count_nonzero(M["R"][s])) for s in range(4))
    vol = 2 * 3 * star_nnz * Bv + 2 * 9 * int(np.count_nonzero(M["Khat"]))
    lift = 2 * 9 * sum(int(np.count_nonzero(M["Rhat"][s])) for s in range(4))
    mix = 4 * 2 * 81 * Bf
    fh = 4 * 2 * 9 * float(np.dot(w, [np.count_nonzero(M["f"][h]) for h in range(3)]))
    predict = ck + ti + traces
    correct = vol + 2 * (lift + mix) + fh
    return dict(ck=ck, ti=ti, traces=traces, volume=vol, local=lift + mix, neighbour=lift + mix + fh,
                step_predict=predict, step_correct=correct, step=predict + correct, step_fused=predict + correct,
                B=B, Bf=Bf)


# ---------------------------------------------------------------------------
# device plans (torch tensors for memory and streams)
# ---------------------------------------------------------------------------
def _torch():
    import torch
    return torch


class Plan:
    """A compiled (degree, precision) configuration of the element kernels."""

    def __init__(self, degree: int, precision: int = DG_FP64):
        lib = _load()
        h = ctypes.c_void_p()
        _check(lib.dg_plan_create(degree, precision, ctypes.byref(h)))
        self._h = h
        self.degree = degree
        self.precision = precision
        B, Bf = ctypes.c_int(), ctypes.c_int()
        _check(lib.dg_plan_sizes(h, ctypes.byref(B), ctypes.byref(Bf)))
        self.B, self.Bf = B.value, Bf.value
        self.fuses_steps = bool(_load().dg_plan_fuses_steps(self._h))
        torch = _torch()
        self.dtype = torch.float64 if precision == DG_FP64 else torch.float32

    def tune(self, E=100_000, stream=None):
        """Time the fused and the two-launch step schedule on E synthetic
        elements and keep the faster for this plan; returns fuses_steps."""
        r = _load().dg_plan_tune(self._h, int(E), self._stream(stream))
        _check(r if r < 0 else 0)
        self.fuses_steps = bool(r)
        return self.fuses_steps

    def set_fusion(self, fused: bool):
        """Force the step schedule: True = corrector of step k and predictor
        of step k+1 in one launch, False = two launches (same result)."""
        _check(_load().dg_plan_set_fusion(self._h, 1 if fused else 0))
        self.fuses_steps = bool(fused)

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.dg_plan_destroy(self._h)
            self._h = None

    # -- argument helpers ----------------------------------------------------
    @staticmethod
    def _check_tensor(t, shape, dtype, name):
        torch = _torch()
        if not isinstance(t, torch.Tensor):
            raise TypeError("%s must be a torch tensor" % name)
        if tuple(t.shape) != tuple(shape):
            raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
        if t.dtype != dtype:
            raise ValueError("%s has dtype %s, expected %s" % (name, t.dtype, dtype))
        if t.numel() and (not t.is_cuda or not t.is_contiguous()):
            raise ValueError("%s must be a contiguous device tensor" % name)
        return t.data_ptr() if t.numel() else None

    def _t(self, t, shape, dtype, name):
        torch = _torch()
        if not isinstance(t, torch.Tensor):
            raise TypeError("%s must be a torch tensor" % name)
        if tuple(t.shape) != tuple(shape):
            raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
        if t.dtype != dtype:
            raise ValueError("%s has dtype %s, expected %s" % (name, t.dtype, dtype))
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("%s must be a contiguous device tensor" % name)
        return ctypes.c_void_p(t.data_ptr())

    @staticmethod
    def _stream(stream=None):
        torch = _torch()
        s = stream if stream is not None else torch.cuda.current_stream()
        return ctypes.c_void_p(s.cuda_stream)

    # -- shapes --------------------------------------------------------------
    def dof_shape(self, E):
        return (E, 9, self.B)

    def trace_shape(self, E):
        """Face-trace work array: one contiguous block of 9*Bf values per
        element and face (internal layout: see include/dg.h)."""
        return (E, 4, 9 * self.Bf)

    def deriv_shape(self, E):
        return (E, self.degree + 1, 9, self.B)

    # -- calls ---------------------------------------------------------------
    def pack_star(self, star_dense, out=None, stream=None):
        torch = _torch()
        E = star_dense.shape[0]
        if out is None:
            out = torch.empty((E, 9, 3, 3), dtype=self.dtype, device=star_dense.device)
        _check(_load().dg_pack_star(self._h, E, self._t(star_dense, (E, 3, 9, 9), torch.float64, "star_dense"),
                                    self._t(out, (E, 9, 3, 3), self.dtype, "star_packed"), self._stream(stream)))
        return out

    def predictor(self, Q, star_packed, dt, T=None, stream=None):
        torch = _torch()
        E = Q.shape[0]
        if T is None:
            T = torch.empty(self.deriv_shape(E), dtype=self.dtype, device=Q.device)
        _check(_load().dg_predictor(self._h, E, float(dt), self._t(Q, self.dof_shape(E), self.dtype, "Q"),
                                    self._t(star_packed, (E, 9, 3, 3), self.dtype, "star_packed"),
                                    self._t(T, self.deriv_shape(E), self.dtype, "T"), self._stream(stream)))
        return T

    def time_integral(self, T, dt, I=None, stream=None):
        torch = _torch()
        E = T.shape[0]
        if I is None:
            I = torch.empty(self.dof_shape(E), dtype=self.dtype, device=T.device)
        _check(_load().dg_time_integral(self._h, E, float(dt), self._t(T, self.deriv_shape(E), self.dtype, "T"),
                                        self._t(I, self.dof_shape(E), self.dtype, "I"), self._stream(stream)))
        return I

    def volume(self, I, star_packed, Q, stream=None):
        E = Q.shape[0]
        _check(_load().dg_volume(self._h, E, self._t(I, self.dof_shape(E), self.dtype, "I"),
                                 self._t(star_packed, (E, 9, 3, 3), self.dtype, "star_packed"),
                                 self._t(Q, self.dof_shape(E), self.dtype, "Q"), self._stream(stream)))
        return Q

    def local_flux(self, I, Aplus, Q, stream=None):
        torch = _torch()
        E = Q.shape[0]
        _check(_load().dg_local_flux(self._h, E, self._t(I, self.dof_shape(E), self.dtype, "I"),
                                     self._t(Aplus, (E, 4, 9, 9), torch.float64, "Aplus"),
                                     self._t(Q, self.dof_shape(E), self.dtype, "Q"), self._stream(stream)))
        return Q

    def neighbour_flux(self, I, neigh, face_rot, Aminus, Q, stream=None):
        torch = _torch()
        E = Q.shape[0]
        EI = I.shape[0]
        _check(_load().dg_neighbour_flux(self._h, E, EI, self._t(I, self.dof_shape(EI), self.dtype, "I"),
                                         self._t(neigh, (E, 4), torch.int32, "neigh"),
                                         self._t(face_rot, (E, 4), torch.uint8, "face_rot"),
                                         self._t(Aminus, (E, 4, 9, 9), torch.float64, "Aminus"),
                                         self._t(Q, self.dof_shape(E), self.dtype, "Q"), self._stream(stream)))
        return Q

    def step(self, Q, I, traces, star_packed, Aplus, Aminus, neigh, face_rot, dt, n_steps=1, stream=None,
             traces_b=None):
        """n_steps time steps; with a second trace array traces_b, one launch
        per step (corrector and next predictor fused)."""
        torch = _torch()
        E = Q.shape[0]
        tb = None if traces_b is None else self._t(traces_b, self.trace_shape(E), self.dtype, "traces_b")
        _check(_load().dg_step(self._h, E, float(dt), int(n_steps),
                               self._t(Q, self.dof_shape(E), self.dtype, "Q"),
                               self._t(I, self.dof_shape(E), self.dtype, "I"),
                               self._t(traces, self.trace_shape(E), self.dtype, "traces"), tb,
                               self._t(star_packed, (E, 9, 3, 3), self.dtype, "star_packed"),
                               self._t(Aplus, (E, 4, 9, 9), torch.float64, "Aplus"),
                               self._t(Aminus, (E, 4, 9, 9), torch.float64, "Aminus"),
                               self._t(neigh, (E, 4), torch.int32, "neigh"),
                               self._t(face_rot, (E, 4), torch.uint8, "face_rot"), self._stream(stream)))
        return Q

    # bytes of the library's fixed face-trace buffer (DG_NOALLOC_SCRATCH_BYTES)
    NOALLOC_SCRATCH_BYTES = 256 << 20

    def noalloc_max_elements(self):
        """Largest E that dg_step_noalloc accepts for this plan."""
        rs = 8 if self.precision == DG_FP64 else 4
        return self.NOALLOC_SCRATCH_BYTES // (4 * 9 * self.Bf * rs)

    def step_noalloc(self, Q, I, star_packed, Aplus, Aminus, neigh, face_rot, dt, n_steps=1, stream=None):
        """dg_step with the face traces in the library's fixed device buffer
        (no device allocation; E up to noalloc_max_elements())."""
        torch = _torch()
        E = Q.shape[0]
        _check(_load().dg_step_noalloc(self._h, E, float(dt), int(n_steps),
                                       self._t(Q, self.dof_shape(E), self.dtype, "Q"),
                                       self._t(I, self.dof_shape(E), self.dtype, "I"),
                                       self._t(star_packed, (E, 9, 3, 3), self.dtype, "star_packed"),
                                       self._t(Aplus, (E, 4, 9, 9), torch.float64, "Aplus"),
                                       self._t(Aminus, (E, 4, 9, 9), torch.float64, "Aminus"),
                                       self._t(neigh, (E, 4), torch.int32, "neigh"),
                                       self._t(face_rot, (E, 4), torch.uint8, "face_rot"), self._stream(stream)))
        return Q

    # simulations advanced together by fused_step (DG_FUSED_SIMS)
    FUSED_SIMS = 16

    def fused_dof_shape(self, E):
        return (E, 9, self.B, self.FUSED_SIMS)

    def fused_trace_shape(self, E):
        return (E, 4, 9, self.Bf, self.FUSED_SIMS)

    def fused_step(self, Q, I, traces, star_packed, Aplus, Aminus, neigh, face_rot, dt, n_steps=1, stream=None):
        """n_steps time steps of 16 simulations on one mesh (dg_fused_step;
        DG_BF16X3 plans): Q, I (E, 9, B, 16), traces (E, 4, 9, Bf, 16)."""
        torch = _torch()
        E = Q.shape[0]
        _check(_load().dg_fused_step(self._h, E, float(dt), int(n_steps),
                                     self._t(Q, self.fused_dof_shape(E), self.dtype, "Q"),
                                     self._t(I, self.fused_dof_shape(E), self.dtype, "I"),
                                     self._t(traces, self.fused_trace_shape(E), self.dtype, "traces"),
                                     self._t(star_packed, (E, 9, 3, 3), self.dtype, "star_packed"),
                                     self._t(Aplus, (E, 4, 9, 9), torch.float64, "Aplus"),
                                     self._t(Aminus, (E, 4, 9, 9), torch.float64, "Aminus"),
                                     self._t(neigh, (E, 4), torch.int32, "neigh"),
                                     self._t(face_rot, (E, 4), torch.uint8, "face_rot"), self._stream(stream)))
        return Q

    def step_predict(self, Q, star_packed, dt, I, traces, stream=None):
        E = Q.shape[0]
        _check(_load().dg_step_predict(self._h, E, float(dt), self._t(Q, self.dof_shape(E), self.dtype, "Q"),
                                       self._t(star_packed, (E, 9, 3, 3), self.dtype, "star_packed"),
                                       self._t(I, self.dof_shape(E), self.dtype, "I"),
                                       self._t(traces, self.trace_shape(E), self.dtype, "traces"),
                                       self._stream(stream)))

    def step_fused(self, Q, I, traces_in, traces_out, star_packed, Aplus, Aminus, neigh, face_rot, dt,
                   stream=None):
        torch = _torch()
        E = Q.shape[0]
        _check(_load().dg_step_fused(self._h, E, float(dt), self._t(Q, self.dof_shape(E), self.dtype, "Q"),
                                     self._t(I, self.dof_shape(E), self.dtype, "I"),
                                     self._t(traces_in, self.trace_shape(E), self.dtype, "traces_in"),
                                     self._t(traces_out, self.trace_shape(E), self.dtype, "traces_out"),
                                     self._t(star_packed, (E, 9, 3, 3), self.dtype, "star_packed"),
                                     self._t(Aplus, (E, 4, 9, 9), torch.float64, "Aplus"),
                                     self._t(Aminus, (E, 4, 9, 9), torch.float64, "Aminus"),
                                     self._t(neigh, (E, 4), torch.int32, "neigh"),
                                     self._t(face_rot, (E, 4), torch.uint8, "face_rot"), self._stream(stream)))

    def step_correct(self, I, traces, star_packed, Aplus, Aminus, neigh, face_rot, Q, stream=None):
        torch = _torch()
        E = Q.shape[0]
        _check(_load().dg_step_correct(self._h, E, self._t(I, self.dof_shape(E), self.dtype, "I"),
                                       self._t(traces, self.trace_shape(E), self.dtype, "traces"),
                                       self._t(star_packed, (E, 9, 3, 3), self.dtype, "star_packed"),
                                       self._t(Aplus, (E, 4, 9, 9), torch.float64, "Aplus"),
                                       self._t(Aminus, (E, 4, 9, 9), torch.float64, "Aminus"),
                                       self._t(neigh, (E, 4), torch.int32, "neigh"),
                                       self._t(face_rot, (E, 4), torch.uint8, "face_rot"),
                                       self._t(Q, self.dof_shape(E), self.dtype, "Q"), self._stream(stream)))

    @staticmethod
    def sync(stream=None):
        _check(_load().dg_sync(Plan._stream(stream)))


class Batch:
    """A batch of independent meshes (any degrees) stepped together: one
    predictor and one corrector launch per degree and material model present,
    replayed as a HIP graph.  `meshes` is a list of dicts with keys degree, E,
    dt, Q, I, traces, star_packed, Aplus, Aminus, neigh, face_rot (device
    tensors owned by the caller and kept alive by this object).  A
    viscoelastic mesh (DG_FP64 batches) has n_quant=27, omega (3 relaxation
    frequencies), star (E, 3, 27, 9) in place of star_packed, Q and I
    (E, 27, B), traces (E, 4, 9, Bf) and Aplus, Aminus (E, 4, 27, 9)."""

    def __init__(self, precision, meshes):
        lib = _load()
        self.precision = precision
        arr, keep = self._items(meshes)
        h = ctypes.c_void_p()
        _check(lib.dg_batch_create(precision, arr, len(meshes), ctypes.byref(h)))
        self._h = h
        self._keep = [keep]
        self.elements = sum(int(m["E"]) for m in meshes)

    def _items(self, meshes):
        torch = _torch()
        dt_ = torch.float64 if self.precision == DG_FP64 else torch.float32
        arr = (BatchItem * max(1, len(meshes)))()
        for i, m in enumerate(meshes):
            N, E = int(m["degree"]), int(m["E"])
            B, Bf = comb(N + 3, 3), comb(N + 2, 2)
            chk = Plan._check_tensor
            if int(m.get("n_quant", 9)) == 27:
                f64 = torch.float64
                om = [float(w) for w in m["omega"]]
                if len(om) != 3:
                    raise ValueError("omega must hold 3 values")
                arr[i] = BatchItem(N, E, float(m["dt"]),
                                   chk(m["Q"], (E, 27, B), f64, "Q"), chk(m["I"], (E, 27, B), f64, "I"),
                                   chk(m["traces"], (E, 4, 9, Bf), f64, "traces"),
                                   chk(m["star"], (E, 3, 27, 9), f64, "star"),
                                   chk(m["Aplus"], (E, 4, 27, 9), f64, "Aplus"),
                                   chk(m["Aminus"], (E, 4, 27, 9), f64, "Aminus"),
                                   chk(m["neigh"], (E, 4), torch.int32, "neigh"),
                                   chk(m["face_rot"], (E, 4), torch.uint8, "face_rot"), 27,
                                   (ctypes.c_double * 3)(*om))
                continue
            arr[i] = BatchItem(N, E, float(m["dt"]),
                               chk(m["Q"], (E, 9, B), dt_, "Q"), chk(m["I"], (E, 9, B), dt_, "I"),
                               chk(m["traces"], (E, 4, 9 * Bf), dt_, "traces"),
                               chk(m["star_packed"], (E, 9, 3, 3), dt_, "star_packed"),
                               chk(m["Aplus"], (E, 4, 9, 9), torch.float64, "Aplus"),
                               chk(m["Aminus"], (E, 4, 9, 9), torch.float64, "Aminus"),
                               chk(m["neigh"], (E, 4), torch.int32, "neigh"),
                               chk(m["face_rot"], (E, 4), torch.uint8, "face_rot"), 9)
        return arr, list(meshes)

    def update(self, meshes):
        """Replace the mesh list (dg_batch_update): steps enqueued from now on
        step `meshes`; steps already enqueued keep their list.  The tensors of
        the previous list stay referenced until the update after next (by
        then no enqueued step reads them)."""
        arr, keep = self._items(meshes)
        _check(_load().dg_batch_update(self._h, arr, len(meshes)))
        self._keep = (self._keep + [keep])[-2:]
        self.elements = sum(int(m["E"]) for m in meshes)

    def step(self, n_steps=1, stream=None):
        _check(_load().dg_batch_step(self._h, int(n_steps), Plan._stream(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.dg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


class Lts:
    """Clustered local time stepping of rate 2 on one mesh (dg_lts_*).
    `cluster` (E,) int32 host array, non-decreasing (elements numbered
    cluster by cluster), `neigh` (E, 4) int32 host array; cluster c steps with
    dt0 * 2^c.  advance() takes the device arrays of dg_step for the mesh."""

    def __init__(self, plan, cluster, neigh, dt0):
        import numpy as np
        lib = _load()
        cl = np.ascontiguousarray(cluster, dtype=np.int32)
        nb = np.ascontiguousarray(neigh, dtype=np.int32)
        E = int(cl.shape[0])
        if nb.shape != (E, 4):
            raise ValueError("neigh has shape %s, expected (%d, 4)" % (nb.shape, E))
        h = ctypes.c_void_p()
        ip = ctypes.POINTER(ctypes.c_int32)
        _check(lib.dg_lts_create(plan._h, E, cl.ctypes.data_as(ip), nb.ctypes.data_as(ip), float(dt0),
                                 ctypes.byref(h)))
        self._h = h
        self.plan = plan
        self.E = E
        nc, upc = ctypes.c_int(), ctypes.c_int64()
        _check(lib.dg_lts_clusters(self._h, ctypes.byref(nc), ctypes.byref(upc)))
        self.n_clusters = nc.value
        self.updates_per_cycle = upc.value

    def advance(self, n_cycles, Q, star_packed, Aplus, Aminus, neigh, face_rot, stream=None):
        torch = _torch()
        p, E = self.plan, self.E
        args = [p._t(Q, p.dof_shape(E), p.dtype, "Q"), p._t(star_packed, (E, 9, 3, 3), p.dtype, "star_packed"),
                p._t(Aplus, (E, 4, 9, 9), torch.float64, "Aplus"),
                p._t(Aminus, (E, 4, 9, 9), torch.float64, "Aminus"),
                p._t(neigh, (E, 4), torch.int32, "neigh"), p._t(face_rot, (E, 4), torch.uint8, "face_rot")]
        _check(_load().dg_lts_advance(self._h, int(n_cycles), *args, Plan._stream(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.dg_lts_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


# ---------------------------------------------------------------------------
# viscoelastic elements (27 quantities)
# ---------------------------------------------------------------------------
def visco_step(degree, Q, I, traces, star, Aplus, Aminus, omega, ref, neigh, face_rot, dt, n_steps=1, stream=None):
    """n_steps viscoelastic steps (dg_visco_step) on FP64 device tensors:
    Q, I (E, 27, B); traces (E, 4, 9, Bf); star (E, 3, 27, 9); Aplus, Aminus
    (E, 4, 27, 9); ref the dg_reference_matrices blob of the degree on the
    device; neigh (E, 4) int32; face_rot (E, 4) uint8; omega 3 floats."""
    torch = _torch()
    E = int(Q.shape[0])
    B, Bf = comb(degree + 3, 3), comb(degree + 2, 2)
    t, f64 = Plan._t, torch.float64
    om = np.ascontiguousarray(omega, dtype=np.float64)
    if om.shape != (3,):
        raise ValueError("omega must hold 3 values")
    args = [t(None, Q, (E, 27, B), f64, "Q"), t(None, I, (E, 27, B), f64, "I"),
            t(None, traces, (E, 4, 9, Bf), f64, "traces"), t(None, star, (E, 3, 27, 9), f64, "star"),
            t(None, Aplus, (E, 4, 27, 9), f64, "Aplus"), t(None, Aminus, (E, 4, 27, 9), f64, "Aminus")]
    refp = t(None, ref, (int(_load().dg_reference_blob_size(degree)),), f64, "ref")
    _check(_load().dg_visco_step(int(degree), E, float(dt), int(n_steps), *args, _dptr(om), refp,
                                 t(None, neigh, (E, 4), torch.int32, "neigh"),
                                 t(None, face_rot, (E, 4), torch.uint8, "face_rot"), Plan._stream(stream)))


def visco_shape(degree, shape=None):
    """The viscoelastic launch shape of a degree, (waves per workgroup,
    workgroups per CU, 0 = all that fit); with `shape` given, set it first
    (dg_visco_set_shape)."""
    lib = _load()
    if shape is not None:
        _check(lib.dg_visco_set_shape(int(degree), int(shape[0]), int(shape[1])))
    w, g = ctypes.c_int(), ctypes.c_int()
    _check(lib.dg_visco_get_shape(int(degree), ctypes.byref(w), ctypes.byref(g)))
    return w.value, g.value


def visco_tune(degree, E=100_000, stream=None):
    """dg_visco_tune: time the viscoelastic launch shapes of `degree` on E
    synthetic elements and keep the fastest for the process; returns
    (waves per workgroup, resident workgroups per CU)."""
    w, g = ctypes.c_int(), ctypes.c_int()
    _check(_load().dg_visco_tune(int(degree), int(E), Plan._stream(stream), ctypes.byref(w), ctypes.byref(g)))
    return w.value, g.value


# ---------------------------------------------------------------------------
# LinA: ADER-DG-SEM on cuboids (Sec. 5.2)
# ---------------------------------------------------------------------------
LINA_MAX_ORDER = {DG_FP64: 12, DG_FP32: 16}


def lina_coefficients(order, rho0, K0, h):
    """Host FP64 coefficient blob (dg_lina_coefficients) as a dict of arrays
    plus the flat blob under "blob"."""
    lib = _load()
    n = lib.dg_lina_blob_size(int(order))
    if n <= 0:
        raise DGError("unsupported LinA order %d" % order)
    buf = np.zeros(n)
    _check(lib.dg_lina_coefficients(int(order), float(rho0), float(K0), float(h), _dptr(buf)))
    O, out, o = int(order), {"blob": buf}, 0
    for name, shape in (("Kt", (O, O)), ("Kh", (O, O)), ("w", (O,)), ("star", (3, 4, 4)), ("Ap", (6, 4, 4)),
                        ("Am", (6, 4, 4))):
        sz = int(np.prod(shape))
        out[name] = buf[o:o + sz].reshape(shape)
        o += sz
    return out


def lina_step(Q, sides, coef, neigh, dt, n_steps=1, stream=None):
    """n_steps LinA steps (dg_lina_step) on device tensors: Q (E, 4, O, O, O)
    float64 or float32, sides (E, 6, 4, O, O) of the same dtype, coef the
    blob on the device in that dtype, neigh (E, 6) int32."""
    torch = _torch()
    E, O = int(Q.shape[0]), int(Q.shape[-1])
    prec = DG_FP64 if Q.dtype == torch.float64 else DG_FP32
    t = Plan._t
    args = [t(None, Q, (E, 4, O, O, O), Q.dtype, "Q"), t(None, sides, (E, 6, 4, O, O), Q.dtype, "sides"),
            t(None, coef, (int(_load().dg_lina_blob_size(O)),), Q.dtype, "coef"),
            t(None, neigh, (E, 6), torch.int32, "neigh")]
    _check(_load().dg_lina_step(prec, O, E, int(n_steps), float(dt), *args, Plan._stream(stream)))


# ---------------------------------------------------------------------------
# the separable contraction of Sec. 7 (Eq. stock_mra)
# ---------------------------------------------------------------------------
MRA_MAX_P = {DG_FP64: 20, DG_FP32: 24}


def mra_apply(S, XL, XR, YL, YR, ZL, ZR, R=None, stream=None):
    """R_ijk = sum S_xyz XL_xl XR_li YL_ym YR_mj ZL_zn ZR_nk for a batch S
    (nb, p, p, p) of device tensors (float64 or float32); factors (p, q) and
    (q, p) of the same dtype.  Returns R (dg_mra_apply)."""
    torch = _torch()
    nb, p = S.shape[0], S.shape[1]
    q = XL.shape[1]
    prec = DG_FP64 if S.dtype == torch.float64 else DG_FP32
    if R is None:
        R = torch.empty_like(S)
    t = Plan._t
    args = [t(None, S, (nb, p, p, p), S.dtype, "S")]
    for name, m, sh in (("XL", XL, (p, q)), ("XR", XR, (q, p)), ("YL", YL, (p, q)), ("YR", YR, (q, p)),
                        ("ZL", ZL, (p, q)), ("ZR", ZR, (q, p))):
        args.append(t(None, m, sh, S.dtype, name))
    args.append(t(None, R, (nb, p, p, p), S.dtype, "R"))
    _check(_load().dg_mra_apply(prec, nb, p, q, *args, Plan._stream(stream)))
    return R
