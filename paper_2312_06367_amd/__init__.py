"""MI355X (gfx950) marching-on-in-time solver for the qHP TD-CFIE.

Thin ctypes binding of ``libqhp.so`` (C ABI in ``include/qhp.h``): argument
marshalling only; every step of the method runs in the library's HIP kernels.
PyTorch supplies device memory and the stream.  Importing this package fails
loudly when the shared library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqhp.so")

QHP_F64, QHP_F32, QHP_BF16, QHP_F32A, QHP_BF16X2, QHP_I8X4, QHP_FAC64, QHP_FAC32 = 0, 1, 2, 3, 4, 5, 6, 7
QHP_FP8E4M3 = 8  # qhp_set_precision only: FP8 values in FP32 words, marched as F32A
QHP_SOLVE_LU, QHP_SOLVE_INV, QHP_SOLVE_GMRES = 0, 1, 2
WARM = {"cold": 0, "prev": 1, "extrap": 2, "quad": 3, "mlp": 4, "best": 5}
MAT = {"gram": 0, "zs": 1, "zh": 2, "m": 3, "psigma": 4, "plambda": 5, "pe": 6, "pm": 7,
       "slab": 8, "a": 9, "b": 10, "c": 11}
ERRORS = {0: "OK", -1: "EINVAL", -2: "EMESH", -3: "ESTATE", -4: "ENOMEM", -5: "EDEVICE",
          -6: "ESINGULAR", -7: "ENOCONV", -8: "EUNSTABLE"}
PRECISIONS = {"f64": QHP_F64, "f32": QHP_F32, "bf16": QHP_BF16, "f32a": QHP_F32A, "bf16x2": QHP_BF16X2,
              "i8x4": QHP_I8X4, "fac64": QHP_FAC64, "fac32": QHP_FAC32, "fp8": QHP_FP8E4M3}
SOLVERS = {"lu": QHP_SOLVE_LU, "inv": QHP_SOLVE_INV, "gmres": QHP_SOLVE_GMRES}


class QhpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class _Params(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("eta_c", ctypes.c_double), ("precision", ctypes.c_int32),
                ("solver", ctypes.c_int32), ("n_psi", ctypes.c_int32), ("device", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("dev_alloc", _ALLOC_FN), ("dev_free", _FREE_FN),
                ("alloc_user", ctypes.c_void_p), ("temporal_order", ctypes.c_int32)]


class TorchAllocator:
    """The dev_alloc / dev_free hook of qhp_params backed by PyTorch's caching
    allocator: the library's device buffers become uint8 tensors held here
    until the library frees them."""

    def __init__(self, device: int):
        self.device = device
        self.live = {}
        self.calls = {"alloc": 0, "free": 0}
        self.alloc_fn = _ALLOC_FN(self._alloc)
        self.free_fn = _FREE_FN(self._free)

    def _alloc(self, nbytes, user):
        import torch
        try:
            t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda:%d" % self.device)
        except RuntimeError:
            return None
        self.live[t.data_ptr()] = t
        self.calls["alloc"] += 1
        return t.data_ptr()

    def _free(self, ptr, user):
        self.live.pop(ptr, None)
        self.calls["free"] += 1

    def bytes_held(self) -> int:
        return sum(t.numel() for t in self.live.values())


class _Wave(ctypes.Structure):
    _fields_ = [("k_hat", ctypes.c_double * 3), ("pol", ctypes.c_double * 3), ("amplitude", ctypes.c_double),
                ("t0", ctypes.c_double), ("pulse", ctypes.c_int32), ("w", ctypes.c_double),
                ("f0", ctypes.c_double), ("bw", ctypes.c_double)]


class _GmresInfo(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("iterations", ctypes.c_int64), ("max_iterations", ctypes.c_int64),
                ("refinements", ctypes.c_int64), ("fallbacks", ctypes.c_int64), ("network_starts", ctypes.c_int64)]


class _Info(ctypes.Structure):
    _fields_ = [("nv", ctypes.c_int64), ("ne", ctypes.c_int64), ("nc", ctypes.c_int64),
                ("n_harmonic", ctypes.c_int64), ("K", ctypes.c_int64), ("n_rhs", ctypes.c_int64),
                ("n_steps", ctypes.c_int64), ("step", ctypes.c_int64), ("ld", ctypes.c_int64),
                ("diameter", ctypes.c_double), ("slab_bytes", ctypes.c_size_t),
                ("hist_variant", ctypes.c_int64), ("hist_splits", ctypes.c_int64), ("raw_nnz", ctypes.c_int64),
                ("band_bytes_pairs", ctypes.c_size_t), ("band_bytes_cells", ctypes.c_size_t),
                ("band_nnz_pairs", ctypes.c_int64), ("band_nnz_cells", ctypes.c_int64),
                ("band_waves_pairs", ctypes.c_int64), ("band_waves_cells", ctypes.c_int64),
                ("band_pieces_pairs", ctypes.c_int64), ("band_pieces_cells", ctypes.c_int64),
                ("band_block", ctypes.c_int64), ("band_bytes_near_pairs", ctypes.c_size_t),
                ("band_bytes_near_cells", ctypes.c_size_t)]


EXPORTS = ["qhp_create", "qhp_mesh", "qhp_assemble", "qhp_set_precision", "qhp_set_solver", "qhp_profile",
           "qhp_hist_time", "qhp_band_time", "qhp_set_incident", "qhp_step", "qhp_run", "qhp_query", "qhp_edges",
           "qhp_get_matrix", "qhp_keep_raw", "qhp_history_sum", "qhp_history_sum_variant", "qhp_history_variants",
           "qhp_t0_condition", "qhp_batch_create", "qhp_batch_create_variant", "qhp_batch_variants", "qhp_batch_history_variant",
           "qhp_batch_run",
           "qhp_batch_step_times", "qhp_batch_last_error", "qhp_batch_destroy", "qhp_last_error",
           "qhp_destroy", "qhp_release_assembly", "qhp_set_gmres", "qhp_gmres_stats", "qhp_gmres_reset", "qhp_mlp_create",
           "qhp_mlp_dims", "qhp_mlp_set_params", "qhp_mlp_get_params", "qhp_mlp_features", "qhp_mlp_guess", "qhp_mlp_reconstruct",
           "qhp_mlp_forward", "qhp_mlp_loss_grad", "qhp_mlp_adam", "qhp_mlp_train", "qhp_attach_mlp",
           "qhp_mlp_last_error", "qhp_mlp_destroy", "qhp_check_mesh", "qhp_set_growth_limit",
           "qhp_history_sum_noalloc"]
_NO_RC = ("qhp_last_error", "qhp_destroy", "qhp_batch_last_error", "qhp_batch_destroy", "qhp_mlp_last_error",
          "qhp_mlp_destroy")

_lib = None


def lib():
    """Load libqhp.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libqhp.so not built: run `python -m paper_2312_06367_amd.build` "
                              "(or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        L.qhp_create.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(vp)]
        L.qhp_mesh.argtypes = [vp, vp, i64, vp, i64]
        L.qhp_assemble.argtypes = [vp]
        L.qhp_set_precision.argtypes = [vp, i32]
        L.qhp_set_solver.argtypes = [vp, i32]
        L.qhp_profile.argtypes = [vp, i32]
        L.qhp_hist_time.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
        L.qhp_band_time.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(i64)]
        L.qhp_set_incident.argtypes = [vp, ctypes.POINTER(_Wave), i32, i32]
        L.qhp_step.argtypes = [vp, vp]
        L.qhp_run.argtypes = [vp, i32, vp, vp]
        L.qhp_query.argtypes = [vp, ctypes.POINTER(_Info)]
        L.qhp_edges.argtypes = [vp, vp, vp]
        L.qhp_get_matrix.argtypes = [vp, i32, i32, vp]
        L.qhp_keep_raw.argtypes = [vp, i32]
        L.qhp_history_sum.argtypes = [vp, i32, i64, i64, i64, i64, vp, vp, vp, i64, i64, vp, vp]
        L.qhp_history_sum_variant.argtypes = [vp, i32, i64, i64, i64, i64, vp, vp, vp, i64, i64, vp, vp, i32]
        L.qhp_history_variants.argtypes = [i32, i64]
        L.qhp_history_sum_noalloc.argtypes = [vp, i32, i64, i64, i64, i64, vp, vp, vp, i64, i64, vp, vp, i32]
        L.qhp_t0_condition.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.qhp_batch_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(vp)]
        L.qhp_batch_create_variant.argtypes = [ctypes.POINTER(vp), i32, i32, ctypes.POINTER(vp)]
        L.qhp_batch_variants.argtypes = [i32, i32]
        L.qhp_batch_variants.restype = i32
        L.qhp_batch_history_variant.argtypes = [vp]
        L.qhp_batch_history_variant.restype = i32
        L.qhp_batch_run.argtypes = [vp, i32, ctypes.POINTER(vp)]
        L.qhp_batch_step_times.argtypes = [vp, ctypes.POINTER(ctypes.c_float), i32]
        L.qhp_batch_last_error.argtypes = [vp]
        L.qhp_batch_last_error.restype = ctypes.c_char_p
        L.qhp_batch_destroy.argtypes = [vp]
        L.qhp_batch_destroy.restype = None
        L.qhp_last_error.argtypes = [vp]
        L.qhp_last_error.restype = ctypes.c_char_p
        L.qhp_destroy.argtypes = [vp]
        L.qhp_destroy.restype = None
        dbl, u64 = ctypes.c_double, ctypes.c_uint64
        L.qhp_set_gmres.argtypes = [vp, dbl, i32, i32, i32]
        L.qhp_release_assembly.argtypes = [vp]
        L.qhp_gmres_stats.argtypes = [vp, ctypes.POINTER(_GmresInfo), vp, vp, i64]
        L.qhp_gmres_reset.argtypes = [vp]
        L.qhp_mlp_create.argtypes = [vp, i32, u64, ctypes.POINTER(vp)]
        L.qhp_mlp_dims.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.qhp_mlp_set_params.argtypes = [vp, vp]
        L.qhp_mlp_get_params.argtypes = [vp, vp]
        L.qhp_mlp_features.argtypes = [vp, vp, i64, vp]
        L.qhp_mlp_guess.argtypes = [vp, vp, vp]
        L.qhp_mlp_reconstruct.argtypes = [vp, vp, i64, vp]
        L.qhp_mlp_forward.argtypes = [vp, vp, i32, vp]
        L.qhp_mlp_loss_grad.argtypes = [vp, vp, vp, i32, ctypes.POINTER(dbl), vp]
        L.qhp_mlp_adam.argtypes = [vp, dbl, dbl, dbl, dbl]
        L.qhp_mlp_train.argtypes = [vp, vp, i64, i64, i32, i32, dbl, u64, vp]
        L.qhp_attach_mlp.argtypes = [vp, vp]
        L.qhp_mlp_last_error.argtypes = [vp]
        L.qhp_mlp_last_error.restype = ctypes.c_char_p
        L.qhp_mlp_destroy.argtypes = [vp]
        L.qhp_mlp_destroy.restype = None
        L.qhp_check_mesh.argtypes = [vp, i64, vp, i64, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.c_char_p, i64]
        L.qhp_set_growth_limit.argtypes = [vp, dbl]
        for name in EXPORTS:
            if name not in _NO_RC:
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def to_cwave(w) -> _Wave:
    cw = _Wave()
    g = (lambda k: w[k]) if isinstance(w, dict) else (lambda k: getattr(w, k))
    for i in range(3):
        cw.k_hat[i] = float(g("k_hat")[i])
        cw.pol[i] = float(g("pol")[i])
    cw.amplitude, cw.t0, cw.pulse = float(g("amplitude")), float(g("t0")), int(g("pulse"))
    cw.w, cw.f0, cw.bw = float(g("w")), float(g("f0")), float(g("bw"))
    return cw


class Solver:
    """One scatterer and time step on one GPU (see include/qhp.h)."""

    def __init__(self, dt: float, precision: str = "f64", solver: str = "lu", n_psi: int = 10,
                 eta_c: float = 1.0, device: int = 0, stream=None, allocator: str = "hip", order: int = 1):
        """allocator: "hip" (the library's hipMalloc) or "torch" (PyTorch's
        caching allocator through the dev_alloc / dev_free hook); order: the
        temporal basis pairs, 1 (hat functions) or 2 (quadratic interpolators)."""
        import torch
        self.L = lib()
        torch.cuda.set_device(device)
        self.allocator = TorchAllocator(device) if allocator == "torch" else None
        if allocator not in ("hip", "torch"):
            raise ValueError("allocator must be 'hip' or 'torch'")
        p = _Params(float(dt), float(eta_c), PRECISIONS[precision], SOLVERS[solver], int(n_psi),
                    int(device), stream if stream is not None else _stream())
        if self.allocator is not None:
            p.dev_alloc, p.dev_free = self.allocator.alloc_fn, self.allocator.free_fn
        p.temporal_order = int(order)
        self._p = p
        h = ctypes.c_void_p()
        self._check(self.L.qhp_create(ctypes.byref(p), ctypes.byref(h)), None)
        self.h = h
        self.device = device
        self.precision = precision

    def _check(self, rc, h="self"):
        if rc != 0:
            hh = self.h if h == "self" else h
            msg = self.L.qhp_last_error(hh).decode() if hh else ""
            raise QhpError(rc, msg)

    def mesh(self, xyz, tri):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        self._check(self.L.qhp_mesh(self.h, xyz.ctypes.data, len(xyz), tri.ctypes.data, len(tri)))

    def keep_raw(self, flag=True):
        self._check(self.L.qhp_keep_raw(self.h, int(bool(flag))))

    def assemble(self):
        self._check(self.L.qhp_assemble(self.h))

    def set_precision(self, precision: str):
        self._check(self.L.qhp_set_precision(self.h, PRECISIONS[precision]))
        self.precision = precision

    def set_solver(self, solver: str):
        self._check(self.L.qhp_set_solver(self.h, SOLVERS[solver]))

    def t0_condition(self, power_iters: int = 800):
        """(|T_0|_1 |T_0^{-1}|_1, sigma_max(T_0) / sigma_min(T_0)) (qhp_t0_condition)"""
        c1, c2 = ctypes.c_double(), ctypes.c_double()
        self._check(self.L.qhp_t0_condition(self.h, int(power_iters), ctypes.byref(c1), ctypes.byref(c2)))
        return float(c1.value), float(c2.value)

    def set_growth_limit(self, limit: float):
        """growth trip of the march (qhp_set_growth_limit; 0 turns it off)"""
        self._check(self.L.qhp_set_growth_limit(self.h, float(limit)))

    def profile(self, enable=True):
        self._check(self.L.qhp_profile(self.h, int(bool(enable))))

    def hist_time(self):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._check(self.L.qhp_hist_time(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def band_time(self):
        """factored history: summed ms of the edge-pair and triangle-pair
        banded products and the steps timed (qhp_band_time)"""
        a, b = ctypes.c_double(), ctypes.c_double()
        n = ctypes.c_int64()
        self._check(self.L.qhp_band_time(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(n)))
        return a.value, b.value, n.value

    def set_incident(self, waves, n_steps: int):
        arr = (_Wave * len(waves))(*[to_cwave(w) for w in waves])
        self._check(self.L.qhp_set_incident(self.h, arr, len(waves), int(n_steps)))

    def step(self, j_out=None):
        self._check(self.L.qhp_step(self.h, _ptr(j_out)))

    def run(self, n_steps: int, j_hist=None, y_hist=None):
        self._check(self.L.qhp_run(self.h, int(n_steps), _ptr(j_hist), _ptr(y_hist)))

    def release_assembly(self):
        self._check(self.L.qhp_release_assembly(self.h))

    def set_gmres(self, tol: float = 1e-10, m_max: int = 40, max_refine: int = 4, warm: str = "cold"):
        self._check(self.L.qhp_set_gmres(self.h, float(tol), int(m_max), int(max_refine), WARM[warm]))

    def gmres_stats(self, n: int = 0):
        """Totals since the last reset, and the first n per-step iteration
        counts and start-vector residuals."""
        inf = _GmresInfo()
        it = np.zeros(max(n, 1), dtype=np.int32)
        r0 = np.zeros(max(n, 1), dtype=np.float32)
        self._check(self.L.qhp_gmres_stats(self.h, ctypes.byref(inf), it.ctypes.data, r0.ctypes.data, int(n)))
        out = {k: getattr(inf, k) for k, _ in _GmresInfo._fields_}
        out["iters"], out["res0"] = it[:n], r0[:n]
        return out

    def gmres_reset(self):
        self._check(self.L.qhp_gmres_reset(self.h))

    def attach_mlp(self, mlp):
        self._check(self.L.qhp_attach_mlp(self.h, None if mlp is None else mlp.h))

    def info(self) -> dict:
        inf = _Info()
        self._check(self.L.qhp_query(self.h, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in _Info._fields_}

    def edges(self):
        ne = self.info()["ne"]
        e = np.zeros((ne, 2), dtype=np.int32)
        c = np.zeros((ne, 2), dtype=np.int32)
        self._check(self.L.qhp_edges(self.h, e.ctypes.data, c.ctypes.data))
        return e, c

    def get_matrix(self, which: str, k: int = 0) -> np.ndarray:
        ne = self.info()["ne"]
        out = np.zeros((ne, ne), dtype=np.float64)
        self._check(self.L.qhp_get_matrix(self.h, MAT[which], int(k), out.ctypes.data))
        return out

    def close(self):
        if getattr(self, "h", None):
            self.L.qhp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def check_mesh(xyz, tri):
    """(code, n_edges, n_harmonic, message) of qhp_check_mesh: host-only
    validation of a closed, connected, orientable surface mesh."""
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    ne, nh = ctypes.c_int64(-1), ctypes.c_int64(-1)
    msg = ctypes.create_string_buffer(256)
    rc = lib().qhp_check_mesh(xyz.ctypes.data, len(xyz), tri.ctypes.data, len(tri), ctypes.byref(ne),
                              ctypes.byref(nh), msg, 256)
    return rc, ne.value, nh.value, msg.value.decode()


def history_variants(precision: str, nrhs: int) -> int:
    """number of history-kernel variants (qhp_history_variants)"""
    return lib().qhp_history_variants(PRECISIONS[precision], int(nrhs))


def batch_variants(precision: str, nrhs: int) -> int:
    """number of history tile shapes of a batch (qhp_batch_variants)"""
    return lib().qhp_batch_variants(PRECISIONS[precision], int(nrhs))


def history_sum(precision: str, slabs, scales, ring, head: int, r, b, kmax: int | None = None, variant: int = -1):
    """b = r - sum_{k=1}^{kmax} T_k y_{i-k} on caller tensors (see qhp_history_sum).

    slabs: [kmax, ne, ld] (float64 / float32 / bfloat16) or, for bf16x2,
    [kmax, ceil(ne/16), ld/32, 2, 512] bfloat16 in matrix-core operand order,
    or, for i8x4, [kmax, block bytes] int8 (digit planes then FP64 row
    scales); scales: float32 [kmax] (bf16 only); ring: [n_slots, ld, nrhs]
    float64 (f64, f32a) or float32, [n_slots, nrp/16, ld/32, 3, 512]
    bfloat16 (bf16 with nrhs > 1, bf16x2) or [n_slots, slot bytes] int8
    (i8x4); r, b: float64 [ne, nrhs]."""
    L = lib()
    kmax = slabs.shape[0] if kmax is None else kmax
    if precision == "bf16x2":  # operand-ordered planes: ld from the tile count, ne from r
        ne, ld = r.shape[0], slabs.shape[2] * 32
    elif precision == "i8x4":  # block bytes = R * ld * 4 + R * 8, R = ne rounded up to 16
        ne = r.shape[0]
        R = (ne + 15) // 16 * 16
        ld = (slabs.shape[-1] - 8 * R) // (4 * R)
    else:
        ne, ld = slabs.shape[-2], slabs.shape[-1]
    nrhs = r.shape[1] if r.dim() == 2 else 1
    rc = L.qhp_history_sum_variant(_stream(), PRECISIONS[precision], ne, ld, nrhs, kmax, _ptr(slabs), _ptr(scales),
                                   _ptr(ring), ring.shape[0], int(head), _ptr(r), _ptr(b), int(variant))
    if rc != 0:
        raise QhpError(rc, "qhp_history_sum")


def history_sum_noalloc(precision: str, slabs, scales, ring, head: int, r, b, kmax: int | None = None,
                        variant: int = -1):
    """qhp_history_sum_noalloc: history_sum's arguments, no device allocation
    (partial sums in the library's fixed per-device array); only enqueues
    the work on the current stream."""
    L = lib()
    kmax = slabs.shape[0] if kmax is None else kmax
    if precision == "bf16x2":
        ne, ld = r.shape[0], slabs.shape[2] * 32
    elif precision == "i8x4":
        ne = r.shape[0]
        R = (ne + 15) // 16 * 16
        ld = (slabs.shape[-1] - 8 * R) // (4 * R)
    else:
        ne, ld = slabs.shape[-2], slabs.shape[-1]
    nrhs = r.shape[1] if r.dim() == 2 else 1
    rc = L.qhp_history_sum_noalloc(_stream(), PRECISIONS[precision], ne, ld, nrhs, kmax, _ptr(slabs), _ptr(scales),
                                   _ptr(ring), ring.shape[0], int(head), _ptr(r), _ptr(b), int(variant))
    if rc != 0:
        raise QhpError(rc, "qhp_history_sum_noalloc")


class Batch:
    """Many scatterers marched together, one graph replay per step
    (qhp_batch_*).  Keeps the solvers alive while it exists."""

    def __init__(self, solvers, variant: int = -1):
        """variant: history tile shape in [0, batch_variants(precision, n_rhs)),
        or -1 to autotune it."""
        self.L = lib()
        self.solvers = list(solvers)
        arr = (ctypes.c_void_p * len(self.solvers))(*[s.h.value for s in self.solvers])
        h = ctypes.c_void_p()
        rc = self.L.qhp_batch_create_variant(arr, len(self.solvers), int(variant), ctypes.byref(h))
        if rc != 0:
            raise QhpError(rc, self.L.qhp_last_error(self.solvers[0].h).decode())
        self.h = h

    @property
    def variant(self) -> int:
        """the history tile shape in use"""
        return int(self.L.qhp_batch_history_variant(self.h))

    def run(self, n_steps: int, j_hists=None):
        ptrs = None
        if j_hists is not None:
            ptrs = (ctypes.c_void_p * len(self.solvers))(*[(None if t is None else t.data_ptr()) for t in j_hists])
        rc = self.L.qhp_batch_run(self.h, int(n_steps), ptrs)
        if rc != 0:
            raise QhpError(rc, self.L.qhp_batch_last_error(self.h).decode())

    def step_times(self, n: int):
        out = (ctypes.c_float * n)()
        self.L.qhp_batch_step_times(self.h, out, n)
        return np.array(out[:], dtype=np.float64)

    def close(self):
        if getattr(self, "h", None):
            self.L.qhp_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MLP:
    """The warm-start perceptron of a solver's mesh (qhp_mlp_*)."""

    def __init__(self, solver: Solver, hidden: int = 256, seed: int = 0):
        self.L = lib()
        self.solver = solver
        h = ctypes.c_void_p()
        rc = self.L.qhp_mlp_create(solver.h, int(hidden), int(seed), ctypes.byref(h))
        if rc != 0:
            raise QhpError(rc, self.L.qhp_last_error(solver.h).decode())
        self.h = h
        nf, npar, hid = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self.L.qhp_mlp_dims(h, ctypes.byref(nf), ctypes.byref(npar), ctypes.byref(hid))
        self.nf, self.n_params, self.hidden = nf.value, npar.value, hid.value
        self.n_in = 4 * self.nf

    def _check(self, rc):
        if rc != 0:
            raise QhpError(rc, self.L.qhp_mlp_last_error(self.h).decode())

    def layout(self):
        """(name, shape) of the parameter vector's segments, in order."""
        H, ni, nf = self.hidden, self.n_in, self.nf
        return [("W1", (H, ni)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (nf, H)), ("b3", (nf,))]

    def unpack(self, flat):
        out, o = {}, 0
        for name, shape in self.layout():
            n = int(np.prod(shape))
            out[name] = flat[o:o + n].reshape(shape)
            o += n
        return out

    def pack(self, params: dict) -> np.ndarray:
        return np.concatenate([np.asarray(params[k], dtype=np.float32).reshape(-1) for k, _ in self.layout()])

    def set_params(self, params):
        flat = np.ascontiguousarray(self.pack(params) if isinstance(params, dict) else params, dtype=np.float32)
        self._check(self.L.qhp_mlp_set_params(self.h, flat.ctypes.data))

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.n_params, dtype=np.float32)
        self._check(self.L.qhp_mlp_get_params(self.h, out.ctypes.data))
        return out

    def features(self, y):
        import torch
        f = torch.empty((y.shape[0], self.nf), dtype=torch.float64, device=y.device)
        self._check(self.L.qhp_mlp_features(self.h, _ptr(y), y.shape[0], _ptr(f)))
        return f

    def guess(self, f4):
        """f4: device float64 [4, nf] (f_{i-1} .. f_{i-4}) -> guess of f_i."""
        import torch
        g = torch.empty((self.nf,), dtype=torch.float64, device=f4.device)
        self._check(self.L.qhp_mlp_guess(self.h, _ptr(f4), _ptr(g)))
        return g

    def reconstruct(self, f):
        import torch
        ne = self.solver.info()["ne"]
        y = torch.empty((f.shape[0], ne), dtype=torch.float64, device=f.device)
        self._check(self.L.qhp_mlp_reconstruct(self.h, _ptr(f), f.shape[0], _ptr(y)))
        return y

    def forward(self, x):
        import torch
        out = torch.empty((x.shape[0], self.nf), dtype=torch.float32, device=x.device)
        self._check(self.L.qhp_mlp_forward(self.h, _ptr(x), x.shape[0], _ptr(out)))
        return out

    def loss_grad(self, x, t):
        loss = ctypes.c_double()
        g = np.zeros(self.n_params, dtype=np.float32)
        self._check(self.L.qhp_mlp_loss_grad(self.h, _ptr(x), _ptr(t), x.shape[0], ctypes.byref(loss),
                                             g.ctypes.data))
        return loss.value, g

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self._check(self.L.qhp_mlp_adam(self.h, lr, beta1, beta2, eps))

    def train(self, y_hist, epochs: int, batch: int = 512, lr: float = 1e-3, seed: int = 0):
        """y_hist: device float64 [n_steps, ne, n_runs]; returns the per-epoch losses."""
        losses = np.zeros(epochs, dtype=np.float64)
        n_steps, _, n_runs = y_hist.shape
        self._check(self.L.qhp_mlp_train(self.h, _ptr(y_hist), n_runs, n_steps, int(epochs), int(batch),
                                         float(lr), int(seed), losses.ctypes.data))
        return losses

    def close(self):
        if getattr(self, "h", None):
            self.L.qhp_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
