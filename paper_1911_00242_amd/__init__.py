"""Python binding of libccsdk (k-point CCSD T2 residual on MI355X).

Argument marshalling only: every step of the residual, the update, the norm, the energy
and DIIS runs in the HIP library ``libccsdk.so`` built next to this file by
``paper_1911_00242_amd.build``.  The functions below carry the names of the C ABI in
``include/ccsd_k.h``; :class:`Context` bundles them with a torch-allocated device
workspace.  Importing this package fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libccsdk.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_1911_00242_amd.build` "
        "(or __graft_entry__.build()); there is no fallback implementation")

# torch ships its own HIP runtime with the same SONAME (libamdhip64.so.7) as the one
# libccsdk links against.  Loading torch first makes the dynamic linker resolve
# libccsdk's dependency to that already-loaded runtime, so the process holds one HIP
# runtime and torch-allocated workspaces and streams are valid inside the library.
import torch  # noqa: E402,F401  (load order matters, see above)

_lib = ctypes.CDLL(LIB_PATH)

OK, NOT_CONVERGED, EINVAL, ENOMEM, EDEVICE, ESTATE, ENUMERIC = 0, 1, -1, -2, -3, -4, -5
PREC_FP64, PREC_MIXED = 0, 1
GROUPING_STANDARD, GROUPING_REARRANGED = 0, 1
FORM_SPLIT2_PRESPLIT, FORM_SPLIT2, FORM_SPLIT3, FORM_FP32 = 0, 1, 2, 3
TILE_32X32, TILE_64X64, TILE_128X64, TILE_64X128 = 0, 1, 2, 3
FORMS = ("split2_presplit", "split2", "split3", "fp32")
CLASSES = ("oooo", "ooov", "oovv", "ovvo", "ovvv", "vvvv")
STAGES = ("pp_ladder", "hh_ladder", "w_mnij", "w_mbej", "ring", "residual")


class ccsd_k_system(ctypes.Structure):
    _fields_ = [("grid", ctypes.c_int32 * 3), ("n_occ", ctypes.c_int32), ("n_vir", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("diis_space", ctypes.c_int32),
                ("synthetic", ctypes.c_int32), ("seed", ctypes.c_uint64), ("eri_scale", ctypes.c_double),
                ("grouping", ctypes.c_int32)]


_p = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_i32, _i64, _u64, _f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double


def _sig(name, res, args):
    fn = getattr(_lib, name)
    fn.restype = res
    fn.argtypes = args
    return fn


_lib_init = _sig("ccsd_k_init", ctypes.c_int, [ctypes.POINTER(ccsd_k_system), _i32, _p, ctypes.POINTER(_p)])
_lib_ws = _sig("ccsd_k_workspace_bytes", ctypes.c_int, [_p, ctypes.POINTER(_u64)])
_lib_bind = _sig("ccsd_k_bind_workspace", ctypes.c_int, [_p, _p, _u64])
_lib_set_inputs = _sig("ccsd_k_set_inputs", ctypes.c_int, [_p, _i32, _dp, ctypes.POINTER(_dp)])
_lib_residual = _sig("ccsd_k_residual", ctypes.c_int, [_p, _i32, _dp, _dp, _dp, _dp])
_lib_iterate = _sig("ccsd_k_iterate", ctypes.c_int, [_p, _i32, _f64, ctypes.POINTER(_i32), _dp])
_lib_rnorm = _sig("ccsd_k_residual_norm", ctypes.c_int, [_p, _i32, _dp])
_lib_energy = _sig("ccsd_k_energy", ctypes.c_int, [_p, _i32, _dp, _dp])
_lib_get_amp = _sig("ccsd_k_get_amplitudes", ctypes.c_int, [_p, _i32, _dp, _dp])
_lib_set_amp = _sig("ccsd_k_set_amplitudes", ctypes.c_int, [_p, _i32, _dp, _dp])
_lib_flops = _sig("ccsd_k_flops", ctypes.c_int, [_p, _i32, _dp, _dp])
_lib_shape = _sig("ccsd_k_product_shape", ctypes.c_int, [_p, _i32, _i32] + [ctypes.POINTER(_i64)] * 4)
_lib_set_form = _sig("ccsd_k_set_product_form", ctypes.c_int, [_p, _i32, _i32, _i32])
_lib_get_form = _sig("ccsd_k_get_product_form", ctypes.c_int, [_p, _i32, _i32, ctypes.POINTER(_i32)])
_lib_set_tile = _sig("ccsd_k_set_product_tile", ctypes.c_int, [_p, _i32, _i32, _i32])
_lib_get_tile = _sig("ccsd_k_get_product_tile", ctypes.c_int, [_p, _i32, _i32, ctypes.POINTER(_i32)])
_lib_autotune = _sig("ccsd_k_autotune", ctypes.c_int, [_p, _i32, _f64, ctypes.c_char_p, ctypes.POINTER(_i32), _dp])
_lib_escalation = _sig("ccsd_k_set_escalation", ctypes.c_int, [_p, _i32])
_lib_graphs = _sig("ccsd_k_set_graphs", ctypes.c_int, [_p, _i32])
_lib_overlap = _sig("ccsd_k_set_overlap", ctypes.c_int, [_p, _i32])
_lib_timing = _sig("ccsd_k_timing", ctypes.c_int, [_p, _i32])
_lib_timing_get = _sig("ccsd_k_timing_get", ctypes.c_int, [_p, _i32, _dp, ctypes.POINTER(_i64)])
_lib_free = _sig("ccsd_k_free", None, [_p])
_lib_dbg_gemm = _sig("ccsd_k_debug_zgemm", ctypes.c_int, [_i32, _i32, _i32, _i32, _dp, _dp, _dp, _i32])
_lib_noalloc_gemm = _sig("ccsd_k_zgemm_noalloc", ctypes.c_int, [_i32, _i32, _i32, _i32, _p, _p, _p, _i32, _p])
_lib_err = _sig("ccsd_k_last_error", ctypes.c_char_p, [_p])

SYMBOLS = ("ccsd_k_init", "ccsd_k_workspace_bytes", "ccsd_k_bind_workspace", "ccsd_k_set_inputs",
           "ccsd_k_residual", "ccsd_k_iterate", "ccsd_k_residual_norm", "ccsd_k_energy",
           "ccsd_k_get_amplitudes", "ccsd_k_set_amplitudes", "ccsd_k_flops", "ccsd_k_product_shape",
           "ccsd_k_set_product_form", "ccsd_k_get_product_form", "ccsd_k_set_product_tile",
           "ccsd_k_get_product_tile", "ccsd_k_autotune", "ccsd_k_set_escalation", "ccsd_k_set_graphs", "ccsd_k_set_overlap",
           "ccsd_k_timing",
           "ccsd_k_timing_get", "ccsd_k_debug_zgemm", "ccsd_k_zgemm_noalloc", "ccsd_k_free", "ccsd_k_last_error")


class CcsdKError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libccsdk error {code}: {msg}")
        self.code = code


def _check(rc, ctx):
    if rc < 0:
        raise CcsdKError(rc, ccsd_k_last_error(ctx))
    return rc


def _ptr(a):
    if a is None:
        return None
    if not (a.flags.c_contiguous and a.dtype in (np.complex128, np.float64)):
        raise ValueError("arrays must be C-contiguous complex128")
    return a.ctypes.data_as(_dp)


# ---------------------------------------------------------------- C ABI, same names
def ccsd_k_last_error(ctx=None) -> str:
    r = _lib_err(ctx)
    return r.decode() if r else ""


def ccsd_k_init(systems, stream=None):
    arr = (ccsd_k_system * len(systems))()
    for i, s in enumerate(systems):
        g = tuple(s["grid"])
        arr[i].grid[:] = g
        arr[i].n_occ, arr[i].n_vir = int(s["no"]), int(s["nv"])
        arr[i].precision = int(s.get("precision", PREC_FP64))
        arr[i].diis_space = int(s.get("diis_space", 0))
        arr[i].synthetic = int(s.get("synthetic", 0))
        arr[i].seed = int(s.get("seed", 0))
        arr[i].eri_scale = float(s.get("eri_scale", 0.05))
        arr[i].grouping = int(s.get("grouping", GROUPING_STANDARD))
    out = _p()
    _check(_lib_init(arr, len(systems), stream, ctypes.byref(out)), None)
    return out


def ccsd_k_workspace_bytes(ctx) -> int:
    b = _u64()
    _check(_lib_ws(ctx, ctypes.byref(b)), ctx)
    return int(b.value)


def ccsd_k_bind_workspace(ctx, device_ptr: int, nbytes: int):
    return _check(_lib_bind(ctx, device_ptr, nbytes), ctx)


def ccsd_k_set_inputs(ctx, sys: int, fock: np.ndarray, eris: dict):
    arrs = [np.ascontiguousarray(eris[c], dtype=np.complex128) for c in CLASSES]
    fock = np.ascontiguousarray(fock, dtype=np.complex128)
    ptrs = (_dp * 6)(*[_ptr(a) for a in arrs])
    return _check(_lib_set_inputs(ctx, sys, _ptr(fock), ptrs), ctx)


def ccsd_k_residual(ctx, sys, t1=None, t2=None, r1=None, r2=None):
    return _check(_lib_residual(ctx, sys, _ptr(t1), _ptr(t2), _ptr(r1), _ptr(r2)), ctx)


def ccsd_k_iterate(ctx, max_iter: int, tol: float):
    it, rn = _i32(), _f64()
    rc = _check(_lib_iterate(ctx, max_iter, tol, ctypes.byref(it), ctypes.byref(rn)), ctx)
    return rc, int(it.value), float(rn.value)


def ccsd_k_residual_norm(ctx, sys) -> float:
    r = _f64()
    _check(_lib_rnorm(ctx, sys, ctypes.byref(r)), ctx)
    return float(r.value)


def ccsd_k_energy(ctx, sys) -> complex:
    re, im = _f64(), _f64()
    _check(_lib_energy(ctx, sys, ctypes.byref(re), ctypes.byref(im)), ctx)
    return complex(re.value, im.value)


def ccsd_k_get_amplitudes(ctx, sys, t1: np.ndarray, t2: np.ndarray):
    return _check(_lib_get_amp(ctx, sys, _ptr(t1), _ptr(t2)), ctx)


def ccsd_k_set_amplitudes(ctx, sys, t1=None, t2=None):
    return _check(_lib_set_amp(ctx, sys, _ptr(t1), _ptr(t2)), ctx)


def ccsd_k_flops(ctx, sys):
    g, o = _f64(), _f64()
    _check(_lib_flops(ctx, sys, ctypes.byref(g), ctypes.byref(o)), ctx)
    return float(g.value), float(o.value)


def ccsd_k_product_shape(ctx, sys, product):
    out = [_i64() for _ in range(4)]
    _check(_lib_shape(ctx, sys, product, *[ctypes.byref(x) for x in out]), ctx)
    return tuple(int(x.value) for x in out)


def ccsd_k_set_product_form(ctx, sys, product, form):
    return _check(_lib_set_form(ctx, sys, product, form), ctx)


def ccsd_k_get_product_form(ctx, sys, product) -> int:
    f = _i32()
    _check(_lib_get_form(ctx, sys, product, ctypes.byref(f)), ctx)
    return int(f.value)


def ccsd_k_set_product_tile(ctx, sys, product, tile):
    return _check(_lib_set_tile(ctx, sys, product, tile), ctx)


def ccsd_k_get_product_tile(ctx, sys, product) -> int:
    t = _i32()
    _check(_lib_get_tile(ctx, sys, product, ctypes.byref(t)), ctx)
    return int(t.value)


def ccsd_k_autotune(ctx, sys, budget, cache_path=None):
    """Returns (forms per product, report[product][form] = (ms, error))."""
    forms = (_i32 * 5)()
    rep = np.zeros((5, 4, 2))
    path = None if cache_path is None else os.fsencode(cache_path)
    _check(_lib_autotune(ctx, sys, float(budget), path, forms, rep.ctypes.data_as(_dp)), ctx)
    return [int(x) for x in forms], rep


def ccsd_k_set_escalation(ctx, enable: bool):
    return _check(_lib_escalation(ctx, 1 if enable else 0), ctx)


def ccsd_k_set_graphs(ctx, enable: bool):
    return _check(_lib_graphs(ctx, 1 if enable else 0), ctx)


def ccsd_k_set_overlap(ctx, enable: bool):
    return _check(_lib_overlap(ctx, 1 if enable else 0), ctx)


def ccsd_k_timing(ctx, enable: bool):
    return _check(_lib_timing(ctx, 1 if enable else 0), ctx)


def ccsd_k_timing_get(ctx, stage: int):
    ms, n = _f64(), _i64()
    _check(_lib_timing_get(ctx, stage, ctypes.byref(ms), ctypes.byref(n)), ctx)
    return float(ms.value), int(n.value)


def ccsd_k_debug_zgemm(A: np.ndarray, B: np.ndarray, reference=False) -> np.ndarray:
    """C[g] = A[g] @ B[g].T on the device (A [G,M,K], B [G,N,K] complex128).
    reference: False/0 tiled FP64 MFMA, True/1 per-element FP64, 2 split-BF16 MFMA on pre-split
    operands; on complex64 operands 3 two-term split-BF16, 4 three-term split-BF16, 5 FP32 MFMA;
    23, 24, 25 the same three forms summed over 64-k chunks in FP64 in one launch;
    10 + t the tiled FP64 kernel in tile shape t (TILE_*)."""
    A = np.ascontiguousarray(A, dtype=np.complex128)
    B = np.ascontiguousarray(B, dtype=np.complex128)
    G, M, K = A.shape
    N = B.shape[1]
    C = np.empty((G, M, N), np.complex128)
    _check(_lib_dbg_gemm(G, M, N, K, _ptr(A), _ptr(B), _ptr(C), int(reference)), None)
    return C


def ccsd_k_zgemm_noalloc(G, M, N, K, a_ptr: int, b_ptr: int, c_ptr: int, variant: int = 0, stream=None):
    """C[g] = A[g] @ B[g].T on device arrays given by address (complex128, dense row-major),
    enqueued on ``stream`` (a hipStream_t address or None) without any allocation."""
    return _check(_lib_noalloc_gemm(G, M, N, K, a_ptr, b_ptr, c_ptr, variant, stream), None)


def ccsd_k_free(ctx):
    _lib_free(ctx)


# ---------------------------------------------------------------- convenience wrapper
class Context:
    """A libccsdk context with its device workspace held by a torch uint8 tensor."""

    def __init__(self, systems, device="cuda", stream=None):
        import torch

        self.systems = [dict(s) for s in systems]
        self._torch = torch
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.ctx = ccsd_k_init(self.systems, ctypes.c_void_p(self.stream.cuda_stream))
        try:
            nbytes = ccsd_k_workspace_bytes(self.ctx)
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
            base = self.workspace.data_ptr()
            aligned = (base + 255) // 256 * 256
            ccsd_k_bind_workspace(self.ctx, aligned, nbytes)
        except Exception:
            ccsd_k_free(self.ctx)
            self.ctx = None
            raise
        self.nbytes = nbytes

    def dims(self, sys):
        s = self.systems[sys]
        N = int(np.prod(s["grid"]))
        return N, int(s["no"]), int(s["nv"])

    def set_inputs(self, sys, fock, eris):
        ccsd_k_set_inputs(self.ctx, sys, fock, eris)

    def residual(self, sys=0, t1=None, t2=None, fetch=True):
        N, no, nv = self.dims(sys)
        t1 = None if t1 is None else np.ascontiguousarray(t1, dtype=np.complex128)
        t2 = None if t2 is None else np.ascontiguousarray(t2, dtype=np.complex128)
        r1 = np.empty((N, no, nv), np.complex128) if fetch else None
        r2 = np.empty((N, N, N, no, no, nv, nv), np.complex128) if fetch else None
        ccsd_k_residual(self.ctx, sys, t1, t2, r1, r2)
        return r1, r2

    def iterate(self, max_iter, tol):
        return ccsd_k_iterate(self.ctx, max_iter, tol)

    def energy(self, sys=0):
        return ccsd_k_energy(self.ctx, sys)

    def residual_norm(self, sys=0):
        return ccsd_k_residual_norm(self.ctx, sys)

    def get_amplitudes(self, sys=0):
        N, no, nv = self.dims(sys)
        t1 = np.empty((N, no, nv), np.complex128)
        t2 = np.empty((N, N, N, no, no, nv, nv), np.complex128)
        ccsd_k_get_amplitudes(self.ctx, sys, t1, t2)
        return t1, t2

    def set_amplitudes(self, sys, t1, t2):
        ccsd_k_set_amplitudes(self.ctx, sys, np.ascontiguousarray(t1, dtype=np.complex128),
                              np.ascontiguousarray(t2, dtype=np.complex128))

    def flops(self, sys=0):
        return ccsd_k_flops(self.ctx, sys)

    def product_shape(self, product, sys=0):
        """(G, M, N, K) of a grouped product as executed; product is a stage name or number."""
        return ccsd_k_product_shape(self.ctx, sys, STAGES.index(product) if isinstance(product, str) else product)

    def set_product_form(self, product, form, sys=0):
        ccsd_k_set_product_form(self.ctx, sys, STAGES.index(product) if isinstance(product, str) else product, form)

    def product_form(self, product, sys=0):
        return ccsd_k_get_product_form(self.ctx, sys, STAGES.index(product) if isinstance(product, str) else product)

    def set_product_tile(self, product, tile, sys=0):
        ccsd_k_set_product_tile(self.ctx, sys, STAGES.index(product) if isinstance(product, str) else product, tile)

    def product_tile(self, product, sys=0):
        return ccsd_k_get_product_tile(self.ctx, sys, STAGES.index(product) if isinstance(product, str) else product)

    def autotune(self, budget, cache_path=None, sys=0):
        return ccsd_k_autotune(self.ctx, sys, budget, cache_path)

    def set_escalation(self, enable=True):
        ccsd_k_set_escalation(self.ctx, enable)

    def set_graphs(self, enable=True):
        ccsd_k_set_graphs(self.ctx, enable)

    def set_overlap(self, enable=True):
        ccsd_k_set_overlap(self.ctx, enable)

    def timing(self, enable=True):
        ccsd_k_timing(self.ctx, enable)

    def timing_get(self, stage):
        return ccsd_k_timing_get(self.ctx, STAGES.index(stage) if isinstance(stage, str) else stage)

    def close(self):
        if self.ctx is not None:
            ccsd_k_free(self.ctx)
            self.ctx = None
            self.workspace = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
