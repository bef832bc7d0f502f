"""Seeded synthetic inputs for k-point CCSD test systems (input generation only).

The recipe is documented at the top of ``synth.c``: counter-based splitmix64 draws,
Box-Muller complex Gaussians scaled by ``scale``, then the antisymmetrizing and
Hermitizing projectors, so that <pq||rs> = -<qp||rs> = -<pq||sr> = conj(<rs||pq>)
(the integral symmetries the paper states for its rearranged equations, Sec. 3.3).

This module serves both the CPU oracle and the tests of the GPU library; it holds none
of the coupled-cluster arithmetic.  The compiled helper ``libsynth.so`` is built with
gcc by :func:`build`.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsynth.so")
_lib = None

CLASSES = ("oooo", "ooov", "oovv", "ovvo", "ovvv", "vvvv")
DEFAULT_SCALE = 0.05


def build() -> str:
    """Compile ``synth.c`` into ``libsynth.so`` (gcc, OpenMP)."""
    src = os.path.join(_HERE, "synth.c")
    tmp = _SO + ".tmp"
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        i32p = ctypes.POINTER(ctypes.c_int32)
        dp = ctypes.POINTER(ctypes.c_double)
        u64, c_int, c_double = ctypes.c_uint64, ctypes.c_int, ctypes.c_double
        lib.synth_stream_state.restype = u64
        lib.synth_stream_state.argtypes = [u64, u64]
        lib.synth_draw.restype = u64
        lib.synth_draw.argtypes = [u64, u64]
        lib.synth_kconserve.restype = c_int
        lib.synth_kconserve.argtypes = [i32p, c_int, c_int, c_int]
        lib.synth_eri_element.restype = None
        lib.synth_eri_element.argtypes = [u64, i32p, c_int, c_double] + [c_int] * 7 + [dp]
        lib.synth_eri_block.restype = c_int
        lib.synth_eri_block.argtypes = [u64, i32p, c_int, c_int, c_double, ctypes.c_char_p,
                                        c_int, c_int, c_int, dp]
        lib.synth_eri_class.restype = c_int
        lib.synth_eri_class.argtypes = [u64, i32p, c_int, c_int, c_double, ctypes.c_char_p, dp]
        lib.synth_fock.restype = c_int
        lib.synth_fock.argtypes = [u64, i32p, c_int, c_int, dp]
        lib.synth_uniforms.restype = c_int
        lib.synth_uniforms.argtypes = [u64, u64, u64, dp]
        lib.synth_test_amplitudes.restype = c_int
        lib.synth_test_amplitudes.argtypes = [u64, i32p, c_int, c_int, c_double, dp, dp]
        _lib = lib
    return _lib


def _grid(grid):
    g = tuple(int(x) for x in grid)
    if len(g) != 3 or min(g) < 1:
        raise ValueError(f"grid must be three positive ints, got {grid}")
    return (ctypes.c_int32 * 3)(*g), g[0] * g[1] * g[2]


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def class_dims(cls: str, no: int, nv: int):
    return tuple({"o": no, "v": nv, "n": no + nv}[c] for c in cls)


def draw(seed: int, tag: int, n: int) -> int:
    lib = _load()
    return int(lib.synth_draw(lib.synth_stream_state(seed, tag), n))


def stream_state(seed: int, tag: int) -> int:
    return int(_load().synth_stream_state(seed, tag))


def kconserve(grid, kp: int, kq: int, kr: int) -> int:
    g, _ = _grid(grid)
    return int(_load().synth_kconserve(g, kp, kq, kr))


def kconserv_table(grid) -> np.ndarray:
    """Table KC[kp,kq,kr] = k_s with k_p + k_q = k_r + k_s (mod the grid), C-order k."""
    g, N = _grid(grid)
    lib = _load()
    kc = np.empty((N, N, N), dtype=np.int64)
    for a in range(N):
        for b in range(N):
            for c in range(N):
                kc[a, b, c] = lib.synth_kconserve(g, a, b, c)
    return kc


def eri_element(seed, grid, no, nv, kp, kq, kr, p, q, r, s, scale=DEFAULT_SCALE) -> complex:
    g, _ = _grid(grid)
    out = np.zeros(2)
    _load().synth_eri_element(seed, g, no + nv, scale, kp, kq, kr, p, q, r, s, _dp(out))
    return complex(out[0], out[1])


def eri_block(seed, grid, no, nv, cls, kp, kq, kr, scale=DEFAULT_SCALE) -> np.ndarray:
    g, _ = _grid(grid)
    dims = class_dims(cls, no, nv)
    out = np.empty(dims, dtype=np.complex128)
    rc = _load().synth_eri_block(seed, g, no, nv, scale, cls.encode(), kp, kq, kr, _dp(out))
    if rc:
        raise ValueError(cls)
    return out


def eri_class(seed, grid, no, nv, cls, scale=DEFAULT_SCALE) -> np.ndarray:
    """Class ``cls`` (4 chars of o/v/n) for every momentum triple: [kp,kq,kr,d0,d1,d2,d3]."""
    g, N = _grid(grid)
    dims = class_dims(cls, no, nv)
    out = np.empty((N, N, N) + dims, dtype=np.complex128)
    rc = _load().synth_eri_class(seed, g, no, nv, scale, cls.encode(), _dp(out))
    if rc:
        raise ValueError(cls)
    return out


def fock(seed, grid, no, nv) -> np.ndarray:
    g, N = _grid(grid)
    out = np.empty((N, no + nv, no + nv), dtype=np.complex128)
    _load().synth_fock(seed, g, no, nv, _dp(out))
    return out


def uniforms(seed, tag, count) -> np.ndarray:
    out = np.empty(int(count), dtype=np.float64)
    _load().synth_uniforms(seed, tag, int(count), _dp(out))
    return out


def test_amplitudes(seed, grid, no, nv, scale=0.02):
    """Random (t1, t2) of magnitude ``scale`` with the symmetry of CCSD amplitudes."""
    g, N = _grid(grid)
    t1 = np.empty((N, no, nv), dtype=np.complex128)
    t2 = np.empty((N, N, N, no, no, nv, nv), dtype=np.complex128)
    _load().synth_test_amplitudes(seed, g, no, nv, scale, _dp(t1), _dp(t2))
    return t1, t2


def system(seed, grid, no, nv, scale=DEFAULT_SCALE):
    """Fock matrix and the six stored integral classes of one synthetic system."""
    f = fock(seed, grid, no, nv)
    eris = {c: eri_class(seed, grid, no, nv, c, scale) for c in CLASSES}
    return f, eris


def batch_shapes(seed: int, count: int):
    """Shapes of a batch of independent systems (tag 3): N_k from {1,2,4,8} (1-D grids up
    to 4, 2x2x2 for 8), n_occ from {4,6,8,12}, n_vir from {8,16,24,32}; system s uses
    seed ``seed + s`` for its integrals."""
    u = uniforms(seed, 3, 3 * count)
    nks, nos, nvs = (1, 2, 4, 8), (4, 6, 8, 12), (8, 16, 24, 32)
    out = []
    for s in range(count):
        nk = nks[min(3, int(u[3 * s] * 4))]
        grid = (2, 2, 2) if nk == 8 else (nk, 1, 1)
        out.append(dict(grid=grid, no=nos[min(3, int(u[3 * s + 1] * 4))],
                        nv=nvs[min(3, int(u[3 * s + 2] * 4))], seed=seed + s))
    return out
