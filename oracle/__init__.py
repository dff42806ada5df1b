"""CPU oracle for the ZNCC -> DT -> WTA stereo path.  TEST INFRASTRUCTURE ONLY.

Plain single-threaded C (``zdt_oracle.c``) in int64 / IEEE double, wrapped with
ctypes.  It follows the paper's definitions: the ZNCC of Eq. ZNCC (Sec. III-A),
the DT recursions Eqs. DT1-DT4 with the weights of Eqs. k1-k4/a (Sec. III-B)
and the WTA of Eq. WTA1 (Sec. III-C).  It shares nothing with the HIP library;
only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it.

Every function here is pinned by ``tests/test_oracle_pins.py`` against
closed forms, independent library routines and brute force; none is "parity
unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from collections import namedtuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "zdt_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        I = ctypes.c_int
        Dbl = ctypes.c_double
        lib.oracle_window_sums.argtypes = [P, P, I, I, I, I, I, P, P, P, P]
        lib.oracle_cross_sums.argtypes = [P, P, I, I, I, I, I, P]
        lib.oracle_cross_sum_at.argtypes = [P, P, I, I, I, I, I, I, I]
        lib.oracle_cross_sum_at.restype = ctypes.c_int64
        lib.oracle_zncc_at.argtypes = [P, P, I, I, I, I, I, I, I]
        lib.oracle_zncc_at.restype = Dbl
        lib.oracle_zncc_cost_slice.argtypes = [P, P, I, I, I, I, I, P]
        lib.oracle_zncc_cost.argtypes = [P, P, I, I, I, I, I, P]
        lib.oracle_dt_weights.argtypes = [P, I, I, I, Dbl, Dbl, P, P]
        lib.oracle_dt_slice.argtypes = [P, I, I, P, P, I]
        lib.oracle_dt_aggregate.argtypes = [P, I, I, I, P, P, I]
        lib.oracle_wta.argtypes = [P, I, I, I, P]
        lib.oracle_stereo_solve.argtypes = [P, P, I, I, I, I, I, Dbl, Dbl, I, I, P, P]
        lib.oracle_sgm_aggregate.argtypes = [P, I, I, I, Dbl, Dbl, Dbl, P]
        lib.oracle_int_solve.argtypes = [P, P, I, I, I, I, I, Dbl, Dbl, I, I, Dbl, I, I, I, P, P, P]
        lib.oracle_dt_passes.argtypes = [P, I, I, P, P, I, I]
        lib.oracle_dt_passes.restype = ctypes.c_int
        lib.oracle_int_solve.restype = ctypes.c_int
        lib.oracle_sgm_aggregate.restype = ctypes.c_int
        lib.oracle_i8_encode.argtypes = [ctypes.c_int16]
        lib.oracle_i8_encode.restype = ctypes.c_uint8
        lib.oracle_i8_decode.argtypes = [ctypes.c_uint8]
        lib.oracle_i8_decode.restype = ctypes.c_int16
        for f in ("oracle_window_sums", "oracle_cross_sums", "oracle_zncc_cost_slice", "oracle_zncc_cost",
                  "oracle_dt_weights", "oracle_dt_slice", "oracle_dt_aggregate", "oracle_wta",
                  "oracle_stereo_solve"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


def _u8(img):
    a = np.ascontiguousarray(img, dtype=np.uint8)
    assert a.ndim == 2
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc, name):
    if rc != 0:
        raise ValueError(f"oracle {name} rejected its arguments (rc={rc})")


def window_sums(left, right, D, r):
    """int64 (S_L, S_LL, S_T, S_TT); S_T/S_TT are [H][W+D-1] over x' = -(D-1)..W-1."""
    L, R = _u8(left), _u8(right)
    H, W = L.shape
    S_L = np.empty((H, W), np.int64)
    S_LL = np.empty((H, W), np.int64)
    S_T = np.empty((H, W + D - 1), np.int64)
    S_TT = np.empty((H, W + D - 1), np.int64)
    _check(_load().oracle_window_sums(_ptr(L), _ptr(R), W, W, H, D, r, _ptr(S_L), _ptr(S_LL), _ptr(S_T),
                                      _ptr(S_TT)), "window_sums")
    return S_L, S_LL, S_T, S_TT


def cross_sums(left, right, D, r):
    """int64 S_RT [H][W][D] by brute force."""
    L, R = _u8(left), _u8(right)
    H, W = L.shape
    out = np.empty((H, W, D), np.int64)
    _check(_load().oracle_cross_sums(_ptr(L), _ptr(R), W, W, H, D, r, _ptr(out)), "cross_sums")
    return out


def cross_sum_at(left, right, r, x, y, d):
    """int S_RT(x, y, d) for one element."""
    L, R = _u8(left), _u8(right)
    H, W = L.shape
    return int(_load().oracle_cross_sum_at(_ptr(L), _ptr(R), W, W, H, r, x, y, d))


def zncc_at(left, right, r, x, y, d):
    """ZNCC z in [-1, 1] at one (x, y, d) by Eq. ZNCC."""
    L, R = _u8(left), _u8(right)
    H, W = L.shape
    return float(_load().oracle_zncc_at(_ptr(L), _ptr(R), W, W, H, r, x, y, d))


def zncc_cost_slice(left, right, r, d):
    """float64 cost 1 - ZNCC, [H][W], for one disparity d."""
    L, R = _u8(left), _u8(right)
    H, W = L.shape
    out = np.empty((H, W), np.float64)
    _check(_load().oracle_zncc_cost_slice(_ptr(L), _ptr(R), W, W, H, r, d, _ptr(out)), "zncc_cost_slice")
    return out


def zncc_cost(left, right, D, r):
    """float64 cost volume 1 - ZNCC, [H][W][D]."""
    L, R = _u8(left), _u8(right)
    H, W = L.shape
    out = np.empty((H, W, D), np.float64)
    _check(_load().oracle_zncc_cost(_ptr(L), _ptr(R), W, W, H, D, r, _ptr(out)), "zncc_cost")
    return out


def dt_weights(guide, sigma_s, sigma_r):
    """float64 (wh, wv) [H][W]: W_L(x,y) and W_U(x,y); zero on the first column / row."""
    G = _u8(guide)
    H, W = G.shape
    wh = np.empty((H, W), np.float64)
    wv = np.empty((H, W), np.float64)
    _check(_load().oracle_dt_weights(_ptr(G), W, W, H, float(sigma_s), float(sigma_r), _ptr(wh), _ptr(wv)),
           "dt_weights")
    return wh, wv


def dt_slice(c_hw, wh, wv, iters):
    """DT of one [H][W] slice (returns a new array)."""
    c = np.array(c_hw, dtype=np.float64, order="C", copy=True)
    H, W = c.shape
    wh = np.ascontiguousarray(wh, np.float64)
    wv = np.ascontiguousarray(wv, np.float64)
    _check(_load().oracle_dt_slice(_ptr(c), W, H, _ptr(wh), _ptr(wv), int(iters)), "dt_slice")
    return c


def dt_aggregate(vol_hwd, wh, wv, iters):
    """DT of a [H][W][D] volume (returns a new array)."""
    v = np.array(vol_hwd, dtype=np.float64, order="C", copy=True)
    H, W, D = v.shape
    wh = np.ascontiguousarray(wh, np.float64)
    wv = np.ascontiguousarray(wv, np.float64)
    _check(_load().oracle_dt_aggregate(_ptr(v), W, H, D, _ptr(wh), _ptr(wv), int(iters)), "dt_aggregate")
    return v


def wta(vol_hwd):
    """int32 [H][W]: smallest d attaining the minimum over d."""
    v = np.ascontiguousarray(vol_hwd, np.float64)
    H, W, D = v.shape
    out = np.empty((H, W), np.int32)
    _check(_load().oracle_wta(_ptr(v), W, H, D, _ptr(out)), "wta")
    return out


def stereo_solve(left, right, D, r, sigma_s, sigma_r, iters, guide_target=False, keep_volume=False):
    """Whole path.  Returns disp [H][W] int32, and the aggregated volume if asked."""
    L, R = _u8(left), _u8(right)
    H, W = L.shape
    disp = np.empty((H, W), np.int32)
    vol = np.empty((H, W, D), np.float64) if keep_volume else None
    _check(_load().oracle_stereo_solve(_ptr(L), _ptr(R), W, W, H, D, r, float(sigma_s), float(sigma_r),
                                       int(iters), int(bool(guide_target)),
                                       _ptr(vol) if vol is not None else None, _ptr(disp)), "stereo_solve")
    return (disp, vol) if keep_volume else disp


IntSolve = namedtuple("IntSolve", "disp volume saturated")


def int_solve(left, right, D, r, sigma_s, sigma_r, iters, T=21.0, code8=False, form="paper", guide_target=False,
              keep_volume=False, npasses=0):
    """The integer-volume path (Sec. IV-C): T-scaled int16 states (or their
    8-bit code), normalized by Eq. DT_new with d_arb = 0, DT, WTA.

    form "paper": the per-pass FastDT of Sec. V-C (a stored state after every
    pass but the last; Int16 normalizes in U2D, Int8 in R2L and codes R2L's
    output).  form "pairs": centred once before the first pass, states stored
    only between pass pairs.  Returns IntSolve(disp [H][W] int32, the last
    pass's output [H][W][D] float64 if asked else None, number of stores that
    saturated).  npasses in 1 .. 4 iters stops after that many passes of the
    sequence L, R, U, D, ... (0: all); the state returned is then the stored
    one if the stop is a store point (the WTA runs on it)."""
    L, R = _u8(left), _u8(right)
    H, W = L.shape
    disp = np.empty((H, W), np.int32)
    vol = np.empty((H, W, D), np.float64) if keep_volume else None
    sat = ctypes.c_int64(0)
    f = {"paper": 0, "pairs": 1}[form]
    _check(_load().oracle_int_solve(_ptr(L), _ptr(R), W, W, H, D, r, float(sigma_s), float(sigma_r), int(iters),
                                    int(bool(guide_target)), float(T), int(bool(code8)), f, int(npasses),
                                    _ptr(vol) if vol is not None else None, _ptr(disp), ctypes.byref(sat)),
           "int_solve")
    return IntSolve(disp, vol, int(sat.value))


def dt_passes(c_hw, wh, wv, first, count):
    """Passes first .. first+count-1 of the sequence L, R, U, D, L, ... on one
    [H][W] slice (returns a new array)."""
    c = np.array(c_hw, dtype=np.float64, order="C", copy=True)
    H, W = c.shape
    wh = np.ascontiguousarray(wh, np.float64)
    wv = np.ascontiguousarray(wv, np.float64)
    _check(_load().oracle_dt_passes(_ptr(c), W, H, _ptr(wh), _ptr(wv), int(first), int(count)), "dt_passes")
    return c


def solve_slices(left, right, r, ds, sigma_s, sigma_r, iters, guide_target=False, threads=1):
    """Aggregated cost slices C_agg(:, :, d) for the disparities in ``ds`` -> [len(ds)][H][W].

    Each slice is the oracle's own cost slice followed by its own DT; the
    slices are independent, so ``threads`` > 1 runs several single-threaded
    oracle calls side by side (ctypes releases the GIL).
    """
    wh, wv = dt_weights(right if guide_target else left, sigma_s, sigma_r)
    ds = list(ds)
    H, W = np.asarray(left).shape
    out = np.empty((len(ds), H, W), np.float64)

    def one(k):
        out[k] = dt_slice(zncc_cost_slice(left, right, r, ds[k]), wh, wv, iters)

    if threads <= 1:
        for k in range(len(ds)):
            one(k)
    else:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(one, range(len(ds))))
    return out


def i8_encode(values):
    """The 8-bit codes (Sec. IV-C) of int16 values, elementwise."""
    lib = _load()
    v = np.asarray(values, np.int16)
    return np.array([lib.oracle_i8_encode(int(x)) for x in v.ravel()], np.uint8).reshape(v.shape)


def i8_decode(codes):
    """The int16 values of 8-bit codes (Sec. IV-C), elementwise."""
    lib = _load()
    c = np.asarray(codes, np.uint8)
    return np.array([lib.oracle_i8_decode(int(x)) for x in c.ravel()], np.int16).reshape(c.shape)


def sgm_aggregate(cost_hwd, p1, p2, scale):
    """Four-path semi-global matching sum [H][W][D] (float64) of scale * cost."""
    c = np.ascontiguousarray(cost_hwd, np.float64)
    H, W, D = c.shape
    out = np.empty_like(c)
    _check(_load().oracle_sgm_aggregate(_ptr(c), W, H, D, float(p1), float(p2), float(scale), _ptr(out)),
           "sgm_aggregate")
    return out
