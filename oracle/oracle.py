"""numpy front end of the plain C oracle (egosgm_oracle.c).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this module; the product library
never does.  Each function here marshals numpy arrays into the C oracle and
back, nothing more: every step of the method's arithmetic lives in the C file.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "egosgm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liborc.so")
_lib = None

CFLAGS = ["-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/liborc.so."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = C.CDLL(_LIB_PATH)
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def census(img: np.ndarray) -> np.ndarray:
    img = np.ascontiguousarray(img, dtype=np.uint8)
    h, w = img.shape
    out = np.zeros((h, w), np.uint64)
    _check(lib().orc_census(_p(img), w, h, _p(out)), "census")
    return out


def cost(cl: np.ndarray, cr: np.ndarray, x: int, y: int, d: int) -> int:
    cl = np.ascontiguousarray(cl, dtype=np.uint64)
    cr = np.ascontiguousarray(cr, dtype=np.uint64)
    return int(lib().orc_cost(_p(cl), _p(cr), cl.shape[1], x, y, d))


def windows(d_pred, p_pred, max_disp, r_fixed=-1, r_min=0, r_max=256, k_sigma=3.0):
    """Returns (lo, hi, off) int16/int16/uint32, off of length n+1."""
    if d_pred is None:
        n = int(np.prod(p_pred)) if isinstance(p_pred, tuple) else int(p_pred)
        lo = np.zeros(n, np.int16)
        hi = np.zeros(n, np.int16)
        off = np.zeros(n + 1, np.uint32)
        _check(lib().orc_windows_full(n, max_disp, _p(lo), _p(hi), _p(off)), "windows_full")
        return lo, hi, off
    d = np.ascontiguousarray(d_pred, dtype=np.float32).ravel()
    p = None if p_pred is None else np.ascontiguousarray(p_pred, dtype=np.float32).ravel()
    n = d.size
    lo = np.zeros(n, np.int16)
    hi = np.zeros(n, np.int16)
    off = np.zeros(n + 1, np.uint32)
    _check(lib().orc_windows(_p(d), _p(p), n, C.c_float(k_sigma), r_fixed, r_min, r_max,
                             max_disp, _p(lo), _p(hi), _p(off)), "windows")
    return lo, hi, off


def cost_volume(cl, cr, lo, hi, off):
    cl = np.ascontiguousarray(cl, dtype=np.uint64)
    cr = np.ascontiguousarray(cr, dtype=np.uint64)
    h, w = cl.shape
    out = np.zeros(int(off[-1]), np.int32)
    _check(lib().orc_cost_volume(_p(cl), _p(cr), w, h, _p(lo), _p(hi), _p(off), _p(out)),
           "cost_volume")
    return out


def path(cost_vol, w, h, lo, hi, off, p1, p2, direction):
    cost_vol = np.ascontiguousarray(cost_vol, dtype=np.int32)
    lo = np.ascontiguousarray(lo, dtype=np.int16)
    hi = np.ascontiguousarray(hi, dtype=np.int16)
    off = np.ascontiguousarray(off, dtype=np.uint32)
    out = np.zeros(int(off[-1]), np.int32)
    _check(lib().orc_path(_p(cost_vol), w, h, _p(lo), _p(hi), _p(off), p1, p2, direction,
                          _p(out)), "path")
    return out


def direction(k):
    dx, dy = C.c_int(), C.c_int()
    _check(lib().orc_direction(k, C.byref(dx), C.byref(dy)), "direction")
    return dx.value, dy.value


def pixel_epilogue(S_row, lo, hi, s_max):
    S_row = np.ascontiguousarray(S_row, dtype=np.int32)
    ds, nl, nr = C.c_int(), C.c_int(), C.c_int()
    sub = C.c_double()
    _check(lib().orc_pixel_epilogue(_p(S_row), lo, hi, s_max, C.byref(ds), C.byref(sub),
                                    C.byref(nl), C.byref(nr)), "pixel_epilogue")
    return ds.value, sub.value, nl.value, nr.value


def sgm(left, right, max_disp, p1=10, p2=120, s_max=80, lr_tol=1, windows=None,
        want_debug=False, n_paths=8):
    """Runs the whole matcher.  windows = (lo, hi, off) or None for full range;
    n_paths 8, or 4 (directions 0-3).

    Returns a dict with disp_wta (int16, -1 invalid), disp_sub (float64),
    var_meas (float64), disp_right (int16), wta_raw (before the LR check) and,
    with want_debug, census_l/census_r, cost, paths (8 x total) and agg."""
    left = np.ascontiguousarray(left, dtype=np.uint8)
    right = np.ascontiguousarray(right, dtype=np.uint8)
    h, w = left.shape
    n = w * h
    if windows is None:
        lo = hi = off = None
        total = n * max_disp
    else:
        lo, hi, off = (np.ascontiguousarray(windows[0], np.int16),
                       np.ascontiguousarray(windows[1], np.int16),
                       np.ascontiguousarray(windows[2], np.uint32))
        total = int(off[-1])
    r = dict(disp_wta=np.zeros((h, w), np.int16), disp_sub=np.zeros((h, w), np.float64),
             var_meas=np.zeros((h, w), np.float64), disp_right=np.zeros((h, w), np.int16),
             wta_raw=np.zeros((h, w), np.int16))
    dbg = {}
    if want_debug:
        dbg = dict(census_l=np.zeros((h, w), np.uint64), census_r=np.zeros((h, w), np.uint64),
                   cost=np.zeros(total, np.int32), paths=np.zeros((n_paths, total), np.int32),
                   agg=np.zeros(total, np.int32))
    rc = lib().orc_sgm(_p(left), _p(right), w, h, max_disp, _p(lo), _p(hi), _p(off),
                       p1, p2, s_max, lr_tol, n_paths,
                       _p(dbg.get("census_l")), _p(dbg.get("census_r")), _p(dbg.get("cost")),
                       _p(dbg.get("paths")), _p(dbg.get("agg")),
                       _p(r["wta_raw"]), _p(r["disp_wta"]), _p(r["disp_sub"]),
                       _p(r["var_meas"]), _p(r["disp_right"]))
    _check(rc, "sgm")
    r.update(dbg)
    return r


def warp_matrix(R, t, f, cx, cy, b):
    R = np.ascontiguousarray(R, dtype=np.float64).ravel()
    t = np.ascontiguousarray(t, dtype=np.float64).ravel()
    H = np.zeros(16, np.float64)
    _check(lib().orc_warp_matrix(_p(R), _p(t), C.c_double(f), C.c_double(cx), C.c_double(cy),
                                 C.c_double(b), _p(H)), "warp_matrix")
    return H.reshape(4, 4)


def warp(d_prev, p_prev, R, t, f, cx, cy, b, q):
    """Returns dict d_pred/p_pred (float64 values), winner (int32 source
    index or -1) and d_key_f32 (the float32 d' the z-buffer compared)."""
    d_prev = np.ascontiguousarray(d_prev, dtype=np.float32)
    p_prev = np.ascontiguousarray(p_prev, dtype=np.float32)
    h, w = d_prev.shape
    R = np.ascontiguousarray(R, dtype=np.float64).ravel()
    t = np.ascontiguousarray(t, dtype=np.float64).ravel()
    out = dict(d_pred=np.zeros((h, w)), p_pred=np.zeros((h, w)),
               winner=np.zeros((h, w), np.int32), d_key_f32=np.zeros((h, w), np.float32))
    _check(lib().orc_warp(_p(d_prev), _p(p_prev), w, h, _p(R), _p(t), C.c_double(f),
                          C.c_double(cx), C.c_double(cy), C.c_double(b), C.c_double(q),
                          _p(out["d_pred"]), _p(out["p_pred"]), _p(out["winner"]),
                          _p(out["d_key_f32"])), "warp")
    return out


def kalman(d_pred, p_pred, z, r, keep_unmeasured=0):
    arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in (d_pred, p_pred, z, r)]
    shape = arrs[0].shape
    n = arrs[0].size
    d = np.zeros(shape)
    p = np.zeros(shape)
    _check(lib().orc_kalman(*[_p(a) for a in arrs], n, keep_unmeasured, _p(d), _p(p)), "kalman")
    return d, p


def right_map(S, w, h, max_disp, lo, hi, off):
    S = np.ascontiguousarray(S, dtype=np.int32)
    out = np.zeros((h, w), np.int16)
    _check(lib().orc_right_map(_p(S), w, h, max_disp, _p(np.ascontiguousarray(lo, np.int16)),
                               _p(np.ascontiguousarray(hi, np.int16)),
                               _p(np.ascontiguousarray(off, np.uint32)), _p(out)), "right_map")
    return out


def lr_check(disp_right, disp_wta, lr_tol=1, disp_sub=None, var_meas=None):
    """Returns copies of (disp_wta, disp_sub, var_meas) after the check."""
    dr = np.ascontiguousarray(disp_right, dtype=np.int16)
    h, w = dr.shape
    wta = np.array(disp_wta, dtype=np.int16, copy=True)
    sub = None if disp_sub is None else np.array(disp_sub, dtype=np.float64, copy=True)
    var = None if var_meas is None else np.array(var_meas, dtype=np.float64, copy=True)
    _check(lib().orc_lr_check(_p(dr), w, h, lr_tol, _p(wta), _p(sub), _p(var)), "lr_check")
    return wta, sub, var


def refine(d_pred, p_pred, edge_tol=-1.0, fill_tol=1.0):
    """Edge rejection + zoom hole filling; returns float32 (d, p)."""
    d = np.ascontiguousarray(d_pred, dtype=np.float32)
    p = np.ascontiguousarray(p_pred, dtype=np.float32)
    h, w = d.shape
    od = np.zeros_like(d)
    op = np.zeros_like(p)
    _check(lib().orc_refine(_p(d), _p(p), w, h, C.c_float(edge_tol), C.c_float(fill_tol),
                            _p(od), _p(op)), "refine")
    return od, op


def sad_check(left, right, disp_wta, radius, sad_max, disp_sub=None, var_meas=None):
    """Returns (disp_wta, disp_sub, var_meas) after the SAD check (copies)."""
    left = np.ascontiguousarray(left, dtype=np.uint8)
    right = np.ascontiguousarray(right, dtype=np.uint8)
    h, w = left.shape
    wta = np.ascontiguousarray(disp_wta, dtype=np.int16).copy()
    sub = None if disp_sub is None else np.ascontiguousarray(disp_sub, dtype=np.float64).copy()
    var = None if var_meas is None else np.ascontiguousarray(var_meas, dtype=np.float64).copy()
    _check(lib().orc_sad_check(_p(left), _p(right), w, h, radius, sad_max, _p(wta), _p(sub), _p(var)),
           "sad_check")
    return wta, sub, var


def lr_check_prediction(d_pred, p_pred, d_right, tol=1.0):
    """Returns float32 (d, p) after the left-right check of a prediction."""
    d = np.ascontiguousarray(d_pred, dtype=np.float32).copy()
    pp = np.ascontiguousarray(p_pred, dtype=np.float32).copy()
    dr = np.ascontiguousarray(d_right, dtype=np.float32)
    h, w = d.shape
    _check(lib().orc_lr_check_prediction(_p(d), _p(pp), _p(dr), w, h, C.c_float(tol)),
           "lr_check_prediction")
    return d, pp


def right_motion(R, t, b):
    R = np.ascontiguousarray(R, dtype=np.float64).ravel()
    t = np.ascontiguousarray(t, dtype=np.float64).ravel()
    out = np.zeros(3)
    _check(lib().orc_right_motion(_p(R), _p(t), C.c_double(b), _p(out)), "right_motion")
    return out
