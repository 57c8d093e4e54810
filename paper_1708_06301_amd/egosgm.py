"""Python binding of libegosgm (include/egosgm.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of libegosgm.so.  Tensors are torch tensors on the GPU (torch provides device
memory and the stream); the functions pass their data pointers and the
current HIP stream to the C ABI and raise on a non-zero status.  There is no
fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libegosgm.so")
_lib = None

_vp, _i, _f, _d, _sz = C.c_void_p, C.c_int, C.c_float, C.c_double, C.c_size_t

_SIGS = {
    "egosgm_abi_version": ([], _i),
    "egosgm_status_string": ([_i], C.c_char_p),
    "egosgm_census": ([_vp, _i, _i, _i, _vp, _vp], _i),
    "egosgm_sgm_workspace_bytes": ([_i, _i, _i], _sz),
    "sgm_full": ([_vp, _vp, _i, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp], _i),
    "egosgm_windows_workspace_bytes": ([_i, _i], _sz),
    "sgm_windows_from_prediction": ([_vp, _vp, _i, _i, _f, _i, _i, _i, _i, _vp, _vp, _vp, _vp,
                                     _sz, _vp], _i),
    "sgm_windows_from_prediction_noalloc": ([_vp, _vp, _i, _i, _f, _i, _i, _i, _i, _vp, _vp, _vp,
                                             _vp], _i),
    "sgm_reduced": ([_vp, _vp, _i, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                     _sz, _vp], _i),
    "egosgm_warp_matrix": ([_vp, _vp, _d, _d, _d, _d, _vp], _i),
    "warp_disparity": ([_vp, _vp, _i, _i, _vp, _vp, _d, _d, _d, _d, _f, _vp, _vp, _vp, _vp], _i),
    "sgm_census": ([_vp, _vp, _i, _i, _i, _i, _vp, _sz, _vp], _i),
    "predict_disparity": ([_vp, _vp, _i, _i, _vp, _vp, _d, _d, _d, _d, _f, _f, _f, _vp, _vp, _vp, _vp], _i),
    "kalman_update": ([_vp, _vp, _vp, _vp, _i, _i, _vp, _vp, _vp], _i),
    "egosgm_refine_workspace_bytes": ([_i, _i], _sz),
    "refine_prediction": ([_vp, _vp, _i, _i, _f, _f, _vp, _vp, _vp, _sz, _vp], _i),
    "egosgm_plan_workspace_bytes": ([_vp, _i], _sz),
    "sgm_plan_create": ([_vp, _i, _vp, _vp, _sz, _vp], _i),
    "sgm_plan_run": ([_vp, _vp], _i),
    "sgm_plan_run_eager": ([_vp, _vp], _i),
    "sgm_plan_update": ([_vp, _vp, _i, _vp], _i),
    "sad_check": ([_vp, _vp, _i, _i, _i, _i, _i, _vp, _vp, _vp, _vp], _i),
    "lr_check_prediction": ([_vp, _vp, _vp, _i, _i, C.c_float, _vp], _i),
    "disparity_to_float": ([_vp, _vp, _i, _vp], _i),
    "egosgm_right_motion": ([_vp, _vp, C.c_double, _vp], _i),
    "sgm_plan_destroy": ([_vp], _i),
    "egosgm_set_tuning": ([_vp], _i),
    "egosgm_get_tuning": ([_vp], _i),
    "egosgm_timing_enable": ([_i], _i),
    "egosgm_timing_read": ([_vp, _vp, _i], _i),
    "egosgm_vo_workspace_bytes": ([_i, _i, _vp], _sz),
    "estimate_motion": ([_vp, _vp, _i, _i, _i, _vp, _d, _d, _d, _d, _vp, _vp, _vp, _sz, _vp], _i),
    "vo_normal_equations": ([_vp, _vp, _i, _i, _i, _vp, _d, _d, _d, _d, _vp, _i, _vp, _vp, _vp, _sz, _vp],
                            _i),
}

STAGES = ("census", "windows", "cost", "paths", "select", "warp", "kalman", "refine",
          "batch_census", "batch_cost", "batch_paths", "batch_select", "vo")


ABI_VERSION = 5   # EGOSGM_ABI_VERSION of include/egosgm.h


def lib():
    """Loads libegosgm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1708_06301_amd.build`")
        h = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(h, name)
            fn.argtypes = args
            fn.restype = res
        if h.egosgm_abi_version() != ABI_VERSION:   # the structs below follow this version
            raise RuntimeError(f"{LIB_PATH} has ABI version {h.egosgm_abi_version()}, "
                               f"this binding expects {ABI_VERSION}: rebuild it")
        _lib = h
    return _lib


class EgoSgmError(RuntimeError):
    pass


def _check(rc: int, what: str):
    if rc != 0:
        msg = lib().egosgm_status_string(rc).decode()
        raise EgoSgmError(f"{what}: {msg} ({rc})")


class SgmParams(C.Structure):
    _fields_ = [("max_disp", C.c_int32), ("p1", C.c_int32), ("p2", C.c_int32),
                ("s_max", C.c_int32), ("lr_tol", C.c_int32), ("n_paths", C.c_int32),
                ("census_ready", C.c_int32)]


class SgmDebug(C.Structure):
    _fields_ = [("census_left", _vp), ("census_right", _vp), ("cost", _vp), ("paths", _vp),
                ("agg", _vp), ("wta_raw", _vp)]


class Tuning(C.Structure):
    _fields_ = [("full_group", C.c_int32), ("ragged_group", C.c_int32),
                ("ragged_schedule", C.c_int32), ("batch_group", C.c_int32),
                ("wide_offsets", C.c_int32), ("batch_persistent", C.c_int32)]


DEFAULT_TUNING = dict(full_group=64, ragged_group=32, ragged_schedule=1, batch_group=16, wide_offsets=0,
                      batch_persistent=0)


def set_tuning(full_group: int | None = None, ragged_group: int | None = None,
               ragged_schedule: int | None = None, batch_group: int | None = None,
               wide_offsets: int | None = None, batch_persistent: int | None = None):
    """Sets the launch shapes; every argument left None keeps its current
    value (the library's own default until something else was set)."""
    cur = get_tuning()
    new = dict(full_group=full_group, ragged_group=ragged_group, ragged_schedule=ragged_schedule,
               batch_group=batch_group, wide_offsets=wide_offsets, batch_persistent=batch_persistent)
    t = Tuning(**{k: cur[k] if v is None else int(v) for k, v in new.items()})
    _check(lib().egosgm_set_tuning(C.byref(t)), "egosgm_set_tuning")


def get_tuning() -> dict:
    t = Tuning()
    _check(lib().egosgm_get_tuning(C.byref(t)), "egosgm_get_tuning")
    return dict(full_group=t.full_group, ragged_group=t.ragged_group,
                ragged_schedule=t.ragged_schedule, batch_group=t.batch_group,
                wide_offsets=t.wide_offsets, batch_persistent=t.batch_persistent)


@dataclass
class MatchParams:
    max_disp: int = 128
    p1: int = 10
    p2: int = 120
    s_max: int = 80
    lr_tol: int = 1
    n_paths: int = 8       # or 4: along and against the rows and the columns only
    census_ready: int = 0  # 1: sgm_census already filled the workspace's census codes

    def c(self) -> SgmParams:
        return SgmParams(self.max_disp, self.p1, self.p2, self.s_max, self.lr_tol, self.n_paths,
                         self.census_ready)


def _stream():
    return _vp(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else _vp(t.data_ptr())


def _need(t: torch.Tensor, dtype, numel=None, name="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise EgoSgmError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise EgoSgmError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise EgoSgmError(f"{name} must be contiguous")
    if numel is not None and t.numel() < numel:
        raise EgoSgmError(f"{name} holds {t.numel()} elements, needs {numel}")
    return t


def abi_version() -> int:
    return lib().egosgm_abi_version()


# ------------------------------------------------------------------ census
def census(img: torch.Tensor) -> torch.Tensor:
    """9x7 census codes (int64 tensor holding the uint64 bit patterns)."""
    _need(img, torch.uint8, name="img")
    h, w = img.shape
    out = torch.empty((h, w), dtype=torch.int64, device=img.device)
    _check(lib().egosgm_census(_ptr(img), w, h, w, _ptr(out), _stream()), "egosgm_census")
    return out


# ------------------------------------------------------------------ workspaces
class Workspace:
    """Device scratch for the matcher, grown on demand and reused."""

    def __init__(self, device="cuda"):
        self.device = torch.device(device)
        self.sgm = None
        self.win = None

    def sgm_bytes(self, w, h, max_disp):
        n = lib().egosgm_sgm_workspace_bytes(w, h, max_disp)
        if n == 0:
            raise EgoSgmError("workspace size: bad shape")
        if self.sgm is None or self.sgm.numel() < n:
            self.sgm = torch.empty(n, dtype=torch.uint8, device=self.device)
        return self.sgm, n

    def refine_bytes(self, w, h):
        n = lib().egosgm_refine_workspace_bytes(w, h)
        if getattr(self, "ref", None) is None or self.ref.numel() < n:
            self.ref = torch.empty(n, dtype=torch.uint8, device=self.device)
        return self.ref, n

    def windows_bytes(self, w, h):
        n = lib().egosgm_windows_workspace_bytes(w, h)
        if self.win is None or self.win.numel() < n:
            self.win = torch.empty(n, dtype=torch.uint8, device=self.device)
        return self.win, n


_default_ws = {}


def _ws(device) -> Workspace:
    key = str(device)
    if key not in _default_ws:
        _default_ws[key] = Workspace(device)
    return _default_ws[key]


def _outputs(h, w, device):
    return dict(disp_wta=torch.empty((h, w), dtype=torch.int16, device=device),
                disp_sub=torch.empty((h, w), dtype=torch.float32, device=device),
                var_meas=torch.empty((h, w), dtype=torch.float32, device=device),
                disp_right=torch.empty((h, w), dtype=torch.int16, device=device))


def _debug(h, w, max_disp, total, device):
    n = h * w
    d = dict(census_left=torch.empty((h, w), dtype=torch.int64, device=device),
             census_right=torch.empty((h, w), dtype=torch.int64, device=device),
             cost=torch.empty(total, dtype=torch.uint8, device=device),
             paths=torch.empty((8, n * max_disp), dtype=torch.uint8, device=device),
             agg=torch.empty(total, dtype=torch.int16, device=device),
             wta_raw=torch.empty((h, w), dtype=torch.int16, device=device))
    s = SgmDebug(*[_ptr(d[k]) for k in ("census_left", "census_right", "cost", "paths", "agg",
                                           "wta_raw")])
    return d, s


# ------------------------------------------------------------------ SGM
def sgm_full(left: torch.Tensor, right: torch.Tensor, params: MatchParams | None = None,
             debug: bool = False, out: dict | None = None, workspace: Workspace | None = None):
    """Full-range SGM; returns dict disp_wta, disp_sub, var_meas, disp_right
    (+ debug tensors: census_left/right, cost, paths, agg (int16 holding
    uint16), wta_raw)."""
    params = params or MatchParams()
    _need(left, torch.uint8, name="left")
    _need(right, torch.uint8, name="right")
    h, w = left.shape
    if right.shape != left.shape:
        raise EgoSgmError("left/right shapes differ")
    o = out if out is not None else _outputs(h, w, left.device)
    ws, nbytes = (workspace or _ws(left.device)).sgm_bytes(w, h, params.max_disp)
    dbg, dbg_c = (None, None)
    if debug:
        dbg, dbg_c = _debug(h, w, params.max_disp, h * w * params.max_disp, left.device)
    prm = params.c()
    rc = lib().sgm_full(_ptr(left), _ptr(right), w, h, w, C.byref(prm), _ptr(o["disp_wta"]),
                        _ptr(o["disp_sub"]), _ptr(o["var_meas"]), _ptr(o.get("disp_right")),
                        C.byref(dbg_c) if debug else None, _ptr(ws), nbytes, _stream())
    _check(rc, "sgm_full")
    if debug:
        o = dict(o)
        o.update(dbg)
    return o


def sgm_census(left: torch.Tensor, right: torch.Tensor, max_disp: int,
               workspace: Workspace | None = None):
    """The matcher's census pass alone, into the workspace; a following
    sgm_full / sgm_reduced with census_ready=1 on that workspace skips it."""
    _need(left, torch.uint8, name="left")
    _need(right, torch.uint8, name="right")
    h, w = left.shape
    if right.shape != left.shape:
        raise EgoSgmError("left/right shapes differ")
    ws, nbytes = (workspace or _ws(left.device)).sgm_bytes(w, h, max_disp)
    _check(lib().sgm_census(_ptr(left), _ptr(right), w, h, w, max_disp, _ptr(ws), nbytes, _stream()),
           "sgm_census")


def windows_from_prediction(d_pred: torch.Tensor, p_pred: torch.Tensor | None, max_disp: int,
                            r_fixed: int = -1, r_min: int = 0, r_max: int = 256,
                            k_sigma: float = 3.0, out=None, workspace: Workspace | None = None):
    """Per-pixel windows (lo, hi, offsets) from a predicted map."""
    _need(d_pred, torch.float32, name="d_pred")
    if p_pred is not None:
        _need(p_pred, torch.float32, d_pred.numel(), name="p_pred")
    h, w = d_pred.shape
    if out is None:
        dev = d_pred.device
        out = (torch.empty((h, w), dtype=torch.int16, device=dev),
               torch.empty((h, w), dtype=torch.int16, device=dev),
               torch.empty(h * w + 1, dtype=torch.int32, device=dev))
    lo, hi, off = out
    ws, nbytes = (workspace or _ws(d_pred.device)).windows_bytes(w, h)
    rc = lib().sgm_windows_from_prediction(_ptr(d_pred), _ptr(p_pred), w, h, k_sigma, r_fixed,
                                           r_min, r_max, max_disp, _ptr(lo), _ptr(hi),
                                           _ptr(off), _ptr(ws), nbytes, _stream())
    _check(rc, "sgm_windows_from_prediction")
    return lo, hi, off


def windows_from_prediction_noalloc(d_pred: torch.Tensor, p_pred: torch.Tensor | None, max_disp: int,
                                    r_fixed: int = -1, r_min: int = 0, r_max: int = 256,
                                    k_sigma: float = 3.0, out=None):
    """windows_from_prediction through the entry point that allocates
    nothing (its scratch is a fixed device array of the library); `out`
    (lo, hi, offsets) must be given where the caller cannot allocate."""
    _need(d_pred, torch.float32, name="d_pred")
    if p_pred is not None:
        _need(p_pred, torch.float32, d_pred.numel(), name="p_pred")
    h, w = d_pred.shape
    if out is None:
        dev = d_pred.device
        out = (torch.empty((h, w), dtype=torch.int16, device=dev),
               torch.empty((h, w), dtype=torch.int16, device=dev),
               torch.empty(h * w + 1, dtype=torch.int32, device=dev))
    lo, hi, off = out
    rc = lib().sgm_windows_from_prediction_noalloc(_ptr(d_pred), _ptr(p_pred), w, h, k_sigma, r_fixed,
                                                   r_min, r_max, max_disp, _ptr(lo), _ptr(hi),
                                                   _ptr(off), _stream())
    _check(rc, "sgm_windows_from_prediction_noalloc")
    return lo, hi, off


def sgm_reduced(left: torch.Tensor, right: torch.Tensor, lo: torch.Tensor, hi: torch.Tensor,
                offsets: torch.Tensor, params: MatchParams | None = None, debug: bool = False,
                out: dict | None = None, workspace: Workspace | None = None, total: int | None = None):
    """SGM over per-pixel windows; debug volumes are sized from `total` (read
    back from offsets when not given)."""
    params = params or MatchParams()
    _need(left, torch.uint8, name="left")
    _need(right, torch.uint8, name="right")
    h, w = left.shape
    _need(lo, torch.int16, h * w, "lo")
    _need(hi, torch.int16, h * w, "hi")
    _need(offsets, torch.int32, h * w + 1, "offsets")
    o = out if out is not None else _outputs(h, w, left.device)
    ws, nbytes = (workspace or _ws(left.device)).sgm_bytes(w, h, params.max_disp)
    dbg, dbg_c = (None, None)
    if debug:
        if total is None:
            total = int(offsets[h * w].item())
        dbg, dbg_c = _debug(h, w, params.max_disp, total, left.device)
    prm = params.c()
    rc = lib().sgm_reduced(_ptr(left), _ptr(right), w, h, w, _ptr(lo), _ptr(hi), _ptr(offsets),
                           C.byref(prm), _ptr(o["disp_wta"]), _ptr(o["disp_sub"]),
                           _ptr(o["var_meas"]), _ptr(o.get("disp_right")),
                           C.byref(dbg_c) if debug else None, _ptr(ws), nbytes, _stream())
    _check(rc, "sgm_reduced")
    if debug:
        o = dict(o)
        o.update(dbg)
    return o


# ------------------------------------------------------------------ warp / update
def warp_matrix(R, t, f, cx, cy, baseline) -> np.ndarray:
    """Host helper: the float32 H the warp uses."""
    R = np.ascontiguousarray(R, dtype=np.float64).ravel()
    t = np.ascontiguousarray(t, dtype=np.float64).ravel()
    H = np.zeros(16, np.float32)
    _check(lib().egosgm_warp_matrix(R.ctypes.data_as(_vp), t.ctypes.data_as(_vp), f, cx, cy,
                                    baseline, H.ctypes.data_as(_vp)), "egosgm_warp_matrix")
    return H.reshape(4, 4)


def warp_disparity(d_prev: torch.Tensor, p_prev: torch.Tensor, R, t, f, cx, cy, baseline, q,
                   out=None, zbuf: torch.Tensor | None = None):
    _need(d_prev, torch.float32, name="d_prev")
    h, w = d_prev.shape
    _need(p_prev, torch.float32, h * w, "p_prev")
    dev = d_prev.device
    if out is None:
        out = (torch.empty((h, w), dtype=torch.float32, device=dev),
               torch.empty((h, w), dtype=torch.float32, device=dev))
    if zbuf is None:
        zbuf = torch.empty(h * w, dtype=torch.int64, device=dev)
    R = np.ascontiguousarray(R, dtype=np.float64).ravel()
    t = np.ascontiguousarray(t, dtype=np.float64).ravel()
    rc = lib().warp_disparity(_ptr(d_prev), _ptr(p_prev), w, h, R.ctypes.data_as(_vp),
                              t.ctypes.data_as(_vp), f, cx, cy, baseline, q, _ptr(out[0]),
                              _ptr(out[1]), _ptr(zbuf), _stream())
    _check(rc, "warp_disparity")
    return out


def predict_disparity(d_prev: torch.Tensor, p_prev: torch.Tensor, R, t, f, cx, cy, baseline, q,
                      edge_tol=2.0, fill_tol=1.0, out=None, zbuf: torch.Tensor | None = None):
    """warp_disparity + refine_prediction in one call (bit-identical)."""
    _need(d_prev, torch.float32, name="d_prev")
    h, w = d_prev.shape
    _need(p_prev, torch.float32, h * w, "p_prev")
    dev = d_prev.device
    if out is None:
        out = (torch.empty((h, w), dtype=torch.float32, device=dev),
               torch.empty((h, w), dtype=torch.float32, device=dev))
    if zbuf is None:
        zbuf = torch.empty(h * w, dtype=torch.int64, device=dev)
    R = np.ascontiguousarray(R, dtype=np.float64).ravel()
    t = np.ascontiguousarray(t, dtype=np.float64).ravel()
    rc = lib().predict_disparity(_ptr(d_prev), _ptr(p_prev), w, h, R.ctypes.data_as(_vp),
                                 t.ctypes.data_as(_vp), f, cx, cy, baseline, q, edge_tol, fill_tol,
                                 _ptr(out[0]), _ptr(out[1]), _ptr(zbuf), _stream())
    _check(rc, "predict_disparity")
    return out


def refine_prediction(d_in, p_in, edge_tol=2.0, fill_tol=1.0, out=None,
                      workspace: Workspace | None = None):
    """Edge rejection + one-pixel hole filling of a predicted map."""
    _need(d_in, torch.float32, name="d_in")
    h, w = d_in.shape
    _need(p_in, torch.float32, h * w, "p_in")
    if out is None:
        out = (torch.empty_like(d_in), torch.empty_like(d_in))
    ws, nbytes = (workspace or _ws(d_in.device)).refine_bytes(w, h)
    rc = lib().refine_prediction(_ptr(d_in), _ptr(p_in), w, h, edge_tol, fill_tol, _ptr(out[0]),
                                 _ptr(out[1]), _ptr(ws), nbytes, _stream())
    _check(rc, "refine_prediction")
    return out


def sad_check(left, right, out, radius: int = 2, sad_max: int = 600):
    """SAD check in place on a matcher's outputs dict (disp_wta, disp_sub,
    var_meas), Sec. 2.4.1."""
    _need(left, torch.uint8, name="left")
    _need(right, torch.uint8, name="right")
    h, w = left.shape
    for k, dt in (("disp_wta", torch.int16), ("disp_sub", torch.float32), ("var_meas", torch.float32)):
        _need(out[k], dt, h * w, k)
    _check(lib().sad_check(_ptr(left), _ptr(right), w, h, w, radius, sad_max, _ptr(out["disp_wta"]),
                           _ptr(out["disp_sub"]), _ptr(out["var_meas"]), _stream()), "sad_check")
    return out


def lr_check_prediction(d_pred, p_pred, d_right, tol: float = 1.0):
    """Left-right check of a prediction in place (Sec. 2.4.1, Fig. 4)."""
    h, w = d_pred.shape
    for t, name in ((d_pred, "d_pred"), (p_pred, "p_pred"), (d_right, "d_right")):
        _need(t, torch.float32, h * w, name)
    _check(lib().lr_check_prediction(_ptr(d_pred), _ptr(p_pred), _ptr(d_right), w, h, float(tol),
                                     _stream()), "lr_check_prediction")
    return d_pred, p_pred


def disparity_to_float(d, out=None):
    _need(d, torch.int16, name="disparity")
    out = out if out is not None else torch.empty(d.shape, dtype=torch.float32, device=d.device)
    _need(out, torch.float32, d.numel(), "out")
    _check(lib().disparity_to_float(_ptr(d), _ptr(out), d.numel(), _stream()), "disparity_to_float")
    return out


def right_motion(R, t, baseline: float):
    """Motion (R, t_R) of the right camera of a rectified rig from the left
    camera's (egosgm_right_motion)."""
    R = np.ascontiguousarray(R, np.float64).reshape(3, 3)
    t = np.ascontiguousarray(t, np.float64).reshape(3)
    tr = np.zeros(3)
    _check(lib().egosgm_right_motion(R.ctypes.data_as(_vp), t.ctypes.data_as(_vp), float(baseline),
                                     tr.ctypes.data_as(_vp)), "egosgm_right_motion")
    return R, tr


def kalman_update(d_pred, p_pred, d_meas, r_meas, keep_unmeasured=0, out=None):
    n = d_pred.numel()
    for name, t in (("d_pred", d_pred), ("p_pred", p_pred), ("d_meas", d_meas), ("r_meas", r_meas)):
        _need(t, torch.float32, n, name)
    if out is None:
        out = (torch.empty_like(d_pred), torch.empty_like(d_pred))
    rc = lib().kalman_update(_ptr(d_pred), _ptr(p_pred), _ptr(d_meas), _ptr(r_meas), n,
                             int(keep_unmeasured), _ptr(out[0]), _ptr(out[1]), _stream())
    _check(rc, "kalman_update")
    return out


# ------------------------------------------------------------------ ego-motion
VO_MAX_LEVELS = 6


class VOParams(C.Structure):
    """egosgm_vo_params: pyramid levels, Gauss-Newton iterations per level
    (finest first), Huber threshold, smallest disparity used."""
    _fields_ = [("levels", C.c_int), ("iters", C.c_int * VO_MAX_LEVELS), ("huber", C.c_float),
                ("min_disp", C.c_float)]


def vo_params(levels=5, iters=(2, 4, 8, 10, 20, 30), huber=8.0, min_disp=1.0) -> VOParams:
    it = list(iters)[:VO_MAX_LEVELS] + [0] * (VO_MAX_LEVELS - len(iters))
    return VOParams(int(levels), (C.c_int * VO_MAX_LEVELS)(*it), float(huber), float(min_disp))


def vo_levels_for(w, h, max_levels=6, min_w=64):
    """Pyramid levels so that the coarsest level stays at least min_w x 16."""
    n = 1
    while n < max_levels and (w >> n) >= min_w and (h >> n) >= 16:
        n += 1
    return n


def vo_workspace(w, h, prm: VOParams, device="cuda"):
    n = lib().egosgm_vo_workspace_bytes(w, h, C.byref(prm))
    if n == 0:
        raise EgoSgmError("egosgm_vo_workspace_bytes: invalid size or parameters")
    return torch.empty(n, dtype=torch.uint8, device=device)


def _vo_args(prev_left, cur_left, prev_disp, prm):
    h, w = cur_left.shape
    _need(prev_left, torch.uint8, name="prev_left")
    _need(cur_left, torch.uint8, name="cur_left")
    if prev_left.shape != cur_left.shape:
        raise EgoSgmError("prev_left and cur_left differ in shape")
    _need(prev_disp, torch.float32, h * w, "prev_disp")
    return w, h


def estimate_motion(prev_left, cur_left, prev_disp, calib, prm: VOParams, pose=None, R0=None, t0=None,
                    workspace=None):
    """Ego-motion (R, t), M_k = R M_{k-1} + t, from the previous left image
    and disparity map and the current left image (estimate_motion).
    calib: (f, cx, cy, baseline).  pose: optional device float64 tensor of 12
    (R row-major, t) holding the initial guess and receiving the estimate;
    else one is made from R0, t0 (identity, zero by default).  Returns the
    pose tensor; pose_to_host() reads it (a synchronisation)."""
    w, h = _vo_args(prev_left, cur_left, prev_disp, prm)
    if pose is None:
        R0 = np.eye(3) if R0 is None else np.asarray(R0, np.float64)
        t0 = np.zeros(3) if t0 is None else np.asarray(t0, np.float64)
        pose = torch.tensor(np.concatenate([R0.ravel(), t0.ravel()]), dtype=torch.float64,
                            device=cur_left.device)
    _need(pose, torch.float64, 12, "pose")
    ws = workspace if workspace is not None else vo_workspace(w, h, prm, cur_left.device)
    f, cx, cy, b = calib
    _check(lib().estimate_motion(_ptr(prev_left), _ptr(cur_left), w, h, w, _ptr(prev_disp), float(f), float(cx),
                                 float(cy), float(b), C.byref(prm), _ptr(pose), _ptr(ws), ws.numel(), _stream()),
           "estimate_motion")
    return pose


def pose_to_host(pose):
    v = pose.cpu().numpy().astype(np.float64)
    return v[:9].reshape(3, 3), v[9:12].copy()


def vo_normal_equations(prev_left, cur_left, prev_disp, calib, prm: VOParams, level, R, t, workspace=None):
    """(H 6x6, g 6, cost, count) of one pyramid level at the pose (R, t)."""
    w, h = _vo_args(prev_left, cur_left, prev_disp, prm)
    pose = torch.tensor(np.concatenate([np.asarray(R, np.float64).ravel(), np.asarray(t, np.float64).ravel()]),
                        dtype=torch.float64, device=cur_left.device)
    out = torch.zeros(44, dtype=torch.float64, device=cur_left.device)
    ws = workspace if workspace is not None else vo_workspace(w, h, prm, cur_left.device)
    f, cx, cy, b = calib
    _check(lib().vo_normal_equations(_ptr(prev_left), _ptr(cur_left), w, h, w, _ptr(prev_disp), float(f), float(cx),
                                     float(cy), float(b), C.byref(prm), int(level), _ptr(pose), _ptr(out), _ptr(ws),
                                     ws.numel(), _stream()), "vo_normal_equations")
    o = out.cpu().numpy()
    return o[:36].reshape(6, 6), o[36:42].copy(), float(o[42]), int(round(o[43]))


# ------------------------------------------------------------------ timing
def timing_enable(on: bool = True):
    _check(lib().egosgm_timing_enable(1 if on else 0), "egosgm_timing_enable")


def timing_read() -> dict:
    """{stage: (total_ms, launches)} for the stages recorded since the last read."""
    ms = (C.c_double * len(STAGES))()
    cnt = (C.c_int * len(STAGES))()
    _check(lib().egosgm_timing_read(ms, cnt, len(STAGES)), "egosgm_timing_read")
    return {s: (ms[i], cnt[i]) for i, s in enumerate(STAGES)}


# ------------------------------------------------------------------ batches
class PairDesc(C.Structure):
    _fields_ = [("left", _vp), ("right", _vp), ("w", C.c_int32), ("h", C.c_int32),
                ("pitch", C.c_int32), ("max_disp", C.c_int32), ("lo", _vp), ("hi", _vp),
                ("offsets", _vp), ("disp_wta", _vp), ("disp_sub", _vp), ("var_meas", _vp),
                ("disp_right", _vp)]


class PairUpdate(C.Structure):
    _fields_ = [("index", C.c_int32), ("active", C.c_int32), ("left", C.c_void_p),
                ("right", C.c_void_p), ("lo", C.c_void_p), ("hi", C.c_void_p),
                ("offsets", C.c_void_p)]


KEEP = object()   # Plan.update: leave this part of the pair as it is


class Plan:
    """Batched matching of many pairs in one captured graph.

    pairs: list of dicts with left, right (uint8 GPU tensors), max_disp and
    optional windows=(lo, hi, offsets) (else full range).  Outputs are
    allocated per pair (plan.outputs[i]) unless given as out=dict.  Every
    tensor is referenced by the plan so its address stays fixed; windows may
    be rewritten in place between runs."""

    def __init__(self, pairs, params: MatchParams | None = None, device=None):
        params = params or MatchParams()
        self._keep = []
        self.outputs = []
        descs = (PairDesc * len(pairs))()
        for i, q in enumerate(pairs):
            L, R = q["left"], q["right"]
            _need(L, torch.uint8, name="left")
            _need(R, torch.uint8, name="right")
            h, w = L.shape
            D = int(q.get("max_disp", params.max_disp))
            win = q.get("windows")
            o = q.get("out") or _outputs(h, w, L.device)
            lo = hi = off = None
            if win is not None:
                lo, hi, off = win
                _need(lo, torch.int16, h * w, "lo")
                _need(hi, torch.int16, h * w, "hi")
                _need(off, torch.int32, h * w + 1, "offsets")
            descs[i] = PairDesc(_ptr(L), _ptr(R), w, h, w, D, _ptr(lo), _ptr(hi), _ptr(off),
                                _ptr(o["disp_wta"]), _ptr(o["disp_sub"]), _ptr(o["var_meas"]),
                                _ptr(o.get("disp_right")))
            self._keep += [L, R, lo, hi, off]
            self.outputs.append(o)
        self._cur = [dict(left=q["left"], right=q["right"], windows=q.get("windows"), active=True)
                     for q in pairs]
        self.n = len(pairs)
        nbytes = lib().egosgm_plan_workspace_bytes(descs, self.n)
        if nbytes == 0:
            raise EgoSgmError("plan workspace: invalid pair descriptors")
        dev = device or pairs[0]["left"].device
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        prm = params.c()
        self._plan = _vp()
        torch.cuda.synchronize(dev)
        _check(lib().sgm_plan_create(descs, self.n, C.byref(prm), _ptr(self.workspace), nbytes,
                                     C.byref(self._plan)), "sgm_plan_create")
        self._descs = descs

    def run(self, eager: bool = False):
        if eager:
            _check(lib().sgm_plan_run_eager(self._plan, _stream()), "sgm_plan_run_eager")
        else:
            _check(lib().sgm_plan_run(self._plan, _stream()), "sgm_plan_run")

    def update(self, changes):
        """Enqueues per-pair changes on the current stream for the runs that
        follow: dicts with index and any of active (bool), left, right (same
        shape as at creation) and windows ((lo, hi, offsets), or None for the
        full range).  Omitted parts stay as they are."""
        ups = (PairUpdate * max(len(changes), 1))()
        staged = []
        for j, c in enumerate(changes):
            i = int(c["index"])
            if not 0 <= i < self.n:
                raise EgoSgmError(f"plan update: pair index {i} out of range")
            cur = dict(self._cur[i])
            h, w = self._cur[i]["left"].shape
            for k in ("left", "right"):
                t = c.get(k, KEEP)
                if t is not KEEP:
                    _need(t, torch.uint8, name=k)
                    if tuple(t.shape) != (h, w):
                        raise EgoSgmError(f"plan update: {k} must be {h}x{w}")
                    cur[k] = t
            win = c.get("windows", KEEP)
            if win is not KEEP:
                if win is not None:
                    lo, hi, off = win
                    _need(lo, torch.int16, h * w, "lo")
                    _need(hi, torch.int16, h * w, "hi")
                    _need(off, torch.int32, h * w + 1, "offsets")
                cur["windows"] = win
            if "active" in c:
                cur["active"] = bool(c["active"])
            lo, hi, off = cur["windows"] if cur["windows"] is not None else (None, None, None)
            ups[j] = PairUpdate(i, int(cur["active"]), _ptr(cur["left"]), _ptr(cur["right"]),
                                _ptr(lo), _ptr(hi), _ptr(off))
            staged.append((i, cur))
        _check(lib().sgm_plan_update(self._plan, ups, len(changes), _stream()), "sgm_plan_update")
        for i, cur in staged:
            self._cur[i] = cur

    def close(self):
        if getattr(self, "_plan", None):
            lib().sgm_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
