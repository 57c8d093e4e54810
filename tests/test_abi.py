"""The C ABI library loads, exports every declared entry point and validates
arguments on the host (no GPU needed: nothing here enqueues work)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1708_06301_amd import egosgm as eg

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "include", "egosgm.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return re.findall(r"^\s*(?:int|size_t|const char\s*\*)\s*(\w+)\s*\(", text, flags=re.M)


def test_every_declared_symbol_is_exported():
    names = declared()
    assert {"sgm_full", "sgm_reduced", "warp_disparity", "kalman_update",
            "sgm_windows_from_prediction", "egosgm_census"} <= set(names)
    lib = eg.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert eg.abi_version() == 5


def test_workspace_sizes():
    lib = eg.lib()
    n = lib.egosgm_sgm_workspace_bytes(1242, 375, 128)
    assert n >= 8 * 1242 * 375 * 128 + 16 * 1242 * 375
    assert lib.egosgm_sgm_workspace_bytes(0, 10, 64) == 0
    assert lib.egosgm_sgm_workspace_bytes(10, 10, 257) == 0
    assert lib.egosgm_windows_workspace_bytes(1242, 375) >= 4 * 375


FAKE = C.c_void_p(0x1000)   # never dereferenced: validation fails first


def _prm(**kw):
    base = dict(max_disp=64, p1=10, p2=120, s_max=80, lr_tol=1, n_paths=8, census_ready=0)
    base.update(kw)
    return eg.SgmParams(*base.values())


@pytest.mark.parametrize("kw,code", [(dict(max_disp=0), -1), (dict(max_disp=257), -1),
                                     (dict(p1=-1), -1), (dict(p1=50, p2=40), -1),
                                     (dict(p2=194), -1), (dict(s_max=-1), -1),
                                     (dict(n_paths=5), -1), (dict(n_paths=16), -1),
                                     (dict(census_ready=2), -1), (dict(census_ready=-1), -1)])
def test_sgm_rejects_bad_params(kw, code):
    lib = eg.lib()
    prm = _prm(**kw)
    rc = lib.sgm_full(FAKE, FAKE, 64, 32, 64, C.byref(prm), FAKE, FAKE, FAKE, None, None,
                      FAKE, 1 << 40, None)
    assert rc == code


def test_sgm_rejects_bad_shapes_and_workspace():
    lib = eg.lib()
    prm = _prm()
    assert lib.sgm_full(None, FAKE, 64, 32, 64, C.byref(prm), FAKE, FAKE, FAKE, None, None,
                        FAKE, 1 << 40, None) == -1
    assert lib.sgm_full(FAKE, FAKE, 64, 32, 63, C.byref(prm), FAKE, FAKE, FAKE, None, None,
                        FAKE, 1 << 40, None) == -1
    assert lib.sgm_full(FAKE, FAKE, 5000, 32, 5000, C.byref(prm), FAKE, FAKE, FAKE, None, None,
                        FAKE, 1 << 40, None) == -4
    assert lib.sgm_full(FAKE, FAKE, 64, 32, 64, C.byref(prm), FAKE, FAKE, FAKE, None, None,
                        FAKE, 100, None) == -2
    assert lib.sgm_reduced(FAKE, FAKE, 64, 32, 64, None, FAKE, FAKE, C.byref(prm), FAKE, FAKE,
                           FAKE, None, None, FAKE, 1 << 40, None) == -1


def test_windows_warp_kalman_validation():
    lib = eg.lib()
    assert lib.sgm_windows_from_prediction(FAKE, None, 64, 32, 3.0, -1, 0, 8, 64, FAKE, FAKE,
                                           FAKE, FAKE, 1 << 20, None) == -1
    assert lib.sgm_windows_from_prediction(FAKE, FAKE, 64, 32, 3.0, -1, 9, 8, 64, FAKE, FAKE,
                                           FAKE, FAKE, 1 << 20, None) == -1
    assert lib.sgm_windows_from_prediction(FAKE, FAKE, 64, 32, 3.0, -1, 0, 8, 64, FAKE, FAKE,
                                           FAKE, FAKE, 4, None) == -2
    # the allocation-free form: same checks, and sizes beyond its fixed scratch
    assert lib.sgm_windows_from_prediction_noalloc(FAKE, None, 64, 32, 3.0, -1, 0, 8, 64, FAKE, FAKE,
                                                   FAKE, None) == -1
    assert lib.sgm_windows_from_prediction_noalloc(FAKE, FAKE, 64, 32, 3.0, -1, 9, 8, 64, FAKE, FAKE,
                                                   FAKE, None) == -1
    assert lib.sgm_windows_from_prediction_noalloc(FAKE, FAKE, 0, 32, 3.0, -1, 0, 8, 64, FAKE, FAKE,
                                                   FAKE, None) == -1
    # 257 x 32769: 2 chunks per row, 65538 chunks > 65536
    assert lib.sgm_windows_from_prediction_noalloc(FAKE, FAKE, 257, 32769, 3.0, 4, 0, 8, 64, FAKE, FAKE,
                                                   FAKE, None) == -4
    R = (C.c_double * 9)(1, 0, 0, 0, 1, 0, 0, 0, 1)
    t = (C.c_double * 3)(0, 0, -1)
    assert lib.warp_disparity(FAKE, FAKE, 64, 32, R, t, 700.0, 32.0, 16.0, 0.54, 0.0, FAKE, FAKE,
                              FAKE, None) == -1
    assert lib.warp_disparity(FAKE, FAKE, 64, 32, R, t, -1.0, 32.0, 16.0, 0.54, 0.5, FAKE, FAKE,
                              FAKE, None) == -1
    assert lib.kalman_update(FAKE, FAKE, FAKE, FAKE, -1, 0, FAKE, FAKE, None) == -1
    assert lib.kalman_update(FAKE, FAKE, FAKE, FAKE, 0, 0, FAKE, FAKE, None) == 0


def test_warp_matrix_host_helper_matches_oracle(orc):
    r = np.random.default_rng(0)
    for _ in range(50):
        a, b, c = r.normal(0, 0.05, 3)
        Ry = np.array([[np.cos(a), 0, np.sin(a)], [0, 1, 0], [-np.sin(a), 0, np.cos(a)]])
        Rx = np.array([[1, 0, 0], [0, np.cos(b), -np.sin(b)], [0, np.sin(b), np.cos(b)]])
        Rz = np.array([[np.cos(c), -np.sin(c), 0], [np.sin(c), np.cos(c), 0], [0, 0, 1]])
        R = Ry @ Rx @ Rz
        t = r.normal(0, 1, 3)
        cam = (r.uniform(300, 1500), r.uniform(100, 1000), r.uniform(50, 500), r.uniform(0.1, 1))
        H = eg.warp_matrix(R, t, *cam)
        Ho = orc.warp_matrix(R, t, *cam)
        assert np.array_equal(H, Ho.astype(np.float32))
    assert np.array_equal(eg.warp_matrix(np.eye(3), np.zeros(3), 718, 620.5, 187, 0.54),
                          np.eye(4, dtype=np.float32))


def test_tuning_validation():
    import ctypes as C
    lib = eg.lib()
    before = eg.get_tuning()
    bad = eg.Tuning(24, 32, 1, 16)
    assert lib.egosgm_set_tuning(C.byref(bad)) == -1
    assert lib.egosgm_set_tuning(None) == -1
    assert eg.get_tuning() == before
    assert lib.egosgm_set_tuning(C.byref(eg.Tuning(32, 32, 9, 16))) == -1
    assert lib.egosgm_set_tuning(C.byref(eg.Tuning(32, 32, -1, 16))) == -1
    assert lib.egosgm_set_tuning(C.byref(eg.Tuning(32, 32, 8, 16))) == 0
    assert lib.egosgm_set_tuning(C.byref(eg.Tuning(32, 32, 3, 16))) == 0
    assert lib.egosgm_set_tuning(C.byref(eg.Tuning(32, 32, 0, 8))) == -1
    assert lib.egosgm_set_tuning(C.byref(eg.Tuning(32, 32, 1, 16, 2))) == -1
    assert lib.egosgm_set_tuning(C.byref(eg.Tuning(32, 32, 1, 16, 1))) == 0
    # arguments left out keep their current value (wide_offsets = 1 from above)
    eg.set_tuning(16, 64, 0, 32)
    assert eg.get_tuning() == dict(full_group=16, ragged_group=64, ragged_schedule=0, batch_group=32,
                                   wide_offsets=1, batch_persistent=0)
    eg.set_tuning(wide_offsets=0, batch_persistent=1)
    assert eg.get_tuning() == dict(full_group=16, ragged_group=64, ragged_schedule=0, batch_group=32,
                                   wide_offsets=0, batch_persistent=1)
    assert lib.egosgm_set_tuning(C.byref(eg.Tuning(32, 32, 1, 16, 0, 2))) == -1
    eg.set_tuning(**before)


def test_plan_validation():
    import ctypes as C
    lib = eg.lib()
    P = (eg.PairDesc * 1)()
    assert lib.egosgm_plan_workspace_bytes(P, 1) == 0           # null pointers
    P[0] = eg.PairDesc(FAKE, FAKE, 64, 32, 64, 128, None, None, None, FAKE, FAKE, FAKE, None)
    n = lib.egosgm_plan_workspace_bytes(P, 1)
    assert n >= lib.egosgm_sgm_workspace_bytes(64, 32, 128)
    P[0].lo = FAKE                                               # lo without hi/offsets
    assert lib.egosgm_plan_workspace_bytes(P, 1) == 0
    out = C.c_void_p()
    prm = _prm()
    P[0].lo = None
    assert lib.sgm_plan_create(P, 1, C.byref(prm), FAKE, 16, C.byref(out)) == -2
    assert lib.sgm_plan_create(P, 0, C.byref(prm), FAKE, n, C.byref(out)) == -1
    assert lib.sgm_plan_run(None, None) == -1
    assert lib.sgm_plan_destroy(None) == 0


def test_sad_check_validation():
    lib = eg.lib()
    f = FAKE
    assert lib.sad_check(None, f, 10, 10, 10, 2, 100, f, f, f, None) == -1
    assert lib.sad_check(f, f, 10, 10, 9, 2, 100, f, f, f, None) == -1     # pitch < w
    assert lib.sad_check(f, f, 10, 10, 10, 8, 100, f, f, f, None) == -1    # radius > 7
    assert lib.sad_check(f, f, 10, 10, 10, 2, -1, f, f, f, None) == -1     # sad_max < 0
    assert lib.sad_check(f, f, 0, 10, 10, 2, 100, f, f, f, None) == -1


def test_prediction_lr_check_validation(orc):
    lib = eg.lib()
    f = FAKE
    assert lib.lr_check_prediction(None, f, f, 10, 10, C.c_float(1.0), None) == -1
    assert lib.lr_check_prediction(f, f, f, 0, 10, C.c_float(1.0), None) == -1
    assert lib.lr_check_prediction(f, f, f, 10, 10, C.c_float(-0.5), None) == -1
    assert lib.lr_check_prediction(f, f, f, 10, 10, C.c_float(float("nan")), None) == -1
    assert lib.lr_check_prediction(f, f, f, 1 << 16, 1 << 15, C.c_float(1.0), None) == -4
    assert lib.disparity_to_float(f, f, 0, None) == -1
    assert lib.disparity_to_float(None, f, 10, None) == -1
    r = np.random.default_rng(3)
    for _ in range(20):
        a, b = r.normal(0, 0.1, 2)
        R = (np.array([[np.cos(a), 0, np.sin(a)], [0, 1, 0], [-np.sin(a), 0, np.cos(a)]]) @
             np.array([[1, 0, 0], [0, np.cos(b), -np.sin(b)], [0, np.sin(b), np.cos(b)]]))
        t, base = r.normal(0, 1, 3), r.uniform(0.1, 1.0)
        Rr, tr = eg.right_motion(R, t, base)
        assert np.array_equal(Rr, R)
        assert np.allclose(tr, orc.right_motion(R, t, base), rtol=0, atol=1e-15)


def test_predict_disparity_validation():
    lib = eg.lib()
    f = FAKE
    R = (C.c_double * 9)(1, 0, 0, 0, 1, 0, 0, 0, 1)
    t = (C.c_double * 3)(0, 0, -1)
    args = lambda **kw: dict(dict(dp=f, pp=f, w=10, h=10, q=0.5, et=2.0, ft=1.0, do=C.c_void_p(0x2000),
                                  po=C.c_void_p(0x3000), z=f), **kw)
    def call(a):
        return lib.predict_disparity(a["dp"], a["pp"], a["w"], a["h"], R, t, 700.0, 5.0, 5.0, 0.5, a["q"],
                                     a["et"], a["ft"], a["do"], a["po"], a["z"], None)
    assert call(args(dp=None)) == -1
    assert call(args(w=0)) == -1
    assert call(args(q=0.0)) == -1
    assert call(args(et=float("nan"))) == -1
    assert call(args(do=f)) == -1          # output aliases an input


def test_sgm_census_validation():
    lib = eg.lib()
    f = FAKE
    n = lib.egosgm_sgm_workspace_bytes(64, 32, 64)
    assert lib.sgm_census(None, f, 64, 32, 64, 64, f, n, None) == -1
    assert lib.sgm_census(f, f, 64, 32, 63, 64, f, n, None) == -1          # pitch < w
    assert lib.sgm_census(f, f, 64, 32, 64, 0, f, n, None) == -1           # max_disp
    assert lib.sgm_census(f, f, 64, 32, 64, 64, f, n - 1, None) == -2      # workspace too small
    assert lib.sgm_census(f, f, 64, 32, 64, 64, None, n, None) == -2


def test_plans_reject_a_precomputed_census():
    lib = eg.lib()
    prm = _prm(census_ready=1)
    P = (eg.PairDesc * 1)()
    out = C.c_void_p()
    assert lib.sgm_plan_create(P, 1, C.byref(prm), FAKE, 1 << 40, C.byref(out)) == -1


def test_vo_workspace_and_validation():
    """estimate_motion / vo_normal_equations validate sizes and parameters on
    the host; the workspace size covers five float images per level."""
    lib = eg.lib()
    prm = eg.vo_params(levels=4, iters=(2, 4, 8, 10))
    n = lib.egosgm_vo_workspace_bytes(1242, 375, C.byref(prm))
    assert n >= 4 * 5 * 1242 * 375
    assert lib.egosgm_vo_workspace_bytes(15, 375, C.byref(prm)) == 0
    assert lib.egosgm_vo_workspace_bytes(100, 100, C.byref(eg.vo_params(levels=4))) == 0   # coarsest 12 x 12
    bad = [eg.vo_params(levels=0), eg.vo_params(levels=7), eg.vo_params(levels=2, iters=(65, 1)),
           eg.vo_params(levels=2, iters=(-1, 1)), eg.vo_params(levels=2, huber=0.0),
           eg.vo_params(levels=2, min_disp=-1.0), eg.vo_params(levels=2, huber=float("nan"))]
    for b in bad:
        assert lib.egosgm_vo_workspace_bytes(640, 192, C.byref(b)) == 0
        rc = lib.estimate_motion(FAKE, FAKE, 640, 192, 640, FAKE, 500.0, 320.0, 96.0, 0.5, C.byref(b), FAKE,
                                 FAKE, 1 << 40, None)
        assert rc == -1
    ok = eg.vo_params(levels=3, iters=(1, 1, 1))
    args = (640, 192, 640, FAKE, 500.0, 320.0, 96.0, 0.5, C.byref(ok))
    assert lib.estimate_motion(None, FAKE, *args, FAKE, FAKE, 1 << 40, None) == -1          # NULL image
    assert lib.estimate_motion(FAKE, FAKE, 640, 192, 639, FAKE, 500.0, 320.0, 96.0, 0.5, C.byref(ok), FAKE,
                               FAKE, 1 << 40, None) == -1                                    # pitch < w
    assert lib.estimate_motion(FAKE, FAKE, 640, 192, 640, FAKE, -1.0, 320.0, 96.0, 0.5, C.byref(ok), FAKE,
                               FAKE, 1 << 40, None) == -1                                    # f <= 0
    assert lib.estimate_motion(FAKE, FAKE, *args, FAKE, FAKE, 16, None) == -2                # small workspace
    assert lib.estimate_motion(FAKE, FAKE, *args, FAKE, None, 1 << 40, None) == -2           # no workspace
    assert lib.vo_normal_equations(FAKE, FAKE, *args, 3, FAKE, FAKE, FAKE, 1 << 40, None) == -1   # level
    assert lib.vo_normal_equations(FAKE, FAKE, *args, -1, FAKE, FAKE, FAKE, 1 << 40, None) == -1
    assert lib.vo_normal_equations(FAKE, FAKE, *args, 0, FAKE, None, FAKE, 1 << 40, None) == -1   # out
