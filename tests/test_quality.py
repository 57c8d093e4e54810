"""Bad-pixel rates (the evaluation of Sec. 3) on hand-built maps."""
import numpy as np

from paper_1708_06301_amd.quality import bad_pixels, summarise


def test_bad_pixel_rates_by_hand():
    gt = np.array([[100.0, 10.0, 100.0, 100.0, 50.0, 200.0, np.inf, -1.0]])
    d = np.array([[102.9, 13.1, 104.0, 106.0, -1.0, 50.0, 5.0, 5.0]])
    # evaluated: first six (gt in [0, 128) -> 200 is out, inf and -1 out) -> five
    r = bad_pixels(d, gt, max_disp=128)
    assert r["n"] == 5
    assert r["density"] == 4 / 5
    # errors: 2.9 of 100 (fine), 3.1 of 10 (bad both ways), 4 of 100 (>3 px only), 6 of 100 (both)
    assert r["bad_or_est"] == 3 / 4
    assert r["bad_and_est"] == 2 / 4
    assert r["bad_or_all"] == (3 + 1) / 5      # the missing estimate counts as bad
    assert r["bad_and_all"] == (2 + 1) / 5


def test_perfect_and_empty_maps():
    gt = np.full((4, 5), 20.0)
    assert bad_pixels(gt.copy(), gt, 64)["bad_or_all"] == 0.0
    r = bad_pixels(np.full((4, 5), -1.0), gt, 64)
    assert r["density"] == 0.0 and r["bad_or_all"] == 1.0 and r["bad_or_est"] == 0.0
    s = summarise([bad_pixels(gt.copy(), gt, 64), r])
    assert s["bad_or_all"] == 0.5 and s["density"] == 0.5
