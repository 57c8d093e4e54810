"""The allocation-free windows entry point (sgm_windows_from_prediction_noalloc)
against the workspace one, through the C ABI: two calls in a row on one GPU,
the second on a smaller map, so the second reuses the library's scratch
array with the first call's totals still in it.  Windows and offsets are
integers: bit-exact."""
import numpy as np
import pytest
import torch

from paper_1708_06301_amd import egosgm as eg

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _prediction(w, h, D, seed):
    r = np.random.default_rng(seed)
    d = r.uniform(0, D - 1, size=(h, w)).astype(np.float32)
    d[r.random((h, w)) < 0.1] = -1.0
    p = r.uniform(0, 5.0, size=(h, w)).astype(np.float32)
    return torch.from_numpy(d).to(DEV), torch.from_numpy(p).to(DEV)


@pytest.mark.parametrize("r_fixed", [-1, 6])
def test_noalloc_windows_equal_the_workspace_call(r_fixed):
    for w, h, D, seed in [(2048, 1024, 256, 1), (333, 77, 96, 2)]:   # second call smaller
        print("CASE noalloc windows", w, h, D, "r_fixed", r_fixed, flush=True)
        d, p = _prediction(w, h, D, seed)
        ref = eg.windows_from_prediction(d, p, D, r_fixed=r_fixed, r_min=1, r_max=16)
        out = (torch.full((h, w), -7, dtype=torch.int16, device=DEV),
               torch.full((h, w), -7, dtype=torch.int16, device=DEV),
               torch.full((h * w + 1,), -7, dtype=torch.int32, device=DEV))
        got = eg.windows_from_prediction_noalloc(d, p, D, r_fixed=r_fixed, r_min=1, r_max=16, out=out)
        torch.cuda.synchronize()
        for a, b, name in zip(ref, got, ("lo", "hi", "offsets")):
            assert torch.equal(a, b), name
