"""usfft_eval_noalloc (the entry point that allocates nothing) against
usfft_eval through the C ABI, on two calls in a row, the second with fewer
points: same kernels, so the outputs agree to rounding (evaluation of
eq. (3.1); the two calls also show the shared scratch carries nothing over)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_eval_noalloc_matches_eval(lib):
    prob, par = W.WORKLOADS["cpu16_d4"]
    plan = lib.Plan(prob, dict(par, precision=lib.FP64, pcg_rtol=1e-13))
    res = lib.detect(plan, 3)
    assert res.n > 0
    g = torch.Generator(device="cuda").manual_seed(11)
    for n in (1000, 203):
        print("eval_noalloc: %d frequencies, %d points, G = %d" % (res.n, n, res.G), flush=True)
        y = torch.rand((n, prob["d"]), dtype=torch.float64, device="cuda", generator=g)
        ref = torch.full((n, res.G), np.nan, dtype=torch.float64, device="cuda")
        out = torch.full((n, res.G), np.nan, dtype=torch.float64, device="cuda")
        lib.eval(res, y, ref)
        lib.eval_noalloc(res, y, out)
        torch.cuda.synchronize()
        a, b = out.cpu().numpy(), ref.cpu().numpy()
        assert np.isfinite(a).all()
        err = np.abs(a - b).max() / np.abs(b).max()
        print("max rel. difference %.2e" % err)
        assert err <= 1e-13
