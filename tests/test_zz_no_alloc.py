"""The no-allocation entry point lgw_hpsi_noalloc (its intermediates in the
library's fixed device scratch) against lgw_hpsi, which allocates its own
workspace: the same kernels on the same inputs, so the results must be
bitwise equal.  Two calls in a row, the second with fewer vectors (the
scratch keeps the first call's contents), in both precisions; a size beyond
the fixed scratch is refused before any device work."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from synthetic import make_workload


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_hpsi_noalloc_matches_hpsi(precision):
    from paper_1408_3036_amd import Lgw
    from paper_1408_3036_amd.lgw import LgwError
    w = make_workload(2)
    lg = Lgw(w.L, w.N, w.ecut, torch.from_numpy(w.V), torch.from_numpy(w.psi), w.eps,
             precision=precision)
    try:
        rng = np.random.default_rng(97)
        shift = -0.37 + 0.21j
        for n in (96, 5):
            print(f"hpsi_noalloc {precision}: n = {n}", flush=True)
            x = torch.from_numpy(rng.standard_normal((n, lg.npw)) + 1j * rng.standard_normal((n, lg.npw))).cuda()
            y = torch.full_like(x, float("nan"))
            lg.hpsi_noalloc(x, y, shift)
            torch.cuda.synchronize()
            ref = lg.hpsi(x, shift)
            torch.cuda.synchronize()
            assert torch.equal(y, ref)
        big = 4096
        x = torch.zeros((big, lg.npw), dtype=torch.complex128, device="cuda")
        with pytest.raises(LgwError) as ei:
            lg.hpsi_noalloc(x, torch.empty_like(x), shift)
        assert ei.value.status == 1 and "at most" in str(ei.value)
    finally:
        lg.close()
