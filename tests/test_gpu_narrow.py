"""GPU checks of the narrow final levels of the triangular solves.

The dependency-driven sweeps leave the final run of levels with few rows each
to one workgroup per slot (values in LDS, a barrier per level).  A row's sum
keeps the sweeps' association (products, trees of 16, balanced trees over
chunks, block folds), so the single-vector apply, which takes the narrow
levels in that workgroup, is bit-identical to the block apply, which runs
every level in the sweeps, in both precisions; and it agrees with the
oracle's apply within the rounding bound.  A factor whose levels are all
narrow (the sweeps then have no unit at all) applies the same bits again and
again."""
import numpy as np
import pytest

from paper_2505_02977_amd import inputs
from tests.bounds import within_apply_bound
from tests.gpu_util import need_gpu, same_bits
from tests.test_gpu_block import single_applies

pytestmark = pytest.mark.gpu


def workload(case):
    if case == "grid3d_24":
        return inputs.grid3d_workload(24)
    return inputs.grid2d_workload(32)


@pytest.mark.parametrize("case", ["grid3d_24", "grid2d_32"])
@pytest.mark.parametrize("precision", [0, 1])
def test_narrow_levels_bit_identical_to_sweeps(orc, case, precision):
    torch = need_gpu()
    from paper_2505_02977_amd import parac
    W = workload(case)
    A = W.A
    f = parac.parac_factor(parac.DeviceCSR(A), perm=W.perm, seed=W.seed, keep_fp32=True)
    info = f.info()
    print("%s: depth %d, narrow levels %d" % (case, info["depth"], info["narrow_levels"]),
          flush=True)
    assert info["narrow_levels"] >= 16
    if case == "grid2d_32":
        # 1,024 positions, short rows: every level is narrow
        assert info["narrow_levels"] == info["depth"]
    else:
        assert info["narrow_levels"] < info["depth"]
    rng = np.random.default_rng(31)
    nrhs = 3
    B = rng.standard_normal((A.n, nrhs))
    B -= B.mean(axis=0)
    want = single_applies(f, B, precision)
    again = single_applies(f, B, precision)
    for j in range(nrhs):
        assert same_bits(again[:, j], want[:, j]), j
    r = torch.tensor(B, device="cuda")
    z = torch.empty_like(r)
    for cps in (1, 2):
        parac.parac_block_shape_set(f, nrhs, precision, cols_per_sweep=cps)
        z.fill_(np.nan)
        parac.parac_apply(f, r, z, precision=precision)
        got = z.cpu().numpy()
        bad = [j for j in range(nrhs) if not same_bits(got[:, j], want[:, j])]
        assert not bad, (case, precision, cps, bad)
    ref = orc.factor(A, perm=W.perm, seed=W.seed)
    b = B[:, 0].copy()
    ok, ratio = within_apply_bound(want[:, 0], orc.apply(ref, b, precision=precision), ref, b,
                                   precision)
    assert ok, ratio
