"""parac_pcg_static, the PCG entry point that allocates no device memory,
against parac_pcg: two calls in a row (the second on a smaller system, so
the fixed array holds the first call's larger contents), in FP64 and with
the FP32 apply; x and the stats must be the same bits, since both run the
same kernels with the same launch shapes.  A system above the array's limit
is rejected with EINVAL before any device work, and the next call works."""
import numpy as np
import pytest

from paper_2505_02977_amd import inputs
from tests.gpu_util import need_gpu, same_bits

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def systems():
    big = inputs.grid3d_workload(40)            # 64,000 vertices, Laplacian
    small = inputs.sddm_system(3, nmax=2e4)     # SDDM: ground vertex added
    return [(big, False), (small, True)]


def run_pair(parac, torch, W, precision):
    dA = parac.DeviceCSR(W.A)
    f = parac.parac_factor(dA, perm=W.perm, seed=W.seed,
                           keep_fp32=precision == parac.PREC_MIXED)
    b = torch.tensor(np.ascontiguousarray(W.b), device="cuda")
    x0 = torch.empty_like(b)
    s0 = parac.parac_pcg(dA, f, b, x0, rtol=1e-6, precision=precision)[0]
    x1 = torch.full_like(b, float("nan"))
    s1 = parac.parac_pcg_static(dA, f, b, x1, rtol=1e-6, precision=precision)
    torch.cuda.synchronize()
    return s0, x0.cpu().numpy(), s1, x1.cpu().numpy()


@pytest.mark.parametrize("precision", [0, 1])
def test_static_pcg_matches_pcg_twice(precision):
    torch = need_gpu()
    from paper_2505_02977_amd import parac
    for W, sddm in systems():
        say("static PCG: %s n=%d precision=%d" % (W.name, W.A.n, precision))
        s0, x0, s1, x1 = run_pair(parac, torch, W, precision)
        assert s0["status"] == 0 and s1["status"] == 0, (s0, s1)
        assert s1["iterations"] == s0["iterations"]
        assert s1["applies"] == s0["applies"]
        assert s1["relres"] == s0["relres"] and s1["true_relres"] == s0["true_relres"]
        assert same_bits(x1, x0), "x differs from parac_pcg"
        res = np.linalg.norm(W.b - W.A.to_scipy() @ x1) / np.linalg.norm(W.b)
        assert res <= 1e-6


def test_static_pcg_rejects_above_limit():
    torch = need_gpu()
    from paper_2505_02977_amd import parac
    n = parac.pcg_static_max_rows() + 1
    say("static PCG limit: path of %d vertices" % n)
    i = np.arange(n - 1)
    A = inputs.laplacian_from_edges(n, i, i + 1, np.ones(n - 1))
    dA = parac.DeviceCSR(A)
    # random labels: a path labelled in order would be one dependent chain
    # of n pivots, eliminated one after another
    perm = np.random.default_rng(5).permutation(n).astype(np.int32)
    f = parac.parac_factor(dA, perm=perm, seed=5)
    b = torch.zeros(n, dtype=torch.float64, device="cuda")
    x = torch.empty_like(b)
    with pytest.raises(parac.ParacError) as e:
        parac.parac_pcg_static(dA, f, b, x)
    assert e.value.status == parac.EINVAL
    assert "too large" in str(e.value)
    del f, dA
    # the next call on a system within the limit works
    W = inputs.grid2d_workload(side=32)
    s0, x0, s1, x1 = run_pair(parac, torch, W, parac.PREC_FP64)
    assert s1["status"] == 0 and same_bits(x1, x0)
