"""GPU parity of the block (several right-hand sides) path.

The block apply is bit-identical, column by column, to the device's
single-vector apply of that column, for every launch shape (columns per lane,
tail threshold) and for the default shape, and agrees with the oracle's apply
of that column within the rounding bound of the two summation orders; block
PCG runs an independent recurrence per column, so each column reaches the
relative residual and agrees with the oracle's single-vector PCG of that
column."""
import numpy as np
import pytest

from paper_2505_02977_amd import inputs
from tests.bounds import within_apply_bound
from tests.gpu_util import need_gpu, same_bits
from tests.test_gpu_solve import MIXED_VS_MIXED

pytestmark = pytest.mark.gpu


def lap(n, i, j, w, excess=None):
    return inputs.laplacian_from_edges(n, i, j, w, excess)


def setup_case(kind, nrhs):
    rng = np.random.default_rng({"grid": 11, "sddm": 12}[kind] * 100 + nrhs)
    if kind == "grid":
        W = inputs.grid2d_workload()
        A, perm, seed, ex = W.A, W.perm, W.seed, None
    else:
        n = 3000
        i, j = inputs.connected_random_edges(n, 4 * n, rng)
        ex = np.zeros(n)
        hot = rng.choice(n, 300, replace=False)
        ex[hot] = rng.random(300)
        A = lap(n, i, j, rng.uniform(0.05, 3.0, len(i)), ex)
        perm = rng.permutation(n).astype(np.int32)
        seed = 777
    B = rng.standard_normal((A.n, nrhs))
    B *= 10.0 ** rng.uniform(-3, 3, nrhs)  # columns of very different scale
    if ex is None:
        B -= B.mean(axis=0)
    return A, perm, seed, np.ascontiguousarray(B), ex is not None


def single_applies(f, B, precision):
    """The device's single-vector apply of every column of B."""
    import torch
    from paper_2505_02977_amd import parac
    out = np.empty_like(B)
    for j in range(B.shape[1]):
        r = torch.tensor(B[:, j].copy(), device="cuda")
        z = torch.empty_like(r)
        parac.parac_apply(f, r, z, precision=precision)
        out[:, j] = z.cpu().numpy()
    return out


# cpl 0: one dependency-driven sweep pair per column; else level-synchronous
SHAPES = [(0, 256)] + [(c, t) for c in (1, 2, 4) for t in (0, 64, 1024, 1 << 40)]


@pytest.mark.parametrize("kind", ["grid", "sddm"])
@pytest.mark.parametrize("precision", [0, 1])
def test_block_apply_every_shape_bit_identical(orc, kind, precision):
    torch = need_gpu()
    from paper_2505_02977_amd import parac
    nrhs = 32
    A, perm, seed, B, _ = setup_case(kind, nrhs)
    ref = orc.factor(A, perm=perm, seed=seed)
    f = parac.parac_factor(parac.DeviceCSR(A), perm=perm, seed=seed, keep_fp32=True)
    want = single_applies(f, B, precision)
    for j in (0, nrhs - 1):
        b = B[:, j].copy()
        ok, ratio = within_apply_bound(want[:, j], orc.apply(ref, b, precision=precision), ref, b,
                                       precision)
        assert ok, (j, ratio)
    r = torch.tensor(B, device="cuda")
    z = torch.empty_like(r)
    for cpl, tail in SHAPES:
        parac.parac_block_shape_set(f, nrhs, precision, cpl=cpl, tail_rows=tail)
        z.fill_(np.nan)
        parac.parac_apply(f, r, z, precision=precision)
        assert same_bits(z.cpu().numpy(), want), (kind, precision, cpl, tail)


@pytest.mark.parametrize("nrhs", [2, 7, 70])
def test_block_apply_default_shape(orc, nrhs):
    torch = need_gpu()
    from paper_2505_02977_amd import parac
    A, perm, seed, B, _ = setup_case("grid", nrhs)
    f = parac.parac_factor(parac.DeviceCSR(A), perm=perm, seed=seed)
    r = torch.tensor(B, device="cuda")
    z = torch.empty_like(r)
    parac.parac_apply(f, r, z)
    got = z.cpu().numpy()
    want = single_applies(f, B, 0)
    for j in range(nrhs):
        assert same_bits(got[:, j], want[:, j]), j
    # chunks of at most 64 columns, each solved by column sweeps unless a
    # level-synchronous shape is fixed
    for cols in sorted({min(64, nrhs - c0) for c0 in range(0, nrhs, 64)}):
        sh = parac.parac_block_shape_get(f, cols)
        assert sh["cpl"] == 0 and sh["tail_rows"] >= 0
    # the single-vector path agrees as well
    z1 = torch.empty(A.n, dtype=torch.float64, device="cuda")
    parac.parac_apply(f, r[:, 0].contiguous(), z1)
    assert same_bits(z1.cpu().numpy(), got[:, 0])


@pytest.mark.parametrize("kind", ["grid", "sddm"])
def test_block_pcg_fp64_per_column(orc, kind):
    torch = need_gpu()
    from paper_2505_02977_amd import parac
    nrhs = 6
    A, perm, seed, B, sddm = setup_case(kind, nrhs)
    B[:, 3] = 0.0  # a zero column is done before the first iteration
    ref = orc.factor(A, perm=perm, seed=seed)
    dA = parac.DeviceCSR(A)
    f = parac.parac_factor(dA, perm=perm, seed=seed)
    bt = torch.tensor(B, device="cuda")
    xt = torch.full_like(bt, np.nan)
    sts = parac.parac_pcg(dA, f, bt, xt, rtol=1e-6)
    X = xt.cpu().numpy()
    L = A.to_scipy()
    for j in range(nrhs):
        st = sts[j]
        assert st["status"] == 0, (j, st)
        if j == 3:
            assert st["iterations"] == 0 and not X[:, j].any()
            continue
        b = B[:, j]
        res = np.linalg.norm(b - L @ X[:, j]) / np.linalg.norm(b)
        assert res <= 1e-6 and abs(res - st["true_relres"]) <= 1e-9, (j, res, st)
        xr, sr = orc.pcg(A, ref, b.copy(), rtol=1e-6)
        if sr["iterations"] != st["iterations"]:
            xr, sr = orc.pcg(A, ref, b.copy(), rtol=0.0, maxit=st["iterations"])
        x = X[:, j]
        if not sddm:
            x, xr = x - x.mean(), xr - xr.mean()
        assert np.linalg.norm(x - xr) <= 1e-8 * np.linalg.norm(xr), j
    # the level-synchronous block apply gives the same bits
    parac.parac_block_shape_set(f, nrhs, 0, cpl=2, tail_rows=64)
    x2 = torch.full_like(bt, np.nan)
    sts2 = parac.parac_pcg(dA, f, bt, x2, rtol=1e-6)
    assert [s["iterations"] for s in sts2] == [s["iterations"] for s in sts]
    assert same_bits(x2.cpu().numpy(), X)


def test_block_pcg_mixed_and_chunks(orc):
    torch = need_gpu()
    from paper_2505_02977_amd import parac
    nrhs = 70  # two chunks: 64 + 6 columns
    A, perm, seed, B, _ = setup_case("grid", nrhs)
    dA = parac.DeviceCSR(A)
    f = parac.parac_factor(dA, perm=perm, seed=seed, keep_fp32=True)
    bt = torch.tensor(B, device="cuda")
    xt = torch.empty_like(bt)
    sts = parac.parac_pcg(dA, f, bt, xt, rtol=1e-6, precision=parac.PREC_MIXED)
    X = xt.cpu().numpy()
    L = A.to_scipy()
    ref = orc.factor(A, perm=perm, seed=seed)
    for j in (0, 5, 63, 64, 69):
        b = B[:, j]
        res = np.linalg.norm(b - L @ X[:, j]) / np.linalg.norm(b)
        assert sts[j]["status"] == 0 and res <= 1e-6, (j, res)
        xm, _ = orc.pcg(A, ref, b.copy(), rtol=0.0, maxit=sts[j]["iterations"], precision=1)
        x = X[:, j] - X[:, j].mean()
        xm = xm - xm.mean()
        assert np.max(np.abs(x - xm)) <= MIXED_VS_MIXED * np.max(np.abs(xm)), j


def test_block_inconsistent_column_rejected(orc):
    torch = need_gpu()
    from paper_2505_02977_amd import parac
    A, perm, seed, B, _ = setup_case("grid", 5)
    B[:, 2] += 1.0
    dA = parac.DeviceCSR(A)
    f = parac.parac_factor(dA, perm=perm, seed=seed)
    bt = torch.tensor(B, device="cuda")
    xt = torch.empty_like(bt)
    with pytest.raises(parac.ParacError) as e:
        parac.parac_pcg(dA, f, bt, xt)
    assert e.value.status == parac.EINCONSISTENT
    assert orc.check_consistent(A, 1, B[:, 2].copy()) == orc.EINCONSISTENT
    assert orc.check_consistent(A, 1, B[:, 1].copy()) == 0
