"""GPU parity of the solve.

The preconditioner apply agrees with the oracle's element by element within
the rounding bound of the two summation orders (the oracle folds each row
left to right, the device adds each row as a balanced tree), in FP64 and
in FP32, and repeated calls give the same bits.  PCG reaches the relative
residual in FP64 and agrees with the oracle's solution to 1e-8 after removing
the null-space component; the mixed-precision PCG agrees with the oracle's
mixed PCG at equal iteration count, and its error against the FP64 oracle
solution is bounded and reported."""
import numpy as np
import pytest

from paper_2505_02977_amd import inputs
from tests.bounds import within_apply_bound
from tests.gpu_util import need_gpu, same_bits

# mixed precision (FP32 apply): agreement of two mixed PCG runs whose FP32
# applies differ only in summation order, at equal iteration count, relative
# to the solution's largest entry, per element, after projection
MIXED_VS_MIXED = 1e-5
# mixed-precision solution against the FP64 oracle solution (both to a
# relative residual of 1e-6), relative 2-norm after projection
MIXED_VS_FP64 = 1e-4

pytestmark = pytest.mark.gpu


def lap(n, i, j, w, excess=None):
    return inputs.laplacian_from_edges(n, i, j, w, excess)


def project(x):
    return x - x.mean()


def setup_case(kind):
    rng = np.random.default_rng({"grid": 1, "sddm": 2, "rand": 3, "star_last": 4,
                                 "star_first": 5, "chunglu": 6}[kind])
    if kind == "grid":
        W = inputs.grid2d_workload()
        return W.A, W.perm, W.seed, W.b, False
    if kind.startswith("star"):
        # a 10,000-leaf star plus a path through the leaves: the hub's row
        # (hub last) or column (hub first) of F runs past 4096 entries, the
        # workgroup row class of the solves
        d = 10000
        i = np.concatenate([np.zeros(d, int), np.arange(1, d)])
        j = np.concatenate([np.arange(1, d + 1), np.arange(2, d + 1)])
        A = lap(d + 1, i, j, rng.uniform(0.5, 2.0, len(i)))
        perm = rng.permutation(d + 1).astype(np.int32)
        k = int(np.argmax(perm == (d if kind == "star_last" else 0)))
        perm[k], perm[0] = perm[0], perm[k]
        b = rng.standard_normal(d + 1)
        return A, perm, 99, b - b.mean(), False
    if kind == "chunglu":
        i, j = inputs.chung_lu_edges(1 << 14, 16.0, 2.1, rng)
        n, i, j, _ = inputs.largest_component(1 << 14, i, j)
        A = lap(n, i, j, rng.uniform(0.5, 2.0, len(i)))
        b = rng.standard_normal(n)
        return A, rng.permutation(n).astype(np.int32), 31, b - b.mean(), False
    n = 2500
    i, j = inputs.connected_random_edges(n, 4 * n, rng)
    ex = None
    if kind == "sddm":
        ex = np.zeros(n)
        hot = rng.choice(n, 250, replace=False)
        ex[hot] = rng.random(250)
    A = lap(n, i, j, rng.uniform(0.05, 3.0, len(i)), ex)
    perm = rng.permutation(n).astype(np.int32)
    b = rng.standard_normal(n)
    if ex is None:
        b -= b.mean()
    return A, perm, 4242, b, ex is not None


@pytest.mark.parametrize("kind", ["grid", "sddm", "rand", "star_last", "star_first", "chunglu"])
@pytest.mark.parametrize("precision", [0, 1])
def test_apply_matches_oracle_within_bound(orc, kind, precision):
    torch = need_gpu()
    from paper_2505_02977_amd import parac
    A, perm, seed, b, _ = setup_case(kind)
    ref = orc.factor(A, perm=perm, seed=seed)
    dA = parac.DeviceCSR(A)
    f = parac.parac_factor(dA, perm=perm, seed=seed, keep_fp32=True)
    r = torch.tensor(b, device="cuda")
    z = torch.empty_like(r)
    zr = orc.apply(ref, b, precision=precision)
    first = None
    for rep in range(2):  # the second call reuses re-armed work vectors
        parac.parac_apply(f, r, z, precision=precision)
        torch.cuda.synchronize()
        got = z.cpu().numpy()
        ok, ratio = within_apply_bound(got, zr, ref, b, precision)
        assert ok, (kind, precision, rep, ratio)
        if first is None:
            first = got
        else:
            assert same_bits(got, first), (kind, precision)


@pytest.mark.parametrize("kind", ["grid", "sddm", "rand"])
def test_pcg_fp64(orc, kind):
    torch = need_gpu()
    from paper_2505_02977_amd import parac
    A, perm, seed, b, sddm = setup_case(kind)
    ref = orc.factor(A, perm=perm, seed=seed)
    dA = parac.DeviceCSR(A)
    f = parac.parac_factor(dA, perm=perm, seed=seed)
    bt = torch.tensor(b, device="cuda")
    xt = torch.empty_like(bt)
    st = parac.parac_pcg(dA, f, bt, xt, rtol=1e-6)[0]
    assert st["status"] == 0
    x = xt.cpu().numpy()
    # true residual recomputed here in FP64 as well
    res = np.linalg.norm(b - A.to_scipy() @ x) / np.linalg.norm(b)
    assert res <= 1e-6 and st["true_relres"] <= 1e-6
    assert abs(res - st["true_relres"]) <= 1e-9
    xr, sr = orc.pcg(A, ref, b, rtol=1e-6)
    if sr["iterations"] != st["iterations"]:
        xr, sr = orc.pcg(A, ref, b, rtol=0.0, maxit=st["iterations"])
    if not sddm:
        x, xr = project(x), project(xr)
    assert np.linalg.norm(x - xr) <= 1e-8 * np.linalg.norm(xr)


def mixed_errors(orc, A, ref, b, x, iterations, sddm):
    """Element-wise agreement with the oracle's mixed PCG at equal iteration
    count, and the relative error against the oracle's FP64 solution."""
    xm, sm = orc.pcg(A, ref, b, rtol=0.0, maxit=iterations, precision=1)
    xd, sd = orc.pcg(A, ref, b, rtol=1e-6)
    assert sd["status"] == 0
    if not sddm:
        x, xm, xd = project(x), project(xm), project(xd)
    vs_mixed = float(np.max(np.abs(x - xm)) / np.max(np.abs(xm)))
    vs_fp64 = float(np.linalg.norm(x - xd) / np.linalg.norm(xd))
    return vs_mixed, vs_fp64


@pytest.mark.parametrize("kind", ["grid", "sddm", "chunglu"])
def test_pcg_mixed(orc, kind):
    torch = need_gpu()
    from paper_2505_02977_amd import parac
    A, perm, seed, b, sddm = setup_case(kind)
    dA = parac.DeviceCSR(A)
    f = parac.parac_factor(dA, perm=perm, seed=seed, keep_fp32=True)
    bt = torch.tensor(b, device="cuda")
    xt = torch.empty_like(bt)
    st = parac.parac_pcg(dA, f, bt, xt, rtol=1e-6, precision=parac.PREC_MIXED)[0]
    assert st["status"] == 0 and st["true_relres"] <= 1e-6
    x = xt.cpu().numpy()
    assert np.linalg.norm(b - A.to_scipy() @ x) <= 1e-6 * np.linalg.norm(b)
    ref = orc.factor(A, perm=perm, seed=seed)
    vs_mixed, vs_fp64 = mixed_errors(orc, A, ref, b, x, st["iterations"], sddm)
    print("mixed %s: iterations %d, vs oracle mixed %.3e, vs oracle FP64 %.3e"
          % (kind, st["iterations"], vs_mixed, vs_fp64))
    assert vs_mixed <= MIXED_VS_MIXED, vs_mixed
    assert vs_fp64 <= MIXED_VS_FP64, vs_fp64


def test_pcg_exact_factor_one_iteration(orc):
    torch = need_gpu()
    from paper_2505_02977_amd import parac
    rng = np.random.default_rng(9)
    n = 500
    i, j = inputs.cycle_edges(n)
    A = lap(n, i, j, rng.uniform(0.5, 2, n))
    perm = rng.permutation(n).astype(np.int32)
    dA = parac.DeviceCSR(A)
    f = parac.parac_factor(dA, perm=perm, seed=1)
    b = inputs.rhs(n, rng)
    bt = torch.tensor(b, device="cuda")
    xt = torch.empty_like(bt)
    st = parac.parac_pcg(dA, f, bt, xt, rtol=1e-10)[0]
    assert st["iterations"] == 1 and st["true_relres"] < 1e-12


def test_inconsistent_rhs_rejected(orc):
    torch = need_gpu()
    from paper_2505_02977_amd import parac
    A, perm, seed, b, _ = setup_case("rand")
    dA = parac.DeviceCSR(A)
    f = parac.parac_factor(dA, perm=perm, seed=seed)
    bt = torch.tensor(b + 1.0, device="cuda")
    xt = torch.empty_like(bt)
    with pytest.raises(parac.ParacError) as e:
        parac.parac_pcg(dA, f, bt, xt)
    assert e.value.status == parac.EINCONSISTENT
    assert orc.check_consistent(A, 1, b + 1.0) == orc.EINCONSISTENT
