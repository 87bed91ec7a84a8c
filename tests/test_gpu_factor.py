"""GPU parity of the factor: the FP64 F and D built by the persistent HIP
elimination are identical, bit for bit, to the CPU oracle's, on the same
seeded inputs -- whatever the grid size, the pool size or the timing."""
import numpy as np
import pytest

from paper_2505_02977_amd import inputs
from tests.gpu_util import compare_factor, need_gpu

pytestmark = pytest.mark.gpu


def lap(n, i, j, w, excess=None):
    return inputs.laplacian_from_edges(n, i, j, w, excess)


def gpu_factor(A, perm, seed, **kw):
    from paper_2505_02977_amd import parac
    dA = parac.DeviceCSR(A)
    return parac.parac_factor(dA, perm=perm, seed=seed, **kw)


def case_graphs():
    rng = np.random.default_rng(77)
    out = []
    # tiny and ragged sizes
    for n in (1, 2, 3, 5, 17, 63, 64, 65, 130):
        if n == 1:
            A = lap(1, np.zeros(0, int), np.zeros(0, int), np.zeros(0))
        else:
            i, j = inputs.connected_random_edges(n, 2 * n, rng)
            A = lap(n, i, j, rng.uniform(0.01, 10.0, len(i)))
        out.append(("rand%d" % n, A, None))
    # unit weights: ties in the sampling order
    i, j = inputs.grid2d_edges(20, 13)
    out.append(("grid_unit", lap(260, i, j, np.ones(len(i))), None))
    # a hub: gathered neighbourhoods beyond one wave (multi-tile suffix sums)
    n = 400
    i = np.concatenate([np.zeros(299, int), np.arange(1, 399)])
    j = np.concatenate([np.arange(1, 300), np.arange(2, 400)])
    i, j = inputs.dedupe_edges(i, j)
    out.append(("hub", lap(n, i, j, rng.uniform(0.1, 1.0, len(i))), None))
    # a big hub on a path of leaves, labelled mid-way: its gathered list runs
    # past the rank-sort limit and holds several records per neighbour (the
    # radix-sort path of both sorts)
    n = 6001
    i = np.concatenate([np.zeros(6000, int), np.arange(1, 6000)])
    j = np.concatenate([np.arange(1, 6001), np.arange(2, 6001)])
    out.append(("bighub", lap(n, i, j, rng.uniform(0.1, 1.0, len(i))), None))
    # power-law degrees (Chung-Lu, beta 2.1)
    i, j = inputs.chung_lu_edges(1 << 14, 16.0, 2.1, rng)
    m, i, j, _ = inputs.largest_component(1 << 14, i, j)
    out.append(("chung_lu_16k", lap(m, i, j, rng.uniform(0.5, 2.0, len(i))), None))
    # SDDM with a ground vertex
    n = 300
    i, j = inputs.connected_random_edges(n, 3 * n, rng)
    ex = np.zeros(n)
    hot = rng.choice(n, 30, replace=False)
    ex[hot] = rng.random(30)
    out.append(("sddm", lap(n, i, j, rng.uniform(0.1, 2.0, len(i)), ex), ex))
    # two components
    i1, j1 = inputs.connected_random_edges(100, 200, rng)
    i2, j2 = inputs.connected_random_edges(80, 150, rng)
    i = np.concatenate([i1, i2 + 100])
    j = np.concatenate([j1, j2 + 100])
    out.append(("two_comp", lap(180, i, j, rng.uniform(0.5, 2, len(i))), None))
    return out


@pytest.mark.parametrize("name,A,ex", case_graphs(), ids=lambda v: v if isinstance(v, str) else "")
def test_factor_bit_identical(orc, name, A, ex):
    need_gpu()
    rng = np.random.default_rng(sum(map(ord, name)) * 131 + A.n)
    perm = rng.permutation(A.n).astype(np.int32)
    if name == "bighub":
        perm[perm == 2500], perm[0] = perm[0], 2500  # the hub gets label 2500
    seed = 12345 + A.n
    ref = orc.factor(A, perm=perm, seed=seed)
    assert ref.status == 0
    if name in ("bighub", "chung_lu_16k"):
        assert ref.stats["max_gather"] > 2048
    f = gpu_factor(A, perm, seed)
    info = f.info()
    assert info["nnz_off"] == ref.nnz_off
    assert info["n_fill"] == ref.stats["n_fill"]
    assert info["max_deg"] == ref.stats["max_deg"]
    assert info["depth"] == ref.stats["depth"]
    compare_factor(f, ref)


def test_grid2d_workload_bit_identical(orc):
    need_gpu()
    W = inputs.grid2d_workload()
    ref = orc.factor(W.A, perm=W.perm, seed=W.seed)
    f = gpu_factor(W.A, W.perm, W.seed)
    compare_factor(f, ref)


@pytest.mark.parametrize("workers", [64, 128, 1024, 0])
def test_grid_size_invariance(orc, workers):
    """Different persistent grids interleave pivots differently; the factor
    must not change (a race detector by differential testing)."""
    need_gpu()
    rng = np.random.default_rng(5)
    i, j = inputs.grid3d_edges(14, 13, 12)
    n = 14 * 13 * 12
    A = lap(n, i, j, 10.0 ** rng.uniform(-2, 2, len(i)))
    perm = rng.permutation(n).astype(np.int32)
    ref = orc.factor(A, perm=perm, seed=99)
    f = gpu_factor(A, perm, 99, workers=workers)
    compare_factor(f, ref)


@pytest.mark.parametrize("tail", [-1.0, 0.3, 1.0])
def test_tail_kernel_split_is_exact(orc, tail):
    """The wide persistent kernel may hand the last pivots to the
    single-workgroup tail kernel at any point (none, 30%, all): the factor
    does not change."""
    need_gpu()
    rng = np.random.default_rng(15)
    i, j = inputs.grid3d_edges(16, 15, 14)
    n = 16 * 15 * 14
    A = lap(n, i, j, 10.0 ** rng.uniform(-2, 2, len(i)))
    perm = rng.permutation(n).astype(np.int32)
    ref = orc.factor(A, perm=perm, seed=21)
    f = gpu_factor(A, perm, 21, tail_fraction=tail)
    compare_factor(f, ref)


_PL = {}


def power_law_case(orc):
    """A Chung-Lu graph (16k vertices, beta 2.1) whose largest gathered
    neighbourhoods are far above a thousand entries, with its oracle factor."""
    if not _PL:
        rng = np.random.default_rng(78)
        i, j = inputs.chung_lu_edges(1 << 14, 16.0, 2.1, rng)
        m, i, j, _ = inputs.largest_component(1 << 14, i, j)
        A = lap(m, i, j, rng.uniform(0.5, 2.0, len(i)))
        perm = np.random.default_rng(79).permutation(m).astype(np.int32)
        ref = orc.factor(A, perm=perm, seed=4242)
        assert ref.status == 0 and ref.stats["max_gather"] > 2048
        _PL.update(A=A, perm=perm, ref=ref)
    return _PL["A"], _PL["perm"], _PL["ref"]


@pytest.mark.parametrize("workers,tail,pool", [(64, -1.0, 4.0), (0, 0.3, 4.0), (0, 1.0, 4.0),
                                               (256, -1.0, 0.02)])
def test_team_path_is_exact(orc, workers, tail, pool):
    """Pivots with more than 128 gathered entries are eliminated by the
    eight waves of a team workgroup, the others by single waves.  The
    factor does not change with the number of single-wave workers, with a
    hand-over to the tail kernel (which has no teams) part-way or from the
    start, or with pool exhaustion and retries inside team pivots."""
    need_gpu()
    A, perm, ref = power_law_case(orc)
    f = gpu_factor(A, perm, 4242, workers=workers, tail_fraction=tail, pool_factor=pool)
    if pool < 1.0:
        assert f.info()["retries"] >= 1
    info = f.info()
    assert info["max_gather"] == ref.stats["max_gather"]
    assert info["depth"] == ref.stats["depth"]
    compare_factor(f, ref)


def test_pool_exhaustion_retry_is_exact(orc):
    """A pool far too small forces EPOOL and internal retries with larger
    pools; the result is unchanged because storage does not enter the
    arithmetic."""
    need_gpu()
    rng = np.random.default_rng(6)
    n = 3000
    i, j = inputs.connected_random_edges(n, 6 * n, rng)
    A = lap(n, i, j, rng.uniform(0.1, 1, len(i)))
    perm = rng.permutation(n).astype(np.int32)
    ref = orc.factor(A, perm=perm, seed=3)
    f = gpu_factor(A, perm, 3, pool_factor=0.02, workers=64)
    assert f.info()["retries"] >= 1
    compare_factor(f, ref)


def test_errors_match_oracle(orc):
    need_gpu()
    from paper_2505_02977_amd import parac
    i, j = inputs.path_edges(6)
    good = lap(6, i, j, np.ones(5))
    bad_sign = lap(6, i, j, np.ones(5))
    bad_sign.val = bad_sign.val.copy()
    bad_sign.val[1] = 0.5
    asym = lap(6, i, j, np.ones(5))
    asym.val = asym.val.copy()
    asym.val[1] = -0.75
    asym.val[0] = 0.75
    for A, perm in ((bad_sign, None), (asym, None), (good, np.array([0, 1, 2, 3, 4, 4]))):
        st_ref = orc.factor(A, perm=perm).status
        with pytest.raises(parac.ParacError) as e:
            gpu_factor(A, perm, 1)
        assert e.value.status == st_ref
    # Laplacian mode forced on an SDDM matrix
    S = lap(6, i, j, np.ones(5), excess=np.array([0.5, 0, 0, 0, 0, 0]))
    with pytest.raises(parac.ParacError) as e:
        gpu_factor(S, None, 1, mode=parac.MODE_LAPLACIAN)
    assert e.value.status == parac.ENOTLAP


@pytest.mark.parametrize("case", ["grid3d", "chung_lu_16k"])
def test_nnz_sorted_order_bit_identical(orc, case):
    """Under the NNZ-sorted elimination order (ascending row count, random
    ties; the ordering recommended for GPUs in §V) the factor is again the
    oracle's, bit for bit."""
    need_gpu()
    if case == "grid3d":
        rng = np.random.default_rng(31)
        i, j = inputs.grid3d_edges(18, 17, 16)
        n = 18 * 17 * 16
        A = lap(n, i, j, 10.0 ** rng.uniform(-2, 2, len(i)))
    else:
        A, _, _ = power_law_case(orc)
    perm = inputs.perm_nnz_sorted(A, np.random.default_rng(32))
    deg = np.diff(A.rowptr)
    order = np.argsort(perm)            # vertices by label
    assert np.all(np.diff(deg[order]) >= 0)
    ref = orc.factor(A, perm=perm, seed=515)
    f = gpu_factor(A, perm, 515)
    assert f.info()["depth"] == ref.stats["depth"]
    compare_factor(f, ref)


@pytest.mark.parametrize("k", [2, 3])
def test_ack_factor_bit_identical(orc, k):
    """AC(k) (k sampling slots per merged neighbour, loops dropped): the
    device factor is the oracle's AC(k) factor bit for bit, on a grid, an
    SDDM system and a power-law graph (large gathered neighbourhoods); k = 1
    is the plain factor."""
    need_gpu()
    from paper_2505_02977_amd import parac
    rng = np.random.default_rng(500 + k)
    cases = []
    i, j = inputs.grid2d_edges(33, 31)
    cases.append((lap(33 * 31, i, j, rng.uniform(1, 2, len(i))), None))
    n = 2000
    i, j = inputs.connected_random_edges(n, 4 * n, rng)
    ex = np.zeros(n)
    ex[rng.choice(n, 200, replace=False)] = rng.random(200)
    cases.append((lap(n, i, j, rng.uniform(0.05, 3.0, len(i)), ex), None))
    i, j = inputs.chung_lu_edges(1 << 12, 16.0, 2.1, rng)
    m, i, j, _ = inputs.largest_component(1 << 12, i, j)
    cases.append((lap(m, i, j, rng.uniform(0.5, 2.0, len(i))), None))
    for A, _ in cases:
        perm = rng.permutation(A.n).astype(np.int32)
        ref = orc.factor(A, perm=perm, seed=321, samples=k)
        assert ref.status == 0
        f = gpu_factor(A, perm, 321, samples=k)
        compare_factor(f, ref)
        assert f.info()["n_fill"] == ref.stats["n_fill"]
    # k = 1 is the plain method
    A = cases[0][0]
    perm = rng.permutation(A.n).astype(np.int32)
    compare_factor(gpu_factor(A, perm, 5, samples=1), orc.factor(A, perm=perm, seed=5))


def test_fig1_trace_forced_on_device(orc):
    """The worked dependency trace of §III (Fig. 1) on the device: the test
    hook forces pivot 0's three slots to their last candidate, which gives
    the sampled tree of the figure; factor and levels equal the oracle's bit
    for bit.  A table of -1 leaves the draws alone, and an offset past its
    candidate range is EINVAL."""
    need_gpu()
    from paper_2505_02977_amd import parac
    from tests.test_oracle_pins import fig1_matrix
    g, A = fig1_matrix()
    tab = -np.ones((g["n"], 4), np.int32)
    tab[0, :3] = [2, 1, 0]
    ref = orc.factor(A, forced=tab)
    assert ref.status == 0
    f = gpu_factor(A, None, 0, forced=tab)
    compare_factor(f, ref)
    colptr, rowind, _, _, lev = f.export()
    assert list(rowind[colptr[0]:colptr[1]]) == [1, 3, 4, 5]
    assert all(list(rowind[colptr[k]:colptr[k + 1]]) == [5] for k in (1, 2, 3, 4))
    assert list(lev) == [0, 1, 0, 1, 1, 2]
    for seed in (5, 6):
        f = gpu_factor(A, None, seed, forced=-np.ones((g["n"], 4), np.int32))
        compare_factor(f, orc.factor(A, seed=seed))
    bad = tab.copy()
    bad[0, 2] = 1
    with pytest.raises(parac.ParacError) as e:
        gpu_factor(A, None, 0, forced=bad)
    assert e.value.status == parac.EINVAL


@pytest.mark.parametrize("case", ["hub", "bighub", "power_law"])
def test_forced_choices_every_path(orc, case):
    """Forced choices keyed by (pivot, slot) act the same way in the one-wave,
    large-neighbourhood and team pivots: a third of the pivots take offset 0
    (the next candidate in sampling order) in their first 64 slots, the rest
    draw; the factor equals the oracle's under the same table."""
    need_gpu()
    if case == "power_law":
        A, perm, _ = power_law_case(orc)
        seed = 4242
    else:
        A = dict((c[0], c[1]) for c in case_graphs())[case]
        perm = np.random.default_rng(5).permutation(A.n).astype(np.int32)
        seed = 99
    rng = np.random.default_rng(A.n)
    tab = -np.ones((A.n, 64), np.int32)
    tab[rng.random(A.n) < 1 / 3] = 0
    ref = orc.factor(A, perm=perm, seed=seed, forced=tab)
    assert ref.status == 0
    f = gpu_factor(A, perm, seed, forced=tab)
    compare_factor(f, ref)
    plain = orc.factor(A, perm=perm, seed=seed)
    assert not np.array_equal(plain.val.view(np.uint64), ref.val.view(np.uint64))
