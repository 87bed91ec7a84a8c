"""GPU tests of the device elimination orders (parac_order) and of the
factor under them.

Each order is integer arithmetic fixed by its definition (a seeded
SplitMix64 hash, row lengths, local-minimum rounds), so the device
permutation must equal, bit for bit, the one written out here in numpy from
the same definition; every MIS round is an independent set; and under the
NNZ and MIS orders the device factor is again the oracle's, bit for bit."""
import numpy as np
import pytest

from paper_2505_02977_amd import inputs
from tests.gpu_util import compare_factor, need_gpu

pytestmark = pytest.mark.gpu

M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix_out(state):
    """SplitMix64 output for states (uint64 array), wrapping arithmetic."""
    with np.errstate(over="ignore"):
        z = state + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def hash_and_pri(A, seed):
    n = A.n
    with np.errstate(over="ignore"):
        h = splitmix_out(np.uint64(seed) + np.arange(n, dtype=np.uint64))
    deg = np.minimum(np.diff(A.rowptr), (1 << 20) - 1).astype(np.uint64)
    pri = (deg << np.uint64(24)) | (h >> np.uint64(40))
    return h, pri


def perm_from_order(order):
    perm = np.empty(len(order), np.int32)
    perm[order] = np.arange(len(order), dtype=np.int32)
    return perm


def mis_rounds(A, pri):
    """Local-minimum rounds written out: in round r an unplaced vertex joins
    when its (pri, index) is below that of every neighbour unplaced at the
    start of the round."""
    n = A.n
    rows = np.repeat(np.arange(n), np.diff(A.rowptr))
    cols = A.col.astype(np.int64)
    off = rows != cols
    rows, cols = rows[off], cols[off]
    rnd = np.full(n, -1, np.int64)
    r = 0
    while (rnd < 0).any():
        open_ = rnd < 0
        e = open_[rows] & open_[cols]
        lt = (pri[cols[e]] < pri[rows[e]]) | ((pri[cols[e]] == pri[rows[e]]) & (cols[e] < rows[e]))
        beaten = np.zeros(n, bool)
        beaten[rows[e][lt]] = True
        join = open_ & ~beaten
        rnd[join] = r
        r += 1
    return rnd, r


def expected(A, kind, seed):
    from paper_2505_02977_amd import parac
    h, pri = hash_and_pri(A, seed)
    idx = np.arange(A.n)
    if kind == parac.ORDER_RANDOM:
        return perm_from_order(np.lexsort((idx, h))), 0
    if kind == parac.ORDER_NNZ:
        return perm_from_order(np.lexsort((idx, pri))), 0
    rnd, r = mis_rounds(A, pri)
    return perm_from_order(np.lexsort((idx, pri, rnd))), r


def cases():
    rng = np.random.default_rng(41)
    out = []
    i, j = inputs.grid3d_edges(20, 19, 18)
    out.append(("grid3d", inputs.laplacian_from_edges(20 * 19 * 18, i, j, np.ones(len(i)))))
    i, j = inputs.chung_lu_edges(1 << 14, 16.0, 2.1, rng)
    n, i, j, _ = inputs.largest_component(1 << 14, i, j)
    out.append(("chunglu", inputs.laplacian_from_edges(n, i, j, rng.uniform(0.5, 2, len(i)))))
    d = 5000  # a star: one hub, every leaf in the first MIS round
    out.append(("star", inputs.laplacian_from_edges(d + 1, np.zeros(d, int), np.arange(1, d + 1),
                                                    np.ones(d))))
    # two components and an isolated vertex
    i = np.array([0, 1, 3, 4, 5])
    j = np.array([1, 2, 4, 5, 6])
    out.append(("pieces", inputs.laplacian_from_edges(8, i, j, np.ones(5))))
    return out


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_order_matches_definition(kind):
    need_gpu()
    from paper_2505_02977_amd import parac
    for name, A in cases():
        for seed in (0, 12345678901234567):
            want, wr = expected(A, kind, seed)
            got, gr = parac.parac_order(parac.DeviceCSR(A), kind, seed)
            assert np.array_equal(got, want), (name, kind, seed)
            assert gr == wr, (name, gr, wr)
            # host arrays in, host permutation out: the same
            got_h, _ = parac.parac_order(A, kind, seed)
            assert np.array_equal(got_h, want), (name, kind, seed)
            if kind == parac.ORDER_MIS:
                # every round is an independent set
                h, pri = hash_and_pri(A, seed)
                rnd, _ = mis_rounds(A, pri)
                rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
                off = rows != A.col
                assert not np.any(rnd[rows[off]] == rnd[A.col[off]]), name
            if kind == parac.ORDER_NNZ:
                deg = np.diff(A.rowptr)
                assert np.all(np.diff(deg[np.argsort(got)]) >= 0)


@pytest.mark.parametrize("kind", [1, 2])
def test_factor_bit_identical_under_device_order(orc, kind):
    need_gpu()
    from paper_2505_02977_amd import parac
    for name, A in cases()[:2]:
        dA = parac.DeviceCSR(A)
        perm, _ = parac.parac_order(dA, kind, 99)
        f = parac.parac_factor(dA, perm=perm, seed=7)
        ref = orc.factor(A, perm=perm, seed=7)
        assert f.info()["depth"] == ref.stats["depth"], name
        compare_factor(f, ref)


def test_order_rejects_bad_kind():
    need_gpu()
    from paper_2505_02977_amd import parac
    A = cases()[3][1]
    with pytest.raises(parac.ParacError) as e:
        parac.parac_order(A, 7, 0)
    assert e.value.status == parac.EINVAL
