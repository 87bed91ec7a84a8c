"""The multithreaded CPU factorisation (parac_factor_host, the paper's CPU
design) gives the oracle's factor bit for bit, whatever the number of
threads, and reports the oracle's errors.  Runs on the CPU only."""
import numpy as np
import pytest

from paper_2505_02977_amd import inputs
from tests.gpu_util import same_bits


def lap(n, i, j, w, excess=None):
    return inputs.laplacian_from_edges(n, i, j, w, excess)


def host(A, perm, seed, threads, **kw):
    from paper_2505_02977_amd import parac
    return parac.parac_factor_host(A, perm=perm, seed=seed, threads=threads, **kw)


def same_as_oracle(h, ref):
    assert h["nnz_off"] == ref.nnz_off
    assert h["n_fill"] == ref.stats["n_fill"]
    assert h["depth"] == ref.stats["depth"]
    assert same_bits(h["colptr"], ref.colptr)
    assert same_bits(h["rowind"], ref.rowind)
    assert same_bits(h["val"], ref.val)
    assert same_bits(h["D"], ref.D)
    assert same_bits(h["level"], ref.level)


def cases():
    rng = np.random.default_rng(90)
    out = []
    n = 2000
    i, j = inputs.connected_random_edges(n, 5 * n, rng)
    out.append(("rand", lap(n, i, j, rng.uniform(0.05, 3.0, len(i)))))
    i, j = inputs.grid3d_edges(14, 13, 12)
    out.append(("grid3d", lap(14 * 13 * 12, i, j, 10.0 ** rng.uniform(-2, 2, len(i)))))
    i, j = inputs.chung_lu_edges(1 << 13, 16.0, 2.1, rng)
    m, i, j, _ = inputs.largest_component(1 << 13, i, j)
    out.append(("chung_lu", lap(m, i, j, rng.uniform(0.5, 2.0, len(i)))))
    n = 500
    i, j = inputs.connected_random_edges(n, 3 * n, rng)
    ex = np.zeros(n)
    ex[rng.choice(n, 50, replace=False)] = rng.random(50)
    out.append(("sddm", lap(n, i, j, rng.uniform(0.1, 2.0, len(i)), ex)))
    d = 3000  # a hub: one neighbourhood of many tiles
    out.append(("star", lap(d + 1, np.zeros(d, int), np.arange(1, d + 1), rng.uniform(0.1, 1, d))))
    i1, j1 = inputs.connected_random_edges(100, 200, rng)
    i2, j2 = inputs.connected_random_edges(80, 150, rng)
    ii, jj = np.concatenate([i1, i2 + 100]), np.concatenate([j1, j2 + 100])
    out.append(("two_comp", lap(180, ii, jj, rng.uniform(0.5, 2, len(ii)))))
    out.append(("single", lap(1, np.zeros(0, int), np.zeros(0, int), np.zeros(0))))
    return out


@pytest.mark.parametrize("name,A", cases(), ids=lambda v: v if isinstance(v, str) else "")
@pytest.mark.parametrize("threads", [1, 3, 8])
def test_host_factor_bit_identical(orc, name, A, threads):
    rng = np.random.default_rng(len(name) * 7 + A.n)
    perm = rng.permutation(A.n).astype(np.int32)
    seed = 1000 + A.n
    ref = orc.factor(A, perm=perm, seed=seed)
    assert ref.status == 0
    h = host(A, perm, seed, threads)
    assert h["threads"] == threads
    same_as_oracle(h, ref)


def test_host_pool_retry_is_exact(orc):
    rng = np.random.default_rng(91)
    n = 1500
    i, j = inputs.connected_random_edges(n, 6 * n, rng)
    A = lap(n, i, j, rng.uniform(0.1, 1, len(i)))
    perm = rng.permutation(n).astype(np.int32)
    ref = orc.factor(A, perm=perm, seed=5)
    same_as_oracle(host(A, perm, 5, 4, pool_factor=0.01), ref)


def test_host_errors_match_oracle(orc):
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
        assert st_ref != 0
        with pytest.raises(parac.ParacError) as e:
            host(A, perm, 1, 2)
        assert e.value.status == st_ref
