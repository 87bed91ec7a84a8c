"""CPU checks of the apply rounding bound used by the GPU parity tests: it
holds between the oracle's left-fold apply and a dense triangular solve (a
different summation order), and it is tight enough to reject a single
perturbed factor value or a dropped product."""
import numpy as np
import pytest

from paper_2505_02977_amd import inputs
from tests.bounds import apply_bound, within_apply_bound


def lap(n, i, j, w, excess=None):
    return inputs.laplacian_from_edges(n, i, j, w, excess)


def cases():
    rng = np.random.default_rng(5)
    out = []
    n = 400
    i, j = inputs.connected_random_edges(n, 4 * n, rng)
    out.append(("rand", lap(n, i, j, rng.uniform(0.05, 3.0, len(i))), False))
    ex = np.zeros(n)
    ex[rng.choice(n, 40, replace=False)] = rng.random(40)
    out.append(("sddm", lap(n, i, j, rng.uniform(0.05, 3.0, len(i)), ex), True))
    d = 300
    out.append(("star", lap(d + 1, np.zeros(d, int), np.arange(1, d + 1), rng.uniform(0.5, 2, d)), False))
    return out


def dense_apply(f, b):
    n = f.n
    F = f.dense_F()[:n, :n]
    D = f.D[:n]
    Dp = np.where(D > 0, 1.0 / np.where(D > 0, D, 1.0), 0.0)
    perm = f.perm
    pb = np.empty(n)
    pb[perm] = b
    y = np.linalg.solve(F, pb)
    x = np.linalg.solve(F.T, Dp * y)
    return x[perm]


@pytest.mark.parametrize("name,A,sddm", cases(), ids=lambda v: v if isinstance(v, str) else "")
def test_bound_holds_across_orders(orc, name, A, sddm):
    rng = np.random.default_rng(len(name))
    perm = rng.permutation(A.n).astype(np.int32)
    f = orc.factor(A, perm=perm, seed=11)
    b = rng.standard_normal(A.n)
    if not sddm:
        b -= b.mean()
    z = orc.apply(f, b)
    zd = dense_apply(f, b)
    ok, ratio = within_apply_bound(z, zd, f, b, 0)
    assert ok, ratio
    # not vacuous: far below the solution's own size
    assert np.max(apply_bound(f, b, 0)) <= 1e-10 * np.max(np.abs(z))
    assert np.max(apply_bound(f, b, 1)) <= 1e-2 * np.max(np.abs(z))


@pytest.mark.parametrize("name,A,sddm", cases(), ids=lambda v: v if isinstance(v, str) else "")
def test_bound_rejects_a_changed_factor(orc, name, A, sddm):
    """A planted mistake on the CPU: one factor value changed in its 30th bit
    (relative 1e-9), applied by the dense solve, must fall outside the
    FP64 bound."""
    rng = np.random.default_rng(len(name) + 100)
    perm = rng.permutation(A.n).astype(np.int32)
    f = orc.factor(A, perm=perm, seed=11)
    b = rng.standard_normal(A.n)
    if not sddm:
        b -= b.mean()
    z = orc.apply(f, b)
    # the largest entry off the last row (the zero pivot's row feeds nothing:
    # D^+ is zero there)
    cand = np.abs(f.val) * (f.rowind < f.n - 1)
    k = int(np.argmax(cand))
    f.val[k] *= 1.0 + 2.0 ** -30
    zd = dense_apply(f, b)
    ok, ratio = within_apply_bound(z, zd, f, b, 0)
    assert not ok, ratio
