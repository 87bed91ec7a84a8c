"""Helpers shared by the GPU tests."""
import numpy as np
import pytest


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def same_bits(a, b):
    a = np.ascontiguousarray(a)
    b = np.ascontiguousarray(b)
    if a.shape != b.shape:
        return False
    if a.dtype == np.float64:
        return np.array_equal(a.view(np.uint64), b.view(np.uint64))
    return np.array_equal(a, b)


def compare_factor(gpu_fac, orc_fac):
    colptr, rowind, val, D, lev = gpu_fac.export()
    assert same_bits(colptr, orc_fac.colptr), "colptr"
    assert same_bits(rowind, orc_fac.rowind), "rowind"
    assert same_bits(val, orc_fac.val), "F values"
    assert same_bits(D, orc_fac.D), "D"
    assert same_bits(lev, orc_fac.level), "levels"
