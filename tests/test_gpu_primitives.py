"""Exhaustive device tests of the bit-sliced primitives against integer
arithmetic: masked +-1 and -1/+2 ripple updates, the sign-extended add, the
schoolbook plane product and the shifted subtraction with and without its
difference, each over every operand combination of a small width (the
device code of bitops.h / wm_device.h, built into a self-test library)."""

import ctypes
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2412_16613_amd", "libbwg_selftest.so")


@pytest.fixture(scope="module")
def run():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lib = ctypes.CDLL(LIB)
    lib.bwg_selftest_prim.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_void_p,
                                      ctypes.c_void_p]

    def go(op, n):
        print("primitive", op, n, flush=True)
        out = torch.zeros(n, dtype=torch.int32, device="cuda")
        rc = lib.bwg_selftest_prim(op, n, ctypes.c_void_p(out.data_ptr()),
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert rc == 0
        torch.cuda.synchronize()
        return out.cpu().numpy().astype(np.int64) & 0xFFFFFFFF

    return go


def test_add_pm1(run):
    k = np.arange(192)
    x, d = k % 64, k // 64
    step = np.where(d == 0, 1, np.where(d == 1, -1, 0))
    np.testing.assert_array_equal(run(0, 192), (x + step) % 64)


def test_add_m1_p2(run):
    k = np.arange(192)
    x, d = k % 64, k // 64
    step = np.where(d == 0, -1, np.where(d == 1, 2, 0))
    np.testing.assert_array_equal(run(1, 192), (x + step) % 64)


def test_add_sign_extended(run):
    n = 1024 * 64 * 2
    k = np.arange(n)
    acc, d6, cin = k % 1024, (k // 1024) % 64, k // 65536
    d = np.where(d6 >= 32, d6 - 64, d6)
    np.testing.assert_array_equal(run(2, n), (acc + d + cin) % 1024)


def test_plane_product(run):
    k = np.arange(4096)
    x, y = k % 64, k // 64
    np.testing.assert_array_equal(run(3, 4096), (x * y) % 1024)


def test_shifted_subtraction_with_difference(run):
    n = 4096 * 64
    k = np.arange(n)
    d, p = k % 4096, k // 4096
    diff = d - (p << 2)
    expect = (diff % 4096) | ((diff < 0).astype(np.int64) << 12)
    np.testing.assert_array_equal(run(4, n), expect)


def test_shifted_subtraction_borrow_of_a_plane_range(run):
    # planes [3, 10) only: the borrow of (d >> 3) mod 2^7 - p, p < 2^6
    n = 1024 * 64
    k = np.arange(n)
    d, p = k % 1024, k // 1024
    expect = (((d >> 3) % 128) < p).astype(np.int64)
    np.testing.assert_array_equal(run(5, n), expect)
