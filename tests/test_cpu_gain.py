"""The host-CPU engines of the paper's gain experiment (Sec. 5): the
bit-parallel method on 64-bit words and the direct method run once per copy,
both with one threshold shared by every copy per iteration, against the
oracle's shared-threshold chain for the same copies, draws and iterations."""

import ctypes
import os

import numpy as np
import pytest

from oracle import ssa
from workloads import paper_network

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2412_16613_amd", "libbwg_cpugain.so")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2412_16613_amd import build
        build._build_calib()
    L = ctypes.CDLL(LIB)
    P = ctypes.POINTER(ctypes.c_int32)
    for f in (L.bwg_cpu_gain_bitwise, L.bwg_cpu_gain_serial):
        f.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, P,
                      ctypes.c_uint64, P]
        f.restype = ctypes.c_int
    return L


@pytest.mark.parametrize("n_tot,M,T", [(32, 64, 3000), (100, 100, 2000), (8, 200, 5000),
                                       (1024, 64, 1500)])
def test_cpu_engines_match_oracle(oracle_lib, lib, n_tot, M, T):
    net = paper_network(n_tot)
    init = ssa.init_multinomial(3, 9, 0, M, n_tot)
    o = ssa.OracleEnsemble(net, M, seed=3, net_id=9, draw=ssa.DRAW_SHARED)
    o.init(("multinomial",))
    o.step(T)
    for f in (lib.bwg_cpu_gain_bitwise, lib.bwg_cpu_gain_serial):
        out = np.zeros((M, 3), dtype=np.int32)
        rc = f(n_tot, M, 3, 9, np.ascontiguousarray(init).ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
               T, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        assert rc == 0
        np.testing.assert_array_equal(out, o.counts)
