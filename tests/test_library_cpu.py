"""Host-side checks of the C-ABI library (no GPU needed)."""

import math
import os
import re

import numpy as np
import pytest

import paper_2412_16613_amd as bwg
from paper_2412_16613_amd import _abi
from oracle.poisson import poisson_table as oracle_table
from oracle.quantize import quantize
from workloads import batch_networks, frank_network, paper_network

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    with open(os.path.join(ROOT, "include", "bwg.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(bwg_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = _abi.load()
    declared = _header_symbols()
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(_abi.SYMBOLS) == declared


def _qcmp(net):
    q_lib = bwg.Network(net).quantized()
    q_orc = quantize(net)
    for k in ("c", "f", "B", "b", "s", "Lambda", "max_total"):
        assert q_lib[k] == q_orc[k], (k, q_lib[k], q_orc[k])
    return q_lib


def test_quantisation_matches_oracle_on_workloads():
    for n in (12, 16, 32, 33, 100, 1000, 1024, 4096):
        q = _qcmp(frank_network(n))
        assert q["gpu_ok"]
    _qcmp(paper_network(32))
    _qcmp(paper_network(9, ghosts=False))
    for cfg in batch_networks()[:64]:
        _qcmp(cfg["net"])


def test_quantisation_matches_oracle_on_random_rates():
    rng = np.random.default_rng(5)
    for _ in range(40):
        n = int(rng.integers(2, 300))
        k = 10.0 ** rng.uniform(-4, 1, 3)
        net = frank_network(n, k0=float(k[0]), k1=float(k[1]), k2=float(k[2]))
        try:
            _qcmp(net)
        except bwg.BwgError as e:
            # beyond 32 threshold planes: the oracle's bound agrees
            assert e.code == _abi.BWG_ERANGE and quantize(net)["B"] > 32


@pytest.mark.parametrize("mu", [1e-6, 0.25, 1.0, 7.5, 63.9, 999.5, 1000.5, 12345.678,
                                51200.0, 409600.0])
def test_poisson_table_matches_oracle(mu):
    k_lo, T = bwg.poisson_table(mu)
    k_lo_o, T_o = oracle_table(mu)
    assert k_lo == k_lo_o and len(T) == len(T_o)
    diff = np.abs(np.array(T, dtype=object) - np.array(T_o, dtype=object))
    # binary128 against 256-bit arithmetic: equal floors except when 2^64 F is
    # within ~1e-10 of an integer
    assert max(diff) <= 1
    assert sum(1 for d in diff if d) <= 1


def test_poisson_tables_of_the_batch():
    for cfg in batch_networks()[:16]:
        q = quantize(cfg["net"])
        mu = q["Lambda"] * (cfg["t_end"] - 0.0)
        k_lo, T = bwg.poisson_table(mu)
        assert (k_lo, T) == oracle_table(mu)


def test_invalid_networks_are_rejected():
    bad_order = frank_network(10)
    bad_order["reactants"] = [(1, 1, 1)] + bad_order["reactants"][1:]
    bad_order["products"] = [(0, 0, 3)] + bad_order["products"][1:]
    with pytest.raises(bwg.BwgError) as e:
        bwg.Network(bad_order)
    assert e.value.code == _abi.BWG_EINVAL
    nonconserving = frank_network(10)
    nonconserving["products"] = [(2, 0, 0)] + nonconserving["products"][1:]
    with pytest.raises(bwg.BwgError) as e:
        bwg.Network(nonconserving)
    assert e.value.code == _abi.BWG_EINVAL
    neg = frank_network(10, k0=-1.0)
    with pytest.raises(bwg.BwgError) as e:
        bwg.Network(neg)
    assert e.value.code == _abi.BWG_EINVAL
    nan = frank_network(10, k0=float("nan"))
    with pytest.raises(bwg.BwgError):
        bwg.Network(nan)
    huge = frank_network(20000)
    with pytest.raises(bwg.BwgError) as e:
        bwg.Network(huge)
    assert e.value.code == _abi.BWG_ERANGE
    lat = frank_network(12, lx=4, ly=4, hop=0.1, site_planes=4)
    with pytest.raises(bwg.BwgError) as e:
        bwg.Network(lat)
    assert e.value.code == _abi.BWG_EUNSUPPORTED


def test_non_frank_order_is_plain_only():
    net = frank_network(16)
    order = [2, 0, 1, 3, 4]
    net["reactants"] = [net["reactants"][i] for i in order]
    net["products"] = [net["products"][i] for i in order]
    net["rates"] = [net["rates"][i] for i in order]
    n = bwg.Network(net)
    assert not n.quantized()["gpu_ok"]
    import ctypes
    nbytes = ctypes.c_uint64()
    o = _abi.Opts()
    o.engine = _abi.BWG_ENGINE_BITWISE
    rc = _abi.load().bwg_ensemble_state_bytes(n.handle, 1024, ctypes.byref(o), ctypes.byref(nbytes))
    assert rc == _abi.BWG_EUNSUPPORTED
    o.engine = _abi.BWG_ENGINE_PLAIN
    rc = _abi.load().bwg_ensemble_state_bytes(n.handle, 1024, ctypes.byref(o), ctypes.byref(nbytes))
    assert rc == 0 and nbytes.value > 1024 * 3 * 4


def test_state_bytes_scale_with_replicas():
    import ctypes
    n = bwg.Network(frank_network(1024))
    sizes = []
    for M in (1, 32, 33, 1 << 20):
        b = ctypes.c_uint64()
        _abi.check(_abi.load().bwg_ensemble_state_bytes(n.handle, M, None, ctypes.byref(b)))
        sizes.append(b.value)
    assert sizes[0] == sizes[1] == sizes[2]
    # 2^20 replicas: 3*11 planes of 2^15 words + 2*8 B per replica + tables
    assert sizes[3] >= (3 * 11 * 4 + 16 * 32) * (1 << 15)
    b = ctypes.c_uint64()
    assert _abi.load().bwg_ensemble_state_bytes(n.handle, 0, None, ctypes.byref(b)) == _abi.BWG_EINVAL
