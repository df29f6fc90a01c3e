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
from workloads import batch_networks, frank_network, paper_network, random_network

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
    for k in ("c", "f", "B", "b", "s", "Lambda", "max_total", "z_shared"):
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


def test_total_weight_range_matches_enumeration_on_random_networks():
    # the library finds the largest and smallest total weight over the simplex
    # from the quadratic in the second count (ends and the integers next to
    # the vertex); the oracle enumerates every state.  Random 3-species tables
    # with dimerisations (concave and convex quadratics), exact-integer and
    # real rates, down to one and two molecules
    rng = np.random.default_rng(11)
    for k in range(60):
        n = int(rng.choice([1, 2, 3, 4, 7])) if k < 15 else int(rng.integers(5, 260))
        net = random_network(1000 + k, n, int(rng.integers(1, 9)), exact_integer=bool(k % 2))
        try:
            _qcmp(net)
        except bwg.BwgError as e:
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


def test_non_frank_networks_take_the_general_kernel():
    """A network outside the Frank family (here its reactions reordered) runs
    on the general bit-sliced kernel and the plain engine, not on the lanes
    engine, shared thresholds or in batches."""
    import ctypes
    net = frank_network(16)
    order = [2, 0, 1, 3, 4]
    net["reactants"] = [net["reactants"][i] for i in order]
    net["products"] = [net["products"][i] for i in order]
    net["rates"] = [net["rates"][i] for i in order]
    n = bwg.Network(net)
    assert n.quantized()["gpu_ok"]
    L = _abi.load()

    def rc(**kw):
        o = _abi.Opts()
        for k, v in kw.items():
            setattr(o, k, v)
        nbytes = ctypes.c_uint64()
        r = L.bwg_ensemble_state_bytes(n.handle, 1024, ctypes.byref(o), ctypes.byref(nbytes))
        return r, nbytes.value

    assert rc(engine=_abi.BWG_ENGINE_BITWISE)[0] == _abi.BWG_OK
    assert rc(engine=_abi.BWG_ENGINE_LANES)[0] == _abi.BWG_EUNSUPPORTED
    assert rc(engine=_abi.BWG_ENGINE_BITWISE,
              flags=_abi.BWG_OPT_SHARED_THRESHOLD)[0] == _abi.BWG_EUNSUPPORTED
    r, nb = rc(engine=_abi.BWG_ENGINE_PLAIN)
    assert r == 0 and nb > 1024 * 3 * 4
    # a Frank-family network may ask for the general kernel
    f = bwg.Network(frank_network(16))
    o = _abi.Opts()
    o.flags = _abi.BWG_OPT_GENERIC_KERNEL
    nbytes = ctypes.c_uint64()
    assert L.bwg_ensemble_state_bytes(f.handle, 64, ctypes.byref(o), ctypes.byref(nbytes)) == 0
    o.engine = _abi.BWG_ENGINE_LANES
    assert (L.bwg_ensemble_state_bytes(f.handle, 64, ctypes.byref(o), ctypes.byref(nbytes))
            == _abi.BWG_EUNSUPPORTED)


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


def test_prepare_refuses_a_null_ensemble():
    """The entry point that builds a network's run-time compiled Frank kernel
    ahead of its first launch validates its argument on the host."""
    assert _abi.load().bwg_ensemble_prepare(None) == _abi.BWG_EINVAL


def test_options_are_checked_before_any_device_work():
    """Block sizes beyond the kernels' launch bounds and shared thresholds
    where no kernel implements them are refused by the size query."""
    import ctypes
    L = _abi.load()

    def rc(net, **kw):
        o = _abi.Opts()
        for k, v in kw.items():
            setattr(o, k, v)
        b = ctypes.c_uint64()
        return L.bwg_ensemble_state_bytes(net.handle, 1000, ctypes.byref(o), ctypes.byref(b))

    n = bwg.Network(paper_network(32))
    for block in (0, 64, 128, 192, 256):
        assert rc(n, block=block) == _abi.BWG_OK
    for block in (-64, 32, 100, 320, 512, 1024):
        assert rc(n, block=block) == _abi.BWG_EINVAL
    shared = _abi.BWG_OPT_SHARED_THRESHOLD
    assert rc(n, flags=shared) == _abi.BWG_OK
    assert rc(n, flags=shared, engine=_abi.BWG_ENGINE_LANES) == _abi.BWG_OK
    assert rc(n, flags=shared, engine=_abi.BWG_ENGINE_PLAIN) == _abi.BWG_EUNSUPPORTED
    lat = bwg.Network(frank_network(12, lx=4, ly=4, hop=0.1, site_planes=4))
    assert rc(lat, flags=shared) == _abi.BWG_EUNSUPPORTED


def test_weights_beyond_32_planes():
    """Rates quantised at more bits of precision: up to 48 threshold planes,
    the same quantisation as the oracle's; the bit-sliced engine takes them on
    the kernels compiled for the network only, the other engines, the
    precompiled kernels, explicit block sizes, other word widths and shared
    thresholds refuse them (before any device work); beyond 48 planes the
    network is refused."""
    import ctypes
    L = _abi.load()

    def rc(net, **kw):
        o = _abi.Opts()
        for k, v in kw.items():
            setattr(o, k, v)
        b = ctypes.c_uint64()
        return L.bwg_ensemble_state_bytes(net.handle, 1000, ctypes.byref(o), ctypes.byref(b))

    for n_tot, bits, B in ((10, 26, 35), (1024, 20, 36), (1024, 26, 42)):
        net = frank_network(n_tot, k0=0.0137 if n_tot == 10 else 0.013)
        q_orc = quantize(net, precision_bits=bits)
        n = bwg.Network(net, precision_bits=bits)
        q_lib = n.quantized()
        assert q_orc["B"] == q_lib["B"] == B
        for k in ("c", "f", "b", "s", "Lambda", "max_total"):
            assert q_lib[k] == q_orc[k], k
        assert q_lib["z_shared"] is None and q_lib["gpu_ok"]
        assert rc(n) == _abi.BWG_OK
        assert rc(n, engine=_abi.BWG_ENGINE_LANES) == _abi.BWG_EUNSUPPORTED
        assert rc(n, engine=_abi.BWG_ENGINE_PLAIN) == _abi.BWG_EUNSUPPORTED
        assert rc(n, flags=_abi.BWG_OPT_NO_JIT) == _abi.BWG_EUNSUPPORTED
        assert rc(n, block=64) == _abi.BWG_EUNSUPPORTED
        assert rc(n, word_bits=16) == _abi.BWG_EUNSUPPORTED
        assert rc(n, flags=_abi.BWG_OPT_SHARED_THRESHOLD) == _abi.BWG_ERANGE
    gen = random_network(0, 12, 5)
    n = bwg.Network(gen, precision_bits=20)
    assert n.quantized()["B"] == quantize(gen, precision_bits=20)["B"] == 33
    assert rc(n) == _abi.BWG_OK
    assert rc(n, flags=_abi.BWG_OPT_NO_JIT) == _abi.BWG_EUNSUPPORTED
    big = frank_network(4096, k0=0.013)
    assert bwg.Network(big, precision_bits=30).quantized()["B"] == 48   # the largest
    with pytest.raises(bwg.BwgError) as e:
        bwg.Network(big, precision_bits=31)
    assert e.value.code == _abi.BWG_ERANGE and quantize(big, precision_bits=31)["B"] == 49


# ---- lattices ----------------------------------------------------------------

def _lat_cmp(net):
    from oracle.lattice import quantize_lattice
    n = bwg.Network(net)
    li, q = n.lattice(), n.quantized()
    o = quantize_lattice(net)
    assert q["c"] == o["c"] and q["f"] == o["f"] and q["s"] == o["s"]
    assert li["c_hop"] == o["c_hop"] and li["B_r"] == o["B_r"] and li["T"] == o["T"]
    assert li["C"] == o["C"] and li["max_site"] == o["max_site"]
    assert li["Lambda"] == o["Lambda"] == q["Lambda"]
    return n


def test_lattice_quantisation_matches_oracle():
    n = _lat_cmp(frank_network(12, lx=64, ly=64, hop=0.1, site_planes=4))
    assert n.quantized()["gpu_ok"]
    assert n.lattice()["C"] == 4096 * ((1 << 18) + 64 * 2458)
    for side in (1, 2, 5, 16, 33):
        _lat_cmp(frank_network(12, lx=side, ly=max(1, side // 2), hop=0.1, site_planes=4))
    _lat_cmp(frank_network(1, k0=0.0, k1=0.0, k2=0.0, lx=5, ly=3, hop=0.1, site_planes=4))
    _lat_cmp(frank_network(4, k0=0.25, k1=1.0, k2=1.0, lx=2, ly=1, hop=0.5, site_planes=2))
    rng = np.random.default_rng(8)
    for _ in range(20):
        k = 10.0 ** rng.uniform(-3, 0, 4)
        _lat_cmp(frank_network(12, k0=float(k[0]), k1=float(k[1]), k2=float(k[2]), lx=8, ly=8,
                               hop=float(k[3]), site_planes=4))


def test_invalid_lattices_are_rejected():
    def code(net):
        with pytest.raises(bwg.BwgError) as ei:
            bwg.Network(net)
        return ei.value.code
    assert code(frank_network(12, lx=65, ly=64, hop=0.1, site_planes=4)) == _abi.BWG_ERANGE
    assert code(frank_network(12, lx=8, ly=8, hop=0.1, site_planes=0)) == _abi.BWG_ERANGE
    bad = frank_network(12, lx=8, ly=8, hop=0.1, site_planes=4)
    bad["hop_rates"] = [0.1, 0.2, 0.1]
    assert code(bad) == _abi.BWG_EUNSUPPORTED
    swapped = frank_network(12, lx=8, ly=8, hop=0.1, site_planes=4)
    swapped["reactants"] = swapped["reactants"][::-1]
    swapped["products"] = swapped["products"][::-1]
    assert code(swapped) == _abi.BWG_EUNSUPPORTED
    neg = frank_network(12, lx=8, ly=8, hop=-0.1, site_planes=4)
    assert code(neg) == _abi.BWG_EINVAL
    # no event kernel for 3-plane sites: the network exists, ensembles do not
    n3 = bwg.Network(frank_network(6, lx=4, ly=4, hop=0.1, site_planes=3))
    assert not n3.quantized()["gpu_ok"]
    nb = ctypes_u64()
    rc = _abi.load().bwg_ensemble_state_bytes(n3.handle, 64, None, nb)
    assert rc == _abi.BWG_EUNSUPPORTED
    # a well-mixed network has no lattice form
    with pytest.raises(bwg.BwgError):
        bwg.Network(frank_network(12)).lattice()


def ctypes_u64():
    import ctypes
    return ctypes.byref(ctypes.c_uint64())


def test_lattice_state_bytes():
    import ctypes
    n = bwg.Network(frank_network(12, lx=64, ly=64, hop=0.1, site_planes=4))
    b = ctypes.c_uint64()
    _abi.check(_abi.load().bwg_ensemble_state_bytes(n.handle, 1 << 16, None, ctypes.byref(b)))
    planes = 2048 * 4096 * 12 * 4
    # the schedule of include/bwg.h's geometry for 32 groups of 2048 replicas
    sched = 32 * _abi.BWG_LAT_PASS_CHUNKS * (3 * _abi.BWG_LAT_CHUNK_EVENTS + 64) * 4
    assert planes + sched <= b.value < planes + sched + (8 << 20)


def test_quantisation_of_wide_and_open_networks_matches_oracle():
    # other species counts and open networks: the library's bound and
    # weights equal the oracle's rule (sum of each reaction's largest factor)
    from workloads import open_network, random_wide_network
    nets = [open_network(n, c) for n, c in (("death", 20), ("birth", 1000),
                                            ("lotka_volterra", 12))]
    nets += [random_wide_network(s, S, n, R, o) for s, S, n, R, o in
             ((0, 4, 8, 5, False), (1, 2, 10, 6, True), (2, 8, 6, 10, False),
              (3, 5, 20, 8, True), (6, 6, 12, 16, True), (7, 2, 200, 7, False))]
    for net in nets:
        q_lib = bwg.Network(net).quantized()
        q_orc = quantize(net)
        assert q_lib["c"] == q_orc["c"] and q_lib["B"] == q_orc["B"]
        assert q_lib["max_total"] == q_orc["max_total"] and q_lib["b"] == q_orc["b"]
        assert q_lib["Lambda"] == q_orc["Lambda"] and q_lib["gpu_ok"]


def test_wide_network_limits():
    from workloads import open_network
    big_jump = open_network("birth", 50)
    big_jump["products"] = [(4,)]                 # A -> 4A: a change of 3
    assert not bwg.Network(big_jump).quantized()["gpu_ok"]
    lat = open_network("lotka_volterra", 12)
    lat.update(lx=4, ly=4, site_planes=4)
    with pytest.raises(bwg.BwgError) as e:
        bwg.Network(lat)
    assert e.value.code == _abi.BWG_EUNSUPPORTED


def test_run_time_kernels_compile_on_the_host():
    """bwg_net_compile builds every kernel a bit-sliced ensemble of the network
    would compile at run time, with no device (there is none here): the
    Frank-family kernel for run-time weights and beyond 32 threshold planes,
    the general kernel for other networks, closed or open, of 3 or more
    species; nothing for networks on precompiled kernels and for lattices.
    A second call reuses the code."""
    from workloads import open_network, random_wide_network
    cases = [
        (frank_network(1024), 0, set()),                 # exact-width precompiled kernel
        (paper_network(32), 0, set()),
        (frank_network(200, k0=0.03), 0, {"frank"}),
        (frank_network(10, k0=0.0137), 26, {"frank"}),   # B = 35
        (random_network(3, 100, 6), 0, {"general"}),
        (random_network(0, 12, 5), 20, {"general"}),     # B = 33
        (random_wide_network(1, 5, 60, 7), 0, {"general"}),
        (open_network("lotka_volterra", 200), 0, {"general"}),
        (frank_network(12, lx=4, ly=4, hop=0.1, site_planes=4), 0, set()),
    ]
    for net, bits, want in cases:
        n = bwg.Network(net, precision_bits=bits)
        assert n.compile() == want
        assert n.compile() == want


def test_bytes_needed_matches_the_library():
    """Ensemble.bytes_needed (the server's admission check) allocates nothing
    and reports bwg_ensemble_state_bytes for the same options."""
    import ctypes
    L = _abi.load()
    n = bwg.Network(frank_network(1024))
    for engine, M in (("bitwise", 1 << 20), ("lanes", 1000), ("plain", 77)):
        o = _abi.Opts()
        o.engine = bwg.ENGINES[engine]
        b = ctypes.c_uint64()
        assert L.bwg_ensemble_state_bytes(n.handle, M, ctypes.byref(o), ctypes.byref(b)) == 0
        assert bwg.Ensemble.bytes_needed(n, M, engine=engine) == b.value
    with pytest.raises(bwg.BwgError):
        bwg.Ensemble.bytes_needed(n, 0)


def test_header_is_plain_c(tmp_path):
    """include/bwg.h compiles as strict C99 and links against libbwg.so from a
    C program: the boundary carries no C++ or torch types."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "use_bwg.c"
    src.write_text(
        '#include "bwg.h"\n'
        "int main(void) {\n"
        "    int64_t k_lo; uint64_t len, t[64];\n"
        "    return bwg_poisson_table(2.0, &k_lo, t, 64, &len) == BWG_OK ? 0 : 1;\n"
        "}\n")
    exe = tmp_path / "use_bwg"
    lib_dir = os.path.join(ROOT, "paper_2412_16613_amd")
    r = subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                        "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe),
                        "-L" + lib_dir, "-lbwg", "-Wl,-rpath," + lib_dir],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    assert subprocess.run([str(exe)]).returncode == 0


def test_quantisation_matches_oracle_on_random_networks():
    """The library's integer form equals the oracle's on 300 seeded random
    networks of every kind (Frank family at 1..8000 molecules, random
    3-species tables, 1..8 species, open networks, the paper's network) at
    the default and at raised precision; where the library refuses one, it
    is for a documented range limit (weights beyond 32 bits, a total weight
    beyond 48 threshold planes)."""
    import random
    from workloads import open_network, random_wide_network
    rng = random.Random(7)
    checked = 0
    for _ in range(300):
        kind = rng.choice(["frank", "random", "wide", "open", "paper"])
        bits = rng.choice([0, 0, 0, 8, 12, 20, 26, 30])
        if kind == "frank":
            net = frank_network(rng.choice([1, 2, 3, 10, 64, 100, 1024, 4096, 8000]),
                                k0=10 ** rng.uniform(-4, 0))
        elif kind == "random":
            net = random_network(rng.randrange(10 ** 6), rng.choice([2, 5, 12, 50, 300]),
                                 rng.choice([1, 3, 5, 8, 12]))
        elif kind == "wide":
            net = random_wide_network(rng.randrange(10 ** 6), rng.choice([1, 2, 4, 8]),
                                      rng.choice([3, 10, 40]), rng.choice([1, 4, 9]),
                                      open_net=rng.random() < 0.5)
        elif kind == "open":
            net = open_network(rng.choice(["death", "birth", "lotka_volterra"]),
                               rng.choice([1, 10, 200, 5000]))
        else:
            net = paper_network(rng.choice([1, 2, 32, 1000, 1448, 3000]))
        orc = quantize(net, precision_bits=bits or 7)
        try:
            lib = bwg.Network(net, precision_bits=bits).quantized()
        except bwg.BwgError as e:
            assert e.code == _abi.BWG_ERANGE
            assert max(orc["c"]) >= 1 << 32 or orc["B"] > 48, (kind, bits, str(e))
            continue
        for k in ("c", "f", "B", "b", "s", "Lambda", "max_total"):
            assert lib[k] == orc[k], (kind, bits, k)
        checked += 1
    assert checked > 200


def test_host_calls_from_several_threads():
    """Network creation, quantisation, Poisson tables, state sizes and the
    run-time compile of one shared network, from eight threads at once (the
    calls release the interpreter lock): every call succeeds and the shared
    network's compile happens once."""
    import random
    import threading
    shared = bwg.Network(frank_network(200, k0=0.03))
    errors = []

    def work(seed):
        rng = random.Random(seed)
        try:
            for _ in range(40):
                k = rng.random()
                if k < 0.4:
                    bwg.Network(random_network(rng.randrange(10 ** 6), rng.choice([5, 50, 300]),
                                               rng.choice([3, 5, 8]))).quantized()
                elif k < 0.7:
                    bwg.poisson_table(rng.uniform(1, 5000))
                else:
                    assert shared.compile() == {"frank"}
                    bwg.Ensemble.bytes_needed(shared, rng.choice([1, 1000, 1 << 20]),
                                              engine=rng.choice(["bitwise", "lanes", "plain"]))
        except Exception as e:  # reported below
            errors.append(repr(e))

    threads = [threading.Thread(target=work, args=(s,)) for s in range(8)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert errors == []
