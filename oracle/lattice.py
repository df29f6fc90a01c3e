"""Compartment (lattice) oracle, Python side — TEST INFRASTRUCTURE ONLY.

Integer form of a lattice network (reading of Sec. 1/Sec. 6 of the paper,
which motivate but do not define the non-well-mixed case): the well-mixed
weight rule of quantize.py applied to the site reactions and to the hop rate
d (per molecule, per direction); a site holds at most T = 2^P - 1 molecules;
B_R is the smallest B with 2^B at or above the largest site weight sum over
every site state with at most T molecules; components: a reaction component
per site (weight 2^B_R) and a hop component per site and direction (weight
(T+1) c_hop); C = S (2^B_R + 4 (T+1) c_hop) and Lambda = C / s events per
replica per unit time.  The chain itself is in lattice.c.
"""

import ctypes
import math

import numpy as np

from . import ssa
from .poisson import poisson_table


class _Lat(ctypes.Structure):
    _fields_ = [("lx", ctypes.c_int32), ("ly", ctypes.c_int32), ("P", ctypes.c_int32),
                ("B_r", ctypes.c_int32), ("c", ctypes.c_int64 * 5), ("c_hop", ctypes.c_int64),
                ("C", ctypes.c_uint64)]


_FRANK_ORDER = [((0, 0, 1), (1, 0, 0)), ((0, 0, 1), (0, 1, 0)), ((1, 0, 1), (2, 0, 0)),
                ((0, 1, 1), (0, 2, 0)), ((1, 1, 0), (0, 0, 2))]


def quantize_lattice(net, precision_bits=7):
    """c (5 Frank weights in table order), c_hop, s, f, P, T, B_r, C, Lambda."""
    rx = [(tuple(r), tuple(p)) for r, p in zip(net["reactants"], net["products"])]
    if rx != _FRANK_ORDER:
        raise ValueError("lattice oracle implements the 5-reaction Frank table")
    hops = net["hop_rates"]
    if len(set(hops)) != 1:
        raise ValueError("equal hop rates for every species")
    d = float(hops[0])
    rates = list(net["rates"])
    orders = [sum(r) for r in net["reactants"]]
    bi = [k for k, o in zip(rates, orders) if o == 2 and k > 0]
    pos = [k for k in rates + [d] if k > 0]
    k_ref = max(bi) if bi else max(pos)
    for f in range(0, 64):
        s = math.ldexp(1.0, f) / k_ref
        ok = True
        for k in rates + [d]:
            if k > 0:
                x = k * s
                c = int(round(x))
                if not (x == c or c >= (1 << precision_bits)):
                    ok = False
        if ok:
            break
    c = [int(round(k * s)) for k in rates]
    c_hop = int(round(d * s))
    P = int(net["site_planes"])
    T = (1 << P) - 1
    best = 0
    for nl in range(T + 1):
        for nd in range(T + 1 - nl):
            for na in range(T + 1 - nl - nd):
                w = c[0] * na + c[1] * na + c[2] * na * nl + c[3] * na * nd + c[4] * nl * nd
                best = max(best, w)
    B_r = max(1, (best - 1).bit_length()) if best > 1 else 1
    S = net["lx"] * net["ly"]
    C = S * ((1 << B_r) + 4 * (T + 1) * c_hop)
    return dict(c=c, c_hop=c_hop, s=s, f=f, P=P, T=T, B_r=B_r, C=C,
                Lambda=float(C) / s, max_site=best)


def c_lat(net, q):
    L = _Lat()
    L.lx, L.ly, L.P, L.B_r = net["lx"], net["ly"], q["P"], q["B_r"]
    for j in range(5):
        L.c[j] = q["c"][j]
    L.c_hop = q["c_hop"]
    L.C = q["C"]
    return L


def _lib():
    lib = ssa.lib()
    if not getattr(lib, "_lat_sigs", False):
        P = ctypes.POINTER
        u64, u32, i32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32
        lib.orc_lat_run.argtypes = [P(_Lat), u64, u32, u64, u64, u64, P(i32), P(u64), P(u64),
                                    P(u64), P(u64), ctypes.c_int]
        lib.orc_lat_run.restype = ctypes.c_int
        lib.orc_lat_init_uniform.argtypes = [u64, u32, u64, u64, u64, i32, i32, i32, P(i32)]
        lib.orc_lat_component.argtypes = [u64, u32, u32, u64, u64]
        lib.orc_lat_component.restype = u64
        lib._lat_sigs = True
    return lib


GROUP_REPLICAS = 2048


def component(seed, net_id, group, e, C):
    return _lib().orc_lat_component(seed, net_id, group, e, C)


class OracleLattice:
    """Replicas first + k*stride (k < count) of an ensemble of one lattice
    network; count defaults to the rest of n_replicas."""

    def __init__(self, net, n_replicas, seed=0, net_id=0, first=0, count=None, threads=0,
                 stride=1):
        self.net = net
        self.q = quantize_lattice(net)
        self.M = n_replicas
        self.first = first
        self.stride = stride
        self.n = (n_replicas - first + stride - 1) // stride if count is None else count
        self.seed, self.net_id, self.threads = seed, net_id, threads
        self.S = net["lx"] * net["ly"]
        self.t_now = 0.0
        self.advance_index = 0
        self.E = np.zeros(self.n, dtype=np.uint64)
        self.real = np.zeros(self.n, dtype=np.uint64)
        self.blocked = np.zeros(self.n, dtype=np.uint64)
        self.sites = None

    def init(self, mode):
        if mode[0] == "uniform_site":
            lo, hi = mode[1], mode[2]
            out = np.zeros((self.n, self.S, 3), dtype=np.int32)
            _lib().orc_lat_init_uniform(self.seed, self.net_id, self.first, self.stride, self.n,
                                        self.S, lo, hi,
                                        out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
            self.sites = out
        elif mode[0] == "fixed_site":
            self.sites = np.tile(np.array(mode[1], np.int32), (self.n, self.S, 1))
        elif mode[0] == "sites":
            self.sites = np.ascontiguousarray(
                np.broadcast_to(np.asarray(mode[1], np.int32), (self.n, self.S, 3)))
        else:
            raise ValueError(mode)
        self.E[:] = 0
        self.real[:] = 0
        self.blocked[:] = 0
        self.t_now = 0.0
        self.advance_index = 0

    def advance(self, t_end):
        if t_end < self.t_now:
            raise ValueError("t_end before the current time")
        mu = self.q["Lambda"] * (t_end - self.t_now)
        if mu > 0:
            if self.stride == 1:
                K = ssa.budgets(self.seed, self.net_id, self.advance_index, self.first, self.n,
                                poisson_table(mu))
            else:
                tab = poisson_table(mu)
                K = np.concatenate([ssa.budgets(self.seed, self.net_id, self.advance_index,
                                                self.first + k * self.stride, 1, tab)
                                    for k in range(self.n)])
        else:
            K = np.zeros(self.n, dtype=np.uint64)
        self._run(K)
        self.t_now = t_end
        self.advance_index += 1
        return K

    def step(self, n_events):
        self._run(np.full(self.n, n_events, dtype=np.uint64))

    def _run(self, K):
        P = ctypes.POINTER
        sites = np.ascontiguousarray(self.sites, dtype=np.int32)
        real = np.zeros(self.n, dtype=np.uint64)
        blk = np.zeros(self.n, dtype=np.uint64)
        E0 = np.ascontiguousarray(self.E, dtype=np.uint64)
        K = np.ascontiguousarray(K, dtype=np.uint64)
        cl = c_lat(self.net, self.q)
        rc = _lib().orc_lat_run(ctypes.byref(cl), self.seed, self.net_id, self.first,
                                self.stride, self.n,
                                sites.ctypes.data_as(P(ctypes.c_int32)),
                                E0.ctypes.data_as(P(ctypes.c_uint64)),
                                K.ctypes.data_as(P(ctypes.c_uint64)),
                                real.ctypes.data_as(P(ctypes.c_uint64)),
                                blk.ctypes.data_as(P(ctypes.c_uint64)), self.threads)
        if rc != 0:
            raise AssertionError("lattice oracle invariant violated")
        self.sites = sites
        self.E = self.E + K
        self.real = self.real + real
        self.blocked = self.blocked + blk

    def totals(self):
        return self.sites.sum(axis=1).astype(np.int32)

    def histogram(self, n_bins=256):
        t = self.totals().astype(np.int64)
        n = t.sum(1)
        d = t[:, 0] - t[:, 1]
        bins = np.where(n > 0, np.minimum(n_bins - 1, ((d + n) * n_bins) // np.maximum(2 * n, 1)),
                        n_bins // 2)
        return np.bincount(bins, minlength=n_bins).astype(np.uint64)
