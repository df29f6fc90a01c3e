"""Python side of the CPU oracle — TEST INFRASTRUCTURE ONLY.

``OracleEnsemble`` mirrors what an ensemble of replicas of one network does
(initial state, advances to a time, fixed numbers of events, readouts) with
every step computed by the plain per-replica direct method of ssa.c.  The
event budgets of each advance come from poisson.py and the draw contract
from philox.py.  ``py_events`` is the same direct method in pure Python, used
to cross-check the C version on tiny cases.
"""

import ctypes
import os
import subprocess

import numpy as np

from . import philox as _ph
from .poisson import poisson_table
from .quantize import quantize, weights, state_change

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liborc.so")
_MAX_S, _MAX_R = 8, 16

DRAW_EVENT = 1
DRAW_PLAIN = 4
DRAW_SHARED = 6
# Replica index of the one budget draw that every copy shares in the
# shared-threshold variant (no replica has it: ensembles hold < 2^32).
SHARED_BUDGET_REPLICA = 0xFFFFFFFF


def build(force=True):
    """Compile ssa.c and lattice.c into liborc.so (gcc, OpenMP)."""
    srcs = [os.path.join(_HERE, f) for f in ("ssa.c", "lattice.c")
            if os.path.exists(os.path.join(_HERE, f))]
    if not force and os.path.exists(_LIB):
        return _LIB
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-o",
           _LIB + ".tmp"] + srcs
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Net(ctypes.Structure):
    _fields_ = [("n_species", ctypes.c_int32), ("n_reactions", ctypes.c_int32),
                ("reactants", (ctypes.c_int32 * _MAX_S) * _MAX_R),
                ("products", (ctypes.c_int32 * _MAX_S) * _MAX_R),
                ("c", ctypes.c_int64 * _MAX_R), ("B", ctypes.c_int32),
                ("z_shared", ctypes.c_uint32), ("n_tot", ctypes.c_int64),
                ("open", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        u64, i64, u32, i32 = (ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32,
                              ctypes.c_int32)
        L.orc_wm_run.argtypes = [P(_Net), u64, u32, ctypes.c_int, u64, u64,
                                 P(i32), P(u64), P(u64), P(u64), P(i32), u64,
                                 ctypes.c_int]
        L.orc_wm_run.restype = ctypes.c_int
        L.orc_budget.argtypes = [u64, u32, u64, u64, u64, P(u64), u64, i64, P(u64)]
        L.orc_init_multinomial.argtypes = [u64, u32, u64, u64, i64, P(i32)]
        L.orc_philox.argtypes = [P(u32), u64, P(u32)]
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_select.argtypes = [P(_Net), P(i32), u64]
        L.orc_draw_shared.argtypes = [u64, u32, u64, u32]
        L.orc_draw_shared.restype = u32
        L.orc_select.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def c_net(net, q):
    S, R = len(net["species"]), len(net["rates"])
    if S > _MAX_S or R > _MAX_R:
        raise ValueError("network too large for the oracle")
    cn = _Net()
    cn.n_species, cn.n_reactions = S, R
    for j in range(R):
        for x in range(S):
            cn.reactants[j][x] = net["reactants"][j][x]
            cn.products[j][x] = net["products"][j][x]
        cn.c[j] = q["c"][j]
    cn.B = q["B"]
    cn.z_shared = q.get("z_shared") or 0
    cn.n_tot = net["n_tot"]
    cn.open = 1 if net.get("open") else 0
    return cn


def philox_c(ctr, seed):
    out = (ctypes.c_uint32 * 4)()
    lib().orc_philox((ctypes.c_uint32 * 4)(*ctr), seed, out)
    return tuple(out)


def run_events(net, q, seed, net_id, first, counts, E0, K, draw=DRAW_EVENT,
               traj_len=0, threads=0):
    """Run K[k] events for replicas first+k; returns (counts, real, traj)."""
    counts = np.ascontiguousarray(counts, dtype=np.int32).copy()
    n = counts.shape[0]
    E0 = np.ascontiguousarray(E0, dtype=np.uint64)
    K = np.ascontiguousarray(K, dtype=np.uint64)
    real = np.zeros(n, dtype=np.uint64)
    traj = None
    tp = ctypes.POINTER(ctypes.c_int32)()
    if traj_len:
        traj = np.zeros((n, traj_len, counts.shape[1]), dtype=np.int32)
        tp = _p(traj, ctypes.c_int32)
    cn = c_net(net, q)
    rc = lib().orc_wm_run(ctypes.byref(cn), seed, net_id, draw, first, n,
                          _p(counts, ctypes.c_int32), _p(E0, ctypes.c_uint64),
                          _p(K, ctypes.c_uint64), _p(real, ctypes.c_uint64),
                          tp, traj_len, threads)
    if rc == -4:
        raise ValueError("the PLAIN draw is one 32-bit word: weights of %d planes need the "
                         "EVENT draw" % q["B"])
    if rc != 0:
        raise AssertionError("oracle invariant violated (negative count, count above the "
                             "cap, or molecule count not conserved)")
    return counts, real, traj


def draw_shared(seed, net_id, e, Z):
    """n shared by every replica at event e (SHARED draw), uniform on [0, Z)."""
    return lib().orc_draw_shared(seed, net_id, e, Z)


def select(net, q, counts, n):
    """Reaction picked by threshold n in state counts (-1: null event)."""
    cn = c_net(net, q)
    c = np.ascontiguousarray(counts, dtype=np.int32)
    return lib().orc_select(ctypes.byref(cn), _p(c, ctypes.c_int32), n)


def budgets(seed, net_id, advance, first, n, table):
    k_lo, T = table
    Ta = np.array(T, dtype=np.uint64)
    out = np.zeros(n, dtype=np.uint64)
    lib().orc_budget(seed, net_id, advance, first, n, _p(Ta, ctypes.c_uint64),
                     len(T), k_lo, _p(out, ctypes.c_uint64))
    return out


def init_multinomial(seed, net_id, first, n, n_tot):
    out = np.zeros((n, 3), dtype=np.int32)
    lib().orc_init_multinomial(seed, net_id, first, n, n_tot,
                               _p(out, ctypes.c_int32))
    return out


def ee_histogram(counts, n_tot, n_bins=256):
    """bin = min(n_bins-1, floor((N_L - N_D + N_tot) n_bins / (2 N_tot)))."""
    d = counts[:, 0].astype(np.int64) - counts[:, 1].astype(np.int64)
    bins = np.minimum(n_bins - 1, ((d + n_tot) * n_bins) // (2 * n_tot))
    return np.bincount(bins, minlength=n_bins).astype(np.uint64)


class OracleEnsemble:
    """Replicas [first, first+n) of an ensemble of one well-mixed network."""

    def __init__(self, net, n_replicas, seed=0, net_id=0, first=0, count=None,
                 draw=DRAW_EVENT, q=None, threads=0):
        self.net = net
        self.q = q if q is not None else quantize(net)
        self.M = n_replicas
        self.first = first
        self.n = n_replicas - first if count is None else count
        self.seed, self.net_id, self.draw, self.threads = seed, net_id, draw, threads
        self.t_now = 0.0
        self.advance_index = 0
        self.E = np.zeros(self.n, dtype=np.uint64)
        self.real = np.zeros(self.n, dtype=np.uint64)
        self.counts = None

    def init(self, mode):
        if mode[0] == "fixed":
            c = np.array(mode[1], dtype=np.int32)
            if len(c) != len(self.net["species"]) or (c < 0).any():
                raise ValueError("one non-negative count per species")
            if self.net.get("open"):
                if (c > self.net["n_tot"]).any():
                    raise ValueError("initial counts above the cap n_tot")
            elif c.sum() != self.net["n_tot"]:
                raise ValueError("initial counts must sum to N_tot")
            self.counts = np.tile(c, (self.n, 1))
        elif mode[0] == "multinomial":
            self.counts = init_multinomial(self.seed, self.net_id, self.first,
                                           self.n, self.net["n_tot"])
        else:
            raise ValueError(mode)
        self.E[:] = 0
        self.real[:] = 0
        self.t_now = 0.0
        self.advance_index = 0

    def event_rate(self):
        """Events per unit time: Lambda = W / s; in the shared-threshold
        variant Z / s (the paper's constant total propensity, Eqs. (9), (12)),
        both divisions in binary64."""
        if self.draw == DRAW_SHARED:
            return self.q["z_shared"] / self.q["s"]
        return self.q["Lambda"]

    def mean_events(self, t_end):
        """mu = rate * (t_end - t_now) in binary64, in that order."""
        return self.event_rate() * (t_end - self.t_now)

    def advance(self, t_end, traj_len=0):
        if t_end < self.t_now:
            raise ValueError("t_end before the current time")
        mu = self.mean_events(t_end)
        if mu > 0.0 and self.draw == DRAW_SHARED:
            # one time step for every copy (the paper's shared tau): a single
            # budget, drawn at the reserved replica index
            k = budgets(self.seed, self.net_id, self.advance_index, SHARED_BUDGET_REPLICA, 1,
                        poisson_table(mu))[0]
            K = np.full(self.n, k, dtype=np.uint64)
        elif mu > 0.0:
            K = budgets(self.seed, self.net_id, self.advance_index, self.first,
                        self.n, poisson_table(mu))
        else:
            K = np.zeros(self.n, dtype=np.uint64)
        traj = self._run(K, traj_len)
        self.t_now = t_end
        self.advance_index += 1
        return K, traj

    def step(self, n_events, traj_len=0):
        K = np.full(self.n, n_events, dtype=np.uint64)
        return K, self._run(K, traj_len)

    def _run(self, K, traj_len):
        self.counts, real, traj = run_events(
            self.net, self.q, self.seed, self.net_id, self.first, self.counts,
            self.E, K, self.draw, traj_len, self.threads)
        self.E = self.E + K
        self.real = self.real + real
        return traj

    def histogram(self, n_bins=256):
        return ee_histogram(self.counts, self.net["n_tot"], n_bins)


# ---------------------------------------------------------------------------
# Pure-Python direct method for tiny cases (cross-checks ssa.c).
# ---------------------------------------------------------------------------

def py_events(net, q, seed, net_id, replica, counts, E0, K, draw=DRAW_EVENT):
    """Return (final counts, list of reaction indices or -1) for one replica."""
    nu = state_change(net)
    N = list(counts)
    picked = []
    if draw == DRAW_PLAIN and q["B"] > 32:
        raise ValueError("the PLAIN draw is one 32-bit word")
    for e in range(E0, E0 + K):
        if draw == DRAW_PLAIN:
            n = _ph.plain_threshold(seed, net_id, replica, e, q["B"])
        elif draw == DRAW_SHARED:
            n = _ph.shared_threshold(seed, net_id, e, q["z_shared"])
        else:
            n = _ph.event_threshold(seed, net_id, replica, e, q["B"])
        w = weights(net, q, N)
        m, r = 0, -1
        for j, wj in enumerate(w):
            m += wj
            if n < m:
                r = j
                break
        if r >= 0 and net.get("open") and any(a + d > net["n_tot"] for a, d in zip(N, nu[r])):
            r = -1          # open network: a firing past the cap does nothing
        picked.append(r)
        if r >= 0:
            N = [a + d for a, d in zip(N, nu[r])]
            assert min(N) >= 0
            assert max(N) <= net["n_tot"] if net.get("open") else sum(N) == net["n_tot"]
    return N, picked
