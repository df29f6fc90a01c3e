"""Bit-parallel Gillespie exact stochastic simulation on MI355X (gfx950).

Python binding of libbwg.so (include/bwg.h): argument marshalling only.
Every step of the simulation runs in the library's HIP kernels; PyTorch
provides the device buffers and the stream.  There is no CPU fallback: the
binding raises if the library has not been built.

    from workloads import frank_network
    import paper_2412_16613_amd as bwg
    net = bwg.Network(frank_network(1024))
    ens = bwg.Ensemble(net, 1 << 20, seed=0)
    ens.init_fixed((0, 0, 1024))
    ens.advance(100.0)
    hist = ens.histogram(256)          # torch.int64 [256] on the GPU
"""

import ctypes

from . import _abi
from ._abi import BwgError  # noqa: F401

ENGINES = {"bitwise": _abi.BWG_ENGINE_BITWISE, "plain": _abi.BWG_ENGINE_PLAIN,
           "lanes": _abi.BWG_ENGINE_LANES}


def _lib():
    return _abi.load()


def _i32arr(vals):
    return (ctypes.c_int32 * len(vals))(*vals)


def poisson_table(mu, cap=1 << 20):
    """The library's budget table for mean mu: (k_lo, list of uint64)."""
    L = _lib()
    k_lo = ctypes.c_int64()
    n = ctypes.c_uint64()
    buf = (ctypes.c_uint64 * cap)()
    _abi.check(L.bwg_poisson_table(float(mu), ctypes.byref(k_lo), buf, cap, ctypes.byref(n)))
    return k_lo.value, list(buf[: n.value])


class Network:
    """A reaction network (see workloads.frank for the dict layout)."""

    def __init__(self, net, precision_bits=0):
        L = _lib()
        S = len(net["species"])
        R = len(net["rates"])
        self.net = net
        self._reac = _i32arr([v for row in net["reactants"] for v in row])
        self._prod = _i32arr([v for row in net["products"] for v in row])
        self._rates = (ctypes.c_double * R)(*net["rates"])
        self._hops = (ctypes.c_double * S)(*net.get("hop_rates", [0.0] * S))
        d = _abi.NetDesc()
        d.n_species, d.n_reactions = S, R
        d.reactants, d.products, d.rates = self._reac, self._prod, self._rates
        d.n_tot = int(net["n_tot"])
        d.lx, d.ly = int(net.get("lx", 0)), int(net.get("ly", 0))
        d.hop_rates = self._hops
        d.site_planes = int(net.get("site_planes", 0))
        d.precision_bits = int(precision_bits)
        d.flags = ((_abi.BWG_EXACT_INTEGER if net.get("exact_integer") else 0) |
                   (_abi.BWG_OPEN if net.get("open") else 0))
        h = ctypes.c_void_p()
        _abi.check(L.bwg_net_create(ctypes.byref(d), ctypes.byref(h)))
        self.handle = h

        self.is_lattice = bool(d.lx or d.ly)

    def quantized(self):
        q = _abi.QNet()
        _abi.check(_lib().bwg_net_quantized(self.handle, ctypes.byref(q)))
        R = q.n_reactions
        return dict(c=list(q.c[:R]), f=q.f, B=q.B, W=1 << q.B, b=q.b, s=q.s,
                    Lambda=q.lambda_, max_total=q.max_total, gpu_ok=bool(q.gpu_ok),
                    z_shared=q.z_shared or None)

    def compile(self):
        """Compile on the host now the run-time kernels a bit-sliced ensemble
        of this network would compile on its first use (bwg_net_compile);
        returns the set of kernels it uses, of "general" and "frank"."""
        built = ctypes.c_uint32()
        _abi.check(_lib().bwg_net_compile(self.handle, ctypes.byref(built)))
        return ({"general"} if built.value & _abi.BWG_JIT_GENERAL else set()) | \
            ({"frank"} if built.value & _abi.BWG_JIT_FRANK else set())

    def lattice(self):
        """Integer form of a lattice network (bwg_net_lattice)."""
        i = _abi.LatticeInfo()
        _abi.check(_lib().bwg_net_lattice(self.handle, ctypes.byref(i)))
        return dict(lx=i.lx, ly=i.ly, sites=i.sites, P=i.P, T=i.T, B_r=i.B_r, c_hop=i.c_hop,
                    C=i.C, max_site=i.max_site, s=i.s, Lambda=i.lambda_)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                _lib().bwg_net_destroy(h)
            except Exception:
                pass
            self.handle = None


def _stream_ptr(stream):
    return ctypes.c_void_p(stream.cuda_stream if stream is not None else 0)


def step_static(network, n_replicas, counts, n_events, seed=0, net_id=0, out=None,
                device="cuda"):
    """bwg_ensemble_step_static: n_replicas from the fixed start counts, run
    n_events each with the ensemble state in the library's static device
    array (no allocation inside the call); returns the counts, int32
    [n_replicas, S], in out if given (a contiguous device tensor)."""
    import torch
    dev = torch.device(device)
    S = len(network.net["species"])
    if out is None:
        out = torch.empty((int(n_replicas), S), dtype=torch.int32, device=dev)
    _abi.check(_lib().bwg_ensemble_step_static(
        network.handle, int(n_replicas), int(seed), int(net_id), _i32arr(counts), int(n_events),
        ctypes.c_void_p(out.data_ptr()), _stream_ptr(torch.cuda.current_stream(dev))))
    return out


def _opts(engine, events_per_launch, table_capacity, block, time_kernels, shared_threshold,
          generic, jit, word_bits, lds_stage):
    o = _abi.Opts()
    o.engine = ENGINES[engine]
    o.block = block
    o.table_capacity = table_capacity
    o.events_per_launch = events_per_launch
    o.word_bits = word_bits
    o.flags = ((_abi.BWG_OPT_TIME_KERNELS if time_kernels else 0) |
               (_abi.BWG_OPT_SHARED_THRESHOLD if shared_threshold else 0) |
               (_abi.BWG_OPT_GENERIC_KERNEL if generic else 0) |
               (0 if jit else _abi.BWG_OPT_NO_JIT) |
               (0 if lds_stage else _abi.BWG_OPT_NO_LDS_STAGE))
    return o


def _state_bytes(network, n_replicas, opts):
    nbytes = ctypes.c_uint64()
    _abi.check(_lib().bwg_ensemble_state_bytes(network.handle, n_replicas, ctypes.byref(opts),
                                               ctypes.byref(nbytes)))
    return nbytes.value


class Ensemble:
    """Replicas of one network in a caller-owned device buffer."""

    def __init__(self, network, n_replicas, seed=0, net_id=0, engine="bitwise",
                 device="cuda", events_per_launch=0, table_capacity=0, block=0,
                 time_kernels=False, shared_threshold=False, generic=False, jit=True,
                 word_bits=0, lds_stage=True):
        import torch
        self.torch = torch
        L = _lib()
        self.network = network
        self.M = int(n_replicas)
        self.device = torch.device(device)
        o = _opts(engine, events_per_launch, table_capacity, block, time_kernels,
                  shared_threshold, generic, jit, word_bits, lds_stage)
        self._opts = o
        self.state_bytes = _state_bytes(network, self.M, o)
        self._buf = torch.empty(self.state_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self._buf.data_ptr()
        off = (-base) % 256
        h = ctypes.c_void_p()
        _abi.check(L.bwg_ensemble_create(network.handle, self.M, int(seed), int(net_id),
                                         ctypes.c_void_p(base + off), self.state_bytes,
                                         ctypes.byref(o), ctypes.byref(h)))
        self.handle = h
        self.groups = (self.M + 31) // 32
        self.engine = engine
        self.n_species = len(network.net["species"])

    @staticmethod
    def bytes_needed(network, n_replicas, engine="bitwise", events_per_launch=0,
                     table_capacity=0, block=0, shared_threshold=False, generic=False,
                     jit=True, word_bits=0, lds_stage=True):
        """Device bytes an ensemble with these arguments takes (no allocation)."""
        return _state_bytes(network, int(n_replicas),
                            _opts(engine, events_per_launch, table_capacity, block, False,
                                  shared_threshold, generic, jit, word_bits, lds_stage))

    def _stream(self):
        return _stream_ptr(self.torch.cuda.current_stream(self.device))

    def init_fixed(self, counts):
        c = _i32arr(list(counts))
        _abi.check(_lib().bwg_ensemble_init(self.handle, _abi.BWG_INIT_FIXED, c, self._stream()))
        return self

    def init_multinomial(self):
        _abi.check(_lib().bwg_ensemble_init(self.handle, _abi.BWG_INIT_MULTINOMIAL, None,
                                            self._stream()))
        return self

    def init_uniform_site(self, lo, hi):
        """Lattice: A uniform in {lo..hi} on every site, L = D = 0."""
        c = _i32arr([int(lo), int(hi)])
        _abi.check(_lib().bwg_ensemble_init(self.handle, _abi.BWG_INIT_UNIFORM_SITE, c,
                                            self._stream()))
        return self

    def init_sites(self, sites):
        """Lattice: every replica starts from sites[s][x] (S x 3 counts)."""
        flat = [int(v) for row in sites for v in row]
        c = _i32arr(flat)
        _abi.check(_lib().bwg_ensemble_init(self.handle, _abi.BWG_INIT_SITES, c, self._stream()))
        return self

    def init(self, mode):
        if mode[0] in ("fixed", "fixed_site"):
            return self.init_fixed(mode[1])
        if mode[0] == "multinomial":
            return self.init_multinomial()
        if mode[0] == "uniform_site":
            return self.init_uniform_site(mode[1], mode[2])
        if mode[0] == "sites":
            return self.init_sites(mode[1])
        raise ValueError(mode)

    def advance(self, t_end):
        _abi.check(_lib().bwg_ensemble_advance(self.handle, float(t_end), self._stream()))
        return self

    def step(self, n_events):
        _abi.check(_lib().bwg_ensemble_step(self.handle, int(n_events), self._stream()))
        return self

    def schedule(self, t_end):
        """Draw the budgets of an advance to t_end without running events."""
        _abi.check(_lib().bwg_ensemble_schedule(self.handle, float(t_end), self._stream()))
        return self

    def run(self, max_events=0):
        """Run pending events, at most max_events per word (0: all)."""
        _abi.check(_lib().bwg_ensemble_run(self.handle, int(max_events), self._stream()))
        return self

    def pending(self):
        b = ctypes.c_uint64()
        _abi.check(_lib().bwg_ensemble_pending(self.handle, ctypes.byref(b)))
        return b.value

    def read_counts(self, out=None):
        t = self.torch
        if out is None:
            out = t.empty((self.M, self.n_species), dtype=t.int32, device=self.device)
        _abi.check(_lib().bwg_ensemble_read_counts(self.handle, ctypes.c_void_p(out.data_ptr()),
                                                   self._stream()))
        return out

    def histogram(self, n_bins=256, out=None):
        t = self.torch
        if out is None:
            out = t.empty(n_bins, dtype=t.int64, device=self.device)
        _abi.check(_lib().bwg_ensemble_histogram(self.handle, n_bins,
                                                 ctypes.c_void_p(out.data_ptr()),
                                                 self._stream()))
        return out

    def read_sites(self, first=0, count=None, out=None):
        """Lattice: site counts of replicas first..first+count-1 as an int32
        tensor [count, sites, 3]."""
        t = self.torch
        S = self.network.lattice()["sites"]
        count = self.M - first if count is None else int(count)
        if out is None:
            out = t.empty((count, S, 3), dtype=t.int32, device=self.device)
        _abi.check(_lib().bwg_ensemble_read_sites(self.handle, int(first), count,
                                                  ctypes.c_void_p(out.data_ptr()),
                                                  self._stream()))
        return out

    def read_blocked(self):
        """Lattice: hops into full sites per 32-replica word (int64)."""
        t = self.torch
        out = t.empty(self.groups, dtype=t.int64, device=self.device)
        _abi.check(_lib().bwg_ensemble_read_blocked(self.handle, ctypes.c_void_p(out.data_ptr()),
                                                    self._stream()))
        return out

    def record(self, t_grid, replicas=(), threshold=None, first=None):
        """Advance through t_grid; return (counts of the chosen replicas after
        each grid time, int32 [n_points, n_sel, 3]; first grid index at which
        |N_L - N_D| >= threshold per replica, int64 [M] with -1 for never, or
        None).  `first` continues an earlier record's first-passage tensor
        (uint32-valued, as returned with -1 entries)."""
        t = self.torch
        grid = [float(x) for x in t_grid]
        arr = (ctypes.c_double * max(len(grid), 1))(*grid)
        # uint32 indices, carried in an int32 tensor (indices of 2^31 and up
        # wrap to negative values and keep their bits)
        idx = [int(r) for r in replicas]
        if any(r < 0 or r >= 1 << 32 for r in idx):
            raise ValueError("replica indices are uint32")
        sel = t.tensor([r - (1 << 32) if r >= 1 << 31 else r for r in idx], dtype=t.int32,
                       device=self.device)
        out = t.empty((len(grid), len(sel), 3), dtype=t.int32, device=self.device)
        fp = None
        if threshold is not None:
            if first is None:
                fp = t.full((self.M,), -1, dtype=t.int32, device=self.device)
            else:
                fp = first.to(device=self.device, dtype=t.int32).clone()
        _abi.check(_lib().bwg_ensemble_record(
            self.handle, arr, len(grid), ctypes.c_void_p(sel.data_ptr() if len(sel) else 0),
            len(sel), ctypes.c_void_p(out.data_ptr() if len(sel) else 0),
            int(threshold or 0), ctypes.c_void_p(fp.data_ptr() if fp is not None else 0),
            self._stream()))
        return out, (fp.to(t.int64) if fp is not None else None)

    def save(self):
        """Checkpoint between advances (bwg_ensemble_save): a bytearray in the
        layout include/bwg.h documents."""
        n = ctypes.c_uint64()
        _abi.check(_lib().bwg_ensemble_checkpoint_bytes(self.handle, ctypes.byref(n)))
        buf = bytearray(n.value)
        ptr = (ctypes.c_char * n.value).from_buffer(buf)
        _abi.check(_lib().bwg_ensemble_save(self.handle, ptr, n.value, self._stream()))
        return buf

    def restore(self, blob):
        """Load a checkpoint (bwg_ensemble_restore); returns self."""
        src = (ctypes.c_char * len(blob)).from_buffer_copy(blob)
        _abi.check(_lib().bwg_ensemble_restore(self.handle, src, len(blob), self._stream()))
        return self

    def read_events(self):
        """(events per replica, real events per 32-lane group (bitwise) or
        per replica (plain)) as int64 tensors."""
        t = self.torch
        ev = t.empty(self.M, dtype=t.int64, device=self.device)
        nr = self.M if self.engine == "plain" else self.groups
        real = t.empty(nr, dtype=t.int64, device=self.device)
        _abi.check(_lib().bwg_ensemble_read_events(self.handle, ctypes.c_void_p(ev.data_ptr()),
                                                   ctypes.c_void_p(real.data_ptr()),
                                                   self._stream()))
        return ev, real

    def prepare(self):
        """Build now any kernel the next bit-sliced launch would compile at
        run time (Frank-family networks on run-time weights)."""
        _abi.check(_lib().bwg_ensemble_prepare(self.handle))
        return self

    def set_engine(self, engine):
        """Switch between the "bitwise" and "lanes" engines (same state and
        results; the lanes engine runs one replica per thread)."""
        _abi.check(_lib().bwg_ensemble_set_engine(self.handle, ENGINES[engine]))
        self.engine = engine
        return self

    def set_lanes_words(self, n_words):
        """In batches, run the last n_words words as lanes items."""
        _abi.check(_lib().bwg_ensemble_set_lanes_words(self.handle, int(n_words)))
        return self

    def kernel_time(self):
        """(ms, launches) of the event-kernel launches since the last call
        (ensembles created with time_kernels=True)."""
        ms = ctypes.c_double()
        n = ctypes.c_uint64()
        _abi.check(_lib().bwg_ensemble_kernel_time(self.handle, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def stats(self):
        s = _abi.Stats()
        _abi.check(_lib().bwg_ensemble_stats(self.handle, self._stream(), ctypes.byref(s)))
        return dict(n_replicas=s.n_replicas, advance_index=s.advance_index, t_now=s.t_now,
                    events_total=s.events_total, real_total=s.real_total)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                _lib().bwg_ensemble_destroy(h)
            except Exception:
                pass
            self.handle = None


class Batch:
    """Several bit-sliced ensembles whose events run in one persistent launch.

    With max_ensembles/max_items the batch keeps room for later member
    changes (set_members), as a continuous-batching server needs."""

    def __init__(self, ensembles, waves=0, order=0, max_ensembles=0, max_items=0,
                 device=None):
        import torch
        self.torch = torch
        L = _lib()
        self.ensembles = list(ensembles)
        n = len(self.ensembles)
        hs = (ctypes.c_void_p * max(n, 1))(*[e.handle.value for e in self.ensembles])
        nbytes = ctypes.c_uint64()
        if max_ensembles or max_items:
            _abi.check(L.bwg_batch_capacity_bytes(max(max_ensembles, n), int(max_items),
                                                  ctypes.byref(nbytes)))
            need = ctypes.c_uint64()
            _abi.check(L.bwg_batch_state_bytes(hs, n, ctypes.byref(need)))
            nbytes.value = max(nbytes.value, need.value)
        else:
            _abi.check(L.bwg_batch_state_bytes(hs, n, ctypes.byref(nbytes)))
        dev = device if device is not None else self.ensembles[0].device
        self.device = torch.device(dev)
        self._buf = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        base = self._buf.data_ptr()
        off = (-base) % 256
        o = _abi.BatchOpts()
        o.waves = int(waves)
        o.order = int(order)
        o.max_ensembles = int(max_ensembles)
        o.max_items = int(max_items)
        h = ctypes.c_void_p()
        _abi.check(L.bwg_batch_create(hs, n, ctypes.c_void_p(base + off), nbytes.value,
                                      ctypes.byref(o), self._stream(), ctypes.byref(h)))
        self.handle = h

    def _stream(self):
        return _stream_ptr(self.torch.cuda.current_stream(self.device))

    def set_members(self, ensembles):
        self.ensembles = list(ensembles)
        n = len(self.ensembles)
        hs = (ctypes.c_void_p * max(n, 1))(*[e.handle.value for e in self.ensembles])
        _abi.check(_lib().bwg_batch_set_members(self.handle, hs, n, self._stream()))
        return self

    def run(self, max_events=0):
        _abi.check(_lib().bwg_batch_run(self.handle, int(max_events), self._stream()))
        return self

    def advance(self, t_end):
        if not hasattr(t_end, "__len__"):
            t_end = [t_end] * len(self.ensembles)
        arr = (ctypes.c_double * max(len(self.ensembles), 1))(*[float(t) for t in t_end])
        _abi.check(_lib().bwg_batch_advance(self.handle, arr, self._stream()))
        return self

    def graph_advance(self, dt, n_steps):
        _abi.check(_lib().bwg_batch_graph_advance(self.handle, float(dt), int(n_steps),
                                                  self._stream()))
        return self

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                _lib().bwg_batch_destroy(h)
            except Exception:
                pass
            self.handle = None
