"""ctypes mirror of include/bwg.h.  Argument marshalling only."""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbwg.so")

BWG_OK = 0
BWG_EINVAL = -1
BWG_ERANGE = -2
BWG_ENOMEM = -3
BWG_EDEVICE = -4
BWG_EUNSUPPORTED = -5
ERROR_NAMES = {BWG_EINVAL: "EINVAL", BWG_ERANGE: "ERANGE", BWG_ENOMEM: "ENOMEM",
               BWG_EDEVICE: "EDEVICE", BWG_EUNSUPPORTED: "EUNSUPPORTED"}

BWG_MAX_SPECIES = 8
BWG_MAX_REACTIONS = 16
BWG_EXACT_INTEGER = 1
BWG_OPEN = 2
BWG_ENGINE_BITWISE = 0
BWG_ENGINE_PLAIN = 1
BWG_ENGINE_LANES = 2
BWG_INIT_FIXED = 0
BWG_INIT_MULTINOMIAL = 1
BWG_INIT_UNIFORM_SITE = 2
BWG_INIT_SITES = 3
BWG_OPT_TIME_KERNELS = 1
BWG_OPT_SHARED_THRESHOLD = 2
BWG_OPT_GENERIC_KERNEL = 4
BWG_OPT_NO_JIT = 8
BWG_OPT_NO_LDS_STAGE = 16
BWG_LAT_STAGE_SITES = 840
BWG_LAT_CHUNK_EVENTS = 8192
BWG_LAT_PASS_CHUNKS = 32
BWG_JIT_GENERAL = 1
BWG_JIT_FRANK = 2

# Every symbol include/bwg.h declares.
SYMBOLS = (
    "bwg_net_create", "bwg_net_quantized", "bwg_net_destroy", "bwg_poisson_table",
    "bwg_ensemble_state_bytes", "bwg_ensemble_create", "bwg_ensemble_init",
    "bwg_ensemble_advance", "bwg_ensemble_step", "bwg_ensemble_read_counts",
    "bwg_ensemble_histogram", "bwg_ensemble_read_events", "bwg_ensemble_stats",
    "bwg_ensemble_destroy", "bwg_last_error", "bwg_batch_state_bytes", "bwg_batch_create",
    "bwg_batch_advance", "bwg_batch_graph_advance", "bwg_batch_destroy",
    "bwg_ensemble_schedule", "bwg_ensemble_run", "bwg_ensemble_pending",
    "bwg_batch_capacity_bytes", "bwg_batch_set_members", "bwg_batch_run",
    "bwg_net_lattice", "bwg_ensemble_read_sites", "bwg_ensemble_read_blocked",
    "bwg_ensemble_kernel_time", "bwg_ensemble_set_engine", "bwg_ensemble_set_lanes_words",
    "bwg_ensemble_record", "bwg_ensemble_prepare", "bwg_ensemble_step_static",
    "bwg_net_compile", "bwg_ensemble_checkpoint_bytes", "bwg_ensemble_save",
    "bwg_ensemble_restore",
)
BWG_STATIC_STATE_BYTES = 64 << 20


class NetDesc(ctypes.Structure):
    _fields_ = [("n_species", ctypes.c_int32), ("n_reactions", ctypes.c_int32),
                ("reactants", ctypes.POINTER(ctypes.c_int32)),
                ("products", ctypes.POINTER(ctypes.c_int32)),
                ("rates", ctypes.POINTER(ctypes.c_double)),
                ("n_tot", ctypes.c_int64), ("lx", ctypes.c_int32), ("ly", ctypes.c_int32),
                ("hop_rates", ctypes.POINTER(ctypes.c_double)),
                ("site_planes", ctypes.c_int32), ("precision_bits", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class QNet(ctypes.Structure):
    _fields_ = [("n_species", ctypes.c_int32), ("n_reactions", ctypes.c_int32),
                ("c", ctypes.c_int64 * BWG_MAX_REACTIONS), ("f", ctypes.c_int32),
                ("B", ctypes.c_int32), ("b", ctypes.c_int32), ("gpu_ok", ctypes.c_int32),
                ("s", ctypes.c_double), ("lambda_", ctypes.c_double),
                ("max_total", ctypes.c_int64), ("z_shared", ctypes.c_int64)]


class LatticeInfo(ctypes.Structure):
    _fields_ = [("lx", ctypes.c_int32), ("ly", ctypes.c_int32), ("sites", ctypes.c_int32),
                ("P", ctypes.c_int32), ("T", ctypes.c_int32), ("B_r", ctypes.c_int32),
                ("c_hop", ctypes.c_int64), ("C", ctypes.c_uint64), ("max_site", ctypes.c_int64),
                ("s", ctypes.c_double), ("lambda_", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("engine", ctypes.c_int32), ("block", ctypes.c_int32),
                ("table_capacity", ctypes.c_uint64), ("events_per_launch", ctypes.c_uint64),
                ("flags", ctypes.c_uint64), ("word_bits", ctypes.c_uint64),
                ("reserved", ctypes.c_uint64 * 2)]


class Stats(ctypes.Structure):
    _fields_ = [("n_replicas", ctypes.c_uint64), ("advance_index", ctypes.c_uint64),
                ("t_now", ctypes.c_double), ("events_total", ctypes.c_uint64),
                ("real_total", ctypes.c_uint64)]


class BatchOpts(ctypes.Structure):
    _fields_ = [("waves", ctypes.c_int32), ("order", ctypes.c_int32),
                ("max_ensembles", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("max_items", ctypes.c_uint64), ("reserved", ctypes.c_uint64 * 3)]


class BwgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERROR_NAMES.get(code, "?"), code, msg))
        self.code = code


_lib = None


def load():
    """Load libbwg.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libbwg.so is not built; run __graft_entry__.build() or "
                          "python paper_2412_16613_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    P, vp = ctypes.POINTER, ctypes.c_void_p
    u64, i64, u32, i32 = ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32, ctypes.c_int32
    sig = {
        "bwg_net_create": (i32, [P(NetDesc), P(vp)]),
        "bwg_net_quantized": (i32, [vp, P(QNet)]),
        "bwg_net_destroy": (None, [vp]),
        "bwg_net_compile": (i32, [vp, P(u32)]),
        "bwg_ensemble_checkpoint_bytes": (i32, [vp, P(u64)]),
        "bwg_ensemble_save": (i32, [vp, vp, u64, vp]),
        "bwg_ensemble_restore": (i32, [vp, vp, u64, vp]),
        "bwg_poisson_table": (i32, [ctypes.c_double, P(i64), P(u64), u64, P(u64)]),
        "bwg_ensemble_state_bytes": (i32, [vp, u64, P(Opts), P(u64)]),
        "bwg_ensemble_create": (i32, [vp, u64, u64, u32, vp, u64, P(Opts), P(vp)]),
        "bwg_ensemble_init": (i32, [vp, i32, P(i32), vp]),
        "bwg_ensemble_advance": (i32, [vp, ctypes.c_double, vp]),
        "bwg_ensemble_step": (i32, [vp, u64, vp]),
        "bwg_ensemble_read_counts": (i32, [vp, vp, vp]),
        "bwg_ensemble_histogram": (i32, [vp, i32, vp, vp]),
        "bwg_ensemble_read_events": (i32, [vp, vp, vp, vp]),
        "bwg_ensemble_stats": (i32, [vp, vp, P(Stats)]),
        "bwg_ensemble_destroy": (None, [vp]),
        "bwg_last_error": (ctypes.c_char_p, []),
        "bwg_batch_state_bytes": (i32, [P(vp), i32, P(u64)]),
        "bwg_batch_create": (i32, [P(vp), i32, vp, u64, P(BatchOpts), vp, P(vp)]),
        "bwg_batch_advance": (i32, [vp, P(ctypes.c_double), vp]),
        "bwg_batch_graph_advance": (i32, [vp, ctypes.c_double, i32, vp]),
        "bwg_batch_destroy": (None, [vp]),
        "bwg_ensemble_schedule": (i32, [vp, ctypes.c_double, vp]),
        "bwg_ensemble_run": (i32, [vp, u64, vp]),
        "bwg_ensemble_pending": (i32, [vp, P(u64)]),
        "bwg_batch_capacity_bytes": (i32, [i32, u64, P(u64)]),
        "bwg_batch_set_members": (i32, [vp, P(vp), i32, vp]),
        "bwg_batch_run": (i32, [vp, u64, vp]),
        "bwg_net_lattice": (i32, [vp, P(LatticeInfo)]),
        "bwg_ensemble_read_sites": (i32, [vp, u64, u64, vp, vp]),
        "bwg_ensemble_read_blocked": (i32, [vp, vp, vp]),
        "bwg_ensemble_kernel_time": (i32, [vp, P(ctypes.c_double), P(u64)]),
        "bwg_ensemble_set_engine": (i32, [vp, i32]),
        "bwg_ensemble_prepare": (i32, [vp]),
        "bwg_ensemble_set_lanes_words": (i32, [vp, u64]),
        "bwg_ensemble_record": (i32, [vp, P(ctypes.c_double), u32, vp, u32, vp, i32, vp, vp]),
        "bwg_ensemble_step_static": (i32, [vp, u64, u64, u32, P(i32), u64, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def check(rc):
    if rc != BWG_OK:
        msg = load().bwg_last_error().decode(errors="replace")
        raise BwgError(rc, msg)
    return rc
