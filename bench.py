"""Throughput of the bit-parallel Gillespie path on one MI355X.

One step = initial state + advance of every replica to t_end (budget draws
and the event kernel) + per-replica counts + enantiomeric-excess histogram,
on the well-mixed Frank workload N_tot = 1024, 2^20 replicas, t_end = 100,
all-A start, seed 0.  The metric counts every uniformised event (null
events included, the paper's "iterations") over all replicas.

Prints one JSON line.  Extra fields: the plain one-replica-per-thread engine
on the same workload, the dominant kernel's roofline, and the CPU oracle on
a bounded sample.
"""

import argparse
import json
import math

import numpy as np
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# VALU issue slots per word-event (32 replica-events) that the bit-sliced method needs, in
# the form the well-mixed kernel computes it (word_event_slots).  One slot is one 32-bit VALU
# instruction per lane; v_mad_u64_u32 issues at the same rate as v_bitop3_b32 (--valu-ref).
PHILOX_SLOTS = 40           # 20 32x32->64 multiply-adds + 20 three-input xors per call


def _bitlen(v):
    return int(v).bit_length()


def _signed_width(lo, hi):
    return max(2, _bitlen(max(hi, -lo - 1)) + 1)


def word_event_slots(q, n_tot):
    """Slots per word-event of the well-mixed Frank event at exact register
    widths (the molecule count known): RNG, the five cumulative comparisons
    (borrow chains, the two that feed later ones keep their difference),
    the changer masks, three masked +-1/+2 ripple updates of the counts, the
    pair counts P_AL, Q_A = N_A (N_tot - N_A), P_LD (masked change formed
    over its exact width, then a sign-extended ripple add) and U = c_u N_A."""
    b, B, N = q["b"], q["B"], n_tot
    BS = B + (1 if q["max_total"] == (1 << B) else 0)
    c = q["c"]
    cu, fa, fi = c[0], _bitlen(c[2]) - 1, _bitlen(c[4]) - 1
    fmin = min(fa, fi)
    UW = max(1, _bitlen(cu * N))
    WP = max(2, _bitlen((N // 2) * (N - N // 2)))
    wd_al = _signed_width(-N + 1, 2 * N - 4)
    wd_qa = _signed_width(-2 * N + 4, 2 * N - 4)
    wd_ld = _signed_width(-N, N - 1)
    rng = ((B + 3) // 4) * PHILOX_SLOTS
    select = (UW + -(-(BS - UW - 1) // 2) + 1) + (fmin - 1) + 2 * (BS - fmin) \
        + (BS - fa) + 2 * (BS - fa) + (BS - fi)
    masks = 10
    counts = 3 * (2 * b - 1)
    products = (5 * wd_al + 2 * WP - 1) + (4 * wd_qa + 2 * WP - 1) + (4 * wd_ld + 2 * WP - 1)
    unimolecular = 2 * UW - 1
    return rng + select + masks + counts + products + unimolecular


# 32-bit VALU lane-operations/s: 256 CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz (a wave64
# instruction in 4 cycles; the fp64 vector peak of 78.6 TFLOP/s is this lane rate of FMAs,
# the fp32 157.3 counts packed pairs, which bitwise instructions do not have).  Measured by
# --valu-ref: v_bitop3_b32 reaches 0.97 of it, v_mad_u64_u32 0.93.
VALU_PEAK = 256 * 4 * 16 * 2.4e9
HBM_PEAK = 8.0e12               # bytes/s, MI355X HBM3E

# HBM bytes per launch of a kernel from rocprofv3 FETCH_SIZE x 2 + WRITE_SIZE x 1
# (the factors of a 1 GiB copy), valid only for the sources they were taken on:
# kernel -> (sha1 prefix of its sources, sources, bytes per launch, summary file).
CSRC = os.path.join(ROOT, "paper_2412_16613_amd", "csrc")
MEASURED_TRAFFIC = {
    "wm_pc_kernel": ("56dc664d5d4c", ("bitops.h", "wm_device.h", "wm_event_body.inc",
                                      "wm_kernel.hip"),
                     (2 * 10822 + 12672) * 1024, "profiles/wm_pc_kernel_frank1024_2p20.md"),
    "lat_event_kernel": ("ed3743083ea0", ("bitops.h", "bwg_internal.h", "lattice.hip"),
                         (2 * 5477457 + 11890680) * 1024,
                         "profiles/lat_event_kernel_lattice64x64_2p16.md"),
}


# VALU wave instructions per launch (rocprofv3 SQ_INSTS_VALU), valid for the same sources:
# kernel -> (sha1 prefix, sources, instructions per launch, summary file).
MEASURED_VALU = {
    "wm_pc_kernel": ("56dc664d5d4c", ("bitops.h", "wm_device.h", "wm_event_body.inc",
                                      "wm_kernel.hip"),
                     20831937027, "profiles/wm_pc_kernel_frank1024_2p20.md"),
}


def _sources_match(entry):
    import hashlib
    sha, files = entry[0], entry[1]
    h = hashlib.sha1()
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12] == sha


def measured_valu(kernel):
    """Counter-measured VALU wave instructions per launch, or None once the
    kernel's sources differ from the ones the counter was taken on."""
    e = MEASURED_VALU.get(kernel)
    return e[2] if e and _sources_match(e) else None


def measured_traffic(kernel):
    """Counter-measured HBM bytes per launch, or None once the kernel's
    sources differ from the ones the counters were taken on."""
    import hashlib
    if kernel not in MEASURED_TRAFFIC:
        return None
    sha, files, nbytes, _ = MEASURED_TRAFFIC[kernel]
    h = hashlib.sha1()
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return nbytes if h.hexdigest()[:12] == sha else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-replicas", type=int, default=65536)
    ap.add_argument("--cpu-replicas-lattice", type=int, default=64)
    ap.add_argument("--workload", default="well-mixed",
                    choices=["well-mixed", "lattice", "batch", "serve", "gain", "gain-cpu",
                             "trajectory", "general"],
                    help="lattice: 64x64 compartments, 2^16 replicas; batch: the 256 uneven "
                         "networks in one persistent launch; gain: the paper's Q(N) sweep")
    ap.add_argument("--gain-n", default="8,16,32,64,128,256,512,1024",
                    help="gain: molecule counts N_tot of the paper's network")
    ap.add_argument("--gain-replicas", default="4194304,64",
                    help="gain: replica counts M, one table each (64: the paper's M)")
    ap.add_argument("--gain-widths", default="16,32,64",
                    help="gain: replicas per thread of the bit-parallel engine")
    ap.add_argument("--gain-steps", type=int, default=100000)
    ap.add_argument("--gain-repeats", type=int, default=3,
                    help="gain: timed steps of T per bit-parallel mode (median taken)")
    ap.add_argument("--batch-nets", type=int, default=256)
    ap.add_argument("--rate", type=float, default=200.0, help="serve: arrivals per second")
    ap.add_argument("--duration", type=float, default=60.0, help="serve: arrival window (s)")
    ap.add_argument("--chunk", type=int, default=4096, help="serve: events per word per pass")
    ap.add_argument("--no-lds-stage", action="store_true",
                    help="lattice: the event kernel that keeps every site in memory")
    ap.add_argument("--lanes-events", type=float, default=0.0,
                    help="serve: requests expecting at least this many events per replica run "
                         "on the lanes engine (0: none)")
    ap.add_argument("--compare-nets", type=int, default=32,
                    help="networks for the one-network-per-launch comparison")
    ap.add_argument("--engine", default="bitwise", choices=["bitwise", "lanes"],
                    help="well-mixed: the engine that runs the replicas (identical results)")
    ap.add_argument("--shard", type=int, default=1,
                    help="well-mixed: time one GPU's share of the workload split by word over this "
                         "many GPUs (replicas 0 .. 2^20/shard - 1, the same draws as in the whole "
                         "run)")
    ap.add_argument("--copy-ref", action="store_true",
                    help="only copy 1 GiB device-to-device (calibrates HBM byte counters)")
    ap.add_argument("--valu-ref", action="store_true",
                    help="only the VALU issue-rate reference: v_bitop3_b32 and v_mad_u64_u32 "
                         "chains at 1, 2, 4 and 8 waves per SIMD")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: replicas are independent and would shard by "
              "word across GPUs, but only the single-GPU path is implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_ref:
        src = torch.ones(1 << 28, dtype=torch.int32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_ref_bytes": 1 << 30}))
        return
    if args.valu_ref:
        return valu_ref()
    if args.workload == "gain-cpu":
        return bench_gain_cpu(args)
    import paper_2412_16613_amd as bwg
    from workloads import config
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "lattice":
        return bench_lattice(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "gain":
        return bench_gain(args)
    if args.workload == "trajectory":
        return bench_trajectory(args)
    if args.workload == "general":
        return bench_general(args)

    c = config("c1")
    net, M, t_end = c["net"], c["replicas"], c["t_end"]
    if args.shard < 1 or M % (32 * args.shard):
        print("--shard must split the replicas into whole words", file=sys.stderr)
        sys.exit(2)
    M //= args.shard
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    network = bwg.Network(net)
    q = network.quantized()
    # counters were taken on the whole workload's bit-sliced launch
    whole = args.shard == 1 and args.engine == "bitwise"
    kernel = "wm_pc_kernel" if args.engine == "bitwise" else "wm_lanes_kernel"

    def make(engine):
        ens = bwg.Ensemble(network, M, seed=c["seed"], net_id=c["net_id"], engine=engine,
                           device=dev, time_kernels=True)
        counts = torch.empty((M, 3), dtype=torch.int32, device=dev)
        hist = torch.empty(256, dtype=torch.int64, device=dev)
        return ens, counts, hist

    def run(engine, steps, warmup):
        ens, counts, hist = make(engine)
        stream = torch.cuda.current_stream(dev)
        k0, k1 = [], []
        for _ in range(warmup):
            ens.init(c["init"]).advance(t_end)
            ens.read_counts(counts)
            ens.histogram(256, hist)
        torch.cuda.synchronize()
        ens.kernel_time()               # start counting event-kernel launches here
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        wall0 = time.perf_counter()
        t0.record(stream)
        for _ in range(steps):
            ens.init(c["init"])
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            ens.advance(t_end)
            b.record(stream)
            k0.append(a)
            k1.append(b)
            ens.read_counts(counts)
            ens.histogram(256, hist)
        t1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall0
        ms = t0.elapsed_time(t1)
        adv_ms = [x.elapsed_time(y) for x, y in zip(k0, k1)]
        kt_ms, kt_n = ens.kernel_time()
        st = ens.stats()
        assert int(hist.sum().item()) == M
        return dict(ms=ms, wall=wall, adv_ms=adv_ms, events=st["events_total"],
                    real=st["real_total"], kt_ms=kt_ms, kt_n=kt_n,
                    counts=counts.cpu().numpy(), hist=hist.cpu().numpy(),
                    ev=ens.read_events()[0].cpu().numpy())

    r = run(args.engine, args.steps, args.warmup)
    ms_step = r["ms"] / args.steps
    events_per_step = r["events"]          # same seed every step: same budgets
    value = events_per_step * args.steps / (r["ms"] / 1e3)
    adv_avg_ms = sum(r["adv_ms"]) / len(r["adv_ms"])
    word_events = events_per_step / 32.0
    slots = word_event_slots(q, net["n_tot"])
    # per event-kernel launch: its share of the step's word-events over its
    # duration (HIP events around each launch, on the launch stream)
    launches_per_step = r["kt_n"] / args.steps
    launch_ms = r["kt_ms"] / r["kt_n"]
    achieved = slots * word_events / launches_per_step / (launch_ms / 1e3)
    out = {
        "metric": "replica-events/sec (bit-parallel vs plain SSA, 1 GPU)",
        "value": value,
        "unit": "replica-events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32 bit-planes",
        "data": "synthetic",
        "config": {"workload": "well-mixed Frank model, N_tot=1024, 2^20 replicas, "
                               "t_end=100, all-A start, seed 0" +
                               ("" if args.shard == 1 else ", one GPU's shard of %d (replicas "
                                "0..%d)" % (args.shard, M - 1)) +
                               ("" if args.engine == "bitwise" else ", lanes engine"),
                   "n_tot": 1024, "replicas": M, "t_end": t_end, "threshold_planes": q["B"],
                   "count_planes": q["b"], "shard": args.shard, "engine": args.engine},
        "real_events_per_s": r["real"] * args.steps / (r["ms"] / 1e3),
        "replica_time_per_s": M * t_end * args.steps / (r["ms"] / 1e3),
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12,
                     "unit": "T VALU lane-slots/s", "frac": achieved / VALU_PEAK,
                     "traffic": measured_traffic("wm_pc_kernel") if whole else None,
                     "traffic_unit": "B/launch",
                     "kernel": kernel, "kernel_ms": launch_ms,
                     "launches_per_step": launches_per_step, "advance_ms": adv_avg_ms,
                     "slots_per_word_event": slots,
                     "valu_insts_per_launch": measured_valu("wm_pc_kernel") if whole else None,
                     "issued_frac": (measured_valu("wm_pc_kernel") * 64 / (launch_ms / 1e3) /
                                     VALU_PEAK if whole and measured_valu("wm_pc_kernel")
                                     else None)},
    }
    if args.engine == "lanes":
        # the lane-slot count above is the bit-sliced word's algorithmic work;
        # the one-replica-per-lane form has no such count of its own
        out["roofline"].update(achieved=None, frac=None, slots_per_word_event=None,
                               note="no algorithmic lane-slot count for the lanes engine")
    if not args.no_plain:
        p = run("plain", max(1, args.steps // 2), 1)
        pv = p["events"] * max(1, args.steps // 2) / (p["ms"] / 1e3)
        out["plain_ssa"] = {"value": pv, "unit": "replica-events/s",
                            "ms_per_step": p["ms"] / max(1, args.steps // 2),
                            "bitwise_over_plain": value / pv}
    # every replica: histogram of the last step's counts by the integer rule
    from oracle import ssa
    hist_ok = bool(np.array_equal(r["hist"].astype(np.uint64),
                                  ssa.ee_histogram(r["counts"], net["n_tot"], 256)))
    out["parity"] = hist_ok
    if not args.no_cpu:
        cb, orc = cpu_baseline(net, c, min(args.cpu_replicas, M))
        n = orc.n
        same = (np.array_equal(r["counts"][:n], orc.counts) and
                np.array_equal(r["ev"][:n].astype(np.uint64), orc.E))
        cb["parity"] = {"replicas": n, "bit_exact": bool(same)}
        out["cpu_baseline"] = cb
        out["parity"] = hist_ok and same
    print(json.dumps(out))
    if not out["parity"]:
        print("parity failure: GPU counts differ from the oracle", file=sys.stderr)
        sys.exit(1)


def valu_ref():
    """Sustained 32-bit VALU lane-operations per second of the two instructions
    the bit-sliced kernels are made of (calib/valu_ref.hip): v_bitop3_b32 and
    Philox's v_mad_u64_u32, eight independent chains per thread, and of the
    two-operand v_add_u32 the lanes engine is mostly made of, with 1, 2,
    4 and 8 waves per SIMD (256, 512, 1024, 2048 blocks of four waves).  Each
    wave64 instruction counts 64 lane-operations; the fraction is of the
    derived peak (256 CUs x 128 lanes per clock x 2.4 GHz)."""
    import ctypes
    import torch
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2412_16613_amd", "libbwg_calib.so"))
    lib.bwg_valu_ref.restype = ctypes.c_double
    lib.bwg_valu_ref.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p,
                                 ctypes.c_void_p]
    lib.bwg_valu_ref_ops_per_thread.restype = ctypes.c_uint64
    lib.bwg_valu_ref_ops_per_thread.argtypes = [ctypes.c_uint32]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    rows = []
    for kind, name, chains, iters in ((0, "v_bitop3_b32", 8, 20000),
                                      (1, "v_mad_u64_u32", 8, 20000),
                                      (3, "v_bitop3_b32", 2, 10000),
                                      (2, "v_bitop3_b32", 1, 5000),
                                      (4, "v_add_u32", 8, 20000)):
        for w in (1, 2, 4, 8):
            blocks = 256 * w
            out = torch.empty(blocks * 256, dtype=torch.int32, device=dev)
            lib.bwg_valu_ref(kind, blocks, 100, ctypes.c_void_p(out.data_ptr()), stream)
            ms = lib.bwg_valu_ref(kind, blocks, iters, ctypes.c_void_p(out.data_ptr()), stream)
            if ms <= 0:
                raise RuntimeError("reference kernel failed (%g)" % ms)
            # every wave issues ops_per_thread instructions of 64 lanes each
            wave_instr = blocks * 4 * lib.bwg_valu_ref_ops_per_thread(iters)
            rate = wave_instr * 64 / (ms / 1e3)
            rows.append({"instruction": name, "chains": chains, "waves_per_simd": w, "ms": ms,
                         "lane_ops_per_s": rate, "frac_of_peak": rate / VALU_PEAK,
                         "cycles_per_wave_instruction_per_simd":
                             (ms / 1e3) * 2.4e9 / (wave_instr / (256 * 4))})
    print(json.dumps({"valu_ref": rows, "peak_lane_ops_per_s": VALU_PEAK}))


def lattice_slots(q, li):
    """VALU issue slots per word-event of the lattice kernel: (reaction, hop).
    Reaction: ceil(B_r/4) Philox calls, the weights cu A (shift-adds over its
    set bits into B_r + 1 planes), three P x P products, three shifted adds
    and five B_r + 1 plane comparisons, masks and the masked +-1 updates; hop:
    one Philox call, two P-plane sums per site, three comparisons, the full
    test and six masked +-1 updates."""
    P, Br = li["P"], li["B_r"]
    BC = Br + 1
    cu = q["c"][0]
    wx = (cu * ((1 << P) - 1)).bit_length()
    shifts = [k for k in range(BC) if (cu >> k) & 1]
    cu_adds = sum(2 * (wx - k) for k in shifts[1:])      # the first is a copy
    product = 4 * P + (P - 1) * (3 * P + 1)              # ANDs + P-plane ripple per row
    ca_add = 2 * (BC - (q["c"][2].bit_length() - 1))
    react = (-(-Br // 4)) * PHILOX_SLOTS + cu_adds + 5 * BC + 3 * (product + ca_add) + 8 + 3 * 2 * P
    hop = PHILOX_SLOTS + 4 * 2 * P + 3 * P + (P - 1) + 6 + 6 * 2 * P
    return react, hop


def bench_lattice(args):
    """64 x 64 periodic lattice of Frank reactors (12 molecules per site on
    average, 4 planes per species per site), hops at d = 0.1, A uniform in
    {9..15} per site, 2^16 replicas, t_end = 20.  One step = init + advance
    + species totals + ee histogram."""
    import torch
    import paper_2412_16613_amd as bwg
    from workloads import config
    c = config("c2")
    net, M, t_end = c["net"], c["replicas"], c["t_end"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    network = bwg.Network(net)
    q, li = network.quantized(), network.lattice()
    ens = bwg.Ensemble(network, M, seed=c["seed"], net_id=c["net_id"], device=dev,
                       time_kernels=True, lds_stage=not args.no_lds_stage)
    counts = torch.empty((M, 3), dtype=torch.int32, device=dev)
    hist = torch.empty(256, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream(dev)
    for _ in range(args.warmup):
        ens.init(c["init"]).advance(t_end)
    torch.cuda.synchronize()
    ens.kernel_time()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    adv = []
    t0.record(stream)
    for _ in range(args.steps):
        ens.init(c["init"])
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        ens.advance(t_end)
        b.record(stream)
        adv.append((a, b))
        ens.read_counts(counts)
        ens.histogram(256, hist)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    adv_ms = sum(a.elapsed_time(b) for a, b in adv) / len(adv)
    kt_ms, kt_n = ens.kernel_time()
    st = ens.stats()
    assert int(hist.sum().item()) == M
    events = st["events_total"]
    value = events * args.steps / (ms / 1e3)
    react, hop = lattice_slots(q, li)
    W_R, W_H = 1 << li["B_r"], ((li["T"] + 1) * li["c_hop"])
    f_r = W_R / (W_R + 4 * W_H)
    slots = f_r * react + (1 - f_r) * hop
    launches_per_step = kt_n / args.steps
    launch_ms = kt_ms / kt_n
    word_events = events / 32.0 / launches_per_step          # per launch
    achieved = slots * word_events / (launch_ms / 1e3)
    # site-plane bytes: a reaction reads and writes the 3 x P planes of its
    # site (one 32-bit word each), a hop those of both sites.  The event
    # kernel keeps the first BWG_LAT_STAGE_SITES sites of every word in LDS
    # for a pass of BWG_LAT_PASS_CHUNKS chunks: its algorithmic HBM bytes are one copy of
    # those sites in and out per word and pass, and the site-plane bytes of
    # the events on the other sites
    from paper_2412_16613_amd import _abi
    site_bytes = 3 * li["P"] * 4
    plane_bytes_we = f_r * 2 * site_bytes + (1 - f_r) * 2 * 2 * site_bytes
    words = (M + 31) // 32
    n_stage = (min(li["sites"], _abi.BWG_LAT_STAGE_SITES)
               if words >= 512 and not args.no_lds_stage else 0)
    passes = math.ceil(events / M / (_abi.BWG_LAT_PASS_CHUNKS * _abi.BWG_LAT_CHUNK_EVENTS))
    stage_bytes = passes * words * 2 * n_stage * site_bytes / launches_per_step
    hbm_bytes = stage_bytes + (1 - n_stage / li["sites"]) * plane_bytes_we * word_events
    bytes_we = hbm_bytes / word_events
    hbm = hbm_bytes / (launch_ms / 1e3)
    alu_side = {"achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12,
                "unit": "T VALU lane-slots/s", "frac": achieved / VALU_PEAK,
                "slots_per_word_event": slots, "slots_reaction": react, "slots_hop": hop}
    hbm_side = {"achieved": hbm / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": hbm / HBM_PEAK, "bytes_per_word_event": bytes_we,
                "site_plane_bytes_per_word_event": plane_bytes_we, "sites_in_lds": n_stage}
    bind = hbm_side if hbm_side["frac"] >= alu_side["frac"] else alu_side
    out = {
        "metric": "replica-events/sec (bit-parallel lattice, 1 GPU)",
        "value": value, "unit": "replica-events/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32 bit-planes", "data": "synthetic",
        "config": {"workload": "64x64 periodic lattice of Frank reactors, 12 per site on "
                               "average (A uniform 9..15), d=0.1, 2^16 replicas, t_end=20, "
                               "seed 0",
                   "sites": li["sites"], "replicas": M, "t_end": t_end, "site_planes": li["P"],
                   "reaction_planes": li["B_r"], "sites_in_lds_per_word": n_stage},
        "real_events_per_s": st["real_total"] * args.steps / (ms / 1e3),
        "roofline": {"bound": "hbm" if bind is hbm_side else "alu",
                     "achieved": bind["achieved"], "peak": bind["peak"], "unit": bind["unit"],
                     "frac": bind["frac"], "alu": alu_side, "hbm": hbm_side,
                     "traffic": measured_traffic("lat_event_kernel"), "traffic_unit": "B/launch",
                     "kernel": "lat_event_kernel", "kernel_ms": launch_ms,
                     "launches_per_step": launches_per_step, "advance_ms": adv_ms},
    }
    out["parity"] = True
    if not args.no_cpu:
        cb, orc = cpu_baseline_lattice(c, args.cpu_replicas_lattice)
        # the last step's state of the sampled replicas, site by site
        got = np.stack([ens.read_sites(orc.first + k * orc.stride, 1).cpu().numpy()[0]
                        for k in range(orc.n)])
        ev = ens.read_events()[0].cpu().numpy().astype(np.uint64)
        same = (np.array_equal(got, orc.sites) and
                np.array_equal(ev[orc.first::orc.stride][:orc.n], orc.E))
        cb["parity"] = {"replicas": orc.n, "stride": orc.stride, "bit_exact": bool(same)}
        out["cpu_baseline"] = cb
        out["parity"] = bool(same)
    print(json.dumps(out))
    if not out["parity"]:
        print("parity failure: GPU sites differ from the oracle", file=sys.stderr)
        sys.exit(1)


def cpu_baseline_lattice(c, n_rep):
    """The lattice oracle on n_rep replicas spread evenly over the ensemble
    (every component group and both launch bands of the 64 x 64 workload);
    returns the report and the oracle (for the parity check)."""
    from oracle.lattice import OracleLattice
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    stride = max(1, c["replicas"] // n_rep)
    o = OracleLattice(c["net"], c["replicas"], seed=c["seed"], net_id=c["net_id"], first=0,
                      count=n_rep, stride=stride, threads=threads)
    o.init(c["init"])
    t = time.perf_counter()
    o.advance(c["t_end"])
    dt = time.perf_counter() - t
    ev = int(o.E.sum())
    out = {"value": ev / dt, "unit": "replica-events/s", "cores": threads, "kind": "oracle",
           "sample": "%d of %d replicas (every %d-th), full t_end (%d events, %.1f s)"
                     % (n_rep, c["replicas"], stride, ev, dt)}
    out.update(cpu_model())
    return out, o


def bench_batch(args):
    """Uneven batch: 256 Frank networks (N_tot log-uniform 16..4096, replicas
    log-uniform 2^10..2^18, k0 uniform 1e-3..1e-1, t_end uniform 10..200) in
    one persistent launch, tuned (lanes members, grid, order), against the
    same networks one launch each (plain engine and bit-sliced engine)."""
    import torch
    import paper_2412_16613_amd as bwg
    from paper_2412_16613_amd import tune
    from workloads import batch_networks

    cfg = batch_networks()[: args.batch_nets]
    sub = cfg[: args.compare_nets]
    nets = [bwg.Network(c["net"]) for c in cfg]

    def make(engine, members, lanes=()):
        ens = []
        for k, c in enumerate(members):
            e = bwg.Ensemble(nets[k], c["replicas"], seed=c["seed"], net_id=c["net_id"],
                             engine="lanes" if k in lanes else engine)
            e.init(c["init"])
            ens.append(e)
        return ens

    def timed(fn):
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / 1e3

    res, tuned = {}, {}

    def run_batched(members, tag):
        items = [(c["net"], c["replicas"], c["t_end"]) for c in members]
        t0 = time.perf_counter()
        tn = tune.tune(items)
        tuned[tag] = dict(tn, tuning_wall_s=time.perf_counter() - t0)
        ens = make("bitwise", members, set(tn["lanes"]))
        batch = bwg.Batch(ens, waves=tn["waves"], order=tn["order"])
        dt = timed(lambda: batch.advance([c["t_end"] for c in members]))
        ev = sum(e.stats()["events_total"] for e in ens)
        res[tag] = {"s": dt, "replica_events_per_s": ev / dt, "networks": len(members),
                    "lanes_members": len(tn["lanes"])}
        return ev, ens

    events, batched_ens = run_batched(cfg, "batched")
    # the first two words (64 replicas) of every network of the batch against
    # the oracle, which is timed on them as the CPU baseline
    first = [(e.read_counts()[:64].cpu().numpy(),
              e.read_events()[0][:64].cpu().numpy().astype(np.uint64)) for e in batched_ens]
    del batched_ens
    cb, parity = cpu_baseline_batch(cfg, first)
    ev_sub, _ = run_batched(sub, "batched_subset")
    for engine in ("bitwise", "plain"):
        ens = make(engine, sub)
        for e in ens:
            e.prepare()         # run-time compiles outside the timed region
        dt = timed(lambda: [e.advance(c["t_end"]) for e, c in zip(ens, sub)])
        ev = sum(e.stats()["events_total"] for e in ens)
        assert ev == ev_sub
        res["one_per_launch_" + engine] = {"s": dt, "replica_events_per_s": ev / dt,
                                           "networks": len(sub)}
        del ens
    out = {"metric": "replica-events/sec (batched persistent vs one network per launch, 1 GPU)",
           "value": res["batched"]["replica_events_per_s"], "unit": "replica-events/s",
           "n_gpus": 1, "higher_is_better": True, "dtype": "u32 bit-planes",
           "data": "synthetic",
           "config": {"workload": "uneven batch of %d Frank networks" % len(cfg),
                      "replica_events": events, "waves": tuned["batched"]["waves"],
                      "order": tuned["batched"]["order"],
                      "lanes_members": len(tuned["batched"]["lanes"])},
           "tuning": tuned, "results": res,
           "speedup_vs_plain_one_per_launch":
               res["batched_subset"]["replica_events_per_s"] /
               res["one_per_launch_plain"]["replica_events_per_s"],
           "speedup_vs_bitwise_one_per_launch":
               res["batched_subset"]["replica_events_per_s"] /
               res["one_per_launch_bitwise"]["replica_events_per_s"],
           "parity": parity, "cpu_baseline": cb}
    print(json.dumps(out))
    if not parity:
        print("parity failure: batched GPU counts differ from the oracle", file=sys.stderr)
        sys.exit(1)


def cpu_baseline_batch(cfg, gpu_first):
    """The oracle on the first 64 replicas of every network of the batch,
    compared bit for bit with the GPU's (counts, events) in gpu_first."""
    from oracle import ssa
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    ssa.lib()
    ev = 0
    dt = 0.0
    bad = []
    for k, (c, (gc, ge)) in enumerate(zip(cfg, gpu_first)):
        n = min(64, c["replicas"])
        E = ssa.OracleEnsemble(c["net"], c["replicas"], seed=c["seed"], net_id=c["net_id"],
                               first=0, count=n, threads=threads)
        E.init(c["init"])
        t = time.perf_counter()
        E.advance(c["t_end"])
        dt += time.perf_counter() - t
        ev += int(E.E.sum())
        if not (np.array_equal(gc[:n], E.counts) and np.array_equal(ge[:n], E.E)):
            bad.append(k)
    out = {"value": ev / dt, "unit": "replica-events/s", "cores": threads, "kind": "oracle",
           "sample": "first 64 replicas of each of the %d networks, full t_end (%d events, "
                     "%.1f s)" % (len(cfg), ev, dt),
           "parity": {"networks": len(cfg), "replicas_each": 64, "bit_exact": not bad,
                      "mismatched_networks": bad[:16]}}
    out.update(cpu_model())
    return out, not bad


def bench_serve(args):
    """Served stream: Poisson arrivals (200/s for 60 s by default) of Frank
    networks drawn like the uneven batch, 30 % of them lattices of side
    16..64, admitted by HBM budget; well-mixed requests share one continuously
    batched persistent launch, lattices run beside it; p50/p99 latency and
    throughput."""
    from paper_2412_16613_amd.serve import Server, summarize
    from workloads import serve_requests
    reqs = serve_requests(rate=args.rate, duration=args.duration)
    n_lat = sum(1 for r in reqs if r["net"].get("lx"))
    srv = Server(chunk=args.chunk, lanes_events=args.lanes_events)
    res = srv.serve(reqs, real_time=True,
                    progress=lambda m: print("serve " + m, file=sys.stderr, flush=True))
    s = summarize(res, srv.stats)
    out = {"metric": "p50/p99 request latency and replica-events/sec (served stream, 1 GPU)",
           "value": s["replica_events_per_s"], "unit": "replica-events/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": "u32 bit-planes", "data": "synthetic",
           "config": {"workload": "Poisson arrivals %.0f/s for %.0f s, 30%% lattice variants"
                                  % (args.rate, args.duration),
                      "requests": len(reqs), "lattice_requests": n_lat,
                      "chunk_events": args.chunk, "lattice_chunk_events": srv.lattice_chunk,
                      "lanes_events": args.lanes_events},
           "p50_latency_s": s["p50_latency_s"], "p99_latency_s": s["p99_latency_s"],
           "summary": s}
    print(json.dumps(out))


def bench_gain(args):
    """The paper's gain experiment (Sec. 5, Efficiency gain) on the GPU.

    For the paper's network (three reactions, unit weights, ghosts making the
    total N(N-1)/2) at each N_tot: M replicas from independent multinomial
    starts, T iterations each (a fixed number of steps, no time), run by
    (1) the plain engine, one replica per thread with its own random number
    per step (the serial algorithm run M times), (2) the bit-parallel engine
    with a random threshold per replica, and (3) the bit-parallel engine with
    one shared threshold on [0, Z) per step (the paper's variant), (2) and (3)
    at every word width (16, 32 or 64 replicas per thread; the paper's words
    are 64-bit).  Q is the plain engine's time over the bit-parallel one's
    (median of the repeats; each repeat continues the same replicas for
    another T steps).  One table per replica count M: 2^22 fills the GPU, 64
    is the paper's own M (one or two words: a latency measurement)."""
    import torch
    import paper_2412_16613_amd as bwg
    from workloads import paper_network
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    T = args.gain_steps
    widths = [int(x) for x in args.gain_widths.split(",")]
    modes = [("plain", "plain", False, 32)]
    for wb in widths:
        modes += [("bitwise_w%d" % wb, "bitwise", False, wb), ("shared_w%d" % wb, "bitwise", True, wb)]
    tables = []
    for M in [int(x) for x in str(args.gain_replicas).split(",")]:
        rows = []
        for N in [int(x) for x in args.gain_n.split(",")]:
            network = bwg.Network(paper_network(N))
            q = network.quantized()
            row = {"n_tot": N, "B": q["B"], "b": q["b"], "Z": q["z_shared"]}
            for name, engine, shared, wb in modes:
                ens = bwg.Ensemble(network, M, seed=1, net_id=N, engine=engine, device=dev,
                                   shared_threshold=shared, time_kernels=True,
                                   word_bits=wb if engine == "bitwise" else 0)
                ens.init(("multinomial",))
                ens.step(max(1, T // 100))                   # warm-up
                torch.cuda.synchronize()
                ens.kernel_time()
                runs = []
                # the plain engine's time varies by well under 1 % between runs
                for _ in range(1 if engine == "plain" else args.gain_repeats):
                    a = torch.cuda.Event(enable_timing=True)
                    b = torch.cuda.Event(enable_timing=True)
                    a.record()
                    ens.step(T)
                    b.record()
                    torch.cuda.synchronize()
                    runs.append(a.elapsed_time(b) / 1e3)
                s = sorted(runs)[len(runs) // 2]
                kt_ms, kt_n = ens.kernel_time()
                row[name] = {"s": s, "runs_s": runs, "replica_steps_per_s": M * T / s,
                             "kernel_ms": kt_ms / kt_n, "launches": kt_n}
                del ens
            for name, engine, _, _ in modes:
                if engine == "bitwise":
                    row["Q_" + name] = row["plain"]["s"] / row[name]["s"]
            rows.append(row)
            print("gain M=%d N=%d: plain %.4f s, " % (M, N, row["plain"]["s"]) +
                  ", ".join("%s %.4f s (Q %.2f)" % (m[0], row[m[0]]["s"], row["Q_" + m[0]])
                            for m in modes[1:]), file=sys.stderr, flush=True)
        tables.append({"replicas": M, "rows": rows})
    last = tables[0]["rows"][-1]
    out = {"metric": "gain Q = plain-SSA time / bit-parallel shared-threshold time "
                     "(same replicas and steps, 1 GPU)",
           "value": last["Q_shared_w32"] if "Q_shared_w32" in last else None, "unit": "x",
           "n_gpus": 1, "higher_is_better": True,
           "vs_baseline": None, "dtype": "u32 bit-planes", "data": "synthetic",
           "config": {"workload": "paper's Frank network with ghosts, multinomial start, "
                                  "M in %s, T=%d steps, N_tot in %s, word widths %s"
                                  % (args.gain_replicas, T, args.gain_n, args.gain_widths),
                      "value_at": {"replicas": tables[0]["replicas"], "n_tot": last["n_tot"],
                                   "word_bits": 32}},
           "tables": tables}
    print(json.dumps(out))


def bench_gain_cpu(args):
    """The paper's gain experiment as the paper ran it: on one host CPU core,
    64-bit words, M = 64 copies (one word), T = 10^5 iterations, one shared
    threshold per iteration, the paper's network with its ghosts; Q = time of
    the direct method run once per copy over the time of the bit-parallel
    method (cpu_gain/gain_cpu.c; both give the same counts, checked here)."""
    import ctypes
    from oracle import ssa
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2412_16613_amd", "libbwg_cpugain.so"))
    P = ctypes.POINTER(ctypes.c_int32)
    for f in (lib.bwg_cpu_gain_bitwise, lib.bwg_cpu_gain_serial):
        f.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, P,
                      ctypes.c_uint64, P]
        f.restype = ctypes.c_int
    M, T = 64, args.gain_steps
    rows = []
    for N in [int(x) for x in args.gain_n.split(",")]:
        init = np.ascontiguousarray(ssa.init_multinomial(1, N, 0, M, N))
        outs, times = [], []
        for f in (lib.bwg_cpu_gain_serial, lib.bwg_cpu_gain_bitwise):
            out = np.zeros((M, 3), dtype=np.int32)
            best = None
            for _ in range(3):
                t = time.perf_counter()
                rc = f(N, M, 1, N, init.ctypes.data_as(P), T, out.ctypes.data_as(P))
                dt = time.perf_counter() - t
                assert rc == 0
                best = dt if best is None else min(best, dt)
            outs.append(out)
            times.append(best)
        same = bool(np.array_equal(outs[0], outs[1]))
        rows.append({"n_tot": N, "serial_s": times[0], "bitwise_s": times[1],
                     "Q": times[0] / times[1], "same_counts": same})
        print("cpu gain N=%d: serial %.3f s, bitwise %.3f s, Q %.1f" % (N, times[0], times[1],
              times[0] / times[1]), file=sys.stderr, flush=True)
        if not same:
            print("the two CPU engines disagree", file=sys.stderr)
            sys.exit(1)
    out = {"metric": "gain Q = direct-method time / bit-parallel time (host CPU, 1 core, "
                     "64-bit words, M = 64)",
           "value": rows[0]["Q"], "unit": "x", "higher_is_better": True, "vs_baseline": None,
           "dtype": "u64 bit-planes", "data": "synthetic",
           "config": {"workload": "paper's Frank network with ghosts, multinomial start, "
                                  "M=64, T=%d, shared threshold, N_tot in %s" % (T, args.gain_n),
                      "value_at_n_tot": rows[0]["n_tot"]},
           "cpu": cpu_model(), "rows": rows}
    print(json.dumps(out))


def bench_general(args):
    """The general bit-sliced kernels (weights recomputed from the planes at
    every event), compiled at run time for the network and precompiled,
    against the Frank kernel on the Frank workload N_tot = 1024, 2^20
    replicas, and against the plain engine on seeded random 3-species
    networks of order <= 2 (2^20 replicas, about 2000 events each)."""
    import torch
    import paper_2412_16613_amd as bwg
    from workloads import config, frank_network, random_network
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    def rate(net, M, init, horizon, **kw):
        e = bwg.Ensemble(bwg.Network(net), M, seed=1, net_id=2, device=dev, **kw)
        e.init(init)
        e.advance(horizon / 20)                                       # warm-up
        torch.cuda.synchronize()
        ev0 = e.stats()["events_total"]
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        e.advance(horizon)
        b.record()
        torch.cuda.synchronize()
        return (e.stats()["events_total"] - ev0) / (a.elapsed_time(b) / 1e3)

    c = config("c1")
    rows = {"frank1024": {
        "frank_kernel": rate(c["net"], c["replicas"], c["init"], c["t_end"] / 4),
        "plain": rate(c["net"], c["replicas"], c["init"], c["t_end"] / 4, engine="plain")}}
    rows["frank1024"]["compiled_kernel"] = rate(c["net"], c["replicas"], c["init"],
                                                c["t_end"] / 4, generic=True)
    rows["frank1024"]["general_kernel"] = rate(c["net"], c["replicas"], c["init"],
                                               c["t_end"] / 4, generic=True, jit=False)
    for seed, n_tot, n_r in ((1, 50, 7), (2, 200, 12), (8, 400, 5)):
        net = random_network(seed, n_tot, n_r)
        t = 2000.0 / bwg.Network(net).quantized()["Lambda"]
        rows["random_s%d_n%d_r%d" % (seed, n_tot, n_r)] = {
            "compiled_kernel": rate(net, 1 << 20, ("multinomial",), t),
            "general_kernel": rate(net, 1 << 20, ("multinomial",), t, jit=False),
            "plain": rate(net, 1 << 20, ("multinomial",), t, engine="plain")}
    for r in rows.values():
        r["compiled_over_plain"] = r["compiled_kernel"] / r["plain"]
        r["general_over_plain"] = r["general_kernel"] / r["plain"]
    # Frank networks whose weights match no precompiled variant: the Frank
    # kernels compiled for the network against the precompiled run-time
    # weight ones (the warm-up advance includes the compile)
    frank_rt = {}
    for n_tot, k0 in ((1024, 0.02), (200, 0.03)):
        net = frank_network(n_tot, k0=k0)
        t = 2000.0 / bwg.Network(net).quantized()["Lambda"]
        r = {"compiled_frank_kernel": rate(net, 1 << 20, ("multinomial",), t),
             "run_time_frank_kernel": rate(net, 1 << 20, ("multinomial",), t, jit=False),
             "plain": rate(net, 1 << 20, ("multinomial",), t, engine="plain")}
        r["compiled_over_run_time"] = r["compiled_frank_kernel"] / r["run_time_frank_kernel"]
        frank_rt["frank%d_k0_%g" % (n_tot, k0)] = r
    out = {"metric": "replica-events/sec of the general bit-sliced kernels (1 GPU)",
           "value": rows["frank1024"]["compiled_kernel"], "unit": "replica-events/s",
           "n_gpus": 1, "higher_is_better": True, "vs_baseline": None,
           "dtype": "u32 bit-planes", "data": "synthetic",
           "config": {"workload": "Frank N_tot=1024 and seeded random 3-species networks, "
                                  "2^20 replicas"},
           "rows": rows, "frank_run_time_weights": frank_rt}
    print(json.dumps(out))


def bench_trajectory(args):
    """The paper's trajectory figure as a workload (Sec. 5, Sec. 6): its
    network at N_tot = 32 with the shared threshold and shared time, 2^22
    replicas from multinomial starts around the racemic state, recorded on a
    grid of 100 times up to t = 2 (L, D, A of 64 replicas after each) with
    every replica's first grid time at |N_L - N_D| >= 24; against the rate of
    one advance to t = 2 (one budget instead of 100, so another count)."""
    import torch
    import paper_2412_16613_amd as bwg
    from workloads import paper_network
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    N, M, t_end, n_grid, thr = 32, 1 << 22, 2.0, 100, 24
    network = bwg.Network(paper_network(N))
    grid = [t_end * (k + 1) / n_grid for k in range(n_grid)]
    sel = list(range(0, M, M // 64))

    def timed(fn):
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        out = fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / 1e3, out

    def make():
        e = bwg.Ensemble(network, M, seed=7, net_id=1, device=dev, shared_threshold=True)
        e.init(("multinomial",))
        return e

    make().record(grid[:10], sel, threshold=thr)                     # warm-up
    e = make()
    s_rec, (traj, first) = timed(lambda: e.record(grid, sel, threshold=thr))
    ev = e.stats()["events_total"]
    f = make()
    s_adv, _ = timed(lambda: f.advance(t_end))
    ev_adv = f.stats()["events_total"]          # one budget instead of 100: another count
    counts = e.read_counts().cpu().numpy()
    first = first.cpu().numpy()
    hit = first >= 0
    out = {"metric": "replica-events/sec recording trajectories (1 GPU)",
           "value": ev / s_rec, "unit": "replica-events/s", "n_gpus": 1,
           "higher_is_better": True, "vs_baseline": None, "dtype": "u32 bit-planes",
           "data": "synthetic",
           "config": {"workload": "paper's network N_tot=32 with ghosts, shared threshold and "
                                  "time, 2^22 replicas, multinomial start, 100 grid times to "
                                  "t=2, 64 recorded replicas, first passage at |L-D| >= 24"},
           "seconds": s_rec, "one_advance_seconds": s_adv,
           "one_advance_replica_events_per_s": ev_adv / s_adv,
           "recording_cost_factor": (ev_adv / s_adv) / (ev / s_rec),
           "homochiral_fraction": float(hit.mean()),
           "L_fraction_of_homochiral": float((counts[hit, 0] > counts[hit, 1]).mean()),
           "median_first_passage_time": float(grid[int(np.median(first[hit]))]) if hit.any()
           else None}
    print(json.dumps(out))


def cpu_model():
    """Host CPU model name (from /proc/cpuinfo) and logical CPU count."""
    name = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": name, "host_logical_cpus": os.cpu_count()}


def cpu_baseline(net, c, n_rep):
    """The CPU oracle on the first n_rep replicas of the same workload;
    returns the report and the oracle ensemble (for the parity check)."""
    from oracle import ssa
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    ssa.lib()
    E = ssa.OracleEnsemble(net, c["replicas"], seed=c["seed"], net_id=c["net_id"], first=0,
                           count=n_rep, threads=threads)
    E.init(c["init"])
    t = time.perf_counter()
    E.advance(c["t_end"])
    dt = time.perf_counter() - t
    ev = int(E.E.sum())
    out = {"value": ev / dt, "unit": "replica-events/s", "cores": threads, "kind": "oracle",
           "sample": "first %d of %d replicas, full t_end (%d events, %.1f s)"
                     % (n_rep, c["replicas"], ev, dt)}
    out.update(cpu_model())
    return out, E


if __name__ == "__main__":
    main()
