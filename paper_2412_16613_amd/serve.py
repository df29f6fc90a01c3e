"""Continuous-batching server for ensemble requests.

A request is (arrival time, network, replicas, seed, net id, initial state,
t_end).  The server admits arrived requests in arrival order while their
device state fits the HBM budget and a member slot is free; an admitted
request gets its own device-resident ensemble and its event budgets for the
whole horizon are drawn at once.  Well-mixed requests join the persistent
batch: every well-mixed pass runs at most `chunk` events per word of every
resident request, so long chains yield to newly admitted requests between
passes and their work overlaps in one launch.  Lattice requests run their
own launches (at most `lattice_chunk` events of their component sequence per
lattice pass), spread round-robin over `lattice_streams` streams beside the
persistent launch: a small lattice ensemble's advance is bound by its own
layer-after-layer latency, so several run at once.  The two kinds of pass
are queued independently (up to `depth` of each in flight), so neither
waits for the other.  A request completes when its pending-event bound
reaches zero (a host-side bound: no device query); its histogram (and, if
asked, its counts) and its event total are copied to pinned host memory
behind its last pass, and a HIP event marks the end of every pass on each of
its streams.  The host does not wait for a pass it has just enqueued: it
admits arrivals and enqueues the next passes while earlier ones run, and
retires a pass (its requests' latency, completion - arrival, recorded and
their memory returned to the budget) once its events have completed.

Results do not depend on the mix: every draw is keyed by (seed, net id,
replica, event), so a request served among others gives bit for bit the
result it gives alone.

Failures stay with their request.  Every result has a status: "ok"; "error"
for a request the library refuses (an invalid network or initial state) or
whose launch fails (the message in "error"; a failed persistent pass fails
the well-mixed requests it ran); "rejected" for a request whose state alone
exceeds the HBM budget or the batch's work items; "cancelled" for a request
not complete `deadline` seconds after its arrival (a request key, optional).
A request leaves the batch before its memory is returned, and only once the
work enqueued for it has completed.
"""

import collections
import json
import time

import numpy as np

import paper_2412_16613_amd as bwg


class Server:
    def __init__(self, hbm_budget=64 << 30, chunk=4096, max_members=1024,
                 max_items=1 << 19, waves=2048, n_bins=256, keep_counts=False,
                 lattice_chunk=1 << 17, depth=2, lanes_events=0, lattice_streams=3,
                 device="cuda", log=None):
        import torch
        self.torch = torch
        # log: a path or a text stream; one JSON line per finished request
        # (status, times, latency, replicas, events run or the error) and a
        # last line with the summary of each serve call
        self.log = log
        # well-mixed requests expecting at least this many events per replica
        # run on the lanes engine (one replica per thread: a word's chain of
        # events an order of magnitude shorter, at about twice the work per
        # replica-event); 0 (the default: served at 200 arrivals/s it changes
        # the latencies by a few per cent and costs throughput at saturation)
        # keeps every request on bit-sliced words
        self.lanes_events = float(lanes_events)
        self.device = torch.device(device)
        self.lattice_chunk = int(lattice_chunk)
        self.lattice_streams = max(1, int(lattice_streams))
        self.sides = None
        self.hbm_budget = int(hbm_budget)
        self.chunk = int(chunk)
        self.max_members = int(max_members)
        self.max_items = int(max_items)
        self.waves = int(waves)
        self.n_bins = int(n_bins)
        self.keep_counts = keep_counts
        self.depth = max(1, int(depth))
        self._nets = {}
        self.batch = None

    def _network(self, net):
        key = (net["n_tot"], tuple(net["rates"]), tuple(map(tuple, net["reactants"])),
               tuple(map(tuple, net["products"])), bool(net.get("exact_integer")),
               net.get("lx", 0), net.get("ly", 0), tuple(net.get("hop_rates", ())),
               net.get("site_planes", 0))
        n = self._nets.get(key)
        if n is None:
            n = bwg.Network(net)
            self._nets[key] = n
        return n

    @staticmethod
    def _items(M, lanes):
        """Work items of a member in the persistent batch: 64-word items, or
        2-word items on the lanes engine."""
        words = (M + 31) // 32
        return (words + 1) // 2 if lanes else (words + 63) // 64

    def serve(self, requests, real_time=True, max_seconds=None, pass_time=1.0, progress=None,
              progress_every=20.0):
        """Serve requests (dicts with arrival, net, replicas, seed, net_id,
        init, t_end); returns one result dict per completed request.  With
        real_time=False the clock is simulated: it advances by pass_time per
        loop that enqueues passes (deterministic interleaving, for tests).
        progress, if given, is called with a status string about every
        progress_every seconds of wall time."""
        torch = self.torch
        reqs = sorted(requests, key=lambda r: r["arrival"])
        incoming = collections.deque(reqs)
        waiting = collections.deque()
        active = []           # dicts: req, ens, bytes, items, lattice, stream, admitted
        used_bytes = 0
        used_items = 0
        results = []
        stats = dict(passes=0, lattice_passes=0, max_active=0, replica_events=0)
        if self.batch is None:
            self.batch = bwg.Batch([], waves=self.waves, max_ensembles=self.max_members,
                                   max_items=self.max_items, device=self.device)
        if self.sides is None:
            self.sides = [torch.cuda.Stream(self.device) for _ in range(self.lattice_streams)]
        main = torch.cuda.current_stream(self.device)
        next_side = 0

        cancelling = []       # (event, entry, status, message): memory back once done

        def log_line(obj):
            if isinstance(self.log, str):
                with open(self.log, "a") as f:
                    f.write(json.dumps(obj) + "\n")
            elif self.log is not None:
                self.log.write(json.dumps(obj) + "\n")

        def record(res, events=None):
            results.append(res)
            if self.log is not None:
                line = {k: res[k] for k in ("id", "status", "arrival", "admitted", "completed",
                                            "latency", "replicas")}
                line["id"] = int(line["id"])
                if events is not None:
                    line["events"] = int(events)
                if res.get("error") is not None:
                    line["error"] = res["error"]
                log_line(line)

        def closed(r, status, message, t_admitted=None):
            t = clock() if real_time else sim_now
            record(dict(id=r["net_id"], arrival=r["arrival"], admitted=t_admitted,
                        completed=t, latency=t - r["arrival"], status=status,
                        error=message, replicas=r["replicas"]))

        def expired(r, now):
            d = r.get("deadline")
            return d is not None and now > r["arrival"] + d

        def drop(entries, status, message):
            """Take entries out of service; their memory returns to the budget
            once the work already enqueued on their stream has completed."""
            nonlocal active
            ids = {id(a) for a in entries}
            active = [a for a in active if id(a) not in ids]
            if any(not a["lattice"] for a in entries):
                self.batch.set_members([a["ens"] for a in active if not a["lattice"]])
            for a in entries:
                ev = torch.cuda.Event()
                ev.record(a["stream"])
                cancelling.append((ev, a, status, message))

        def to_host(t):
            h = torch.empty(t.shape, dtype=t.dtype, pin_memory=True)
            h.copy_(t, non_blocking=True)
            return h

        # passes in flight: well-mixed ones on the main stream, lattice ones
        # on the side streams; each entry: events, requests finished, order
        wm_inflight = collections.deque()
        lat_inflight = collections.deque()
        order = 0
        t0 = time.perf_counter()
        clock = (lambda: time.perf_counter() - t0) if real_time else None
        sim_now = 0.0

        def retire(p):
            """Requests of a completed pass: results, memory back to the budget."""
            nonlocal used_bytes, used_items
            t_done = clock() if real_time else p["sim_done"]
            for a in p["done"]:
                r = a["req"]
                res = dict(id=r["net_id"], arrival=r["arrival"], admitted=a["admitted"],
                           completed=t_done, latency=t_done - r["arrival"], status="ok",
                           hist=a["hist_host"].numpy().copy(), replicas=r["replicas"])
                if self.keep_counts:
                    res["counts"] = a["counts_host"].numpy().copy()
                events = int(a["events_host"].numpy()[0])
                stats["replica_events"] += events
                record(res, events)
                used_bytes -= a["bytes"]
                used_items -= a["items"]

        def readouts(done):
            for a in done:
                with torch.cuda.stream(a["stream"]):
                    a["hist_host"] = to_host(a["ens"].histogram(self.n_bins))
                    a["events_host"] = to_host(a["ens"].read_events()[0].sum().view(1))
                    if self.keep_counts:
                        a["counts_host"] = to_host(a["ens"].read_counts())

        def ready(p):
            return all(ev.query() for ev in p["ev"])

        wm_changed = True     # the batch may still list an earlier call's members
        next_report = progress_every
        while incoming or waiting or active or wm_inflight or lat_inflight or cancelling:
            if progress is not None and time.perf_counter() - t0 >= next_report:
                next_report += progress_every
                progress("t=%.0fs: %d done, %d active, %d waiting, %d not yet arrived, %d passes"
                         % (time.perf_counter() - t0, len(results), len(active), len(waiting),
                            len(incoming), stats["passes"] + stats["lattice_passes"]))
            now = clock() if real_time else sim_now
            if max_seconds is not None and now > max_seconds:
                break
            while incoming and incoming[0]["arrival"] <= now:
                waiting.append(incoming.popleft())
            # deadlines: waiting requests leave the queue, active ones the service
            for r in [r for r in waiting if expired(r, now)]:
                waiting.remove(r)
                closed(r, "cancelled", "deadline passed before admission")
            late = [a for a in active if expired(a["req"], now)]
            if late:
                drop(late, "cancelled", "deadline passed")
                wm_changed = True
            while waiting and len(active) < self.max_members:
                r = waiting[0]
                try:
                    net = self._network(r["net"])
                    lattice = net.is_lattice
                    lanes = (not lattice and self.lanes_events > 0 and
                             net.quantized()["Lambda"] * r["t_end"] >= self.lanes_events)
                    nbytes = bwg.Ensemble.bytes_needed(
                        net, r["replicas"], engine="lanes" if lanes else "bitwise")
                except (bwg.BwgError, ValueError, KeyError, TypeError) as exc:
                    waiting.popleft()
                    closed(r, "error", str(exc))
                    continue
                items = 0 if lattice else self._items(r["replicas"], lanes)
                if nbytes > self.hbm_budget or items > self.max_items:
                    waiting.popleft()
                    closed(r, "rejected", "state of %d bytes and %d work items exceeds the "
                           "server's budget" % (nbytes, items))
                    continue
                busy = active or wm_inflight or lat_inflight or cancelling
                if busy and (used_bytes + nbytes > self.hbm_budget
                             or used_items + items > self.max_items):
                    break
                waiting.popleft()
                # a lattice ensemble lives on its side stream from its first call
                stream = main
                if lattice:
                    stream = self.sides[next_side % len(self.sides)]
                    next_side += 1
                try:
                    ens = bwg.Ensemble(net, r["replicas"], seed=r["seed"], net_id=r["net_id"],
                                       device=self.device, engine="lanes" if lanes else "bitwise")
                    with torch.cuda.stream(stream):
                        ens.init(r["init"])
                        ens.schedule(r["t_end"])
                except (bwg.BwgError, ValueError, KeyError, TypeError) as exc:
                    # whatever init enqueued finishes before the buffer can
                    # be handed out again
                    stream.synchronize()
                    closed(r, "error", str(exc))
                    continue
                active.append(dict(req=r, ens=ens, bytes=nbytes, items=items, lattice=lattice,
                                   stream=stream, admitted=clock() if real_time else now))
                used_bytes += nbytes
                used_items += items
                wm_changed = wm_changed or not lattice
            stats["max_active"] = max(stats["max_active"], len(active))
            enqueued = False
            wm = [a for a in active if not a["lattice"]]
            lat = [a for a in active if a["lattice"]]
            if wm and len(wm_inflight) < self.depth:
                if wm_changed:
                    self.batch.set_members([a["ens"] for a in wm])
                try:
                    self.batch.run(self.chunk)
                except bwg.BwgError as exc:
                    # the pass's members are in an unknown state: all fail
                    drop(wm, "error", "persistent pass failed: %s" % exc)
                    wm_changed = True
                    continue
                done = [a for a in wm if a["ens"].pending() == 0]
                readouts(done)
                ev = torch.cuda.Event()
                ev.record(main)
                wm_inflight.append(dict(ev=[ev], done=done, order=order))
                order += 1
                stats["passes"] += 1
                enqueued = True
                wm_changed = False
                if done:
                    # out of the batch before their ensembles can be freed
                    active = [a for a in active if a["lattice"] or a["ens"].pending() != 0]
                    self.batch.set_members([a["ens"] for a in active if not a["lattice"]])
            if lat and len(lat_inflight) < self.depth:
                streams = []
                failed = []
                for a in lat:
                    try:
                        with torch.cuda.stream(a["stream"]):
                            a["ens"].run(self.lattice_chunk)
                    except bwg.BwgError as exc:
                        failed.append((a, str(exc)))
                        continue
                    if a["stream"] not in streams:
                        streams.append(a["stream"])
                for a, msg in failed:
                    drop([a], "error", "lattice pass failed: %s" % msg)
                lat = [a for a in lat if all(a is not f for f, _ in failed)]
                done = [a for a in lat if a["ens"].pending() == 0]
                readouts(done)
                evs = []
                for st in streams:
                    ev = torch.cuda.Event()
                    ev.record(st)
                    evs.append(ev)
                lat_inflight.append(dict(ev=evs, done=done, order=order))
                order += 1
                stats["lattice_passes"] += 1
                enqueued = True
                if done:
                    active = [a for a in active if not a["lattice"] or a["ens"].pending() != 0]
            if enqueued and not real_time:
                sim_now += pass_time
            for q in (wm_inflight, lat_inflight):
                for p in q:
                    p.setdefault("sim_done", sim_now)
            if not enqueued and not wm_inflight and not lat_inflight:
                if incoming and not waiting and not active:
                    if real_time:
                        time.sleep(max(0.0, incoming[0]["arrival"] - clock()))
                    else:
                        sim_now = incoming[0]["arrival"]
                    continue
            # retire finished passes; when nothing could be enqueued, wait for
            # the oldest pass in flight
            retired = False
            for q in (wm_inflight, lat_inflight):
                while q and ready(q[0]):
                    retire(q.popleft())
                    retired = True
            still = []
            for ev, a, status, msg in cancelling:
                if ev.query():
                    closed(a["req"], status, msg, a["admitted"])
                    used_bytes -= a["bytes"]
                    used_items -= a["items"]
                    retired = True
                else:
                    still.append((ev, a, status, msg))
            cancelling = still
            if not enqueued and not retired and cancelling and not (wm_inflight or
                                                                    lat_inflight):
                cancelling[0][0].synchronize()
                continue
            if not enqueued and not retired and (wm_inflight or lat_inflight):
                heads = [q for q in (wm_inflight, lat_inflight) if q]
                q = min(heads, key=lambda d: d[0]["order"])
                for ev in q[0]["ev"]:
                    ev.synchronize()
                retire(q.popleft())
        stats["wall_s"] = (time.perf_counter() - t0)
        self.stats = stats
        if self.log is not None:
            log_line(dict(summary=summarize(results, stats)))
            if not isinstance(self.log, str):
                self.log.flush()
        return results


def summarize(results, stats):
    ok = [r for r in results if r.get("status", "ok") == "ok"]
    lat = np.array([r["latency"] for r in ok])
    return dict(requests=len(ok),
                failed={s: sum(r.get("status") == s for r in results)
                        for s in ("error", "rejected", "cancelled")},
                p50_latency_s=float(np.percentile(lat, 50)) if len(lat) else None,
                p99_latency_s=float(np.percentile(lat, 99)) if len(lat) else None,
                mean_latency_s=float(lat.mean()) if len(lat) else None,
                replica_events_per_s=stats["replica_events"] / stats["wall_s"],
                passes=stats["passes"], lattice_passes=stats.get("lattice_passes", 0),
                max_active=stats["max_active"],
                wall_s=stats["wall_s"])
