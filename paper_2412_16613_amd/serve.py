"""Continuous-batching server for ensemble requests.

A request is (arrival time, network, replicas, seed, net id, initial state,
t_end).  The server admits arrived requests in arrival order while their
device state fits the HBM budget and a member slot is free; an admitted
request gets its own device-resident ensemble and its event budgets for the
whole horizon are drawn at once.  Well-mixed requests join the persistent
batch: every pass runs at most `chunk` events per word of every resident
request, so long chains yield to newly admitted requests between passes and
their work overlaps in one launch.  Lattice requests run their own launches
(at most `lattice_chunk` events of their component sequence per pass) on a
second stream, beside the persistent launch.  A request completes when its
pending-event bound reaches zero; its histogram (and, if asked, its counts)
is read back, the latency (completion - arrival) recorded and its memory
returned to the budget.

Results do not depend on the mix: every draw is keyed by (seed, net id,
replica, event), so a request served among others gives bit for bit the
result it gives alone.
"""

import collections
import time

import numpy as np

import paper_2412_16613_amd as bwg


class Server:
    def __init__(self, hbm_budget=64 << 30, chunk=4096, max_members=1024,
                 max_items=1 << 16, waves=2048, n_bins=256, keep_counts=False,
                 lattice_chunk=1 << 17, device="cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.lattice_chunk = int(lattice_chunk)
        self.side = None
        self.hbm_budget = int(hbm_budget)
        self.chunk = int(chunk)
        self.max_members = int(max_members)
        self.max_items = int(max_items)
        self.waves = int(waves)
        self.n_bins = int(n_bins)
        self.keep_counts = keep_counts
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
    def _items(M):
        return (((M + 31) // 32) + 63) // 64

    def serve(self, requests, real_time=True, max_seconds=None, pass_time=1.0):
        """Serve requests (dicts with arrival, net, replicas, seed, net_id,
        init, t_end); returns one result dict per completed request.  With
        real_time=False the clock is simulated: it advances by pass_time per
        pass (deterministic interleaving, for tests)."""
        torch = self.torch
        reqs = sorted(requests, key=lambda r: r["arrival"])
        incoming = collections.deque(reqs)
        waiting = collections.deque()
        active = []           # dicts: req, ens, bytes, items, lattice, admitted
        used_bytes = 0
        used_items = 0
        results = []
        stats = dict(passes=0, max_active=0, replica_events=0)
        if self.batch is None:
            self.batch = bwg.Batch([], waves=self.waves, max_ensembles=self.max_members,
                                   max_items=self.max_items, device=self.device)
        if self.side is None:
            self.side = torch.cuda.Stream(self.device)
        main = torch.cuda.current_stream(self.device)

        def well_mixed(act):
            return [a["ens"] for a in act if not a["lattice"]]
        t0 = time.perf_counter()
        clock = (lambda: time.perf_counter() - t0) if real_time else None
        sim_now = 0.0
        while incoming or waiting or active:
            now = clock() if real_time else sim_now
            if max_seconds is not None and now > max_seconds:
                break
            while incoming and incoming[0]["arrival"] <= now:
                waiting.append(incoming.popleft())
            changed = False
            while waiting and len(active) < self.max_members:
                r = waiting[0]
                net = self._network(r["net"])
                lattice = net.is_lattice
                ens = bwg.Ensemble(net, r["replicas"], seed=r["seed"], net_id=r["net_id"],
                                   device=self.device)
                nbytes = ens.state_bytes
                items = 0 if lattice else self._items(r["replicas"])
                if active and (used_bytes + nbytes > self.hbm_budget
                               or used_items + items > self.max_items):
                    del ens
                    break
                waiting.popleft()
                # lattice ensembles live on the side stream from their first call
                with torch.cuda.stream(self.side if lattice else main):
                    ens.init(r["init"])
                    ens.schedule(r["t_end"])
                active.append(dict(req=r, ens=ens, bytes=nbytes, items=items, lattice=lattice,
                                   admitted=clock() if real_time else now))
                used_bytes += nbytes
                used_items += items
                changed = True
            if not active:
                if incoming:
                    if real_time:
                        time.sleep(max(0.0, incoming[0]["arrival"] - clock()))
                    else:
                        sim_now = incoming[0]["arrival"]
                continue
            stats["max_active"] = max(stats["max_active"], len(active))
            if changed:
                self.batch.set_members(well_mixed(active))
            if any(not a["lattice"] for a in active):
                self.batch.run(self.chunk)
            with torch.cuda.stream(self.side):
                for a in active:
                    if a["lattice"]:
                        a["ens"].run(self.lattice_chunk)
            stats["passes"] += 1
            done = [a for a in active if a["ens"].pending() == 0]
            if done:
                for a in done:
                    with torch.cuda.stream(self.side if a["lattice"] else main):
                        a["hist_dev"] = a["ens"].histogram(self.n_bins)
                        if self.keep_counts:
                            a["counts_dev"] = a["ens"].read_counts()
            main.synchronize()
            self.side.synchronize()
            if not real_time:
                sim_now += pass_time
            if done:
                t_done = clock() if real_time else sim_now
                for a in done:
                    r = a["req"]
                    hist = a["hist_dev"].cpu().numpy()
                    res = dict(id=r["net_id"], arrival=r["arrival"], admitted=a["admitted"],
                               completed=t_done, latency=t_done - r["arrival"], hist=hist,
                               replicas=r["replicas"])
                    if self.keep_counts:
                        res["counts"] = a["counts_dev"].cpu().numpy()
                    stats["replica_events"] += a["ens"].stats()["events_total"]
                    results.append(res)
                    used_bytes -= a["bytes"]
                    used_items -= a["items"]
                active = [a for a in active if a["ens"].pending() != 0]
                self.batch.set_members(well_mixed(active))
        stats["wall_s"] = (time.perf_counter() - t0)
        self.stats = stats
        return results


def summarize(results, stats):
    lat = np.array([r["latency"] for r in results])
    return dict(requests=len(results),
                p50_latency_s=float(np.percentile(lat, 50)) if len(lat) else None,
                p99_latency_s=float(np.percentile(lat, 99)) if len(lat) else None,
                mean_latency_s=float(lat.mean()) if len(lat) else None,
                replica_events_per_s=stats["replica_events"] / stats["wall_s"],
                passes=stats["passes"], max_active=stats["max_active"],
                wall_s=stats["wall_s"])
