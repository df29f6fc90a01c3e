"""Continuous batching: results alone and in the mix are bit-identical."""

import json

import numpy as np
import pytest

import paper_2412_16613_amd as bwg
from paper_2412_16613_amd.serve import Server, summarize
from oracle import ssa
from workloads import frank_network, serve_requests

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _requests():
    nets = [(frank_network(16, k0=0.05), 33, 10.0), (frank_network(100), 1000, 3.0),
            (frank_network(300, k0=0.003), 2048, 1.5), (frank_network(1000, k0=0.02), 97, 0.6),
            (frank_network(40, k0=0.1), 5000, 6.0), (frank_network(2000, k0=0.001), 64, 0.3),
            (frank_network(24, k0=0.02), 700, 8.0), (frank_network(64), 4096, 2.0)]
    out = []
    for k, (net, M, t) in enumerate(nets):
        out.append(dict(arrival=0.7 * k, net=net, replicas=M, seed=17, net_id=500 + k,
                        init=("fixed", (0, 0, net["n_tot"])), t_end=t))
    return out


@pytest.mark.parametrize("lanes_events", [0, 1e5, 1])
def test_served_results_equal_results_alone(torch, lanes_events):
    # lanes_events: none, the long chains, or every well-mixed request on
    # the lanes engine (2-word items in the persistent batch)
    reqs = _requests()
    srv = Server(chunk=200, max_members=4, keep_counts=True, lanes_events=lanes_events)
    res = srv.serve(reqs, real_time=False, pass_time=1.0)
    assert len(res) == len(reqs)
    assert srv.stats["max_active"] >= 2          # the mix really overlapped
    by_id = {r["id"]: r for r in res}
    for r in reqs:
        e = bwg.Ensemble(bwg.Network(r["net"]), r["replicas"], seed=r["seed"],
                         net_id=r["net_id"])
        e.init(r["init"]).advance(r["t_end"])
        h = e.histogram(256).cpu().numpy()
        c = e.read_counts().cpu().numpy()
        got = by_id[r["net_id"]]
        np.testing.assert_array_equal(got["hist"], h)
        np.testing.assert_array_equal(got["counts"], c)


def test_served_small_requests_match_oracle(torch):
    reqs = _requests()[:2]
    res = Server(chunk=150, keep_counts=True).serve(reqs, real_time=False)
    for r, got in zip(reqs, sorted(res, key=lambda x: x["id"])):
        o = ssa.OracleEnsemble(r["net"], r["replicas"], seed=r["seed"], net_id=r["net_id"])
        o.init(r["init"])
        o.advance(r["t_end"])
        np.testing.assert_array_equal(got["counts"], o.counts)


def _lattice_requests():
    reqs = _requests()[:4]
    lat = [(frank_network(12, lx=8, ly=8, hop=0.1, site_planes=4), 300, 1.5),
           (frank_network(12, lx=16, ly=12, hop=0.1, site_planes=4), 70, 0.4),
           (frank_network(12, lx=5, ly=7, k0=0.05, hop=0.3, site_planes=4), 2100, 2.0)]
    for k, (net, M, t) in enumerate(lat):
        reqs.append(dict(arrival=0.5 + 0.9 * k, net=net, replicas=M, seed=21, net_id=700 + k,
                         init=("uniform_site", 9, 15), t_end=t))
    return reqs


def test_lattice_requests_in_the_mix(torch):
    """Lattice requests run beside the persistent batch on a second stream;
    every request's histogram and totals equal its run alone, and the
    lattice ones equal the lattice oracle."""
    from oracle.lattice import OracleLattice
    reqs = _lattice_requests()
    srv = Server(chunk=200, max_members=5, keep_counts=True, lattice_chunk=8192)
    res = srv.serve(reqs, real_time=False, pass_time=1.0)
    assert len(res) == len(reqs)
    assert srv.stats["max_active"] >= 3
    by_id = {r["id"]: r for r in res}
    for r in reqs:
        e = bwg.Ensemble(bwg.Network(r["net"]), r["replicas"], seed=r["seed"],
                         net_id=r["net_id"])
        e.init(r["init"]).advance(r["t_end"])
        got = by_id[r["net_id"]]
        np.testing.assert_array_equal(got["hist"], e.histogram(256).cpu().numpy())
        np.testing.assert_array_equal(got["counts"], e.read_counts().cpu().numpy())
        if r["net"].get("lx"):
            o = OracleLattice(r["net"], r["replicas"], seed=r["seed"], net_id=r["net_id"],
                              threads=8)
            o.init(r["init"])
            o.advance(r["t_end"])
            np.testing.assert_array_equal(got["counts"], o.totals())


def test_admission_respects_the_memory_budget(torch):
    reqs = _requests()
    one = max(bwg.Ensemble(bwg.Network(r["net"]), r["replicas"]).state_bytes for r in reqs)
    srv = Server(hbm_budget=one + 1, chunk=300)
    res = srv.serve(reqs, real_time=False)
    assert len(res) == len(reqs)
    assert srv.stats["max_active"] <= 2


def test_real_time_stream_reports_latency(torch):
    reqs = [r for r in serve_requests(rate=50.0, duration=1.0, lattice_frac=0.0)]
    for r in reqs:           # keep the test short: small horizons and sizes
        r["t_end"] = r["t_end"] / 100.0
        r["replicas"] = min(r["replicas"], 4096)
    srv = Server(chunk=1024)
    res = srv.serve(reqs, real_time=True)
    s = summarize(res, srv.stats)
    assert len(res) == len(reqs)
    assert all(r["latency"] >= 0 for r in res)
    assert s["p99_latency_s"] >= s["p50_latency_s"]


def _alone(r, keep_counts=True):
    e = bwg.Ensemble(bwg.Network(r["net"]), r["replicas"], seed=r["seed"], net_id=r["net_id"])
    e.init(r["init"]).advance(r["t_end"])
    return e.histogram(256).cpu().numpy(), e.read_counts().cpu().numpy()


def test_failures_stay_with_their_request(torch, monkeypatch, tmp_path):
    """An invalid network, an invalid start, a request larger than the whole
    budget, one past its deadline and a lattice whose launch fails (injected)
    each end with their own status; every other request completes with
    the result it gives alone."""
    reqs = _lattice_requests()
    base = len(reqs)
    bad_rates = dict(frank_network(16), rates=[-1.0] + frank_network(16)["rates"][1:])
    bad = [dict(arrival=0.2, net=bad_rates, replicas=100, seed=1, net_id=900,
                init=("fixed", (0, 0, 16)), t_end=1.0),
           dict(arrival=0.4, net=frank_network(16), replicas=100, seed=1, net_id=901,
                init=("fixed", (0, 0, 15)), t_end=1.0),
           dict(arrival=0.6, net=frank_network(64), replicas=1 << 31, seed=1, net_id=902,
                init=("fixed", (0, 0, 64)), t_end=1.0),
           dict(arrival=0.8, net=frank_network(64), replicas=4096, seed=1, net_id=903,
                init=("fixed", (0, 0, 64)), t_end=1e4, deadline=2.5)]
    orig = bwg.Ensemble.run

    def flaky(self, max_events=0):
        if self.network.net.get("lx") == 16:
            raise bwg.BwgError(_abi_edevice(), "injected launch failure")
        return orig(self, max_events)

    monkeypatch.setattr(bwg.Ensemble, "run", flaky)
    log = tmp_path / "serve.jsonl"
    srv = Server(hbm_budget=8 << 30, chunk=200, max_members=6, keep_counts=True,
                 lattice_chunk=8192, log=str(log))
    res = srv.serve(reqs + bad, real_time=False, pass_time=1.0)
    by_id = {r["id"]: r for r in res}
    # the log: one JSON line per request, then the summary
    lines = [json.loads(x) for x in log.read_text().splitlines()]
    assert [x["id"] for x in lines[:-1]] == [r["id"] for r in res]
    assert all(x["status"] == r["status"] for x, r in zip(lines, res))
    assert all(("events" in x) == (x["status"] == "ok") for x in lines[:-1])
    assert lines[-1]["summary"]["failed"] == dict(error=3, rejected=1, cancelled=1)
    assert len(res) == base + len(bad)
    assert by_id[900]["status"] == "error" and "rate" in by_id[900]["error"]
    assert by_id[901]["status"] == "error"
    assert by_id[902]["status"] == "rejected"
    assert by_id[903]["status"] == "cancelled"
    assert by_id[701]["status"] == "error" and "injected" in by_id[701]["error"]
    for r in reqs:
        if r["net_id"] == 701:
            continue
        got = by_id[r["net_id"]]
        assert got["status"] == "ok", got
        h, c = _alone(r)
        np.testing.assert_array_equal(got["hist"], h)
        np.testing.assert_array_equal(got["counts"], c)
    s = summarize(res, srv.stats)
    assert s["requests"] == base - 1
    assert s["failed"] == dict(error=3, rejected=1, cancelled=1)


def test_failed_persistent_pass_fails_only_its_members(torch, monkeypatch):
    reqs = _requests()
    orig = bwg.Batch.run
    calls = {"n": 0}

    def flaky(self, max_events=0):
        calls["n"] += 1
        if calls["n"] == 3:
            raise bwg.BwgError(_abi_edevice(), "injected launch failure")
        return orig(self, max_events)

    monkeypatch.setattr(bwg.Batch, "run", flaky)
    srv = Server(chunk=200, max_members=3, keep_counts=True)
    res = srv.serve(reqs, real_time=False, pass_time=1.0)
    assert len(res) == len(reqs)
    failed = [r for r in res if r["status"] != "ok"]
    assert failed and all(r["status"] == "error" and "injected" in r["error"] for r in failed)
    assert len(failed) <= 3
    by_id = {r["id"]: r for r in res}
    for r in reqs:
        got = by_id[r["net_id"]]
        if got["status"] == "ok":
            h, c = _alone(r)
            np.testing.assert_array_equal(got["hist"], h)
            np.testing.assert_array_equal(got["counts"], c)
    assert sum(r["status"] == "ok" for r in res) >= len(reqs) - 3


def _abi_edevice():
    from paper_2412_16613_amd import _abi
    return _abi.BWG_EDEVICE
