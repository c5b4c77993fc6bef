"""Served stream: requests admitted by footprint and overlapped on the device give
the same bits as each request run alone (every handle is independent and
deterministic) and, for small requests, as the FP32 oracle; admission respects the
HBM budget and the slot limit."""
import sys

import numpy as np
import pytest

from netgen import configs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _requests(count, seed, n_hi, d_hi_s, gap_s):
    from paper_2211_15963_amd.serve import Request
    out = []
    for r in range(count):
        spec, steps = configs.served_request(r, seed=seed, n_lo=1e4, n_hi=n_hi, d_lo_s=0.05, d_hi_s=d_hi_s)
        out.append(Request(r, spec, steps, arrival_s=r * gap_s))
    return out


def _alone(req):
    from paper_2211_15963_amd import Simulator
    from paper_2211_15963_amd.serve import summarize
    bins = -(-req.n_steps // req.spec.steps_per_bin)
    sim = Simulator(req.spec, record_regions=True, record_bins=max(4096, bins))
    sim.step(req.n_steps)
    sim.sync()
    out = summarize(sim)
    sim.close()
    return out


def _same(a, b):
    assert a["steps"] == b["steps"] and a["bins"] == b["bins"]
    assert a["spikes"] == b["spikes"] and a["edge_events"] == b["edge_events"]
    assert np.array_equal(a["bin_spikes"], b["bin_spikes"])
    assert a["state_sha256"] == b["state_sha256"]


def test_served_results_equal_alone():
    from paper_2211_15963_amd.serve import Server
    reqs = _requests(8, seed=11, n_hi=8e4, d_hi_s=0.2, gap_s=0.02)
    _say(f"serve 8 requests, sizes {[r.spec.num_neurons for r in reqs]}, steps {[r.n_steps for r in reqs]}")
    srv = Server(max_active=4, slice_bins=10, build_workers=2)
    out = srv.run(reqs)
    assert out["completed"] == 8 and out["failed"] == 0
    assert 1 <= out["peak_active"] <= 4
    for r in out["requests"]:
        assert r.result["spikes"] > 0
        assert r.t_admit >= r.arrival_s - 1e-9 and r.t_built >= r.t_admit and r.t_done >= r.t_built
    for r in sorted(out["requests"], key=lambda r: r.rid):
        _say(f"  request {r.rid}: {r.spec.num_neurons} neurons, latency {r.latency_s:.3f} s; alone run")
        _same(r.result, _alone(r))


def test_served_results_equal_the_oracle():
    """Two small requests served among larger ones (overlapping on the device with them)
    against the FP32 oracle: raster, final V, J, refractory counters and delivered events
    bit for bit."""
    from oracle import Oracle
    from paper_2211_15963_amd.serve import Request, Server
    reqs = _requests(4, seed=15, n_hi=6e4, d_hi_s=0.1, gap_s=0.01)
    for k, rid in enumerate((4, 5)):
        spec, _ = configs.served_request(rid, seed=15, n_lo=2000, n_hi=4000)
        reqs.insert(1 + 2 * k, Request(rid, spec, 40 * spec.steps_per_bin, arrival_s=0.005 + 0.01 * k))
    _say(f"serve 6 requests, sizes {[r.spec.num_neurons for r in reqs]}; requests 4 and 5 against the oracle")
    out = Server(max_active=4, slice_bins=10, build_workers=2, full_results=True).run(reqs)
    assert out["completed"] == 6
    for r in out["requests"]:
        if r.rid not in (4, 5):
            continue
        orc = Oracle(r.spec, 32)
        orc.step(r.n_steps)
        so, io = orc.spikes()
        sg, ig = r.result["raster"]
        assert len(so) > 0 and np.array_equal(sg, so) and np.array_equal(ig, io), f"request {r.rid}: raster"
        Vo, Jo, ro = orc.state()
        Vg, Jg, rg = r.result["state"]
        assert np.array_equal(Vg.astype(np.float64), Vo) and np.array_equal(Jg.astype(np.float64), Jo)
        assert np.array_equal(rg, ro) and r.result["edge_events"] == orc.edge_events
        _say(f"  request {r.rid} ({r.spec.num_neurons} neurons, {len(so)} spikes): bit-identical to the oracle")


def test_admission_by_footprint():
    from paper_2211_15963_amd.dbsim import footprint
    from paper_2211_15963_amd.serve import Server
    reqs = _requests(6, seed=12, n_hi=5e4, d_hi_s=0.1, gap_s=0.0)
    fps = sorted(footprint(r.spec, record_regions=True) for r in reqs)
    budget = fps[-1] + fps[-2]  # room for two of the largest at most
    _say(f"serve 6 requests with an HBM budget of {budget} B")
    srv = Server(hbm_budget=budget, max_active=16, slice_bins=5, build_workers=2)
    out = srv.run(reqs)
    assert out["completed"] == 6
    # no more than the budget resident at once: replay admissions and retirements
    events = sorted([(r.t_admit, r.footprint) for r in out["requests"]] +
                    [(r.t_done, -r.footprint) for r in out["requests"]], key=lambda e: (e[0], e[1]))
    use = 0
    for _, d in events:
        use += d
        assert use <= budget
    too_big = _requests(1, seed=13, n_hi=2e4, d_hi_s=0.06, gap_s=0.0)
    out = Server(hbm_budget=1 << 20, max_active=2).run(too_big)
    assert out["completed"] == 0 and out["failed"] == 1 and "exceeds" in out["requests"][0].error


def test_a_failing_request_retires_alone(monkeypatch):
    """A request whose stepping fails (the failure is forced from the host, before any
    device work of that slice is queued) retires with its error and frees its memory; the
    other requests complete with the same bits as alone."""
    import torch
    from paper_2211_15963_amd import dbsim as D
    from paper_2211_15963_amd.serve import Server
    reqs = _requests(4, seed=14, n_hi=5e4, d_hi_s=0.1, gap_s=0.0)
    bad = reqs[1].spec
    real_step = D.Simulator.step

    def step(self, n):
        if self.spec is bad and self.steps_done > 0:
            raise D.DbsimError(D.EDEVICE, "stepping failure forced from the host")
        real_step(self, n)

    monkeypatch.setattr(D.Simulator, "step", step)
    _say(f"serve 4 requests, request 1 fails on its second slice; sizes {[r.spec.num_neurons for r in reqs]}")
    torch.cuda.synchronize()
    m0 = torch.cuda.memory_allocated()
    out = Server(max_active=4, slice_bins=5, build_workers=2).run(reqs)
    assert out["completed"] == 3 and out["failed"] == 1
    failed = [r for r in out["requests"] if r.error is not None]
    assert failed[0].rid == 1 and "forced" in failed[0].error and failed[0].result is None
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == m0
    for r in sorted(out["requests"], key=lambda r: r.rid):
        if r.error is None:
            _say(f"  request {r.rid}: alone run")
            _same(r.result, _alone(r))


def test_cancelled_requests_retire_and_free_their_memory():
    """Requests withdrawn while waiting (at arrival), while resident (by their cancel time)
    and from another thread (Server.cancel) retire with the error "cancelled" whatever state
    they were in, and free their memory; the other requests complete with the same bits as
    alone."""
    import threading
    import torch
    from paper_2211_15963_amd.serve import Request, Server
    reqs = _requests(5, seed=15, n_hi=5e4, d_hi_s=0.1, gap_s=0.0)
    reqs[1].cancel_at_s = 0.0                                   # withdrawn on arrival
    for k in (2, 3):                                            # long: 200 s of biological time
        reqs[k] = Request(k, reqs[k].spec, 2_000_000, arrival_s=0.0)
    reqs[2].cancel_at_s = 1.5
    _say(f"serve 5 requests, 1 withdrawn on arrival, 2 at 1.5 s, 3 from another thread at 2.0 s; "
         f"sizes {[r.spec.num_neurons for r in reqs]}")
    torch.cuda.synchronize()
    m0 = torch.cuda.memory_allocated()
    srv = Server(max_active=4, slice_bins=5, build_workers=2)
    timer = threading.Timer(2.0, srv.cancel, args=(3,))
    timer.start()
    try:
        out = srv.run(reqs)
    finally:
        timer.cancel()
    by = {r.rid: r for r in out["requests"]}
    assert sorted(by) == [0, 1, 2, 3, 4]
    for k in (1, 2, 3):
        assert by[k].error == "cancelled" and by[k].result is None, (k, by[k].error)
    # 2 and 3 were resident (deployed) when withdrawn, and 3 was withdrawn by the thread
    assert by[2].t_built < 1.5 <= by[2].t_done and by[3].t_built < 2.0 <= by[3].t_done
    assert out["completed"] == 2 and out["failed"] == 3
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == m0
    for k in (0, 4):
        _say(f"  request {k}: alone run")
        _same(by[k].result, _alone(by[k]))
