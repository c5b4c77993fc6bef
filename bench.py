"""Benchmark of the per-timestep spiking-network step on one MI355X.

One benchmark step is one 1 ms spike bin of the whole hot path: the radix-partitioned
fan-in of the bin's arrivals (k_part, k_bucket when two passes are needed, k_gather),
ten fused 0.1 ms Euler substeps of every neuron with Poisson background (k_neuron),
the spike-list compaction (k_compact), and the region readout and bin close
(k_region_partials, k_readout_close).

Workload (default): one GPU's share of the whole-brain model, 6.1 M LIF neurons,
in-degree 556 (3.39e9 synapses, two weights each), 4 receptors, delays uniform in
1..10 ms, background tuned for a mean rate near 15 Hz. All inputs are synthetic
and seeded (the paper's networks come from private MRI data).

Prints one JSON line: synaptic events/s over the timed bins (inputs resident in
HBM), the real-time factor, the HBM roofline of the dominant fan-out phase, the
batched-ensemble comparison (64 uneven networks advanced together vs one after
another: ensemble sims/s and per-member p50/p99 completion latency), the served
stream (seeded Poisson arrivals of requests admitted by footprint: p50/p99
latency and sustained events/s, at the offered rate and at a stable rate), and the
CPU oracle's throughput on a bounded sample of the same recipe.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
BYTES_PER_EVENT = 44.0         # fan-out: 4 B target + 2 x 4 B weights + 2 x (8 B read + 8 B write) accumulators
BYTES_PER_NEURON_BIN = 128.0   # neuron step: V, J[4], ref read+write, g_u[4], arrivals[4] int64 read+clear


FANIN_KERNELS = ("k_part", "k_bucket", "k_gather")
PHASES = ("ms_scatter", "ms_gather", "ms_neuron", "ms_readout")
COUNTERS_JSON = os.path.join(ROOT, "profiles", "fanin_share6.1M_15hz_counters.json")
KERNEL_SOURCES = ("paper_2211_15963_amd/csrc/kernels.hip", "paper_2211_15963_amd/csrc/dbsim_internal.hpp")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(events_per_bin: float):
    """HBM bytes per bin of the fan-out phase from the committed counter summary, scaled
    to this run's events per bin; None when the kernels changed since the counters."""
    try:
        with open(COUNTERS_JSON) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    if c.get("kernel_source_hash") != kernel_source_hash():
        return None
    per_bin = sum(c["bytes_per_bin"][k]["read"] + c["bytes_per_bin"][k]["write"]
                  for k in FANIN_KERNELS if k in c["bytes_per_bin"])
    return per_bin * events_per_bin / c["edge_events_per_bin"]


def run_gpu(args):
    import torch
    from netgen import configs
    from paper_2211_15963_amd import Simulator

    spec = configs.share(n=args.n, indegree=args.indegree, regime_hz=args.regime, seed=args.seed)
    log(f"building {spec.name}: {spec.num_neurons} neurons, {spec.num_edges()} synapses")
    t0 = time.time()
    sim = Simulator(spec, record_regions=True, device=0, no_graph=args.mode == "direct")
    log(f"built in {time.time() - t0:.1f} s (construction {sim.stats()['build_seconds']:.1f} s), "
        f"device bytes {sim.stats()['hbm_bytes'] / 1e9:.2f} GB")
    S = sim.S
    # the network starts from a synchronous transient (every V drawn in [V_reset, V_th), no
    # conductances yet): a fixed settling period, independent of --warmup, brings it to its
    # stationary rate before anything is tuned or timed (the paper times the tail of longer runs)
    sim.step(args.settle * S)
    sim.sync()
    log(f"settled {args.settle} bins")
    tuned = None
    if args.autotune:
        from paper_2211_15963_amd.tune import autotune
        # fan-in kernels on one stream (phase events), ranked over trials of at least ten bins
        tuned = autotune(sim, bins_per_trial=max(10, args.tune_bins))
        log(f"autotuned fan-in schedule: {tuned['chosen']}")
    sim.step(args.warmup * S)
    sim.sync()
    log(f"warmup {args.warmup} bins done")
    s0 = sim.stats()
    if args.mode == "timed":
        sim.set_timing(True)
    torch.cuda.synchronize()
    sim.sync()
    t0 = time.perf_counter()
    sim.step(args.steps * S)
    sim.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s1 = sim.stats()
    log(f"timed {args.steps} bins in {wall:.3f} s ({args.mode} launches)")
    events = s1["edge_events"] - s0["edge_events"]
    spikes = s1["spikes"] - s0["spikes"]
    bio_s = args.steps * spec.bin_ms * 1e-3
    # per-kernel durations: HIP events between the phases on the handle's stream (one
    # stream, nothing overlapped), over a further window of the same run
    p0, p1, pbins = s0, s1, args.steps
    if args.mode == "graph" and args.phase_bins > 0:
        sim.set_timing(True)
        p0 = sim.stats()
        sim.step(args.phase_bins * S)
        sim.sync()
        p1 = sim.stats()
        sim.set_timing(False)
        pbins = args.phase_bins
        log(f"phase timing window: {pbins} bins, {sum(p1[k] - p0[k] for k in PHASES) / pbins:.3f} ms per bin "
            f"without overlap")
    s2 = sim.stats()
    out = {
        "events": events, "spikes": spikes, "wall": wall, "bio_s": bio_s,
        "rate_hz": spikes / (spec.num_neurons * bio_s),
        "phase_events": p1["edge_events"] - p0["edge_events"],
        "ms_scatter": p1["ms_scatter"] - p0["ms_scatter"], "ms_gather": p1["ms_gather"] - p0["ms_gather"],
        "ms_neuron": p1["ms_neuron"] - p0["ms_neuron"], "ms_readout": p1["ms_readout"] - p0["ms_readout"],
        "timed_bins": p1["timed_bins"] - p0["timed_bins"], "spec": spec, "build_s": s1["build_seconds"],
        "hbm_bytes": s1["hbm_bytes"], "tuning": sim.tuning(),
        "buffers": {"stream_records": int(sim.info.stream_records), "arena_records": int(sim.info.arena_records),
                    "stream_record_bytes": int(sim.info.stream_record_bytes)},
        "run_totals": {"bins": s2["bins"], "edge_events": s2["edge_events"], "spilled_events": s2["spilled_events"],
                       "overflow_events": s2["overflow_events"]},
    }
    sim.close()
    return out


def run_regimes(args, regimes, tuning=None):
    """Real-time factor of the same share workload in the other firing regimes (the
    background rate set for a 7 or 30 Hz population rate), graph launches, after a warm-up."""
    import torch
    from netgen import configs
    from paper_2211_15963_amd import Simulator

    out = {}
    for r in regimes:
        spec = configs.share(n=args.n, indegree=args.indegree, regime_hz=r, seed=args.seed)
        sim = Simulator(spec, record_regions=True, device=0)
        if tuning:  # the schedule the autotuner chose for the headline regime
            sim.set_tuning(**tuning)
        S = sim.S
        sim.step(args.settle * S)
        sim.sync()
        s0 = sim.stats()
        bins = 300
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(bins * S)
        sim.sync()
        wall = time.perf_counter() - t0
        s1 = sim.stats()
        sim.close()
        bio = bins * spec.bin_ms * 1e-3
        out[str(r)] = {"rtf": wall / bio, "events_per_s": (s1["edge_events"] - s0["edge_events"]) / wall,
                       "mean_rate_hz": round((s1["spikes"] - s0["spikes"]) / (spec.num_neurons * bio), 3),
                       "bins": bins}
        log(f"regime {r} Hz: real-time factor {wall / bio:.3f}, {out[str(r)]['events_per_s']:.3e} events/s")
    return out


def run_small_configs(args):
    """Real-time factor of the other single-GPU workloads: the tiny 1,000-neuron network for
    1 s of biological time (launch-bound; the paper's debug-graph scale) and the 200-region
    network (200 x 5,000 neurons, long-range delays up to 20 ms) after a settling period."""
    import torch
    from netgen import configs
    from paper_2211_15963_amd import Simulator

    out = {}
    for name, spec, settle, bins in (("tiny", configs.tiny(seed=args.seed), 0, 1000),
                                     ("multi_region", configs.multi_region(seed=args.seed), args.settle, 300)):
        sim = Simulator(spec, record_regions=True, device=0)
        S = sim.S
        if settle:
            sim.step(settle * S)
        sim.sync()
        s0 = sim.stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(bins * S)
        sim.sync()
        wall = time.perf_counter() - t0
        s1 = sim.stats()
        sim.close()
        bio = bins * spec.bin_ms * 1e-3
        out[name] = {"neurons": spec.num_neurons, "synapses": spec.num_edges(), "bins": bins, "settle_bins": settle,
                     "rtf": wall / bio, "events_per_s": (s1["edge_events"] - s0["edge_events"]) / wall,
                     "mean_rate_hz": round((s1["spikes"] - s0["spikes"]) / (spec.num_neurons * bio), 3)}
        log(f"{name}: real-time factor {wall / bio:.4f}, {out[name]['events_per_s']:.3e} events/s, "
            f"{out[name]['mean_rate_hz']} Hz")
    return out


def run_served(args):
    """Served stream: seeded Poisson arrivals of requests of log-uniform size, admitted by
    footprint, built on host threads (connection tables on the device) and advanced
    together on the device. First at the offered rate (an overload: the device's throughput
    on many small networks bounds the service rate), then at 70% of the sustained
    completion rate measured there, where queues are stable."""
    from netgen import configs
    from paper_2211_15963_amd.serve import Request, Server

    def window(rate, count, seed):
        t = configs.arrival_times(count, rate, seed=seed)
        reqs = []
        for r in range(count):
            spec, steps = configs.served_request(r, seed=seed)
            reqs.append(Request(r, spec, steps, arrival_s=float(t[r])))
        srv = Server(max_active=args.serve_slots, slice_bins=25, build_workers=2, state_digest=False)
        out = srv.run(reqs)
        done = [r for r in out["requests"] if r.error is None]
        return {"offered_per_s": rate, "requests": count, "completed": out["completed"],
                "wall_s": round(out["wall_s"], 3), "completed_per_s": out["completed"] / out["wall_s"],
                "p50_latency_s": out["p50_latency_s"], "p99_latency_s": out["p99_latency_s"],
                "events_per_s": out["events_per_s"], "peak_resident": out["peak_active"],
                "mean_wait_s": out["mean_wait_s"], "mean_build_s": out["mean_build_s"],
                "neurons": int(sum(r.spec.num_neurons for r in done)),
                "synapses": int(sum(r.spec.num_edges() for r in done))}

    log(f"served stream: {args.serve_requests} requests at {args.serve_rate}/s")
    over = window(args.serve_rate, args.serve_requests, args.seed + 100)
    log(f"served (offered {args.serve_rate}/s): p50 {over['p50_latency_s']:.2f} s, p99 {over['p99_latency_s']:.2f} s, "
        f"{over['completed_per_s']:.2f} req/s, {over['events_per_s']:.3g} events/s")
    stable_rate = 0.7 * over["completed_per_s"]
    n_stable = max(4, args.serve_requests // 2)
    stable = window(stable_rate, n_stable, args.seed + 200)
    log(f"served (offered {stable_rate:.2f}/s): p50 {stable['p50_latency_s']:.2f} s, "
        f"p99 {stable['p99_latency_s']:.2f} s")
    return {"offered": over, "stable": stable,
            "recipe": "sizes log-uniform 1e4..2e6 neurons, in-degree U{200..600}, regime U{7,15,30} Hz, "
                      "duration U[0.1, 2] s bio; latency = completion - arrival (host build included)"}


def _host_info():
    model, ram = None, None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    ram = round(int(line.split()[1]) / 2**20, 1)
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model, "ram_gib": ram}


def _host_cores() -> int:
    """Cores this process may use: its CPU affinity, capped by OMP_NUM_THREADS when set."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cap = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    return max(1, min(n, cap) if cap > 0 else n)


def cpu_baseline(args, budget_s: float):
    """The FP32 oracle on a 1/64 share of the same recipe: on one host core, then split over
    every core this process may use (neuron ranges per thread; identical results). Also the
    FP32 state error of the GPU path against the FP64 oracle on the tiny network."""
    from netgen import configs
    from oracle import Oracle

    n = max(1000, args.n // 64)
    spec = configs.share(n=n, indegree=args.indegree, regime_hz=args.regime, seed=args.seed)
    t0 = time.time()
    o = Oracle(spec, 32)
    log(f"cpu baseline: oracle network {n} neurons built in {time.time() - t0:.1f} s")
    S = spec.steps_per_bin
    o.step(20 * S)  # 20 ms warm-up so that delayed arrivals are flowing

    def timed(threads, budget):
        o.set_threads(threads)
        ev0 = o.edge_events
        t0 = time.perf_counter()
        bins = 0
        while time.perf_counter() - t0 < budget:
            o.step(S)
            bins += 1
        wall = time.perf_counter() - t0
        return (o.edge_events - ev0) / wall, wall / (bins * 1e-3), bins

    v1, rtf1, b1 = timed(1, budget_s / 2)
    cores = _host_cores()
    vn, rtfn, bn = timed(cores, budget_s / 2)
    log(f"cpu baseline: {v1:.3e} events/s on one core, {vn:.3e} on {cores} cores")
    sample = (f"share recipe at N={n} (1/64 of the GPU share), in-degree {args.indegree}, delays 1..10 ms, "
              f"after 20 ms warm-up; FP32 oracle")
    return {"value": v1, "unit": "synaptic events/s", "cores": 1, "kind": "oracle",
            "sample": f"{sample} on one host core, {b1} bins ({b1} ms bio); real-time factor {rtf1:.1f}",
            "rtf": rtf1,
            # the oracle's work per bin grows linearly with N at a fixed rate and in-degree
            "rtf_full_share_extrapolated": rtf1 * args.n / n,
            "all_cores": {"value": vn, "unit": "synaptic events/s", "cores": cores, "kind": "oracle",
                          "sample": f"{sample} split over {cores} host threads (same results), {bn} bins",
                          "rtf": rtfn, "rtf_full_share_extrapolated": rtfn * args.n / n, **_host_info()},
            "fp32_vs_fp64": fp32_vs_fp64(args)}


def fp32_vs_fp64(args, bins: int = 1000):
    """FP32 state error of the GPU path against the FP64 oracle on the tiny network (1 s):
    the largest relative V error and the largest J error (relative to the largest |J|) over
    the bins before the first raster divergence, and the step of that divergence."""
    import numpy as np
    from netgen import configs
    from oracle import Oracle
    from paper_2211_15963_amd import Simulator

    spec = configs.tiny(seed=args.seed)
    sim = Simulator(spec, record_regions=False, device=0)
    o64 = Oracle(spec, 64)
    S = sim.S
    v_err = j_err = 0.0
    diverged = None
    seen = 0
    for b in range(bins):
        sim.step(S)
        o64.step(S)
        st, ids = sim.spikes(b * S, (b + 1) * S)
        so, io = o64.spikes()
        so, io = so[seen:], io[seen:]
        seen += len(so)
        if not (np.array_equal(st, so) and np.array_equal(ids, io)):
            diverged = b * S
            break
        V, J, _ = sim.state()
        V64, J64, _ = o64.state()
        v_err = max(v_err, float(np.max(np.abs(V - V64) / np.abs(V64))))
        j_err = max(j_err, float(np.max(np.abs(J - J64))) / max(float(np.max(np.abs(J64))), 1e-30))
    sim.close()
    log(f"FP32 (GPU) vs FP64 (oracle), tiny network: max relative V error {v_err:.3e}, J {j_err:.3e}, "
        f"first raster divergence at {'none' if diverged is None else f'step {diverged}'}")
    return {"workload": "tiny (1,000 neurons), 1 s", "max_rel_V_err": v_err, "max_rel_J_err": j_err,
            "bins_compared": bins if diverged is None else diverged // S,
            "first_raster_divergence_step": diverged}


def run_ensemble(args):
    """Batched ensemble: members advanced together vs the same members one after another."""
    import numpy as np
    import torch
    from netgen import configs
    from paper_2211_15963_amd import Simulator

    members = [configs.ensemble_member(m, seed=args.seed) for m in range(args.members)]
    nn = sum(s.num_neurons for s in members)
    ne = sum(s.num_edges() for s in members)
    bins = args.ensemble_bins
    log(f"ensemble: {len(members)} members, {nn} neurons, {ne} synapses, {bins} bins each")
    t0 = time.time()
    ens = Simulator(members, record_regions=True)
    log(f"ensemble built in {time.time() - t0:.1f} s")
    S = ens.S
    ens.step(args.ensemble_warmup * S)
    if args.autotune:
        from paper_2211_15963_amd.tune import autotune
        autotune(ens, bins_per_trial=4)
    ens.sync()
    s0 = ens.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.step(bins * S)
    ens.sync()
    torch.cuda.synchronize()
    wall_ens = time.perf_counter() - t0
    ev_ens = ens.stats()["edge_events"] - s0["edge_events"]
    tuning = ens.tuning()
    ens.close()
    log(f"ensemble: {bins} bins in {wall_ens:.3f} s")
    # the same members one after another, each on its own handle
    walls = []
    ev_seq = 0
    for m, spec in enumerate(members):
        sim = Simulator(spec, record_regions=True)
        sim.step(args.ensemble_warmup * S)
        sim.sync()
        e0 = sim.stats()["edge_events"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(bins * S)
        sim.sync()
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        ev_seq += sim.stats()["edge_events"] - e0
        sim.close()
    wall_seq = float(np.sum(walls))
    log(f"one after another: {wall_seq:.3f} s")
    done_seq = np.cumsum(walls)  # completion time of each member when run in sequence
    return {"members": len(members), "neurons": nn, "synapses": ne, "bio_s": bins * 1e-3,
            "ensemble": {"wall_s": wall_ens, "sims_per_s": len(members) / wall_ens,
                         "p50_latency_s": wall_ens, "p99_latency_s": wall_ens, "events_per_s": ev_ens / wall_ens,
                         "tuning": tuning},
            "one_after_another": {"wall_s": wall_seq, "sims_per_s": len(members) / wall_seq,
                                  "p50_latency_s": float(np.percentile(done_seq, 50)),
                                  "p99_latency_s": float(np.percentile(done_seq, 99)),
                                  "events_per_s": ev_seq / wall_seq},
            "speedup": wall_seq / wall_ens}


def copy_bandwidth() -> float:
    """Achievable HBM bandwidth: a plain 2 GiB device-to-device copy (read + write bytes
    per second), timed with HIP events; the best of five."""
    import torch
    n = 1 << 29
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = 0.0
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = max(best, 8.0 * n / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del a, b
    torch.cuda.empty_cache()
    return best


def calibrate_copy(args):
    """A plain device copy of known size, so that profiler byte counters can be scaled."""
    import torch
    n = 1 << 29  # 2 GiB of float32 per buffer
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}))


def _rocpd(db):
    """Per-kernel dispatch count, mean duration (us) and mean counter values from a rocprofv3 database."""
    import collections
    import sqlite3
    c = sqlite3.connect(db)
    q = ("select k.kernel_name, d.start, d.end from rocpd_kernel_dispatch d "
         "join rocpd_info_kernel_symbol k on d.kernel_id = k.id")
    dur = collections.defaultdict(list)
    rows = sorted(c.execute(q), key=lambda r: r[1])
    for name, t0, t1 in rows:
        dur[name].append((t1 - t0) / 1e3)
    # the one-stream timed window at the end of the run: every dispatch after the last two
    # that overlapped by more than 2 us (back-to-back dispatches touch within the clocks' jitter)
    lib_rows = [r for r in rows if "dbs" in r[0]]
    last = 0
    end_so_far = 0
    for x, (name, t0, t1) in enumerate(lib_rows):
        if x and t0 + 2000 < end_so_far:
            last = x + 1
        end_so_far = max(end_so_far, t1)
    alone = collections.defaultdict(list)
    for name, t0, t1 in lib_rows[last:]:
        alone[name].append((t1 - t0) / 1e3)
    pmc = collections.defaultdict(lambda: collections.defaultdict(float))
    try:
        q = ("select k.kernel_name, d.event_id, p.name, e.value from rocpd_pmc_event e "
             "join rocpd_info_pmc p on e.pmc_id = p.id join rocpd_kernel_dispatch d on d.event_id = e.event_id "
             "join rocpd_info_kernel_symbol k on d.kernel_id = k.id")
        for name, ev, pn, val in c.execute(q):
            pmc[(name, pn)][ev] += val  # sum over counter instances of one dispatch
    except sqlite3.Error:
        pass
    out = {}
    for name, v in dur.items():
        a = alone.get(name, [])
        out[name] = {"calls": len(v), "avg_us": sum(v) / len(v), "alone_calls": len(a),
                     "alone_avg_us": sum(a) / len(a) if a else None}
    for (name, pn), per_disp in pmc.items():
        out.setdefault(name, {})[pn] = sum(per_disp.values()) / len(per_disp)
    return out


def _short(name):
    for k in ("k_part", "k_bucket", "k_gather_blk", "k_gather", "k_fan", "k_neuron", "k_compact", "k_drain",
              "k_region_partials", "k_readout_close", "k_pass_reset", "k_gen_count", "k_gen_fill", "k_gen_sort",
              "k_gen_rows", "k_gen_cursors", "k_gen_clear", "k_scan_a", "k_scan_b", "k_scan_c", "copyBuffer"):
        if k in name:
            return k
    return name


def _construction(name):
    """Kernels of the device construction of the connection table (once per network)."""
    return "k_gen_" in name or "k_scan_" in name


def summarize_profiles(args):
    """Writes the committed text summary and counter file from a directory of rocprofv3 runs:
    trace/, fetch/, write/ (the bench command), cal_fetch/, cal_write/ (--calibrate-copy), and
    fetch.log (the profiled bench run's output, for its event totals)."""
    d = args.summarize_profiles
    trace = _rocpd(os.path.join(d, "trace", "run_results.db"))
    fetch = _rocpd(os.path.join(d, "fetch", "run_results.db"))
    write = _rocpd(os.path.join(d, "write", "run_results.db"))
    cf = _rocpd(os.path.join(d, "cal_fetch", "run_results.db"))
    cw = _rocpd(os.path.join(d, "cal_write", "run_results.db"))
    copy_bytes = 4 << 29
    cal_f = next(v["FETCH_SIZE"] for k, v in cf.items() if "copyBuffer" in k and "FETCH_SIZE" in v)
    cal_w = next(v["WRITE_SIZE"] for k, v in cw.items() if "copyBuffer" in k and "WRITE_SIZE" in v)
    f_fac, w_fac = copy_bytes / (cal_f * 1024), copy_bytes / (cal_w * 1024)
    run = None
    with open(os.path.join(d, "fetch.log")) as f:
        for line in f:
            if line.startswith("{"):
                run = json.loads(line)
    tot = run["config"]["run_totals"]
    ev_per_bin = tot["edge_events"] / tot["bins"]
    per_bin = {}
    for name in set(fetch) | set(write):
        # the library's per-bin kernels only (not the runtime's copy/fill kernels, not the
        # one-time construction)
        if "dbs" not in name or _construction(name):
            continue
        if "FETCH_SIZE" in fetch.get(name, {}) and "WRITE_SIZE" in write.get(name, {}):
            # mean per dispatch x dispatches per bin (the partition kernels run twice a bin)
            fr, wr = fetch[name]["calls"] / tot["bins"], write[name]["calls"] / tot["bins"]
            per_bin[_short(name)] = {"read": fetch[name]["FETCH_SIZE"] * 1024 * f_fac * fr,
                                     "write": write[name]["WRITE_SIZE"] * 1024 * w_fac * wr,
                                     "dispatches_per_bin": fr}
    cmd = args.profile_command
    lines = [f"# Kernel trace and HBM byte counters: {run['config']['workload']}", "",
             "Commands (from the repository root, PYTHONPATH=., TMPDIR=/tmp):",
             f"  rocprofv3 --kernel-trace --stats -d OUT/trace -o run -- {cmd}",
             f"  rocprofv3 --pmc FETCH_SIZE -d OUT/fetch -o run -- {cmd} > OUT/fetch.log",
             f"  rocprofv3 --pmc WRITE_SIZE -d OUT/write -o run -- {cmd}",
             "  rocprofv3 --pmc FETCH_SIZE -d OUT/cal_fetch -o run -- python3 bench.py --calibrate-copy",
             "  rocprofv3 --pmc WRITE_SIZE -d OUT/cal_write -o run -- python3 bench.py --calibrate-copy",
             "  python3 bench.py --summarize-profiles OUT", "",
             f"Profiled run: {tot['bins']} bins in all (warm-up included), {ev_per_bin:.4g} edge events per bin "
             f"on average; fan-in schedule {run['config']['fanin_schedule']}.", "",
             "Kernel durations (kernel trace, every dispatch of the run; the next bin's delay >= 2 "
             "partition overlaps the neuron step on a second stream, so per-bin sums exceed the bin time):",
             f"  {'kernel':46s} {'calls':>6s} {'avg us':>10s}"]
    for name, v in sorted(trace.items(), key=lambda kv: -kv[1]["calls"] * kv[1]["avg_us"]):
        if _construction(name):
            continue
        lines.append(f"  {name[:46]:46s} {v['calls']:6d} {v['avg_us']:10.2f}  "
                     f"({v['calls'] * v['avg_us'] / tot['bins']:8.2f} us per bin)")
    cons = {k: v for k, v in trace.items() if _construction(k)}
    if cons:
        lines += ["", "Network construction on the device (once, before the first bin):"]
        for name, v in sorted(cons.items(), key=lambda kv: -kv[1]["calls"] * kv[1]["avg_us"]):
            lines.append(f"  {_short(name):16s} {v['calls']:4d} launches  {v['calls'] * v['avg_us'] / 1e3:9.1f} ms")
        lines.append(f"  total {sum(v['calls'] * v['avg_us'] for v in cons.values()) / 1e6:.2f} s")
    # the one-stream timed window: what bench.py's phase timers measure (roofline.avg_launch_ms)
    alone_bins = max((v["alone_calls"] for k, v in trace.items() if "k_neuron" in k), default=0)
    if alone_bins:
        lines += ["", f"Same kernels in the one-stream timed window at the end of the run (every dispatch "
                      f"after the last overlap; {alone_bins} bins):"]
        fan_us = 0.0
        for name, v in sorted(trace.items(), key=lambda kv: -(kv[1]["alone_calls"] * (kv[1]["alone_avg_us"] or 0))):
            if not v["alone_calls"] or "dbs" not in name:
                continue
            per_bin_us = v["alone_calls"] * v["alone_avg_us"] / alone_bins
            if _short(name) in FANIN_KERNELS:
                fan_us += per_bin_us
            lines.append(f"  {name[:46]:46s} {v['alone_calls']:6d} {v['alone_avg_us']:10.2f}  "
                         f"({per_bin_us:8.2f} us per bin)")
        lines.append(f"  fan-out phase (k_part + k_bucket + k_gather): {fan_us:.1f} us per bin")
    lines += ["", f"Counter calibration: a 2 GiB device copy reads FETCH_SIZE {cal_f:.4g} KiB and WRITE_SIZE "
                  f"{cal_w:.4g} KiB per launch -> scale factors FETCH x{f_fac:.3f}, WRITE x{w_fac:.3f}.", "",
              "HBM-side bytes per bin (calibrated) and per edge event:"]
    for k, v in sorted(per_bin.items()):
        lines.append(f"  {k:18s} read {v['read'] / 1e6:9.1f} MB  write {v['write'] / 1e6:8.1f} MB   "
                     f"({v['read'] / ev_per_bin:6.2f} + {v['write'] / ev_per_bin:6.2f} B/event)")
    fan = sum(per_bin[k]["read"] + per_bin[k]["write"] for k in FANIN_KERNELS if k in per_bin)
    lines.append(f"  fan-out phase total {fan / ev_per_bin:.2f} B per edge event (algorithmic model "
                 f"{BYTES_PER_EVENT:.0f} B)")
    base = os.path.join(ROOT, "profiles", "fanin_share6.1M_15hz")
    with open(base + ".txt", "w") as f:
        f.write("\n".join(lines) + "\n")
    with open(base + "_counters.json", "w") as f:
        json.dump({"kernel_source_hash": kernel_source_hash(), "edge_events_per_bin": ev_per_bin,
                   "bins": tot["bins"], "copy_factors": {"fetch": f_fac, "write": w_fac},
                   "bytes_per_bin": per_bin,
                   "avg_us": {_short(k): v["avg_us"] for k, v in trace.items()}}, f, indent=1)
    print("\n".join(lines))


def tune(args):
    """Bisection of the background rate for target population rates (writes nothing)."""
    from netgen import configs
    from paper_2211_15963_amd import Simulator

    res = {}
    for target in (7, 15, 30):
        lo, hi = 2000.0, 12000.0
        for it in range(args.tune_iters):
            mid = 0.5 * (lo + hi)
            spec = configs.share(n=args.n, indegree=args.indegree, seed=args.seed, bg_rate_hz=mid)
            sim = Simulator(spec, record_regions=False)
            sim.step(200 * sim.S)
            s0 = sim.stats()["spikes"]
            sim.step(300 * sim.S)
            r = (sim.stats()["spikes"] - s0) / (spec.num_neurons * 0.3)
            sim.close()
            log(f"target {target} Hz: bg {mid:.1f} Hz -> {r:.2f} Hz")
            if r < target:
                lo = mid
            else:
                hi = mid
        res[target] = 0.5 * (lo + hi)
    print(json.dumps({"tuned_bg_hz": res}))


def main():
    import faulthandler
    faulthandler.enable()  # a fatal signal prints every thread's Python stack to stderr
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000, help="timed 1 ms bins")
    ap.add_argument("--warmup", type=int, default=200, help="untimed 1 ms bins (after the settling period)")
    ap.add_argument("--settle", type=int, default=300,
                    help="bins run first, before tuning and warm-up, so that the start-up transient has passed")
    ap.add_argument("--tune-bins", type=int, default=10, help="bins per autotuner trial (at least 10)")
    ap.add_argument("--rate-tolerance", type=float, default=0.05,
                    help="largest relative gap between the timed window's mean rate and the regime")
    ap.add_argument("--n", type=int, default=6_100_000)
    ap.add_argument("--indegree", type=int, default=556)
    ap.add_argument("--regime", type=int, default=15, choices=[7, 15, 30])
    ap.add_argument("--regimes", type=int, default=1, help="also time the other firing regimes (1) or not (0)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--mode", default="graph", choices=["graph", "timed", "direct"],
                    help="graph: replayed HIP graphs with the next bin's fan-in overlapped (headline), then a "
                         "window of timed phases for the roofline; timed: timed phases only")
    ap.add_argument("--phase-bins", type=int, default=300, help="bins of the per-kernel timing window")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune", action="store_true")
    ap.add_argument("--tune-iters", type=int, default=9)
    ap.add_argument("--calibrate-copy", action="store_true", help="run only a 2 GiB device copy (counter scaling)")
    ap.add_argument("--summarize-profiles", default=None, help="directory of rocprofv3 runs to summarise (CPU only)")
    ap.add_argument("--profile-command", default="python3 bench.py --steps 20 --warmup 5 --no-cpu-baseline "
                    "--ensemble 0 --serve 0 --regimes 0 --small-configs 0",
                    help="the profiled command, quoted in the summary")
    ap.add_argument("--autotune", type=int, default=1, help="autotune the fan-in schedule during warm-up")
    ap.add_argument("--ensemble", type=int, default=1, help="also run the batched-ensemble comparison")
    ap.add_argument("--small-configs", type=int, default=1,
                    help="also time the tiny and the 200-region networks (real-time factor)")
    ap.add_argument("--members", type=int, default=64)
    ap.add_argument("--serve", type=int, default=1, help="also run the served-stream leg")
    ap.add_argument("--serve-rate", type=float, default=50.0, help="offered request arrivals per second")
    ap.add_argument("--serve-requests", type=int, default=24, help="arrivals in the offered-rate window")
    ap.add_argument("--serve-slots", type=int, default=16, help="most requests resident at once")
    ap.add_argument("--ensemble-bins", type=int, default=500, help="bins (ms) each member advances")
    ap.add_argument("--ensemble-warmup", type=int, default=50)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU's share of the network; runs on more than one GPU are not supported "
              "(the multi-GPU spike exchange is not part of this library)", file=sys.stderr)
        sys.exit(2)
    if args.tune:
        tune(args)
        return
    if args.calibrate_copy:
        calibrate_copy(args)
        return
    if args.summarize_profiles:
        summarize_profiles(args)
        return
    g = run_gpu(args)
    spec = g["spec"]
    value = g["events"] / g["wall"]
    fan_ms = g["ms_scatter"] + g["ms_gather"]
    nb = max(1, g["timed_bins"])
    roof = None
    if g["timed_bins"]:
        achieved = BYTES_PER_EVENT * g["phase_events"] / (fan_ms * 1e-3) / 1e9
        traffic = measured_traffic(g["phase_events"] / nb)
        copy_gbs = copy_bandwidth()
        roof = {"bound": "hbm", "kernel": "fan-out phase (k_part + k_bucket + k_gather), per bin",
                "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4),
                "traffic": None if traffic is None else round(traffic),
                "traffic_unit": "bytes per bin (FETCH_SIZE x copy factor + WRITE_SIZE x copy factor)",
                "traffic_bytes_per_event": None if traffic is None else round(traffic * nb / g["phase_events"], 2),
                "measured_gbs": None if traffic is None else round(traffic / (fan_ms / nb * 1e-3) / 1e9, 1),
                "measured_frac": None if traffic is None else round(traffic / (fan_ms / nb * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                "copy_gbs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4),
                "measured_frac_of_copy": None if traffic is None else round(traffic / (fan_ms / nb * 1e-3) / 1e9 / copy_gbs, 4),
                "bytes_per_event": BYTES_PER_EVENT, "events_per_launch": g["phase_events"] / nb,
                "phase_window_bins": nb,
                "avg_launch_ms": {"k_part+k_bucket": g["ms_scatter"] / nb, "k_gather": g["ms_gather"] / nb,
                                  "k_neuron": g["ms_neuron"] / nb, "readout_close": g["ms_readout"] / nb}}
    regimes = None
    if args.regimes:
        regimes = {str(args.regime): {"rtf": g["wall"] / g["bio_s"], "events_per_s": value,
                                      "mean_rate_hz": round(g["rate_hz"], 3), "bins": args.steps}}
        regimes.update(run_regimes(args, [r for r in (7, 15, 30) if r != args.regime], g["tuning"]))
    small = run_small_configs(args) if args.small_configs else None
    ens = run_ensemble(args) if args.ensemble else None
    served = run_served(args) if args.serve else None
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args, args.cpu_seconds)
    line = {
        "metric": "synaptic events/s", "value": value, "unit": "synaptic events/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * g["wall"] / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded fixed in-degree network, Poisson background)",
        "config": {"workload": f"one GPU share: {spec.num_neurons} LIF neurons, in-degree {args.indegree}, "
                               f"delays 1-10 ms, 4 receptors, dt 0.1 ms, {args.regime} Hz regime",
                   "neurons": spec.num_neurons, "synapses": spec.num_edges(), "dt_ms": spec.dt_ms,
                   "bin_ms": spec.bin_ms, "regime_hz": args.regime, "mean_rate_hz": round(g["rate_hz"], 3),
                   "rtf": g["wall"] / g["bio_s"], "launch": args.mode, "build_s": round(g["build_s"], 1),
                   "device_gb": round(g["hbm_bytes"] / 1e9, 2), "fanin_buffers": g["buffers"],
                   "fanin_schedule": g["tuning"],
                   "run_totals": g["run_totals"]},
        "rtf_15hz": g["wall"] / g["bio_s"] if args.regime == 15 else None,
        "regimes": regimes,
        "other_workloads": small,
        "ensemble": ens,
        "served": served,
        "roofline": roof, "cpu_baseline": cpu,
    }
    # the timed window must sit in the stated regime: a window inside the start-up transient (or a
    # network tuned for another rate) would label another workload's numbers with this one's name
    gap = abs(g["rate_hz"] - args.regime) / args.regime
    line["config"]["rate_within_tolerance"] = gap <= args.rate_tolerance
    print(json.dumps(line), flush=True)
    if gap > args.rate_tolerance:
        log(f"timed window's mean rate {g['rate_hz']:.3f} Hz is {100 * gap:.1f} % away from the {args.regime} Hz "
            f"regime (tolerance {100 * args.rate_tolerance:.0f} %)")
        sys.exit(3)


if __name__ == "__main__":
    main()
