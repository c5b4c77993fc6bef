"""Benchmark of the per-timestep spiking-network step on one MI355X.

One benchmark step is one 1 ms spike bin of the whole hot path: the bucketed
fan-in of the bin's arrivals (k_scatter + k_gather), ten fused 0.1 ms Euler
substeps of every neuron with Poisson background (k_neuron), the spike-list
compaction (k_compact), and the region readout and bin close (k_readout_close).

Workload (default): one GPU's share of the whole-brain model, 6.1 M LIF neurons,
in-degree 556 (3.39e9 synapses, two weights each), 4 receptors, delays uniform in
1..10 ms, background tuned for a mean rate near 15 Hz. All inputs are synthetic
and seeded (the paper's networks come from private MRI data).

Prints one JSON line: synaptic events/s over the timed bins (inputs resident in
HBM), the real-time factor, the HBM roofline of the dominant fan-out phase, the
batched-ensemble comparison (64 uneven networks advanced together vs one after
another: ensemble sims/s and per-member p50/p99 completion latency), and the CPU
oracle's throughput on a bounded sample of the same recipe.
"""
import argparse
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


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_gpu(args):
    import torch
    from netgen import configs
    from paper_2211_15963_amd import Simulator

    spec = configs.share(n=args.n, indegree=args.indegree, regime_hz=args.regime, seed=args.seed)
    log(f"building {spec.name}: {spec.num_neurons} neurons, {spec.num_edges()} synapses")
    t0 = time.time()
    sim = Simulator(spec, record_regions=True, device=0, no_graph=args.mode == "direct")
    log(f"built in {time.time() - t0:.1f} s (host construction {sim.stats()['build_seconds']:.1f} s), "
        f"device bytes {sim.stats()['hbm_bytes'] / 1e9:.2f} GB")
    S = sim.S
    tuned = None
    if args.autotune:
        sim.step((args.warmup // 2) * S)
        from paper_2211_15963_amd.tune import autotune
        tuned = autotune(sim, bins_per_trial=max(2, args.warmup // 40))
        log(f"autotuned fan-in schedule: {tuned['chosen']}")
        sim.step((args.warmup - args.warmup // 2) * S)
    else:
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
    log(f"timed {args.steps} bins in {wall:.3f} s")
    events = s1["edge_events"] - s0["edge_events"]
    spikes = s1["spikes"] - s0["spikes"]
    bio_s = args.steps * spec.bin_ms * 1e-3
    out = {
        "events": events, "spikes": spikes, "wall": wall, "bio_s": bio_s,
        "rate_hz": spikes / (spec.num_neurons * bio_s),
        "ms_scatter": s1["ms_scatter"] - s0["ms_scatter"], "ms_gather": s1["ms_gather"] - s0["ms_gather"],
        "ms_neuron": s1["ms_neuron"] - s0["ms_neuron"], "ms_readout": s1["ms_readout"] - s0["ms_readout"],
        "timed_bins": s1["timed_bins"] - s0["timed_bins"], "spec": spec, "build_s": s1["build_seconds"],
        "hbm_bytes": s1["hbm_bytes"], "tuning": sim.tuning(),
    }
    sim.close()
    return out


def cpu_baseline(args, budget_s: float):
    """The FP32 oracle, single-threaded, on a 1/64 share of the same recipe."""
    from netgen import configs
    from oracle import Oracle

    n = max(1000, args.n // 64)
    spec = configs.share(n=n, indegree=args.indegree, regime_hz=args.regime, seed=args.seed)
    t0 = time.time()
    o = Oracle(spec, 32)
    log(f"cpu baseline: oracle network {n} neurons built in {time.time() - t0:.1f} s")
    S = spec.steps_per_bin
    o.step(20 * S)  # 20 ms warm-up so that delayed arrivals are flowing
    ev0, b0 = o.edge_events, 0
    t0 = time.perf_counter()
    bins = 0
    while time.perf_counter() - t0 < budget_s:
        o.step(S)
        bins += 1
    wall = time.perf_counter() - t0
    ev = o.edge_events - ev0
    return {"value": ev / wall, "unit": "synaptic events/s", "cores": 1, "kind": "oracle",
            "sample": f"share recipe at N={n} (1/64 of the GPU share), in-degree {args.indegree}, delays 1..10 ms, "
                      f"{bins} bins ({bins} ms bio) after 20 ms warm-up, FP32 oracle on one host core; "
                      f"real-time factor {wall / (bins * 1e-3):.1f}",
            "rtf": wall / (bins * 1e-3)}


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
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000, help="timed 1 ms bins")
    ap.add_argument("--warmup", type=int, default=200, help="untimed 1 ms bins")
    ap.add_argument("--n", type=int, default=6_100_000)
    ap.add_argument("--indegree", type=int, default=556)
    ap.add_argument("--regime", type=int, default=15, choices=[7, 15, 30])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--mode", default="timed", choices=["timed", "graph", "direct"])
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune", action="store_true")
    ap.add_argument("--tune-iters", type=int, default=9)
    ap.add_argument("--calibrate-copy", action="store_true", help="run only a 2 GiB device copy (counter scaling)")
    ap.add_argument("--autotune", type=int, default=1, help="autotune the fan-in schedule during warm-up")
    ap.add_argument("--ensemble", type=int, default=1, help="also run the batched-ensemble comparison")
    ap.add_argument("--members", type=int, default=64)
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
    g = run_gpu(args)
    spec = g["spec"]
    value = g["events"] / g["wall"]
    fan_ms = g["ms_scatter"] + g["ms_gather"]
    nb = max(1, g["timed_bins"])
    roof = None
    if g["timed_bins"]:
        achieved = BYTES_PER_EVENT * g["events"] / (fan_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": "fan-out phase (k_scatter + k_gather)", "achieved": round(achieved, 1),
                "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
                "bytes_per_event": BYTES_PER_EVENT, "events_per_launch": g["events"] / nb,
                "avg_launch_ms": {"k_scatter": g["ms_scatter"] / nb, "k_gather": g["ms_gather"] / nb,
                                  "k_neuron": g["ms_neuron"] / nb, "readout_close": g["ms_readout"] / nb}}
    ens = run_ensemble(args) if args.ensemble else None
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
                   "device_gb": round(g["hbm_bytes"] / 1e9, 2), "fanin_schedule": g["tuning"]},
        "rtf_15hz": g["wall"] / g["bio_s"] if args.regime == 15 else None,
        "ensemble": ens,
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
