"""Autotuner of the fan-in schedule.

Tries scatter schedules (workgroups per CU, LDS round size, chunks per workgroup) on a
live simulator for a few bins each and keeps the fastest per delivered event, timed
either as the fan-in kernels alone (the library's phase events, one stream) or as the
wall time of whole bins replayed from graphs (the partition then shares the CUs with the
neuron step, and its registers and workgroup count matter beyond its own speed). Every
schedule gives bit-identical results (the arrival sums are exact integers), so tuning
changes speed only; the bins it runs are ordinary simulation steps.
"""
from __future__ import annotations

import time
from typing import Dict, List, Optional, Tuple

from .dbsim import DbsimError, Simulator


def candidates(sim: Simulator) -> List[Tuple[int, int, int]]:
    """(workgroups per CU, round-size divisor, chunks per workgroup). The single-pass form
    runs one or two workgroups of 1,024 threads per CU; the two-pass form two to eight of 512."""
    out = []
    wgs_set = (1, 2) if sim.info.fanin_passes == 1 else (2, 4, 6, 8)
    for wgs in wgs_set:
        for cpw in (1, 4):
            for re_div in (1, 2):
                out.append((wgs, re_div, cpw))
    return out


def autotune(sim: Simulator, bins_per_trial: int = 10, verbose: bool = False, mode: str = "phases") -> Dict:
    """Returns the chosen schedule and the per-candidate timings (ms per million events).
    mode: "phases" (fan-in kernels, phase events) or "wall" (whole replayed bins)."""
    if mode not in ("phases", "wall"):
        raise ValueError("mode must be 'phases' or 'wall'")
    was = sim.tuning()
    sim.set_timing(mode == "phases")
    results = []
    best: Optional[Tuple[float, Dict]] = None
    for wgs, re_div, cpw in candidates(sim):
        try:
            sim.set_tuning(scatter_wgs_per_cu=wgs, round_events=0, chunks_per_wg=cpw)
            if re_div > 1:
                cur = sim.tuning()["round_events"]
                re = max(256, (cur // re_div) // 256 * 256)
                sim.set_tuning(scatter_wgs_per_cu=wgs, round_events=re, chunks_per_wg=cpw)
        except DbsimError:
            continue
        if mode == "wall":
            sim.step(2 * sim.S)  # the new schedule's graphs are captured here
            sim.sync()
        s0 = sim.stats()
        t0 = time.perf_counter()
        sim.step(bins_per_trial * sim.S)
        if mode == "wall":
            sim.sync()
        wall_ms = (time.perf_counter() - t0) * 1e3
        s1 = sim.stats()
        ev = s1["edge_events"] - s0["edge_events"]
        if mode == "wall":
            ms = wall_ms
        else:
            ms = (s1["ms_scatter"] - s0["ms_scatter"]) + (s1["ms_gather"] - s0["ms_gather"])
        score = ms / max(ev, 1) * 1e6
        t = sim.tuning()
        results.append({**t, "ms_per_mevent": score})
        if verbose:
            print(f"[autotune] {t} -> {score:.4f} ms per 1e6 events", flush=True)
        if best is None or score < best[0]:
            best = (score, t)
    sim.set_timing(False)
    if best is None:
        sim.set_tuning(**was)
        return {"chosen": was, "trials": results}
    sim.set_tuning(**best[1])
    return {"chosen": best[1], "trials": results}
