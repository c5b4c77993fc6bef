"""Autotuner of the fan-in schedule.

Tries scatter schedules (workgroups per CU, LDS round size, chunks per workgroup) on a
live simulator for a few bins each, timing the fan-in kernels with the library's
phase events, and keeps the fastest per delivered event. Every schedule gives
bit-identical results (the arrival sums are exact integers), so tuning changes speed
only; the bins it runs are ordinary simulation steps.
"""
from __future__ import annotations

from typing import Dict, List, Optional, Tuple

from .dbsim import DbsimError, Simulator


def candidates(sim: Simulator) -> List[Tuple[int, int, int]]:
    out = []
    for wgs in (2, 4, 6, 8):
        for cpw in (1, 4):
            for re_div in (1, 2):
                out.append((wgs, re_div, cpw))
    return out


def autotune(sim: Simulator, bins_per_trial: int = 10, verbose: bool = False) -> Dict:
    """Returns the chosen schedule and the per-candidate timings (ms per million events)."""
    was = sim.tuning()
    sim.set_timing(True)
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
        s0 = sim.stats()
        sim.step(bins_per_trial * sim.S)
        s1 = sim.stats()
        ev = s1["edge_events"] - s0["edge_events"]
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
