"""Conductance initialisation by iterative rescaling (Supplementary Algorithm 1).

The paper initialises the receptor conductances g_u of the resting-state model
off-network: a small unit of the network is simulated, its mean synaptic current
per receptor is measured, and each g_u is multiplied by the ratio of the wanted
current to the measured one, until the measured currents match (Supplementary
Algorithm 1; Methods: it converged in fewer than 20 iterations).

Here the "off-line model" is any network description (typically a scaled-down
recipe), simulated on the GPU through the library. The measured current of
receptor u is the mean over neurons and over sampled bin ends of
g_u J_u (V_u - V), the same per-receptor term whose sum is the region signal,
reduced on the device (dbsim_receptor_currents); the host only averages the
samples and applies the rescaling.
"""
from __future__ import annotations

import copy
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

from .dbsim import Simulator

RECEPTOR_NAMES = ("AMPA", "NMDA", "GABA_A", "GABA_B")


def receptor_currents(sim: Simulator, spec, warm_bins: int, measure_bins: int, every: int = 10) -> np.ndarray:
    """Mean synaptic current per receptor (pA per neuron; AMPA, NMDA, GABA_A, GABA_B) over the
    network, sampled at every `every`-th bin end after warm_bins: each sample is the library's
    device reduction (per-population means of g_u J_u (V_u - V)), weighted by population size."""
    sizes = np.array([p.size for p in spec.pops], np.float64)
    sim.step(warm_bins * sim.S)
    acc = np.zeros(4)
    n = 0
    for _ in range(max(1, measure_bins // every)):
        sim.step(every * sim.S)
        acc += sizes @ sim.receptor_currents() / sizes.sum()
        n += 1
    return acc / n


def gpu_measure(spec, warm_bins: int, measure_bins: int, every: int = 10) -> np.ndarray:
    """The off-line model of Suppl. Algorithm 1 run on the GPU through the library."""
    sim = Simulator(spec, record_regions=False)
    try:
        return receptor_currents(sim, spec, warm_bins, measure_bins, every)
    finally:
        sim.close()


def calibrate_conductances(spec, target_currents: Sequence[float], iterations: int = 20, tol: float = 0.02,
                           warm_bins: int = 100, measure_bins: int = 200, verbose: bool = False,
                           measure: Optional[Callable] = None) -> Dict:
    """Rescales every population's g_u by target_u / measured_u until all present
    receptors are within tol (relative) of their targets, or the iterations run out.
    measure(spec, warm_bins, measure_bins) runs the off-line model (default: gpu_measure).
    Returns the calibrated description, the final conductances and the history."""
    measure = gpu_measure if measure is None else measure
    spec = copy.deepcopy(spec)
    target = np.asarray(target_currents, np.float64)
    present = [u for u in range(4) if any(p.g[u] != 0 for p in spec.pops) and target[u] != 0]
    history: List[Dict] = []
    converged = False
    for it in range(iterations):
        meas = np.asarray(measure(spec, warm_bins, measure_bins), np.float64)
        ratio = np.ones(4)
        for u in present:
            ratio[u] = target[u] / meas[u] if meas[u] != 0 else 2.0
        err = max(abs(1.0 / ratio[u] - 1.0) for u in present) if present else 0.0
        history.append({"iteration": it, "g": [list(p.g) for p in spec.pops], "measured": meas.tolist(),
                        "max_rel_error": err})
        if verbose:
            print(f"[calibrate] it {it}: measured {meas} (max rel error {err:.3g})", flush=True)
        if err <= tol:
            converged = True
            break
        for p in spec.pops:
            p.g = tuple(float(p.g[u] * ratio[u]) if u in present else p.g[u] for u in range(4))
    return {"spec": spec, "g": [list(p.g) for p in spec.pops], "converged": converged, "history": history}
