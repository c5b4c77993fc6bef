"""Conductance initialisation by iterative rescaling (Supplementary Algorithm 1).

The paper initialises the receptor conductances g_u of the resting-state model
off-network: a small unit of the network is simulated, its mean synaptic current
per receptor is measured, and each g_u is multiplied by the ratio of the wanted
current to the measured one, until the measured currents match (Supplementary
Algorithm 1; Methods: it converged in fewer than 20 iterations).

Here the "off-line model" is any network description (typically a scaled-down
recipe), simulated on the GPU through the library. The measured current of
receptor u is the mean over neurons and over sampled bin ends of
g_u J_u (V_u - V), the same per-receptor term whose sum is the region signal.
"""
from __future__ import annotations

import copy
from typing import Dict, List, Optional, Sequence

import numpy as np

from .dbsim import Simulator

RECEPTOR_NAMES = ("AMPA", "NMDA", "GABA_A", "GABA_B")


def receptor_currents(sim: Simulator, spec, warm_bins: int, measure_bins: int, every: int = 10) -> np.ndarray:
    """Mean synaptic current per receptor slot (pA per neuron), sampled at bin ends."""
    U = sim.U
    slots = [0, 1, 2, 3] if U == 4 else [0, 2]
    g = np.zeros((U, spec.num_neurons), np.float64)
    Vu = np.zeros((U, spec.num_neurons), np.float64)
    off = 0
    for p in spec.pops:
        for j, u in enumerate(slots):
            g[j, off:off + p.size] = p.g[u]
            Vu[j, off:off + p.size] = p.V_rev[u]
        off += p.size
    sim.step(warm_bins * sim.S)
    acc = np.zeros(U)
    n = 0
    for _ in range(max(1, measure_bins // every)):
        sim.step(every * sim.S)
        V, J, _ = sim.state()
        acc += np.mean(g * J.astype(np.float64) * (Vu - V.astype(np.float64)[None, :]), axis=1)
        n += 1
    out = np.zeros(4)
    out[slots] = acc / n
    return out


def calibrate_conductances(spec, target_currents: Sequence[float], iterations: int = 20, tol: float = 0.02,
                           warm_bins: int = 100, measure_bins: int = 200, verbose: bool = False) -> Dict:
    """Rescales every population's g_u by target_u / measured_u until all present
    receptors are within tol (relative) of their targets, or the iterations run out.
    Returns the calibrated description, the final conductances and the history."""
    spec = copy.deepcopy(spec)
    target = np.asarray(target_currents, np.float64)
    present = [u for u in range(4) if any(p.g[u] != 0 for p in spec.pops) and target[u] != 0]
    history: List[Dict] = []
    converged = False
    for it in range(iterations):
        sim = Simulator(spec, record_regions=False)
        meas = receptor_currents(sim, spec, warm_bins, measure_bins)
        sim.close()
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
