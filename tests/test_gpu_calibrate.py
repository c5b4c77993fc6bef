"""Conductance initialisation (Supplementary Algorithm 1) on the GPU: starting from
perturbed conductances, iterative rescaling recovers per-receptor currents measured
at known conductances."""
import sys

import numpy as np
import pytest

from netgen import configs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def test_calibration_recovers_target_currents():
    from paper_2211_15963_amd import Simulator
    from paper_2211_15963_amd.calibrate import calibrate_conductances, receptor_currents
    spec = configs.share(n=20000, indegree=300, seed=21)
    _say("share 20000 / k300: currents at the recipe's conductances")
    sim = Simulator(spec, record_regions=False)
    target = receptor_currents(sim, spec, 100, 200)
    sim.close()
    assert target[0] > 0 and target[2] < 0  # excitatory inward, inhibitory outward
    start = configs.share(n=20000, indegree=300, seed=21)
    for p in start.pops:
        p.g = tuple(x * f for x, f in zip(p.g, (1.3, 0.8, 1.2, 0.85)))
    _say(f"calibrating from perturbed conductances towards {np.round(target, 3)} pA")
    out = calibrate_conductances(start, target, iterations=20, tol=0.03)
    errs = [h["max_rel_error"] for h in out["history"]]
    _say(f"relative errors per iteration: {np.round(errs, 4)}")
    assert out["converged"], errs
    assert errs[-1] < errs[0]
