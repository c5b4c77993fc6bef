"""Conductance initialisation (Supplementary Algorithm 1) on the GPU.

* The measurement (mean current per receptor and population, reduced on the device) equals
  the FP32 oracle's at the same state, within the rounding bound of two summation orders of
  the same double terms.
* The calibration iteration run on the GPU and the same iteration run on the FP32 oracle give
  the same conductances and measurements, iteration by iteration.
* Starting from perturbed conductances, the GPU calibration recovers the per-receptor
  currents the oracle measures at the recipe's conductances.
"""
import os
import sys

import numpy as np
import pytest

from netgen import configs
from oracle import Oracle

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _oracle_measure(spec, warm_bins, measure_bins, every=10):
    """The same off-line model on the FP32 oracle: population-size-weighted means of the
    oracle's per-population receptor currents, sampled every `every` bins."""
    o = Oracle(spec, 32)
    o.set_threads(max(1, min(16, len(os.sched_getaffinity(0)))))
    S = spec.steps_per_bin
    sizes = np.array([p.size for p in spec.pops], np.float64)
    o.step(warm_bins * S)
    acc = np.zeros(4)
    n = 0
    for _ in range(max(1, measure_bins // every)):
        o.step(every * S)
        acc += sizes @ o.receptor_currents() / sizes.sum()
        n += 1
    return acc / n


def test_receptor_currents_equal_the_oracle():
    from paper_2211_15963_amd import Simulator
    for spec in (configs.share(n=6000, indegree=150, seed=22), configs.tiny(seed=23),
                 configs.multi_region(n_regions=4, per_region=1500, seed=24)):
        _say(f"{spec.name}: receptor currents after 25 bins, GPU vs oracle")
        sim = Simulator(spec, record_regions=False)
        sim.step(25 * spec.steps_per_bin)
        got = sim.receptor_currents()
        sim.close()
        o = Oracle(spec, 32)
        o.step(25 * spec.steps_per_bin)
        want = o.receptor_currents()
        assert got.shape == want.shape == (len(spec.pops), 4)
        assert np.any(want != 0)
        # the same double terms summed in two orders: (n - 1) eps sum |t| / n, |t| < 1e5 pA
        assert np.all(np.abs(got - want) <= 1e5 * np.finfo(np.float64).eps), np.max(np.abs(got - want))


def test_calibration_iteration_equals_the_oracle_iteration():
    from paper_2211_15963_amd.calibrate import calibrate_conductances
    spec = configs.share(n=3000, indegree=120, seed=25)
    for p in spec.pops:
        p.g = tuple(x * f for x, f in zip(p.g, (1.2, 0.9, 1.15, 0.8)))
    target = (60.0, 20.0, -50.0, -10.0)
    _say("share 3000 / k120: 3 calibration iterations on the GPU and on the oracle")
    gpu = calibrate_conductances(spec, target, iterations=3, tol=0.0, warm_bins=20, measure_bins=30)
    orc = calibrate_conductances(spec, target, iterations=3, tol=0.0, warm_bins=20, measure_bins=30,
                                 measure=_oracle_measure)
    assert len(gpu["history"]) == len(orc["history"]) == 3
    for a, b in zip(gpu["history"], orc["history"]):
        assert a["g"] == b["g"], (a["g"], b["g"])
        np.testing.assert_allclose(a["measured"], b["measured"], rtol=1e-12, atol=1e-9)
    assert gpu["g"] == orc["g"]


def test_calibration_recovers_oracle_currents():
    from paper_2211_15963_amd.calibrate import calibrate_conductances
    spec = configs.share(n=20000, indegree=300, seed=21)
    _say("share 20000 / k300: target currents measured by the oracle at the recipe's conductances")
    target = _oracle_measure(spec, 100, 200)
    assert target[0] > 0 and target[2] < 0  # excitatory inward, inhibitory outward
    start = configs.share(n=20000, indegree=300, seed=21)
    for p in start.pops:
        p.g = tuple(x * f for x, f in zip(p.g, (1.3, 0.8, 1.2, 0.85)))
    _say(f"calibrating on the GPU from perturbed conductances towards {np.round(target, 3)} pA")
    out = calibrate_conductances(start, target, iterations=20, tol=0.03)
    errs = [h["max_rel_error"] for h in out["history"]]
    _say(f"relative errors per iteration: {np.round(errs, 4)}")
    assert out["converged"], errs
    assert errs[-1] < errs[0]
