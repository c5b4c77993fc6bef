"""CPU pins of the library's derived constants against the oracle's (no device needed).

Every per-population constant the kernels use (dt/C, the receptor decays exp(-dt/tau),
the refractory steps and the Poisson background inversion table) is derived on the host
from the description. A one-count error in one Poisson threshold would flip a background
draw with probability about 2^-32 per step, so no trajectory comparison would see it;
these tests compare the library's table with the oracle's bit for bit instead, for every
workload recipe and across the range of background rates the table accepts (the paper's
GPU-vs-CPU check of a debug graph, Results, precision of the simulation)."""
import math

import numpy as np
import pytest

from netgen import configs
from netgen.desc import NetSpec, PopSpec, RECEPTORS_2, RECEPTORS_4
from oracle import Oracle, poisson_table

MAX_POISSON = 64


@pytest.fixture(scope="module")
def D():
    from paper_2211_15963_amd import dbsim
    return dbsim


def _check_equal(lib_pops, spec_list):
    q = 0
    first = 0
    for m, spec in enumerate(spec_list):
        orc = Oracle(spec, 32, params_only=True)
        for p, pop in enumerate(spec.pops):
            L = lib_pops[q]
            O = orc.pop_constants(p)
            assert L["member"] == m
            assert L["first_neuron"] == first and L["end_neuron"] == first + pop.size
            assert L["k"].tobytes() == O["k"].tobytes(), (m, p)
            assert L["decay"].tobytes() == O["decay"].tobytes(), (m, p)
            assert L["ref_steps"] == O["ref_steps"], (m, p)
            assert len(L["poisson_T"]) == len(O["poisson_T"]), (m, p)
            assert np.array_equal(L["poisson_T"], O["poisson_T"]), (m, p)
            first += pop.size
            q += 1
        del orc
    assert q == len(lib_pops)


@pytest.mark.parametrize("name,spec", [
    ("tiny", configs.tiny(seed=0)),
    ("tiny_dt1", configs.tiny(seed=0, dt_ms=1.0)),
    ("share7", configs.share(n=20000, regime_hz=7)),
    ("share15", configs.share(n=20000, regime_hz=15)),
    ("share30", configs.share(n=20000, regime_hz=30)),
    ("multi_region", configs.multi_region(n_regions=20, per_region=1000)),
])
def test_recipe_constants_equal_oracle(D, name, spec):
    _check_equal(D.derive_constants(spec), [spec])


def test_ensemble_and_served_constants_equal_oracle(D):
    members = [configs.ensemble_member(m, seed=0) for m in range(64)]
    _check_equal(D.derive_constants(members), members)
    for r in range(40):
        spec, _ = configs.served_request(r, seed=0)
        _check_equal(D.derive_constants(spec), [spec])


def _rate_spec(rates_hz, dt_ms=0.1):
    pops = [PopSpec(10, True, g=configs.SHARE_G, bg_rate_hz=float(r), w_bg=configs.SHARE_W_BG) for r in rates_hz]
    return NetSpec(pops, [], seed=3, dt_ms=dt_ms, bin_ms=1.0, receptor_mask=RECEPTORS_4, name="rates")


def _lambda_of_length(n):
    """Smallest lambda (bisection on the oracle's table length) whose table has more than n entries."""
    lo, hi = 0.0, 100.0
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        if len(poisson_table(mid)) > n:
            hi = mid
        else:
            lo = mid
    return hi


def test_poisson_tables_across_rates(D):
    """Background rates from zero up to the last one whose table fits 64 entries: the library's
    thresholds equal the oracle's; just above it, the library refuses the description."""
    dt = 0.1
    lam_max = _lambda_of_length(MAX_POISSON)  # first lambda with 65 entries
    lams = [0.0, 1e-9, 1e-4, 0.2, 0.659, 0.823, 1.1277, 2.0, 5.0, 10.0]
    for n in (40, 50, 60, 62, 63, 64):
        lo = _lambda_of_length(n - 1)
        lams += [lo, np.nextafter(lo, 0.0) if lo > 0 else lo]
    lams += [np.nextafter(lam_max, 0.0) * (1 - 1e-12)]
    rates = [float(l) / (dt * 1e-3) for l in lams]
    # the description carries the rate as float32; keep only rates whose float32 value stays
    # inside the 64-entry range
    rates = [r for r in rates if len(poisson_table(float(np.float32(r)) * dt * 1e-3)) <= MAX_POISSON]
    spec = _rate_spec(rates, dt)
    lib = D.derive_constants(spec)
    _check_equal(lib, [spec])
    lens = sorted({len(p["poisson_T"]) for p in lib})
    assert lens[0] == 0 and lens[-1] >= 60
    # one step past the limit: the oracle's longer table, and the library's refusal
    r_over = float(np.float32(lam_max * 1.001 / (dt * 1e-3)))
    assert len(poisson_table(r_over * dt * 1e-3)) > MAX_POISSON
    with pytest.raises(D.DbsimError) as e:
        D.derive_constants(_rate_spec([r_over], dt))
    assert e.value.code == D.EINVAL


def test_random_descriptions(D):
    """Random parameter values (capacitance, time constants including +inf, refractory
    periods, rates, dt of 0.1 and 1 ms): k, decays and refractory steps agree bit for bit."""
    rng = np.random.default_rng(7)
    for dt in (0.1, 1.0):
        pops = []
        for _ in range(200):
            tau = [float(x) for x in rng.uniform(0.3, 400.0, 4)]
            tau[int(rng.integers(4))] = math.inf
            pops.append(PopSpec(int(rng.integers(1, 50)), bool(rng.integers(2)), C=float(rng.uniform(20, 2000)),
                                g_L=float(rng.uniform(1, 60)), T_ref=float(rng.uniform(1.0, 25.0)),
                                tau=tuple(tau), g=configs.SHARE_G, bg_rate_hz=float(rng.uniform(0, 20000 if dt < 1 else 2000)),
                                w_bg=1.0))
        for mask in (RECEPTORS_2, RECEPTORS_4):
            spec = NetSpec(pops, [], seed=5, dt_ms=dt, bin_ms=1.0, receptor_mask=mask, name="random")
            _check_equal(D.derive_constants(spec), [spec])


def test_derive_constants_errors(D):
    spec = configs.tiny(seed=0)
    spec.pops[0].T_ref = 0.5  # below bin - dt: a neuron could spike twice in a bin
    with pytest.raises(D.DbsimError) as e:
        D.derive_constants(spec)
    assert e.value.code == D.EINVAL
