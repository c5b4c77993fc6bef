"""Seeded synthetic workload recipes.

Every input is synthetic: the paper's networks are built from a subject's
MRI/DWI/PET data that are not available, so these recipes reproduce the shapes
the paper works at (population sizes, 4:1 excitatory:inhibitory ratio,
fixed in-degree, U[0,1] weights, two weight channels, 1 ms bins with a
0.1 ms Euler step) with seeded random draws.

Recipes
-------
tiny            1,000 neurons (800 E / 200 I), in-degree 100, lognormal weights
                (mean 0.5, s.d. 0.5; inhibitory x4), one 1 ms delay, AMPA + GABA_A,
                2 kHz Poisson background.
share           one GPU's share of the whole-brain model: N neurons (default 6.1 M),
                80/20 E/I, in-degree 556 from all other neurons, U[0,1] weights
                (inhibitory x4), two weights per edge, 4 receptors, delays uniform
                1..10 ms, Poisson background tuned for 7 / 15 / 30 Hz.
multi_region    R regions x M neurons (default 200 x 5,000), 80/20 E/I, intra-region
                in-degree 400 (delay 1 ms) plus 100 excitatory long-range inputs from
                the other regions, delay = ceil(distance / 5 mm/ms) clamped to 1..20 ms,
                region centres uniform in a 57.7 mm cube.
ensemble_member member m of a batched ensemble: N log-uniform in [2e4, 5e5],
                in-degree uniform in 200..600, background rate and per-receptor
                conductances each scaled by U[0.7, 1.3].
served_request  request r of a served stream: N log-uniform in [1e4, 2e6], in-degree
                uniform in 200..600, regime uniform over 7 / 15 / 30 Hz, duration
                uniform in [0.1, 2] s of biological time (whole 1 ms bins); the
                arrival times form a seeded Poisson process (arrival_times).
"""
from __future__ import annotations

import math

import numpy as np

from .desc import (NetSpec, PopSpec, ProjSpec, RECEPTORS_2, RECEPTORS_4, SRC_ALL, SRC_SAME_REGION,
                   SRC_OTHER_REGIONS, CLASS_ANY, CLASS_EXC, W_UNIFORM, W_LOGNORMAL, D_FIXED, D_UNIFORM,
                   D_DISTANCE)

# lognormal with mean 0.5 and s.d. 0.5: sigma^2 = ln(1 + CV^2) = ln 2, mu = ln(mean) - sigma^2/2
LOGN_SIGMA = math.sqrt(math.log(2.0))
LOGN_MU = math.log(0.5) - math.log(2.0) / 2.0

# conductances (nS) for the two-receptor tiny network: AMPA, -, GABA_A, -
TINY_G = (2.0, 0.0, 2.5, 0.0)
TINY_W_BG = 1.2

# four-receptor networks: AMPA:NMDA current split 0.3:0.7 and GABA_A:GABA_B 0.5:0.5
# (Suppl. Section 2, parameter initialisation) at the default time constants.
SHARE_G = (0.20, 0.0096, 0.40, 0.0115)
SHARE_W_BG = 4.0
# Poisson background rate (Hz per neuron) per target regime, found by bisection on the
# population rate of the seeded 'share' recipe (see the benchmark's tuning mode).
SHARE_BG_HZ = {7: 6590.0, 15: 8230.0, 30: 11277.0}

REGION_G = (0.22, 0.0106, 0.44, 0.0126)
REGION_BG_HZ = 8230.0


def tiny(seed: int = 0, dt_ms: float = 0.1, n_exc: int = 800, n_inh: int = 200, indegree: int = 100,
         bg_rate_hz: float = 2000.0) -> NetSpec:
    common = dict(g=TINY_G, bg_rate_hz=bg_rate_hz, w_bg=TINY_W_BG, v0_lo=-55.0, v0_hi=-50.0)
    pops = [PopSpec(n_exc, True, **common), PopSpec(n_inh, False, **common)]
    projs = [ProjSpec(indegree, src_mode=SRC_ALL, w_dist=W_LOGNORMAL, w_a=LOGN_MU, w_b=LOGN_SIGMA,
                      w_scale_exc=1.0, w_scale_inh=4.0, d_mode=D_FIXED, d_min=1, d_max=1)]
    return NetSpec(pops, projs, seed=seed, dt_ms=dt_ms, bin_ms=1.0, receptor_mask=RECEPTORS_2,
                   name=f"tiny-{n_exc + n_inh}")


def share(n: int = 6_100_000, indegree: int = 556, regime_hz: int = 15, seed: int = 0, d_max: int = 10,
          bg_rate_hz: float | None = None, g_scale: float = 1.0) -> NetSpec:
    n_exc = int(round(0.8 * n))
    n_inh = n - n_exc
    bg = SHARE_BG_HZ[regime_hz] if bg_rate_hz is None else bg_rate_hz
    g = tuple(x * g_scale for x in SHARE_G)
    common = dict(g=g, bg_rate_hz=bg, w_bg=SHARE_W_BG, v0_lo=-55.0, v0_hi=-50.0)
    pops = [PopSpec(n_exc, True, **common), PopSpec(n_inh, False, **common)]
    projs = [ProjSpec(indegree, src_mode=SRC_ALL, w_dist=W_UNIFORM, w_a=0.0, w_b=1.0,
                      w_scale_exc=1.0, w_scale_inh=4.0, d_mode=D_UNIFORM, d_min=1, d_max=d_max)]
    return NetSpec(pops, projs, seed=seed, dt_ms=0.1, bin_ms=1.0, receptor_mask=RECEPTORS_4,
                   name=f"share-{n}-k{indegree}-{regime_hz}hz")


def region_layout(n_regions: int, seed: int, side_mm: float = 57.7) -> np.ndarray:
    rng = np.random.default_rng([seed, 0x5EED, n_regions])
    return (rng.random((n_regions, 3)) * side_mm).astype(np.float32)


def multi_region(n_regions: int = 200, per_region: int = 5000, intra_indegree: int = 400,
                 long_indegree: int = 100, seed: int = 0, bg_rate_hz: float = REGION_BG_HZ,
                 d_max: int = 20) -> NetSpec:
    n_exc = int(round(0.8 * per_region))
    n_inh = per_region - n_exc
    common = dict(g=REGION_G, bg_rate_hz=bg_rate_hz, w_bg=SHARE_W_BG, v0_lo=-55.0, v0_hi=-50.0)
    pops = []
    for r in range(n_regions):
        pops.append(PopSpec(n_exc, True, region=r, **common))
        pops.append(PopSpec(n_inh, False, region=r, **common))
    projs = [ProjSpec(intra_indegree, src_mode=SRC_SAME_REGION, src_class=CLASS_ANY, w_dist=W_UNIFORM,
                      w_a=0.0, w_b=1.0, w_scale_inh=4.0, d_mode=D_FIXED, d_min=1, d_max=1)]
    if long_indegree > 0 and n_regions > 1:
        projs.append(ProjSpec(long_indegree, src_mode=SRC_OTHER_REGIONS, src_class=CLASS_EXC, w_dist=W_UNIFORM,
                              w_a=0.0, w_b=1.0, d_mode=D_DISTANCE, d_min=1, d_max=d_max))
    return NetSpec(pops, projs, n_regions=n_regions, seed=seed, dt_ms=0.1, bin_ms=1.0,
                   receptor_mask=RECEPTORS_4, velocity_mm_per_ms=5.0,
                   region_xyz_mm=region_layout(n_regions, seed), name=f"regions-{n_regions}x{per_region}")


def ensemble_member(m: int, seed: int = 0, n_lo: float = 2e4, n_hi: float = 5e5) -> NetSpec:
    rng = np.random.default_rng([seed, 0xE25E, m])
    n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
    k = int(rng.integers(200, 601))
    bg_scale = rng.uniform(0.7, 1.3)
    g_scale = rng.uniform(0.7, 1.3, size=4)
    n_exc = int(round(0.8 * n))
    g = tuple(float(SHARE_G[u] * g_scale[u]) for u in range(4))
    common = dict(g=g, bg_rate_hz=float(SHARE_BG_HZ[15] * bg_scale), w_bg=SHARE_W_BG, v0_lo=-55.0, v0_hi=-50.0)
    pops = [PopSpec(n_exc, True, **common), PopSpec(n - n_exc, False, **common)]
    projs = [ProjSpec(k, src_mode=SRC_ALL, w_dist=W_UNIFORM, w_a=0.0, w_b=1.0, w_scale_inh=4.0,
                      d_mode=D_UNIFORM, d_min=1, d_max=10)]
    return NetSpec(pops, projs, seed=seed * 1000003 + m, net_id=m, dt_ms=0.1, bin_ms=1.0,
                   receptor_mask=RECEPTORS_4, name=f"member-{m}")


def served_request(r: int, seed: int = 0, n_lo: float = 1e4, n_hi: float = 2e6, d_lo_s: float = 0.1,
                   d_hi_s: float = 2.0):
    """(network, biological duration in steps) of request r of a served stream."""
    rng = np.random.default_rng([seed, 0x5E7E, r])
    n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
    k = int(rng.integers(200, 601))
    regime = int(rng.choice([7, 15, 30]))
    bins = int(round(rng.uniform(d_lo_s, d_hi_s) * 1000.0))
    spec = share(n=n, indegree=k, regime_hz=regime, seed=seed * 1000003 + r)
    spec.net_id = r & 0xFFFFFF
    spec.name = f"request-{r}-{n}-k{k}-{regime}hz"
    return spec, bins * spec.steps_per_bin


def arrival_times(count: int, rate_per_s: float, seed: int = 0) -> np.ndarray:
    """Seeded Poisson arrival process: cumulative exponential gaps (seconds)."""
    rng = np.random.default_rng([seed, 0xA11E])
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=count))
