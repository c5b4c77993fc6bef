"""GPU path vs the FP32 oracle, element by element, on the code paths that only run at
larger sizes or in rare numerical regimes.

* A 600,000-neuron share network (in-degree 125, delays 1..10 ms): 147 accumulation tiles
  (four per super-tile in the two-pass fan-in), 2,344 neuron blocks (ten compaction groups of
  256 blocks) and one region of 600,000 neurons (ten level-1 readout groups). Full raster,
  V, J, refractory counters, delivered events and region signals, in both fan-in forms.
* FP32 subnormals: a network without background, kicked once by injected spikes, then
  silent long enough for the AMPA and GABA_A conductances to decay into the subnormal
  range (the library keeps denormals; so does the oracle).
* Fixed-point conversion ties: constant weights and a saturating drive make every target's
  bin sum exactly n q(w), chosen half-way between two floats both below and above 2^24,
  with both rounding directions of round-half-even.
* A synchronous burst: nearly every neuron fires in one bin and every delay is one bin, so
  the next bin delivers nearly every edge of the table at once.
"""
import os
import sys

import numpy as np
import pytest

from netgen import configs
from netgen.desc import NetSpec, PopSpec, ProjSpec, RECEPTORS_4, SRC_POP, W_CONST, D_FIXED
from oracle import Oracle, quantize

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _threads():
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _compare(sim, orc, spec, what):
    st_g, id_g = sim.spikes()
    st_o, id_o = orc.spikes()
    assert len(st_o) > 0, f"{what}: no spikes"
    assert len(st_g) == len(st_o), f"{what}: spike counts differ: gpu {len(st_g)} oracle {len(st_o)}"
    assert np.array_equal(st_g, st_o) and np.array_equal(id_g, id_o), f"{what}: rasters differ"
    Vg, Jg, rg = sim.state()
    Vo, Jo, ro = orc.state()
    assert np.array_equal(Vg.astype(np.float64), Vo), f"{what}: V differs"
    assert np.array_equal(Jg.astype(np.float64), Jo), f"{what}: J differs"
    assert np.array_equal(rg, ro), f"{what}: refractory counters differ"
    assert sim.stats()["edge_events"] == orc.edge_events, f"{what}: delivered events differ"


def _compare_regions(sim, orc, spec, what):
    sg, cg = sim.region_signal()
    so, co = orc.region_signal()
    assert sg.shape == so.shape
    assert np.array_equal(cg, co), f"{what}: region spike counts differ"
    # the same double terms summed in two orders differ by at most (n - 1) eps sum |terms|;
    # divided by n, with |current| < 1e5 pA per neuron: n eps 1e5 per region
    n_reg = np.bincount(spec.region_of_neuron(), minlength=spec.n_regions)
    bound = n_reg[None, :] * np.finfo(np.float64).eps * 1e5
    assert np.all(np.abs(sg - so) <= bound), f"{what}: region signals differ beyond the two-order bound"


@pytest.fixture(scope="module")
def Sim():
    from paper_2211_15963_amd import Simulator
    return Simulator


def test_share_600k_element_wise_both_forms(Sim):
    spec = configs.share(n=600_000, indegree=125, seed=31)
    K = 25
    S = spec.steps_per_bin
    _say(f"share 600000 / k125 seed 31: oracle, {K} bins on {_threads()} threads")
    orc = Oracle(spec, 32)
    orc.set_threads(_threads())
    orc.step(K * S)
    assert orc.spikes()[0].size > 100_000
    for single_pass in (False, True):
        _say(f"share 600000 / k125 seed 31: GPU, {K} bins, single_pass={single_pass}")
        sim = Sim(spec, single_pass=single_pass)
        info = sim.info
        assert info.n_tiles == 147
        assert info.fanin_passes == (1 if single_pass else 2)
        assert info.stream_record_bytes == (0 if single_pass else 10)
        n_blocks = (spec.num_neurons + 255) // 256
        assert n_blocks > 2000  # several compaction groups and level-1 readout groups of 256 blocks
        sim.step(K * S)
        _compare(sim, orc, spec, f"600k single_pass={single_pass}")
        _compare_regions(sim, orc, spec, f"600k single_pass={single_pass}")
        sim.close()


def test_subnormal_conductances_bit_exact(Sim):
    spec = configs.tiny(seed=41, bg_rate_hz=0.0)
    for p in spec.pops:
        p.v0_lo, p.v0_hi = -60.0, -55.0
    S = spec.steps_per_bin
    _say("tiny seed 41, no background: injected spikes in bin 0, then 2 s of silence")
    sim = Sim(spec)
    sim.set_spike_injection([0.05, 0.05], 1)
    orc = Oracle(spec, 32)
    orc.set_injection([0.05, 0.05], 1)
    tiny32 = np.finfo(np.float32).tiny
    seen_sub = np.zeros(2, bool)
    for chunk in range(40):
        sim.step(50 * S)
        orc.step(50 * S)
        Jg = sim.state()[1]
        _, Jo, _ = orc.state()
        assert np.array_equal(Jg.astype(np.float64), Jo), f"J differs after {(chunk + 1) * 50} bins"
        sub = (Jo != 0.0) & (np.abs(Jo) < tiny32)
        seen_sub |= sub.any(axis=1)
    # (the decay of a few-ulp subnormal rounds back to itself, so the conductances settle on
    # subnormal values rather than zero: both sides must settle on the same ones)
    assert seen_sub.all(), "the case never reached subnormal AMPA and GABA_A conductances"
    _compare(sim, orc, spec, "subnormal case")
    sim.close()


def _tie_network(seed=51):
    """Four excitatory populations driven to fire at the start of every bin; population p
    receives n_p inputs per bin of the constant weight w_p (both weights of the edge)."""
    cases = [(6, np.float32(0.5 + 2.0 ** -24)),        # 6 q = 3 2^32 + 1536: tie, rounds up
             (6, np.float32(0.5 + 3 * 2.0 ** -24)),    # 6 q = 3 2^32 + 4608: tie, rounds down
             (17, np.float32(2.0 ** -12 + 2.0 ** -32)),  # 17 (2^20 + 1): odd, in [2^24, 2^25): rounds down
             (19, np.float32(2.0 ** -12 + 2.0 ** -32))]  # 19 (2^20 + 1): rounds up
    pops, projs = [], []
    for p, (n, w) in enumerate(cases):
        pops.append(PopSpec(500, True, g=configs.SHARE_G, I_ext=2e5, T_ref=0.9, v0_lo=-55.0, v0_hi=-50.0))
        projs.append(ProjSpec(n, dst_pop=p, src_mode=SRC_POP, src_pop=p, w_dist=W_CONST, w_a=float(w),
                              d_mode=D_FIXED, d_min=1, d_max=1))
    return NetSpec(pops, projs, seed=seed, receptor_mask=RECEPTORS_4, name="ties"), cases


def test_conversion_ties_bit_exact(Sim):
    spec, cases = _tie_network()
    # every case is a true tie of the int64 -> float conversion, in both directions
    dirs = set()
    for n, w in cases:
        s = n * quantize(float(w), 32)
        e = s.bit_length() - 24          # spacing of floats at s is 2^e
        assert e >= 1 and s % (1 << e) == 1 << (e - 1), (n, w, s)
        f = float(np.float32(s))
        dirs.add("up" if f > s else "down")
        assert int(f) == (s + (1 << (e - 1)) if ((s >> e) & 1) else s - (1 << (e - 1)))
    assert dirs == {"up", "down"}
    S = spec.steps_per_bin
    orc = Oracle(spec, 32)
    orc.step(20 * S)
    st, _ = orc.spikes()
    assert len(st) == 20 * spec.num_neurons, "the drive does not fire every neuron in every bin"
    for single_pass in (False, True):
        _say(f"conversion ties, saturated 4 x 500 neurons, 20 bins, single_pass={single_pass}")
        sim = Sim(spec, single_pass=single_pass)
        sim.step(20 * S)
        _compare(sim, orc, spec, f"ties single_pass={single_pass}")
        sim.close()


def test_synchronous_burst_through_the_buffers(Sim):
    """99 % of a 600,000-neuron network fires in bin 0 (spike injection) and every delay is
    one bin, so bin 1 delivers ~99 % of the 6e7 edges at once. Streams and arena sized for
    every edge (1000 per mille) take it without a slow-path event (the worst case of one
    bin); the default shares send most of it past their slices (spills into the arena,
    overflow sums) and give the same bits. Bins 0-1 are checked against the oracle too."""
    spec = configs.share(n=600_000, indegree=100, seed=71, d_max=1)
    S, E = spec.steps_per_bin, spec.num_edges()
    _say("share 600000 / k100, all delays 1, 99 % injected in bin 0: every-edge vs default buffers, 5 bins")
    full = Sim(spec, stream_permille=1000, arena_permille=1000)
    full.set_spike_injection(0.99, 1)
    full.step(2 * S)
    st2 = full.stats()
    assert st2["edge_events"] >= 0.98 * E and st2["spilled_events"] == 0 and st2["overflow_events"] == 0
    orc = Oracle(spec, 32)
    orc.set_threads(_threads())
    orc.set_injection(0.99, 1)
    orc.step(2 * S)
    _compare(full, orc, spec, "burst, bins 0-1")
    full.step(3 * S)
    assert full.stats()["spilled_events"] == 0 and full.stats()["overflow_events"] == 0
    small = Sim(spec)
    small.set_spike_injection(0.99, 1)
    small.step(5 * S)
    st = small.stats()
    assert st["spilled_events"] > 0.1 * E and st["overflow_events"] > 0.5 * E
    a, b = full.spikes(), small.spikes()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    for x, y in zip(full.state(), small.state()):
        assert np.array_equal(x, y)
    assert st["edge_events"] == full.stats()["edge_events"]
    full.close()
    small.close()
