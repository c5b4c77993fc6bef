"""GPU path vs the FP32 oracle on degenerate networks, bit for bit: no synapses (E = 0),
one neuron, a network that never fires (every bin's fan-in is empty), and a saturated
network whose every bin's spike list holds all N neurons (the largest fan-in per bin the
method allows), each in both fan-in forms."""
import sys

import numpy as np
import pytest

from oracle import Oracle

import edge_networks as nets

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _same(sim, orc, spec):
    st_g, id_g = sim.spikes()
    st_o, id_o = orc.spikes()
    assert np.array_equal(st_g, st_o) and np.array_equal(id_g, id_o), "rasters differ"
    Vg, Jg, rg = sim.state()
    Vo, Jo, ro = orc.state()
    assert np.array_equal(Vg.astype(np.float64), Vo), "V differs"
    assert np.array_equal(Jg.astype(np.float64), Jo), "J differs"
    assert np.array_equal(rg, ro), "refractory counters differ"
    assert sim.stats()["edge_events"] == orc.edge_events
    sg, cg = sim.region_signal()
    so, co = orc.region_signal()
    assert sg.shape == so.shape and np.array_equal(cg, co), "region spike counts differ"
    n_reg = np.bincount(spec.region_of_neuron(), minlength=spec.n_regions)
    assert np.all(np.abs(sg - so) <= n_reg[None, :] * np.finfo(np.float64).eps * 1e5)
    return len(st_o)


@pytest.fixture(scope="module")
def Sim():
    from paper_2211_15963_amd import Simulator
    return Simulator


@pytest.mark.parametrize("name,bins", [("no_edges", 200), ("no_edges_share", 30), ("one_neuron", 300),
                                       ("silent", 100), ("saturated", 40)])
def test_degenerate_network_bit_exact(Sim, name, bins):
    spec = getattr(nets, name)()
    S = spec.steps_per_bin
    orc = Oracle(spec, 32)
    orc.step(bins * S)
    n_spk = len(orc.spikes()[0])
    if name == "silent":
        assert n_spk == 0
    elif name == "saturated":
        assert n_spk == bins * spec.num_neurons
    else:
        assert n_spk > 0 and orc.edge_events == 0
    for single_pass in (False, True):
        _say(f"{name}: N={spec.num_neurons}, {bins} bins, single_pass={single_pass}")
        sim = Sim(spec, single_pass=single_pass)
        sim.step(bins * S)
        assert _same(sim, orc, spec) == n_spk
        sim.close()


def test_longest_delays_and_finest_step(Sim):
    """The largest delay a description may hold (255 bins) and the most substeps per bin
    (dt = 1/16 ms, S = 16): 300 bins, so spikes of the first bins arrive 255 bins later."""
    from netgen import configs
    spec = configs.share(n=3000, indegree=100, seed=51, d_max=255)
    spec.dt_ms = 0.0625
    assert spec.steps_per_bin == 16 and spec.max_delay == 255
    S, bins = spec.steps_per_bin, 300
    _say(f"share 3000 / k100, delays 1..255 bins, dt 1/16 ms: oracle, {bins} bins")
    orc = Oracle(spec, 32)
    orc.step(bins * S)
    assert len(orc.spikes()[0]) > 1000
    for single_pass in (False, True):
        _say(f"  GPU, single_pass={single_pass}")
        sim = Sim(spec, single_pass=single_pass)
        assert sim.info.max_delay == 255 and sim.info.steps_per_bin == 16
        sim.step(bins * S)
        _same(sim, orc, spec)
        sim.close()
