"""Oracle pins on degenerate networks: what the method fixes when there are no synapses,
no spikes, or as many spikes as it allows. Each expected value follows from the step's
definition (the explicit Euler update, the refractory hold of r steps after the spike
step, delivery at the start of bin b + d) without running the step itself."""
import numpy as np

from oracle import Oracle

import edge_networks as nets


def test_saturating_drive_fires_every_neuron_at_every_bin_start():
    """With a drive that crosses threshold from V_reset in one step and r = S - 1, a neuron
    fires at step 0 (every V0 is within 40 mV of threshold) and then after every hold of r
    steps: its spike steps are exactly 0, S, 2S, ... (the refractory reading: the minimum
    interspike interval is r + 1 steps)."""
    spec = nets.saturated(n=300, indegree=40)
    S = spec.steps_per_bin
    N = spec.num_neurons
    B = 50
    o = Oracle(spec, 32)
    o.step(B * S)
    st, ids = o.spikes()
    want_st = np.repeat(np.arange(B, dtype=np.uint64) * S, N)
    want_ids = np.tile(np.arange(N, dtype=np.uint32), B)
    np.testing.assert_array_equal(st, want_st)
    np.testing.assert_array_equal(ids, want_ids)
    # the last spike was at step (B-1) S; the r = S - 1 steps after it held V at V_reset and
    # counted the hold down to zero
    V, J, ref = o.state()
    assert np.all(V == np.float64(np.float32(spec.pops[0].V_reset)))
    assert np.all(ref == 0)
    # delivery: a spike of bin b reaches its delay-d edges at the start of bin b + d, so
    # after B bins edge e (delay d_e) has delivered once for each b <= B - 1 - d_e
    ptr, src, w0, w1, dl = o.in_edges()
    assert o.edge_events == int(np.maximum(0, B - dl.astype(np.int64)).sum())


def test_network_without_synapses_has_no_arrivals():
    """E = 0: no event is delivered, the GABA_A conductance never leaves zero, the AMPA one
    carries the Poisson background alone, and neurons still fire from it."""
    spec = nets.no_edges()
    o = Oracle(spec, 32)
    o.step(200 * spec.steps_per_bin)
    assert o.edge_events == 0
    st, _ = o.spikes()
    assert len(st) > 0
    V, J, ref = o.state()
    assert np.all(J[1] == 0.0)
    assert np.all(J[0] >= 0.0) and np.any(J[0] > 0.0)


def test_silent_network_relaxes_without_spikes():
    """No background and every V below threshold: nothing fires, no conductance is ever
    opened, and every V moves monotonically toward V_L (the relaxation factor 1 - k g_L
    lies in (0, 1))."""
    spec = nets.silent()
    o = Oracle(spec, 32)
    V0 = o.state()[0].copy()
    o.step(100 * spec.steps_per_bin)
    st, _ = o.spikes()
    assert len(st) == 0 and o.edge_events == 0
    V, J, ref = o.state()
    assert np.all(J == 0.0) and np.all(ref == 0)
    V_L = float(spec.pops[0].V_L)
    assert np.all(np.abs(V - V_L) <= np.abs(V0 - V_L))
    assert np.all(np.sign(V - V_L) == np.sign(V0 - V_L))
