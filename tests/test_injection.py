"""Initial spike injection (Methods: the output train of every neuron carries a spike with
a small probability per bin at the start) in the oracle, pinned by an independent
numpy Philox and by the delivered-event count."""
import numpy as np

from netgen import configs
from oracle import Oracle
from oracle.brute import philox_np


def _silent(seed=2):
    """tiny network with no background and a low start: nothing fires by itself"""
    s = configs.tiny(seed=seed, bg_rate_hz=0.0)
    for p in s.pops:
        p.v0_lo, p.v0_hi = -69.0, -68.0
    return s


def _expected(spec, p, bins):
    """(bin, id) pairs whose injection word falls below floor(p 2^32)"""
    N = spec.num_neurons
    T = int(np.floor(np.float64(np.float32(p)) * 2.0**32))
    ids = np.arange(N)
    out = []
    for k in range(bins):
        w0, _, _, _ = philox_np(np.full(N, k), np.full(N, k >> 32), ids, np.full(N, (2 << 24) | spec.net_id),
                                spec.seed & 0xFFFFFFFF, spec.seed >> 32)
        for i in np.nonzero(w0 < T)[0]:
            out.append((k, int(i)))
    return out


def test_silent_network_raster_is_the_injection():
    spec = _silent()
    S = spec.steps_per_bin
    o = Oracle(spec, 32)
    o.set_injection(0.01, 150)
    o.step(200 * S)
    st, ids = o.spikes()
    exp = _expected(spec, 0.01, 150)
    assert len(exp) > 1000  # about 1 % of 1000 neurons over 150 bins
    assert np.array_equal(st, np.array([k * S + S - 1 for k, _ in exp], np.uint64))
    assert np.array_equal(ids, np.array([i for _, i in exp], np.uint32))
    # the injected spikes are delivered: one event per out-edge of every injected spike
    _, src, _, _, _ = o.in_edges()
    outdeg = np.bincount(src, minlength=spec.num_neurons)
    delivered = sum(int(outdeg[i]) for k, i in exp if k + 1 < 200)
    assert o.edge_events == delivered


def test_injection_does_not_reset_and_keeps_one_spike_per_bin():
    spec = configs.tiny(seed=4)
    S = spec.steps_per_bin
    plain = Oracle(spec, 32)
    plain.step(5 * S)
    inj = Oracle(spec, 32)
    inj.set_injection([0.3, 0.0], 5)  # excitatory population only
    inj.step(5 * S)
    a, b = plain.spikes(), inj.spikes()
    st, ids = b
    keys = st // S * spec.num_neurons + ids
    assert len(np.unique(keys)) == len(keys)  # at most one output spike per neuron and bin
    # bin 0 (before anything injected is delivered): the real spikes are the plain run's,
    # the extra ones are excitatory neurons stamped at the bin's last step
    pa = set(zip(a[0][a[0] < S].tolist(), a[1][a[0] < S].tolist()))
    pb = set(zip(st[st < S].tolist(), ids[st < S].tolist()))
    assert pa <= pb
    extra = pb - pa
    assert extra and all(s_ == S - 1 and i < 800 for s_, i in extra)
    assert not any(i in {i2 for _, i2 in pa} for _, i in extra)
    # off: bins = 0
    off = Oracle(spec, 32)
    off.set_injection(0.5, 0)
    off.step(5 * S)
    assert np.array_equal(off.spikes()[0], plain.spikes()[0])
