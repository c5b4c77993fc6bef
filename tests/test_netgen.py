"""Host tests of the seeded network generator (fixed in-degree sampling without
replacement, no autapses or multapses; Extended Data Table 2 "Connectivity")."""
import math

import numpy as np
import pytest

from netgen import configs
from netgen.desc import (NetSpec, PopSpec, ProjSpec, RECEPTORS_4, SRC_ALL, SRC_SAME_REGION, SRC_OTHER_REGIONS,
                         CLASS_EXC, W_UNIFORM, D_DISTANCE, generate, validate)


def _check_graph(spec, net):
    N = spec.num_neurons
    off = spec.pop_offsets()
    region = spec.region_of_neuron()
    exc = spec.is_exc_neuron()
    ptr, src, dl = net["ptr"], net["src"], net["delay"]
    for i in range(N):
        s = src[ptr[i]:ptr[i + 1]]
        assert i not in set(s.tolist()), "autapse"
        assert len(set(s.tolist())) == len(s), "multapse"
        assert np.all(s < N)
    return off, region, exc


def test_tiny_fixed_indegree_and_weights():
    spec = configs.tiny()
    net = generate(spec)
    assert np.all(np.diff(net["ptr"]) == 100)
    _check_graph(spec, net)
    exc = spec.is_exc_neuron()
    w = net["w0"]
    we = w[exc[net["src"]]]
    wi = w[~exc[net["src"]]]
    # lognormal with mean 0.5 and s.d. 0.5; inhibitory weights are 4x an independent draw
    assert abs(we.mean() - 0.5) < 0.01 and abs(we.std() - 0.5) < 0.03
    assert abs(wi.mean() - 2.0) < 0.06 and abs(wi.std() - 2.0) < 0.2
    assert np.all(net["w1"] == 0.0)
    assert np.all(net["delay"] == 1)
    # sources are uniform over all other neurons: E fraction near 0.8
    assert abs(exc[net["src"]].mean() - 0.8) < 0.01


def test_share_uniform_weights_and_delays():
    spec = configs.share(n=5000, indegree=556, seed=1)
    net = generate(spec)
    assert np.all(np.diff(net["ptr"]) == 556)
    _check_graph(spec, net)
    exc = spec.is_exc_neuron()
    e = exc[net["src"]]
    for w in (net["w0"], net["w1"]):
        assert abs(w[e].mean() - 0.5) < 0.005 and abs(w[e].var() - 1 / 12) < 0.002
        assert abs(w[~e].mean() - 2.0) < 0.02
    assert np.corrcoef(net["w0"][e], net["w1"][e])[0, 1] < 0.01     # independent channels
    d = net["delay"]
    assert d.min() == 1 and d.max() == 10
    hist = np.bincount(d, minlength=11)[1:]
    assert np.all(np.abs(hist / len(d) - 0.1) < 0.005)
    # sources within a target's list are ascending
    for i in range(0, 5000, 97):
        s = net["src"][net["ptr"][i]:net["ptr"][i + 1]]
        assert np.all(np.diff(s.astype(np.int64)) > 0)


def test_multi_region_sources_and_distance_delays():
    spec = configs.multi_region(n_regions=12, per_region=50, intra_indegree=20, long_indegree=10, seed=4)
    net = generate(spec)
    off, region, exc = _check_graph(spec, net)
    xyz = spec.region_xyz_mm.astype(np.float64)
    N = spec.num_neurons
    for i in range(N):
        a, b = net["ptr"][i], net["ptr"][i + 1]
        s, d = net["src"][a:b], net["delay"][a:b]
        assert b - a == 30
        intra, lr = s[:20], s[20:]
        assert np.all(region[intra] == region[i]) and np.all(d[:20] == 1)
        assert np.all(region[lr] != region[i]) and np.all(exc[lr])
        dist = np.linalg.norm(xyz[region[lr]] - xyz[region[i]], axis=1)
        want = np.clip(np.ceil(dist / 5.0), 1, 20)
        assert np.array_equal(d[20:].astype(np.float64), want)


def test_generator_is_deterministic_and_seeded():
    spec = configs.share(n=2000, indegree=50, seed=7)
    a, b = generate(spec), generate(spec)
    for k in a:
        assert np.array_equal(a[k], b[k])
    spec2 = configs.share(n=2000, indegree=50, seed=8)
    c = generate(spec2)
    assert not np.array_equal(a["src"], c["src"])
    v0 = a["v0"]
    assert v0.min() >= -55.0 and v0.max() < -50.0


def test_sampling_covers_candidates_uniformly():
    # in-degree close to the candidate count exercises Floyd's algorithm near its limit
    spec = configs.tiny(n_exc=40, n_inh=10, indegree=45, seed=3)
    net = generate(spec)
    _check_graph(spec, net)
    counts = np.bincount(net["src"], minlength=50)
    # each neuron is a source of about 45 * 49 / 49 targets
    assert abs(counts.mean() - 45) < 1e-9 and counts.min() > 30


def test_validation_errors():
    spec = configs.tiny(n_exc=10, n_inh=2, indegree=12)
    assert "more sources" in validate(spec)
    spec = configs.tiny()
    spec.bin_ms = 0.35
    assert "integer" in validate(spec)
    spec = configs.tiny()
    spec.receptor_mask = 0x3
    assert "receptor_mask" in validate(spec)
    spec = configs.multi_region(n_regions=3, per_region=20, intra_indegree=4, long_indegree=2)
    spec.region_xyz_mm = None
    assert "distance" in validate(spec)
