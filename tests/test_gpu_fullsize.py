"""Full-size runs on the GPU, checked on sampled outputs the oracle computes one by one.

The one-GPU share (6.1 M neurons, in-degree 556, 3.39e9 synapses) and the 200-region
network (1 M neurons) are far beyond what the oracle can simulate, so after K bins on
the GPU (same launch configuration as the benchmark: replayed graphs) the test takes
the GPU's recorded spikes and state at the start of bin K and checks, for a random
sample of neurons, that

* the arrivals due at bin K (pull form of eq. 3 over the generator's in-edges of each
  sampled neuron, fixed point) and one Euler step from the GPU's state reproduce the
  GPU's state after that step bit for bit (oracle point evaluations);

and, over the whole network, properties that hold at any size: at most one spike per
neuron per bin, ids in range, delivered events equal the summed delay-segment lengths
of the recorded spikes.
"""
import sys

import numpy as np
import pytest

from netgen import configs
from oracle import Oracle

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _run_and_check(spec, K, n_sample=1500, seed=0):
    from paper_2211_15963_amd import Simulator
    _say(f"{spec.name}: building {spec.num_neurons} neurons / {spec.num_edges()} synapses")
    sim = Simulator(spec, record_regions=True, spike_record_capacity=1 << 26)
    S = sim.S
    _say(f"{spec.name}: built; running {K} bins")
    sim.step(K * S)
    st, ids = sim.spikes()
    V0, J0, r0 = sim.state()
    sim.step(1)
    V1, J1, r1 = sim.state()
    stats = sim.stats()
    row_ptr, seg, _, _, _ = sim.export_csr(edges=False)
    sim.close()
    N = spec.num_neurons
    _say(f"{spec.name}: {len(st)} spikes in {K} bins ({len(st) / (N * K * 1e-3):.2f} Hz); checking")
    assert len(st) > 0 and ids.max() < N
    bins = st // S
    key = bins.astype(np.int64) * N + ids.astype(np.int64)
    assert len(np.unique(key)) == len(key), "a neuron spiked twice in one bin"
    # delivered events through bin K: every recorded spike (bin b) delivers its delay-d
    # segment at bin b + d <= K
    D = seg.shape[1] - 1
    seglen = np.diff(seg.astype(np.int64), axis=1)          # [N, D]
    want = 0
    for d in range(1, D + 1):
        sel = bins + d <= K
        want += int(seglen[ids[sel], d - 1].sum())
    assert stats["edge_events"] == want
    # sampled point evaluations
    rng = np.random.default_rng(seed)
    sample = np.sort(rng.choice(N, size=n_sample, replace=False)).astype(np.uint32)
    o = Oracle(spec, 32, params_only=True)
    A, ev = o.point_arrivals(K, st, ids, sample)
    assert ev > 0
    n = K * S
    for t, i in enumerate(sample):
        v, j, r, _ = o.point_step(int(i), n, A[t], float(V0[i]), J0[:, i], int(r0[i]))
        assert np.float32(v) == V1[i], (i, v, V1[i])
        assert np.array_equal(j, J1[:, i]), (i, j, J1[:, i])
        assert r == r1[i]
    _say(f"{spec.name}: {n_sample} sampled neurons bit-identical after the bin-start step")


def test_one_gpu_share_full_size_sampled():
    _run_and_check(configs.share(), K=30)


def test_multi_region_full_size_sampled():
    _run_and_check(configs.multi_region(), K=40)
