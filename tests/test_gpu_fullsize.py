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
of the recorded spikes; the record is complete (the neurons whose refractory counter at
the start of each of the last three bins says they fired in the bin before, and at which
step, are exactly that bin's recorded spikes); and every region's signal for the last
bin equals its definition evaluated on the recorded state (the mean over the region of
each neuron's FP32 current sum_u (g_u J_u)(V_u - V), summed in double), within the
rounding bound of two summation orders.
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
    sim = Simulator(spec, record_regions=True, host_spike_capacity=1 << 26)
    S = sim.S
    _say(f"{spec.name}: built; running {K} bins")
    sim.step((K - 3) * S)
    refs = {}
    for b in range(K - 3, K):
        sim.step(S)
        V0, J0, r0 = sim.state()
        refs[b] = r0  # state at the start of bin b + 1
    st, ids = sim.spikes()
    sig, _ = sim.region_signal(K - 1, K)
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
    _check_record_complete(spec, S, st, ids, refs)
    _check_region_signal(spec, V0, J0, sig[0])
    _say(f"{spec.name}: spike record complete over the last 3 bins; region signals equal their definition")
    _check_points(spec, K, S, st, ids, (V0, J0, r0), (V1, J1, r1), n_sample, seed)
    _say(f"{spec.name}: {n_sample} sampled neurons bit-identical after the bin-start step")


def _check_record_complete(spec, S, st, ids, refs):
    """A neuron that fired at step n of bin b (n in bS .. bS + S - 1) holds r - ((b + 1) S - 1 - n)
    refractory steps at the start of bin b + 1 (r = round(T_ref / dt) >= S), one that fired
    earlier holds at most r - S: the counters name every spike of bin b and its step."""
    from paper_2211_15963_amd.dbsim import derive_constants
    N = spec.num_neurons
    r = np.zeros(N, np.int64)
    for p in derive_constants(spec):
        r[p["first_neuron"]:p["end_neuron"]] = p["ref_steps"]
    assert r.min() >= S
    for b, ref in refs.items():
        ref = ref.astype(np.int64)
        fired = np.nonzero(ref >= r - S + 1)[0]
        steps = (b + 1) * S - 1 - (r[fired] - ref[fired])
        sel = (st // S) == b
        got = sorted(zip(st[sel].tolist(), ids[sel].tolist()))
        want = sorted(zip(steps.tolist(), fired.tolist()))
        assert got == want, f"bin {b}: recorded spikes differ from those the refractory counters imply"


def _check_region_signal(spec, V, J, sig):
    from paper_2211_15963_amd.dbsim import derive_constants
    cur = np.zeros(spec.num_neurons, np.float32)
    for p in derive_constants(spec):
        a, b = p["first_neuron"], p["end_neuron"]
        for u in range(len(p["g"])):
            cur[a:b] = cur[a:b] + (p["g"][u] * J[u, a:b]) * (p["V_rev"][u] - V[a:b])
    reg = spec.region_of_neuron()
    n_reg = np.bincount(reg, minlength=spec.n_regions)
    want = np.bincount(reg, weights=cur.astype(np.float64), minlength=spec.n_regions) / n_reg
    bound = n_reg * np.finfo(np.float64).eps * 1e5
    assert np.all(np.abs(sig - want) <= bound), np.max(np.abs(sig - want) / bound)


def _check_points(spec, K, S, st, ids, before, after, n_sample, seed):
    """oracle point evaluations: for sampled neurons, the arrivals due at bin K (from the
    recorded spikes and the generator's in-edges) and one Euler step from the recorded
    state reproduce the recorded state after that step bit for bit"""
    V0, J0, r0 = before
    V1, J1, r1 = after
    N = spec.num_neurons
    rng = np.random.default_rng(seed)
    sample = np.sort(rng.choice(N, size=min(n_sample, N), replace=False)).astype(np.uint32)
    o = Oracle(spec, 32, params_only=True)
    A, ev = o.point_arrivals(K, st, ids, sample)
    assert ev > 0
    n = K * S
    for t, i in enumerate(sample):
        v, j, r, _ = o.point_step(int(i), n, A[t], float(V0[i]), J0[:, i], int(r0[i]))
        assert np.float32(v) == V1[i], (i, v, V1[i])
        assert np.array_equal(j, J1[:, i]), (i, j, J1[:, i])
        assert r == r1[i]


def test_one_gpu_share_full_size_sampled():
    _run_and_check(configs.share(), K=30)


def test_multi_region_full_size_sampled():
    _run_and_check(configs.multi_region(), K=40)


def test_ensemble_full_size_sampled():
    """The 64-member ensemble as the benchmark runs it (10.3 M neurons, 3.96e9 synapses,
    one handle, replayed graphs, one chunk per partition workgroup): per member, the
    properties that hold at any size and sampled oracle point evaluations on eight
    members (the smallest, the largest and six others)."""
    from paper_2211_15963_amd import Simulator
    members = [configs.ensemble_member(m, seed=0) for m in range(64)]
    _say(f"ensemble: building 64 members, {sum(s.num_neurons for s in members)} neurons")
    ens = Simulator(members, record_regions=True, host_spike_capacity=1 << 27)
    ens.set_tuning(scatter_wgs_per_cu=ens.tuning()["scatter_wgs_per_cu"], round_events=0, chunks_per_wg=1)
    S = ens.S
    K = 30
    _say(f"ensemble: built; running {K} bins")
    ens.step(K * S)
    st, ids = ens.spikes()
    V0, J0, r0 = ens.state()
    ens.step(1)
    V1, J1, r1 = ens.state()
    stats = ens.stats()
    row_ptr, seg, _, _, _ = ens.export_csr(edges=False)
    spans = [ens.member(m) for m in range(len(members))]
    ens.close()
    N = V0.size
    assert len(st) > 0 and ids.max() < N
    bins = st // S
    key = bins.astype(np.int64) * N + ids.astype(np.int64)
    assert len(np.unique(key)) == len(key), "a neuron spiked twice in one bin"
    D = seg.shape[1] - 1
    seglen = np.diff(seg.astype(np.int64), axis=1)
    want = 0
    for d in range(1, D + 1):
        sel = bins + d <= K
        want += int(seglen[ids[sel], d - 1].sum())
    assert stats["edge_events"] == want
    sizes = [s.num_neurons for s in members]
    chosen = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 5, 17, 29, 41, 50, 63})
    for m in chosen:
        a, n, _, _ = spans[m]
        sel = (ids >= a) & (ids < a + n)
        local = (st[sel], (ids[sel] - a).astype(np.uint32))
        cut = lambda x: x[..., a:a + n]
        _check_points(members[m], K, S, local[0], local[1], (cut(V0), cut(J0), cut(r0)), (cut(V1), cut(J1), cut(r1)),
                      250, m)
        _say(f"ensemble member {m} ({n} neurons): 250 sampled neurons bit-identical after the bin-start step")
