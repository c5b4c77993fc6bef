"""GPU path (through the C ABI) vs the FP32 CPU oracle, element by element.

Bar: spike rasters, V, J and refractory counters bit-identical; delivered-event
counts identical; region signals equal within the rounding bound of two
different summation orders of the same double terms.
"""
import sys

import numpy as np
import pytest

from netgen import configs
from oracle import Oracle

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def Sim():
    from paper_2211_15963_amd import Simulator
    return Simulator


def _compare(sim, orc, spec, check_regions=True):
    st_g, id_g = sim.spikes()
    st_o, id_o = orc.spikes()
    assert len(st_o) > 0, "the case produced no spikes"
    assert len(st_g) == len(st_o), f"spike counts differ: gpu {len(st_g)} oracle {len(st_o)}"
    assert np.array_equal(st_g, st_o) and np.array_equal(id_g, id_o), "rasters differ"
    Vg, Jg, rg = sim.state()
    Vo, Jo, ro = orc.state()
    assert np.array_equal(Vg.astype(np.float64), Vo), "V differs"
    assert np.array_equal(Jg.astype(np.float64), Jo), "J differs"
    assert np.array_equal(rg, ro), "refractory counters differ"
    assert sim.stats()["edge_events"] == orc.edge_events
    if check_regions:
        sg, cg = sim.region_signal()
        so, co = orc.region_signal()
        assert sg.shape == so.shape
        assert np.array_equal(cg, co), "region spike counts differ"
        # the same double terms summed in two orders differ by at most (n-1) eps sum|terms|;
        # divided by n and with |current| < 1e5 pA per neuron: n eps 1e5 per region
        n_reg = np.bincount(spec.region_of_neuron(), minlength=spec.n_regions)
        bound = n_reg[None, :] * np.finfo(np.float64).eps * 1e5
        assert np.all(np.abs(sg - so) <= bound)


def test_tiny_one_second_bit_exact(Sim):
    spec = configs.tiny()
    _say("tiny 1000 neurons, 10000 steps (1 s)")
    sim = Sim(spec)
    sim.step(10000)
    orc = Oracle(spec, 32)
    orc.step(10000)
    _compare(sim, orc, spec)
    sim.close()


def test_tiny_partial_bins_and_splits(Sim):
    spec = configs.tiny(seed=3)
    chunks = [3, 7, 10, 15, 1, 4, 5, 955, 9, 1, 990]
    _say(f"tiny seed 3, step chunks {chunks}")
    sim = Sim(spec)
    for c in chunks:
        sim.step(c)
    orc = Oracle(spec, 32)
    orc.step(sum(chunks))
    _compare(sim, orc, spec)
    sim.close()


def test_share_scaled_bit_exact(Sim):
    spec = configs.share(n=20000, indegree=556, seed=1)
    _say("share 20000 neurons, in-degree 556, delays 1..10, 400 steps")
    sim = Sim(spec)
    sim.step(400)
    orc = Oracle(spec, 32)
    orc.step(400)
    _compare(sim, orc, spec)
    sim.close()


def test_multi_region_scaled_bit_exact(Sim):
    spec = configs.multi_region(n_regions=20, per_region=1000, seed=2)
    _say("multi-region 20 x 1000, in-degree 400 + 100 long-range, delays 1..20, 500 steps")
    sim = Sim(spec)
    sim.step(500)
    orc = Oracle(spec, 32)
    orc.step(500)
    _compare(sim, orc, spec)
    sim.close()


def test_launch_modes_agree(Sim):
    spec = configs.share(n=6000, indegree=200, seed=4, bg_rate_hz=6500.0)
    _say("share 6000 / k200: graph replay vs direct launches vs timed launches")
    a = Sim(spec)
    a.step(300)
    b = Sim(spec, no_graph=True)
    b.step(300)
    c = Sim(spec)
    c.set_timing(True)
    c.step(300)
    ra, rb, rc = a.spikes(), b.spikes(), c.spikes()
    assert len(ra[0]) > 0
    for x, y in ((ra, rb), (ra, rc)):
        assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)
    st = c.stats()
    assert st["timed_bins"] == 30 and st["ms_scatter"] > 0 and st["ms_neuron"] > 0
    for s in (a, b, c):
        s.close()


def test_mixed_launch_sequence_bit_exact(Sim):
    """One handle driven through replayed graphs, direct and timed launches, partial bins
    and a schedule change (the partition kernels' work-queue counters and stream fills are
    reset by whichever kernel follows them), in both fan-in forms, against the oracle."""
    spec = configs.share(n=20000, indegree=300, seed=16)
    S = spec.steps_per_bin
    for single_pass in (False, True):
        _say(f"share 20000 / k300 seed 16: mixed launch sequence, single_pass={single_pass}")
        sim = Sim(spec, single_pass=single_pass)
        orc = Oracle(spec, 32)
        plan = [("graph", 20 * S), ("step", 3), ("step", S - 3), ("timed", 7 * S + 4), ("graph", 9 * S - 4),
                ("tune", 0), ("graph", 12 * S), ("timed", 5), ("step", 2 * S - 5)]
        for what, n in plan:
            if what == "tune":
                sim.set_tuning(scatter_wgs_per_cu=2, round_events=0, chunks_per_wg=2, ahead_passes=0)
                continue
            sim.set_timing(what == "timed")
            sim.step(n)
            orc.step(n)
        _compare(sim, orc, spec)
        sim.close()


def test_exported_table_is_the_generated_network(Sim):
    from netgen.desc import generate
    spec = configs.share(n=3000, indegree=50, seed=5)
    _say("export of the presynaptic table, 3000 neurons")
    sim = Sim(spec)
    row_ptr, seg, tgt, w0, w1 = sim.export_csr()
    net = generate(spec)
    D = spec.max_delay
    got = []
    for j in range(spec.num_neurons):
        a = int(row_ptr[j])
        for d in range(1, D + 1):
            for e in range(a + int(seg[j, d - 1]), a + int(seg[j, d])):
                got.append((int(tgt[e]), j, d, float(w0[e]), float(w1[e])))
        # rows sorted by (delay, target)
        t = tgt[a:int(row_ptr[j + 1])].astype(np.int64)
        for d in range(1, D + 1):
            blk = t[int(seg[j, d - 1]):int(seg[j, d])]
            assert np.all(np.diff(blk) > 0)
    want = []
    for i in range(spec.num_neurons):
        for e in range(int(net["ptr"][i]), int(net["ptr"][i + 1])):
            want.append((i, int(net["src"][e]), int(net["delay"][e]), float(net["w0"][e]), float(net["w1"][e])))
    assert sorted(got) == sorted(want)
    sim.close()


def test_state_roundtrip_is_invisible(Sim):
    spec = configs.tiny(seed=6)
    _say("tiny seed 6: read/write state at a bin boundary")
    a = Sim(spec)
    a.step(2000)
    b = Sim(spec)
    b.step(1000)
    V, J, ref = b.state()
    b.write_state(V, J, ref)
    b.step(1000)
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)
    a.close()
    b.close()


def test_spike_read_windows(Sim):
    spec = configs.tiny(seed=7)
    _say("tiny seed 7: windowed spike reads and truncation")
    sim = Sim(spec)
    sim.step(1234)
    st, ids = sim.spikes()
    assert st.max() < 1230  # only completed bins are visible
    st2, ids2 = sim.spikes(500, 800)
    sel = (st >= 500) & (st < 800)
    assert np.array_equal(st2, st[sel]) and np.array_equal(ids2, ids[sel])
    sim.close()


def test_one_hip_runtime_in_process(Sim):
    import torch
    _say("HIP runtime libraries mapped in this process")
    torch.zeros(1, device="cuda")
    maps = sorted(set(l.split()[-1] for l in open("/proc/self/maps") if "libamdhip64" in l))
    assert len(maps) == 1, maps


def test_single_pass_fanin_bit_exact(Sim):
    spec = configs.share(n=20000, indegree=556, seed=5)
    _say("share 20000 / k556 seed 5, single-pass fan-in, 400 steps")
    sim = Sim(spec, single_pass=True)
    assert sim.info.fanin_passes == 1
    sim.step(400)
    orc = Oracle(spec, 32)
    orc.step(400)
    _compare(sim, orc, spec)
    sim.close()
    # one weight per edge (8-byte records) over 5 tiles
    spec = configs.tiny(seed=8, n_exc=16000, n_inh=4000, indegree=100)
    _say("tiny-recipe 20000 / k100 seed 8 (one weight per edge), single-pass fan-in, 300 steps")
    sim = Sim(spec, single_pass=True)
    assert sim.info.fanin_passes == 1
    sim.step(300)
    orc = Oracle(spec, 32)
    orc.step(300)
    assert orc.spikes()[0].size > 1000
    _compare(sim, orc, spec)
    sim.close()
    spec = configs.multi_region(n_regions=20, per_region=1000, seed=6)
    _say("multi-region 20 x 1000 seed 6, single-pass fan-in, 300 steps")
    sim = Sim(spec, single_pass=True)
    sim.step(300)
    orc = Oracle(spec, 32)
    orc.step(300)
    _compare(sim, orc, spec)
    sim.close()


def test_stream_record_formats(Sim):
    """Non-negative weights with two per edge use 10-byte super-tile stream records (a 2-byte
    key beside the weight pair, two key bits in the weights' sign bits); a description with
    negative weights keeps the 12-byte records. Both equal the oracle bit for bit."""
    spec = configs.share(n=20000, indegree=300, seed=61)
    sim = Sim(spec)
    assert sim.info.stream_record_bytes == 10
    sim.close()
    neg = configs.share(n=20000, indegree=300, seed=62)
    for p in neg.projs:
        p.w_a = -0.25   # weights uniform in [-0.25, 1)
    _say("share 20000 / k300 seed 62 with negative weights: 12-byte stream records, 300 steps")
    sim = Sim(neg)
    assert sim.info.stream_record_bytes == 12
    sim.step(300)
    orc = Oracle(neg, 32)
    orc.step(300)
    _compare(sim, orc, neg)
    sim.close()


@pytest.mark.parametrize("negative", [False, True])
def test_full_streams_spill_to_arena(Sim, negative):
    """Super-tile streams smaller than a pass's events: with one in a thousand of each
    super-tile's in-edges nearly every run finds its stream full and goes to the tile arena
    event by event; with one in a hundred only some do. Both equal the oracle bit for bit, in
    both stream record formats."""
    spec = configs.share(n=20000, indegree=300, seed=63)
    if negative:
        for p in spec.projs:
            p.w_a = -0.25
    orc = Oracle(spec, 32)
    orc.step(300)
    for permille in (1, 10):
        _say(f"share 20000 / k300 seed 63, negative weights {negative}, stream_permille {permille}, 300 steps")
        sim = Sim(spec, stream_permille=permille)
        assert sim.info.stream_record_bytes == (12 if negative else 10)
        E = spec.num_edges()
        assert sim.info.stream_records <= E * permille // 1000 + 64
        sim.step(300)
        st = sim.stats()
        assert st["spilled_events"] > 0
        if permille == 10:
            assert st["spilled_events"] < st["edge_events"]
        _compare(sim, orc, spec)
        sim.close()


@pytest.mark.parametrize("negative", [False, True])
def test_full_arena_slices_sum_exactly(Sim, negative):
    """Tile arena slices smaller than a bin's events: the events past a full slice (from the
    bucketing, and from full streams, which place events in the arena one by one) are summed
    into the per-target overflow accumulator, which the tile's gather adds. With one in a
    thousand, one in a hundred of the in-edges, and both buffers tiny, the results equal the
    oracle bit for bit, in both stream record formats."""
    spec = configs.share(n=20000, indegree=300, seed=64)
    if negative:
        for p in spec.projs:
            p.w_a = -0.25
    orc = Oracle(spec, 32)
    orc.step(300)
    for sp, ap in ((0, 1), (0, 10), (1, 1)):
        _say(f"share 20000 / k300 seed 64, negative weights {negative}, stream_permille {sp}, arena_permille {ap}")
        sim = Sim(spec, stream_permille=sp, arena_permille=ap)
        assert sim.info.arena_records <= spec.num_edges() * ap // 1000 + 8
        sim.step(300)
        st = sim.stats()
        # (the counters include the next bin's events assembled ahead, not yet delivered)
        assert st["overflow_events"] > 0
        if ap == 10:
            assert st["overflow_events"] < st["edge_events"]
        if sp:
            assert st["spilled_events"] > 0
        _compare(sim, orc, spec)
        sim.close()


def test_small_buffers_one_weight_per_edge(Sim):
    """The one-weight form (two receptors, 12-byte stream records) with streams and arena
    slices of one in a thousand of their in-edges: spills and overflow sums, against the
    oracle over a second of biological time."""
    spec = configs.tiny(seed=13)
    _say("tiny seed 13, stream_permille 1, arena_permille 1, 10000 steps")
    sim = Sim(spec, stream_permille=1, arena_permille=1)
    assert sim.info.weights_per_edge == 1 and sim.info.stream_record_bytes == 8
    sim.step(10000)
    st = sim.stats()
    assert st["spilled_events"] > 0 and st["overflow_events"] > 0
    orc = Oracle(spec, 32)
    orc.step(10000)
    _compare(sim, orc, spec)
    sim.close()


def test_small_buffers_on_a_region_network(Sim):
    """A region network (neurons project mostly into their own region, so a few tiles take
    a bin's events in bursts) with streams and arena slices of one in a hundred of their
    in-edges, against the oracle."""
    spec = configs.multi_region(n_regions=20, per_region=1000, seed=12)
    _say("multi-region 20 x 1000 seed 12, stream_permille 10, arena_permille 10, 400 steps")
    sim = Sim(spec, stream_permille=10, arena_permille=10)
    sim.step(400)
    st = sim.stats()
    assert st["overflow_events"] > 0
    orc = Oracle(spec, 32)
    orc.step(400)
    _compare(sim, orc, spec)
    sim.close()


@pytest.mark.parametrize("single_pass", [False, True])
def test_fanin_schedules_agree(Sim, single_pass):
    """Every partition schedule gives the same bits (exact integer arrival sums)."""
    spec = configs.share(n=60000, indegree=300, seed=7)
    _say(f"share 60000 / k300, schedules compared, single_pass={single_pass}")
    ref = Sim(spec, single_pass=single_pass)
    assert ref.info.fanin_passes == (1 if single_pass else 2)
    ref.step(200)
    r_sp, r_st = ref.spikes(), ref.state()
    r_ev = ref.stats()["edge_events"]
    assert len(r_sp[0]) > 0
    ref.close()
    for wgs, re, cpw, ap in ((1, 0, 1, 1), (2, 256, 64, 9), (3, 512, 2, 2), (8, 0, 8, 0), (4, 1536, 4, 5)):
        sim = Sim(spec, single_pass=single_pass)
        try:
            sim.set_tuning(scatter_wgs_per_cu=wgs, round_events=re, chunks_per_wg=cpw, ahead_passes=ap)
        except Exception as ex:  # a schedule that does not fit the LDS is refused up front
            assert "LDS" in str(ex)
            sim.close()
            continue
        _say(f"  schedule {sim.tuning()}")
        sim.step(200)
        sp, st = sim.spikes(), sim.state()
        assert np.array_equal(sp[0], r_sp[0]) and np.array_equal(sp[1], r_sp[1])
        for x, y in zip(st, r_st):
            assert np.array_equal(x, y)
        assert sim.stats()["edge_events"] == r_ev
        sim.close()


def test_one_ms_euler_step_bit_exact(Sim):
    """The paper's Delta_t = 1 ms setting (one Euler step per bin, S = 1)."""
    spec = configs.tiny(dt_ms=1.0, seed=8)
    _say("tiny with dt = bin = 1 ms (S = 1), 1000 steps")
    sim = Sim(spec)
    assert sim.S == 1
    sim.step(1000)
    orc = Oracle(spec, 32)
    orc.step(1000)
    _compare(sim, orc, spec)
    sim.close()
    spec = configs.share(n=20000, indegree=300, seed=9)
    spec.dt_ms = 1.0
    spec.pops[0].T_ref = spec.pops[1].T_ref = 2.0
    _say("share 20000 / k300 with dt = 1 ms, 300 steps")
    sim = Sim(spec)
    sim.step(300)
    orc = Oracle(spec, 32)
    orc.step(300)
    _compare(sim, orc, spec)
    sim.close()


def test_ou_background_bit_exact(Sim):
    """OU background current (eq. 1 / eq. 4) on the GPU vs the oracle: the increments, the
    recurrence and its effect on V, spikes and delivery, bit for bit."""
    spec = configs.tiny(seed=14, bg_rate_hz=0.0)
    S = spec.steps_per_bin
    _say("tiny seed 14, no Poisson background: OU mu = (450, 400), sigma = 150, tau = 3 ms, 200 bins")
    sim = Sim(spec)
    sim.set_ou_background([450.0, 400.0], 150.0, 3.0)
    sim.step(200 * S)
    orc = Oracle(spec, 32)
    orc.set_ou([450.0, 400.0], 150.0, 3.0)
    orc.step(200 * S)
    assert orc.spikes()[0].size > 1000
    _compare(sim, orc, spec)
    sim.close()
    spec = configs.share(n=20000, indegree=300, seed=15)
    for single_pass in (False, True):
        _say(f"share 20000 / k300 seed 15: OU on the inhibitory population from bin 5, single_pass={single_pass}")
        sim = Sim(spec, single_pass=single_pass)
        sim.step(5 * S + 3)  # switched on mid-bin
        sim.set_ou_background([0.0, 20.0], [0.0, 40.0], [0.0, 4.0])
        sim.step(25 * S - 3)
        orc = Oracle(spec, 32)
        orc.step(5 * S + 3)
        orc.set_ou([0.0, 20.0], [0.0, 40.0], [0.0, 4.0])
        orc.step(25 * S - 3)
        _compare(sim, orc, spec)
        sim.close()


def test_spike_injection_bit_exact(Sim):
    """Initial spike injection (Methods) on the GPU vs the oracle: injected output spikes,
    their delivery and the rest of the trajectory."""
    spec = configs.tiny(seed=12)
    S = spec.steps_per_bin
    _say("tiny seed 12: injection p = (0.01, 0.005) for 200 bins, 400 bins run")
    sim = Sim(spec)
    sim.set_spike_injection([0.01, 0.005], 200)
    sim.step(400 * S)
    orc = Oracle(spec, 32)
    orc.set_injection([0.01, 0.005], 200)
    orc.step(400 * S)
    _compare(sim, orc, spec)
    sim.close()
    spec = configs.share(n=20000, indegree=300, seed=13)
    for single_pass in (False, True):
        _say(f"share 20000 / k300 seed 13: injection 0.02 for 20 bins from bin 10, single_pass={single_pass}")
        sim = Sim(spec, single_pass=single_pass)
        sim.step(10 * S)
        sim.set_spike_injection(0.02, 20)
        sim.step(30 * S)
        orc = Oracle(spec, 32)
        orc.step(10 * S)
        orc.set_injection(0.02, 30)  # absolute bin index: bins 10..29
        orc.step(30 * S)
        _compare(sim, orc, spec)
        sim.close()


def test_host_record_with_minimal_device_ring(Sim):
    """Every bin's spikes are copied to the pinned host ring while the device keeps only the
    last max delay + 1 bins the fan-in reads: over 1 s the device ring (2,048 entries) wraps
    several times and the raster read back still equals the oracle's; a host ring smaller
    than the raster keeps its most recent part and refuses older reads."""
    from paper_2211_15963_amd import dbsim as D
    spec = configs.tiny(seed=17)
    _say("tiny seed 17, 1 s, device ring at its minimum, raster from the host ring")
    sim = Sim(spec)
    sim.step(10000)
    orc = Oracle(spec, 32)
    orc.step(10000)
    assert orc.spikes()[0].size > 4 * 2048  # the device ring wrapped at least four times
    _compare(sim, orc, spec)
    sim.close()
    spec = configs.share(n=20000, indegree=300, seed=18)
    S = spec.steps_per_bin
    _say("share 20000 / k300 seed 18: host ring of 4096 entries, 60 bins, graph and partial launches")
    sim = Sim(spec, host_spike_capacity=4096)
    sim.step(30 * S)
    sim.step(7)
    sim.step(30 * S - 7)
    orc = Oracle(spec, 32)
    orc.step(60 * S)
    so, io = orc.spikes()
    keep = so >= 55 * S
    assert 0 < keep.sum() <= 4096 and len(so) > 4096
    st, ids = sim.spikes(55 * S, 60 * S)
    assert np.array_equal(st, so[keep]) and np.array_equal(ids, io[keep])
    with pytest.raises(D.DbsimError) as ex:
        sim.spikes(0, 10 * S)
    assert ex.value.code == D.ERANGE
    sim.close()
