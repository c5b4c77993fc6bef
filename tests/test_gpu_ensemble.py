"""Ensembles (many independent networks advanced by the same launches): each member's
spikes and state inside the ensemble are bit-identical to the member run alone on the
GPU and to the FP32 oracle."""
import numpy as np
import pytest

from netgen import configs
from oracle import Oracle

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def test_ensemble_members_equal_alone_and_oracle():
    from paper_2211_15963_amd import Simulator
    members = [configs.ensemble_member(m, seed=3, n_lo=1500, n_hi=12000) for m in range(6)]
    steps = 300
    _say(f"ensemble of {len(members)} members, sizes {[s.num_neurons for s in members]}, {steps} steps")
    ens = Simulator(members)
    ens.step(steps)
    for m, spec in enumerate(members):
        alone = Simulator(spec)
        alone.step(steps)
        st_a, id_a = alone.spikes()
        st_e, id_e = ens.member_spikes(m)
        assert len(st_a) > 0
        assert np.array_equal(st_a, st_e) and np.array_equal(id_a, id_e), f"member {m} raster differs"
        for x, y in zip(alone.state(), ens.member_state(m)):
            assert np.array_equal(x, y), f"member {m} state differs"
        alone.close()
        if spec.num_neurons <= 6000:
            o = Oracle(spec, 32)
            o.step(steps)
            so, io = o.spikes()
            assert np.array_equal(so, st_e) and np.array_equal(io, id_e), f"member {m} differs from the oracle"
            Vo, Jo, ro = o.state()
            Ve, Je, re = ens.member_state(m)
            assert np.array_equal(Ve.astype(np.float64), Vo) and np.array_equal(Je.astype(np.float64), Jo)
    ens.close()


def test_ensemble_with_small_buffers_equals_default():
    """The whole ensemble's streams and arena slices at one in a hundred of their in-edges
    (spills and overflow sums across members): every member bit-identical to the default
    buffers' run."""
    from paper_2211_15963_amd import Simulator
    members = [configs.ensemble_member(m, seed=4, n_lo=1500, n_hi=12000) for m in range(5)]
    steps = 300
    _say(f"ensemble of {len(members)} members with 10 per mille buffers vs default, {steps} steps")
    ref = Simulator(members)
    ref.step(steps)
    small = Simulator(members, stream_permille=10, arena_permille=10)
    small.step(steps)
    st = small.stats()
    assert st["overflow_events"] > 0 and st["edge_events"] == ref.stats()["edge_events"]
    for m in range(len(members)):
        a, b = ref.member_spikes(m), small.member_spikes(m)
        assert len(a[0]) > 0 and np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), m
        for x, y in zip(ref.member_state(m), small.member_state(m)):
            assert np.array_equal(x, y), m
    ref.close()
    small.close()
