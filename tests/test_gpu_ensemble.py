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
