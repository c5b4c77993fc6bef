"""dbsim_create_static: the handle's device arrays in the library's static region (no
device allocation), checked against dbsim_create on the same networks, bit for bit.

Two creations in a row on one device, the second network smaller than the first (the
region keeps the first handle's contents; everything the kernels read must be set up
again), each compared with a handle of dbsim_create: raster, V, J, refractory counters,
region signal and delivered events. Also: the size limit and the one-handle-per-device
rule give their errors.
"""
import ctypes
import sys

import numpy as np
import pytest

from netgen import configs


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def test_static_create_refuses_networks_beyond_the_region():
    """Host-side check, before any device work (runs without a GPU)."""
    from paper_2211_15963_amd import dbsim as D
    L = D.lib()
    spec = configs.share(n=20000, indegree=556)
    need = D.footprint(spec, host_record=False)  # the static handle keeps its raster on the device
    assert need > D.STATIC_BYTES
    d, holder = D.make_desc(spec)
    h = ctypes.c_void_p()
    rc = L.dbsim_create_static(ctypes.byref(d), ctypes.byref(h))
    msg = L.dbsim_last_error().decode()
    assert rc == D.EINVAL and not h.value
    assert str(need) in msg and str(D.STATIC_BYTES) in msg


def _run(Sim, spec, steps, static):
    sim = Sim(spec, static_region=static, spike_record_capacity=1 << 16)
    for n in steps:
        sim.step(n)
    out = (sim.spikes(), sim.state(), sim.region_signal(), sim.stats()["edge_events"])
    return sim, out


def _same(a, b):
    (sa, ia), (Va, Ja, ra), (ga, ca), ea = a
    (sb, ib), (Vb, Jb, rb), (gb, cb), eb = b
    assert len(sa) > 0
    assert np.array_equal(sa, sb) and np.array_equal(ia, ib), "rasters differ"
    assert np.array_equal(Va, Vb) and np.array_equal(Ja, Jb) and np.array_equal(ra, rb), "states differ"
    # same kernels, same reduction order: the region signal is the same bits
    assert np.array_equal(ga, gb) and np.array_equal(ca, cb), "region signals differ"
    assert ea == eb, "delivered events differ"


@pytest.mark.gpu
def test_static_create_equals_create_twice_smaller_second():
    from paper_2211_15963_amd import DbsimError, Simulator
    from paper_2211_15963_amd import dbsim as D
    first = configs.share(n=6000, indegree=200, seed=61, bg_rate_hz=6500.0)
    second = configs.tiny(seed=62, n_exc=480, n_inh=120, indegree=60)
    fp = lambda spec: D.footprint(spec, spike_record_capacity=1 << 16, host_record=False)
    assert fp(second) < fp(first) <= D.STATIC_BYTES
    for spec, steps in ((first, [3000, 7, 993]), (second, [1500, 4, 496])):
        _say(f"static region: {spec.name} ({spec.num_neurons} neurons), steps {steps}")
        ref, want = _run(Simulator, spec, steps, static=False)
        ref.close()
        sim, got = _run(Simulator, spec, steps, static=True)
        _same(got, want)
        # one handle per device in the region; timers need events the handle does not create
        with pytest.raises(DbsimError) as ex:
            Simulator(spec, static_region=True)
        assert ex.value.code == D.ESTATE
        with pytest.raises(DbsimError) as ex:
            sim.set_timing(True)
        assert ex.value.code == D.ESTATE
        sim.close()
