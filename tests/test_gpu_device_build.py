"""Connection table generated on the device (the default where it applies) against the
host construction (DBSIM_F_HOST_BUILD): the same rows, delay segments, targets and weight
bit patterns on the share and region recipes, an ensemble, constant weights, one weight
per edge, long segments, and an in-degree that takes the thread-per-target generator;
descriptions with lognormal weights stay on the host. The oracle parity tests
run on device-built tables too, since that is the default."""
import sys

import numpy as np
import pytest

import edge_networks
from netgen import configs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def Sim():
    from paper_2211_15963_amd import Simulator
    return Simulator


def _same_tables(Sim, spec, name):
    _say(f"{name}: device construction vs host construction")
    a = Sim(spec)
    b = Sim(spec, host_build=True)
    assert a.info.device_built == 1 and b.info.device_built == 0
    ta, tb = a.export_csr(), b.export_csr()
    for x, y, what in zip(ta, tb, ("row_ptr", "seg", "tgt", "w0", "w1")):
        if x is None or y is None:
            assert x is None and y is None
            continue
        xv = x.view(np.uint32) if x.dtype == np.float32 else x
        yv = y.view(np.uint32) if y.dtype == np.float32 else y
        assert np.array_equal(xv, yv), f"{name}: {what} differs"
    sa, sb = a.stats(), b.stats()
    _say(f"  construction {sa['build_seconds']:.3f} s on the device, {sb['build_seconds']:.3f} s on the host")
    a.close()
    b.close()


def test_share_and_region_recipes(Sim):
    _same_tables(Sim, configs.share(n=60000, indegree=556, seed=7), "share 60000 / k556")
    _same_tables(Sim, configs.multi_region(n_regions=12, per_region=1500, seed=41), "regions 12 x 1500")


def test_ensemble_constant_weights_one_weight_per_edge(Sim):
    a = configs.share(n=20000, indegree=300, seed=1)
    b = configs.multi_region(n_regions=4, per_region=1500, seed=2)
    a.net_id, b.net_id = 3, 4
    _say("ensemble of a share and a region network: device vs host construction")
    x = Sim([a, b])
    y = Sim([a, b], host_build=True)
    assert x.info.device_built == 1 and y.info.device_built == 0
    for u, v in zip(x.export_csr(), y.export_csr()):
        if u is not None:
            assert np.array_equal(u.view(np.uint32) if u.dtype == np.float32 else u,
                                  v.view(np.uint32) if v.dtype == np.float32 else v)
    x.close()
    y.close()
    sat = edge_networks.saturated(n=20000, indegree=100)
    for p in sat.projs:
        p.w_dist, p.w_a = 2, 0.3
    _same_tables(Sim, sat, "constant weights 20000 / k100")
    tw = configs.tiny(seed=9, n_exc=16000, n_inh=4000, indegree=100)
    for p in tw.projs:
        p.w_dist, p.w_a, p.w_b = 0, 0.0, 1.0
    _same_tables(Sim, tw, "one weight per edge, uniform, 20000 / k100")


def test_long_segments_and_duplicate_pairs(Sim):
    """16 hub neurons feed every one of 20,000 targets 8 times at delay 1 (segments of about
    10,000 records, beyond the LDS sort), and an all-to-all projection can pick a hub for
    the same target again (equal targets in one segment, ordered by projection)."""
    from netgen.desc import NetSpec, PopSpec, ProjSpec, SRC_POP, D_UNIFORM
    pops = [PopSpec(16, True), PopSpec(20000, True)]
    projs = [ProjSpec(8, dst_pop=1, src_mode=SRC_POP, src_pop=0), ProjSpec(50, d_mode=D_UNIFORM, d_min=1, d_max=3)]
    _same_tables(Sim, NetSpec(pops, projs, seed=17, name="hubs"), "hubs 16 -> 20000")


def test_thread_per_target_generator(Sim):
    """In-degree 5,000: the wavefront generator's LDS sets would not fit, so one thread per
    target draws the in-edges with scratch in the streams (batches of targets)."""
    _same_tables(Sim, configs.share(n=12000, indegree=5000, seed=19), "share 12000 / k5000")


def test_lognormal_weights_stay_on_the_host(Sim):
    sim = Sim(configs.tiny(seed=0))
    assert sim.info.device_built == 0
    sim.close()


def test_construction_time_at_600k(Sim):
    spec = configs.share(n=600_000, indegree=556, seed=31)
    _say("share 600000 / k556: construction time, device vs host")
    _same_tables(Sim, spec, "share 600000 / k556")
