"""The generator step of the device construction of the connection table, evaluated on
the host (dbsim_check_device_generator), against the input generator (dbnet_in_edges):
for every target of several networks, the same in-edges in the same order, with the
same source ids, weight bit patterns and delays. Covers uniform weights with uniform
delays (share recipe), two projections with same-region and other-region sources and
distance delays (region recipe), constant weights, one weight per edge, ensembles
(members with their own seeds, net ids and id offsets), and the refusal of lognormal
weights (drawn through libm, so built on the host)."""
import numpy as np
import pytest

import edge_networks
from netgen import configs
from netgen.desc import generate


@pytest.fixture(scope="module")
def D():
    from paper_2211_15963_amd import dbsim
    dbsim.lib()
    return dbsim


def _check_all(D, specs):
    base = 0
    for sp in specs:
        ref = generate(sp)
        for i in range(sp.num_neurons):
            a, b = int(ref["ptr"][i]), int(ref["ptr"][i + 1])
            src, w0, w1, dl, _ = D.device_generator_in_edges(specs, base + i)
            assert src.size == b - a, (sp.name, i)
            assert np.array_equal(src, ref["src"][a:b] + base), (sp.name, i)
            assert np.array_equal(w0.view(np.uint32), ref["w0"][a:b].view(np.uint32)), (sp.name, i)
            assert np.array_equal(w1.view(np.uint32), ref["w1"][a:b].view(np.uint32)), (sp.name, i)
            assert np.array_equal(dl, ref["delay"][a:b]), (sp.name, i)
        base += sp.num_neurons


def test_share_recipe_every_target(D):
    _check_all(D, [configs.share(n=3000, indegree=300, seed=3)])


def test_region_recipe_every_target(D):
    sp = configs.multi_region(n_regions=6, per_region=700, intra_indegree=200, long_indegree=60, seed=4)
    assert sp.max_delay > 1
    _check_all(D, [sp])


def test_constant_weights_and_one_weight_per_edge(D):
    sp = edge_networks.saturated(n=2000, indegree=50)
    for p in sp.projs:
        p.w_dist, p.w_a = 2, 0.3   # constant weights
    _check_all(D, [sp])
    tw = configs.tiny(seed=9)
    for p in tw.projs:
        p.w_dist, p.w_a, p.w_b = 0, 0.0, 1.0   # uniform instead of lognormal
    assert tw.weights_per_edge == 1
    _check_all(D, [tw])


def test_ensemble_members_every_target(D):
    a = configs.share(n=1500, indegree=120, seed=5)
    b = configs.multi_region(n_regions=3, per_region=600, intra_indegree=100, long_indegree=30, seed=6)
    a.net_id, b.net_id = 11, 12
    _check_all(D, [a, b])


def test_lognormal_weights_are_refused(D):
    with pytest.raises(D.DbsimError, match="lognormal"):
        D.device_generator_in_edges(configs.tiny(seed=0), 0)
