"""CPU checks of the served-stream recipes: seeded, within their ranges."""
import numpy as np

from netgen import configs


def test_served_request_recipe():
    sizes, ks, steps, regimes = [], [], [], set()
    for r in range(200):
        spec, n = configs.served_request(r, seed=3)
        a, b = configs.served_request(r, seed=3)
        assert a.num_neurons == spec.num_neurons and b == n
        assert 1e4 - 1 <= spec.num_neurons <= 2e6 + 1
        assert 200 <= spec.projs[0].indegree <= 600
        assert n % spec.steps_per_bin == 0 and 100 * 10 <= n <= 2000 * 10
        sizes.append(spec.num_neurons)
        regimes.add(spec.name.split("-")[-1])
    assert regimes == {"7hz", "15hz", "30hz"}
    # log-uniform: the median is near the geometric midpoint sqrt(1e4 * 2e6) ~ 1.4e5
    assert 6e4 < np.median(sizes) < 3.5e5


def test_arrival_times_poisson():
    t = configs.arrival_times(4000, 50.0, seed=1)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert np.all(gaps > 0)
    assert abs(gaps.mean() - 0.02) < 0.002
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.08  # exponential: CV = 1
    assert np.array_equal(t, configs.arrival_times(4000, 50.0, seed=1))
