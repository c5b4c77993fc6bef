"""FP32 GPU path vs the FP64 oracle (the paper's precedent compares its GPU and CPU
runs: identical spike times and relative V error below 1e-4 over 1 s).

Reported as numbers: the largest relative V error before the first raster difference
(per seed), and, after the trajectories separate, the population rate and the mean
ISI coefficient of variation over five seeds, which must agree within stated
tolerances (rate: max(3 standard errors, 2 %) relative; CV: 0.05 absolute).
"""
import numpy as np
import pytest

from netgen import configs
from oracle import Oracle

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]


def _cv(steps, ids, n, dt):
    order = np.lexsort((steps, ids))
    s, i = steps[order].astype(np.float64) * dt, ids[order]
    cvs = []
    starts = np.searchsorted(i, np.arange(n))
    ends = np.searchsorted(i, np.arange(n), side="right")
    for a, b in zip(starts, ends):
        if b - a >= 4:
            isi = np.diff(s[a:b])
            cvs.append(isi.std() / isi.mean())
    return float(np.mean(cvs)) if cvs else float("nan")


def test_fp32_gpu_against_fp64_oracle():
    from paper_2211_15963_amd import Simulator
    rates32, rates64, cv32, cv64, errs = [], [], [], [], []
    T, chunk = 10000, 100
    for seed in range(5):
        spec = configs.multi_region(n_regions=10, per_region=400, intra_indegree=150, long_indegree=30, seed=seed)
        print(f"[gpu-case] precision seed {seed}: {spec.num_neurons} neurons, 1 s", flush=True)
        sim = Simulator(spec)
        o = Oracle(spec, 64)
        worst, diverged = 0.0, None
        for c in range(T // chunk):
            sim.step(chunk)
            o.step(chunk)
            if diverged is None:
                a, b = sim.spikes(), o.spikes()
                done = (c + 1) * chunk // 10 * 10
                sa = a[0] < done
                sb = b[0] < done
                if not (np.array_equal(a[0][sa], b[0][sb]) and np.array_equal(a[1][sa], b[1][sb])):
                    diverged = (c + 1) * chunk
                else:
                    V32 = sim.state()[0].astype(np.float64)
                    V64 = o.state()[0]
                    worst = max(worst, float(np.max(np.abs(V32 - V64) / np.abs(V64))))
        st32, id32 = sim.spikes()
        st64, id64 = o.spikes()
        n = spec.num_neurons
        rates32.append(len(st32) / (n * 1.0))
        rates64.append(len(st64) / (n * 1.0))
        cv32.append(_cv(st32, id32, n, spec.dt_ms))
        cv64.append(_cv(st64, id64, n, spec.dt_ms))
        errs.append(worst)
        print(f"  max rel V error before divergence {worst:.2e}, rasters separate at step {diverged}; "
              f"rate {rates32[-1]:.2f} vs {rates64[-1]:.2f} Hz; CV {cv32[-1]:.3f} vs {cv64[-1]:.3f}", flush=True)
        sim.close()
    r32, r64 = np.array(rates32), np.array(rates64)
    se = np.sqrt(r32.var(ddof=1) / len(r32) + r64.var(ddof=1) / len(r64))
    assert abs(r32.mean() - r64.mean()) <= max(3 * se, 0.02 * r64.mean())
    assert abs(np.mean(cv32) - np.mean(cv64)) <= 0.05
    assert max(errs) < 1e-4
