"""Region BOLD on the GPU vs the FP64 Balloon-Windkessel oracle, fed with the same
per-bin region spike counts (the GPU's, and the FP32 oracle's own).

Tolerance: both sides evaluate the same FP64 expressions in the same order (no FMA);
only pow() may differ by an ulp between the device and host math libraries. The
model is contracting, so per-step differences of a few 1e-16 relative stay below
1e-12 relative over the run; the test allows 1e-10 of the signal's range."""
import sys

import numpy as np
import pytest

from netgen import configs
from oracle import bold as obold

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def test_bold_matches_oracle():
    from paper_2211_15963_amd import Simulator
    from paper_2211_15963_amd.dbsim import bold_defaults
    spec = configs.multi_region(n_regions=20, per_region=1000, seed=3)
    _say("multi-region 20 x 1000: BOLD with TR = 50 bins over 3000 bins, then 1000 more")
    sim = Simulator(spec, record_regions=True)
    p = bold_defaults(tr_bins=50, activity_scale=0.02)
    sim.set_bold(p)
    sim.step(3000 * sim.S)
    y_gpu = sim.bold()
    st_gpu, n = sim.bold_state()
    assert n == 60 and y_gpu.shape == (60, 20)
    _, counts = sim.region_signal(0, 3000)
    sizes = np.bincount(spec.region_of_neuron(), minlength=spec.n_regions)
    y_orc, st_orc = obold.run(counts, sizes, p.as_dict(), spec.bin_ms)
    scale = np.max(np.abs(y_orc))
    assert scale > 0
    assert np.max(np.abs(y_gpu - y_orc)) <= 1e-10 * scale
    assert np.allclose(st_gpu, st_orc, rtol=1e-10, atol=1e-14)
    # continuing: samples keep their numbering and the state carries over
    sim.step(1000 * sim.S)
    _, c2 = sim.region_signal(3000, 4000)
    y2, _ = obold.run(c2, sizes, p.as_dict(), spec.bin_ms, state=st_orc, bins_done=3000)
    assert np.max(np.abs(sim.bold(60, 80) - y2)) <= 1e-10 * scale
    # reset to rest, and off
    sim.set_bold(p)
    st, n = sim.bold_state()
    assert n == 0 and np.array_equal(st, obold.rest_state(20))
    sim.set_bold(False)
    sim.step(100 * sim.S)
    assert sim.bold_state()[1] == 0
    sim.close()


def test_bold_from_the_oracles_own_counts():
    """The whole chain against the oracles alone: the FP32 oracle simulates the network, its
    per-bin region spike counts drive the FP64 Balloon-Windkessel oracle, and the GPU's BOLD
    samples (computed on the device from the GPU's own counts) must match."""
    from oracle import Oracle
    from paper_2211_15963_amd import Simulator
    from paper_2211_15963_amd.dbsim import bold_defaults
    spec = configs.multi_region(n_regions=6, per_region=600, seed=9)
    bins = 1200
    _say(f"multi-region 6 x 600: BOLD with TR = 40 bins over {bins} bins, counts from the FP32 oracle")
    sim = Simulator(spec, record_regions=True)
    p = bold_defaults(tr_bins=40, activity_scale=0.02)
    sim.set_bold(p)
    sim.step(bins * sim.S)
    y_gpu = sim.bold()
    st_gpu, n = sim.bold_state()
    sim.close()
    orc = Oracle(spec, 32)
    orc.step(bins * spec.steps_per_bin)
    _, counts = orc.region_signal()
    assert counts.shape == (bins, 6) and counts.sum() > 0
    sizes = np.bincount(spec.region_of_neuron(), minlength=spec.n_regions)
    y_orc, st_orc = obold.run(counts, sizes, p.as_dict(), spec.bin_ms)
    assert n == bins // 40 and y_gpu.shape == y_orc.shape
    scale = np.max(np.abs(y_orc))
    assert scale > 0
    assert np.max(np.abs(y_gpu - y_orc)) <= 1e-10 * scale
    assert np.allclose(st_gpu, st_orc, rtol=1e-10, atol=1e-14)


def test_bold_requires_regions_and_valid_params():
    from paper_2211_15963_amd import Simulator
    from paper_2211_15963_amd.dbsim import DbsimError, bold_defaults
    spec = configs.tiny()
    sim = Simulator(spec, record_regions=False)
    with pytest.raises(DbsimError, match="REC_REGIONS"):
        sim.set_bold()
    sim.close()
    sim = Simulator(spec, record_regions=True)
    with pytest.raises(DbsimError, match="out of range"):
        sim.set_bold(bold_defaults(rho=1.5))
    sim.close()
