"""Checkpoint and resume through the C ABI (dbsim_checkpoint_save / _restore).

A run saved at a bin boundary and restored into a fresh handle of the same description
continues bit-identically to the saved run: raster, V, J, refractory counters, delivered
events, spike count, region signals and BOLD samples after the checkpoint, with delays
up to 20 bins (the restored spike history feeds the fan-in), with the OU background and
spike injection switched on before the checkpoint, in both fan-in forms, and with a
checkpoint taken before the first max-delay bins have passed. The continued run also
equals the FP32 oracle run straight through. Error paths: a stepped handle, another
network, a damaged image, a mid-bin checkpoint, reads of bins before the checkpoint.
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


def _same_after(a, b, spec, K, M):
    S = spec.steps_per_bin
    sa, ia = a.spikes(K * S, (K + M) * S)
    sb, ib = b.spikes(K * S, (K + M) * S)
    assert sa.size > 0
    assert np.array_equal(sa, sb) and np.array_equal(ia, ib)
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x.view(np.uint32) if x.dtype == np.float32 else x,
                              y.view(np.uint32) if y.dtype == np.float32 else y)
    ta, tb = a.stats(), b.stats()
    for k in ("steps", "bins", "spikes", "edge_events"):
        assert ta[k] == tb[k], (k, ta[k], tb[k])
    if int(a.info.n_regions) > 0:
        ga, ca = a.region_signal(K, K + M)
        gb, cb = b.region_signal(K, K + M)
        assert np.array_equal(ga.view(np.uint64), gb.view(np.uint64)) and np.array_equal(ca, cb)


@pytest.mark.parametrize("single_pass", [False, True])
def test_resume_equals_uninterrupted_run(Sim, single_pass):
    spec = configs.multi_region(n_regions=12, per_region=1500, seed=41)
    S, K, M = spec.steps_per_bin, 37, 30
    _say(f"multi-region 12 x 1500 (delays up to {spec.max_delay}), checkpoint at bin {K}, "
         f"{M} more bins, single_pass={single_pass}")
    a = Sim(spec, single_pass=single_pass)
    a.set_bold(tr_bins=5)
    a.set_ou_background(mu=5.0, sigma=20.0, tau_ms=[5.0] + [0.0] * (len(spec.pops) - 1))
    a.step(10 * S)
    a.set_spike_injection(0.01, 40)
    a.step((K - 10) * S)
    image = a.checkpoint()
    a.step(M * S)
    b = Sim(spec, single_pass=single_pass)
    b.restore(image)
    assert b.stats()["bins"] == K
    b.step(M * S)
    _same_after(a, b, spec, K, M)
    ya, na = a.bold_state()
    yb, nb = b.bold_state()
    assert na == nb and np.array_equal(ya, yb)
    assert np.array_equal(a.bold(0, na), b.bold(0, nb))
    # bins before the checkpoint are not in the restored handle's history
    from paper_2211_15963_amd.dbsim import DbsimError
    with pytest.raises(DbsimError, match="precede the checkpoint"):
        b.spikes((K - 1) * S, K * S)
    with pytest.raises(DbsimError, match="precede the checkpoint"):
        b.region_signal(K - 1, K)
    a.close()
    b.close()


def test_resume_equals_oracle_and_early_checkpoint(Sim):
    spec = configs.share(n=20000, indegree=300, seed=42)
    S = spec.steps_per_bin
    orc = Oracle(spec, 32)
    K, M = 4, 26   # before the first ten bins (max delay) have passed
    _say(f"share 20000 / k300 seed 42, checkpoint at bin {K} (< max delay), {M} more bins vs the oracle")
    a = Sim(spec)
    a.step(K * S)
    image = a.checkpoint()
    a.close()
    b = Sim(spec)
    b.restore(image)
    b.step(M * S)
    orc.step((K + M) * S)
    st, ids = b.spikes(K * S, (K + M) * S)
    ost, oids = orc.spikes()
    sel = ost >= K * S
    assert st.size > 0
    assert np.array_equal(st, ost[sel].astype(np.uint64)) and np.array_equal(ids, oids[sel].astype(np.uint32))
    V, J, ref = b.state()
    oV, oJ, oref = orc.state()
    assert np.array_equal(V.astype(np.float64), oV) and np.array_equal(J.astype(np.float64), oJ)
    assert np.array_equal(ref, oref)
    assert b.stats()["edge_events"] == orc.edge_events
    b.close()


def test_checkpoint_errors(Sim):
    from paper_2211_15963_amd.dbsim import DbsimError
    spec = configs.tiny(seed=43)
    S = spec.steps_per_bin
    _say("tiny seed 43: checkpoint error paths")
    a = Sim(spec)
    a.step(5 * S + 3)
    with pytest.raises(DbsimError, match="bin boundaries"):
        a.checkpoint()
    a.step(S - 3)
    image = a.checkpoint()
    b = Sim(spec)
    b.step(S)
    with pytest.raises(DbsimError, match="not been stepped"):
        b.restore(image)
    b.close()
    d = Sim(configs.tiny(seed=44))
    with pytest.raises(DbsimError, match="another network"):
        d.restore(image)
    d.close()
    c = Sim(spec)
    with pytest.raises(DbsimError, match="shorter"):
        c.restore(image[: len(image) // 2])
    bad = bytearray(image)
    bad[0] ^= 0xFF
    with pytest.raises(DbsimError, match="not a checkpoint"):
        c.restore(bytes(bad))
    c.restore(image)  # the failed attempts left the fresh handle usable
    c.step(10 * S)
    a.step(10 * S)
    _same_after(a, c, spec, 6, 10)
    a.close()
    c.close()


def test_resume_with_small_buffers(Sim):
    """Streams and arena slices of one in a hundred of their in-edges on both sides: the
    restore re-assembles the next bin's delay >= 2 events through the slow paths (spills and
    overflow sums) and the continued run equals the uninterrupted one."""
    spec = configs.share(n=20000, indegree=300, seed=43)
    S, K, M = spec.steps_per_bin, 25, 25
    _say(f"share 20000 / k300 seed 43, stream and arena shares 10 per mille, checkpoint at bin {K}, {M} more")
    a = Sim(spec, stream_permille=10, arena_permille=10)
    a.step(K * S)
    image = a.checkpoint()
    a.step(M * S)
    assert a.stats()["overflow_events"] > 0
    b = Sim(spec, stream_permille=10, arena_permille=10)
    b.restore(image)
    b.step(M * S)
    _same_after(a, b, spec, K, M)
    a.close()
    b.close()
