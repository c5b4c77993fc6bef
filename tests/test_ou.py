"""Ornstein-Uhlenbeck background current (eq. 1 with its Euler form, eq. 4) in the oracle.

The increment draw is pinned bit for bit by an independent numpy Philox and by the
moments of the twelve-term Irwin-Hall sum it is built from; the recurrence is pinned by
the closed forms of the discrete OU (AR(1)) process it must follow (stationary mean and
variance, lag autocorrelation) and by the noiseless case, which must equal a constant
external current bit for bit."""
import numpy as np

from netgen import configs
from oracle import Oracle, ou_normal
from oracle.brute import philox_np


def _z_np(seed, net_id, n, ids):
    """twelve 10-bit fields of one Philox block, standardised (independent of the C oracle)"""
    ids = np.asarray(ids)
    w = philox_np(np.full(ids.shape, n & 0xFFFFFFFF), np.full(ids.shape, n >> 32), ids,
                  np.full(ids.shape, (3 << 24) | net_id), seed & 0xFFFFFFFF, seed >> 32)
    s = sum(((x >> np.uint64(10 * f)) & np.uint64(1023)).astype(np.int64) for x in w for f in range(3))
    return (2 * s - 12276).astype(np.float64) / 2048.0


def test_increment_matches_independent_philox_bits():
    for seed, net_id, n in ((0, 0, 0), (12345, 7, 99), (2**40 + 3, 0xABCDEF, 2**33 + 5)):
        ids = np.arange(0, 4000, 13)
        exp = _z_np(seed, net_id, n, ids)
        got = np.array([ou_normal(seed, net_id, n, int(i)) for i in ids], np.float64)
        assert np.array_equal(got, exp)


def test_increment_moments_are_irwin_hall_twelve():
    ids = np.arange(20000)
    z = np.concatenate([_z_np(3, 1, n, ids) for n in range(10)])
    assert z.min() >= -6.0 and z.max() <= 6.0 - 12.0 / 2048.0  # bounded support
    # twelve uniform fields: mean 0, variance 1 - 2^-20, excess kurtosis -6/(5*12) = -0.1
    se = 1.0 / np.sqrt(z.size)
    assert abs(z.mean()) < 5 * se
    assert abs(z.var() - (1.0 - 2.0**-20)) < 5 * np.sqrt(2.0) * se
    kurt = np.mean((z - z.mean())**4) / z.var()**2 - 3.0
    assert abs(kurt + 0.1) < 5 * np.sqrt(24.0) * se
    # every value is an exact multiple of 2^-10 (integer arithmetic, no rounding)
    assert np.array_equal(z * 1024.0, np.round(z * 1024.0))


def _silent(seed=5):
    s = configs.tiny(seed=seed, bg_rate_hz=0.0)
    for p in s.pops:
        p.v0_lo, p.v0_hi = -69.0, -68.0
    return s


def test_ou_process_stationary_moments_and_autocorrelation():
    spec = _silent()
    mu, sigma, tau = 10.0, 25.0, 2.0  # pA, pA, ms
    dt = spec.dt_ms
    c1 = dt / tau
    c2 = sigma * np.sqrt(2.0 * dt / tau)
    o = Oracle(spec, 32)
    o.set_ou(mu, sigma, tau)
    assert np.all(o.ou_current() == np.float32(mu))  # starts at the mean
    o.step(200)  # 10 time constants of burn-in
    trace = []
    for _ in range(600):
        o.step(1)
        trace.append(o.ou_current())
    x = np.array(trace)  # [steps, N]
    var_inf = c2**2 / (1.0 - (1.0 - c1)**2)  # stationary variance of the discrete recurrence
    # independent neurons; ~x.shape[0] * c1 / 2 effectively independent samples per neuron
    n_eff = x.shape[1] * x.shape[0] * c1 / 2.0
    assert abs(x.mean() - mu) < 5 * np.sqrt(var_inf / n_eff)
    assert abs(x.var() / var_inf - 1.0) < 0.05
    xc = x - mu
    for m in (1, 5, 20):
        rho = np.mean(xc[m:] * xc[:-m]) / np.mean(xc * xc)
        assert abs(rho - (1.0 - c1)**m) < 0.03


def test_noiseless_ou_equals_a_constant_external_current():
    base = configs.tiny(seed=6)
    assert all(p.I_ext == 0.0 for p in base.pops)
    S = base.steps_per_bin
    ou = Oracle(base, 32)
    ou.set_ou([40.0, 30.0], 0.0, [3.0, 3.0])
    ou.step(30 * S)
    ext = configs.tiny(seed=6)
    ext.pops[0].I_ext, ext.pops[1].I_ext = 40.0, 30.0
    ref = Oracle(ext, 32)
    ref.step(30 * S)
    a, b = ou.spikes(), ref.spikes()
    assert len(a[0]) > 100
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    for x, y in zip(ou.state(), ref.state()):
        assert np.array_equal(x, y)


def test_ou_off_is_the_plain_run_and_fp64_agrees_in_distribution():
    spec = configs.tiny(seed=7)
    S = spec.steps_per_bin
    plain = Oracle(spec, 32)
    plain.step(10 * S)
    off = Oracle(spec, 32)
    off.set_ou(5.0, 5.0, 0.0)  # tau <= 0: off
    off.step(10 * S)
    assert np.array_equal(plain.spikes()[1], off.spikes()[1])
    assert np.all(off.ou_current() == 0.0)
    # FP64 oracle runs the same recurrence on the same draws: its current tracks the FP32 one
    o32, o64 = Oracle(spec, 32), Oracle(spec, 64)
    for o in (o32, o64):
        o.set_ou(0.0, 20.0, 5.0)
        o.step(3 * S)
    d = np.abs(o32.ou_current() - o64.ou_current())
    assert d.max() < 1e-3
