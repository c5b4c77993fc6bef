"""Pins of the Balloon-Windkessel oracle (Extended Data Table 4) against what the
mathematics fixes: the rest state, the closed-form fixed point under constant
activity, first-order convergence of the Euler step to a high-accuracy
integration of the same ODE (scipy RK45), linearity for small inputs, and the
textbook time-to-peak of the haemodynamic response."""
import numpy as np
from scipy.integrate import solve_ivp

from oracle import bold

# the standard constants of the Balloon-Windkessel literature (the paper gives none)
P = dict(kappa=0.65, gamma=0.41, tau=0.98, alpha=0.32, rho=0.34, V0=0.02, k1=7 * 0.34, k2=2.0,
         k3=2 * 0.34 - 0.2, activity_scale=0.01, tr_bins=1)


def _rhs(t, x, zf):
    s, f, v, q = x
    z = zf(t)
    fout = v ** (1 / P["alpha"])
    E = 1 - (1 - P["rho"]) ** (1 / f)
    return [z - P["kappa"] * s - P["gamma"] * (f - 1), s, (f - fout) / P["tau"],
            (f * E / P["rho"] - fout * q / v) / P["tau"]]


def test_rest_is_stationary():
    ys, st = bold.run_activity(np.zeros((20000, 3)), P, 1e-3)
    assert np.all(np.abs(st - bold.rest_state(3)) < 1e-12)
    assert np.max(np.abs(ys)) < 1e-12


def test_constant_activity_reaches_closed_form_fixed_point():
    z = np.array([0.05, 0.2, 0.6])
    _, st = bold.run_activity(np.tile(z, (200000, 1)), P, 1e-3)  # 200 s
    fp = bold.fixed_point(z, P)
    assert np.allclose(st, fp, rtol=1e-9, atol=1e-11)
    # at the fixed point the flow balance holds: f = v^(1/alpha)
    assert np.allclose(fp[1], fp[2] ** (1 / P["alpha"]), rtol=1e-12)


def test_euler_converges_at_first_order_to_rk45():
    T = 20.0

    def zf(t):
        return 0.3 if 1.0 <= t < 3.0 else 0.0

    ref = solve_ivp(_rhs, (0, T), [0, 1, 1, 1], args=(zf,), method="RK45", rtol=1e-11, atol=1e-13,
                    dense_output=True, max_step=0.01)
    errs = []
    for h in (2e-3, 1e-3, 5e-4):
        n = int(round(T / h))
        t = (np.arange(n) + 1) * h
        zt = np.array([zf(tk - h) for tk in t])[:, None]  # step k uses the activity of its interval
        ys, _ = bold.run_activity(zt, P, h)
        x = ref.sol(t)
        yr = bold.bold_of(x[3], x[2], P)
        errs.append(np.max(np.abs(ys[:, 0] - yr)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 1.6 < r1 < 2.4 and 1.6 < r2 < 2.4, errs
    assert errs[1] < 1e-3 * np.max(np.abs(yr))


def test_small_inputs_respond_linearly():
    z = np.zeros((15000, 2))
    z[:1000, 0] = 1e-4
    z[:1000, 1] = 2e-4
    ys, _ = bold.run_activity(z, P, 1e-3)
    k = np.argmax(np.abs(ys[:, 0]))
    assert abs(ys[k, 1] / ys[k, 0] - 2.0) < 1e-3


def test_response_peaks_a_few_seconds_after_a_brief_burst():
    z = np.zeros((20000, 1))
    z[:500, 0] = 0.5  # 0.5 s of activity
    ys, _ = bold.run_activity(z, P, 1e-3)
    t_peak = (np.argmax(ys[:, 0]) + 1) * 1e-3
    assert 3.0 < t_peak < 7.0
    assert ys[:, 0].max() > 0 and ys[-1, 0] < 0.2 * ys[:, 0].max()  # decays (with an undershoot)


def test_sampling_and_counts_interface():
    rng = np.random.default_rng(0)
    counts = rng.poisson(3.0, size=(100, 4))
    sizes = np.array([100, 200, 0, 50])
    p = dict(P, tr_bins=25)
    ys, st = bold.run(counts, sizes, p, 1.0)
    assert ys.shape == (4, 4)
    # a region of size 0 has no activity and stays at rest
    assert np.allclose(st[:, 2], [0, 1, 1, 1], atol=1e-12)
    # splitting the run gives the same result
    y1, s1 = bold.run(counts[:60], sizes, p, 1.0)
    y2, s2 = bold.run(counts[60:], sizes, p, 1.0, state=s1, bins_done=60)
    assert np.array_equal(np.concatenate([y1, y2]), ys) and np.array_equal(s2, st)
