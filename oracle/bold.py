"""Balloon-Windkessel haemodynamic model of the region BOLD signal.

TEST INFRASTRUCTURE ONLY: the plain CPU reference that the GPU BOLD step is
checked against (tests, smoke check). Never part of the product path.

The model is the one of Extended Data Table 4 (z the neural activity, s the
vasodilatory signal, f the inflow, v the blood volume, q the deoxyhaemoglobin
content, y the BOLD signal):

    ds/dt = z - kappa s - gamma (f - 1)
    df/dt = s
    tau dv/dt = f - v^(1/alpha)
    tau dq/dt = f E(f, rho) / rho - v^(1/alpha) q / v,   E(f, rho) = 1 - (1 - rho)^(1/f)
    y = V0 (k1 (1 - q) + k2 (1 - q / v) + k3 (1 - v))

discretised, as the Supplementary Information's HMDA framework does (an
Euler-Maruyama step of the model per time step, here without noise), with one
explicit Euler step per spike bin of length h, every right-hand side at the old
state. The activity of region r in bin k is its firing rate scaled,
z = activity_scale / (N_r h) * count_r(k) (Fig. 2a: rates from spike counts feed
the model). A sample y is taken after every tr_bins bins.

FP64 numpy; each expression is written in the order the equations give so that
a reader can check it against the table.
"""
from __future__ import annotations

from typing import Dict, Optional, Tuple

import numpy as np


def rest_state(n_regions: int) -> np.ndarray:
    st = np.ones((4, n_regions), np.float64)
    st[0] = 0.0
    return st


def fixed_point(z: np.ndarray, p: Dict) -> np.ndarray:
    """Stationary state under constant activity z: s = 0, f = 1 + z / gamma,
    v = f^alpha (outflow equals inflow), q = v E(f) / rho."""
    f = 1.0 + np.asarray(z, np.float64) / p["gamma"]
    v = f ** p["alpha"]
    E = 1.0 - (1.0 - p["rho"]) ** (1.0 / f)
    q = v * E / p["rho"]
    return np.stack([np.zeros_like(f), f, v, q])


def bold_of(q: np.ndarray, v: np.ndarray, p: Dict) -> np.ndarray:
    return p["V0"] * (p["k1"] * (1.0 - q) + p["k2"] * (1.0 - q / v) + p["k3"] * (1.0 - v))


def euler_step(st: np.ndarray, z: np.ndarray, h: float, p: Dict) -> np.ndarray:
    s, f, v, q = st
    ht = h / p["tau"]
    fout = v ** (1.0 / p["alpha"])
    E = 1.0 - (1.0 - p["rho"]) ** (1.0 / f)
    s1 = s + h * (z - p["kappa"] * s - p["gamma"] * (f - 1.0))
    f1 = f + h * s
    v1 = v + ht * (f - fout)
    q1 = q + ht * (f * E / p["rho"] - fout * q / v)
    return np.stack([s1, f1, v1, q1])


def run(counts: np.ndarray, region_sizes: np.ndarray, p: Dict, bin_ms: float,
        state: Optional[np.ndarray] = None, bins_done: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """Steps the model over counts[bins][regions]; returns (samples [m][regions], final state).
    bins_done: bins already stepped since rest (for the sampling phase)."""
    counts = np.asarray(counts)
    R = counts.shape[1]
    h = float(np.float32(bin_ms)) * 1e-3  # the network description holds bin_ms as f32
    sizes = np.asarray(region_sizes, np.float64)
    zs = np.where(sizes > 0, p["activity_scale"] / (np.maximum(sizes, 1.0) * h), 0.0)
    st = rest_state(R) if state is None else np.array(state, np.float64)
    ys = []
    for k in range(counts.shape[0]):
        z = zs * counts[k].astype(np.float64)
        st = euler_step(st, z, h, p)
        if (bins_done + k + 1) % p["tr_bins"] == 0:
            ys.append(bold_of(st[3], st[2], p))
    return (np.array(ys) if ys else np.zeros((0, R))), st


def run_activity(z: np.ndarray, p: Dict, h: float) -> Tuple[np.ndarray, np.ndarray]:
    """Euler trajectory for a given activity time course z[steps][regions]; returns
    (y at every step, final state). For the pins below."""
    z = np.asarray(z, np.float64)
    st = rest_state(z.shape[1])
    ys = np.empty(z.shape)
    for k in range(z.shape[0]):
        st = euler_step(st, z[k], h, p)
        ys[k] = bold_of(st[3], st[2], p)
    return ys, st
