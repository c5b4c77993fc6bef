"""Dense brute-force simulator for tiny networks (N <= ~50). TEST INFRASTRUCTURE ONLY.

An independent restatement of the same discrete method with a different data
representation: dense weight matrices W[u][i, j] (fixed point, int64) and a
dense delay matrix Dm[i, j] replace the oracle's per-target edge lists, and a
spike history matrix replaces its bitmaps. Philox4x32-10 and the Poisson
inversion table are re-implemented here in numpy/Python from their published
definitions. It is used only to pin the oracle's sparse fan-in, delays and
receptor routing (a transposed operand, an off-by-one delay or a wrong
receptor fails the bit-exact comparison).

Only the FP32 variant is provided; all float arithmetic is numpy float32
element-wise, one IEEE operation at a time, in the oracle's order.
"""
from __future__ import annotations

import math

import numpy as np

from netgen.desc import NetSpec, generate

M0, M1, W0, W1 = 0xD2511F53, 0xCD9E8D57, 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox_np(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10 over uint64 arrays holding 32-bit values."""
    c0, c1, c2, c3 = (np.asarray(x, np.uint64) & MASK for x in (c0, c1, c2, c3))
    k0, k1 = int(k0) & MASK, int(k1) & MASK
    for r in range(10):
        if r:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = c0 * np.uint64(M0)
        p1 = c2 * np.uint64(M1)
        c0, c1, c2, c3 = ((p1 >> np.uint64(32)) ^ c1 ^ np.uint64(k0), p1 & np.uint64(MASK),
                          (p0 >> np.uint64(32)) ^ c3 ^ np.uint64(k1), p0 & np.uint64(MASK))
    return c0, c1, c2, c3


def poisson_thresholds(lam: float):
    p = math.exp(-lam)
    F = p
    T = []
    c = 0
    while not (1.0 - F < 2.0 ** -32):
        T.append(int(math.floor(F * 2.0 ** 32)))
        c += 1
        p = p * lam / c
        F = F + p
    return np.array(T, dtype=np.uint64)


def simulate(spec: NetSpec, n_steps: int, regions: bool = False):
    """Returns (raster list of (step, id), V float32 [N], J float32 [U, N], ref int32 [N], edge_events);
    with regions=True also (sig float64 [bins, regions], counts int64 [bins, regions]): at every bin
    end, the mean over each region's neurons of the FP32 current sum_u (g_u J_u)(V_u - V) (each
    neuron's current in float32, receptor order, one operation at a time; the region sum in double in
    ascending neuron id) and the region's spike count in the bin."""
    net = generate(spec)
    N = spec.num_neurons
    S = spec.steps_per_bin
    KW = spec.weights_per_edge
    U = 2 * KW
    F = spec.frac_bits
    umap = [0, 2] if KW == 1 else [0, 1, 2, 3]
    off = spec.pop_offsets()
    pop = np.searchsorted(off[1:], np.arange(N), side="right")
    exc = spec.is_exc_neuron()
    D = spec.max_delay
    # dense fixed-point weights W[u, i, j] and delays Dm[i, j] (0 = no edge)
    W = np.zeros((U, N, N), np.int64)
    Dm = np.zeros((N, N), np.int64)
    for i in range(N):
        for e in range(int(net["ptr"][i]), int(net["ptr"][i + 1])):
            j = int(net["src"][e])
            assert Dm[i, j] == 0, "multapse"
            Dm[i, j] = int(net["delay"][e])
            base = 0 if exc[j] else KW
            W[base, i, j] = int(np.rint(np.float64(net["w0"][e]) * 2.0 ** F))
            if KW == 2:
                W[base + 1, i, j] = int(np.rint(np.float64(net["w1"][e]) * 2.0 ** F))
    f32 = np.float32
    P = spec.pops
    dt = float(np.float32(spec.dt_ms))
    k = np.array([f32(dt / float(f32(P[p].C))) for p in pop], f32)
    gL = np.array([P[p].g_L for p in pop], f32)
    VL = np.array([P[p].V_L for p in pop], f32)
    Vth = np.array([P[p].V_th for p in pop], f32)
    Vr = np.array([P[p].V_reset for p in pop], f32)
    Iext = np.array([P[p].I_ext for p in pop], f32)
    g = np.array([[P[p].g[umap[u]] for p in pop] for u in range(U)], f32)
    Vu = np.array([[P[p].V_rev[umap[u]] for p in pop] for u in range(U)], f32)
    dec = np.array([[f32(math.exp(-dt / float(f32(P[p].tau[umap[u]])))) for p in pop] for u in range(U)], f32)
    wbg = np.array([P[p].w_bg for p in pop], f32)
    r = np.array([int(round(float(f32(P[p].T_ref)) / dt)) for p in pop], np.int32)
    tables = [poisson_thresholds(float(f32(P[p].bg_rate_hz)) * dt * 1e-3) for p in range(len(P))]
    V = net["v0"].astype(f32).copy()
    J = np.zeros((U, N), f32)
    ref = np.zeros(N, np.int32)
    spk_hist = np.zeros((n_steps // S + 2, N), bool)  # spikes per bin
    raster = []
    events = 0
    reg = np.array([P[p].region for p in pop], np.int64)
    R = spec.n_regions
    sigs, cnts = [], []
    seed = int(spec.seed)
    ids = np.arange(N, dtype=np.uint64)
    for n in range(n_steps):
        kb, s = divmod(n, S)
        if s == 0:
            acc = np.zeros((U, N), np.int64)
            for d in range(1, D + 1):
                b = kb - d
                if b < 0:
                    continue
                a = spk_hist[b].astype(np.int64)           # A_j at bin b
                mask = (Dm == d).astype(np.int64)           # edges with delay d
                for u in range(U):
                    acc[u] += (W[u] * mask) @ a
                events += int(((Dm == d) & spk_hist[b][None, :]).sum())
            A = acc.astype(f32) * f32(2.0 ** -F)
        else:
            A = np.zeros((U, N), f32)
        blk = n // 4
        words = philox_np(np.full(N, blk & MASK), np.full(N, blk >> 32), ids,
                          np.full(N, (1 << 24) | (spec.net_id & 0xFFFFFF)), seed & MASK, seed >> 32)
        x = words[n % 4]
        c = np.array([int((x[i] >= tables[pop[i]]).sum()) for i in range(N)], np.int64)
        # voltage (old V and J)
        I = gL * (VL - V)
        for u in range(U):
            I = I + (g[u] * J[u]) * (Vu[u] - V)
        I = I + Iext
        Vn = V + k * I
        refr = ref > 0
        fire = (~refr) & (Vn >= Vth)
        Vn = np.where(refr | fire, Vr, Vn).astype(f32)
        ref = np.where(refr, ref - 1, np.where(fire, r, 0)).astype(np.int32)
        B = wbg * c.astype(f32)
        Jn = dec * J + A
        Jn[0] = Jn[0] + B
        V, J = Vn, Jn.astype(f32)
        for i in np.nonzero(fire)[0]:
            raster.append((n, int(i)))
        spk_hist[kb] |= fire
        if regions and s == S - 1:
            cur = np.zeros(N, f32)
            for u in range(U):
                cur = cur + (g[u] * J[u]) * (Vu[u] - V)
            sig = np.zeros(R)
            cnt = np.zeros(R, np.int64)
            for rr in range(R):
                idx = np.nonzero(reg == rr)[0]
                acc = 0.0
                for i in idx:  # ascending neuron id, double accumulator
                    acc = acc + float(cur[i])
                sig[rr] = acc / len(idx) if len(idx) else 0.0
                cnt[rr] = int(spk_hist[kb][idx].sum())
            sigs.append(sig)
            cnts.append(cnt)
    if regions:
        return raster, V, J, ref, events, np.array(sigs).reshape(-1, R), np.array(cnts).reshape(-1, R)
    return raster, V, J, ref, events
