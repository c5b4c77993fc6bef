// kernels.hip - gfx950 kernels of one spike bin.
//
// Per bin k (S Euler steps of dt, SI Section 3):
//   k_scatter  fan-in of the arrivals due at the start of bin k. Every spike j
//              of bin k-d (d = 1..D) contributes its delay-d edges (Suppl.
//              Algorithm 2 pushes a spike list through destination lists;
//              here the delay ring is read backwards, so all events of a bin
//              land in one accumulator). Events are bucketed by target tile
//              into a per-tile arena slice, one reservation atomic per
//              (chunk, tile) instead of one global atomic per event.
//   k_gather   one workgroup per tile: sums its events in LDS as int64 fixed
//              point (exact, so any order gives the same bits), converts once
//              to float, writes A.
//   k_neuron   one lane per neuron, S substeps fused in registers: Philox
//              Poisson background, Euler update of V (CV equation), threshold,
//              reset and refractory clamp, receptor decay (eq. 3); at the bin
//              end, wavefront-ballot compaction of the spike list and the
//              per-block region partial sums.
//   k_readout  per-region mean synaptic current and spike count (fixed-order
//              tree over the region's block partials).
//   k_close    advances the bin counter and the spike-history ring.
//
// All float arithmetic is single IEEE operations in a fixed order (the file
// is built with -ffp-contract=off and f32 denormals preserved) so the result
// equals a scalar CPU evaluation of the same expressions.
#include "dbsim_internal.hpp"

namespace dbs {

namespace {

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Exclusive prefix sum over a 1024-thread block; *total receives the block sum.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* s_wave, uint32_t* total) {
    const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6;
    const uint32_t nw = blockDim.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= (uint32_t)o) x += y;
    }
    if (lane == 63u) s_wave[wid] = x;
    __syncthreads();
    if (wid == 0) {
        uint32_t t = lane < nw ? s_wave[lane] : 0u;
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            uint32_t y = __shfl_up(t, o, 64);
            if (lane >= (uint32_t)o) t += y;
        }
        if (lane < nw) s_wave[lane] = t;
    }
    __syncthreads();
    const uint32_t off = wid ? s_wave[wid - 1] : 0u;
    *total = s_wave[nw - 1];
    return off + x - v;
}

// index s in [0, n) with pre[s] <= e < pre[s+1] (largest s with pre[s] <= e)
__device__ __forceinline__ uint32_t seg_search(const uint32_t* pre, uint32_t n, uint32_t e) {
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1u) {
        uint32_t mid = (lo + hi) >> 1;
        if (pre[mid] <= e) lo = mid;
        else hi = mid;
    }
    return lo;
}

// fixed-point weight: round_half_even(w * 2^F) (exact: w * 2^F is exact in double)
__device__ __forceinline__ unsigned long long quant(float w, double qscale) {
    return (unsigned long long)(long long)__builtin_rint((double)w * qscale);
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two 32x32->64
// multiplies and a Weyl-sequence key schedule.
__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3, uint32_t k0,
                                              uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; r++) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
}

} // namespace

// ------------------------------------------------------------------ scatter

__global__ void __launch_bounds__(kScatterThreads) k_scatter(DevNet net) {
    extern __shared__ __align__(16) unsigned char dyn[];
    uint32_t* hist = reinterpret_cast<uint32_t*>(dyn);
    unsigned long long* cursor = reinterpret_cast<unsigned long long*>(dyn + ((4u * net.T + 15u) & ~15u));
    __shared__ unsigned long long s_sstart[kScatterSegs];
    __shared__ uint32_t s_spre[kScatterSegs + 1];
    __shared__ uint8_t s_scls[kScatterSegs];
    __shared__ unsigned long long s_dpre[DBNET_MAX_DELAY + 1];
    __shared__ unsigned long long s_dstart[DBNET_MAX_DELAY];
    __shared__ uint32_t s_wave[kScatterThreads / 64];

    const unsigned long long k = net.ctl->bin;
    const uint32_t D = net.D;
    const uint32_t tid = threadIdx.x;
    if (tid == 0) {
        unsigned long long tot = 0;
        for (uint32_t d = 1; d <= D; d++) {
            s_dpre[d - 1] = tot;
            s_dstart[d - 1] = 0;
            if (k >= d) {
                const uint32_t b = (uint32_t)((k - d) & net.MBmask);
                s_dstart[d - 1] = net.bin_start[b];
                tot += net.bin_cnt[b];
            }
        }
        s_dpre[D] = tot;
    }
    __syncthreads();
    const unsigned long long total = s_dpre[D];
    const unsigned long long nchunks = (total + kScatterSegs - 1) / kScatterSegs;
    const uint32_t tb = net.tile_bits, tmask = (1u << tb) - 1u, T = net.T;
    unsigned long long my_events = 0;

    for (unsigned long long c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const unsigned long long g0 = c * kScatterSegs;
        const uint32_t nseg = (uint32_t)min((unsigned long long)kScatterSegs, total - g0);
        uint32_t len = 0;
        if (tid < nseg) {
            const unsigned long long g = g0 + tid;
            uint32_t lo = 0, hi = D;
            while (hi - lo > 1u) {
                const uint32_t mid = (lo + hi) >> 1;
                if (s_dpre[mid] <= g) lo = mid;
                else hi = mid;
            }
            const uint32_t d = lo + 1;
            const unsigned long long idx = g - s_dpre[lo];
            const uint32_t j = net.rec[(s_dstart[lo] + idx) & net.RCmask] >> 4;
            const uint32_t* sg = net.seg + (size_t)j * (D + 1);
            const uint32_t so = sg[d - 1], eo = sg[d];
            s_sstart[tid] = net.row_ptr[j] + so;
            s_scls[tid] = net.src_inh[j];
            len = eo - so;
        }
        uint32_t ec;
        const uint32_t ex = block_exclusive_scan(len, s_wave, &ec);
        s_spre[tid] = ex;
        if (tid == 0) s_spre[kScatterSegs] = ec;
        for (uint32_t t = tid; t < T; t += blockDim.x) hist[t] = 0;
        __syncthreads();
        // sweep 1: events per tile
        for (uint32_t e = tid; e < ec; e += blockDim.x) {
            const uint32_t s = seg_search(s_spre, nseg, e);
            const unsigned long long edge = s_sstart[s] + (e - s_spre[s]);
            atomicAdd(&hist[net.col[edge] >> tb], 1u);
        }
        __syncthreads();
        // one reservation per non-empty tile
        for (uint32_t t = tid; t < T; t += blockDim.x) {
            const uint32_t h = hist[t];
            unsigned long long cur = ~0ull;
            if (h) {
                const uint32_t base = atomicAdd(&net.tile_fill[t], h);
                const unsigned long long cap = net.tile_base[t + 1] - net.tile_base[t];
                if ((unsigned long long)base + h <= cap) cur = net.tile_base[t] + base;
                else atomicOr(&net.ctl->err, kErrArena);
            }
            cursor[t] = cur;
        }
        __syncthreads();
        // sweep 2: write the events into the reserved slices
        for (uint32_t e = tid; e < ec; e += blockDim.x) {
            const uint32_t s = seg_search(s_spre, nseg, e);
            const unsigned long long edge = s_sstart[s] + (e - s_spre[s]);
            const uint32_t tgt = net.col[edge];
            const uint32_t t = tgt >> tb;
            if (cursor[t] != ~0ull) {
                const unsigned long long pos = atomicAdd(&cursor[t], 1ull);
                net.ev_tgt[pos] = (uint16_t)((tgt & tmask) | ((uint32_t)s_scls[s] << 15));
                if (net.KW == 2)
                    reinterpret_cast<float2*>(net.ev_w)[pos] = reinterpret_cast<const float2*>(net.w)[edge];
                else
                    net.ev_w[pos] = net.w[edge];
            }
        }
        my_events += ec;
        __syncthreads();
    }
    if (tid == 0 && my_events) atomicAdd(&net.ctl->edge_events, my_events);
}

// ------------------------------------------------------------------ gather

template <int KW>
__global__ void __launch_bounds__(kGatherThreads) k_gather(DevNet net) {
    extern __shared__ __align__(16) unsigned long long acc[];
    constexpr uint32_t U = 2 * KW;
    const uint32_t t = blockIdx.x;
    const uint32_t i0 = t << net.tile_bits;
    const uint32_t nt = min(1u << net.tile_bits, net.N - i0);
    const uint32_t lmask = (1u << net.tile_bits) - 1u;
    for (uint32_t x = threadIdx.x; x < nt * U; x += blockDim.x) acc[x] = 0ull;
    __syncthreads();
    const unsigned long long b0 = net.tile_base[t];
    const uint32_t cnt = net.tile_fill[t];
    const double qs = net.qscale;
    for (uint32_t e = threadIdx.x; e < cnt; e += blockDim.x) {
        const uint32_t v = net.ev_tgt[b0 + e];
        const uint32_t lt = v & lmask;
        const uint32_t u0 = (v >> 15) ? (uint32_t)KW : 0u;
        if (KW == 2) {
            const float2 w = reinterpret_cast<const float2*>(net.ev_w)[b0 + e];
            atomicAdd(&acc[lt * U + u0], quant(w.x, qs));
            atomicAdd(&acc[lt * U + u0 + 1], quant(w.y, qs));
        } else {
            atomicAdd(&acc[lt * U + u0], quant(net.ev_w[b0 + e], qs));
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) net.tile_fill[t] = 0;
    const float qinv = net.qinv;
    for (uint32_t x = threadIdx.x; x < nt; x += blockDim.x) {
#pragma unroll
        for (uint32_t u = 0; u < U; u++)
            net.A[(size_t)u * net.N + i0 + x] = (float)(long long)acc[x * U + u] * qinv;
    }
}

// ------------------------------------------------------------------ neuron

template <int U>
__global__ void __launch_bounds__(kNeuronBlock) k_neuron(DevNet net, int s0, int s1) {
    __shared__ uint32_t s_T[kMaxPoisson];
    __shared__ double s_red[kNeuronBlock];
    __shared__ uint32_t s_wcnt[kNeuronBlock / 64];
    const uint2 bi = net.blk[blockIdx.x];
    const PopParams& P = net.pops[bi.y];
    const int cmax = P.cmax;
    if ((int)threadIdx.x < cmax) s_T[threadIdx.x] = net.ptab[(size_t)bi.y * kMaxPoisson + threadIdx.x];
    const uint32_t i = bi.x + threadIdx.x;
    const bool active = i < P.end;
    const unsigned long long k = net.ctl->bin;
    const uint32_t N = net.N;
    const uint32_t S = net.S;

    float V = 0.0f, J[U], A[U];
    int ref = 0;
    uint32_t sub = 0xFFu;
#pragma unroll
    for (int u = 0; u < U; u++) {
        J[u] = 0.0f;
        A[u] = 0.0f;
    }
    if (active) {
        V = net.V[i];
#pragma unroll
        for (int u = 0; u < U; u++) J[u] = net.J[(size_t)u * N + i];
        ref = net.ref[i];
        if (s0 == 0) {
#pragma unroll
            for (int u = 0; u < U; u++) A[u] = net.A[(size_t)u * N + i];
        } else {
            sub = net.pend[i];
        }
    }
    __syncthreads();

    const float k_dt = P.k, gL = P.gL, VL = P.VL, Vth = P.Vth, Vr = P.Vr, Iext = P.Iext, wbg = P.wbg;
    float g[U], Vu[U], dec[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
        g[u] = P.g[u];
        Vu[u] = P.Vu[u];
        dec[u] = P.dec[u];
    }
    const int rsteps = P.r;
    const uint32_t key0 = (uint32_t)net.seed, key1 = (uint32_t)(net.seed >> 32);
    const uint32_t tag = (1u << 24) | (net.net_id & 0xFFFFFFu);
    uint32_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;
    unsigned long long cur_blk = ~0ull;

    for (int s = s0; s < s1; s++) {
        const unsigned long long n = k * S + (unsigned long long)s;
        const unsigned long long blk = n >> 2;
        if (blk != cur_blk) {
            w0 = (uint32_t)blk;
            w1 = (uint32_t)(blk >> 32);
            w2 = i;
            w3 = tag;
            philox4x32_10(w0, w1, w2, w3, key0, key1);
            cur_blk = blk;
        }
        const uint32_t sel = (uint32_t)(n & 3ull);
        const uint32_t x = sel == 0 ? w0 : sel == 1 ? w1 : sel == 2 ? w2 : w3;
        uint32_t c = 0;
        for (int m = 0; m < cmax; m++) c += (x >= s_T[m]) ? 1u : 0u;

        float Vn;
        if (ref > 0) {
            Vn = Vr;
            ref -= 1;
        } else {
            float I = gL * (VL - V);
#pragma unroll
            for (int u = 0; u < U; u++) {
                const float gJ = g[u] * J[u];
                I = I + gJ * (Vu[u] - V);
            }
            I = I + Iext;
            Vn = V + k_dt * I;
            if (Vn >= Vth) {
                Vn = Vr;
                ref = rsteps;
                sub = (uint32_t)s;
            }
        }
        V = Vn;
        const float B = wbg * (float)c;
#pragma unroll
        for (int u = 0; u < U; u++) {
            const float a = (s == 0) ? A[u] : 0.0f;
            float Jn = dec[u] * J[u] + a;
            if (u == 0) Jn = Jn + B;
            J[u] = Jn;
        }
    }
    if (active) {
        net.V[i] = V;
#pragma unroll
        for (int u = 0; u < U; u++) net.J[(size_t)u * N + i] = J[u];
        net.ref[i] = (uint8_t)ref;
        if (s1 < (int)S) net.pend[i] = (uint8_t)sub;
    }
    if (s1 < (int)S) return; // block-uniform: the bin continues in a later launch

    // bin end: spike-list compaction (one atomic per wavefront)
    const bool spiked = active && sub != 0xFFu;
    const unsigned long long mask = __ballot(spiked);
    const uint32_t nw = (uint32_t)__popcll(mask);
    const uint32_t slot = (uint32_t)(k & net.MBmask);
    uint32_t base = 0;
    if (nw) {
        if (lane_id() == 0) base = atomicAdd(&net.bin_cnt[slot], nw);
        base = __shfl(base, 0, 64);
        if (spiked) {
            const uint32_t rank = (uint32_t)__popcll(mask & ((1ull << lane_id()) - 1ull));
            const unsigned long long pos = net.bin_start[slot] + base + rank;
            net.rec[pos & net.RCmask] = (i << 4) | sub;
        }
    }
    if (!net.regions_on) return;
    // region partials: total synaptic current per neuron, summed in a fixed tree
    float cur = 0.0f;
#pragma unroll
    for (int u = 0; u < U; u++) {
        const float t = (g[u] * J[u]) * (Vu[u] - V);
        cur = cur + t;
    }
    s_red[threadIdx.x] = active ? (double)cur : 0.0;
    if (lane_id() == 0) s_wcnt[threadIdx.x >> 6] = nw;
    __syncthreads();
    for (uint32_t st = kNeuronBlock / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) s_red[threadIdx.x] += s_red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        uint32_t c = 0;
        for (int w = 0; w < kNeuronBlock / 64; w++) c += s_wcnt[w];
        net.blk_sig[blockIdx.x] = s_red[0];
        net.blk_cnt[blockIdx.x] = c;
    }
}

// ------------------------------------------------------------------ readout

__global__ void __launch_bounds__(256) k_readout(DevNet net) {
    __shared__ double s[256];
    __shared__ uint32_t sc[256];
    const uint32_t r = blockIdx.x;
    const unsigned long long k = net.ctl->bin;
    const uint32_t b0 = net.reg_blk_ptr[r], b1 = net.reg_blk_ptr[r + 1];
    double a = 0.0;
    uint32_t c = 0;
    for (uint32_t b = b0 + threadIdx.x; b < b1; b += blockDim.x) {
        a += net.blk_sig[net.reg_blk[b]];
        c += net.blk_cnt[net.reg_blk[b]];
    }
    s[threadIdx.x] = a;
    sc[threadIdx.x] = c;
    __syncthreads();
    for (uint32_t st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            s[threadIdx.x] += s[threadIdx.x + st];
            sc[threadIdx.x] += sc[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const size_t o = (size_t)(k & net.MBmask) * net.n_regions + r;
        net.sig[o] = s[0] / (double)net.reg_size[r];
        net.sig_cnt[o] = sc[0];
    }
}

__global__ void k_close(DevNet net) {
    if (threadIdx.x == 0) {
        const unsigned long long k = net.ctl->bin;
        const uint32_t m = net.MBmask;
        const uint32_t c = net.bin_cnt[k & m];
        net.bin_start[(k + 1) & m] = net.bin_start[k & m] + c;
        net.bin_cnt[(k + 1) & m] = 0;
        net.ctl->spikes += c;
        net.ctl->bin = k + 1;
    }
}

// ------------------------------------------------------------------ launchers

size_t scatter_lds_bytes(const DevNet& n) { return ((4u * n.T + 15u) & ~15u) + 8u * (size_t)n.T; }

size_t gather_lds_bytes(const DevNet& n) { return ((size_t)1 << n.tile_bits) * n.U * 8u; }

hipError_t launch_scatter(const DevNet& n, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_scatter, dim3(grid), dim3(kScatterThreads), scatter_lds_bytes(n), st, n);
    return hipGetLastError();
}

hipError_t prepare_kernels() {
    hipError_t e = hipFuncSetAttribute((const void*)k_gather<1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)kTileLdsBytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_gather<2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)kTileLdsBytes);
}

hipError_t launch_gather(const DevNet& n, hipStream_t st) {
    if (n.KW == 2)
        hipLaunchKernelGGL(k_gather<2>, dim3(n.T), dim3(kGatherThreads), gather_lds_bytes(n), st, n);
    else
        hipLaunchKernelGGL(k_gather<1>, dim3(n.T), dim3(kGatherThreads), gather_lds_bytes(n), st, n);
    return hipGetLastError();
}

hipError_t launch_neuron(const DevNet& n, int s0, int s1, hipStream_t st) {
    if (n.U == 4)
        hipLaunchKernelGGL(k_neuron<4>, dim3(n.n_blocks), dim3(kNeuronBlock), 0, st, n, s0, s1);
    else
        hipLaunchKernelGGL(k_neuron<2>, dim3(n.n_blocks), dim3(kNeuronBlock), 0, st, n, s0, s1);
    return hipGetLastError();
}

hipError_t launch_readout(const DevNet& n, hipStream_t st) {
    hipLaunchKernelGGL(k_readout, dim3(n.n_regions), dim3(256), 0, st, n);
    return hipGetLastError();
}

hipError_t launch_close(const DevNet& n, hipStream_t st) {
    hipLaunchKernelGGL(k_close, dim3(1), dim3(64), 0, st, n);
    return hipGetLastError();
}

} // namespace dbs
