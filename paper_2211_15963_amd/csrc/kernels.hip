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
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
    }
}

} // namespace

// ------------------------------------------------------------------ scatter

namespace {

// XCC (accelerator complex die) this wavefront runs on; used only to pick which tile
// group a workgroup serves first, never for correctness.
__device__ __forceinline__ uint32_t xcc_id() { return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20); }

// exclusive scan of v[0..n) in place (n <= 2 * blockDim.x), returns the total
__device__ uint32_t block_scan_inplace(uint32_t* v, uint32_t n, uint32_t* s_wave) {
    const uint32_t t = threadIdx.x;
    const uint32_t a = 2 * t < n ? v[2 * t] : 0u, b = 2 * t + 1 < n ? v[2 * t + 1] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(a + b, s_wave, &tot);
    if (2 * t < n) v[2 * t] = ex;
    if (2 * t + 1 < n) v[2 * t + 1] = ex + a;
    return tot;
}

} // namespace

// Fan-in of the arrivals due at the start of bin k (see the file header). Targets are
// split into kTileGroups groups of consecutive tiles; every (spike, delay) segment of a
// row is further split by group (rows are sorted by delay, then target). Work items are
// (group, chunk of segments) taken from one queue per group; a workgroup serves the group
// of its own XCC first (its arena writes then stay in that XCC's L2) and then helps the
// others, so the bin completes whatever the placement. Each chunk is processed in rounds
// that stage the events in LDS, sort them by tile, reserve one slice per non-empty tile
// and write the records out in runs of consecutive addresses.
__global__ void __launch_bounds__(kScatterThreads) k_scatter(DevNet net) {
    extern __shared__ __align__(16) unsigned char dyn[];
    const uint32_t D = net.D, G = kTileGroups, TG = net.TG, RE = net.round_events;
    unsigned char* p = dyn;
    unsigned long long* s_dpre = reinterpret_cast<unsigned long long*>(p); p += 8 * (DBNET_MAX_DELAY + 1);
    unsigned long long* s_dstart = reinterpret_cast<unsigned long long*>(p); p += 8 * DBNET_MAX_DELAY;
    unsigned long long* s_sstart = reinterpret_cast<unsigned long long*>(p); p += 8 * kScatterSegs;
    unsigned long long* gbase = reinterpret_cast<unsigned long long*>(p); p += 8 * ((TG + 1) & ~1u);
    float2* r_w = reinterpret_cast<float2*>(p); p += 8 * RE;
    uint32_t* r_col = reinterpret_cast<uint32_t*>(p); p += 4 * RE;
    uint32_t* s_spre = reinterpret_cast<uint32_t*>(p); p += 4 * (kScatterSegs + 4);
    uint32_t* hist = reinterpret_cast<uint32_t*>(p); p += 4 * TG;
    uint32_t* lstart = reinterpret_cast<uint32_t*>(p); p += 4 * TG;
    uint32_t* lcur = reinterpret_cast<uint32_t*>(p); p += 4 * TG;
    uint32_t* s_misc = reinterpret_cast<uint32_t*>(p); p += 4 * 20; // [0..15] scan scratch, [16] queue ticket
    uint16_t* r_idx = reinterpret_cast<uint16_t*>(p); p += 2 * RE;
    uint8_t* s_scls = reinterpret_cast<uint8_t*>(p);

    const unsigned long long k = net.ctl->bin;
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
    if (total == 0) return;
    // segments per chunk: about chunks_per_wg chunks per workgroup over all groups, at most kScatterSegs
    const unsigned long long cw = (unsigned long long)net.chunks_per_wg * gridDim.x;
    const unsigned long long want = (total * G + cw - 1) / cw;
    const uint32_t spc = (uint32_t)min((unsigned long long)kScatterSegs, max(32ull, want));
    const uint32_t nchunks = (uint32_t)((total + spc - 1) / spc);
    const uint32_t tb = net.tile_bits, tmask = (1u << tb) - 1u, DG1 = D * G + 1;
    const uint32_t g0 = xcc_id() % G;
    unsigned long long my_events = 0;

    for (uint32_t gi = 0; gi < G; gi++) {
        const uint32_t g = (g0 + gi) % G;
        const uint32_t t0 = g * TG;                       // first tile of the group
        const uint32_t ntg = t0 < net.T ? min(TG, net.T - t0) : 0u;
        for (;;) {
            if (tid == 0) s_misc[16] = atomicAdd(&net.sq[g], 1u);
            __syncthreads();
            const uint32_t c = s_misc[16];
            __syncthreads();
            if (c >= nchunks || ntg == 0) break;
            const unsigned long long i0 = (unsigned long long)c * spc;
            const uint32_t nseg = (uint32_t)min((unsigned long long)spc, total - i0);
            uint32_t len = 0;
            if (tid < nseg) {
                const unsigned long long it = i0 + tid;
                uint32_t lo = 0, hi = D;
                while (hi - lo > 1u) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (s_dpre[mid] <= it) lo = mid;
                    else hi = mid;
                }
                const uint32_t d = lo + 1;
                const uint32_t j = net.rec[(s_dstart[lo] + (it - s_dpre[lo])) & net.RCmask] >> 4;
                const uint32_t* sg = net.seg + (size_t)j * DG1 + (d - 1) * G + g;
                const uint32_t so = sg[0], eo = sg[1];
                s_sstart[tid] = net.row_ptr[j] + so;
                s_scls[tid] = net.src_inh[j];
                len = eo - so;
            }
            uint32_t ec;
            const uint32_t ex = block_exclusive_scan(len, s_misc, &ec);
            s_spre[tid] = ex;
            if (tid == 0) s_spre[kScatterSegs] = ec;
            __syncthreads();
            for (uint32_t r0 = 0; r0 < ec; r0 += RE) {
                const uint32_t ne = min(RE, ec - r0);
                for (uint32_t t = tid; t < ntg; t += blockDim.x) hist[t] = 0;
                __syncthreads();
                // stage the round's events in LDS and count them per tile
                uint32_t s_lo = 0;
                for (uint32_t e = tid; e < ne; e += blockDim.x) {
                    const uint32_t ge = r0 + e;
                    const uint32_t s = s_lo + seg_search(s_spre + s_lo, nseg - s_lo, ge);
                    s_lo = s;
                    const unsigned long long edge = s_sstart[s] + (ge - s_spre[s]);
                    const uint32_t tgt = net.col[edge];
                    r_col[e] = tgt | ((uint32_t)s_scls[s] << 31);
                    r_w[e] = net.KW == 2 ? reinterpret_cast<const float2*>(net.w)[edge] : make_float2(net.w[edge], 0.0f);
                    uint32_t lt = (tgt >> tb) - t0;
                    if (lt >= ntg) { // a target outside the group: the table is inconsistent
                        atomicOr(&net.ctl->err, kErrLayout);
                        lt = 0;
                    }
                    atomicAdd(&hist[lt], 1u);
                }
                __syncthreads();
                // one global reservation per non-empty tile; local offsets by a scan
                for (uint32_t t = tid; t < ntg; t += blockDim.x) {
                    const uint32_t h = hist[t];
                    unsigned long long gb = ~0ull;
                    if (h) {
                        const uint32_t base = atomicAdd(&net.tile_fill[t0 + t], h);
                        const unsigned long long tb0 = net.tile_base[t0 + t];
                        if ((unsigned long long)base + h <= net.tile_base[t0 + t + 1] - tb0) gb = tb0 + base;
                        else atomicOr(&net.ctl->err, kErrArena);
                    }
                    gbase[t] = gb;
                    lstart[t] = h;
                }
                __syncthreads();
                block_scan_inplace(lstart, ntg, s_misc);
                __syncthreads();
                for (uint32_t t = tid; t < ntg; t += blockDim.x) lcur[t] = lstart[t];
                __syncthreads();
                // counting sort of the staged events by tile
                for (uint32_t e = tid; e < ne; e += blockDim.x) {
                    uint32_t lt = ((r_col[e] & 0x7FFFFFFFu) >> tb) - t0;
                    lt = lt < ntg ? lt : 0u;
                    r_idx[atomicAdd(&lcur[lt], 1u)] = (uint16_t)e;
                }
                __syncthreads();
                // write-out: consecutive threads write consecutive records of a tile's run
                for (uint32_t q = tid; q < ne; q += blockDim.x) {
                    const uint32_t e = r_idx[q];
                    const uint32_t v = r_col[e];
                    const uint32_t tgt = v & 0x7FFFFFFFu;
                    uint32_t lt = (tgt >> tb) - t0;
                    lt = lt < ntg ? lt : 0u;
                    const unsigned long long gb = gbase[lt];
                    if (gb != ~0ull) {
                        const unsigned long long pos = gb + (q - lstart[lt]);
                        const uint32_t key = (tgt & tmask) | (v & 0x80000000u);
                        const float2 w = r_w[e];
                        if (net.KW == 2)
                            reinterpret_cast<uint3*>(net.ev)[pos] = make_uint3(key, __float_as_uint(w.x), __float_as_uint(w.y));
                        else
                            reinterpret_cast<uint2*>(net.ev)[pos] = make_uint2(key, __float_as_uint(w.x));
                    }
                }
                __syncthreads();
            }
            my_events += ec;
        }
    }
    if (tid == 0 && my_events) atomicAdd(&net.ctl->edge_events, my_events);
}

size_t scatter_fixed_lds(uint32_t TG) {
    return 8 * (DBNET_MAX_DELAY + 1) + 8 * DBNET_MAX_DELAY + 8 * kScatterSegs + 8 * ((TG + 1) & ~1u) +
           4 * (kScatterSegs + 4) + 12 * (size_t)TG + 4 * 20 + kScatterSegs + 16;
}

size_t scatter_lds_bytes(const DevNet& n) { return scatter_fixed_lds(n.TG) + 14 * (size_t)n.round_events; }

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
        if (KW == 2) {
            const uint3 r = reinterpret_cast<const uint3*>(net.ev)[b0 + e];
            const uint32_t lt = r.x & lmask;
            const uint32_t u0 = (r.x >> 31) ? 2u : 0u;
            atomicAdd(&acc[lt * U + u0], quant(__uint_as_float(r.y), qs));
            atomicAdd(&acc[lt * U + u0 + 1], quant(__uint_as_float(r.z), qs));
        } else {
            const uint2 r = reinterpret_cast<const uint2*>(net.ev)[b0 + e];
            const uint32_t lt = r.x & lmask;
            const uint32_t u0 = (r.x >> 31) ? 1u : 0u;
            atomicAdd(&acc[lt * U + u0], quant(__uint_as_float(r.y), qs));
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) net.tile_fill[t] = 0;
    if (t == 0 && threadIdx.x < kTileGroups) net.sq[threadIdx.x] = 0;
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
    const unsigned long long seed = P.seed;
    const uint32_t key0 = (uint32_t)seed, key1 = (uint32_t)(seed >> 32);
    const uint32_t tag = (1u << 24) | (P.net_id & 0xFFFFFFu);
    const uint32_t local = i - P.id_base; // neuron index within its own network
    uint32_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;
    unsigned long long cur_blk = ~0ull;

    for (int s = s0; s < s1; s++) {
        const unsigned long long n = k * S + (unsigned long long)s;
        const unsigned long long blk = n >> 2;
        if (blk != cur_blk) {
            w0 = (uint32_t)blk;
            w1 = (uint32_t)(blk >> 32);
            w2 = local;
            w3 = tag;
            philox4x32_10(w0, w1, w2, w3, key0, key1);
            cur_blk = blk;
        }
        const uint32_t sel = (uint32_t)(n & 3ull);
        const uint32_t x = sel == 0 ? w0 : sel == 1 ? w1 : sel == 2 ? w2 : w3;
        // c = #{m < cmax : T_m <= x}; T is nondecreasing, so a binary search counts it
        uint32_t c = 0;
#pragma unroll
        for (uint32_t step = kMaxPoisson / 2; step > 0; step >>= 1) {
            const uint32_t probe = c + step;
            if (probe <= (uint32_t)cmax && s_T[probe - 1] <= x) c = probe;
        }

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

    // bin end: compact this block's spikes into its own staging slots (no global atomics
    // per wavefront); k_compact then places every block's spikes in the bin's dense list
    const bool spiked = active && sub != 0xFFu;
    const unsigned long long mask = __ballot(spiked);
    const uint32_t nw = (uint32_t)__popcll(mask);
    const uint32_t wid = threadIdx.x >> 6;
    if (lane_id() == 0) s_wcnt[wid] = nw;
    __syncthreads();
    uint32_t woff = 0, btot = 0;
    for (uint32_t w = 0; w < kNeuronBlock / 64; w++) {
        woff += (w < wid) ? s_wcnt[w] : 0u;
        btot += s_wcnt[w];
    }
    if (spiked) {
        const uint32_t rank = (uint32_t)__popcll(mask & ((1ull << lane_id()) - 1ull));
        net.stage[(size_t)blockIdx.x * kNeuronBlock + woff + rank] = (i << 4) | sub;
    }
    if (threadIdx.x == 0) {
        net.blk_cnt[blockIdx.x] = btot;
        if (btot) atomicAdd(&net.grp_cnt[(k & 1ull) * net.n_grp + (blockIdx.x >> 8)], btot);
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
    __syncthreads();
    for (uint32_t st = kNeuronBlock / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) s_red[threadIdx.x] += s_red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) net.blk_sig[blockIdx.x] = s_red[0];
}

// ------------------------------------------------------------------ compaction

// Group g of 256 neuron blocks: its offset in the bin's spike list is the sum of the
// counts of groups 0..g-1 (each block added its count to its group in k_neuron), the
// blocks' offsets inside the group come from a block-wide scan, and each thread copies
// one block's staged spikes. Group 0 also records the bin's spike count; every group
// clears its counter of the other bin parity for the next bin.
__global__ void __launch_bounds__(256) k_compact(DevNet net) {
    __shared__ uint32_t s_wave[4];
    __shared__ uint32_t s_part[256];
    const unsigned long long k = net.ctl->bin;
    const uint32_t par = (uint32_t)(k & 1ull);
    const uint32_t* gc = net.grp_cnt + (size_t)par * net.n_grp;
    const uint32_t g = blockIdx.x;
    // offset of this group and (for group 0) the bin total
    uint32_t before = 0, all = 0;
    for (uint32_t x = threadIdx.x; x < net.n_grp; x += blockDim.x) {
        const uint32_t v = gc[x];
        before += x < g ? v : 0u;
        all += v;
    }
    s_part[threadIdx.x] = before;
    __syncthreads();
    for (uint32_t st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) s_part[threadIdx.x] += s_part[threadIdx.x + st];
        __syncthreads();
    }
    const uint32_t goff = s_part[0];
    __syncthreads();
    if (g == 0) {
        s_part[threadIdx.x] = all;
        __syncthreads();
        for (uint32_t st = 128; st > 0; st >>= 1) {
            if (threadIdx.x < st) s_part[threadIdx.x] += s_part[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == 0) net.bin_cnt[k & net.MBmask] = s_part[0];
    }
    const uint32_t b = g * 256u + threadIdx.x;
    const uint32_t c = b < net.n_blocks ? net.blk_cnt[b] : 0u;
    // exclusive scan of the 256 block counts (4 wavefronts)
    const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6;
    uint32_t x = c;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= (uint32_t)o) x += y;
    }
    if (lane == 63u) s_wave[wid] = x;
    __syncthreads();
    uint32_t woff = 0;
    for (uint32_t w = 0; w < wid; w++) woff += s_wave[w];
    const unsigned long long base = net.bin_start[k & net.MBmask] + goff + woff + x - c;
    for (uint32_t r = 0; r < c; r++) net.rec[(base + r) & net.RCmask] = net.stage[(size_t)b * kNeuronBlock + r];
    if (threadIdx.x == 0) net.grp_cnt[(size_t)(par ^ 1u) * net.n_grp + g] = 0;
}


// ------------------------------------------------------------------ readout + close

// Level 1: workgroup (region r, group g) sums the block partials g*256 .. g*256+255 of
// region r in a fixed tree. The last workgroup to finish sums each region's level-1
// partials in ascending g (so the result does not depend on which workgroup is last),
// then closes the bin: advances the spike-history ring and the bin counter.
__global__ void __launch_bounds__(256) k_readout_close(DevNet net) {
    __shared__ double s[256];
    __shared__ uint32_t sc[256];
    __shared__ bool last;
    const unsigned long long k = net.ctl->bin;
    if (net.regions_on) {
        const uint32_t gid = blockIdx.x;
        const uint32_t r = net.l1_region[gid];
        const uint32_t b0 = net.reg_blk_ptr[r] + (gid - net.l1_ptr[r]) * 256u;
        const uint32_t b1 = min(b0 + 256u, net.reg_blk_ptr[r + 1]);
        const uint32_t b = b0 + threadIdx.x;
        s[threadIdx.x] = b < b1 ? net.blk_sig[net.reg_blk[b]] : 0.0;
        sc[threadIdx.x] = b < b1 ? net.blk_cnt[net.reg_blk[b]] : 0u;
        __syncthreads();
        for (uint32_t st = 128; st > 0; st >>= 1) {
            if (threadIdx.x < st) {
                s[threadIdx.x] += s[threadIdx.x + st];
                sc[threadIdx.x] += sc[threadIdx.x + st];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            net.l1_sig[gid] = s[0];
            net.l1_cnt[gid] = sc[0];
            __threadfence();
            last = atomicAdd(&net.ctl->done, 1u) == gridDim.x - 1;
        }
        __syncthreads();
        if (!last) return;
        __threadfence();
        for (uint32_t rr = threadIdx.x; rr < net.n_regions; rr += blockDim.x) {
            double a = 0.0;
            uint32_t c = 0;
            for (uint32_t g = net.l1_ptr[rr]; g < net.l1_ptr[rr + 1]; g++) {
                a += __hip_atomic_load(&net.l1_sig[g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                c += __hip_atomic_load(&net.l1_cnt[g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            const size_t o = (size_t)(k & net.MBmask) * net.n_regions + rr;
            net.sig[o] = net.reg_size[rr] ? a / (double)net.reg_size[rr] : 0.0;
            net.sig_cnt[o] = c;
        }
    }
    if (threadIdx.x == 0) {
        const uint32_t m = net.MBmask;
        const uint32_t c = net.bin_cnt[k & m];
        net.bin_start[(k + 1) & m] = net.bin_start[k & m] + c;
        net.bin_cnt[(k + 1) & m] = 0;
        net.ctl->spikes += c;
        net.ctl->done = 0;
        net.ctl->bin = k + 1;
    }
}

// ------------------------------------------------------------------ launchers

size_t gather_lds_bytes(const DevNet& n) { return ((size_t)1 << n.tile_bits) * n.U * 8u; }

hipError_t launch_scatter(const DevNet& n, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_scatter, dim3(grid), dim3(kScatterThreads), scatter_lds_bytes(n), st, n);
    return hipGetLastError();
}

hipError_t prepare_kernels() {
    hipError_t e = hipFuncSetAttribute((const void*)k_scatter, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)kMaxLdsBytes);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)k_gather<1>, hipFuncAttributeMaxDynamicSharedMemorySize,
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

hipError_t launch_compact(const DevNet& n, hipStream_t st) {
    hipLaunchKernelGGL(k_compact, dim3(n.n_grp), dim3(256), 0, st, n);
    return hipGetLastError();
}

hipError_t launch_readout_close(const DevNet& n, hipStream_t st) {
    hipLaunchKernelGGL(k_readout_close, dim3(n.regions_on ? n.n_l1 : 1u), dim3(256), 0, st, n);
    return hipGetLastError();
}

} // namespace dbs
