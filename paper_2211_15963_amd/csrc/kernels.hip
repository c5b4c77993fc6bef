// kernels.hip - gfx950 kernels of one spike bin.
//
// Per bin k (S Euler steps of dt, SI Section 3):
//   k_part     fan-in of the arrivals due at the start of bin k: every spike j of
//              bin k-d (d = 1..D) contributes its delay-d edges (Suppl. Algorithm 2
//              pushes a spike list through destination lists; here the delay ring
//              is read backwards, so all events of a bin land in one accumulator).
//              Whole delay segments are read (contiguous 12-byte edge records) and
//              their events are radix-partitioned through LDS into at most 64
//              super-tile streams, with one global reservation per non-empty bucket
//              per round instead of one atomic per event. Launched twice per bin:
//              delays 2..D of bin k+1 while bin k's neurons are stepped (side
//              stream), delay 1 at the start of bin k+1.
//              After each workgroup's first chunk the chunks come from a counter.
//   k_bucket   second pass: each super-tile stream is partitioned into its tiles
//              the same way, in rounds handed out by a counter; the next round's
//              records are copied global -> LDS directly (no registers) while the
//              current round is reserved and written.
//   k_gather   one workgroup per tile: sums its events in LDS as int64 fixed
//              point (exact, so any order gives the same bits), converts once
//              to float, writes A.
//   k_fan, k_gather_blk  the single-pass form (on request): the partition goes
//              straight into per-workgroup blocks of every tile through carry
//              buffers in LDS, and the gather reads the tile's blocks.
//   k_neuron   one lane per neuron, S substeps fused in registers: Philox
//              Poisson background, Euler update of V (CV equation), threshold,
//              reset and refractory clamp, receptor decay (eq. 3); at the bin
//              end, wavefront-ballot compaction of the spike list and the
//              per-block region partial sums.
//   k_compact  places every block's staged spikes in the bin's dense spike list.
//   k_region_partials, k_readout_close  per-region mean synaptic current and spike
//              count (fixed-order tree over groups of 256 block partials, then the
//              groups in order), the region BOLD step (Extended Data Table 4), and the
//              bin close (bin counter, spike ring).
//
// All float arithmetic is single IEEE operations in a fixed order (the file
// is built with -ffp-contract=off and f32 denormals preserved) so the result
// equals a scalar CPU evaluation of the same expressions.
#include "dbsim_internal.hpp"

namespace dbs {

namespace {

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Exclusive prefix sum over a workgroup of NT threads (NT <= 1024); *total receives the block
// sum. s_wave holds NT / 64 words.
template <int NT = kScatterThreads>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* s_wave, uint32_t* total) {
    const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6;
    constexpr uint32_t nw = NT >> 6;
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

// ------------------------------------------------------------------ fan-in partition

namespace {

// exclusive scan of v[0..n) in place (n <= 2 * kScatterThreads), returns the total
__device__ uint32_t block_scan_inplace(uint32_t* v, uint32_t n, uint32_t* s_wave) {
    const uint32_t t = threadIdx.x;
    const uint32_t a = 2 * t < n ? v[2 * t] : 0u, b = 2 * t + 1 < n ? v[2 * t + 1] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(a + b, s_wave, &tot);
    if (2 * t < n) v[2 * t] = ex;
    if (2 * t + 1 < n) v[2 * t + 1] = ex + a;
    return tot;
}

// bump allocator over the dynamic LDS (host and device compute the same offsets)
struct LdsLayout {
    size_t off = 0;
    __host__ __device__ size_t take(size_t bytes, size_t align) {
        off = (off + align - 1) & ~(align - 1);
        const size_t o = off;
        off += bytes;
        return o;
    }
};

// one partition round: the round's events sorted by bucket, per-bucket counts,
// sorted starts and reserved output positions
struct RoundLayout {
    size_t gbase, s_w, s_key, hist, lstart, s_wave;
    __host__ __device__ void place(LdsLayout& L, uint32_t nb, uint32_t RE) {
        gbase = L.take(8 * (size_t)nb, 8);
        s_w = L.take(8 * (size_t)RE, 8);
        s_key = L.take(4 * (size_t)RE, 4);
        hist = L.take(4 * (size_t)nb, 4);
        lstart = L.take(4 * (size_t)nb, 4);
        s_wave = L.take(4 * 20, 4);
    }
};

struct PartLayout {
    size_t dpre, dstart, sstart, spre, dcnt, smap, total;
    RoundLayout r;
    __host__ __device__ PartLayout(uint32_t nb, uint32_t RE, uint32_t D) {
        LdsLayout L;
        dpre = L.take(8 * ((size_t)D + 1), 8);
        dstart = L.take(8 * (size_t)D, 8);
        sstart = L.take(8 * kScatterSegs, 8);
        r.place(L, nb, RE);
        spre = L.take(4 * (kScatterSegs + 4), 4);
        dcnt = L.take(4 * ((size_t)D + 1), 4);
        smap = L.take(2 * (kScatterSegs + 2), 2);
        total = L.take(0, 16);
    }
};

struct BucketLayout {
    size_t stage, cpre, sbase, ccnt, fill, total;
    RoundLayout r;
    __host__ __device__ BucketLayout(uint32_t nb, uint32_t RE) {
        LdsLayout L;
        stage = L.take(16 * (size_t)RE, 16);
        cpre = L.take(8 * (kMaxSuperTiles + 2), 8);
        sbase = L.take(8 * (kMaxSuperTiles + 2), 8);
        ccnt = L.take(4 * (kMaxSuperTiles + 2), 4);
        fill = L.take(4 * (kMaxSuperTiles + 2), 4);
        r.place(L, nb, RE);
        total = L.take(0, 16);
    }
};

struct Round {
    unsigned long long* gbase; // reserved output position of each bucket (~0 on overflow)
    float2* s_w;               // the round's weights, sorted by bucket
    uint32_t* s_key;           // the round's keys (target | source class << 31), sorted by bucket
    uint32_t* hist;            // events per bucket
    uint32_t* lstart;          // first sorted position of each bucket
    uint32_t* s_wave;
    __device__ void at(unsigned char* base, const RoundLayout& l) {
        gbase = reinterpret_cast<unsigned long long*>(base + l.gbase);
        s_w = reinterpret_cast<float2*>(base + l.s_w);
        s_key = reinterpret_cast<uint32_t*>(base + l.s_key);
        hist = reinterpret_cast<uint32_t*>(base + l.hist);
        lstart = reinterpret_cast<uint32_t*>(base + l.lstart);
        s_wave = reinterpret_cast<uint32_t*>(base + l.s_wave);
    }
};

// the events of one thread in one round, held in registers from the load to the placement
struct Batch {
    uint32_t key[kMaxBatch];
    float2 w[kMaxBatch];
    uint32_t br[kMaxBatch]; // bucket << 16 | rank within the bucket
};

// Direct global -> LDS copy of records (12 bytes each; an 8-byte record brings the next
// record's first word along, which is never used): one instruction per wavefront moves 64
// records into 64 consecutive 16-byte LDS slots (lane l lands at byte 16 l) without passing
// through registers. The copy is counted like a vector load of the issuing wavefront; it has
// landed after that wavefront's next wait for all its vector memory operations (dma_wait),
// so every read of the slots follows dma_wait and a barrier. The compiler builtin sets the
// wave-uniform LDS base itself (the slots of one instruction start at a wave-uniform address).
__device__ __forceinline__ void dma_records64(const uint32_t* g, uint4* lds) {
    __builtin_amdgcn_global_load_lds((__attribute__((address_space(1))) void*)g,
                                     (__attribute__((address_space(3))) void*)lds, 12, 0, 0);
}

__device__ __forceinline__ void dma_wait() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Wavefronts w0 .. of the block copy records src[first + e], e < ne, into stage[e] (64 per
// instruction; the lanes past ne repeat the last record, so every access stays in the round).
template <int KW>
__device__ __forceinline__ void dma_round(const uint32_t* src, unsigned long long first, uint32_t ne, uint4* stage,
                                          uint32_t w0) {
    const uint32_t w = threadIdx.x >> 6, nw = kScatterThreads >> 6, l = threadIdx.x & 63u;
    const uint32_t nch = (ne + 63u) >> 6;
    for (uint32_t c = w - w0; c < nch; c += nw - w0) {
        const uint32_t e = min(c * 64u + l, ne - 1u);
        dma_records64(src + (first + e) * (1u + KW), stage + (size_t)c * 64u);
    }
}

// The same for narrow stream records: per instruction pair, 128 records' weights (16 bytes
// per lane, lane l at byte 16 l) and keys (4 bytes per lane, lane l at byte 4 l). The round
// starts at an even record, so every copy is aligned; lanes past ne repeat the last pair,
// which lies inside the slice (slices start even, so the record after an odd count does).
__device__ __forceinline__ void dma_round_narrow(const DevNet& net, unsigned long long first, uint32_t ne,
                                                 uint2* stage_w, uint16_t* stage_k, uint32_t w0) {
    const uint32_t w = threadIdx.x >> 6, nw = kScatterThreads >> 6, l = threadIdx.x & 63u;
    const uint32_t nch = (ne + 127u) >> 7;
    const uint32_t last = (ne - 1u) & ~1u;
    for (uint32_t c = w - w0; c < nch; c += nw - w0) {
        const uint32_t e = min(c * 128u + 2u * l, last);
        __builtin_amdgcn_global_load_lds((__attribute__((address_space(1))) void*)(net.sevw + first + e),
                                         (__attribute__((address_space(3))) void*)(stage_w + (size_t)c * 128u), 16, 0,
                                         0);
        __builtin_amdgcn_global_load_lds((__attribute__((address_space(1))) void*)(net.sevk + first + e),
                                         (__attribute__((address_space(3))) void*)(stage_k + (size_t)c * 128u), 4, 0,
                                         0);
    }
}

__device__ __forceinline__ uint32_t bucket_of(const DevNet& net, uint32_t key, uint32_t nb, uint32_t b0, uint32_t bshift) {
    const uint32_t b = ((key & 0x7FFFFFFFu) >> bshift) - b0;
    return b < nb ? b : 0u;
}

// counts an event in its bucket; returns bucket << 16 | its rank among the bucket's events
__device__ __forceinline__ uint32_t rank_event(const DevNet& net, Round& R, uint32_t key, uint32_t nb, uint32_t b0,
                                               uint32_t bshift) {
    uint32_t b = ((key & 0x7FFFFFFFu) >> bshift) - b0;
    if (b >= nb) { // cannot happen for a consistent table
        atomicOr(&net.ctl->err, kErrLayout);
        b = 0;
    }
    return (b << 16) | atomicAdd(&R.hist[b], 1u);
}

// moves this thread's events of the round to their sorted LDS positions
__device__ __forceinline__ void place_batch(Round& R, const Batch& B, uint32_t ne, uint32_t nbt) {
#pragma unroll
    for (int u = 0; u < kMaxBatch; u++) {
        const uint32_t e = u * kScatterThreads + threadIdx.x;
        if (u < (int)nbt && e < ne) {
            const uint32_t pos = R.lstart[B.br[u] >> 16] + (B.br[u] & 0xFFFFu);
            R.s_key[pos] = B.key[u];
            R.s_w[pos] = B.w[u];
        }
    }
}

template <int KW>
__device__ __forceinline__ void store_record(uint32_t* out, unsigned long long pos, uint32_t key, float2 w) {
    if (KW == 2)
        reinterpret_cast<uint3*>(out)[pos] = make_uint3(key, __float_as_uint(w.x), __float_as_uint(w.y));
    else
        reinterpret_cast<uint2*>(out)[pos] = make_uint2(key, __float_as_uint(w.x));
}

constexpr unsigned long long kSpillRun = ~1ull; // gbase of a run whose slice is full

// Runs (unbuffered): one reservation per non-empty bucket in out_fill (slice of bucket b:
// out_base[b0+b] .. out_base[b0+b+1]); sets gbase and the sorted starts. A slice holds a
// share of the events its bucket can receive in a pass (super-tile streams) or a bin (tile
// arena): a run that does not fit is marked kSpillRun and counted in *marked, and the
// slice's valid records end at the first such reservation, kept as the largest ~base in
// out_fill[nlim + b0 + b] (the reservations that fit are exactly those before it, since
// the fill only grows). Returns whether a run of the round was marked (on every thread).
__device__ bool reserve_runs(const DevNet& net, Round& R, uint32_t nb, uint32_t b0, const uint64_t* out_base,
                             uint32_t* out_fill, uint32_t nlim, unsigned long long* marked) {
    int spilled = 0;
    for (uint32_t t = threadIdx.x; t < nb; t += kScatterThreads) {
        const uint32_t h = R.hist[t];
        unsigned long long gb = ~0ull;
        if (h) {
            const uint32_t base = atomicAdd(&out_fill[b0 + t], h);
            const unsigned long long s0 = out_base[b0 + t];
            if ((unsigned long long)base + h <= out_base[b0 + t + 1] - s0) {
                gb = s0 + base;
            } else {
                atomicMax(&out_fill[nlim + b0 + t], ~base);
                atomicAdd(marked, (unsigned long long)h);
                gb = kSpillRun;
                spilled = 1;
            }
        }
        R.gbase[t] = gb;
        R.lstart[t] = h;
    }
    const bool any = __syncthreads_or(spilled) != 0;
    block_scan_inplace(R.lstart, nb, R.s_wave);
    __syncthreads();
    return any;
}

// An event past its tile's arena slice: its fixed-point weights are added to the target's
// per-receptor sums in ovf (one atomic each; exact in any order), which the tile's gather
// adds to the slice's sums.
template <int KW>
__device__ void overflow_event(const DevNet& net, uint32_t tgt, uint32_t inh, float2 w) {
    unsigned long long* o = net.ovf + (size_t)tgt * (2 * KW) + (inh ? KW : 0);
    atomicAdd(o, quant(w.x, net.qscale));
    if (KW == 2) atomicAdd(o + 1, quant(w.y, net.qscale));
}

// An event whose super-tile stream was full goes straight to its tile's arena slice, with
// one atomic for its place (the bucketing of the stream's records reserves after it), or,
// if that is full too, to the overflow sums. Returns whether it overflowed.
template <int KW>
__device__ bool spill_event(const DevNet& net, uint32_t key, float2 w) {
    const uint32_t tgt = key & 0x7FFFFFFFu, t = tgt >> net.tile_bits;
    const uint32_t slot = atomicAdd(&net.tile_fill[t], 1u);
    const unsigned long long s0 = net.tile_base[t];
    if (slot < net.tile_base[t + 1] - s0) {
        const unsigned long long pos = s0 + slot;
        net.evk[pos] = (uint16_t)((tgt & ((1u << net.tile_bits) - 1u)) | ((key >> 31) << 15));
        if (KW == 2) reinterpret_cast<float2*>(net.ev)[pos] = w;
        else reinterpret_cast<float*>(net.ev)[pos] = w.x;
        return false;
    }
    atomicMax(&net.tile_fill[net.T + t], ~slot);
    overflow_event<KW>(net, tgt, key >> 31, w);
    return true;
}

// consecutive threads write consecutive records of a bucket's run (SPILL: some runs of the
// round are marked and go to the tile arena instead)
template <int KW, bool SPILL>
__device__ void write_runs(const DevNet& net, Round& R, uint32_t ne, uint32_t nb, uint32_t b0, uint32_t bshift,
                           uint32_t* out) {
    uint32_t nov = 0;
    for (uint32_t q = threadIdx.x; q < ne; q += kScatterThreads) {
        const uint32_t key = R.s_key[q];
        const uint32_t b = bucket_of(net, key, nb, b0, bshift);
        const unsigned long long gb = R.gbase[b];
        if (SPILL && gb == kSpillRun) nov += spill_event<KW>(net, key, R.s_w[q]) ? 1u : 0u;
        else if (gb != ~0ull) store_record<KW>(out, gb + (q - R.lstart[b]), key, R.s_w[q]);
    }
    if (SPILL && nov) atomicAdd(&net.ctl->overflow, (unsigned long long)nov);
    __syncthreads();
}

// Narrow stream records: the key within the super-tile (17 bits at most) as a 16-bit key
// beside the weight pair, whose sign bits (free: every weight is non-negative) carry the
// source class (w0) and the key's bit 16 (w1).
template <bool SPILL>
__device__ void write_runs_narrow(const DevNet& net, Round& R, uint32_t ne, uint32_t nb, uint32_t bshift) {
    const uint32_t smask = (1u << (net.tile_bits + net.ts_bits)) - 1u;
    uint32_t nov = 0;
    for (uint32_t q = threadIdx.x; q < ne; q += kScatterThreads) {
        const uint32_t key = R.s_key[q];
        const uint32_t b = bucket_of(net, key, nb, 0, bshift);
        const unsigned long long gb = R.gbase[b];
        if (SPILL && gb == kSpillRun) {
            nov += spill_event<2>(net, key, R.s_w[q]) ? 1u : 0u;
        } else if (gb != ~0ull) {
            const unsigned long long pos = gb + (q - R.lstart[b]);
            const uint32_t loc = key & smask;
            const float2 w = R.s_w[q];
            net.sevk[pos] = (uint16_t)loc;
            net.sevw[pos] = make_uint2(__float_as_uint(w.x) | (key & 0x80000000u), __float_as_uint(w.y) | ((loc >> 16) << 31));
        }
    }
    if (SPILL && nov) atomicAdd(&net.ctl->overflow, (unsigned long long)nov);
    __syncthreads();
}

// The tile arena's records: a 16-bit key (target within the tile | inhibitory source << 15)
// in evk beside the weights in ev, consecutive threads writing consecutive records of a run.
// SPILL: some runs of the round are marked; their events go to the overflow sums (target =
// tbase + the key's target field: the super-tile's first neuron for the narrow stream keys).
template <int KW, bool SPILL>
__device__ void write_runs_arena(const DevNet& net, Round& R, uint32_t ne, uint32_t nb, uint32_t b0, uint32_t tbase) {
    const uint32_t lmask = (1u << net.tile_bits) - 1u;
    for (uint32_t q = threadIdx.x; q < ne; q += kScatterThreads) {
        const uint32_t key = R.s_key[q];
        const uint32_t b = bucket_of(net, key, nb, b0, net.tile_bits);
        const unsigned long long gb = R.gbase[b];
        if (SPILL && gb == kSpillRun) {
            overflow_event<KW>(net, tbase + (key & 0x7FFFFFFFu), key >> 31, R.s_w[q]);
        } else if (gb != ~0ull) {
            const unsigned long long pos = gb + (q - R.lstart[b]);
            net.evk[pos] = (uint16_t)((key & lmask) | ((key >> 31) << 15));
            if (KW == 2) reinterpret_cast<float2*>(net.ev)[pos] = R.s_w[q];
            else reinterpret_cast<float*>(net.ev)[pos] = R.s_w[q].x;
        }
    }
    __syncthreads();
}

} // namespace

// The fan-in of the arrivals due at the start of bin k: the delay-d segments of the rows of
// every neuron that spiked in bin k-d, d = 1..D. Workgroups take chunks of these segments
// (read whole, so the table reads are contiguous) and process them in rounds of up to
// round_events events: each thread loads its events into registers, ranks them by bucket
// with LDS counters, the round is placed in LDS sorted by bucket and written out.
// The buckets are the super-tile streams (runs), re-bucketed by k_bucket.
template <int KW>
__global__ void __launch_bounds__(kScatterThreads) k_part(DevNet net, uint32_t d_lo, uint32_t d_hi, uint32_t ahead) {
    extern __shared__ __align__(16) unsigned char dyn[];
    const uint32_t D = net.D, RE = net.round_events;
    const uint32_t nb = net.NS;
    const PartLayout L(nb, RE, D);
    unsigned long long* s_dpre = reinterpret_cast<unsigned long long*>(dyn + L.dpre);
    unsigned long long* s_dstart = reinterpret_cast<unsigned long long*>(dyn + L.dstart);
    unsigned long long* s_sstart = reinterpret_cast<unsigned long long*>(dyn + L.sstart);
    uint32_t* s_spre = reinterpret_cast<uint32_t*>(dyn + L.spre);
    Round R;
    R.at(dyn, L.r);

    uint32_t* s_dcnt = reinterpret_cast<uint32_t*>(dyn + L.dcnt);
    uint16_t* s_map = reinterpret_cast<uint16_t*>(dyn + L.smap);
    // the bin whose arrivals are assembled: the current one, or (ahead = 1, while the
    // current bin's neurons are still being stepped) the next one
    const unsigned long long k = net.ctl->bin + ahead;
    const uint32_t tid = threadIdx.x;
    // spike lists of bins k-d for the delays d_lo <= d <= d_hi (one thread per delay),
    // then their prefix over all D delays (the other delays contribute nothing)
    for (uint32_t x = tid; x < D; x += kScatterThreads) {
        const uint32_t d = x + 1;
        uint32_t cnt = 0;
        unsigned long long st = 0;
        if (k >= d && d >= d_lo && d <= d_hi) {
            const uint32_t b = (uint32_t)((k - d) & net.MBmask);
            st = net.bin_start[b];
            cnt = net.bin_cnt[b];
        }
        s_dstart[x] = st;
        s_dcnt[x] = cnt;
    }
    __syncthreads();
    for (uint32_t x = tid; x <= D; x += kScatterThreads) {
        unsigned long long tot = 0;
        for (uint32_t y = 0; y < x; y++) tot += s_dcnt[y];
        s_dpre[x] = tot;
    }
    __syncthreads();
    const unsigned long long total = s_dpre[D];
    if (total == 0) return;
    // segments per chunk: about chunks_per_wg chunks per workgroup (one for the small
    // delay-1 pass, where a chunk's fixed cost weighs most), at most kScatterSegs
    const uint32_t G = gridDim.x;
    const unsigned long long cw = (unsigned long long)(ahead ? net.chunks_per_wg : 1u) * G;
    const uint32_t spc = (uint32_t)min((unsigned long long)kScatterSegs, max(32ull, (total + cw - 1) / cw));
    const unsigned long long nchunks = (total + spc - 1) / spc;
    const uint32_t bshift = net.tile_bits + net.ts_bits;
    unsigned long long my_events = 0;
    // the first chunk of every workgroup is fixed, the others are handed out through a
    // counter (a workgroup that starts late, behind another kernel's workgroups, takes
    // fewer); the next one is claimed while this one is read
    __shared__ unsigned long long s_pc;
    // this thread's segment of a chunk: the spiking neuron j, then its row header (row start,
    // bit 63: inhibitory source; the delay segment offsets). For the next chunk both are
    // fetched during the current chunk's first two rounds (pf: 1 neuron, 2 header too)
    uint32_t pf = 0, pf_d = 0, pf_j = 0, pf_so = 0, pf_eo = 0;
    uint2 pf_rs = make_uint2(0u, 0u);
    unsigned long long pf_c = ~0ull;
    auto fetch_id = [&](unsigned long long cn) {
        pf = 0;
        pf_c = cn;
        const unsigned long long in0 = cn * spc;
        if (cn < nchunks && tid < min((unsigned long long)spc, total - in0)) {
            const unsigned long long it = in0 + tid;
            uint32_t lo = 0, hi = D;
            while (hi - lo > 1u) {
                const uint32_t mid = (lo + hi) >> 1;
                if (s_dpre[mid] <= it) lo = mid;
                else hi = mid;
            }
            pf_d = lo + 1;
            pf_j = net.rec[(s_dstart[lo] + (it - s_dpre[lo])) & net.RCmask] >> 4;
            pf = 1;
        }
    };
    auto fetch_hdr = [&]() {
        if (pf == 1) {
            const uint32_t* hp = net.hdr + (size_t)pf_j * net.HW;
            pf_rs = *reinterpret_cast<const uint2*>(hp);
            pf_so = hp[1 + pf_d];
            pf_eo = hp[2 + pf_d];
            pf = 2;
        }
    };
    unsigned long long c = blockIdx.x;
    while (c < nchunks) {
        const unsigned long long i0 = c * spc;
        const uint32_t nseg = (uint32_t)min((unsigned long long)spc, total - i0);
        uint32_t len = 0;
        if (pf_c != c) fetch_id(c);
        fetch_hdr();
        if (tid < nseg) {
            s_sstart[tid] = (((unsigned long long)(pf_rs.y & 0x7FFFFFFFu) << 32) | pf_rs.x) + pf_so;
            len = pf_eo - pf_so;
        }
        pf_c = ~0ull;
        uint32_t ec;
        const uint32_t ex = block_exclusive_scan(len, R.s_wave, &ec);
        s_spre[tid] = ex;
        if (tid == 0) s_spre[kScatterSegs] = ec;
        // coarse map: the segment holding event m << mb_bits, for the at most
        // kScatterSegs blocks of 2^mb_bits events of the chunk
        uint32_t mb_bits = 0;
        while (((ec + (1u << mb_bits) - 1) >> mb_bits) > (uint32_t)kScatterSegs) mb_bits++;
        if (len) {
            const uint32_t m0 = (ex + (1u << mb_bits) - 1) >> mb_bits;
            const uint32_t m1 = (ex + len + (1u << mb_bits) - 1) >> mb_bits;
            for (uint32_t m = m0; m < m1; m++) s_map[m] = (uint16_t)tid;
        }
        const uint32_t nmap = (ec + (1u << mb_bits) - 1) >> mb_bits;
        __syncthreads();
        // a round's loads: all of them issued before any is used (latency cover); the segment
        // of each event is found from the coarse map, independently per event
        Batch B;
        auto load_round = [&](uint32_t ra) {
            const uint32_t na = min(RE, ec - ra);
            const uint32_t nba = (na + kScatterThreads - 1) / kScatterThreads;
#pragma unroll
            for (int u = 0; u < kMaxBatch; u++) {
                if (u < (int)nba) {
                    const uint32_t ge = ra + min(u * kScatterThreads + tid, na - 1);
                    const uint32_t m = ge >> mb_bits;
                    const uint32_t lo = s_map[m], hi = m + 1 < nmap ? s_map[m + 1] : nseg - 1;
                    const uint32_t sg = lo + seg_search(s_spre + lo, hi - lo + 1, ge);
                    const unsigned long long edge = s_sstart[sg] + (ge - s_spre[sg]);
                    if (KW == 2) { // weights, then target | source class << 31
                        const uint3 r = reinterpret_cast<const uint3*>(net.edge)[edge];
                        B.key[u] = r.z;
                        B.w[u] = make_float2(__uint_as_float(r.x), __uint_as_float(r.y));
                    } else {
                        const uint2 r = reinterpret_cast<const uint2*>(net.edge)[edge];
                        B.key[u] = r.y;
                        B.w[u] = make_float2(__uint_as_float(r.x), 0.0f);
                    }
                }
            }
        };
        if (ec) load_round(0);
        for (uint32_t r0 = 0; r0 < ec; r0 += RE) {
            const uint32_t ne = min(RE, ec - r0);
            const uint32_t nbt = (ne + kScatterThreads - 1) / kScatterThreads;
            for (uint32_t t = tid; t < nb; t += kScatterThreads) R.hist[t] = 0;
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kMaxBatch; u++)
                if (u < (int)nbt && u * kScatterThreads + tid < ne) B.br[u] = rank_event(net, R, B.key[u], nb, 0, bshift);
            __syncthreads();
            // the next chunk is claimed in the first round, alongside wavefront 0's
            // reservations (one wait for both)
            unsigned long long claim = 0;
            if (tid == 0 && r0 == 0) claim = atomicAdd(&net.ctl->pnext, 1ull);
            const bool spill = reserve_runs(net, R, nb, 0, net.st_base, net.st_fill, net.NS, &net.ctl->spilled);
            place_batch(R, B, ne, nbt);
            if (tid == 0 && r0 == 0) s_pc = G + claim; // read by every thread at the end of the chunk
            __syncthreads();
            // this round's events are in LDS: the next round's loads go out now and land
            // while the runs are written, and with them the next chunk's segment lookups
            if (r0 + RE < ec) load_round(r0 + RE);
            if (r0 == 0) fetch_id(s_pc);
            else if (r0 == RE) fetch_hdr();
            if (KW == 2 && net.narrow) {
                if (spill) write_runs_narrow<true>(net, R, ne, nb, bshift);
                else write_runs_narrow<false>(net, R, ne, nb, bshift);
            } else {
                if (spill) write_runs<KW, true>(net, R, ne, nb, 0, bshift, net.sev);
                else write_runs<KW, false>(net, R, ne, nb, 0, bshift, net.sev);
            }
        }
        if (ec == 0) { // no round: claim here
            if (tid == 0) s_pc = G + atomicAdd(&net.ctl->pnext, 1ull);
            __syncthreads();
        }
        my_events += ec;
        c = s_pc;
    }
    // events count as delivered when their bin's arrivals are consumed (the gather moves
    // the ahead count over)
    if (tid == 0 && my_events) atomicAdd(ahead ? &net.ctl->ahead_events : &net.ctl->edge_events, my_events);
    // the chunk counter is reset by the next kernel of the stream (k_bucket, k_gather or the
    // bin close): no grid-wide completion count, whose same-address atomics cost tens of us
}

// Records in super-tile stream st: the reservations that fit its slice (the others went
// to the tile arena directly), which end at the first one that did not.
__device__ __forceinline__ uint32_t stream_fill(const DevNet& net, uint32_t st) {
    const uint32_t lim = net.st_fill[net.NS + st];
    const uint32_t f = lim ? min(net.st_fill[st], ~lim) : net.st_fill[st];
    return (uint32_t)min((unsigned long long)f, net.st_base[st + 1] - net.st_base[st]);
}

// Second pass when the tiles are too many for the carry buffers: each super-tile stream is
// cut into rounds of contiguous records, which are partitioned into the super-tile's tiles.
template <int KW>
__global__ void __launch_bounds__(kScatterThreads) k_bucket(DevNet net) {
    extern __shared__ __align__(16) unsigned char dyn[];
    const uint32_t RE = net.bucket_events, NS = net.NS, TS = 1u << net.ts_bits, G = gridDim.x;
    const BucketLayout L(TS, RE);
    uint4* stage = reinterpret_cast<uint4*>(dyn + L.stage);
    // narrow records: the weights, then the keys, in the same staging bytes
    const bool narrow = KW == 2 && net.narrow;
    uint2* stage_w = reinterpret_cast<uint2*>(dyn + L.stage);
    uint16_t* stage_k = reinterpret_cast<uint16_t*>(dyn + L.stage + 8 * (size_t)RE);
    unsigned long long* s_cpre = reinterpret_cast<unsigned long long*>(dyn + L.cpre);
    unsigned long long* s_sbase = reinterpret_cast<unsigned long long*>(dyn + L.sbase);
    Round R;
    R.at(dyn, L.r);
    uint32_t* s_ccnt = reinterpret_cast<uint32_t*>(dyn + L.ccnt);
    uint32_t* s_fill = reinterpret_cast<uint32_t*>(dyn + L.fill);
    const uint32_t tid = threadIdx.x;
    if (blockIdx.x == 0 && tid == 0) net.ctl->pnext = 0; // the partition pass has finished
    // records and rounds per stream (one thread per stream), then the rounds' prefix
    for (uint32_t st = tid; st < NS; st += kScatterThreads) {
        const uint32_t f = stream_fill(net, st);
        s_fill[st] = f;
        s_sbase[st] = net.st_base[st];
        s_ccnt[st] = (f + RE - 1) / RE;
    }
    __syncthreads();
    for (uint32_t st = tid; st <= NS; st += kScatterThreads) {
        unsigned long long tot = 0;
        for (uint32_t y = 0; y < st; y++) tot += s_ccnt[y];
        s_cpre[st] = tot;
    }
    __syncthreads();
    const unsigned long long nchunks = s_cpre[NS];
    // round c: stream, first record and size
    auto locate = [&](unsigned long long c, uint32_t& st, unsigned long long& r0, uint32_t& ne) {
        uint32_t lo = 0, hi = NS;
        while (hi - lo > 1u) {
            const uint32_t mid = (lo + hi) >> 1;
            if (s_cpre[mid] <= c) lo = mid;
            else hi = mid;
        }
        st = lo;
        r0 = (c - s_cpre[st]) * RE;
        ne = (uint32_t)min((unsigned long long)RE, s_fill[st] - r0);
    };
    // Rounds: the first two of every workgroup are fixed, the others are handed out through
    // a counter (a workgroup that starts late, behind another kernel's workgroups, takes
    // fewer), two ahead: while round c is processed, the records of the next round cn are
    // copied into the staging slots (free once c is ranked) and the round after it is claimed.
    __shared__ unsigned long long s_claim;
    unsigned long long c = blockIdx.x, cn = blockIdx.x + G;
    if (c < nchunks) {
        uint32_t st, ne;
        unsigned long long r0;
        locate(c, st, r0, ne);
        if (narrow) dma_round_narrow(net, s_sbase[st] + r0, ne, stage_w, stage_k, 0);
        else dma_round<KW>(net.sev, s_sbase[st] + r0, ne, stage, 0);
    }
    while (c < nchunks) {
        uint32_t st, ne;
        unsigned long long r0;
        locate(c, st, r0, ne);
        const uint32_t nbt = (ne + kScatterThreads - 1) / kScatterThreads;
        const uint32_t t0 = st * TS;
        const uint32_t nt = min(TS, net.T - t0);
        for (uint32_t t = tid; t < nt; t += kScatterThreads) R.hist[t] = 0;
        dma_wait();
        __syncthreads();
        Batch B;
#pragma unroll
        for (int u = 0; u < kMaxBatch; u++) {
            const uint32_t e = u * kScatterThreads + tid;
            if (u < (int)nbt && e < ne) {
                if (narrow) { // key within the super-tile, so the tiles count from 0
                    const uint2 wv = stage_w[e];
                    B.key[u] = (uint32_t)stage_k[e] | ((wv.y >> 31) << 16) | (wv.x & 0x80000000u);
                    B.w[u] = make_float2(__uint_as_float(wv.x & 0x7FFFFFFFu), __uint_as_float(wv.y & 0x7FFFFFFFu));
                    B.br[u] = rank_event(net, R, B.key[u], nt, 0, net.tile_bits);
                } else {
                    const uint4 q = stage[e];
                    B.key[u] = q.x;
                    B.w[u] = make_float2(__uint_as_float(q.y), KW == 2 ? __uint_as_float(q.z) : 0.0f);
                    B.br[u] = rank_event(net, R, B.key[u], nt, t0, net.tile_bits);
                }
            }
        }
        __syncthreads();
        if (cn < nchunks && tid >= 64u) { // wavefront 0 makes the reservations meanwhile
            uint32_t st2, ne2;
            unsigned long long r2;
            locate(cn, st2, r2, ne2);
            if (narrow) dma_round_narrow(net, s_sbase[st2] + r2, ne2, stage_w, stage_k, 1);
            else dma_round<KW>(net.sev, s_sbase[st2] + r2, ne2, stage, 1);
        }
        // the claim travels with wavefront 0's reservations (one wait for both)
        unsigned long long claim = 0;
        if (tid == 0 && cn < nchunks) claim = atomicAdd(&net.ctl->bnext, 1ull);
        const bool spill = reserve_runs(net, R, nt, t0, net.tile_base, net.tile_fill, net.T, &net.ctl->overflow);
        place_batch(R, B, ne, nbt);
        if (tid == 0) s_claim = cn < nchunks ? 2ull * G + claim : ~0ull;
        __syncthreads();
        const uint32_t tbase = narrow ? st << (net.tile_bits + net.ts_bits) : 0u;
        if (spill) write_runs_arena<KW, true>(net, R, ne, nt, narrow ? 0u : t0, tbase);
        else write_runs_arena<KW, false>(net, R, ne, nt, narrow ? 0u : t0, tbase);
        c = cn;
        cn = s_claim;
    }
    // the round counter and the stream fills are reset by the next kernel of the stream
    // (k_gather, the bin close, or the reset between two ahead passes)
}

// between two partition passes of one bin: empty streams and work-queue counters
__global__ void __launch_bounds__(256) k_pass_reset(DevNet net) {
    for (uint32_t x = threadIdx.x; x < 2 * net.NS; x += blockDim.x) net.st_fill[x] = 0;
    if (threadIdx.x == 0) {
        net.ctl->pnext = 0;
        net.ctl->bnext = 0;
    }
}

// ------------------------------------------------------------------ single-pass blocked fan-in

namespace {

template <int KW> struct WeightOf;
template <> struct WeightOf<1> { using type = float; };
template <> struct WeightOf<2> { using type = float2; };

// an edge record as loaded: the weights, then the key (target | inhibitory source << 31)
template <int KW> struct RecOf;
template <> struct RecOf<1> {
    using type = uint2;
    __device__ static uint32_t key(const uint2& r) { return r.y; }
    __device__ static float weights(const uint2& r) { return __uint_as_float(r.x); }
};
template <> struct RecOf<2> {
    using type = uint3;
    __device__ static uint32_t key(const uint3& r) { return r.z; }
    __device__ static float2 weights(const uint3& r) { return make_float2(__uint_as_float(r.x), __uint_as_float(r.y)); }
};

constexpr uint32_t kNoBlock = 0xFFFFFFFFu; // the workgroup holds no block of the tile
constexpr uint32_t kNoSpace = 0xFFFFFFFEu; // the tile's blocks ran out (kErrArena raised)

// LDS of k_fan: the delay lists, one chunk's segments (start, length) and its segment counter,
// and per tile a carry buffer of C records (16-bit key: target within the tile | inhibitory
// source << 15, and the weights), its claimed slots, the workgroup's current block of the tile
// and the records already in that block, and the list of tiles to move out.
struct FanLayout {
    size_t dpre, dstart, sstart, bufw, cnt, blk, slen, dcnt, wave, bufk, fill, flist, total;
    __host__ __device__ FanLayout(uint32_t T, uint32_t C, uint32_t KW, uint32_t D) {
        LdsLayout L;
        dpre = L.take(8 * ((size_t)D + 1), 8);
        dstart = L.take(8 * (size_t)D, 8);
        sstart = L.take(8 * (size_t)kFanThreads, 8);
        bufw = L.take(4 * (size_t)KW * C * T, 16);
        cnt = L.take(4 * (size_t)T, 4);
        blk = L.take(4 * (size_t)T, 4);
        slen = L.take(4 * (size_t)kFanThreads, 4);
        dcnt = L.take(4 * ((size_t)D + 1), 4);
        wave = L.take(4 * 32, 4);
        bufk = L.take(2 * (size_t)C * T, 16);
        fill = L.take(2 * (size_t)T, 2);
        flist = L.take(2 * (size_t)T, 2);
        total = L.take(0, 16);
    }
};

template <int KW>
struct Fan {
    using W = typename WeightOf<KW>::type;
    W* bufw;
    uint16_t* bufk;
    uint32_t* cnt;   // slots claimed in the carry buffer (claims beyond C wait for the next move)
    uint32_t* blk;   // current block (kNoBlock / kNoSpace)
    uint16_t* fill;  // records in the current block
    uint16_t* flist; // tiles to move out
    uint32_t* nfl;   // their number: three counters used in turn by the iterations, and a fourth
                     // for the final list
    __device__ void at(unsigned char* base, const FanLayout& l) {
        bufw = reinterpret_cast<W*>(base + l.bufw);
        bufk = reinterpret_cast<uint16_t*>(base + l.bufk);
        cnt = reinterpret_cast<uint32_t*>(base + l.cnt);
        blk = reinterpret_cast<uint32_t*>(base + l.blk);
        fill = reinterpret_cast<uint16_t*>(base + l.fill);
        flist = reinterpret_cast<uint16_t*>(base + l.flist);
        nfl = reinterpret_cast<uint32_t*>(base + l.wave) + 20;
    }
};

// Moves the carry buffers of the listed tiles into the workgroup's blocks: C records each
// (full buffers), or cnt[t] (the rest, at the end of a pass). One lane per tile: it takes a
// new block of the tile when the current one cannot hold them (the block left behind is full:
// its count is K), copies the records in 16-byte pieces (a full buffer starts at a multiple of
// C records in its block, so the pieces are aligned) and empties the buffer. Ends with a
// barrier.
template <int KW>
__device__ void fan_move(const DevNet& net, Fan<KW>& F, uint32_t nfl, bool full) {
    const uint32_t tid = threadIdx.x, C = net.fan_C, K = net.fan_K;
    for (uint32_t x = tid; x < nfl; x += kFanThreads) {
        const uint32_t t = F.flist[x];
        const uint32_t n = full ? C : F.cnt[t];
        uint32_t b = F.blk[t], f = F.fill[t];
        if (b == kNoBlock || (b != kNoSpace && f + n > K)) {
            if (b != kNoBlock) net.bcnt[b] = f;
            const uint32_t got = atomicAdd(&net.tile_fill[t], 1u);
            const unsigned long long b0 = net.tile_base[t];
            if (b0 + got < net.tile_base[t + 1]) {
                b = (uint32_t)(b0 + got);
            } else { // cannot happen: a tile's blocks cover its in-degree plus two part-filled
                     // blocks per workgroup and bin
                b = kNoSpace;
                atomicOr(&net.ctl->err, kErrArena);
            }
            f = 0;
        }
        F.blk[t] = b;
        F.fill[t] = (uint16_t)(f + n);
        if (b < kNoSpace) {
            const size_t pos = (size_t)b * K + f;
            if (full) { // C records: keys 2C bytes (C / 4 pieces of 8), weights 4 KW C bytes
                const uint2* sk = reinterpret_cast<const uint2*>(F.bufk + (size_t)t * C);
                uint2* dk = reinterpret_cast<uint2*>(net.evk + pos);
                for (uint32_t q = 0; q < C / 4u; q++) dk[q] = sk[q];
                const uint4* sw = reinterpret_cast<const uint4*>(F.bufw + (size_t)t * C);
                uint4* dw = reinterpret_cast<uint4*>(reinterpret_cast<typename WeightOf<KW>::type*>(net.ev) + pos);
                for (uint32_t q = 0; q < C * KW / 4u; q++) dw[q] = sw[q];
            } else {
                for (uint32_t q = 0; q < n; q++) {
                    net.evk[pos + q] = F.bufk[t * C + q];
                    reinterpret_cast<typename WeightOf<KW>::type*>(net.ev)[pos + q] = F.bufw[t * C + q];
                }
            }
        }
        // claims past C belong to events still held in registers, which claim again
        F.cnt[t] = 0u;
    }
    __syncthreads();
}

} // namespace

// Single-pass fan-in (the tiles fit the LDS carry buffers). A chunk is up to kFanThreads
// (spike, delay) segments (one row-header read each); every wavefront takes whole segments
// from the chunk's counter and fills each of its kMaxBatch register slots with up to 64
// consecutive records of its current segment (one per lane: coalesced loads, no search). Every
// held event claims a slot in the carry buffer of its target tile (one LDS counter); a full
// buffer is moved out as C contiguous records into a block of K records that the workgroup
// took from the tile's block range (one global claim per block, not per event). An event that
// finds its buffer full stays in its slot and claims again in the next iteration; a slot is
// refilled when it is free in every lane of the wavefront, and the loads are issued right after
// the claims, so they are in flight while the full buffers are moved. At the end every
// part-filled buffer is moved and every block the workgroup holds gets its record count, so
// k_gather_blk reads each tile's blocks in full.
template <int KW>
__global__ void __launch_bounds__(kFanThreads) k_fan(DevNet net, uint32_t d_lo, uint32_t d_hi, uint32_t ahead) {
    extern __shared__ __align__(16) unsigned char dyn[];
    const uint32_t D = net.D, T = net.T, C = net.fan_C;
    const FanLayout L(T, C, KW, D);
    unsigned long long* s_dpre = reinterpret_cast<unsigned long long*>(dyn + L.dpre);
    unsigned long long* s_dstart = reinterpret_cast<unsigned long long*>(dyn + L.dstart);
    unsigned long long* s_sstart = reinterpret_cast<unsigned long long*>(dyn + L.sstart);
    uint32_t* s_slen = reinterpret_cast<uint32_t*>(dyn + L.slen);
    uint32_t* s_dcnt = reinterpret_cast<uint32_t*>(dyn + L.dcnt);
    uint32_t* s_wave = reinterpret_cast<uint32_t*>(dyn + L.wave);
    uint32_t* s_flag = s_wave + 24; // three vote words, used in turn
    uint32_t* s_segnext = s_wave + 28; // next segment of the chunk to hand to a wavefront
    Fan<KW> F;
    F.at(dyn, L);
    const unsigned long long k = net.ctl->bin + ahead;
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    for (uint32_t x = tid; x < D; x += kFanThreads) {
        const uint32_t d = x + 1;
        uint32_t cnt = 0;
        unsigned long long st = 0;
        if (k >= d && d >= d_lo && d <= d_hi) {
            const uint32_t b = (uint32_t)((k - d) & net.MBmask);
            st = net.bin_start[b];
            cnt = net.bin_cnt[b];
        }
        s_dstart[x] = st;
        s_dcnt[x] = cnt;
    }
    __syncthreads();
    for (uint32_t x = tid; x <= D; x += kFanThreads) {
        unsigned long long tot = 0;
        for (uint32_t y = 0; y < x; y++) tot += s_dcnt[y];
        s_dpre[x] = tot;
    }
    __syncthreads();
    const unsigned long long total = s_dpre[D];
    if (total == 0) return;
    for (uint32_t t = tid; t < T; t += kFanThreads) {
        F.cnt[t] = 0u;
        F.blk[t] = kNoBlock;
        F.fill[t] = 0;
    }
    if (tid == 0)
        for (int x = 0; x < 4; x++) F.nfl[x] = s_flag[x] = 0u;
    const uint32_t G = gridDim.x;
    const unsigned long long cw = (unsigned long long)(ahead ? net.chunks_per_wg : 1u) * G;
    const uint32_t spc = (uint32_t)min((unsigned long long)kFanThreads, max(32ull, (total + cw - 1) / cw));
    const unsigned long long nchunks = (total + spc - 1) / spc;
    const uint32_t tb = net.tile_bits, lmask = (1u << tb) - 1u;
    const uint32_t nslots = max(1u, min((uint32_t)kMaxBatch, net.round_events / kFanThreads));
    unsigned long long my_events = 0;
    __shared__ unsigned long long s_pc;
    // the current chunk (uniform); this wavefront's current segment (wave-uniform)
    unsigned long long c = blockIdx.x;
    uint32_t nseg = 0;
    bool have = false;
    unsigned long long seg_base = 0;
    uint32_t seg_left = 0;
    // Reads the row headers of chunk c's segments and claims the next chunk; every thread's
    // loads of the previous chunk have been issued before this.
    auto setup_chunk = [&]() {
        __syncthreads();
        have = c < nchunks;
        if (!have) return;
        const unsigned long long i0 = c * spc;
        nseg = (uint32_t)min((unsigned long long)spc, total - i0);
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
            const uint32_t* hp = net.hdr + (size_t)j * net.HW;
            const uint2 rs = *reinterpret_cast<const uint2*>(hp);
            const uint32_t so = hp[1 + d], eo = hp[2 + d];
            s_sstart[tid] = (((unsigned long long)(rs.y & 0x7FFFFFFFu) << 32) | rs.x) + so;
            len = eo - so;
            s_slen[tid] = len;
        }
        uint32_t ec;
        (void)block_exclusive_scan<kFanThreads>(len, s_wave, &ec);
        if (tid == 0) {
            *s_segnext = 0u;
            s_pc = G + atomicAdd(&net.ctl->pnext, 1ull);
        }
        __syncthreads();
        c = s_pc;
        seg_left = 0;
        my_events += ec;
    };
    // The held events: their edge index and the record as loaded (weights, then target |
    // class << 31). Every slot is reloaded in every iteration, unconditionally (a held event
    // reads its own record again, an empty slot any valid one), so the loads land straight in
    // the slots' registers and are first waited for by the next iteration's claims.
    using Rec = typename RecOf<KW>::type;
    Rec rec[kMaxBatch];
    unsigned long long eidx[kMaxBatch];
    uint32_t pend = 0u;
#pragma unroll
    for (int u = 0; u < kMaxBatch; u++) {
        rec[u] = Rec{};
        eidx[u] = 0ull;
    }
    setup_chunk();
    for (uint32_t it = 0;; it++) {
        uint32_t* nfl_it = &F.nfl[it % 3u]; // list counter of this iteration
        // claims of the events held (loaded in the previous iteration, or waiting for a buffer)
#pragma unroll
        for (int u = 0; u < kMaxBatch; u++) {
            if (pend & (1u << u)) {
                const uint32_t key = RecOf<KW>::key(rec[u]), tgt = key & 0x7FFFFFFFu;
                const uint32_t t = tgt >> tb;
                if (t >= T) { // cannot happen for a consistent table
                    atomicOr(&net.ctl->err, kErrLayout);
                    pend &= ~(1u << u);
                    continue;
                }
                const uint32_t slot = atomicAdd(&F.cnt[t], 1u);
                if (slot < C) {
                    F.bufk[t * C + slot] = (uint16_t)((tgt & lmask) | ((key >> 31) << 15));
                    F.bufw[t * C + slot] = RecOf<KW>::weights(rec[u]);
                    if (slot == C - 1u) F.flist[atomicAdd(nfl_it, 1u)] = (uint16_t)t;
                    pend &= ~(1u << u);
                }
            }
        }
        // refill the slots that are free in the whole wavefront with up to 64 consecutive
        // records of the wavefront's current segment (taking whole segments from the chunk)
        if (have) {
#pragma unroll
            for (int u = 0; u < kMaxBatch; u++) {
                if (u < (int)nslots && __ballot((pend >> u) & 1u) == 0ull) {
                    while (seg_left == 0u) { // the next nonempty segment of the chunk, if any
                        uint32_t sg = 0;
                        if (lane == 0) sg = atomicAdd(s_segnext, 1u);
                        sg = __shfl(sg, 0, 64);
                        if (sg >= nseg) break;
                        seg_base = s_sstart[sg];
                        seg_left = s_slen[sg];
                    }
                    if (seg_left) {
                        const uint32_t n = min(64u, seg_left);
                        if (lane < n) {
                            eidx[u] = seg_base + lane;
                            pend |= 1u << u;
                        }
                        seg_base += n;
                        seg_left -= n;
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kMaxBatch; u++) rec[u] = reinterpret_cast<const Rec*>(net.edge)[eidx[u]];
        // vote: 1 = this chunk may still hold events to load, 2 = events held. The vote words
        // and list counters are used in turn by three iterations: read after this barrier, the
        // ones for two iterations ahead are cleared here (their last readers passed the
        // previous barrier, their next writers start after the next one)
        const bool more = have && (seg_left != 0u || *s_segnext < nseg);
        const uint32_t vote = (more ? 1u : 0u) | (pend ? 2u : 0u);
        if (vote) atomicOr(&s_flag[it % 3u], vote);
        __syncthreads();
        const uint32_t fl = s_flag[it % 3u], nfl = *nfl_it;
        if (tid == 0) s_flag[(it + 2u) % 3u] = F.nfl[(it + 2u) % 3u] = 0u;
        if (nfl) fan_move<KW>(net, F, nfl, true);
        if (!(fl & 1u)) {
            if (have) setup_chunk(); // every event of this chunk is loaded: the next chunk
            if (!have && !(fl & 2u)) break;
        }
    }
    // the part-filled buffers (listed with the fourth counter), then the record count of every
    // block held
    __syncthreads();
    for (uint32_t t = tid; t < T; t += kFanThreads)
        if (F.cnt[t]) F.flist[atomicAdd(&F.nfl[3], 1u)] = (uint16_t)t;
    __syncthreads();
    const uint32_t nfl = F.nfl[3];
    if (nfl) fan_move<KW>(net, F, nfl, false);
    for (uint32_t t = tid; t < T; t += kFanThreads) {
        const uint32_t b = F.blk[t];
        if (b < kNoSpace) net.bcnt[b] = F.fill[t];
    }
    if (tid == 0 && my_events) atomicAdd(ahead ? &net.ctl->ahead_events : &net.ctl->edge_events, my_events);
    // the chunk counter is reset by the next kernel of the stream (the gather or the bin close)
}

size_t fan_lds_bytes(uint32_t T, uint32_t C, uint32_t KW, uint32_t D) { return FanLayout(T, C, KW, D).total; }

size_t part_lds_bytes(uint32_t nb, uint32_t RE, uint32_t D) { return PartLayout(nb, RE, D).total; }

size_t bucket_lds_bytes(uint32_t TS, uint32_t RE) { return BucketLayout(TS, RE).total; }

// ------------------------------------------------------------------ gather

template <int KW>
__global__ void __launch_bounds__(kGatherThreads) k_gather(DevNet net) {
    extern __shared__ __align__(16) unsigned long long acc[];
    constexpr uint32_t U = 2 * KW;
    const uint32_t t = blockIdx.x;
    const uint32_t i0 = t << net.tile_bits;
    const uint32_t nt = min(1u << net.tile_bits, net.N - i0);
    for (uint32_t x = threadIdx.x; x < nt * U; x += blockDim.x) acc[x] = 0ull;
    __syncthreads();
    const unsigned long long b0 = net.tile_base[t];
    // the slice's records: the reservations before the first that did not fit (lim != 0),
    // whose events and all after it were summed in ovf
    const uint32_t lim = net.tile_fill[net.T + t];
    const uint32_t f = lim ? min(net.tile_fill[t], ~lim) : net.tile_fill[t];
    const uint32_t cnt = (uint32_t)min((unsigned long long)f, net.tile_base[t + 1] - b0);
    const double qs = net.qscale;
    const uint16_t* kk = net.evk + b0;
    for (uint32_t eb = 0; eb < cnt; eb += kLoadBatch * blockDim.x) {
        // load a batch of records first (latency cover), then accumulate them
        uint32_t key[kLoadBatch];
        float2 w[kLoadBatch];
#pragma unroll
        for (int u = 0; u < kLoadBatch; u++) {
            // clamped, so the loads are unconditional (no branch between them)
            const uint32_t e = min(eb + u * blockDim.x + threadIdx.x, cnt - 1);
            key[u] = kk[e];
            if (KW == 2) w[u] = reinterpret_cast<const float2*>(net.ev)[b0 + e];
            else w[u] = make_float2(reinterpret_cast<const float*>(net.ev)[b0 + e], 0.0f);
        }
#pragma unroll
        for (int u = 0; u < kLoadBatch; u++) {
            const uint32_t e = eb + u * blockDim.x + threadIdx.x;
            if (e < cnt) {
                const uint32_t lt = key[u] & 0x7FFFu;
                const uint32_t u0 = (key[u] >> 15) ? (uint32_t)KW : 0u;
                atomicAdd(&acc[lt * U + u0], quant(w[u].x, qs));
                if (KW == 2) atomicAdd(&acc[lt * U + u0 + 1], quant(w[u].y, qs));
            }
        }
    }
    __syncthreads();
    if (lim) { // the overflow sums of the tile's targets, cleared for the next bin
        unsigned long long* o = net.ovf + (size_t)i0 * U;
        for (uint32_t x = threadIdx.x; x < nt * U; x += blockDim.x) {
            acc[x] += o[x];
            o[x] = 0ull;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        net.tile_fill[t] = 0;
        net.tile_fill[net.T + t] = 0;
    }
    // the super-tile streams are empty again: this bin's delay-1 records are in the tile
    // arena, and the next bin's delay >= 2 records start from the front (the bin close
    // clears them again after those have been bucketed)
    if (t == 0)
        for (uint32_t x = threadIdx.x; x < 2 * net.NS; x += blockDim.x) net.st_fill[x] = 0;
    // this bin's events assembled ahead are delivered now (no partition of the next bin
    // runs before the gather has finished)
    if (t == 0 && threadIdx.x == 0) {
        net.ctl->edge_events += net.ctl->ahead_events;
        net.ctl->ahead_events = 0;
        net.ctl->pnext = 0; // work-queue counters of the partition kernels
        net.ctl->bnext = 0;
    }
    const float qinv = net.qinv;
    for (uint32_t x = threadIdx.x; x < nt; x += blockDim.x) {
#pragma unroll
        for (uint32_t u = 0; u < U; u++)
            net.A[(size_t)u * net.N + i0 + x] = (float)(long long)acc[x * U + u] * qinv;
    }
}

// Gather of the single-pass form: one workgroup per tile reads the tile's blocks (record
// counts first, in batches of up to kGatherThreads blocks whose prefix, with a coarse map of
// every 2^m-th record, locates every record in one or two LDS probes), sums them in LDS as
// int64 fixed point, converts once, writes A.
template <int KW>
__global__ void __launch_bounds__(kGatherThreads) k_gather_blk(DevNet net) {
    using W = typename WeightOf<KW>::type;
    extern __shared__ __align__(16) unsigned long long acc[];
    __shared__ uint32_t s_pre[kGatherThreads];
    __shared__ uint16_t s_map[kGatherThreads + 2];
    __shared__ uint32_t s_wave[kGatherThreads / 64];
    constexpr uint32_t U = 2 * KW;
    const uint32_t t = blockIdx.x, tid = threadIdx.x;
    const uint32_t i0 = t << net.tile_bits;
    const uint32_t nt = min(1u << net.tile_bits, net.N - i0);
    const uint32_t lmask = (1u << net.tile_bits) - 1u;
    for (uint32_t x = tid; x < nt * U; x += kGatherThreads) acc[x] = 0ull;
    const unsigned long long b0 = net.tile_base[t];
    const uint32_t nb = (uint32_t)min((unsigned long long)net.tile_fill[t], net.tile_base[t + 1] - b0);
    const uint32_t K = net.fan_K;
    const double qs = net.qscale;
    const uint16_t* evk = net.evk;
    const W* evw = reinterpret_cast<const W*>(net.ev);
    for (uint32_t bb = 0; bb < nb; bb += kGatherThreads) {
        const uint32_t nbb = min(kGatherThreads, nb - bb);
        const uint32_t cnt = tid < nbb ? min(net.bcnt[b0 + bb + tid], K) : 0u;
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan<kGatherThreads>(cnt, s_wave, &tot);
        s_pre[tid] = ex;
        uint32_t mb = 0;
        while (((tot + (1u << mb) - 1) >> mb) > (uint32_t)kGatherThreads) mb++;
        if (cnt) {
            const uint32_t m0 = (ex + (1u << mb) - 1) >> mb, m1 = (ex + cnt + (1u << mb) - 1) >> mb;
            for (uint32_t m = m0; m < m1; m++) s_map[m] = (uint16_t)tid;
        }
        const uint32_t nmap = (tot + (1u << mb) - 1) >> mb;
        __syncthreads();
        const size_t base = (size_t)(b0 + bb) * K;
        for (uint32_t e0 = 0; e0 < tot; e0 += kLoadBatch * kGatherThreads) {
            uint32_t kk[kLoadBatch];
            W ww[kLoadBatch];
#pragma unroll
            for (int u = 0; u < kLoadBatch; u++) { // clamped: every load is issued, none branches
                const uint32_t e = min(e0 + u * kGatherThreads + tid, tot - 1);
                const uint32_t m = e >> mb;
                const uint32_t lo = s_map[m], hi = m + 1 < nmap ? s_map[m + 1] : nbb - 1;
                const uint32_t j = lo + seg_search(s_pre + lo, hi - lo + 1, e);
                const size_t pos = base + (size_t)j * K + (e - s_pre[j]);
                kk[u] = evk[pos];
                ww[u] = evw[pos];
            }
#pragma unroll
            for (int u = 0; u < kLoadBatch; u++) {
                if (e0 + u * kGatherThreads + tid < tot) {
                    const uint32_t lt = kk[u] & lmask;
                    const uint32_t u0 = (kk[u] >> 15) ? (uint32_t)KW : 0u;
                    if constexpr (KW == 2) {
                        atomicAdd(&acc[lt * U + u0], quant(ww[u].x, qs));
                        atomicAdd(&acc[lt * U + u0 + 1], quant(ww[u].y, qs));
                    } else {
                        atomicAdd(&acc[lt * U + u0], quant(ww[u], qs));
                    }
                }
            }
        }
        __syncthreads(); // s_pre is rewritten by the next batch
    }
    __syncthreads();
    if (tid == 0) net.tile_fill[t] = 0;
    if (t == 0 && tid == 0) {
        net.ctl->edge_events += net.ctl->ahead_events;
        net.ctl->ahead_events = 0;
        net.ctl->pnext = 0;
        net.ctl->bnext = 0;
    }
    const float qinv = net.qinv;
    for (uint32_t x = tid; x < nt; x += kGatherThreads) {
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

    float V = 0.0f, J[U], A[U], Iou = 0.0f;
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
        if (P.ou_on) Iou = net.Iou[i];
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
    // the first Poisson thresholds in registers (uniform: the block's population)
    constexpr int kTr = 8;
    uint32_t Tr[kTr];
#pragma unroll
    for (int m = 0; m < kTr; m++) Tr[m] = m < cmax ? s_T[m] : 0u;
    const bool ou = P.ou_on != 0u; // uniform: neuron blocks never straddle populations
    const float ou_mu = P.ou_mu, ou_c1 = P.ou_c1, ou_c2 = P.ou_c2;
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
        // c = #{m < cmax : T_m <= x}. T is nondecreasing, so every lane's condition holds
        // for m below its count and fails above: a linear scan over m that stops at the first
        // threshold above the x of every lane of the wavefront counts exactly (the counts are
        // small, so it stops after a few thresholds)
        uint32_t c = 0;
        bool more = true;
#pragma unroll
        for (int m = 0; m < kTr; m++) {
            if (more && m < cmax) { // wavefront-uniform
                const bool ge = Tr[m] <= x;
                c += ge ? 1u : 0u;
                more = __any(ge);
            }
        }
        if (more)
            for (int m = kTr; m < cmax; m++) {
                const bool ge = s_T[m] <= x;
                if (!__any(ge)) break;
                c += ge ? 1u : 0u;
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
            if (ou) I = I + Iou;
            Vn = V + k_dt * I;
            if (Vn >= Vth) {
                Vn = Vr;
                ref = rsteps;
                sub = (uint32_t)s;
            }
        }
        V = Vn;
        if (ou) { // Ornstein-Uhlenbeck background current (eq. 1, discretised as eq. 4), old value above
            uint32_t y0 = (uint32_t)n, y1 = (uint32_t)(n >> 32), y2 = local, y3 = (3u << 24) | (P.net_id & 0xFFFFFFu);
            philox4x32_10(y0, y1, y2, y3, key0, key1);
            // twelve 10-bit uniforms; their standardised sum is the increment (exact integers)
            const uint32_t sum = (y0 & 1023u) + ((y0 >> 10) & 1023u) + ((y0 >> 20) & 1023u) + (y1 & 1023u) +
                                 ((y1 >> 10) & 1023u) + ((y1 >> 20) & 1023u) + (y2 & 1023u) + ((y2 >> 10) & 1023u) +
                                 ((y2 >> 20) & 1023u) + (y3 & 1023u) + ((y3 >> 10) & 1023u) + ((y3 >> 20) & 1023u);
            const float z = (float)((int)(2u * sum) - 12276) * 0x1p-11f;
            const float drift = ou_c1 * (ou_mu - Iou);
            const float Ih = Iou + drift;
            Iou = Ih + ou_c2 * z;
        }
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
        if (ou) net.Iou[i] = Iou;
        if (s1 < (int)S) net.pend[i] = (uint8_t)sub;
    }
    if (s1 < (int)S) return; // block-uniform: the bin continues in a later launch

    // initial spike injection (Methods): in the bins below inject_until the output train
    // of a neuron carries a spike with probability inject_t / 2^32 per bin (its own Philox
    // stream, word 0 of counter (k, local id, 2 << 24 | net_id)); the spike is delivered
    // like any other but does not reset the neuron; alone it is stamped at the bin's last step
    if (active && P.inject_t != 0u && k < net.ctl->inject_until && sub == 0xFFu) {
        uint32_t x0 = (uint32_t)k, x1 = (uint32_t)(k >> 32), x2 = local, x3 = (2u << 24) | (P.net_id & 0xFFFFFFu);
        philox4x32_10(x0, x1, x2, x3, key0, key1);
        if (x0 < P.inject_t) sub = S - 1;
    }
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


// ------------------------------------------------------------------ receptor currents

// The measurement step of Suppl. Algorithm 1 at the current state: per neuron block, the sum
// of each receptor's term g_u J_u (V_u - V) (float, the region signal's expression) in a fixed
// tree (double); then per population the sum of its blocks in ascending order, divided by its
// size. rblk [n_blocks][4] and rpop [n_pops][4] (paper receptor order) are device arrays.
template <int U>
__global__ void __launch_bounds__(kNeuronBlock) k_receptor_blocks(DevNet net, double* rblk) {
    __shared__ double s_red[U][kNeuronBlock];
    const uint2 bi = net.blk[blockIdx.x];
    const PopParams& P = net.pops[bi.y];
    const uint32_t i = bi.x + threadIdx.x;
    const bool active = i < P.end;
    const float V = active ? net.V[i] : 0.0f;
#pragma unroll
    for (int u = 0; u < U; u++) {
        const float t = active ? (P.g[u] * net.J[(size_t)u * net.N + i]) * (P.Vu[u] - V) : 0.0f;
        s_red[u][threadIdx.x] = active ? (double)t : 0.0;
    }
    __syncthreads();
    for (uint32_t st = kNeuronBlock / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st)
#pragma unroll
            for (int u = 0; u < U; u++) s_red[u][threadIdx.x] += s_red[u][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x < 4) {
        // paper order: AMPA, NMDA, GABA_A, GABA_B; with two receptors, AMPA and GABA_A
        const int u = U == 4 ? (int)threadIdx.x : (threadIdx.x == 0 ? 0 : threadIdx.x == 2 ? 1 : -1);
        rblk[(size_t)blockIdx.x * 4 + threadIdx.x] = u >= 0 ? s_red[u][0] : 0.0;
    }
}

__global__ void __launch_bounds__(256) k_receptor_pops(DevNet net, uint32_t n_pops, const double* rblk, double* rpop) {
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_pops) return;
    // blocks are laid out population by population: the first block of q and of q + 1
    auto first = [&](uint32_t pq) {
        uint32_t lo = 0, hi = net.n_blocks;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (net.blk[mid].y < pq) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    };
    const uint32_t b0 = first(q), b1 = first(q + 1);
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (uint32_t b = b0; b < b1; b++)
        for (int u = 0; u < 4; u++) s[u] += rblk[(size_t)b * 4 + u];
    const uint32_t n = b1 > b0 ? net.pops[q].end - net.blk[b0].x : 0u;
    for (int u = 0; u < 4; u++) rpop[(size_t)q * 4 + u] = n ? s[u] / (double)n : 0.0;
}

// ------------------------------------------------------------------ recording to host memory

// Copies the spike list of the bin being closed (compacted, not yet closed) into the pinned
// host ring at the same offsets (mod its size) and stores the bin's end offset. Runs on a
// second stream beside the rest of the bin; the host reads the ring after a synchronisation.
__global__ void __launch_bounds__(256) k_drain(DevNet net) {
    const unsigned long long k = net.ctl->bin;
    const uint32_t m = net.MBmask;
    const unsigned long long st = net.bin_start[k & m];
    const uint32_t c = net.bin_cnt[k & m];
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < c; x += gridDim.x * blockDim.x)
        net.hrec[(st + x) & net.HCmask] = net.rec[(st + x) & net.RCmask];
    if (blockIdx.x == 0 && threadIdx.x == 0) net.hbend[(k + 1) & net.HMBmask] = st + c;
}

// ------------------------------------------------------------------ readout + close

// Level 1: workgroup (region r, group g) sums the block partials g*256 .. g*256+255 of
// region r in a fixed tree. The last workgroup to finish sums each region's level-1
// partials in ascending g (so the result does not depend on which workgroup is last),
// then closes the bin: advances the spike-history ring and the bin counter.
// One explicit Euler step (h = one bin) of region r's Balloon-Windkessel model driven by
// the bin's spike count c, in the order of the equations of Extended Data Table 4 (all
// right-hand sides at the old state), and the BOLD sample when a TR is complete.
__device__ void bold_step(const DevNet& net, uint32_t r, uint32_t c) {
    const uint32_t R = net.n_regions;
    double* B = net.bold;
    const double z = net.bold_zs[r] * (double)c;
    const double s = B[r], f = B[R + r], v = B[2 * R + r], q = B[3 * R + r];
    const double h = net.bw_h, ht = net.bw_htau, rho = net.bw_rho;
    const double fout = pow(v, net.bw_inv_alpha);
    const double E = 1.0 - pow(1.0 - rho, 1.0 / f);
    const double s1 = s + h * (z - net.bw_kappa * s - net.bw_gamma * (f - 1.0));
    const double f1 = f + h * s;
    const double v1 = v + ht * (f - fout);
    const double q1 = q + ht * (f * E / rho - fout * q / v);
    B[r] = s1;
    B[R + r] = f1;
    B[2 * R + r] = v1;
    B[3 * R + r] = q1;
    const unsigned long long bb = net.bold_ctl[0] + 1; // bins stepped including this one
    if (bb % net.tr_bins == 0) {
        const unsigned long long m = bb / net.tr_bins - 1;
        const double y = net.bw_V0 * (net.bw_k1 * (1.0 - q1) + net.bw_k2 * (1.0 - q1 / v1) + net.bw_k3 * (1.0 - v1));
        net.bold_y[(size_t)(m & (kBoldRing - 1)) * R + r] = y;
    }
}

// Level 1 of the region readout: workgroup g sums up to 256 neuron blocks of one region
// (fixed tree).
__global__ void __launch_bounds__(256) k_region_partials(DevNet net) {
    __shared__ double s[256];
    __shared__ uint32_t sc[256];
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
    }
}

// Region sums over their level-1 partials in order, the BOLD step, and the bin close
// (one workgroup).
__global__ void __launch_bounds__(256) k_readout_close(DevNet net) {
    const unsigned long long k = net.ctl->bin;
    if (net.regions_on) {
        for (uint32_t rr = threadIdx.x; rr < net.n_regions; rr += blockDim.x) {
            // in group order; eight loads in flight at a time
            double a = 0.0;
            uint32_t c = 0;
            const uint32_t g0 = net.l1_ptr[rr], g1 = net.l1_ptr[rr + 1];
            uint32_t g = g0;
            for (; g + 8u <= g1; g += 8u) {
                double v[8];
                uint32_t w[8];
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    v[q] = net.l1_sig[g + q];
                    w[q] = net.l1_cnt[g + q];
                }
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    a += v[q];
                    c += w[q];
                }
            }
            for (; g < g1; g++) {
                a += net.l1_sig[g];
                c += net.l1_cnt[g];
            }
            const size_t o = (size_t)(k & net.MBmask) * net.n_regions + rr;
            net.sig[o] = net.reg_size[rr] ? a / (double)net.reg_size[rr] : 0.0;
            net.sig_cnt[o] = c;
            if (net.bold_on) bold_step(net, rr, c);
        }
        __syncthreads(); // every region has read the BOLD bin counter
        if (net.bold_on && threadIdx.x == 0) {
            const unsigned long long bb = net.bold_ctl[0] + 1;
            net.bold_ctl[0] = bb;
            if (bb % net.tr_bins == 0) net.bold_ctl[1] = bb / net.tr_bins;
        }
    }
    // the super-tile streams are empty again: the next bin's delay >= 2 records have been
    // bucketed before this kernel starts, its delay-1 records come next
    for (uint32_t x = threadIdx.x; x < 2 * net.NS; x += blockDim.x) net.st_fill[x] = 0;
    if (threadIdx.x == 0) {
        const uint32_t m = net.MBmask;
        const uint32_t c = net.bin_cnt[k & m];
        net.bin_start[(k + 1) & m] = net.bin_start[k & m] + c;
        net.bin_cnt[(k + 1) & m] = 0;
        net.ctl->spikes += c;
        net.ctl->pnext = 0;
        net.ctl->bnext = 0;
        net.ctl->bin = k + 1;
    }
}

// ------------------------------------------------------------------ launchers

size_t gather_lds_bytes(const DevNet& n) { return ((size_t)1 << n.tile_bits) * n.U * 8u; }


hipError_t prepare_kernels() {
    const void* big[] = {(const void*)k_part<1>, (const void*)k_part<2>, (const void*)k_bucket<1>,
                         (const void*)k_bucket<2>, (const void*)k_fan<1>, (const void*)k_fan<2>};
    hipError_t e = hipSuccess;
    for (const void* f : big) { // leave room for the kernels' few static LDS bytes
        e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kMaxLdsBytes - kStaticLds));
        if (e != hipSuccess) return e;
    }
    const void* gat[] = {(const void*)k_gather<1>, (const void*)k_gather<2>, (const void*)k_gather_blk<1>,
                         (const void*)k_gather_blk<2>};
    for (const void* f : gat) {
        e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kTileLdsBytes);
        if (e != hipSuccess) return e;
    }
    return e;
}

hipError_t launch_part(const DevNet& n, int grid, hipStream_t st, uint32_t d_lo, uint32_t d_hi, uint32_t ahead) {
    const size_t la = part_lds_bytes(n.NS, n.round_events, n.D);
    if (n.KW == 2)
        hipLaunchKernelGGL(k_part<2>, dim3(grid), dim3(kScatterThreads), la, st, n, d_lo, d_hi, ahead);
    else
        hipLaunchKernelGGL(k_part<1>, dim3(grid), dim3(kScatterThreads), la, st, n, d_lo, d_hi, ahead);
    return hipGetLastError();
}

hipError_t launch_bucket(const DevNet& n, int grid, hipStream_t st) {
    const size_t lb = bucket_lds_bytes(1u << n.ts_bits, n.bucket_events);
    if (n.KW == 2)
        hipLaunchKernelGGL(k_bucket<2>, dim3(grid), dim3(kScatterThreads), lb, st, n);
    else
        hipLaunchKernelGGL(k_bucket<1>, dim3(grid), dim3(kScatterThreads), lb, st, n);
    return hipGetLastError();
}

hipError_t launch_scatter(const DevNet& n, int grid, hipStream_t st, uint32_t d_lo, uint32_t d_hi, uint32_t ahead) {
    if (n.blocked) {
        const size_t lf = fan_lds_bytes(n.T, n.fan_C, n.KW, n.D);
        if (n.KW == 2)
            hipLaunchKernelGGL(k_fan<2>, dim3(grid), dim3(kFanThreads), lf, st, n, d_lo, d_hi, ahead);
        else
            hipLaunchKernelGGL(k_fan<1>, dim3(grid), dim3(kFanThreads), lf, st, n, d_lo, d_hi, ahead);
        return hipGetLastError();
    }
    hipError_t e = launch_part(n, grid, st, d_lo, d_hi, ahead);
    if (e != hipSuccess) return e;
    return launch_bucket(n, grid, st);
}

hipError_t launch_pass_reset(const DevNet& n, hipStream_t st) {
    hipLaunchKernelGGL(k_pass_reset, dim3(1), dim3(256), 0, st, n);
    return hipGetLastError();
}

hipError_t launch_gather(const DevNet& n, hipStream_t st) {
    if (n.blocked) {
        if (n.KW == 2)
            hipLaunchKernelGGL(k_gather_blk<2>, dim3(n.T), dim3(kGatherThreads), gather_lds_bytes(n), st, n);
        else
            hipLaunchKernelGGL(k_gather_blk<1>, dim3(n.T), dim3(kGatherThreads), gather_lds_bytes(n), st, n);
        return hipGetLastError();
    }
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

hipError_t launch_receptor_currents(const DevNet& n, uint32_t n_pops, double* rblk, double* rpop, hipStream_t st) {
    if (n.U == 4)
        hipLaunchKernelGGL(k_receptor_blocks<4>, dim3(n.n_blocks), dim3(kNeuronBlock), 0, st, n, rblk);
    else
        hipLaunchKernelGGL(k_receptor_blocks<2>, dim3(n.n_blocks), dim3(kNeuronBlock), 0, st, n, rblk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_receptor_pops, dim3((n_pops + 255) / 256), dim3(256), 0, st, n, n_pops, rblk, rpop);
    return hipGetLastError();
}

hipError_t launch_drain(const DevNet& n, hipStream_t st) {
    hipLaunchKernelGGL(k_drain, dim3(64), dim3(256), 0, st, n);
    return hipGetLastError();
}

hipError_t launch_readout_close(const DevNet& n, hipStream_t st) {
    if (n.regions_on) {
        hipLaunchKernelGGL(k_region_partials, dim3(n.n_l1), dim3(256), 0, st, n);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_readout_close, dim3(1), dim3(256), 0, st, n);
    return hipGetLastError();
}

} // namespace dbs
