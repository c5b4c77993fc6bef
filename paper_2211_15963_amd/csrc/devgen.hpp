// devgen.hpp - the seeded network generator's per-target step, as the device construction
// of the connection table runs it (one thread per target), also callable on the host.
//
// It draws exactly the network of the input generator (netgen/dbnet.c): for every target,
// fixed in-degree sampling without replacement (Floyd's algorithm over the candidate
// index space with the target itself removed), the sampled indices in ascending order
// mapped to source ids, weights and delays from the same counter-based hash of (seed,
// net_id, stream, target, projection, index). Only the weight distributions made of exact
// double arithmetic (uniform, constant) are covered; descriptions with lognormal weights,
// whose draws go through libm, are built on the host. Distance delays come from a
// per-(projection, source region, target region) table computed on the host with the
// generator's own formula.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dbs {

// one population of the handle (all members)
struct GenPop {
    uint64_t first;    // global id of its first neuron
    uint64_t off;      // member-local id of its first neuron
    uint32_t size;
    uint32_t exc;      // 1: excitatory source
    uint32_t member;
    uint32_t local;    // index within its member
    uint32_t region;   // member-local region
    uint32_t pad;
};

struct GenMember {
    uint64_t seed;
    uint64_t nbase;    // global id of its first neuron
    uint32_t net_id;
    uint32_t kw;       // weights per edge
    uint32_t n_pops;
    uint32_t n_regions;
    uint32_t proj0;    // its first projection in the handle's list
    uint32_t n_projs;
};

struct GenProj {
    int32_t dst_pop;   // member-local target population, -1 = every population
    uint32_t indegree;
    uint32_t w_dist;   // DBNET_W_UNIFORM or DBNET_W_CONST
    uint32_t d_mode;
    uint32_t d_min, d_max;
    float w_a, w_b, w_scale_exc, w_scale_inh;
    uint32_t dtab;     // distance mode: offset of its [n_regions][n_regions] delay table
    uint32_t cand0;    // first GenCand entry: one per member-local target population
};

// candidates of one (projection, target population)
struct GenCand {
    uint64_t M;        // candidate indices, the target itself excluded
    uint64_t self_base;// candidate index of the target population's first neuron (~0: none)
    uint32_t c0, nc;   // its candidate populations: GenCandPop entries c0 .. c0 + nc
};

struct GenCandPop {
    uint64_t end;      // one past its last candidate index
    uint64_t first;    // global id of its first neuron
    uint32_t size;
    uint32_t exc;
};

struct GenTables {
    const GenPop* pops;
    const GenMember* members;
    const GenProj* projs;
    const GenCand* cands;
    const GenCandPop* cpops;
    const uint8_t* dtab;
    uint32_t n_pops;   // all members
    uint32_t kmax;     // largest in-degree of one projection
    uint32_t hcap;     // hash-set slots per thread (power of two >= 2 kmax + 2)
    uint32_t scratch_words; // u32 words of scratch per thread
};

__host__ __device__ inline uint64_t gen_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// high 64 bits of a 64 x 64 product, from 32-bit halves
__host__ __device__ inline uint64_t gen_mulhi(uint64_t a, uint64_t b) {
    const uint64_t al = a & 0xFFFFFFFFull, ah = a >> 32, bl = b & 0xFFFFFFFFull, bh = b >> 32;
    const uint64_t ll = al * bl, lh = al * bh, hl = ah * bl, hh = ah * bh;
    const uint64_t mid = (ll >> 32) + (lh & 0xFFFFFFFFull) + (hl & 0xFFFFFFFFull);
    return hh + (lh >> 32) + (hl >> 32) + (mid >> 32);
}

__host__ __device__ inline uint64_t gen_stream_key(uint64_t seed, uint32_t net_id, uint32_t stream, uint32_t target) {
    const uint64_t h = gen_mix64(seed + 0x9E3779B97F4A7C15ULL * (uint64_t)(1u + stream));
    return gen_mix64(h ^ (((uint64_t)net_id << 32) | target));
}

__host__ __device__ inline uint64_t gen_draw(uint64_t key, uint32_t proj, uint64_t idx) {
    return gen_mix64(key ^ ((uint64_t)proj << 48) ^ idx);
}

__host__ __device__ inline double gen_u01(uint64_t h) { return (double)(h >> 11) * 0x1p-53; }

// uniform integer in [0, n) by multiply-high
__host__ __device__ inline uint64_t gen_below(uint64_t h, uint64_t n) { return gen_mulhi(h, n); }

// Global population of global neuron id i (binary search over the first ids).
__host__ __device__ inline uint32_t gen_pop_of(const GenTables& g, uint64_t i) {
    uint32_t lo = 0, hi = g.n_pops;
    while (hi - lo > 1u) {
        const uint32_t mid = (lo + hi) >> 1;
        if (g.pops[mid].first <= i) lo = mid;
        else hi = mid;
    }
    return lo;
}

// The in-edges of global target i in the generator's order: emit(src global id, source
// excitatory (1) or inhibitory (0), w0, w1, delay, projection index within the member).
// scratch: g.scratch_words u32 words of this thread's own (hash set, picked indices, bucket
// counts, sorted indices).
// Returns false if a candidate set is smaller than its in-degree (the description is then
// invalid; validation refuses it before).
template <class Emit>
__host__ __device__ bool gen_target(const GenTables& g, uint64_t i, uint32_t* scratch, Emit&& emit) {
    const uint32_t gq = gen_pop_of(g, i);
    const GenPop& T = g.pops[gq];
    const GenMember& mb = g.members[T.member];
    const uint32_t il = (uint32_t)(i - mb.nbase); // member-local target id
    enum { ST_SAMPLE = 1, ST_W0 = 2, ST_W1 = 3, ST_DELAY = 4 }; // the generator's stream numbers
    const uint64_t k_sample = gen_stream_key(mb.seed, mb.net_id, ST_SAMPLE, il);
    const uint64_t k_delay = gen_stream_key(mb.seed, mb.net_id, ST_DELAY, il);
    const uint64_t k_w0 = gen_stream_key(mb.seed, mb.net_id, ST_W0, il);
    const uint64_t k_w1 = gen_stream_key(mb.seed, mb.net_id, ST_W1, il);
    uint32_t* hash = scratch;               // hcap slots of (index + 1), 0 = empty
    uint32_t* picked = hash + g.hcap;       // kmax
    uint32_t* bucket = picked + g.kmax;     // kmax + 1
    uint32_t* sorted = bucket + g.kmax + 1; // kmax
    const uint32_t hmask = g.hcap - 1u;
    for (uint32_t j = 0; j < mb.n_projs; j++) {
        const GenProj& pr = g.projs[mb.proj0 + j];
        if ((pr.dst_pop >= 0 && (uint32_t)pr.dst_pop != T.local) || pr.indegree == 0) continue;
        const GenCand& C = g.cands[pr.cand0 + T.local];
        const uint64_t M = C.M;
        const uint32_t k = pr.indegree;
        if (M < k) return false;
        const uint64_t self_pos = C.self_base != ~0ull ? C.self_base + (il - T.off) : ~0ull;
        // Floyd's algorithm: k distinct indices uniform in [0, M) (indices < 2^28 fit u32)
        for (uint32_t x = 0; x <= hmask; x++) hash[x] = 0u;
        uint32_t np = 0;
        for (uint64_t t = M - k; t < M; t++) {
            const uint32_t r = (uint32_t)gen_below(gen_draw(k_sample, j, t), t + 1);
            uint32_t v = r, h = (uint32_t)(gen_mix64(r) & hmask);
            bool present = false;
            while (hash[h] != 0u) {
                if (hash[h] == r + 1u) {
                    present = true;
                    break;
                }
                h = (h + 1u) & hmask;
            }
            if (present) { // t itself is new: every earlier draw was below t
                v = (uint32_t)t;
                h = (uint32_t)(gen_mix64(t) & hmask);
                while (hash[h] != 0u) h = (h + 1u) & hmask;
            }
            hash[h] = v + 1u;
            picked[np++] = v;
        }
        // ascending order: counting by value range, then insertion within each range
        for (uint32_t a = 0; a <= k; a++) bucket[a] = 0u;
        const uint64_t scale = ~0ull / M;
        for (uint32_t a = 0; a < k; a++) bucket[gen_below((uint64_t)picked[a] * scale, k) + 1]++;
        for (uint32_t a = 0; a < k; a++) bucket[a + 1] += bucket[a];
        for (uint32_t a = 0; a < k; a++) sorted[bucket[gen_below((uint64_t)picked[a] * scale, k)]++] = picked[a];
        for (uint32_t a = 1; a < k; a++) {
            const uint32_t v = sorted[a];
            uint32_t b = a;
            while (b > 0 && sorted[b - 1] > v) {
                sorted[b] = sorted[b - 1];
                b--;
            }
            sorted[b] = v;
        }
        // indices -> source ids, then weights and delays in index order
        uint32_t c = 0;
        const GenCandPop* cp = g.cpops + C.c0;
        for (uint32_t a = 0; a < k; a++) {
            uint64_t x = sorted[a];
            if (x >= self_pos) x++;
            while (x >= cp[c].end) c++;
            const GenCandPop& Q = cp[c];
            const uint64_t s = Q.first + (x - (Q.end - Q.size));
            const double sc = Q.exc ? (double)pr.w_scale_exc : (double)pr.w_scale_inh;
            double d0, d1;
            if (pr.w_dist == 0u) { // uniform [a, b)
                d0 = (double)pr.w_a + ((double)pr.w_b - (double)pr.w_a) * gen_u01(gen_draw(k_w0, j, a));
                d1 = (double)pr.w_a + ((double)pr.w_b - (double)pr.w_a) * gen_u01(gen_draw(k_w1, j, a));
            } else { // constant
                d0 = (double)pr.w_a;
                d1 = (double)pr.w_a;
            }
            const float w0 = (float)(sc * d0);
            const float w1 = mb.kw == 2u ? (float)(sc * d1) : 0.0f;
            uint32_t dl;
            if (pr.d_mode == 0u) {
                dl = pr.d_min;
            } else if (pr.d_mode == 1u) {
                dl = pr.d_min + (uint32_t)gen_below(gen_draw(k_delay, j, a), pr.d_max - pr.d_min + 1);
            } else {
                const uint32_t sr = g.pops[gen_pop_of(g, s)].region;
                dl = g.dtab[pr.dtab + (size_t)sr * mb.n_regions + T.region];
            }
            emit(s, Q.exc, w0, w1, dl, j);
        }
    }
    return true;
}

// Device construction of the connection table (devbuild.hip): the generator's tables and
// the temporaries (in the handle's tile arena and super-tile streams, free before the first
// bin), and the table it writes.
struct DevBuild {
    GenTables g;
    uint32_t* scratch;            // batch * g.scratch_words u32
    uint32_t batch;               // targets per generation launch
    uint32_t* cnt;                // [N * D] edges per (source, delay)
    unsigned long long* cur;      // [N * D] placement cursors
    unsigned long long* rowlen;   // [N + 1]
    unsigned long long* rowptr;   // [N + 1]
    unsigned long long* sums;     // [N / 1024 + 2] block sums of the row scan
    uint8_t* tb;                  // [E] projection of every placed edge (order of equal targets)
    uint32_t* err;                // the handle's sticky error word (a failed check sets kErrBuild)
    uint32_t* edge;               // the edge records [E][1 + KW]
    uint32_t* hdr;                // the row headers [N][HW]
    uint64_t N, E;
    uint32_t D, HW, KW;
    double wlim;                  // |w| must stay below 2^(52 - F)
};
constexpr uint32_t kGenSortMax = 2048; // delay segments up to this length are ordered in LDS
// LDS bytes of the wavefront generator per wavefront (hash set and two index buffers); it
// runs where one wavefront's fit 64 KiB, else one thread per target with scratch
inline size_t gen_wave_lds(uint32_t kmax, uint32_t hcap) { return 4ull * (hcap + 2ull * kmax); }
constexpr size_t kGenWaveLds = 65536;
constexpr uint32_t kErrBuild = 4u;      // error-word bit: a consistency check of the construction failed

// Enqueues the whole construction on st; nothing is awaited. Checks that cannot fail for
// a validated description (delays in range, the edge total, no placement past a segment)
// set kErrBuild in the handle's error word, which the next synchronisation reports.
hipError_t launch_device_build(const DevBuild& b, hipStream_t st);

} // namespace dbs
