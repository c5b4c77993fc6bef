// devbuild.hip - construction of the connection table on the device.
//
// The same table the host construction builds (netbuild.cpp): rows by presynaptic neuron,
// delay segments in ascending delay, each segment sorted by target (equal targets, which
// only distinct projections can give, in projection order), records of (weights, target |
// inhibitory source << 31), and 64-byte row headers. Steps, all on the handle's stream:
//   k_gen_wave    one wavefront per target draws its in-edges (gen_target_wave: the
//                 generator's step spread over the lanes, its sets in LDS) and counts them
//                 per (source, delay); k_gen_count does the same with one thread per target
//                 and global scratch, in batches, where the LDS sets would not fit;
//   k_gen_rows    per source: delay-segment offsets within the row, row length;
//   k_scan_*      row starts (exclusive scan of the row lengths, 64-bit);
//   k_gen_cursors per source: row header (start | class bit), one cursor per segment;
//   k_gen_wave / k_gen_fill  the in-edges drawn again, each placed at its segment's cursor;
//   k_gen_sort    one wavefront per row orders every segment by (target, projection).
// The draws are counter-based, so the second generation repeats the first exactly.
#include <algorithm>

#include "dbsim_internal.hpp"
#include "devgen.hpp"

namespace dbs {

__global__ void __launch_bounds__(256) k_gen_clear(uint32_t* p, uint64_t n) {
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (uint64_t)gridDim.x * blockDim.x)
        p[x] = 0u;
}

__global__ void __launch_bounds__(256) k_gen_count(DevBuild b, uint64_t i0, uint64_t i1) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t i = i0 + t;
    if (i >= i1) return;
    uint32_t* sc = b.scratch + t * b.g.scratch_words;
    const uint32_t D = b.D;
    const uint64_t N = b.N;
    bool bad = false;
    const bool ok = gen_target(b.g, i, sc, [&](uint64_t s, uint32_t, float, float, uint32_t dl, uint32_t) {
        if (dl >= 1u && dl <= D && s < N) atomicAdd(&b.cnt[s * D + dl - 1], 1u);
        else bad = true;
    });
    if (bad || !ok) atomicOr(b.err, kErrBuild);
}

// Wavefront variant of the generator's per-target step (gen_target): the same draws and
// the same result, with the draws, the ordering and the mapping spread over the 64 lanes
// and the sampling loop, sequential by nature, on lane 0; the hash set and the index
// buffers live in this wavefront's LDS (hash: hcap words, pk and srt: kmax words each).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

template <class Emit>
__device__ bool gen_target_wave(const GenTables& g, uint64_t i, uint32_t* hash, uint32_t* pk, uint32_t* srt,
                                Emit&& emit) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t gq = gen_pop_of(g, i);
    const GenPop& T = g.pops[gq];
    const GenMember& mb = g.members[T.member];
    const uint32_t il = (uint32_t)(i - mb.nbase);
    enum { ST_SAMPLE = 1, ST_W0 = 2, ST_W1 = 3, ST_DELAY = 4 }; // the generator's stream numbers
    const uint64_t k_sample = gen_stream_key(mb.seed, mb.net_id, ST_SAMPLE, il);
    const uint64_t k_delay = gen_stream_key(mb.seed, mb.net_id, ST_DELAY, il);
    const uint64_t k_w0 = gen_stream_key(mb.seed, mb.net_id, ST_W0, il);
    const uint64_t k_w1 = gen_stream_key(mb.seed, mb.net_id, ST_W1, il);
    const uint32_t hmask = g.hcap - 1u;
    for (uint32_t j = 0; j < mb.n_projs; j++) {
        const GenProj& pr = g.projs[mb.proj0 + j];
        if ((pr.dst_pop >= 0 && (uint32_t)pr.dst_pop != T.local) || pr.indegree == 0) continue;
        const GenCand& C = g.cands[pr.cand0 + T.local];
        const uint64_t M = C.M;
        const uint32_t k = pr.indegree;
        if (M < k) return false;
        const uint64_t self_pos = C.self_base != ~0ull ? C.self_base + (il - T.off) : ~0ull;
        for (uint32_t x = lane; x <= hmask; x += 64) hash[x] = 0u;
        for (uint32_t a = lane; a < k; a += 64) {
            const uint64_t t = M - k + a;
            pk[a] = (uint32_t)gen_below(gen_draw(k_sample, j, t), t + 1);
        }
        wave_sync();
        if (lane == 0) { // Floyd's algorithm over the draws, in order
            for (uint32_t a = 0; a < k; a++) {
                const uint32_t t = (uint32_t)(M - k + a), r = pk[a];
                uint32_t h = (uint32_t)(gen_mix64(r) & hmask);
                bool present = false;
                while (hash[h] != 0u) {
                    if (hash[h] == r + 1u) {
                        present = true;
                        break;
                    }
                    h = (h + 1u) & hmask;
                }
                uint32_t v = r;
                if (present) {
                    v = t;
                    h = (uint32_t)(gen_mix64(t) & hmask);
                    while (hash[h] != 0u) h = (h + 1u) & hmask;
                }
                hash[h] = v + 1u;
                pk[a] = v;
            }
        }
        wave_sync();
        // ascending order: the indices are distinct, so each one's rank is its position
        for (uint32_t e = lane; e < k; e += 64) {
            const uint32_t v = pk[e];
            uint32_t rank = 0;
            for (uint32_t f = 0; f < k; f++) rank += pk[f] < v ? 1u : 0u;
            srt[rank] = v;
        }
        wave_sync();
        const GenCandPop* cp = g.cpops + C.c0;
        for (uint32_t a = lane; a < k; a += 64) {
            uint64_t x = srt[a];
            if (x >= self_pos) x++;
            uint32_t lo = 0, hi = C.nc - 1u; // first candidate population with end > x
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (cp[mid].end > x) hi = mid;
                else lo = mid + 1u;
            }
            const GenCandPop& Q = cp[lo];
            const uint64_t s = Q.first + (x - (Q.end - Q.size));
            const double sc = Q.exc ? (double)pr.w_scale_exc : (double)pr.w_scale_inh;
            double d0, d1;
            if (pr.w_dist == 0u) {
                d0 = (double)pr.w_a + ((double)pr.w_b - (double)pr.w_a) * gen_u01(gen_draw(k_w0, j, a));
                d1 = (double)pr.w_a + ((double)pr.w_b - (double)pr.w_a) * gen_u01(gen_draw(k_w1, j, a));
            } else {
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
        wave_sync(); // the buffers are reused by the next projection
    }
    return true;
}

// Counting (FILL = false) or placing (FILL = true) pass, one wavefront per target at a time.
template <bool FILL, int KW>
__global__ void __launch_bounds__(256) k_gen_wave(DevBuild b) {
    extern __shared__ uint32_t lds[];
    const uint32_t wpb = blockDim.x >> 6, w = threadIdx.x >> 6;
    const uint32_t per = b.g.hcap + 2u * b.g.kmax;
    uint32_t* hash = lds + (size_t)w * per;
    uint32_t* pk = hash + b.g.hcap;
    uint32_t* srt = pk + b.g.kmax;
    const uint32_t D = b.D;
    const uint64_t N = b.N, E = b.E;
    const double wlim = b.wlim;
    for (uint64_t i = (uint64_t)blockIdx.x * wpb + w; i < N; i += (uint64_t)gridDim.x * wpb) {
        bool bad = false;
        const bool ok = gen_target_wave(b.g, i, hash, pk, srt, [&](uint64_t s, uint32_t exc, float w0, float w1,
                                                                   uint32_t dl, uint32_t j) {
            if (!(dl >= 1u && dl <= D && s < N)) {
                bad = true;
                return;
            }
            if (!FILL) {
                atomicAdd(&b.cnt[s * D + dl - 1], 1u);
                return;
            }
            const unsigned long long pos = atomicAdd(&b.cur[s * D + dl - 1], 1ull);
            if (pos >= E) {
                bad = true;
                return;
            }
            const uint32_t key = (uint32_t)i | ((exc ? 0u : 1u) << 31);
            if (KW == 2)
                reinterpret_cast<uint3*>(b.edge)[pos] = make_uint3(__float_as_uint(w0), __float_as_uint(w1), key);
            else
                reinterpret_cast<uint2*>(b.edge)[pos] = make_uint2(__float_as_uint(w0), key);
            b.tb[pos] = (uint8_t)j;
            if (!(fabs((double)w0) < wlim) || !(fabs((double)w1) < wlim)) bad = true;
        });
        if (bad || !ok) atomicOr(b.err, kErrBuild);
    }
}

__global__ void __launch_bounds__(256) k_gen_rows(DevBuild b) {
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= b.N) return;
    uint32_t* hp = b.hdr + j * b.HW;
    unsigned long long acc = 0;
    hp[2] = 0u;
    for (uint32_t x = 0; x < b.D; x++) {
        acc += b.cnt[j * b.D + x];
        hp[3 + x] = (uint32_t)acc;
    }
    b.rowlen[j] = acc;
}

// exclusive scan of n 64-bit values, 1024 per block (256 threads x 4)
__device__ unsigned long long block_scan_u64(unsigned long long v, unsigned long long* sh, unsigned long long* total) {
    const uint32_t tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (uint32_t o = 1; o < blockDim.x; o <<= 1) {
        const unsigned long long y = tid >= o ? sh[tid - o] : 0ull;
        __syncthreads();
        sh[tid] += y;
        __syncthreads();
    }
    *total = sh[blockDim.x - 1];
    const unsigned long long r = sh[tid] - v;
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(256) k_scan_a(const unsigned long long* in, unsigned long long* out, uint64_t n,
                                                unsigned long long* sums) {
    __shared__ unsigned long long sh[256];
    const uint64_t base = (uint64_t)blockIdx.x * 1024 + 4ull * threadIdx.x;
    unsigned long long v[4], loc = 0;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        v[q] = base + q < n ? in[base + q] : 0ull;
        loc += v[q];
    }
    unsigned long long tot;
    unsigned long long ex = block_scan_u64(loc, sh, &tot);
#pragma unroll
    for (int q = 0; q < 4; q++) {
        if (base + q < n) out[base + q] = ex;
        ex += v[q];
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// one block: exclusive scan of the nb block sums in place, the total at sums[nb] (which
// must be the edge count E)
__global__ void __launch_bounds__(256) k_scan_b(unsigned long long* sums, uint64_t nb, uint64_t E, uint32_t* err) {
    __shared__ unsigned long long sh[256];
    unsigned long long carry = 0;
    for (uint64_t c0 = 0; c0 < nb; c0 += 256) {
        const uint64_t x = c0 + threadIdx.x;
        const unsigned long long v = x < nb ? sums[x] : 0ull;
        unsigned long long tot;
        const unsigned long long ex = block_scan_u64(v, sh, &tot);
        if (x < nb) sums[x] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        sums[nb] = carry;
        if (carry != E) atomicOr(err, kErrBuild);
    }
}

__global__ void __launch_bounds__(256) k_scan_c(unsigned long long* out, uint64_t n, const unsigned long long* sums) {
    const uint64_t base = (uint64_t)blockIdx.x * 1024 + 4ull * threadIdx.x;
    const unsigned long long add = sums[blockIdx.x];
#pragma unroll
    for (int q = 0; q < 4; q++)
        if (base + q < n) out[base + q] += add;
}

__global__ void __launch_bounds__(256) k_gen_cursors(DevBuild b) {
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= b.N) return;
    uint32_t* hp = b.hdr + j * b.HW;
    const unsigned long long r0 = b.rowptr[j];
    const unsigned long long inh = b.g.pops[gen_pop_of(b.g, j)].exc ? 0ull : 1ull;
    const unsigned long long rs = r0 | (inh << 63);
    hp[0] = (uint32_t)rs;
    hp[1] = (uint32_t)(rs >> 32);
    for (uint32_t x = 0; x < b.D; x++) b.cur[j * b.D + x] = r0 + hp[2 + x];
}

template <int KW>
__global__ void __launch_bounds__(256) k_gen_fill(DevBuild b, uint64_t i0, uint64_t i1) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t i = i0 + t;
    if (i >= i1) return;
    uint32_t* sc = b.scratch + t * b.g.scratch_words;
    const uint32_t D = b.D;
    const uint64_t N = b.N, E = b.E;
    const double wlim = b.wlim;
    bool bad = false, wbad = false;
    gen_target(b.g, i, sc, [&](uint64_t s, uint32_t exc, float w0, float w1, uint32_t dl, uint32_t j) {
        if (!(dl >= 1u && dl <= D && s < N)) {
            bad = true;
            return;
        }
        const unsigned long long pos = atomicAdd(&b.cur[s * D + dl - 1], 1ull);
        if (pos >= E) {
            bad = true;
            return;
        }
        const uint32_t key = (uint32_t)i | ((exc ? 0u : 1u) << 31);
        if (KW == 2)
            reinterpret_cast<uint3*>(b.edge)[pos] = make_uint3(__float_as_uint(w0), __float_as_uint(w1), key);
        else
            reinterpret_cast<uint2*>(b.edge)[pos] = make_uint2(__float_as_uint(w0), key);
        b.tb[pos] = (uint8_t)j;
        if (!(fabs((double)w0) < wlim) || !(fabs((double)w1) < wlim)) wbad = true;
    });
    if (bad || wbad) atomicOr(b.err, kErrBuild);
}

// one wavefront per row: every delay segment ordered by (target, projection), through LDS
// up to kGenSortMax records, else in place (keys distinct: a projection draws a source at
// most once per target)
template <int KW>
__global__ void __launch_bounds__(64) k_gen_sort(DevBuild b) {
    constexpr uint32_t RW = 1 + KW;
    __shared__ uint32_t s_rec[kGenSortMax * RW];
    __shared__ uint8_t s_tb[kGenSortMax];
    const uint64_t j = blockIdx.x;
    const uint32_t lane = threadIdx.x;
    const uint32_t* hp = b.hdr + j * b.HW;
    const unsigned long long r0 = (unsigned long long)hp[0] | ((unsigned long long)(hp[1] & 0x7FFFFFFFu) << 32);
    for (uint32_t x = 0; x < b.D; x++) {
        const unsigned long long s0 = r0 + hp[2 + x];
        const uint32_t L = hp[3 + x] - hp[2 + x];
        if (L < 2u) continue;
        if (s0 + L > b.E) {
            if (lane == 0) atomicOr(b.err, kErrBuild);
            continue;
        }
        if (L <= kGenSortMax) {
            for (uint32_t e = lane; e < L; e += 64) {
#pragma unroll
                for (uint32_t w = 0; w < RW; w++) s_rec[e * RW + w] = b.edge[(s0 + e) * RW + w];
                s_tb[e] = b.tb[s0 + e];
            }
            __syncthreads();
            for (uint32_t e = lane; e < L; e += 64) {
                const unsigned long long ke = ((unsigned long long)(s_rec[e * RW + KW] & 0x7FFFFFFFu) << 8) | s_tb[e];
                uint32_t rank = 0;
                for (uint32_t f = 0; f < L; f++) {
                    const unsigned long long kf = ((unsigned long long)(s_rec[f * RW + KW] & 0x7FFFFFFFu) << 8) | s_tb[f];
                    rank += kf < ke ? 1u : 0u;
                }
#pragma unroll
                for (uint32_t w = 0; w < RW; w++) b.edge[(s0 + rank) * RW + w] = s_rec[e * RW + w];
            }
            __syncthreads();
        } else {
            // longer segments in place, by a bitonic network whose comparators all put the
            // smaller key first (a flip over each block of k, then half-cleaners): the
            // positions from L up to the next power of two stand for keys above every key
            // and are never touched
            uint32_t P = 2;
            while (P < L) P <<= 1;
            for (uint32_t k = 2; k <= P; k <<= 1) {
                for (uint32_t jd = k >> 1; jd > 0; jd >>= 1) {
                    for (uint32_t q = lane; q < P / 2; q += 64) {
                        const uint32_t i = ((q & ~(jd - 1)) << 1) | (q & (jd - 1)); // bit jd clear
                        const uint32_t pi = jd == (k >> 1) ? (i ^ (k - 1)) : (i | jd);
                        if (pi >= L) continue;
                        const unsigned long long ei = s0 + i, ep = s0 + pi;
                        const unsigned long long ki = ((unsigned long long)(b.edge[ei * RW + KW] & 0x7FFFFFFFu) << 8) | b.tb[ei];
                        const unsigned long long kp = ((unsigned long long)(b.edge[ep * RW + KW] & 0x7FFFFFFFu) << 8) | b.tb[ep];
                        if (ki > kp) {
#pragma unroll
                            for (uint32_t w = 0; w < RW; w++) {
                                const uint32_t a = b.edge[ei * RW + w];
                                b.edge[ei * RW + w] = b.edge[ep * RW + w];
                                b.edge[ep * RW + w] = a;
                            }
                            const uint8_t ta = b.tb[ei];
                            b.tb[ei] = b.tb[ep];
                            b.tb[ep] = ta;
                        }
                    }
                    __syncthreads();
                }
            }
        }
    }
}

static unsigned grid_of(uint64_t n, unsigned bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t launch_device_build(const DevBuild& b, hipStream_t st) {
    const uint64_t N = b.N;
    // wavefront generator when its LDS (hash set and two index buffers per wavefront) fits
    // 64 KiB per block of up to four wavefronts; else one thread per target with scratch
    const size_t per = gen_wave_lds(b.g.kmax, b.g.hcap);
    const uint32_t wpb = per <= kGenWaveLds ? (uint32_t)std::min<size_t>(4, kGenWaveLds / per) : 0u;
    const unsigned wgrid = wpb ? (unsigned)std::min<uint64_t>((N + wpb - 1) / wpb, 256ull * 64) : 0u;
    hipLaunchKernelGGL(k_gen_clear, dim3(grid_of(N * b.D, 256 * 16) + 1), dim3(256), 0, st, b.cnt, N * b.D);
    hipError_t e = hipGetLastError();
    if (wpb) {
        hipLaunchKernelGGL((k_gen_wave<false, 2>), dim3(wgrid), dim3(64 * wpb), wpb * per, st, b);
        e = hipGetLastError();
    }
    for (uint64_t i0 = 0; !wpb && i0 < N && e == hipSuccess; i0 += b.batch) {
        const uint64_t i1 = std::min<uint64_t>(N, i0 + b.batch);
        hipLaunchKernelGGL(k_gen_count, dim3(grid_of(i1 - i0, 256)), dim3(256), 0, st, b, i0, i1);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gen_rows, dim3(grid_of(N, 256)), dim3(256), 0, st, b);
    const uint64_t nb = (N + 1023) / 1024;
    hipLaunchKernelGGL(k_scan_a, dim3((unsigned)nb), dim3(256), 0, st, b.rowlen, b.rowptr, N, b.sums);
    hipLaunchKernelGGL(k_scan_b, dim3(1), dim3(256), 0, st, b.sums, nb, b.E, b.err);
    hipLaunchKernelGGL(k_scan_c, dim3((unsigned)nb), dim3(256), 0, st, b.rowptr, N, b.sums);
    hipLaunchKernelGGL(k_gen_cursors, dim3(grid_of(N, 256)), dim3(256), 0, st, b);
    e = hipGetLastError();
    if (wpb && e == hipSuccess) {
        if (b.KW == 2)
            hipLaunchKernelGGL((k_gen_wave<true, 2>), dim3(wgrid), dim3(64 * wpb), wpb * per, st, b);
        else
            hipLaunchKernelGGL((k_gen_wave<true, 1>), dim3(wgrid), dim3(64 * wpb), wpb * per, st, b);
        e = hipGetLastError();
    }
    for (uint64_t i0 = 0; !wpb && i0 < N && e == hipSuccess; i0 += b.batch) {
        const uint64_t i1 = std::min<uint64_t>(N, i0 + b.batch);
        if (b.KW == 2)
            hipLaunchKernelGGL(k_gen_fill<2>, dim3(grid_of(i1 - i0, 256)), dim3(256), 0, st, b, i0, i1);
        else
            hipLaunchKernelGGL(k_gen_fill<1>, dim3(grid_of(i1 - i0, 256)), dim3(256), 0, st, b, i0, i1);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    if (b.KW == 2)
        hipLaunchKernelGGL(k_gen_sort<2>, dim3((unsigned)N), dim3(64), 0, st, b);
    else
        hipLaunchKernelGGL(k_gen_sort<1>, dim3((unsigned)N), dim3(64), 0, st, b);
    return hipGetLastError();
}

} // namespace dbs
