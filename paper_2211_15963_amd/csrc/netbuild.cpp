// netbuild.cpp - validation, memory plan and host construction of the tables.
//
// The connection table is generated per target by the seeded generator
// (fixed in-degree, sources drawn without replacement) and transposed here
// into rows by presynaptic neuron, each row split into delay segments and
// sorted by (delay, target) so the layout is deterministic. Two generator
// passes (count, then fill) avoid holding a by-target copy of the table.
#include "netbuild.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <thread>

#include <unistd.h>

namespace dbs {

namespace {

template <class F>
void parallel_chunks(uint64_t n, uint64_t chunk, unsigned nt, F f) {
    std::atomic<uint64_t> next{0};
    auto worker = [&](unsigned tid) {
        for (;;) {
            const uint64_t a = next.fetch_add(chunk);
            if (a >= n) break;
            f(tid, a, std::min(n, a + chunk));
        }
    };
    std::vector<std::thread> th;
    for (unsigned t = 1; t < nt; t++) th.emplace_back(worker, t);
    worker(0);
    for (auto& x : th) x.join();
}

uint32_t pow2_at_least32(uint64_t x) {
    uint64_t c = 1;
    while (c < x) c <<= 1;
    return (uint32_t)c;
}

uint64_t pow2_at_least64(uint64_t x) {
    uint64_t c = 1;
    while (c < x) c <<= 1;
    return c;
}

// Poisson inversion thresholds T_c = floor(2^32 * CDF(c)) of Poisson(lambda),
// CDF summed in ascending c from p_0 = exp(-lambda), p_c = p_{c-1} lambda / c;
// stops at the first c whose upper tail is below 2^-32. Returns the length or -1.
int poisson_thresholds(double lambda, uint32_t* T, int cap) {
    double p = std::exp(-lambda), F = p;
    int c = 0;
    for (;;) {
        if (1.0 - F < 0x1p-32) return c;
        if (c >= cap) return -1;
        T[c] = (uint32_t)std::floor(F * 0x1p32);
        c++;
        p = p * lambda / (double)c;
        F = F + p;
    }
}

uint32_t indeg_of_pop(const dbnet_desc& d, uint32_t p) {
    uint32_t k = 0;
    for (uint32_t j = 0; j < d.n_projs; j++)
        if (d.projs[j].dst_pop < 0 || (uint32_t)d.projs[j].dst_pop == p) k += d.projs[j].indegree;
    return k;
}

} // namespace

// one edge on its way from its target to its source's row (bucketed construction)
struct BucketEdge {
    uint32_t src_dl; // source index within its block << 8 | delay
    uint32_t tgt;
    uint32_t w0, w1; // weight bit patterns
};
// host memory the bucketed construction may hold: 30 % of the machine's memory, at most
// 64 GiB (larger networks take the two-pass construction)
static double bucket_build_bytes() {
    const long pages = sysconf(_SC_PHYS_PAGES), psz = sysconf(_SC_PAGE_SIZE);
    const double phys = pages > 0 && psz > 0 ? (double)pages * (double)psz : 16.0 * (1ull << 30);
    return std::min(0.3 * phys, 64.0 * (1ull << 30));
}

uint32_t max_round_events(const Plan& p, uint32_t wgs_per_cu) {
    if (p.blocked) return (uint32_t)(kFanThreads * kMaxBatch); // events stay in registers
    const size_t budget = kMaxLdsBytes / wgs_per_cu - kStaticLds;
    uint32_t best = 0;
    for (uint32_t re = kScatterThreads; re <= (uint32_t)(kScatterThreads * kMaxBatch); re += kScatterThreads)
        if (part_lds_bytes(p.NS, re, p.D) <= budget) best = re;
    return best;
}

uint32_t max_bucket_events(const Plan& p, uint32_t wgs_per_cu) {
    if (p.blocked) return kScatterThreads; // no second pass
    const size_t budget = kMaxLdsBytes / wgs_per_cu - kStaticLds;
    uint32_t best = 0;
    for (uint32_t re = kScatterThreads; re <= (uint32_t)(kScatterThreads * kMaxBatch); re += kScatterThreads)
        if (bucket_lds_bytes(1u << p.ts_bits, re) <= budget) best = re;
    return best;
}

uint32_t fan_chunk_records(const Plan& p, uint32_t wgs_per_cu) {
    if (wgs_per_cu == 0) return 0;
    const size_t budget = kMaxLdsBytes / wgs_per_cu - kStaticLds;
    uint32_t best = 0;
    for (uint32_t c = kFanMinChunk; c <= kFanMaxChunk; c *= 2)
        if (fan_lds_bytes(p.T, c, p.KW, p.D) <= budget) best = c;
    return best;
}

void Members::assign(const dbnet_desc* descs, uint32_t n) {
    m.assign(descs, descs + n);
    pops.resize(n);
    projs.resize(n);
    xyz.resize(n);
    nbase.assign(n + 1, 0);
    pbase.assign(n + 1, 0);
    rbase.assign(n + 1, 0);
    for (uint32_t k = 0; k < n; k++) {
        const dbnet_desc& d = descs[k];
        if (d.pops && d.n_pops) pops[k].assign(d.pops, d.pops + d.n_pops);
        if (d.projs && d.n_projs) projs[k].assign(d.projs, d.projs + d.n_projs);
        if (d.region_xyz_mm) xyz[k].assign(d.region_xyz_mm, d.region_xyz_mm + 3 * (size_t)d.n_regions);
        m[k].pops = pops[k].empty() ? nullptr : pops[k].data();
        m[k].projs = projs[k].empty() ? nullptr : projs[k].data();
        m[k].region_xyz_mm = xyz[k].empty() ? nullptr : xyz[k].data();
        uint64_t nn = 0;
        for (const auto& q : pops[k]) nn += q.size;
        nbase[k + 1] = nbase[k] + nn;
        pbase[k + 1] = pbase[k] + d.n_pops;
        rbase[k + 1] = rbase[k] + d.n_regions;
    }
}

uint32_t Members::member_of(uint64_t i) const {
    return (uint32_t)(std::upper_bound(nbase.begin(), nbase.end(), i) - nbase.begin()) - 1;
}

// Candidate rule of the input generator: is population q a source of projection pr for
// targets in population tp (class filter, then the source mode)?
static bool gen_candidate(const dbnet_desc& d, const dbnet_proj& pr, uint32_t tp, uint32_t q) {
    const dbnet_pop& P = d.pops[q];
    if (pr.src_class == DBNET_CLASS_EXC && !P.exc) return false;
    if (pr.src_class == DBNET_CLASS_INH && P.exc) return false;
    switch (pr.src_mode) {
    case DBNET_SRC_ALL: return true;
    case DBNET_SRC_SAME_REGION: return P.region == d.pops[tp].region;
    case DBNET_SRC_OTHER_REGIONS: return P.region != d.pops[tp].region;
    case DBNET_SRC_POP: return (int32_t)q == pr.src_pop;
    default: return false;
    }
}

std::string make_gen_tables(const Members& mem, HostTables& h) {
    h.gpops.clear();
    h.gmembers.clear();
    h.gprojs.clear();
    h.gcands.clear();
    h.gcpops.clear();
    h.gdtab.clear();
    h.gkmax = 1;
    for (size_t m = 0; m < mem.m.size(); m++) {
        const dbnet_desc& d = mem.m[m];
        GenMember gm{};
        gm.seed = d.seed;
        gm.nbase = mem.nbase[m];
        gm.net_id = d.net_id;
        gm.kw = dbnet_weights_per_edge(&d);
        gm.n_pops = d.n_pops;
        gm.n_regions = d.n_regions;
        gm.proj0 = (uint32_t)h.gprojs.size();
        gm.n_projs = d.n_projs;
        std::vector<uint64_t> off(d.n_pops + 1, 0);
        for (uint32_t q = 0; q < d.n_pops; q++) off[q + 1] = off[q] + d.pops[q].size;
        for (uint32_t q = 0; q < d.n_pops; q++) {
            GenPop gp{};
            gp.first = mem.nbase[m] + off[q];
            gp.off = off[q];
            gp.size = d.pops[q].size;
            gp.exc = d.pops[q].exc ? 1u : 0u;
            gp.member = (uint32_t)m;
            gp.local = q;
            gp.region = d.pops[q].region;
            h.gpops.push_back(gp);
        }
        for (uint32_t j = 0; j < d.n_projs; j++) {
            const dbnet_proj& pr = d.projs[j];
            if (pr.indegree > 0 && pr.w_dist == DBNET_W_LOGNORMAL)
                return "lognormal weights are drawn through libm and generated on the host";
            GenProj gj{};
            gj.dst_pop = pr.dst_pop;
            gj.indegree = pr.indegree;
            gj.w_dist = pr.w_dist == DBNET_W_UNIFORM ? 0u : 1u;
            gj.d_mode = pr.d_mode;
            gj.d_min = pr.d_min;
            gj.d_max = pr.d_max;
            gj.w_a = pr.w_a;
            gj.w_b = pr.w_b;
            gj.w_scale_exc = pr.w_scale_exc;
            gj.w_scale_inh = pr.w_scale_inh;
            gj.cand0 = (uint32_t)h.gcands.size();
            h.gkmax = std::max(h.gkmax, pr.indegree);
            if (pr.d_mode == DBNET_D_DISTANCE && pr.indegree > 0) {
                // the generator's delay of a source in region a for a target in region b
                gj.dtab = (uint32_t)h.gdtab.size();
                const uint32_t R = d.n_regions;
                h.gdtab.resize(h.gdtab.size() + (size_t)R * R);
                for (uint32_t a = 0; a < R; a++)
                    for (uint32_t b = 0; b < R; b++) {
                        const float* xs = d.region_xyz_mm + 3 * a;
                        const float* xt = d.region_xyz_mm + 3 * b;
                        const double dx = (double)xs[0] - xt[0], dy = (double)xs[1] - xt[1], dz = (double)xs[2] - xt[2];
                        const double dist = std::sqrt(dx * dx + dy * dy + dz * dz);
                        const double bins = std::ceil(dist / ((double)d.velocity_mm_per_ms * (double)d.bin_ms));
                        const uint32_t dl = bins < (double)pr.d_min ? pr.d_min
                                            : bins > (double)pr.d_max ? pr.d_max : (uint32_t)bins;
                        h.gdtab[gj.dtab + (size_t)a * R + b] = (uint8_t)dl;
                    }
            }
            // candidates for every target population (ascending population order, the target
            // itself removed from the index space)
            for (uint32_t tp = 0; tp < d.n_pops; tp++) {
                GenCand c{};
                c.c0 = (uint32_t)h.gcpops.size();
                c.self_base = ~0ull;
                uint64_t mm = 0;
                for (uint32_t q = 0; q < d.n_pops; q++) {
                    if (!gen_candidate(d, pr, tp, q)) continue;
                    if (q == tp) c.self_base = mm;
                    mm += d.pops[q].size;
                    GenCandPop cp{};
                    cp.end = mm;
                    cp.first = mem.nbase[m] + off[q];
                    cp.size = d.pops[q].size;
                    cp.exc = d.pops[q].exc ? 1u : 0u;
                    h.gcpops.push_back(cp);
                }
                c.nc = (uint32_t)h.gcpops.size() - c.c0;
                c.M = mm - (c.self_base != ~0ull ? 1 : 0);
                h.gcands.push_back(c);
            }
            h.gprojs.push_back(gj);
        }
        h.gmembers.push_back(gm);
    }
    h.ghcap = pow2_at_least32(2ull * h.gkmax + 2);
    return "";
}

size_t gen_tables_bytes(const HostTables& h) {
    auto a = [](size_t b) { return (b + 255) & ~(size_t)255; };
    return a(sizeof(GenPop) * h.gpops.size()) + a(sizeof(GenMember) * h.gmembers.size()) +
           a(sizeof(GenProj) * h.gprojs.size()) + a(sizeof(GenCand) * h.gcands.size()) +
           a(sizeof(GenCandPop) * h.gcpops.size()) + a(h.gdtab.size() + 1);
}

std::string make_plan(const dbsim_desc& opts, const Members& mem, Plan& p) {
    if (opts.abi_version != DBSIM_ABI_VERSION) return "dbsim_desc.abi_version does not match the library";
    if (mem.m.empty()) return "no network given";
    char err[512];
    for (size_t k = 0; k < mem.m.size(); k++) {
        if (dbnet_validate(&mem.m[k], err, sizeof err) != 0)
            return mem.m.size() > 1 ? "member " + std::to_string(k) + ": " + err : std::string(err);
    }
    const dbnet_desc& m0 = mem.m[0];
    for (size_t k = 1; k < mem.m.size(); k++) {
        const dbnet_desc& d = mem.m[k];
        if (d.dt_ms != m0.dt_ms || d.bin_ms != m0.bin_ms || d.receptor_mask != m0.receptor_mask ||
            d.frac_bits != m0.frac_bits)
            return "ensemble members must share dt_ms, bin_ms, receptor_mask and frac_bits";
    }
    if (mem.nbase.back() >= DBNET_MAX_NEURONS) return "too many neurons in total (ids must fit in 28 bits)";
    p.n_members = (uint32_t)mem.m.size();
    p.N = (uint32_t)mem.nbase.back();
    p.KW = dbnet_weights_per_edge(&m0);
    p.U = 2 * p.KW;
    p.S = (uint32_t)std::lround((double)m0.bin_ms / (double)m0.dt_ms);
    p.D = 1;
    for (const auto& d : mem.m) p.D = std::max(p.D, dbnet_max_delay(&d));
    p.F = m0.frac_bits;
    p.n_pops = mem.pbase.back();
    p.n_regions = mem.rbase.back();
    p.regions_on = (opts.record_flags & DBSIM_REC_REGIONS) != 0;
    // tiles: the LDS accumulator of a tile holds tile_neurons * U int64 sums
    const uint32_t tile_neurons = kTileLdsBytes / (8u * p.U);
    p.tile_bits = 0;
    while ((1u << (p.tile_bits + 1)) <= tile_neurons) p.tile_bits++;
    p.T = (p.N + (1u << p.tile_bits) - 1) >> p.tile_bits;
    if (p.T > (uint32_t)kMaxTilesLds) return "network too large for the tile histogram (too many neurons)";
    // fan-in form: two passes through at most kMaxSuperTiles super-tile streams of a
    // power-of-two number of tiles each (the faster form on every measured network); on
    // request, one pass straight into per-workgroup tile blocks when a carry buffer of at
    // least kFanMinChunk records per tile fits one workgroup's LDS (T up to about 2,900
    // tiles with two weights per edge), which needs no streams
    p.blocked = (opts.flags & DBSIM_F_SINGLE_PASS) != 0 && p.T <= 65535u && fan_chunk_records(p, 1) != 0;
    p.ts_bits = 0;
    if (!p.blocked)
        while (((p.T + (1u << p.ts_bits) - 1) >> p.ts_bits) > kMaxSuperTiles) p.ts_bits++;
    p.NS = p.blocked ? 0u : (p.T + (1u << p.ts_bits) - 1) >> p.ts_bits;
    p.HW = (p.D + 3 + 3) & ~3u;
    // default schedule: two passes, two partition workgroups per CU and the largest LDS
    // round that fits; single pass, one workgroup per CU with the largest carry buffers
    p.scatter_wgs_per_cu = p.blocked ? 1 : 2;
    p.round_events = max_round_events(p, p.scatter_wgs_per_cu);
    p.bucket_events = max_bucket_events(p, p.scatter_wgs_per_cu);
    if (p.round_events == 0 || p.bucket_events == 0) return "too many tiles per super-tile for the LDS budget";
    const double dt = (double)m0.dt_ms;
    p.E = 0;
    p.n_blocks = 0;
    std::vector<uint64_t> rblocks(p.n_regions, 0);
    for (size_t k = 0; k < mem.m.size(); k++) {
        const dbnet_desc& n = mem.m[k];
        for (uint32_t q = 0; q < n.n_pops; q++) {
            const dbnet_pop& P = n.pops[q];
            const long r = std::lround((double)P.T_ref / dt);
            if (r < (long)p.S - 1)
                return "T_ref must be at least bin_ms - dt_ms so that a neuron spikes at most once per bin";
            if (r > 255) return "T_ref / dt_ms must not exceed 255 steps";
            uint32_t T[kMaxPoisson];
            if (poisson_thresholds((double)P.bg_rate_hz * dt * 1e-3, T, kMaxPoisson) < 0)
                return "background rate too high for the Poisson table (rate * dt above about 20)";
            const uint32_t kin = indeg_of_pop(n, q);
            // super-tile streams and tile slices are indexed with 32-bit fill counters
            if (((uint64_t)kin << (p.tile_bits + p.ts_bits)) >= (1ull << 32))
                return "in-degree too large for a super-tile stream";
            p.E += (uint64_t)P.size * kin;
            const uint32_t nb = (P.size + kNeuronBlock - 1) / kNeuronBlock;
            p.n_blocks += nb;
            rblocks[mem.rbase[k] + P.region] += nb;
        }
    }
    p.n_l1 = 0;
    for (uint32_t r = 0; r < p.n_regions; r++) p.n_l1 += (uint32_t)std::max<uint64_t>(1, (rblocks[r] + 255) / 256);
    const uint32_t rb = opts.record_bins ? opts.record_bins : 4096u;
    p.MB = pow2_at_least32(std::max<uint64_t>(rb, (uint64_t)p.D + 1));
    // spike history: at least the last D + 1 bins for the fan-in, plus (when the raster is
    // read from the device) a default reading window; the host ring takes the raster otherwise
    p.host_record = !(opts.flags & DBSIM_F_NO_HOST_RECORD);
    const uint64_t want = opts.spike_record_capacity ? opts.spike_record_capacity : (p.host_record ? 0 : (1ull << 22));
    p.RC = pow2_at_least64(std::max<uint64_t>(want, ((uint64_t)p.D + 1) * p.N));
    p.HC = p.host_record ? pow2_at_least64(std::max<uint64_t>(opts.host_spike_capacity ? opts.host_spike_capacity
                                                                                      : (1ull << 24), 64)) : 0;
    p.HMB = p.host_record ? (1u << 20) : 0;
    // memory plan (one allocation, 256-byte aligned slots)
    size_t off = 0;
    auto slot = [&](Plan::Slot& s, size_t bytes) {
        s.off = off;
        s.bytes = bytes;
        off += (bytes + 255) & ~(size_t)255;
    };
    // in-edges of every tile (the most events it can receive in one bin)
    std::vector<uint64_t> tin(p.T, 0);
    {
        uint64_t i0 = 0;
        for (size_t k = 0; k < mem.m.size(); k++)
            for (uint32_t q = 0; q < mem.m[k].n_pops; q++) {
                const uint64_t kin = indeg_of_pop(mem.m[k], q), i1 = i0 + mem.m[k].pops[q].size;
                for (uint64_t a = i0; a < i1;) {
                    const uint64_t t = a >> p.tile_bits, b = std::min(i1, (t + 1) << p.tile_bits);
                    tin[t] += kin * (b - a);
                    a = b;
                }
                i0 = i1;
            }
    }
    // single-pass form: tile t's blocks hold its total in-degree in whole blocks plus two
    // part-filled blocks per workgroup and bin (one per workgroup and pass)
    p.tile_blk.clear();
    if (p.blocked) {
        p.tile_blk.assign((size_t)p.T + 1, 0);
        for (uint32_t t = 0; t < p.T; t++)
            p.tile_blk[t + 1] = p.tile_blk[t] + tin[t] / kFanBlock + 2ull * kFanMaxGrid;
        if (p.tile_blk[p.T] >= 0xFFFFFFF0ull) return "network too large for the single-pass event arena";
    }
    const size_t N = p.N, U = p.U, E = p.E;
    // the device checks nothing it could report before the first bin, so the fixed-point
    // range of the weights (|w| 2^F < 2^52) is bounded here from the distributions' limits;
    // a description that may exceed it is built and checked exactly on the host
    bool wfit = true;
    for (const auto& d : mem.m)
        for (uint32_t j = 0; j < d.n_projs; j++) {
            const dbnet_proj& pr = d.projs[j];
            const double a = std::max(std::fabs((double)pr.w_a), pr.w_dist == DBNET_W_CONST ? 0.0 : std::fabs((double)pr.w_b));
            const double sc = std::max(std::fabs((double)pr.w_scale_exc), std::fabs((double)pr.w_scale_inh));
            if (!(a * sc * (1.0 + 0x1p-20) < std::ldexp(1.0, 52 - (int)p.F))) wfit = false;
        }
    HostTables gt;
    const bool gen_ok = !p.blocked && !(opts.flags & DBSIM_F_HOST_BUILD) && p.E > 0 && wfit &&
                        make_gen_tables(mem, gt).empty();
    // per-target scratch of the thread-per-target generator (in the streams, which are free
    // before the first bin); the wavefront generator needs none
    const size_t gen_sw = gen_ok ? 4 * (size_t)gen_scratch_words(gt.gkmax, gt.ghcap) : 1;
    const bool gen_threads = gen_ok && gen_wave_lds(gt.gkmax, gt.ghcap) > kGenWaveLds;
    // the construction's temporaries in the arena's weight slot (free before the first bin)
    p.gl = Plan::GenLayout{};
    if (gen_ok) {
        size_t o = 0;
        auto take = [&](size_t bytes) {
            const size_t at = o;
            o += (bytes + 255) & ~(size_t)255;
            return at;
        };
        Plan::GenLayout& g = p.gl;
        g.tables = take(gen_tables_bytes(gt));
        g.cnt = take(4 * (size_t)N * p.D);
        g.cur = take(8 * (size_t)N * p.D);
        g.rowlen = take(8 * (N + 1));
        g.rowptr = take(8 * (N + 1));
        g.sums = take(8 * (N / 1024 + 2));
        g.tb = take(E);
        g.flags = take(16);
        g.end = o;
    }
    // tile arena slices of the two-pass form: a share of each tile's in-edges (all of them
    // would cover the worst case, every edge firing in one bin; a bin at 15 Hz fills about
    // 1.5 %); the events past a full slice go to the per-target overflow sums
    if (opts.arena_permille > 1000) return "arena_permille must lie in 0..1000";
    p.ta_permille = opts.arena_permille ? opts.arena_permille : kArenaPermille;
    p.ta_len.assign(p.blocked ? 0 : p.T, 0);
    p.ta_total = 0;
    for (uint32_t t = 0; !p.blocked && t < p.T; t++) {
        uint64_t len = (tin[t] * p.ta_permille + 999) / 1000;
        if (!opts.arena_permille) len = std::max(len, std::min<uint64_t>(tin[t], kArenaFloor));
        len = std::max<uint64_t>(len, 1);
        p.ta_len[t] = len;
        p.ta_total += len;
    }
    slot(p.V, 4 * N);
    slot(p.J, 4 * U * N);
    slot(p.ref, N);
    slot(p.pend, N);
    slot(p.A, 4 * U * N);
    slot(p.Iou, 4 * N);
    slot(p.pops, sizeof(PopParams) * p.n_pops);
    slot(p.ptab, 4 * (size_t)kMaxPoisson * p.n_pops);
    slot(p.blk, sizeof(uint2) * p.n_blocks);
    slot(p.hdr, 4 * N * (size_t)p.HW);
    slot(p.edge, 4 * (size_t)(1 + p.KW) * E + 64); // spare: 8-byte records are copied with 12-byte reads
    // event arena
    if (p.blocked) {
        const size_t recs = (size_t)p.tile_blk[p.T] * kFanBlock;
        slot(p.ev, 4 * (size_t)p.KW * recs);
        slot(p.evk, 2 * recs);
        slot(p.bcnt, 4 * (size_t)p.tile_blk[p.T]);
    } else { // records of a 16-bit key array beside the weights
        slot(p.ev, std::max(4 * (size_t)p.KW * p.ta_total + 64, p.gl.end));
        slot(p.evk, 2 * (size_t)p.ta_total + 64);
        slot(p.bcnt, 16);
    }
    // per-target int64 sums of the events past their tile's arena slice ([N][U])
    slot(p.ovf, p.blocked ? 16 : 8 * U * N);
    slot(p.tile_base, 8 * ((size_t)p.T + 1));
    // fill counters of the tiles, then the first failed reservation of each
    slot(p.tile_fill, 8 * (size_t)p.T);
    // fill counters of the super-tile streams, then the first failed reservation of each
    slot(p.st_base, 8 * ((size_t)p.NS + 1));
    slot(p.st_fill, 8 * (size_t)p.NS + 4);
    // narrow stream records: two weights per edge, every weight non-negative (its sign bit
    // free: the parameters that shape it are not negative and not -0), and a key within the
    // super-tile of at most 17 bits
    p.narrow = false;
    if (!p.blocked && p.KW == 2 && p.tile_bits + p.ts_bits <= 17) {
        bool nonneg = true;
        for (const auto& d : mem.m)
            for (uint32_t j = 0; j < d.n_projs; j++) {
                const dbnet_proj& pr = d.projs[j];
                if (std::signbit(pr.w_scale_exc) || std::signbit(pr.w_scale_inh)) nonneg = false;
                if (pr.w_dist != DBNET_W_LOGNORMAL && std::signbit(pr.w_a)) nonneg = false;
            }
        p.narrow = nonneg;
    }
    // stream slices: a share of each super-tile's in-edges (all of them would cover the
    // worst case, every edge firing in one pass; a pass at 15 Hz fills about 1.4 %), even
    // sized for the narrow records (the bucketing copies record pairs); the runs past a
    // full slice go to the tile arena event by event
    if (opts.stream_permille > 1000) return "stream_permille must lie in 0..1000";
    p.st_permille = opts.stream_permille ? opts.stream_permille : kStreamPermille;
    p.st_len.assign(p.NS, 0);
    p.st_total = 0;
    for (uint32_t x = 0; x < p.NS; x++) {
        uint64_t in = 0;
        for (uint32_t t = x << p.ts_bits; t < std::min<uint32_t>(p.T, (x + 1) << p.ts_bits); t++) in += tin[t];
        uint64_t len = (in * p.st_permille + 999) / 1000;
        if (!opts.stream_permille) len = std::max(len, std::min<uint64_t>(in, kStreamFloor));
        len = std::max<uint64_t>(len, 2);
        if (p.narrow) len = (len + 1) & ~1ull;
        p.st_len[x] = len;
        p.st_total += len;
    }
    // 64 spare bytes: the partition kernels copy 8-byte records with 12-byte reads
    p.st_cap = p.narrow ? p.st_total + 128 : 0;
    if (p.blocked) {
        slot(p.sev, 16);
    } else {
        size_t sb = p.narrow ? ((2 * (size_t)p.st_cap + 255) & ~(size_t)255) + 8 * (size_t)p.st_cap
                             : 4 * (size_t)(1 + p.KW) * p.st_total + 64;
        // the thread-per-target generator's batches of up to 2^20 targets, within the
        // worst-case stream size
        if (gen_threads)
            sb = std::max(sb, std::min(4 * (size_t)(1 + p.KW) * E + 64, gen_sw * std::min<size_t>(N, 1u << 20)));
        slot(p.sev, sb);
    }
    p.n_grp = (p.n_blocks + 255) / 256;
    slot(p.stage, 4 * (size_t)p.n_blocks * kNeuronBlock);
    slot(p.grp_cnt, 4 * 2 * (size_t)p.n_grp);
    slot(p.rec, 4 * p.RC);
    slot(p.bin_start, 8 * (size_t)p.MB);
    slot(p.bin_cnt, 4 * (size_t)p.MB);
    slot(p.blk_sig, 8 * (size_t)p.n_blocks);
    slot(p.blk_cnt, 4 * (size_t)p.n_blocks);
    slot(p.reg_blk_ptr, 4 * ((size_t)p.n_regions + 1));
    slot(p.reg_blk, 4 * (size_t)p.n_blocks);
    slot(p.reg_size, 4 * (size_t)p.n_regions);
    slot(p.l1_ptr, 4 * ((size_t)p.n_regions + 1));
    slot(p.l1_region, 4 * (size_t)p.n_l1);
    slot(p.l1_sig, 8 * (size_t)p.n_l1);
    slot(p.l1_cnt, 4 * (size_t)p.n_l1);
    slot(p.sig, p.regions_on ? 8 * (size_t)p.MB * p.n_regions : 8);
    slot(p.sig_cnt, p.regions_on ? 4 * (size_t)p.MB * p.n_regions : 4);
    const size_t RB = p.regions_on ? p.n_regions : 1;
    slot(p.bold_zs, 8 * RB);
    slot(p.bold, 8 * 4 * RB);
    slot(p.bold_y, 8 * (size_t)kBoldRing * RB);
    slot(p.bold_ctl, 16);
    slot(p.rblk, 8 * 4 * (size_t)p.n_blocks); // receptor-current measurement (block sums)
    slot(p.rpop, 8 * 4 * (size_t)p.n_pops);
    slot(p.ctl, sizeof(Ctl));
    p.total = off;
    // connection table on the device: two-pass form (its streams and arena are free before
    // the first bin), weights of exact double arithmetic, and room for the temporaries
    p.dev_build = false;
    p.gen_batch = 0;
    if (gen_ok) {
        const Plan::GenLayout& g = p.gl;
        const uint64_t batch = std::min<uint64_t>({(uint64_t)N, p.sev.bytes / gen_sw, 1ull << 20});
        if (g.end <= p.ev.bytes && batch >= std::min<uint64_t>(N, 4096)) {
            p.dev_build = true;
            p.gen_batch = (uint32_t)batch;
        }
    }
    return "";
}

void fill_populations(const Members& mem, const Plan& p, std::vector<PopParams>& pops, std::vector<uint32_t>& ptab,
                      std::vector<uint64_t>* first, std::vector<uint32_t>* indeg) {
    const uint32_t KW = p.KW;
    const uint32_t M = (uint32_t)mem.m.size();
    const double dt = (double)mem.m[0].dt_ms;
    // derived constants, computed in double and rounded once to float
    pops.assign(p.n_pops, PopParams{});
    ptab.assign((size_t)p.n_pops * kMaxPoisson, 0u);
    static const uint32_t umap2[2] = {DBNET_AMPA, DBNET_GABA_A};
    static const uint32_t umap4[4] = {DBNET_AMPA, DBNET_NMDA, DBNET_GABA_A, DBNET_GABA_B};
    const uint32_t* umap = KW == 1 ? umap2 : umap4;
    if (indeg) indeg->assign(p.n_pops, 0u);
    if (first) first->assign((size_t)p.n_pops + 1, 0ull);
    uint64_t off = 0;
    for (uint32_t m = 0; m < M; m++) {
        const dbnet_desc& d = mem.m[m];
        for (uint32_t q = 0; q < d.n_pops; q++) {
            const uint32_t gq = mem.pbase[m] + q;
            const dbnet_pop& Q = d.pops[q];
            PopParams& P = pops[gq];
            P.k = (float)(dt / (double)Q.C);
            P.gL = Q.g_L;
            P.VL = Q.V_L;
            P.Vth = Q.V_th;
            P.Vr = Q.V_reset;
            P.Iext = Q.I_ext;
            P.wbg = Q.w_bg;
            for (uint32_t c = 0; c < p.U; c++) {
                const uint32_t u = umap[c];
                P.g[c] = Q.g[u];
                P.Vu[c] = Q.V_rev[u];
                P.dec[c] = (float)std::exp(-dt / (double)Q.tau[u]);
            }
            P.r = (int32_t)std::lround((double)Q.T_ref / dt);
            P.cmax = poisson_thresholds((double)Q.bg_rate_hz * dt * 1e-3, &ptab[(size_t)gq * kMaxPoisson], kMaxPoisson);
            if (first) (*first)[gq] = off;
            off += Q.size;
            P.end = (uint32_t)off;
            P.region = mem.rbase[m] + Q.region;
            P.net_id = d.net_id;
            P.id_base = (uint32_t)mem.nbase[m];
            P.seed = d.seed;
            if (indeg) (*indeg)[gq] = indeg_of_pop(d, q);
        }
    }
    if (first) (*first)[p.n_pops] = off;
}

std::string build_tables(const Members& mem, const Plan& p, unsigned threads, HostTables& h, bool with_edges) {
    const unsigned nt = threads ? threads : std::max(1u, std::thread::hardware_concurrency());
    const uint32_t N = p.N, D = p.D, KW = p.KW;
    const uint32_t M = (uint32_t)mem.m.size();

    std::vector<uint32_t> pop_indeg;
    std::vector<uint64_t> pop_first;
    fill_populations(mem, p, h.pops, h.ptab, &pop_first, &pop_indeg);
    // neuron blocks never straddle populations; regions list their blocks
    h.blk.clear();
    h.reg_size.assign(p.n_regions, 0u);
    std::vector<std::vector<uint32_t>> rb(p.n_regions);
    for (uint32_t gq = 0; gq < p.n_pops; gq++) {
        const uint32_t r = h.pops[gq].region;
        for (uint64_t s = pop_first[gq]; s < pop_first[gq + 1]; s += kNeuronBlock) {
            rb[r].push_back((uint32_t)h.blk.size());
            h.blk.push_back(make_uint2((uint32_t)s, gq));
        }
        h.reg_size[r] += (uint32_t)(pop_first[gq + 1] - pop_first[gq]);
    }
    h.reg_blk_ptr.assign(p.n_regions + 1, 0u);
    h.reg_blk.clear();
    h.l1_ptr.assign(p.n_regions + 1, 0u);
    h.l1_region.clear();
    for (uint32_t r = 0; r < p.n_regions; r++) {
        h.reg_blk.insert(h.reg_blk.end(), rb[r].begin(), rb[r].end());
        h.reg_blk_ptr[r + 1] = (uint32_t)h.reg_blk.size();
        const uint32_t g = std::max<uint32_t>(1u, ((uint32_t)rb[r].size() + 255u) / 256u);
        for (uint32_t x = 0; x < g; x++) h.l1_region.push_back(r);
        h.l1_ptr[r + 1] = (uint32_t)h.l1_region.size();
    }
    if (h.l1_region.size() != p.n_l1) return "internal error: readout group count mismatch";
    // per-neuron source class and in-degree prefix by tile
    h.src_inh.assign(N, 0);
    h.tile_base.assign((size_t)p.T + 1, 0ull);
    for (uint32_t m = 0; m < M; m++)
        for (uint32_t q = 0; q < mem.m[m].n_pops; q++) {
            const uint32_t gq = mem.pbase[m] + q;
            const uint8_t inh = mem.m[m].pops[q].exc ? 0 : 1;
            for (uint64_t i = pop_first[gq]; i < pop_first[gq + 1]; i++) {
                h.src_inh[i] = inh;
                h.tile_base[(i >> p.tile_bits) + 1] += pop_indeg[gq];
            }
        }
    {
        uint64_t sum = 0;
        for (uint32_t t = 0; t < p.T; t++) sum += h.tile_base[t + 1];
        if (sum != p.E) return "internal error: edge count mismatch";
    }
    // record slices of the two-pass form; block ranges of the single-pass form (the plan's)
    if (p.blocked) {
        h.tile_base = p.tile_blk;
    } else {
        for (uint32_t t = 0; t < p.T; t++) h.tile_base[t + 1] = h.tile_base[t] + p.ta_len[t];
    }

    // initial membrane potentials
    h.V0.resize(N);
    parallel_chunks(N, 1 << 16, nt, [&](unsigned, uint64_t a, uint64_t b) {
        for (uint64_t i = a; i < b; i++) {
            const uint32_t m = mem.member_of(i);
            h.V0[i] = dbnet_v0(&mem.m[m], (uint32_t)(i - mem.nbase[m]));
        }
    });

    // super-tile stream slices (the plan's sizes, one after another)
    h.st_base.assign((size_t)p.NS + 1, 0ull);
    for (uint32_t x = 0; x < p.NS; x++) h.st_base[x + 1] = h.st_base[x] + p.st_len[x];
    if (!with_edges) return make_gen_tables(mem, h);

    size_t scratch_bytes = 0;
    uint32_t kmax = 1;
    for (const auto& d : mem.m) {
        scratch_bytes = std::max(scratch_bytes, dbnet_scratch_bytes(&d));
        kmax = std::max(kmax, dbnet_max_indegree(&d));
    }
    const size_t RW = 1 + KW; // words per edge record: the weights, then the target (key)
    const double wlim = std::ldexp(1.0, 52 - (int)p.F);
    std::atomic<int> gen_fail{0}, wbad{0};
    if ((double)p.E * sizeof(BucketEdge) <= bucket_build_bytes()) {
        // Bucketed transposition. The edges are generated by target and stored by source.
        // Phase 1: thread t generates the targets of its static range in ascending order and
        // appends each edge to its bucket of the source's block. Phase 2: every source block
        // is placed on its own: counts per (source, delay), block-local offsets, then the
        // block's buckets in thread order, which is ascending target order, so every delay
        // segment comes out sorted by target. No atomics, no random writes across the table.
        const uint32_t SB = std::max<uint32_t>(1, std::min<uint32_t>(4096, N / 2048)); // source blocks
        const uint32_t bsz = (N + SB - 1) / SB;                                        // sources per block
        const unsigned T = nt;
        std::vector<std::vector<BucketEdge>> bucket((size_t)T * SB);
        std::vector<std::thread> th;
        auto gen = [&](unsigned t) {
            const uint64_t i0 = (uint64_t)N * t / T, i1 = (uint64_t)N * (t + 1) / T;
            // room for this thread's share of every block with sources drawn uniformly (a
            // bucket that outgrows it still grows)
            const double share = (double)p.E / T / SB;
            for (uint32_t b = 0; b < SB; b++) bucket[(size_t)t * SB + b].reserve((size_t)(1.15 * share) + 256);
            std::vector<uint32_t> src(kmax);
            std::vector<float> w0(kmax), w1(kmax);
            std::vector<uint8_t> dl(kmax);
            std::vector<unsigned char> scratch(scratch_bytes);
            for (uint64_t i = i0; i < i1; i++) {
                const uint32_t m = mem.member_of(i);
                const uint64_t base = mem.nbase[m];
                const int64_t k = dbnet_in_edges(&mem.m[m], (uint32_t)(i - base), src.data(), w0.data(), w1.data(),
                                                 dl.data(), scratch.data());
                if (k < 0) {
                    gen_fail.store(1);
                    return;
                }
                for (int64_t e = 0; e < k; e++) {
                    const uint32_t s = (uint32_t)(src[e] + base);
                    BucketEdge be;
                    be.src_dl = ((s % bsz) << 8) | dl[e];
                    be.tgt = (uint32_t)i;
                    std::memcpy(&be.w0, &w0[e], 4);
                    std::memcpy(&be.w1, &w1[e], 4);
                    if (!(std::fabs((double)w0[e]) < wlim) || !(std::fabs((double)w1[e]) < wlim)) wbad.store(1);
                    bucket[(size_t)t * SB + s / bsz].push_back(be);
                }
            }
        };
        for (unsigned t = 1; t < T; t++) th.emplace_back(gen, t);
        gen(0);
        for (auto& x : th) x.join();
        if (gen_fail.load()) return "network generator failed";
        if (wbad.load()) return "a weight is too large for the fixed-point format (|w| * 2^frac_bits must stay below 2^52)";
        std::vector<uint64_t> bbase((size_t)SB + 1, 0ull); // first edge of every source block
        for (uint32_t b = 0; b < SB; b++) {
            uint64_t n = 0;
            for (unsigned t = 0; t < T; t++) n += bucket[(size_t)t * SB + b].size();
            bbase[b + 1] = bbase[b] + n;
        }
        if (bbase[SB] != p.E) return "internal error: transposed edge count mismatch";
        h.row_ptr.assign((size_t)N + 1, 0ull);
        h.seg.assign((size_t)N * (D + 1), 0u);
        h.edge.reset(new uint32_t[(size_t)p.E * RW]);
        h.edge_words = (size_t)p.E * RW;
        std::atomic<int> too_big{0};
        parallel_chunks(SB, 1, nt, [&](unsigned, uint64_t b0, uint64_t b1) {
            std::vector<uint64_t> cur;
            for (uint64_t b = b0; b < b1; b++) {
                const uint32_t j0 = (uint32_t)(b * bsz), j1 = std::min<uint32_t>(N, j0 + bsz);
                const uint32_t nj = j1 - j0;
                cur.assign((size_t)nj * D, 0ull);
                for (unsigned t = 0; t < T; t++)
                    for (const BucketEdge& be : bucket[(size_t)t * SB + b]) cur[(size_t)(be.src_dl >> 8) * D + (be.src_dl & 0xFF) - 1]++;
                uint64_t pos = bbase[b];
                for (uint32_t jl = 0; jl < nj; jl++) {
                    const uint32_t j = j0 + jl;
                    h.row_ptr[j] = pos;
                    uint32_t* sg = &h.seg[(size_t)j * (D + 1)];
                    uint64_t acc = 0;
                    sg[0] = 0;
                    for (uint32_t x = 0; x < D; x++) {
                        const uint64_t c = cur[(size_t)jl * D + x];
                        cur[(size_t)jl * D + x] = pos + acc; // cursor of (j, delay x + 1)
                        acc += c;
                        sg[x + 1] = (uint32_t)acc;
                    }
                    if (acc >= (1ull << 32)) too_big.store(1);
                    pos += acc;
                }
                for (unsigned t = 0; t < T; t++)
                    for (const BucketEdge& be : bucket[(size_t)t * SB + b]) {
                        const uint64_t e = cur[(size_t)(be.src_dl >> 8) * D + (be.src_dl & 0xFF) - 1]++;
                        uint32_t* rec = &h.edge[e * RW];
                        rec[KW] = be.tgt | ((uint32_t)h.src_inh[j0 + (be.src_dl >> 8)] << 31);
                        rec[0] = be.w0;
                        if (KW == 2) rec[1] = be.w1;
                    }
                for (unsigned t = 0; t < T; t++) std::vector<BucketEdge>().swap(bucket[(size_t)t * SB + b]);
            }
        });
        if (too_big.load()) return "out-degree too large";
        h.row_ptr[N] = p.E;
    } else {
        // Two generation passes for networks whose buckets would not fit in host memory:
        // count per (source, delay), then fill through atomic cursors, then sort every
        // delay segment by target.
        std::unique_ptr<std::atomic<uint32_t>[]> cnt(new std::atomic<uint32_t>[(size_t)N * D]);
        for (size_t x = 0; x < (size_t)N * D; x++) cnt[x].store(0, std::memory_order_relaxed);
        parallel_chunks(N, 256, nt, [&](unsigned, uint64_t a, uint64_t b) {
            std::vector<uint32_t> src(kmax);
            std::vector<uint8_t> dl(kmax);
            std::vector<unsigned char> scratch(scratch_bytes);
            for (uint64_t i = a; i < b; i++) {
                const uint32_t m = mem.member_of(i);
                const uint64_t base = mem.nbase[m];
                const int64_t k = dbnet_in_edges(&mem.m[m], (uint32_t)(i - base), src.data(), nullptr, nullptr, dl.data(),
                                                 scratch.data());
                if (k < 0) {
                    gen_fail.store(1);
                    return;
                }
                for (int64_t e = 0; e < k; e++)
                    cnt[(size_t)(src[e] + base) * D + dl[e] - 1].fetch_add(1, std::memory_order_relaxed);
            }
        });
        if (gen_fail.load()) return "network generator failed";
        h.row_ptr.assign((size_t)N + 1, 0ull);
        h.seg.assign((size_t)N * (D + 1), 0u);
        for (uint32_t j = 0; j < N; j++) {
            uint64_t acc = 0;
            uint32_t* sg = &h.seg[(size_t)j * (D + 1)];
            sg[0] = 0;
            for (uint32_t x = 0; x < D; x++) {
                acc += cnt[(size_t)j * D + x].load(std::memory_order_relaxed);
                sg[x + 1] = (uint32_t)acc;
            }
            if (acc >= (1ull << 32)) return "out-degree too large";
            h.row_ptr[j + 1] = h.row_ptr[j] + acc;
        }
        if (h.row_ptr[N] != p.E) return "internal error: transposed edge count mismatch";
        // pass 2: fill rows (cursor per (source, delay))
        std::unique_ptr<std::atomic<uint64_t>[]> cur(new std::atomic<uint64_t>[(size_t)N * D]);
        for (uint32_t j = 0; j < N; j++)
            for (uint32_t x = 0; x < D; x++)
                cur[(size_t)j * D + x].store(h.row_ptr[j] + h.seg[(size_t)j * (D + 1) + x], std::memory_order_relaxed);
        cnt.reset();
            h.edge.reset(new uint32_t[(size_t)p.E * RW]);
            h.edge_words = (size_t)p.E * RW;
            parallel_chunks(N, 256, nt, [&](unsigned, uint64_t a, uint64_t b) {
            std::vector<uint32_t> src(kmax);
            std::vector<float> w0(kmax), w1(kmax);
            std::vector<uint8_t> dl(kmax);
            std::vector<unsigned char> scratch(scratch_bytes);
            for (uint64_t i = a; i < b; i++) {
                const uint32_t m = mem.member_of(i);
                const uint64_t base = mem.nbase[m];
                const int64_t k = dbnet_in_edges(&mem.m[m], (uint32_t)(i - base), src.data(), w0.data(), w1.data(),
                                                 dl.data(), scratch.data());
                if (k < 0) {
                    gen_fail.store(1);
                    return;
                }
                for (int64_t e = 0; e < k; e++) {
                    const uint64_t pos = cur[(size_t)(src[e] + base) * D + dl[e] - 1].fetch_add(1, std::memory_order_relaxed);
                    uint32_t* rec = &h.edge[pos * RW];
                    rec[KW] = (uint32_t)i | ((uint32_t)h.src_inh[src[e] + base] << 31);
                    std::memcpy(&rec[0], &w0[e], 4);
                    if (KW == 2) std::memcpy(&rec[1], &w1[e], 4);
                    if (!(std::fabs((double)w0[e]) < wlim) || !(std::fabs((double)w1[e]) < wlim)) wbad.store(1);
                }
            }
        });
        if (gen_fail.load()) return "network generator failed";
        if (wbad.load()) return "a weight is too large for the fixed-point format (|w| * 2^frac_bits must stay below 2^52)";
        cur.reset();
        // deterministic layout: sort every delay segment by target (tile groups are ranges of
        // consecutive targets, so each delay segment splits into contiguous group sub-segments)
        parallel_chunks(N, 1024, nt, [&](unsigned, uint64_t a, uint64_t b) {
            struct Ed {
                uint32_t t, w0, w1; // target and the weights' bit patterns
            };
            std::vector<Ed> tmp;
            for (uint64_t j = a; j < b; j++) {
                const uint32_t* sg = &h.seg[(size_t)j * (D + 1)];
                for (uint32_t x = 0; x < D; x++) {
                    const uint64_t s0 = h.row_ptr[j] + sg[x], s1 = h.row_ptr[j] + sg[x + 1];
                    if (s1 - s0 < 2) continue;
                    tmp.resize(s1 - s0);
                    for (uint64_t e = s0; e < s1; e++)
                        tmp[e - s0] = Ed{h.edge[e * RW + KW], h.edge[e * RW], KW == 2 ? h.edge[e * RW + 1] : 0u};
                    std::sort(tmp.begin(), tmp.end(), [](const Ed& A, const Ed& B) { return A.t < B.t; });
                    for (uint64_t e = s0; e < s1; e++) {
                        h.edge[e * RW + KW] = tmp[e - s0].t;
                        h.edge[e * RW] = tmp[e - s0].w0;
                        if (KW == 2) h.edge[e * RW + 1] = tmp[e - s0].w1;
                    }
                }
            }
        });
    }
    // row headers
    h.hdr.assign((size_t)N * p.HW, 0u);
    for (uint32_t j = 0; j < N; j++) {
        uint32_t* hp = &h.hdr[(size_t)j * p.HW];
        const uint64_t rs = h.row_ptr[j] | ((uint64_t)h.src_inh[j] << 63);
        hp[0] = (uint32_t)rs;
        hp[1] = (uint32_t)(rs >> 32);
        for (uint32_t x = 0; x <= D; x++) hp[2 + x] = h.seg[(size_t)j * (D + 1) + x];
    }
    return "";
}

} // namespace dbs
