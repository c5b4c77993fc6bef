// netbuild.hpp - host-side construction of the device tables from descriptions.
//
// A handle simulates one network or an ensemble of independent networks
// ("members"). Members are laid out one after another: member m owns global
// neuron ids nbase[m] .. nbase[m+1]-1, populations pbase[m].., regions rbase[m]..
// Edges never cross members, and each member keeps its own seed and noise
// stream, so its results do not depend on the other members.
#pragma once

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "dbnet.h"
#include "dbsim.h"
#include "dbsim_internal.hpp"
#include "devgen.hpp"

namespace dbs {

// Deep copies of the member descriptions (the dbnet_desc pointers point into them).
struct Members {
    std::vector<dbnet_desc> m;
    std::vector<std::vector<dbnet_pop>> pops;
    std::vector<std::vector<dbnet_proj>> projs;
    std::vector<std::vector<float>> xyz;
    std::vector<uint64_t> nbase; // [M+1] first global neuron of each member
    std::vector<uint32_t> pbase; // [M+1] first global population
    std::vector<uint32_t> rbase; // [M+1] first global region
    void assign(const dbnet_desc* descs, uint32_t n);
    uint32_t member_of(uint64_t i) const;
};

// Sizes derived from the descriptions without generating the networks.
struct Plan {
    uint32_t N = 0, U = 0, KW = 0, S = 0, D = 0, F = 0;
    uint32_t tile_bits = 0, T = 0, n_blocks = 0, n_regions = 0, n_pops = 0, n_members = 0;
    uint32_t MB = 0;    // bins kept in the per-bin rings (power of two)
    uint32_t n_l1 = 0;  // level-1 readout groups (256 neuron blocks each, per region)
    uint32_t n_grp = 0; // compaction groups (256 consecutive neuron blocks each)
    bool blocked = false;         // single-pass fan-in into tile blocks (else two passes)
    bool narrow = false;          // two-pass form with 10-byte stream records
    uint32_t st_permille = 0;     // stream slice per super-tile, in thousandths of its in-edges
    std::vector<uint64_t> st_len; // records of every super-tile's stream slice [NS]
    uint64_t st_total = 0;        // their sum
    uint64_t st_cap = 0;          // narrow: stream record capacity (the slices and a margin)
    uint32_t ta_permille = 0;     // tile arena slice, in thousandths of the tile's in-edges
    std::vector<uint64_t> ta_len; // records of every tile's arena slice [T] (two-pass form)
    uint64_t ta_total = 0;        // their sum
    uint32_t NS = 0, ts_bits = 0; // super-tiles, log2(tiles per super-tile) of the two-pass form
    std::vector<uint64_t> tile_blk; // single-pass form: first block of every tile [T + 1]
    uint32_t HW = 0;              // words per row header
    uint32_t round_events = 0, bucket_events = 0, scatter_wgs_per_cu = 0;
    uint64_t RC = 0; // spike-history ring entries (power of two)
    bool host_record = false; // every bin's spikes are copied to a pinned host ring
    uint64_t HC = 0;          // host ring entries (power of two)
    uint32_t HMB = 0;         // bins of offsets kept beside it (power of two)
    uint64_t E = 0;  // edges
    bool regions_on = false;
    // connection table built on the device (else on the host): the temporaries live in the
    // tile arena (counts, cursors, row lengths, tie-breaks, the generator's tables) and the
    // super-tile streams (per-thread generator scratch, gen_batch targets at a time)
    bool dev_build = false;
    uint32_t gen_batch = 0;
    struct GenLayout {
        size_t tables = 0, cnt = 0, cur = 0, rowlen = 0, rowptr = 0, sums = 0, tb = 0, flags = 0, end = 0;
    } gl;
    // byte offsets of every device array inside one allocation
    struct Slot {
        size_t off = 0, bytes = 0;
    };
    Slot V, J, ref, pend, A, Iou, pops, ptab, blk, hdr, edge, ev, evk, bcnt, ovf, tile_base, tile_fill, st_base, st_fill,
        sev, stage,
        grp_cnt, rec, bin_start, bin_cnt, blk_sig, blk_cnt, reg_blk_ptr, reg_blk, reg_size, l1_ptr, l1_region, l1_sig,
        l1_cnt, sig, sig_cnt, bold_zs, bold, bold_y, bold_ctl, rblk, rpop, ctl;
    size_t total = 0;
};

// Largest multiple of kScatterThreads events (at most 4096) a round of the two-pass form can
// stage in LDS (0 if none fits); the single-pass form keeps its rounds in registers (at most
// kMaxBatch * kFanThreads events).
uint32_t max_round_events(const Plan& p, uint32_t wgs_per_cu);
uint32_t max_bucket_events(const Plan& p, uint32_t wgs_per_cu);
// Single-pass form: the largest carry buffer (records per tile, a power of two in
// kFanMinChunk .. kFanMaxChunk) whose LDS fits wgs_per_cu workgroups per CU (0 if none).
uint32_t fan_chunk_records(const Plan& p, uint32_t wgs_per_cu);

// Validates the runtime options and the members for this simulator and fills the plan.
// Returns an empty string on success, else the reason.
std::string make_plan(const dbsim_desc& opts, const Members& mem, Plan& p);

// Host images of every device table.
struct HostTables {
    std::vector<float> V0;
    std::vector<PopParams> pops;
    std::vector<uint32_t> ptab;
    std::vector<uint2> blk;
    std::vector<uint64_t> row_ptr;
    std::vector<uint32_t> seg; // [N][D+1] delay segments
    // [E][1 + KW]: target, then the weights (bit patterns); left uninitialised at allocation
    // so that the parallel placement threads touch its pages first
    std::unique_ptr<uint32_t[]> edge;
    size_t edge_words = 0;
    std::vector<uint8_t> src_inh;
    std::vector<uint32_t> hdr; // [N][HW] device row headers
    std::vector<uint64_t> tile_base, st_base;
    std::vector<uint32_t> reg_blk_ptr, reg_blk, reg_size, l1_ptr, l1_region;
    // the generator's tables for the device construction (plan.dev_build)
    std::vector<GenPop> gpops;
    std::vector<GenMember> gmembers;
    std::vector<GenProj> gprojs;
    std::vector<GenCand> gcands;
    std::vector<GenCandPop> gcpops;
    std::vector<uint8_t> gdtab;
    uint32_t gkmax = 0, ghcap = 0;
};

// The generator's tables of the members for the device construction. Returns an empty
// string, or why the device construction does not apply (lognormal weights).
std::string make_gen_tables(const Members& mem, HostTables& h);
// Bytes of the tables as laid out in device memory (each array 256-byte aligned).
size_t gen_tables_bytes(const HostTables& h);
// u32 words of generator scratch per target thread.
inline uint32_t gen_scratch_words(uint32_t kmax, uint32_t hcap) { return hcap + 3u * kmax + 1u; }

// Per-population parameters and derived constants of the plan's populations (members one
// after another): PopParams and the Poisson thresholds [n_pops][kMaxPoisson]; optionally the
// first global neuron of every population [n_pops + 1] and its in-degree. Host only.
void fill_populations(const Members& mem, const Plan& p, std::vector<PopParams>& pops, std::vector<uint32_t>& ptab,
                      std::vector<uint64_t>* first, std::vector<uint32_t>* indeg);

// Builds every host table (threads: 0 = all cores); the connection table (edge records and
// row headers) too when with_edges, else the generator's tables for the device construction.
// Returns an empty string on success, else the reason.
std::string build_tables(const Members& mem, const Plan& p, unsigned threads, HostTables& h, bool with_edges);

} // namespace dbs
