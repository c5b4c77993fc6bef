// dbsim_internal.hpp - device data layout and kernel interfaces of libdbsim.
//
// Layout in HBM (one handle):
//   neuron state, structure of arrays: V f32[N], J f32[U][N] (receptor-major),
//     ref u8[N] (refractory steps left), pend u8[N] (spike substep carried
//     across a bin split over two step calls), A f32[U][N] (arrival sums of the
//     current bin, already converted from fixed point);
//   populations: PopParams[n_pops] and Poisson thresholds u32[n_pops][kMaxPoisson];
//     neuron blocks never straddle populations, so a block's parameters are
//     uniform (scalar registers);
//   connection table by presynaptic neuron (Suppl. Table 5's table is stored
//     by target; the push-based fan-out of Suppl. Algorithm 2 wants it by
//     source): one record of 1 + KW words per edge (the weights, then target |
//     source class << 31, the fan-in's event key; weights first, so a whole-record
//     load puts them in an aligned register pair),
//     so that a (spike, delay) segment is one contiguous run; rows sorted by
//     delay, then target; one row header per neuron, hdr u32[N][HW]
//     (HW = D + 3 rounded up to 4 words: the row start as u64 with the source
//     class in bit 63, then the D + 1 delay segment offsets inside the row), so
//     that one 64-byte read gives everything a (spike, delay) segment needs;
//   the event arena of the fan-in. Single-pass form (on request, where the tiles'
//     carry buffers fit a workgroup's LDS): blocks of kFanBlock records, a 16-bit key
//     array (target within the tile | inhibitory source << 15) beside the weights; tile
//     t owns blocks tile_base[t] .. tile_base[t+1]: its in-degree in whole blocks (the
//     most events a tile can receive in one bin: an edge delivers at most once per bin)
//     plus two part-filled blocks per workgroup and bin (each workgroup and pass leaves
//     at most one). Two-pass form: the same 16-bit keys beside the weights, tile t's
//     slice tile_base[t] .. tile_base[t+1] a share of its in-edges, the events past a
//     full slice summed in the per-target overflow sums ovf; the super-tile streams
//     (slices of a share of each super-tile's in-edges) hold records of 1 + KW words
//     (target | source class << 31, then the weights) or the narrow form below;
//   spike history: rec u32[RC] ring of (id << 4 | substep), per-bin start u64[MB]
//     and count u32[MB] (rings indexed by bin & (MB-1));
//   region readout: per-block partial sums f64/u32, per-region block lists,
//     and a ring of MB bins of region signal f64[MB][n_regions] and counts;
//   region BOLD: per-region activity scale f64[n_regions], Balloon-Windkessel state
//     f64[4][n_regions] and a ring of kBoldRing samples f64[kBoldRing][n_regions];
//   ctl: bin counter, delivered-event counter, sticky error bits.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "dbnet.h"

namespace dbs {

constexpr int kMaxPoisson = 64;       // Poisson thresholds per population
constexpr int kNeuronBlock = 256;     // neurons per block of the neuron kernel
constexpr int kScatterThreads = 512;  // threads per block of the partition kernels (several blocks per CU)
constexpr int kScatterSegs = 512;     // (spike, delay) segments per partition chunk (one per thread)
constexpr int kGatherThreads = 1024;
constexpr int kMaxTilesLds = 16384;   // most tiles (at most 256 buckets in the second partition pass)
constexpr uint32_t kTileLdsBytes = 128u * 1024u; // LDS accumulator per tile
constexpr uint32_t kErrArena = 1u;    // single-pass block arena overflow (cannot happen by construction)
constexpr uint32_t kErrLayout = 2u;   // a table entry outside its tile group (cannot happen by construction)
constexpr uint32_t kMaxSuperTiles = 64; // buckets of the first partition pass
constexpr uint32_t kStreamPermille = 125; // default stream slice: 1/8 of the super-tile's in-edges,
constexpr uint64_t kStreamFloor = 1ull << 20; // and at least this many records (or all of them)
constexpr uint32_t kArenaPermille = 125;  // default tile arena slice: 1/8 of the tile's in-edges,
constexpr uint64_t kArenaFloor = 1ull << 16; // and at least this many records (or all of them)
constexpr uint32_t kBoldRing = 1024;     // BOLD samples kept per region (power of two)
constexpr int kLoadBatch = 8;          // gather: records loaded per thread before they are consumed
constexpr int kMaxBatch = 8;           // partition: events per thread per round
constexpr uint32_t kMaxPartGrid = 2048; // most partition workgroups
constexpr int kFanThreads = 1024;       // threads per workgroup of the single-pass fan-in
constexpr uint32_t kFanBlock = 256;     // records per block of the single-pass event arena
constexpr uint32_t kFanMaxGrid = 512;   // most single-pass workgroups (bounds the part-filled blocks)
constexpr uint32_t kFanMinChunk = 4, kFanMaxChunk = 64; // records per carry buffer (power of two)
constexpr uint32_t kMaxLdsBytes = 160u * 1024u;
constexpr uint32_t kStaticLds = 1024u; // room left per workgroup for the kernels' static LDS

struct PopParams {
    float k;      // dt / C
    float gL, VL, Vth, Vr, Iext, wbg;
    float g[4], Vu[4], dec[4]; // compact receptor order (AMPA, [NMDA], GABA_A, [GABA_B])
    int32_t r;                  // refractory steps
    int32_t cmax;               // Poisson table length
    uint32_t end;               // one past the population's last neuron id
    uint32_t region;
    uint32_t net_id;            // noise stream of the population's network
    uint32_t id_base;           // global id of its network's first neuron (noise counters use local ids)
    unsigned long long seed;    // its network's seed (Philox key)
    uint32_t inject_t;          // injected output spike when a Philox word < inject_t (0: none)
    uint32_t ou_on;             // Ornstein-Uhlenbeck background current on
    float ou_mu;                // its mean (pA)
    float ou_c1, ou_c2;         // dt / tau and sigma * sqrt(2 dt / tau), rounded once
    uint32_t pad;
};

struct Ctl {
    unsigned long long bin;         // bin being processed (advanced at the bin close)
    unsigned long long edge_events; // delivered synaptic events
    unsigned long long spikes;      // spikes emitted in closed bins
    unsigned int err;               // sticky error bits
    unsigned int pad1;
    unsigned long long ahead_events; // events of the next bin assembled ahead, not yet delivered
    unsigned int pad0;
    unsigned long long bnext;        // next k_bucket round to hand out (work queue)
    unsigned long long pnext;        // next k_part chunk to hand out (work queue)
    unsigned long long inject_until; // output spikes are injected in bins below this one
    unsigned long long spilled;      // partitioned events whose super-tile stream was full
    unsigned long long overflow;     // events whose tile arena slice was full (summed in ovf)
};

struct DevNet {
    uint32_t N, U, KW, S, D, F;
    uint32_t tile_bits, T, n_blocks, n_regions;
    uint32_t blocked;      // 1: single-pass fan-in (k_fan into tile blocks), 0: two passes
    uint32_t NS;           // super-tiles (buckets of k_part in the two-pass form; 0 otherwise)
    uint32_t ts_bits;      // log2(tiles per super-tile)
    uint32_t HW;           // words per row header
    uint32_t round_events; // events staged in LDS per partition round (k_part)
    uint32_t bucket_events; // events per round of the second pass (k_bucket)
    uint32_t chunks_per_wg; // target scatter chunks per workgroup and bin
    uint32_t ahead_passes;  // partition passes of the next bin's delay >= 2 fan-in (two-pass form)
    uint32_t fan_C;         // single-pass form: records per carry buffer
    uint32_t fan_K;         // single-pass form: records per block
    uint32_t narrow;        // two-pass form: 10-byte stream records (sevk beside sevw)
    uint64_t RCmask;
    uint32_t MBmask;
    double qscale;   // 2^F
    float qinv;      // 2^-F
    uint32_t regions_on;
    // state
    float* V;
    float* J;
    uint8_t* ref;
    uint8_t* pend;
    float* A;
    float* Iou; // Ornstein-Uhlenbeck background current per neuron (populations with it on)
    // populations and neuron blocks
    const PopParams* pops;
    const uint32_t* ptab;
    const uint2* blk; // (first neuron, population)
    // connection table
    const uint32_t* hdr;  // [N][HW] row headers
    const uint32_t* edge; // [E][1 + KW] records: the weights, then target | inhibitory source << 31
    // event arena: keys evk (target within tile | inhibitory source << 15) beside the weights
    // ev (KW floats per record). Two-pass form: tile t's slice tile_base[t] .. tile_base[t+1],
    // tile_fill[t] records reserved this bin, tile_fill[T + t] the complement of the first
    // reservation that did not fit (0: none), whose events were summed into ovf (int64 fixed
    // point, [N][U], zero again after the tile's gather). Single-pass form: blocks of fan_K
    // records; tile t owns blocks tile_base[t] .. tile_base[t+1], tile_fill[t] of them taken
    // this bin, bcnt[b] records in b.
    uint32_t* ev;
    uint16_t* evk;
    uint32_t* bcnt;
    unsigned long long* ovf;
    const uint64_t* tile_base;
    uint32_t* tile_fill;
    const uint64_t* st_base; // super-tile stream slices [NS + 1]
    uint32_t* st_fill;       // [2 NS] records reserved per super-tile this pass, then the
                             // complement of the first reservation that did not fit (0: none)
    uint32_t* sev;           // super-tile stream records: (target | source class << 31, weights)
    // or, narrow (every weight non-negative, two weights per edge): a 16-bit key array sevk
    // (target within the super-tile, low 16 bits) beside the weight pairs sevw, whose sign
    // bits carry the source class (w0) and the key's bit 16 (w1); slices start at even records
    uint16_t* sevk;
    uint2* sevw;
    // spikes: per-block staging (256 slots per neuron block), per-group counts (two bin
    // parities x groups of 256 blocks), then the dense history ring
    uint32_t* stage;
    uint32_t* grp_cnt;
    uint32_t n_grp;
    uint32_t* rec;
    unsigned long long* bin_start;
    uint32_t* bin_cnt;
    // host recording (pinned host memory, written by k_drain): ring of spike entries at the
    // same offsets as rec (mod HCmask + 1), and the end offset of every bin k at (k + 1) & HMBmask
    uint32_t* hrec;
    unsigned long long* hbend;
    uint64_t HCmask;
    uint32_t HMBmask;
    // regions
    double* blk_sig;
    uint32_t* blk_cnt;
    const uint32_t* reg_blk_ptr;
    const uint32_t* reg_blk;
    const uint32_t* reg_size;
    const uint32_t* l1_ptr;    // first level-1 readout group of each region [n_regions + 1]
    const uint32_t* l1_region; // region of each level-1 group [n_l1]
    double* l1_sig;
    uint32_t* l1_cnt;
    uint32_t n_l1;
    double* sig;
    uint32_t* sig_cnt;
    // region BOLD (Balloon-Windkessel, Extended Data Table 4), stepped at every bin end
    uint32_t bold_on, tr_bins;
    double bw_h, bw_htau, bw_kappa, bw_gamma, bw_inv_alpha, bw_rho, bw_V0, bw_k1, bw_k2, bw_k3;
    const double* bold_zs;           // per region: activity_scale / (N_r * h)
    double* bold;                    // [4][n_regions]: s, f, v, q
    double* bold_y;                  // [kBoldRing][n_regions] samples
    unsigned long long* bold_ctl;    // [0] bins since enabled, [1] samples taken
    Ctl* ctl;
};

// kernel launchers (kernels.hip); each enqueues on `st` and returns the launch status
hipError_t prepare_kernels(); // one-time function attributes (LDS opt-in); call outside graph capture
// fan-in of the delays d_lo..d_hi of the current bin (ahead = 0) or of the next one (ahead = 1)
hipError_t launch_scatter(const DevNet& n, int grid, hipStream_t st, uint32_t d_lo, uint32_t d_hi, uint32_t ahead);
// the two halves of launch_scatter in the two-pass form: the partition into the super-tile
// streams (k_part), and their bucketing into the tile arena (k_bucket)
hipError_t launch_part(const DevNet& n, int grid, hipStream_t st, uint32_t d_lo, uint32_t d_hi, uint32_t ahead);
hipError_t launch_bucket(const DevNet& n, int grid, hipStream_t st);
hipError_t launch_gather(const DevNet& n, hipStream_t st);
hipError_t launch_pass_reset(const DevNet& n, hipStream_t st);
hipError_t launch_neuron(const DevNet& n, int s0, int s1, hipStream_t st);
hipError_t launch_compact(const DevNet& n, hipStream_t st);
hipError_t launch_drain(const DevNet& n, hipStream_t st);
// per-population mean current per receptor at the current state: rblk [n_blocks][4] scratch,
// rpop [n_pops][4] result (paper receptor order)
hipError_t launch_receptor_currents(const DevNet& n, uint32_t n_pops, double* rblk, double* rpop, hipStream_t st);
hipError_t launch_readout_close(const DevNet& n, hipStream_t st);
size_t part_lds_bytes(uint32_t nb, uint32_t RE, uint32_t D);
size_t fan_lds_bytes(uint32_t T, uint32_t C, uint32_t KW, uint32_t D);
size_t bucket_lds_bytes(uint32_t TS, uint32_t RE);
size_t gather_lds_bytes(const DevNet& n);

} // namespace dbs
