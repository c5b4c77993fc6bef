// abi.cpp - the C ABI of libdbsim: handle lifecycle, the bin driver (direct
// launches or replayed HIP graphs), recording reads and error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "dbsim.h"
#include "dbsim_internal.hpp"
#include "netbuild.hpp"

using namespace dbs;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (dev >= 0 && hipGetDevice(&prev) == hipSuccess && prev != dev) {
            if (hipSetDevice(dev) != hipSuccess) prev = -1;
        } else {
            prev = -1;
        }
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

constexpr int kGraphBins = 8; // bins captured in one replayable graph
constexpr int kPhases = 4;    // reported phases: scatter (partition), gather, neuron, bin end
constexpr int kMarks = 7;     // events per timed bin (six intervals, see resolve_timers)

} // namespace

// Device memory of the handles made by dbsim_create_static: one region per GPU, held from the
// library's load to the end of the process. In host code the array's name is only a host-side
// stand-in, so its device address is looked up once per device (static_region_of) and only
// that address is used afterwards (kernel arguments, copies, fills).
static __device__ __align__(256) unsigned char scratch[DBSIM_STATIC_BYTES];

namespace {
constexpr int kStaticDevices = 64;
std::mutex g_static_mu;
unsigned char* g_static_ptr[kStaticDevices] = {};
bool g_static_busy[kStaticDevices] = {};
} // namespace

// The region's device address on `device` (current device set by the caller); nullptr with
// *err set when the lookup fails.
static unsigned char* static_region_of(int device, hipError_t* err) {
    *err = hipSuccess;
    if (!g_static_ptr[device]) {
        void* ptr = nullptr;
        *err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (*err != hipSuccess || !ptr) {
            if (*err == hipSuccess) *err = hipErrorInvalidSymbol;
            return nullptr;
        }
        g_static_ptr[device] = static_cast<unsigned char*>(ptr);
    }
    return g_static_ptr[device];
}

// The kernels' LDS limits are set once per device and process, not at every create:
// handles are created on host threads while other handles' kernels are being launched and
// captured, and a set that is already in place needs no repeating.
static hipError_t prepare_kernels_once(int device) {
    static std::mutex mu;
    static std::set<int> done;
    std::lock_guard<std::mutex> lock(mu);
    if (done.count(device)) return hipSuccess;
    const hipError_t e = prepare_kernels();
    if (e == hipSuccess) done.insert(device);
    return e;
}

struct dbsim {
    dbsim_desc desc{};
    Members mem;
    Plan plan;
    int device = -1;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t cap_stream = nullptr;
    hipStream_t side_stream = nullptr; // the next bin's delay >= 2 fan-in, beside the neuron step
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipStream_t drain_stream = nullptr; // copies each bin's spikes to the pinned host ring
    hipEvent_t ev_dfork = nullptr, ev_djoin = nullptr;
    uint32_t* hrec = nullptr;             // pinned host ring of spike entries (host recording)
    unsigned long long* hbend = nullptr;  // pinned: end offset of bin k at (k + 1) & (HMB - 1)
    unsigned char* dev = nullptr;
    bool static_mem = false; // dev is the device's static region (dbsim_create_static)
    DevNet net{};
    int scatter_grid = 256;
    int num_cus = 256;
    uint32_t scatter_wgs = 1;
    hipGraphExec_t g_multi = nullptr;
    hipGraphExec_t g_one = nullptr;
    uint64_t step = 0;
    uint64_t first_bin = 0; // first bin whose spikes and region signal can be read (restores)
    int dead = 0; // sticky error code
    bool timing = false;
    std::vector<std::array<hipEvent_t, kMarks>> ev_pending;
    std::vector<std::array<hipEvent_t, kMarks>> ev_pool;
    double ms[kPhases] = {0, 0, 0, 0};
    uint64_t timed_bins = 0;
    double build_seconds = 0.0;
    bool device_built = false; // the connection table was generated on the device
    hipEvent_t ev_build[2] = {nullptr, nullptr}; // around the device construction, until timed
};

// A network built on the host and not yet deployed (dbsim_build -> dbsim_create_built).
struct dbsim_built {
    dbsim_desc desc{};
    Members mem;
    Plan plan;
    HostTables ht;
    double build_seconds = 0.0;
    bool in_static = false;
};

namespace {

int hip_fail(dbsim* h, hipError_t e, const char* what) {
    if (h) h->dead = DBSIM_EDEVICE;
    return fail(DBSIM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(h, x, what)                                                                                             \
    do {                                                                                                               \
        hipError_t e_ = (x);                                                                                           \
        if (e_ != hipSuccess) return hip_fail((h), e_, (what));                                                        \
    } while (0)

template <class T>
T* at(unsigned char* base, const Plan::Slot& s) {
    return reinterpret_cast<T*>(base + s.off);
}

// One pass: each further pass costs about 80 us of fill and drain on the 6.1 M share and
// no cache retention of the smaller streams was measurable.
uint32_t default_ahead_passes(const Plan&) { return 1u; }

void fill_devnet(dbsim* h) {
    const Plan& p = h->plan;
    unsigned char* b = h->dev;
    DevNet& n = h->net;
    n.N = p.N;
    n.U = p.U;
    n.KW = p.KW;
    n.S = p.S;
    n.D = p.D;
    n.F = p.F;
    n.tile_bits = p.tile_bits;
    n.blocked = p.blocked ? 1u : 0u;
    n.NS = p.NS;
    n.ts_bits = p.ts_bits;
    n.HW = p.HW;
    n.round_events = p.round_events;
    n.bucket_events = p.bucket_events;
    n.chunks_per_wg = 4;
    n.fan_K = kFanBlock;
    n.fan_C = p.blocked ? fan_chunk_records(p, p.scatter_wgs_per_cu) : 0u;
    n.ahead_passes = default_ahead_passes(p);
    n.T = p.T;
    n.n_blocks = p.n_blocks;
    n.n_regions = p.n_regions;
    n.RCmask = p.RC - 1;
    n.MBmask = p.MB - 1;
    n.qscale = std::ldexp(1.0, (int)p.F);
    n.qinv = std::ldexp(1.0f, -(int)p.F);
    n.regions_on = p.regions_on ? 1u : 0u;
    n.V = at<float>(b, p.V);
    n.J = at<float>(b, p.J);
    n.ref = at<uint8_t>(b, p.ref);
    n.pend = at<uint8_t>(b, p.pend);
    n.A = at<float>(b, p.A);
    n.Iou = at<float>(b, p.Iou);
    n.pops = at<const PopParams>(b, p.pops);
    n.ptab = at<const uint32_t>(b, p.ptab);
    n.blk = at<const uint2>(b, p.blk);
    n.hdr = at<const uint32_t>(b, p.hdr);
    n.edge = at<const uint32_t>(b, p.edge);
    n.ev = at<uint32_t>(b, p.ev);
    n.evk = at<uint16_t>(b, p.evk);
    n.bcnt = at<uint32_t>(b, p.bcnt);
    n.tile_base = at<const uint64_t>(b, p.tile_base);
    n.ovf = at<unsigned long long>(b, p.ovf);
    n.tile_fill = at<uint32_t>(b, p.tile_fill);
    n.st_base = at<const uint64_t>(b, p.st_base);
    n.st_fill = at<uint32_t>(b, p.st_fill);
    n.sev = at<uint32_t>(b, p.sev);
    n.narrow = p.narrow ? 1u : 0u;
    n.sevk = reinterpret_cast<uint16_t*>(b + p.sev.off);
    n.sevw = reinterpret_cast<uint2*>(b + p.sev.off + ((2 * (size_t)p.st_cap + 255) & ~(size_t)255));
    n.stage = at<uint32_t>(b, p.stage);
    n.grp_cnt = at<uint32_t>(b, p.grp_cnt);
    n.n_grp = p.n_grp;
    n.rec = at<uint32_t>(b, p.rec);
    n.bin_start = at<unsigned long long>(b, p.bin_start);
    n.bin_cnt = at<uint32_t>(b, p.bin_cnt);
    n.hrec = nullptr; // set once the pinned host ring exists
    n.hbend = nullptr;
    n.HCmask = p.HC ? p.HC - 1 : 0;
    n.HMBmask = p.HMB ? p.HMB - 1 : 0;
    n.blk_sig = at<double>(b, p.blk_sig);
    n.blk_cnt = at<uint32_t>(b, p.blk_cnt);
    n.reg_blk_ptr = at<const uint32_t>(b, p.reg_blk_ptr);
    n.reg_blk = at<const uint32_t>(b, p.reg_blk);
    n.reg_size = at<const uint32_t>(b, p.reg_size);
    n.l1_ptr = at<const uint32_t>(b, p.l1_ptr);
    n.l1_region = at<const uint32_t>(b, p.l1_region);
    n.l1_sig = at<double>(b, p.l1_sig);
    n.l1_cnt = at<uint32_t>(b, p.l1_cnt);
    n.n_l1 = p.n_l1;
    n.sig = at<double>(b, p.sig);
    n.sig_cnt = at<uint32_t>(b, p.sig_cnt);
    n.bold_on = 0;
    n.tr_bins = 1;
    n.bold_zs = at<const double>(b, p.bold_zs);
    n.bold = at<double>(b, p.bold);
    n.bold_y = at<double>(b, p.bold_y);
    n.bold_ctl = at<unsigned long long>(b, p.bold_ctl);
    n.ctl = at<Ctl>(b, p.ctl);
}

// Bin schedule. The arrivals due at the start of bin k come from the spikes of bins k-d,
// d = 1..D. Those with d >= 2 only need bins that are already complete while bin k-1's
// neurons are being stepped, so they are assembled then ("ahead", on a side stream when
// the bin runs as a whole); at the start of bin k only the delay-1 part is left. Bin 0
// has nothing to assemble ahead. Order per bin k:
//   start: partition d = 1 (bin k) -> gather (A for bin k)
//   step:  neuron (bin k)                 | side: partition d = 2..D (bin k+1)
//   end:   compact (bin k) -> join side -> readout and bin close (resets the streams)
hipError_t enqueue_bin_start(dbsim* h, hipStream_t st) {
    hipError_t e = launch_scatter(h->net, h->scatter_grid, st, 1, 1, 0);
    if (e != hipSuccess) return e;
    return launch_gather(h->net, st);
}

// The next bin's delay >= 2 fan-in on `st`, after this bin's gather (which empties the
// super-tile streams). Two-pass form: consecutive delay groups, one partition pass
// (k_part + k_bucket) each, with a reset between two passes.
hipError_t enqueue_ahead(dbsim* h, hipStream_t st) {
    const uint32_t D = h->plan.D;
    if (D < 2) return hipSuccess;
    if (h->plan.blocked) return launch_scatter(h->net, h->scatter_grid, st, 2, D, 1);
    const uint32_t P = std::min(h->net.ahead_passes, D - 1);
    hipError_t e = hipSuccess;
    for (uint32_t g = 0; g < P && e == hipSuccess; g++) {
        const uint32_t lo = 2 + (D - 1) * g / P, hi = 1 + (D - 1) * (g + 1) / P;
        if (g > 0) e = launch_pass_reset(h->net, st);
        if (e == hipSuccess) e = launch_scatter(h->net, h->scatter_grid, st, lo, hi, 1);
    }
    return e;
}

hipError_t enqueue_bin_end(dbsim* h, hipStream_t st) {
    hipError_t e = launch_compact(h->net, st);
    if (e == hipSuccess && h->plan.host_record) e = launch_drain(h->net, st);
    if (e == hipSuccess) e = enqueue_ahead(h, st);
    if (e != hipSuccess) return e;
    return launch_readout_close(h->net, st);
}

// One whole bin with the next bin's delay >= 2 fan-in forked onto the side stream right
// after the gather (it touches neither the neuron state nor this bin's spike list) and
// joined before the bin close; the spike recording of the bin runs on the drain stream
// beside the close. (Forking earlier, after the delay-1 bucketing, so that the side
// partition overlaps the gather, was measured 13 % slower: the partition's workgroups take
// the CUs' LDS before the gather's, which is on the critical path.)
hipError_t enqueue_full_bin(dbsim* h, hipStream_t st, hipStream_t side) {
    const bool fork = h->plan.D >= 2;
    hipError_t e = enqueue_bin_start(h, st);
    if (e == hipSuccess && fork) e = hipEventRecord(h->ev_fork, st);
    if (e == hipSuccess && fork) e = hipStreamWaitEvent(side, h->ev_fork, 0);
    if (e == hipSuccess && fork) e = enqueue_ahead(h, side);
    if (e == hipSuccess && fork) e = hipEventRecord(h->ev_join, side);
    if (e == hipSuccess) e = launch_neuron(h->net, 0, (int)h->plan.S, st);
    if (e == hipSuccess) e = launch_compact(h->net, st);
    const bool drain = h->plan.host_record;
    if (e == hipSuccess && drain) e = hipEventRecord(h->ev_dfork, st);
    if (e == hipSuccess && drain) e = hipStreamWaitEvent(h->drain_stream, h->ev_dfork, 0);
    if (e == hipSuccess && drain) e = launch_drain(h->net, h->drain_stream);
    if (e == hipSuccess && drain) e = hipEventRecord(h->ev_djoin, h->drain_stream);
    if (e == hipSuccess && fork) e = hipStreamWaitEvent(st, h->ev_join, 0);
    if (e == hipSuccess && drain) e = hipStreamWaitEvent(st, h->ev_djoin, 0);
    if (e != hipSuccess) return e;
    return launch_readout_close(h->net, st);
}

// One whole bin on one stream, kernel after kernel (the order of the timed bins, without
// their events): the same results as the two-stream form.
hipError_t enqueue_serial_bin(dbsim* h, hipStream_t st) {
    hipError_t e = enqueue_bin_start(h, st);
    if (e == hipSuccess) e = launch_neuron(h->net, 0, (int)h->plan.S, st);
    if (e == hipSuccess) e = enqueue_bin_end(h, st);
    return e;
}

hipError_t capture_graph(dbsim* h, int bins, hipGraphExec_t* out) {
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    for (int b = 0; b < bins && e == hipSuccess; b++) e = enqueue_full_bin(h, h->cap_stream, h->side_stream);
    hipError_t e2 = hipStreamEndCapture(h->cap_stream, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    return e;
}

std::array<hipEvent_t, kMarks> take_events(dbsim* h, hipError_t* e) {
    std::array<hipEvent_t, kMarks> ev{};
    *e = hipSuccess;
    if (!h->ev_pool.empty()) {
        ev = h->ev_pool.back();
        h->ev_pool.pop_back();
        return ev;
    }
    for (auto& x : ev) {
        *e = hipEventCreate(&x);
        if (*e != hipSuccess) return ev;
    }
    return ev;
}

int resolve_timers(dbsim* h) {
    // marks of a timed bin: 0 partition d=1 | 1 gather | 2 neuron | 3 compact | 4 partition
    // d>=2 of the next bin | 5 readout and close | 6; the partition intervals add up to the
    // scatter phase, compact and readout to the bin-end phase
    static const int phase_of[kMarks - 1] = {0, 1, 2, 3, 0, 3};
    for (auto& ev : h->ev_pending) {
        for (int k = 0; k < kMarks - 1; k++) {
            float ms = 0.0f;
            hipError_t e = hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
            if (e != hipSuccess) return hip_fail(h, e, "hipEventElapsedTime");
            h->ms[phase_of[k]] += ms;
        }
        h->timed_bins++;
        h->ev_pool.push_back(ev);
    }
    h->ev_pending.clear();
    return DBSIM_OK;
}

int check_usable(dbsim* h) {
    if (!h) return fail(DBSIM_EINVAL, "null handle");
    if (h->dead) return fail(h->dead, "handle is unusable after an earlier device error: " + g_err);
    return DBSIM_OK;
}

int sync_and_check(dbsim* h) {
    HIPCHK(h, hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    Ctl c;
    HIPCHK(h, hipMemcpy(&c, h->net.ctl, sizeof c, hipMemcpyDeviceToHost), "hipMemcpy(ctl)");
    if (h->ev_build[0]) { // the device construction's duration joins the construction time
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, h->ev_build[0], h->ev_build[1]) == hipSuccess) h->build_seconds += 1e-3 * ms;
        (void)hipEventDestroy(h->ev_build[0]);
        (void)hipEventDestroy(h->ev_build[1]);
        h->ev_build[0] = h->ev_build[1] = nullptr;
    }
    if (c.err & kErrBuild) {
        h->dead = DBSIM_EDEVICE;
        return fail(DBSIM_EDEVICE, "device construction of the connection table failed a consistency check");
    }
    if (c.err) {
        h->dead = DBSIM_EOVERFLOW;
        return fail(DBSIM_EOVERFLOW, "device-side capacity exceeded (error bits " + std::to_string(c.err) + ")");
    }
    return resolve_timers(h);
}

void release_device(dbsim* h) {
    for (auto& x : h->ev_build)
        if (x) {
            (void)hipEventDestroy(x);
            x = nullptr;
        }
    if (h->g_multi) (void)hipGraphExecDestroy(h->g_multi);
    if (h->g_one) (void)hipGraphExecDestroy(h->g_one);
    h->g_multi = h->g_one = nullptr;
    for (auto& ev : h->ev_pending)
        for (auto x : ev) (void)hipEventDestroy(x);
    for (auto& ev : h->ev_pool)
        for (auto x : ev) (void)hipEventDestroy(x);
    h->ev_pending.clear();
    h->ev_pool.clear();
    if (h->dev) {
        if (h->static_mem) {
            std::lock_guard<std::mutex> lock(g_static_mu);
            g_static_busy[h->device] = false;
        } else if (h->desc.dev_alloc) {
            h->desc.dev_free(h->desc.alloc_ctx, h->dev, h->plan.total);
        } else {
            (void)hipFree(h->dev);
        }
        h->dev = nullptr;
    }
    if (h->hrec) (void)hipHostFree(h->hrec);
    if (h->hbend) (void)hipHostFree(h->hbend);
    h->hrec = nullptr;
    h->hbend = nullptr;
    if (h->drain_stream) (void)hipStreamDestroy(h->drain_stream);
    if (h->ev_dfork) (void)hipEventDestroy(h->ev_dfork);
    if (h->ev_djoin) (void)hipEventDestroy(h->ev_djoin);
    h->drain_stream = nullptr;
    h->ev_dfork = h->ev_djoin = nullptr;
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    if (h->side_stream) (void)hipStreamDestroy(h->side_stream);
    if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
    if (h->ev_join) (void)hipEventDestroy(h->ev_join);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    h->cap_stream = h->side_stream = h->stream = nullptr;
    h->ev_fork = h->ev_join = nullptr;
}

} // namespace

extern "C" {

uint32_t dbsim_abi_version(void) { return DBSIM_ABI_VERSION; }

const char* dbsim_last_error(void) { return g_err.c_str(); }

static int footprint_impl(const dbsim_desc* desc, const dbnet_desc* members, uint32_t n, uint64_t* hbm_bytes) {
    if (!desc || !hbm_bytes || !members || n == 0) return fail(DBSIM_EINVAL, "null argument or no network");
    try {
        Members mem;
        mem.assign(members, n);
        Plan p;
        std::string m = make_plan(*desc, mem, p);
        if (!m.empty()) return fail(DBSIM_EINVAL, m);
        *hbm_bytes = p.total;
        return DBSIM_OK;
    } catch (const std::bad_alloc&) {
        return fail(DBSIM_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(DBSIM_EINVAL, "unexpected exception");
    }
}

int dbsim_footprint(const dbsim_desc* desc, uint64_t* hbm_bytes) {
    if (!desc) return fail(DBSIM_EINVAL, "null argument");
    return footprint_impl(desc, &desc->net, 1, hbm_bytes);
}

int dbsim_footprint_ensemble(const dbsim_desc* common, const dbnet_desc* members, uint32_t n_members,
                             uint64_t* hbm_bytes) {
    return footprint_impl(common, members, n_members, hbm_bytes);
}

// Host phase of the creation: validation, memory plan and every host table (no HIP call, so
// it may run on any thread while other threads drive the device).
static int build_impl(const dbsim_desc* desc, const dbnet_desc* members, uint32_t n_members, bool in_static,
                      dbsim_built** out) {
    if (!desc || !out || !members || n_members == 0) return fail(DBSIM_EINVAL, "null argument or no network");
    *out = nullptr;
    if (desc->dev_alloc && !desc->dev_free) return fail(DBSIM_EINVAL, "dev_alloc given without dev_free");
    if (in_static && desc->dev_alloc)
        return fail(DBSIM_EINVAL, "dbsim_create_static allocates nothing: dev_alloc must be NULL");
    dbsim_built* b = nullptr;
    try {
        b = new dbsim_built();
        b->in_static = in_static;
        b->desc = *desc;
        b->mem.assign(members, n_members);
        b->desc.net = b->mem.m[0];
        if (in_static) b->desc.flags |= DBSIM_F_NO_HOST_RECORD; // pinned host memory is an allocation
        std::string m = make_plan(b->desc, b->mem, b->plan);
        if (!m.empty()) {
            delete b;
            return fail(DBSIM_EINVAL, m);
        }
        if (in_static && b->plan.total > (size_t)DBSIM_STATIC_BYTES) {
            const std::string need = std::to_string(b->plan.total);
            delete b;
            return fail(DBSIM_EINVAL, "the network needs " + need + " bytes of device memory; the static region of "
                                      "dbsim_create_static holds " + std::to_string((size_t)DBSIM_STATIC_BYTES));
        }
        auto t0 = std::chrono::steady_clock::now();
        m = build_tables(b->mem, b->plan, desc->host_threads, b->ht, !b->plan.dev_build);
        if (!m.empty()) {
            delete b;
            return fail(DBSIM_EINVAL, m);
        }
        b->build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        *out = b;
        return DBSIM_OK;
    } catch (const std::bad_alloc&) {
        delete b;
        return fail(DBSIM_ENOMEM, "host allocation failed while building the network");
    } catch (...) {
        delete b;
        return fail(DBSIM_EINVAL, "unexpected exception while building the network");
    }
}

// Connection table generated on the device (plan.dev_build), into the handle's edge and
// header arrays, with the temporaries in its tile arena and super-tile streams. Only the
// copies of the generator's tables are awaited (their host memory dies with the built
// network); the construction itself runs on the handle's stream ahead of the first bin,
// and its duration joins build_seconds at the next synchronisation.
static int device_build(dbsim* h, HostTables& ht) {
    const Plan& p = h->plan;
    unsigned char* ev = h->dev + p.ev.off;
    // the generator's tables, in the order gen_tables_bytes lays them out
    size_t o = p.gl.tables;
    hipError_t pe = hipSuccess;
    auto put = [&](const void* src, size_t bytes) -> unsigned char* {
        unsigned char* d = ev + o;
        if (bytes && pe == hipSuccess) pe = hipMemcpyAsync(d, src, bytes, hipMemcpyHostToDevice, h->stream);
        o += (bytes + 255) & ~(size_t)255;
        return d;
    };
    DevBuild b{};
    b.g.pops = reinterpret_cast<const GenPop*>(put(ht.gpops.data(), sizeof(GenPop) * ht.gpops.size()));
    b.g.members = reinterpret_cast<const GenMember*>(put(ht.gmembers.data(), sizeof(GenMember) * ht.gmembers.size()));
    b.g.projs = reinterpret_cast<const GenProj*>(put(ht.gprojs.data(), sizeof(GenProj) * ht.gprojs.size()));
    b.g.cands = reinterpret_cast<const GenCand*>(put(ht.gcands.data(), sizeof(GenCand) * ht.gcands.size()));
    b.g.cpops = reinterpret_cast<const GenCandPop*>(put(ht.gcpops.data(), sizeof(GenCandPop) * ht.gcpops.size()));
    const uint8_t zero = 0;
    b.g.dtab = put(ht.gdtab.empty() ? &zero : ht.gdtab.data(), ht.gdtab.empty() ? 1 : ht.gdtab.size());
    if (o > p.gl.cnt) return fail(DBSIM_EINVAL, "internal error: generator tables overrun their slot");
    HIPCHK(h, pe, "hipMemcpy(generator tables)");
    HIPCHK(h, hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    b.g.n_pops = (uint32_t)ht.gpops.size();
    b.g.kmax = ht.gkmax;
    b.g.hcap = ht.ghcap;
    b.g.scratch_words = gen_scratch_words(ht.gkmax, ht.ghcap);
    b.scratch = reinterpret_cast<uint32_t*>(h->dev + p.sev.off);
    b.batch = p.gen_batch;
    b.cnt = reinterpret_cast<uint32_t*>(ev + p.gl.cnt);
    b.cur = reinterpret_cast<unsigned long long*>(ev + p.gl.cur);
    b.rowlen = reinterpret_cast<unsigned long long*>(ev + p.gl.rowlen);
    b.rowptr = reinterpret_cast<unsigned long long*>(ev + p.gl.rowptr);
    b.sums = reinterpret_cast<unsigned long long*>(ev + p.gl.sums);
    b.tb = ev + p.gl.tb;
    b.err = &h->net.ctl->err;
    b.edge = reinterpret_cast<uint32_t*>(h->dev + p.edge.off);
    b.hdr = reinterpret_cast<uint32_t*>(h->dev + p.hdr.off);
    b.N = p.N;
    b.E = p.E;
    b.D = p.D;
    b.HW = p.HW;
    b.KW = p.KW;
    b.wlim = std::ldexp(1.0, 52 - (int)p.F);
    const bool timed = !h->static_mem; // a handle in the static region creates no events
    if (timed) {
        HIPCHK(h, hipEventCreate(&h->ev_build[0]), "hipEventCreate");
        HIPCHK(h, hipEventCreate(&h->ev_build[1]), "hipEventCreate");
        HIPCHK(h, hipEventRecord(h->ev_build[0], h->stream), "hipEventRecord");
    }
    HIPCHK(h, launch_device_build(b, h->stream), "device construction launch");
    if (timed) HIPCHK(h, hipEventRecord(h->ev_build[1], h->stream), "hipEventRecord");
    h->device_built = true;
    return DBSIM_OK;
}

// Device phase: allocation, streams, upload and initial state from a built network, which
// it consumes. dev_opts (may be NULL) replaces the device, stream and allocator options.
static int deploy_impl(dbsim_built* bt, const dbsim_desc* dev_opts, dbsim** out) {
    std::unique_ptr<dbsim_built> own(bt);
    if (!bt || !out) return fail(DBSIM_EINVAL, "null argument");
    *out = nullptr;
    const bool in_static = bt->in_static;
    dbsim_desc dsc = bt->desc;
    if (dev_opts) {
        if (dev_opts->dev_alloc && !dev_opts->dev_free) return fail(DBSIM_EINVAL, "dev_alloc given without dev_free");
        if (in_static && dev_opts->dev_alloc)
            return fail(DBSIM_EINVAL, "dbsim_create_static allocates nothing: dev_alloc must be NULL");
        dsc.device = dev_opts->device;
        dsc.hip_stream = dev_opts->hip_stream;
        dsc.dev_alloc = dev_opts->dev_alloc;
        dsc.dev_free = dev_opts->dev_free;
        dsc.alloc_ctx = dev_opts->alloc_ctx;
    }
    const dbsim_desc* desc = &dsc;
    dbsim* h = nullptr;
    try {
        h = new dbsim();
        h->desc = dsc;
        h->mem = std::move(bt->mem);
        h->plan = std::move(bt->plan);
        h->desc.net = h->mem.m[0];
        h->build_seconds = bt->build_seconds;
        HostTables& ht = bt->ht;
        h->device = desc->device;
        if (h->device < 0 && hipGetDevice(&h->device) != hipSuccess) {
            delete h;
            return fail(DBSIM_EDEVICE, "no HIP device");
        }
        DeviceGuard dg(h->device);
        const Plan& p = h->plan;
        if (in_static) {
            if (h->device >= kStaticDevices) {
                delete h;
                return fail(DBSIM_EINVAL, "device ordinal too large for the static regions");
            }
            std::lock_guard<std::mutex> lock(g_static_mu);
            hipError_t se;
            unsigned char* region = static_region_of(h->device, &se);
            if (!region) {
                delete h;
                return fail(DBSIM_EDEVICE, std::string("hipGetSymbolAddress(static region): ") + hipGetErrorString(se));
            }
            if (g_static_busy[h->device]) {
                delete h;
                return fail(DBSIM_ESTATE, "the static region of this device is held by another handle of "
                                          "dbsim_create_static; destroy that one first");
            }
            g_static_busy[h->device] = true;
            h->dev = region;
            h->static_mem = true;
        } else if (desc->dev_alloc) {
            h->dev = (unsigned char*)desc->dev_alloc(desc->alloc_ctx, p.total);
            if (!h->dev) {
                delete h;
                return fail(DBSIM_EHBM, "device allocator returned NULL for " + std::to_string(p.total) + " bytes");
            }
        } else {
            void* ptr = nullptr;
            if (hipMalloc(&ptr, p.total) != hipSuccess || !ptr) {
                (void)hipGetLastError();
                delete h;
                return fail(DBSIM_EHBM, "hipMalloc failed for " + std::to_string(p.total) + " bytes");
            }
            h->dev = (unsigned char*)ptr;
        }
        fill_devnet(h);
        // streams (a handle in the static region creates none: its bins run on the caller's
        // stream, or the default stream, one kernel after another)
        if (in_static) {
            h->stream = (hipStream_t)desc->hip_stream;
        } else if (desc->hip_stream) {
            h->stream = (hipStream_t)desc->hip_stream;
        } else {
            hipError_t se = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
            if (se != hipSuccess) {
                release_device(h);
                delete h;
                return fail(DBSIM_EDEVICE, std::string("hipStreamCreateWithFlags: ") + hipGetErrorString(se));
            }
            h->own_stream = true;
        }
        if (!in_static) {
            hipError_t se = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
            if (se == hipSuccess) se = hipStreamCreateWithFlags(&h->side_stream, hipStreamNonBlocking);
            if (se == hipSuccess) se = hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming);
            if (se == hipSuccess) se = hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming);
            if (se == hipSuccess && p.host_record) {
                // the recording ring: pinned, coherent host memory the drain kernel writes
                void *a = nullptr, *b = nullptr, *da = nullptr, *db = nullptr;
                se = hipHostMalloc(&a, 4 * (size_t)p.HC, hipHostMallocCoherent);
                if (se == hipSuccess) h->hrec = static_cast<uint32_t*>(a);
                if (se == hipSuccess) se = hipHostMalloc(&b, 8 * (size_t)p.HMB, hipHostMallocCoherent);
                if (se == hipSuccess) h->hbend = static_cast<unsigned long long*>(b);
                if (se == hipSuccess) std::memset(h->hbend, 0, 8 * (size_t)p.HMB);
                if (se == hipSuccess) se = hipHostGetDevicePointer(&da, a, 0);
                if (se == hipSuccess) se = hipHostGetDevicePointer(&db, b, 0);
                if (se == hipSuccess) {
                    h->net.hrec = static_cast<uint32_t*>(da);
                    h->net.hbend = static_cast<unsigned long long*>(db);
                }
                if (se == hipSuccess) se = hipStreamCreateWithFlags(&h->drain_stream, hipStreamNonBlocking);
                if (se == hipSuccess) se = hipEventCreateWithFlags(&h->ev_dfork, hipEventDisableTiming);
                if (se == hipSuccess) se = hipEventCreateWithFlags(&h->ev_djoin, hipEventDisableTiming);
            }
            if (se != hipSuccess) {
                release_device(h);
                delete h;
                return fail(DBSIM_EDEVICE, std::string("stream/event creation or pinned host ring: ") +
                                                hipGetErrorString(se));
            }
        }
        // upload
        auto up = [&](const Plan::Slot& s, const void* src, size_t bytes) -> hipError_t {
            if (!bytes) return hipSuccess;
            return hipMemcpyAsync(h->dev + s.off, src, bytes, hipMemcpyHostToDevice, h->stream);
        };
        hipError_t e = prepare_kernels_once(h->device);
        const size_t N = p.N;
        auto fill = [&](const Plan::Slot& sl, int v) -> hipError_t {
            return hipMemsetAsync(h->dev + sl.off, v, sl.bytes, h->stream);
        };
        if (e == hipSuccess) e = up(p.V, ht.V0.data(), 4 * N);
        if (e == hipSuccess) e = fill(p.J, 0);   // +0.0f
        if (e == hipSuccess) e = fill(p.A, 0);
        if (e == hipSuccess) e = fill(p.Iou, 0);
        if (e == hipSuccess) e = fill(p.ref, 0);
        if (e == hipSuccess) e = fill(p.pend, 0xFF); // no partial bin pending
        if (e == hipSuccess) e = up(p.pops, ht.pops.data(), sizeof(PopParams) * ht.pops.size());
        if (e == hipSuccess) e = up(p.ptab, ht.ptab.data(), 4 * ht.ptab.size());
        if (e == hipSuccess) e = up(p.blk, ht.blk.data(), sizeof(uint2) * ht.blk.size());
        if (e == hipSuccess && !p.dev_build) e = up(p.hdr, ht.hdr.data(), 4 * ht.hdr.size());
        if (e == hipSuccess) e = up(p.st_base, ht.st_base.data(), 8 * ht.st_base.size());
        if (e == hipSuccess) e = hipMemsetAsync(h->dev + p.st_fill.off, 0, p.st_fill.bytes, h->stream);
        if (e == hipSuccess && !p.dev_build) e = up(p.edge, ht.edge.get(), 4 * ht.edge_words);
        if (e == hipSuccess) e = up(p.tile_base, ht.tile_base.data(), 8 * ht.tile_base.size());
        if (e == hipSuccess) e = hipMemsetAsync(h->dev + p.tile_fill.off, 0, p.tile_fill.bytes, h->stream);
        if (e == hipSuccess) e = hipMemsetAsync(h->dev + p.ovf.off, 0, p.ovf.bytes, h->stream);
        if (e == hipSuccess) e = hipMemsetAsync(h->dev + p.grp_cnt.off, 0, p.grp_cnt.bytes, h->stream);
        if (e == hipSuccess) e = hipMemsetAsync(h->dev + p.bin_start.off, 0, p.bin_start.bytes, h->stream);
        if (e == hipSuccess) e = hipMemsetAsync(h->dev + p.bin_cnt.off, 0, p.bin_cnt.bytes, h->stream);
        if (e == hipSuccess) e = hipMemsetAsync(h->dev + p.blk_sig.off, 0, p.blk_sig.bytes, h->stream);
        if (e == hipSuccess) e = hipMemsetAsync(h->dev + p.blk_cnt.off, 0, p.blk_cnt.bytes, h->stream);
        if (e == hipSuccess) e = up(p.reg_blk_ptr, ht.reg_blk_ptr.data(), 4 * ht.reg_blk_ptr.size());
        if (e == hipSuccess) e = up(p.reg_blk, ht.reg_blk.data(), 4 * ht.reg_blk.size());
        if (e == hipSuccess) e = up(p.reg_size, ht.reg_size.data(), 4 * ht.reg_size.size());
        if (e == hipSuccess) e = up(p.l1_ptr, ht.l1_ptr.data(), 4 * ht.l1_ptr.size());
        if (e == hipSuccess) e = up(p.l1_region, ht.l1_region.data(), 4 * ht.l1_region.size());
        if (e == hipSuccess) e = hipMemsetAsync(h->dev + p.sig.off, 0, p.sig.bytes, h->stream);
        if (e == hipSuccess) e = hipMemsetAsync(h->dev + p.sig_cnt.off, 0, p.sig_cnt.bytes, h->stream);
        if (e == hipSuccess) e = hipMemsetAsync(h->dev + p.ctl.off, 0, p.ctl.bytes, h->stream);
        if (e == hipSuccess) e = hipMemsetAsync(h->dev + p.bold_ctl.off, 0, p.bold_ctl.bytes, h->stream);
        // the host tables die with this call: wait for the copies on this handle's stream
        // only (other handles keep running on theirs)
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) {
            std::string msg = std::string("upload failed: ") + hipGetErrorString(e);
            release_device(h);
            delete h;
            return fail(DBSIM_EDEVICE, msg);
        }
        if (p.dev_build) {
            const int rc = device_build(h, ht);
            if (rc) {
                release_device(h);
                delete h;
                return rc;
            }
        }
        // grid of the partition kernels: scatter_wgs_per_cu blocks per CU
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) h->num_cus = prop.multiProcessorCount;
        h->scatter_wgs = p.scatter_wgs_per_cu;
        h->scatter_grid = std::min((int)(p.blocked ? kFanMaxGrid : kMaxPartGrid), (int)h->scatter_wgs * h->num_cus);
        *out = h;
        return DBSIM_OK;
    } catch (const std::bad_alloc&) {
        if (h) {
            release_device(h);
            delete h;
        }
        return fail(DBSIM_ENOMEM, "host allocation failed while building the network");
    } catch (...) {
        if (h) {
            release_device(h);
            delete h;
        }
        return fail(DBSIM_EINVAL, "unexpected exception while deploying the network");
    }
}


static int create_impl(const dbsim_desc* desc, const dbnet_desc* members, uint32_t n_members, dbsim** out,
                       bool in_static = false) {
    if (!out) return fail(DBSIM_EINVAL, "null argument");
    *out = nullptr;
    dbsim_built* b = nullptr;
    const int rc = build_impl(desc, members, n_members, in_static, &b);
    if (rc) return rc;
    return deploy_impl(b, nullptr, out);
}

static void to_constants(const Members& mem, const Plan& p, const std::vector<PopParams>& pops,
                         const std::vector<uint32_t>& ptab, dbsim_pop_constants* out) {
    for (uint32_t gq = 0; gq < p.n_pops; gq++) {
        const PopParams& P = pops[gq];
        dbsim_pop_constants& c = out[gq];
        std::memset(&c, 0, sizeof c);
        c.first_neuron = gq ? pops[gq - 1].end : 0u;
        c.end_neuron = P.end;
        c.member = (uint32_t)(std::upper_bound(mem.pbase.begin(), mem.pbase.end(), gq) - mem.pbase.begin()) - 1;
        c.region = P.region;
        c.k = P.k;
        c.g_L = P.gL;
        c.V_L = P.VL;
        c.V_th = P.Vth;
        c.V_reset = P.Vr;
        c.I_ext = P.Iext;
        c.w_bg = P.wbg;
        for (uint32_t u = 0; u < p.U; u++) {
            c.g[u] = P.g[u];
            c.V_rev[u] = P.Vu[u];
            c.decay[u] = P.dec[u];
        }
        c.ref_steps = P.r;
        c.poisson_len = (uint32_t)P.cmax;
        for (int x = 0; x < P.cmax && x < (int)kMaxPoisson; x++) c.poisson_T[x] = ptab[(size_t)gq * kMaxPoisson + x];
    }
}

int dbsim_derive_constants(const dbsim_desc* common, const dbnet_desc* members, uint32_t n_members,
                           dbsim_pop_constants* out, uint32_t cap, uint32_t* n_out) {
    if (!common || !members || n_members == 0 || !n_out) return fail(DBSIM_EINVAL, "null argument or no network");
    try {
        Members mem;
        mem.assign(members, n_members);
        Plan p;
        std::string m = make_plan(*common, mem, p);
        if (!m.empty()) return fail(DBSIM_EINVAL, m);
        *n_out = p.n_pops;
        if (cap < p.n_pops) return fail(DBSIM_ETRUNC, "buffer too small; *n_out holds the count needed");
        if (!out) return fail(DBSIM_EINVAL, "out is NULL");
        std::vector<PopParams> pops;
        std::vector<uint32_t> ptab;
        fill_populations(mem, p, pops, ptab, nullptr, nullptr);
        to_constants(mem, p, pops, ptab, out);
        return DBSIM_OK;
    } catch (const std::bad_alloc&) {
        return fail(DBSIM_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(DBSIM_EINVAL, "unexpected exception");
    }
}

int dbsim_create(const dbsim_desc* desc, dbsim** out) {
    if (!desc) return fail(DBSIM_EINVAL, "null argument");
    return create_impl(desc, &desc->net, 1, out);
}

int dbsim_create_static(const dbsim_desc* desc, dbsim** out) {
    if (!desc) return fail(DBSIM_EINVAL, "null argument");
    return create_impl(desc, &desc->net, 1, out, true);
}

int dbsim_build(const dbsim_desc* desc, dbsim_built** out) {
    if (!desc) return fail(DBSIM_EINVAL, "null argument");
    return build_impl(desc, &desc->net, 1, false, out);
}

int dbsim_create_built(dbsim_built* b, const dbsim_desc* device_opts, dbsim** out) {
    return deploy_impl(b, device_opts, out);
}

void dbsim_built_free(dbsim_built* b) { delete b; }

int dbsim_create_ensemble(const dbsim_desc* common, const dbnet_desc* members, uint32_t n_members, dbsim** out) {
    return create_impl(common, members, n_members, out);
}

int dbsim_member_info(dbsim* h, uint32_t member, dbsim_member* info) {
    if (!h || !info) return fail(DBSIM_EINVAL, "null argument");
    if (member >= h->mem.m.size()) return fail(DBSIM_EINVAL, "member index out of range");
    info->first_neuron = h->mem.nbase[member];
    info->num_neurons = h->mem.nbase[member + 1] - h->mem.nbase[member];
    info->first_region = h->mem.rbase[member];
    info->num_regions = h->mem.rbase[member + 1] - h->mem.rbase[member];
    return DBSIM_OK;
}

int dbsim_get_info(dbsim* h, dbsim_info* info) {
    if (!h || !info) return fail(DBSIM_EINVAL, "null argument");
    const Plan& p = h->plan;
    info->num_neurons = p.N;
    info->num_edges = p.E;
    info->receptors = p.U;
    info->weights_per_edge = p.KW;
    info->steps_per_bin = p.S;
    info->max_delay = p.D;
    info->n_regions = p.n_regions;
    info->tile_neurons = 1u << p.tile_bits;
    info->n_tiles = p.T;
    info->frac_bits = p.F;
    info->n_members = p.n_members;
    info->fanin_passes = p.blocked ? 1u : 2u;
    info->device_built = h->device_built ? 1u : 0u;
    info->stream_record_bytes = p.blocked ? 0u : p.narrow ? 10u : 4u * (1u + p.KW);
    info->stream_records = p.blocked ? 0u : p.st_total;
    info->arena_records = p.blocked ? (uint64_t)p.tile_blk[p.T] * kFanBlock : p.ta_total;
    return DBSIM_OK;
}

int dbsim_step(dbsim* h, uint64_t n_steps) {
    int rc = check_usable(h);
    if (rc) return rc;
    DeviceGuard dg(h->device);
    const uint32_t S = h->plan.S;
    const bool direct = h->timing || h->static_mem || (h->desc.flags & DBSIM_F_NO_GRAPH);
    while (n_steps > 0) {
        const uint32_t s0 = (uint32_t)(h->step % S);
        if (s0 == 0 && n_steps >= S) {
            uint64_t nb = n_steps / S;
            if (direct) {
                for (uint64_t b = 0; b < nb; b++) {
                    if (h->timing) {
                        hipError_t e;
                        auto ev = take_events(h, &e);
                        HIPCHK(h, e, "hipEventCreate");
                        // one stream, an event between phases (no overlap, so that each
                        // kernel's duration is its own)
                        hipStream_t st = h->stream;
                        HIPCHK(h, hipEventRecord(ev[0], st), "hipEventRecord");
                        HIPCHK(h, launch_scatter(h->net, h->scatter_grid, st, 1, 1, 0), "partition launch");
                        HIPCHK(h, hipEventRecord(ev[1], st), "hipEventRecord");
                        HIPCHK(h, launch_gather(h->net, st), "gather launch");
                        HIPCHK(h, hipEventRecord(ev[2], st), "hipEventRecord");
                        HIPCHK(h, launch_neuron(h->net, 0, (int)S, st), "neuron launch");
                        HIPCHK(h, hipEventRecord(ev[3], st), "hipEventRecord");
                        HIPCHK(h, launch_compact(h->net, st), "compact launch");
                        if (h->plan.host_record) HIPCHK(h, launch_drain(h->net, st), "recording launch");
                        HIPCHK(h, hipEventRecord(ev[4], st), "hipEventRecord");
                        HIPCHK(h, enqueue_ahead(h, st), "partition launch");
                        HIPCHK(h, hipEventRecord(ev[5], st), "hipEventRecord");
                        HIPCHK(h, launch_readout_close(h->net, st), "readout launch");
                        HIPCHK(h, hipEventRecord(ev[6], st), "hipEventRecord");
                        h->ev_pending.push_back(ev);
                    } else if (h->static_mem) {
                        HIPCHK(h, enqueue_serial_bin(h, h->stream), "bin launch");
                    } else {
                        HIPCHK(h, enqueue_full_bin(h, h->stream, h->side_stream), "bin launch");
                    }
                }
            } else {
                if (!h->g_multi) HIPCHK(h, capture_graph(h, kGraphBins, &h->g_multi), "graph capture");
                if (!h->g_one) HIPCHK(h, capture_graph(h, 1, &h->g_one), "graph capture");
                for (uint64_t b = 0; b + kGraphBins <= nb; b += kGraphBins)
                    HIPCHK(h, hipGraphLaunch(h->g_multi, h->stream), "hipGraphLaunch");
                for (uint64_t b = 0; b < nb % kGraphBins; b++)
                    HIPCHK(h, hipGraphLaunch(h->g_one, h->stream), "hipGraphLaunch");
            }
            h->step += nb * S;
            n_steps -= nb * S;
        } else {
            const uint32_t s1 = (uint32_t)std::min<uint64_t>(S, s0 + n_steps);
            if (s0 == 0) HIPCHK(h, enqueue_bin_start(h, h->stream), "bin start launch");
            HIPCHK(h, launch_neuron(h->net, (int)s0, (int)s1, h->stream), "neuron launch");
            if (s1 == S) HIPCHK(h, enqueue_bin_end(h, h->stream), "bin end launch");
            h->step += s1 - s0;
            n_steps -= s1 - s0;
        }
    }
    return DBSIM_OK;
}

int dbsim_sync(dbsim* h) {
    int rc = check_usable(h);
    if (rc) return rc;
    DeviceGuard dg(h->device);
    return sync_and_check(h);
}

int dbsim_read_spikes(dbsim* h, uint64_t step_lo, uint64_t step_hi, uint64_t* steps, uint32_t* ids, uint64_t cap,
                      uint64_t* n_out) {
    int rc = check_usable(h);
    if (rc) return rc;
    if (!n_out) return fail(DBSIM_EINVAL, "n_out is NULL");
    DeviceGuard dg(h->device);
    rc = sync_and_check(h);
    if (rc) return rc;
    const Plan& p = h->plan;
    const uint64_t S = p.S, done_bins = h->step / S;
    step_hi = std::min(step_hi, done_bins * S);
    *n_out = 0;
    if (step_lo >= step_hi) return DBSIM_OK;
    const uint64_t b_lo = step_lo / S, b_hi = (step_hi + S - 1) / S;
    if (b_lo < h->first_bin)
        return fail(DBSIM_ERANGE, "requested bins precede the checkpoint this handle was restored from");
    std::vector<std::pair<uint64_t, uint32_t>> out;
    if (p.host_record) { // the pinned host ring, complete up to the last synchronised bin
        if (done_bins - b_lo > p.HMB - 1) return fail(DBSIM_ERANGE, "requested bins have left the host record");
        const uint64_t hm = p.HMB - 1, cm = p.HC - 1;
        const uint64_t head = h->hbend[done_bins & hm], first = h->hbend[b_lo & hm];
        if (head - first > p.HC) return fail(DBSIM_ERANGE, "requested spikes have been overwritten in the host record");
        for (uint64_t b = b_lo; b < b_hi; b++) {
            const uint64_t s0 = h->hbend[b & hm], s1 = h->hbend[(b + 1) & hm];
            for (uint64_t o = s0; o < s1; o++) {
                const uint32_t v = h->hrec[o & cm];
                const uint64_t st = b * S + (v & 15u);
                if (st >= step_lo && st < step_hi) out.emplace_back(st, v >> 4);
            }
        }
    } else {
        if (done_bins - b_lo > p.MB - 1) return fail(DBSIM_ERANGE, "requested bins have left the device history");
        std::vector<unsigned long long> bstart(p.MB);
        std::vector<uint32_t> bcnt(p.MB);
        HIPCHK(h, hipMemcpy(bstart.data(), h->net.bin_start, 8 * (size_t)p.MB, hipMemcpyDeviceToHost), "hipMemcpy");
        HIPCHK(h, hipMemcpy(bcnt.data(), h->net.bin_cnt, 4 * (size_t)p.MB, hipMemcpyDeviceToHost), "hipMemcpy");
        const uint64_t head = bstart[done_bins & (p.MB - 1)];
        const uint64_t first = bstart[b_lo & (p.MB - 1)];
        if (head - first > p.RC) return fail(DBSIM_ERANGE, "requested spikes have been overwritten in the device ring");
        std::vector<uint32_t> raw(head - first);
        uint64_t a = first & (p.RC - 1), left = head - first, o = 0;
        while (left) {
            const uint64_t n = std::min(left, p.RC - a);
            HIPCHK(h, hipMemcpy(raw.data() + o, h->net.rec + a, 4 * n, hipMemcpyDeviceToHost), "hipMemcpy");
            o += n;
            left -= n;
            a = 0;
        }
        for (uint64_t b = b_lo; b < b_hi; b++) {
            const uint64_t s = bstart[b & (p.MB - 1)] - first;
            const uint32_t c = bcnt[b & (p.MB - 1)];
            for (uint32_t x = 0; x < c; x++) {
                const uint32_t v = raw[s + x];
                const uint64_t st = b * S + (v & 15u);
                if (st >= step_lo && st < step_hi) out.emplace_back(st, v >> 4);
            }
        }
    }
    std::sort(out.begin(), out.end());
    *n_out = out.size();
    if (out.size() > cap) return fail(DBSIM_ETRUNC, "buffer too small; *n_out holds the count needed");
    if (!out.empty() && (!steps || !ids)) return fail(DBSIM_EINVAL, "output arrays are NULL");
    for (size_t x = 0; x < out.size(); x++) {
        steps[x] = out[x].first;
        ids[x] = out[x].second;
    }
    return DBSIM_OK;
}

int dbsim_read_region_signal(dbsim* h, uint64_t bin_lo, uint64_t bin_hi, double* sig, uint32_t* counts, uint64_t cap,
                             uint64_t* n_out) {
    int rc = check_usable(h);
    if (rc) return rc;
    if (!n_out) return fail(DBSIM_EINVAL, "n_out is NULL");
    const Plan& p = h->plan;
    if (!p.regions_on) return fail(DBSIM_ESTATE, "region recording was not requested (DBSIM_REC_REGIONS)");
    DeviceGuard dg(h->device);
    rc = sync_and_check(h);
    if (rc) return rc;
    const uint64_t done_bins = h->step / p.S;
    bin_hi = std::min(bin_hi, done_bins);
    *n_out = 0;
    if (bin_lo >= bin_hi) return DBSIM_OK;
    if (done_bins - bin_lo > p.MB) return fail(DBSIM_ERANGE, "requested bins have left the device history");
    if (bin_lo < h->first_bin)
        return fail(DBSIM_ERANGE, "requested bins precede the checkpoint this handle was restored from");
    const uint64_t R = p.n_regions, need = (bin_hi - bin_lo) * R;
    *n_out = need;
    if (need > cap) return fail(DBSIM_ETRUNC, "buffer too small; *n_out holds the count needed");
    if (!sig) return fail(DBSIM_EINVAL, "sig is NULL");
    for (uint64_t b = bin_lo; b < bin_hi; b++) {
        const size_t slot = (size_t)(b & (p.MB - 1)) * R;
        HIPCHK(h, hipMemcpy(sig + (b - bin_lo) * R, h->net.sig + slot, 8 * R, hipMemcpyDeviceToHost), "hipMemcpy");
        if (counts)
            HIPCHK(h, hipMemcpy(counts + (b - bin_lo) * R, h->net.sig_cnt + slot, 4 * R, hipMemcpyDeviceToHost),
                   "hipMemcpy");
    }
    return DBSIM_OK;
}

int dbsim_read_state(dbsim* h, float* V, float* J, int32_t* ref) {
    int rc = check_usable(h);
    if (rc) return rc;
    DeviceGuard dg(h->device);
    rc = sync_and_check(h);
    if (rc) return rc;
    const size_t N = h->plan.N;
    if (V) HIPCHK(h, hipMemcpy(V, h->net.V, 4 * N, hipMemcpyDeviceToHost), "hipMemcpy");
    if (J) HIPCHK(h, hipMemcpy(J, h->net.J, 4 * N * h->plan.U, hipMemcpyDeviceToHost), "hipMemcpy");
    if (ref) {
        std::vector<uint8_t> r(N);
        HIPCHK(h, hipMemcpy(r.data(), h->net.ref, N, hipMemcpyDeviceToHost), "hipMemcpy");
        for (size_t i = 0; i < N; i++) ref[i] = r[i];
    }
    return DBSIM_OK;
}

int dbsim_receptor_currents(dbsim* h, double* mean, uint32_t n_pops) {
    int rc = check_usable(h);
    if (rc) return rc;
    if (!mean) return fail(DBSIM_EINVAL, "mean is NULL");
    const Plan& p = h->plan;
    if (n_pops != p.n_pops) return fail(DBSIM_EINVAL, "n_pops does not match the handle's population count");
    DeviceGuard dg(h->device);
    rc = sync_and_check(h);
    if (rc) return rc;
    double* rblk = at<double>(h->dev, p.rblk);
    double* rpop = at<double>(h->dev, p.rpop);
    HIPCHK(h, launch_receptor_currents(h->net, p.n_pops, rblk, rpop, h->stream), "receptor current launch");
    HIPCHK(h, hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    HIPCHK(h, hipMemcpy(mean, rpop, 8 * 4 * (size_t)p.n_pops, hipMemcpyDeviceToHost), "hipMemcpy");
    return DBSIM_OK;
}

int dbsim_write_state(dbsim* h, const float* V, const float* J, const int32_t* ref) {
    int rc = check_usable(h);
    if (rc) return rc;
    if (h->step % h->plan.S) return fail(DBSIM_ESTATE, "state can only be written at a bin boundary");
    DeviceGuard dg(h->device);
    rc = sync_and_check(h);
    if (rc) return rc;
    const size_t N = h->plan.N;
    if (ref)
        for (size_t i = 0; i < N; i++)
            if (ref[i] < 0 || ref[i] > 255) return fail(DBSIM_EINVAL, "ref values must lie in [0, 255]");
    if (V) HIPCHK(h, hipMemcpy(h->net.V, V, 4 * N, hipMemcpyHostToDevice), "hipMemcpy");
    if (J) HIPCHK(h, hipMemcpy(h->net.J, J, 4 * N * h->plan.U, hipMemcpyHostToDevice), "hipMemcpy");
    if (ref) {
        std::vector<uint8_t> r(N);
        for (size_t i = 0; i < N; i++) r[i] = (uint8_t)ref[i];
        HIPCHK(h, hipMemcpy(h->net.ref, r.data(), N, hipMemcpyHostToDevice), "hipMemcpy");
    }
    return DBSIM_OK;
}

int dbsim_check_device_generator(const dbnet_desc* members, uint32_t n_members, uint64_t target, uint32_t* src,
                                 float* w0, float* w1, uint8_t* delay, uint32_t* proj, uint64_t cap,
                                 uint64_t* n_out) {
    if (!members || !n_members || !n_out) return fail(DBSIM_EINVAL, "null argument or no network");
    try {
        Members mem;
        mem.assign(members, n_members);
        char err[512];
        for (uint32_t k = 0; k < n_members; k++)
            if (dbnet_validate(&mem.m[k], err, sizeof err) != 0) return fail(DBSIM_EINVAL, err);
        if (target >= mem.nbase.back()) return fail(DBSIM_EINVAL, "target out of range");
        HostTables ht;
        const std::string m = make_gen_tables(mem, ht);
        if (!m.empty()) return fail(DBSIM_EINVAL, m);
        GenTables g{};
        g.pops = ht.gpops.data();
        g.members = ht.gmembers.data();
        g.projs = ht.gprojs.data();
        g.cands = ht.gcands.data();
        g.cpops = ht.gcpops.data();
        g.dtab = ht.gdtab.data();
        g.n_pops = (uint32_t)ht.gpops.size();
        g.kmax = ht.gkmax;
        g.hcap = ht.ghcap;
        g.scratch_words = gen_scratch_words(ht.gkmax, ht.ghcap);
        std::vector<uint32_t> scratch(g.scratch_words);
        uint64_t n = 0;
        const bool ok = gen_target(g, target, scratch.data(),
                                   [&](uint64_t s, uint32_t, float a, float b, uint32_t dl, uint32_t j) {
                                       if (n < cap) {
                                           if (src) src[n] = (uint32_t)s;
                                           if (w0) w0[n] = a;
                                           if (w1) w1[n] = b;
                                           if (delay) delay[n] = (uint8_t)dl;
                                           if (proj) proj[n] = j;
                                       }
                                       n++;
                                   });
        *n_out = n;
        if (!ok) return fail(DBSIM_EINVAL, "a candidate set is smaller than its in-degree");
        if (n > cap) return fail(DBSIM_ETRUNC, "buffers too small; *n_out holds the in-degree");
        return DBSIM_OK;
    } catch (const std::bad_alloc&) {
        return fail(DBSIM_ENOMEM, "host allocation failed");
    }
}

// ------------------------------------------------------------------ checkpoint and resume

namespace {

struct CkHeader {
    char magic[8];
    uint64_t fingerprint;
    uint64_t N, U, n_pops, n_regions, D, S;
    uint64_t bin, edge_events, spikes, inject_until;
    uint64_t b0;    // first bin of the saved spike history
    uint64_t off0;  // spike-stream offset of bin b0's first entry
    uint64_t n_spk; // saved spike entries, bins b0 .. bin - 1
    uint64_t bold_on, tr_bins;
    double bw[10];  // h, h/tau, kappa, gamma, 1/alpha, rho, V0, k1, k2, k3
    uint64_t bold_ctl[2];
};
constexpr char kCkMagic[8] = {'D', 'B', 'S', 'I', 'M', 'C', 'K', '1'};

inline size_t up8(size_t x) { return (x + 7) & ~(size_t)7; }

void fnv(uint64_t& h, const void* p, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; i++) {
        h ^= b[i];
        h *= 0x100000001b3ull;
    }
}

// Identity of the network a checkpoint belongs to: sizes, the members' descriptions (their
// reserved words excluded) and the first and last 4 KiB of the device edge table.
int ck_fingerprint(dbsim* h, uint64_t* out) {
    const Plan& p = h->plan;
    uint64_t f = 0xcbf29ce484222325ull;
    const uint64_t sc[] = {p.N, p.E, p.U, p.KW, p.S, p.D, p.F, p.n_pops, p.n_regions, p.n_members};
    fnv(f, sc, sizeof sc);
    for (const dbnet_desc& d : h->mem.m) {
        const uint64_t ds[] = {d.seed, d.n_pops, d.n_projs, d.n_regions, d.receptor_mask, d.frac_bits, d.net_id};
        fnv(f, ds, sizeof ds);
        const float df[] = {d.dt_ms, d.bin_ms, d.velocity_mm_per_ms};
        fnv(f, df, sizeof df);
        for (uint32_t q = 0; q < d.n_pops; q++) {
            fnv(f, &d.pops[q], offsetof(dbnet_pop, reserved));
            fnv(f, &d.pops[q].C, sizeof(dbnet_pop) - offsetof(dbnet_pop, C));
        }
        for (uint32_t q = 0; q < d.n_projs; q++) fnv(f, &d.projs[q], offsetof(dbnet_proj, reserved));
        if (d.region_xyz_mm) fnv(f, d.region_xyz_mm, 12 * (size_t)d.n_regions);
    }
    const size_t eb = 4 * (size_t)(1 + p.KW) * p.E, n = std::min<size_t>(eb, 4096);
    if (n) {
        std::vector<unsigned char> a(2 * n);
        const unsigned char* e = reinterpret_cast<const unsigned char*>(h->net.edge);
        HIPCHK(h, hipMemcpy(a.data(), e, n, hipMemcpyDeviceToHost), "hipMemcpy");
        HIPCHK(h, hipMemcpy(a.data() + n, e + eb - n, n, hipMemcpyDeviceToHost), "hipMemcpy");
        fnv(f, a.data(), a.size());
    }
    *out = f;
    return DBSIM_OK;
}

// Saved spike history of the bins b0 .. bin-1 (the fan-in of the coming bins reads them).
int ck_history(dbsim* h, uint64_t bin, uint64_t* b0, std::vector<unsigned long long>& st,
               std::vector<uint32_t>& cnt) {
    const Plan& p = h->plan;
    *b0 = bin > p.D ? bin - p.D : 0;
    st.assign(p.MB, 0);
    cnt.assign(p.MB, 0);
    HIPCHK(h, hipMemcpy(st.data(), h->net.bin_start, 8 * (size_t)p.MB, hipMemcpyDeviceToHost), "hipMemcpy");
    HIPCHK(h, hipMemcpy(cnt.data(), h->net.bin_cnt, 4 * (size_t)p.MB, hipMemcpyDeviceToHost), "hipMemcpy");
    return DBSIM_OK;
}

size_t ck_bytes(const Plan& p, uint64_t nb, uint64_t n_spk, bool bold) {
    size_t b = up8(sizeof(CkHeader));
    b += up8(4 * (size_t)p.N) * (2 + p.U); // V, Iou, J
    b += up8((size_t)p.N);                 // ref
    b += up8(sizeof(PopParams) * p.n_pops);
    b += up8(4 * nb);                      // per-bin counts
    b += up8(4 * n_spk);
    if (bold) b += 8 * (size_t)p.n_regions * (5 + kBoldRing);
    return b;
}

int ck_check_boundary(dbsim* h) {
    if (h->step % h->plan.S) return fail(DBSIM_ESTATE, "checkpoints are taken at bin boundaries");
    return DBSIM_OK;
}

} // namespace

int dbsim_checkpoint_size(dbsim* h, uint64_t* bytes) {
    int rc = check_usable(h);
    if (rc) return rc;
    if (!bytes) return fail(DBSIM_EINVAL, "bytes is NULL");
    if ((rc = ck_check_boundary(h))) return rc;
    DeviceGuard dg(h->device);
    if ((rc = sync_and_check(h))) return rc;
    const Plan& p = h->plan;
    const uint64_t bin = h->step / p.S;
    uint64_t b0;
    std::vector<unsigned long long> st;
    std::vector<uint32_t> cnt;
    if ((rc = ck_history(h, bin, &b0, st, cnt))) return rc;
    uint64_t n_spk = 0;
    for (uint64_t b = b0; b < bin; b++) n_spk += cnt[b & (p.MB - 1)];
    *bytes = ck_bytes(p, bin - b0, n_spk, h->net.bold_on != 0);
    return DBSIM_OK;
}

int dbsim_checkpoint_save(dbsim* h, void* buf, uint64_t cap, uint64_t* n_out) {
    int rc = check_usable(h);
    if (rc) return rc;
    if (!n_out) return fail(DBSIM_EINVAL, "n_out is NULL");
    if ((rc = ck_check_boundary(h))) return rc;
    DeviceGuard dg(h->device);
    if ((rc = sync_and_check(h))) return rc;
    const Plan& p = h->plan;
    const DevNet& n = h->net;
    const uint64_t bin = h->step / p.S;
    uint64_t b0;
    std::vector<unsigned long long> st;
    std::vector<uint32_t> cnt;
    if ((rc = ck_history(h, bin, &b0, st, cnt))) return rc;
    const uint64_t m = p.MB - 1;
    uint64_t n_spk = 0;
    for (uint64_t b = b0; b < bin; b++) n_spk += cnt[b & m];
    const bool bold = n.bold_on != 0;
    const size_t need = ck_bytes(p, bin - b0, n_spk, bold);
    *n_out = need;
    if (cap < need) return fail(DBSIM_ETRUNC, "buffer too small; *n_out holds the size needed");
    if (!buf) return fail(DBSIM_EINVAL, "buf is NULL");
    Ctl c{};
    HIPCHK(h, hipMemcpy(&c, n.ctl, sizeof c, hipMemcpyDeviceToHost), "hipMemcpy(ctl)");
    CkHeader hd{};
    std::memcpy(hd.magic, kCkMagic, 8);
    if ((rc = ck_fingerprint(h, &hd.fingerprint))) return rc;
    hd.N = p.N;
    hd.U = p.U;
    hd.n_pops = p.n_pops;
    hd.n_regions = p.n_regions;
    hd.D = p.D;
    hd.S = p.S;
    hd.bin = bin;
    hd.edge_events = c.edge_events;
    hd.spikes = c.spikes;
    hd.inject_until = c.inject_until;
    hd.b0 = b0;
    hd.off0 = st[b0 & m];
    hd.n_spk = n_spk;
    hd.bold_on = bold;
    hd.tr_bins = n.tr_bins;
    const double bw[10] = {n.bw_h, n.bw_htau, n.bw_kappa, n.bw_gamma, n.bw_inv_alpha,
                           n.bw_rho, n.bw_V0, n.bw_k1, n.bw_k2, n.bw_k3};
    std::memcpy(hd.bw, bw, sizeof bw);
    if (bold) HIPCHK(h, hipMemcpy(hd.bold_ctl, n.bold_ctl, 16, hipMemcpyDeviceToHost), "hipMemcpy");
    unsigned char* o = static_cast<unsigned char*>(buf);
    std::memset(o, 0, need);
    std::memcpy(o, &hd, sizeof hd);
    size_t at_ = up8(sizeof hd);
    const size_t N = p.N;
    HIPCHK(h, hipMemcpy(o + at_, n.V, 4 * N, hipMemcpyDeviceToHost), "hipMemcpy");
    at_ += up8(4 * N);
    HIPCHK(h, hipMemcpy(o + at_, n.Iou, 4 * N, hipMemcpyDeviceToHost), "hipMemcpy");
    at_ += up8(4 * N);
    HIPCHK(h, hipMemcpy(o + at_, n.J, 4 * N * p.U, hipMemcpyDeviceToHost), "hipMemcpy");
    at_ += up8(4 * N) * p.U;
    HIPCHK(h, hipMemcpy(o + at_, n.ref, N, hipMemcpyDeviceToHost), "hipMemcpy");
    at_ += up8(N);
    HIPCHK(h, hipMemcpy(o + at_, n.pops, sizeof(PopParams) * p.n_pops, hipMemcpyDeviceToHost), "hipMemcpy");
    at_ += up8(sizeof(PopParams) * p.n_pops);
    uint32_t* bc = reinterpret_cast<uint32_t*>(o + at_);
    for (uint64_t b = b0; b < bin; b++) bc[b - b0] = cnt[b & m];
    at_ += up8(4 * (bin - b0));
    // the entries of bins b0 .. bin-1 are contiguous in the ring (mod its size)
    {
        uint64_t a = hd.off0 & (p.RC - 1), left = n_spk, w = 0;
        while (left) {
            const uint64_t k = std::min<uint64_t>(left, p.RC - a);
            HIPCHK(h, hipMemcpy(o + at_ + 4 * w, n.rec + a, 4 * k, hipMemcpyDeviceToHost), "hipMemcpy");
            w += k;
            left -= k;
            a = 0;
        }
    }
    at_ += up8(4 * n_spk);
    if (bold) {
        const size_t R = p.n_regions;
        HIPCHK(h, hipMemcpy(o + at_, n.bold_zs, 8 * R, hipMemcpyDeviceToHost), "hipMemcpy");
        at_ += 8 * R;
        HIPCHK(h, hipMemcpy(o + at_, n.bold, 8 * 4 * R, hipMemcpyDeviceToHost), "hipMemcpy");
        at_ += 8 * 4 * R;
        HIPCHK(h, hipMemcpy(o + at_, n.bold_y, 8 * (size_t)kBoldRing * R, hipMemcpyDeviceToHost), "hipMemcpy");
        at_ += 8 * (size_t)kBoldRing * R;
    }
    return DBSIM_OK;
}

int dbsim_checkpoint_restore(dbsim* h, const void* buf, uint64_t len) {
    int rc = check_usable(h);
    if (rc) return rc;
    if (!buf) return fail(DBSIM_EINVAL, "buf is NULL");
    if (h->step != 0) return fail(DBSIM_ESTATE, "a checkpoint is restored into a handle that has not been stepped");
    const Plan& p = h->plan;
    CkHeader hd;
    if (len < sizeof hd) return fail(DBSIM_EINVAL, "checkpoint too short");
    std::memcpy(&hd, buf, sizeof hd);
    if (std::memcmp(hd.magic, kCkMagic, 8) != 0) return fail(DBSIM_EINVAL, "not a checkpoint of this library");
    if (hd.N != p.N || hd.U != p.U || hd.n_pops != p.n_pops || hd.n_regions != p.n_regions || hd.D != p.D ||
        hd.S != p.S)
        return fail(DBSIM_EINVAL, "the checkpoint belongs to a network of other sizes");
    if (hd.b0 > hd.bin || hd.bin - hd.b0 > p.D || hd.n_spk > (uint64_t)p.D * p.N || hd.tr_bins == 0)
        return fail(DBSIM_EINVAL, "corrupt checkpoint header");
    const bool bold = hd.bold_on != 0;
    if (bold && !p.regions_on) return fail(DBSIM_EINVAL, "the checkpoint has BOLD state; the handle records no regions");
    const size_t need = ck_bytes(p, hd.bin - hd.b0, hd.n_spk, bold);
    if (len < need) return fail(DBSIM_EINVAL, "checkpoint shorter than its header says");
    DeviceGuard dg(h->device);
    if ((rc = sync_and_check(h))) return rc;
    uint64_t fp;
    if ((rc = ck_fingerprint(h, &fp))) return rc;
    if (fp != hd.fingerprint) return fail(DBSIM_EINVAL, "the checkpoint belongs to another network");
    const unsigned char* in = static_cast<const unsigned char*>(buf);
    const size_t N = p.N;
    DevNet& n = h->net;
    size_t at_ = up8(sizeof hd);
    const unsigned char* V = in + at_;
    at_ += up8(4 * N);
    const unsigned char* Iou = in + at_;
    at_ += up8(4 * N);
    const unsigned char* J = in + at_;
    at_ += up8(4 * N) * p.U;
    const unsigned char* ref = in + at_;
    at_ += up8(N);
    const unsigned char* pops = in + at_;
    at_ += up8(sizeof(PopParams) * p.n_pops);
    const uint32_t* bc = reinterpret_cast<const uint32_t*>(in + at_);
    at_ += up8(4 * (hd.bin - hd.b0));
    const unsigned char* spk = in + at_;
    at_ += up8(4 * hd.n_spk);
    uint64_t tot = 0;
    for (uint64_t b = hd.b0; b < hd.bin; b++) tot += bc[b - hd.b0];
    if (tot != hd.n_spk) return fail(DBSIM_EINVAL, "corrupt checkpoint: spike counts do not add up");
    HIPCHK(h, hipMemcpy(n.V, V, 4 * N, hipMemcpyHostToDevice), "hipMemcpy");
    HIPCHK(h, hipMemcpy(n.Iou, Iou, 4 * N, hipMemcpyHostToDevice), "hipMemcpy");
    HIPCHK(h, hipMemcpy(n.J, J, 4 * N * p.U, hipMemcpyHostToDevice), "hipMemcpy");
    HIPCHK(h, hipMemcpy(n.ref, ref, N, hipMemcpyHostToDevice), "hipMemcpy");
    HIPCHK(h, hipMemcpy((void*)n.pops, pops, sizeof(PopParams) * p.n_pops, hipMemcpyHostToDevice), "hipMemcpy");
    // spike history: the saved bins at their original stream offsets
    const uint64_t m = p.MB - 1;
    std::vector<unsigned long long> st(p.MB, 0);
    std::vector<uint32_t> cnt(p.MB, 0);
    uint64_t off = hd.off0;
    for (uint64_t b = hd.b0; b < hd.bin; b++) {
        st[b & m] = off;
        cnt[b & m] = bc[b - hd.b0];
        off += bc[b - hd.b0];
    }
    st[hd.bin & m] = off;
    HIPCHK(h, hipMemcpy(n.bin_start, st.data(), 8 * (size_t)p.MB, hipMemcpyHostToDevice), "hipMemcpy");
    HIPCHK(h, hipMemcpy(n.bin_cnt, cnt.data(), 4 * (size_t)p.MB, hipMemcpyHostToDevice), "hipMemcpy");
    {
        uint64_t a = hd.off0 & (p.RC - 1), left = hd.n_spk, w = 0;
        while (left) {
            const uint64_t k = std::min<uint64_t>(left, p.RC - a);
            HIPCHK(h, hipMemcpy(n.rec + a, spk + 4 * w, 4 * k, hipMemcpyHostToDevice), "hipMemcpy");
            w += k;
            left -= k;
            a = 0;
        }
    }
    if (p.host_record) h->hbend[hd.bin & (p.HMB - 1)] = off; // the host record starts at this bin
    if (bold) {
        const size_t R = p.n_regions;
        HIPCHK(h, hipMemcpy((void*)n.bold_zs, in + at_, 8 * R, hipMemcpyHostToDevice), "hipMemcpy");
        at_ += 8 * R;
        HIPCHK(h, hipMemcpy(n.bold, in + at_, 8 * 4 * R, hipMemcpyHostToDevice), "hipMemcpy");
        at_ += 8 * 4 * R;
        HIPCHK(h, hipMemcpy(n.bold_y, in + at_, 8 * (size_t)kBoldRing * R, hipMemcpyHostToDevice), "hipMemcpy");
        at_ += 8 * (size_t)kBoldRing * R;
        HIPCHK(h, hipMemcpy(n.bold_ctl, hd.bold_ctl, 16, hipMemcpyHostToDevice), "hipMemcpy");
        n.bw_h = hd.bw[0];
        n.bw_htau = hd.bw[1];
        n.bw_kappa = hd.bw[2];
        n.bw_gamma = hd.bw[3];
        n.bw_inv_alpha = hd.bw[4];
        n.bw_rho = hd.bw[5];
        n.bw_V0 = hd.bw[6];
        n.bw_k1 = hd.bw[7];
        n.bw_k2 = hd.bw[8];
        n.bw_k3 = hd.bw[9];
        n.tr_bins = (uint32_t)hd.tr_bins;
    }
    n.bold_on = bold ? 1 : 0;
    // counters; the next bin's delay >= 2 events, which the saved handle had assembled ahead
    // while its last bin ran, are assembled again here from the restored spike history
    Ctl c{};
    c.edge_events = hd.edge_events;
    c.spikes = hd.spikes;
    c.inject_until = hd.inject_until;
    const bool ahead = hd.bin >= 1 && p.D >= 2;
    c.bin = ahead ? hd.bin - 1 : hd.bin;
    HIPCHK(h, hipMemcpy(n.ctl, &c, sizeof c, hipMemcpyHostToDevice), "hipMemcpy(ctl)");
    if (ahead) {
        HIPCHK(h, enqueue_ahead(h, h->stream), "partition launch");
        HIPCHK(h, launch_pass_reset(n, h->stream), "reset launch");
        HIPCHK(h, hipStreamSynchronize(h->stream), "hipStreamSynchronize");
        const unsigned long long b = hd.bin;
        HIPCHK(h, hipMemcpy(&n.ctl->bin, &b, sizeof b, hipMemcpyHostToDevice), "hipMemcpy(ctl)");
    }
    // the kernels take the network descriptor by value: re-capture the graphs
    if (h->g_multi) (void)hipGraphExecDestroy(h->g_multi);
    if (h->g_one) (void)hipGraphExecDestroy(h->g_one);
    h->g_multi = h->g_one = nullptr;
    h->step = hd.bin * p.S;
    h->first_bin = hd.bin;
    return sync_and_check(h);
}


int dbsim_export_csr(dbsim* h, uint64_t* row_ptr, uint32_t* seg, uint32_t* tgt, float* w0, float* w1) {
    int rc = check_usable(h);
    if (rc) return rc;
    DeviceGuard dg(h->device);
    rc = sync_and_check(h);
    if (rc) return rc;
    const Plan& p = h->plan;
    if (row_ptr || seg) { // unpacked from the row headers
        std::vector<uint32_t> hd((size_t)p.N * p.HW);
        HIPCHK(h, hipMemcpy(hd.data(), h->net.hdr, 4 * hd.size(), hipMemcpyDeviceToHost), "hipMemcpy");
        for (size_t j = 0; j < p.N; j++) {
            const uint32_t* hp = &hd[j * p.HW];
            if (row_ptr) row_ptr[j] = ((uint64_t)(hp[1] & 0x7FFFFFFFu) << 32) | hp[0];
            if (seg)
                for (size_t x = 0; x <= p.D; x++) seg[j * (p.D + 1) + x] = hp[2 + x];
        }
        if (row_ptr) row_ptr[p.N] = p.E;
    }
    if (tgt || w0 || w1) { // split the edge records
        const size_t RW = 1 + p.KW;
        std::vector<uint32_t> rec((size_t)p.E * RW);
        HIPCHK(h, hipMemcpy(rec.data(), h->net.edge, 4 * rec.size(), hipMemcpyDeviceToHost), "hipMemcpy");
        for (uint64_t e = 0; e < p.E; e++) { // weights first, then the target
            if (tgt) tgt[e] = rec[e * RW + p.KW] & 0x7FFFFFFFu; // bit 31: the source is inhibitory
            if (w0) std::memcpy(&w0[e], &rec[e * RW], 4);
            if (w1) {
                if (p.KW == 2) std::memcpy(&w1[e], &rec[e * RW + 1], 4);
                else w1[e] = 0.0f;
            }
        }
    }
    return DBSIM_OK;
}

int dbsim_export_network(dbsim* h, dbsim_network_view* v) {
    int rc = check_usable(h);
    if (rc) return rc;
    if (!v) return fail(DBSIM_EINVAL, "null argument");
    const Plan& p = h->plan;
    v->n_pops = p.n_pops;
    if (v->pops && v->pops_cap < p.n_pops) return fail(DBSIM_ETRUNC, "pops_cap too small; n_pops holds the count needed");
    rc = dbsim_export_csr(h, v->row_ptr, v->seg, v->tgt, v->w0, v->w1);
    if (rc) return rc;
    DeviceGuard dg(h->device);
    try {
        if (v->pops) { // what the kernels read: the device copies of the tables
            std::vector<PopParams> pops(p.n_pops);
            std::vector<uint32_t> ptab((size_t)p.n_pops * kMaxPoisson);
            HIPCHK(h, hipMemcpy(pops.data(), h->net.pops, sizeof(PopParams) * pops.size(), hipMemcpyDeviceToHost),
                   "hipMemcpy");
            HIPCHK(h, hipMemcpy(ptab.data(), h->net.ptab, 4 * ptab.size(), hipMemcpyDeviceToHost), "hipMemcpy");
            to_constants(h->mem, p, pops, ptab, v->pops);
        }
        if (v->V0) // the generator's initial potentials, as uploaded at creation
            for (uint32_t m = 0; m < p.n_members; m++)
                for (uint64_t i = h->mem.nbase[m]; i < h->mem.nbase[m + 1]; i++)
                    v->V0[i] = dbnet_v0(&h->mem.m[m], (uint32_t)(i - h->mem.nbase[m]));
    } catch (const std::bad_alloc&) {
        return fail(DBSIM_ENOMEM, "host allocation failed");
    }
    return DBSIM_OK;
}

void dbsim_bold_defaults(dbsim_bold_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->kappa = 0.65;
    p->gamma = 0.41;
    p->tau = 0.98;
    p->alpha = 0.32;
    p->rho = 0.34;
    p->V0 = 0.02;
    p->k1 = 7.0 * p->rho;
    p->k2 = 2.0;
    p->k3 = 2.0 * p->rho - 0.2;
    p->activity_scale = 0.01;
    p->tr_bins = 800;
}

int dbsim_set_bold(dbsim* h, const dbsim_bold_params* bp) {
    int rc = check_usable(h);
    if (rc) return rc;
    const Plan& p = h->plan;
    if (bp) {
        if (!p.regions_on) return fail(DBSIM_EINVAL, "the BOLD model needs DBSIM_REC_REGIONS");
        const double v[] = {bp->kappa, bp->gamma, bp->tau, bp->alpha, bp->rho, bp->V0,
                            bp->k1, bp->k2, bp->k3, bp->activity_scale};
        for (double x : v)
            if (!std::isfinite(x)) return fail(DBSIM_EINVAL, "BOLD parameters must be finite");
        if (!(bp->tau > 0) || !(bp->alpha > 0) || !(bp->rho > 0 && bp->rho < 1) || bp->kappa < 0 ||
            bp->gamma < 0 || bp->activity_scale < 0 || bp->tr_bins < 1)
            return fail(DBSIM_EINVAL, "BOLD parameters out of range (tau, alpha > 0; 0 < rho < 1; kappa, gamma, "
                                      "activity_scale >= 0; tr_bins >= 1)");
    }
    DeviceGuard dg(h->device);
    rc = sync_and_check(h);
    if (rc) return rc;
    DevNet& n = h->net;
    if (bp) {
        const double hs = (double)h->mem.m[0].bin_ms * 1e-3;
        std::vector<uint32_t> rs(p.n_regions);
        HIPCHK(h, hipMemcpy(rs.data(), n.reg_size, 4 * rs.size(), hipMemcpyDeviceToHost), "hipMemcpy");
        std::vector<double> zs(p.n_regions), st(4 * (size_t)p.n_regions, 1.0);
        for (uint32_t r = 0; r < p.n_regions; r++) {
            zs[r] = rs[r] ? bp->activity_scale / ((double)rs[r] * hs) : 0.0;
            st[r] = 0.0; // s = 0, f = v = q = 1
        }
        const unsigned long long zero[2] = {0ull, 0ull};
        HIPCHK(h, hipMemcpy((void*)n.bold_zs, zs.data(), 8 * zs.size(), hipMemcpyHostToDevice), "hipMemcpy");
        HIPCHK(h, hipMemcpy(n.bold, st.data(), 8 * st.size(), hipMemcpyHostToDevice), "hipMemcpy");
        HIPCHK(h, hipMemcpy(n.bold_ctl, zero, sizeof zero, hipMemcpyHostToDevice), "hipMemcpy");
        n.bw_h = hs;
        n.bw_htau = hs / bp->tau;
        n.bw_kappa = bp->kappa;
        n.bw_gamma = bp->gamma;
        n.bw_inv_alpha = 1.0 / bp->alpha;
        n.bw_rho = bp->rho;
        n.bw_V0 = bp->V0;
        n.bw_k1 = bp->k1;
        n.bw_k2 = bp->k2;
        n.bw_k3 = bp->k3;
        n.tr_bins = bp->tr_bins;
        n.bold_on = 1;
    } else {
        n.bold_on = 0;
    }
    // the kernels take the network descriptor by value: re-capture the graphs
    if (h->g_multi) (void)hipGraphExecDestroy(h->g_multi);
    if (h->g_one) (void)hipGraphExecDestroy(h->g_one);
    h->g_multi = h->g_one = nullptr;
    return DBSIM_OK;
}

int dbsim_read_bold(dbsim* h, uint64_t sample_lo, uint64_t sample_hi, double* y, uint64_t cap, uint64_t* n_out) {
    int rc = check_usable(h);
    if (rc) return rc;
    if (!n_out || sample_hi < sample_lo) return fail(DBSIM_EINVAL, "bad arguments");
    const Plan& p = h->plan;
    if (!p.regions_on) return fail(DBSIM_EINVAL, "the BOLD model needs DBSIM_REC_REGIONS");
    DeviceGuard dg(h->device);
    rc = sync_and_check(h);
    if (rc) return rc;
    unsigned long long c[2];
    HIPCHK(h, hipMemcpy(c, h->net.bold_ctl, sizeof c, hipMemcpyDeviceToHost), "hipMemcpy");
    const uint64_t have = c[1], first = have > kBoldRing ? have - kBoldRing : 0;
    if (sample_hi > have || sample_lo < first)
        return fail(DBSIM_ERANGE, "BOLD samples " + std::to_string(sample_lo) + ".." + std::to_string(sample_hi) +
                                      " not recorded (have " + std::to_string(first) + ".." + std::to_string(have) + ")");
    const uint64_t R = p.n_regions, need = (sample_hi - sample_lo) * R;
    *n_out = need;
    if (!y || cap < need) return need ? fail(DBSIM_ETRUNC, "output buffer too small") : DBSIM_OK;
    for (uint64_t m = sample_lo; m < sample_hi; m++)
        HIPCHK(h, hipMemcpy(y + (m - sample_lo) * R, h->net.bold_y + (m & (kBoldRing - 1)) * R, 8 * R,
                            hipMemcpyDeviceToHost), "hipMemcpy");
    return DBSIM_OK;
}

int dbsim_read_bold_state(dbsim* h, double* sfvq, uint64_t* n_samples) {
    int rc = check_usable(h);
    if (rc) return rc;
    const Plan& p = h->plan;
    if (!p.regions_on) return fail(DBSIM_EINVAL, "the BOLD model needs DBSIM_REC_REGIONS");
    DeviceGuard dg(h->device);
    rc = sync_and_check(h);
    if (rc) return rc;
    if (sfvq) HIPCHK(h, hipMemcpy(sfvq, h->net.bold, 8 * 4 * (size_t)p.n_regions, hipMemcpyDeviceToHost), "hipMemcpy");
    if (n_samples) {
        unsigned long long c[2];
        HIPCHK(h, hipMemcpy(c, h->net.bold_ctl, sizeof c, hipMemcpyDeviceToHost), "hipMemcpy");
        *n_samples = c[1];
    }
    return DBSIM_OK;
}

int dbsim_set_spike_injection(dbsim* h, const float* prob, uint32_t n_pops, uint64_t bins) {
    int rc = check_usable(h);
    if (rc) return rc;
    const Plan& p = h->plan;
    if (bins && !prob) return fail(DBSIM_EINVAL, "prob is NULL");
    if (bins && n_pops != p.n_pops)
        return fail(DBSIM_EINVAL, "n_pops must equal the handle's " + std::to_string(p.n_pops) + " populations");
    if (h->step % p.S) return fail(DBSIM_ESTATE, "spike injection can only be set at a bin boundary");
    std::vector<uint32_t> thr(p.n_pops, 0u);
    for (uint32_t q = 0; bins && q < p.n_pops; q++) {
        if (!(prob[q] >= 0.0f && prob[q] < 1.0f)) return fail(DBSIM_EINVAL, "injection probabilities must lie in [0, 1)");
        thr[q] = (uint32_t)std::floor((double)prob[q] * 4294967296.0);
    }
    DeviceGuard dg(h->device);
    rc = sync_and_check(h);
    if (rc) return rc;
    std::vector<PopParams> pp(p.n_pops);
    HIPCHK(h, hipMemcpy(pp.data(), h->net.pops, sizeof(PopParams) * pp.size(), hipMemcpyDeviceToHost), "hipMemcpy");
    for (uint32_t q = 0; q < p.n_pops; q++) pp[q].inject_t = thr[q];
    HIPCHK(h, hipMemcpy((void*)h->net.pops, pp.data(), sizeof(PopParams) * pp.size(), hipMemcpyHostToDevice), "hipMemcpy");
    const unsigned long long until = bins ? h->step / p.S + bins : 0ull;
    HIPCHK(h, hipMemcpy(&h->net.ctl->inject_until, &until, sizeof until, hipMemcpyHostToDevice), "hipMemcpy");
    return DBSIM_OK;
}

int dbsim_set_ou_background(dbsim* h, const float* mu, const float* sigma, const float* tau_ms, uint32_t n_pops) {
    int rc = check_usable(h);
    if (rc) return rc;
    const Plan& p = h->plan;
    if (!mu || !sigma || !tau_ms) return fail(DBSIM_EINVAL, "null argument");
    if (n_pops != p.n_pops)
        return fail(DBSIM_EINVAL, "n_pops must equal the handle's " + std::to_string(p.n_pops) + " populations");
    for (uint32_t q = 0; q < n_pops; q++)
        if (!std::isfinite(mu[q]) || !std::isfinite(sigma[q]) || !std::isfinite(tau_ms[q]) || sigma[q] < 0.0f)
            return fail(DBSIM_EINVAL, "OU parameters must be finite with sigma >= 0");
    DeviceGuard dg(h->device);
    rc = sync_and_check(h);
    if (rc) return rc;
    std::vector<PopParams> pp(p.n_pops);
    HIPCHK(h, hipMemcpy(pp.data(), h->net.pops, sizeof(PopParams) * pp.size(), hipMemcpyDeviceToHost), "hipMemcpy");
    std::vector<float> I(p.N); // every neuron belongs to one population: all overwritten below
    uint32_t q = 0;
    for (size_t m = 0; m < h->mem.m.size(); m++) {
        const dbnet_desc& d = h->mem.m[m];
        const double dt = (double)d.dt_ms;
        uint64_t first = h->mem.nbase[m];
        for (uint32_t lq = 0; lq < d.n_pops; lq++, q++) {
            const uint32_t sz = d.pops[lq].size;
            PopParams& P = pp[q];
            P.ou_on = tau_ms[q] > 0.0f ? 1u : 0u;
            P.ou_mu = mu[q];
            P.ou_c1 = P.ou_on ? (float)(dt / (double)tau_ms[q]) : 0.0f;
            P.ou_c2 = P.ou_on ? (float)((double)sigma[q] * std::sqrt(2.0 * dt / (double)tau_ms[q])) : 0.0f;
            // the current starts at its mean (or 0 when off)
            for (uint64_t i = first; i < first + sz; i++) I[i] = P.ou_on ? mu[q] : 0.0f;
            first += sz;
        }
    }
    HIPCHK(h, hipMemcpy((void*)h->net.pops, pp.data(), sizeof(PopParams) * pp.size(), hipMemcpyHostToDevice), "hipMemcpy");
    HIPCHK(h, hipMemcpy(h->net.Iou, I.data(), 4 * I.size(), hipMemcpyHostToDevice), "hipMemcpy");
    return DBSIM_OK;
}

int dbsim_get_tuning(dbsim* h, dbsim_tuning* t) {
    if (!h || !t) return fail(DBSIM_EINVAL, "null argument");
    t->scatter_wgs_per_cu = h->scatter_wgs;
    t->round_events = h->net.round_events;
    t->chunks_per_wg = h->net.chunks_per_wg;
    t->ahead_passes = h->plan.blocked ? 1u : h->net.ahead_passes;
    return DBSIM_OK;
}

int dbsim_set_tuning(dbsim* h, const dbsim_tuning* t) {
    int rc = check_usable(h);
    if (rc) return rc;
    if (!t) return fail(DBSIM_EINVAL, "null argument");
    if (t->scatter_wgs_per_cu < 1 || t->scatter_wgs_per_cu > 8) return fail(DBSIM_EINVAL, "scatter_wgs_per_cu must lie in 1..8");
    const bool blocked = h->plan.blocked;
    // single pass: workgroups of kFanThreads threads, at most two per CU, whose carry buffers fit
    const uint32_t fan_c = blocked ? fan_chunk_records(h->plan, t->scatter_wgs_per_cu) : 0u;
    if (blocked && (t->scatter_wgs_per_cu > 2 || fan_c == 0))
        return fail(DBSIM_EINVAL, "this schedule does not fit the LDS (single pass: 1 or 2 workgroups per CU)");
    if (t->chunks_per_wg < 1 || t->chunks_per_wg > 64) return fail(DBSIM_EINVAL, "chunks_per_wg must lie in 1..64");
    const uint32_t pmax = std::max(1u, h->plan.D - 1);
    if (t->ahead_passes > pmax) return fail(DBSIM_EINVAL, "ahead_passes must lie in 0..max delay - 1");
    const uint32_t rmax = max_round_events(h->plan, t->scatter_wgs_per_cu);
    const uint32_t bmax = max_bucket_events(h->plan, t->scatter_wgs_per_cu);
    if (rmax == 0 || bmax == 0) return fail(DBSIM_EINVAL, "this schedule does not fit the LDS");
    const uint32_t re = t->round_events ? t->round_events : rmax;
    if (re % 256 || re > rmax) return fail(DBSIM_EINVAL, "round_events must be a multiple of 256 that fits the LDS");
    DeviceGuard dg(h->device);
    rc = sync_and_check(h);
    if (rc) return rc;
    h->scatter_wgs = t->scatter_wgs_per_cu;
    h->scatter_grid = std::min((int)(blocked ? kFanMaxGrid : kMaxPartGrid), (int)h->scatter_wgs * h->num_cus);
    h->net.fan_C = fan_c;
    h->net.round_events = re;
    h->net.bucket_events = std::min(bmax, std::max<uint32_t>(re / kScatterThreads, 1u) * kScatterThreads);
    h->net.chunks_per_wg = t->chunks_per_wg;
    h->net.ahead_passes = t->ahead_passes ? t->ahead_passes : default_ahead_passes(h->plan);
    if (h->g_multi) (void)hipGraphExecDestroy(h->g_multi);
    if (h->g_one) (void)hipGraphExecDestroy(h->g_one);
    h->g_multi = h->g_one = nullptr;
    return DBSIM_OK;
}

int dbsim_set_timing(dbsim* h, int on) {
    int rc = check_usable(h);
    if (rc) return rc;
    if (on && h->static_mem) return fail(DBSIM_ESTATE, "phase timers create HIP events; a handle of "
                                                       "dbsim_create_static has none");
    h->timing = on != 0;
    return DBSIM_OK;
}

int dbsim_get_stats(dbsim* h, dbsim_stats* s) {
    if (!h || !s) return fail(DBSIM_EINVAL, "null argument");
    std::memset(s, 0, sizeof *s);
    DeviceGuard dg(h->device);
    Ctl c{};
    if (!h->dead) {
        int rc = sync_and_check(h);
        if (rc) return rc;
        HIPCHK(h, hipMemcpy(&c, h->net.ctl, sizeof c, hipMemcpyDeviceToHost), "hipMemcpy(ctl)");
    }
    s->steps = h->step;
    s->bins = c.bin;
    s->spikes = c.spikes;
    s->edge_events = c.edge_events;
    s->num_neurons = h->plan.N;
    s->num_edges = h->plan.E;
    s->hbm_bytes = h->plan.total;
    s->timed_bins = h->timed_bins;
    s->ms_scatter = h->ms[0];
    s->ms_gather = h->ms[1];
    s->ms_neuron = h->ms[2];
    s->ms_readout = h->ms[3];
    s->build_seconds = h->build_seconds;
    s->spilled_events = c.spilled;
    s->overflow_events = c.overflow;
    return DBSIM_OK;
}

int dbsim_destroy(dbsim* h) {
    if (!h) return DBSIM_OK;
    {
        DeviceGuard dg(h->device);
        if (h->stream || h->static_mem) (void)hipStreamSynchronize(h->stream);
        release_device(h);
    }
    delete h;
    return DBSIM_OK;
}

} // extern "C"
