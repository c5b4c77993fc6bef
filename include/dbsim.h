/*
 * dbsim.h - C ABI of the MI355X spiking-network step library (libdbsim.so).
 *
 * The library advances one GPU's share of a Digital Brain network
 * (Lu et al., "Simulation and assimilation of the digital human brain"):
 * leaky integrate-and-fire neurons with four receptor conductances
 * (Methods, CV equation and eq. 2), explicit Euler-Maruyama steps of dt with
 * spikes exchanged once per bin b_t (SI Section 3, eqs. 3 and 5 and the
 * definition of A_j), and the fan-out of each bin's spikes through a sparse
 * synapse table (the push-based integration of Suppl. Algorithm 2), extended
 * with integer synaptic delays (the paper has none; one bin reproduces it).
 *
 * The workflow follows the paper's statement of the simulation steps
 * (Methods, end of "Simulating Digital Brain on GPUs"): build the neuron
 * attribute and connection tables from a description, load and deploy them,
 * initialise, run while recording spikes and population signals.
 *
 * Conventions
 *  - All functions return a dbsim_status (0 = success, negative = error);
 *    dbsim_last_error() gives a message for the calling thread.
 *  - Host buffers passed in are owned by the caller and are not retained.
 *    Device memory is owned by the library (allocated through the caller's
 *    callbacks when given, else hipMalloc) and released by dbsim_destroy.
 *  - A handle is not thread-safe; distinct handles may be used concurrently.
 *  - After DBSIM_EDEVICE or DBSIM_EOVERFLOW the handle is dead: only
 *    dbsim_destroy (and the read-only query calls) remain valid.
 *  - Step n covers simulated time [n dt, (n+1) dt); bin k covers steps
 *    kS .. kS+S-1 with S = bin_ms / dt_ms.
 */
#ifndef DBSIM_H
#define DBSIM_H

#include <stddef.h>
#include <stdint.h>

#include "dbnet.h"

#ifdef __cplusplus
extern "C" {
#endif

#define DBSIM_ABI_VERSION 3u

typedef enum dbsim_status {
    DBSIM_OK = 0,
    DBSIM_EINVAL = -1,    /* invalid argument or description */
    DBSIM_ENOMEM = -2,    /* host allocation failed */
    DBSIM_EHBM = -3,      /* device allocation failed (handle not created) */
    DBSIM_EDEVICE = -4,   /* HIP runtime error (sticky) */
    DBSIM_ETRUNC = -5,    /* output buffer too small; the needed count is returned */
    DBSIM_EOVERFLOW = -6, /* a device-side capacity was exceeded (sticky) */
    DBSIM_ESTATE = -7,    /* call not valid in the handle's current state */
    DBSIM_ERANGE = -8     /* requested steps/bins are not (or no longer) recorded */
} dbsim_status;

/* Device-memory callbacks (e.g. a framework's caching allocator). alloc
   returns a device pointer aligned to at least 256 bytes, or NULL. */
typedef void* (*dbsim_alloc_fn)(void* ctx, size_t bytes);
typedef void (*dbsim_free_fn)(void* ctx, void* ptr, size_t bytes);

/* record_flags */
#define DBSIM_REC_REGIONS 1u /* per-bin region signal and spike counts */

typedef struct dbsim_desc {
    uint32_t abi_version;           /* DBSIM_ABI_VERSION */
    uint32_t record_flags;          /* DBSIM_REC_* */
    dbnet_desc net;                 /* the seeded network description (dbnet.h) */
    uint64_t spike_record_capacity; /* spike entries kept on the device (rounded up to
                                       a power of two >= (max delay + 1) * N); 0 = that
                                       minimum while spikes are recorded to host memory
                                       (host_spike_capacity), else 2^22 */
    uint32_t record_bins;           /* bins of spike/region history kept (power of two,
                                       >= max delay + 1); 0 = 4096 */
    int32_t device;                 /* HIP device ordinal, -1 = the current device */
    void* hip_stream;               /* hipStream_t to run on; NULL = a stream of the library */
    dbsim_alloc_fn dev_alloc;       /* optional device allocator (NULL = hipMalloc) */
    dbsim_free_fn dev_free;         /* required when dev_alloc is given */
    void* alloc_ctx;
    uint32_t host_threads;          /* threads for network construction, 0 = all cores */
    uint32_t flags;                 /* DBSIM_F_* */
    uint64_t host_spike_capacity;   /* spike entries recorded in pinned host memory (rounded
                                       up to a power of two); 0 = 2^24; unused with
                                       DBSIM_F_NO_HOST_RECORD. The last 2^20 bins' offsets are
                                       kept beside them. */
    uint32_t stream_permille;       /* two-pass form: records each super-tile stream holds per
                                       partition pass, in thousandths of the super-tile's
                                       in-edges (1..1000; 1000 = every edge, the most one pass
                                       can carry). 0 = 125, and at least 2^20 records (or all
                                       in-edges, if fewer). Runs that find their stream full
                                       go straight to the tile arena, one atomic per event:
                                       slower, same results (dbsim_stats.spilled_events). */
    uint32_t arena_permille;        /* two-pass form: records each tile's arena slice holds per
                                       bin, in thousandths of the tile's in-edges (1..1000;
                                       1000 = every edge, the most one bin can deliver). 0 =
                                       125, and at least 2^16 records (or all in-edges, if
                                       fewer). Events that find their slice full are summed
                                       into an exact int64 accumulator per target with one
                                       atomic each: slower, same results
                                       (dbsim_stats.overflow_events). */
} dbsim_desc;

/* flags */
#define DBSIM_F_NO_GRAPH 1u /* launch kernels directly instead of replaying HIP graphs */
#define DBSIM_F_NO_HOST_RECORD 4u /* keep the raster only in the device ring (no pinned host
                                     memory; reads copy from the device) */
#define DBSIM_F_HOST_BUILD 8u /* build the connection table on the host threads even where the
                                 device construction applies (same table; for comparisons) */
#define DBSIM_F_SINGLE_PASS 2u /* fan-in in one pass into per-workgroup blocks of each tile
                                  (no super-tile streams; slower on every measured network);
                                  taken where the tiles' carry buffers fit one workgroup's
                                  LDS (up to about 2,900 tiles), else the default two
                                  passes. Same results. */

typedef struct dbsim_stats {
    uint64_t steps;        /* Euler steps completed (queued) */
    uint64_t bins;         /* bins completed */
    uint64_t spikes;       /* spikes emitted in completed bins */
    uint64_t edge_events;  /* synaptic events delivered (edge whose source spike arrived) */
    uint64_t num_neurons;
    uint64_t num_edges;
    uint64_t hbm_bytes;    /* device bytes held by the handle */
    uint64_t timed_bins;   /* bins covered by the phase timers below */
    double ms_scatter;     /* summed kernel time per phase while timing is on */
    double ms_gather;
    double ms_neuron;
    double ms_readout;
    double build_seconds;  /* time spent constructing the network: the host phase, plus the
                              device construction of the connection table where it ran (its
                              duration is added at the first synchronisation after create) */
    uint64_t spilled_events;  /* partitioned events (this handle's bins, and the next bin's
                                 part assembled ahead) that found their super-tile stream
                                 full and were placed in the tile arena directly */
    uint64_t overflow_events; /* likewise, events that found their tile's arena slice full
                                 and were summed into the per-target accumulator */
} dbsim_stats;

typedef struct dbsim_info {
    uint64_t num_neurons, num_edges;
    uint32_t receptors;        /* |U|: 2 or 4 */
    uint32_t weights_per_edge; /* 1 or 2 */
    uint32_t steps_per_bin;    /* S */
    uint32_t max_delay;        /* D (bins) */
    uint32_t n_regions;
    uint32_t tile_neurons;     /* targets per accumulation tile */
    uint32_t n_tiles;
    uint32_t frac_bits;        /* F of the fixed-point arrival sums */
    uint32_t n_members;        /* networks in the handle (1 unless an ensemble) */
    uint32_t fanin_passes;     /* 1: single-pass fan-in into tile blocks, 2: through super-tile streams */
    uint32_t device_built;     /* 1: the connection table was generated on the device */
    uint32_t stream_record_bytes; /* super-tile stream record: 4 bytes per weight and 4 for
                                     the key (12 or 8), or 10 (a 2-byte key beside the weight
                                     pair, when every weight is non-negative and there are two
                                     per edge); 0 in the single-pass form */
    uint32_t reserved;
    uint64_t stream_records;   /* records the super-tile streams hold in all (0 in the
                                  single-pass form) */
    uint64_t arena_records;    /* records the tile arena holds in all (two-pass form; the
                                  single-pass form's blocks otherwise) */
} dbsim_info;

typedef struct dbsim_member {
    uint64_t first_neuron; /* global id of the member's neuron 0 */
    uint64_t num_neurons;
    uint32_t first_region; /* global index of the member's region 0 */
    uint32_t num_regions;
} dbsim_member;

/* Library ABI version (DBSIM_ABI_VERSION of the build). */
uint32_t dbsim_abi_version(void);

/* Message of the last failure on the calling thread ("" if none). */
const char* dbsim_last_error(void);

/*
 * Builds the network from the seeded description (neuron attribute table,
 * connection table re-laid out by presynaptic neuron, derived constants),
 * allocates device memory, uploads, and sets the initial state (V from the
 * generator, J = 0, not refractory). Host work runs on host_threads threads.
 * Errors: EINVAL (description; message says why), ENOMEM, EHBM (allocation
 * failed; nothing is leaked), EDEVICE.
 */
int dbsim_create(const dbsim_desc* desc, struct dbsim** out);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): dbsim_create with every device array of
 * the handle placed in a static region of DBSIM_STATIC_BYTES per GPU that the library holds
 * from its load to the end of the process. No hipMalloc, hipFree, stream, event or graph
 * is created: dev_alloc must be NULL, and the handle's bins run on desc->hip_stream (NULL:
 * the default stream) as direct launches, one kernel after another, with the same results
 * as dbsim_create (no phase timers: dbsim_set_timing(h, 1) gives ESTATE; spikes are read
 * from the device ring, as with DBSIM_F_NO_HOST_RECORD). Everything the
 * kernels read is initialised here, whatever the region held before (creation copies the
 * tables and synchronises the stream, so it runs outside a capture; the bins it then runs
 * allocate nothing and may be captured by the caller). The region is shared:
 * one such handle per device at a time (ESTATE while another is alive; dbsim_destroy frees
 * the region for the next). Errors: EINVAL when the footprint (dbsim_footprint) exceeds
 * DBSIM_STATIC_BYTES (checked before any device work) or dev_alloc is set; otherwise as
 * dbsim_create.
 */
#define DBSIM_STATIC_BYTES (64u << 20)
int dbsim_create_static(const dbsim_desc* desc, struct dbsim** out);

/*
 * The two steps of dbsim_create apart, following the paper's workflow (Methods: generate the
 * neuron attribute and connection tables, then load and deploy them). dbsim_build validates
 * the description and builds every host table; it makes no HIP call and touches no device, so
 * it may run on worker threads while another thread drives the GPU (a server builds requests
 * that way). dbsim_create_built allocates, uploads and initialises the handle; it consumes b
 * (freed whether it succeeds or not). device_opts (may be NULL: those given to dbsim_build)
 * supplies device, hip_stream, dev_alloc, dev_free and alloc_ctx; its other fields are
 * ignored. dbsim_built_free releases a built network that is not deployed (NULL: no-op).
 * Errors: as dbsim_create.
 */
typedef struct dbsim_built dbsim_built;
int dbsim_build(const dbsim_desc* desc, dbsim_built** out);
int dbsim_create_built(dbsim_built* b, const dbsim_desc* device_opts, struct dbsim** out);
void dbsim_built_free(dbsim_built* b);

/* Exact device bytes dbsim_create would allocate for desc, without building. */
int dbsim_footprint(const dbsim_desc* desc, uint64_t* hbm_bytes);

/*
 * Ensemble of independent networks advanced together by the same kernel
 * launches (the ensemble forward pass of the diffusion ensemble Kalman filter,
 * Suppl. Algorithm 3, evolves many model instances with their own parameters).
 * members[m] are full network descriptions (own seed, net_id, populations,
 * projections, regions); they must share dt_ms, bin_ms, receptor_mask and
 * frac_bits. Runtime options come from common (its net field is ignored).
 * Member m's neurons and regions occupy consecutive global ids (see
 * dbsim_member_info); edges never cross members and each member keeps its own
 * noise stream, so every member's spikes and state are bit-identical to
 * running it alone. Reads return global ids; errors as dbsim_create.
 */
int dbsim_create_ensemble(const dbsim_desc* common, const dbnet_desc* members, uint32_t n_members,
                          struct dbsim** out);

/* Exact device bytes dbsim_create_ensemble would allocate (admission control). */
int dbsim_footprint_ensemble(const dbsim_desc* common, const dbnet_desc* members, uint32_t n_members,
                             uint64_t* hbm_bytes);

/* Global id range and region range of ensemble member `member` (0 for a single network). */
int dbsim_member_info(struct dbsim* h, uint32_t member, dbsim_member* info);

/* Queries sizes of a built network. */
int dbsim_get_info(struct dbsim* h, dbsim_info* info);

/*
 * Advances n_steps Euler steps (any count; partial bins are legal).
 * Asynchronous on the handle's stream; errors from device work surface at
 * the next dbsim_sync or read call.
 */
int dbsim_step(struct dbsim* h, uint64_t n_steps);

/* Waits for queued work; surfaces deferred device errors (EDEVICE, EOVERFLOW). */
int dbsim_sync(struct dbsim* h);

/*
 * Spikes with step_lo <= step < step_hi, sorted by (step, id), copied to
 * steps[] / ids[] (cap entries each). Only completed bins are visible. If
 * cap is too small returns ETRUNC with *n_out = the count needed. ERANGE if
 * part of the range is no longer recorded. Synchronises.
 *
 * Recording (SI Section 3: a second stream copies every iteration's spikes to CPU
 * memory): at the end of every bin, once its spike list is compacted, a kernel on a
 * second stream copies the list into a ring of host_spike_capacity entries in pinned
 * host memory, concurrently with the rest of the bin; reads are served from that ring,
 * so the device ring only needs the last max delay + 1 bins the fan-in reads. With
 * DBSIM_F_NO_HOST_RECORD (and for handles of dbsim_create_static) reads copy from the
 * device ring instead.
 */
int dbsim_read_spikes(struct dbsim* h, uint64_t step_lo, uint64_t step_hi, uint64_t* steps,
                      uint32_t* ids, uint64_t cap, uint64_t* n_out);

/*
 * Region signal for bins bin_lo <= k < bin_hi: sig[(k - bin_lo) * n_regions + r]
 * is the mean over region r's neurons of the total synaptic current
 * sum_u g_u J_u (V_u - V) at the end of bin k (pA); counts (may be NULL)
 * holds the region's spike count in that bin. cap counts entries
 * (bins * regions). Requires DBSIM_REC_REGIONS. Synchronises.
 */
int dbsim_read_region_signal(struct dbsim* h, uint64_t bin_lo, uint64_t bin_hi, double* sig,
                             uint32_t* counts, uint64_t cap, uint64_t* n_out);

/* Host copies of the state: V[N], J[|U| * N] (receptor-major: AMPA, [NMDA],
   GABA_A, [GABA_B]), refractory steps left ref[N]. Any pointer may be NULL. */
int dbsim_read_state(struct dbsim* h, float* V, float* J, int32_t* ref);

/*
 * Region BOLD signal: the Balloon-Windkessel model of Extended Data Table 4,
 * one per region, driven by the region's firing rate (Fig. 2a: firing rates from
 * spike counts feed the haemodynamic model). At the end of every bin k each
 * region r takes one explicit Euler step of length h = bin_ms / 1000 s (FP64):
 *   z  = activity_scale * count_r(k) / (N_r * h)          (rate in Hz, scaled)
 *   s' = s + h * (z - kappa * s - gamma * (f - 1))
 *   f' = f + h * s
 *   v' = v + (h / tau) * (f - v^(1/alpha))
 *   q' = q + (h / tau) * (f * (1 - (1 - rho)^(1/f)) / rho - v^(1/alpha) * q / v)
 * all right-hand sides at the old state; after every tr_bins bins the sample
 *   y = V0 * (k1 * (1 - q) + k2 * (1 - q / v) + k3 * (1 - v))
 * is recorded (a ring of the last 1024 samples per region). The paper gives no
 * constants; the defaults (dbsim_bold_defaults) are the standard ones of the
 * Balloon-Windkessel literature. Requires DBSIM_REC_REGIONS.
 */
typedef struct dbsim_bold_params {
    double kappa;          /* 1/s, decay of the vasodilatory signal (0.65) */
    double gamma;          /* 1/s, autoregulatory feedback (0.41) */
    double tau;            /* s, haemodynamic transit time (0.98) */
    double alpha;          /* Grubb's exponent (0.32) */
    double rho;            /* resting oxygen extraction fraction (0.34) */
    double V0;             /* resting blood volume fraction (0.02) */
    double k1, k2, k3;     /* BOLD coefficients (7 rho, 2, 2 rho - 0.2) */
    double activity_scale; /* z per Hz of region firing rate (0.01) */
    uint32_t tr_bins;      /* bins per BOLD sample, >= 1 (800: TR = 0.8 s at 1 ms bins) */
    uint32_t reserved;
} dbsim_bold_params;

/* Fills the default parameters. */
void dbsim_bold_defaults(dbsim_bold_params* p);

/* Turns the BOLD model on with these parameters (NULL: off) and resets every
   region to rest (s = 0, f = v = q = 1) and the sample count to 0; sampling is
   counted from the next completed bin. EINVAL for non-positive constants or
   without DBSIM_REC_REGIONS. Synchronises. */
int dbsim_set_bold(struct dbsim* h, const dbsim_bold_params* p);

/* BOLD samples m with sample_lo <= m < sample_hi: y[(m - sample_lo) * n_regions + r].
   cap counts entries. ERANGE if part of the range is not (or no longer) recorded;
   ETRUNC if cap is too small (*n_out = entries needed). Synchronises. */
int dbsim_read_bold(struct dbsim* h, uint64_t sample_lo, uint64_t sample_hi, double* y, uint64_t cap,
                    uint64_t* n_out);

/* The Balloon-Windkessel state, sfvq[4 * n_regions]: s, then f, v, q (region-major
   within each). *n_samples (may be NULL) receives the samples taken so far. */
int dbsim_read_bold_state(struct dbsim* h, double* sfvq, uint64_t* n_samples);

/*
 * Initial spike injection (Methods, initialisation of the spike trains): during the next
 * `bins` bins, the output spike train of every neuron of population p carries a spike in
 * a bin with probability prob[p] (the neuron's own draw: word 0 of Philox4x32-10 with key =
 * its network's seed and counter (bin, bin >> 32, local neuron id, 2 << 24 | net_id), below
 * floor(prob * 2^32)). An injected spike is delivered through the neuron's edges like any
 * other and recorded (at the bin's last step when the neuron did not fire itself), but it
 * does not reset the neuron. prob[n_pops] over all populations of the handle (members of an
 * ensemble one after another), each in [0, 1); n_pops must match; bins = 0 turns injection
 * off. Call at a bin boundary (ESTATE otherwise); takes effect from the next bin. Synchronises.
 */
int dbsim_set_spike_injection(struct dbsim* h, const float* prob, uint32_t n_pops, uint64_t bins);

/*
 * Ornstein-Uhlenbeck background current (eq. 1; eq. 4 discretised with the noise scaled as
 * the continuous process requires): for the neurons of population p with tau_ms[p] > 0,
 *   I_bg' = I_bg + c1 (mu - I_bg),   I_bg'' = I_bg' + c2 z,
 * c1 = dt / tau, c2 = sigma sqrt(2 dt / tau) (rounded once to f32), z the standardised sum of
 * twelve 10-bit fields of one Philox4x32-10 block (counter (n, n >> 32, local id,
 * 3 << 24 | net_id)): an exact integer, variance 1 - 2^-20. I_bg enters the membrane current
 * after I_ext (I = I + I_ext, then I = I + I_bg) at the old value, every step, also while
 * refractory. The current is set to mu (0 where tau <= 0, which turns it off). It adds to the
 * Poisson background (set bg_rate_hz = 0 for OU alone). Arrays of n_pops over all populations
 * (members one after another). Synchronises.
 */
int dbsim_set_ou_background(struct dbsim* h, const float* mu, const float* sigma, const float* tau_ms,
                            uint32_t n_pops);

/*
 * The measurement step of the conductance initialisation (Suppl. Algorithm 1: run the
 * off-line model, obtain the mean current of each receptor type) at the current state:
 * mean[q * 4 + u] = the mean over population q's neurons of g_u J_u (V_u - V), u in the
 * paper's order AMPA, NMDA, GABA_A, GABA_B (0 for receptors the network lacks). Each
 * neuron's term is evaluated in float as in the region signal; sums are in double, in a
 * fixed order on the device. n_pops must be the handle's population count (members of an
 * ensemble one after another; EINVAL otherwise). Synchronises.
 */
int dbsim_receptor_currents(struct dbsim* h, double* mean, uint32_t n_pops);

/* Overwrites V, J and the refractory counters of this handle. Only at a bin boundary
   (ESTATE otherwise). ref values must lie in [0, 255]. */
int dbsim_write_state(struct dbsim* h, const float* V, const float* J, const int32_t* ref);

/*
 * Checkpoint and resume of a run (a long simulation continued in another process or
 * after a failure; the clock-driven step of SI Section 3 depends only on this state).
 * A checkpoint is an opaque byte image of everything the coming bins depend on, taken
 * at a bin boundary (ESTATE otherwise): V, J, refractory counters, OU currents, the
 * per-population settings (spike injection, OU background), the spike lists of the last
 * max-delay bins (the fan-in of the coming bins reads them), the counters (steps, bins,
 * spikes, delivered events) and, when the BOLD model is on, its parameters, state and
 * sample ring.
 *
 * dbsim_checkpoint_size: the image's size now (synchronises).
 * dbsim_checkpoint_save: writes it to buf (host memory, caller-owned, cap bytes);
 *   *n_out = the size; ETRUNC if cap is smaller.
 * dbsim_checkpoint_restore: loads an image into a handle created from the same network
 *   description that has not been stepped (ESTATE otherwise); EINVAL for an image of
 *   another network (sizes, descriptions and a sample of the connection table are
 *   compared) or a damaged one. The handle then continues bit-identically to the saved
 *   one. Its spike and region-signal history starts at the checkpoint's bin (earlier bins:
 *   ERANGE); its tuning, timing and launch mode stay its own.
 */
/*
 * The in-edges of one target as the device construction of the connection table draws
 * them, evaluated on the host threads (no device needed): for checking the device
 * generator against the input generator (dbnet_in_edges) edge by edge. members as for
 * dbsim_create_ensemble; target is a global neuron id (members one after another).
 * Writes up to cap edges in the generator's order: global source ids, weights, delays
 * (bins) and the projection index within the member; *n_out = the in-degree (ETRUNC if
 * cap is smaller). EINVAL where the device construction does not apply (lognormal
 * weights) or for an invalid description or target.
 */
int dbsim_check_device_generator(const dbnet_desc* members, uint32_t n_members, uint64_t target, uint32_t* src,
                                 float* w0, float* w1, uint8_t* delay, uint32_t* proj, uint64_t cap,
                                 uint64_t* n_out);

int dbsim_checkpoint_size(struct dbsim* h, uint64_t* bytes);
int dbsim_checkpoint_save(struct dbsim* h, void* buf, uint64_t cap, uint64_t* n_out);
int dbsim_checkpoint_restore(struct dbsim* h, const void* buf, uint64_t len);

/*
 * Host copy of the device connection table: row_ptr[N+1] (edge offsets of
 * each presynaptic row), seg[N * (D+1)] (offset of each delay's first edge
 * within the row; seg[j*(D+1)+d-1] .. seg[j*(D+1)+d] are the delay-d edges),
 * tgt[E], w0[E], w1[E] (w1 ignored and may be NULL with one weight per
 * edge). Rows hold edges sorted by (delay, target).
 */
int dbsim_export_csr(struct dbsim* h, uint64_t* row_ptr, uint32_t* seg, uint32_t* tgt, float* w0,
                     float* w1);

/*
 * Derived constants of one population, as the kernels use them (the discrete step
 * of the Methods' CV equation and eq. 2, SI Section 3, with the readings stated in
 * the header comment): every value is computed in double from the description and
 * rounded once to float, so a CPU implementation of the same step can check them
 * bit for bit (the paper validates its GPU code against a CPU run of a debug graph).
 */
#define DBSIM_MAX_POISSON 64u
typedef struct dbsim_pop_constants {
    uint32_t first_neuron;  /* global id of the population's first neuron */
    uint32_t end_neuron;    /* one past its last neuron */
    uint32_t member;        /* network of the handle (ensemble member) it belongs to */
    uint32_t region;        /* global region index */
    float k;                /* dt / C */
    float g_L, V_L, V_th, V_reset, I_ext, w_bg; /* copied from the description */
    float g[4], V_rev[4];   /* compact receptor order: AMPA, [NMDA], GABA_A, [GABA_B] */
    float decay[4];         /* exp(-dt / tau_u); 1 for tau = +inf */
    int32_t ref_steps;      /* round(T_ref / dt): steps held after a spike */
    uint32_t poisson_len;   /* c_max: entries of poisson_T in use */
    uint32_t poisson_T[DBSIM_MAX_POISSON]; /* T_c = floor(2^32 P(Poisson(lambda) <= c)), lambda =
                                              bg_rate dt, pmf by p_0 = exp(-lambda), p_c = p_{c-1}
                                              lambda / c summed in ascending c; the table ends at
                                              the first c whose upper tail is below 2^-32; the
                                              background count of a step is #{c : T_c <= x} for
                                              the step's 32-bit Philox word x */
} dbsim_pop_constants;

/*
 * Host only (no device is touched, nothing is generated): validates the description(s)
 * as dbsim_create / dbsim_create_ensemble would and writes the derived constants of
 * every population (members one after another) to out[0 .. cap). *n_out receives the
 * population count; ETRUNC if cap is smaller; EINVAL for an invalid description.
 * n_members = 1 with members = &common->net for a single network.
 */
int dbsim_derive_constants(const dbsim_desc* common, const dbnet_desc* members, uint32_t n_members,
                           dbsim_pop_constants* out, uint32_t cap, uint32_t* n_out);

/*
 * Everything the handle built from its description, for a CPU check of the same
 * network (the paper's GPU-vs-CPU comparison of a debug graph): each pointer may be
 * NULL; arrays are caller-owned and sized as stated.
 */
typedef struct dbsim_network_view {
    uint64_t* row_ptr;          /* [N + 1] edge offset of each presynaptic row */
    uint32_t* seg;              /* [N * (D + 1)] delay segment offsets inside each row (as dbsim_export_csr) */
    uint32_t* tgt;              /* [E] target of each edge (rows sorted by delay, then target) */
    float* w0;                  /* [E] first weight */
    float* w1;                  /* [E] second weight (zero with one weight per edge) */
    float* V0;                  /* [N] initial membrane potentials (the values set at creation) */
    dbsim_pop_constants* pops;  /* [pops_cap] read back from the device copy the kernels use */
    uint32_t pops_cap;          /* entries available in pops */
    uint32_t n_pops;            /* out: populations of the handle */
} dbsim_network_view;

/* Fills the view (ETRUNC, with n_pops set, if pops_cap is too small). Synchronises. */
int dbsim_export_network(struct dbsim* h, dbsim_network_view* v);

/*
 * Launch schedule of the fan-in partition kernels. Any valid schedule gives
 * bit-identical results (the arrival sums are exact integers); it only changes
 * speed, so an autotuner may try schedules on a live handle.
 */
typedef struct dbsim_tuning {
    uint32_t scatter_wgs_per_cu; /* partition workgroups per CU (they split the LDS): 1..8 of 512
                                    threads in the two-pass form, 1..2 of 1,024 in the single-pass
                                    form (whose per-tile carry buffers shrink with the LDS share) */
    uint32_t round_events;       /* events per round of the first partition pass, multiple of 256:
                                    two-pass form, staged in LDS, at most 4096 (0 = the most that
                                    fit; the second pass takes the most that fit beside its staging
                                    copy, at most this, rounded down to whole 512-event batches);
                                    single-pass form, held in registers, at most 8192 (0 = 8192) */
    uint32_t chunks_per_wg;      /* target (spike, delay) chunks per partition workgroup in the pass of
                                    delays >= 2, 1..64 (the delay-1 pass uses one) */
    uint32_t ahead_passes;       /* two-pass form: the next bin's delay >= 2 fan-in runs as this many
                                    partition passes over consecutive delay groups (smaller passes keep
                                    their streams cache-resident), 1..max delay - 1; 0 = default; the
                                    single-pass form always runs one */
} dbsim_tuning;

/* Reads / sets the schedule (EINVAL if it does not fit the LDS). Takes effect
   for the next step call; replayed graphs are re-captured. */
int dbsim_get_tuning(struct dbsim* h, dbsim_tuning* t);
int dbsim_set_tuning(struct dbsim* h, const dbsim_tuning* t);

/* Turns per-phase kernel timing (HIP events around each phase of every
   bin) on or off; while on, bins are launched directly, not via graphs. */
int dbsim_set_timing(struct dbsim* h, int on);

/* Counters and timers (synchronises to resolve timers). */
int dbsim_get_stats(struct dbsim* h, dbsim_stats* s);

/* Frees everything; NULL is a no-op. */
int dbsim_destroy(struct dbsim* h);

typedef struct dbsim dbsim;

#ifdef __cplusplus
}
#endif
#endif /* DBSIM_H */
