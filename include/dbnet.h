/*
 * dbnet.h - seeded synthetic network description and its generator.
 *
 * This is the input-generator module. It turns a small description
 * (populations, projections, regions, seed) into a concrete network: the
 * incoming edges of every neuron (source, receptor weights, integer delay)
 * and every neuron's initial membrane potential. It contains none of the
 * simulation arithmetic; the simulator library (dbsim.h) and the CPU oracle
 * both call it so that they see the same network.
 *
 * Network model (Methods "Constructing the Digital Brain model", Suppl.
 * Section 2 and Extended Data Table 2):
 *  - neurons belong to excitatory or inhibitory populations (the 4:1 ratio is
 *    a choice of the description, not of this code);
 *  - excitatory sources act through AMPA and NMDA, inhibitory ones through
 *    GABA_A and GABA_B; each edge carries one weight per receptor of its
 *    source class (Suppl. Table 5 stores two weight channels per edge);
 *  - connectivity is a fixed in-degree ("k-random") graph: for every target,
 *    sources are drawn uniformly *without replacement* from the candidate
 *    set, never the target itself (no autapses, no multapses);
 *  - weights are fixed; Extended Data Table 2 uses U[0,1];
 *  - integer synaptic delays (in spike bins) are an extension: the paper's
 *    Discussion states its model has none. A delay of one bin reproduces the
 *    paper's delivery at the next bin boundary exactly.
 *
 * Determinism: every random draw comes from a counter-based hash keyed by
 * (seed, net_id, target, projection, index), so the network does not depend
 * on thread count or generation order.
 *
 * All functions are plain C, thread-safe (no global state) and allocate
 * nothing except where stated.
 */
#ifndef DBNET_H
#define DBNET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DBNET_ABI_VERSION 1u

/* Receptor indices in the paper's order (Methods eq. 2). */
enum { DBNET_AMPA = 0, DBNET_NMDA = 1, DBNET_GABA_A = 2, DBNET_GABA_B = 3 };

/* Receptor masks accepted by the generator and both simulators. */
#define DBNET_RECEPTORS_2 0x5u /* AMPA + GABA_A: one weight per edge */
#define DBNET_RECEPTORS_4 0xFu /* AMPA, NMDA, GABA_A, GABA_B: two weights per edge */

/* Source candidate sets of a projection, relative to the target neuron. */
enum {
    DBNET_SRC_ALL = 0,           /* every population */
    DBNET_SRC_SAME_REGION = 1,   /* populations of the target's region */
    DBNET_SRC_OTHER_REGIONS = 2, /* populations of every other region */
    DBNET_SRC_POP = 3            /* the single population src_pop */
};
/* Class filter applied on top of the candidate set. */
enum { DBNET_CLASS_ANY = 0, DBNET_CLASS_EXC = 1, DBNET_CLASS_INH = 2 };
/* Weight distributions. */
enum { DBNET_W_UNIFORM = 0, DBNET_W_LOGNORMAL = 1, DBNET_W_CONST = 2 };
/* Delay rules (delays are in bins of bin_ms). */
enum { DBNET_D_FIXED = 0, DBNET_D_UNIFORM = 1, DBNET_D_DISTANCE = 2 };

/*
 * One population: a contiguous block of neuron ids, homogeneous parameters
 * (Suppl. Table 5 lists the per-neuron property columns; the paper sets
 * homogeneous values per parameter type, SI Section 3 "Numerical method").
 * Units: mV, ms, nS, pF, pA, Hz.
 */
typedef struct dbnet_pop {
    uint32_t size;    /* number of neurons */
    uint32_t exc;     /* 1: excitatory source (AMPA/NMDA), 0: inhibitory (GABA_A/GABA_B) */
    uint32_t region;  /* region index < n_regions */
    uint32_t reserved;
    float C;          /* membrane capacitance (pF) */
    float g_L;        /* leak conductance (nS) */
    float V_L;        /* leak reversal (mV) */
    float V_th;       /* threshold (mV) */
    float V_reset;    /* reset / refractory clamp (mV) */
    float T_ref;      /* refractory period (ms) */
    float I_ext;      /* constant external current (pA) */
    float g[4];       /* maximal conductance per receptor (nS), AMPA..GABA_B */
    float V_rev[4];   /* receptor reversal potentials (mV) */
    float tau[4];     /* receptor decay time constants (ms); +inf means no decay */
    float bg_rate_hz; /* Poisson background rate per neuron (Hz) */
    float w_bg;       /* weight of one background spike on AMPA */
    float v0_lo;      /* initial V ~ U[v0_lo, v0_hi) */
    float v0_hi;
} dbnet_pop;

/* One projection: rule for part of the in-degree of every target in dst_pop. */
typedef struct dbnet_proj {
    int32_t dst_pop;     /* target population, or -1 for every population */
    uint32_t src_mode;   /* DBNET_SRC_* */
    uint32_t src_class;  /* DBNET_CLASS_* */
    int32_t src_pop;     /* population for DBNET_SRC_POP, else ignored */
    uint32_t indegree;   /* sources drawn per target */
    uint32_t w_dist;     /* DBNET_W_* */
    float w_a, w_b;      /* uniform [a,b); lognormal (mu, sigma) of log w; const a */
    float w_scale_exc;   /* weight multiplier for excitatory sources */
    float w_scale_inh;   /* weight multiplier for inhibitory sources */
    uint32_t d_mode;     /* DBNET_D_* */
    uint32_t d_min;      /* delay bins: fixed value, or lower clamp / bound */
    uint32_t d_max;      /* delay bins: upper clamp / bound */
    uint32_t reserved;
} dbnet_proj;

typedef struct dbnet_desc {
    uint32_t abi_version;   /* DBNET_ABI_VERSION */
    uint32_t n_pops;
    uint32_t n_projs;
    uint32_t n_regions;
    uint64_t seed;          /* network and background-noise seed */
    float dt_ms;            /* Euler step */
    float bin_ms;           /* spike bin; bin_ms/dt_ms must be an integer */
    uint32_t receptor_mask; /* DBNET_RECEPTORS_2 or DBNET_RECEPTORS_4 */
    uint32_t frac_bits;     /* fixed-point fraction bits of the arrival sums, 1..40 */
    float velocity_mm_per_ms; /* conduction velocity for DBNET_D_DISTANCE */
    uint32_t net_id;        /* distinguishes the noise streams of networks sharing a seed */
    const dbnet_pop* pops;
    const dbnet_proj* projs;
    const float* region_xyz_mm; /* n_regions*3 centres; needed only for distance delays */
} dbnet_desc;

/* Limits checked by dbnet_validate. */
#define DBNET_MAX_POPS 4096u
#define DBNET_MAX_NEURONS (1u << 28)
#define DBNET_MAX_DELAY 255u
#define DBNET_MAX_STEPS_PER_BIN 16u

/*
 * Checks the description for structural errors (sizes, counts, ranges,
 * enough candidate sources for every in-degree, region coordinates present
 * when needed). Returns 0 if valid, else -1 with a message in err (if
 * errlen > 0). Does not check simulator-specific rules.
 */
int dbnet_validate(const dbnet_desc* d, char* err, size_t errlen);

/* Total neurons (sum of population sizes). */
uint64_t dbnet_num_neurons(const dbnet_desc* d);

/* First neuron id of population p (p may equal n_pops: returns N). */
uint64_t dbnet_pop_offset(const dbnet_desc* d, uint32_t p);

/* Population of neuron i (binary search over the offsets). */
uint32_t dbnet_pop_of(const dbnet_desc* d, uint32_t i);

/* Weights per edge implied by receptor_mask (1 or 2), 0 if the mask is invalid. */
uint32_t dbnet_weights_per_edge(const dbnet_desc* d);

/* Total in-degree of target i (sum over projections that apply to it). */
uint32_t dbnet_indegree(const dbnet_desc* d, uint32_t i);

/* Largest in-degree over all neurons and largest delay over all projections. */
uint32_t dbnet_max_indegree(const dbnet_desc* d);
uint32_t dbnet_max_delay(const dbnet_desc* d);

/* Bytes of caller scratch needed by dbnet_in_edges. */
size_t dbnet_scratch_bytes(const dbnet_desc* d);

/*
 * Incoming edges of target i, written to the caller's arrays (each sized
 * at least dbnet_indegree(d, i)): source ids, first and second weight (w1 is
 * 0 when one weight per edge), delay in bins. Edge order: projections in
 * description order, ascending source id within a projection. scratch must
 * hold dbnet_scratch_bytes(d) bytes. Returns the number of edges, or -1 if
 * the description is invalid for this target (run dbnet_validate first).
 * w0, w1 and delay may be NULL to skip those draws (the sources and the other
 * outputs are unchanged).
 */
int64_t dbnet_in_edges(const dbnet_desc* d, uint32_t i, uint32_t* src, float* w0, float* w1,
                       uint8_t* delay, void* scratch);

/* Initial membrane potential of neuron i, U[v0_lo, v0_hi) of its population. */
float dbnet_v0(const dbnet_desc* d, uint32_t i);

#ifdef __cplusplus
}
#endif
#endif /* DBNET_H */
