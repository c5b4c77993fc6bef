/*
 * oracle.h - CPU oracle of the Digital Brain per-timestep step.
 *
 * TEST INFRASTRUCTURE ONLY: used by the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark. Never part of the product path.
 * See oracle.c for the equations, the readings of the paper and the
 * operation order.
 */
#ifndef DB_ORACLE_H
#define DB_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#include "dbnet.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc orc;

/* Builds the network from the seeded description (via the dbnet
   generator) and the initial state. precision is 32 or 64. Returns NULL
   with a message in err on failure. */
orc* orc_create(const dbnet_desc* d, int precision, char* err, size_t errlen);
/* flags: ORC_PARAMS_ONLY builds the constants and the state but not the edge
   table (for point evaluations of networks too large to simulate here). */
#define ORC_PARAMS_ONLY 1u
orc* orc_create_ex(const dbnet_desc* d, int precision, uint32_t flags, char* err, size_t errlen);
void orc_destroy(orc* o);

/* Host threads used by orc_step (default 1, at most 256): the neurons are split into
   contiguous ranges; results do not depend on the count. Returns 0, or -1. */
int orc_set_threads(orc* o, uint32_t threads);

/* Advances n Euler steps. Returns 0, or -1 if host memory ran out. */
int orc_step(orc* o, uint64_t n);

uint32_t orc_num_neurons(const orc* o);
uint32_t orc_num_receptors(const orc* o);
uint32_t orc_steps_per_bin(const orc* o);
uint64_t orc_steps_done(const orc* o);
uint64_t orc_num_edges(const orc* o);
/* Synaptic events delivered so far (one per edge whose source spike arrived). */
uint64_t orc_edge_events(const orc* o);
uint64_t orc_num_spikes(const orc* o);
uint64_t orc_bins_recorded(const orc* o);

/* All spikes so far, ordered by (step, id). Arrays sized orc_num_spikes. */
void orc_get_spikes(const orc* o, uint64_t* steps, uint32_t* ids);
/* Region signal and spike counts per completed bin, row-major [bin][region]. */
void orc_get_region_signal(const orc* o, double* sig, uint32_t* cnt);
/* State as double: V[N], J[U*N] (receptor-major), ref[N]. */
void orc_get_state(const orc* o, double* V, double* J, int32_t* ref);
/* Overwrites the state (FP32 variant rounds to float). */
int orc_set_state(orc* o, const double* V, const double* J, const int32_t* ref);
/* The incoming-edge table the oracle works from (ptr[N+1], then E entries). */
void orc_get_in_edges(const orc* o, uint64_t* ptr, uint32_t* src, float* w0, float* w1, uint8_t* dl);

/* Initial spike injection: in bins k < until_bin the output train of every neuron of
   population q carries a spike with probability p[q] per bin (see oracle.c); npops must
   equal the description's. Returns 0, or -1 on bad arguments. */
int orc_set_injection(orc* o, const float* p, uint32_t npops, uint64_t until_bin);

/* Ornstein-Uhlenbeck background current (eq. 1 / eq. 4) per population (tau_ms <= 0: off);
   the current starts at mu. Returns 0, or -1 on bad arguments. orc_get_ou copies the
   current per neuron; orc_ou_normal is its increment draw (see oracle.c). */
int orc_set_ou(orc* o, const float* mu, const float* sigma, const float* tau_ms, uint32_t npops);
void orc_get_ou(const orc* o, double* I);
float orc_ou_normal(uint64_t seed, uint32_t net_id, uint64_t n, uint32_t i);

/* Mean synaptic current per receptor of every population at the current state (the
   measurement step of Suppl. Algorithm 1): out[q*4 + u] = the mean over population q's
   neurons, in ascending id, of g_u J_u (V_u - V), u in the paper's receptor order (AMPA,
   NMDA, GABA_A, GABA_B; absent receptors 0). The FP32 oracle evaluates each neuron's term in
   float (the region signal's expression), the FP64 one in double; sums are in double. */
void orc_receptor_currents(const orc* o, double* out);

/* Point evaluations for sampled checks of large runs (FP32 oracle):
   arrivals A[t*U+u] due at the start of `bin` for each target, from the given
   spike list (pull form of eq. 3, fixed point), and one Euler step of neuron
   i at step n from a given state (A is used only when n is a bin start). */
int orc_point_arrivals(orc* o, uint64_t bin, uint64_t nspk, const uint64_t* spk_steps, const uint32_t* spk_ids,
                       uint32_t ntargets, const uint32_t* targets, float* A, uint64_t* events);
int orc_point_step(orc* o, uint32_t i, uint64_t n, const float* A, float* V, float* J, int32_t* ref, int* spiked);

/* Derived constants of population p as the FP32 oracle uses them (each computed in
   double from the description and rounded once to float): dt/C, the receptor decays
   in compact receptor order, the refractory steps, and the Poisson inversion table
   (its length, then up to cap thresholds). Returns 0, or -1 for a bad p. */
int orc_pop_constants(const orc* o, uint32_t p, float* k, float* decay4, int32_t* ref_steps, int* table_len,
                      uint32_t* T, int cap);

/* Building blocks, exported so that the tests can pin them. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
uint32_t orc_bg_word(uint64_t seed, uint32_t net_id, uint64_t n, uint32_t i);
int orc_poisson_table(double lambda, uint32_t* T, int cap);
uint32_t orc_poisson_count(uint32_t x, const uint32_t* T, int cmax);
int64_t orc_quantize(float w, uint32_t F);
float orc_i64_to_f32(int64_t v);

#ifdef __cplusplus
}
#endif
#endif
