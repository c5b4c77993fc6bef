/*
 * oracle.c - plain, slow CPU oracle of the Digital Brain per-timestep step.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load or run this code. It shares no
 * code with the GPU library: its only dependency is the seeded network
 * generator (dbnet), which both sides call to obtain the same network.
 *
 * What it computes (one neuron i, one Euler step n, all right-hand sides at
 * time n; notation of the paper):
 *
 *   LIF capacitance-voltage equation (Methods, CV equation; SI Section 2):
 *     C dV/dt = -g_L (V - V_L) + sum_u g_u J_u (V_u - V) + I_ext + I_bg
 *   receptor kinetics (Methods eq. 2): dJ_u/dt = -J_u/tau_u + sum_j w_ij^u delta(t - t_j)
 *   explicit Euler-Maruyama discretisation (SI Section 3, eqs. 3 and 5):
 *     J_u(t+dt) = exp(-dt/tau_u) J_u(t) + sum_j w_ij^u A_j(t)
 *     V(t+dt)   = V(t) + (dt/C) * (the CV right-hand side at t)
 *   spike when V reaches V_th, reset and clamp for T_ref (Methods; SI eq. after 5);
 *   spikes are accumulated per bin b_t and delivered at bin boundaries
 *   (SI Section 3, definition of A_j(t)).
 *
 * Readings where the paper is silent or garbled (each is listed in the
 * design notes with its justification):
 *   - eq. 5 as printed lacks 1/C and I_ext: the continuous CV equation is
 *     followed, V += (dt/C) * I_total;
 *   - a spike is registered when the updated V' >= V_th; V' is then set to
 *     V_reset and held there for r = round(T_ref/dt) further steps;
 *   - bin k covers steps kS .. kS+S-1 (S = b_t/dt); A_j is binary; a spike
 *     in bin k reaches its target at step (k+d)S where d >= 1 is the edge's
 *     integer delay in bins (d = 1 is the paper's delivery at the next bin
 *     boundary; delays themselves are an extension, the paper has none);
 *   - the arrival sum of eq. 3 is taken exactly: each weight is rounded once
 *     to fixed point q(w) = round_half_even(w * 2^F), the integer sum is exact
 *     (so its order does not matter) and is converted once to float, times
 *     2^-F. The FP64 variant uses the unrounded weights instead;
 *   - the background input is an independent Poisson count c per neuron and
 *     step with mean lambda = rate * dt (a sum of per-synapse Poisson trains,
 *     Extended Data Table 2), added to the AMPA variable with weight w_bg.
 *     c is drawn by inverting the Poisson CDF with a 32-bit word of the
 *     counter-based generator Philox4x32-10 (Salmon, Moraes, Dror and Shaw,
 *     SC'11, "Parallel random numbers: as easy as 1, 2, 3");
 *   - NMDA has no voltage dependence: all four receptors use the linear
 *     form g_u J_u (V_u - V) written in eq. 2;
 *   - the region signal is the mean over a region's neurons of the total
 *     synaptic current sum_u g_u J_u (V_u - V) at each bin end.
 *
 * FP32 variant: every operation is one IEEE binary32 operation, in the order
 * written below, with no contraction and no flush-to-zero (build with
 * -ffp-contract=off, no fast-math). The FP64 variant runs the same
 * algorithm in binary64 and serves as the reference trajectory.
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ---------------- Philox4x32-10 (Salmon et al., SC'11) ---------------- */

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; r++) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The 32-bit background word of neuron i at step n: word (n mod 4) of the
   block with counter (floor(n/4), i, stream tag | net_id), key = seed. */
uint32_t orc_bg_word(uint64_t seed, uint32_t net_id, uint64_t n, uint32_t i) {
    uint64_t blk = n / 4;
    uint32_t ctr[4] = {(uint32_t)blk, (uint32_t)(blk >> 32), i, (1u << 24) | (net_id & 0xFFFFFFu)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[n % 4];
}

/* ---------------- Poisson inversion table ----------------
   T_c = floor(2^32 * P(Poisson(lambda) <= c)), CDF by the recurrence
   p_0 = exp(-lambda), p_c = p_{c-1} * lambda / c, summed in ascending c.
   The table stops at cmax, the first c whose upper tail 1 - CDF(c) is below
   2^-32 (so T_cmax would be 2^32). A word x maps to the count
   c = #{ m < cmax : x >= T_m }, the smallest c with x < T_c. */
int orc_poisson_table(double lambda, uint32_t* T, int cap) {
    if (!(lambda >= 0.0) || lambda > 64.0) return -1;
    double p = exp(-lambda), F = p;
    int c = 0;
    for (;;) {
        if (1.0 - F < 0x1p-32) return c;
        if (c >= cap) return -1;
        T[c] = (uint32_t)floor(F * 0x1p32);
        c++;
        p = p * lambda / (double)c;
        F = F + p;
    }
}

uint32_t orc_poisson_count(uint32_t x, const uint32_t* T, int cmax) {
    uint32_t c = 0;
    for (int m = 0; m < cmax; m++) c += (x >= T[m]) ? 1u : 0u;
    return c;
}

/* ---------------- fixed point ---------------- */

int64_t orc_quantize(float w, uint32_t F) { return (int64_t)nearbyint((double)w * ldexp(1.0, (int)F)); }

float orc_i64_to_f32(int64_t v) { return (float)v; }

/* ---------------- the simulator state ---------------- */

#define ORC_MAX_TABLE 160
#define ORC_MAX_THREADS 256

typedef struct {
    /* membrane and receptor parameters, per population */
    double k64, gL64, VL64, Vth64, Vr64, Iext64, g64[4], Vu64[4], d64[4], wbg64;
    float k32, gL32, VL32, Vth32, Vr32, Iext32, g32[4], Vu32[4], d32[4], wbg32;
    int32_t r;
    int cmax;
    uint32_t T[ORC_MAX_TABLE];
    /* Ornstein-Uhlenbeck background current (eq. 1, eq. 4): on, mean, dt/tau, sigma sqrt(2 dt/tau) */
    int ou;
    float ou_mu32, ou_c1_32, ou_c2_32;
    double ou_mu64, ou_c1_64, ou_c2_64;
} orc_pop;

struct orc {
    dbnet_desc d;
    dbnet_pop* pops;
    dbnet_proj* projs;
    float* xyz;
    int prec;
    uint32_t N, S, U, KW, R, F, n_regions;
    uint32_t umap[4]; /* compact receptor index -> paper receptor index */
    uint32_t* pop_of;
    uint8_t* is_exc;
    uint32_t* region_of;
    uint32_t* region_size;
    orc_pop* P;
    /* incoming edges, grouped by target, in generator order */
    uint64_t* in_ptr;
    uint32_t* in_src;
    float* in_w0;
    float* in_w1;
    uint8_t* in_d;
    /* state */
    float* V32; float* J32; /* J[u*N + i] */
    double* V64; double* J64;
    int32_t* ref;
    uint8_t* hist;    /* [R][N] spike flags of recent bins */
    uint8_t* binspk;  /* spike flag of the current bin */
    uint8_t* stepspk; /* spike flag of the current step */
    uint32_t threads; /* host threads of orc_step (1 unless set) */
    float* A32; double* A64;
    uint64_t step, edge_events;
    /* recordings */
    uint64_t nspk, capspk;
    uint64_t* spk_step; uint32_t* spk_id;
    uint64_t nbins_rec, capbins;
    double* sig; uint32_t* cnt;
    int params_only;
    /* initial spike injection (Methods): per-population threshold, active below inj_until */
    uint32_t* inj_T;
    uint64_t inj_until;
    /* OU background current per neuron */
    float* Iou32;
    double* Iou64;
};

static void* xcalloc(size_t n, size_t s) {
    void* p = calloc(n ? n : 1, s ? s : 1);
    return p;
}

void orc_destroy(orc* o) {
    if (!o) return;
    free(o->inj_T);
    free(o->Iou32);
    free(o->Iou64);
    free(o->pops); free(o->projs); free(o->xyz);
    free(o->pop_of); free(o->is_exc); free(o->region_of); free(o->region_size); free(o->P);
    free(o->in_ptr); free(o->in_src); free(o->in_w0); free(o->in_w1); free(o->in_d);
    free(o->V32); free(o->J32); free(o->V64); free(o->J64); free(o->ref);
    free(o->hist); free(o->binspk); free(o->stepspk); free(o->A32); free(o->A64);
    free(o->spk_step); free(o->spk_id); free(o->sig); free(o->cnt);
    free(o);
}

static void seterr(char* err, size_t len, const char* m) {
    if (err && len) snprintf(err, len, "%s", m);
}

orc* orc_create(const dbnet_desc* d, int precision, char* err, size_t errlen) {
    return orc_create_ex(d, precision, 0, err, errlen);
}

orc* orc_create_ex(const dbnet_desc* d, int precision, uint32_t flags, char* err, size_t errlen) {
    if (dbnet_validate(d, err, errlen) != 0) return NULL;
    if (precision != 32 && precision != 64) { seterr(err, errlen, "precision must be 32 or 64"); return NULL; }
    orc* o = (orc*)xcalloc(1, sizeof(orc));
    if (!o) return NULL;
    o->d = *d;
    o->pops = (dbnet_pop*)malloc(sizeof(dbnet_pop) * d->n_pops);
    memcpy(o->pops, d->pops, sizeof(dbnet_pop) * d->n_pops);
    o->d.pops = o->pops;
    o->projs = (dbnet_proj*)malloc(sizeof(dbnet_proj) * (d->n_projs ? d->n_projs : 1));
    if (d->n_projs) memcpy(o->projs, d->projs, sizeof(dbnet_proj) * d->n_projs);
    o->d.projs = o->projs;
    if (d->region_xyz_mm) {
        o->xyz = (float*)malloc(sizeof(float) * 3 * d->n_regions);
        memcpy(o->xyz, d->region_xyz_mm, sizeof(float) * 3 * d->n_regions);
        o->d.region_xyz_mm = o->xyz;
    }
    o->prec = precision;
    o->N = (uint32_t)dbnet_num_neurons(d);
    o->S = (uint32_t)lround((double)d->bin_ms / (double)d->dt_ms);
    o->KW = dbnet_weights_per_edge(d);
    o->U = 2 * o->KW;
    if (o->KW == 1) { o->umap[0] = DBNET_AMPA; o->umap[1] = DBNET_GABA_A; }
    else { o->umap[0] = DBNET_AMPA; o->umap[1] = DBNET_NMDA; o->umap[2] = DBNET_GABA_A; o->umap[3] = DBNET_GABA_B; }
    o->R = dbnet_max_delay(d) + 1;
    o->F = d->frac_bits;
    o->n_regions = d->n_regions;
    uint32_t N = o->N;

    /* per-population constants, computed in double and (FP32) rounded once */
    o->P = (orc_pop*)xcalloc(d->n_pops, sizeof(orc_pop));
    double dt = (double)d->dt_ms;
    for (uint32_t p = 0; p < d->n_pops; p++) {
        const dbnet_pop* Q = &d->pops[p];
        orc_pop* P = &o->P[p];
        P->k64 = dt / (double)Q->C;
        P->k32 = (float)P->k64;
        P->gL64 = Q->g_L; P->gL32 = Q->g_L;
        P->VL64 = Q->V_L; P->VL32 = Q->V_L;
        P->Vth64 = Q->V_th; P->Vth32 = Q->V_th;
        P->Vr64 = Q->V_reset; P->Vr32 = Q->V_reset;
        P->Iext64 = Q->I_ext; P->Iext32 = Q->I_ext;
        for (uint32_t c = 0; c < o->U; c++) {
            uint32_t u = o->umap[c];
            P->g64[c] = Q->g[u]; P->g32[c] = Q->g[u];
            P->Vu64[c] = Q->V_rev[u]; P->Vu32[c] = Q->V_rev[u];
            P->d64[c] = exp(-dt / (double)Q->tau[u]);
            P->d32[c] = (float)P->d64[c];
        }
        P->wbg64 = Q->w_bg; P->wbg32 = Q->w_bg;
        P->r = (int32_t)lround((double)Q->T_ref / dt);
        if (P->r < (int32_t)o->S - 1) {
            seterr(err, errlen, "T_ref must cover a bin minus one step (at most one spike per bin)");
            orc_destroy(o);
            return NULL;
        }
        double lambda = (double)Q->bg_rate_hz * dt * 1e-3;
        P->cmax = orc_poisson_table(lambda, P->T, ORC_MAX_TABLE);
        if (P->cmax < 0) { seterr(err, errlen, "background rate too high"); orc_destroy(o); return NULL; }
    }
    o->pop_of = (uint32_t*)malloc(sizeof(uint32_t) * N);
    o->is_exc = (uint8_t*)malloc(N);
    o->region_of = (uint32_t*)malloc(sizeof(uint32_t) * N);
    o->region_size = (uint32_t*)xcalloc(o->n_regions, sizeof(uint32_t));
    {
        uint32_t i = 0;
        for (uint32_t p = 0; p < d->n_pops; p++)
            for (uint32_t a = 0; a < d->pops[p].size; a++, i++) {
                o->pop_of[i] = p;
                o->is_exc[i] = (uint8_t)(d->pops[p].exc != 0);
                o->region_of[i] = d->pops[p].region;
                o->region_size[d->pops[p].region]++;
            }
    }
    /* incoming edges straight from the generator */
    o->in_ptr = (uint64_t*)malloc(sizeof(uint64_t) * (N + 1));
    o->in_ptr[0] = 0;
    for (uint32_t i = 0; i < N; i++) o->in_ptr[i + 1] = o->in_ptr[i] + dbnet_indegree(d, i);
    o->params_only = (flags & ORC_PARAMS_ONLY) != 0;
    uint64_t E = o->params_only ? 0 : o->in_ptr[N];
    o->in_src = (uint32_t*)malloc(sizeof(uint32_t) * (E ? E : 1));
    o->in_w0 = (float*)malloc(sizeof(float) * (E ? E : 1));
    o->in_w1 = (float*)malloc(sizeof(float) * (E ? E : 1));
    o->in_d = (uint8_t*)malloc(E ? E : 1);
    void* scratch = malloc(dbnet_scratch_bytes(d));
    if (!o->in_src || !o->in_w0 || !o->in_w1 || !o->in_d || !scratch) {
        free(scratch); seterr(err, errlen, "out of host memory"); orc_destroy(o); return NULL;
    }
    for (uint32_t i = 0; i < N && !o->params_only; i++) {
        uint64_t a = o->in_ptr[i];
        int64_t k = dbnet_in_edges(d, i, o->in_src + a, o->in_w0 + a, o->in_w1 + a, o->in_d + a, scratch);
        if (k != (int64_t)(o->in_ptr[i + 1] - a)) {
            free(scratch); seterr(err, errlen, "generator failed"); orc_destroy(o); return NULL;
        }
    }
    free(scratch);
    /* fixed-point range check: every q(w) must stay far from int64 overflow */
    for (uint64_t e = 0; e < E; e++) {
        double m = fabs((double)o->in_w0[e]) > fabs((double)o->in_w1[e]) ? fabs((double)o->in_w0[e]) : fabs((double)o->in_w1[e]);
        if (!(m * ldexp(1.0, (int)o->F) < 0x1p52)) { seterr(err, errlen, "weight too large for the fixed-point format"); orc_destroy(o); return NULL; }
    }
    /* state: V0 from the generator, J = 0, not refractory */
    o->ref = (int32_t*)xcalloc(N, sizeof(int32_t));
    if (precision == 32) {
        o->V32 = (float*)malloc(sizeof(float) * N);
        o->J32 = (float*)xcalloc((size_t)o->U * N, sizeof(float));
        o->A32 = (float*)xcalloc((size_t)o->U * N, sizeof(float));
        for (uint32_t i = 0; i < N; i++) o->V32[i] = dbnet_v0(d, i);
    } else {
        o->V64 = (double*)malloc(sizeof(double) * N);
        o->J64 = (double*)xcalloc((size_t)o->U * N, sizeof(double));
        o->A64 = (double*)xcalloc((size_t)o->U * N, sizeof(double));
        for (uint32_t i = 0; i < N; i++) o->V64[i] = (double)dbnet_v0(d, i);
    }
    o->hist = (uint8_t*)xcalloc((size_t)o->R * N, 1);
    o->binspk = (uint8_t*)xcalloc(N, 1);
    o->stepspk = (uint8_t*)xcalloc(N, 1);
    o->threads = 1;
    return o;
}

static int record_spike(orc* o, uint64_t n, uint32_t i) {
    if (o->nspk == o->capspk) {
        uint64_t c = o->capspk ? 2 * o->capspk : 1024;
        uint64_t* a = (uint64_t*)realloc(o->spk_step, sizeof(uint64_t) * c);
        if (!a) return -1;
        o->spk_step = a;
        uint32_t* b = (uint32_t*)realloc(o->spk_id, sizeof(uint32_t) * c);
        if (!b) return -1;
        o->spk_id = b;
        o->capspk = c;
    }
    o->spk_step[o->nspk] = n;
    o->spk_id[o->nspk] = i;
    o->nspk++;
    return 0;
}

static int record_bin(orc* o) {
    if (o->nbins_rec == o->capbins) {
        uint64_t c = o->capbins ? 2 * o->capbins : 64;
        double* a = (double*)realloc(o->sig, sizeof(double) * c * o->n_regions);
        if (!a) return -1;
        o->sig = a;
        uint32_t* b = (uint32_t*)realloc(o->cnt, sizeof(uint32_t) * c * o->n_regions);
        if (!b) return -1;
        o->cnt = b;
        o->capbins = c;
    }
    double* sig = o->sig + o->nbins_rec * o->n_regions;
    uint32_t* cnt = o->cnt + o->nbins_rec * o->n_regions;
    for (uint32_t r = 0; r < o->n_regions; r++) { sig[r] = 0.0; cnt[r] = 0; }
    const uint32_t N = o->N, U = o->U;
    for (uint32_t i = 0; i < N; i++) {
        const orc_pop* P = &o->P[o->pop_of[i]];
        double cur;
        if (o->prec == 32) {
            float V = o->V32[i];
            float acc = 0.0f;
            for (uint32_t u = 0; u < U; u++) {
                float t = (P->g32[u] * o->J32[(size_t)u * N + i]) * (P->Vu32[u] - V);
                acc = acc + t;
            }
            cur = (double)acc;
        } else {
            double V = o->V64[i];
            double acc = 0.0;
            for (uint32_t u = 0; u < U; u++) acc = acc + (P->g64[u] * o->J64[(size_t)u * N + i]) * (P->Vu64[u] - V);
            cur = acc;
        }
        sig[o->region_of[i]] += cur;
        cnt[o->region_of[i]] += o->binspk[i];
    }
    for (uint32_t r = 0; r < o->n_regions; r++) sig[r] = o->region_size[r] ? sig[r] / (double)o->region_size[r] : 0.0;
    o->nbins_rec++;
    return 0;
}

/* Suppl. Algorithm 1 measures the mean current of each receptor type: per population,
   the mean over its neurons of g_u J_u (V_u - V) (the same per-receptor term as the region
   signal), summed in ascending neuron id. */
void orc_receptor_currents(const orc* o, double* out) {
    const uint32_t N = o->N, U = o->U, Q = o->d.n_pops;
    for (uint32_t q = 0; q < 4 * Q; q++) out[q] = 0.0;
    uint64_t i0 = 0;
    for (uint32_t q = 0; q < Q; q++) {
        const orc_pop* P = &o->P[q];
        const uint64_t i1 = i0 + o->pops[q].size;
        for (uint32_t u = 0; u < U; u++) {
            double s = 0.0;
            for (uint64_t i = i0; i < i1; i++) {
                if (o->prec == 32) {
                    const float t = (P->g32[u] * o->J32[(size_t)u * N + i]) * (P->Vu32[u] - o->V32[i]);
                    s += (double)t;
                } else {
                    s += (P->g64[u] * o->J64[(size_t)u * N + i]) * (P->Vu64[u] - o->V64[i]);
                }
            }
            out[(size_t)q * 4 + o->umap[u]] = i1 > i0 ? s / (double)(i1 - i0) : 0.0;
        }
        i0 = i1;
    }
}

/* Arrival sums for the bin starting at step kS: eq. 3's sum_j w_ij^u A_j
   with A_j taken at bin k - d_ij (pull form of the definition). */
static uint64_t arrivals(orc* o, uint64_t k, uint32_t i0, uint32_t i1) {
    const uint32_t N = o->N, KW = o->KW;
    uint64_t events = 0;
    for (uint32_t i = i0; i < i1; i++) {
        int64_t q[4] = {0, 0, 0, 0};
        double s[4] = {0.0, 0.0, 0.0, 0.0};
        for (uint64_t e = o->in_ptr[i]; e < o->in_ptr[i + 1]; e++) {
            uint32_t dl = o->in_d[e];
            if ((uint64_t)dl > k) continue;
            uint32_t j = o->in_src[e];
            if (!o->hist[(size_t)((k - dl) % o->R) * N + j]) continue;
            uint32_t base = o->is_exc[j] ? 0u : KW;
            events++;
            if (o->prec == 32) {
                q[base] += orc_quantize(o->in_w0[e], o->F);
                if (KW == 2) q[base + 1] += orc_quantize(o->in_w1[e], o->F);
            } else {
                s[base] += (double)o->in_w0[e];
                if (KW == 2) s[base + 1] += (double)o->in_w1[e];
            }
        }
        for (uint32_t u = 0; u < o->U; u++) {
            if (o->prec == 32) o->A32[(size_t)u * N + i] = orc_i64_to_f32(q[u]) * ldexpf(1.0f, -(int)o->F);
            else o->A64[(size_t)u * N + i] = s[u];
        }
    }
    return events;
}

/* One Euler step of one neuron (FP32): all right-hand sides use the old V and
   J; A is this step's arrival (zero except at a bin start), c the background
   count. Returns 1 if the neuron spiked. */
static int neuron_step32(const orc_pop* P, uint32_t U, uint32_t c, const float* A, float* Vp, float* J, int32_t* ref,
                         float Ibg) {
    const float V = *Vp;
    float Vn;
    int spiked = 0;
    if (*ref > 0) {
        Vn = P->Vr32;
        *ref -= 1;
    } else {
        float I = P->gL32 * (P->VL32 - V);
        for (uint32_t u = 0; u < U; u++) {
            float gJ = P->g32[u] * J[u];
            I = I + gJ * (P->Vu32[u] - V);
        }
        I = I + P->Iext32;
        if (P->ou) I = I + Ibg;
        Vn = V + P->k32 * I;
        if (Vn >= P->Vth32) { spiked = 1; Vn = P->Vr32; *ref = P->r; }
    }
    *Vp = Vn;
    float B = P->wbg32 * (float)c;
    for (uint32_t u = 0; u < U; u++) {
        float Jn = P->d32[u] * J[u] + A[u];
        if (u == 0) Jn = Jn + B;
        J[u] = Jn;
    }
    return spiked;
}

/* The same step in FP64. */
static int neuron_step64(const orc_pop* P, uint32_t U, uint32_t c, const double* A, double* Vp, double* J, int32_t* ref,
                         double Ibg) {
    const double V = *Vp;
    double Vn;
    int spiked = 0;
    if (*ref > 0) {
        Vn = P->Vr64;
        *ref -= 1;
    } else {
        double I = P->gL64 * (P->VL64 - V);
        for (uint32_t u = 0; u < U; u++) I = I + (P->g64[u] * J[u]) * (P->Vu64[u] - V);
        I = I + P->Iext64;
        if (P->ou) I = I + Ibg;
        Vn = V + P->k64 * I;
        if (Vn >= P->Vth64) { spiked = 1; Vn = P->Vr64; *ref = P->r; }
    }
    *Vp = Vn;
    double B = P->wbg64 * (double)c;
    for (uint32_t u = 0; u < U; u++) {
        double Jn = P->d64[u] * J[u] + A[u];
        if (u == 0) Jn = Jn + B;
        J[u] = Jn;
    }
    return spiked;
}

/* Initial spike injection (Methods: to start the spike trains without synchrony, every
   neuron's output train gets a spike with a small probability): in bins k < inj_until
   neuron i's train carries a spike when word 0 of Philox4x32-10 with key = seed and
   counter (k, k >> 32, i, 2 << 24 | net_id) is below floor(p * 2^32). */
static int injected(const orc* o, uint64_t k, uint32_t i) {
    if (!o->inj_T || k >= o->inj_until) return 0;
    const uint32_t T = o->inj_T[o->pop_of[i]];
    if (T == 0) return 0;
    uint32_t ctr[4] = {(uint32_t)k, (uint32_t)(k >> 32), i, (2u << 24) | (o->d.net_id & 0xFFFFFFu)};
    uint32_t key[2] = {(uint32_t)o->d.seed, (uint32_t)(o->d.seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[0] < T;
}

/* Gaussian-like increment of the OU background: the 128 bits of Philox4x32-10 with key =
   seed and counter (n, n >> 32, i, 3 << 24 | net_id) as twelve 10-bit uniform integers
   (bits 0-9, 10-19, 20-29 of each word); each field has mean 511.5 and variance
   (1024^2 - 1) / 12, so z = (2 s - 12276) / 2048 for their sum s has mean 0 and variance
   1 - 2^-20 (Irwin-Hall with twelve terms). Computed exactly. */
float orc_ou_normal(uint64_t seed, uint32_t net_id, uint64_t n, uint32_t i) {
    uint32_t ctr[4] = {(uint32_t)n, (uint32_t)(n >> 32), i, (3u << 24) | (net_id & 0xFFFFFFu)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    uint32_t sum = 0;
    for (int q = 0; q < 4; q++)
        for (int f = 0; f < 3; f++) sum += (w[q] >> (10 * f)) & 1023u;
    return (float)((int)(2u * sum) - 12276) * 0x1p-11f;
}

int orc_set_ou(orc* o, const float* mu, const float* sigma, const float* tau_ms, uint32_t npops) {
    if (!o || npops != o->d.n_pops || !mu || !sigma || !tau_ms) return -1;
    if (!o->Iou32) o->Iou32 = (float*)xcalloc(o->N, sizeof(float));
    if (!o->Iou64) o->Iou64 = (double*)xcalloc(o->N, sizeof(double));
    const double dt = (double)o->d.dt_ms;
    uint64_t first = 0;
    for (uint32_t q = 0; q < npops; q++) {
        if (!isfinite(mu[q]) || !isfinite(sigma[q]) || !isfinite(tau_ms[q]) || sigma[q] < 0.0f) return -1;
        orc_pop* P = &o->P[q];
        P->ou = tau_ms[q] > 0.0f;
        P->ou_mu32 = mu[q];
        P->ou_c1_32 = P->ou ? (float)(dt / (double)tau_ms[q]) : 0.0f;
        P->ou_c2_32 = P->ou ? (float)((double)sigma[q] * sqrt(2.0 * dt / (double)tau_ms[q])) : 0.0f;
        P->ou_mu64 = (double)mu[q];
        P->ou_c1_64 = P->ou ? dt / (double)tau_ms[q] : 0.0;
        P->ou_c2_64 = P->ou ? (double)sigma[q] * sqrt(2.0 * dt / (double)tau_ms[q]) : 0.0;
        for (uint64_t i = first; i < first + o->pops[q].size; i++) {
            o->Iou32[i] = P->ou ? mu[q] : 0.0f;
            o->Iou64[i] = P->ou ? (double)mu[q] : 0.0;
        }
        first += o->pops[q].size;
    }
    return 0;
}

void orc_get_ou(const orc* o, double* I) {
    for (uint32_t i = 0; i < o->N; i++)
        I[i] = o->Iou32 ? (o->prec == 32 ? (double)o->Iou32[i] : o->Iou64[i]) : 0.0;
}

int orc_set_injection(orc* o, const float* p, uint32_t npops, uint64_t until_bin) {
    if (!o || npops != o->d.n_pops || (until_bin && !p)) return -1;
    if (!o->inj_T) o->inj_T = (uint32_t*)xcalloc(npops, sizeof(uint32_t));
    for (uint32_t q = 0; q < npops; q++) {
        if (until_bin && !(p[q] >= 0.0f && p[q] < 1.0f)) return -1;
        o->inj_T[q] = until_bin ? (uint32_t)floor((double)p[q] * 4294967296.0) : 0u;
    }
    o->inj_until = until_bin;
    return 0;
}

/* One Euler step n of the neurons i0 <= i < i1 (each independent of the others within the
   step): background draw, membrane and synapse update; the spike flag of each neuron (own
   spike or injected output spike) goes to spk[i]. */
static void neurons(orc* o, uint64_t n, uint32_t i0, uint32_t i1, uint8_t* spk) {
    const uint32_t N = o->N, U = o->U, S = o->S;
    const uint64_t k = n / S;
    const uint32_t s = (uint32_t)(n % S);
    for (uint32_t i = i0; i < i1; i++) {
        const orc_pop* P = &o->P[o->pop_of[i]];
        /* background Poisson count */
        uint32_t x = orc_bg_word(o->d.seed, o->d.net_id, n, i);
        uint32_t c = orc_poisson_count(x, P->T, P->cmax);
        int spiked;
        if (o->prec == 32) {
            float J[4], A[4];
            for (uint32_t u = 0; u < U; u++) {
                J[u] = o->J32[(size_t)u * N + i];
                A[u] = (s == 0) ? o->A32[(size_t)u * N + i] : 0.0f;
            }
            const float Ibg = P->ou ? o->Iou32[i] : 0.0f;
            spiked = neuron_step32(P, U, c, A, &o->V32[i], J, &o->ref[i], Ibg);
            for (uint32_t u = 0; u < U; u++) o->J32[(size_t)u * N + i] = J[u];
            if (P->ou) { /* OU current: drift towards mu, then the scaled increment */
                const float z = orc_ou_normal(o->d.seed, o->d.net_id, n, i);
                const float drift = P->ou_c1_32 * (P->ou_mu32 - Ibg);
                const float Ih = Ibg + drift;
                o->Iou32[i] = Ih + P->ou_c2_32 * z;
            }
        } else {
            double J[4], A[4];
            for (uint32_t u = 0; u < U; u++) {
                J[u] = o->J64[(size_t)u * N + i];
                A[u] = (s == 0) ? o->A64[(size_t)u * N + i] : 0.0;
            }
            const double Ibg = P->ou ? o->Iou64[i] : 0.0;
            spiked = neuron_step64(P, U, c, A, &o->V64[i], J, &o->ref[i], Ibg);
            for (uint32_t u = 0; u < U; u++) o->J64[(size_t)u * N + i] = J[u];
            if (P->ou) {
                const double z = (double)orc_ou_normal(o->d.seed, o->d.net_id, n, i);
                o->Iou64[i] = (Ibg + P->ou_c1_64 * (P->ou_mu64 - Ibg)) + P->ou_c2_64 * z;
            }
        }
        /* an injected output spike is delivered and recorded, the neuron is not reset */
        spk[i] = (uint8_t)(spiked || (s == S - 1 && !o->binspk[i] && injected(o, k, i)));
    }
}

/* Host threads: the neurons (and the targets of the arrival sums) are split into
   contiguous ranges, one per thread; every neuron's arithmetic is the same as on one
   thread, and spikes are recorded afterwards in ascending id. */
typedef struct {
    orc* o;
    uint64_t n, k;
    uint32_t i0, i1;
    int phase; /* 0: arrivals of bin k, 1: neurons of step n */
    uint64_t events;
} orc_job;

static void* run_job(void* arg) {
    orc_job* j = (orc_job*)arg;
    if (j->phase == 0) j->events = arrivals(j->o, j->k, j->i0, j->i1);
    else neurons(j->o, j->n, j->i0, j->i1, j->o->stepspk);
    return NULL;
}

static uint64_t run_split(orc* o, int phase, uint64_t n, uint64_t k) {
    const uint32_t T = o->threads > 1 ? o->threads : 1, N = o->N;
    orc_job jobs[ORC_MAX_THREADS];
    pthread_t th[ORC_MAX_THREADS];
    int started[ORC_MAX_THREADS];
    for (uint32_t t = 0; t < T; t++) {
        jobs[t] = (orc_job){o, n, k, (uint32_t)((uint64_t)N * t / T), (uint32_t)((uint64_t)N * (t + 1) / T), phase, 0};
        started[t] = t > 0 && pthread_create(&th[t], NULL, run_job, &jobs[t]) == 0;
        if (t > 0 && !started[t]) run_job(&jobs[t]); /* no thread: run the range here */
    }
    run_job(&jobs[0]);
    uint64_t ev = 0;
    for (uint32_t t = 0; t < T; t++) {
        if (started[t]) pthread_join(th[t], NULL);
        ev += jobs[t].events;
    }
    return ev;
}

int orc_set_threads(orc* o, uint32_t threads) {
    if (!o || threads < 1 || threads > ORC_MAX_THREADS) return -1;
    o->threads = threads;
    return 0;
}

int orc_step(orc* o, uint64_t nsteps) {
    const uint32_t N = o->N, S = o->S;
    if (o->params_only) return -2;
    for (uint64_t t = 0; t < nsteps; t++) {
        const uint64_t n = o->step;
        const uint64_t k = n / S;
        const uint32_t s = (uint32_t)(n % S);
        if (s == 0) {
            memset(o->binspk, 0, N);
            o->edge_events += run_split(o, 0, n, k);
        }
        run_split(o, 1, n, k);
        for (uint32_t i = 0; i < N; i++) {
            if (!o->stepspk[i]) continue;
            o->binspk[i] = 1;
            if (record_spike(o, n, i)) return -1;
        }
        if (s == S - 1) {
            memcpy(o->hist + (size_t)(k % o->R) * N, o->binspk, N);
            if (record_bin(o)) return -1;
        }
        o->step++;
    }
    return 0;
}

/* ---------------- accessors ---------------- */

uint32_t orc_num_neurons(const orc* o) { return o->N; }
uint32_t orc_num_receptors(const orc* o) { return o->U; }
uint32_t orc_steps_per_bin(const orc* o) { return o->S; }
uint64_t orc_steps_done(const orc* o) { return o->step; }
uint64_t orc_num_edges(const orc* o) { return o->params_only ? 0 : o->in_ptr[o->N]; }
uint64_t orc_edge_events(const orc* o) { return o->edge_events; }
uint64_t orc_num_spikes(const orc* o) { return o->nspk; }
uint64_t orc_bins_recorded(const orc* o) { return o->nbins_rec; }

void orc_get_spikes(const orc* o, uint64_t* steps, uint32_t* ids) {
    memcpy(steps, o->spk_step, sizeof(uint64_t) * o->nspk);
    memcpy(ids, o->spk_id, sizeof(uint32_t) * o->nspk);
}

void orc_get_region_signal(const orc* o, double* sig, uint32_t* cnt) {
    memcpy(sig, o->sig, sizeof(double) * o->nbins_rec * o->n_regions);
    memcpy(cnt, o->cnt, sizeof(uint32_t) * o->nbins_rec * o->n_regions);
}

void orc_get_state(const orc* o, double* V, double* J, int32_t* ref) {
    const size_t N = o->N, U = o->U;
    for (size_t i = 0; i < N; i++) V[i] = o->prec == 32 ? (double)o->V32[i] : o->V64[i];
    for (size_t i = 0; i < U * N; i++) J[i] = o->prec == 32 ? (double)o->J32[i] : o->J64[i];
    memcpy(ref, o->ref, sizeof(int32_t) * N);
}

int orc_set_state(orc* o, const double* V, const double* J, const int32_t* ref) {
    const size_t N = o->N, U = o->U;
    for (size_t i = 0; i < N; i++) {
        if (o->prec == 32) o->V32[i] = (float)V[i];
        else o->V64[i] = V[i];
    }
    for (size_t i = 0; i < U * N; i++) {
        if (o->prec == 32) o->J32[i] = (float)J[i];
        else o->J64[i] = J[i];
    }
    memcpy(o->ref, ref, sizeof(int32_t) * N);
    return 0;
}

void orc_get_in_edges(const orc* o, uint64_t* ptr, uint32_t* src, float* w0, float* w1, uint8_t* dl) {
    uint64_t E = o->in_ptr[o->N];
    memcpy(ptr, o->in_ptr, sizeof(uint64_t) * (o->N + 1));
    memcpy(src, o->in_src, sizeof(uint32_t) * E);
    memcpy(w0, o->in_w0, sizeof(float) * E);
    memcpy(w1, o->in_w1, sizeof(float) * E);
    memcpy(dl, o->in_d, E);
}

/* ---------------- point evaluations (sampled checks of large runs) ---------------- */

static int cmp_u64(const void* a, const void* b) {
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : x > y;
}

int orc_point_arrivals(orc* o, uint64_t bin, uint64_t nspk, const uint64_t* spk_steps, const uint32_t* spk_ids,
                       uint32_t ntargets, const uint32_t* targets, float* A, uint64_t* events) {
    const uint32_t U = o->U, KW = o->KW, S = o->S;
    /* spikes of bins bin-D .. bin-1 as sorted (bin << 32 | id) keys */
    uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (nspk ? nspk : 1));
    if (!keys) return -1;
    uint64_t nk = 0;
    for (uint64_t x = 0; x < nspk; x++) {
        uint64_t b = spk_steps[x] / S;
        if (b < bin && bin - b < o->R) keys[nk++] = (b << 32) | spk_ids[x];
    }
    qsort(keys, nk, sizeof(uint64_t), cmp_u64);
    uint32_t kmax = dbnet_max_indegree(&o->d);
    uint32_t* src = (uint32_t*)malloc(sizeof(uint32_t) * (kmax ? kmax : 1));
    float* w0 = (float*)malloc(sizeof(float) * (kmax ? kmax : 1));
    float* w1 = (float*)malloc(sizeof(float) * (kmax ? kmax : 1));
    uint8_t* dl = (uint8_t*)malloc(kmax ? kmax : 1);
    void* scratch = malloc(dbnet_scratch_bytes(&o->d));
    int rc = (src && w0 && w1 && dl && scratch) ? 0 : -1;
    uint64_t ev = 0;
    for (uint32_t t = 0; t < ntargets && rc == 0; t++) {
        int64_t k = dbnet_in_edges(&o->d, targets[t], src, w0, w1, dl, scratch);
        if (k < 0) { rc = -1; break; }
        int64_t q[4] = {0, 0, 0, 0};
        for (int64_t e = 0; e < k; e++) {
            if ((uint64_t)dl[e] > bin) continue;
            uint64_t key = ((bin - dl[e]) << 32) | src[e];
            if (!bsearch(&key, keys, nk, sizeof(uint64_t), cmp_u64)) continue;
            uint32_t base = o->is_exc[src[e]] ? 0u : KW;
            q[base] += orc_quantize(w0[e], o->F);
            if (KW == 2) q[base + 1] += orc_quantize(w1[e], o->F);
            ev++;
        }
        for (uint32_t u = 0; u < U; u++) A[(size_t)t * U + u] = orc_i64_to_f32(q[u]) * ldexpf(1.0f, -(int)o->F);
    }
    if (events) *events = ev;
    free(keys); free(src); free(w0); free(w1); free(dl); free(scratch);
    return rc;
}

int orc_point_step(orc* o, uint32_t i, uint64_t n, const float* A, float* V, float* J, int32_t* ref, int* spiked) {
    if (o->prec != 32 || i >= o->N) return -1;
    const orc_pop* P = &o->P[o->pop_of[i]];
    if (P->ou) return -1; /* the OU current is state of its own; point checks run without it */
    uint32_t c = orc_poisson_count(orc_bg_word(o->d.seed, o->d.net_id, n, i), P->T, P->cmax);
    float Az[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    int s = neuron_step32(P, o->U, c, (n % o->S == 0 && A) ? A : Az, V, J, ref, 0.0f);
    if (spiked) *spiked = s;
    return 0;
}

int orc_pop_constants(const orc* o, uint32_t p, float* k, float* decay4, int32_t* ref_steps, int* table_len,
                      uint32_t* T, int cap) {
    if (!o || p >= o->d.n_pops) return -1;
    const orc_pop* P = &o->P[p];
    if (k) *k = P->k32;
    if (decay4)
        for (uint32_t u = 0; u < 4; u++) decay4[u] = u < o->U ? P->d32[u] : 0.0f;
    if (ref_steps) *ref_steps = P->r;
    if (table_len) *table_len = P->cmax;
    if (T)
        for (int c = 0; c < P->cmax && c < cap; c++) T[c] = P->T[c];
    return 0;
}
