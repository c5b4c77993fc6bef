/*
 * dbnet.c - seeded synthetic network generator (see include/dbnet.h).
 *
 * Input generation only: fixed in-degree sampling without replacement
 * (Suppl. Section 2, "k-random graph"; Extended Data Table 2
 * "Connectivity"), weight and delay draws, initial potentials. Random
 * numbers come from a counter-based hash built on the SplitMix64 output
 * function (Steele, Lea and Flood, OOPSLA 2014), so every draw is a pure
 * function of (seed, net_id, stream, target, projection, index).
 *
 * Compiled with gcc -O2 -ffp-contract=off; libm log/exp/cos/sqrt are used
 * only to shape weight and delay distributions.
 */
#include "dbnet.h"

#include <math.h>
#include <stdio.h>
#include <string.h>

enum { ST_SAMPLE = 1, ST_W0 = 2, ST_W1 = 3, ST_DELAY = 4, ST_V0 = 5, ST_W0B = 6, ST_W1B = 7 };

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* the draws of one (stream, target): key = the first two rounds, which do not depend on
   the projection and index; draw = the third */
static inline uint64_t stream_key(const dbnet_desc* d, uint32_t stream, uint32_t target) {
    uint64_t h = mix64(d->seed + 0x9E3779B97F4A7C15ULL * (uint64_t)(1u + stream));
    return mix64(h ^ (((uint64_t)d->net_id << 32) | target));
}

static inline uint64_t draw_k(uint64_t key, uint32_t proj, uint64_t idx) {
    return mix64(key ^ ((uint64_t)proj << 48) ^ idx);
}

static inline uint64_t draw(const dbnet_desc* d, uint32_t stream, uint32_t target, uint32_t proj,
                            uint64_t idx) {
    return draw_k(stream_key(d, stream, target), proj, idx);
}

/* uniform double in [0,1) from the top 53 bits */
static inline double u01(uint64_t h) { return (double)(h >> 11) * 0x1p-53; }
/* uniform double in (0,1] */
static inline double u01_open0(uint64_t h) { return (double)((h >> 11) + 1) * 0x1p-53; }
/* uniform integer in [0, n) by multiply-high (bias below n / 2^64) */
static inline uint64_t below(uint64_t h, uint64_t n) {
    return (uint64_t)(((unsigned __int128)h * n) >> 64);
}

static void set_err(char* err, size_t errlen, const char* msg, long a) {
    if (err && errlen) snprintf(err, errlen, msg, a);
}

uint64_t dbnet_num_neurons(const dbnet_desc* d) {
    uint64_t n = 0;
    for (uint32_t p = 0; p < d->n_pops; p++) n += d->pops[p].size;
    return n;
}

uint64_t dbnet_pop_offset(const dbnet_desc* d, uint32_t p) {
    uint64_t n = 0;
    for (uint32_t q = 0; q < p && q < d->n_pops; q++) n += d->pops[q].size;
    return n;
}

uint32_t dbnet_pop_of(const dbnet_desc* d, uint32_t i) {
    uint64_t off = 0;
    for (uint32_t p = 0; p < d->n_pops; p++) {
        off += d->pops[p].size;
        if (i < off) return p;
    }
    return d->n_pops;
}

uint32_t dbnet_weights_per_edge(const dbnet_desc* d) {
    if (d->receptor_mask == DBNET_RECEPTORS_2) return 1;
    if (d->receptor_mask == DBNET_RECEPTORS_4) return 2;
    return 0;
}

static int proj_applies(const dbnet_proj* pr, uint32_t pop) {
    return pr->dst_pop < 0 || (uint32_t)pr->dst_pop == pop;
}

/* Is population q a candidate source of projection pr for a target in population tp? */
static int candidate(const dbnet_desc* d, const dbnet_proj* pr, uint32_t tp, uint32_t q) {
    const dbnet_pop* P = &d->pops[q];
    if (pr->src_class == DBNET_CLASS_EXC && !P->exc) return 0;
    if (pr->src_class == DBNET_CLASS_INH && P->exc) return 0;
    switch (pr->src_mode) {
    case DBNET_SRC_ALL: return 1;
    case DBNET_SRC_SAME_REGION: return P->region == d->pops[tp].region;
    case DBNET_SRC_OTHER_REGIONS: return P->region != d->pops[tp].region;
    case DBNET_SRC_POP: return (int32_t)q == pr->src_pop;
    default: return 0;
    }
}

/* Number of candidate sources for a target in population tp, self excluded. */
static uint64_t candidate_count(const dbnet_desc* d, const dbnet_proj* pr, uint32_t tp) {
    uint64_t m = 0;
    for (uint32_t q = 0; q < d->n_pops; q++)
        if (candidate(d, pr, tp, q)) m += d->pops[q].size - (q == tp ? 1u : 0u);
    return m;
}

int dbnet_validate(const dbnet_desc* d, char* err, size_t errlen) {
    if (!d) { set_err(err, errlen, "null description%ld", 0); return -1; }
    if (d->abi_version != DBNET_ABI_VERSION) {
        set_err(err, errlen, "dbnet abi_version %ld unsupported", (long)d->abi_version);
        return -1;
    }
    if (d->n_pops < 1 || d->n_pops > DBNET_MAX_POPS || !d->pops) {
        set_err(err, errlen, "n_pops=%ld out of range or pops missing", (long)d->n_pops);
        return -1;
    }
    if (d->n_regions < 1) { set_err(err, errlen, "n_regions must be >= 1 (got %ld)", 0); return -1; }
    if (d->n_projs > 0 && !d->projs) { set_err(err, errlen, "projs missing%ld", 0); return -1; }
    if (!(d->dt_ms > 0.0f) || !(d->bin_ms > 0.0f) || !isfinite(d->dt_ms) || !isfinite(d->bin_ms)) {
        set_err(err, errlen, "dt_ms and bin_ms must be positive%ld", 0);
        return -1;
    }
    double ratio = (double)d->bin_ms / (double)d->dt_ms;
    long S = lround(ratio);
    if (fabs(ratio - (double)S) > 1e-6 * ratio || S < 1 || S > (long)DBNET_MAX_STEPS_PER_BIN) {
        set_err(err, errlen, "bin_ms/dt_ms must be an integer in [1,16] (steps per bin %ld)", S);
        return -1;
    }
    if (!dbnet_weights_per_edge(d)) {
        set_err(err, errlen, "receptor_mask 0x%lx unsupported (0x5 or 0xF)", (long)d->receptor_mask);
        return -1;
    }
    if (d->frac_bits < 1 || d->frac_bits > 40) {
        set_err(err, errlen, "frac_bits %ld out of [1,40]", (long)d->frac_bits);
        return -1;
    }
    uint64_t n = 0;
    for (uint32_t p = 0; p < d->n_pops; p++) {
        const dbnet_pop* P = &d->pops[p];
        if (P->size < 1) { set_err(err, errlen, "population %ld is empty", p); return -1; }
        if (P->region >= d->n_regions) { set_err(err, errlen, "population %ld region out of range", p); return -1; }
        if (!(P->C > 0.0f) || !isfinite(P->C) || !(P->g_L >= 0.0f) || !isfinite(P->g_L) ||
            !isfinite(P->V_L) || isnan(P->V_th) || !isfinite(P->V_reset) || !(P->T_ref >= 0.0f) ||
            !isfinite(P->T_ref) || !isfinite(P->I_ext)) {
            set_err(err, errlen, "population %ld has invalid membrane parameters", p);
            return -1;
        }
        for (int u = 0; u < 4; u++)
            if (!(P->g[u] >= 0.0f) || !isfinite(P->g[u]) || !isfinite(P->V_rev[u]) || !(P->tau[u] > 0.0f)) {
                set_err(err, errlen, "population %ld has invalid receptor parameters", p);
                return -1;
            }
        if (!(P->bg_rate_hz >= 0.0f) || !isfinite(P->bg_rate_hz) || !isfinite(P->w_bg) ||
            !isfinite(P->v0_lo) || !isfinite(P->v0_hi) || P->v0_hi < P->v0_lo) {
            set_err(err, errlen, "population %ld has invalid background or initial-state parameters", p);
            return -1;
        }
        n += P->size;
    }
    if (n >= DBNET_MAX_NEURONS) { set_err(err, errlen, "too many neurons (%ld)", (long)n); return -1; }
    int need_xyz = 0;
    for (uint32_t j = 0; j < d->n_projs; j++) {
        const dbnet_proj* pr = &d->projs[j];
        if (pr->dst_pop < -1 || pr->dst_pop >= (int32_t)d->n_pops) {
            set_err(err, errlen, "projection %ld dst_pop out of range", j); return -1;
        }
        if (pr->src_mode > DBNET_SRC_POP || pr->src_class > DBNET_CLASS_INH) {
            set_err(err, errlen, "projection %ld has an unknown source rule", j); return -1;
        }
        if (pr->src_mode == DBNET_SRC_POP && (pr->src_pop < 0 || pr->src_pop >= (int32_t)d->n_pops)) {
            set_err(err, errlen, "projection %ld src_pop out of range", j); return -1;
        }
        if (pr->w_dist > DBNET_W_CONST || !isfinite(pr->w_a) || !isfinite(pr->w_b) ||
            !isfinite(pr->w_scale_exc) || !isfinite(pr->w_scale_inh) ||
            (pr->w_dist == DBNET_W_UNIFORM && pr->w_b < pr->w_a) ||
            (pr->w_dist == DBNET_W_LOGNORMAL && pr->w_b < 0.0f)) {
            set_err(err, errlen, "projection %ld has invalid weight parameters", j); return -1;
        }
        if (pr->d_mode > DBNET_D_DISTANCE || pr->d_min < 1 || pr->d_max < pr->d_min ||
            pr->d_max > DBNET_MAX_DELAY) {
            set_err(err, errlen, "projection %ld has invalid delays (need 1 <= d_min <= d_max <= 255)", j);
            return -1;
        }
        if (pr->d_mode == DBNET_D_DISTANCE) need_xyz = 1;
        for (uint32_t p = 0; p < d->n_pops; p++) {
            if (!proj_applies(pr, p)) continue;
            if (candidate_count(d, pr, p) < pr->indegree) {
                set_err(err, errlen, "projection %ld asks more sources than exist", j);
                return -1;
            }
        }
    }
    if (need_xyz && (!d->region_xyz_mm || !(d->velocity_mm_per_ms > 0.0f))) {
        set_err(err, errlen, "distance delays need region_xyz_mm and velocity_mm_per_ms%ld", 0);
        return -1;
    }
    return 0;
}

uint32_t dbnet_indegree(const dbnet_desc* d, uint32_t i) {
    uint32_t tp = dbnet_pop_of(d, i), k = 0;
    for (uint32_t j = 0; j < d->n_projs; j++)
        if (proj_applies(&d->projs[j], tp)) k += d->projs[j].indegree;
    return k;
}

uint32_t dbnet_max_indegree(const dbnet_desc* d) {
    uint32_t m = 0;
    for (uint32_t p = 0; p < d->n_pops; p++) {
        uint32_t k = 0;
        for (uint32_t j = 0; j < d->n_projs; j++)
            if (proj_applies(&d->projs[j], p)) k += d->projs[j].indegree;
        if (k > m) m = k;
    }
    return m;
}

uint32_t dbnet_max_delay(const dbnet_desc* d) {
    uint32_t m = 1;
    for (uint32_t j = 0; j < d->n_projs; j++)
        if (d->projs[j].d_max > m && d->projs[j].indegree > 0) m = d->projs[j].d_max;
    return m;
}

static uint32_t pow2_at_least(uint64_t x) {
    uint32_t c = 1;
    while (c < x) c <<= 1;
    return c;
}

/* scratch layout: hash[hcap] u64 | picked[kmax] u64 | sorted[kmax] u64 | bucket[kmax+1] u32 |
   candpop[n_pops] u32 | (align 8) candend[n_pops] u64 | candoff[n_pops] u64 */
size_t dbnet_scratch_bytes(const dbnet_desc* d) {
    uint64_t kmax = 1;
    for (uint32_t j = 0; j < d->n_projs; j++)
        if (d->projs[j].indegree > kmax) kmax = d->projs[j].indegree;
    uint32_t hcap = pow2_at_least(2 * kmax + 2);
    return (size_t)hcap * 8 + (size_t)kmax * 16 + (size_t)(kmax + 1) * 4 + (size_t)d->n_pops * 20 + 64;
}

/* open-addressing set of u64 keys (stored +1 so 0 marks empty) */
static int set_insert(uint64_t* tab, uint32_t cap, uint64_t key) {
    uint32_t h = (uint32_t)(mix64(key) & (cap - 1));
    for (;;) {
        if (tab[h] == 0) { tab[h] = key + 1; return 1; }
        if (tab[h] == key + 1) return 0;
        h = (h + 1) & (cap - 1);
    }
}

/* key_a / key_b: stream keys of the weight's two streams for this target */
static double weight_draw(const dbnet_proj* pr, uint64_t key_a, uint64_t key_b, uint32_t j, uint64_t e) {
    switch (pr->w_dist) {
    case DBNET_W_UNIFORM: return (double)pr->w_a + ((double)pr->w_b - (double)pr->w_a) * u01(draw_k(key_a, j, e));
    case DBNET_W_LOGNORMAL: {
        /* Box-Muller normal deviate */
        double r = sqrt(-2.0 * log(u01_open0(draw_k(key_a, j, e))));
        double z = r * cos(6.283185307179586 * u01(draw_k(key_b, j, e)));
        return exp((double)pr->w_a + (double)pr->w_b * z);
    }
    default: return (double)pr->w_a;
    }
}

int64_t dbnet_in_edges(const dbnet_desc* d, uint32_t i, uint32_t* src, float* w0, float* w1,
                       uint8_t* delay, void* scratch) {
    uint32_t tp = dbnet_pop_of(d, i);
    if (tp >= d->n_pops) return -1;
    uint64_t kmax = 1;
    for (uint32_t j = 0; j < d->n_projs; j++)
        if (d->projs[j].indegree > kmax) kmax = d->projs[j].indegree;
    uint32_t hcap = pow2_at_least(2 * kmax + 2);
    uint64_t* hash = (uint64_t*)scratch;
    uint64_t* picked = hash + hcap;
    uint64_t* sorted = picked + kmax;
    uint32_t* bucket = (uint32_t*)(sorted + kmax);
    uint32_t* candpop = bucket + (kmax + 1);
    uint64_t* candend = (uint64_t*)(((uintptr_t)(candpop + d->n_pops) + 7) & ~(uintptr_t)7);
    uint64_t* candoff = candend + d->n_pops;
    const uint32_t kw = dbnet_weights_per_edge(d);
    const dbnet_pop* T = &d->pops[tp];
    int64_t out = 0;
    const uint64_t k_sample = stream_key(d, ST_SAMPLE, i), k_delay = stream_key(d, ST_DELAY, i);
    const uint64_t k_w0 = stream_key(d, ST_W0, i), k_w0b = stream_key(d, ST_W0B, i);
    const uint64_t k_w1 = stream_key(d, ST_W1, i), k_w1b = stream_key(d, ST_W1B, i);

    for (uint32_t j = 0; j < d->n_projs; j++) {
        const dbnet_proj* pr = &d->projs[j];
        if (!proj_applies(pr, tp) || pr->indegree == 0) continue;
        /* candidate populations in ascending id order, self removed from the index space */
        uint32_t nc = 0;
        uint64_t m = 0, self_pos = UINT64_MAX, off = 0;
        for (uint32_t q = 0; q < d->n_pops; off += d->pops[q].size, q++) {
            if (!candidate(d, pr, tp, q)) continue;
            if (q == tp) self_pos = m + (i - off);
            m += d->pops[q].size;
            candpop[nc] = q;
            candend[nc] = m;
            candoff[nc] = off;
            nc++;
        }
        uint64_t M = m - (self_pos != UINT64_MAX ? 1 : 0);
        uint32_t k = pr->indegree;
        if (M < k) return -1;
        /* Floyd's algorithm: k distinct indices uniform in [0, M) */
        memset(hash, 0, (size_t)hcap * 8);
        uint32_t np = 0;
        for (uint64_t t = M - k; t < M; t++) {
            uint64_t r = below(draw_k(k_sample, j, t), t + 1);
            if (set_insert(hash, hcap, r)) picked[np++] = r;
            else { set_insert(hash, hcap, t); picked[np++] = t; }
        }
        /* sort: bucket by value then insertion sort (expected linear for uniform values) */
        memset(bucket, 0, (size_t)(k + 1) * 4);
        for (uint32_t a = 0; a < k; a++) bucket[below(picked[a] * (UINT64_MAX / M), k) + 1]++;
        for (uint32_t a = 0; a < k; a++) bucket[a + 1] += bucket[a];
        for (uint32_t a = 0; a < k; a++) sorted[bucket[below(picked[a] * (UINT64_MAX / M), k)]++] = picked[a];
        for (uint32_t a = 1; a < k; a++) {
            uint64_t v = sorted[a];
            uint32_t b = a;
            while (b > 0 && sorted[b - 1] > v) { sorted[b] = sorted[b - 1]; b--; }
            sorted[b] = v;
        }
        /* map indices to neuron ids, then draw weights and delays */
        uint32_t c = 0;
        for (uint32_t a = 0; a < k; a++) {
            uint64_t x = sorted[a];
            if (x >= self_pos) x++;
            while (x >= candend[c]) c++;
            uint32_t q = candpop[c];
            uint64_t base = candend[c] - d->pops[q].size;
            uint32_t s = (uint32_t)(candoff[c] + (x - base));
            const dbnet_pop* Sp = &d->pops[q];
            double scale = Sp->exc ? (double)pr->w_scale_exc : (double)pr->w_scale_inh;
            src[out] = s;
            if (w0) w0[out] = (float)(scale * weight_draw(pr, k_w0, k_w0b, j, a));
            if (w1) w1[out] = kw == 2 ? (float)(scale * weight_draw(pr, k_w1, k_w1b, j, a)) : 0.0f;
            uint32_t dl;
            if (pr->d_mode == DBNET_D_FIXED) {
                dl = pr->d_min;
            } else if (pr->d_mode == DBNET_D_UNIFORM) {
                dl = pr->d_min + (uint32_t)below(draw_k(k_delay, j, a), pr->d_max - pr->d_min + 1);
            } else {
                const float* xs = d->region_xyz_mm + 3 * Sp->region;
                const float* xt = d->region_xyz_mm + 3 * T->region;
                double dx = (double)xs[0] - xt[0], dy = (double)xs[1] - xt[1], dz = (double)xs[2] - xt[2];
                double dist = sqrt(dx * dx + dy * dy + dz * dz);
                double bins = ceil(dist / ((double)d->velocity_mm_per_ms * (double)d->bin_ms));
                dl = bins < (double)pr->d_min ? pr->d_min : bins > (double)pr->d_max ? pr->d_max : (uint32_t)bins;
            }
            if (delay) delay[out] = (uint8_t)dl;
            out++;
        }
    }
    return out;
}

float dbnet_v0(const dbnet_desc* d, uint32_t i) {
    const dbnet_pop* P = &d->pops[dbnet_pop_of(d, i)];
    double u = u01(draw(d, ST_V0, i, 0, 0));
    return (float)((double)P->v0_lo + ((double)P->v0_hi - (double)P->v0_lo) * u);
}
