/*
 * snnc_oracle.c -- CPU oracle for on-device spiking-network construction.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this code.  It shares no source,
 * header, table or helper with the GPU library: every step below is written
 * out again from the paper (Golosio, Tiddia, Villamar et al., "Scalable
 * Construction of Spiking Neural Networks using up to thousands of GPUs",
 * arXiv:2512.09502) and from the published definitions it relies on.
 *
 * Plain, single-threaded, deliberately slow: nested loops, linear searches,
 * qsort.  Floating point is IEEE double except where the result format is
 * fixed (fp32 weights, integer delay steps).
 *
 * What it computes (one virtual host's share, host P_local of P):
 *   - Philox4x32-10 blocks keyed by (seed, call id), counter (e, purpose).
 *   - Connection draws of the five Connect rules (Methods, "Creation of the
 *     remote connection structures"; the rules are those of the
 *     connectivity-concepts reference the paper cites), in canonical
 *     generation order (call, e).  Sources are kept as their position in the
 *     call's source set, the paper's temporary source positions.
 *   - Synapse values: fp32 weight (Box-Muller), integer delay step.
 *   - Prepare: the remote-source image map per (alpha+1, sigma) (Methods,
 *     point-to-point and collective sections: flag, compact, sort, search,
 *     append, remap), the source-major connection sort with its first-index
 *     array (Methods, "GPU memory levels"), the point-to-point send lists
 *     S, T, P, and the collective arrays H, I, G, Q.
 *
 * Readings where the paper leaves a choice open (RNG, value mappings, image
 * numbering, tie order) are listed at each function.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ESTATE (-4)
#define ORC_EUNSUPPORTED (-5)

enum { R_ONE_TO_ONE = 0, R_INDEGREE = 1, R_OUTDEGREE = 2, R_TOTAL = 3, R_BERNOULLI = 4, R_ASSIGNED = 5 };
enum { D_CONST = 0, D_NORMAL = 1 };
enum { PURPOSE_IDX = 0, PURPOSE_SYN = 1, PURPOSE_BERN = 2 };

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, "Parallel random       */
/* numbers: as easy as 1, 2, 3").  One round multiplies counter words 0 and */
/* 2 by the two round constants as 32x32->64 products and mixes the high    */
/* halves with the other counter words and the key; the key is bumped by    */
/* the two Weyl constants between rounds.  Ten rounds.                      */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(prod1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)prod1;
        uint32_t n2 = (uint32_t)(prod0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)prod0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The stream of one Connect call: key = (seed, call id), counter =
 * (low and high word of the element index e, purpose, 0).  This replaces the
 * paper's aligned generator array RNG_{sigma,tau}, which it only requires to
 * give source and target process the same numbers. */
static void draw_block(uint32_t seed, uint32_t call_id, uint64_t e, uint32_t purpose, uint32_t w[4])
{
    uint32_t ctr[4] = { (uint32_t)(e & 0xffffffffu), (uint32_t)(e >> 32), purpose, 0u };
    uint32_t key[2] = { seed, call_id };
    orc_philox4x32_10(ctr, key, w);
}

/* Uniform index in [0, n) from two 32-bit words: the 64-bit fraction
 * u = (hi:lo) / 2^64 scaled by n and truncated, i.e. floor(u * n / 2^64). */
uint64_t orc_uniform_index(uint32_t lo, uint32_t hi, uint64_t n)
{
    uint64_t u = ((uint64_t)hi << 32) | (uint64_t)lo;
    unsigned __int128 prod = (unsigned __int128)u * (unsigned __int128)n;
    return (uint64_t)(prod >> 64);
}

/* Acceptance threshold of a pairwise Bernoulli(p) test on a uniform 32-bit
 * word w: the pair connects iff w < floor(p 2^32); p = 1 gives 2^32, so every
 * word passes.  The probability is floor(p 2^32) / 2^32, within 2^-32 of p. */
static uint64_t bern_threshold(double p)
{
    if (p >= 1.0) return 4294967296ull;
    return (uint64_t)floor(p * 4294967296.0);
}

/* Normal weight by the Box-Muller transform, cosine branch, in double,
 * rounded once to fp32: u1 = (w0 + 1) / 2^32 in (0, 1], u2 = w1 / 2^32,
 * z = sqrt(-2 ln u1) cos(2 pi u2), weight = (float)(mean + sd * z). */
float orc_normal_weight(uint32_t w0, uint32_t w1, double mean, double sd)
{
    const double two_pi = 6.283185307179586476925286766559;
    double u1 = ((double)w0 + 1.0) * (1.0 / 4294967296.0);
    double u2 = (double)w1 * (1.0 / 4294967296.0);
    double radius = sqrt(-2.0 * log(u1));
    double angle = two_pi * u2;
    double z = radius * cos(angle);
    double scaled = sd * z;
    double value = mean + scaled;
    return (float)value;
}

/* Standard normal CDF from the complementary error function. */
static double std_normal_cdf(double x)
{
    return 0.5 * erfc(-x / 1.41421356237309504880168872420969808);
}

/* Delays are integer multiples of the time step (App. E, delivery example).
 * A normally distributed delay d ~ N(mean, sd) in ms, clipped from below at
 * lo, becomes round(max(d, lo) / dt) steps (ties away from zero).  It is
 * sampled exactly by inversion of that discrete distribution on a 32-bit
 * uniform word:  with k_lo = round(lo / dt) and, for k >= k_lo,
 * F(k) = Phi(((k + 1/2) dt - mean) / sd), threshold t_k = ceil(F(k) 2^32);
 * the step is k_lo + #{k : word >= t_k}.  The table keeps the thresholds
 * below 2^32.  Returns the table length, or -1 if it would not fit. */
int64_t orc_delay_table(double mean, double sd, double lo, double dt,
                        uint32_t* table, uint64_t cap, uint32_t* k_lo_out)
{
    double k_lo_d = round(lo / dt);
    if (!(k_lo_d >= 1.0) || k_lo_d > 65535.0) return -1;
    uint32_t k_lo = (uint32_t)k_lo_d;
    uint64_t len = 0;
    for (uint64_t k = k_lo; ; k++) {
        double x = (((double)k + 0.5) * dt - mean) / sd;
        double F = std_normal_cdf(x);
        double t = ceil(F * 4294967296.0);
        if (t >= 4294967296.0) break;
        if (k >= 65535) return -1;      /* step k+1 would not fit uint16 */
        if (len >= cap) return -1;
        table[len++] = (uint32_t)t;
    }
    *k_lo_out = k_lo;
    return (int64_t)len;
}

/* ------------------------------------------------------------------------ */
/* Network description                                                      */
/* ------------------------------------------------------------------------ */
typedef struct { uint32_t host, first, n; } orc_seg;

typedef struct {
    orc_seg* seg;
    uint32_t nseg;
    uint64_t total;
} orc_set;

typedef struct {
    int kind;
    double mean, sd, lo;
} orc_dist;

typedef struct {
    uint32_t id;
    int rule;
    uint64_t n;
    double p;
    int autapses, multapses;
    orc_set S, T;
    int32_t alpha;
    orc_dist w, d;
    float w_const;
    uint16_t d_const;
    uint32_t* dtab;
    uint32_t dtab_len;
    uint32_t d_klo;
    uint32_t* pair_s;     /* assigned nodes: source and target ordinal of pair i (n pairs) */
    uint32_t* pair_t;
    uint64_t gen_begin, gen_count;
} orc_call;

typedef struct orc_net {
    uint32_t P, P_local, seed;
    double dt;
    uint32_t* M;
    orc_call* calls;
    uint32_t ncalls, capcalls;
    /* local share, generation order */
    uint32_t* g_src;
    uint32_t* g_tgt;
    uint16_t* g_delay;
    float* g_weight;
    uint64_t* g_e;
    uint64_t n_gen, cap_gen;
    uint64_t* call_off;
    int prepared;
    /* map policy: image numbering (0 canonical, 1 in call order) and which
     * sources get images (0 used, 1 threshold heuristic, 2 all passed) */
    int numbering, img_sources;
    double xi;
    /* GPU memory level (Methods, GPU memory levels subsection), -1 when not
     * set; decides which of the first-index and count arrays of the image
     * rows exist (placement in host or device memory has no counterpart here) */
    int mem_level;
    uint64_t* img_first;
    uint32_t* img_count;
    /* image map */
    uint32_t n_a;
    uint64_t* r_off;
    int32_t* r_val;
    int32_t* l_val;
    int64_t* img_base;
    uint64_t n_img;
    /* sorted connections and first-index array */
    int32_t* s_src;
    int32_t* s_tgt;
    uint16_t* s_delay;
    float* s_weight;
    uint64_t* row_ptr;
    uint64_t n_rows;
    /* point-to-point send lists */
    uint64_t* S_off;
    int32_t* S_val;
    uint64_t* TP_ptr;
    uint32_t* T_val;
    uint32_t* P_val;
    /* collective arrays */
    uint32_t n_groups;
    int32_t* groups;
    uint64_t* H_off;
    int32_t* H_val;
    int32_t* I_val;
    uint64_t* GQ_ptr;
    int32_t* G_val;
    uint32_t* Q_val;
    char err[256];
} orc_net;

static int fail(orc_net* net, int code, const char* msg)
{
    snprintf(net->err, sizeof net->err, "%s", msg);
    return code;
}

const char* orc_last_error(const orc_net* net) { return net->err; }

orc_net* orc_new(uint32_t P, uint32_t P_local, uint32_t seed, double dt)
{
    if (P == 0 || P_local >= P || !(dt > 0.0)) return NULL;
    orc_net* net = (orc_net*)calloc(1, sizeof(orc_net));
    net->P = P; net->P_local = P_local; net->seed = seed; net->dt = dt;
    net->M = (uint32_t*)calloc(P, sizeof(uint32_t));
    net->xi = 1.0;
    net->mem_level = -1;
    return net;
}

int orc_set_map_policy(orc_net* net, int numbering, int img_sources, double xi)
{
    if (net->prepared) return fail(net, ORC_ESTATE, "map policy after prepare");
    if (numbering < 0 || numbering > 1 || img_sources < 0 || img_sources > 2 || !(xi >= 0.0) || xi > 1e300)
        return fail(net, ORC_EINVAL, "bad map policy");
    net->numbering = numbering; net->img_sources = img_sources; net->xi = xi;
    return ORC_OK;
}

/* GPU memory level 0..3 (Methods, GPU memory levels subsection), before
 * prepare: level 0 gives images to the used sources only, levels 1 to 3 to
 * every source passed to a call (the image-source choice of the map policy,
 * which a later orc_set_map_policy overrides); the level also decides which
 * first-index and count arrays of the image rows exist. */
int orc_set_memory_level(orc_net* net, int level)
{
    if (net->prepared) return fail(net, ORC_ESTATE, "memory level after prepare");
    if (level < 0 || level > 3) return fail(net, ORC_EINVAL, "memory level out of range");
    net->mem_level = level;
    net->img_sources = level == 0 ? 0 : 2;
    return ORC_OK;
}

static void free_prepared(orc_net* net)
{
    free(net->r_off); free(net->r_val); free(net->l_val); free(net->img_base);
    free(net->s_src); free(net->s_tgt); free(net->s_delay); free(net->s_weight); free(net->row_ptr);
    free(net->S_off); free(net->S_val); free(net->TP_ptr); free(net->T_val); free(net->P_val);
    free(net->groups); free(net->H_off); free(net->H_val); free(net->I_val);
    free(net->GQ_ptr); free(net->G_val); free(net->Q_val);
    free(net->img_first); free(net->img_count);
}

void orc_free(orc_net* net)
{
    if (!net) return;
    for (uint32_t c = 0; c < net->ncalls; c++) {
        free(net->calls[c].S.seg); free(net->calls[c].T.seg); free(net->calls[c].dtab);
        free(net->calls[c].pair_s); free(net->calls[c].pair_t);
    }
    free(net->calls); free(net->M);
    free(net->g_src); free(net->g_tgt); free(net->g_delay); free(net->g_weight); free(net->g_e);
    free(net->call_off);
    free_prepared(net);
    free(net);
}

/* Create(population, n): n new neurons on a host get the next local ids. */
int orc_create(orc_net* net, uint32_t host, uint32_t n, uint32_t* first_out)
{
    if (net->prepared) return fail(net, ORC_ESTATE, "create after prepare");
    if (host >= net->P) return fail(net, ORC_EINVAL, "host out of range");
    if ((uint64_t)net->M[host] + n > 0x7fffffffu) return fail(net, ORC_EINVAL, "too many neurons on host");
    *first_out = net->M[host];
    net->M[host] += n;
    return ORC_OK;
}

/* Ordinal -> (host, local id): walk the segments in order. */
static void set_at(const orc_set* s, uint64_t ord, uint32_t* host, uint32_t* local)
{
    for (uint32_t i = 0; i < s->nseg; i++) {
        if (ord < s->seg[i].n) {
            *host = s->seg[i].host;
            *local = s->seg[i].first + (uint32_t)ord;
            return;
        }
        ord -= s->seg[i].n;
    }
    *host = 0xffffffffu; *local = 0xffffffffu;   /* not reached for valid ordinals */
}

/* Position of neuron (host, local) in a set, or -1. */
static int64_t set_pos(const orc_set* s, uint32_t host, uint32_t local)
{
    uint64_t base = 0;
    for (uint32_t i = 0; i < s->nseg; i++) {
        const orc_seg* g = &s->seg[i];
        if (g->host == host && local >= g->first && local < g->first + g->n)
            return (int64_t)(base + (local - g->first));
        base += g->n;
    }
    return -1;
}

/* Number of neurons that belong to both sets. */
static uint64_t set_overlap(const orc_set* a, const orc_set* b)
{
    uint64_t total = 0;
    for (uint32_t i = 0; i < a->nseg; i++)
        for (uint32_t j = 0; j < b->nseg; j++) {
            const orc_seg* x = &a->seg[i];
            const orc_seg* y = &b->seg[j];
            if (x->host != y->host) continue;
            uint64_t lo = x->first > y->first ? x->first : y->first;
            uint64_t hi_x = (uint64_t)x->first + x->n, hi_y = (uint64_t)y->first + y->n;
            uint64_t hi = hi_x < hi_y ? hi_x : hi_y;
            if (hi > lo) total += hi - lo;
        }
    return total;
}

static int copy_set(orc_net* net, const uint32_t* triples, uint32_t nseg, orc_set* out)
{
    out->seg = (orc_seg*)calloc(nseg ? nseg : 1, sizeof(orc_seg));
    out->nseg = nseg;
    out->total = 0;
    for (uint32_t i = 0; i < nseg; i++) {
        orc_seg g = { triples[3 * i], triples[3 * i + 1], triples[3 * i + 2] };
        if (g.host >= net->P) return fail(net, ORC_EINVAL, "segment host out of range");
        if ((uint64_t)g.first + g.n > net->M[g.host]) return fail(net, ORC_EINVAL, "segment outside created neurons");
        out->seg[i] = g;
        out->total += g.n;
    }
    /* a set lists each neuron at most once */
    if (set_overlap(out, out) != out->total) return fail(net, ORC_EINVAL, "segments of a set overlap");
    if (out->total > 0xffffffffull) return fail(net, ORC_EINVAL, "set larger than 2^32-1 neurons");
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Rule draws.  gen_call walks the draws of one call that land on a given    */
/* host's share and hands each accepted connection (source position in S,   */
/* target local id, element index e) to a sink.  `lo`/`hi` restrict the     */
/* primary ordinal (target ordinal for in-degree, Bernoulli and one-to-one, */
/* source ordinal for out-degree, candidate index for total number).        */
/* ------------------------------------------------------------------------ */
typedef struct {
    void (*emit)(void* ctx, uint64_t src_ord, uint32_t tgt_local, uint64_t e);
    void* ctx;
} sink_t;

static int cmp_u64(const void* a, const void* b)
{
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* Robert Floyd's sampling of k distinct values in [0, n): for j = 0..k-1,
 * with m = n - k + j, draw r uniform in [0, m]; take r unless it was taken,
 * else take m.  The draws use element indices base + j.  The chosen values
 * are returned sorted ascending (membership test by linear scan). */
static void floyd_sample(const orc_net* net, uint32_t call_id, uint64_t base, uint64_t k, uint64_t n,
                         uint64_t* chosen)
{
    for (uint64_t j = 0; j < k; j++) {
        uint64_t m = n - k + j;
        uint32_t w[4];
        draw_block(net->seed, call_id, base + j, PURPOSE_IDX, w);
        uint64_t r = orc_uniform_index(w[0], w[1], m + 1);
        int taken = 0;
        for (uint64_t i = 0; i < j; i++)
            if (chosen[i] == r) { taken = 1; break; }
        chosen[j] = taken ? m : r;
    }
    qsort(chosen, k, sizeof(uint64_t), cmp_u64);
}

/* One "K draws from a set of size n_set" group: fixed in-degree draws K
 * sources for a target, fixed out-degree K targets for a source.  self_pos is
 * the position of the other end in the drawn set when autapses are excluded
 * (else -1): the draw then runs over n_set - 1 values and skips self_pos. */
static void draw_k(const orc_net* net, const orc_call* c, uint64_t base, uint64_t K, uint64_t n_set,
                   int64_t self_pos, uint64_t* out)
{
    uint64_t n_eff = n_set - (self_pos >= 0 ? 1 : 0);
    if (c->multapses) {
        for (uint64_t j = 0; j < K; j++) {
            uint32_t w[4];
            draw_block(net->seed, c->id, base + j, PURPOSE_IDX, w);
            out[j] = orc_uniform_index(w[0], w[1], n_eff);
        }
    } else {
        floyd_sample(net, c->id, base, K, n_eff, out);
    }
    if (self_pos >= 0)
        for (uint64_t j = 0; j < K; j++)
            if (out[j] >= (uint64_t)self_pos) out[j] += 1;
}

/* Open-addressing set of (source ordinal, target ordinal) pairs. */
typedef struct { uint64_t* key; uint64_t cap; uint64_t n; } pairset;

static uint64_t mix64(uint64_t x)
{
    x ^= x >> 33; x *= 0xff51afd7ed558ccdull; x ^= x >> 33; x *= 0xc4ceb9fe1a85ec53ull; x ^= x >> 33;
    return x;
}

static int pairset_insert(pairset* s, uint64_t a, uint64_t b)   /* 1 if new */
{
    if (2 * (s->n + 1) > s->cap) {
        uint64_t ncap = s->cap ? s->cap * 2 : 1024;
        uint64_t* nk = (uint64_t*)malloc(ncap * 2 * sizeof(uint64_t));
        for (uint64_t i = 0; i < ncap; i++) nk[2 * i] = UINT64_MAX;
        for (uint64_t i = 0; i < s->cap; i++) {
            if (s->key[2 * i] == UINT64_MAX) continue;
            uint64_t h = mix64(s->key[2 * i] * 0x9E3779B97F4A7C15ull ^ s->key[2 * i + 1]) & (ncap - 1);
            while (nk[2 * h] != UINT64_MAX) h = (h + 1) & (ncap - 1);
            nk[2 * h] = s->key[2 * i]; nk[2 * h + 1] = s->key[2 * i + 1];
        }
        free(s->key); s->key = nk; s->cap = ncap;
    }
    uint64_t h = mix64(a * 0x9E3779B97F4A7C15ull ^ b) & (s->cap - 1);
    while (s->key[2 * h] != UINT64_MAX) {
        if (s->key[2 * h] == a && s->key[2 * h + 1] == b) return 0;
        h = (h + 1) & (s->cap - 1);
    }
    s->key[2 * h] = a; s->key[2 * h + 1] = b; s->n++;
    return 1;
}

static void gen_call(const orc_net* net, const orc_call* c, uint32_t host, uint64_t lo, uint64_t hi, sink_t sink)
{
    const uint64_t ns = c->S.total, nt = c->T.total;
    uint32_t h, l, h2, l2;
    switch (c->rule) {
    case R_INDEGREE: {
        uint64_t K = c->n;
        uint64_t* buf = (uint64_t*)malloc((K ? K : 1) * sizeof(uint64_t));
        for (uint64_t t = lo; t < hi && t < nt; t++) {
            set_at(&c->T, t, &h, &l);
            if (h != host) continue;
            int64_t self_pos = c->autapses ? -1 : set_pos(&c->S, h, l);
            draw_k(net, c, t * K, K, ns, self_pos, buf);
            for (uint64_t j = 0; j < K; j++) sink.emit(sink.ctx, buf[j], l, t * K + j);
        }
        free(buf);
        break;
    }
    case R_OUTDEGREE: {
        uint64_t K = c->n;
        uint64_t* buf = (uint64_t*)malloc((K ? K : 1) * sizeof(uint64_t));
        for (uint64_t s = lo; s < hi && s < ns; s++) {
            set_at(&c->S, s, &h, &l);
            int64_t self_pos = c->autapses ? -1 : set_pos(&c->T, h, l);
            draw_k(net, c, s * K, K, nt, self_pos, buf);
            for (uint64_t j = 0; j < K; j++) {
                set_at(&c->T, buf[j], &h2, &l2);
                if (h2 == host) sink.emit(sink.ctx, s, l2, s * K + j);
            }
        }
        free(buf);
        break;
    }
    case R_TOTAL: {
        /* The rule over the whole target set (reading for targets on several
         * hosts): candidates c = 0, 1, ... draw a pair over S x T, the first
         * N valid ones are the connections, and each host keeps those whose
         * target it holds.  Every host evaluates every candidate. */
        pairset seen = { NULL, 0, 0 };
        uint64_t accepted = 0;
        for (uint64_t cand = 0; accepted < c->n && cand < hi; cand++) {
            uint32_t w[4];
            draw_block(net->seed, c->id, cand, PURPOSE_IDX, w);
            uint64_t s = orc_uniform_index(w[0], w[1], ns);
            uint64_t t = orc_uniform_index(w[2], w[3], nt);
            set_at(&c->S, s, &h, &l);
            set_at(&c->T, t, &h2, &l2);
            if (!c->autapses && h == h2 && l == l2) continue;
            if (!c->multapses && !pairset_insert(&seen, s, t)) continue;
            accepted++;
            if (cand >= lo && h2 == host) sink.emit(sink.ctx, s, l2, cand);
        }
        free(seen.key);
        break;
    }
    case R_BERNOULLI: {
        /* Pairwise Bernoulli (the rule dictionary C; realisation is a
         * reading): every (source, target) pair is an independent test.  The
         * pairs are numbered target-major, q = t n_s + s, and four pairs share
         * one Philox block: pair q connects iff word (q mod 4) of BERN(q / 4)
         * is below T_p = floor(p 2^32), with T_p = 2^32 for p = 1 (every pair
         * connects).  The connection's element index is q. */
        const uint64_t thr = bern_threshold(c->p);
        for (uint64_t t = lo; t < hi && t < nt; t++) {
            set_at(&c->T, t, &h2, &l2);
            if (h2 != host) continue;
            for (uint64_t s = 0; s < ns; s++) {
                const uint64_t q = t * ns + s;
                uint32_t w[4];
                draw_block(net->seed, c->id, q / 4, PURPOSE_BERN, w);
                if ((uint64_t)w[q % 4] >= thr) continue;
                if (!c->autapses) {
                    set_at(&c->S, s, &h, &l);
                    if (h == h2 && l == l2) continue;
                }
                sink.emit(sink.ctx, s, l2, q);
            }
        }
        break;
    }
    case R_ONE_TO_ONE: {
        for (uint64_t i = lo; i < hi && i < nt; i++) {
            set_at(&c->T, i, &h2, &l2);
            if (h2 != host) continue;
            if (!c->autapses) {
                set_at(&c->S, i, &h, &l);
                if (h == h2 && l == l2) continue;
            }
            sink.emit(sink.ctx, i, l2, i);
        }
        break;
    }
    case R_ASSIGNED: {
        /* assigned nodes (distributed fixed in-degree subsection): pair i
         * gives the source and target positions itself; the host of the
         * target keeps it.  Element index i. */
        for (uint64_t i = lo; i < hi && i < c->n; i++) {
            set_at(&c->T, c->pair_t[i], &h2, &l2);
            if (h2 == host) sink.emit(sink.ctx, c->pair_s[i], l2, i);
        }
        break;
    }
    }
}

/* ------------------------------------------------------------------------ */
/* Connect                                                                   */
/* ------------------------------------------------------------------------ */
typedef struct { orc_net* net; const orc_call* c; } local_sink_ctx;

static void grow_gen(orc_net* net, uint64_t need)
{
    if (need <= net->cap_gen) return;
    uint64_t cap = net->cap_gen ? net->cap_gen : 1024;
    while (cap < need) cap *= 2;
    net->g_src = (uint32_t*)realloc(net->g_src, cap * sizeof(uint32_t));
    net->g_tgt = (uint32_t*)realloc(net->g_tgt, cap * sizeof(uint32_t));
    net->g_delay = (uint16_t*)realloc(net->g_delay, cap * sizeof(uint16_t));
    net->g_weight = (float*)realloc(net->g_weight, cap * sizeof(float));
    net->g_e = (uint64_t*)realloc(net->g_e, cap * sizeof(uint64_t));
    net->cap_gen = cap;
}

/* The synapse values of element e always come from block SYN(e) of the same
 * call: weight from words 0 and 1, delay step from word 2. */
static void emit_local(void* vctx, uint64_t src_ord, uint32_t tgt_local, uint64_t e)
{
    local_sink_ctx* ctx = (local_sink_ctx*)vctx;
    orc_net* net = ctx->net;
    const orc_call* c = ctx->c;
    grow_gen(net, net->n_gen + 1);
    uint64_t i = net->n_gen++;
    net->g_src[i] = (uint32_t)src_ord;
    net->g_tgt[i] = tgt_local;
    net->g_e[i] = e;
    uint32_t w[4] = { 0, 0, 0, 0 };
    if (c->w.kind != D_CONST || c->d.kind != D_CONST)
        draw_block(net->seed, c->id, e, PURPOSE_SYN, w);
    net->g_weight[i] = (c->w.kind == D_CONST) ? c->w_const : orc_normal_weight(w[0], w[1], c->w.mean, c->w.sd);
    if (c->d.kind == D_CONST) {
        net->g_delay[i] = c->d_const;
    } else {
        uint32_t count = 0;
        for (uint32_t k = 0; k < c->dtab_len; k++)
            if (w[2] >= c->dtab[k]) count++;
        net->g_delay[i] = (uint16_t)(c->d_klo + count);
    }
}

static int validate_and_fill(orc_net* net, orc_call* c)
{
    const uint64_t ns = c->S.total, nt = c->T.total;
    uint64_t ov = c->autapses ? 0 : set_overlap(&c->S, &c->T);
    switch (c->rule) {
    case R_ONE_TO_ONE:
        if (ns != nt) return fail(net, ORC_EINVAL, "one-to-one needs equal set sizes");
        break;
    case R_INDEGREE:
        if (c->n > 0 && nt > 0) {
            uint64_t n_eff = ns - (ov > 0 ? 1 : 0);
            if (ns == 0 || n_eff == 0) return fail(net, ORC_EINVAL, "no source to draw from");
            if (!c->multapses && c->n > n_eff) return fail(net, ORC_EINVAL, "in-degree exceeds candidates without multapses");
        }
        break;
    case R_OUTDEGREE:
        if (c->n > 0 && ns > 0) {
            uint64_t n_eff = nt - (ov > 0 ? 1 : 0);
            if (nt == 0 || n_eff == 0) return fail(net, ORC_EINVAL, "no target to draw from");
            if (!c->multapses && c->n > n_eff) return fail(net, ORC_EINVAL, "out-degree exceeds candidates without multapses");
        }
        break;
    case R_TOTAL: {
        if (c->n > 0) {
            if (ns == 0 || nt == 0) return fail(net, ORC_EINVAL, "empty set");
            unsigned __int128 pairs = (unsigned __int128)ns * nt - ov;
            if (pairs == 0) return fail(net, ORC_EINVAL, "no valid pair");
            if (!c->multapses && (unsigned __int128)c->n > pairs) return fail(net, ORC_EINVAL, "total number exceeds pairs without multapses");
        }
        break;
    }
    case R_BERNOULLI:
        if (!(c->p >= 0.0 && c->p <= 1.0)) return fail(net, ORC_EINVAL, "probability outside [0,1]");
        break;
    case R_ASSIGNED:
        if (c->n > 0 && (!c->pair_s || !c->pair_t)) return fail(net, ORC_EINVAL, "assigned nodes without pairs");
        for (uint64_t i = 0; i < c->n; i++)
            if (c->pair_s[i] >= ns || c->pair_t[i] >= nt) return fail(net, ORC_EINVAL, "assigned pair outside the sets");
        break;
    default:
        return fail(net, ORC_EINVAL, "unknown rule");
    }
    if (c->alpha < -1) return fail(net, ORC_EINVAL, "group index below -1");
    /* synapse values */
    if (c->w.kind == D_CONST) c->w_const = (float)c->w.mean;
    else if (c->w.kind == D_NORMAL) { if (!(c->w.sd >= 0.0)) return fail(net, ORC_EINVAL, "weight sd < 0"); }
    else return fail(net, ORC_EINVAL, "unknown weight distribution");
    if (c->d.kind == D_CONST) {
        if (!(c->d.mean >= net->dt)) return fail(net, ORC_EINVAL, "delay below one time step");
        double steps = round(c->d.mean / net->dt);
        if (steps > 65535.0) return fail(net, ORC_EINVAL, "delay too long for uint16 steps");
        c->d_const = (uint16_t)steps;
    } else if (c->d.kind == D_NORMAL) {
        if (!(c->d.sd > 0.0)) return fail(net, ORC_EINVAL, "delay sd must be > 0");
        if (!(c->d.lo >= net->dt)) return fail(net, ORC_EINVAL, "delay clip below one time step");
        uint64_t cap = 65536;
        c->dtab = (uint32_t*)malloc(cap * sizeof(uint32_t));
        int64_t len = orc_delay_table(c->d.mean, c->d.sd, c->d.lo, net->dt, c->dtab, cap, &c->d_klo);
        if (len < 0) return fail(net, ORC_EINVAL, "delay distribution does not fit uint16 steps");
        c->dtab_len = (uint32_t)len;
    } else {
        return fail(net, ORC_EINVAL, "unknown delay distribution");
    }
    return ORC_OK;
}

/* Validates a call record, appends it and generates P_local's share. */
static int add_call(orc_net* net, orc_call* c, uint32_t* call_id_out)
{
    int st = validate_and_fill(net, c);
    if (st != ORC_OK) {
        free(c->S.seg); free(c->T.seg); free(c->dtab); free(c->pair_s); free(c->pair_t);
        return st;
    }
    if (net->ncalls == net->capcalls) {
        net->capcalls = net->capcalls ? 2 * net->capcalls : 16;
        net->calls = (orc_call*)realloc(net->calls, net->capcalls * sizeof(orc_call));
    }
    net->calls[net->ncalls] = *c;
    orc_call* cp = &net->calls[net->ncalls];
    net->ncalls++;
    cp->gen_begin = net->n_gen;
    local_sink_ctx ctx = { net, cp };
    sink_t sink = { emit_local, &ctx };
    gen_call(net, cp, net->P_local, 0, UINT64_MAX, sink);
    cp->gen_count = net->n_gen - cp->gen_begin;
    *call_id_out = cp->id;
    return ORC_OK;
}

static int init_call(orc_net* net, orc_call* c, const uint32_t* src_triples, uint32_t n_src_seg,
                     const uint32_t* tgt_triples, uint32_t n_tgt_seg,
                     int rule, uint64_t n, double p, int autapses, int multapses,
                     int w_kind, double w_mean, double w_sd,
                     int d_kind, double d_mean, double d_sd, double d_lo, int32_t alpha)
{
    memset(c, 0, sizeof *c);
    c->id = net->ncalls;
    c->rule = rule; c->n = n; c->p = p; c->autapses = autapses != 0; c->multapses = multapses != 0;
    c->alpha = alpha;
    c->w.kind = w_kind; c->w.mean = w_mean; c->w.sd = w_sd; c->w.lo = 0.0;
    c->d.kind = d_kind; c->d.mean = d_mean; c->d.sd = d_sd; c->d.lo = d_lo;
    int st = copy_set(net, src_triples, n_src_seg, &c->S);
    if (st == ORC_OK) st = copy_set(net, tgt_triples, n_tgt_seg, &c->T);
    if (st != ORC_OK) { free(c->S.seg); free(c->T.seg); }
    return st;
}

/* Connect(src, tgt, rule, syn_spec) with group alpha (-1: point-to-point).
 * Sets are lists of (host, first, n) triples; the position of a neuron in a
 * set is its rank in the concatenation of the segments. */
int orc_connect(orc_net* net, const uint32_t* src_triples, uint32_t n_src_seg,
                const uint32_t* tgt_triples, uint32_t n_tgt_seg,
                int rule, uint64_t n, double p, int autapses, int multapses,
                int w_kind, double w_mean, double w_sd,
                int d_kind, double d_mean, double d_sd, double d_lo,
                int32_t alpha, uint32_t* call_id_out)
{
    if (net->prepared) return fail(net, ORC_ESTATE, "connect after prepare");
    if (rule == R_ASSIGNED) return fail(net, ORC_EINVAL, "assigned nodes take their pairs (orc_connect_assigned)");
    orc_call c;
    int st = init_call(net, &c, src_triples, n_src_seg, tgt_triples, n_tgt_seg, rule, n, p, autapses, multapses,
                       w_kind, w_mean, w_sd, d_kind, d_mean, d_sd, d_lo, alpha);
    if (st != ORC_OK) return st;
    return add_call(net, &c, call_id_out);
}

/* Connect with the assigned-nodes rule: n pairs (pair_s[i], pair_t[i]) of
 * source and target positions in the two sets (copied). */
int orc_connect_assigned(orc_net* net, const uint32_t* src_triples, uint32_t n_src_seg,
                         const uint32_t* tgt_triples, uint32_t n_tgt_seg,
                         const uint32_t* pair_s, const uint32_t* pair_t, uint64_t n,
                         int w_kind, double w_mean, double w_sd,
                         int d_kind, double d_mean, double d_sd, double d_lo,
                         int32_t alpha, uint32_t* call_id_out)
{
    if (net->prepared) return fail(net, ORC_ESTATE, "connect after prepare");
    orc_call c;
    int st = init_call(net, &c, src_triples, n_src_seg, tgt_triples, n_tgt_seg, R_ASSIGNED, n, 0.0, 1, 1,
                       w_kind, w_mean, w_sd, d_kind, d_mean, d_sd, d_lo, alpha);
    if (st != ORC_OK) return st;
    if (n > 0 && pair_s && pair_t) {
        c.pair_s = (uint32_t*)malloc(n * sizeof(uint32_t));
        c.pair_t = (uint32_t*)malloc(n * sizeof(uint32_t));
        memcpy(c.pair_s, pair_s, n * sizeof(uint32_t));
        memcpy(c.pair_t, pair_t, n * sizeof(uint32_t));
    }
    return add_call(net, &c, call_id_out);
}

/* ------------------------------------------------------------------------ */
/* Prepare                                                                   */
/* ------------------------------------------------------------------------ */
static int cmp_i32(const void* a, const void* b)
{
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* sorted unique, in place; returns new length */
static uint64_t sort_unique_i32(int32_t* v, uint64_t n)
{
    if (n == 0) return 0;
    qsort(v, n, sizeof(int32_t), cmp_i32);
    uint64_t m = 1;
    for (uint64_t i = 1; i < n; i++)
        if (v[i] != v[m - 1]) v[m++] = v[i];
    return m;
}

/* growable int32 list */
typedef struct { int32_t* v; uint64_t n, cap; } ilist;

static void ilist_push(ilist* l, int32_t x)
{
    if (l->n == l->cap) {
        l->cap = l->cap ? 2 * l->cap : 16;
        l->v = (int32_t*)realloc(l->v, l->cap * sizeof(int32_t));
    }
    l->v[l->n++] = x;
}

/* sort key of the source-major order: (source', target, generation index) */
static const int32_t* g_sort_src;
static const uint32_t* g_sort_tgt;
static int cmp_conn(const void* a, const void* b)
{
    uint64_t i = *(const uint64_t*)a, j = *(const uint64_t*)b;
    if (g_sort_src[i] != g_sort_src[j]) return g_sort_src[i] < g_sort_src[j] ? -1 : 1;
    if (g_sort_tgt[i] != g_sort_tgt[j]) return g_sort_tgt[i] < g_sort_tgt[j] ? -1 : 1;
    return i < j ? -1 : (i > j ? 1 : 0);
}

/* Source-major order (Methods, GPU memory levels: connections sorted with
 * the source as first key, so a source's connections are one block given by
 * its first index and count).  Reading: the second key is the target, ties
 * keep generation order.  row_ptr[r] = first connection of source r,
 * row_ptr[n_rows] = n (counts, then a running sum). */
void orc_sort_csr(uint64_t n, const int32_t* src, const uint32_t* tgt, const uint16_t* delay,
                  const float* weight, uint64_t n_rows,
                  int32_t* o_src, int32_t* o_tgt, uint16_t* o_delay, float* o_weight, uint64_t* row_ptr)
{
    uint64_t* order = (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t));
    for (uint64_t i = 0; i < n; i++) order[i] = i;
    g_sort_src = src; g_sort_tgt = tgt;
    qsort(order, n, sizeof(uint64_t), cmp_conn);
    for (uint64_t i = 0; i < n; i++) {
        uint64_t j = order[i];
        o_src[i] = src[j];
        o_tgt[i] = (int32_t)tgt[j];
        o_delay[i] = delay[j];
        o_weight[i] = weight[j];
    }
    free(order);
    for (uint64_t r = 0; r <= n_rows; r++) row_ptr[r] = 0;
    for (uint64_t i = 0; i < n; i++) row_ptr[(uint64_t)o_src[i] + 1] += 1;
    for (uint64_t r = 0; r < n_rows; r++) row_ptr[r + 1] += row_ptr[r];
}

/* The per-source lists of the send tables.  Given sorted lists
 * list_val[list_off[k] .. list_off[k+1]) for k = 0..n_lists-1 (the S_tau of
 * the point-to-point layout, or H_{alpha,P_local} of the collective one), for
 * each local neuron s = 0..M-1 collect the pairs (k, i) with list k holding s
 * at position i, k ascending (the appends to T/P and to G/Q).  out_ptr has
 * M+1 entries; returns the number of pairs. */
uint64_t orc_transpose_lists(uint32_t n_lists, const uint64_t* list_off, const int32_t* list_val,
                             uint32_t M, uint64_t* out_ptr, uint32_t* out_list, uint32_t* out_pos)
{
    uint64_t count = 0;
    for (uint32_t s = 0; s < M; s++) {
        out_ptr[s] = count;
        for (uint32_t k = 0; k < n_lists; k++) {
            for (uint64_t i = list_off[k]; i < list_off[k + 1]; i++)
                if (list_val[i] == (int32_t)s) {
                    out_list[count] = k;
                    out_pos[count] = (uint32_t)(i - list_off[k]);
                    count++;
                    break;
                }
        }
    }
    out_ptr[M] = count;
    return count;
}

typedef struct { ilist* lists; uint32_t P_local; const orc_call* c; } mark_ctx;

/* point-to-point regeneration: keep the sources that live on P_local */
static void emit_mark_local_source(void* vctx, uint64_t src_ord, uint32_t tgt_local, uint64_t e)
{
    (void)tgt_local; (void)e;
    mark_ctx* ctx = (mark_ctx*)vctx;
    uint32_t h, l;
    set_at(&ctx->c->S, src_ord, &h, &l);
    if (h == ctx->P_local) ilist_push(ctx->lists, (int32_t)l);
}

static int32_t max_alpha(const orc_net* net)
{
    int32_t a = -1;
    for (uint32_t c = 0; c < net->ncalls; c++)
        if (net->calls[c].alpha > a) a = net->calls[c].alpha;
    return a;
}

/* (R, L) map of one (alpha+1, sigma): R sorted ascending except while a
 * call appends to it. */
typedef struct { int32_t* r; int32_t* l; uint64_t n, cap; } omap;

static void omap_append(omap* m, int32_t r, int32_t l)
{
    if (m->n == m->cap) {
        m->cap = m->cap ? 2 * m->cap : 16;
        m->r = (int32_t*)realloc(m->r, m->cap * sizeof(int32_t));
        m->l = (int32_t*)realloc(m->l, m->cap * sizeof(int32_t));
    }
    m->r[m->n] = r; m->l[m->n] = l; m->n++;
}

/* position of r among the first n (sorted) entries, or -1: binary search */
static int64_t omap_find(const omap* m, uint64_t n, int32_t r)
{
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        uint64_t mid = (lo + hi) / 2;
        if (m->r[mid] < r) lo = mid + 1; else hi = mid;
    }
    return (lo < n && m->r[lo] == r) ? (int64_t)lo : -1;
}

static void omap_sort(omap* m)   /* insertion sort by R (carries L) */
{
    for (uint64_t i = 1; i < m->n; i++) {
        int32_t r = m->r[i], l = m->l[i];
        uint64_t j = i;
        while (j > 0 && m->r[j - 1] > r) { m->r[j] = m->r[j - 1]; m->l[j] = m->l[j - 1]; j--; }
        m->r[j] = r; m->l[j] = l;
    }
}

/* Number of neurons of a set that live on `host`. */
static uint64_t set_count_on(const orc_set* s, uint32_t host)
{
    uint64_t n = 0;
    for (uint32_t i = 0; i < s->nseg; i++)
        if (s->seg[i].host == host) n += s->seg[i].n;
    return n;
}

/* Does call c map only its used sources onto host tau (flagging), or all the
 * sources passed to it?  Policy 0 always flags, policy 2 never does.  Policy 1
 * is the threshold heuristic of the point-to-point creation subsection:
 * flag when the rule draws its source indices at random and the estimated
 * number of new connections on tau divided by the number of sources is below
 * xi.  Estimates (reading): fixed in-degree K N_t, fixed total number
 * N N_t / (all targets of the call), pairwise Bernoulli p N_s N_t, assigned
 * nodes the number of its pairs with the target on tau, with N_t the call's
 * targets on tau and N_s all its sources; one-to-one and fixed out-degree use
 * every source and are never flagged. */
static int flag_sources(const orc_net* net, const orc_call* c, uint32_t tau)
{
    if (net->img_sources == 0) return 1;
    if (net->img_sources == 2) return 0;
    const double n_s = (double)c->S.total, n_t = (double)set_count_on(&c->T, tau);
    if (n_s == 0.0) return 1;
    double est;
    switch (c->rule) {
    case R_INDEGREE: est = (double)c->n * n_t; break;
    case R_TOTAL: est = (double)c->n * n_t / (double)c->T.total; break;
    case R_BERNOULLI: est = c->p * n_s * n_t; break;
    case R_ASSIGNED: {     /* the pairs whose target is on tau */
        uint32_t h, l;
        est = 0.0;
        for (uint64_t i = 0; i < c->n; i++) {
            set_at(&c->T, c->pair_t[i], &h, &l);
            if (h == tau) est += 1.0;
        }
        break;
    }
    default: return 0;
    }
    return est / n_s < net->xi;
}

int orc_prepare(orc_net* net)
{
    if (net->prepared) return fail(net, ORC_ESTATE, "prepare called twice");
    const uint32_t P = net->P, PL = net->P_local;
    const uint32_t M_local = net->M[PL];
    const uint64_t N = net->n_gen;

    net->call_off = (uint64_t*)malloc((net->ncalls + 1) * sizeof(uint64_t));
    for (uint32_t c = 0; c < net->ncalls; c++) net->call_off[c] = net->calls[c].gen_begin;
    net->call_off[net->ncalls] = N;

    /* --- image maps (R, L) per (alpha+1, sigma), built call by call in the
     * order of the point-to-point creation subsection: for every call with
     * targets on P_local and every source host sigma != P_local (ascending),
     * flag b over the call's sources on sigma (the used ones, or all of them
     * when the call is not flagged, see flag_sources), compact to u~ / s~,
     * sort by s~, search each s~_j in R: found -> its L; not found ->
     * append (s~_j, M), M += 1; re-sort the map by R.  M starts at the
     * number of local neurons (reading: all Create calls precede the remote
     * connections).  With the canonical numbering the finished maps are
     * renumbered after the local neurons in (alpha+1, sigma, s) order. --- */
    net->n_a = (uint32_t)(max_alpha(net) + 2);
    const uint32_t n_a = net->n_a;
    omap* maps = (omap*)calloc((size_t)n_a * P, sizeof(omap));
    uint32_t* conn_host = (uint32_t*)malloc((N ? N : 1) * sizeof(uint32_t));
    uint32_t* conn_local = (uint32_t*)malloc((N ? N : 1) * sizeof(uint32_t));
    uint32_t* conn_a = (uint32_t*)malloc((N ? N : 1) * sizeof(uint32_t));
    uint32_t M_next = M_local;
    for (uint32_t c = 0; c < net->ncalls; c++) {
        const orc_call* cl = &net->calls[c];
        for (uint64_t i = cl->gen_begin; i < cl->gen_begin + cl->gen_count; i++) {
            set_at(&cl->S, net->g_src[i], &conn_host[i], &conn_local[i]);
            conn_a[i] = (uint32_t)(cl->alpha + 1);
        }
        if (set_count_on(&cl->T, PL) == 0 || cl->S.total == 0) continue;
        const int flagged = flag_sources(net, cl, PL);
        unsigned char* b = (unsigned char*)calloc(cl->S.total, 1);
        if (flagged) {
            for (uint64_t i = cl->gen_begin; i < cl->gen_begin + cl->gen_count; i++) b[net->g_src[i]] = 1;
        } else {
            memset(b, 1, cl->S.total);
        }
        const uint32_t a = (uint32_t)(cl->alpha + 1);
        for (uint32_t sigma = 0; sigma < P; sigma++) {
            if (sigma == PL) continue;
            ilist st = {0};   /* s~ : flagged sources on sigma */
            uint64_t ord = 0;
            for (uint32_t k = 0; k < cl->S.nseg; k++) {
                const orc_seg* sg = &cl->S.seg[k];
                for (uint32_t x = 0; x < sg->n; x++, ord++)
                    if (sg->host == sigma && b[ord]) ilist_push(&st, (int32_t)(sg->first + x));
            }
            if (st.n == 0) { free(st.v); continue; }
            qsort(st.v, st.n, sizeof(int32_t), cmp_i32);
            omap* m = &maps[(size_t)a * P + sigma];
            const uint64_t n_before = m->n;
            for (uint64_t j = 0; j < st.n; j++) {
                if (omap_find(m, n_before, st.v[j]) >= 0) continue;   /* already has an image */
                omap_append(m, st.v[j], (int32_t)M_next);
                M_next++;
            }
            omap_sort(m);
            free(st.v);
        }
        free(b);
    }
    net->r_off = (uint64_t*)calloc((size_t)n_a * P + 1, sizeof(uint64_t));
    net->img_base = (int64_t*)calloc((size_t)n_a * P, sizeof(int64_t));
    uint64_t total = 0;
    for (uint64_t k = 0; k < (uint64_t)n_a * P; k++) {
        net->r_off[k] = total;
        total += maps[k].n;
    }
    net->r_off[(size_t)n_a * P] = total;
    net->n_img = total;
    net->r_val = (int32_t*)malloc((total ? total : 1) * sizeof(int32_t));
    net->l_val = (int32_t*)malloc((total ? total : 1) * sizeof(int32_t));
    for (uint64_t k = 0; k < (uint64_t)n_a * P; k++) {
        for (uint64_t i = 0; i < maps[k].n; i++) {
            net->r_val[net->r_off[k] + i] = maps[k].r[i];
            if (net->numbering == 0) maps[k].l[i] = (int32_t)(M_local + net->r_off[k] + i);
            net->l_val[net->r_off[k] + i] = maps[k].l[i];
        }
        net->img_base[k] = net->numbering == 0 ? (int64_t)M_local + (int64_t)net->r_off[k] : -1;
    }

    /* --- remap: source' = local id, or the image index L of the source --- */
    int32_t* src2 = (int32_t*)malloc((N ? N : 1) * sizeof(int32_t));
    for (uint64_t i = 0; i < N; i++) {
        if (conn_host[i] == PL) {
            src2[i] = (int32_t)conn_local[i];
        } else {
            const omap* m = &maps[(size_t)conn_a[i] * P + conn_host[i]];
            int64_t pos = omap_find(m, m->n, (int32_t)conn_local[i]);
            src2[i] = pos >= 0 ? m->l[pos] : -1;   /* -1 is not reached: every remote source has an image */
        }
    }
    for (uint64_t k = 0; k < (uint64_t)n_a * P; k++) { free(maps[k].r); free(maps[k].l); }
    free(maps);
    free(conn_host); free(conn_local); free(conn_a);

    /* --- source-major sort and first-index array --- */
    net->n_rows = (uint64_t)M_local + net->n_img;
    net->s_src = (int32_t*)malloc((N ? N : 1) * sizeof(int32_t));
    net->s_tgt = (int32_t*)malloc((N ? N : 1) * sizeof(int32_t));
    net->s_delay = (uint16_t*)malloc((N ? N : 1) * sizeof(uint16_t));
    net->s_weight = (float*)malloc((N ? N : 1) * sizeof(float));
    net->row_ptr = (uint64_t*)calloc(net->n_rows + 1, sizeof(uint64_t));
    orc_sort_csr(N, src2, net->g_tgt, net->g_delay, net->g_weight, net->n_rows,
                 net->s_src, net->s_tgt, net->s_delay, net->s_weight, net->row_ptr);
    free(src2);

    /* --- point-to-point send lists.  For each target host tau and every
     * alpha = -1 call with targets on tau: when the call is flagged for tau,
     * regenerate its draws for tau's share (the source-process variant of
     * RemoteConnect) and keep the sources on P_local; otherwise take all its
     * sources on P_local.  S_tau = their sorted unique local ids.  Then T/P: for each local s,
     * the (tau, position of s in S_tau), tau ascending. --- */
    ilist* S = (ilist*)calloc(P, sizeof(ilist));
    for (uint32_t tau = 0; tau < P; tau++) {
        if (tau == PL) continue;
        for (uint32_t c = 0; c < net->ncalls; c++) {
            const orc_call* cl = &net->calls[c];
            if (cl->alpha != -1 || set_count_on(&cl->T, tau) == 0) continue;
            if (flag_sources(net, cl, tau)) {
                mark_ctx mctx = { &S[tau], PL, cl };
                sink_t sink = { emit_mark_local_source, &mctx };
                gen_call(net, cl, tau, 0, UINT64_MAX, sink);
            } else {   /* not flagged: every source of the call on P_local */
                for (uint32_t k = 0; k < cl->S.nseg; k++)
                    if (cl->S.seg[k].host == PL)
                        for (uint32_t x = 0; x < cl->S.seg[k].n; x++) ilist_push(&S[tau], (int32_t)(cl->S.seg[k].first + x));
            }
        }
        S[tau].n = sort_unique_i32(S[tau].v, S[tau].n);
    }
    net->S_off = (uint64_t*)calloc(P + 1, sizeof(uint64_t));
    uint64_t s_total = 0;
    for (uint32_t tau = 0; tau < P; tau++) { net->S_off[tau] = s_total; s_total += S[tau].n; }
    net->S_off[P] = s_total;
    net->S_val = (int32_t*)malloc((s_total ? s_total : 1) * sizeof(int32_t));
    for (uint32_t tau = 0; tau < P; tau++)
        if (S[tau].n) memcpy(net->S_val + net->S_off[tau], S[tau].v, S[tau].n * sizeof(int32_t));
    net->TP_ptr = (uint64_t*)calloc((uint64_t)M_local + 1, sizeof(uint64_t));
    net->T_val = (uint32_t*)malloc((s_total ? s_total : 1) * sizeof(uint32_t));
    net->P_val = (uint32_t*)malloc((s_total ? s_total : 1) * sizeof(uint32_t));
    orc_transpose_lists(P, net->S_off, net->S_val, M_local, net->TP_ptr, net->T_val, net->P_val);
    for (uint32_t tau = 0; tau < P; tau++) free(S[tau].v);
    free(S);

    /* --- collective arrays.  For each group alpha >= 0 and host sigma:
     * H = sorted union of the sources on sigma passed to group-alpha calls
     * (all passed sources, used or not); I aligned with H holds the image
     * index on P_local or -1 (also -1 for sigma = P_local, whose sources are
     * real local neurons); G/Q list, for each local s, the groups whose H on
     * P_local contains s and the position there, groups ascending. --- */
    int32_t amax = max_alpha(net);
    net->n_groups = 0;
    net->groups = (int32_t*)malloc((amax >= 0 ? (size_t)amax + 1 : 1) * sizeof(int32_t));
    for (int32_t a = 0; a <= amax; a++) {
        int present = 0;
        for (uint32_t c = 0; c < net->ncalls; c++)
            if (net->calls[c].alpha == a) { present = 1; break; }
        if (present) net->groups[net->n_groups++] = a;
    }
    const uint32_t G = net->n_groups;
    ilist* H = (ilist*)calloc((size_t)G * P + 1, sizeof(ilist));
    for (uint32_t g = 0; g < G; g++) {
        for (uint32_t c = 0; c < net->ncalls; c++) {
            const orc_call* cl = &net->calls[c];
            if (cl->alpha != net->groups[g]) continue;
            for (uint32_t k = 0; k < cl->S.nseg; k++) {
                const orc_seg* sg = &cl->S.seg[k];
                for (uint32_t x = 0; x < sg->n; x++) ilist_push(&H[(size_t)g * P + sg->host], (int32_t)(sg->first + x));
            }
        }
        for (uint32_t sigma = 0; sigma < P; sigma++) {
            ilist* hl = &H[(size_t)g * P + sigma];
            hl->n = sort_unique_i32(hl->v, hl->n);
        }
    }
    net->H_off = (uint64_t*)calloc((size_t)G * P + 1, sizeof(uint64_t));
    uint64_t h_total = 0;
    for (uint64_t k = 0; k < (uint64_t)G * P; k++) { net->H_off[k] = h_total; h_total += H[k].n; }
    net->H_off[(size_t)G * P] = h_total;
    net->H_val = (int32_t*)malloc((h_total ? h_total : 1) * sizeof(int32_t));
    net->I_val = (int32_t*)malloc((h_total ? h_total : 1) * sizeof(int32_t));
    for (uint32_t g = 0; g < G; g++) {
        uint32_t a = (uint32_t)(net->groups[g] + 1);
        for (uint32_t sigma = 0; sigma < P; sigma++) {
            uint64_t k = (uint64_t)g * P + sigma;
            size_t rk = (size_t)a * P + sigma;
            uint64_t rn = net->r_off[rk + 1] - net->r_off[rk];
            const int32_t* R = net->r_val + net->r_off[rk];
            for (uint64_t j = 0; j < H[k].n; j++) {
                int32_t hv = H[k].v[j];
                net->H_val[net->H_off[k] + j] = hv;
                int32_t img = -1;
                if (sigma != PL) {
                    for (uint64_t i = 0; i < rn; i++)
                        if (R[i] == hv) { img = net->l_val[net->r_off[rk] + i]; break; }
                }
                net->I_val[net->H_off[k] + j] = img;
            }
        }
    }
    /* lists H_{alpha, P_local} for the groups in ascending order */
    uint64_t* hl_off = (uint64_t*)calloc((size_t)G + 1, sizeof(uint64_t));
    for (uint32_t g = 0; g < G; g++) hl_off[g + 1] = hl_off[g] + H[(size_t)g * P + PL].n;
    int32_t* hl_val = (int32_t*)malloc((hl_off[G] ? hl_off[G] : 1) * sizeof(int32_t));
    for (uint32_t g = 0; g < G; g++)
        if (H[(size_t)g * P + PL].n)
            memcpy(hl_val + hl_off[g], H[(size_t)g * P + PL].v, H[(size_t)g * P + PL].n * sizeof(int32_t));
    net->GQ_ptr = (uint64_t*)calloc((uint64_t)M_local + 1, sizeof(uint64_t));
    net->G_val = (int32_t*)malloc((hl_off[G] ? hl_off[G] : 1) * sizeof(int32_t));
    net->Q_val = (uint32_t*)malloc((hl_off[G] ? hl_off[G] : 1) * sizeof(uint32_t));
    uint64_t gq = orc_transpose_lists(G, hl_off, hl_val, M_local, net->GQ_ptr, (uint32_t*)net->G_val, net->Q_val);
    for (uint64_t i = 0; i < gq; i++) net->G_val[i] = net->groups[net->G_val[i]];
    free(hl_off); free(hl_val);
    for (uint64_t k = 0; k < (uint64_t)G * P; k++) free(H[k].v);
    free(H);

    /* first index and count of the image rows, as the memory level keeps
     * them: levels 0 and 1 both (in host memory in the library), level 3 the
     * count beside the first-index array; level 2 derives the count from it */
    const uint64_t n_img_rows = net->n_rows - M_local;
    if (net->mem_level == 0 || net->mem_level == 1) {
        net->img_first = (uint64_t*)malloc((n_img_rows ? n_img_rows : 1) * sizeof(uint64_t));
        for (uint64_t i = 0; i < n_img_rows; i++) net->img_first[i] = net->row_ptr[M_local + i];
    }
    if (net->mem_level == 0 || net->mem_level == 1 || net->mem_level == 3) {
        net->img_count = (uint32_t*)malloc((n_img_rows ? n_img_rows : 1) * sizeof(uint32_t));
        for (uint64_t i = 0; i < n_img_rows; i++)
            net->img_count[i] = (uint32_t)(net->row_ptr[M_local + i + 1] - net->row_ptr[M_local + i]);
    }

    net->prepared = 1;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Spike exchange with the built maps (Appendix E: packet and delivery        */
/* figures; collective subsection for groups).                               */
/* ------------------------------------------------------------------------ */

/* Packets of one time step from per-source lists (ptr over M sources;
 * dest[j], where[j]): spike k of source spikes[k] (multiplicity mult[k], or 1
 * when mult is NULL) appends (where[j], mult) to packet dest[j] for each of its
 * list entries j; packets keep the spike order.  off has n_dest + 1 entries.
 * Returns the number of packet entries, or -1 for a spike id >= M or a
 * capacity below the count (nothing written then). */
int64_t orc_packets_from_lists(const uint64_t* ptr, const uint32_t* dest, const uint32_t* where, uint32_t M,
                               uint32_t n_dest, const uint32_t* spikes, const uint32_t* mult, uint64_t n,
                               uint64_t* off, uint32_t* pos_out, uint32_t* mult_out, uint64_t cap)
{
    uint64_t total = 0;
    for (uint64_t k = 0; k < n; k++) {
        if (spikes[k] >= M) return -1;
        total += ptr[spikes[k] + 1] - ptr[spikes[k]];
    }
    if (total > cap) return -1;
    for (uint32_t d = 0; d <= n_dest; d++) off[d] = 0;
    for (uint64_t k = 0; k < n; k++)          /* packet sizes */
        for (uint64_t j = ptr[spikes[k]]; j < ptr[spikes[k] + 1]; j++) off[dest[j] + 1]++;
    for (uint32_t d = 0; d < n_dest; d++) off[d + 1] += off[d];
    uint64_t* fill = (uint64_t*)malloc(((size_t)n_dest + 1) * sizeof(uint64_t));
    for (uint32_t d = 0; d <= n_dest; d++) fill[d] = off[d];
    for (uint64_t k = 0; k < n; k++)          /* append in spike order */
        for (uint64_t j = ptr[spikes[k]]; j < ptr[spikes[k] + 1]; j++) {
            uint64_t o = fill[dest[j]]++;
            pos_out[o] = where[j];
            mult_out[o] = mult ? mult[k] : 1u;
        }
    free(fill);
    return (int64_t)total;
}

/* Packets of the local host: kind 0 point-to-point (destinations = hosts,
 * lists T/P), kind 1 collective (destinations = the groups in ascending
 * order, lists G/Q with the group replaced by its rank). */
int64_t orc_spike_packets(const orc_net* net, int kind, const uint32_t* spikes, const uint32_t* mult, uint64_t n,
                          uint64_t* off, uint32_t* pos_out, uint32_t* mult_out, uint64_t cap)
{
    if (!net->prepared) return -1;
    const uint32_t M = net->M[net->P_local];
    if (kind == 0)
        return orc_packets_from_lists(net->TP_ptr, net->T_val, net->P_val, M, net->P, spikes, mult, n,
                                      off, pos_out, mult_out, cap);
    if (kind != 1) return -1;
    const uint64_t m = net->GQ_ptr[M];
    uint32_t* grank = (uint32_t*)malloc((m ? m : 1) * sizeof(uint32_t));
    for (uint64_t j = 0; j < m; j++) {
        uint32_t g = 0;
        while (g < net->n_groups && net->groups[g] != net->G_val[j]) g++;
        grank[j] = g;
    }
    int64_t r = orc_packets_from_lists(net->GQ_ptr, grank, net->Q_val, M, net->n_groups, spikes, mult, n,
                                       off, pos_out, mult_out, cap);
    free(grank);
    return r;
}

/* Delivery from explicit maps: entry e names a received position pos[e] in
 * map key[e] (map_off over n_maps maps, map_img the local image index or -1
 * for none); the image's outgoing connections are its row of the sorted
 * arrays.  Per entry: image (or -1), row [begin, end).  Events, for entries
 * in order and their connections in row order: (target, delay,
 * weight * multiplicity in fp32).  Returns the event count, -1 for an entry
 * outside its map, -2 when the events exceed ev_cap (the per-entry outputs
 * are written, the events are not). */
int64_t orc_deliver_from_maps(const uint64_t* map_off, const int32_t* map_img, uint64_t n_maps,
                              const uint64_t* row_ptr, const int32_t* tgt, const uint16_t* delay, const float* weight,
                              const uint32_t* key, const uint32_t* pos, const uint32_t* mult, uint64_t n,
                              int32_t* image, uint64_t* rb, uint64_t* re,
                              int32_t* ev_tgt, uint16_t* ev_delay, float* ev_weight, uint64_t ev_cap)
{
    uint64_t total = 0;
    for (uint64_t e = 0; e < n; e++) {
        if (key[e] >= n_maps || pos[e] >= map_off[key[e] + 1] - map_off[key[e]]) return -1;
        int32_t img = map_img[map_off[key[e]] + pos[e]];
        image[e] = img;
        rb[e] = img >= 0 ? row_ptr[img] : 0;
        re[e] = img >= 0 ? row_ptr[img + 1] : 0;
        total += re[e] - rb[e];
    }
    if (!ev_tgt) return (int64_t)total;
    if (total > ev_cap) return -2;
    uint64_t o = 0;
    for (uint64_t e = 0; e < n; e++) {
        const float m = mult ? (float)mult[e] : 1.0f;
        for (uint64_t c = rb[e]; c < re[e]; c++, o++) {
            ev_tgt[o] = tgt[c];
            ev_delay[o] = delay[c];
            ev_weight[o] = weight[c] * m;
        }
    }
    return (int64_t)total;
}

/* Delivery on the local host.  kind 0: entry = (source host sigma, position
 * i in the point-to-point map R_{P_local,sigma}) -> L; kind 1: entry = (group
 * rank g, source host sigma, position j in H_{alpha_g,sigma}) -> I (-1: the
 * source has no image here).  grp is ignored for kind 0. */
int64_t orc_deliver(const orc_net* net, int kind, const uint32_t* grp, const uint32_t* host, const uint32_t* pos,
                    const uint32_t* mult, uint64_t n, int32_t* image, uint64_t* rb, uint64_t* re,
                    int32_t* ev_tgt, uint16_t* ev_delay, float* ev_weight, uint64_t ev_cap)
{
    if (!net->prepared || (kind != 0 && kind != 1)) return -1;
    const uint32_t P = net->P;
    uint32_t* key = (uint32_t*)malloc((n ? n : 1) * sizeof(uint32_t));
    for (uint64_t e = 0; e < n; e++) {
        if (host[e] >= P || (kind == 0 && host[e] == net->P_local) || (kind == 1 && grp[e] >= net->n_groups)) {
            free(key);
            return -1;
        }
        key[e] = kind == 0 ? host[e] : grp[e] * P + host[e];   /* map (alpha+1 = 0, sigma) / (g, sigma) */
    }
    int64_t r = kind == 0
        ? orc_deliver_from_maps(net->r_off, net->l_val, P, net->row_ptr, net->s_tgt,
                                net->s_delay, net->s_weight, key, pos, mult, n, image, rb, re,
                                ev_tgt, ev_delay, ev_weight, ev_cap)
        : orc_deliver_from_maps(net->H_off, net->I_val, (uint64_t)net->n_groups * P, net->row_ptr, net->s_tgt,
                                net->s_delay, net->s_weight, key, pos, mult, n, image, rb, re,
                                ev_tgt, ev_delay, ev_weight, ev_cap);
    free(key);
    return r;
}

/* ------------------------------------------------------------------------ */
/* Access                                                                    */
/* ------------------------------------------------------------------------ */
enum {
    A_GEN_SRC = 0, A_GEN_TGT = 1, A_GEN_DELAY = 2, A_GEN_WEIGHT = 3, A_GEN_E = 4, A_CALL_OFF = 5,
    A_SRC = 10, A_TGT = 11, A_DELAY = 12, A_WEIGHT = 13, A_ROW_PTR = 14, A_IMG_FIRST = 15, A_IMG_COUNT = 16,
    A_R_OFF = 20, A_R_VAL = 21, A_IMG_BASE = 22, A_L_VAL = 23,
    A_S_OFF = 30, A_S_VAL = 31, A_TP_PTR = 32, A_T_VAL = 33, A_P_VAL = 34,
    A_GROUPS = 40, A_H_OFF = 41, A_H_VAL = 42, A_I_VAL = 43, A_GQ_PTR = 44, A_G_VAL = 45, A_Q_VAL = 46
};

/* element count of an array, or -1 if not available (yet) */
int64_t orc_len(const orc_net* net, int which)
{
    const uint32_t PL = net->P_local;
    switch (which) {
    case A_GEN_SRC: case A_GEN_TGT: case A_GEN_DELAY: case A_GEN_WEIGHT: case A_GEN_E: return (int64_t)net->n_gen;
    default: break;
    }
    if (!net->prepared) return -1;
    switch (which) {
    case A_CALL_OFF: return net->ncalls + 1;
    case A_SRC: case A_TGT: case A_DELAY: case A_WEIGHT: return (int64_t)net->n_gen;
    case A_ROW_PTR:     /* levels 0 and 1 keep the image rows apart */
        return (net->mem_level == 0 || net->mem_level == 1) ? (int64_t)net->M[PL] + 1 : (int64_t)net->n_rows + 1;
    case A_IMG_FIRST: return net->img_first ? (int64_t)(net->n_rows - net->M[PL]) : -1;
    case A_IMG_COUNT: return net->img_count ? (int64_t)(net->n_rows - net->M[PL]) : -1;
    case A_R_OFF: return (int64_t)net->n_a * net->P + 1;
    case A_R_VAL: case A_L_VAL: return (int64_t)net->n_img;
    case A_IMG_BASE: return (int64_t)net->n_a * net->P;
    case A_S_OFF: return net->P + 1;
    case A_S_VAL: case A_T_VAL: case A_P_VAL: return (int64_t)net->S_off[net->P];
    case A_TP_PTR: case A_GQ_PTR: return (int64_t)net->M[PL] + 1;
    case A_GROUPS: return net->n_groups;
    case A_H_OFF: return (int64_t)net->n_groups * net->P + 1;
    case A_H_VAL: case A_I_VAL: return (int64_t)net->H_off[(size_t)net->n_groups * net->P];
    case A_G_VAL: case A_Q_VAL: return (int64_t)net->GQ_ptr[net->M[PL]];
    }
    return -1;
}

static const void* array_ptr(const orc_net* net, int which, size_t* elem)
{
    switch (which) {
    case A_GEN_SRC: *elem = 4; return net->g_src;
    case A_GEN_TGT: *elem = 4; return net->g_tgt;
    case A_GEN_DELAY: *elem = 2; return net->g_delay;
    case A_GEN_WEIGHT: *elem = 4; return net->g_weight;
    case A_GEN_E: *elem = 8; return net->g_e;
    case A_CALL_OFF: *elem = 8; return net->call_off;
    case A_SRC: *elem = 4; return net->s_src;
    case A_TGT: *elem = 4; return net->s_tgt;
    case A_DELAY: *elem = 2; return net->s_delay;
    case A_WEIGHT: *elem = 4; return net->s_weight;
    case A_ROW_PTR: *elem = 8; return net->row_ptr;
    case A_IMG_FIRST: *elem = 8; return net->img_first;
    case A_IMG_COUNT: *elem = 4; return net->img_count;
    case A_R_OFF: *elem = 8; return net->r_off;
    case A_R_VAL: *elem = 4; return net->r_val;
    case A_IMG_BASE: *elem = 8; return net->img_base;
    case A_L_VAL: *elem = 4; return net->l_val;
    case A_S_OFF: *elem = 8; return net->S_off;
    case A_S_VAL: *elem = 4; return net->S_val;
    case A_TP_PTR: *elem = 8; return net->TP_ptr;
    case A_T_VAL: *elem = 4; return net->T_val;
    case A_P_VAL: *elem = 4; return net->P_val;
    case A_GROUPS: *elem = 4; return net->groups;
    case A_H_OFF: *elem = 8; return net->H_off;
    case A_H_VAL: *elem = 4; return net->H_val;
    case A_I_VAL: *elem = 4; return net->I_val;
    case A_GQ_PTR: *elem = 8; return net->GQ_ptr;
    case A_G_VAL: *elem = 4; return net->G_val;
    case A_Q_VAL: *elem = 4; return net->Q_val;
    }
    *elem = 0;
    return NULL;
}

int orc_copy(const orc_net* net, int which, void* dst, uint64_t cap_bytes)
{
    int64_t n = orc_len(net, which);
    size_t elem;
    const void* src = array_ptr(net, which, &elem);
    if (n < 0 || elem == 0) return ORC_ESTATE;
    if ((uint64_t)n * elem > cap_bytes) return ORC_EINVAL;
    if (n > 0) memcpy(dst, src, (size_t)n * elem);
    return ORC_OK;
}

uint32_t orc_neurons(const orc_net* net, uint32_t host) { return host < net->P ? net->M[host] : 0; }

/* Sampled checks at full size: the draws of one call restricted to a range
 * of its primary ordinal, on a given host's share, written to caller arrays
 * (source position, target local id, element index, weight, delay).
 * Returns the number written, or -1 if cap is too small. */
typedef struct {
    const orc_net* net; const orc_call* c;
    uint32_t* src; uint32_t* tgt; uint64_t* e; float* w; uint16_t* d; uint64_t n, cap; int overflow;
} range_ctx;

static void emit_range(void* vctx, uint64_t src_ord, uint32_t tgt_local, uint64_t e)
{
    range_ctx* ctx = (range_ctx*)vctx;
    if (ctx->n >= ctx->cap) { ctx->overflow = 1; return; }
    const orc_call* c = ctx->c;
    uint32_t w[4] = { 0, 0, 0, 0 };
    if (c->w.kind != D_CONST || c->d.kind != D_CONST)
        draw_block(ctx->net->seed, c->id, e, PURPOSE_SYN, w);
    uint64_t i = ctx->n++;
    ctx->src[i] = (uint32_t)src_ord; ctx->tgt[i] = tgt_local; ctx->e[i] = e;
    ctx->w[i] = (c->w.kind == D_CONST) ? c->w_const : orc_normal_weight(w[0], w[1], c->w.mean, c->w.sd);
    if (c->d.kind == D_CONST) ctx->d[i] = c->d_const;
    else {
        uint32_t count = 0;
        for (uint32_t k = 0; k < c->dtab_len; k++) if (w[2] >= c->dtab[k]) count++;
        ctx->d[i] = (uint16_t)(c->d_klo + count);
    }
}

int64_t orc_call_range(const orc_net* net, uint32_t call_id, uint32_t host, uint64_t lo, uint64_t hi,
                       uint32_t* src, uint32_t* tgt, uint64_t* e, float* w, uint16_t* d, uint64_t cap)
{
    if (call_id >= net->ncalls) return -1;
    range_ctx ctx = { net, &net->calls[call_id], src, tgt, e, w, d, 0, cap, 0 };
    sink_t sink = { emit_range, &ctx };
    gen_call(net, &net->calls[call_id], host, lo, hi, sink);
    return ctx.overflow ? -1 : (int64_t)ctx.n;
}

/* One element of a call, computed on its own, for the rules whose elements
 * do not depend on each other: fixed in-degree and out-degree with
 * multapses (element e = unit * K + j), fixed total number with autapses and
 * multapses (candidate e), pairwise Bernoulli (pair e) and one-to-one (e).
 * Returns 1 and the element's values when the element is a connection, 0
 * when it is not (a pair that does not connect, a skipped autapse), -1 for
 * a rule or flag combination where elements depend on each other. */
int orc_call_element(const orc_net* net, uint32_t call_id, uint64_t e, uint32_t* src_ord, uint32_t* tgt_host,
                     uint32_t* tgt_local, float* weight, uint16_t* delay)
{
    if (call_id >= net->ncalls) return -1;
    const orc_call* c = &net->calls[call_id];
    const uint64_t ns = c->S.total, nt = c->T.total;
    uint64_t s = 0, t = 0;
    uint32_t h, l, h2, l2;
    switch (c->rule) {
    case R_INDEGREE: {
        if (!c->multapses || c->n == 0) return -1;
        t = e / c->n;
        if (t >= nt) return -1;
        set_at(&c->T, t, &h2, &l2);
        int64_t self_pos = c->autapses ? -1 : set_pos(&c->S, h2, l2);
        uint64_t pick;
        draw_k(net, c, e, 1, ns, self_pos, &pick);     /* one draw with element index e */
        s = pick;
        break;
    }
    case R_OUTDEGREE: {
        if (!c->multapses || c->n == 0) return -1;
        s = e / c->n;
        if (s >= ns) return -1;
        set_at(&c->S, s, &h, &l);
        int64_t self_pos = c->autapses ? -1 : set_pos(&c->T, h, l);
        uint64_t pick;
        draw_k(net, c, e, 1, nt, self_pos, &pick);
        t = pick;
        set_at(&c->T, t, &h2, &l2);
        break;
    }
    case R_TOTAL: {
        if (!c->autapses || !c->multapses) return -1;
        uint32_t w[4];
        draw_block(net->seed, c->id, e, PURPOSE_IDX, w);
        s = orc_uniform_index(w[0], w[1], ns);
        t = orc_uniform_index(w[2], w[3], nt);
        set_at(&c->T, t, &h2, &l2);
        break;
    }
    case R_BERNOULLI: {
        if (ns == 0) return -1;
        t = e / ns;
        s = e % ns;
        if (t >= nt) return -1;
        uint32_t w[4];
        draw_block(net->seed, c->id, e / 4, PURPOSE_BERN, w);
        if ((uint64_t)w[e % 4] >= bern_threshold(c->p)) return 0;
        set_at(&c->T, t, &h2, &l2);
        if (!c->autapses) {
            set_at(&c->S, s, &h, &l);
            if (h == h2 && l == l2) return 0;
        }
        break;
    }
    case R_ASSIGNED: {
        if (e >= c->n) return -1;
        s = c->pair_s[e];
        t = c->pair_t[e];
        set_at(&c->T, t, &h2, &l2);
        break;
    }
    case R_ONE_TO_ONE: {
        if (e >= nt) return -1;
        s = t = e;
        set_at(&c->T, t, &h2, &l2);
        if (!c->autapses) {
            set_at(&c->S, s, &h, &l);
            if (h == h2 && l == l2) return 0;
        }
        break;
    }
    default:
        return -1;
    }
    uint32_t w[4] = { 0, 0, 0, 0 };
    if (c->w.kind != D_CONST || c->d.kind != D_CONST) draw_block(net->seed, c->id, e, PURPOSE_SYN, w);
    *weight = (c->w.kind == D_CONST) ? c->w_const : orc_normal_weight(w[0], w[1], c->w.mean, c->w.sd);
    if (c->d.kind == D_CONST) {
        *delay = c->d_const;
    } else {
        uint32_t count = 0;
        for (uint32_t k = 0; k < c->dtab_len; k++) if (w[2] >= c->dtab[k]) count++;
        *delay = (uint16_t)(c->d_klo + count);
    }
    *src_ord = (uint32_t)s;
    *tgt_host = h2;
    *tgt_local = l2;
    return 1;
}

/* A connect that only records the call (no local generation): lets sampled
 * checks at full size describe a huge network without building it. */
int orc_declare(orc_net* net, const uint32_t* src_triples, uint32_t n_src_seg,
                const uint32_t* tgt_triples, uint32_t n_tgt_seg,
                int rule, uint64_t n, double p, int autapses, int multapses,
                int w_kind, double w_mean, double w_sd,
                int d_kind, double d_mean, double d_sd, double d_lo,
                int32_t alpha, uint32_t* call_id_out)
{
    if (net->prepared) return fail(net, ORC_ESTATE, "declare after prepare");
    if (rule == R_ASSIGNED) return fail(net, ORC_EINVAL, "assigned nodes cannot be declared");
    orc_call c;
    memset(&c, 0, sizeof c);
    c.id = net->ncalls;
    c.rule = rule; c.n = n; c.p = p; c.autapses = autapses != 0; c.multapses = multapses != 0;
    c.alpha = alpha;
    c.w.kind = w_kind; c.w.mean = w_mean; c.w.sd = w_sd;
    c.d.kind = d_kind; c.d.mean = d_mean; c.d.sd = d_sd; c.d.lo = d_lo;
    int st = copy_set(net, src_triples, n_src_seg, &c.S);
    if (st == ORC_OK) st = copy_set(net, tgt_triples, n_tgt_seg, &c.T);
    if (st == ORC_OK) st = validate_and_fill(net, &c);
    if (st != ORC_OK) { free(c.S.seg); free(c.T.seg); free(c.dtab); return st; }
    if (net->ncalls == net->capcalls) {
        net->capcalls = net->capcalls ? 2 * net->capcalls : 16;
        net->calls = (orc_call*)realloc(net->calls, net->capcalls * sizeof(orc_call));
    }
    c.gen_begin = net->n_gen; c.gen_count = 0;
    net->calls[net->ncalls++] = c;
    *call_id_out = c.id;
    return ORC_OK;
}

/* Number of connections of one call on one host's share whose primary
 * ordinal lies in [lo, hi): the same walk of the rule's draws as the
 * generation (gen_call), counting each accepted connection instead of
 * drawing its synapse values.  Used to decide admission against a resident
 * budget without generating.  -1 for an unknown call. */
typedef struct { uint64_t n; } count_ctx;

static void emit_count(void* vctx, uint64_t src_ord, uint32_t tgt_local, uint64_t e)
{
    (void)src_ord; (void)tgt_local; (void)e;
    ((count_ctx*)vctx)->n++;
}

int64_t orc_call_count(const orc_net* net, uint32_t call_id, uint32_t host, uint64_t lo, uint64_t hi)
{
    if (call_id >= net->ncalls) return -1;
    count_ctx ctx = { 0 };
    sink_t sink = { emit_count, &ctx };
    gen_call(net, &net->calls[call_id], host, lo, hi, sink);
    return (int64_t)ctx.n;
}
