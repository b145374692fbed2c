/*
 * snnc.h -- C ABI of the MI355X (gfx950) spiking-network construction library.
 *
 * The library builds, on one GPU, the share of a distributed spiking-network
 * connectivity that belongs to one virtual host P_local of P hosts, following
 * the construction method of Golosio, Tiddia, Villamar et al., "Scalable
 * Construction of Spiking Neural Networks using up to thousands of GPUs"
 * (arXiv:2512.09502), section Methods ("Remote connections" and its
 * subsections).  Other hosts exist only as ranges of neuron ids: each host
 * runs the same script and builds its own share without communication
 * (Results, first subsection; Methods, point-to-point creation subsection).
 *
 * Calls follow the paper's problem statement: Create(population, n),
 * Connect / RemoteConnect(sigma, s, tau, t, p, C, D, alpha) (Methods,
 * "Creation of the remote connection structures for point-to-point MPI
 * communication"), and the simulation-preparation phase (Methods,
 * "Simulation phases and optimization").  Connect and RemoteConnect are one
 * call here: every node set lists its segments with their host.
 *
 * Conventions
 *  - Every function returns an snnc_status; nothing is thrown across the ABI.
 *    snnc_last_error() gives a message for the last failure of a context.
 *    A failed call leaves the context as it was before the call.
 *  - Device memory: the context owns every device buffer.  It allocates
 *    through the caller's snnc_allocator (for instance a framework's caching
 *    allocator) or, if none is given, stream-ordered from a memory pool the
 *    library keeps per device.  Pointers handed out by
 *    snnc_get_array() are device pointers, valid until the next mutating call
 *    (connect, prepare, destroy) on the context.
 *  - Streams: all device work of a context is ordered on the HIP stream given
 *    at init (0 = the null stream).  Calls return once the work is enqueued,
 *    except where a host-visible result (a count, a status) requires a
 *    synchronisation; snnc_sync() waits for the stream.
 *  - Determinism: the call id of a Connect is its ordinal among the accepted
 *    connect calls of the context.  Every random number is a Philox4x32-10
 *    block keyed by (seed, call id) with counter (element index e, purpose),
 *    so every host regenerates any draw of any call exactly.  Results do not
 *    depend on launch shapes.
 */
#ifndef SNNC_H
#define SNNC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct snnc_ctx snnc_ctx;

typedef enum {
    SNNC_OK = 0,
    SNNC_EINVAL = -1,       /* invalid argument or connection spec              */
    SNNC_ENOMEM = -2,       /* the allocator returned NULL                      */
    SNNC_EBUDGET = -3,      /* the device-memory budget would be exceeded       */
    SNNC_ESTATE = -4,       /* call not allowed in the current state            */
    SNNC_EUNSUPPORTED = -5, /* valid request outside what this library builds   */
    SNNC_EDEVICE = -6       /* a HIP runtime call or a kernel reported an error */
} snnc_status;

/* A range of local neuron ids [first, first + n) on virtual host `host`. */
typedef struct {
    uint32_t host, first, n;
} snnc_segment;

/* A node set: the concatenation of its segments.  The position of a neuron in
 * the set (its ordinal) is its rank in that concatenation.  A set lists each
 * neuron at most once.  Host memory, read during the call only. */
typedef struct {
    const snnc_segment* seg;
    uint32_t n_seg;
} snnc_nodeset;

/* Connection rules (the paper's rule dictionary C, rules as defined in the
 * connectivity-concepts reference it cites). */
typedef enum {
    SNNC_ONE_TO_ONE = 0,          /* s_i -> t_i, n_s == n_t                         */
    SNNC_FIXED_INDEGREE = 1,      /* n sources drawn for every target               */
    SNNC_FIXED_OUTDEGREE = 2,     /* n targets drawn for every source               */
    SNNC_FIXED_TOTAL_NUMBER = 3,  /* n connections drawn over all pairs             */
    SNNC_PAIRWISE_BERNOULLI = 4,  /* every pair connected with probability p        */
    SNNC_ASSIGNED_NODES = 5       /* explicit (source, target) pairs: only through
                                     snnc_connect_assigned                          */
} snnc_rule_kind;

typedef struct {
    uint32_t kind;            /* snnc_rule_kind                                   */
    uint32_t allow_autapses;  /* 0: no connection from a neuron to itself         */
    uint32_t allow_multapses; /* 0: at most one connection per (source, target)   */
    uint32_t reserved;
    uint64_t n;               /* in-degree, out-degree or total number            */
    double p;                 /* Bernoulli probability                            */
} snnc_conn_spec;

typedef enum { SNNC_CONST = 0, SNNC_NORMAL = 1 } snnc_dist_kind;

/* CONST uses mean.  NORMAL draws N(mean, sd); for delays the draw is clipped
 * from below at lo (ms) before it is turned into an integer number of steps. */
typedef struct {
    uint32_t kind;
    uint32_t reserved;
    double mean, sd, lo;
} snnc_dist;

/* The synapse dictionary D: weight (stored as fp32) and delay in ms (stored
 * as uint16 time steps of dt, see snnc_delay_table); receptor port p must be
 * 0 (ports are not stored). */
typedef struct {
    snnc_dist weight;
    snnc_dist delay_ms;
    uint32_t port;
    uint32_t reserved;
} snnc_syn_spec;

/* Device-memory callbacks.  alloc returns NULL on failure; the library then
 * returns SNNC_ENOMEM.  `stream` is the context's stream. */
typedef struct {
    void* (*alloc)(size_t bytes, void* stream, void* user);
    void (*free)(void* ptr, void* user);
    void* user;
} snnc_allocator;

/* ---------------------------------------------------------------- lifecycle */

/* Create a context for host P_local of P virtual hosts.  seed keys every
 * Philox stream; dt_ms is the time step that delays are counted in.
 * `alloc` may be NULL (stream-ordered allocation from the library's pool).  budget_bytes > 0 caps the device
 * bytes the context may hold at once (SNNC_EBUDGET beyond).  The current HIP
 * device at the time of the call is the context's device.
 * Errors: SNNC_EINVAL for P == 0, P_local >= P, dt_ms <= 0. */
snnc_status snnc_init(snnc_ctx** out, uint32_t P, uint32_t P_local, uint32_t seed, double dt_ms,
                      const snnc_allocator* alloc, void* hip_stream, uint64_t budget_bytes);

/* Free every device buffer of the context (after waiting for its streams).
 * Buffers the caller's allocator gave go back to it.  The library's own
 * stream-ordered blocks are kept, up to 8 GiB per device, in a per-device
 * cache that later contexts on that device draw exact-size blocks from
 * (and pinned host staging buffers likewise); the rest return to the
 * library's memory pool, which keeps its memory until the process ends. */
snnc_status snnc_destroy(snnc_ctx* ctx);

/* Message of the last failed call on this context ("" if none). */
const char* snnc_last_error(const snnc_ctx* ctx);

/* Wait for all work enqueued by the context. */
snnc_status snnc_sync(snnc_ctx* ctx);

/* ---------------------------------------------------------------- building */

/* Create(population, n): n neurons on `host` get the next free local ids of
 * that host; *out receives the segment.  Every host's context must see the
 * same creates in the same order.  Host-side bookkeeping only.
 * Errors: SNNC_EINVAL (host >= P, more than 2^31-1 neurons on a host),
 * SNNC_ESTATE after snnc_prepare. */
snnc_status snnc_create(snnc_ctx* ctx, uint32_t host, uint32_t n, snnc_segment* out);

/* Connect(src, tgt, rule, syn_spec) with group alpha (-1: point-to-point
 * exchange; >= 0: collective group alpha).  Generates on the GPU, in
 * canonical generation order (element index e ascending), every connection
 * of the call whose target lives on P_local: the source as its ordinal in
 * `src` (the paper's temporary source position), the target as its local id,
 * the delay in steps and the fp32 weight.  *call_id_out gets the call id.
 * Element index and draws per rule:
 *   fixed in-degree K:   e = t_ord * K + j; source ordinal from block IDX(e);
 *                        without multapses Robert Floyd's sampling over the
 *                        K draws of a target, then sorted ascending;
 *                        without autapses the draw skips the target itself;
 *   fixed out-degree K:  mirror image with sources and targets swapped;
 *   fixed total number:  candidate c draws (source, target) from IDX(c) over
 *                        the whole sets; the first n candidates that are valid
 *                        (no autapse if excluded, no repeated pair if
 *                        multapses excluded) are the connections, e = c; with
 *                        targets on several hosts every host evaluates every
 *                        candidate and keeps those whose target it holds;
 *   pairwise Bernoulli:  pairs numbered target-major, q = t_ord * n_s +
 *                        s_ord; pair q connects iff word q % 4 of block
 *                        BERN(q / 4) is below floor(p * 2^32) (every pair
 *                        for p = 1); e = q;
 *   one-to-one:          e = i;
 *   assigned nodes:      see snnc_connect_assigned (snnc_connect rejects it).
 * Synapse values of element e come from block SYN(e) of the same call.
 * Errors: SNNC_EINVAL (bad segment, overlapping segments within a set, rule
 * parameters impossible for the sets, port != 0, delay below one step or
 * beyond 65535 steps, sd < 0), SNNC_EUNSUPPORTED (more than 2^32-1 neurons
 * in a set, total number or degree above 2^32-1, degree above 8192 without
 * multapses),
 * SNNC_ESTATE after prepare, SNNC_ENOMEM / SNNC_EBUDGET, SNNC_EDEVICE. */
snnc_status snnc_connect(snnc_ctx* ctx, const snnc_nodeset* src, const snnc_nodeset* tgt,
                         const snnc_conn_spec* conn, const snnc_syn_spec* syn, int32_t alpha,
                         uint32_t* call_id_out);

/* Connect with the assigned-nodes rule (Methods, distributed fixed in-degree
 * subsection: after the source draws of a target host are sorted by source
 * host and position, each source host's part is connected with a rule that
 * takes the source and target of every connection as given).  Pair i
 * connects source position src_pos[i] of `src` to target position
 * tgt_pos[i] of `tgt` (positions = ordinals in the concatenated segments);
 * element index e = i, synapse values from block SYN(i).  The connection
 * belongs to the share of the target's host, so every host passes the same
 * pairs (as for every Connect).  src_pos, tgt_pos: host arrays of n uint32,
 * read during the call and copied to the device (the library keeps the copy
 * until snnc_destroy, since Prepare regenerates the point-to-point lists from
 * it).  Autapse and multapse flags do not apply.  Under the threshold map
 * policy the estimate is the number of pairs with a target on the host.
 * Errors: SNNC_EINVAL (null arrays with n > 0, a position outside its set,
 * bad segments or synapse spec as snnc_connect), SNNC_ESTATE after prepare,
 * SNNC_ENOMEM / SNNC_EBUDGET, SNNC_EDEVICE.  Per call only: snnc_submit
 * rejects SNNC_ASSIGNED_NODES (SNNC_EINVAL). */
snnc_status snnc_connect_assigned(snnc_ctx* ctx, const snnc_nodeset* src, const snnc_nodeset* tgt,
                                  const uint32_t* src_pos, const uint32_t* tgt_pos, uint64_t n,
                                  const snnc_syn_spec* syn, int32_t alpha, uint32_t* call_id_out);

/* Reserve room for n generated connections (optional; avoids regrowth). */
snnc_status snnc_reserve(snnc_ctx* ctx, uint64_t n_connections);

/* ---------------------------------------------------------------- served construction
 * A construction server keeps the growing network resident in HBM and admits
 * each Connect request against a budget on the resident network: 14 bytes
 * per connection (source, target, delay, weight) plus the request's metadata
 * (16 bytes per segment of each node set, at least one per set, and 4 bytes
 * per delay-table threshold plus a 257-word guide for a normal delay, or 4
 * bytes for a constant one; assigned nodes add 8 bytes per pair; a request
 * with no source or target on P_local has no metadata and no connections).
 * Admission uses the exact connection count of the request on P_local's share
 * (a counting pass where the count depends on the draws), in submission
 * order, so it is deterministic; a rejected request changes nothing and gets
 * no call id.  The budget applies to snnc_connect as well, so per-call and
 * batched construction of the same request stream admit the same requests
 * and build bit-identical networks.  (This is the served form of the paper's
 * dynamic construction, where the maps are kept in blocks allocated as they
 * grow; the budget plays the role of the GPU memory limit that bounds the
 * paper's scaling.) */

/* Set the resident budget in bytes (0 = none).  SNNC_ESTATE after prepare. */
snnc_status snnc_set_resident_budget(snnc_ctx* ctx, uint64_t bytes);

/* Submit a Connect request (arguments as snnc_connect): validate, count,
 * admit and reserve its positions now; generate it at the next snnc_flush.
 * *call_id_out receives its call id.  Errors: as snnc_connect, plus
 * SNNC_EBUDGET when the request does not fit the resident budget.  A request
 * whose smallest possible count already exceeds what the budget has left (a
 * fixed total number with every target on this host keeps exactly N) gets
 * SNNC_EBUDGET without its count being drawn on the device. */
snnc_status snnc_submit(snnc_ctx* ctx, const snnc_nodeset* src, const snnc_nodeset* tgt,
                        const snnc_conn_spec* conn, const snnc_syn_spec* syn, int32_t alpha, uint32_t* call_id_out);

/* Submit n requests at once (array i of each argument is request i): the
 * same as n snnc_submit calls in order -- same admissions, call ids and
 * network -- except that the host waits for the device once for all counts
 * that need it instead of once per such request.  Those counts are queued
 * assuming every earlier request of the batch is admitted (consecutive call
 * ids); a request whose id moves because an earlier one was rejected, or
 * whose fixed-total-number window held too few valid candidates, is counted
 * again at its admission.  status_out[i] receives request i's status
 * (SNNC_OK, SNNC_EBUDGET, or the SNNC_EINVAL / SNNC_EUNSUPPORTED of an
 * invalid request, which then gets no call id) and call_ids_out[i] its call
 * id (UINT32_MAX when not admitted); both are caller arrays of n entries.
 * The call itself returns SNNC_EINVAL for null arrays with n > 0,
 * SNNC_ESTATE after prepare, and SNNC_ENOMEM / SNNC_EDEVICE, after which the
 * requests not yet admitted are dropped. */
snnc_status snnc_submit_many(snnc_ctx* ctx, uint32_t n, const snnc_nodeset* src, const snnc_nodeset* tgt,
                             const snnc_conn_spec* conn, const snnc_syn_spec* syn, const int32_t* alpha,
                             snnc_status* status_out, uint32_t* call_ids_out);

/* Launch every submitted, not yet generated request as one batch: requests
 * whose connections are one per element (fixed in-degree and out-degree with
 * multapses, fixed total number with autapses and multapses, one-to-one
 * without skipped autapses) run in one persistent launch replayed from a
 * captured HIP graph; the others run their own launches.  Returns once the
 * batch is enqueued. */
snnc_status snnc_flush(snnc_ctx* ctx);

/* *done = 1 when the call's connections are generated (its batch has
 * completed on the device, or it was made by snnc_connect), 0 otherwise. */
snnc_status snnc_poll(snnc_ctx* ctx, uint32_t call_id, int32_t* done);

/* Simulation preparation (Methods, point-to-point and collective creation
 * subsections; "GPU memory levels" for the source-major order):
 *  1. image map: for every map index a = alpha + 1 and remote host sigma, R
 *     = sorted unique local ids of the sigma-sources used by local
 *     connections of group-alpha calls; images are numbered after the M_local
 *     local neurons, in (a, sigma, source id) order, L = img_base + position;
 *  2. remap: every connection's source becomes its local id (source on
 *     P_local) or its image index;
 *  3. sort: all connections by (source, target), ties in generation order;
 *  4. first-index array row_ptr over M_local + n_images sources;
 *  5. point-to-point send lists: S_tau = sorted local sources that host tau's
 *     share of the alpha = -1 calls uses (regenerated here, no communication),
 *     and per local source the (tau, position in S_tau) pairs T/P;
 *  6. collective arrays per group alpha: H_{alpha,sigma} = sorted union of the
 *     sigma-sources passed to group-alpha calls, I aligned with H (image index
 *     on P_local or -1; -1 for sigma = P_local), and per local source the
 *     (alpha, position in H_{alpha,P_local}) pairs G/Q.
 * Errors: SNNC_ESTATE if already prepared, SNNC_EUNSUPPORTED if
 * bits(sources) + bits(targets) > 48, SNNC_ENOMEM/EBUDGET, SNNC_EDEVICE. */
snnc_status snnc_prepare(snnc_ctx* ctx);

/* ---------------------------------------------------------------- results */

typedef enum {
    /* generation order (available after connect, until prepare) */
    SNNC_GEN_SRC = 0,      /* uint32 source ordinal in the call's source set  */
    SNNC_GEN_TGT = 1,      /* uint32 target local id                           */
    SNNC_GEN_DELAY = 2,    /* uint16 steps                                     */
    SNNC_GEN_WEIGHT = 3,   /* float                                            */
    SNNC_CALL_OFF = 5,     /* uint64 [n_calls + 1] first generated index/call  */
    /* after prepare */
    SNNC_SRC = 10,         /* int32 source' (local id or image index), sorted  */
    SNNC_TGT = 11,         /* int32 target local id                            */
    SNNC_DELAY = 12,       /* uint16                                           */
    SNNC_WEIGHT = 13,      /* float                                            */
    SNNC_ROW_PTR = 14,     /* uint64 [M_local + n_img + 1]; [M_local + 1] at   */
                           /* GPU memory levels 0 and 1 (image rows apart)     */
    SNNC_IMG_FIRST = 15,   /* uint64 [n_img] first connection of each image    */
                           /* row (levels 0 and 1, host memory)                */
    SNNC_IMG_COUNT = 16,   /* uint32 [n_img] connections of each image row     */
                           /* (levels 0 and 1 host memory, level 3 device)     */
    SNNC_R_OFF = 20,       /* uint64 [n_a * P + 1] offsets of R per (a, sigma) */
    SNNC_R_VAL = 21,       /* int32 remote source ids                          */
    SNNC_IMG_BASE = 22,    /* int64 [n_a * P] first image index per (a, sigma); */
                           /* -1 under SNNC_NUMBER_CALL_ORDER (not contiguous) */
    SNNC_L_VAL = 23,       /* int32 image index L, aligned with R              */
    SNNC_S_OFF = 30,       /* uint64 [P + 1] offsets of S per target host      */
    SNNC_S_VAL = 31,       /* int32 local source ids                           */
    SNNC_TP_PTR = 32,      /* uint64 [M_local + 1]                             */
    SNNC_T_VAL = 33,       /* uint32 target host                               */
    SNNC_P_VAL = 34,       /* uint32 position in S_tau (= in R_{tau,P_local})  */
    SNNC_GROUPS = 40,      /* int32 [n_groups] group ids ascending             */
    SNNC_H_OFF = 41,       /* uint64 [n_groups * P + 1]                        */
    SNNC_H_VAL = 42,       /* int32 source ids                                 */
    SNNC_I_VAL = 43,       /* int32 image index or -1, aligned with H          */
    SNNC_GQ_PTR = 44,      /* uint64 [M_local + 1]                             */
    SNNC_G_VAL = 45,       /* int32 group                                      */
    SNNC_Q_VAL = 46        /* uint32 position in H_{group, P_local}            */
} snnc_array_id;

/* Pointer and element count of an array (count 0 and ptr NULL for an empty
 * array): device memory, except the arrays that GPU memory levels 0 and 1
 * keep in pinned host memory (snnc_array_on_host).  SNNC_ESTATE if the array
 * does not exist in this state. */
snnc_status snnc_get_array(const snnc_ctx* ctx, int32_t id, const void** dev_ptr, uint64_t* count);

/* *on_host = 1 when the array lives in pinned host memory (readable by
 * kernels through the mapping), 0 for device memory.  SNNC_ESTATE as
 * snnc_get_array. */
snnc_status snnc_array_on_host(const snnc_ctx* ctx, int32_t id, int32_t* on_host);

/* Copy an array to dst (host or device memory, hipMemcpyDefault), waiting
 * for completion.  SNNC_EINVAL if cap_bytes is too small. */
snnc_status snnc_copy_array(snnc_ctx* ctx, int32_t id, void* dst, uint64_t cap_bytes);

/* Copy elements [first, first + count) of an array to dst (host or device
 * memory), waiting for completion.  SNNC_EINVAL if the range is outside the
 * array. */
snnc_status snnc_copy_range(snnc_ctx* ctx, int32_t id, uint64_t first, uint64_t count, void* dst);

/* ---------------------------------------------------------------- typed views
 * Views gather the pointers and sizes of the prepared arrays (no copy, no
 * device work).  Pointers are device memory except where a GPU memory level
 * keeps an array in pinned host memory (flagged in the view); they stay
 * valid until snnc_destroy (nothing mutates a prepared network).  Every view
 * call returns SNNC_ESTATE before snnc_prepare. */

/* The sorted connections and their first-index array (Methods, "GPU memory
 * levels": connections stored in blocks sorted by source, with the first
 * index and the number of outgoing connections of every source; Methods,
 * point-to-point creation subsection, for the image indices of remote
 * sources).  src[i] is a local id (< M_local) or an image index (M_local ..
 * M_local + n_images - 1); connections of a source are contiguous, ordered by
 * target, ties in generation order.  Row s is [row_ptr[s], row_ptr[s+1]) for
 * s < n_rows: n_rows = M_local + n_images at levels 2 and 3, M_local at
 * levels 0 and 1, where image row i is [img_first[i], img_first[i] +
 * img_count[i]) (host memory, img_rows_on_host = 1); img_count is also
 * present at level 3 (device).  Absent arrays are NULL. */
typedef struct {
    const int32_t* src;        /* [n] */
    const int32_t* tgt;        /* [n] target local id */
    const uint16_t* delay;     /* [n] steps of dt */
    const float* weight;       /* [n] */
    const uint64_t* row_ptr;   /* [n_rows + 1] */
    const uint64_t* img_first; /* [n_images] or NULL */
    const uint32_t* img_count; /* [n_images] or NULL */
    uint64_t n;
    uint64_t n_rows;
    uint64_t n_images;
    uint32_t M_local;
    int32_t img_rows_on_host;
} snnc_conn_view;

snnc_status snnc_get_connections(const snnc_ctx* ctx, snnc_conn_view* out);

/* The image map of remote host sigma for group alpha (map index alpha + 1;
 * Methods, point-to-point creation subsection: the sorted array of the
 * remote sources of sigma that have an image on this host, and the map of
 * each to its image index; collective subsection for alpha >= 0).  *R gets
 * the n sorted source local ids of sigma, *L (when L is not NULL) their
 * image indices, *img_base the first image index when the images of the map
 * are contiguous (canonical numbering: L[i] = img_base + i) and -1 under
 * call-order numbering.  A map that does not exist (no image, a map index
 * above the network's groups, sigma = P_local) gives n = 0 and NULL
 * pointers.  Pointers are into SNNC_R_VAL / SNNC_L_VAL (host memory at GPU
 * memory levels 0 and 1).  Errors: SNNC_EINVAL for alpha < -1 or sigma >= P,
 * SNNC_ESTATE before prepare. */
snnc_status snnc_get_image_map(const snnc_ctx* ctx, int32_t alpha, uint32_t sigma, const int32_t** R, uint64_t* n,
                               int64_t* img_base, const int32_t** L);

/* The point-to-point send lists (Methods, point-to-point creation
 * subsection, source-process side; Eq. of the map alignment: S_{tau,P_local}
 * equals the map R_{tau,P_local} that host tau builds; simulation
 * preparation: the per-source lists of target hosts and positions).  S_tau =
 * s_val[s_off[tau] .. s_off[tau+1]), sorted local ids; for local source s,
 * entries tp_ptr[s] .. tp_ptr[s+1] give (t_val = target host tau, ascending,
 * p_val = position of s in S_tau).  Device memory. */
typedef struct {
    const uint64_t* s_off;   /* [P + 1] */
    const int32_t* s_val;    /* [n_s] */
    const uint64_t* tp_ptr;  /* [M_local + 1] */
    const uint32_t* t_val;   /* [n_tp] */
    const uint32_t* p_val;   /* [n_tp] */
    uint64_t n_s, n_tp;
    uint32_t P, M_local;
} snnc_p2p_view;

snnc_status snnc_get_p2p_send(const snnc_ctx* ctx, snnc_p2p_view* out);

/* The collective arrays of group alpha >= 0 (Methods, collective
 * communication subsection): H_{alpha,sigma} = h_val[h_off[sigma] ..
 * h_off[sigma+1]) for sigma < P (offsets index the whole h_val / i_val
 * arrays: h_off points at this group's P + 1 entries of SNNC_H_OFF), the
 * sorted union of the sigma-sources passed to the group's calls; i_val
 * aligned with h_val: the image index of that source on this host or -1
 * (always -1 for sigma = P_local); and, over all groups, for local source s
 * the entries gq_ptr[s] .. gq_ptr[s+1] of (g_val = group id, q_val =
 * position of s in H_{group,P_local}).  rank = the group's rank in
 * SNNC_GROUPS; on_host = 1 when H and I live in pinned host memory (GPU
 * memory levels 0 and 1).  Errors: SNNC_EINVAL for alpha < 0 or a group
 * without calls, SNNC_ESTATE before prepare. */
typedef struct {
    const uint64_t* h_off;   /* [P + 1] */
    const int32_t* h_val;    /* [n_h], all groups */
    const int32_t* i_val;    /* [n_h], all groups */
    const uint64_t* gq_ptr;  /* [M_local + 1] */
    const int32_t* g_val;    /* [n_gq] */
    const uint32_t* q_val;   /* [n_gq] */
    uint64_t n_h, n_gq;
    int32_t alpha;
    uint32_t rank, P, M_local;
    int32_t on_host;
} snnc_coll_view;

snnc_status snnc_get_collective(const snnc_ctx* ctx, int32_t alpha, snnc_coll_view* out);

/* Copy a whole array into caller host memory of `bytes` (at least the
 * array's size; snnc_get_array gives its element count), waiting for
 * completion; the caller owns dst.  Errors: SNNC_EINVAL (dst NULL with bytes
 * > 0, or bytes too small), SNNC_ESTATE as snnc_get_array. */
snnc_status snnc_copy_to_host(const snnc_ctx* ctx, int32_t id, void* dst, uint64_t bytes);

/* Counters of the context. */
typedef struct {
    uint64_t n_connections;   /* local-share connections generated       */
    uint64_t n_images;        /* image neurons (after prepare)            */
    uint32_t n_calls;
    uint32_t M_local;
    uint64_t bytes_live;      /* device bytes held now                    */
    uint64_t bytes_peak;      /* high-water mark                          */
    uint32_t sort_passes;     /* radix passes of the last prepare         */
    uint32_t key_bits;        /* bits(sources) + bits(targets)            */
    double ms_connect;        /* stream time from the first connect call to the start of prepare (events) */
    double ms_prepare;        /* GPU time of prepare                      */
} snnc_stats_t;

snnc_status snnc_stats(snnc_ctx* ctx, snnc_stats_t* out);

/* Per-kernel GPU timing with HIP events on the context stream.  enable = 1:
 * every kernel launch is bracketed by an event pair; 2: only the radix-sort
 * passes (the brackets cost host time per launch); 0: off.  snnc_kernel_times
 * reports, per kernel name, the launch count and the summed milliseconds
 * (names as NUL-terminated strings of at most 47 characters).  SNNC_EINVAL
 * for other values of enable. */
snnc_status snnc_set_timing(snnc_ctx* ctx, int enable);
snnc_status snnc_kernel_times(snnc_ctx* ctx, uint32_t cap, char (*names)[48], uint64_t* launches,
                              double* ms, uint32_t* n_out);

/* Map policy (Methods, point-to-point creation subsection; used for the
 * collective maps alike), set before snnc_prepare.
 * numbering: SNNC_NUMBER_CANONICAL numbers all images after the local neurons
 *   in (alpha+1, sigma, s) order; SNNC_NUMBER_CALL_ORDER is the paper's
 *   incremental numbering: calls in order, each call's new images in
 *   (sigma, s) order, the counter starting at M_local.
 * image_sources: SNNC_IMAGES_USED gives images only to remote sources used by
 *   a local connection (flagging on every call); SNNC_IMAGES_ALL to every
 *   source passed to a call with targets on this host (no flagging, the
 *   paper's GPU memory levels >= 1); SNNC_IMAGES_THRESHOLD decides per call
 *   and target host: flag when the rule draws sources at random (fixed
 *   in-degree, fixed total number, pairwise Bernoulli) and the estimated
 *   connections on that host per source, K N_t / N_s, N / N_s or p N_t, is
 *   below xi; fixed out-degree and one-to-one calls are never flagged.
 * The point-to-point send lists S follow the same decision on the source
 * host, so S_{tau,sigma} stays equal to R_{tau,sigma}.  Default: CANONICAL,
 * USED, xi = 1.  Errors: SNNC_EINVAL for unknown values or xi < 0 / not
 * finite, SNNC_ESTATE after snnc_prepare. */
/* GPU memory level 0 .. 3 (Methods, GPU memory levels subsection), set before
 * snnc_prepare.  Levels 0 and 1 keep the maps of the remote sources to their
 * images (R_OFF, R_VAL, IMG_BASE, L_VAL; H_OFF, H_VAL, I_VAL) and the first
 * index and count of every image row (IMG_FIRST, IMG_COUNT) in pinned host
 * memory; the device keeps ROW_PTR over the local rows only.  Level 2 keeps
 * everything in device memory and a row's count is the difference of two
 * ROW_PTR entries; level 3 adds IMG_COUNT in device memory.  Level 0 gives
 * images to the used remote sources only, levels 1 to 3 to every source
 * passed to a call with targets on this host: the level sets the map
 * policy's image sources (SNNC_IMAGES_USED, SNNC_IMAGES_ALL), which a later
 * snnc_set_map_policy overrides.  Without a level the placement is level 2's
 * and the image sources are the map policy's.  Errors: SNNC_EINVAL outside
 * 0 .. 3, SNNC_ESTATE after snnc_prepare. */
snnc_status snnc_set_memory_level(snnc_ctx* ctx, int32_t level);

typedef enum { SNNC_NUMBER_CANONICAL = 0, SNNC_NUMBER_CALL_ORDER = 1 } snnc_numbering;
typedef enum { SNNC_IMAGES_USED = 0, SNNC_IMAGES_THRESHOLD = 1, SNNC_IMAGES_ALL = 2 } snnc_image_sources;
snnc_status snnc_set_map_policy(snnc_ctx* ctx, int32_t numbering, int32_t image_sources, double xi);

/* Tuning knobs of the context, by name.  "sort_variant": tile shape of the
 * radix-sort passes, 0 .. 13, as threads x keys per thread: 0 = 512x16 with
 * keys and payloads staged through LDS one after the other (70 KB, two
 * workgroups per compute unit; default), 1 = 256x8, 2 = 512x8, 3 = 512x16,
 * 4 = 256x16, 5 = 256x12, 6 = 1024x8, and staged in two phases like 0:
 * 7 = 1024x8, 8 = 512x8, 9 = 512x12, 10 = 256x16, 11 = 512x11, 12 = 1024x16,
 * 13 = 768x12.  SNNC_EINVAL for an unknown key or value. */
snnc_status snnc_tune(snnc_ctx* ctx, const char* key, int64_t value);
/* "sort_mode": 0 = single-pass onesweep passes (decoupled look-back), 1 =
 * reduce-then-scan passes (per-tile digit counts, one scan, scatter).
 * Further keys: "fuse_batches" (0/1, default 1), "fused_wgs_per_cu"
 * (workgroups per compute unit of the persistent batch launch, 1 .. 64) and
 * "map_path" (0: automatic, 1: number images before the sort even under the
 * default map policy, the path the other policies take) and "digit_bits"
 * (0: 9-bit digits, 512 buckets, when they save a pass and the tile has at
 * least 512 threads; 8 or 9: forced where the tile allows), "number_variant"
 * (tile shape of the image-numbering pass after the sort, 0 .. 11; default 10 =
 * 1024 threads x 10 items with the payload loaded before the look-back) and
 * "mark_in_lds" (1, default: regeneration for the point-to-point lists marks
 * its bit row in LDS when the row has at most 2^19 neurons; 0: a global
 * atomic per draw) and "floyd_wave_max" (0 .. 8192, default 1024: Floyd's
 * sampling of a unit runs in a one-wave workgroup when the degree rounded up
 * to a power of two is at most this, else in 256 threads up to 2048 and in
 * 1024 threads above) and "total_hash_max" (0 .. 2^32: fixed
 * total number without multapses finds each pair's first candidate by
 * hashing for candidate windows up to this size -- a two-bit-per-slot filter
 * of at least 16 slots per candidate settles the candidates alone in their
 * slot, an exact table the rest; 23 - 45 transient bytes per candidate --
 * and by sorting the pair keys above it (25 bytes per candidate); default
 * 2^28) and "total_small_max" (0 .. 2^15, default 8192: windows up to this
 * size run the first occurrences, the valid counts and their scan in one
 * launch of one workgroup instead of six launches) and "bern_masks" (1, default: the counting pass of
 * pairwise Bernoulli keeps each item's 4-bit pair mask for the writing pass;
 * 0: the writing pass draws them again) and "gen_blocks" (1, default where
 * the device supports virtual memory management: the generation-order arrays
 * live in fixed-size blocks of 2^26 connections mapped as calls and admitted
 * requests need them, kept mapped for the next context on the device after
 * Prepare; 0: arrays grown by doubling; set before the first connection,
 * SNNC_EUNSUPPORTED for 1 without support).  Every setting gives the same
 * arrays. */

/* Autotuner of the source-major sort: times every pass algorithm and tile
 * shape (sort_mode x sort_variant) on n synthetic keys with `bits` sorted
 * bits (1 .. 48), on the context's device, and sets the fastest on the
 * context.  Results are cached per (floor(log2 n), bits) for the process and
 * used by every later sort of that size class on any context whose sort
 * settings were not set with snnc_tune; a cached size class returns at once
 * with *ms_out = -1.  Allocates scratch of about 24 n bytes.
 * Errors: SNNC_EINVAL, SNNC_ENOMEM, SNNC_EDEVICE. */
snnc_status snnc_autotune_sort(snnc_ctx* ctx, uint64_t n, uint32_t bits, int32_t* mode_out, int32_t* variant_out,
                               float* ms_out);

/* Autotuner of the persistent batch launch of snnc_flush: times the launch at
 * 1, 2, 4, 8, 16 and 32 workgroups per compute unit on a synthetic batch of
 * 48 fusable requests (fixed in-degree and out-degree with multapses, total
 * number with autapses and multapses, one-to-one; sizes spread over three
 * decades; about n connections) built in scratch contexts on this context's
 * device, allocator and stream, and sets the fastest on the context.  The
 * choice is cached for the device for the process: a later call returns at
 * once with *ms_out = -1.  The grid changes no result.  Allocates about
 * 2 x 14 n bytes while it runs.  Errors: SNNC_EINVAL (n = 0, null outputs),
 * SNNC_ESTATE after prepare, SNNC_ENOMEM, SNNC_EDEVICE. */
snnc_status snnc_autotune_fused(snnc_ctx* ctx, uint64_t n, int32_t* wgs_out, float* ms_out);

/* ---------------------------------------------------------- spike exchange */

/* Spike packets of one time step on this host (Appendix E, packet figure;
 * collective subsection).  kind 0 (point-to-point): spike k of local neuron
 * spikes[k] appends (P_{s,j}, mult[k]) to the packet of target host T_{s,j}
 * for each of its (T, P) pairs; kind 1 (collective): appends (Q_{s,j},
 * mult[k]) to the packet of group G_{s,j}, groups numbered by their rank in
 * SNNC_GROUPS.  Packets keep the spike order.  All pointers are the caller's
 * device memory: spikes, mult (NULL: multiplicity 1) [n]; off [n_dest + 1],
 * n_dest = P (kind 0) or the number of groups (kind 1), packet d is
 * [off[d], off[d+1]); pos_out, mult_out [cap].  *n_out receives the number
 * of entries; when it exceeds cap nothing is written and SNNC_EINVAL is
 * returned.  Runs on the context stream and waits for completion.
 * Errors: SNNC_ESTATE before snnc_prepare; SNNC_EINVAL for an unknown kind,
 * a spike id >= M_local or a small cap. */
snnc_status snnc_spike_packets(snnc_ctx* ctx, int32_t kind, const uint32_t* spikes, const uint32_t* mult,
                               uint64_t n, uint64_t* off, uint32_t* pos_out, uint32_t* mult_out, uint64_t cap,
                               uint64_t* n_out);

/* Delivery of received packet entries on this host (Appendix E, delivery
 * figure).  kind 0: entry e = (source host host[e] != P_local, position
 * pos[e] in the point-to-point map R_{P_local,host[e]}) -> its image L; kind
 * 1: entry e = (group rank grp[e], source host host[e], position pos[e] in
 * H_{group,host}) -> its image I, or -1 when the source has no image here.
 * Per entry (caller device arrays of n): image[e] and the image's row
 * [row_begin[e], row_end[e]) in the sorted connection arrays (empty for -1).
 * Events (skipped when ev_tgt is NULL): for the entries in order and their
 * connections in row order, (target, delay steps, weight x multiplicity in
 * fp32) into ev_tgt, ev_delay, ev_weight of ev_cap; mult NULL means 1.
 * *n_events receives the number of events.  Runs on the context stream and
 * waits for completion.  Errors: SNNC_ESTATE before snnc_prepare;
 * SNNC_EINVAL for an unknown kind, an entry outside its map, or more events
 * than ev_cap (per-entry outputs written, events not). */
snnc_status snnc_deliver(snnc_ctx* ctx, int32_t kind, const uint32_t* grp, const uint32_t* host,
                         const uint32_t* pos, const uint32_t* mult, uint64_t n, int32_t* image,
                         uint64_t* row_begin, uint64_t* row_end, int32_t* ev_tgt, uint16_t* ev_delay,
                         float* ev_weight, uint64_t ev_cap, uint64_t* n_events);

/* ---------------------------------------------------------------- helpers */

/* The source-major sort of Prepare on its own: stable LSD radix sort of n
 * (key, payload) pairs in device memory by key bits [bit_lo, bit_hi) (ties
 * keep their input order), on the context stream, with the context's sort
 * variant.  keys_tmp/vals_tmp are device scratch of the same sizes.  On
 * return *result_in_tmp says whether the sorted pairs are in (keys, vals)
 * (0) or in (keys_tmp, vals_tmp) (1).  Errors: SNNC_EINVAL for bad bit
 * ranges or null pointers, SNNC_EDEVICE if a device wait exceeded its bound. */
snnc_status snnc_sort_pairs(snnc_ctx* ctx, uint64_t* keys, uint32_t* vals, uint64_t* keys_tmp, uint32_t* vals_tmp,
                            uint64_t n, uint32_t bit_lo, uint32_t bit_hi, int32_t* result_in_tmp);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * snnc_sort_pairs (same arguments, same result) without any allocation.  The
 * digit histograms, tile counters, status word and look-back table live in
 * one static device array of 16 MiB per GPU owned by the library (set up by
 * the first snnc_init on that GPU and held until the process ends); the
 * caller passes keys, vals and the keys_tmp/vals_tmp ping-pong buffers as
 * for snnc_sort_pairs.  Limit: the look-back table (tiles x digit buckets x
 * 8 B, tiles of the context's sort variant, 8192 pairs by default) must fit
 * 16 MiB - 64.25 KiB: about 33 million pairs with 9-bit digits and 67 million
 * with 8-bit digits at the default tile; larger n returns SNNC_EINVAL before
 * any device work.  Every call on a GPU shares that GPU's array and keeps its
 * contents between calls (the library clears what must start at zero);
 * calls are serialised by a host lock and each waits for its sort, so calls
 * from several contexts or threads do not overlap on the array.  No timing
 * brackets are recorded.  Errors: as snnc_sort_pairs, SNNC_ESTATE if the
 * device's scratch was not set up (no snnc_init on it). */
snnc_status snnc_sort_pairs_noalloc(snnc_ctx* ctx, uint64_t* keys, uint32_t* vals, uint64_t* keys_tmp,
                                    uint32_t* vals_tmp, uint64_t n, uint32_t bit_lo, uint32_t bit_hi,
                                    int32_t* result_in_tmp);

/* The delay-step table of a NORMAL(mean, sd) delay clipped at lo (ms) for
 * time step dt (ms): k_lo = round(lo / dt) and thresholds
 * t_k = ceil(Phi(((k + 1/2) dt - mean) / sd) 2^32) for k = k_lo, k_lo+1, ...
 * while below 2^32; a 32-bit uniform word w maps to k_lo + #{k : w >= t_k}.
 * Host computation.  *len_out = number of thresholds.
 * Errors: SNNC_EINVAL if lo < dt, sd <= 0 or the steps would exceed 65535
 * or cap entries. */
snnc_status snnc_delay_table(double mean, double sd, double lo, double dt, uint32_t* table,
                             uint64_t cap, uint32_t* k_lo_out, uint64_t* len_out);

/* Device check of the random stream: out[4 i .. 4 i + 3] = Philox4x32-10
 * block for key (seed, call_id) and counter (e_begin + i, purpose) for
 * i < n.  `out` is device memory of 4 n uint32; runs on the context stream. */
snnc_status snnc_philox_blocks(snnc_ctx* ctx, uint32_t seed, uint32_t call_id, uint64_t e_begin,
                               uint32_t purpose, uint64_t n, uint32_t* out);

#ifdef __cplusplus
}
#endif
#endif /* SNNC_H */
