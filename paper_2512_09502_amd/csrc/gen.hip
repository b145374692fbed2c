// Connection generation on the GPU: one thread per element (or per Philox
// block for Bernoulli), coalesced structure-of-arrays stores, per-thread
// Philox counters.  Rules with a data-dependent count run a counting pass,
// a scan of the per-tile counts and a writing pass that compacts in element
// order with a workgroup scan.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "device_common.h"
#include "internal.h"

namespace snnc {

namespace {

constexpr int NT = 256;          // threads per workgroup
constexpr int IPT = 4;           // items per thread
constexpr uint64_t TILE = NT * IPT;
constexpr uint64_t MAX_TILES_PER_LAUNCH = 1u << 22;
constexpr uint32_t BERN_WGS_PER_CU = 16;   // grid cap of the Bernoulli counting and marking passes

enum Mode { DIRECT = 0, COUNT = 1, WRITE = 2, MARK = 3 };

struct Res {
    uint32_t src;   // source ordinal
    uint32_t tgt;   // target local id
    uint64_t e;     // element index
};

// ------------------------------------------------------------------ sinks
struct WriteSink {
    uint32_t* src;
    uint32_t* tgt;
    uint16_t* delay;
    float* weight;
    uint64_t base;
    SynD syn;
    uint32_t seed, call;
    __device__ __forceinline__ void put(uint64_t pos, const Res& r) const {
        float w;
        uint16_t d;
        syn_values(syn, seed, call, r.e, w, d);
        const uint64_t i = base + pos;
        src[i] = r.src;
        tgt[i] = r.tgt;
        delay[i] = d;
        weight[i] = w;
    }
    __device__ __forceinline__ void mark(const Res&) const {}
};

// Source and target only, for Floyd's sampling (its synapse values are filled
// afterwards by k_syn_fill: the sampling kernel then needs far fewer registers
// than with the Box-Muller draw inline, and more of its waves fit a CU).
struct IdSink {
    uint32_t* src;
    uint32_t* tgt;
    uint64_t base;
    __device__ __forceinline__ void put(uint64_t pos, const Res& r) const {
        src[base + pos] = r.src;
        tgt[base + pos] = r.tgt;
    }
    __device__ __forceinline__ void mark(const Res&) const {}
};

// Point-to-point regeneration: set the bit of every source that lives on
// `host` (one bit row over that host's neurons).
struct MarkSink {
    const SegD* S;
    uint32_t nS;
    uint32_t host;
    uint32_t* bits;
    uint32_t words;   // words of the row: (neurons on `host` + 31) / 32
    __device__ __forceinline__ void mark(const Res& r) const {
        uint32_t h, l;
        set_lookup(S, nS, r.src, h, l);
        if (h != host) return;
        // most draws hit sources already marked: a plain read skips their atomics
        // (a stale read only costs a redundant atomic)
        const uint32_t m = 1u << (l & 31);
        if (!(bits[l >> 5] & m)) atomicOr(bits + (l >> 5), m);
    }
    __device__ __forceinline__ void put(uint64_t, const Res& r) const { mark(r); }
};

__device__ __forceinline__ uint32_t find_chunk(const TChunk* ch, uint32_t nch, uint64_t g) {
    uint32_t a = 0, b = nch;
    while (b - a > 1) {
        const uint32_t m = (a + b) >> 1;
        if (ch[m].out_begin <= g) a = m; else b = m;
    }
    return a;
}

// A call's run table.  Up to CH_INLINE runs (a call over one source and one
// target segment has one) travel inline with the kernel's arguments, so the
// call needs no upload; longer tables live in device memory.
constexpr uint32_t CH_INLINE = 4;

struct ChunkTab {
    const TChunk* d;            // device table when n > CH_INLINE, else null
    uint32_t n;
    TChunk in[CH_INLINE];
    // the run holding element g (the last run starting at or before g)
    __device__ __forceinline__ TChunk at(uint64_t g) const {
        if (n <= CH_INLINE) {
            TChunk c = in[0];
#pragma unroll
            for (uint32_t k = 1; k < CH_INLINE; ++k)
                if (k < n && in[k].out_begin <= g) c = in[k];
            return c;
        }
        return d[find_chunk(d, n, g)];
    }
};

// ------------------------------------------------------------------ rules
// Fixed in-degree with multapses: element e = t_ord K + j draws its source
// ordinal from IDX(e) over the n_s candidates (n_s - 1 with the target itself
// skipped when autapses are excluded).
struct InDegree {
    static constexpr int R = 1;
    ChunkTab ch;
    uint32_t K;
    FastDiv fk;
    uint32_t n_s;
    uint32_t seed, call;
    __device__ __forceinline__ int eval(uint64_t g, Res* r) const {
        const TChunk c = ch.at(g);
        const uint32_t rel = (uint32_t)(g - c.out_begin);
        const uint32_t t_rel = fastdiv(rel, fk);
        const uint32_t j = rel - t_rel * K;
        const uint64_t t_ord = c.t_ord + t_rel;
        const uint64_t e = t_ord * K + j;
        const bool skip = c.self_base >= 0;
        const uint4 b = draw(seed, call, e, PURPOSE_IDX);
        uint32_t s = uniform_index(b.x, b.y, n_s - (skip ? 1u : 0u));
        if (skip && s >= (uint64_t)c.self_base + t_rel) ++s;
        r[0] = Res{s, c.local_first + t_rel, e};
        return 1;
    }
};

// Fixed out-degree with multapses: element e = s_ord K + j draws a target
// ordinal; the connection belongs to the share of the target's host.
struct OutDegree {
    static constexpr int R = 1;
    ChunkTab ch;        // runs of source ordinals (local_first unused)
    uint32_t K;
    FastDiv fk;
    uint32_t n_t;
    const SegD* T;
    uint32_t nT;
    uint32_t host;
    uint32_t seed, call;
    __device__ __forceinline__ int eval(uint64_t g, Res* r) const {
        const TChunk c = ch.at(g);
        const uint32_t rel = (uint32_t)(g - c.out_begin);
        const uint32_t s_rel = fastdiv(rel, fk);
        const uint32_t j = rel - s_rel * K;
        const uint64_t s_ord = c.t_ord + s_rel;
        const uint64_t e = s_ord * K + j;
        const bool skip = c.self_base >= 0;
        const uint4 b = draw(seed, call, e, PURPOSE_IDX);
        uint32_t t = uniform_index(b.x, b.y, n_t - (skip ? 1u : 0u));
        if (skip && t >= (uint64_t)c.self_base + s_rel) ++t;
        uint32_t h, l;
        set_lookup(T, nT, t, h, l);
        if (h != host) return 0;
        r[0] = Res{(uint32_t)s_ord, l, e};
        return 1;
    }
};

// Fixed total number: candidate c draws (source, target) ordinals from the
// two halves of IDX(c).  Invalid candidates: autapses when excluded, and
// repeats of an earlier valid pair when multapses are excluded (first[c] = 0).
struct Total {
    static constexpr int R = 1;
    const SegD* S;
    uint32_t nS;
    const SegD* T;
    uint32_t nT;
    uint32_t n_s, n_t;
    uint32_t autapses;
    const uint8_t* first;   // null when multapses are allowed
    uint32_t seed, call;
    __device__ __forceinline__ int eval(uint64_t cand, Res* r, uint32_t* th_out = nullptr) const {
        const uint4 b = draw(seed, call, cand, PURPOSE_IDX);
        const uint32_t s = uniform_index(b.x, b.y, n_s);
        const uint32_t t = uniform_index(b.z, b.w, n_t);
        uint32_t th, tl;
        set_lookup(T, nT, t, th, tl);
        if (th_out) *th_out = th;
        if (!autapses) {
            uint32_t sh, sl;
            set_lookup(S, nS, s, sh, sl);
            if (sh == th && sl == tl) return 0;
        }
        if (first && !first[cand]) return 0;
        r[0] = Res{s, tl, cand};
        return 1;
    }
};

// Assigned nodes: pair i names its source and target positions; the
// connection belongs to the share of the target's host.  Element index i.
struct Assigned {
    static constexpr int R = 1;
    const uint32_t* src_pos;
    const uint32_t* tgt_pos;
    const SegD* T;
    uint32_t nT;
    uint32_t host;
    __device__ __forceinline__ int eval(uint64_t i, Res* r) const {
        uint32_t h, l;
        set_lookup(T, nT, tgt_pos[i], h, l);
        if (h != host) return 0;
        r[0] = Res{src_pos[i], l, i};
        return 1;
    }
};

// Pairwise Bernoulli: pair q = t_ord n_s + s_ord (target-major) connects iff
// word q % 4 of BERN(q / 4) is below thr = floor(p 2^32) (2^32 for p = 1).
// Item = (target, k-th Philox block of the blocks that hold its pairs): the
// pairs of target t start at q0 = t_ord n_s, its blocks at q0 / 4; nb =
// ceil(n_s / 4) + 1 items per target cover a pair range that may start and
// end inside a block (a block shared by two targets is drawn by both, each
// keeping its own pairs).  A connection's element index is q.
struct BernPair {
    ChunkTab ch;
    uint32_t nb;      // items per target
    FastDiv fnb;
    uint32_t n_s;
    uint64_t thr;     // floor(p 2^32), 2^32 for p = 1
    uint32_t autapses;
    uint32_t seed, call;
};

struct BernItem {
    uint64_t q0;      // first pair of the target
    uint64_t blk;     // Philox block of this item
    uint32_t tgt;     // target local id
    uint32_t k;       // the item's index among its target's nb items
    int64_t self;     // the target's own source ordinal, or -1
};

// whether the item's block still holds pairs of its target
__device__ __forceinline__ bool bern_valid(const BernPair& r, const BernItem& it) {
    return it.blk * 4 < it.q0 + r.n_s;
}

// the item's target and pair block, without the draw; false past the target's pairs
__device__ __forceinline__ bool bern_item(const BernPair& r, uint64_t g, BernItem& it) {
    const TChunk c = r.ch.at(g);
    const uint32_t rel = (uint32_t)(g - c.out_begin);
    const uint32_t t_rel = fastdiv(rel, r.fnb);
    it.k = rel - t_rel * r.nb;
    it.q0 = (c.t_ord + t_rel) * (uint64_t)r.n_s;
    it.blk = (it.q0 >> 2) + it.k;
    it.tgt = c.local_first + t_rel;
    it.self = c.self_base >= 0 ? c.self_base + t_rel : -1;
    return bern_valid(r, it);
}

// the item after `it` (item g): the next block of the same target while the
// target has items left (runs hold whole targets), else decoded afresh
__device__ __forceinline__ bool bern_next(const BernPair& r, uint64_t g, BernItem& it) {
    if (it.k + 1 < r.nb) {
        ++it.k;
        ++it.blk;
        return bern_valid(r, it);
    }
    return bern_item(r, g, it);
}

// bit i set = pair 4 blk + i connects (inside the target's range, autapse
// rule applied).  The block's pairs sit at positions d0 .. d1 - 1 of the
// target's range (d0 = q0 - 4 blk), so the range and the autapse become two
// shifts of the 4-bit mask.
__device__ __forceinline__ uint32_t bern_draw_mask(const BernPair& r, const BernItem& it) {
    const uint4 b = draw(r.seed, r.call, it.blk, PURPOSE_BERN);
    uint32_t mask = 15u;                                   // p = 1: every pair
    if (!(r.thr >> 32)) {
        const uint32_t t = (uint32_t)r.thr;
        mask = (b.x < t ? 1u : 0u) | (b.y < t ? 2u : 0u) | (b.z < t ? 4u : 0u) | (b.w < t ? 8u : 0u);
    }
    const int64_t d0 = (int64_t)(it.q0 - it.blk * 4);
    const int64_t d1 = d0 + r.n_s;
    if (d0 > 0) mask &= d0 >= 4 ? 0u : (15u << d0) & 15u;
    if (d1 < 4) mask &= d1 <= 0 ? 0u : (1u << d1) - 1u;
    if (!r.autapses && it.self >= 0) {
        const int64_t si = it.self + d0;                   // position of the pair (target, target)
        if (si >= 0 && si < 4) mask &= ~(1u << si);
    }
    return mask;
}

__device__ __forceinline__ uint32_t bern_mask(const BernPair& r, uint64_t g, BernItem& it) {
    if (!bern_item(r, g, it)) return 0;
    return bern_draw_mask(r, it);
}

__device__ __forceinline__ Res bern_res(const BernItem& it, uint32_t i) {
    const uint64_t q = it.blk * 4 + i;
    return Res{(uint32_t)(q - it.q0), it.tgt, q};
}

// COUNT: connections per tile, and each item's 4-bit mask into `masks` (when
// given); MARK: the connections' marks.  WRITE: each thread takes IPT consecutive items of the tile, their
// masks from `masks` when given (the counting pass drew them; no second
// Philox draw), else drawn again; one workgroup scan of the per-thread counts
// places every connection of the tile in an LDS list in pair order (its pair
// within the tile, 2 bytes); then all lanes take list entries in turn for the
// synapse values and the stores, so the sparse hits of a low p leave no lane
// idle, with three barriers per tile.
template <class Sink, int MODE>
__global__ __launch_bounds__(NT) void k_bern(BernPair r, Sink sink, uint64_t n_items, uint64_t tile0, uint32_t n_tiles,
                                             uint32_t* tile_counts, const uint64_t* tile_offsets, uint8_t* masks) {
    __shared__ uint32_t scratch[NT / 64];
    if constexpr (MODE == WRITE) {
        static_assert(4 * TILE <= 65536 && IPT <= 8, "pair index within a tile fits 16 bits, masks 32 bits");
        const uint64_t tile = tile0 + blockIdx.x;
        const uint64_t base = tile * TILE;
        const uint64_t running = tile_offsets[tile];
        if (tile_offsets[tile + 1] == running) return;     // no connection in the tile
        __shared__ uint16_t hits[4 * TILE];
        const uint64_t first = base + (uint64_t)threadIdx.x * IPT;
        uint32_t mk = 0;   // 4 bits per item, item k at bits [4k, 4k + 4)
        if (masks && first + IPT <= n_items && IPT == 4) {
            const uint32_t w = *reinterpret_cast<const uint32_t*>(masks + first);   // 4-byte aligned: TILE, IPT multiples of 4
#pragma unroll
            for (int k = 0; k < IPT; ++k) mk |= ((w >> (8 * k)) & 15u) << (4 * k);
        } else {
#pragma unroll
            for (int k = 0; k < IPT; ++k) {
                const uint64_t item = first + k;
                if (item >= n_items) break;
                BernItem it{};
                const uint32_t m = masks ? (uint32_t)masks[item] : bern_mask(r, item, it);
                mk |= (m & 15u) << (4 * k);
            }
        }
        uint32_t tot;
        uint32_t pre = block_excl_scan<NT>((uint32_t)__builtin_popcount(mk), scratch, &tot);
        for (uint32_t m = mk; m; m &= m - 1) {
            const uint32_t b = __builtin_ctz(m);   // = 4 k + pair within the item
            hits[pre++] = (uint16_t)(threadIdx.x * IPT * 4 + b);
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < tot; i += NT) {
            const uint32_t h = hits[i];
            BernItem it{};
            (void)bern_item(r, base + (h >> 2), it);
            sink.put(running + i, bern_res(it, h & 3u));
        }
        return;
    }
    // COUNT and MARK: the launch's tiles in turn (a capped grid); each
    // thread takes IPT consecutive items, so it decodes its first item only
    // and steps through the target's blocks, and stores its masks in one word
    const uint64_t t_end = tile0 + n_tiles;
    for (uint64_t tile = tile0 + blockIdx.x; tile < t_end; tile += gridDim.x) {
        const uint64_t first = tile * TILE + (uint64_t)threadIdx.x * IPT;
        uint32_t counted = 0, packed = 0;
        BernItem it{};
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
            const uint64_t item = first + k;
            uint32_t mask = 0;
            if (item < n_items && (k == 0 ? bern_item(r, item, it) : bern_next(r, item, it)))
                mask = bern_draw_mask(r, it);
            packed |= mask << (8 * k);
            if constexpr (MODE == MARK) {
                for (uint32_t m = mask; m; m &= m - 1) sink.mark(bern_res(it, __builtin_ctz(m)));
            } else {
                counted += __builtin_popcount(mask);
            }
        }
        if constexpr (MODE == COUNT) {
            if (masks) {
                if (first + IPT <= n_items) {
                    *reinterpret_cast<uint32_t*>(masks + first) = packed;   // 4-byte aligned: TILE, IPT multiples of 4
                } else {
                    for (int k = 0; k < IPT; ++k)
                        if (first + k < n_items) masks[first + k] = (uint8_t)(packed >> (8 * k));
                }
            }
            uint32_t tot;
            block_excl_scan<NT>(counted, scratch, &tot);
            if (threadIdx.x == 0) tile_counts[tile] = tot;
            __syncthreads();   // the scan's scratch is written again by the next tile
        }
    }
}

template <class Sink, int MODE>
void launch_bern(Ctx& c, const BernPair& r, const Sink& sink, uint64_t n_items, uint32_t* tile_counts,
                 const uint64_t* tile_offsets, uint8_t* masks = nullptr) {
    const uint64_t tiles = (n_items + TILE - 1) / TILE;
    for (uint64_t t0 = 0; t0 < tiles; t0 += MAX_TILES_PER_LAUNCH) {
        const uint32_t nb = (uint32_t)std::min<uint64_t>(MAX_TILES_PER_LAUNCH, tiles - t0);
        // WRITE: one workgroup per tile; COUNT and MARK: at most BERN_WGS_PER_CU
        // workgroups per compute unit, each taking tiles in turn
        const uint32_t grid = MODE == WRITE ? nb : std::min<uint32_t>(nb, (uint32_t)c.n_cu * BERN_WGS_PER_CU);
        tstart(c, MODE == MARK ? "prep_mark" : "gen_bernoulli");
        hipLaunchKernelGGL((k_bern<Sink, MODE>), dim3(grid), dim3(NT), 0, c.stream, r, sink, n_items, t0, nb,
                           tile_counts, tile_offsets, masks);
        tstop(c);
        HIPCHK(hipGetLastError());
    }
}

// One-to-one: element i connects source ordinal i to target ordinal i; it is
// an autapse exactly when the target's own source ordinal equals i.
struct OneToOne {
    static constexpr int R = 1;
    ChunkTab ch;
    uint32_t autapses;
    __device__ __forceinline__ int eval(uint64_t g, Res* r) const {
        const TChunk c = ch.at(g);
        const uint32_t rel = (uint32_t)(g - c.out_begin);
        const uint64_t i = c.t_ord + rel;
        if (!autapses && c.self_base >= 0 && (uint64_t)c.self_base + rel == i) return 0;
        r[0] = Res{(uint32_t)i, c.local_first + rel, i};
        return 1;
    }
};

// ------------------------------------------------------------------ generic kernel
template <class Rule, class Sink, int MODE>
__global__ __launch_bounds__(NT) void k_gen(Rule rule, Sink sink, uint64_t n_items, uint64_t tile0,
                                            uint32_t* tile_counts, const uint64_t* tile_offsets, uint64_t limit) {
    __shared__ uint32_t scratch[NT / 64];
    const uint64_t tile = tile0 + blockIdx.x;
    const uint64_t base = tile * TILE;
    uint64_t running = 0;
    if constexpr (MODE == WRITE) running = tile_offsets[tile];
    uint32_t counted = 0;
#pragma unroll 1
    for (int it = 0; it < IPT; ++it) {
        const uint64_t item = base + (uint64_t)it * NT + threadIdx.x;
        Res r[Rule::R];
        int n = 0;
        if (item < n_items) n = rule.eval(item, r);
        if constexpr (MODE == DIRECT) {
            if (n) sink.put(item, r[0]);
        } else if constexpr (MODE == MARK) {
            for (int k = 0; k < n; ++k) sink.mark(r[k]);
        } else if constexpr (MODE == COUNT) {
            counted += (uint32_t)n;
        } else {
            uint32_t tot;
            const uint32_t pre = block_excl_scan<NT>((uint32_t)n, scratch, &tot);
            for (int k = 0; k < n; ++k) {
                const uint64_t pos = running + pre + k;
                if (pos < limit) sink.put(pos, r[k]);
            }
            running += tot;
        }
    }
    if constexpr (MODE == COUNT) {
        uint32_t tot;
        block_excl_scan<NT>(counted, scratch, &tot);
        if (threadIdx.x == 0) tile_counts[tile] = tot;
    }
}

// Regeneration for the point-to-point lists with the bit row in LDS: every
// workgroup marks the draws of a long item range in its own copy of the row
// and ORs the words it set into the global row once, so the global atomics
// scale with workgroups x row words instead of with draws (most draws hit
// sources already marked).
constexpr uint32_t MARK_LDS_WORDS = 16384;   // rows up to 2^19 neurons (64 KB of LDS)

template <class Rule>
__global__ __launch_bounds__(NT) void k_gen_mark_lds(Rule rule, MarkSink sink, uint64_t n_items,
                                                     uint64_t per_block) {
    extern __shared__ uint32_t row[];
    for (uint32_t w = threadIdx.x; w < sink.words; w += NT) row[w] = 0;
    __syncthreads();
    const uint64_t lo = (uint64_t)blockIdx.x * per_block;
    const uint64_t hi = lo + per_block < n_items ? lo + per_block : n_items;
#pragma unroll 1
    for (uint64_t item = lo + threadIdx.x; item < hi; item += NT) {
        Res r[Rule::R];
        const int n = rule.eval(item, r);
        for (int k = 0; k < n; ++k) {
            uint32_t h, l;
            set_lookup(sink.S, sink.nS, r[k].src, h, l);
            if (h == sink.host) atomicOr(&row[l >> 5], 1u << (l & 31));
        }
    }
    __syncthreads();
    for (uint32_t w = threadIdx.x; w < sink.words; w += NT)
        if (row[w]) atomicOr(sink.bits + w, row[w]);
}

template <class Rule, class Sink, int MODE>
void launch_gen(Ctx& c, const char* name, const Rule& rule, const Sink& sink, uint64_t n_items,
                uint32_t* tile_counts, const uint64_t* tile_offsets, uint64_t limit) {
    if constexpr (MODE == MARK) {
        if (c.mark_in_lds && sink.words <= MARK_LDS_WORDS && n_items) {
            // about 2048 workgroups, each over at least 8192 items
            const uint64_t per_block = std::max<uint64_t>(8192, (n_items + 2047) / 2048);
            const uint64_t blocks = (n_items + per_block - 1) / per_block;
            tstart(c, "prep_mark");
            hipLaunchKernelGGL(k_gen_mark_lds<Rule>, dim3((unsigned)blocks), dim3(NT), sink.words * 4, c.stream, rule,
                               sink, n_items, per_block);
            tstop(c);
            HIPCHK(hipGetLastError());
            return;
        }
    }
    const uint64_t tiles = (n_items + TILE - 1) / TILE;
    for (uint64_t t0 = 0; t0 < tiles; t0 += MAX_TILES_PER_LAUNCH) {
        const uint32_t nb = (uint32_t)std::min<uint64_t>(MAX_TILES_PER_LAUNCH, tiles - t0);
        tstart(c, MODE == MARK ? "prep_mark" : name);   // regeneration for the send lists
        hipLaunchKernelGGL((k_gen<Rule, Sink, MODE>), dim3(nb), dim3(NT), 0, c.stream, rule, sink, n_items, t0,
                           tile_counts, tile_offsets, limit);
        tstop(c);
        HIPCHK(hipGetLastError());
    }
}

// ------------------------------------------------------------------ fixed total number
// Candidates of a fixed-total-number call in order; the first `limit` valid
// ones (global rank over all targets) are the connections, and a host keeps
// those whose target it holds.  CNT_VALID counts valid candidates per tile;
// CNT_KEEP counts the kept ones (ranks from the scanned valid counts);
// WRITE_KEEP writes them at the scanned kept counts (ALL_LOCAL: every target
// is on the host, the position is the rank itself); MARK_KEEP marks them.
enum DistMode { CNT_VALID = 0, CNT_KEEP = 1, WRITE_KEEP = 2, MARK_KEEP = 3 };

constexpr uint8_t FIRST_PENDING = 2;   // shares its filter slot: resolved from the exact table

// The exact table of the filtered first occurrences, read by the counting
// pass (CNT_VALID) to settle the candidates still pending (tab null: none).
struct PendingTab {
    const uint64_t* tab;
    const uint32_t* minidx;
    uint64_t mask;
    uint8_t* first;
};
__device__ uint8_t settle_pending(const Total& t, uint64_t i, const PendingTab& p);

template <class Sink, int MODE, bool ALL_LOCAL>
__global__ __launch_bounds__(NT) void k_total_dist(Total rule, uint32_t host, Sink sink, uint64_t n_items,
                                                   uint64_t tile0, uint32_t* tile_counts, const uint64_t* valid_off,
                                                   const uint64_t* keep_off, uint64_t limit, PendingTab pend) {
    __shared__ uint32_t scratch[NT / 64];
    const uint64_t tile = tile0 + blockIdx.x;
    const uint64_t base = tile * TILE;
    uint64_t vrun = 0, krun = 0;
    if constexpr (MODE != CNT_VALID) vrun = valid_off[tile];
    if constexpr (MODE == WRITE_KEEP && !ALL_LOCAL) krun = keep_off[tile];
    if constexpr (MODE == WRITE_KEEP && ALL_LOCAL) {
        // every target on the host: a valid candidate's position is its rank;
        // each thread takes IPT consecutive candidates, one scan per tile
        const uint64_t first_item = base + (uint64_t)threadIdx.x * IPT;
        Res rr[IPT];
        uint32_t vmask = 0, nv = 0;
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
            const uint64_t item = first_item + k;
            uint32_t th = 0;
            rr[k] = Res{};
            const bool v = item < n_items && rule.eval(item, &rr[k], &th) != 0;
            vmask |= (v ? 1u : 0u) << k;
            nv += v ? 1u : 0u;
        }
        uint32_t tot;
        uint64_t rank = vrun + block_excl_scan<NT>(nv, scratch, &tot);
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
            if (!((vmask >> k) & 1u)) continue;
            if (rank < limit) sink.put(rank, rr[k]);
            ++rank;
        }
        return;
    }
    if constexpr (MODE == CNT_VALID) {
        // valid candidates per tile: each thread takes IPT consecutive
        // candidates (independent draws in flight); a candidate sharing its
        // filter slot is settled first, and its flag written back
        const uint64_t first_item = base + (uint64_t)threadIdx.x * IPT;
        uint32_t nv = 0;
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
            const uint64_t item = first_item + k;
            if (item >= n_items) continue;
            if (pend.tab && pend.first[item] == FIRST_PENDING) pend.first[item] = settle_pending(rule, item, pend);
            Res r{};
            uint32_t th = 0;
            nv += (uint32_t)rule.eval(item, &r, &th);
        }
        uint32_t tot;
        block_excl_scan<NT>(nv, scratch, &tot);
        if (threadIdx.x == 0) tile_counts[tile] = tot;
        return;
    }
    uint32_t counted = 0;
#pragma unroll 1
    for (int it = 0; it < IPT; ++it) {
        const uint64_t item = base + (uint64_t)it * NT + threadIdx.x;
        Res r{};
        uint32_t th = 0;
        const uint32_t v = item < n_items ? (uint32_t)rule.eval(item, &r, &th) : 0u;
        {
            uint32_t vtot;
            const uint32_t vpre = block_excl_scan<NT>(v, scratch, &vtot);
            const uint64_t rank = vrun + vpre;
            const bool keep = v && (ALL_LOCAL || th == host) && rank < limit;
            vrun += vtot;
            if constexpr (MODE == CNT_KEEP) {
                counted += keep ? 1u : 0u;
            } else if constexpr (MODE == MARK_KEEP) {
                if (keep) sink.mark(r);
            } else if constexpr (ALL_LOCAL) {
                if (keep) sink.put(rank, r);
            } else {
                uint32_t ktot;
                const uint32_t kpre = block_excl_scan<NT>(keep ? 1u : 0u, scratch, &ktot);
                if (keep) sink.put(krun + kpre, r);
                krun += ktot;
            }
        }
    }
    if constexpr (MODE == CNT_KEEP) {
        uint32_t tot;
        block_excl_scan<NT>(counted, scratch, &tot);
        if (threadIdx.x == 0) tile_counts[tile] = tot;
    }
}

template <class Sink, int MODE, bool ALL_LOCAL>
void launch_total_dist(Ctx& c, const Total& rule, uint32_t host, const Sink& sink, uint64_t n_items,
                       uint32_t* tile_counts, const uint64_t* valid_off, const uint64_t* keep_off, uint64_t limit,
                       const PendingTab& pend = PendingTab{}) {
    const uint64_t tiles = (n_items + TILE - 1) / TILE;
    for (uint64_t t0 = 0; t0 < tiles; t0 += MAX_TILES_PER_LAUNCH) {
        const uint32_t nb = (uint32_t)std::min<uint64_t>(MAX_TILES_PER_LAUNCH, tiles - t0);
        tstart(c, MODE == MARK_KEEP ? "prep_mark" : "gen_total");
        hipLaunchKernelGGL((k_total_dist<Sink, MODE, ALL_LOCAL>), dim3(nb), dim3(NT), 0, c.stream, rule, host, sink,
                           n_items, t0, tile_counts, valid_off, keep_off, limit, pend);
        tstop(c);
        HIPCHK(hipGetLastError());
    }
}

// Count, scan, write: returns the number of results kept (at most `limit`,
// the first ones in element order).  `provide(n)` returns the sink for the
// n results (or null to only count).
template <class Rule, class Provider>
uint64_t count_and_write(Ctx& c, const char* name, const Rule& rule, Provider provide, uint64_t n_items,
                         uint64_t limit) {
    using SinkPtr = decltype(provide(0));
    using Sink = std::remove_cv_t<std::remove_pointer_t<SinkPtr>>;
    const uint64_t tiles = (n_items + TILE - 1) / TILE;
    if (!tiles) return 0;
    uint32_t* counts = dalloc_n<uint32_t>(c, tiles);
    uint64_t* offs = dalloc_n<uint64_t>(c, tiles + 1);
    uint64_t total = 0;
    try {
        launch_gen<Rule, Sink, COUNT>(c, name, rule, Sink{}, n_items, counts, nullptr, 0);
        total = scan_u32_u64(c, counts, offs, tiles, true);
        const uint64_t kept = std::min(total, limit);
        if (kept) {
            SinkPtr sink = provide(kept);
            if (sink) launch_gen<Rule, Sink, WRITE>(c, name, rule, *sink, n_items, counts, offs, limit);
        }
    } catch (...) {
        dfree(c, counts);
        dfree(c, offs);
        throw;
    }
    dfree(c, counts);
    dfree(c, offs);
    return std::min(total, limit);
}

// Synapse values of a call written unit by unit (K elements per unit, in the
// order of the unit runs): position p of the call holds element (t_ord + rel)
// K + j of its run, rel = unit within the run, j = rank within the unit.
__global__ __launch_bounds__(NT) void k_syn_fill(ChunkTab ch, uint32_t K, FastDiv fK,
                                                 uint64_t items, SynD syn, uint32_t seed, uint32_t call,
                                                 uint16_t* delay, float* weight, uint64_t base) {
    for (uint64_t p = (uint64_t)blockIdx.x * NT + threadIdx.x; p < items; p += (uint64_t)gridDim.x * NT) {
        const TChunk c = ch.at(p);
        const uint64_t off = p - c.out_begin;
        const uint32_t rel = fastdiv((uint32_t)off, fK);   // a run holds fewer than 2^32 elements
        const uint32_t j = (uint32_t)off - rel * K;
        float w;
        uint16_t d;
        syn_values(syn, seed, call, (c.t_ord + rel) * (uint64_t)K + j, w, d);
        delay[base + p] = d;
        weight[base + p] = w;
    }
}

// ------------------------------------------------------------------ Floyd's sampling
// One workgroup per unit draws K distinct values in [0, n_eff) with the
// draws r_j = index(IDX(base + j), n_eff - K + j + 1) of Floyd's sampling and
// emits them in ascending order (j = rank).  In-degree: unit = target, all K
// kept.  Out-degree: unit = source, a value is kept when its target is on
// `host`.
struct FloydArgs {
    ChunkTab ch;
    uint64_t n_units;
    uint32_t K, n_set;     // draws per unit, candidate set size
    uint32_t in_degree;
    const SegD* T;         // out-degree: target set
    uint32_t nT;
    uint32_t host;
    uint32_t kpad;         // power of two >= K
    uint32_t kshift;       // log2(kpad): step bits of a 32-bit sort key
    uint32_t seed, call;
};

// Bitonic sort of kp = NT * E keys by a workgroup of NT threads, E keys
// per thread in registers (element tid * E + e in r[e]).  Strides below E
// compare registers of the thread, strides below 64 * E exchange register e
// with lane lane ^ (stride / E) of the same wave, and larger strides (several
// waves) go through LDS.  The keys come from and go back to `key`; the caller
// synchronises before and after.
constexpr uint32_t FLOYD_REG_E = 16;   // at most 16 keys per thread in registers

template <int NT, int E, class KeyT>
__device__ __forceinline__ void reg_bitonic_sort(KeyT* key, uint32_t kp) {
    constexpr uint32_t W = 64u * E;    // keys of one wave
    const uint32_t tid = threadIdx.x;
    const uint32_t base = tid * E;
    KeyT r[E];
#pragma unroll
    for (int e = 0; e < E; ++e) r[e] = key[base + e];
    for (uint32_t size = 2; size <= kp; size <<= 1) {
        uint32_t stride = size >> 1;
        if constexpr (NT > 64) {
            if (stride >= W) {
#pragma unroll
                for (int e = 0; e < E; ++e) key[base + e] = r[e];
                __syncthreads();
                for (; stride >= W; stride >>= 1) {
                    for (uint32_t i = tid; i < kp / 2; i += NT) {
                        const uint32_t lo_i = 2 * i - (i & (stride - 1));
                        const uint32_t hi_i = lo_i + stride;
                        const bool up = ((lo_i & size) == 0);
                        const KeyT x = key[lo_i], y = key[hi_i];
                        if ((x > y) == up) {
                            key[lo_i] = y;
                            key[hi_i] = x;
                        }
                    }
                    __syncthreads();
                }
#pragma unroll
                for (int e = 0; e < E; ++e) r[e] = key[base + e];
            }
        }
        for (; stride >= (uint32_t)E; stride >>= 1) {
            const int m = (int)(stride / E);
            const bool take_min = ((tid & (uint32_t)m) == 0) == ((base & size) == 0);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const KeyT y = __shfl_xor(r[e], m, 64);
                r[e] = take_min ? (y < r[e] ? y : r[e]) : (y < r[e] ? r[e] : y);
            }
        }
#pragma unroll
        for (int S = E / 2; S >= 1; S >>= 1) {
            if ((uint32_t)S < size) {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    if ((e & S) == 0) {
                        const bool up = ((base + (uint32_t)e) & size) == 0;
                        const KeyT x = r[e], y = r[e + S];
                        const KeyT lo = x < y ? x : y, hi = x < y ? y : x;
                        r[e] = up ? lo : hi;
                        r[e + S] = up ? hi : lo;
                    }
                }
            }
        }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) key[base + e] = r[e];
}

// Floyd's sampling without the sequential loop.  Step j draws r_j in
// [0, m_j], m_j = n - K + j, and takes m_j instead exactly when r_j is already
// chosen.  A low value (< n - K) is chosen at its first draw, so a repeat is
// detected by an earlier occurrence (A_j).  A high value m_i (i < j) is chosen
// at step i when step i took its fallback or drew m_i itself, else at its
// first later draw; so dup_j = A_j or dup_i.  These links point to earlier
// steps and are resolved by pointer jumping.  The chosen values -- the same
// set as inserting one by one -- are then listed in ascending order from the
// one sort of the draws and flags over the top window.  K <= 8192, so a step
// index fits 13 bits of the sort key.  The sort runs in registers where the
// padded degree gives each thread 1 to 16 keys (8 for the larger workgroups),
// in LDS otherwise.
// NT threads per unit: one wave (64) for padded degrees up to the context's
// floyd_wave_max, where the barriers of a one-wave workgroup cost next to
// nothing and many units share a compute unit; 256 up to 2048; 1024 above,
// where the LDS of a unit leaves room for one or two units per compute unit.
// KeyT: the sort keys (value << SH | step) in 64 bits with SH = 13, or in 32
// bits with SH = log2(kpad) when every value is below 2^(32 - SH) (half the
// LDS bytes of the sort, and a smaller footprint per unit).
template <int NT, class Sink, int MODE, class KeyT>
__global__ __launch_bounds__(NT) void k_floyd(FloydArgs a, Sink sink, uint32_t* unit_counts, const uint64_t* unit_offsets) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const uint32_t kp = a.kpad;
    const uint32_t SH = sizeof(KeyT) == 8 ? 13u : a.kshift;
    const KeyT SM = (KeyT)((1u << SH) - 1u);
    KeyT* key = reinterpret_cast<KeyT*>(lds_raw);                   // (value << SH | step), later the chosen values
    uint32_t* rv = reinterpret_cast<uint32_t*>(key + kp);           // draw of step j
    uint16_t* par0 = reinterpret_cast<uint16_t*>(rv + kp);
    uint16_t* par1 = par0 + kp;
    uint8_t* dup0 = reinterpret_cast<uint8_t*>(par1 + kp);
    uint8_t* dup1 = dup0 + kp;
    const uint32_t tid = threadIdx.x;
    for (uint64_t u = blockIdx.x; u < a.n_units; u += gridDim.x) {
        const uint64_t g = u * a.K;
        const TChunk c = a.ch.at(g);
        const uint32_t rel = (uint32_t)((g - c.out_begin) / a.K);
        const uint64_t ord = c.t_ord + rel;
        const int64_t self = c.self_base >= 0 ? c.self_base + rel : -1;
        const uint32_t n_eff = a.n_set - (self >= 0 ? 1u : 0u);
        const uint32_t base_m = n_eff - a.K;                    // m_j = base_m + j
        const uint64_t e0 = ord * a.K;
        for (uint32_t j = tid; j < kp; j += NT) {
            if (j < a.K) {
                const uint4 b = draw(a.seed, a.call, e0 + j, PURPOSE_IDX);
                const uint32_t r = uniform_index(b.x, b.y, base_m + j + 1);
                rv[j] = r;
                key[j] = ((KeyT)r << SH) | (KeyT)j;
            } else {
                key[j] = (KeyT)~(KeyT)0;
            }
        }
        __syncthreads();
        bool sorted = false;
        // keys per thread in registers: up to 16 for one wave, 8 for the
        // larger workgroups (whose padded degrees stop at 8 per thread)
        constexpr uint32_t EMAX = NT == 64 ? FLOYD_REG_E : FLOYD_REG_E / 2;
        if (kp >= NT && kp <= NT * EMAX) {
            switch (kp / NT) {
            case 1: reg_bitonic_sort<NT, 1, KeyT>(key, kp); break;
            case 2: reg_bitonic_sort<NT, 2, KeyT>(key, kp); break;
            case 4: reg_bitonic_sort<NT, 4, KeyT>(key, kp); break;
            case 8: reg_bitonic_sort<NT, 8, KeyT>(key, kp); break;
            default:
                if constexpr (EMAX == 16) reg_bitonic_sort<NT, 16, KeyT>(key, kp);
                break;
            }
            __syncthreads();
            sorted = true;
        }
        if (!sorted) {
            for (uint32_t size = 2; size <= kp; size <<= 1) {  // bitonic sort of (value, step) in LDS
                for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
                    for (uint32_t i = tid; i < kp / 2; i += NT) {
                        const uint32_t lo_i = 2 * i - (i & (stride - 1));
                        const uint32_t hi_i = lo_i + stride;
                        const bool up = ((lo_i & size) == 0);
                        const KeyT x = key[lo_i], y = key[hi_i];
                        if ((x > y) == up) {
                            key[lo_i] = y;
                            key[hi_i] = x;
                        }
                    }
                    __syncthreads();
                }
            }
        }
        // A_j: an earlier step drew the same value.  Equal values sort by
        // step, so exactly the first key of each run of equal values has none.
        for (uint32_t p = tid; p < a.K; p += NT) {
            const KeyT k = key[p];
            const uint32_t j = (uint32_t)(k & SM);
            dup0[j] = (p > 0 && (key[p - 1] >> SH) == (k >> SH)) ? 1 : 0;
            const uint32_t r = rv[j];
            par0[j] = (uint16_t)(r >= base_m ? r - base_m : j);   // link to the step whose fallback is r
        }
        __syncthreads();
        uint16_t* pa = par0;
        uint16_t* pb = par1;
        uint8_t* da = dup0;
        uint8_t* db = dup1;
        for (uint32_t span = 1; span < a.K; span <<= 1) {     // pointer jumping
            for (uint32_t j = tid; j < a.K; j += NT) {
                const uint32_t q = pa[j];
                db[j] = da[j] | da[q];
                pb[j] = pa[q];
            }
            __syncthreads();
            uint16_t* tp = pa; pa = pb; pb = tp;
            uint8_t* td = da; da = db; db = td;
        }
        // The chosen values in ascending order, without sorting them again: a
        // low value (< base_m) is chosen at its first draw, so the distinct low
        // draws are the run starts of the sorted keys; every other chosen value
        // lies in the window [base_m, base_m + K) and is flagged there (step
        // j's fallback base_m + j, or a high draw kept as drawn).  Low values
        // come first, then the flagged window positions; each thread takes a
        // contiguous range of positions, one scan gives its output offsets.
        __shared__ uint32_t wsum[NT / 64];
        for (uint32_t i = tid; i < a.K; i += NT) db[i] = 0;
        __syncthreads();
        for (uint32_t j = tid; j < a.K; j += NT) {
            if (da[j]) db[j] = 1;
            else if (rv[j] >= base_m) db[rv[j] - base_m] = 1;
        }
        __syncthreads();
        uint32_t* vals = rv;   // the draws are no longer needed: chosen values in rank order
        const uint32_t per = (a.K + NT - 1) / NT;
        const uint32_t q0 = min(tid * per, a.K), q1 = min(q0 + per, a.K);
        auto low_start = [&](uint32_t q) {
            const uint64_t v = (uint64_t)(key[q] >> SH);
            return v < base_m && (q == 0 || (uint64_t)(key[q - 1] >> SH) != v);
        };
        uint32_t n_low = 0, n_high = 0;
        for (uint32_t q = q0; q < q1; ++q) {
            n_low += low_start(q) ? 1u : 0u;
            n_high += db[q];
        }
        uint32_t tot_low, tot_high;
        uint32_t at_low = block_excl_scan<NT>(n_low, wsum, &tot_low);
        uint32_t at_high = tot_low + block_excl_scan<NT>(n_high, wsum, &tot_high);
        for (uint32_t q = q0; q < q1; ++q) {
            if (low_start(q)) vals[at_low++] = (uint32_t)(key[q] >> SH);
            if (db[q]) vals[at_high++] = base_m + q;
        }
        __syncthreads();
        // emit in ascending order (j = rank)
        uint64_t running = 0;
        if constexpr (MODE == WRITE) running = unit_offsets[u];
        uint32_t counted = 0;
        for (uint32_t j0 = 0; j0 < a.K; j0 += NT) {
            const uint32_t j = j0 + tid;
            Res r{};
            bool ok = false;
            if (j < a.K) {
                uint32_t v = vals[j];
                if (self >= 0 && v >= (uint64_t)self) ++v;
                if (a.in_degree) {
                    r = Res{v, c.local_first + rel, e0 + j};
                    ok = true;
                } else {
                    uint32_t h, l;
                    set_lookup(a.T, a.nT, v, h, l);
                    r = Res{(uint32_t)ord, l, e0 + j};
                    ok = (h == a.host);
                }
            }
            if constexpr (MODE == DIRECT) {
                if (ok) sink.put(c.out_begin + (uint64_t)rel * a.K + j, r);
            } else if constexpr (MODE == MARK) {
                if (ok) sink.mark(r);
            } else {
                uint32_t tot;
                const uint32_t before = block_excl_scan<NT>(ok ? 1u : 0u, wsum, &tot);
                if constexpr (MODE == COUNT) counted += tot;
                else {
                    if (ok) sink.put(running + before, r);
                    running += tot;
                }
            }
        }
        if constexpr (MODE == COUNT) {
            if (tid == 0) unit_counts[u] = counted;
        }
        __syncthreads();
    }
}

// Small degrees (K <= FLOYD_SMALL): one lane per unit, the same draws and
// Floyd's insertions one by one (membership by a scan of the K chosen values), the
// chosen values sorted ascending and emitted with j = rank.  LDS slot j of
// lane t is [j * FNT + t], so the lanes of a wave hit distinct banks.
constexpr uint32_t FLOYD_SMALL = 32;
constexpr int FNT = 256;

// One unit of the small-degree sampler; x points at the unit's first value
// slot, slot j at x[j * stride].
template <class Sink, int MODE>
__device__ __forceinline__ void floyd_small_unit(const FloydArgs& a, uint64_t u, uint32_t* x, uint32_t stride,
                                                 const Sink& sink, uint32_t* unit_counts,
                                                 const uint64_t* unit_offsets) {
    const uint64_t g = u * a.K;
    const TChunk c = a.ch.at(g);
    const uint32_t rel = (uint32_t)((g - c.out_begin) / a.K);
    const uint64_t ord = c.t_ord + rel;
    const int64_t self = c.self_base >= 0 ? c.self_base + rel : -1;
    const uint32_t n_eff = a.n_set - (self >= 0 ? 1u : 0u);
    const uint64_t e0 = ord * a.K;
    for (uint32_t j = 0; j < a.K; ++j) {
        const uint4 b = draw(a.seed, a.call, e0 + j, PURPOSE_IDX);
        const uint32_t r = uniform_index(b.x, b.y, n_eff - a.K + j + 1);
        bool found = false;
        for (uint32_t i = 0; i < j; ++i) found |= x[i * stride] == r;
        x[j * stride] = found ? n_eff - a.K + j : r;   // the fallback was never chosen before step j
    }
    for (uint32_t j = 1; j < a.K; ++j) {   // insertion sort, ascending
        const uint32_t v = x[j * stride];
        uint32_t i = j;
        while (i > 0 && x[(i - 1) * stride] > v) {
            x[i * stride] = x[(i - 1) * stride];
            --i;
        }
        x[i * stride] = v;
    }
    uint64_t running = 0;
    if constexpr (MODE == WRITE) running = unit_offsets[u];
    uint32_t counted = 0;
    for (uint32_t j = 0; j < a.K; ++j) {
        uint32_t v = x[j * stride];
        if (self >= 0 && v >= (uint64_t)self) ++v;
        Res r{};
        bool ok;
        if (a.in_degree) {
            r = Res{v, c.local_first + rel, e0 + j};
            ok = true;
        } else {
            uint32_t h, l;
            set_lookup(a.T, a.nT, v, h, l);
            r = Res{(uint32_t)ord, l, e0 + j};
            ok = (h == a.host);
        }
        if (!ok) continue;
        if constexpr (MODE == DIRECT) sink.put(c.out_begin + (uint64_t)rel * a.K + j, r);
        else if constexpr (MODE == MARK) sink.mark(r);
        else if constexpr (MODE == COUNT) ++counted;
        else sink.put(running++, r);
    }
    if constexpr (MODE == COUNT) unit_counts[u] = counted;
}

template <class Sink, int MODE>
__global__ __launch_bounds__(FNT) void k_floyd_small(FloydArgs a, Sink sink, uint32_t* unit_counts,
                                                     const uint64_t* unit_offsets) {
    __shared__ uint32_t x[FLOYD_SMALL * FNT];
    const uint32_t t = threadIdx.x;
    for (uint64_t u = (uint64_t)blockIdx.x * FNT + t; u < a.n_units; u += (uint64_t)gridDim.x * FNT)
        floyd_small_unit<Sink, MODE>(a, u, x + t, FNT, sink, unit_counts, unit_offsets);
}

template <class Sink, int MODE, class KeyT>
void launch_floyd_keys(Ctx& c, const FloydArgs& a, const Sink& sink, uint32_t* unit_counts,
                       const uint64_t* unit_offsets) {
    const uint32_t grid = (uint32_t)std::min<uint64_t>(a.n_units, 65536);
    const size_t shmem = (size_t)a.kpad * (sizeof(KeyT) + 4 + 2 * 2 + 2 * 1);
    tstart(c, MODE == MARK ? "prep_mark" : "gen_floyd");
    if (a.kpad <= c.floyd_wave_max) {
        hipLaunchKernelGGL((k_floyd<64, Sink, MODE, KeyT>), dim3(grid), dim3(64), shmem, c.stream, a, sink,
                           unit_counts, unit_offsets);
    } else if (a.kpad <= 2048) {
        hipLaunchKernelGGL((k_floyd<256, Sink, MODE, KeyT>), dim3(grid), dim3(256), shmem, c.stream, a, sink,
                           unit_counts, unit_offsets);
    } else {
        // 57 .. 147 KB of LDS leave room for one or two units per compute unit: 16 waves each
        HIPCHK(hipFuncSetAttribute((const void*)k_floyd<1024, Sink, MODE, KeyT>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
        hipLaunchKernelGGL((k_floyd<1024, Sink, MODE, KeyT>), dim3(grid), dim3(1024), shmem, c.stream, a, sink,
                           unit_counts, unit_offsets);
    }
    tstop(c);
    HIPCHK(hipGetLastError());
}

template <class Sink, int MODE>
void launch_floyd(Ctx& c, const FloydArgs& a, const Sink& sink, uint32_t* unit_counts, const uint64_t* unit_offsets) {
    if (!a.n_units) return;
    if (a.K <= FLOYD_SMALL) {
        const uint32_t grid = (uint32_t)std::min<uint64_t>((a.n_units + FNT - 1) / FNT, 65536);
        tstart(c, MODE == MARK ? "prep_mark" : "gen_floyd");
        hipLaunchKernelGGL((k_floyd_small<Sink, MODE>), dim3(grid), dim3(FNT), 0, c.stream, a, sink, unit_counts,
                           unit_offsets);
        tstop(c);
        HIPCHK(hipGetLastError());
        return;
    }
    const uint32_t grid = (uint32_t)std::min<uint64_t>(a.n_units, 65536);
    if (a.kpad > 8192) raise(SNNC_EUNSUPPORTED, "degree above 8192 without multapses");
    // 32-bit sort keys when (value << log2(kpad) | step) stays below 2^32
    if (((uint64_t)a.n_set << a.kshift) < (1ull << 32)) launch_floyd_keys<Sink, MODE, uint32_t>(c, a, sink, unit_counts, unit_offsets);
    else launch_floyd_keys<Sink, MODE, uint64_t>(c, a, sink, unit_counts, unit_offsets);
}

// Floyd's sampling written directly (one unit after another): sources and
// targets by the sampler, then the synapse values by element index.
bool defer_syn_fill(Ctx& c, const FloydArgs& a, const WriteSink& ws, uint64_t items);
bool defer_floyd_small(Ctx& c, const FloydArgs& a, const WriteSink& ws);

void launch_floyd_direct(Ctx& c, const FloydArgs& a, const WriteSink& ws, uint64_t items) {
    IdSink ids{ws.src, ws.tgt, ws.base};
    if (!(a.K <= FLOYD_SMALL && defer_floyd_small(c, a, ws))) launch_floyd<IdSink, DIRECT>(c, a, ids, nullptr, nullptr);
    if (!items) return;
    if (defer_syn_fill(c, a, ws, items)) return;   // the batch's fused launch writes them
    const uint32_t grid = (uint32_t)std::min<uint64_t>((items + NT - 1) / NT, 1u << 20);
    tstart(c, "gen_floyd");
    hipLaunchKernelGGL(k_syn_fill, dim3(grid), dim3(NT), 0, c.stream, a.ch, a.K, make_fastdiv(a.K), items,
                       ws.syn, ws.seed, ws.call, ws.delay, ws.weight, ws.base);
    tstop(c);
    HIPCHK(hipGetLastError());
}

uint32_t next_pow2(uint32_t x) {
    uint32_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

uint32_t log2_pow2(uint32_t p) {
    uint32_t l = 0;
    while ((1u << l) < p) ++l;
    return l;
}

// ------------------------------------------------------------------ total number, restricted
// First-occurrence flags for the multapse-free total number: sort the
// candidates' (source, target) pair keys stably and keep the first of every
// run of equal keys.
__global__ void k_total_keys(const Total t, uint64_t n, uint32_t n_t, uint64_t* keys, uint32_t* vals) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 b = draw(t.seed, t.call, i, PURPOSE_IDX);
    const uint32_t s = uniform_index(b.x, b.y, t.n_s);
    const uint32_t tt = uniform_index(b.z, b.w, t.n_t);
    keys[i] = (uint64_t)s * n_t + tt;
    vals[i] = (uint32_t)i;
}

__global__ void k_first_flags(const uint64_t* keys, const uint32_t* vals, uint64_t n, uint8_t* first) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    first[vals[i]] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

// First occurrences by hashing behind a filter.  Every candidate clears the
// "unseen" bit of its slot in a bitmap of at least 16 slots per candidate
// (all bits start at one, so the table and the filter take one fill) and,
// when that bit was clear already, the slot's "alone" bit.  A candidate alone
// in its slot draws a pair that no other candidate draws, so it is the first
// (and only) occurrence of that pair.  The others, about one in 16, resolve
// exactly in an open-addressing table of at least 1.5 slots per distinct pair
// they can hold: each claims the slot of its pair (compare-and-swap) and
// lowers the slot's smallest candidate index; the candidate holding the
// minimum is the first occurrence.  No result depends on the order of the
// atomics.
constexpr uint64_t HASH_EMPTY = ~0ull;

__device__ __forceinline__ uint64_t pair_hash(uint64_t x) {
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return x;
}

__device__ __forceinline__ uint64_t total_pair_key(const Total& t, uint64_t i, uint32_t n_t) {
    const uint4 b = draw(t.seed, t.call, i, PURPOSE_IDX);
    return (uint64_t)uniform_index(b.x, b.y, t.n_s) * n_t + uniform_index(b.z, b.w, t.n_t);
}

// filter slot of a pair: two bits (seen, shared) in word slot / 16
__device__ __forceinline__ uint64_t filter_slot(uint64_t key, uint64_t slot_mask) {
    return pair_hash(key) & slot_mask;
}

// table slot of a pair: the other half of the hash, so that pairs sharing a
// filter slot spread over the table
__device__ __forceinline__ uint64_t table_slot(uint64_t key, uint64_t mask) {
    const uint64_t h = pair_hash(key);
    return ((h >> 32) | (h << 32)) & mask;
}

__global__ void k_first_filter(const Total t, uint64_t n, uint32_t n_t, uint32_t* bm, uint64_t slot_mask) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t h = filter_slot(total_pair_key(t, i, n_t), slot_mask);
    const uint32_t sh = (uint32_t)(h & 15) * 2;
    const uint32_t old = atomicAnd(&bm[h >> 4], ~(1u << sh));
    if (!((old >> sh) & 1u)) atomicAnd(&bm[h >> 4], ~(2u << sh));
}

__global__ void k_first_resolve(const Total t, uint64_t n, uint32_t n_t, const uint32_t* bm, uint64_t slot_mask,
                                uint64_t* tab, uint32_t* minidx, uint64_t mask, uint8_t* first) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t key = total_pair_key(t, i, n_t);
    const uint64_t h = filter_slot(key, slot_mask);
    if ((bm[h >> 4] >> ((uint32_t)(h & 15) * 2 + 1)) & 1u) {   // still alone
        first[i] = 1;
        return;
    }
    first[i] = FIRST_PENDING;
    uint64_t s = table_slot(key, mask);
    for (uint64_t probe = 0; probe <= mask; ++probe) {   // never full: 1.5 slots per possible pair
        const uint64_t prev = atomicCAS((unsigned long long*)&tab[s], (unsigned long long)HASH_EMPTY,
                                        (unsigned long long)key);
        if (prev == HASH_EMPTY || prev == key) {
            atomicMin(&minidx[s], (uint32_t)i);
            return;
        }
        s = (s + 1) & mask;
    }
}

// the first-occurrence flag of pending candidate i: whether it holds the
// smallest index among the candidates of its pair
__device__ uint8_t settle_pending(const Total& t, uint64_t i, const PendingTab& p) {
    const uint64_t key = total_pair_key(t, i, t.n_t);
    uint64_t s = table_slot(key, p.mask);
    for (uint64_t probe = 0; probe <= p.mask; ++probe) {
        if (p.tab[s] == key) return p.minidx[s] == (uint32_t)i ? 1 : 0;
        s = (s + 1) & p.mask;
    }
    return 0;   // not reached: every pending candidate's pair is in the table
}

// Small candidate windows: the whole first-occurrence pipeline and the
// valid counts with their scan in one launch of one workgroup, the phases
// separated by barriers (fill the table and filter with ones; filter;
// resolve; settle the pending candidates; valid candidates per tile of TILE
// and the tiles' exclusive offsets, the total to out[tiles] and *total_out).
// Every candidate stays with one thread through all phases (candidate
// i = k FS_NT + thread, and TILE == FS_NT), so its flag is read back by the
// thread that wrote it; the filter and table words other threads wrote are
// read with device-scope atomic loads.  Same flags, offsets and total as the
// filter, resolve, pending, counting and scan launches.
constexpr uint32_t FS_NT = 1024;
static_assert(TILE == FS_NT, "one tile per iteration of the workgroup");

struct FirstSmallJob {
    Total t;
    uint64_t n;
    uint32_t n_t;
    uint64_t* block;
    uint64_t words, H, slot_mask;
    uint8_t* first;
    uint64_t* voff;
    uint64_t* total_out;
};

__device__ __forceinline__ void first_small_window(const Total& t, uint64_t n, uint32_t n_t, uint64_t* block,
                                                   uint64_t words, uint64_t H, uint64_t slot_mask, uint8_t* first,
                                                   uint64_t* voff, uint64_t* total_out, uint32_t* scratch) {
    const uint32_t tid = threadIdx.x;
    uint64_t* tab = block;
    uint32_t* minidx = reinterpret_cast<uint32_t*>(block + H);
    uint32_t* bm = minidx + H;
    const uint64_t mask = H - 1;
    for (uint64_t w = tid; w < words; w += FS_NT) block[w] = ~0ull;
    __syncthreads();
    for (uint64_t i = tid; i < n; i += FS_NT) {   // filter
        const uint64_t h = filter_slot(total_pair_key(t, i, n_t), slot_mask);
        const uint32_t sh = (uint32_t)(h & 15) * 2;
        const uint32_t old = atomicAnd(&bm[h >> 4], ~(1u << sh));
        if (!((old >> sh) & 1u)) atomicAnd(&bm[h >> 4], ~(2u << sh));
    }
    __syncthreads();
    for (uint64_t i = tid; i < n; i += FS_NT) {   // resolve
        const uint64_t key = total_pair_key(t, i, n_t);
        const uint64_t h = filter_slot(key, slot_mask);
        const uint32_t word = __hip_atomic_load(&bm[h >> 4], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((word >> ((uint32_t)(h & 15) * 2 + 1)) & 1u) {
            first[i] = 1;
            continue;
        }
        first[i] = FIRST_PENDING;
        uint64_t s = table_slot(key, mask);
        for (uint64_t probe = 0; probe <= mask; ++probe) {   // never full: 1.5 slots per possible pair
            const uint64_t prev = atomicCAS((unsigned long long*)&tab[s], (unsigned long long)HASH_EMPTY,
                                            (unsigned long long)key);
            if (prev == HASH_EMPTY || prev == key) {
                atomicMin(&minidx[s], (uint32_t)i);
                break;
            }
            s = (s + 1) & mask;
        }
    }
    __syncthreads();
    for (uint64_t i = tid; i < n; i += FS_NT) {   // pending
        if (first[i] != FIRST_PENDING) continue;
        const uint64_t key = total_pair_key(t, i, n_t);
        uint64_t s = table_slot(key, mask);
        uint8_t f = 0;
        for (uint64_t probe = 0; probe <= mask; ++probe) {
            if (__hip_atomic_load(&tab[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == key) {
                f = __hip_atomic_load(&minidx[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == (uint32_t)i ? 1 : 0;
                break;
            }
            s = (s + 1) & mask;
        }
        first[i] = f;
    }
    Total tv = t;
    tv.first = first;
    const uint64_t tiles = (n + TILE - 1) / TILE;
    uint64_t running = 0;
    for (uint64_t tile = 0; tile < tiles; ++tile) {   // valid counts and their scan
        const uint64_t i = tile * TILE + tid;
        Res r{};
        const uint32_t v = i < n ? (uint32_t)tv.eval(i, &r) : 0u;
        uint32_t tot;
        block_excl_scan<FS_NT, uint32_t>(v, scratch, &tot);
        if (tid == 0) voff[tile] = running;
        running += tot;
    }
    if (tid == 0) {
        voff[tiles] = running;
        *total_out = running;
    }
}

__global__ __launch_bounds__(FS_NT) void k_first_small(Total t, uint64_t n, uint32_t n_t, uint64_t* block,
                                                       uint64_t words, uint64_t H, uint64_t slot_mask,
                                                       uint8_t* first, uint64_t* voff, uint64_t* total_out) {
    __shared__ uint32_t scratch[FS_NT / 64];
    first_small_window(t, n, n_t, block, words, H, slot_mask, first, voff, total_out, scratch);
}

// The small windows of a batch's admission counts: one workgroup per window.
__global__ __launch_bounds__(FS_NT) void k_first_small_multi(const FirstSmallJob* jobs) {
    __shared__ uint32_t scratch[FS_NT / 64];
    const FirstSmallJob j = jobs[blockIdx.x];
    first_small_window(j.t, j.n, j.n_t, j.block, j.words, j.H, j.slot_mask, j.first, j.voff, j.total_out, scratch);
}

struct DeviceChunks {
    ChunkTab tab{};
    TChunk* d = nullptr;   // device copy of a table too long to go inline (owned)
    uint64_t items = 0;
};

DeviceChunks upload_chunks(Ctx& c, const std::vector<TChunk>& v, uint64_t items) {
    DeviceChunks dc;
    dc.tab.n = (uint32_t)v.size();
    dc.items = items;
    if (v.size() <= CH_INLINE) {
        std::copy(v.begin(), v.end(), dc.tab.in);
        return dc;
    }
    dc.d = dalloc_n<TChunk>(c, v.size());
    upload(c, dc.d, v.data(), v.size() * sizeof(TChunk));
    dc.tab.d = dc.d;
    return dc;
}

// Runs of units of set U (optionally only those on `host`) with their self
// positions in set O (when autapses are excluded), each run holding at most
// max_elems / per_unit units; out_begin counts per_unit elements per unit.
std::vector<TChunk> unit_runs(const HostSet& U, const HostSet* O, int64_t host, uint64_t per_unit,
                              uint64_t max_elems) {
    std::vector<TChunk> out;
    uint64_t acc = 0;
    const uint64_t max_units = std::max<uint64_t>(1, max_elems / std::max<uint64_t>(per_unit, 1));
    auto emit = [&](uint64_t ord, uint32_t local, uint64_t n, int64_t self) {
        while (n) {
            const uint64_t k = std::min(n, max_units);
            out.push_back(TChunk{ord, acc, self, local, (uint32_t)k});
            acc += k * per_unit;
            ord += k;
            local += (uint32_t)k;
            if (self >= 0) self += (int64_t)k;
            n -= k;
        }
    };
    for (size_t i = 0; i < U.seg.size(); ++i) {
        const snnc_segment g = U.seg[i];
        if (host >= 0 && g.host != (uint32_t)host) continue;
        const uint64_t ord0 = U.ord_begin[i];
        if (!O) {
            emit(ord0, g.first, g.n, -1);
            continue;
        }
        // pieces of g inside the other set's segments on the same host
        std::vector<std::pair<uint32_t, uint32_t>> cuts;   // [lo, hi) local ranges with self mapping
        std::vector<int64_t> selfs;
        for (size_t j = 0; j < O->seg.size(); ++j) {
            const snnc_segment o = O->seg[j];
            if (o.host != g.host) continue;
            const uint64_t lo = std::max<uint64_t>(g.first, o.first);
            const uint64_t hi = std::min<uint64_t>((uint64_t)g.first + g.n, (uint64_t)o.first + o.n);
            if (hi <= lo) continue;
            cuts.push_back({(uint32_t)lo, (uint32_t)hi});
            selfs.push_back((int64_t)(O->ord_begin[j] + (lo - o.first)));
        }
        std::vector<size_t> idx(cuts.size());
        for (size_t k = 0; k < idx.size(); ++k) idx[k] = k;
        std::sort(idx.begin(), idx.end(), [&](size_t x, size_t y) { return cuts[x].first < cuts[y].first; });
        uint32_t cur = g.first;
        const uint32_t end = g.first + g.n;
        for (size_t k : idx) {
            if (cuts[k].first > cur) emit(ord0 + (cur - g.first), cur, cuts[k].first - cur, -1);
            emit(ord0 + (cuts[k].first - g.first), cuts[k].first, cuts[k].second - cuts[k].first, selfs[k]);
            cur = cuts[k].second;
        }
        if (cur < end) emit(ord0 + (cur - g.first), cur, end - cur, -1);
    }
    return out;
}

constexpr uint64_t MAX_RUN_ELEMS = 1ull << 30;

uint64_t runs_elems(const std::vector<TChunk>& v, uint64_t per_unit) {
    return v.empty() ? 0 : v.back().out_begin + (uint64_t)v.back().n * per_unit;
}

SynD syn_of(const Call& cl) {
    SynD s{};
    s.w_mean = cl.w.mean;
    s.w_sd = cl.w.sd;
    s.w_const = cl.w_const;
    s.w_normal = cl.w.kind == SNNC_NORMAL;
    s.d_normal = cl.d.kind == SNNC_NORMAL;
    s.d_const = cl.d_const;
    s.dtab = cl.dtab_dev;
    s.dguide = cl.dguide_dev;
    s.dtab_len = cl.dtab ? (uint32_t)cl.dtab->tab.size() : 0u;
    s.d_klo = cl.d_klo;
    return s;
}

// Thrown by the output provider in counting mode, once the count is known.
struct CountOnly {
    uint64_t n;
};

enum class Out { APPEND, AT_BASE, COUNT, MARK };

// The whole generation of one call on one host's share.
//   APPEND:  append the connections to the generation-order arrays;
//   AT_BASE: write them at [cl.gen_begin, cl.gen_begin + cl.gen_count), room
//            reserved by the caller (served batches);
//   COUNT:   only count them (launches counting passes where the count
//            depends on the draws);
//   MARK:    mark the sources on P_local (point-to-point regeneration).
uint64_t run_call(Ctx& c, Call& cl, uint32_t host, Out mode, uint32_t* mark_bits) {
    if (!cl.meta) upload_meta(c, cl);
    const bool mark = mode == Out::MARK;
    WriteSink ws{};
    MarkSink ms{};
    if (mark) ms = MarkSink{cl.dS, (uint32_t)cl.S.seg.size(), c.P_local, mark_bits, (c.M[c.P_local] + 31) / 32};
    // room for the n connections; returns the sink writing them
    auto reserve = [&](uint64_t n) -> WriteSink* {
        uint64_t base = c.n_gen;
        if (mode == Out::COUNT) throw CountOnly{n};
        if (mode == Out::AT_BASE) {
            if (n != cl.gen_count) raise(SNNC_EDEVICE, "generated count differs from the admitted count");
            base = cl.gen_begin;
        } else {
            grow_gen(c, c.n_gen + n);
        }
        ws = WriteSink{c.g_src, c.g_tgt, c.g_delay, c.g_weight, base, syn_of(cl), c.seed, cl.id};
        return &ws;
    };

    const uint32_t nS = (uint32_t)cl.S.seg.size(), nT = (uint32_t)cl.T.seg.size();
    const uint64_t ns = cl.S.total, nt = cl.T.total;
    uint64_t result = 0;
    std::vector<void*> temps;
    auto cleanup = [&] {
        for (void* p : temps) dfree(c, p);
    };
    try {
        switch (cl.rule) {
        case SNNC_FIXED_INDEGREE: {
            const uint64_t K = cl.n;
            if (!K || !ns) break;
            auto runs = unit_runs(cl.T, cl.autapses ? nullptr : &cl.S, host, K, MAX_RUN_ELEMS);
            const uint64_t items = runs_elems(runs, K);
            result = items;
            if (!items || mode == Out::COUNT) break;     // every target keeps its K draws
            DeviceChunks dc = upload_chunks(c, runs, items);
            temps.push_back(dc.d);
            if (cl.multapses) {
                InDegree r{dc.tab, (uint32_t)K, make_fastdiv((uint32_t)K), (uint32_t)ns, c.seed, cl.id};
                if (mark) launch_gen<InDegree, MarkSink, MARK>(c, "gen_indegree", r, ms, items, nullptr, nullptr, 0);
                else launch_gen<InDegree, WriteSink, DIRECT>(c, "gen_indegree", r, *reserve(items), items, nullptr, nullptr, 0);
            } else {
                FloydArgs a{dc.tab, items / K, (uint32_t)K, (uint32_t)ns, 1, cl.dT, nT, host,
                            next_pow2((uint32_t)K), log2_pow2(next_pow2((uint32_t)K)), c.seed, cl.id};
                if (mark) launch_floyd<MarkSink, MARK>(c, a, ms, nullptr, nullptr);
                else launch_floyd_direct(c, a, *reserve(items), items);
            }
            break;
        }
        case SNNC_FIXED_OUTDEGREE: {
            const uint64_t K = cl.n;
            if (!K || !nt) break;
            // regeneration for the point-to-point lists only needs the sources on the marked host
            const int64_t unit_host = mark ? (int64_t)c.P_local : -1;
            auto runs = unit_runs(cl.S, cl.autapses ? nullptr : &cl.T, unit_host, K, MAX_RUN_ELEMS);
            const uint64_t items = runs_elems(runs, K);
            if (!items) break;
            uint64_t on_host = 0;
            for (auto& g : cl.T.seg) if (g.host == host) on_host += g.n;
            const bool all_local = on_host == nt;
            if (all_local && mode == Out::COUNT) {   // every draw is kept
                result = items;
                break;
            }
            DeviceChunks dc = upload_chunks(c, runs, items);
            temps.push_back(dc.d);
            if (cl.multapses) {
                OutDegree r{dc.tab, (uint32_t)K, make_fastdiv((uint32_t)K), (uint32_t)nt, cl.dT, nT, host,
                            c.seed, cl.id};
                if (mark) {
                    launch_gen<OutDegree, MarkSink, MARK>(c, "gen_outdegree", r, ms, items, nullptr, nullptr, 0);
                } else if (all_local) {
                    result = items;
                    launch_gen<OutDegree, WriteSink, DIRECT>(c, "gen_outdegree", r, *reserve(items), items, nullptr, nullptr, 0);
                } else {
                    result = count_and_write<OutDegree>(c, "gen_outdegree", r, reserve, items, UINT64_MAX);
                }
            } else {
                const uint64_t units = items / K;
                FloydArgs a{dc.tab, units, (uint32_t)K, (uint32_t)nt, 0, cl.dT, nT, host,
                            next_pow2((uint32_t)K), log2_pow2(next_pow2((uint32_t)K)), c.seed, cl.id};
                if (mark) {
                    launch_floyd<MarkSink, MARK>(c, a, ms, nullptr, nullptr);
                } else if (all_local) {
                    result = items;
                    launch_floyd_direct(c, a, *reserve(items), items);
                } else {
                    uint32_t* cnt = dalloc_n<uint32_t>(c, units);
                    temps.push_back(cnt);
                    uint64_t* off = dalloc_n<uint64_t>(c, units + 1);
                    temps.push_back(off);
                    launch_floyd<WriteSink, COUNT>(c, a, ws, cnt, nullptr);
                    result = scan_u32_u64(c, cnt, off, units, true);
                    if (result) launch_floyd<WriteSink, WRITE>(c, a, *reserve(result), cnt, off);
                }
            }
            break;
        }
        case SNNC_FIXED_TOTAL_NUMBER: {
            // targets on several hosts: every host evaluates every candidate and
            // keeps the first N valid ones whose target it holds
            const uint64_t on_host = [&] {
                uint64_t k = 0;
                for (auto& g : cl.T.seg) if (g.host == host) k += g.n;
                return k;
            }();
            if (!cl.n || !on_host) break;
            const bool all_local = on_host == nt;
            const uint64_t N = cl.n;
            Total r{cl.dS, nS, cl.dT, nT, (uint32_t)ns, (uint32_t)nt, cl.autapses ? 1u : 0u, nullptr, c.seed, cl.id};
            if (cl.autapses && cl.multapses && all_local) {
                result = N;
                if (mark) launch_gen<Total, MarkSink, MARK>(c, "gen_total", r, ms, N, nullptr, nullptr, 0);
                else launch_gen<Total, WriteSink, DIRECT>(c, "gen_total", r, *reserve(N), N, nullptr, nullptr, 0);
                break;
            }
            // candidate window: enough draws for N valid ones (expected), grown until it is
            const double V = (double)ns * (double)nt;
            double est = cl.autapses && cl.multapses ? (double)N : (double)N * 1.05 + 1024.0;
            if (!cl.multapses) {
                const double frac = std::min(0.999999, (double)N / V);
                est = std::max(est, -V * std::log1p(-frac) * 1.05 + 1024.0);
            }
            uint64_t C = (uint64_t)std::min(est, 4.0e9);
            if (cl.pre_off && mode != Out::COUNT && !mark) {
                // counted at admission: window, flags and offsets are kept with the call
                C = cl.pre_window;
                Total rr = r;
                rr.first = cl.pre_first;
                uint64_t* voff = cl.pre_off;
                uint64_t* koff = cl.pre_koff;
                result = cl.pre_count;
                temps.insert(temps.end(), {(void*)voff, (void*)koff, (void*)cl.pre_first});
                cl.pre_off = cl.pre_koff = nullptr;
                cl.pre_first = nullptr;
                WriteSink* sink = reserve(result);
                if (result) {
                    if (all_local)
                        launch_total_dist<WriteSink, WRITE_KEEP, true>(c, rr, host, *sink, C, nullptr, voff, koff, N);
                    else
                        launch_total_dist<WriteSink, WRITE_KEEP, false>(c, rr, host, *sink, C, nullptr, voff, koff, N);
                }
                break;
            }
            for (;;) {
                uint8_t* first = nullptr;
                const uint64_t tiles = (C + TILE - 1) / TILE;
                const bool deferred = mode == Out::COUNT && c.defer_slot;
                uint64_t* voff = nullptr;   // set here when the small-window launch counted and scanned
                PendingTab pend{};          // filtered windows: the exact table, read by the counting pass
                if (!cl.multapses && C <= c.total_small_max && C <= c.total_hash_max) {
                    uint64_t m = 1024;
                    while (m < 16 * C) m <<= 1;
                    const uint64_t distinct = std::min<uint64_t>(C, ns * nt);
                    uint64_t H = 1024;
                    while (H < distinct + distinct / 2) H <<= 1;
                    uint64_t* block = dalloc_n<uint64_t>(c, H + H / 2 + m / 32);
                    first = dalloc_n<uint8_t>(c, C);
                    voff = dalloc_n<uint64_t>(c, tiles + 1);
                    temps.insert(temps.end(), {block, first, voff});
                    uint64_t* total_out = deferred ? c.defer_slot : c.tot_pin_dev + (c.stream == c.count_stream ? 1 : 0);
                    temps.erase(std::remove(temps.begin(), temps.end(), (void*)block), temps.end());
                    if (deferred && all_local && c.scan_batching) {
                        // batched admission: launched with the batch's other small windows, before
                        // the scans (no later count of this call reads its flags or offsets)
                        const FirstSmallJob job{r, C, (uint32_t)nt, block, H + H / 2 + m / 32, H, m - 1,
                                                first, voff, total_out};
                        const uint8_t* b = reinterpret_cast<const uint8_t*>(&job);
                        c.first_jobs.insert(c.first_jobs.end(), b, b + sizeof job);
                        c.scan_owned.push_back(block);   // released after that launch
                    } else {
                        tstart(c, "gen_total_first");
                        hipLaunchKernelGGL(k_first_small, dim3(1), dim3(FS_NT), 0, c.stream, r, C, (uint32_t)nt,
                                           block, H + H / 2 + m / 32, H, m - 1, first, voff, total_out);
                        tstop(c);
                        const hipError_t e = hipGetLastError();
                        dfree(c, block);
                        HIPCHK(e);
                    }
                } else if (!cl.multapses && C <= c.total_hash_max) {
                    // filter: 2 bits per slot, at least 16 slots per candidate
                    uint64_t m = 1024;
                    while (m < 16 * C) m <<= 1;
                    // table: 1.5 slots per pair a pending candidate can hold (at most min(C, pairs))
                    const uint64_t distinct = std::min<uint64_t>(C, ns * nt);
                    uint64_t H = 1024;
                    while (H < distinct + distinct / 2) H <<= 1;
                    // keys (HASH_EMPTY), earliest candidates (none yet) and the filter (unseen, alone) in
                    // one block, all bits one, cleared by one fill
                    uint64_t* tab = dalloc_n<uint64_t>(c, H + H / 2 + m / 32);
                    uint32_t* minidx = reinterpret_cast<uint32_t*>(tab + H);
                    uint32_t* bm = minidx + H;
                    first = dalloc_n<uint8_t>(c, C);
                    temps.insert(temps.end(), {tab, first});
                    HIPCHK(hipMemsetAsync(tab, 0xff, H * 12 + m / 4, c.stream));
                    const dim3 grid((unsigned)((C + 255) / 256));
                    tstart(c, "gen_total_first");
                    hipLaunchKernelGGL(k_first_filter, grid, dim3(256), 0, c.stream, r, C, (uint32_t)nt, bm, m - 1);
                    hipLaunchKernelGGL(k_first_resolve, grid, dim3(256), 0, c.stream, r, C, (uint32_t)nt,
                                       (const uint32_t*)bm, m - 1, tab, minidx, H - 1, first);
                    tstop(c);
                    HIPCHK(hipGetLastError());
                    // the pending candidates are settled by the counting pass below; the block
                    // is released after it
                    pend = PendingTab{tab, minidx, H - 1, first};
                } else if (!cl.multapses) {
                    uint64_t* k0 = dalloc_n<uint64_t>(c, C);
                    uint64_t* k1 = dalloc_n<uint64_t>(c, C);
                    uint32_t* v0 = dalloc_n<uint32_t>(c, C);
                    uint32_t* v1 = dalloc_n<uint32_t>(c, C);
                    first = dalloc_n<uint8_t>(c, C);
                    temps.insert(temps.end(), {k0, k1, v0, v1, first});
                    tstart(c, "gen_total_keys");
                    hipLaunchKernelGGL(k_total_keys, dim3((unsigned)((C + 255) / 256)), dim3(256), 0, c.stream, r, C,
                                       (uint32_t)nt, k0, v0);
                    tstop(c);
                    HIPCHK(hipGetLastError());
                    uint32_t bits = 0;
                    while (bits < 64 && (ns * nt - 1) >> bits) ++bits;
                    // every pass runs (no wait for the digit histograms): the pair keys are random
                    c.sort_tag = "gen_total_sort";
                    int which = 0;
                    try {
                        which = radix_sort(c, k0, v0, k1, v1, C, 0, bits, nullptr, nullptr, false);
                    } catch (...) {
                        c.sort_tag = nullptr;
                        throw;
                    }
                    c.sort_tag = nullptr;
                    tstart(c, "gen_total_first");
                    hipLaunchKernelGGL(k_first_flags, dim3((unsigned)((C + 255) / 256)), dim3(256), 0, c.stream,
                                       which ? k1 : k0, which ? v1 : v0, C, first);
                    tstop(c);
                    HIPCHK(hipGetLastError());
                    dfree(c, k0); dfree(c, k1); dfree(c, v0); dfree(c, v1);
                    temps.resize(temps.size() - 5);
                    temps.push_back(first);
                }
                Total rr = r;
                rr.first = first;
                uint32_t* cnt = dalloc_n<uint32_t>(c, tiles);
                temps.push_back(cnt);
                const bool counted = voff != nullptr;
                if (!counted) {
                    voff = dalloc_n<uint64_t>(c, tiles + 1);
                    temps.push_back(voff);
                    launch_total_dist<WriteSink, CNT_VALID, true>(c, rr, host, ws, C, cnt, nullptr, nullptr, 0, pend);
                }
                if (pend.tab) {   // released in stream order, after the counting pass
                    void* blk = const_cast<uint64_t*>(pend.tab);
                    dfree(c, blk);
                    temps.erase(std::remove(temps.begin(), temps.end(), blk), temps.end());
                    pend = PendingTab{};
                }
                if (deferred) {
                    // batched admission: valid candidates of this window (and the kept ones) go to
                    // the caller's mapped words; a window with fewer than N valid candidates is
                    // counted again, without deferral, when the batch is admitted
                    if (!counted && all_local) {   // queued with the batch's scans
                        temps.erase(std::remove(temps.begin(), temps.end(), (void*)cnt), temps.end());
                        scan_u32_u64_later(c, cnt, voff, tiles, c.defer_slot);
                        cnt = nullptr;
                    } else if (!counted) {
                        scan_u32_u64_to(c, cnt, voff, tiles, c.defer_slot);
                    }
                    uint64_t* koff = nullptr;
                    if (!all_local) {
                        koff = dalloc_n<uint64_t>(c, tiles + 1);
                        launch_total_dist<WriteSink, CNT_KEEP, false>(c, rr, host, ws, C, cnt, voff, nullptr, N);
                        scan_u32_u64_to(c, cnt, koff, tiles, c.defer_slot + 1);
                    }
                    release_pre(c, cl);
                    cl.pre_off = voff;
                    cl.pre_koff = koff;
                    cl.pre_first = first;
                    cl.pre_window = C;
                    cl.deferred = all_local ? 2 : 3;
                    temps.erase(std::remove_if(temps.begin(), temps.end(),
                                               [&](void* q) { return q == voff || q == first; }),
                                temps.end());
                    break;
                }
                uint64_t valid;
                if (counted) {   // the small-window launch wrote the total to the lane's mapped word
                    sync(c);
                    valid = *reinterpret_cast<volatile uint64_t*>(c.tot_pin + (c.stream == c.count_stream ? 1 : 0));
                } else {
                    valid = scan_u32_u64(c, cnt, voff, tiles, true);
                }
                if (valid >= N) {
                    uint64_t kept = N;
                    uint64_t* koff = nullptr;
                    if (!all_local) {
                        koff = dalloc_n<uint64_t>(c, tiles + 1);
                        temps.push_back(koff);
                        launch_total_dist<WriteSink, CNT_KEEP, false>(c, rr, host, ws, C, cnt, voff, nullptr, N);
                        kept = scan_u32_u64(c, cnt, koff, tiles, true);
                    }
                    result = kept;
                    if (mode == Out::COUNT) {
                        // keep the window, flags and offsets for the generation
                        release_pre(c, cl);
                        cl.pre_off = voff;
                        cl.pre_koff = koff;
                        cl.pre_first = first;
                        cl.pre_window = C;
                        cl.pre_count = kept;
                        temps.erase(std::remove_if(temps.begin(), temps.end(),
                                                   [&](void* q) { return q == voff || q == koff || q == first; }),
                                    temps.end());
                    }
                    if (mark) {
                        if (all_local) launch_total_dist<MarkSink, MARK_KEEP, true>(c, rr, host, ms, C, nullptr, voff, nullptr, N);
                        else launch_total_dist<MarkSink, MARK_KEEP, false>(c, rr, host, ms, C, nullptr, voff, nullptr, N);
                    } else {
                        WriteSink* sink = reserve(kept);
                        if (kept) {
                            if (all_local)
                                launch_total_dist<WriteSink, WRITE_KEEP, true>(c, rr, host, *sink, C, nullptr, voff, koff, N);
                            else
                                launch_total_dist<WriteSink, WRITE_KEEP, false>(c, rr, host, *sink, C, nullptr, voff, koff, N);
                        }
                    }
                    break;
                }
                dfree(c, cnt);
                dfree(c, voff);
                temps.resize(temps.size() - 2);
                if (first) {
                    dfree(c, first);
                    temps.pop_back();
                }
                if (C >= 4000000000ull) raise(SNNC_EUNSUPPORTED, "total number needs more than 4e9 candidates");
                C = std::min<uint64_t>(C * 2, 4000000000ull);
            }
            break;
        }
        case SNNC_PAIRWISE_BERNOULLI: {
            if (!ns || !nt) break;
            const uint32_t nb = (uint32_t)((ns + 3) / 4 + 1);
            auto runs = unit_runs(cl.T, cl.autapses ? nullptr : &cl.S, host, nb, MAX_RUN_ELEMS);
            const uint64_t items = runs_elems(runs, nb);
            if (!items) break;
            DeviceChunks dc = upload_chunks(c, runs, items);
            temps.push_back(dc.d);
            const uint64_t thr = cl.p >= 1.0 ? (1ull << 32) : (uint64_t)std::floor(cl.p * 4294967296.0);
            BernPair r{dc.tab, nb, make_fastdiv(nb), (uint32_t)ns, thr, cl.autapses ? 1u : 0u, c.seed, cl.id};
            if (mark) {
                launch_bern<MarkSink, MARK>(c, r, ms, items, nullptr, nullptr);
                break;
            }
            const uint64_t tiles = (items + TILE - 1) / TILE;
            uint64_t* off = nullptr;
            uint8_t* masks = nullptr;   // the counting pass's item masks, read by the writing pass
            if (cl.pre_off && mode != Out::COUNT) {
                // counted at admission: the tile offsets and item masks are kept with the call
                off = cl.pre_off;
                masks = cl.pre_first;
                result = cl.pre_count;
                cl.pre_off = nullptr;
                cl.pre_first = nullptr;
                temps.push_back(off);
                temps.push_back(masks);
            } else {
                uint32_t* cnt = dalloc_n<uint32_t>(c, tiles);
                temps.push_back(cnt);
                off = dalloc_n<uint64_t>(c, tiles + 1);
                if (c.bern_masks) masks = dalloc_n<uint8_t>(c, items);
                launch_bern<WriteSink, COUNT>(c, r, ws, items, cnt, nullptr, masks);
                if (mode == Out::COUNT && c.defer_slot) {
                    // batched admission: the total goes to the caller's mapped word, read after one
                    // wait for the whole batch (the scan queued with the batch's others); the tile
                    // offsets and masks stay with the call
                    temps.erase(std::remove(temps.begin(), temps.end(), (void*)cnt), temps.end());
                    scan_u32_u64_later(c, cnt, off, tiles, c.defer_slot);
                    release_pre(c, cl);
                    cl.pre_off = off;
                    cl.pre_first = masks;
                    cl.deferred = 1;
                    break;
                }
                result = scan_u32_u64(c, cnt, off, tiles, true);
                if (mode == Out::COUNT) {
                    release_pre(c, cl);
                    cl.pre_off = off;
                    cl.pre_first = masks;
                    cl.pre_count = result;
                } else {
                    temps.push_back(off);
                    temps.push_back(masks);
                }
            }
            WriteSink* sink = reserve(result);
            if (result) launch_bern<WriteSink, WRITE>(c, r, *sink, items, nullptr, off, masks);
            break;
        }
        case SNNC_ONE_TO_ONE: {
            auto runs = unit_runs(cl.T, cl.autapses ? nullptr : &cl.S, host, 1, MAX_RUN_ELEMS);
            // a run is all autapses (its self position is its target ordinal) or none:
            // drop those runs on the host, so the count is known and one launch writes
            // element g of the kept runs at position g
            std::vector<TChunk> kept;
            uint64_t items = 0;
            for (const TChunk& ch : runs) {
                if (!cl.autapses && ch.self_base >= 0 && (uint64_t)ch.self_base == ch.t_ord) continue;
                TChunk k = ch;
                k.out_begin = items;
                items += ch.n;
                kept.push_back(k);
            }
            result = items;
            if (!items) {
                if (!mark) reserve(0);
                break;
            }
            if (mode == Out::COUNT) break;
            DeviceChunks dc = upload_chunks(c, kept, items);
            temps.push_back(dc.d);
            OneToOne r{dc.tab, 1u};   // autapse runs are gone
            if (mark) launch_gen<OneToOne, MarkSink, MARK>(c, "gen_one_to_one", r, ms, items, nullptr, nullptr, 0);
            else launch_gen<OneToOne, WriteSink, DIRECT>(c, "gen_one_to_one", r, *reserve(items), items, nullptr, nullptr, 0);
            break;
        }
        case SNNC_ASSIGNED_NODES: {
            const uint64_t n = cl.n;
            if (!n) break;
            uint64_t on_host = 0;
            for (auto& g : cl.T.seg) if (g.host == host) on_host += g.n;
            if (!on_host && !mark) break;
            Assigned r{cl.pairs, cl.pairs + n, cl.dT, nT, host};
            if (mark) {
                launch_gen<Assigned, MarkSink, MARK>(c, "gen_assigned", r, ms, n, nullptr, nullptr, 0);
            } else if (on_host == nt) {      // every target here: every pair is kept
                result = n;
                if (mode == Out::COUNT) break;
                launch_gen<Assigned, WriteSink, DIRECT>(c, "gen_assigned", r, *reserve(n), n, nullptr, nullptr, 0);
            } else {
                result = count_and_write<Assigned>(c, "gen_assigned", r, reserve, n, UINT64_MAX);
            }
            break;
        }
        default:
            raise(SNNC_EINVAL, "unknown rule");
        }
    } catch (const CountOnly& co) {
        cleanup();
        return co.n;
    } catch (...) {
        cleanup();
        throw;
    }
    // buffers are released in stream order: later work on the stream may reuse them
    cleanup();
    if (mode == Out::COUNT) return result;
    return result;
}

// ------------------------------------------------------------------ fused batches
// Many small calls whose connections are written one per element (no count
// depends on the draws) run as one persistent launch: a descriptor per call
// gives its item range in the batch and its rule parameters; every item finds
// its call by binary search and is generated exactly as in the per-call
// kernel, at the position the call was admitted to.
// F_SYN_FILL: the synapse values of a Floyd call (its sources and targets
// written by its own launch), element index from the run table as in
// k_syn_fill; `ind` holds the run table and K.
// F_FLOYD_SMALL: the sources and targets of a Floyd call of degree up to
// FLOYD_SMALL, one item per unit (`fl` holds the sampler's arguments).
enum FusedKind : uint32_t {
    F_INDEGREE = 0, F_TOTAL = 1, F_OUTDEGREE = 2, F_ONE_TO_ONE = 3, F_SYN_FILL = 4, F_FLOYD_SMALL = 5
};

struct FusedReq {
    uint64_t item_begin;
    uint64_t out_base;
    uint32_t kind, call;
    SynD syn;
    InDegree ind;
    OutDegree outd;
    Total tot;
    OneToOne o2o;
    FloydArgs fl;
};

struct FusedHdr {
    uint64_t n_req, total;
    uint32_t* src;
    uint32_t* tgt;
    uint16_t* delay;
    float* weight;
    uint32_t seed;
};

// During a batch flush, a Floyd call whose run table travels inline leaves
// its synapse values to the batch's fused launch (a descriptor whose
// item_begin holds the element count until the flush places it).
bool defer_syn_fill(Ctx& c, const FloydArgs& a, const WriteSink& ws, uint64_t items) {
    if (!c.gen_defer || a.ch.d) return false;
    FusedReq q;
    memset(&q, 0, sizeof q);
    q.kind = F_SYN_FILL;
    q.item_begin = items;
    q.out_base = ws.base;
    q.call = ws.call;
    q.syn = ws.syn;
    q.ind = InDegree{a.ch, a.K, make_fastdiv(a.K), 0u, ws.seed, ws.call};
    static_cast<std::vector<FusedReq>*>(c.gen_defer)->push_back(q);
    return true;
}

// During a batch flush, a Floyd call of degree up to FLOYD_SMALL whose run
// table travels inline leaves its sampling to the batch's fused launch (one
// item per unit; item_begin holds the unit count until the flush places it).
bool defer_floyd_small(Ctx& c, const FloydArgs& a, const WriteSink& ws) {
    if (!c.gen_defer || a.ch.d || !a.n_units) return false;
    FusedReq q;
    memset(&q, 0, sizeof q);
    q.kind = F_FLOYD_SMALL;
    q.item_begin = a.n_units;
    q.out_base = ws.base;
    q.call = ws.call;
    q.fl = a;
    static_cast<std::vector<FusedReq>*>(c.gen_defer)->push_back(q);
    return true;
}

// the descriptor holding item g among reqs[lo, hi) (g at or after reqs[lo])
__device__ __forceinline__ uint32_t find_req(const FusedReq* reqs, uint32_t lo, uint32_t hi, uint64_t g) {
    while (hi - lo > 1) {
        const uint32_t m = (lo + hi) >> 1;
        if (reqs[m].item_begin <= g) lo = m; else hi = m;
    }
    return lo;
}

// one item of the fused launch, generated by its call's descriptor q; fx is
// the thread's first slot of the small Floyd sampler's LDS values
__device__ __forceinline__ void fused_item(const FusedReq* __restrict__ q, const FusedHdr& h, uint64_t item,
                                           uint32_t* fx) {
    const uint64_t local = item - q->item_begin;
    if (q->kind == F_FLOYD_SMALL) {
        const IdSink ids{h.src, h.tgt, q->out_base};
        floyd_small_unit<IdSink, DIRECT>(q->fl, local, fx, NT, ids, nullptr, nullptr);
        return;
    }
    if (q->kind == F_SYN_FILL) {
        const TChunk ck = q->ind.ch.at(local);
        const uint64_t off = local - ck.out_begin;
        const uint32_t rel = fastdiv((uint32_t)off, q->ind.fk);   // a run holds fewer than 2^32 elements
        const uint32_t j = (uint32_t)off - rel * q->ind.K;
        float w;
        uint16_t d;
        syn_values(q->syn, h.seed, q->call, (ck.t_ord + rel) * (uint64_t)q->ind.K + j, w, d);
        h.delay[q->out_base + local] = d;
        h.weight[q->out_base + local] = w;
        return;
    }
    Res r[1];
    int n = 0;
    switch (q->kind) {
    case F_INDEGREE: n = q->ind.eval(local, r); break;
    case F_TOTAL: n = q->tot.eval(local, r); break;
    case F_OUTDEGREE: n = q->outd.eval(local, r); break;
    default: n = q->o2o.eval(local, r); break;
    }
    if (n) {
        const WriteSink ws{h.src, h.tgt, h.delay, h.weight, q->out_base, q->syn, h.seed, q->call};
        ws.put(local, r[0]);
    }
}

__global__ __launch_bounds__(NT) void k_fused(const FusedReq* __restrict__ reqs, const FusedHdr* __restrict__ hdr) {
    static_assert(NT == FNT, "the small Floyd sampler's LDS layout");
    __shared__ uint32_t s_range[2];
    __shared__ uint32_t fx[FLOYD_SMALL * NT];
    uint32_t* const my_fx = fx + threadIdx.x;
    const FusedHdr h = *hdr;
    for (uint64_t tile = blockIdx.x; tile * TILE < h.total; tile += gridDim.x) {
        // the descriptors of the tile's first and last items, found once: the
        // items' own searches then run over that range only
        if (threadIdx.x == 0) {
            const uint64_t first = tile * TILE, last = min(first + TILE, h.total) - 1;
            const uint32_t lo = find_req(reqs, 0, (uint32_t)h.n_req, first);
            s_range[0] = lo;
            s_range[1] = find_req(reqs, lo, (uint32_t)h.n_req, last) + 1;
        }
        __syncthreads();
        const uint32_t r_lo = __builtin_amdgcn_readfirstlane(s_range[0]);
        const uint32_t r_hi = __builtin_amdgcn_readfirstlane(s_range[1]);
        __syncthreads();   // read before thread 0 writes the next tile's range
        if (r_hi - r_lo == 1) {
            // the usual case, one call for the whole tile: its descriptor is
            // the same for every lane (scalar loads, uniform branches)
            const FusedReq* q = reqs + r_lo;
#pragma unroll 1
            for (int it = 0; it < IPT; ++it) {
                const uint64_t item = tile * TILE + (uint64_t)it * NT + threadIdx.x;
                if (item < h.total) fused_item(q, h, item, my_fx);
            }
        } else {
#pragma unroll 1
            for (int it = 0; it < IPT; ++it) {
                const uint64_t item = tile * TILE + (uint64_t)it * NT + threadIdx.x;
                if (item < h.total) fused_item(reqs + find_req(reqs, r_lo, r_hi, item), h, item, my_fx);
            }
        }
    }
}

// Descriptor of a call for the fused launch, or false if the call needs its
// own launches (counting passes, Floyd's sampling, restricted total number).
// The call's chunk table is appended to `chunks` (all tables of a batch go to
// the device in one block); the descriptor's table pointer is set by the
// caller once that block exists (`*chunk_at` = first entry in `chunks`).
// A fused call's run table: inline when short, else appended to the batch's
// table (*chunk_at = its first entry; the device address is set after the
// batch's one upload).
ChunkTab batch_tab(const std::vector<TChunk>& runs, std::vector<TChunk>& chunks, size_t* chunk_at) {
    ChunkTab t{};
    t.n = (uint32_t)runs.size();
    if (runs.size() <= CH_INLINE) {
        std::copy(runs.begin(), runs.end(), t.in);
    } else {
        *chunk_at = chunks.size();
        chunks.insert(chunks.end(), runs.begin(), runs.end());
    }
    return t;
}

bool fused_desc(Ctx& c, Call& cl, FusedReq& q, std::vector<TChunk>& chunks, size_t* chunk_at) {
    const uint32_t host = c.P_local;
    const uint32_t nS = (uint32_t)cl.S.seg.size(), nT = (uint32_t)cl.T.seg.size();
    const uint64_t ns = cl.S.total, nt = cl.T.total;
    memset(&q, 0, sizeof q);
    q.out_base = cl.gen_begin;
    q.call = cl.id;
    q.syn = syn_of(cl);
    if (!cl.gen_count) return false;
    switch (cl.rule) {
    case SNNC_FIXED_INDEGREE: {
        if (!cl.multapses) return false;
        const uint64_t K = cl.n;
        auto runs = unit_runs(cl.T, cl.autapses ? nullptr : &cl.S, host, K, MAX_RUN_ELEMS);
        q.kind = F_INDEGREE;
        q.ind = InDegree{batch_tab(runs, chunks, chunk_at), (uint32_t)K, make_fastdiv((uint32_t)K), (uint32_t)ns,
                         c.seed, cl.id};
        return true;
    }
    case SNNC_FIXED_OUTDEGREE: {
        if (!cl.multapses) return false;
        uint64_t on_host = 0;
        for (auto& g : cl.T.seg) if (g.host == host) on_host += g.n;
        if (on_host != nt) return false;
        const uint64_t K = cl.n;
        auto runs = unit_runs(cl.S, cl.autapses ? nullptr : &cl.T, -1, K, MAX_RUN_ELEMS);
        q.kind = F_OUTDEGREE;
        q.outd = OutDegree{batch_tab(runs, chunks, chunk_at), (uint32_t)K, make_fastdiv((uint32_t)K), (uint32_t)nt,
                           cl.dT, nT, host, c.seed, cl.id};
        return true;
    }
    case SNNC_FIXED_TOTAL_NUMBER: {
        if (!cl.autapses || !cl.multapses) return false;
        uint64_t on_host = 0;
        for (auto& g : cl.T.seg) if (g.host == host) on_host += g.n;
        if (on_host != nt) return false;   // targets on several hosts: candidates are filtered
        q.kind = F_TOTAL;
        q.tot = Total{cl.dS, nS, cl.dT, nT, (uint32_t)ns, (uint32_t)nt, 1u, nullptr, c.seed, cl.id};
        return true;
    }
    case SNNC_ONE_TO_ONE: {
        auto runs = unit_runs(cl.T, cl.autapses ? nullptr : &cl.S, host, 1, MAX_RUN_ELEMS);
        std::vector<TChunk> kept;   // runs that are all autapses are dropped (as in run_call)
        uint64_t items = 0;
        for (const TChunk& ch : runs) {
            if (!cl.autapses && ch.self_base >= 0 && (uint64_t)ch.self_base == ch.t_ord) continue;
            TChunk k = ch;
            k.out_begin = items;
            items += ch.n;
            kept.push_back(k);
        }
        if (items != cl.gen_count) return false;
        q.kind = F_ONE_TO_ONE;
        q.o2o = OneToOne{batch_tab(kept, chunks, chunk_at), 1u};   // autapse runs are gone
        return true;
    }
    default:
        return false;
    }
}

__global__ void k_philox_blocks(uint32_t seed, uint32_t call, uint64_t e0, uint32_t purpose, uint64_t n, uint4* out) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = draw(seed, call, e0 + i, purpose);
}

}  // namespace

uint64_t gen_local(Ctx& c, Call& cl) { return run_call(c, cl, c.P_local, Out::APPEND, nullptr); }

void first_small_batch_run(Ctx& c) {
    if (c.first_jobs.empty()) return;
    const size_t bytes = c.first_jobs.size();
    const unsigned n = (unsigned)(bytes / sizeof(FirstSmallJob));
    void* dev = dalloc(c, bytes);
    try {
        upload(c, dev, c.first_jobs.data(), bytes);
    } catch (...) {
        dfree(c, dev);
        throw;
    }
    c.first_jobs.clear();
    tstart(c, "gen_total_first");
    hipLaunchKernelGGL(k_first_small_multi, dim3(n), dim3(FS_NT), 0, c.stream, static_cast<const FirstSmallJob*>(dev));
    tstop(c);
    const hipError_t e = hipGetLastError();
    dfree(c, dev);   // in stream order, after the launch
    HIPCHK(e);
}

uint64_t gen_count_local(Ctx& c, Call& cl) { return run_call(c, cl, c.P_local, Out::COUNT, nullptr); }

// Whether counting the call's local connections launches device work (the
// counting branches of run_call): Bernoulli draws, total number unless every
// candidate is kept, out-degree and assigned pairs with targets on other hosts.
bool count_on_device(const Ctx& c, const Call& cl) {
    uint64_t on_host = 0;
    for (auto& g : cl.T.seg) if (g.host == c.P_local) on_host += g.n;
    const bool all_local = on_host == cl.T.total;
    switch (cl.rule) {
    case SNNC_PAIRWISE_BERNOULLI: return cl.S.total && cl.T.total;
    case SNNC_FIXED_TOTAL_NUMBER: return cl.n && on_host && !(cl.autapses && cl.multapses && all_local);
    case SNNC_FIXED_OUTDEGREE: return cl.n && cl.T.total && !all_local;
    case SNNC_ASSIGNED_NODES: return cl.n && on_host && !all_local;
    default: return false;
    }
}

void release_pre(Ctx& c, Call& cl) {
    dfree(c, cl.pre_off);
    dfree(c, cl.pre_koff);
    dfree(c, cl.pre_first);
    cl.pre_off = cl.pre_koff = nullptr;
    cl.pre_first = nullptr;
}

void gen_mark(Ctx& c, Call& cl, uint32_t host, uint32_t* bits) { run_call(c, cl, host, Out::MARK, bits); }

// One batch of admitted calls: the fusable ones in one persistent launch
// (replayed from a captured graph), the others with their own launches, all
// writing at their admitted positions.  Records the batch's completion event.
void flush_batch(Ctx& c, const std::vector<uint32_t>& ids, hipEvent_t done) {
    std::vector<FusedReq> reqs;
    std::vector<size_t> chunk_at;
    std::vector<TChunk> chunks;
    std::vector<uint32_t> rest;
    uint64_t total = 0;
    uint32_t first_fused = UINT32_MAX;
    for (uint32_t id : ids) {
        Call& cl = c.calls[id];
        FusedReq q;
        size_t at = SIZE_MAX;
        if (!cl.gen_count) {           // nothing to generate on this host
            release_pre(c, cl);
            continue;
        }
        if (c.fuse_batches && fused_desc(c, cl, q, chunks, &at)) {
            q.item_begin = total;
            total += cl.gen_count;
            reqs.push_back(q);
            chunk_at.push_back(at);
            if (first_fused == UINT32_MAX) first_fused = id;
        } else if (cl.gen_count) {
            rest.push_back(id);
        }
    }
    // the other calls with their own launches; Floyd calls among them leave
    // their synapse values to the fused launch below
    std::vector<FusedReq> deferred;
    c.gen_defer = &deferred;
    try {
        for (uint32_t id : rest) run_call(c, c.calls[id], c.P_local, Out::AT_BASE, nullptr);
    } catch (...) {
        c.gen_defer = nullptr;
        throw;
    }
    c.gen_defer = nullptr;
    for (FusedReq& q : deferred) {
        const uint64_t items = q.item_begin;
        q.item_begin = total;
        total += items;
        reqs.push_back(q);
        chunk_at.push_back(SIZE_MAX);
    }
    if (!chunks.empty()) {
        // the chunk tables of every fused call: one block, one copy (kept until Prepare)
        TChunk* dev = dalloc_n<TChunk>(c, chunks.size());
        c.calls[first_fused].owned.push_back(dev);
        upload(c, dev, chunks.data(), chunks.size() * sizeof(TChunk));
        for (size_t k = 0; k < reqs.size(); ++k) {
            if (chunk_at[k] == SIZE_MAX) continue;
            TChunk* t = dev + chunk_at[k];
            switch (reqs[k].kind) {
            case F_INDEGREE: reqs[k].ind.ch.d = t; break;
            case F_OUTDEGREE: reqs[k].outd.ch.d = t; break;
            case F_ONE_TO_ONE: reqs[k].o2o.ch.d = t; break;
            default: break;
            }
        }
    }
    if (!reqs.empty()) {
        // device descriptor table and header at fixed addresses, so that one
        // captured graph serves every batch
        if (c.fused_cap < reqs.size() || !c.fused_exec) {
            if (c.fused_exec) HIPCHK(hipGraphExecDestroy(c.fused_exec));
            c.fused_exec = nullptr;
            dfree(c, c.fused_reqs);
            dfree(c, c.fused_hdr);
            c.fused_cap = std::max<size_t>(reqs.size() * 2, 256);
            c.fused_reqs = dalloc(c, c.fused_cap * sizeof(FusedReq));
            c.fused_hdr = dalloc(c, sizeof(FusedHdr));
            if (!c.capture_stream) HIPCHK(hipStreamCreateWithFlags(&c.capture_stream, hipStreamNonBlocking));
            int cus = 256;
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c.device);
            const unsigned grid = (unsigned)std::max(1, cus * c.fused_wgs_per_cu);
            hipGraph_t g;
            HIPCHK(hipStreamBeginCapture(c.capture_stream, hipStreamCaptureModeRelaxed));
            hipLaunchKernelGGL(k_fused, dim3(grid), dim3(NT), 0, c.capture_stream,
                               static_cast<const FusedReq*>(c.fused_reqs), static_cast<const FusedHdr*>(c.fused_hdr));
            HIPCHK(hipStreamEndCapture(c.capture_stream, &g));
            HIPCHK(hipGraphInstantiate(&c.fused_exec, g, nullptr, nullptr, 0));
            HIPCHK(hipGraphDestroy(g));
        }
        FusedHdr h{reqs.size(), total, c.g_src, c.g_tgt, c.g_delay, c.g_weight, c.seed};
        upload(c, c.fused_reqs, reqs.data(), reqs.size() * sizeof(FusedReq));
        upload(c, c.fused_hdr, &h, sizeof h);
        tstart(c, "gen_fused");
        HIPCHK(hipGraphLaunch(c.fused_exec, c.stream));
        tstop(c);
    }
    HIPCHK(hipEventRecord(done, c.stream));
}

std::vector<TChunk> target_chunks(const Call& cl, uint32_t host, uint64_t K, uint64_t max_elems) {
    return unit_runs(cl.T, cl.autapses ? nullptr : &cl.S, host, K, max_elems);
}

}  // namespace snnc

extern "C" snnc_status snnc_philox_blocks(snnc_ctx* ctx, uint32_t seed, uint32_t call_id, uint64_t e_begin,
                                          uint32_t purpose, uint64_t n, uint32_t* out) {
    using namespace snnc;
    Ctx* c = ctx;
    if (!c || (!out && n)) return SNNC_EINVAL;
    try {
        HIPCHK(hipSetDevice(c->device));
        if (n) {
            hipLaunchKernelGGL(k_philox_blocks, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, seed,
                               call_id, e_begin, purpose, n, reinterpret_cast<uint4*>(out));
            HIPCHK(hipGetLastError());
            sync(*c);
        }
        return SNNC_OK;
    } catch (const Error& e) {
        c->last_error = e.msg;
        return e.code;
    }
}
