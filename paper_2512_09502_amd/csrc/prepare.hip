// Simulation preparation on the GPU:
//  1. build the 64-bit sort key of every connection, (source prefix, target,
//     delay), with the digit histograms of every radix pass in the same
//     read; the source prefix is the local id of a local source, and
//     M_local + (alpha+1) G + global id of a remote one (global id = host
//     base + local id), an order that agrees with (alpha+1, sigma, source);
//  2. source-major radix sort;
//  3. without remote sources the last pass unpacks the result arrays; with
//     them, one scan over the sorted keys numbers the images: the first
//     connection of every distinct remote prefix starts the next image after
//     the local neurons (the sorted-unique map R of every (alpha+1, sigma) and
//     the remap of the paper's flag/compact/sort/search/append steps in one
//     pass), and the same pass unpacks the arrays;
//  4. R, its per-(alpha+1, sigma) offsets and a bit set of the images;
//  5. first-index array from the sorted sources;
//  6. point-to-point send lists: regenerate alpha = -1 draws per target host,
//     bit rows of the local sources they use, their compaction (S) and the
//     per-source transpose (T/P);
//  7. collective arrays H, I, G/Q from the source ranges of each group.
#include <algorithm>
#include <numeric>

#include "device_common.h"
#include "internal.h"

namespace snnc {

namespace {

constexpr int PNT = 256;

struct CallD {
    uint64_t gen_begin;
    const SegD* S;
    uint32_t nS;
    uint32_t a;      // alpha + 1
    uint32_t order;  // position of the call in call order
    uint32_t flag;   // 1: only the sources its local connections use get images
    uint32_t uniform;   // 1: all source segments have the same length (segment = ordinal / length)
    FastDiv seg_div;
    const int64_t* seg_base;   // per segment: bit of its first neuron minus its first ordinal
    uint64_t local_lo;         // bit of P_local's neuron 0 in this call's map index
};

// segment lookup by division when every source segment of the call has the same length
CallD make_calld(const Call& cl, uint32_t order, uint32_t flag) {
    CallD d{cl.gen_begin, cl.dS, (uint32_t)cl.S.seg.size(), (uint32_t)(cl.alpha + 1), order, flag, 0, FastDiv{},
            nullptr, 0};
    const auto& seg = cl.S.seg;
    bool uniform = seg.size() > 1 && seg[0].n > 0 && cl.S.total < (1ull << 31);
    for (const auto& g : seg) uniform = uniform && g.n == seg[0].n;
    if (uniform) {
        d.uniform = 1;
        d.seg_div = make_fastdiv(seg[0].n);
    }
    return d;
}

struct Lookup {
    const CallD* calls;
    uint32_t ncalls;
    const uint64_t* host_base;   // [P + 1]
    uint32_t P, PL;
    uint64_t G;                  // neurons over all hosts
};

__device__ __forceinline__ uint32_t find_call(const CallD* calls, uint32_t n, uint64_t i) {
    uint32_t a = 0, b = n;
    while (b - a > 1) {
        const uint32_t m = (a + b) >> 1;
        if (calls[m].gen_begin <= i) a = m; else b = m;
    }
    return a;
}

// Source of connection i (host, local id and bit index (alpha+1) G + global
// id), with a per-thread cache of the current call and source segment:
// a thread walks increasing positions, so the binary searches run only when
// the position leaves the cached call or the ordinal leaves the cached segment.
struct SourceCursor {
    uint64_t call_lo = 1, call_hi = 0;   // cached call covers [call_lo, call_hi)
    CallD call{};
    uint64_t seg_lo = 1, seg_hi = 0;     // cached segment covers ordinals [seg_lo, seg_hi)
    uint32_t seg_host = 0, seg_first = 0;
    uint64_t bit_base = 0;               // a G + host_base[seg_host] + seg_first - seg_lo

    __device__ __forceinline__ const CallD& call_at(const Lookup& L, uint64_t i) {
        if (i < call_lo || i >= call_hi) {
            const uint32_t k = find_call(L.calls, L.ncalls, i);
            call = L.calls[k];
            call_lo = call.gen_begin;
            call_hi = k + 1 < L.ncalls ? L.calls[k + 1].gen_begin : ~0ull;
            seg_lo = 1;
            seg_hi = 0;
        }
        return call;
    }

    __device__ __forceinline__ void at(const Lookup& L, uint64_t i, uint32_t ord, uint32_t& host, uint32_t& local,
                                       uint64_t& bit) {
        call_at(L, i);
        if (ord < seg_lo || ord >= seg_hi) {
            uint32_t a = 0, b = call.nS;
            if (call.uniform) {
                a = fastdiv(ord, call.seg_div);
            } else {
                while (b - a > 1) {
                    const uint32_t m = (a + b) >> 1;
                    if (call.S[m].ord_begin <= ord) a = m; else b = m;
                }
            }
            const SegD s = call.S[a];
            seg_lo = s.ord_begin;
            seg_hi = a + 1 < call.nS ? call.S[a + 1].ord_begin : ~0ull;
            seg_host = s.host;
            seg_first = s.first;
            bit_base = (uint64_t)call.a * L.G + L.host_base[s.host] + s.first - s.ord_begin;
        }
        host = seg_host;
        local = seg_first + (uint32_t)(ord - seg_lo);
        bit = bit_base + ord;
    }
};

// contiguous range of positions for workgroup b of g over n (multiple of the block size)
__device__ __forceinline__ void block_range(uint64_t n, uint64_t& lo, uint64_t& hi) {
    const uint64_t per = ((n + gridDim.x - 1) / gridDim.x + PNT - 1) / PNT * PNT;
    lo = (uint64_t)blockIdx.x * per;
    hi = lo + per < n ? lo + per : n;
}

__device__ __forceinline__ uint64_t rank_of(const uint32_t* bits, const uint64_t* word_rank, uint64_t bit) {
    const uint64_t w = bit >> 5;
    return word_rank[w] + (uint64_t)__popc(bits[w] & ((1u << (bit & 31)) - 1u));
}

// source' and the sort key (source' << tgt_shift | target << 16 | delay),
// with the digit histograms of all radix passes
__global__ __launch_bounds__(PNT) void k_keys(Lookup L, const uint32_t* g_src, const uint32_t* g_tgt,
                                              const uint16_t* g_delay, uint64_t n, const uint32_t* bits,
                                              const uint64_t* word_rank, const int32_t* Lmap, uint32_t M_local,
                                              uint32_t tgt_shift, uint32_t n9,
                                              uint32_t dbits, uint32_t passes, uint64_t* keys, uint64_t* hist) {
    __shared__ uint32_t h[8 * HIST_STRIDE];
    for (uint32_t i = threadIdx.x; i < passes * HIST_STRIDE; i += PNT) h[i] = 0;
    __syncthreads();
    uint64_t lo, hi;
    block_range(n, lo, hi);
    // call of the current window (a workgroup's range crosses few calls)
    uint64_t call_lo = 1, call_hi = 0;
    CallD cd{};
    uint32_t last_sidx = ~0u;   // segment whose base is cached (single-segment calls load it once)
    int64_t last_base = 0;
    constexpr int KU = 4;   // independent elements per thread per step: their table loads overlap
    for (uint64_t base = lo; base < hi; base += (uint64_t)PNT * KU) {
        uint32_t ord[KU], tg[KU];
        uint16_t dl[KU];
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            const uint64_t i = base + (uint64_t)u * PNT + threadIdx.x;
            if (i < hi) {
                ord[u] = g_src[i];
                tg[u] = g_tgt[i];
                dl[u] = g_delay[i];
            }
        }
        uint64_t key[KU];
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            const uint64_t i = base + (uint64_t)u * PNT + threadIdx.x;
            key[u] = 0;
            if (i >= hi) continue;
            if (i < call_lo || i >= call_hi) {
                const uint32_t k = find_call(L.calls, L.ncalls, i);
                cd = L.calls[k];
                call_lo = cd.gen_begin;
                call_hi = k + 1 < L.ncalls ? L.calls[k + 1].gen_begin : ~0ull;
                last_sidx = ~0u;
            }
            uint32_t sidx;
            if (cd.uniform) {
                sidx = fastdiv(ord[u], cd.seg_div);
            } else {
                uint32_t a = 0, b = cd.nS;
                while (b - a > 1) {
                    const uint32_t m = (a + b) >> 1;
                    if (cd.S[m].ord_begin <= ord[u]) a = m; else b = m;
                }
                sidx = a;
            }
            if (sidx != last_sidx) {
                last_base = cd.seg_base[sidx];
                last_sidx = sidx;
            }
            const uint64_t bit = (uint64_t)(last_base + (int64_t)ord[u]);
            const uint64_t rel = bit - cd.local_lo;   // the local neuron, when below M_local
            // remote sources: the image index L when the images were numbered before the sort,
            // else the global prefix M_local + bit (images are numbered after the sort)
            const uint64_t src2 = rel < M_local ? rel
                                  : bits        ? (uint64_t)Lmap[rank_of(bits, word_rank, bit)]
                                                : (uint64_t)M_local + bit;
            key[u] = (src2 << tgt_shift) | ((uint64_t)tg[u] << 16) | dl[u];
            keys[i] = key[u];
        }
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            const bool valid = base + (uint64_t)u * PNT + threadIdx.x < hi;
            for (uint32_t p = 0; p < passes; ++p)   // bits above the key's top are zero
                wave_hist_add(&h[p * HIST_STRIDE],
                              (uint32_t)((key[u] >> pass_shift(16, n9, dbits, p)) & ((p < n9 ? 0x1ffu : (1u << dbits) - 1))),
                              valid);
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < passes * HIST_STRIDE; i += PNT)
        if (h[i]) atomicAdd((unsigned long long*)&hist[i], (unsigned long long)h[i]);
}

// ---- image numbering after the sort (networks with remote sources)
// The keys were sorted with source prefix p = local id (local source) or
// M_local + (alpha+1) G + global id (remote source); both orders agree with
// (alpha+1, sigma, s).  One pass over the sorted keys numbers the images: the
// first key of every distinct remote prefix starts a new image, and a scan of
// these flags (decoupled look-back across tiles) gives each connection its
// image index.  The same pass unpacks the connection arrays, records each
// image's prefix and writes the first-index array.
// Tile shapes (threads, items per thread; whether the payload is loaded with
// the keys, before the look-back).  Measured on the 6.4e8- and 2.25e9-connection
// remote-source networks: larger tiles win (fewer look-back steps per element)
// and loading the payload early hides its latency behind the look-back; 1024
// threads x 10 items with the early payload is the fastest shape that does
// not spill (variant 10, the default).
struct NumberShape {
    int nt, ipt;
    bool early_vals;
};
constexpr NumberShape NUMBER_SHAPES[] = {{1024, 12, false}, {512, 12, false}, {256, 12, false},
                                         {512, 12, true},   {256, 12, true},  {256, 16, true},
                                         {256, 8, true},    {256, 6, true},   {512, 8, true},
                                         {1024, 12, true},  {1024, 10, true}, {1024, 8, true}};
constexpr int NUMBER_VARIANTS = (int)(sizeof(NUMBER_SHAPES) / sizeof(NUMBER_SHAPES[0]));
constexpr uint64_t XFLAG_AGG = 1ull << 62, XFLAG_INC = 2ull << 62, XVALUE = (1ull << 40) - 1;
constexpr uint32_t XEPOCH_MAX = (1u << 22) - 1;

template <int XNT, int XIPT, bool EARLY_VALS>
__global__ __launch_bounds__(XNT) void k_number(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ vals,
                                                uint64_t n, uint32_t tgt_shift, uint64_t tgt_mask, uint32_t M_local,
                                                uint64_t* lookback, uint32_t* tile_counter, uint32_t epoch,
                                                uint32_t* status, int32_t* o_src, int32_t* o_tgt, uint16_t* o_delay,
                                                float* o_weight, uint64_t* img_key, uint64_t* row_ptr,
                                                uint64_t* n_img_out) {
    __shared__ uint32_t s_tile;
    __shared__ uint64_t wave_tot[XNT / 64];
    __shared__ uint64_t s_excl;
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) s_tile = atomicAdd(tile_counter, 1u);
    __syncthreads();
    const uint64_t tile = s_tile;
    constexpr uint64_t XTILE = (uint64_t)XNT * XIPT;
    const uint64_t wbase = tile * XTILE + (uint64_t)wave * 64 * XIPT;
    // element of item k on this lane: wbase + k*64 + lane (wave-striped, so loads and stores coalesce);
    // the keys stay in registers for the second half (a reload would come from HBM again)
    uint64_t key[XIPT];
    uint32_t val[EARLY_VALS ? XIPT : 1];
    uint32_t incl[XIPT];          // flags up to and including the item, within the wave
    uint32_t fl = 0;              // bit k: item k starts a new image
    const uint64_t before_wave = wbase > 0 && wbase - 1 < n ? (keys[wbase - 1] >> tgt_shift) : ~0ull;
    uint64_t last = before_wave;  // prefix before the wave
    uint32_t carry = 0;
#pragma unroll
    for (int k = 0; k < XIPT; ++k) {
        const uint64_t i = wbase + (uint64_t)k * 64 + lane;
        key[k] = i < n ? keys[i] : ~0ull;
        if constexpr (EARLY_VALS) val[k] = i < n ? vals[i] : 0u;
        const uint64_t pk = i < n ? key[k] >> tgt_shift : ~0ull;
        uint64_t prev = __shfl_up(pk, 1, 64);
        const uint64_t last_lane = __shfl(pk, 63, 64);
        if (lane == 0) prev = last;
        last = last_lane;
        const uint32_t f = (i < n && pk >= M_local && (i == 0 || pk != prev)) ? 1u : 0u;
        fl |= f << k;
        const uint32_t s = wave_incl_scan(f);
        incl[k] = carry + s;
        carry += __shfl(s, 63, 64);
    }
    if (lane == 63) wave_tot[wave] = carry;
    __syncthreads();
    uint64_t wave_excl = 0, tile_tot = 0;
#pragma unroll
    for (int w = 0; w < XNT / 64; ++w) {
        if (w < (int)wave) wave_excl += wave_tot[w];
        tile_tot += wave_tot[w];
    }
    if (threadIdx.x == 0) {
        uint64_t* my = lookback + tile;
        uint64_t excl = 0;
        if (tile == 0) {
            __hip_atomic_store(my, XFLAG_INC | ((uint64_t)epoch << 40) | tile_tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(my, XFLAG_AGG | ((uint64_t)epoch << 40) | tile_tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            int64_t pred = (int64_t)tile - 1;
            uint32_t spins = 0;
            while (pred >= 0) {
                const uint64_t st = __hip_atomic_load(lookback + pred, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint64_t flag = st & (3ull << 62);
                if (flag != 0 && (uint32_t)((st >> 40) & XEPOCH_MAX) == epoch) {
                    excl += st & XVALUE;
                    if (flag == XFLAG_INC) break;
                    --pred;
                    continue;
                }
                if (++spins > (1u << 22) || __hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    atomicOr(status, 2u);   // bounded wait exceeded: flag the failure and finish the tile
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            __hip_atomic_store(my, XFLAG_INC | ((uint64_t)epoch << 40) | (excl + tile_tot), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        s_excl = excl;
    }
    __syncthreads();
    const uint64_t before = s_excl + wave_excl;   // images started before this wave
    last = before_wave;
#pragma unroll
    for (int k = 0; k < XIPT; ++k) {
        const uint64_t i = wbase + (uint64_t)k * 64 + lane;
        const uint64_t pk = key[k] >> tgt_shift;
        // prefix of the previous connection, again from the neighbouring lane
        uint64_t pp = __shfl_up(pk, 1, 64);
        const uint64_t last_lane = __shfl(pk, 63, 64);
        if (lane == 0) pp = last;
        last = last_lane;
        if (i >= n) continue;
        const uint64_t rank = before + incl[k];                 // images started up to and including i
        const bool local = pk < M_local;
        const int64_t src2 = local ? (int64_t)pk : (int64_t)(M_local + rank - 1);
        o_src[i] = (int32_t)src2;
        o_tgt[i] = (int32_t)((key[k] >> 16) & tgt_mask);
        o_delay[i] = (uint16_t)(key[k] & 0xffffu);
        if constexpr (EARLY_VALS) o_weight[i] = __uint_as_float(val[k]);
        else o_weight[i] = __uint_as_float(vals[i]);
        // previous connection's source' (its flag count is rank minus this item's flag)
        const bool flag_here = (fl >> k) & 1u;
        int64_t prev2 = -1;
        if (i > 0) prev2 = pp < M_local ? (int64_t)pp : (int64_t)(M_local + rank - (flag_here ? 1 : 0) - 1);
        if (flag_here) img_key[rank - 1] = pk - M_local;
        for (int64_t r = prev2 + 1; r <= src2; ++r) row_ptr[r] = i;
        if (i + 1 == n) {
            const int64_t n_rows = (int64_t)M_local + (int64_t)rank;
            for (int64_t r = src2 + 1; r <= n_rows; ++r) row_ptr[r] = n;
            *n_img_out = rank;
        }
    }
}

// R value and (alpha+1, sigma) boundaries from the image prefixes a G + gid.
// Each thread takes RV_RUN consecutive images (sorted): the map slot a and the
// host are found for the first and kept while the next ones stay inside them.
constexpr int RV_RUN = 8;

__global__ void k_rvals_sorted(const uint64_t* img_key, uint64_t n_img, const uint64_t* host_base, uint32_t P,
                               uint64_t G, int32_t* R) {
    const uint64_t j0 = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * RV_RUN;
    if (j0 >= n_img) return;
    const uint64_t j1 = j0 + RV_RUN < n_img ? j0 + RV_RUN : n_img;
    uint64_t base = 0;             // a G of the current slot
    uint64_t hlo = 1, hhi = 0;     // [host_base[h], host_base[h + 1]) of the current host (empty: none yet)
    for (uint64_t j = j0; j < j1; ++j) {
        const uint64_t key = img_key[j];
        if (key < base || key - base >= G) base = key / G * G;
        const uint64_t gid = key - base;
        if (gid < hlo || gid >= hhi) {
            uint32_t lo = 0, hi = P;
            while (hi - lo > 1) {
                const uint32_t m = (lo + hi) >> 1;
                if (host_base[m] <= gid) lo = m; else hi = m;
            }
            hlo = host_base[lo];
            hhi = host_base[lo + 1];
        }
        R[j] = (int32_t)(gid - hlo);
    }
}

__global__ void k_bounds_sorted(const uint64_t* img_key, uint64_t n_img, const uint64_t* host_base, uint32_t P,
                                uint32_t n_a, uint64_t G, uint32_t M_local, uint64_t* r_off, int64_t* img_base) {
    const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t nk = (uint64_t)n_a * P;
    if (k > nk) return;
    const uint64_t x = k == nk ? (uint64_t)n_a * G : (k / P) * G + host_base[k % P];
    uint64_t a = 0, b = n_img;   // lower_bound of x
    while (a < b) {
        const uint64_t m = (a + b) >> 1;
        if (img_key[m] < x) a = m + 1; else b = m;
    }
    r_off[k] = a;
    if (k < nk) img_base[k] = (int64_t)M_local + (int64_t)a;
}

// Bit of every image prefix (bits is zero before).  The prefixes are sorted,
// so the lanes of one word are contiguous in a wave: a segmented OR across
// them leaves the word's bits in its last lane, which sets them with one
// atomic (a word can continue in the next wave).
__global__ void k_bits_sorted(const uint64_t* img_key, uint64_t n_img, uint32_t* bits) {
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool valid = j < n_img;
    const uint64_t key = valid ? img_key[j] : ~0ull;
    const uint64_t w = key >> 5;
    uint32_t acc = valid ? 1u << (key & 31) : 0u;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t a = __shfl_up(acc, o, 64);
        const uint64_t wo = __shfl_up(w, o, 64);
        if (lane >= o && wo == w) acc |= a;
    }
    const uint64_t wn = __shfl_down(w, 1, 64);
    if (valid && (lane == 63 || wn != w)) atomicOr(bits + w, acc);
}

// ---- images numbered before the sort (map policies other than the default)
// fc[(alpha+1) G + gid] = first call (in call order) that gives the source an
// image; ~0 = none.  Flagged calls: the sources their local connections use.
__global__ __launch_bounds__(PNT) void k_first_use(Lookup L, const uint32_t* g_src, uint64_t n, uint32_t* fc) {
    uint64_t lo, hi;
    block_range(n, lo, hi);
    SourceCursor cur;
    for (uint64_t i = lo + threadIdx.x; i < hi; i += PNT) {
        if (!cur.call_at(L, i).flag) continue;
        uint32_t host, local;
        uint64_t bit;
        cur.at(L, i, g_src[i], host, local, bit);
        if (host == L.PL) continue;
        const uint32_t ord = cur.call.order;
        if (fc[bit] > ord) atomicMin(&fc[bit], ord);   // fc only decreases: a stale read never skips wrongly
    }
}

// Unflagged calls: every source passed to them (bit ranges, concatenated)
struct FRange {
    uint64_t begin;   // first position in the concatenation
    uint64_t bit;     // bit of the range's first source
    uint32_t order;   // call order
    uint32_t pad;
};

__global__ __launch_bounds__(PNT) void k_first_pass(const FRange* rg, uint32_t n_rg, uint64_t total, uint32_t* fc) {
    for (uint64_t j = (uint64_t)blockIdx.x * PNT + threadIdx.x; j < total; j += (uint64_t)gridDim.x * PNT) {
        uint32_t a = 0, b = n_rg;
        while (b - a > 1) {
            const uint32_t m = (a + b) >> 1;
            if (rg[m].begin <= j) a = m; else b = m;
        }
        const uint64_t bit = rg[a].bit + (j - rg[a].begin);
        const uint32_t ord = rg[a].order;
        if (fc[bit] > ord) atomicMin(&fc[bit], ord);
    }
}

// bit set of the sources with an image: one ballot per wave covers 64 bits
__global__ __launch_bounds__(PNT) void k_fc_bits(const uint32_t* fc, uint64_t n_bits, uint64_t n_words, uint32_t* bits) {
    for (uint64_t base = (uint64_t)blockIdx.x * PNT; base < n_bits; base += (uint64_t)gridDim.x * PNT) {
        const uint64_t b = base + threadIdx.x;   // the loop bound is uniform per workgroup: whole waves ballot
        const uint64_t m = __ballot(b < n_bits && fc[b] != ~0u);
        if ((threadIdx.x & 63) == 0) {
            const uint64_t w = (b >> 6) * 2;
            if (w < n_words) bits[w] = (uint32_t)m;
            if (w + 1 < n_words) bits[w + 1] = (uint32_t)(m >> 32);
        }
    }
}

// images in canonical order: R value, and (first call << 16, canonical index)
// pairs for the numbering in call order
__global__ __launch_bounds__(PNT) void k_img_list(const uint32_t* bits, const uint64_t* word_rank, uint64_t n_words,
                                                  const uint32_t* fc, const uint64_t* host_base, uint32_t P, uint64_t G,
                                                  int32_t* R, uint64_t* okey, uint32_t* oval) {
    for (uint64_t w = (uint64_t)blockIdx.x * PNT + threadIdx.x; w < n_words; w += (uint64_t)gridDim.x * PNT) {
        uint32_t word = bits[w];
        uint64_t pos = word_rank[w];
        while (word) {
            const uint32_t bb = __ffs(word) - 1;
            word &= word - 1;
            const uint64_t bit = w * 32 + bb;
            const uint64_t gid = bit % G;
            uint32_t lo = 0, hi = P;
            while (hi - lo > 1) {
                const uint32_t m = (lo + hi) >> 1;
                if (host_base[m] <= gid) lo = m; else hi = m;
            }
            R[pos] = (int32_t)(gid - host_base[lo]);
            if (okey) {
                okey[pos] = (uint64_t)fc[bit] << 16;
                oval[pos] = (uint32_t)pos;
            }
            ++pos;
        }
    }
}

// L[j] = M_local + j (canonical numbering)
__global__ void k_iota_l(int32_t* Lv, uint64_t n, uint32_t M_local) {
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) Lv[j] = (int32_t)((uint64_t)M_local + j);
}

// L[canonical index] = M_local + position in call order
__global__ void k_scatter_l(const uint32_t* canon, uint64_t n, uint32_t M_local, int32_t* Lv) {
    const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) Lv[canon[k]] = (int32_t)((uint64_t)M_local + k);
}

// R offsets per (alpha+1, sigma) from the bit set ranks
__global__ void k_bounds_bits(const uint32_t* bits, const uint64_t* word_rank, const uint64_t* host_base, uint32_t P,
                              uint32_t n_a, uint64_t G, uint32_t M_local, int canonical, uint64_t* r_off,
                              int64_t* img_base) {
    const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t nk = (uint64_t)n_a * P;
    if (k > nk) return;
    const uint64_t x = k == nk ? (uint64_t)n_a * G : (k / P) * G + host_base[k % P];
    const uint64_t r = rank_of(bits, word_rank, x);
    r_off[k] = r;
    if (k < nk) img_base[k] = canonical ? (int64_t)M_local + (int64_t)r : -1;
}

// point-to-point rows: set the bits of local-id ranges (unflagged calls)
struct WRange {
    uint64_t begin;   // first position in the concatenation of word counts
    uint64_t row;     // first word of the row
    uint32_t lo, hi;  // local ids [lo, hi)
};

__global__ __launch_bounds__(PNT) void k_set_ranges(const WRange* rg, uint32_t n_rg, uint64_t total, uint32_t* rows) {
    for (uint64_t j = (uint64_t)blockIdx.x * PNT + threadIdx.x; j < total; j += (uint64_t)gridDim.x * PNT) {
        uint32_t a = 0, b = n_rg;
        while (b - a > 1) {
            const uint32_t m = (a + b) >> 1;
            if (rg[m].begin <= j) a = m; else b = m;
        }
        const WRange r = rg[a];
        const uint32_t w = (r.lo >> 5) + (uint32_t)(j - r.begin);
        const uint32_t first = max(r.lo, w * 32), last = min(r.hi, w * 32 + 32);   // [first, last) in this word
        const uint32_t nb = last - first;
        const uint32_t mask = (nb == 32 ? ~0u : ((1u << nb) - 1u)) << (first & 31);
        atomicOr(&rows[r.row + w], mask);
    }
}

// first-index array: row_ptr[r] = first position with source >= r
// Each thread takes 4 consecutive positions with one 16-byte load; position
// i closes the rows (src[i-1], src[i]] (position n closes the rest).
__global__ __launch_bounds__(PNT) void k_csr(const int32_t* src, uint64_t n, uint64_t n_rows, uint64_t* row_ptr) {
    const uint64_t quads = n / 4 + 1;   // the last quad holds the tail and position n
    for (uint64_t q = (uint64_t)blockIdx.x * PNT + threadIdx.x; q < quads; q += (uint64_t)gridDim.x * PNT) {
        const uint64_t i0 = q * 4;
        int64_t v[4];
        if (i0 + 4 <= n) {
            const int4 x = *reinterpret_cast<const int4*>(src + i0);
            v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
        } else {
            for (int k = 0; k < 4; ++k) v[k] = i0 + k < n ? (int64_t)src[i0 + k] : (int64_t)n_rows;
        }
        int64_t prev = i0 == 0 ? -1 : (int64_t)src[i0 - 1];
        for (int k = 0; k < 4; ++k) {
            const uint64_t i = i0 + k;
            if (i > n) break;
            for (int64_t r = prev + 1; r <= v[k]; ++r) row_ptr[r] = i;
            prev = v[k];
        }
    }
}

// The same by a binary search per row, for few rows against many connections:
// a search reads about log2(n) positions where the pass above reads all n.
__global__ void k_csr_search(const int32_t* src, uint64_t n, uint64_t n_rows, uint64_t* row_ptr) {
    const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r > n_rows) return;
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if ((int64_t)src[mid] < (int64_t)r) lo = mid + 1; else hi = mid;
    }
    row_ptr[r] = lo;
}

__global__ void k_fill_u64(uint64_t* p, uint64_t n, uint64_t v) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---- point-to-point lists
// S values: set bits of row tau as local ids, at their rank
__global__ __launch_bounds__(PNT) void k_s_vals(const uint32_t* rows, const uint64_t* word_rank, uint64_t n_words,
                                                uint32_t words_per_row, int32_t* S) {
    for (uint64_t w = (uint64_t)blockIdx.x * PNT + threadIdx.x; w < n_words; w += (uint64_t)gridDim.x * PNT) {
        uint32_t word = rows[w];
        uint64_t pos = word_rank[w];
        const uint32_t s0 = (uint32_t)(w % words_per_row) * 32;
        while (word) {
            const uint32_t b = __ffs(word) - 1;
            word &= word - 1;
            S[pos++] = (int32_t)(s0 + b);
        }
    }
}

// per local source: number of target hosts whose row has its bit
__global__ __launch_bounds__(PNT) void k_tp_count(const uint32_t* rows, uint32_t P, uint32_t words_per_row,
                                                  uint32_t M, uint32_t* cnt) {
    const uint32_t s = blockIdx.x * PNT + threadIdx.x;
    if (s >= M) return;
    uint32_t c = 0;
    for (uint32_t tau = 0; tau < P; ++tau) c += (rows[(uint64_t)tau * words_per_row + (s >> 5)] >> (s & 31)) & 1u;
    cnt[s] = c;
}

__global__ __launch_bounds__(PNT) void k_tp_fill(const uint32_t* rows, const uint64_t* word_rank, const uint64_t* s_off,
                                                 uint32_t P, uint32_t words_per_row, uint32_t M, const uint64_t* tp_ptr,
                                                 uint32_t* T, uint32_t* Pos) {
    const uint32_t s = blockIdx.x * PNT + threadIdx.x;
    if (s >= M) return;
    uint64_t o = tp_ptr[s];
    for (uint32_t tau = 0; tau < P; ++tau) {
        const uint64_t w = (uint64_t)tau * words_per_row + (s >> 5);
        const uint32_t word = rows[w];
        if ((word >> (s & 31)) & 1u) {
            T[o] = tau;
            Pos[o] = (uint32_t)(word_rank[w] + (uint64_t)__popc(word & ((1u << (s & 31)) - 1u)) - s_off[tau]);
            ++o;
        }
    }
}

// ---- collective arrays
struct HRange {
    uint64_t h_begin;   // first position in H
    uint32_t lo, len;   // source ids [lo, lo + len)
    uint32_t a, sigma;  // map index alpha + 1 and host
};

__global__ __launch_bounds__(PNT) void k_hi(const HRange* rg, uint32_t n_rg, uint64_t n_h, const uint32_t* bits,
                                            const uint64_t* word_rank, const int32_t* Lmap, const uint64_t* host_base,
                                            uint64_t G, uint32_t PL, int32_t* H, int32_t* I) {
    for (uint64_t j = (uint64_t)blockIdx.x * PNT + threadIdx.x; j < n_h; j += (uint64_t)gridDim.x * PNT) {
        uint32_t a = 0, b = n_rg;
        while (b - a > 1) {
            const uint32_t m = (a + b) >> 1;
            if (rg[m].h_begin <= j) a = m; else b = m;
        }
        const HRange r = rg[a];
        const uint32_t s = r.lo + (uint32_t)(j - r.h_begin);
        H[j] = (int32_t)s;
        int32_t img = -1;
        if (r.sigma != PL) {
            const uint64_t bit = (uint64_t)r.a * G + host_base[r.sigma] + s;
            if ((bits[bit >> 5] >> (bit & 31)) & 1u) img = Lmap[rank_of(bits, word_rank, bit)];
        }
        I[j] = img;
    }
}

// G/Q of local source s: groups (ascending) whose H on P_local contains s
struct LRange {
    uint32_t lo, hi;    // [lo, hi)
    uint64_t pos;       // position of lo in H_{g, P_local}
};

__global__ __launch_bounds__(PNT) void k_gq(const LRange* lr, const uint32_t* g_first, uint32_t n_groups,
                                            const int32_t* groups, uint32_t M, const uint64_t* gq_ptr, uint32_t* cnt,
                                            int32_t* Gv, uint32_t* Qv) {
    const uint32_t s = blockIdx.x * PNT + threadIdx.x;
    if (s >= M) return;
    uint64_t o = gq_ptr ? gq_ptr[s] : 0;
    uint32_t c = 0;
    for (uint32_t g = 0; g < n_groups; ++g) {
        uint32_t a = g_first[g], b = g_first[g + 1];
        if (a == b) continue;
        while (b - a > 1) {   // last range with lo <= s
            const uint32_t m = (a + b) >> 1;
            if (lr[m].lo <= s) a = m; else b = m;
        }
        const LRange r = lr[a];
        if (s >= r.lo && s < r.hi) {
            if (gq_ptr) {
                Gv[o] = groups[g];
                Qv[o] = (uint32_t)(r.pos + (s - r.lo));
                ++o;
            }
            ++c;
        }
    }
    if (!gq_ptr) cnt[s] = c;
}

uint64_t count_on(const HostSet& s, uint32_t host) {
    uint64_t n = 0;
    for (auto& g : s.seg)
        if (g.host == host) n += g.n;
    return n;
}

// Map policy: does call cl give images on host tau only to the sources its
// connections there use (flagging)?  The threshold heuristic flags rules that
// draw their sources at random (and assigned pairs) when the estimated
// connections on tau per source fall below xi; out-degree and one-to-one calls
// use every source.
bool flag_sources(const Ctx& c, const Call& cl, uint32_t tau) {
    if (c.img_sources == 0) return true;
    if (c.img_sources == 2) return false;
    if (cl.S.total == 0) return true;
    const double n_s = (double)cl.S.total, n_t = (double)count_on(cl.T, tau);
    double est;
    switch (cl.rule) {
        case SNNC_FIXED_INDEGREE: est = (double)cl.n * n_t; break;
        case SNNC_FIXED_TOTAL_NUMBER: est = (double)cl.n * n_t / (double)cl.T.total; break;
        case SNNC_PAIRWISE_BERNOULLI: est = cl.p * n_s * n_t; break;
        case SNNC_ASSIGNED_NODES: {
            auto it = cl.pairs_on.find(tau);
            est = it == cl.pairs_on.end() ? 0.0 : (double)it->second;
            break;
        }
        default: return false;
    }
    return est / n_s < c.xi;
}

template <class T>
T* result(Ctx& c, int32_t id, uint64_t n) {
    auto& a = c.arrays[id];
    dfree(c, a.p);
    a.p = dalloc(c, (size_t)std::max<uint64_t>(n, 1) * sizeof(T));
    a.bytes = (size_t)n * sizeof(T);
    c.counts[id] = n;
    return static_cast<T*>(a.p);
}

unsigned grid_for(uint64_t n, uint64_t cap = 1u << 20) {
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n + PNT - 1) / PNT, cap));
}

uint32_t bits_for(uint64_t n_values) {   // bits to hold 0 .. n_values - 1
    uint32_t b = 0;
    while (b < 64 && (n_values > 0 ? (n_values - 1) >> b : 0)) ++b;
    return b;
}

}  // namespace

namespace {

// first index and count of the image rows [M_local, M_local + n_img)
__global__ void k_img_rows(const uint64_t* row_ptr, uint32_t M_local, uint64_t n_img, uint64_t* first,
                           uint32_t* count) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_img; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t a = row_ptr[(uint64_t)M_local + i], b = row_ptr[(uint64_t)M_local + i + 1];
        if (first) first[i] = a;
        if (count) count[i] = (uint32_t)(b - a);
    }
}

// Moves a result array into pinned host memory that kernels can read.
void to_host(Ctx& c, int32_t id) {
    auto it = c.arrays.find(id);
    if (it == c.arrays.end() || it->second.host) return;
    DevArray& a = it->second;
    void* h = nullptr;
    HIPCHK(hipHostMalloc(&h, std::max<size_t>(a.bytes, 1), hipHostMallocMapped));
    void* d = nullptr;
    if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipHostFree(h);
        raise(SNNC_EDEVICE, "pinned host memory without a device address");
    }
    if (a.bytes) HIPCHK(hipMemcpyAsync(h, a.p, a.bytes, hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
    dfree(c, a.p);
    a.p = h;
    a.dev = d;
    a.host = true;
}

// GPU memory levels (Methods, GPU memory levels subsection).  Levels 0 and 1:
// the maps of the remote sources to their images (R, L, img_base and their
// offsets; H and I of the collective layout) and the first index and count
// of every image row live in pinned host memory, the device keeps the
// first-index array of the local rows only.  Level 2: everything in device
// memory, the count of a row from two first-index entries.  Level 3: level 2
// plus the counts of the image rows as an array.  (Images of every passed
// source from level 1 on: set with the level.)
void place_memory_level(Ctx& c, uint32_t M_local) {
    const int L = c.mem_level;
    if (L != 0 && L != 1 && L != 3) return;
    const uint64_t n_img = c.n_img;
    const uint64_t* rp = static_cast<const uint64_t*>(c.arrays[SNNC_ROW_PTR].p);
    uint64_t* first = (L <= 1) ? result<uint64_t>(c, SNNC_IMG_FIRST, n_img) : nullptr;
    uint32_t* count = result<uint32_t>(c, SNNC_IMG_COUNT, n_img);
    if (n_img) {
        tstart(c, "prep_img_rows");
        hipLaunchKernelGGL(k_img_rows, dim3(grid_for(n_img)), dim3(PNT), 0, c.stream, rp, M_local, n_img, first, count);
        tstop(c);
        HIPCHK(hipGetLastError());
    }
    if (L == 3) return;
    // the device keeps the local rows of the first-index array
    const uint64_t keep = (uint64_t)M_local + 1;
    DevArray old = c.arrays[SNNC_ROW_PTR];
    c.arrays[SNNC_ROW_PTR] = DevArray{};
    uint64_t* nrp = result<uint64_t>(c, SNNC_ROW_PTR, keep);
    HIPCHK(hipMemcpyAsync(nrp, old.p, keep * 8, hipMemcpyDeviceToDevice, c.stream));
    free_array(c, old);
    for (int32_t id : {SNNC_IMG_FIRST, SNNC_IMG_COUNT, SNNC_R_OFF, SNNC_R_VAL, SNNC_IMG_BASE, SNNC_L_VAL, SNNC_H_OFF,
                       SNNC_H_VAL, SNNC_I_VAL})
        to_host(c, id);
}

}  // namespace

int number_variant_count() { return NUMBER_VARIANTS; }

void prepare_all(Ctx& c) {
    const uint32_t P = c.P, PL = c.P_local;
    const uint64_t N = c.n_gen;
    const uint32_t M_local = c.M[PL];
    std::vector<void*> temps;
    auto tmp = [&](size_t bytes) {
        void* p = dalloc(c, bytes);
        temps.push_back(p);
        return p;
    };
    auto cleanup = [&] {
        for (void* p : temps) dfree(c, p);
        temps.clear();
    };
    try {
        // ---------------------------------------------------------- layout tables
        std::vector<uint64_t> host_base(P + 1, 0);
        for (uint32_t h = 0; h < P; ++h) host_base[h + 1] = host_base[h] + c.M[h];
        const uint64_t G = std::max<uint64_t>(host_base[P], 1);
        int32_t amax = -1;
        for (auto& cl : c.calls) amax = std::max(amax, cl.alpha);
        const uint32_t n_a = (uint32_t)(amax + 2);
        const uint32_t n_calls = (uint32_t)c.calls.size();
        std::vector<uint8_t> flag_local(n_calls);
        for (uint32_t k = 0; k < n_calls; ++k) flag_local[k] = flag_sources(c, c.calls[k], PL) ? 1 : 0;
        std::vector<CallD> calls;
        std::vector<int64_t> seg_base;   // all calls' segment tables, concatenated
        std::vector<size_t> seg_at;
        for (uint32_t k = 0; k < n_calls; ++k) {
            const Call& cl = c.calls[k];
            if (!cl.gen_count) continue;
            CallD d = make_calld(cl, k, flag_local[k]);
            const uint64_t a = (uint64_t)(cl.alpha + 1);
            seg_at.push_back(seg_base.size());
            for (size_t j = 0; j < cl.S.seg.size(); ++j)
                seg_base.push_back((int64_t)(a * G + host_base[cl.S.seg[j].host] + cl.S.seg[j].first) -
                                   (int64_t)cl.S.ord_begin[j]);
            d.local_lo = a * G + host_base[PL];
            calls.push_back(d);
        }
        int64_t* d_seg_base = static_cast<int64_t*>(tmp(std::max<size_t>(seg_base.size(), 1) * 8));
        upload(c, d_seg_base, seg_base.data(), seg_base.size() * 8);
        for (size_t k = 0; k < calls.size(); ++k) calls[k].seg_base = d_seg_base + seg_at[k];
        if (calls.empty()) calls.push_back(CallD{0, nullptr, 0, 0, 0, 0, 0, FastDiv{}, nullptr, 0});
        CallD* d_calls = static_cast<CallD*>(tmp(calls.size() * sizeof(CallD)));
        upload(c, d_calls, calls.data(), calls.size() * sizeof(CallD));
        uint64_t* d_hb = static_cast<uint64_t*>(tmp((P + 1) * 8));
        upload(c, d_hb, host_base.data(), (P + 1) * 8);
        Lookup L{d_calls, (uint32_t)calls.size(), d_hb, P, PL, G};

        // ---------------------------------------------------------- 1-5 image map, keys, sort, first index
        // Default policy: without remote sources the keys hold final sources and
        // the last radix pass unpacks; with remote sources the keys hold global
        // source ids and the images are numbered by a scan over the sorted keys.
        // Other policies (or "map_path"): the images are numbered first (first
        // call of every image source, its order), the keys hold image indices
        // and the last pass unpacks.
        bool remote_net = false;
        for (auto& cl : c.calls)
            for (auto& g : cl.S.seg) remote_net |= (g.host != PL && cl.gen_count > 0);
        const bool mapped = c.numbering != 0 || c.img_sources != 0 || c.force_map_path;
        const uint64_t n_bits = (uint64_t)n_a * G;
        const uint64_t n_words = n_bits / 32 + 1;    // one spare word: rank of the end bit
        uint32_t* bits = static_cast<uint32_t*>(tmp(n_words * 4));
        HIPCHK(hipMemsetAsync(bits, 0, n_words * 4, c.stream));
        uint64_t* word_rank = static_cast<uint64_t*>(tmp((n_words + 1) * 8));
        uint64_t n_img = 0;
        int32_t* Lmap = nullptr;
        if (mapped) {
            uint32_t* fc = static_cast<uint32_t*>(dalloc(c, n_bits * 4));
            try {
                HIPCHK(hipMemsetAsync(fc, 0xff, n_bits * 4, c.stream));
                bool any_flagged = false;
                for (auto& cd : calls) any_flagged |= (cd.flag && cd.nS > 0);
                if (N && remote_net && any_flagged) {
                    tstart(c, "prep_first_use");
                    hipLaunchKernelGGL(k_first_use, dim3(grid_for(N, 8192)), dim3(PNT), 0, c.stream, L, c.g_src, N, fc);
                    tstop(c);
                    HIPCHK(hipGetLastError());
                }
                std::vector<FRange> fr;
                uint64_t f_total = 0;
                for (uint32_t k = 0; k < n_calls; ++k) {
                    const Call& cl = c.calls[k];
                    if (flag_local[k] || count_on(cl.T, PL) == 0) continue;
                    for (auto& g : cl.S.seg)
                        if (g.host != PL && g.n) {
                            fr.push_back(FRange{f_total, (uint64_t)(cl.alpha + 1) * G + host_base[g.host] + g.first, k, 0});
                            f_total += g.n;
                        }
                }
                if (f_total) {
                    FRange* d_fr = static_cast<FRange*>(tmp(fr.size() * sizeof(FRange)));
                    upload(c, d_fr, fr.data(), fr.size() * sizeof(FRange));
                    tstart(c, "prep_first_pass");
                    hipLaunchKernelGGL(k_first_pass, dim3(grid_for(f_total)), dim3(PNT), 0, c.stream, d_fr,
                                       (uint32_t)fr.size(), f_total, fc);
                    tstop(c);
                    HIPCHK(hipGetLastError());
                }
                tstart(c, "prep_fc_bits");
                hipLaunchKernelGGL(k_fc_bits, dim3(grid_for(n_bits)), dim3(PNT), 0, c.stream, fc, n_bits, n_words, bits);
                tstop(c);
                HIPCHK(hipGetLastError());
                n_img = scan_popc_u64(c, bits, word_rank, n_words, true);
                if ((uint64_t)M_local + n_img > 0x7fffffffull)
                    raise(SNNC_EUNSUPPORTED, "more than 2^31-1 local and image neurons");
                int32_t* R = result<int32_t>(c, SNNC_R_VAL, n_img);
                Lmap = result<int32_t>(c, SNNC_L_VAL, n_img);
                const uint32_t call_bits = bits_for(n_calls);
                const bool by_call = c.numbering == 1 && call_bits > 0;
                uint64_t* ik0 = nullptr;
                uint32_t* iv0 = nullptr;
                if (by_call && n_img) {
                    ik0 = static_cast<uint64_t*>(tmp(n_img * 8));
                    iv0 = static_cast<uint32_t*>(tmp(n_img * 4));
                }
                if (n_img) {
                    tstart(c, "prep_img_list");
                    hipLaunchKernelGGL(k_img_list, dim3(grid_for(n_words)), dim3(PNT), 0, c.stream, bits, word_rank,
                                       n_words, fc, d_hb, P, G, R, ik0, iv0);
                    tstop(c);
                    HIPCHK(hipGetLastError());
                }
                dfree(c, fc);
                fc = nullptr;
                if (n_img && by_call) {
                    // stable sort of the canonical indices by first call: the paper's order
                    uint64_t* ik1 = static_cast<uint64_t*>(tmp(n_img * 8));
                    uint32_t* iv1 = static_cast<uint32_t*>(tmp(n_img * 4));
                    const int w = radix_sort(c, ik0, iv0, ik1, iv1, n_img, 16, 16 + call_bits, nullptr, nullptr);
                    tstart(c, "prep_number_calls");
                    hipLaunchKernelGGL(k_scatter_l, dim3((unsigned)((n_img + 255) / 256)), dim3(256), 0, c.stream,
                                       w ? iv1 : iv0, n_img, M_local, Lmap);
                    tstop(c);
                    HIPCHK(hipGetLastError());
                } else if (n_img) {
                    hipLaunchKernelGGL(k_iota_l, dim3((unsigned)((n_img + 255) / 256)), dim3(256), 0, c.stream, Lmap,
                                       n_img, M_local);
                    HIPCHK(hipGetLastError());
                }
                uint64_t* r_off = result<uint64_t>(c, SNNC_R_OFF, (uint64_t)n_a * P + 1);
                int64_t* img_base = result<int64_t>(c, SNNC_IMG_BASE, (uint64_t)n_a * P);
                const uint64_t nk = (uint64_t)n_a * P + 1;
                hipLaunchKernelGGL(k_bounds_bits, dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, c.stream, bits,
                                   word_rank, d_hb, P, n_a, G, M_local, c.numbering == 0 ? 1 : 0, r_off, img_base);
                HIPCHK(hipGetLastError());
            } catch (...) {
                if (fc) dfree(c, fc);
                throw;
            }
        }
        const uint32_t tbits = bits_for(M_local);
        const uint64_t prefix_span = mapped       ? (uint64_t)M_local + n_img
                                     : remote_net ? (uint64_t)M_local + n_bits
                                                  : (uint64_t)M_local;
        const uint32_t sbits = bits_for(prefix_span);
        c.key_bits = sbits + tbits;
        if (sbits + tbits > 48) raise(SNNC_EUNSUPPORTED, "source and target ids need more than 48 key bits");
        const SortPlan plan = plan_sort(c, N, sbits + tbits);   // the sort below takes the same plan
        const uint32_t passes = plan.passes, dbits = plan.dbits;
        const bool unpack_in_sort = !remote_net || mapped;
        int32_t* o_src = nullptr;
        uint64_t* row_ptr = nullptr;
        uint64_t* keys0 = nullptr;
        uint64_t* keys1 = nullptr;
        uint32_t* vals1 = nullptr;
        if (N) {
            keys0 = static_cast<uint64_t*>(tmp(N * 8));
            uint64_t* hist = static_cast<uint64_t*>(tmp(8 * HIST_STRIDE * 8));
            HIPCHK(hipMemsetAsync(hist, 0, 8 * HIST_STRIDE * 8, c.stream));
            tstart(c, "prep_keys");
            hipLaunchKernelGGL(k_keys, dim3(grid_for(N, 8192)), dim3(PNT), 0, c.stream, L, c.g_src, c.g_tgt, c.g_delay,
                               N, mapped ? bits : (const uint32_t*)nullptr, mapped ? word_rank : (const uint64_t*)nullptr,
                               Lmap, M_local, 16 + tbits, plan.n9, dbits, passes, keys0, hist);
            tstop(c);
            HIPCHK(hipGetLastError());
            // the source ordinals, targets and delays now live in the keys (released in stream order)
            if (!c.gen_vmm) {   // block store: handed back after Prepare's final wait
                dfree(c, c.g_src); c.g_src = nullptr;
                dfree(c, c.g_tgt); c.g_tgt = nullptr;
                dfree(c, c.g_delay); c.g_delay = nullptr;
            }
            keys1 = static_cast<uint64_t*>(tmp(N * 8));
            vals1 = static_cast<uint32_t*>(tmp(N * 4));
            // outputs allocated only now, so they reuse the memory just released
            o_src = result<int32_t>(c, SNNC_SRC, N);
            int32_t* o_tgt = result<int32_t>(c, SNNC_TGT, N);
            uint16_t* o_delay = result<uint16_t>(c, SNNC_DELAY, N);
            float* o_weight = result<float>(c, SNNC_WEIGHT, N);
            FinalOut fo{o_src, o_tgt, o_delay, o_weight, 16 + tbits, tbits ? (1ull << tbits) - 1 : 0};
            if (unpack_in_sort) {
                radix_sort(c, keys0, reinterpret_cast<uint32_t*>(c.g_weight), keys1, vals1, N, 16, 16 + sbits + tbits,
                           hist, &fo);
                const uint64_t n_rows = (uint64_t)M_local + n_img;
                row_ptr = result<uint64_t>(c, SNNC_ROW_PTR, n_rows + 1);
                tstart(c, "prep_csr");
                if (n_rows * 64 < N)   // rows few against connections: search instead of reading every source
                    hipLaunchKernelGGL(k_csr_search, dim3((unsigned)((n_rows + 1 + 255) / 256)), dim3(256), 0,
                                       c.stream, o_src, N, n_rows, row_ptr);
                else
                    hipLaunchKernelGGL(k_csr, dim3(grid_for(N / 4 + 1, 16384)), dim3(PNT), 0, c.stream, o_src, N,
                                       n_rows, row_ptr);
                tstop(c);
                HIPCHK(hipGetLastError());
            } else {
                const int which = radix_sort(c, keys0, reinterpret_cast<uint32_t*>(c.g_weight), keys1, vals1, N, 16,
                                             16 + sbits + tbits, hist, nullptr);
                const uint64_t max_img = std::min<uint64_t>(N, n_bits);
                uint64_t* img_key = static_cast<uint64_t*>(tmp(max_img * 8 + 8));
                row_ptr = result<uint64_t>(c, SNNC_ROW_PTR, (uint64_t)M_local + max_img + 1);
                uint64_t* d_nimg = static_cast<uint64_t*>(tmp(8));
                const NumberShape shape = NUMBER_SHAPES[c.number_variant];
                const uint64_t xtile = (uint64_t)shape.nt * shape.ipt;
                const uint64_t tiles = (N + xtile - 1) / xtile;
                if (c.lookback_bytes < tiles * 8) raise(SNNC_EDEVICE, "look-back table too small");
                if (++c.sort_epoch > XEPOCH_MAX) {
                    HIPCHK(hipMemsetAsync(c.lookback, 0, c.lookback_bytes, c.stream));
                    c.sort_epoch = 1;
                }
                uint32_t* counter = static_cast<uint32_t*>(tmp(4));
                HIPCHK(hipMemsetAsync(counter, 0, 4, c.stream));
                const uint32_t* vsorted = which ? vals1 : reinterpret_cast<uint32_t*>(c.g_weight);
                tstart(c, "prep_number");
                auto number = [&](auto kern, int nt) {
                    hipLaunchKernelGGL(kern, dim3((unsigned)tiles), dim3(nt), 0, c.stream, which ? keys1 : keys0,
                                   vsorted, N, 16 + tbits, fo.tgt_mask, M_local, (uint64_t*)c.lookback, counter,
                                   c.sort_epoch, c.d_status, o_src, o_tgt, o_delay, o_weight, img_key, row_ptr, d_nimg);
                };
                switch (c.number_variant) {
                case 0: number(k_number<1024, 12, false>, 1024); break;
                case 1: number(k_number<512, 12, false>, 512); break;
                case 2: number(k_number<256, 12, false>, 256); break;
                case 3: number(k_number<512, 12, true>, 512); break;
                case 4: number(k_number<256, 12, true>, 256); break;
                case 5: number(k_number<256, 16, true>, 256); break;
                case 6: number(k_number<256, 8, true>, 256); break;
                case 7: number(k_number<256, 6, true>, 256); break;
                case 8: number(k_number<512, 8, true>, 512); break;
                case 9: number(k_number<1024, 12, true>, 1024); break;
                case 10: number(k_number<1024, 10, true>, 1024); break;
                default: number(k_number<1024, 8, true>, 1024); break;
                }
                tstop(c);
                HIPCHK(hipGetLastError());
                download(c, &n_img, d_nimg, 8);
                c.counts[SNNC_ROW_PTR] = (uint64_t)M_local + n_img + 1;
                if ((uint64_t)M_local + n_img > 0x7fffffffull)
                    raise(SNNC_EUNSUPPORTED, "more than 2^31-1 local and image neurons");
                int32_t* R = result<int32_t>(c, SNNC_R_VAL, n_img);
                Lmap = result<int32_t>(c, SNNC_L_VAL, n_img);
                uint64_t* r_off = result<uint64_t>(c, SNNC_R_OFF, (uint64_t)n_a * P + 1);
                int64_t* img_base = result<int64_t>(c, SNNC_IMG_BASE, (uint64_t)n_a * P);
                if (n_img) {
                    tstart(c, "prep_rvals");
                    hipLaunchKernelGGL(k_rvals_sorted, dim3((unsigned)((n_img + 256 * RV_RUN - 1) / (256 * RV_RUN))),
                                       dim3(256), 0, c.stream,
                                       img_key, n_img, d_hb, P, G, R);
                    tstop(c);
                    HIPCHK(hipGetLastError());
                    tstart(c, "prep_bits");
                    hipLaunchKernelGGL(k_bits_sorted, dim3((unsigned)((n_img + 255) / 256)), dim3(256), 0, c.stream,
                                       img_key, n_img, bits);
                    tstop(c);
                    HIPCHK(hipGetLastError());
                    hipLaunchKernelGGL(k_iota_l, dim3((unsigned)((n_img + 255) / 256)), dim3(256), 0, c.stream, Lmap,
                                       n_img, M_local);
                    HIPCHK(hipGetLastError());
                }
                const uint64_t nk = (uint64_t)n_a * P + 1;
                tstart(c, "prep_bounds");
                hipLaunchKernelGGL(k_bounds_sorted, dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, c.stream, img_key,
                                   n_img, d_hb, P, n_a, G, M_local, r_off, img_base);
                tstop(c);
                HIPCHK(hipGetLastError());
            }
        } else {
            o_src = result<int32_t>(c, SNNC_SRC, 0);
            result<int32_t>(c, SNNC_TGT, 0);
            result<uint16_t>(c, SNNC_DELAY, 0);
            result<float>(c, SNNC_WEIGHT, 0);
            const uint64_t n_rows = (uint64_t)M_local + n_img;
            row_ptr = result<uint64_t>(c, SNNC_ROW_PTR, n_rows + 1);
            hipLaunchKernelGGL(k_fill_u64, dim3((n_rows + 1 + 255) / 256), dim3(256), 0, c.stream, row_ptr, n_rows + 1,
                               (uint64_t)0);
            HIPCHK(hipGetLastError());
        }
        if (!mapped && (!remote_net || !N)) {
            result<int32_t>(c, SNNC_R_VAL, 0);
            result<int32_t>(c, SNNC_L_VAL, 0);
            uint64_t* r_off = result<uint64_t>(c, SNNC_R_OFF, (uint64_t)n_a * P + 1);
            int64_t* img_base = result<int64_t>(c, SNNC_IMG_BASE, (uint64_t)n_a * P);
            HIPCHK(hipMemsetAsync(r_off, 0, ((uint64_t)n_a * P + 1) * 8, c.stream));
            std::vector<int64_t> ib((size_t)n_a * P, (int64_t)M_local);
            upload(c, img_base, ib.data(), ib.size() * 8);
        }
        c.n_img = n_img;
        // word ranks of the image bit set (the collective arrays look images up by bit)
        if (!mapped) scan_popc_u64(c, bits, word_rank, n_words, false);
        if (!c.gen_vmm) {   // block store: unmapped after the final wait of Prepare
            dfree(c, c.g_weight);
            c.g_weight = nullptr;
            c.cap_gen = 0;
        }
        (void)row_ptr;

        // ---------------------------------------------------------- 6 point-to-point lists
        const uint32_t wpr = (M_local + 31) / 32 + 1;     // words per row (+1 spare)
        const uint64_t n_rw = (uint64_t)P * wpr;
        uint32_t* rows = static_cast<uint32_t*>(tmp(n_rw * 4));
        HIPCHK(hipMemsetAsync(rows, 0, n_rw * 4, c.stream));
        std::vector<WRange> wr;
        uint64_t w_total = 0;
        for (auto& cl : c.calls) {
            if (cl.alpha != -1) continue;
            bool has_local_source = false;
            for (auto& g : cl.S.seg) has_local_source |= (g.host == PL && g.n > 0);
            if (!has_local_source) continue;
            for (uint32_t tau = 0; tau < P; ++tau) {
                if (tau == PL || count_on(cl.T, tau) == 0) continue;
                if (flag_sources(c, cl, tau)) {   // regenerate tau's draws, keep the local sources they use
                    gen_mark(c, cl, tau, rows + (uint64_t)tau * wpr);
                    continue;
                }
                for (auto& g : cl.S.seg)          // not flagged: every local source of the call
                    if (g.host == PL && g.n) {
                        wr.push_back(WRange{w_total, (uint64_t)tau * wpr, g.first, g.first + g.n});
                        w_total += ((g.first + g.n - 1) >> 5) - (g.first >> 5) + 1;
                    }
            }
        }
        if (w_total) {
            WRange* d_wr = static_cast<WRange*>(tmp(wr.size() * sizeof(WRange)));
            upload(c, d_wr, wr.data(), wr.size() * sizeof(WRange));
            tstart(c, "prep_s_ranges");
            hipLaunchKernelGGL(k_set_ranges, dim3(grid_for(w_total)), dim3(PNT), 0, c.stream, d_wr, (uint32_t)wr.size(),
                               w_total, rows);
            tstop(c);
            HIPCHK(hipGetLastError());
        }
        uint64_t* row_rank = static_cast<uint64_t*>(tmp((n_rw + 1) * 8));
        const uint64_t n_s = scan_popc_u64(c, rows, row_rank, n_rw, true);
        std::vector<uint64_t> rank_host(n_rw + 1);
        download(c, rank_host.data(), row_rank, (n_rw + 1) * 8);
        std::vector<uint64_t> s_off_h(P + 1);
        for (uint32_t tau = 0; tau <= P; ++tau) s_off_h[tau] = rank_host[(uint64_t)tau * wpr];
        uint64_t* s_off = result<uint64_t>(c, SNNC_S_OFF, P + 1);
        upload(c, s_off, s_off_h.data(), (P + 1) * 8);
        int32_t* S = result<int32_t>(c, SNNC_S_VAL, n_s);
        uint64_t* tp_ptr = result<uint64_t>(c, SNNC_TP_PTR, (uint64_t)M_local + 1);
        uint32_t* Tv = result<uint32_t>(c, SNNC_T_VAL, n_s);
        uint32_t* Pv = result<uint32_t>(c, SNNC_P_VAL, n_s);
        if (n_s) {
            tstart(c, "prep_s_vals");
            hipLaunchKernelGGL(k_s_vals, dim3(grid_for(n_rw)), dim3(PNT), 0, c.stream, rows, row_rank, n_rw, wpr, S);
            tstop(c);
            HIPCHK(hipGetLastError());
        }
        if (M_local) {
            uint32_t* cnt = static_cast<uint32_t*>(tmp((size_t)M_local * 4));
            tstart(c, "prep_tp");
            hipLaunchKernelGGL(k_tp_count, dim3((M_local + PNT - 1) / PNT), dim3(PNT), 0, c.stream, rows, P, wpr,
                               M_local, cnt);
            tstop(c);
            HIPCHK(hipGetLastError());
            scan_u32_u64(c, cnt, tp_ptr, M_local, false);
            if (n_s) {
                tstart(c, "prep_tp");
                hipLaunchKernelGGL(k_tp_fill, dim3((M_local + PNT - 1) / PNT), dim3(PNT), 0, c.stream, rows, row_rank,
                                   s_off, P, wpr, M_local, tp_ptr, Tv, Pv);
                tstop(c);
                HIPCHK(hipGetLastError());
            }
        } else {
            HIPCHK(hipMemsetAsync(tp_ptr, 0, 8, c.stream));
        }

        // ---------------------------------------------------------- 7 collective arrays
        std::vector<int32_t> groups;
        for (auto& cl : c.calls)
            if (cl.alpha >= 0) groups.push_back(cl.alpha);
        std::sort(groups.begin(), groups.end());
        groups.erase(std::unique(groups.begin(), groups.end()), groups.end());
        const uint32_t NG = (uint32_t)groups.size();
        std::vector<HRange> ranges;
        std::vector<uint64_t> h_off_h((size_t)NG * P + 1, 0);
        std::vector<LRange> lranges;
        std::vector<uint32_t> g_first(NG + 1, 0);
        uint64_t h_total = 0;
        for (uint32_t g = 0; g < NG; ++g) {
            std::vector<std::vector<std::pair<uint32_t, uint32_t>>> per(P);
            for (auto& cl : c.calls)
                if (cl.alpha == groups[g])
                    for (auto& sg : cl.S.seg) per[sg.host].push_back({sg.first, sg.first + sg.n});
            g_first[g] = (uint32_t)lranges.size();
            for (uint32_t sigma = 0; sigma < P; ++sigma) {
                auto& v = per[sigma];
                std::sort(v.begin(), v.end());
                std::vector<std::pair<uint32_t, uint32_t>> merged;
                for (auto& r : v) {
                    if (!merged.empty() && r.first <= merged.back().second) merged.back().second = std::max(merged.back().second, r.second);
                    else merged.push_back(r);
                }
                h_off_h[(size_t)g * P + sigma] = h_total;
                uint64_t pos = 0;
                for (auto& r : merged) {
                    ranges.push_back(HRange{h_total, r.first, r.second - r.first, (uint32_t)(groups[g] + 1), sigma});
                    if (sigma == PL) lranges.push_back(LRange{r.first, r.second, pos});
                    h_total += r.second - r.first;
                    pos += r.second - r.first;
                }
            }
        }
        g_first[NG] = (uint32_t)lranges.size();
        h_off_h[(size_t)NG * P] = h_total;
        int32_t* d_groups = result<int32_t>(c, SNNC_GROUPS, NG);
        upload(c, d_groups, groups.data(), NG * 4);
        uint64_t* h_off = result<uint64_t>(c, SNNC_H_OFF, (uint64_t)NG * P + 1);
        upload(c, h_off, h_off_h.data(), h_off_h.size() * 8);
        int32_t* Hv = result<int32_t>(c, SNNC_H_VAL, h_total);
        int32_t* Iv = result<int32_t>(c, SNNC_I_VAL, h_total);
        if (h_total) {
            HRange* d_rg = static_cast<HRange*>(tmp(ranges.size() * sizeof(HRange)));
            upload(c, d_rg, ranges.data(), ranges.size() * sizeof(HRange));
            tstart(c, "prep_hi");
            hipLaunchKernelGGL(k_hi, dim3(grid_for(h_total)), dim3(PNT), 0, c.stream, d_rg, (uint32_t)ranges.size(),
                               h_total, bits, word_rank, Lmap, d_hb, G, PL, Hv, Iv);
            tstop(c);
            HIPCHK(hipGetLastError());
        }
        uint64_t* gq_ptr = result<uint64_t>(c, SNNC_GQ_PTR, (uint64_t)M_local + 1);
        uint64_t n_gq = 0;
        if (M_local && !lranges.empty()) {
            LRange* d_lr = static_cast<LRange*>(tmp(lranges.size() * sizeof(LRange)));
            upload(c, d_lr, lranges.data(), lranges.size() * sizeof(LRange));
            uint32_t* d_gf = static_cast<uint32_t*>(tmp((NG + 1) * 4));
            upload(c, d_gf, g_first.data(), (NG + 1) * 4);
            uint32_t* cnt = static_cast<uint32_t*>(tmp((size_t)M_local * 4));
            tstart(c, "prep_gq");
            hipLaunchKernelGGL(k_gq, dim3((M_local + PNT - 1) / PNT), dim3(PNT), 0, c.stream, d_lr, d_gf, NG, d_groups,
                               M_local, (const uint64_t*)nullptr, cnt, (int32_t*)nullptr, (uint32_t*)nullptr);
            tstop(c);
            HIPCHK(hipGetLastError());
            n_gq = scan_u32_u64(c, cnt, gq_ptr, M_local, true);
            int32_t* Gv = result<int32_t>(c, SNNC_G_VAL, n_gq);
            uint32_t* Qv = result<uint32_t>(c, SNNC_Q_VAL, n_gq);
            if (n_gq) {
                tstart(c, "prep_gq");
                hipLaunchKernelGGL(k_gq, dim3((M_local + PNT - 1) / PNT), dim3(PNT), 0, c.stream, d_lr, d_gf, NG,
                                   d_groups, M_local, (const uint64_t*)gq_ptr, cnt, Gv, Qv);
                tstop(c);
                HIPCHK(hipGetLastError());
            }
        } else {
            tstart(c, "prep_gq");
            hipLaunchKernelGGL(k_fill_u64, dim3(((uint64_t)M_local + 1 + 255) / 256), dim3(256), 0, c.stream, gq_ptr,
                               (uint64_t)M_local + 1, (uint64_t)0);
            tstop(c);
            HIPCHK(hipGetLastError());
            result<int32_t>(c, SNNC_G_VAL, 0);
            result<uint32_t>(c, SNNC_Q_VAL, 0);
        }
        sync(c);
        place_memory_level(c, M_local);
    } catch (...) {
        cleanup();
        throw;
    }
    cleanup();
}

void free_array(Ctx& c, DevArray& a) {
    if (a.host) (void)hipHostFree(a.p);
    else dfree(c, a.p);
    a = DevArray{};
}

}  // namespace snnc
