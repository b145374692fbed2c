// Stable LSD radix sort of 64-bit keys with a 32-bit payload, one pass per
// digit of at most 8 bits, in the single-pass "onesweep" form: every
// workgroup takes the next tile in launch order, ranks its keys within the
// tile with wave64 ballots, publishes its per-digit count, resolves the
// counts of all earlier tiles by decoupled look-back, stages the tile in LDS
// in digit order and writes runs of equal digits with consecutive stores.
// The digit histograms of all passes come from one reading pass (fused into
// the key builder in the prepare pipeline).  Tile shapes (threads x keys per
// thread) are template variants; the context picks one (tunable).
#include <algorithm>
#include <map>
#include <mutex>

#include "device_common.h"
#include "internal.h"

namespace snnc {

namespace {

constexpr int RADIX = 256;          // buckets of an 8-bit digit
constexpr int HSTRIDE = HIST_STRIDE; // histogram entries per pass (up to 9-bit digits)

// look-back status word: [63:62] flag, [61:40] epoch, [39:0] count
constexpr uint64_t FLAG_AGG = 1ull << 62;
constexpr uint64_t FLAG_INC = 2ull << 62;
constexpr uint64_t VALUE_MASK = (1ull << 40) - 1;
constexpr uint32_t EPOCH_MAX = (1u << 22) - 1;
constexpr uint32_t SPIN_LIMIT = 1u << 22;

__device__ __forceinline__ uint64_t pack_status(uint64_t flag, uint32_t epoch, uint64_t v) {
    return flag | ((uint64_t)epoch << 40) | (v & VALUE_MASK);
}

}  // namespace

namespace {

constexpr int HNT = 256;

__global__ __launch_bounds__(HNT) void k_hist(const uint64_t* keys, uint64_t n, uint32_t bit_lo, uint32_t bit_hi,
                                              uint32_t n9, uint32_t dbits, uint32_t passes, uint64_t* hist) {
    __shared__ uint32_t h[8 * HSTRIDE];
    for (uint32_t i = threadIdx.x; i < passes * HSTRIDE; i += HNT) h[i] = 0;
    __syncthreads();
    for (uint64_t base = (uint64_t)blockIdx.x * HNT; base < n; base += (uint64_t)gridDim.x * HNT) {
        const uint64_t i = base + threadIdx.x;
        const bool valid = i < n;
        const uint64_t k = valid ? keys[i] : 0;
        for (uint32_t p = 0; p < passes; ++p) {
            const uint32_t mask = (1u << pass_bits(bit_lo, bit_hi, n9, dbits, p)) - 1;
            wave_hist_add(&h[p * HSTRIDE], (uint32_t)((k >> pass_shift(bit_lo, n9, dbits, p)) & mask), valid);
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < passes * HSTRIDE; i += HNT)
        if (h[i]) atomicAdd((unsigned long long*)&hist[i], (unsigned long long)h[i]);
}

// exclusive scan over the buckets of each pass (one workgroup per pass)
__global__ __launch_bounds__(HSTRIDE) void k_hist_scan(const uint64_t* hist, uint64_t* off) {
    __shared__ uint64_t scratch[HSTRIDE / 64];
    const uint64_t v = hist[blockIdx.x * HSTRIDE + threadIdx.x];
    uint64_t tot;
    const uint64_t ex = block_excl_scan<HSTRIDE, uint64_t>(v, scratch, &tot);
    off[blockIdx.x * HSTRIDE + threadIdx.x] = ex;
}

// LB = true: onesweep (dynamic tile order, decoupled look-back, digit_off =
// exclusive digit totals).  LB = false: the scatter of a reduce-then-scan pass
// (tile = block index, digit_off = exclusive scan of the per-tile counts laid
// out digit-major, so entry d * tiles + t is the tile's global base for d).
// RB: buckets of the digit (256, or 512 for 9-bit digits).  SPLIT: stage the
// keys, then the payloads (with their digits), through one LDS buffer of
// 8 B per pair that also holds the per-wave digit counts while the tile is
// ranked: about 70 KB for an 8192-pair tile, so two workgroups share a compute
// unit and one's ranking and look-back overlap the other's memory traffic.
template <int NT, int IPT, bool FINAL, bool LB, int RB, bool SPLIT>
__global__ __launch_bounds__(NT) void k_onesweep(const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                 uint64_t* __restrict__ kout, uint32_t* __restrict__ vout, uint64_t n,
                                                 uint32_t shift, uint32_t dbits, const uint64_t* __restrict__ digit_off,
                                                 uint64_t* lookback, uint32_t* tile_counter, uint32_t epoch,
                                                 uint32_t* status, FinalOut fo) {
    constexpr int TILE = NT * IPT;
    constexpr int WAVES = NT / 64;
    static_assert(NT >= RB, "one thread per digit");
    constexpr int STAGE_K = TILE * 8;            // bytes of the staged keys
    constexpr int WH = WAVES * RB * 4;           // bytes of the per-wave digit counts
    static_assert(!SPLIT || (WH <= STAGE_K && TILE * 6 <= STAGE_K), "split staging layout");
    __shared__ uint32_t s_tile;
    __shared__ uint32_t tile_start[RB];          // first LDS slot of each digit in the tile
    __shared__ uint64_t glob_base[RB];           // global position of the tile's first key of each digit
    __shared__ uint64_t scan_scratch[NT / 64];
    __shared__ __align__(16) unsigned char pool[SPLIT ? STAGE_K : STAGE_K + TILE * 4 + WH];
    auto wave_hist = reinterpret_cast<uint32_t (*)[RB]>(SPLIT ? pool : pool + STAGE_K + TILE * 4);
    uint64_t* stage_k = reinterpret_cast<uint64_t*>(pool);
    uint32_t* stage_v = reinterpret_cast<uint32_t*>(SPLIT ? pool : pool + STAGE_K);
    uint16_t* stage_d = reinterpret_cast<uint16_t*>(pool + TILE * 4);   // SPLIT: digit of each staged payload

    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (LB && threadIdx.x == 0) s_tile = atomicAdd(tile_counter, 1u);
    for (uint32_t i = threadIdx.x; i < WAVES * RB; i += NT) (&wave_hist[0][0])[i] = 0;
    __syncthreads();
    const uint64_t tile = LB ? (uint64_t)s_tile : (uint64_t)blockIdx.x;
    const uint64_t base = tile * TILE;
    const uint32_t mask = (1u << dbits) - 1;

    // striped load within each wave: item k of lane l is element base + wave*64*IPT + k*64 + l
    uint64_t key[IPT];
    uint32_t val[IPT];
    uint32_t rank[IPT];
    const uint64_t wbase = base + (uint64_t)wave * 64 * IPT + lane;
    if (base + TILE <= n) {      // full tile: no per-element guards
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
            key[k] = kin[wbase + (uint64_t)k * 64];
            val[k] = vin[wbase + (uint64_t)k * 64];
        }
    } else {
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
            const uint64_t i = wbase + (uint64_t)k * 64;
            key[k] = i < n ? kin[i] : 0ull;
            val[k] = i < n ? vin[i] : 0u;
        }
    }
    const uint64_t lt_mask = (1ull << lane) - 1;
    constexpr int MAXBITS = RB == 512 ? 9 : 8;   // digits of a pass have at most this many bits
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const uint64_t i = wbase + (uint64_t)k * 64;
        const bool valid = i < n;
        const uint32_t d = valid ? (uint32_t)((key[k] >> shift) & mask) : 0u;
        // lanes holding the same digit: one ballot per digit bit (bits above
        // dbits are zero in every lane and leave the set unchanged)
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < MAXBITS; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        uint32_t r = 0;
        if (valid) {
            const uint32_t before = wave_hist[wave][d];
            r = before + (uint32_t)__popcll(peers & lt_mask);
            // the highest peer advances the wave's counter of this digit
            if ((peers >> lane) == 1ull) wave_hist[wave][d] = before + (uint32_t)__popcll(peers);
        }
        rank[k] = r;
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();

    // per digit: tile count, per-wave offsets, look-back over earlier tiles
    const uint32_t d = threadIdx.x;
    const bool digit_thread = d < RB;
    uint32_t cnt = 0;
    uint32_t woff[WAVES];
    uint64_t excl = 0;
    if (digit_thread) {
#pragma unroll
        for (int w = 0; w < WAVES; ++w) {
            woff[w] = cnt;
            cnt += wave_hist[w][d];
        }
        uint64_t* my = lookback + tile * RB + d;
        if (!LB) {
            // offsets known from the reduce-then-scan counts
        } else if (tile == 0) {
            __hip_atomic_store(my, pack_status(FLAG_INC, epoch, cnt), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(my, pack_status(FLAG_AGG, epoch, cnt), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            int64_t pred = (int64_t)tile - 1;
            uint32_t spins = 0;
            while (pred >= 0) {
                const uint64_t st = __hip_atomic_load(lookback + (uint64_t)pred * RB + d, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
                const uint64_t flag = st & (3ull << 62);
                const uint32_t ep = (uint32_t)((st >> 40) & EPOCH_MAX);
                if (flag != 0 && ep == epoch) {
                    excl += st & VALUE_MASK;
                    if (flag == FLAG_INC) break;
                    --pred;
                    continue;
                }
                if (++spins > SPIN_LIMIT || __hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    atomicOr(status, 1u);   // bounded wait exceeded: flag the failure and finish the tile
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            __hip_atomic_store(my, pack_status(FLAG_INC, epoch, excl + cnt), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    // digit start within the tile (exclusive scan over digits)
    uint64_t tot;
    const uint32_t start = (uint32_t)block_excl_scan<NT, uint64_t>((uint64_t)cnt, scan_scratch, &tot);
    if (digit_thread) {
        tile_start[d] = start;
        glob_base[d] = LB ? digit_off[d] + excl : digit_off[(uint64_t)d * ((n + TILE - 1) / TILE) + tile];
#pragma unroll
        for (int w = 0; w < WAVES; ++w) wave_hist[w][d] = start + woff[w];
    }
    __syncthreads();

    const uint32_t tile_n = (uint32_t)min((uint64_t)TILE, n - base);
    if constexpr (SPLIT) {
        // slots first: the counts share the staging buffer
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
            const uint32_t dd = (uint32_t)((key[k] >> shift) & mask);
            rank[k] += wave_hist[wave][dd];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < IPT; ++k)
            if (wbase + (uint64_t)k * 64 < n) stage_k[rank[k]] = key[k];
        __syncthreads();
#pragma unroll 4
        for (uint32_t s = threadIdx.x; s < tile_n; s += NT) {
            const uint64_t k = stage_k[s];
            const uint32_t dd = (uint32_t)((k >> shift) & mask);
            const uint64_t g = glob_base[dd] + (s - tile_start[dd]);
            if constexpr (FINAL) {
                fo.src[g] = (int32_t)(k >> fo.tgt_shift);
                fo.tgt[g] = (int32_t)((k >> 16) & fo.tgt_mask);
                fo.delay[g] = (uint16_t)(k & 0xffffu);
            } else {
                kout[g] = k;
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < IPT; ++k)
            if (wbase + (uint64_t)k * 64 < n) {
                stage_v[rank[k]] = val[k];
                stage_d[rank[k]] = (uint16_t)((key[k] >> shift) & mask);
            }
        __syncthreads();
#pragma unroll 4
        for (uint32_t s = threadIdx.x; s < tile_n; s += NT) {
            const uint32_t dd = stage_d[s];
            const uint64_t g = glob_base[dd] + (s - tile_start[dd]);
            if constexpr (FINAL) fo.weight[g] = __uint_as_float(stage_v[s]);
            else vout[g] = stage_v[s];
        }
        return;
    }

    // stage in digit order
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const uint64_t i = wbase + (uint64_t)k * 64;
        if (i < n) {
            const uint32_t dd = (uint32_t)((key[k] >> shift) & mask);
            const uint32_t slot = wave_hist[wave][dd] + rank[k];
            stage_k[slot] = key[k];
            stage_v[slot] = val[k];
        }
    }
    __syncthreads();

#pragma unroll 4
    for (uint32_t s = threadIdx.x; s < tile_n; s += NT) {
        const uint64_t k = stage_k[s];
        const uint32_t dd = (uint32_t)((k >> shift) & mask);
        const uint64_t g = glob_base[dd] + (s - tile_start[dd]);
        if constexpr (FINAL) {
            fo.src[g] = (int32_t)(k >> fo.tgt_shift);
            fo.tgt[g] = (int32_t)((k >> 16) & fo.tgt_mask);
            fo.delay[g] = (uint16_t)(k & 0xffffu);
            fo.weight[g] = __uint_as_float(stage_v[s]);
        } else {
            kout[g] = k;
            vout[g] = stage_v[s];
        }
    }
}

__global__ void k_unpack(const uint64_t* keys, const uint32_t* vals, uint64_t n, FinalOut fo) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t k = keys[i];
    fo.src[i] = (int32_t)(k >> fo.tgt_shift);
    fo.tgt[i] = (int32_t)((k >> 16) & fo.tgt_mask);
    fo.delay[i] = (uint16_t)(k & 0xffffu);
    fo.weight[i] = __uint_as_float(vals[i]);
}

struct PassArgs {
    const uint64_t* kin;
    const uint32_t* vin;
    uint64_t* kout;
    uint32_t* vout;
    uint64_t n;
    uint32_t shift, dbits;
    const uint64_t* off;
    uint64_t* lookback;
    uint32_t* counter;
    uint32_t epoch;
    uint32_t* status;
    FinalOut fo;
    int mode;   // 0: onesweep, 1: reduce-then-scan
};

// Digit counts of every tile of a pass, digit-major (counts[d * tiles + t]),
// for the reduce-then-scan form of a pass.
template <int NT, int IPT, int RB>
__global__ __launch_bounds__(NT) void k_tile_counts(const uint64_t* __restrict__ kin, uint64_t n, uint32_t shift,
                                                    uint32_t dbits, uint32_t* counts) {
    constexpr int TILE = NT * IPT;
    __shared__ uint32_t h[RB];
    for (uint32_t i = threadIdx.x; i < RB; i += NT) h[i] = 0;
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t tiles = (n + TILE - 1) / TILE;
    const uint64_t wbase = (uint64_t)blockIdx.x * TILE + (uint64_t)wave * 64 * IPT + lane;
    const uint32_t mask = (1u << dbits) - 1;
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const uint64_t i = wbase + (uint64_t)k * 64;
        const bool valid = i < n;
        const uint32_t d = valid ? (uint32_t)((kin[i] >> shift) & mask) : 0u;
        wave_hist_add(h, d, valid);
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < RB; d += NT) counts[(uint64_t)d * tiles + blockIdx.x] = h[d];
}

template <int NT, int IPT, int RB, bool SPLIT = false>
void launch_pass(Ctx& c, const PassArgs& a, bool final) {
    constexpr int TILE = NT * IPT;
    const uint64_t tiles = (a.n + TILE - 1) / TILE;
    const uint64_t* off = a.off;
    std::vector<void*> temps;
    if (a.mode == 1) {
        // reduce-then-scan: per-tile counts, one scan, scatter with known bases
        uint32_t* counts = dalloc_n<uint32_t>(c, tiles * RB);
        temps.push_back(counts);
        uint64_t* scanned = dalloc_n<uint64_t>(c, tiles * RB + 1);
        temps.push_back(scanned);
        hipLaunchKernelGGL((k_tile_counts<NT, IPT, RB>), dim3((unsigned)tiles), dim3(NT), 0, c.stream, a.kin, a.n,
                           a.shift, a.dbits, counts);
        HIPCHK(hipGetLastError());
        scan_u32_u64(c, counts, scanned, tiles * RB, false);
        off = scanned;
        if (final)
            hipLaunchKernelGGL((k_onesweep<NT, IPT, true, false, RB, SPLIT>), dim3((unsigned)tiles), dim3(NT), 0, c.stream,
                               a.kin, a.vin, a.kout, a.vout, a.n, a.shift, a.dbits, off, a.lookback, a.counter, a.epoch,
                               a.status, a.fo);
        else
            hipLaunchKernelGGL((k_onesweep<NT, IPT, false, false, RB, SPLIT>), dim3((unsigned)tiles), dim3(NT), 0, c.stream,
                               a.kin, a.vin, a.kout, a.vout, a.n, a.shift, a.dbits, off, a.lookback, a.counter, a.epoch,
                               a.status, a.fo);
    } else if (final) {
        hipLaunchKernelGGL((k_onesweep<NT, IPT, true, true, RB, SPLIT>), dim3((unsigned)tiles), dim3(NT), 0, c.stream, a.kin,
                           a.vin, a.kout, a.vout, a.n, a.shift, a.dbits, off, a.lookback, a.counter, a.epoch, a.status,
                           a.fo);
    } else {
        hipLaunchKernelGGL((k_onesweep<NT, IPT, false, true, RB, SPLIT>), dim3((unsigned)tiles), dim3(NT), 0, c.stream, a.kin,
                           a.vin, a.kout, a.vout, a.n, a.shift, a.dbits, off, a.lookback, a.counter, a.epoch, a.status,
                           a.fo);
    }
    HIPCHK(hipGetLastError());
    for (void* p : temps) dfree(c, p);   // stream-ordered release
}

struct Variant {
    int nt, ipt;
    bool split;   // keys and payloads staged through LDS one after the other
};
// tile shapes available to the tuner; index 0 is the default, the fastest
// measured for sorts of 4e8 .. 2e9 pairs: 8192-pair tiles (digit runs long
// enough for whole-line writes) staged in two phases, so that two workgroups
// share each compute unit
constexpr Variant VARIANTS[] = {{512, 16, true},  {256, 8, false},  {512, 8, false}, {512, 16, false},
                                {256, 16, false}, {256, 12, false}, {1024, 8, false}, {1024, 8, true},
                                {512, 8, true},   {512, 12, true},  {256, 16, true},  {512, 11, true},
                                {1024, 16, true}, {768, 12, true}};
constexpr int N_VARIANTS = sizeof(VARIANTS) / sizeof(VARIANTS[0]);

// autotuner results for the process: (pass algorithm, tile shape) per size
// class; used by every context whose sort settings were not set by hand
struct TuneKey {
    int size_class;   // floor(log2 n)
    uint32_t bits;
    bool operator<(const TuneKey& o) const { return size_class != o.size_class ? size_class < o.size_class : bits < o.bits; }
};

std::map<TuneKey, std::pair<int, int>>& tune_cache() {
    static std::map<TuneKey, std::pair<int, int>> m;
    return m;
}

int log2_floor(uint64_t n) {
    int l = 0;
    while (n >>= 1) ++l;
    return l;
}

void launch_variant(Ctx& c, int v, const PassArgs& a, bool final, bool wide) {
    if (wide) {   // 9-bit digits: tile shapes with at least 512 threads
        switch (v) {
        case 2: launch_pass<512, 8, 512>(c, a, final); break;
        case 3: launch_pass<512, 16, 512>(c, a, final); break;
        case 0: launch_pass<512, 16, 512, true>(c, a, final); break;
        case 6: launch_pass<1024, 8, 512>(c, a, final); break;
        case 7: launch_pass<1024, 8, 512, true>(c, a, final); break;
        case 8: launch_pass<512, 8, 512, true>(c, a, final); break;
        case 9: launch_pass<512, 12, 512, true>(c, a, final); break;
        case 11: launch_pass<512, 11, 512, true>(c, a, final); break;
        case 12: launch_pass<1024, 16, 512, true>(c, a, final); break;
        case 13: launch_pass<768, 12, 512, true>(c, a, final); break;
        default: raise(SNNC_EINVAL, "9-bit digits need a tile of at least 512 threads");
        }
        return;
    }
    switch (v) {
    case 1: launch_pass<256, 8, RADIX>(c, a, final); break;
    case 2: launch_pass<512, 8, RADIX>(c, a, final); break;
    case 3: launch_pass<512, 16, RADIX>(c, a, final); break;
    case 4: launch_pass<256, 16, RADIX>(c, a, final); break;
    case 5: launch_pass<256, 12, RADIX>(c, a, final); break;
    case 6: launch_pass<1024, 8, RADIX>(c, a, final); break;
    case 7: launch_pass<1024, 8, RADIX, true>(c, a, final); break;
    case 8: launch_pass<512, 8, RADIX, true>(c, a, final); break;
    case 9: launch_pass<512, 12, RADIX, true>(c, a, final); break;
    case 10: launch_pass<256, 16, RADIX, true>(c, a, final); break;
    case 11: launch_pass<512, 11, RADIX, true>(c, a, final); break;
    case 12: launch_pass<1024, 16, RADIX, true>(c, a, final); break;
    case 13: launch_pass<768, 12, RADIX, true>(c, a, final); break;
    default: launch_pass<512, 16, RADIX, true>(c, a, final); break;
    }
}

}  // namespace

int sort_variant_count() { return N_VARIANTS; }

// Pass algorithm, tile shape and digit plan of a sort of n keys over `bits`
// bits.  9-bit digits (512 buckets) are taken when the tile has at least 512
// threads and they save a pass over 8-bit digits (or when forced).
SortPlan plan_sort(const Ctx& c, uint64_t n, uint32_t bits) {
    SortPlan p;
    p.variant = (c.sort_variant >= 0 && c.sort_variant < N_VARIANTS) ? c.sort_variant : 0;
    p.mode = c.sort_mode;
    if (!c.sort_pinned) {
        auto it = tune_cache().find(TuneKey{log2_floor(std::max<uint64_t>(n, 1)), bits});
        if (it != tune_cache().end()) {
            p.mode = it->second.first;
            p.variant = it->second.second;
        }
    }
    const uint32_t p8 = (bits + 7) / 8, p9 = (bits + 8) / 9;
    const bool can9 = VARIANTS[p.variant].nt >= 512;
    const bool use9 = can9 && (c.digit_bits == 9 || (c.digit_bits == 0 && p9 < p8));
    p.passes = use9 ? p9 : p8;
    if (use9 && c.digit_bits == 9) {          // forced: every pass 9 bits
        p.n9 = p.passes;
        p.dbits = 9;
    } else if (use9) {                         // as few 9-bit passes as the pass count allows
        p.n9 = bits - 8 * p.passes;           // (a 9-bit pass costs more than an 8-bit one)
        p.dbits = 8;
    } else {
        p.n9 = 0;
        p.dbits = p.passes ? (bits + p.passes - 1) / p.passes : 0;
    }
    p.wide = p.n9 > 0;
    return p;
}

// Timer name of a radix-sort step: "sort_<step>", or "<sort_tag>_<step>" for
// the sorts that generation runs (kept out of the Prepare phase's figures).
std::string sort_timer(const Ctx& c, const char* step) {
    return std::string(c.sort_tag ? c.sort_tag : "sort") + "_" + step;
}

void launch_hist(Ctx& c, const uint64_t* keys, uint64_t n, uint32_t bit_lo, uint32_t bit_hi, uint32_t n9,
                 uint32_t dbits, uint32_t passes, uint64_t* hist) {
    HIPCHK(hipMemsetAsync(hist, 0, (size_t)passes * HSTRIDE * 8, c.stream));
    if (!n || !passes) return;
    const uint32_t grid = (uint32_t)std::min<uint64_t>((n + HNT - 1) / HNT, 4096);
    tstart(c, sort_timer(c, "hist").c_str());
    hipLaunchKernelGGL(k_hist, dim3(grid), dim3(HNT), 0, c.stream, keys, n, bit_lo, bit_hi, n9, dbits, passes, hist);
    tstop(c);
    HIPCHK(hipGetLastError());
}

namespace {

__global__ void k_fill_words(uint64_t* p, uint64_t n, uint64_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// clears n 64-bit words with a kernel (no memset node in a captured stream)
void fill_words(Ctx& c, uint64_t* p, uint64_t n) {
    if (!n) return;
    const unsigned grid = (unsigned)std::min<uint64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_words, dim3(grid), dim3(256), 0, c.stream, p, n, 0ull);
    HIPCHK(hipGetLastError());
}

// Scratch of a sort that allocates nothing: digit histograms and offsets,
// tile counters, a status word and the look-back table, all at fixed
// addresses; the look-back epoch persists with the table.
struct FixedScratch {
    uint64_t* hist;
    uint64_t* off;
    uint32_t* counter;
    uint32_t* status;
    void* lookback;
    size_t lookback_bytes;
    uint32_t* epoch;
};

int radix_sort_impl(Ctx& c, uint64_t* keys0, uint32_t* vals0, uint64_t* keys1, uint32_t* vals1, uint64_t n,
                    uint32_t bit_lo, uint32_t bit_hi, const uint64_t* digit_hist, const FinalOut* final_out,
                    bool wait_for_plan, const FixedScratch* fs) {
    const SortPlan plan = plan_sort(c, n, bit_hi > bit_lo ? bit_hi - bit_lo : 0);
    const uint32_t passes = plan.passes, dbits = plan.dbits;
    // the reduce-then-scan passes allocate per-tile counts: fixed scratch takes onesweep passes
    const int variant = plan.variant, mode = fs ? 0 : plan.mode;
    const uint32_t rb = plan.wide ? 512 : RADIX;
    if (passes > 8) raise(SNNC_EUNSUPPORTED, "radix sort over more than 64 bits");
    const uint64_t tile = (uint64_t)VARIANTS[variant].nt * VARIANTS[variant].ipt;
    const uint64_t tiles = (n + tile - 1) / tile;
    if (fs && passes && n && (size_t)tiles * rb * 8 > fs->lookback_bytes)
        raise(SNNC_EINVAL, "sort of " + std::to_string(n) + " keys needs a look-back table of " +
                               std::to_string((size_t)tiles * rb * 8) + " bytes, above the " +
                               std::to_string(fs->lookback_bytes) + " of the static scratch");
    void* temps[3] = {nullptr, nullptr, nullptr};
    auto cleanup = [&] {
        for (void* p : temps) dfree(c, p);
    };
    uint32_t* status = fs ? fs->status : c.d_status;
    void* lookback = fs ? fs->lookback : c.lookback;
    uint32_t& epoch = fs ? *fs->epoch : c.sort_epoch;
    const size_t lookback_bytes = fs ? fs->lookback_bytes : 0;
    int cur = 0;
    try {
        uint64_t hh[8 * HSTRIDE];
        memset(hh, 0, sizeof hh);
        uint64_t* off = nullptr;
        if (passes && n) {
            uint64_t* hist = const_cast<uint64_t*>(digit_hist);
            if (!hist && fs) {
                hist = fs->hist;
                fill_words(c, hist, (uint64_t)passes * HSTRIDE);
                const uint32_t grid = (uint32_t)std::min<uint64_t>((n + HNT - 1) / HNT, 4096);
                hipLaunchKernelGGL(k_hist, dim3(grid), dim3(HNT), 0, c.stream, keys0, n, bit_lo, bit_hi, plan.n9, dbits,
                                   passes, hist);
                HIPCHK(hipGetLastError());
            } else if (!hist) {
                hist = dalloc_n<uint64_t>(c, (uint64_t)passes * HSTRIDE);
                temps[0] = hist;
                launch_hist(c, keys0, n, bit_lo, bit_hi, plan.n9, dbits, passes, hist);
            }
            if (fs) {
                off = fs->off;
            } else {
                off = dalloc_n<uint64_t>(c, (uint64_t)passes * HSTRIDE);
                temps[1] = off;
            }
            tstart(c, sort_timer(c, "hist_scan").c_str());
            hipLaunchKernelGGL(k_hist_scan, dim3(passes), dim3(HSTRIDE), 0, c.stream, hist, off);
            tstop(c);
            HIPCHK(hipGetLastError());
            if (wait_for_plan) download(c, hh, hist, (size_t)passes * HSTRIDE * 8);
            // look-back table: tiles x buckets status words, zeroed once when (re)allocated
            const size_t need = (size_t)tiles * rb * 8;
            if (!fs && c.lookback_bytes < need) {
                dfree(c, c.lookback);
                c.lookback = nullptr;
                c.lookback_bytes = 0;
                c.lookback = dalloc(c, need);
                c.lookback_bytes = need;
                HIPCHK(hipMemsetAsync(c.lookback, 0, need, c.stream));
                c.sort_epoch = 0;
                lookback = c.lookback;
            }
        }
        uint32_t* counter;
        if (fs) {
            counter = fs->counter;
            fill_words(c, reinterpret_cast<uint64_t*>(counter), 4);   // 8 tile counters
        } else {
            counter = dalloc_n<uint32_t>(c, std::max<uint32_t>(passes, 1));
            temps[2] = counter;
            HIPCHK(hipMemsetAsync(counter, 0, std::max<uint32_t>(passes, 1) * 4, c.stream));
        }
        // passes whose digit is the same for every key leave the order unchanged
        uint32_t live[8];
        uint32_t n_live = 0;
        for (uint32_t p = 0; p < passes; ++p) {
            bool trivial = false;
            for (int b = 0; b < HSTRIDE; ++b)
                if (hh[(size_t)p * HSTRIDE + b] == n) trivial = true;
            if (!trivial) live[n_live++] = p;
        }
        c.sort_passes = n_live;
        uint64_t* kb[2] = {keys0, keys1};
        uint32_t* vb[2] = {vals0, vals1};
        for (uint32_t li = 0; li < n_live; ++li) {
            const uint32_t p = live[li];
            if (++epoch > EPOCH_MAX) {
                if (fs) fill_words(c, static_cast<uint64_t*>(lookback), lookback_bytes / 8);
                else HIPCHK(hipMemsetAsync(c.lookback, 0, c.lookback_bytes, c.stream));
                epoch = 1;
            }
            const bool last = (li + 1 == n_live) && final_out;
            const uint32_t width = pass_bits(bit_lo, bit_hi, plan.n9, dbits, p);
            PassArgs a{kb[cur], vb[cur], kb[cur ^ 1], vb[cur ^ 1], n, pass_shift(bit_lo, plan.n9, dbits, p), width,
                       off + (size_t)p * HSTRIDE, (uint64_t*)lookback, counter + p, epoch, status,
                       final_out ? *final_out : FinalOut{}, mode};
            tstart(c, sort_timer(c, last ? "pass_final" : "pass").c_str());
            launch_variant(c, variant, a, last, width > 8);
            tstop(c);
            HIPCHK(hipGetLastError());
            cur ^= 1;
        }
        if (final_out && !n_live && n) {
            tstart(c, sort_timer(c, "unpack").c_str());
            hipLaunchKernelGGL(k_unpack, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c.stream, kb[cur], vb[cur], n,
                               *final_out);
            tstop(c);
            HIPCHK(hipGetLastError());
        }
    } catch (...) {
        cleanup();
        throw;
    }
    cleanup();
    return cur;
}

}  // namespace

int radix_sort(Ctx& c, uint64_t* keys0, uint32_t* vals0, uint64_t* keys1, uint32_t* vals1, uint64_t n,
               uint32_t bit_lo, uint32_t bit_hi, const uint64_t* digit_hist, const FinalOut* final_out,
               bool wait_for_plan) {
    return radix_sort_impl(c, keys0, vals0, keys1, vals1, n, bit_lo, bit_hi, digit_hist, final_out, wait_for_plan,
                           nullptr);
}

}  // namespace snnc

// ------------------------------------------------------------------ autotuner
namespace snnc {
namespace {

__global__ void k_random_keys(uint64_t* keys, uint32_t* vals, uint64_t n, uint32_t bit_lo, uint32_t bits,
                              uint32_t seed) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 b = draw(seed, 0x7ea5u, i, PURPOSE_IDX);
    const uint64_t r = ((uint64_t)b.y << 32) | b.x;
    keys[i] = bits >= 64 ? r : ((r & ((1ull << bits) - 1)) << bit_lo);
    vals[i] = (uint32_t)i;
}

}  // namespace

// Time every (pass algorithm, tile shape) on n synthetic keys with `bits`
// sorted bits; keep the fastest in the context and in the process cache.
void autotune_sort(Ctx& c, uint64_t n, uint32_t bits, int* mode_out, int* variant_out, float* ms_out) {
    const TuneKey key{log2_floor(std::max<uint64_t>(n, 1)), bits};
    auto it = tune_cache().find(key);
    if (it != tune_cache().end()) {
        c.sort_mode = it->second.first;
        c.sort_variant = it->second.second;
        *mode_out = c.sort_mode;
        *variant_out = c.sort_variant;
        *ms_out = -1.f;
        return;
    }
    uint64_t* k0 = dalloc_n<uint64_t>(c, n);
    uint64_t* k1 = dalloc_n<uint64_t>(c, n);
    uint32_t* v0 = dalloc_n<uint32_t>(c, n);
    uint32_t* v1 = dalloc_n<uint32_t>(c, n);
    hipEvent_t a, b;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    int best_mode = 0, best_var = 0;
    float best = 1e30f;
    const int saved_mode = c.sort_mode, saved_var = c.sort_variant;
    const bool saved_timing = c.timing, saved_pinned = c.sort_pinned;
    c.timing = false;
    c.sort_pinned = true;   // each candidate runs as set
    try {
        for (int mode = 0; mode < 2; ++mode) {
            for (int v = 0; v < N_VARIANTS; ++v) {
                c.sort_mode = mode;
                c.sort_variant = v;
                float t_best = 1e30f;
                for (int rep = 0; rep < 2; ++rep) {
                    hipLaunchKernelGGL(k_random_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c.stream, k0, v0,
                                       n, 16, bits, 1234u);
                    HIPCHK(hipGetLastError());
                    HIPCHK(hipEventRecord(a, c.stream));
                    radix_sort(c, k0, v0, k1, v1, n, 16, 16 + bits, nullptr, nullptr);
                    HIPCHK(hipEventRecord(b, c.stream));
                    HIPCHK(hipEventSynchronize(b));
                    float ms = 0.f;
                    HIPCHK(hipEventElapsedTime(&ms, a, b));
                    t_best = std::min(t_best, ms);
                }
                if (t_best < best) {
                    best = t_best;
                    best_mode = mode;
                    best_var = v;
                }
            }
        }
    } catch (...) {
        c.sort_mode = saved_mode;
        c.sort_variant = saved_var;
        c.timing = saved_timing;
        c.sort_pinned = saved_pinned;
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        dfree(c, k0); dfree(c, k1); dfree(c, v0); dfree(c, v1);
        throw;
    }
    c.timing = saved_timing;
    c.sort_pinned = saved_pinned;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    dfree(c, k0); dfree(c, k1); dfree(c, v0); dfree(c, v1);
    c.sort_mode = best_mode;
    c.sort_variant = best_var;
    tune_cache()[key] = {best_mode, best_var};
    *mode_out = best_mode;
    *variant_out = best_var;
    *ms_out = best;
}

}  // namespace snnc

extern "C" snnc_status snnc_autotune_sort(snnc_ctx* ctx, uint64_t n, uint32_t bits, int32_t* mode_out,
                                          int32_t* variant_out, float* ms_out) {
    using namespace snnc;
    if (!ctx || !mode_out || !variant_out || !ms_out || bits == 0 || bits > 48) return SNNC_EINVAL;
    try {
        HIPCHK(hipSetDevice(ctx->device));
        int m = 0, v = 0;
        float ms = 0.f;
        autotune_sort(*ctx, std::max<uint64_t>(n, 1), bits, &m, &v, &ms);
        *mode_out = m;
        *variant_out = v;
        *ms_out = ms;
        return SNNC_OK;
    } catch (const Error& e) {
        ctx->last_error = e.msg;
        return e.code;
    }
}

extern "C" snnc_status snnc_sort_pairs(snnc_ctx* ctx, uint64_t* keys, uint32_t* vals, uint64_t* keys_tmp,
                                       uint32_t* vals_tmp, uint64_t n, uint32_t bit_lo, uint32_t bit_hi,
                                       int32_t* result_in_tmp) {
    using namespace snnc;
    if (!ctx || !result_in_tmp || (n && (!keys || !vals || !keys_tmp || !vals_tmp)) || bit_hi > 64 || bit_lo > bit_hi)
        return SNNC_EINVAL;
    try {
        HIPCHK(hipSetDevice(ctx->device));
        *result_in_tmp = radix_sort(*ctx, keys, vals, keys_tmp, vals_tmp, n, bit_lo, bit_hi, nullptr, nullptr);
        uint32_t status = 0;
        download(*ctx, &status, ctx->d_status, 4);
        if (status) raise(SNNC_EDEVICE, "a device wait exceeded its bound");
        return SNNC_OK;
    } catch (const Error& e) {
        ctx->last_error = e.msg;
        return e.code;
    }
}

// ------------------------------------------------------------------ allocation-free sort
// One static scratch array per GPU, for callers that cannot allocate device
// memory.  Layout: digit histograms (8 passes x 512 u64), their offsets
// (same), 8 tile counters and a status word (256 B), then the look-back
// table.  Host code reaches it only through the address that
// hipGetSymbolAddress gives for the current device.
namespace snnc {
namespace {

constexpr size_t NA_BYTES = 16u << 20;
constexpr size_t NA_HIST = 0;
constexpr size_t NA_OFF = NA_HIST + 8 * HSTRIDE * 8;
constexpr size_t NA_CNT = NA_OFF + 8 * HSTRIDE * 8;
constexpr size_t NA_STATUS = NA_CNT + 8 * 4;
constexpr size_t NA_LB = NA_CNT + 256;
constexpr size_t NA_LB_BYTES = NA_BYTES - NA_LB;
constexpr int NA_MAX_DEVICES = 64;

struct NoallocDevice {
    char* ptr = nullptr;    // device address of `scratch` on this GPU
    uint32_t epoch = 0;     // look-back epoch of the last pass run on it
};

std::mutex& na_mutex() {
    static std::mutex m;
    return m;
}

NoallocDevice* na_devices() {
    static NoallocDevice d[NA_MAX_DEVICES];
    return d;
}

}  // namespace
}  // namespace snnc

static __device__ __align__(256) unsigned char scratch[snnc::NA_BYTES];

namespace snnc {

// Called by snnc_init with the context's device current: takes the device
// address of the static scratch once per device and clears its look-back
// table (a fill kernel on the context stream, waited for).
void noalloc_setup(Ctx& c) {
    if (c.device < 0 || c.device >= NA_MAX_DEVICES) return;
    std::lock_guard<std::mutex> lock(na_mutex());
    NoallocDevice& d = na_devices()[c.device];
    if (d.ptr) return;
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    char* base = static_cast<char*>(p);
    fill_words(c, reinterpret_cast<uint64_t*>(base + NA_LB), NA_LB_BYTES / 8);
    HIPCHK(hipStreamSynchronize(c.stream));
    d.ptr = base;
    d.epoch = 0;
}

}  // namespace snnc

extern "C" snnc_status snnc_sort_pairs_noalloc(snnc_ctx* ctx, uint64_t* keys, uint32_t* vals, uint64_t* keys_tmp,
                                               uint32_t* vals_tmp, uint64_t n, uint32_t bit_lo, uint32_t bit_hi,
                                               int32_t* result_in_tmp) {
    using namespace snnc;
    if (!ctx || !result_in_tmp || (n && (!keys || !vals || !keys_tmp || !vals_tmp)) || bit_hi > 64 || bit_lo > bit_hi)
        return SNNC_EINVAL;
    try {
        HIPCHK(hipSetDevice(ctx->device));
        if (ctx->device < 0 || ctx->device >= NA_MAX_DEVICES) raise(SNNC_EUNSUPPORTED, "device ordinal above 63");
        std::lock_guard<std::mutex> lock(na_mutex());
        NoallocDevice& d = na_devices()[ctx->device];
        if (!d.ptr) raise(SNNC_ESTATE, "static scratch not set up on this device");
        FixedScratch fs{reinterpret_cast<uint64_t*>(d.ptr + NA_HIST), reinterpret_cast<uint64_t*>(d.ptr + NA_OFF),
                        reinterpret_cast<uint32_t*>(d.ptr + NA_CNT), reinterpret_cast<uint32_t*>(d.ptr + NA_STATUS),
                        d.ptr + NA_LB, NA_LB_BYTES, &d.epoch};
        const int saved_timing = ctx->timing;
        ctx->timing = 0;   // timing brackets would create events
        fill_words(*ctx, reinterpret_cast<uint64_t*>(d.ptr + NA_CNT), 32);   // counters and status word
        int which = 0;
        try {
            which = radix_sort_impl(*ctx, keys, vals, keys_tmp, vals_tmp, n, bit_lo, bit_hi, nullptr, nullptr, true,
                                    &fs);
        } catch (...) {
            ctx->timing = saved_timing;
            throw;
        }
        ctx->timing = saved_timing;
        uint32_t status = 0;
        download(*ctx, &status, d.ptr + NA_STATUS, 4);
        if (status) raise(SNNC_EDEVICE, "a device wait exceeded its bound");
        *result_in_tmp = which;
        return SNNC_OK;
    } catch (const Error& e) {
        ctx->last_error = e.msg;
        return e.code;
    }
}
