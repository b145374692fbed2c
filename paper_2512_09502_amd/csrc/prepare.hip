// Simulation preparation on the GPU:
//  1. mark every remote source used by a local connection in a bit set over
//     (a = alpha + 1, global neuron id), global id = host base + local id;
//  2. popcount prefix of the bit set = image numbering in (a, sigma, source)
//     order; R = the set bits per (a, sigma);
//  3. remap each connection's source (local id, or M_local + rank of its bit:
//     the lower_bound of the source in R plus the map's first image) and
//     build the 64-bit sort key (source', target, delay), with the digit
//     histograms of every radix pass in the same read;
//  4. source-major radix sort, unpacked into the result arrays;
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
    uint32_t a;   // alpha + 1
};

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

// source of connection i: host, local id and the bit index (a G + global id)
__device__ __forceinline__ void source_of(const Lookup& L, const uint32_t* g_src, uint64_t i, uint32_t& host,
                                          uint32_t& local, uint64_t& bit) {
    const CallD c = L.calls[find_call(L.calls, L.ncalls, i)];
    set_lookup(c.S, c.nS, g_src[i], host, local);
    bit = (uint64_t)c.a * L.G + L.host_base[host] + local;
}

// The same with a per-thread cache of the current call and source segment:
// a thread walks increasing positions, so the binary searches run only when
// the position leaves the cached call or the ordinal leaves the cached segment.
struct SourceCursor {
    uint64_t call_lo = 1, call_hi = 0;   // cached call covers [call_lo, call_hi)
    CallD call{};
    uint64_t seg_lo = 1, seg_hi = 0;     // cached segment covers ordinals [seg_lo, seg_hi)
    uint32_t seg_host = 0, seg_first = 0;
    uint64_t bit_base = 0;               // a G + host_base[seg_host] + seg_first - seg_lo

    __device__ __forceinline__ void at(const Lookup& L, uint64_t i, uint32_t ord, uint32_t& host, uint32_t& local,
                                       uint64_t& bit) {
        if (i < call_lo || i >= call_hi) {
            const uint32_t k = find_call(L.calls, L.ncalls, i);
            call = L.calls[k];
            call_lo = call.gen_begin;
            call_hi = k + 1 < L.ncalls ? L.calls[k + 1].gen_begin : ~0ull;
            seg_lo = 1;
            seg_hi = 0;
        }
        if (ord < seg_lo || ord >= seg_hi) {
            uint32_t a = 0, b = call.nS;
            while (b - a > 1) {
                const uint32_t m = (a + b) >> 1;
                if (call.S[m].ord_begin <= ord) a = m; else b = m;
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

__global__ __launch_bounds__(PNT) void k_mark(Lookup L, const uint32_t* g_src, uint64_t first, uint64_t end,
                                              uint32_t* bits) {
    uint64_t lo, hi;
    block_range(end - first, lo, hi);
    SourceCursor cur;
    for (uint64_t i = first + lo + threadIdx.x; i < first + hi; i += PNT) {
        uint32_t h, l;
        uint64_t bit;
        cur.at(L, i, g_src[i], h, l, bit);
        if (h != L.PL) atomicOr(bits + (bit >> 5), 1u << (bit & 31));
    }
}

__device__ __forceinline__ uint64_t rank_of(const uint32_t* bits, const uint64_t* word_rank, uint64_t bit) {
    const uint64_t w = bit >> 5;
    return word_rank[w] + (uint64_t)__popc(bits[w] & ((1u << (bit & 31)) - 1u));
}

// R: the set bits, in order, as local ids of their host
__global__ __launch_bounds__(PNT) void k_rvals(const uint32_t* bits, const uint64_t* word_rank, uint64_t n_words,
                                               const uint64_t* host_base, uint32_t P, uint64_t G, int32_t* R) {
    for (uint64_t w = (uint64_t)blockIdx.x * PNT + threadIdx.x; w < n_words; w += (uint64_t)gridDim.x * PNT) {
        uint32_t word = bits[w];
        uint64_t pos = word_rank[w];
        while (word) {
            const uint32_t b = __ffs(word) - 1;
            word &= word - 1;
            const uint64_t gid = (w * 32 + b) % G;
            uint32_t lo = 0, hi = P;   // host: last with host_base <= gid
            while (hi - lo > 1) {
                const uint32_t m = (lo + hi) >> 1;
                if (host_base[m] <= gid) lo = m; else hi = m;
            }
            R[pos++] = (int32_t)(gid - host_base[lo]);
        }
    }
}

// r_off[a P + sigma] = rank of the first bit of (a, sigma); r_off[n_a P] = n_img
__global__ void k_bounds(const uint32_t* bits, const uint64_t* word_rank, const uint64_t* host_base, uint32_t P,
                         uint32_t n_a, uint64_t G, uint32_t M_local, uint64_t* r_off, int64_t* img_base) {
    const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t nk = (uint64_t)n_a * P;
    if (k > nk) return;
    uint64_t r;
    if (k == nk) {
        r = rank_of(bits, word_rank, (uint64_t)n_a * G);
    } else {
        const uint64_t a = k / P, sigma = k % P;
        r = rank_of(bits, word_rank, a * G + host_base[sigma]);
        img_base[k] = (int64_t)M_local + (int64_t)r;
    }
    r_off[k] = r;
}

// source' and the sort key (source' << tgt_shift | target << 16 | delay),
// with the digit histograms of all radix passes
__global__ __launch_bounds__(PNT) void k_keys(Lookup L, const uint32_t* g_src, const uint32_t* g_tgt,
                                              const uint16_t* g_delay, uint64_t n, const uint32_t* bits,
                                              const uint64_t* word_rank, uint32_t M_local, uint32_t tgt_shift,
                                              uint32_t dbits, uint32_t passes, uint64_t* keys, uint64_t* hist) {
    __shared__ uint32_t h[8 * 256];
    for (uint32_t i = threadIdx.x; i < passes * 256; i += PNT) h[i] = 0;
    __syncthreads();
    const uint32_t dmask = (1u << dbits) - 1;
    uint64_t lo, hi;
    block_range(n, lo, hi);
    SourceCursor cur;
    for (uint64_t base = lo; base < hi; base += PNT) {
        const uint64_t i = base + threadIdx.x;
        const bool valid = i < hi;
        uint64_t key = 0;
        if (valid) {
            uint32_t host, local;
            uint64_t bit;
            cur.at(L, i, g_src[i], host, local, bit);
            const uint64_t src2 = host == L.PL ? local : (uint64_t)M_local + rank_of(bits, word_rank, bit);
            key = (src2 << tgt_shift) | ((uint64_t)g_tgt[i] << 16) | g_delay[i];
            keys[i] = key;
        }
        for (uint32_t p = 0; p < passes; ++p)
            wave_hist_add(&h[p * 256], (uint32_t)((key >> (16 + p * dbits)) & dmask), valid);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < passes * 256; i += PNT)
        if (h[i]) atomicAdd((unsigned long long*)&hist[i], (unsigned long long)h[i]);
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
                                            const uint64_t* word_rank, const uint64_t* host_base, uint64_t G,
                                            uint32_t PL, uint32_t M_local, int32_t* H, int32_t* I) {
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
            if ((bits[bit >> 5] >> (bit & 31)) & 1u) img = (int32_t)((uint64_t)M_local + rank_of(bits, word_rank, bit));
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
        std::vector<CallD> calls;
        for (auto& cl : c.calls)
            if (cl.gen_count) calls.push_back(CallD{cl.gen_begin, cl.dS, (uint32_t)cl.S.seg.size(), (uint32_t)(cl.alpha + 1)});
        if (calls.empty()) calls.push_back(CallD{0, nullptr, 0, 0});
        CallD* d_calls = static_cast<CallD*>(tmp(calls.size() * sizeof(CallD)));
        upload(c, d_calls, calls.data(), calls.size() * sizeof(CallD));
        uint64_t* d_hb = static_cast<uint64_t*>(tmp((P + 1) * 8));
        upload(c, d_hb, host_base.data(), (P + 1) * 8);
        Lookup L{d_calls, (uint32_t)calls.size(), d_hb, P, PL, G};

        // ---------------------------------------------------------- 1-2 image map
        const uint64_t n_bits = (uint64_t)n_a * G;
        const uint64_t n_words = n_bits / 32 + 1;    // one spare word: rank of the end bit
        uint32_t* bits = static_cast<uint32_t*>(tmp(n_words * 4));
        HIPCHK(hipMemsetAsync(bits, 0, n_words * 4, c.stream));
        // only the connections of calls with a source segment off P_local can need an image
        std::vector<std::pair<uint64_t, uint64_t>> mark_ranges;
        for (auto& cl : c.calls) {
            bool remote = false;
            for (auto& g : cl.S.seg) remote |= (g.host != PL);
            if (!remote || !cl.gen_count) continue;
            if (!mark_ranges.empty() && mark_ranges.back().second == cl.gen_begin)
                mark_ranges.back().second += cl.gen_count;
            else
                mark_ranges.push_back({cl.gen_begin, cl.gen_begin + cl.gen_count});
        }
        for (auto& r : mark_ranges) {
            tstart(c, "prep_mark");
            hipLaunchKernelGGL(k_mark, dim3(grid_for(r.second - r.first, 8192)), dim3(PNT), 0, c.stream, L, c.g_src, r.first,
                               r.second, bits);
            tstop(c);
            HIPCHK(hipGetLastError());
        }
        uint64_t* word_rank = static_cast<uint64_t*>(tmp((n_words + 1) * 8));
        const uint64_t n_img = scan_popc_u64(c, bits, word_rank, n_words, true);
        c.n_img = n_img;
        if ((uint64_t)M_local + n_img > 0x7fffffffull) raise(SNNC_EUNSUPPORTED, "more than 2^31-1 local and image neurons");
        int32_t* R = result<int32_t>(c, SNNC_R_VAL, n_img);
        if (n_img) {
            tstart(c, "prep_rvals");
            hipLaunchKernelGGL(k_rvals, dim3(grid_for(n_words)), dim3(PNT), 0, c.stream, bits, word_rank, n_words,
                               d_hb, P, G, R);
            tstop(c);
            HIPCHK(hipGetLastError());
        }
        uint64_t* r_off = result<uint64_t>(c, SNNC_R_OFF, (uint64_t)n_a * P + 1);
        int64_t* img_base = result<int64_t>(c, SNNC_IMG_BASE, (uint64_t)n_a * P);
        {
            const uint64_t nk = (uint64_t)n_a * P + 1;
            tstart(c, "prep_bounds");
            hipLaunchKernelGGL(k_bounds, dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, c.stream, bits, word_rank,
                               d_hb, P, n_a, G, M_local, r_off, img_base);
            tstop(c);
            HIPCHK(hipGetLastError());
        }

        // ---------------------------------------------------------- 3-4 keys and sort
        const uint64_t n_rows = (uint64_t)M_local + n_img;
        const uint32_t sbits = bits_for(n_rows), tbits = bits_for(M_local);
        c.key_bits = sbits + tbits;
        if (sbits + tbits > 48) raise(SNNC_EUNSUPPORTED, "source and target ids need more than 48 key bits");
        uint32_t passes, dbits;
        radix_plan(sbits + tbits, passes, dbits);
        int32_t* o_src = nullptr;
        if (N) {
            uint64_t* keys0 = static_cast<uint64_t*>(tmp(N * 8));
            uint64_t* hist = static_cast<uint64_t*>(tmp(8 * 256 * 8));
            HIPCHK(hipMemsetAsync(hist, 0, 8 * 256 * 8, c.stream));
            tstart(c, "prep_keys");
            hipLaunchKernelGGL(k_keys, dim3(grid_for(N, 8192)), dim3(PNT), 0, c.stream, L, c.g_src, c.g_tgt, c.g_delay,
                               N, bits, word_rank, M_local, 16 + tbits, dbits, passes, keys0, hist);
            tstop(c);
            HIPCHK(hipGetLastError());
            // the source ordinals, targets and delays now live in the keys (released in stream order)
            dfree(c, c.g_src); c.g_src = nullptr;
            dfree(c, c.g_tgt); c.g_tgt = nullptr;
            dfree(c, c.g_delay); c.g_delay = nullptr;
            uint64_t* keys1 = static_cast<uint64_t*>(tmp(N * 8));
            uint32_t* vals1 = static_cast<uint32_t*>(tmp(N * 4));
            // outputs allocated only now, so they reuse the memory just released
            o_src = result<int32_t>(c, SNNC_SRC, N);
            int32_t* o_tgt = result<int32_t>(c, SNNC_TGT, N);
            uint16_t* o_delay = result<uint16_t>(c, SNNC_DELAY, N);
            float* o_weight = result<float>(c, SNNC_WEIGHT, N);
            FinalOut fo{o_src, o_tgt, o_delay, o_weight, 16 + tbits, (1ull << tbits) - 1};
            if (tbits == 0) fo.tgt_mask = 0;
            radix_sort(c, keys0, reinterpret_cast<uint32_t*>(c.g_weight), keys1, vals1, N, 16, 16 + sbits + tbits,
                       hist, &fo);
        } else {
            o_src = result<int32_t>(c, SNNC_SRC, 0);
            result<int32_t>(c, SNNC_TGT, 0);
            result<uint16_t>(c, SNNC_DELAY, 0);
            result<float>(c, SNNC_WEIGHT, 0);
        }
        dfree(c, c.g_src); c.g_src = nullptr;
        dfree(c, c.g_tgt); c.g_tgt = nullptr;
        dfree(c, c.g_delay); c.g_delay = nullptr;
        dfree(c, c.g_weight); c.g_weight = nullptr;
        c.cap_gen = 0;

        // ---------------------------------------------------------- 5 first-index array
        uint64_t* row_ptr = result<uint64_t>(c, SNNC_ROW_PTR, n_rows + 1);
        tstart(c, "prep_csr");
        hipLaunchKernelGGL(k_csr, dim3(grid_for(N / 4 + 1, 16384)), dim3(PNT), 0, c.stream, o_src, N, n_rows, row_ptr);
        tstop(c);
        HIPCHK(hipGetLastError());

        // ---------------------------------------------------------- 6 point-to-point lists
        const uint32_t wpr = (M_local + 31) / 32 + 1;     // words per row (+1 spare)
        const uint64_t n_rw = (uint64_t)P * wpr;
        uint32_t* rows = static_cast<uint32_t*>(tmp(n_rw * 4));
        HIPCHK(hipMemsetAsync(rows, 0, n_rw * 4, c.stream));
        for (auto& cl : c.calls) {
            if (cl.alpha != -1) continue;
            bool has_local_source = false;
            for (auto& g : cl.S.seg) has_local_source |= (g.host == PL);
            if (!has_local_source) continue;
            std::vector<bool> tgt_host(P, false);
            for (auto& g : cl.T.seg) tgt_host[g.host] = true;
            for (uint32_t tau = 0; tau < P; ++tau)
                if (tau != PL && tgt_host[tau]) gen_mark(c, cl, tau, rows + (uint64_t)tau * wpr);
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
                               h_total, bits, word_rank, d_hb, G, PL, M_local, Hv, Iv);
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
    } catch (...) {
        cleanup();
        throw;
    }
    cleanup();
}

}  // namespace snnc
