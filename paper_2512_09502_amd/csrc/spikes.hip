// Spike exchange through the built maps (the paper's Appendix E example and
// the collective subsection): per-destination packets of one time step on
// the source host, and on the target host the lookup of received map
// positions (L for point-to-point, I for collective groups) into the image's
// row of the source-sorted connections, expanded into (target, delay,
// weight x multiplicity) events.
//
// Packets: each spike contributes one record per (destination, position)
// pair of its source; records carry (destination << 32 | spike index) as
// key, so a stable radix sort on the destination bits groups them by packet
// and keeps the spike order inside a packet.
#include <algorithm>

#include "device_common.h"
#include "internal.h"

namespace snnc {
namespace {

constexpr int SNT = 256;

unsigned sgrid(uint64_t n) { return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n + SNT - 1) / SNT, 1u << 20)); }

// The exchange's error word: a mapped pinned word that the kernels set with a
// plain store (any lane, same value) and the host reads after the stream's
// wait; cleared by the host before the launches (the previous call waited).
static uint32_t* err_word(Ctx& c) {
    *reinterpret_cast<volatile uint32_t*>(c.tot_pin + 2) = 0u;
    return reinterpret_cast<uint32_t*>(c.tot_pin_dev + 2);
}

// status word of the packet sort's look-back waits (mapped pinned memory,
// cleared here while no kernel of the context runs)
static uint32_t* sort_status_word(Ctx& c) {
    *reinterpret_cast<volatile uint32_t*>(c.tot_pin + 3) = 0u;
    return reinterpret_cast<uint32_t*>(c.tot_pin_dev + 3);
}

// after the stream's final wait: whether a look-back wait gave up
bool sort_status_failed(Ctx& c) { return *reinterpret_cast<volatile uint32_t*>(c.tot_pin + 3) != 0u; }

// records per spike; spike ids beyond M set the error word
__global__ __launch_bounds__(SNT) void k_spike_deg(const uint32_t* spikes, uint64_t n, uint32_t M, const uint64_t* ptr,
                                                   uint32_t* deg, uint32_t* err) {
    for (uint64_t k = (uint64_t)blockIdx.x * SNT + threadIdx.x; k < n; k += (uint64_t)gridDim.x * SNT) {
        const uint32_t s = spikes[k];
        uint32_t d = 0;
        if (s >= M) *err = 1u;   // any lane may set it
        else d = (uint32_t)(ptr[s + 1] - ptr[s]);
        deg[k] = d;
    }
}

// destination rank of a list entry: the host itself (point-to-point) or the
// group's rank among the sorted group ids (collective)
__device__ __forceinline__ uint32_t dest_rank(uint32_t v, const int32_t* groups, uint32_t n_groups) {
    if (!groups) return v;
    uint32_t a = 0, b = n_groups;   // lower_bound
    while (a < b) {
        const uint32_t m = (a + b) >> 1;
        if (groups[m] < (int32_t)v) a = m + 1; else b = m;
    }
    return a;
}

__global__ __launch_bounds__(SNT) void k_spike_records(const uint32_t* spikes, uint64_t n, const uint64_t* ptr,
                                                       const uint32_t* dest, const uint32_t* where,
                                                       const int32_t* groups, uint32_t n_groups,
                                                       const uint64_t* rec_off, uint64_t* keys, uint32_t* vals) {
    for (uint64_t k = (uint64_t)blockIdx.x * SNT + threadIdx.x; k < n; k += (uint64_t)gridDim.x * SNT) {
        const uint32_t s = spikes[k];
        uint64_t r = rec_off[k];
        for (uint64_t j = ptr[s]; j < ptr[s + 1]; ++j, ++r) {
            keys[r] = ((uint64_t)dest_rank(dest[j], groups, n_groups) << 32) | k;
            vals[r] = where[j];
        }
    }
}

__global__ __launch_bounds__(SNT) void k_packets_out(const uint64_t* keys, const uint32_t* vals, uint64_t total,
                                                     const uint32_t* mult, uint32_t* pos_out, uint32_t* mult_out) {
    for (uint64_t o = (uint64_t)blockIdx.x * SNT + threadIdx.x; o < total; o += (uint64_t)gridDim.x * SNT) {
        pos_out[o] = vals[o];
        mult_out[o] = mult ? mult[(uint32_t)keys[o]] : 1u;
    }
}

// off[d] = first record of destination d (records sorted by destination)
__global__ __launch_bounds__(SNT) void k_packet_bounds(const uint64_t* keys, uint64_t total, uint32_t n_dest,
                                                       uint64_t* off) {
    const uint32_t d = blockIdx.x * SNT + threadIdx.x;
    if (d > n_dest) return;
    const uint64_t x = (uint64_t)d << 32;
    uint64_t a = 0, b = total;
    while (a < b) {
        const uint64_t m = (a + b) >> 1;
        if (keys[m] < x) a = m + 1; else b = m;
    }
    off[d] = a;
}

// delivery: image and row of every received entry
__global__ __launch_bounds__(SNT) void k_deliver_lookup(const uint32_t* grp, const uint32_t* host, const uint32_t* pos,
                                                        uint64_t n, uint32_t P, uint32_t PL, uint32_t n_maps_grp,
                                                        int kind, const uint64_t* map_off, const int32_t* map_img,
                                                        const uint64_t* row_ptr, const uint64_t* img_first,
                                                        const uint32_t* img_count, uint32_t M_local, int32_t* image,
                                                        uint64_t* rb, uint64_t* re, uint64_t* cnt, uint32_t* err) {
    for (uint64_t e = (uint64_t)blockIdx.x * SNT + threadIdx.x; e < n; e += (uint64_t)gridDim.x * SNT) {
        const uint32_t h = host[e];
        bool ok = h < P && (kind == 1 || h != PL);
        uint64_t key = h;
        if (kind == 1) {
            const uint32_t g = grp[e];
            ok = ok && g < n_maps_grp;
            key = (uint64_t)g * P + h;
        }
        int32_t img = -1;
        if (ok) {
            const uint64_t a = map_off[key], b = map_off[key + 1];
            if ((uint64_t)pos[e] < b - a) img = map_img[a + pos[e]];
            else ok = false;
        }
        if (!ok) *err = 1u;   // any lane may set it
        uint64_t lo = 0, hi = 0;
        if (img >= 0 && img_first) {     // image rows kept apart (GPU memory levels 0 and 1)
            lo = img_first[(uint32_t)img - M_local];
            hi = lo + img_count[(uint32_t)img - M_local];
        } else if (img >= 0) {
            lo = row_ptr[img];
            hi = row_ptr[img + 1];
        }
        image[e] = img;
        rb[e] = lo;
        re[e] = hi;
        cnt[e] = hi - lo;
    }
}

// events: one thread per event, its entry found by binary search over the offsets
__global__ __launch_bounds__(SNT) void k_deliver_events(const uint64_t* ev_off, uint64_t n, uint64_t total,
                                                        const uint64_t* rb, const uint32_t* mult, const int32_t* tgt,
                                                        const uint16_t* delay, const float* weight, int32_t* ev_tgt,
                                                        uint16_t* ev_delay, float* ev_weight) {
    for (uint64_t o = (uint64_t)blockIdx.x * SNT + threadIdx.x; o < total; o += (uint64_t)gridDim.x * SNT) {
        uint64_t a = 0, b = n;   // last entry with ev_off <= o
        while (b - a > 1) {
            const uint64_t m = (a + b) >> 1;
            if (ev_off[m] <= o) a = m; else b = m;
        }
        const uint64_t c = rb[a] + (o - ev_off[a]);
        const float m = mult ? (float)mult[a] : 1.0f;
        ev_tgt[o] = tgt[c];
        ev_delay[o] = delay[c];
        ev_weight[o] = weight[c] * m;
    }
}

// address of a result array for kernels (host-resident arrays through their mapping)
template <class T>
const T* arr(Ctx& c, int32_t id) {
    auto it = c.arrays.find(id);
    if (it == c.arrays.end()) raise(SNNC_ESTATE, "array not available");
    return static_cast<const T*>(it->second.host ? it->second.dev : it->second.p);
}

template <class T>
const T* arr_or_null(Ctx& c, int32_t id) {
    return c.arrays.count(id) ? arr<T>(c, id) : nullptr;
}

uint32_t bits_for_values(uint64_t n_values) {
    uint32_t b = 0;
    while (b < 64 && (n_values > 0 ? (n_values - 1) >> b : 0)) ++b;
    return b;
}

}  // namespace

uint64_t spike_packets(Ctx& c, int kind, const uint32_t* spikes, const uint32_t* mult, uint64_t n, uint64_t* off,
                       uint32_t* pos_out, uint32_t* mult_out, uint64_t cap) {
    if (!c.prepared) raise(SNNC_ESTATE, "spike packets need a prepared network");
    if (kind != 0 && kind != 1) raise(SNNC_EINVAL, "kind must be 0 (point-to-point) or 1 (collective)");
    if (n >= (1ull << 32)) raise(SNNC_EINVAL, "more than 2^32 - 1 spikes");
    const uint32_t M = c.M[c.P_local];
    const uint64_t* ptr = arr<uint64_t>(c, kind == 0 ? SNNC_TP_PTR : SNNC_GQ_PTR);
    const uint32_t* dest = kind == 0 ? arr<uint32_t>(c, SNNC_T_VAL) : reinterpret_cast<const uint32_t*>(arr<int32_t>(c, SNNC_G_VAL));
    const uint32_t* where = arr<uint32_t>(c, kind == 0 ? SNNC_P_VAL : SNNC_Q_VAL);
    const int32_t* groups = kind == 1 ? arr<int32_t>(c, SNNC_GROUPS) : nullptr;
    const uint32_t n_groups = (uint32_t)c.counts[SNNC_GROUPS];
    const uint32_t n_dest = kind == 0 ? c.P : n_groups;
    std::vector<void*> temps;
    auto tmp = [&](size_t bytes) {
        void* p = dalloc(c, bytes);
        temps.push_back(p);
        return p;
    };
    uint64_t total = 0;
    try {
        // the error word lives in mapped pinned memory: read after the scan's wait, no copy
        uint32_t* err = err_word(c);
        uint32_t* deg = static_cast<uint32_t*>(tmp(std::max<uint64_t>(n, 1) * 4));
        uint64_t* rec_off = static_cast<uint64_t*>(tmp((n + 1) * 8));
        if (n) {
            hipLaunchKernelGGL(k_spike_deg, dim3(sgrid(n)), dim3(SNT), 0, c.stream, spikes, n, M, ptr, deg, err);
            HIPCHK(hipGetLastError());
        }
        total = n ? scan_u32_u64(c, deg, rec_off, n, true) : 0;   // waits for the stream
        if (*reinterpret_cast<volatile uint32_t*>(c.tot_pin + 2)) raise(SNNC_EINVAL, "spike id is not a local neuron");
        if (total > cap) {
            for (void* p : temps) dfree(c, p);
            temps.clear();
            return total;   // caller reports the small capacity
        }
        if (total) {
            uint64_t* k0 = static_cast<uint64_t*>(tmp(total * 8));
            uint64_t* k1 = static_cast<uint64_t*>(tmp(total * 8));
            uint32_t* v0 = static_cast<uint32_t*>(tmp(total * 4));
            uint32_t* v1 = static_cast<uint32_t*>(tmp(total * 4));
            tstart(c, "spike_records");
            hipLaunchKernelGGL(k_spike_records, dim3(sgrid(n)), dim3(SNT), 0, c.stream, spikes, n, ptr, dest, where,
                               groups, n_groups, rec_off, k0, v0);
            tstop(c);
            HIPCHK(hipGetLastError());
            // a look-back wait that gives up flags the sort's status word: here the
            // fourth mapped pinned word, read after the final wait below
            uint32_t* const saved_status = c.d_status;
            c.d_status = sort_status_word(c);
            int w = 0;
            try {
                w = radix_sort(c, k0, v0, k1, v1, total, 32, 32 + bits_for_values(n_dest), nullptr, nullptr,
                               false);   // every pass runs: no wait for the digit histograms
            } catch (...) {
                c.d_status = saved_status;
                throw;
            }
            c.d_status = saved_status;
            const uint64_t* ks = w ? k1 : k0;
            const uint32_t* vs = w ? v1 : v0;
            tstart(c, "spike_packets");
            hipLaunchKernelGGL(k_packets_out, dim3(sgrid(total)), dim3(SNT), 0, c.stream, ks, vs, total, mult, pos_out,
                               mult_out);
            hipLaunchKernelGGL(k_packet_bounds, dim3((n_dest + 1 + SNT - 1) / SNT), dim3(SNT), 0, c.stream, ks, total,
                               n_dest, off);
            tstop(c);
            HIPCHK(hipGetLastError());
        } else {
            HIPCHK(hipMemsetAsync(off, 0, ((uint64_t)n_dest + 1) * 8, c.stream));
        }
        sync(c);
        if (sort_status_failed(c)) raise(SNNC_EDEVICE, "a look-back wait of the packet sort exceeded its bound");
    } catch (...) {
        for (void* p : temps) dfree(c, p);
        throw;
    }
    for (void* p : temps) dfree(c, p);
    return total;
}

uint64_t deliver(Ctx& c, int kind, const uint32_t* grp, const uint32_t* host, const uint32_t* pos,
                 const uint32_t* mult, uint64_t n, int32_t* image, uint64_t* rb, uint64_t* re, int32_t* ev_tgt,
                 uint16_t* ev_delay, float* ev_weight, uint64_t ev_cap, bool* too_small) {
    if (!c.prepared) raise(SNNC_ESTATE, "delivery needs a prepared network");
    if (kind != 0 && kind != 1) raise(SNNC_EINVAL, "kind must be 0 (point-to-point) or 1 (collective)");
    if (kind == 1 && !grp) raise(SNNC_EINVAL, "collective delivery needs the group ranks");
    *too_small = false;
    const uint64_t* map_off = arr<uint64_t>(c, kind == 0 ? SNNC_R_OFF : SNNC_H_OFF);
    const int32_t* map_img = arr<int32_t>(c, kind == 0 ? SNNC_L_VAL : SNNC_I_VAL);
    const uint64_t* row_ptr = arr<uint64_t>(c, SNNC_ROW_PTR);
    std::vector<void*> temps;
    auto tmp = [&](size_t bytes) {
        void* p = dalloc(c, bytes);
        temps.push_back(p);
        return p;
    };
    uint64_t total = 0;
    try {
        uint32_t* err = err_word(c);   // mapped pinned memory, read after the scan's wait
        uint64_t* cnt = static_cast<uint64_t*>(tmp(std::max<uint64_t>(n, 1) * 8));
        uint64_t* ev_off = static_cast<uint64_t*>(tmp((n + 1) * 8));
        if (n) {
            tstart(c, "deliver_lookup");
            hipLaunchKernelGGL(k_deliver_lookup, dim3(sgrid(n)), dim3(SNT), 0, c.stream, grp, host, pos, n, c.P,
                               c.P_local, (uint32_t)c.counts[SNNC_GROUPS], kind, map_off, map_img, row_ptr,
                               arr_or_null<uint64_t>(c, SNNC_IMG_FIRST), arr_or_null<uint32_t>(c, SNNC_IMG_COUNT),
                               c.M[c.P_local], image, rb, re, cnt, err);
            tstop(c);
            HIPCHK(hipGetLastError());
        }
        total = n ? scan_u64_u64(c, cnt, ev_off, n, true) : 0;   // waits for the stream
        if (*reinterpret_cast<volatile uint32_t*>(c.tot_pin + 2)) raise(SNNC_EINVAL, "received entry outside its map");
        if (ev_tgt && total > ev_cap) {
            *too_small = true;
        } else if (ev_tgt && total) {
            tstart(c, "deliver_events");
            hipLaunchKernelGGL(k_deliver_events, dim3(sgrid(total)), dim3(SNT), 0, c.stream, ev_off, n, total, rb, mult,
                               arr<int32_t>(c, SNNC_TGT), arr<uint16_t>(c, SNNC_DELAY), arr<float>(c, SNNC_WEIGHT),
                               ev_tgt, ev_delay, ev_weight);
            tstop(c);
            HIPCHK(hipGetLastError());
        }
        sync(c);
    } catch (...) {
        for (void* p : temps) dfree(c, p);
        throw;
    }
    for (void* p : temps) dfree(c, p);
    return total;
}

}  // namespace snnc

extern "C" snnc_status snnc_spike_packets(snnc_ctx* ctx, int32_t kind, const uint32_t* spikes, const uint32_t* mult,
                                          uint64_t n, uint64_t* off, uint32_t* pos_out, uint32_t* mult_out,
                                          uint64_t cap, uint64_t* n_out) {
    using namespace snnc;
    if (!ctx || !n_out || (n && !spikes) || !off) return SNNC_EINVAL;
    try {
        HIPCHK(hipSetDevice(ctx->device));
        const uint64_t total = spike_packets(*ctx, kind, spikes, mult, n, off, pos_out, mult_out, cap);
        *n_out = total;
        if (total > cap) {
            ctx->last_error = "packet capacity " + std::to_string(cap) + " below " + std::to_string(total) + " entries";
            return SNNC_EINVAL;
        }
        return SNNC_OK;
    } catch (const Error& e) {
        ctx->last_error = e.msg;
        return e.code;
    }
}

extern "C" snnc_status snnc_deliver(snnc_ctx* ctx, int32_t kind, const uint32_t* grp, const uint32_t* host,
                                    const uint32_t* pos, const uint32_t* mult, uint64_t n, int32_t* image,
                                    uint64_t* row_begin, uint64_t* row_end, int32_t* ev_tgt, uint16_t* ev_delay,
                                    float* ev_weight, uint64_t ev_cap, uint64_t* n_events) {
    using namespace snnc;
    if (!ctx || !n_events || (n && (!host || !pos || !image || !row_begin || !row_end))) return SNNC_EINVAL;
    if (ev_tgt && (!ev_delay || !ev_weight)) return SNNC_EINVAL;
    try {
        HIPCHK(hipSetDevice(ctx->device));
        bool small = false;
        const uint64_t total = deliver(*ctx, kind, grp, host, pos, mult, n, image, row_begin, row_end, ev_tgt,
                                       ev_delay, ev_weight, ev_cap, &small);
        *n_events = total;
        if (small) {
            ctx->last_error = "event capacity " + std::to_string(ev_cap) + " below " + std::to_string(total);
            return SNNC_EINVAL;
        }
        return SNNC_OK;
    } catch (const Error& e) {
        ctx->last_error = e.msg;
        return e.code;
    }
}
