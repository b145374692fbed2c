// C ABI and host planner: context state, allocation against the budget,
// validation of Connect specs, kernel timing, array access.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <stdexcept>

#include "device_common.h"
#include "internal.h"

namespace snnc {

[[noreturn]] void raise(snnc_status code, const std::string& msg) { throw Error{code, msg}; }

void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) raise(SNNC_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

constexpr size_t SMALL_MAX = 1u << 20;   // blocks up to this size come from the slabs
constexpr size_t SLAB_BYTES = 8u << 20;

// Stream-ordered allocations come from one memory pool per device owned by
// the library, which keeps freed memory (no release threshold): a served
// stream makes a context per build, and memory returned to the driver at
// every context's end would be mapped again by the next.
static hipMemPool_t lib_pool(int device) {
    static std::mutex m;
    static hipMemPool_t pools[64] = {};
    if (device < 0 || device >= 64) return nullptr;
    std::lock_guard<std::mutex> lock(m);
    if (!pools[device]) {
        hipMemPoolProps props{};
        props.allocType = hipMemAllocationTypePinned;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = device;
        hipMemPool_t p = nullptr;
        if (hipMemPoolCreate(&p, &props) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        uint64_t keep = UINT64_MAX;
        (void)hipMemPoolSetAttribute(p, hipMemPoolAttrReleaseThreshold, &keep);
        pools[device] = p;
    }
    return pools[device];
}

// Blocks of stream-ordered memory that a destroyed context held (after its
// final wait) wait here for the next context on the device: freeing them
// back to the pool costs milliseconds per block.  At most 8 GiB per device.
namespace {
constexpr size_t BLOCK_CACHE_MAX = 8ull << 30;

struct BlockCache {
    std::mutex m;
    std::map<size_t, std::vector<void*>> free;
    size_t bytes = 0;
};

BlockCache& block_cache(int device) {
    static BlockCache caches[64];
    return caches[device < 0 || device >= 64 ? 0 : device];
}
}  // namespace

// Memory from the outer allocator.  `live` keeps the size with the lane in
// bit 0: lane 0 uses the caller's allocator (else stream-ordered allocation
// on the caller's stream), lane 1 stream-ordered allocation on the counting
// stream.
static void* raw_alloc(Ctx& c, size_t bytes, int lane) {
    bytes = (bytes + 255) & ~(size_t)255;
    if (c.budget && c.bytes_live + bytes > c.budget)
        raise(SNNC_EBUDGET, "device-memory budget exceeded (" + std::to_string(c.bytes_live + bytes) + " > " +
                                std::to_string(c.budget) + " bytes)");
    void* p = nullptr;
    if (lane == 0 && c.has_alloc) {
        p = c.alloc.alloc(bytes, (void*)c.main_stream, c.alloc.user);
        if (!p) raise(SNNC_ENOMEM, "allocator returned NULL for " + std::to_string(bytes) + " bytes");
    } else {
        // stream-ordered: a buffer freed after enqueued work is reused only by later work
        hipStream_t strm = lane == 0 ? c.main_stream : c.count_stream;
        {
            BlockCache& bc = block_cache(c.device);
            std::lock_guard<std::mutex> lock(bc.m);
            auto it = bc.free.find(bytes);
            if (it != bc.free.end() && !it->second.empty()) {
                p = it->second.back();
                it->second.pop_back();
                bc.bytes -= bytes;
            }
        }
        hipMemPool_t pool = p ? nullptr : lib_pool(c.device);
        hipError_t e = p ? hipSuccess
                         : pool ? hipMallocFromPoolAsync(&p, bytes, pool, strm) : hipMallocAsync(&p, bytes, strm);
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            raise(SNNC_ENOMEM, "hipMallocAsync failed for " + std::to_string(bytes) + " bytes");
        }
    }
    c.live[p] = bytes | (size_t)lane;
    c.bytes_live += bytes;
    c.bytes_peak = std::max(c.bytes_peak, c.bytes_live);
    return p;
}

// to_cache: the context is being destroyed and its streams have drained, so a
// stream-ordered block may go to the device's block cache instead.
static void raw_free(Ctx& c, void* p, bool to_cache = false) {
    auto it = c.live.find(p);
    if (it == c.live.end()) return;
    const size_t bytes = it->second & ~(size_t)255;
    const int lane = (int)(it->second & 1);
    c.bytes_live -= bytes;
    c.live.erase(it);
    if (lane == 0 && c.has_alloc) {
        c.alloc.free(p, c.alloc.user);
        return;
    }
    if (to_cache) {
        BlockCache& bc = block_cache(c.device);
        std::lock_guard<std::mutex> lock(bc.m);
        if (bc.bytes + bytes <= BLOCK_CACHE_MAX) {
            bc.free[bytes].push_back(p);
            bc.bytes += bytes;
            return;
        }
    }
    (void)hipFreeAsync(p, lane == 0 ? c.main_stream : c.count_stream);
}

// Blocks up to SMALL_MAX come from a free list per power-of-two class,
// refilled from 8 MB slabs; larger blocks of the caller's lane go to the outer
// allocator.  A block freed after the work that uses it was enqueued is
// reused only by later work of the same stream.  The counting lane keeps every
// block it allocates (large ones too) in its own class lists; its blocks freed
// while the caller's stream may still use them wait for a fence (see
// CountScope).
void* dalloc(Ctx& c, size_t bytes) {
    if (bytes == 0) bytes = 1;
    if (c.lane == 0 && bytes > SMALL_MAX) return raw_alloc(c, bytes, 0);
    size_t cls = 256;
    while (cls < bytes) cls <<= 1;
    auto& fl = c.small_free[cls];
    void* p = nullptr;
    if (!fl.empty()) {
        p = fl.back();
        fl.pop_back();
    } else if (cls > SMALL_MAX) {
        p = raw_alloc(c, cls, c.lane);
    } else {
        if (c.slab_left < cls) {
            c.slab_cur = static_cast<char*>(raw_alloc(c, SLAB_BYTES, c.lane));
            c.slabs.push_back(c.slab_cur);
            c.slab_left = SLAB_BYTES;
        }
        p = c.slab_cur;
        c.slab_cur += cls;
        c.slab_left -= cls;
    }
    c.small_live[p] = cls | (size_t)c.lane;
    return p;
}

void dfree(Ctx& c, void* p) {
    if (!p) return;
    auto sm = c.small_live.find(p);
    if (sm != c.small_live.end()) {
        const size_t cls = sm->second & ~(size_t)1;
        const int lane = (int)(sm->second & 1);
        c.small_live.erase(sm);
        if (lane == c.lane) c.small_free[cls].push_back(p);
        else if (lane == 1) c.deferred.push_back(Ctx::Deferred{c.fence_seq, p, cls});
        else c.parked.small_free[cls].push_back(p);     // the caller's stream orders its later use
        return;
    }
    raw_free(c, p);
}

static void swap_lane(Ctx& c) {
    LaneState& o = c.parked;
    std::swap(c.stream, o.stream);
    std::swap(c.ring, o.ring);
    std::swap(c.lookback, o.lookback);
    std::swap(c.lookback_bytes, o.lookback_bytes);
    std::swap(c.sort_epoch, o.sort_epoch);
    std::swap(c.slab_cur, o.slab_cur);
    std::swap(c.slab_left, o.slab_left);
    std::swap(c.small_free, o.small_free);
    c.lane ^= 1;
}

CountScope::CountScope(Ctx& ctx) : c(ctx) {
    if (c.lane != 0) raise(SNNC_ESTATE, "nested counting section");
    if (!c.count_stream) {
        HIPCHK(hipStreamCreateWithFlags(&c.count_stream, hipStreamNonBlocking));
        c.parked.stream = c.count_stream;
        HIPCHK(hipEventCreateWithFlags(&c.count_done, hipEventDisableTiming));
        init_ring(c.parked.ring, 4u << 20);
    }
    // fence the blocks freed since the last fence, then take back those whose
    // fence the caller's stream has passed
    if (!c.deferred.empty() && c.deferred.back().seq == c.fence_seq) {
        hipEvent_t e = nullptr;
        if (!c.fence_pool.empty()) {
            e = c.fence_pool.back();
            c.fence_pool.pop_back();
        } else {
            HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        }
        HIPCHK(hipEventRecord(e, c.main_stream));
        c.fences.emplace_back(c.fence_seq, e);
        ++c.fence_seq;
    }
    bool any = false;
    uint64_t done = 0;
    while (!c.fences.empty()) {
        const hipError_t q = hipEventQuery(c.fences.front().second);
        if (q == hipErrorNotReady) break;
        HIPCHK(q);
        done = c.fences.front().first;
        any = true;
        c.fence_pool.push_back(c.fences.front().second);
        c.fences.pop_front();
    }
    while (any && !c.deferred.empty() && c.deferred.front().seq <= done) {
        c.parked.small_free[c.deferred.front().cls].push_back(c.deferred.front().p);
        c.deferred.pop_front();
    }
    swap_lane(c);
}

CountScope::~CountScope() {
    (void)hipEventRecord(c.count_done, c.stream);
    swap_lane(c);
    (void)hipStreamWaitEvent(c.stream, c.count_done, 0);
}

static hipEvent_t get_event(Ctx& c) {
    if (!c.event_pool.empty()) {
        hipEvent_t e = c.event_pool.back();
        c.event_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    return e;
}

void tstart(Ctx& c, const char* name) {
    if (!c.timing) return;
    if (c.timing == 2 && strncmp(name, "sort_pass", 9) != 0) {
        c.open_timers.push_back(SIZE_MAX);   // bracket not timed
        return;
    }
    Ctx::Pending p;
    p.name = name;
    p.a = get_event(c);
    p.b = get_event(c);
    HIPCHK(hipEventRecord(p.a, c.stream));
    c.open_timers.push_back(c.pending.size());
    c.pending.push_back(p);
}

// closes the innermost open bracket (brackets nest: a scan inside a sort pass)
void tstop(Ctx& c) {
    if (!c.timing || c.open_timers.empty()) return;
    const size_t k = c.open_timers.back();
    c.open_timers.pop_back();
    if (k == SIZE_MAX) return;
    HIPCHK(hipEventRecord(c.pending[k].b, c.stream));
}

void resolve_times(Ctx& c) {
    if (c.pending.empty()) return;
    for (size_t k : c.open_timers)   // left open by an error
        if (k != SIZE_MAX) HIPCHK(hipEventRecord(c.pending[k].b, c.stream));
    c.open_timers.clear();
    HIPCHK(hipStreamSynchronize(c.main_stream));
    if (c.count_stream) HIPCHK(hipStreamSynchronize(c.count_stream));
    for (auto& p : c.pending) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, p.a, p.b));
        auto& k = c.ktimes[p.name];
        k.launches += 1;
        k.ms += ms;
        c.event_pool.push_back(p.a);
        c.event_pool.push_back(p.b);
    }
    c.pending.clear();
}

// Pinned host buffers (staging rings, read-back and mapped words) outlive
// their context in a process-wide cache keyed by size and flags: pinning and
// unpinning pages costs milliseconds, and a served stream makes a context per
// build.  The cache keeps a few buffers per key.
namespace {
std::mutex& pinned_mutex() {
    static std::mutex m;
    return m;
}

std::map<std::pair<size_t, unsigned>, std::vector<void*>>& pinned_cache() {
    static std::map<std::pair<size_t, unsigned>, std::vector<void*>> m;
    return m;
}
}  // namespace

void* pinned_take(size_t bytes, unsigned flags) {
    {
        std::lock_guard<std::mutex> lock(pinned_mutex());
        auto& v = pinned_cache()[{bytes, flags}];
        if (!v.empty()) {
            void* p = v.back();
            v.pop_back();
            return p;
        }
    }
    void* p = nullptr;
    HIPCHK(hipHostMalloc(&p, bytes, flags));
    return p;
}

void pinned_give(void* p, size_t bytes, unsigned flags) {
    if (!p) return;
    {
        std::lock_guard<std::mutex> lock(pinned_mutex());
        auto& v = pinned_cache()[{bytes, flags}];
        if (v.size() < 4) {
            v.push_back(p);
            return;
        }
    }
    (void)hipHostFree(p);
}

void init_ring(StageRing& r, size_t bytes) {
    for (auto& e : r.ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    r.buf = static_cast<char*>(pinned_take(bytes, hipHostMallocDefault));
    r.bytes = bytes;
}

void free_ring(StageRing& r) {
    for (auto& e : r.ev)
        if (e) (void)hipEventDestroy(e);
    pinned_give(r.buf, r.bytes, hipHostMallocDefault);
    r = StageRing{};
}

// the writer moves into quarter nq: close the quarter it leaves, and wait
// for the copies out of nq's previous contents
static void enter_quarter(Ctx& c, StageRing& r, int nq) {
    if (nq == r.q) return;
    HIPCHK(hipEventRecord(r.ev[r.q], c.stream));
    r.pending[r.q] = true;
    if (r.pending[nq]) HIPCHK(hipEventSynchronize(r.ev[nq]));
    r.pending[nq] = false;
    r.q = nq;
}

void upload(Ctx& c, void* dst, const void* src, size_t bytes) {
    if (!bytes) return;
    StageRing& r = c.ring;
    const size_t quarter = r.bytes / 4;
    if (!r.buf || bytes > quarter) {
        HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c.stream));
        HIPCHK(hipStreamSynchronize(c.stream));
        return;
    }
    size_t at = (r.used + 255) & ~(size_t)255;
    if (at + bytes > r.bytes) at = 0;                      // wrap
    enter_quarter(c, r, (int)(at / quarter));
    enter_quarter(c, r, (int)((at + bytes - 1) / quarter));   // a copy spans at most two quarters
    memcpy(r.buf + at, src, bytes);
    HIPCHK(hipMemcpyAsync(dst, r.buf + at, bytes, hipMemcpyHostToDevice, c.stream));
    r.used = at + bytes;
}

void download(Ctx& c, void* dst, const void* src, size_t bytes) {
    if (!bytes) return;
    if (c.dl_pin && bytes <= c.dl_pin_bytes) {
        // small read-backs (counts, histograms) land in pinned memory: a direct DMA
        // instead of the runtime's staged copy into pageable memory
        HIPCHK(hipMemcpyAsync(c.dl_pin, src, bytes, hipMemcpyDeviceToHost, c.stream));
        HIPCHK(hipStreamSynchronize(c.stream));
        memcpy(dst, c.dl_pin, bytes);
        return;
    }
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, c.stream));
    HIPCHK(hipStreamSynchronize(c.stream));
}

void sync(Ctx& c) { HIPCHK(hipStreamSynchronize(c.stream)); }

// ------------------------------------------------------------------ node sets
bool set_lookup_host(const HostSet& s, uint64_t ord, uint32_t& host, uint32_t& local) {
    if (ord >= s.total) return false;
    size_t k = std::upper_bound(s.ord_begin.begin(), s.ord_begin.end(), ord) - s.ord_begin.begin() - 1;
    host = s.seg[k].host;
    local = s.seg[k].first + (uint32_t)(ord - s.ord_begin[k]);
    return true;
}

static HostSet make_set(const Ctx& c, const snnc_nodeset* ns) {
    HostSet s;
    if (!ns) raise(SNNC_EINVAL, "null node set");
    if (ns->n_seg && !ns->seg) raise(SNNC_EINVAL, "node set without segments array");
    std::vector<snnc_segment> order;
    for (uint32_t i = 0; i < ns->n_seg; ++i) {
        const snnc_segment g = ns->seg[i];
        if (g.host >= c.P) raise(SNNC_EINVAL, "segment host out of range");
        if ((uint64_t)g.first + g.n > c.M[g.host]) raise(SNNC_EINVAL, "segment outside the created neurons");
        if (g.n == 0) continue;     // empty segments hold no ordinals
        s.seg.push_back(g);
        s.ord_begin.push_back(s.total);
        s.total += g.n;
        order.push_back(g);
    }
    if (s.total > 0xffffffffull) raise(SNNC_EUNSUPPORTED, "node set larger than 2^32-1 neurons");
    std::sort(order.begin(), order.end(), [](const snnc_segment& a, const snnc_segment& b) {
        return a.host != b.host ? a.host < b.host : a.first < b.first;
    });
    for (size_t i = 1; i < order.size(); ++i)
        if (order[i].host == order[i - 1].host && order[i].first < (uint64_t)order[i - 1].first + order[i - 1].n)
            raise(SNNC_EINVAL, "segments of a node set overlap");
    return s;
}

// neurons present in both sets
static uint64_t set_overlap(const HostSet& a, const HostSet& b) {
    uint64_t total = 0;
    std::vector<snnc_segment> x = a.seg, y = b.seg;
    auto key = [](const snnc_segment& s) { return ((uint64_t)s.host << 32) | s.first; };
    std::sort(x.begin(), x.end(), [&](auto& p, auto& q) { return key(p) < key(q); });
    std::sort(y.begin(), y.end(), [&](auto& p, auto& q) { return key(p) < key(q); });
    size_t i = 0, j = 0;
    while (i < x.size() && j < y.size()) {
        const uint64_t xa = key(x[i]), xb = xa + x[i].n, ya = key(y[j]), yb = ya + y[j].n;
        const uint64_t lo = std::max(xa, ya), hi = std::min(xb, yb);
        if (hi > lo) total += hi - lo;
        if (xb < yb) ++i; else ++j;
    }
    return total;
}

// Standard normal CDF via the complementary error function.
static double phi(double x) { return 0.5 * std::erfc(-x / 1.41421356237309504880168872420969808); }

static bool build_delay_table(double mean, double sd, double lo, double dt, std::vector<uint32_t>& tab,
                              uint32_t& klo, uint64_t cap) {
    const double klo_d = std::round(lo / dt);
    if (!(klo_d >= 1.0) || klo_d > 65535.0) return false;
    klo = (uint32_t)klo_d;
    tab.clear();
    for (uint64_t k = klo;; ++k) {
        const double x = (((double)k + 0.5) * dt - mean) / sd;
        const double t = std::ceil(phi(x) * 4294967296.0);
        if (t >= 4294967296.0) break;
        if (k >= 65535 || tab.size() >= cap) return false;
        tab.push_back((uint32_t)t);
    }
    return true;
}

// The context's table of a normal delay distribution, built on first use
// (null when the distribution does not fit uint16 steps).
static std::shared_ptr<const DelayTable> delay_table_for(Ctx& c, const snnc_dist& d) {
    std::array<uint64_t, 3> key;
    memcpy(&key[0], &d.mean, 8);
    memcpy(&key[1], &d.sd, 8);
    memcpy(&key[2], &d.lo, 8);
    auto it = c.delay_tables.find(key);
    if (it != c.delay_tables.end()) return it->second;
    auto t = std::make_shared<DelayTable>();
    if (!build_delay_table(d.mean, d.sd, d.lo, c.dt, t->tab, t->klo, 65536)) return nullptr;
    if (!t->tab.empty()) {   // the thresholds do not decrease: one merge against the slice edges
        t->guide.resize(257);
        size_t i = 0;
        for (uint32_t j = 0; j <= 256; ++j) {
            const uint64_t edge = (uint64_t)j << 24;
            while (i < t->tab.size() && t->tab[i] < edge) ++i;
            t->guide[j] = (uint32_t)i;
        }
    }
    if (c.delay_tables.size() >= 4096) c.delay_tables.clear();   // bound the cache
    c.delay_tables.emplace(key, t);
    return t;
}

static void validate(Ctx& c, Call& cl, const snnc_syn_spec* syn) {
    const uint64_t ns = cl.S.total, nt = cl.T.total;
    const uint64_t ov = cl.autapses ? 0 : set_overlap(cl.S, cl.T);
    switch (cl.rule) {
    case SNNC_ONE_TO_ONE:
        if (ns != nt) raise(SNNC_EINVAL, "one-to-one needs equal set sizes");
        break;
    case SNNC_FIXED_INDEGREE:
    case SNNC_FIXED_OUTDEGREE: {
        const bool in = cl.rule == SNNC_FIXED_INDEGREE;
        const uint64_t units = in ? nt : ns, cand = in ? ns : nt;
        if (cl.n > 0 && units > 0) {
            const uint64_t n_eff = cand - (ov > 0 ? 1 : 0);
            if (cand == 0 || n_eff == 0) raise(SNNC_EINVAL, "no candidate to draw from");
            if (!cl.multapses && cl.n > n_eff) raise(SNNC_EINVAL, "degree exceeds the candidates without multapses");
            if (!cl.multapses && cl.n > 8192) raise(SNNC_EUNSUPPORTED, "degree above 8192 without multapses");
            if (cl.n > 0xffffffffull) raise(SNNC_EUNSUPPORTED, "degree above 2^32-1");
        }
        break;
    }
    case SNNC_FIXED_TOTAL_NUMBER: {
        if (cl.n > 0) {
            if (ns == 0 || nt == 0) raise(SNNC_EINVAL, "empty node set");
            const unsigned __int128 pairs = (unsigned __int128)ns * nt - ov;
            if (pairs == 0) raise(SNNC_EINVAL, "no valid pair");
            if (!cl.multapses && (unsigned __int128)cl.n > pairs) raise(SNNC_EINVAL, "total number exceeds the pairs without multapses");
            if (cl.n > 0xffffffffull) raise(SNNC_EUNSUPPORTED, "total number above 2^32-1");
        }
        break;
    }
    case SNNC_PAIRWISE_BERNOULLI:
        if (!(cl.p >= 0.0 && cl.p <= 1.0)) raise(SNNC_EINVAL, "probability outside [0, 1]");
        break;
    case SNNC_ASSIGNED_NODES: {
        if (cl.n && (!cl.in_src_pos || !cl.in_tgt_pos))
            raise(SNNC_EINVAL, "assigned nodes take their pairs through snnc_connect_assigned");
        uint32_t smax = 0, tmax = 0;
        for (uint64_t i = 0; i < cl.n; ++i) {
            smax = std::max(smax, cl.in_src_pos[i]);
            tmax = std::max(tmax, cl.in_tgt_pos[i]);
        }
        if (cl.n && (smax >= ns || tmax >= nt)) raise(SNNC_EINVAL, "assigned pair outside the node sets");
        // pairs per target host (the threshold map policy's estimate)
        bool one_host = true;
        for (auto& g : cl.T.seg) one_host = one_host && g.host == cl.T.seg[0].host;
        if (cl.n && one_host) {
            cl.pairs_on[cl.T.seg[0].host] = cl.n;
        } else {
            for (uint64_t i = 0; i < cl.n; ++i) {
                uint32_t h, l;
                set_lookup_host(cl.T, cl.in_tgt_pos[i], h, l);
                cl.pairs_on[h] += 1;
            }
        }
        break;
    }
    default:
        raise(SNNC_EINVAL, "unknown rule");
    }
    if (cl.alpha < -1) raise(SNNC_EINVAL, "group index below -1");
    if (!syn) raise(SNNC_EINVAL, "null synapse spec");
    if (syn->port != 0) raise(SNNC_EINVAL, "receptor port must be 0");
    cl.w = syn->weight;
    cl.d = syn->delay_ms;
    if (cl.w.kind == SNNC_CONST) cl.w_const = (float)cl.w.mean;
    else if (cl.w.kind == SNNC_NORMAL) {
        if (!(cl.w.sd >= 0.0)) raise(SNNC_EINVAL, "weight sd < 0");
    } else raise(SNNC_EINVAL, "unknown weight distribution");
    if (cl.d.kind == SNNC_CONST) {
        if (!(cl.d.mean >= c.dt)) raise(SNNC_EINVAL, "delay below one time step");
        const double steps = std::round(cl.d.mean / c.dt);
        if (steps > 65535.0) raise(SNNC_EINVAL, "delay beyond 65535 steps");
        cl.d_const = (uint16_t)steps;
    } else if (cl.d.kind == SNNC_NORMAL) {
        if (!(cl.d.sd > 0.0)) raise(SNNC_EINVAL, "delay sd must be > 0");
        if (!(cl.d.lo >= c.dt)) raise(SNNC_EINVAL, "delay clip below one time step");
        cl.dtab = delay_table_for(c, cl.d);
        if (!cl.dtab) raise(SNNC_EINVAL, "delay distribution does not fit uint16 steps");
        cl.d_klo = cl.dtab->klo;
    } else raise(SNNC_EINVAL, "unknown delay distribution");
}

// device copies of a call's sets and delay table (one allocation): layout
// S segments, T segments, delay thresholds, their 257-entry guide
static size_t meta_size(const Call& cl) {
    const size_t nS = std::max<size_t>(cl.S.seg.size(), 1), nT = std::max<size_t>(cl.T.seg.size(), 1);
    const bool tab = cl.dtab && !cl.dtab->tab.empty();
    const size_t nD = tab ? cl.dtab->tab.size() : 1;
    const size_t nG = tab ? 257 : 0;
    return (nS + nT) * sizeof(SegD) + (nD + nG) * sizeof(uint32_t);
}

static void fill_meta(const Call& cl, char* host) {
    const size_t nS = std::max<size_t>(cl.S.seg.size(), 1), nT = std::max<size_t>(cl.T.seg.size(), 1);
    memset(host, 0, meta_size(cl));
    SegD* hS = reinterpret_cast<SegD*>(host);
    SegD* hT = hS + nS;
    for (size_t i = 0; i < cl.S.seg.size(); ++i) hS[i] = SegD{cl.S.ord_begin[i], cl.S.seg[i].host, cl.S.seg[i].first};
    for (size_t i = 0; i < cl.T.seg.size(); ++i) hT[i] = SegD{cl.T.ord_begin[i], cl.T.seg[i].host, cl.T.seg[i].first};
    if (cl.dtab && !cl.dtab->tab.empty()) {
        uint32_t* hD = reinterpret_cast<uint32_t*>(hT + nT);
        const size_t nD = cl.dtab->tab.size();
        memcpy(hD, cl.dtab->tab.data(), nD * sizeof(uint32_t));
        memcpy(hD + nD, cl.dtab->guide.data(), 257 * sizeof(uint32_t));
    }
}

static void bind_meta(Call& cl, void* dev) {
    const size_t nS = std::max<size_t>(cl.S.seg.size(), 1), nT = std::max<size_t>(cl.T.seg.size(), 1);
    const bool tab = cl.dtab && !cl.dtab->tab.empty();
    const size_t nD = tab ? cl.dtab->tab.size() : 1;
    cl.meta = dev;
    cl.meta_bytes = meta_size(cl);
    cl.dS = static_cast<SegD*>(dev);
    cl.dT = cl.dS + nS;
    cl.dtab_dev = reinterpret_cast<uint32_t*>(cl.dT + nT);
    cl.dguide_dev = tab ? cl.dtab_dev + nD : nullptr;
}

void upload_meta(Ctx& c, Call& cl) {
    const size_t bytes = meta_size(cl);
    std::vector<char> host(bytes);
    fill_meta(cl, host.data());
    void* dev = dalloc(c, bytes);
    upload(c, dev, host.data(), bytes);
    bind_meta(cl, dev);
    if (cl.rule == SNNC_ASSIGNED_NODES && cl.n) {
        cl.pairs = dalloc_n<uint32_t>(c, 2 * cl.n);
        upload(c, cl.pairs, cl.in_src_pos, cl.n * 4);
        upload(c, cl.pairs + cl.n, cl.in_tgt_pos, cl.n * 4);
        cl.meta_bytes += 8 * cl.n;
    }
    cl.in_src_pos = cl.in_tgt_pos = nullptr;
}

// Metadata of several calls in one device block and one copy (batched
// submission).  The calls share the block: it is released with the context.
static void upload_meta_batch(Ctx& c, std::vector<Call*>& calls) {
    if (calls.empty()) return;
    std::vector<size_t> at(calls.size());
    size_t total = 0;
    for (size_t i = 0; i < calls.size(); ++i) {
        at[i] = total;
        total += (meta_size(*calls[i]) + 15) & ~(size_t)15;
    }
    std::vector<char> host(total);
    for (size_t i = 0; i < calls.size(); ++i) fill_meta(*calls[i], host.data() + at[i]);
    char* dev = static_cast<char*>(dalloc(c, total));
    upload(c, dev, host.data(), total);
    for (size_t i = 0; i < calls.size(); ++i) {
        bind_meta(*calls[i], dev + at[i]);
        calls[i]->meta_shared = true;
        calls[i]->in_src_pos = calls[i]->in_tgt_pos = nullptr;
    }
}

static void free_meta(Ctx& c, Call& cl) {
    if (!cl.meta_shared) dfree(c, cl.meta);
    cl.meta = nullptr;
}

// ------------------------------------------------------------------ generation store in blocks
// The generation-order arrays (source ordinal, target, delay, weight) live in
// fixed-size blocks of physical device memory (GEN_BLOCK connections each)
// mapped on demand behind four reserved virtual ranges: kernels see
// contiguous arrays and growth maps the next blocks (no copy, no wait for the
// device).  After Prepare (or at destroy) a context hands its ranges, still
// mapped, to a per-device store that the next context takes whole, so a
// steady stream of contexts maps nothing; a context that finds the store in
// use maps its own blocks and releases them at its end unless the store is
// empty, which it then fills.
namespace {
constexpr uint64_t GEN_BLOCK = 1ull << 26;                 // connections per block
constexpr uint64_t GEN_VA_CONNS = 1ull << 35;              // reserved connections per array
constexpr size_t GEN_BPC[4] = {4, 4, 2, 4};                // bytes per connection of each array
constexpr int GEN_MAX_DEVICES = 64;

struct MappedStore {
    std::mutex m;
    bool in_use = false;
    char* va[4] = {nullptr, nullptr, nullptr, nullptr};
    std::vector<std::array<void*, 4>> blocks;
    uint64_t mapped = 0;
};

MappedStore& mapped_store(int device) {
    static MappedStore stores[GEN_MAX_DEVICES];
    return stores[device];
}

void unmap_all(char* const va[4], const std::vector<std::array<void*, 4>>& blocks) {
    for (int a = 0; a < 4; ++a) {
        const size_t bytes = GEN_BPC[a] * GEN_BLOCK;
        for (size_t b = 0; b < blocks.size(); ++b) {
            (void)hipMemUnmap(va[a] + bytes * b, bytes);
            (void)hipMemRelease(static_cast<hipMemGenericAllocationHandle_t>(blocks[b][a]));
        }
        (void)hipMemAddressFree(va[a], GEN_BPC[a] * GEN_VA_CONNS);
    }
}

void gen_map(Ctx& c, uint64_t need) {
    if (need > GEN_VA_CONNS) raise(SNNC_EUNSUPPORTED, "more than 2^35 generated connections");
    if (!c.gen_va[0]) {
        MappedStore& st = mapped_store(c.device);
        std::lock_guard<std::mutex> lock(st.m);
        if (st.va[0] && !st.in_use) {   // take the device's mapped store whole
            st.in_use = true;
            c.gen_pooled = true;
            for (int a = 0; a < 4; ++a) c.gen_va[a] = st.va[a];
            c.gen_handles = st.blocks;
            c.gen_mapped = st.mapped;
            c.bytes_live += 14 * GEN_BLOCK * c.gen_handles.size();
            c.bytes_peak = std::max(c.bytes_peak, c.bytes_live);
        }
    }
    if (!c.gen_va[0]) {
        for (int a = 0; a < 4; ++a) {
            void* p = nullptr;
            if (hipMemAddressReserve(&p, GEN_BPC[a] * GEN_VA_CONNS, 0, nullptr, 0) != hipSuccess) {
                (void)hipGetLastError();
                for (int b = 0; b < a; ++b) (void)hipMemAddressFree(c.gen_va[b], GEN_BPC[b] * GEN_VA_CONNS);
                for (int b = 0; b < 4; ++b) c.gen_va[b] = nullptr;
                raise(SNNC_ENOMEM, "virtual address range for the generation arrays");
            }
            c.gen_va[a] = static_cast<char*>(p);
        }
        c.gen_pooled = false;
    }
    hipMemAllocationProp prop{};
    prop.type = hipMemAllocationTypePinned;
    prop.location.type = hipMemLocationTypeDevice;
    prop.location.id = c.device;
    hipMemAccessDesc acc{};
    acc.location = prop.location;
    acc.flags = hipMemAccessFlagsProtReadWrite;
    while (c.gen_mapped < need) {
        const size_t block_bytes = 14 * GEN_BLOCK;
        if (c.budget && c.bytes_live + block_bytes > c.budget)
            raise(SNNC_EBUDGET, "device-memory budget exceeded by a generation block");
        std::array<void*, 4> hs{};
        int done = 0;
        try {
            for (; done < 4; ++done) {
                const size_t bytes = GEN_BPC[done] * GEN_BLOCK;
                hipMemGenericAllocationHandle_t h{};
                if (hipMemCreate(&h, bytes, &prop, 0) != hipSuccess) {
                    (void)hipGetLastError();
                    raise(SNNC_ENOMEM, "no device memory for a generation block of " + std::to_string(bytes) + " bytes");
                }
                char* at = c.gen_va[done] + GEN_BPC[done] * c.gen_mapped;
                if (hipMemMap(at, bytes, 0, h, 0) != hipSuccess) {
                    (void)hipMemRelease(h);
                    (void)hipGetLastError();
                    raise(SNNC_EDEVICE, "mapping a generation block failed");
                }
                if (hipMemSetAccess(at, bytes, &acc, 1) != hipSuccess) {
                    (void)hipMemUnmap(at, bytes);
                    (void)hipMemRelease(h);
                    (void)hipGetLastError();
                    raise(SNNC_EDEVICE, "access to a generation block failed");
                }
                hs[done] = h;
            }
        } catch (...) {
            for (int a = 0; a < done; ++a) {
                (void)hipMemUnmap(c.gen_va[a] + GEN_BPC[a] * c.gen_mapped, GEN_BPC[a] * GEN_BLOCK);
                (void)hipMemRelease(static_cast<hipMemGenericAllocationHandle_t>(hs[a]));
            }
            throw;
        }
        c.gen_handles.push_back(hs);
        c.gen_mapped += GEN_BLOCK;
        c.bytes_live += block_bytes;
        c.bytes_peak = std::max(c.bytes_peak, c.bytes_live);
    }
    c.g_src = reinterpret_cast<uint32_t*>(c.gen_va[0]);
    c.g_tgt = reinterpret_cast<uint32_t*>(c.gen_va[1]);
    c.g_delay = reinterpret_cast<uint16_t*>(c.gen_va[2]);
    c.g_weight = reinterpret_cast<float*>(c.gen_va[3]);
    c.cap_gen = c.gen_mapped;
}

}  // namespace

bool gen_blocks_supported(int device) {
    if (device < 0 || device >= GEN_MAX_DEVICES) return false;
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeVirtualMemoryManagementSupported, device) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    hipMemAllocationProp prop{};
    prop.type = hipMemAllocationTypePinned;
    prop.location.type = hipMemLocationTypeDevice;
    prop.location.id = device;
    size_t gran = 0;
    if (hipMemGetAllocationGranularity(&gran, &prop, hipMemAllocationGranularityMinimum) != hipSuccess || !gran) {
        (void)hipGetLastError();
        return false;
    }
    return v != 0 && (2 * GEN_BLOCK) % gran == 0;
}

// Hands the context's generation store back (the caller has waited for every
// kernel that uses it): into the device's store, still mapped, when it came
// from there or the store is empty; else unmapped and released.
void gen_release(Ctx& c) {
    if (!c.gen_vmm || !c.gen_va[0]) return;
    bool kept = false;
    {
        MappedStore& st = mapped_store(c.device);
        std::lock_guard<std::mutex> lock(st.m);
        if (c.gen_pooled || !st.va[0]) {
            for (int a = 0; a < 4; ++a) st.va[a] = c.gen_va[a];
            st.blocks = c.gen_handles;
            st.mapped = c.gen_mapped;
            st.in_use = false;
            kept = true;
        }
    }
    if (!kept) unmap_all(c.gen_va, c.gen_handles);
    c.bytes_live -= 14 * GEN_BLOCK * c.gen_handles.size();
    for (int a = 0; a < 4; ++a) c.gen_va[a] = nullptr;
    c.gen_handles.clear();
    c.gen_mapped = 0;
    c.gen_pooled = false;
    c.g_src = c.g_tgt = nullptr;
    c.g_delay = nullptr;
    c.g_weight = nullptr;
    c.cap_gen = 0;
}

void grow_gen(Ctx& c, uint64_t need) {
    if (need <= c.cap_gen) return;
    if (c.gen_vmm) {
        gen_map(c, need);
        return;
    }
    uint64_t cap = std::max<uint64_t>(c.cap_gen ? c.cap_gen : 1 << 16, 1 << 16);
    while (cap < need) cap *= 2;
    if (c.cap_gen && need <= c.cap_gen + (c.cap_gen >> 2)) cap = std::max(cap, need);
    uint32_t* s = dalloc_n<uint32_t>(c, cap);
    uint32_t* t = nullptr;
    uint16_t* d = nullptr;
    float* w = nullptr;
    try {
        t = dalloc_n<uint32_t>(c, cap);
        d = dalloc_n<uint16_t>(c, cap);
        w = dalloc_n<float>(c, cap);
    } catch (...) {
        dfree(c, s); dfree(c, t); dfree(c, d);
        throw;
    }
    if (c.n_gen) {
        HIPCHK(hipMemcpyAsync(s, c.g_src, c.n_gen * 4, hipMemcpyDeviceToDevice, c.stream));
        HIPCHK(hipMemcpyAsync(t, c.g_tgt, c.n_gen * 4, hipMemcpyDeviceToDevice, c.stream));
        HIPCHK(hipMemcpyAsync(d, c.g_delay, c.n_gen * 2, hipMemcpyDeviceToDevice, c.stream));
        HIPCHK(hipMemcpyAsync(w, c.g_weight, c.n_gen * 4, hipMemcpyDeviceToDevice, c.stream));
        sync(c);
    }
    dfree(c, c.g_src); dfree(c, c.g_tgt); dfree(c, c.g_delay); dfree(c, c.g_weight);
    c.g_src = s; c.g_tgt = t; c.g_delay = d; c.g_weight = w;
    c.cap_gen = cap;
}

// A validated call record without its device metadata (not yet admitted).
// Assigned nodes come only through snnc_connect_assigned, which passes the
// pair arrays (`pairs` true, arrays may be null when n is 0).
static Call make_call_host(Ctx& c, const snnc_nodeset* src, const snnc_nodeset* tgt, const snnc_conn_spec* conn,
                           const snnc_syn_spec* syn, int32_t alpha, bool pairs = false,
                           const uint32_t* src_pos = nullptr, const uint32_t* tgt_pos = nullptr) {
    if (c.prepared) raise(SNNC_ESTATE, "connect after prepare");
    if (!conn) raise(SNNC_EINVAL, "null argument");
    if ((conn->kind == SNNC_ASSIGNED_NODES) != pairs)
        raise(SNNC_EINVAL, "assigned nodes take their pairs through snnc_connect_assigned");
    Call cl;
    cl.in_src_pos = src_pos;
    cl.in_tgt_pos = tgt_pos;
    cl.id = (uint32_t)c.calls.size();
    cl.rule = conn->kind;
    cl.n = conn->n;
    cl.p = conn->p;
    cl.autapses = conn->allow_autapses != 0;
    cl.multapses = conn->allow_multapses != 0;
    cl.alpha = alpha;
    cl.S = make_set(c, src);
    cl.T = make_set(c, tgt);
    validate(c, cl, syn);
    return cl;
}

// Whether the call's device tables are needed on this host: it has local
// sources or targets (a call with neither adds no local connection and no
// entry to the local send lists), or it takes assigned pairs (the caller's
// pair arrays are copied during the call).  Other calls keep host records only;
// run_call uploads the tables if it is ever asked to run one.
static bool needs_meta(const Ctx& c, const Call& cl) {
    if (cl.rule == SNNC_ASSIGNED_NODES) return true;
    for (auto& g : cl.S.seg) if (g.host == c.P_local && g.n) return true;
    for (auto& g : cl.T.seg) if (g.host == c.P_local && g.n) return true;
    return false;
}

// ... with its device metadata where this host needs it.
static Call make_call(Ctx& c, const snnc_nodeset* src, const snnc_nodeset* tgt, const snnc_conn_spec* conn,
                      const snnc_syn_spec* syn, int32_t alpha, bool pairs = false,
                      const uint32_t* src_pos = nullptr, const uint32_t* tgt_pos = nullptr) {
    Call cl = make_call_host(c, src, tgt, conn, syn, alpha, pairs, src_pos, tgt_pos);
    if (needs_meta(c, cl)) upload_meta(c, cl);
    return cl;
}

// resident bytes of a call with n connections: 14 B per connection + metadata
static uint64_t resident_cost(const Call& cl, uint64_t n) { return n * 14 + cl.meta_bytes; }

// A lower bound of a call's local connection count, known without draws: a
// fixed total number with every target on this host keeps exactly N, and the
// other rules counted on the device may keep none.
static uint64_t min_local_count(const Ctx& c, const Call& cl) {
    if (cl.rule != SNNC_FIXED_TOTAL_NUMBER) return 0;
    uint64_t on_host = 0;
    for (auto& g : cl.T.seg) if (g.host == c.P_local) on_host += g.n;
    return on_host == cl.T.total ? cl.n : 0;
}

// Whether admission rejects the call whatever its draws give: the budget is
// exceeded already by its smallest possible count (the resident bytes only
// grow until then), so its device count can be skipped.
static bool surely_over_budget(const Ctx& c, const Call& cl) {
    return c.resident_budget && c.resident_bytes + resident_cost(cl, min_local_count(c, cl)) > c.resident_budget;
}

static void admit(Ctx& c, Call& cl, uint64_t n) {
    const uint64_t cost = resident_cost(cl, n);
    if (c.resident_budget && c.resident_bytes + cost > c.resident_budget)
        raise(SNNC_EBUDGET, "request of " + std::to_string(n) + " connections exceeds the resident budget");
}

// Builds the call record and counts its local connections (served mode).  A
// count that needs device work runs on the counting lane, so that the host
// reads it back without waiting for generation already queued on the
// caller's stream.
static Call counted_call(Ctx& c, const snnc_nodeset* src, const snnc_nodeset* tgt, const snnc_conn_spec* conn,
                         const snnc_syn_spec* syn, int32_t alpha, uint64_t* n_out, bool pairs = false,
                         const uint32_t* src_pos = nullptr, const uint32_t* tgt_pos = nullptr) {
    Call cl = make_call_host(c, src, tgt, conn, syn, alpha, pairs, src_pos, tgt_pos);
    if (!needs_meta(c, cl)) {          // no local target: nothing to count or generate here
        *n_out = 0;
        return cl;
    }
    if (!count_on_device(c, cl)) {     // counted on the host: no second stream needed
        upload_meta(c, cl);
        try {
            *n_out = gen_count_local(c, cl);
        } catch (...) {
            free_meta(c, cl);
            dfree(c, cl.pairs);
            throw;
        }
        return cl;
    }
    CountScope lane(c);
    upload_meta(c, cl);
    if (surely_over_budget(c, cl)) {   // the caller's admission rejects it: no device count
        *n_out = min_local_count(c, cl);
        return cl;
    }
    try {
        *n_out = gen_count_local(c, cl);
    } catch (...) {
        free_meta(c, cl);
        dfree(c, cl.pairs);
        release_pre(c, cl);
        throw;
    }
    return cl;
}

static void connect_impl(Ctx& c, const snnc_nodeset* src, const snnc_nodeset* tgt, const snnc_conn_spec* conn,
                         const snnc_syn_spec* syn, int32_t alpha, uint32_t* call_id_out, bool pairs = false,
                         const uint32_t* src_pos = nullptr, const uint32_t* tgt_pos = nullptr) {
    if (!call_id_out) raise(SNNC_EINVAL, "null argument");
    uint64_t n = 0;
    Call cl = c.resident_budget ? counted_call(c, src, tgt, conn, syn, alpha, &n, pairs, src_pos, tgt_pos)
                                : make_call(c, src, tgt, conn, syn, alpha, pairs, src_pos, tgt_pos);
    try {
        if (c.resident_budget) admit(c, cl, n);
        if (!c.conn_started) {
            HIPCHK(hipEventRecord(c.conn_first, c.stream));
            c.conn_started = true;
        }
        cl.gen_begin = c.n_gen;
        cl.gen_count = cl.meta ? gen_local(c, cl) : 0;   // no tables: no local target
        HIPCHK(hipGetLastError());
    } catch (...) {
        free_meta(c, cl);
        dfree(c, cl.pairs);
        release_pre(c, cl);
        throw;
    }
    c.n_gen += cl.gen_count;
    c.resident_bytes += resident_cost(cl, cl.gen_count);
    c.calls.push_back(std::move(cl));
    *call_id_out = c.calls.back().id;
}

static void submit_impl(Ctx& c, const snnc_nodeset* src, const snnc_nodeset* tgt, const snnc_conn_spec* conn,
                        const snnc_syn_spec* syn, int32_t alpha, uint32_t* call_id_out) {
    if (!call_id_out) raise(SNNC_EINVAL, "null argument");
    uint64_t n = 0;
    Call cl = counted_call(c, src, tgt, conn, syn, alpha, &n);
    try {
        admit(c, cl, n);
        grow_gen(c, c.n_gen + n);
        if (!c.conn_started) {
            HIPCHK(hipEventRecord(c.conn_first, c.stream));
            c.conn_started = true;
        }
        cl.gen_begin = c.n_gen;
        cl.gen_count = n;
    } catch (...) {
        free_meta(c, cl);
        dfree(c, cl.pairs);
        release_pre(c, cl);
        throw;
    }
    c.n_gen += cl.gen_count;
    c.resident_bytes += resident_cost(cl, cl.gen_count);
    c.queued.push_back(cl.id);
    c.calls.push_back(std::move(cl));
    *call_id_out = c.calls.back().id;
}

// Several requests with one wait for the device counts: as submit_impl for
// each request in order, but the counts that need the device are queued on
// the counting lane for all requests first, their totals read after one
// wait, and then the requests are admitted in order.  The counts depend on
// the call id, so they are drawn with the ids the requests get if the
// predicted admissions hold (exact host counts, expected device counts
// against the budget); where an id turns out different, the rest of the
// batch is counted again from there with the ids now known.
static void submit_many_impl(Ctx& c, uint32_t n, const snnc_nodeset* src, const snnc_nodeset* tgt,
                             const snnc_conn_spec* conn, const snnc_syn_spec* syn, const int32_t* alpha,
                             snnc_status* status, uint32_t* ids) {
    if (c.prepared) raise(SNNC_ESTATE, "submit after prepare");
    if (n && (!src || !tgt || !conn || !syn || !alpha || !status || !ids)) raise(SNNC_EINVAL, "null argument");
    if (c.defer_cap < n) {
        if (c.defer_pin) {
            if (c.count_stream) HIPCHK(hipStreamSynchronize(c.count_stream));   // no count still writes to it
            pinned_give(c.defer_pin, c.defer_cap * 2 * sizeof(uint64_t), hipHostMallocMapped);
        }
        c.defer_pin = c.defer_pin_dev = nullptr;
        c.defer_cap = 0;
        const size_t cap = std::max<size_t>(n, 256);
        c.defer_pin = static_cast<uint64_t*>(pinned_take(cap * 2 * sizeof(uint64_t), hipHostMallocMapped));
        HIPCHK(hipHostGetDevicePointer((void**)&c.defer_pin_dev, c.defer_pin, 0));
        c.defer_cap = cap;
    }
    std::vector<Call> cls(n);
    std::vector<uint64_t> count(n, 0);
    std::vector<char> ok(n, 0), on_device(n, 0);
    auto drop = [&](Call& cl) {
        free_meta(c, cl);
        dfree(c, cl.pairs);
        release_pre(c, cl);
        cl.meta = nullptr;
        cl.pairs = nullptr;
    };
    auto fatal = [](const Error& e) {
        return e.code == SNNC_EDEVICE || e.code == SNNC_ENOMEM || e.code == SNNC_ESTATE;
    };
    auto expected = [&](const Call& cl) -> uint64_t {   // expected local count of a device-counted request
        uint64_t on_host = 0;
        for (auto& g : cl.T.seg) if (g.host == c.P_local) on_host += g.n;
        const double share = cl.T.total ? (double)on_host / (double)cl.T.total : 0.0;
        switch (cl.rule) {
        case SNNC_PAIRWISE_BERNOULLI: return (uint64_t)(cl.p * (double)cl.S.total * (double)on_host);
        case SNNC_FIXED_TOTAL_NUMBER: return (uint64_t)((double)cl.n * share);
        case SNNC_FIXED_OUTDEGREE: return (uint64_t)((double)cl.S.total * (double)cl.n * share);
        case SNNC_ASSIGNED_NODES: {
            const auto it = cl.pairs_on.find(c.P_local);
            return it == cl.pairs_on.end() ? 0 : it->second;
        }
        default: return 0;
        }
    };
    // 1. records, tables and host counts (on the counting lane; the caller's
    // stream waits for it at the end of each counting section)
    {
        CountScope lane(c);
        std::vector<char> meta(n, 0);
        std::vector<Call*> with_meta;
        for (uint32_t i = 0; i < n; ++i) {
            status[i] = SNNC_OK;
            ids[i] = UINT32_MAX;
            Call& cl = cls[i];
            try {
                cl = make_call_host(c, &src[i], &tgt[i], &conn[i], &syn[i], alpha[i]);
                if (needs_meta(c, cl)) {
                    meta[i] = 1;
                    with_meta.push_back(&cl);
                }
                ok[i] = 1;
            } catch (const Error& e) {
                drop(cl);
                if (fatal(e)) {
                    for (uint32_t k = 0; k < i; ++k) drop(cls[k]);
                    throw;
                }
                status[i] = e.code;
            }
        }
        try {
            upload_meta_batch(c, with_meta);   // the tables of the whole batch: one block, one copy
        } catch (...) {
            for (uint32_t k = 0; k < n; ++k) drop(cls[k]);
            throw;
        }
        for (uint32_t i = 0; i < n; ++i) {
            if (!meta[i]) continue;
            Call& cl = cls[i];
            try {
                if (count_on_device(c, cl)) on_device[i] = 1;
                else count[i] = gen_count_local(c, cl);   // no draws: independent of the call id
            } catch (const Error& e) {
                drop(cl);
                if (fatal(e)) {
                    for (uint32_t k = 0; k < n; ++k) drop(cls[k]);
                    throw;
                }
                ok[i] = 0;
                status[i] = e.code;
            }
        }
    }
    uint32_t start = 0;
    try {
        while (start < n) {
            // 2. device counts of requests start.. with their predicted ids, then one wait
            bool queued = false;
            {
                CountScope lane(c);
                // the counts' tile scans are queued and launched together before the wait
                c.scan_batching = true;
                struct ScanBatch {
                    Ctx& c;
                    ~ScanBatch() {   // on an error: drop the queued scans, release their inputs
                        c.scan_batching = false;
                        for (void* p : c.scan_owned) dfree(c, p);
                        c.scan_jobs.clear();
                        c.first_jobs.clear();
                        c.scan_owned.clear();
                    }
                } scan_batch{c};
                uint32_t next = (uint32_t)c.calls.size();
                uint64_t predicted = c.resident_bytes;
                for (uint32_t i = start; i < n; ++i) {
                    if (!ok[i]) continue;
                    Call& cl = cls[i];
                    cl.id = next;
                    uint64_t est = count[i];
                    if (on_device[i] && surely_over_budget(c, cl)) {
                        // rejected at admission whatever the draws give: no device count
                        on_device[i] = 0;
                        est = count[i] = min_local_count(c, cl);
                    }
                    if (on_device[i]) {
                        release_pre(c, cl);
                        cl.deferred = 0;
                        c.defer_slot = c.defer_pin_dev + 2 * i;
                        try {
                            count[i] = gen_count_local(c, cl);
                        } catch (const Error& e) {
                            c.defer_slot = nullptr;
                            if (fatal(e)) throw;
                            drop(cl);
                            ok[i] = 0;
                            status[i] = e.code;
                            continue;
                        }
                        c.defer_slot = nullptr;
                        if (cl.deferred) {
                            queued = true;
                            est = expected(cl);
                        } else {
                            est = count[i];
                        }
                    }
                    const uint64_t cost = resident_cost(cl, est);
                    if (!c.resident_budget || predicted + cost <= c.resident_budget) {
                        predicted += cost;
                        ++next;
                    }
                }
                c.scan_batching = false;
                scan_batch_run(c);
            }
            if (queued) HIPCHK(hipStreamSynchronize(c.count_stream));
            // 3. admission in order, up to the first request whose id moved
            uint32_t restart = n;
            for (uint32_t i = start; i < n; ++i) {
                if (!ok[i]) continue;
                Call& cl = cls[i];
                const uint32_t id = (uint32_t)c.calls.size();
                if (cl.id != id) {
                    if (on_device[i]) {   // its draws used another id: count again from here
                        restart = i;
                        break;
                    }
                    cl.id = id;
                }
                try {
                    if (cl.deferred) {
                        const volatile uint64_t* w = c.defer_pin + 2 * i;
                        bool again = false;
                        if (cl.deferred == 1) count[i] = w[0];
                        else if (w[0] >= cl.n) count[i] = cl.deferred == 2 ? cl.n : w[1];
                        else again = true;   // too few valid candidates in the window
                        cl.deferred = 0;
                        if (again) {
                            release_pre(c, cl);
                            CountScope lane(c);
                            count[i] = gen_count_local(c, cl);
                        } else {
                            cl.pre_count = count[i];
                        }
                    }
                    admit(c, cl, count[i]);
                    grow_gen(c, c.n_gen + count[i]);
                } catch (const Error& e) {
                    if (fatal(e)) throw;
                    drop(cl);
                    ok[i] = 0;
                    status[i] = e.code;
                    continue;
                }
                if (!c.conn_started) {
                    HIPCHK(hipEventRecord(c.conn_first, c.stream));
                    c.conn_started = true;
                }
                cl.gen_begin = c.n_gen;
                cl.gen_count = count[i];
                c.n_gen += cl.gen_count;
                c.resident_bytes += resident_cost(cl, cl.gen_count);
                c.queued.push_back(cl.id);
                ids[i] = cl.id;
                ok[i] = 0;   // moved into the context
                c.calls.push_back(std::move(cl));
            }
            start = restart;
        }
    } catch (...) {
        for (uint32_t k = 0; k < n; ++k)
            if (ok[k]) drop(cls[k]);
        c.defer_slot = nullptr;
        throw;
    }
}

void flush_pending(Ctx& c) {
    if (c.queued.empty()) return;
    hipEvent_t ev;
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    c.batch_done.push_back(ev);
    const int32_t b = (int32_t)c.batch_done.size() - 1;
    std::vector<uint32_t> ids;
    ids.swap(c.queued);
    for (uint32_t id : ids) c.calls[id].batch = b;
    flush_batch(c, ids, ev);
}

static void free_results(Ctx& c) {
    for (auto& kv : c.arrays) free_array(c, kv.second);
    c.arrays.clear();
    c.counts.clear();
}

// ------------------------------------------------------------------ fused-launch autotuner
// Times the persistent batch launch at 1 .. 32 workgroups per compute unit on
// a synthetic batch of fusable requests (fixed in-degree and out-degree with
// multapses, total number with autapses and multapses, one-to-one; sizes
// spread over three decades) of about n connections, in scratch contexts on
// the same device, allocator and stream, and keeps the fastest grid for the
// process.  The grid changes no result: items are addressed by index.
namespace {

// serialises tuner runs (the scratch contexts of a run read the cache at init)
std::mutex& fused_tune_mutex() {
    static std::mutex m;
    return m;
}

std::atomic<int>* fused_tune_cache() {
    static std::atomic<int> best[64] = {};
    return best;
}

float time_fused_grid(snnc_ctx* ctx, int wgs, uint64_t n) {
    snnc_ctx* t = nullptr;
    auto check = [&](snnc_status st) {
        if (st != SNNC_OK) {
            const std::string msg = t ? snnc_last_error(t) : "scratch context";
            if (t) snnc_destroy(t);
            raise(st, "fused autotuner: " + msg);
        }
    };
    check(snnc_init(&t, 1, 0, 7, 0.1, ctx->has_alloc ? &ctx->alloc : nullptr, ctx->stream, 0));
    check(snnc_tune(t, "fused_wgs_per_cu", wgs));
    check(snnc_set_resident_budget(t, ~0ull >> 1));
    snnc_segment a{}, b{};
    check(snnc_create(t, 0, 100000, &a));
    check(snnc_create(t, 0, 80000, &b));
    // about n connections per batch in 48 requests, sizes log-spread over 1e3 .. 1e6 x scale
    std::vector<snnc_conn_spec> cs;
    std::vector<snnc_nodeset> S, T;
    std::vector<snnc_segment> segs;
    segs.reserve(2 * 48);
    const double scale = std::max(1.0, (double)n / 48.0 / 3.0e5);
    for (int i = 0; i < 48; ++i) {
        const double size = 1.0e3 * std::pow(1.0e3, (double)i / 47.0) * scale;
        snnc_conn_spec c{};
        c.allow_autapses = c.allow_multapses = 1;
        snnc_segment src = (i & 1) ? a : b, tgt = (i & 1) ? b : a;
        switch (i % 4) {
        case 0:   // in-degree over a prefix of the targets
            tgt.n = (uint32_t)std::min<double>(tgt.n, std::max(1.0, size / 100.0));
            c.kind = SNNC_FIXED_INDEGREE;
            c.n = std::max<uint64_t>(1, (uint64_t)(size / tgt.n));
            break;
        case 1:
            src.n = (uint32_t)std::min<double>(src.n, std::max(1.0, size / 50.0));
            c.kind = SNNC_FIXED_OUTDEGREE;
            c.n = std::max<uint64_t>(1, (uint64_t)(size / src.n));
            break;
        case 2:
            c.kind = SNNC_FIXED_TOTAL_NUMBER;
            c.n = (uint64_t)size;
            break;
        default:
            src.n = tgt.n = (uint32_t)std::min<double>(std::min(src.n, tgt.n), size);
            c.kind = SNNC_ONE_TO_ONE;
            break;
        }
        segs.push_back(src);
        segs.push_back(tgt);
        cs.push_back(c);
    }
    for (int i = 0; i < 48; ++i) {
        S.push_back(snnc_nodeset{&segs[2 * i], 1});
        T.push_back(snnc_nodeset{&segs[2 * i + 1], 1});
    }
    snnc_syn_spec syn{};
    syn.weight.kind = SNNC_NORMAL;
    syn.weight.mean = 0.1;
    syn.weight.sd = 0.01;
    syn.delay_ms.kind = SNNC_NORMAL;
    syn.delay_ms.mean = 1.5;
    syn.delay_ms.sd = 0.75;
    syn.delay_ms.lo = 0.1;
    std::vector<snnc_syn_spec> Y(48, syn);
    std::vector<int32_t> A(48, -1);
    std::vector<snnc_status> st(48);
    std::vector<uint32_t> ids(48);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float best = 1e30f;
    try {
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        for (int rep = 0; rep < 3; ++rep) {   // the first run captures the graph
            check(snnc_submit_many(t, 48, S.data(), T.data(), cs.data(), Y.data(), A.data(), st.data(), ids.data()));
            for (int i = 0; i < 48; ++i) check(st[i]);
            check(snnc_sync(t));
            HIPCHK(hipEventRecord(e0, t->stream));
            check(snnc_flush(t));
            HIPCHK(hipEventRecord(e1, t->stream));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            if (rep) best = std::min(best, ms);
        }
    } catch (...) {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        snnc_destroy(t);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    snnc_destroy(t);
    return best;
}

}  // namespace

int fused_grid_tuned(int device) {
    if (device < 0 || device >= 64) return 0;
    return fused_tune_cache()[device].load();
}

}  // namespace snnc

using namespace snnc;

template <class F>
static snnc_status guarded(snnc_ctx* ctx, F&& f) {
    try {
        if (ctx) HIPCHK(hipSetDevice(ctx->device));
        f();
        if (ctx) ctx->last_error.clear();
        return SNNC_OK;
    } catch (const Error& e) {
        if (ctx) ctx->last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        if (ctx) ctx->last_error = "host allocation failed";
        return SNNC_ENOMEM;
    } catch (const std::exception& e) {
        if (ctx) ctx->last_error = e.what();
        return SNNC_EDEVICE;
    }
}

extern "C" {

snnc_status snnc_init(snnc_ctx** out, uint32_t P, uint32_t P_local, uint32_t seed, double dt_ms,
                      const snnc_allocator* alloc, void* hip_stream, uint64_t budget_bytes) {
    if (!out) return SNNC_EINVAL;
    *out = nullptr;
    if (P == 0 || P_local >= P || !(dt_ms > 0.0)) return SNNC_EINVAL;
    if (alloc && (!alloc->alloc || !alloc->free)) return SNNC_EINVAL;
    snnc_ctx* c = new (std::nothrow) snnc_ctx();
    if (!c) return SNNC_ENOMEM;
    c->P = P;
    c->P_local = P_local;
    c->seed = seed;
    c->dt = dt_ms;
    c->stream = (hipStream_t)hip_stream;
    c->main_stream = c->stream;
    c->budget = budget_bytes;
    if (alloc) {
        c->alloc = *alloc;
        c->has_alloc = true;
    }
    c->M.assign(P, 0);
    snnc_status st = guarded(nullptr, [&] {
        HIPCHK(hipGetDevice(&c->device));
        (void)hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, c->device);
        if (c->n_cu < 1) c->n_cu = 256;
        HIPCHK(hipEventCreate(&c->phase_a));
        HIPCHK(hipEventCreate(&c->phase_b));
        HIPCHK(hipEventCreate(&c->conn_first));
        HIPCHK(hipEventCreate(&c->conn_last));
        init_ring(c->ring, 16u << 20);
        c->dl_pin_bytes = 64u << 10;
        c->dl_pin = static_cast<char*>(pinned_take(c->dl_pin_bytes, hipHostMallocDefault));
        c->tot_pin = static_cast<uint64_t*>(pinned_take(4 * sizeof(uint64_t), hipHostMallocMapped));
        HIPCHK(hipHostGetDevicePointer((void**)&c->tot_pin_dev, c->tot_pin, 0));
        c->d_status = dalloc_n<uint32_t>(*c, 1);
        HIPCHK(hipMemsetAsync(c->d_status, 0, 4, c->stream));
        sync(*c);
        noalloc_setup(*c);   // device address of the allocation-free sort's static scratch
        c->gen_vmm = gen_blocks_supported(c->device);
        const int tuned = fused_grid_tuned(c->device);   // the fused-launch autotuner's choice, if any
        if (tuned) c->fused_wgs_per_cu = tuned;
    });
    if (st != SNNC_OK) {
        snnc_destroy(c);
        return st;
    }
    *out = c;
    return SNNC_OK;
}

snnc_status snnc_destroy(snnc_ctx* c) {
    if (!c) return SNNC_OK;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->main_stream);
    if (c->count_stream) (void)hipStreamSynchronize(c->count_stream);
    for (auto& kv : c->arrays)
        if (kv.second.host) (void)hipHostFree(kv.second.p);
    c->arrays.clear();
    gen_release(*c);
    std::vector<void*> ptrs;
    for (auto& kv : c->live) ptrs.push_back(kv.first);
    for (void* p : ptrs) raw_free(*c, p, true);   // the streams have drained
    if (c->count_stream) (void)hipStreamSynchronize(c->count_stream);
    (void)hipStreamSynchronize(c->main_stream);
    for (auto& p : c->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : c->event_pool) (void)hipEventDestroy(e);
    if (c->phase_a) (void)hipEventDestroy(c->phase_a);
    if (c->phase_b) (void)hipEventDestroy(c->phase_b);
    if (c->conn_first) (void)hipEventDestroy(c->conn_first);
    if (c->conn_last) (void)hipEventDestroy(c->conn_last);
    free_ring(c->ring);
    pinned_give(c->dl_pin, c->dl_pin_bytes, hipHostMallocDefault);
    pinned_give(c->tot_pin, 4 * sizeof(uint64_t), hipHostMallocMapped);
    pinned_give(c->defer_pin, c->defer_cap * 2 * sizeof(uint64_t), hipHostMallocMapped);
    for (auto e : c->batch_done) (void)hipEventDestroy(e);
    if (c->fused_exec) (void)hipGraphExecDestroy(c->fused_exec);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    for (auto& f : c->fences) (void)hipEventDestroy(f.second);
    for (auto e : c->fence_pool) (void)hipEventDestroy(e);
    if (c->count_done) (void)hipEventDestroy(c->count_done);
    free_ring(c->parked.ring);
    if (c->count_stream) (void)hipStreamDestroy(c->count_stream);
    delete c;
    return SNNC_OK;
}

const char* snnc_last_error(const snnc_ctx* c) { return c ? c->last_error.c_str() : "null context"; }

snnc_status snnc_sync(snnc_ctx* c) {
    if (!c) return SNNC_EINVAL;
    return guarded(c, [&] { sync(*c); });
}

snnc_status snnc_create(snnc_ctx* c, uint32_t host, uint32_t n, snnc_segment* out) {
    if (!c || !out) return SNNC_EINVAL;
    return guarded(c, [&] {
        if (c->prepared) raise(SNNC_ESTATE, "create after prepare");
        if (host >= c->P) raise(SNNC_EINVAL, "host out of range");
        if ((uint64_t)c->M[host] + n > 0x7fffffffull) raise(SNNC_EINVAL, "more than 2^31-1 neurons on a host");
        out->host = host;
        out->first = c->M[host];
        out->n = n;
        c->M[host] += n;
    });
}

snnc_status snnc_connect(snnc_ctx* c, const snnc_nodeset* src, const snnc_nodeset* tgt,
                         const snnc_conn_spec* conn, const snnc_syn_spec* syn, int32_t alpha,
                         uint32_t* call_id_out) {
    if (!c) return SNNC_EINVAL;
    return guarded(c, [&] { connect_impl(*c, src, tgt, conn, syn, alpha, call_id_out); });
}

snnc_status snnc_connect_assigned(snnc_ctx* c, const snnc_nodeset* src, const snnc_nodeset* tgt,
                                  const uint32_t* src_pos, const uint32_t* tgt_pos, uint64_t n,
                                  const snnc_syn_spec* syn, int32_t alpha, uint32_t* call_id_out) {
    if (!c) return SNNC_EINVAL;
    return guarded(c, [&] {
        snnc_conn_spec conn{};
        conn.kind = SNNC_ASSIGNED_NODES;
        conn.allow_autapses = 1;
        conn.allow_multapses = 1;
        conn.n = n;
        connect_impl(*c, src, tgt, &conn, syn, alpha, call_id_out, true, src_pos, tgt_pos);
    });
}

snnc_status snnc_set_resident_budget(snnc_ctx* c, uint64_t bytes) {
    if (!c) return SNNC_EINVAL;
    return guarded(c, [&] {
        if (c->prepared) raise(SNNC_ESTATE, "budget after prepare");
        c->resident_budget = bytes;
    });
}

snnc_status snnc_submit(snnc_ctx* c, const snnc_nodeset* src, const snnc_nodeset* tgt, const snnc_conn_spec* conn,
                        const snnc_syn_spec* syn, int32_t alpha, uint32_t* call_id_out) {
    if (!c) return SNNC_EINVAL;
    return guarded(c, [&] { submit_impl(*c, src, tgt, conn, syn, alpha, call_id_out); });
}

snnc_status snnc_submit_many(snnc_ctx* c, uint32_t n, const snnc_nodeset* src, const snnc_nodeset* tgt,
                             const snnc_conn_spec* conn, const snnc_syn_spec* syn, const int32_t* alpha,
                             snnc_status* status_out, uint32_t* call_ids_out) {
    if (!c) return SNNC_EINVAL;
    return guarded(c, [&] { submit_many_impl(*c, n, src, tgt, conn, syn, alpha, status_out, call_ids_out); });
}

snnc_status snnc_flush(snnc_ctx* c) {
    if (!c) return SNNC_EINVAL;
    return guarded(c, [&] {
        if (c->prepared) raise(SNNC_ESTATE, "flush after prepare");
        flush_pending(*c);
    });
}

snnc_status snnc_poll(snnc_ctx* c, uint32_t call_id, int32_t* done) {
    if (!c || !done) return SNNC_EINVAL;
    return guarded(c, [&] {
        if (call_id >= c->calls.size()) raise(SNNC_EINVAL, "unknown call id");
        const int32_t b = c->calls[call_id].batch;
        if (b < 0) {   // generated by connect, or waiting for a flush
            *done = 0;
            for (uint32_t id : c->queued)
                if (id == call_id) return;
            *done = 1;
            return;
        }
        const hipError_t e = hipEventQuery(c->batch_done[b]);
        if (e == hipErrorNotReady) {
            *done = 0;
            return;
        }
        HIPCHK(e);
        *done = 1;
    });
}

snnc_status snnc_reserve(snnc_ctx* c, uint64_t n) {
    if (!c) return SNNC_EINVAL;
    return guarded(c, [&] {
        if (c->prepared) raise(SNNC_ESTATE, "reserve after prepare");
        grow_gen(*c, n);
    });
}

snnc_status snnc_prepare(snnc_ctx* c) {
    if (!c) return SNNC_EINVAL;
    return guarded(c, [&] {
        if (c->prepared) raise(SNNC_ESTATE, "prepare called twice");
        flush_pending(*c);
        if (c->conn_started) {   // the connect phase ends where prepare's work begins
            HIPCHK(hipEventRecord(c->conn_last, c->stream));
            HIPCHK(hipEventSynchronize(c->conn_last));
            float cms = 0.f;
            HIPCHK(hipEventElapsedTime(&cms, c->conn_first, c->conn_last));
            c->ms_connect = cms;
        }
        HIPCHK(hipEventRecord(c->phase_a, c->stream));
        try {
            for (auto& cl : c->calls) {   // per-call launch tables are no longer needed (stream order)
                for (void* p : cl.owned) dfree(*c, p);
                cl.owned.clear();
            }
            prepare_all(*c);
        } catch (...) {
            free_results(*c);
            throw;
        }
        HIPCHK(hipEventRecord(c->phase_b, c->stream));
        HIPCHK(hipEventSynchronize(c->phase_b));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, c->phase_a, c->phase_b));
        c->ms_prepare = ms;
        uint32_t status = 0;
        download(*c, &status, c->d_status, 4);
        gen_release(*c);   // the stream has drained: the generation store goes back, still mapped
        if (status) raise(SNNC_EDEVICE, "a device wait exceeded its bound (status " + std::to_string(status) + ")");
        c->prepared = true;
    });
}

snnc_status snnc_get_array(const snnc_ctx* cc, int32_t id, const void** ptr, uint64_t* count) {
    snnc_ctx* c = const_cast<snnc_ctx*>(cc);
    if (!c || !ptr || !count) return SNNC_EINVAL;
    return guarded(c, [&] {
        *ptr = nullptr;
        *count = 0;
        switch (id) {
        case SNNC_GEN_SRC: case SNNC_GEN_TGT: case SNNC_GEN_DELAY: case SNNC_GEN_WEIGHT:
            if (c->prepared) raise(SNNC_ESTATE, "generation-order arrays are consumed by prepare");
            *count = c->n_gen;
            *ptr = id == SNNC_GEN_SRC ? (const void*)c->g_src
                 : id == SNNC_GEN_TGT ? (const void*)c->g_tgt
                 : id == SNNC_GEN_DELAY ? (const void*)c->g_delay : (const void*)c->g_weight;
            if (!c->n_gen) *ptr = nullptr;
            return;
        default:
            break;
        }
        auto it = c->arrays.find(id);
        if (it == c->arrays.end()) {
            if (id == SNNC_CALL_OFF || !c->prepared) {
                if (id != SNNC_CALL_OFF) raise(SNNC_ESTATE, "array not available before prepare");
            }
            if (id != SNNC_CALL_OFF) raise(SNNC_EINVAL, "unknown array id");
        }
        if (id == SNNC_CALL_OFF) {
            // host-derived; materialised on demand
            std::vector<uint64_t> off(c->calls.size() + 1);
            for (size_t i = 0; i < c->calls.size(); ++i) off[i] = c->calls[i].gen_begin;
            off.back() = c->n_gen;
            auto& a = c->arrays[SNNC_CALL_OFF];
            dfree(*c, a.p);
            a.p = dalloc(*c, off.size() * 8);
            a.bytes = off.size() * 8;
            upload(*c, a.p, off.data(), off.size() * 8);
            c->counts[SNNC_CALL_OFF] = off.size();
            it = c->arrays.find(id);
        }
        *count = c->counts[id];
        *ptr = *count ? it->second.p : nullptr;
    });
}

static size_t elem_size(int32_t id) {
    switch (id) {
    case SNNC_GEN_DELAY: case SNNC_DELAY: return 2;
    case SNNC_CALL_OFF: case SNNC_ROW_PTR: case SNNC_R_OFF: case SNNC_IMG_BASE: case SNNC_S_OFF:
    case SNNC_TP_PTR: case SNNC_H_OFF: case SNNC_GQ_PTR: case SNNC_IMG_FIRST: return 8;
    default: return 4;
    }
}

snnc_status snnc_copy_array(snnc_ctx* c, int32_t id, void* dst, uint64_t cap_bytes) {
    if (!c) return SNNC_EINVAL;
    const void* p = nullptr;
    uint64_t n = 0;
    snnc_status st = snnc_get_array(c, id, &p, &n);
    if (st != SNNC_OK) return st;
    return guarded(c, [&] {
        const uint64_t bytes = n * elem_size(id);
        if (bytes > cap_bytes) raise(SNNC_EINVAL, "destination too small");
        if (!bytes) return;
        HIPCHK(hipMemcpyAsync(dst, p, bytes, hipMemcpyDefault, c->stream));
        sync(*c);
    });
}

snnc_status snnc_copy_range(snnc_ctx* c, int32_t id, uint64_t first, uint64_t count, void* dst) {
    if (!c) return SNNC_EINVAL;
    const void* p = nullptr;
    uint64_t n = 0;
    snnc_status st = snnc_get_array(c, id, &p, &n);
    if (st != SNNC_OK) return st;
    return guarded(c, [&] {
        if (first > n || count > n - first) raise(SNNC_EINVAL, "range outside the array");
        if (!count) return;
        const size_t es = elem_size(id);
        HIPCHK(hipMemcpyAsync(dst, static_cast<const char*>(p) + first * es, count * es, hipMemcpyDefault, c->stream));
        sync(*c);
    });
}

snnc_status snnc_stats(snnc_ctx* c, snnc_stats_t* out) {
    if (!c || !out) return SNNC_EINVAL;
    return guarded(c, [&] {
        out->n_connections = c->n_gen;
        out->n_images = c->n_img;
        out->n_calls = (uint32_t)c->calls.size();
        out->M_local = c->M[c->P_local];
        out->bytes_live = c->bytes_live;
        out->bytes_peak = c->bytes_peak;
        out->sort_passes = c->sort_passes;
        out->key_bits = c->key_bits;
        out->ms_connect = c->ms_connect;
        out->ms_prepare = c->ms_prepare;
    });
}

snnc_status snnc_tune(snnc_ctx* c, const char* key, int64_t value) {
    if (!c || !key) return SNNC_EINVAL;
    return guarded(c, [&] {
        if (!strcmp(key, "sort_variant")) {
            if (value < 0 || value >= sort_variant_count()) raise(SNNC_EINVAL, "sort_variant out of range");
            c->sort_variant = (int)value;
            c->sort_pinned = true;
        } else if (!strcmp(key, "number_variant")) {
            if (value < 0 || value >= number_variant_count()) raise(SNNC_EINVAL, "number_variant out of range");
            c->number_variant = (int)value;
        } else if (!strcmp(key, "mark_in_lds")) {
            if (value < 0 || value > 1) raise(SNNC_EINVAL, "mark_in_lds must be 0 or 1");
            c->mark_in_lds = value == 1;
        } else if (!strcmp(key, "sort_mode")) {
            if (value < 0 || value > 1) raise(SNNC_EINVAL, "sort_mode out of range");
            c->sort_mode = (int)value;
            c->sort_pinned = true;
        } else if (!strcmp(key, "digit_bits")) {
            if (value != 0 && value != 8 && value != 9) raise(SNNC_EINVAL, "digit_bits must be 0, 8 or 9");
            c->digit_bits = (int)value;
        } else if (!strcmp(key, "map_path")) {
            if (value < 0 || value > 1) raise(SNNC_EINVAL, "map_path out of range");
            c->force_map_path = value == 1;
        } else if (!strcmp(key, "gen_blocks")) {
            if (value < 0 || value > 1) raise(SNNC_EINVAL, "gen_blocks must be 0 or 1");
            if (c->cap_gen) raise(SNNC_ESTATE, "gen_blocks before the first connection");
            if (value == 1 && !gen_blocks_supported(c->device))
                raise(SNNC_EUNSUPPORTED, "the device has no virtual memory management");
            c->gen_vmm = value == 1;
        } else if (!strcmp(key, "bern_masks")) {
            if (value < 0 || value > 1) raise(SNNC_EINVAL, "bern_masks must be 0 or 1");
            c->bern_masks = value == 1;
        } else if (!strcmp(key, "total_small_max")) {
            if (value < 0 || value > (1ll << 15)) raise(SNNC_EINVAL, "total_small_max out of range");
            c->total_small_max = (uint64_t)value;
        } else if (!strcmp(key, "total_hash_max")) {
            if (value < 0 || value > (1ll << 32)) raise(SNNC_EINVAL, "total_hash_max out of range");
            c->total_hash_max = (uint64_t)value;
        } else if (!strcmp(key, "floyd_wave_max")) {
            if (value < 0 || value > 8192) raise(SNNC_EINVAL, "floyd_wave_max out of range");
            c->floyd_wave_max = (uint32_t)value;
        } else if (!strcmp(key, "fuse_batches")) {
            c->fuse_batches = value != 0;
        } else if (!strcmp(key, "fused_wgs_per_cu")) {
            if (value < 1 || value > 64) raise(SNNC_EINVAL, "fused_wgs_per_cu out of range");
            c->fused_wgs_per_cu = (int)value;
            if (c->fused_exec) HIPCHK(hipGraphExecDestroy(c->fused_exec));
            c->fused_exec = nullptr;
        } else {
            raise(SNNC_EINVAL, std::string("unknown tuning key ") + key);
        }
    });
}


snnc_status snnc_autotune_fused(snnc_ctx* c, uint64_t n, int32_t* wgs_out, float* ms_out) {
    if (!c || !wgs_out || !ms_out || n == 0) return SNNC_EINVAL;
    return guarded(c, [&] {
        if (c->prepared) raise(SNNC_ESTATE, "autotune after prepare");
        if (c->device < 0 || c->device >= 64) raise(SNNC_EUNSUPPORTED, "device ordinal above 63");
        std::lock_guard<std::mutex> lock(fused_tune_mutex());
        int best_w = fused_tune_cache()[c->device].load();
        float best = -1.f;
        if (!best_w) {
            best = 1e30f;
            for (int w : {1, 2, 4, 8, 16, 32}) {
                const float ms = time_fused_grid(c, w, n);
                if (ms < best) {
                    best = ms;
                    best_w = w;
                }
            }
            fused_tune_cache()[c->device].store(best_w);
        }
        c->fused_wgs_per_cu = best_w;
        if (c->fused_exec) HIPCHK(hipGraphExecDestroy(c->fused_exec));
        c->fused_exec = nullptr;
        *wgs_out = best_w;
        *ms_out = best;
    });
}

snnc_status snnc_set_memory_level(snnc_ctx* c, int32_t level) {
    if (!c) return SNNC_EINVAL;
    return guarded(c, [&] {
        if (c->prepared) raise(SNNC_ESTATE, "memory level after prepare");
        if (level < 0 || level > 3) raise(SNNC_EINVAL, "memory level out of range");
        c->mem_level = level;
        c->img_sources = level == 0 ? SNNC_IMAGES_USED : SNNC_IMAGES_ALL;
    });
}

snnc_status snnc_array_on_host(const snnc_ctx* cc, int32_t id, int32_t* on_host) {
    snnc_ctx* c = const_cast<snnc_ctx*>(cc);
    if (!c || !on_host) return SNNC_EINVAL;
    const void* p = nullptr;
    uint64_t n = 0;
    snnc_status st = snnc_get_array(c, id, &p, &n);
    if (st != SNNC_OK) return st;
    auto it = c->arrays.find(id);
    *on_host = (it != c->arrays.end() && it->second.host) ? 1 : 0;
    return SNNC_OK;
}

snnc_status snnc_set_map_policy(snnc_ctx* c, int32_t numbering, int32_t image_sources, double xi) {
    if (!c) return SNNC_EINVAL;
    return guarded(c, [&] {
        if (c->prepared) raise(SNNC_ESTATE, "map policy after prepare");
        if (numbering < 0 || numbering > 1) raise(SNNC_EINVAL, "numbering out of range");
        if (image_sources < 0 || image_sources > 2) raise(SNNC_EINVAL, "image_sources out of range");
        if (!(xi >= 0.0) || !std::isfinite(xi)) raise(SNNC_EINVAL, "xi must be finite and >= 0");
        c->numbering = numbering;
        c->img_sources = image_sources;
        c->xi = xi;
    });
}

snnc_status snnc_set_timing(snnc_ctx* c, int enable) {
    if (!c) return SNNC_EINVAL;
    return guarded(c, [&] {
        if (enable < 0 || enable > 2) raise(SNNC_EINVAL, "timing must be 0, 1 or 2");
        resolve_times(*c);
        c->timing = enable;
        if (enable) c->ktimes.clear();
    });
}

snnc_status snnc_kernel_times(snnc_ctx* c, uint32_t cap, char (*names)[48], uint64_t* launches, double* ms,
                              uint32_t* n_out) {
    if (!c || !n_out) return SNNC_EINVAL;
    return guarded(c, [&] {
        resolve_times(*c);
        uint32_t i = 0;
        for (auto& kv : c->ktimes) {
            if (i < cap) {
                snprintf(names[i], 48, "%s", kv.first.c_str());
                launches[i] = kv.second.launches;
                ms[i] = kv.second.ms;
            }
            ++i;
        }
        *n_out = i;
    });
}

snnc_status snnc_delay_table(double mean, double sd, double lo, double dt, uint32_t* table, uint64_t cap,
                             uint32_t* k_lo_out, uint64_t* len_out) {
    if (!table || !k_lo_out || !len_out) return SNNC_EINVAL;
    if (!(sd > 0.0) || !(dt > 0.0) || !(lo >= dt)) return SNNC_EINVAL;
    std::vector<uint32_t> tab;
    uint32_t klo = 0;
    if (!build_delay_table(mean, sd, lo, dt, tab, klo, cap)) return SNNC_EINVAL;
    memcpy(table, tab.data(), tab.size() * sizeof(uint32_t));
    *k_lo_out = klo;
    *len_out = tab.size();
    return SNNC_OK;
}

}  // extern "C"
