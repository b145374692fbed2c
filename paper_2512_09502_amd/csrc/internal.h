// Internal declarations of the construction library (host planner side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <deque>
#include <array>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/snnc.h"

namespace snnc {

// ------------------------------------------------------------------ errors
struct Error {
    snnc_status code;
    std::string msg;
};

[[noreturn]] void raise(snnc_status code, const std::string& msg);
void hip_check(hipError_t e, const char* what);
#define HIPCHK(x) ::snnc::hip_check((x), #x)

// ------------------------------------------------------------------ device-side descriptors
// A segment of a node set: ordinals [ord_begin, ord_begin + n) are the local
// ids [first, first + n) on `host`.
struct SegD {
    uint64_t ord_begin;
    uint32_t host, first;
};

// A run of consecutive target ordinals that live on the generating host, for
// the rules whose unit is a target.  Within a run the "self position" (the
// ordinal of the same neuron in the source set, for autapse exclusion) is
// either absent (self_base < 0) or self_base + (t - t_ord).
struct TChunk {
    uint64_t t_ord;      // first target ordinal of the run
    uint64_t out_begin;  // first element of the run in the call's element space
    int64_t self_base;   // source ordinal of the first target, or -1
    uint32_t local_first;
    uint32_t n;          // targets in the run
};

// Synapse-value parameters of a call.
struct SynD {
    double w_mean, w_sd;
    const uint32_t* dtab;  // delay thresholds (device)
    const uint32_t* dguide;   // 257 entries: thresholds below j * 2^24 (device)
    uint32_t dtab_len;
    uint32_t d_klo;
    float w_const;
    uint32_t w_normal;     // 1: normal weight, 0: constant
    uint32_t d_normal;     // 1: table delay, 0: constant
    uint32_t d_const;
};

// ------------------------------------------------------------------ host-side call record
struct HostSet {
    std::vector<snnc_segment> seg;
    std::vector<uint64_t> ord_begin;
    uint64_t total = 0;
};

// Threshold table of a normal delay distribution (delay step klo + i while the
// word is at or above tab[i]) and its guide: guide[j] counts the thresholds
// below j 2^24, so a word in [j 2^24, (j + 1) 2^24) has its step between
// guide[j] and guide[j + 1].  Built once per distribution and context.
struct DelayTable {
    uint32_t klo = 0;
    std::vector<uint32_t> tab, guide;
};

struct Call {
    uint32_t id = 0;
    uint32_t rule = 0;
    uint64_t n = 0;
    double p = 0.0;
    bool autapses = true, multapses = true;
    int32_t alpha = -1;
    HostSet S, T;
    snnc_dist w{}, d{};
    float w_const = 0.f;
    uint16_t d_const = 0;
    uint32_t d_klo = 0;
    std::shared_ptr<const DelayTable> dtab;   // normal delays only
    // device copies
    void* meta = nullptr;       // one allocation: S segs, T segs, delay table
    bool meta_shared = false;   // meta lies in a block shared by a batch of calls (released with the context)
    size_t meta_bytes = 0;
    SegD* dS = nullptr;
    SegD* dT = nullptr;
    uint32_t* dtab_dev = nullptr;
    uint32_t* dguide_dev = nullptr;
    uint64_t gen_begin = 0, gen_count = 0;
    std::vector<void*> owned;   // device tables kept until the call's batch has run
    int32_t batch = -1;         // served mode: batch that generates the call (-1: not yet flushed)
    // results of the admission count, reused by the generation: tile offsets
    // (Bernoulli; valid-candidate offsets for fixed total number), per-item
    // bytes (Bernoulli: the 4-bit pair masks of each item; fixed total number:
    // first-occurrence flags), and for fixed total number the kept-candidate
    // offsets and the window
    uint64_t* pre_off = nullptr;
    uint64_t* pre_koff = nullptr;
    uint8_t* pre_first = nullptr;
    uint64_t pre_count = 0, pre_window = 0;
    // batched admission: the count was queued and its total is read later
    // (1 Bernoulli; 2 fixed total number, all targets local; 3 the same with
    // targets elsewhere, kept count in the second word)
    uint8_t deferred = 0;
    // assigned nodes: the caller's pair arrays during the call, then the
    // device copy (n source positions, then n target positions) and the
    // number of pairs per target host
    const uint32_t* in_src_pos = nullptr;
    const uint32_t* in_tgt_pos = nullptr;
    uint32_t* pairs = nullptr;
    std::map<uint32_t, uint64_t> pairs_on;
};

// ------------------------------------------------------------------ context
struct DevArray {
    void* p = nullptr;
    size_t bytes = 0;
    bool host = false;       // pinned host memory (GPU memory levels 0 and 1)
    void* dev = nullptr;     // its address for kernels when host
};

struct KernelTime {
    uint64_t launches = 0;
    double ms = 0.0;
};

// Per-stream state that changes hands when admission counting runs on its own
// stream: the stream, the pinned staging area, the radix-sort look-back table
// and the free lists of the small-block pool.
// Pinned staging ring for host-to-device uploads, in four quarters: an event
// recorded when the writer leaves a quarter covers every copy out of it, and
// the writer waits for that event only when it comes back to the quarter.
struct StageRing {
    char* buf = nullptr;
    size_t bytes = 0, used = 0;
    int q = 0;                           // quarter being filled
    hipEvent_t ev[4] = {};
    bool pending[4] = {};
};

// One queued exclusive scan of per-tile counts (out[n] and *total_out get the total).
struct ScanJob {
    const uint32_t* in;
    uint64_t* out;
    uint64_t* total_out;
    uint64_t n;
};

struct LaneState {
    hipStream_t stream = nullptr;
    StageRing ring;
    void* lookback = nullptr;
    size_t lookback_bytes = 0;
    uint32_t sort_epoch = 0;
    char* slab_cur = nullptr;
    size_t slab_left = 0;
    std::map<size_t, std::vector<void*>> small_free;
};

struct Ctx {
    uint32_t P = 1, P_local = 0, seed = 0;
    double dt = 0.1;
    hipStream_t stream = nullptr;        // stream of the active lane (the caller's stream outside counting)
    int device = 0;
    int n_cu = 256;                      // compute units of the device
    snnc_allocator alloc{};
    bool has_alloc = false;
    uint64_t budget = 0;
    uint64_t bytes_live = 0, bytes_peak = 0;
    std::map<void*, size_t> live;
    // small blocks (metadata, tables, tile counts) carved from slabs, so that
    // requests do not call the outer allocator: free lists per power-of-two class
    std::vector<void*> slabs;
    char* slab_cur = nullptr;                        // per lane
    size_t slab_left = 0;                            // per lane
    std::map<size_t, std::vector<void*>> small_free; // per lane
    std::map<void*, size_t> small_live;              // class | lane of each block in use
    std::string last_error;

    std::vector<uint32_t> M;          // neurons per host
    std::vector<Call> calls;
    bool prepared = false;

    // generation-order arrays (local share), capacity cap_gen
    uint32_t* g_src = nullptr;
    uint32_t* g_tgt = nullptr;
    uint16_t* g_delay = nullptr;
    float* g_weight = nullptr;
    uint64_t n_gen = 0, cap_gen = 0;
    // generation store in fixed-size blocks of physical memory mapped behind
    // reserved virtual ranges (when the device supports it; tunable gen_blocks)
    bool gen_vmm = false;
    void* gen_defer = nullptr;           // during a batch flush: descriptors of work left to the fused launch
    char* gen_va[4] = {nullptr, nullptr, nullptr, nullptr};   // src, tgt, delay, weight
    bool gen_pooled = false;                                   // taken from the device's mapped store
    uint64_t gen_mapped = 0;                                   // connections mapped
    std::vector<std::array<void*, 4>> gen_handles;             // physical blocks (hipMemGenericAllocationHandle_t)

    // results of prepare
    std::map<int32_t, DevArray> arrays;    // by snnc_array_id
    std::map<int32_t, uint64_t> counts;
    uint64_t n_img = 0;
    uint32_t sort_passes = 0, key_bits = 0;

    // timing
    int timing = 0;                      // 0 off, 1 every launch, 2 radix passes only
    const char* sort_tag = nullptr;      // timer prefix of radix sorts outside Prepare (null: "sort")
    struct Pending {
        std::string name;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    std::vector<size_t> open_timers;      // indices into pending of brackets not yet closed
    std::vector<hipEvent_t> event_pool;
    std::map<std::string, KernelTime> ktimes;
    double ms_connect = 0.0, ms_prepare = 0.0;
    hipEvent_t phase_a = nullptr, phase_b = nullptr;

    // device status word for bounded waits (0 = fine)
    uint32_t* d_status = nullptr;
    // radix-sort look-back epoch (never reset, so status tables need no clearing)
    uint32_t sort_epoch = 0;             // per lane
    void* lookback = nullptr;            // per lane
    size_t lookback_bytes = 0;           // per lane
    int sort_variant = 0;                // tile shape of the radix passes (tunable)
    bool mark_in_lds = true;             // regeneration marks bit rows in LDS when they fit (tunable)
    int number_variant = 10;             // tile shape of the image-numbering pass (tunable; 1024 x 10, payload early)
    int sort_mode = 0;                   // 0: onesweep (look-back), 1: reduce-then-scan (tunable)
    bool sort_pinned = false;            // set by hand: the autotuner's process-wide choice is not used
    int digit_bits = 0;                  // 0: 9-bit digits when they save a pass; 8 or 9: forced
    // map policy: image numbering (0 canonical, 1 call order), image sources
    // (0 used, 1 threshold heuristic, 2 all passed), threshold xi
    int numbering = 0, img_sources = 0;
    double xi = 1.0;
    bool force_map_path = false;         // number images before the sort under the default policy
    // GPU memory level 0..3, -1 when not set (then: maps and first-index array
    // in device memory, counts from the first-index array, as level 2)
    int mem_level = -1;

    // pinned staging for host-to-device uploads (no synchronisation per upload)
    StageRing ring;                      // per lane
    // pinned landing area of small device-to-host reads (each read waits for its copy)
    char* dl_pin = nullptr;
    // scan totals read back without a copy: mapped pinned words (main stream,
    // counting stream), written by the scan's last kernel; word 2 is the
    // spike exchange's error word, word 3 spare
    uint64_t* tot_pin = nullptr;
    uint64_t* tot_pin_dev = nullptr;
    // batched admission: where the counting sections write their totals
    // (null: counts are read back at once); mapped pinned words, two per request
    uint64_t* defer_slot = nullptr;
    // batched admission: tile-count scans queued by scan_u32_u64_later and
    // launched together by scan_batch_run (their count arrays owned here until then)
    bool scan_batching = false;
    std::vector<ScanJob> scan_jobs;
    std::vector<void*> scan_owned;
    // small first-occurrence windows queued the same way (launched together,
    // one workgroup each, by scan_batch_run); the job records as bytes
    std::vector<uint8_t> first_jobs;
    uint64_t* defer_pin = nullptr;
    uint64_t* defer_pin_dev = nullptr;
    size_t defer_cap = 0;                // requests the pinned words hold
    size_t dl_pin_bytes = 0;
    // delay tables by distribution (bit patterns of mean, sd, lo)
    std::map<std::array<uint64_t, 3>, std::shared_ptr<const DelayTable>> delay_tables;
    // connect timing: first connect start, prepare entry
    hipEvent_t conn_first = nullptr, conn_last = nullptr;
    bool conn_started = false;

    // admission: bytes of the resident network (14 B per connection plus call
    // metadata) may not exceed this (0: no limit)
    uint64_t resident_budget = 0;
    uint64_t resident_bytes = 0;
    // served mode: admitted calls waiting for a flush, and the batches
    std::vector<uint32_t> queued;
    std::vector<hipEvent_t> batch_done;
    bool fuse_batches = true;
    int fused_wgs_per_cu = 8;
    uint32_t floyd_wave_max = 1024;      // Floyd's sampling: one-wave workgroups up to this padded degree
    uint64_t total_small_max = 8192;      // first occurrences, counts and scan in one workgroup up to this window
    uint64_t total_hash_max = 1ull << 28;  // first occurrences by filtered hashing up to this candidate window, else by sorting
    bool bern_masks = true;              // Bernoulli: the counting pass keeps item masks for the writing pass
    size_t fused_cap = 0;
    void* fused_reqs = nullptr;
    void* fused_hdr = nullptr;
    hipGraphExec_t fused_exec = nullptr;
    hipStream_t capture_stream = nullptr;

    // admission counting lane: counts of served requests run on their own
    // stream, so that reading a count back does not wait for queued
    // generation.  The fields above marked per lane (stream, staging,
    // look-back, small-block free lists) belong to the active lane; the
    // other lane's are parked here.
    int lane = 0;                        // 0: caller's stream, 1: counting stream
    hipStream_t main_stream = nullptr, count_stream = nullptr;
    LaneState parked;
    hipEvent_t count_done = nullptr;     // end of the last counting section
    // blocks of the counting lane freed while the caller's stream may still
    // use them: reusable once the fence event recorded after that use completes
    struct Deferred {
        uint64_t seq;
        void* p;
        size_t cls;
    };
    std::deque<Deferred> deferred;
    std::deque<std::pair<uint64_t, hipEvent_t>> fences;
    std::vector<hipEvent_t> fence_pool;
    uint64_t fence_seq = 0;
};

// Runs its scope on the counting lane: swaps the per-lane state, and on exit
// makes the caller's stream wait for everything the scope enqueued.
struct CountScope {
    Ctx& c;
    explicit CountScope(Ctx& ctx);
    ~CountScope();
    CountScope(const CountScope&) = delete;
    CountScope& operator=(const CountScope&) = delete;
};

// allocation through the context (budget-checked); throws on failure
void* dalloc(Ctx& c, size_t bytes);
void dfree(Ctx& c, void* p);
template <class T>
T* dalloc_n(Ctx& c, uint64_t n) {
    return static_cast<T*>(dalloc(c, (size_t)(n ? n : 1) * sizeof(T)));
}

// kernel timing brackets (no-ops unless timing is enabled)
void tstart(Ctx& c, const char* name);
void tstop(Ctx& c);
void resolve_times(Ctx& c);

// upload helpers: the host buffer may be reused as soon as upload returns
// (small copies go through the pinned staging area without a stream sync)
void upload(Ctx& c, void* dst, const void* src, size_t bytes);
void download(Ctx& c, void* dst, const void* src, size_t bytes);
void sync(Ctx& c);

// ------------------------------------------------------------------ entry points of the device code
// Generation of one call (gen.hip).
// gen_local: the call's connections on P_local's share, appended to the
//   context's generation-order arrays (grown once the count is known);
//   returns the number appended.
// gen_mark: regenerate the draws of the call on `host`'s share and set, in
//   the bit row `bits` (over P_local's neurons), the bit of every source that
//   lives on P_local (point-to-point send lists).
uint64_t gen_local(Ctx& c, Call& cl);
void gen_mark(Ctx& c, Call& cl, uint32_t host, uint32_t* bits);
// frees what the admission count kept with a call
void release_pre(Ctx& c, Call& cl);
// number of tile shapes of the image-numbering pass
int number_variant_count();
bool count_on_device(const Ctx& c, const Call& cl);
// device copies of a call's sets and tables (cl.meta), once
void upload_meta(Ctx& c, Call& cl);
// exact number of connections the call has on P_local's share (may launch a
// counting pass)
uint64_t gen_count_local(Ctx& c, Call& cl);
// generate the admitted calls `ids` at their reserved positions as one batch
void flush_batch(Ctx& c, const std::vector<uint32_t>& ids, hipEvent_t done);
// served mode: flush whatever is pending (no-op if nothing is)
void flush_pending(Ctx& c);
// grow the generation-order arrays to hold `need` connections
void grow_gen(Ctx& c, uint64_t need);
// hands the generation block store back after the caller has waited for every
// kernel that uses it (kept mapped for the next context on the device)
void gen_release(Ctx& c);
// workgroups per compute unit that the fused-launch autotuner chose for the
// device in this process (0: not tuned)
int fused_grid_tuned(int device);
bool gen_blocks_supported(int device);

// host-side helpers shared by the planner files
std::vector<TChunk> target_chunks(const Call& cl, uint32_t host, uint64_t K, uint64_t max_elems);
bool set_lookup_host(const HostSet& s, uint64_t ord, uint32_t& host, uint32_t& local);

// device-wide scans (scan.hip)
// out[i] = sum_{k<i} in[i] for i <= n (out has n + 1 entries); returns total
// after synchronising when want_total.
uint64_t scan_u32_u64(Ctx& c, const uint32_t* in, uint64_t* out, uint64_t n, bool want_total);
// the same without a wait: the total is written to total_dev (a mapped host word)
void scan_u32_u64_to(Ctx& c, const uint32_t* in, uint64_t* out, uint64_t n, uint64_t* total_dev);
// scan_u32_u64_to, queued while c.scan_batching is set (and n is at most
// SCAN_BATCH_MAX); takes ownership of `in` (freed once the scan has been enqueued)
constexpr uint64_t SCAN_BATCH_MAX = 1u << 16;
void scan_u32_u64_later(Ctx& c, uint32_t* in, uint64_t* out, uint64_t n, uint64_t* total_dev);
// launches every queued scan in one kernel on the active lane and frees their inputs
void scan_batch_run(Ctx& c);
// launches the queued small first-occurrence windows (part of scan_batch_run)
void first_small_batch_run(Ctx& c);
// the same over popcounts of 32-bit words
uint64_t scan_popc_u64(Ctx& c, const uint32_t* words, uint64_t* out, uint64_t n_words, bool want_total);
uint64_t scan_u64_u64(Ctx& c, const uint64_t* in, uint64_t* out, uint64_t n, bool want_total);

// stable LSD radix sort on bits [bit_lo, bit_hi) of 64-bit keys with a
// 32-bit payload (sort.hip).  Ping-pong buffers are supplied by the caller;
// returns 0 if the result is in (keys0, vals0), 1 if in (keys1, vals1).
// When `final_out` is set, the last pass writes the unpacked connection
// arrays instead (see sort.hip).
struct FinalOut {
    int32_t* src;
    int32_t* tgt;
    uint16_t* delay;
    float* weight;
    uint32_t tgt_shift;   // key = src << tgt_shift | tgt << 16 | delay
    uint64_t tgt_mask;
};
// wait_for_plan: read the digit histograms back to skip passes whose digit is
// the same for every key (a wait on the stream); false runs every pass
// without waiting (the result is the same: such a pass keeps the order).
// takes the device address of the allocation-free sort's static scratch
// (once per device; called by snnc_init with the context's device current)
void noalloc_setup(Ctx& c);
int radix_sort(Ctx& c, uint64_t* keys0, uint32_t* vals0, uint64_t* keys1, uint32_t* vals1, uint64_t n,
               uint32_t bit_lo, uint32_t bit_hi, const uint64_t* digit_hist /* may be null */,
               const FinalOut* final_out, bool wait_for_plan = true);
// digit histograms for all passes of a sort (radix 256, D bits per pass)
// digit histograms: entries per pass (buckets of digits up to 9 bits)
constexpr int HIST_STRIDE = 512;
// Digits of radix pass p over bits [bit_lo, bit_hi): the first n9 passes take
// 9 bits, the others dbits; the last pass ends at bit_hi.
__host__ __device__ inline uint32_t pass_shift(uint32_t bit_lo, uint32_t n9, uint32_t dbits, uint32_t p) {
    const uint32_t a = p < n9 ? p : n9;
    return bit_lo + 9 * a + dbits * (p - a);
}
__host__ __device__ inline uint32_t pass_bits(uint32_t bit_lo, uint32_t bit_hi, uint32_t n9, uint32_t dbits,
                                              uint32_t p) {
    const uint32_t s = pass_shift(bit_lo, n9, dbits, p);
    const uint32_t w = p < n9 ? 9u : dbits;
    return bit_hi - s < w ? bit_hi - s : w;
}

struct SortPlan {
    int mode = 0, variant = 0;
    uint32_t passes = 0, dbits = 0;
    uint32_t n9 = 0;     // leading passes with 9-bit digits
    bool wide = false;   // some pass has 9-bit digits
};
SortPlan plan_sort(const Ctx& c, uint64_t n, uint32_t bits);
// 64 geometric-gap thresholds of a Bernoulli(p) sequence (pairwise Bernoulli rule)
int sort_variant_count();

// prepare pipeline (prepare.hip)
void prepare_all(Ctx& c);
void init_ring(StageRing& r, size_t bytes);
void free_ring(StageRing& r);
void free_array(Ctx& c, DevArray& a);

}  // namespace snnc

// The opaque handle of the C ABI is the context itself.
struct snnc_ctx : public snnc::Ctx {};
