// Device-wide exclusive scans (reduce, scan of the block sums, scan): used
// for per-tile counts, popcounts of bit sets and first-index arrays.
#include <algorithm>

#include "device_common.h"
#include "internal.h"

namespace snnc {

namespace {

constexpr int SNT = 256;
constexpr int SIPT = 16;
constexpr uint64_t STILE = SNT * SIPT;

struct LoadU32 {
    const uint32_t* p;
    __device__ __forceinline__ uint64_t operator()(uint64_t i) const { return p[i]; }
};
struct LoadPopc {
    const uint32_t* p;
    __device__ __forceinline__ uint64_t operator()(uint64_t i) const { return (uint64_t)__popc(p[i]); }
};
struct LoadU64 {
    const uint64_t* p;
    __device__ __forceinline__ uint64_t operator()(uint64_t i) const { return p[i]; }
};

template <class L>
__global__ __launch_bounds__(SNT) void k_reduce(L load, uint64_t n, uint64_t* partial) {
    __shared__ uint64_t scratch[SNT / 64];
    const uint64_t base = (uint64_t)blockIdx.x * STILE;
    uint64_t s = 0;
#pragma unroll 4
    for (int k = 0; k < SIPT; ++k) {
        const uint64_t i = base + (uint64_t)k * SNT + threadIdx.x;
        if (i < n) s += load(i);
    }
    uint64_t tot;
    block_excl_scan<SNT, uint64_t>(s, scratch, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// Each thread owns SIPT consecutive elements; out[n] receives the total (and
// *total_out, when given: a mapped host word the caller reads after a sync).
template <class L>
__global__ __launch_bounds__(SNT) void k_scan(L load, uint64_t n, const uint64_t* block_off, uint64_t* out,
                                              uint64_t* total_out) {
    __shared__ uint64_t scratch[SNT / 64];
    const uint64_t base = (uint64_t)blockIdx.x * STILE + (uint64_t)threadIdx.x * SIPT;
    uint64_t v[SIPT];
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < SIPT; ++k) {
        const uint64_t i = base + k;
        v[k] = i < n ? load(i) : 0;
        s += v[k];
    }
    uint64_t tot;
    uint64_t run = block_excl_scan<SNT, uint64_t>(s, scratch, &tot) + (block_off ? block_off[blockIdx.x] : 0);
#pragma unroll
    for (int k = 0; k < SIPT; ++k) {
        const uint64_t i = base + k;
        if (i < n) out[i] = run;
        run += v[k];
        if (i + 1 == n) {
            out[n] = run;
            if (total_out) *total_out = run;
        }
    }
}

// the total of an empty scan: out[0] and the caller's word are zero
__global__ void k_put_u64(uint64_t* out, uint64_t* total_out) {
    out[0] = 0;
    *total_out = 0;
}

template <class L>
void scan_impl(Ctx& c, L load, uint64_t n, uint64_t* out, uint64_t* total_out = nullptr) {
    const uint64_t nb = (n + STILE - 1) / STILE;
    if (nb <= 1) {
        tstart(c, "scan");
        hipLaunchKernelGGL(k_scan<L>, dim3(1), dim3(SNT), 0, c.stream, load, n, (const uint64_t*)nullptr, out,
                           total_out);
        tstop(c);
        HIPCHK(hipGetLastError());
        return;
    }
    uint64_t* partial = dalloc_n<uint64_t>(c, nb);
    uint64_t* off = nullptr;
    try {
        off = dalloc_n<uint64_t>(c, nb + 1);
        tstart(c, "scan");
        hipLaunchKernelGGL(k_reduce<L>, dim3((unsigned)nb), dim3(SNT), 0, c.stream, load, n, partial);
        tstop(c);
        HIPCHK(hipGetLastError());
        scan_impl(c, LoadU64{partial}, nb, off);
        tstart(c, "scan");
        hipLaunchKernelGGL(k_scan<L>, dim3((unsigned)nb), dim3(SNT), 0, c.stream, load, n, (const uint64_t*)off, out,
                           total_out);
        tstop(c);
        HIPCHK(hipGetLastError());
    } catch (...) {
        dfree(c, partial);
        dfree(c, off);
        throw;
    }
    // released in stream order: only later work on the stream can reuse them
    dfree(c, partial);
    dfree(c, off);
}

template <class L>
uint64_t scan_any(Ctx& c, L load, uint64_t* out, uint64_t n, bool want_total) {
    if (n == 0) {
        HIPCHK(hipMemsetAsync(out, 0, 8, c.stream));
        if (want_total) sync(c);
        return 0;
    }
    if (!want_total || !c.tot_pin) {
        scan_impl(c, load, n, out);
        uint64_t total = 0;
        if (want_total) download(c, &total, out + n, 8);
        return total;
    }
    // the total lands in mapped host memory: no copy between the scan and the read
    const int slot = c.stream == c.count_stream ? 1 : 0;
    scan_impl(c, load, n, out, c.tot_pin_dev + slot);
    sync(c);
    return *reinterpret_cast<volatile uint64_t*>(c.tot_pin + slot);
}

// One workgroup per queued scan: chunks of STILE counts in order, the running
// total carried from chunk to chunk.
__global__ __launch_bounds__(SNT) void k_multi_scan(const ScanJob* jobs) {
    __shared__ uint64_t scratch[SNT / 64];
    const ScanJob j = jobs[blockIdx.x];
    uint64_t carry = 0;
    for (uint64_t base = 0; base < j.n; base += STILE) {
        const uint64_t first = base + (uint64_t)threadIdx.x * SIPT;
        uint64_t v[SIPT];
        uint64_t sum = 0;
#pragma unroll
        for (int k = 0; k < SIPT; ++k) {
            v[k] = first + k < j.n ? j.in[first + k] : 0;
            sum += v[k];
        }
        uint64_t tot;
        uint64_t run = carry + block_excl_scan<SNT, uint64_t>(sum, scratch, &tot);
#pragma unroll
        for (int k = 0; k < SIPT; ++k) {
            if (first + k < j.n) j.out[first + k] = run;
            run += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) {
        j.out[j.n] = carry;
        if (j.total_out) *j.total_out = carry;
    }
}

}  // namespace

void scan_u32_u64_later(Ctx& c, uint32_t* in, uint64_t* out, uint64_t n, uint64_t* total_dev) {
    if (!c.scan_batching || n > SCAN_BATCH_MAX) {
        scan_u32_u64_to(c, in, out, n, total_dev);
        dfree(c, in);   // in stream order: only later work reuses it
        return;
    }
    c.scan_jobs.push_back(ScanJob{in, out, total_dev, n});
    c.scan_owned.push_back(in);
}

void scan_batch_run(Ctx& c) {
    first_small_batch_run(c);
    if (!c.scan_jobs.empty()) {
        const size_t bytes = c.scan_jobs.size() * sizeof(ScanJob);
        ScanJob* dev = static_cast<ScanJob*>(dalloc(c, bytes));
        upload(c, dev, c.scan_jobs.data(), bytes);
        tstart(c, "scan");
        hipLaunchKernelGGL(k_multi_scan, dim3((unsigned)c.scan_jobs.size()), dim3(SNT), 0, c.stream,
                           (const ScanJob*)dev);
        tstop(c);
        const hipError_t e = hipGetLastError();
        dfree(c, dev);
        HIPCHK(e);
    }
    for (void* p : c.scan_owned) dfree(c, p);
    c.scan_jobs.clear();
    c.scan_owned.clear();
}

uint64_t scan_u32_u64(Ctx& c, const uint32_t* in, uint64_t* out, uint64_t n, bool want_total) {
    return scan_any(c, LoadU32{in}, out, n, want_total);
}

void scan_u32_u64_to(Ctx& c, const uint32_t* in, uint64_t* out, uint64_t n, uint64_t* total_dev) {
    if (n == 0) {
        hipLaunchKernelGGL(k_put_u64, dim3(1), dim3(1), 0, c.stream, out, total_dev);
        HIPCHK(hipGetLastError());
        return;
    }
    scan_impl(c, LoadU32{in}, n, out, total_dev);
}

uint64_t scan_popc_u64(Ctx& c, const uint32_t* words, uint64_t* out, uint64_t n_words, bool want_total) {
    return scan_any(c, LoadPopc{words}, out, n_words, want_total);
}

uint64_t scan_u64_u64(Ctx& c, const uint64_t* in, uint64_t* out, uint64_t n, bool want_total) {
    return scan_any(c, LoadU64{in}, out, n, want_total);
}

}  // namespace snnc
