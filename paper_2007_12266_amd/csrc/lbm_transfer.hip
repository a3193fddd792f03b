// Host <-> device copies of large caller buffers (images, neighbour tables, fields, states).
//
// The caller's host memory is pageable. A copy from pageable memory is staged by the runtime
// through pinned memory with one host thread, which caps it well below what the link carries.
// Here the staging is explicit: two pinned buffers of kChunk bytes, filled (or drained) by up
// to kThreads host threads while the DMA of the other buffer runs. The buffers are allocated
// once per process (pinned with hipHostMalloc) and shared under a mutex, so concurrent callers
// take turns; copies below kDirect bytes go straight to hipMemcpyAsync.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <system_error>
#include <thread>
#include <vector>

#include "lbm_internal.h"

namespace lbm {
namespace {

constexpr size_t kChunk = 32u << 20;
constexpr size_t kDirect = 4u << 20;
constexpr unsigned kThreads = 8;

struct Staging {
    std::mutex mu;
    void* buf[2] = {nullptr, nullptr};
};

Staging& staging() {
    static Staging st;
    return st;
}

hipError_t ensure_buffers(Staging& st) {
    for (void*& b : st.buf)
        if (!b) {
            const hipError_t e = hipHostMalloc(&b, kChunk, hipHostMallocPortable);
            if (e != hipSuccess) {
                b = nullptr;
                return e;
            }
        }
    return hipSuccess;
}

// memcpy on up to kThreads threads, each a contiguous slice.
void copy_threads(void* dst, const void* src, size_t n) {
    const unsigned hw = std::max(1u, std::min(kThreads, std::thread::hardware_concurrency()));
    if (n < (1u << 20) || hw == 1) {
        std::memcpy(dst, src, n);
        return;
    }
    const size_t slice = (n + hw - 1) / hw;
    std::vector<std::thread> pool;
    for (unsigned t = 0; t < hw; ++t) {
        const size_t b = t * slice;
        if (b >= n) break;
        const size_t len = std::min(slice, n - b);
        try {
            pool.emplace_back([=] { std::memcpy((char*)dst + b, (const char*)src + b, len); });
        } catch (const std::system_error&) {
            std::memcpy((char*)dst + b, (const char*)src + b, len);   // no thread: copy here
        }
    }
    for (std::thread& th : pool) th.join();
}

// Two events per call (created on the current device, like the stream's work).
struct Events {
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t err = hipSuccess;
    Events() {
        for (hipEvent_t& e : ev)
            if (err == hipSuccess) err = hipEventCreateWithFlags(&e, hipEventDisableTiming);
    }
    ~Events() {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

// An error return leaves no DMA running on a staging buffer that the next caller would reuse.
hipError_t drained(hipError_t e, hipStream_t s) {
    (void)hipStreamSynchronize(s);
    return e;
}

}  // namespace

hipError_t copy_to_device(void* dst, const void* src, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    if (bytes < kDirect) {
        const hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
        return e != hipSuccess ? e : hipStreamSynchronize(s);
    }
    Staging& st = staging();
    std::lock_guard<std::mutex> lock(st.mu);
    if (hipError_t e = ensure_buffers(st)) return e;
    Events evs;
    if (evs.err != hipSuccess) return evs.err;
    bool pending[2] = {false, false};
    size_t off = 0;
    for (int k = 0; off < bytes; ++k) {
        const int b = k & 1;
        const size_t len = std::min(kChunk, bytes - off);
        if (pending[b])   // the DMA that last read this buffer has finished
            if (hipError_t e = hipEventSynchronize(evs.ev[b])) return drained(e, s);
        copy_threads(st.buf[b], (const char*)src + off, len);
        if (hipError_t e = hipMemcpyAsync((char*)dst + off, st.buf[b], len,
                                          hipMemcpyHostToDevice, s))
            return drained(e, s);
        if (hipError_t e = hipEventRecord(evs.ev[b], s)) return drained(e, s);
        pending[b] = true;
        off += len;
    }
    return hipStreamSynchronize(s);
}

hipError_t copy_to_host(void* dst, const void* src, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    if (bytes < kDirect) {
        const hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s);
        return e != hipSuccess ? e : hipStreamSynchronize(s);
    }
    Staging& st = staging();
    std::lock_guard<std::mutex> lock(st.mu);
    if (hipError_t e = ensure_buffers(st)) return e;
    Events evs;
    if (evs.err != hipSuccess) return evs.err;
    const size_t nchunks = (bytes + kChunk - 1) / kChunk;
    // Chunk k is copied into buffer k % 2 while the host drains chunk k - 1; the host drained
    // chunk k - 2 (same buffer) before chunk k was queued.
    for (size_t k = 0; k <= nchunks; ++k) {
        if (k < nchunks) {
            const size_t off = k * kChunk, len = std::min(kChunk, bytes - off);
            if (hipError_t e = hipMemcpyAsync(st.buf[k & 1], (const char*)src + off, len,
                                              hipMemcpyDeviceToHost, s))
                return drained(e, s);
            if (hipError_t e = hipEventRecord(evs.ev[k & 1], s)) return drained(e, s);
        }
        if (k > 0) {
            const size_t j = k - 1, off = j * kChunk, len = std::min(kChunk, bytes - off);
            if (hipError_t e = hipEventSynchronize(evs.ev[j & 1])) return drained(e, s);
            copy_threads((char*)dst + off, st.buf[j & 1], len);
        }
    }
    return hipStreamSynchronize(s);
}

}  // namespace lbm
