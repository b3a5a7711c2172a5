// Internal helpers shared by the libmbamg translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <cstring>
#include <vector>

#include "../../include/mbamg.h"

namespace mbamg {

// Error carried from deep inside the host code to the C-ABI boundary.
struct Error : std::runtime_error {
    mbamg_status code;
    Error(mbamg_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define MB_HIP(call)                                                                    \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            throw ::mbamg::Error(MBAMG_E_HIP, std::string(#call) + ": " +               \
                                                  hipGetErrorString(e_) + " at " +      \
                                                  __FILE__ + ":" + std::to_string(__LINE__)); \
    } while (0)

#define MB_CHECK(cond, code, msg)                                  \
    do {                                                           \
        if (!(cond)) throw ::mbamg::Error((code), (msg));          \
    } while (0)

#define MB_LAUNCH_CHECK() MB_HIP(hipGetLastError())

constexpr int WAVE = 64;

// Device memory comes from a process-wide cache (memory.hip): a freed block
// is parked as pending in a per-thread list and becomes reusable only at a
// point where the caller has made the whole device idle (pool_device_idle),
// so a block is never handed out while a kernel may still use it.  Cached
// blocks stay mapped, which keeps the large allocations of repeated setups
// off the driver's map/unmap path.
void* dev_alloc(size_t bytes);
void dev_free(void* p, size_t bytes);
// Call right after hipDeviceSynchronize(): this thread's pending blocks become reusable.
void pool_device_idle();

// Page-locked host memory from a process-wide pool (memory.hip): a copy to or
// from pageable memory is staged by the runtime and ran at 1.6-2.6 GB/s here.
// Buffers are kept for the life of the process; a taken buffer is the
// caller's until it is given back.
void* pinned_take(size_t bytes);
void pinned_give(void* p);

template <class T>
struct PinnedBuf {
    T* p = nullptr;
    explicit PinnedBuf(size_t count) : p((T*)pinned_take((count ? count : 1) * sizeof(T))) {}
    ~PinnedBuf() { pinned_give(p); }
    PinnedBuf(const PinnedBuf&) = delete;
    PinnedBuf& operator=(const PinnedBuf&) = delete;
};

// transfers of at least this many bytes go through a page-locked buffer
constexpr size_t PINNED_STAGING_MIN = (size_t)1 << 20;

// Owning device buffer.
template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    explicit DevBuf(size_t count) { alloc(count); }
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t count) {
        release();
        if (count) {
            p = static_cast<T*>(dev_alloc(count * sizeof(T)));
            n = count;
        }
    }
    void release() {
        if (p) dev_free(p, n * sizeof(T));
        p = nullptr;
        n = 0;
    }
    size_t bytes() const { return n * sizeof(T); }
    // Synchronous with respect to the host buffer, which may be released on return.
    void upload(const T* h, size_t count, hipStream_t s) {
        if (count > n) alloc(count);
        if (!count) return;
        const size_t bytes = count * sizeof(T);
        if (bytes < PINNED_STAGING_MIN) {
            MB_HIP(hipMemcpyAsync(p, h, bytes, hipMemcpyHostToDevice, s));
            MB_HIP(hipStreamSynchronize(s));
            return;
        }
        PinnedBuf<T> st(count);
        std::copy(h, h + count, st.p);
        MB_HIP(hipMemcpyAsync(p, st.p, bytes, hipMemcpyHostToDevice, s));
        MB_HIP(hipStreamSynchronize(s));   // the staging buffer goes back to the pool
    }
    void upload(const std::vector<T>& v, hipStream_t s) { upload(v.data(), v.size(), s); }
    std::vector<T> download(hipStream_t s, size_t count = SIZE_MAX) const {
        size_t c = count == SIZE_MAX ? n : count;
        std::vector<T> h(c);
        if (!c) return h;
        const size_t bytes = c * sizeof(T);
        if (bytes < PINNED_STAGING_MIN) {
            MB_HIP(hipMemcpyAsync(h.data(), p, bytes, hipMemcpyDeviceToHost, s));
            MB_HIP(hipStreamSynchronize(s));
            return h;
        }
        PinnedBuf<T> st(c);
        MB_HIP(hipMemcpyAsync(st.p, p, bytes, hipMemcpyDeviceToHost, s));
        MB_HIP(hipStreamSynchronize(s));
        std::copy(st.p, st.p + c, h.data());
        return h;
    }
};
// Several device arrays copied to host vectors through one page-locked buffer
// with one synchronisation of the stream.
struct HostCopies {
    struct Item {
        const void* src;
        void* dst;
        size_t bytes;
    };
    std::vector<Item> items;
    template <class T>
    void add(const DevBuf<T>& b, std::vector<T>& out, size_t count) {
        out.resize(count);
        if (count) items.push_back({b.p, out.data(), count * sizeof(T)});
    }
    void run(hipStream_t s) {
        size_t total = 0;
        for (const Item& it : items) total += (it.bytes + 15) & ~(size_t)15;
        if (!total) return;
        PinnedBuf<char> st(total);
        size_t off = 0;
        for (const Item& it : items) {
            MB_HIP(hipMemcpyAsync(st.p + off, it.src, it.bytes, hipMemcpyDeviceToHost, s));
            off += (it.bytes + 15) & ~(size_t)15;
        }
        MB_HIP(hipStreamSynchronize(s));
        off = 0;
        for (const Item& it : items) {
            std::memcpy(it.dst, st.p + off, it.bytes);
            off += (it.bytes + 15) & ~(size_t)15;
        }
        items.clear();
    }
};


inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace mbamg
