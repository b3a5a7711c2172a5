// Internal helpers shared by the libmbamg translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
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
        if (count) {
            MB_HIP(hipMemcpyAsync(p, h, count * sizeof(T), hipMemcpyHostToDevice, s));
            MB_HIP(hipStreamSynchronize(s));
        }
    }
    void upload(const std::vector<T>& v, hipStream_t s) { upload(v.data(), v.size(), s); }
    std::vector<T> download(hipStream_t s, size_t count = SIZE_MAX) const {
        size_t c = count == SIZE_MAX ? n : count;
        std::vector<T> h(c);
        if (c) {
            MB_HIP(hipMemcpyAsync(h.data(), p, c * sizeof(T), hipMemcpyDeviceToHost, s));
            MB_HIP(hipStreamSynchronize(s));
        }
        return h;
    }
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace mbamg
