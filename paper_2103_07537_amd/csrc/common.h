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
        n = count;
        if (count) {
            hipError_t e = hipMalloc(reinterpret_cast<void**>(&p), count * sizeof(T));
            if (e != hipSuccess) {
                p = nullptr;
                n = 0;
                (void)hipGetLastError();
                throw Error(MBAMG_E_NOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
            }
        }
    }
    void release() {
        if (p) (void)hipFree(p);
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
