// Caching device allocator behind DevBuf.
//
// Blocks are rounded up to 1/8-octave size classes (at least 4 KiB) and kept
// per device in free lists keyed by their rounded size.  A freed block first
// goes to the freeing thread's pending list: the library only knows that the
// block is idle once the device has been synchronised, so pending blocks are
// moved to the free lists by pool_device_idle(), which the library calls right
// after hipDeviceSynchronize().  A thread that ends hands its pending blocks
// to a shared list that the next pool_device_idle() promotes as well.  When
// hipMalloc fails, the cached free blocks are released and the allocation is
// retried once.
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "common.h"

namespace mbamg {
namespace {

struct Block {
    int dev;
    size_t bytes;
    void* p;
};

struct Pool {
    std::mutex m;
    std::unordered_map<int, std::multimap<size_t, void*>> free_lists;   // device -> (size class -> block)
};

Pool& pool() {
    static Pool* p = new Pool;   // never destroyed: blocks may be freed during process teardown
    return *p;
}

// blocks freed by threads that have ended, promoted by the next idle point
std::vector<Block>& orphans() {
    static auto* v = new std::vector<Block>;   // guarded by pool().m
    return *v;
}
struct Pending {
    std::vector<Block> v;
    ~Pending() {
        if (v.empty()) return;
        std::lock_guard<std::mutex> g(pool().m);
        orphans().insert(orphans().end(), v.begin(), v.end());
    }
};
thread_local Pending t_pending;

size_t size_class(size_t b) {
    if (b <= 4096) return 4096;
    int e = 63 - __builtin_clzll((unsigned long long)b);
    size_t step = (size_t)1 << (e > 3 ? e - 3 : 0);
    if (step < 4096) step = 4096;
    return (b + step - 1) / step * step;
}

int current_device() {
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess) {
        (void)hipGetLastError();
        d = 0;
    }
    return d;
}

void release_cached(int dev) {
    std::multimap<size_t, void*> drop;
    {
        std::lock_guard<std::mutex> g(pool().m);
        drop.swap(pool().free_lists[dev]);
    }
    for (auto& kv : drop) (void)hipFree(kv.second);
}

}  // namespace

void* dev_alloc(size_t bytes) {
    const size_t r = size_class(bytes);
    const int dev = current_device();
    {
        std::lock_guard<std::mutex> g(pool().m);
        auto& fl = pool().free_lists[dev];
        auto it = fl.find(r);
        if (it != fl.end()) {
            void* p = it->second;
            fl.erase(it);
            return p;
        }
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, r);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        release_cached(dev);
        e = hipMalloc(&p, r);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw Error(MBAMG_E_NOMEM, "hipMalloc of " + std::to_string(r) + " bytes failed");
        }
    }
    return p;
}

void dev_free(void* p, size_t bytes) {
    if (!p) return;
    t_pending.v.push_back({current_device(), size_class(bytes), p});
}

// the current device has been synchronised: its pending blocks are idle
namespace {
struct PinnedPool {
    std::mutex m;
    std::vector<std::pair<void*, size_t>> free_list;   // buffers not handed out
    std::unordered_map<void*, size_t> taken;
    size_t total = 0;                                    // bytes held, free or taken
};
// above this many pinned bytes, idle buffers are released before a new one is made
constexpr size_t PINNED_POOL_CAP = (size_t)1 << 30;
PinnedPool& pinned_pool() {
    static PinnedPool* pool = new PinnedPool();   // never destroyed: its buffers live as long as the process
    return *pool;
}
}  // namespace

void* pinned_take(size_t bytes) {
    PinnedPool& P = pinned_pool();
    {
        std::lock_guard<std::mutex> g(P.m);
        size_t best = P.free_list.size();
        for (size_t k = 0; k < P.free_list.size(); ++k)
            if (P.free_list[k].second >= bytes &&
                (best == P.free_list.size() || P.free_list[k].second < P.free_list[best].second))
                best = k;
        if (best < P.free_list.size()) {
            const auto e = P.free_list[best];
            P.free_list.erase(P.free_list.begin() + (std::ptrdiff_t)best);
            P.taken[e.first] = e.second;
            return e.first;
        }
    }
    std::vector<std::pair<void*, size_t>> drop;
    {
        std::lock_guard<std::mutex> g(P.m);
        if (P.total + bytes > PINNED_POOL_CAP) {
            drop.swap(P.free_list);
            for (const auto& e : drop) P.total -= e.second;
        }
    }
    for (const auto& e : drop) (void)hipHostFree(e.first);
    void* p = nullptr;
    MB_HIP(hipHostMalloc(&p, bytes, hipHostMallocDefault));
    std::lock_guard<std::mutex> g(P.m);
    P.taken[p] = bytes;
    P.total += bytes;
    return p;
}

void pinned_give(void* p) {
    if (!p) return;
    PinnedPool& P = pinned_pool();
    std::lock_guard<std::mutex> g(P.m);
    const auto it = P.taken.find(p);
    if (it == P.taken.end()) return;
    P.free_list.emplace_back(p, it->second);
    P.taken.erase(it);
}

void pool_device_idle() {
    const int dev = current_device();
    std::lock_guard<std::mutex> g(pool().m);
    auto promote = [dev](std::vector<Block>& list) {
        size_t keep = 0;
        for (const Block& b : list) {
            if (b.dev == dev) pool().free_lists[dev].emplace(b.bytes, b.p);
            else list[keep++] = b;
        }
        list.resize(keep);
    };
    promote(t_pending.v);
    promote(orphans());
}

}  // namespace mbamg
