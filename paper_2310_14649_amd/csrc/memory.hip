// Device memory of the library's handles: every device buffer the library
// holds comes from device_alloc, which takes it from hipMalloc (default),
// from functions the caller installed (sg_set_allocator), or from a
// caller-owned arena (sg_set_arena, bump allocation, 256-byte aligned).
// Each live allocation remembers where it came from, so a buffer is given
// back to the source it was taken from even if the caller switched sources
// while handles were alive.
#include "common.hpp"

#include <mutex>
#include <unordered_map>

namespace sg {
namespace {

enum class Source { Hip, Hook, Arena };

struct Origin {
    Source src;
    size_t bytes;
    int device;
    sg_device_free_fn release;
    void* ctx;
};

struct MemState {
    std::mutex mu;
    Source mode = Source::Hip;
    sg_device_alloc_fn alloc = nullptr;
    sg_device_free_fn release = nullptr;
    void* ctx = nullptr;
    char* arena = nullptr;
    size_t arena_bytes = 0, arena_used = 0;
    int arena_device = -1;
    int64_t live = 0, peak = 0;
    std::unordered_map<void*, Origin> origin;
};

MemState& mem() {
    static MemState m;
    return m;
}

constexpr size_t kAlign = 256;

}  // namespace

void* device_alloc(size_t bytes) {
    if (bytes == 0) return nullptr;
    MemState& m = mem();
    const int dev = current_device();
    std::lock_guard<std::mutex> lk(m.mu);
    void* p = nullptr;
    Origin o{m.mode, bytes, dev, m.release, m.ctx};
    if (m.mode == Source::Arena) {
        SG_REQUIRE(dev == m.arena_device, "arena set on device %d, allocation on device %d",
                   m.arena_device, dev);
        const size_t need = (bytes + kAlign - 1) & ~(kAlign - 1);
        if (m.arena_used + need > m.arena_bytes)
            SG_THROW(SG_ERR_WORKSPACE, "arena exhausted: %zu bytes requested, %zu of %zu used",
                     bytes, m.arena_used, m.arena_bytes);
        p = m.arena + m.arena_used;
        m.arena_used += need;
    } else if (m.mode == Source::Hook) {
        p = m.alloc(bytes, dev, m.ctx);
        if (!p) SG_THROW(SG_ERR_WORKSPACE, "caller allocator returned no memory for %zu bytes",
                         bytes);
        SG_REQUIRE(reinterpret_cast<uintptr_t>(p) % kAlign == 0,
                   "caller allocator returned a pointer not aligned to %zu bytes", kAlign);
    } else {
        HIP_OK(hipMalloc(&p, bytes));
    }
    m.origin[p] = o;
    m.live += (int64_t)bytes;
    if (m.live > m.peak) m.peak = m.live;
    return p;
}

void device_free(void* p) {
    if (!p) return;
    MemState& m = mem();
    Origin o;
    {
        std::lock_guard<std::mutex> lk(m.mu);
        auto it = m.origin.find(p);
        if (it == m.origin.end()) return;
        o = it->second;
        m.origin.erase(it);
        m.live -= (int64_t)o.bytes;
    }
    if (o.src == Source::Hip) (void)hipFree(p);
    else if (o.src == Source::Hook && o.release) o.release(p, o.bytes, o.device, o.ctx);
    // arena memory goes back only with sg_set_arena / sg_arena_reset
}

}  // namespace sg

using namespace sg;

extern "C" {

int sg_set_allocator(sg_device_alloc_fn alloc, sg_device_free_fn release, void* ctx) {
    return guarded([&]() -> int {
        SG_REQUIRE((alloc == nullptr) == (release == nullptr),
                   "give both allocator functions or neither");
        MemState& m = mem();
        std::lock_guard<std::mutex> lk(m.mu);
        m.mode = alloc ? Source::Hook : Source::Hip;
        m.alloc = alloc;
        m.release = release;
        m.ctx = ctx;
        m.arena = nullptr;
        m.arena_bytes = m.arena_used = 0;
        m.arena_device = -1;
        return SG_OK;
    });
}

int sg_set_arena(void* base, size_t bytes) {
    return guarded([&]() -> int {
        MemState& m = mem();
        if (base == nullptr) {
            std::lock_guard<std::mutex> lk(m.mu);
            if (m.mode == Source::Arena) m.mode = m.alloc ? Source::Hook : Source::Hip;
            m.arena = nullptr;
            m.arena_bytes = m.arena_used = 0;
            m.arena_device = -1;
            return SG_OK;
        }
        SG_REQUIRE(reinterpret_cast<uintptr_t>(base) % kAlign == 0,
                   "arena base must be %zu-byte aligned", kAlign);
        const int dev = current_device();
        std::lock_guard<std::mutex> lk(m.mu);
        m.mode = Source::Arena;
        m.arena = static_cast<char*>(base);
        m.arena_bytes = bytes;
        m.arena_used = 0;
        m.arena_device = dev;
        return SG_OK;
    });
}

int sg_arena_reset(void) {
    return guarded([&]() -> int {
        MemState& m = mem();
        std::lock_guard<std::mutex> lk(m.mu);
        SG_REQUIRE(m.mode == Source::Arena, "no arena is set");
        for (const auto& kv : m.origin)
            SG_REQUIRE(kv.second.src != Source::Arena,
                       "arena still holds live buffers (destroy the handles first)");
        m.arena_used = 0;
        return SG_OK;
    });
}

int sg_memory_stats(int64_t* live_bytes, int64_t* peak_bytes, int64_t* arena_used) {
    return guarded([&]() -> int {
        MemState& m = mem();
        std::lock_guard<std::mutex> lk(m.mu);
        if (live_bytes) *live_bytes = m.live;
        if (peak_bytes) *peak_bytes = m.peak;
        if (arena_used) *arena_used = (int64_t)m.arena_used;
        return SG_OK;
    });
}

int sg_memory_reset_peak(void) {
    MemState& m = mem();
    std::lock_guard<std::mutex> lk(m.mu);
    m.peak = m.live;
    return SG_OK;
}

}  // extern "C"
