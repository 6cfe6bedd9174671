// Internal helpers shared by the libatsne sources (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/atsne.h"

namespace atsne {

// Thread-local error text behind atsne_last_error().
void set_error(const char* fmt, ...) __attribute__((format(printf, 1, 2)));
void clear_error();

#define ATSNE_REQUIRE(cond, code, ...)        \
    do {                                      \
        if (!(cond)) {                        \
            ::atsne::set_error(__VA_ARGS__);  \
            return (code);                    \
        }                                     \
    } while (0)

#define ATSNE_HIP(call)                                                                           \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) {                                                                   \
            ::atsne::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                               __LINE__);                                                         \
            return ATSNE_E_HIP;                                                                   \
        }                                                                                         \
    } while (0)

#define ATSNE_LAUNCH_CHECK()                                                                     \
    do {                                                                                         \
        hipError_t e_ = hipGetLastError();                                                       \
        if (e_ != hipSuccess) {                                                                  \
            ::atsne::set_error("kernel launch failed: %s (%s:%d)", hipGetErrorString(e_),       \
                               __FILE__, __LINE__);                                              \
            return ATSNE_E_HIP;                                                                  \
        }                                                                                        \
    } while (0)

#define ATSNE_TRY(expr)                      \
    do {                                     \
        atsne_status s_ = (expr);            \
        if (s_ != ATSNE_OK) return s_;       \
    } while (0)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Bump allocator over a caller workspace.
struct Arena {
    char* base = nullptr;
    size_t cap = 0, used = 0;
    Arena() = default;
    Arena(void* p, size_t c) : base(static_cast<char*>(p)), cap(c) {}
    template <class T>
    T* take(size_t count) {
        size_t off = align_up(used, 256);
        used = off + align_up(count * sizeof(T), 256);
        return base ? reinterpret_cast<T*>(base + off) : nullptr;
    }
};

// Workspace holder: uses the caller's buffer or a stream-ordered allocation.
struct Scratch {
    void* ptr = nullptr;
    bool owned = false;
    hipStream_t stream = nullptr;
    atsne_status acquire(void* ws, size_t ws_bytes, size_t need, hipStream_t s) {
        stream = s;
        if (ws) {
            if (ws_bytes < need) {
                set_error("workspace too small: %zu bytes given, %zu needed", ws_bytes, need);
                return ATSNE_E_NOMEM;
            }
            ptr = ws;
            return ATSNE_OK;
        }
        if (need == 0) return ATSNE_OK;
        hipError_t e = hipMallocAsync(&ptr, need, s);
        if (e != hipSuccess) {
            set_error("workspace allocation of %zu bytes failed: %s", need, hipGetErrorString(e));
            ptr = nullptr;
            return ATSNE_E_NOMEM;
        }
        owned = true;
        return ATSNE_OK;
    }
    ~Scratch() {
        if (owned && ptr) (void)hipFreeAsync(ptr, stream);
    }
};

// Number of compute units of the current device (cached per device).
int device_cu_count();
// Global memory of the current device in bytes (0 when there is no device).
size_t device_hbm_bytes();

// Optional per-kernel timing: brackets a launch with HIP events on its
// stream while profiling is enabled (atsne_profile_enable).
struct ProfScope {
    int slot = -1;
    hipStream_t stream;
    ProfScope(const char* name, hipStream_t s);
    ~ProfScope() { stop(); }
    void stop();  // records the end event now (idempotent)
};
// While one is alive on this thread, ProfScopes record nothing: a stage
// reported as a whole (the FP8 seeding pass) hides the kernels inside it.
struct ProfQuiet {
    ProfQuiet();
    ~ProfQuiet();
};

}  // namespace atsne
