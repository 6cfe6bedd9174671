// Error reporting, version and device queries of libatsne.
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"

namespace atsne {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = '\0'; }

size_t device_hbm_bytes() {
    static std::mutex mu;
    static std::vector<size_t> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lk(mu);
    if (dev >= (int)cache.size()) cache.resize(dev + 1, 0);
    if (cache[dev] == 0) {
        size_t bytes = 0;
        if (hipDeviceTotalMem(&bytes, dev) != hipSuccess) bytes = 0;
        cache[dev] = bytes;
    }
    return cache[dev];
}

int device_cu_count() {
    static std::mutex mu;
    static std::vector<int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    std::lock_guard<std::mutex> lk(mu);
    if (dev >= (int)cache.size()) cache.resize(dev + 1, 0);
    if (cache[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            n = 256;
        cache[dev] = n;
    }
    return cache[dev];
}

// ---- kernel timing ----
namespace {
struct ProfRec {
    std::string name;
    hipEvent_t a = nullptr, b = nullptr;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;
thread_local int g_prof_quiet = 0;
}  // namespace

ProfQuiet::ProfQuiet() { ++g_prof_quiet; }
ProfQuiet::~ProfQuiet() { --g_prof_quiet; }

ProfScope::ProfScope(const char* name, hipStream_t s) : stream(s) {
    if (g_prof_quiet > 0) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on) return;
    ProfRec r;
    r.name = name;
    if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return;
    if (hipEventRecord(r.a, s) != hipSuccess) return;
    slot = (int)g_prof.size();
    g_prof.push_back(r);
}

void ProfScope::stop() {
    if (slot < 0) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (slot < (int)g_prof.size()) (void)hipEventRecord(g_prof[slot].b, stream);
    slot = -1;
}

}  // namespace atsne

extern "C" atsne_status atsne_profile_enable(int32_t on) {
    using namespace atsne;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto& r : g_prof) {
        if (r.a) (void)hipEventDestroy(r.a);
        if (r.b) (void)hipEventDestroy(r.b);
    }
    g_prof.clear();
    g_prof_on = on != 0;
    return ATSNE_OK;
}

extern "C" atsne_status atsne_profile_read(const char* name, double* total_ms, int64_t* count) {
    using namespace atsne;
    ATSNE_REQUIRE(name && total_ms && count, ATSNE_E_INVALID_ARG, "null argument");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    double tot = 0.0;
    int64_t n = 0;
    const size_t len = strlen(name);
    for (auto& r : g_prof) {
        if (r.name.compare(0, len, name) != 0) continue;
        ATSNE_HIP(hipEventSynchronize(r.b));
        float ms = 0.f;
        ATSNE_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        tot += ms;
        ++n;
    }
    *total_ms = tot;
    *count = n;
    return ATSNE_OK;
}

extern "C" const char* atsne_last_error(void) { return atsne::g_err; }

extern "C" const char* atsne_version(void) { return "atsne-mi355x 0.1 (gfx950)"; }

extern "C" atsne_status atsne_device_info(int32_t* n_cu, int32_t* clock_khz, int32_t* gcn_arch_major) {
    ATSNE_REQUIRE(n_cu && clock_khz && gcn_arch_major, ATSNE_E_INVALID_ARG, "null output pointer");
    int dev = 0;
    ATSNE_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    ATSNE_HIP(hipGetDeviceProperties(&prop, dev));
    *n_cu = prop.multiProcessorCount;
    *clock_khz = prop.clockRate;
    *gcn_arch_major = prop.major;
    return ATSNE_OK;
}
