// Library runtime: error reporting, version, device tables.
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "wk_internal.h"
#include "lowp.h"

namespace wk {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

int check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(WK_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    return WK_OK;
}

// S[jj][t] = sin(2 pi (jj+1)(t+1)/n_m) for jj, t < P, zero elsewhere, in the requested form.
__global__ void build_sine_table(void* out, int n_m, int Pk, int Pn, int kind) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)Pk * Pn) return;
    const int P = n_m / 2;
    const int jj = (int)(idx / Pn), t = (int)(idx % Pn);
    double v = 0.0;
    if (jj < P && t < P) v = sin_2pi_ratio((long)(jj + 1) * (t + 1), n_m);
    switch (kind) {
        case 0: reinterpret_cast<double*>(out)[idx] = v; break;
        case 1: reinterpret_cast<uint16_t*>(out)[idx] = bf16_bits(v); break;
        case 2: reinterpret_cast<uint16_t*>(out)[idx] = bf16_bits(v - bf16_value(bf16_bits(v))); break;
        case 3: reinterpret_cast<uint16_t*>(out)[idx] = f16_bits(v); break;
        case 4: reinterpret_cast<uint16_t*>(out)[idx] = f16_bits(v - f16_value(f16_bits(v))); break;
        default: break;
    }
}

const void* sine_table(int n_m, int kind, int Pk, int Pn, hipStream_t stream, int* err) {
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int, int>, void*> cache;
    *err = WK_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        *err = fail(WK_EHIP, "hipGetDevice failed");
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(mu);
    auto key = std::make_tuple(dev, n_m, kind, Pk, Pn);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    const size_t elem = kind == 0 ? sizeof(double) : sizeof(uint16_t);
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, elem * (size_t)Pk * Pn);
    if (e != hipSuccess) {
        *err = fail(WK_EHIP, std::string("sine table hipMalloc: ") + hipGetErrorString(e));
        return nullptr;
    }
    const long n = (long)Pk * Pn;
    hipLaunchKernelGGL(build_sine_table, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                       p, n_m, Pk, Pn, kind);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        *err = fail(WK_EHIP, std::string("sine table build: ") + hipGetErrorString(e));
        return nullptr;
    }
    cache[key] = p;
    return p;
}


// ----------------------------------------------------------------------------- tracing
// Optional per-kernel timing: when enabled, launches wrapped by trace_begin/trace_end are
// bracketed by events (from a pool created at enable time) on the launch stream.
namespace {
struct TraceRec {
    std::string name;
    hipEvent_t a, b;
};
std::mutex g_trace_mu;
bool g_trace_on = false;
std::vector<hipEvent_t> g_pool;
size_t g_pool_next = 0;
std::vector<TraceRec> g_recs;
}  // namespace

int trace_begin(const char* name, hipStream_t s) {
    if (!g_trace_on) return -1;
    std::lock_guard<std::mutex> lock(g_trace_mu);
    if (g_pool_next + 2 > g_pool.size()) return -1;
    TraceRec r{name, g_pool[g_pool_next], g_pool[g_pool_next + 1]};
    g_pool_next += 2;
    (void)hipEventRecord(r.a, s);
    g_recs.push_back(r);
    return (int)g_recs.size() - 1;
}

void trace_end(int h, hipStream_t s) {
    if (h < 0) return;
    std::lock_guard<std::mutex> lock(g_trace_mu);
    (void)hipEventRecord(g_recs[h].b, s);
}

}  // namespace wk

extern "C" int wk_trace_enable(int32_t max_launches) {
    using namespace wk;
    WK_REQUIRE(max_launches > 0, "wk_trace_enable: max_launches must be positive");
    std::lock_guard<std::mutex> lock(g_trace_mu);
    while ((int)g_pool.size() < 2 * max_launches) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return fail(WK_EHIP, "wk_trace_enable: hipEventCreate failed");
        g_pool.push_back(e);
    }
    g_pool_next = 0;
    g_recs.clear();
    g_trace_on = true;
    return WK_OK;
}

extern "C" int wk_trace_disable(void) {
    using namespace wk;
    std::lock_guard<std::mutex> lock(g_trace_mu);
    g_trace_on = false;
    return WK_OK;
}

extern "C" int wk_trace_read(const char* name, double* total_ms, int64_t* count) {
    using namespace wk;
    WK_REQUIRE(name && total_ms && count, "wk_trace_read: NULL argument");
    std::lock_guard<std::mutex> lock(g_trace_mu);
    double t = 0.0;
    int64_t c = 0;
    for (const auto& r : g_recs) {
        if (r.name != name) continue;
        if (hipEventSynchronize(r.b) != hipSuccess) return fail(WK_EHIP, "wk_trace_read: event sync failed");
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
            return fail(WK_EHIP, "wk_trace_read: elapsed time failed");
        t += ms;
        ++c;
    }
    *total_ms = t;
    *count = c;
    return WK_OK;
}

extern "C" int wk_trace_names(char* buf, size_t len) {
    using namespace wk;
    WK_REQUIRE(buf && len > 0, "wk_trace_names: bad buffer");
    std::lock_guard<std::mutex> lock(g_trace_mu);
    std::string all;
    std::map<std::string, int> seen;
    for (const auto& r : g_recs)
        if (!seen.count(r.name)) {
            seen[r.name] = 1;
            all += r.name + "\n";
        }
    std::strncpy(buf, all.c_str(), len - 1);
    buf[len - 1] = 0;
    return WK_OK;
}

namespace wk {
}  // namespace wk

extern "C" {

const char* wk_last_error(void) { return wk::g_last_error.c_str(); }

int wk_version(void) { return WK_VERSION; }

int wk_device_count(void) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return 0;
    return n;
}

}  // extern "C"
