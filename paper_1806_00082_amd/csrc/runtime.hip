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

// Sine tables of eq.(4), kind = format | (part << 3).  Formats: 0 FP64, 1 BF16, 2 BF16
// remainder (v - bf16(v)), 3 FP16, 4 FP16 remainder, 5 FP32.  Parts (a = row, b = column):
//   0: S[a][b] = sin(2 pi (a+1)(b+1) / n_m) for a, b < P = n_m / 2;
//   1: odd-j fold  So[a][b] = sin(2 pi (2a+1)(b+1) / n_m),   a, b < H = floor(P / 2);
//   2: even-j fold Se[a][b] = sin(2 pi (2a+2)(b+1) / n_m),   a, b < H;
//   3, 4: parts 1 and 2 transposed, T[a][b] = fold[b][a].
// Entries outside those ranges are zero (padding of the tiles).
__global__ void build_sine_table(void* out, int n_m, int rows, int cols, int kind) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)rows * cols) return;
    const int P = n_m / 2, H = P / 2;
    const int a = (int)(idx / cols), b = (int)(idx % cols);
    const int fmt = kind & 7, part = kind >> 3;
    double v = 0.0;
    if (part == 0) {
        if (a < P && b < P) v = sin_2pi_ratio((long)(a + 1) * (b + 1), n_m);
    } else {
        const int k = part <= 2 ? a : b, t = part <= 2 ? b : a;
        const int even = (part == 2 || part == 4) ? 1 : 0;
        if (k < H && t < H) v = sin_2pi_ratio((long)(2 * k + 1 + even) * (t + 1), n_m);
    }
    switch (fmt) {
        case 0: reinterpret_cast<double*>(out)[idx] = v; break;
        case 1: reinterpret_cast<uint16_t*>(out)[idx] = bf16_bits(v); break;
        case 2: reinterpret_cast<uint16_t*>(out)[idx] = bf16_bits(v - bf16_value(bf16_bits(v))); break;
        case 3: reinterpret_cast<uint16_t*>(out)[idx] = f16_bits(v); break;
        case 4: reinterpret_cast<uint16_t*>(out)[idx] = f16_bits(v - f16_value(f16_bits(v))); break;
        case 5: reinterpret_cast<float*>(out)[idx] = (float)v; break;
        default: break;
    }
}

namespace {
std::mutex g_sine_mu;
std::map<std::tuple<int, int, int, int, int>, void*> g_sine;

size_t sine_elem(int kind) {
    const int fmt = kind & 7;
    return fmt == 0 ? sizeof(double) : (fmt == 5 ? sizeof(float) : sizeof(uint16_t));
}
}  // namespace

int sine_table_build(int n_m, int kind, int rows, int cols, hipStream_t stream) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(WK_EHIP, "hipGetDevice failed");
    std::lock_guard<std::mutex> lock(g_sine_mu);
    auto key = std::make_tuple(dev, n_m, kind, rows, cols);
    if (g_sine.count(key)) return WK_OK;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, sine_elem(kind) * (size_t)rows * cols);
    if (e != hipSuccess) return fail(WK_EHIP, std::string("wk_prepare: hipMalloc: ") + hipGetErrorString(e));
    const long n = (long)rows * cols;
    hipLaunchKernelGGL(build_sine_table, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                       p, n_m, rows, cols, kind);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        (void)hipFree(p);
        return fail(WK_EHIP, std::string("wk_prepare: sine table build: ") + hipGetErrorString(e));
    }
    g_sine[key] = p;
    return WK_OK;
}

const void* sine_table(int n_m, int kind, int rows, int cols, int* err) {
    *err = WK_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        *err = fail(WK_EHIP, "hipGetDevice failed");
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_sine_mu);
    auto it = g_sine.find(std::make_tuple(dev, n_m, kind, rows, cols));
    if (it != g_sine.end()) return it->second;
    *err = fail(WK_EINVAL, "sine tables for n_m = " + std::to_string(n_m) +
                               " are not prepared on this device: call wk_prepare first");
    return nullptr;
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
