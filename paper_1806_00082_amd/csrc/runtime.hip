// Library runtime: error reporting, version, device tables.
#include <map>
#include <mutex>
#include <tuple>

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
