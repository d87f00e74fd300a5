// Internal helpers of libwigner (gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/wigner.h"

namespace wk {

// ----------------------------------------------------------------------------- errors
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

#define WK_REQUIRE(cond, msg)                                \
    do {                                                     \
        if (!(cond)) return ::wk::fail(WK_EINVAL, (msg));    \
    } while (0)

#define WK_HIP(call)                                                                    \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return ::wk::fail(WK_EHIP, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

// Checks the launch that was just enqueued.
int check_launch(const char* what);

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Optional per-kernel timing (wk_trace_enable): bracket a launch with events on its stream.
int trace_begin(const char* name, hipStream_t s);
void trace_end(int handle, hipStream_t s);

#define WK_LAUNCH(NAME, KERNEL, GRID, BLOCK, SHMEM, STREAM, ...)                          \
    do {                                                                                 \
        const int th_ = ::wk::trace_begin(NAME, STREAM);                                 \
        hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM, __VA_ARGS__);             \
        ::wk::trace_end(th_, STREAM);                                                    \
    } while (0)

// Device sine tables for n_m, [rows][cols] arrays with zero padding, one per device, kind and
// shape.  kind = format | (part << 3); format 0: double, 1: bf16 hi, 2: bf16 lo, 3: fp16 hi,
// 4: fp16 lo (hi/lo of the double), 5: float; part 0: the plain table
// S[jj][t] = sin(2 pi (jj+1)(t+1) / n_m), jj, t < P; parts 1 / 2: the odd-j / even-j fold
// So[k][t] = sin(2 pi (2k+1)(t+1) / n_m), Se[k][t] = sin(2 pi (2k+2)(t+1) / n_m),
// k, t < floor(P / 2); parts 3 / 4: those two transposed.
// sine_table_build allocates, fills and synchronises (set-up only: wk_prepare);
// sine_table only looks a built table up and fails with WK_EINVAL when it is absent.
enum { SINE_PLAIN = 0, SINE_ODD = 1 << 3, SINE_EVEN = 2 << 3, SINE_ODD_T = 3 << 3, SINE_EVEN_T = 4 << 3 };
enum { SINE_F64 = 0, SINE_F32 = 5 };
int sine_table_build(int n_m, int kind, int rows, int cols, hipStream_t stream);
const void* sine_table(int n_m, int kind, int rows, int cols, int* err);

// ----------------------------------------------------------------------------- device utils
__device__ __forceinline__ long mod_pos(long a, long n) {
    long r = a % n;
    return r < 0 ? r + n : r;
}

// sin(2 pi k / n) after an exact integer reduction to the first quarter period, so that
// zeros (k = 0, n/2) and oddness are exact.
__device__ __forceinline__ double sin_2pi_ratio(long k, long n) {
    long t = mod_pos(k, n);
    if (t == 0 || 2 * t == n) return 0.0;
    double sg = 1.0;
    if (2 * t > n) {
        t = n - t;
        sg = -1.0;
    }
    if (4 * t > n) return sg * sinpi((double)(n - 2 * t) / (double)n);  // sin(pi - a) = sin a
    return sg * sinpi(2.0 * (double)t / (double)n);
}

// cos(2 pi k / n) = sin(2 pi (k + n/4) / n) for n divisible by 4, else through cospi.
__device__ __forceinline__ double cos_2pi_ratio(long k, long n) {
    if ((n & 3) == 0) return sin_2pi_ratio(k + n / 4, n);
    return cospi(2.0 * (double)mod_pos(k, n) / (double)n);
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, multipliers
// 0xD2511F53 / 0xCD9E8D57, round keys bumped by 0x9E3779B9 / 0xBB67AE85.
struct u32x4 {
    uint32_t v[4];
};

__device__ __forceinline__ u32x4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint64_t seed) {
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // full 32 x 32 -> 64-bit products: one v_mad_u64_u32 each instead of mul_lo + mul_hi
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    u32x4 o;
    o.v[0] = c0;
    o.v[1] = c1;
    o.v[2] = c2;
    o.v[3] = c3;
    return o;
}

enum : uint32_t { TAG_CREATE = 1, TAG_ANNIH = 2, TAG_INIT = 3 };

// Fraction bits fb such that cell + k 2^-fb is exact in the position type for any cell
// index < n_max.
inline int frac_bits_host(int n_max, int pos_f64) {
    int k = 0;
    while ((1L << k) < (long)n_max) ++k;
    int fb = (pos_f64 ? 53 : 24) - k;
    return fb > 32 ? 32 : fb;
}

// Wave-level inclusive scan of an int (64 lanes, all active): a Hillis-Steele scan inside each
// row of 16 lanes by DPP row shifts (VALU moves; a shuffle is an LDS permute with its round
// trip), then each row adds the totals of the rows below it, read from lanes 15, 31 and 47.
// Lanes whose row-shift source lies outside their row add 0 (the `old` operand).
__device__ __forceinline__ int wave_incl_scan(int v) {
    constexpr int ROW_SHR = 0x110;  // DPP control row_shr:n is ROW_SHR + n
    v += __builtin_amdgcn_update_dpp(0, v, ROW_SHR + 1, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, ROW_SHR + 2, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, ROW_SHR + 4, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, ROW_SHR + 8, 0xf, 0xf, false);
    const int row = (threadIdx.x & 63) >> 4;
    const int t0 = __builtin_amdgcn_readlane(v, 15), t1 = __builtin_amdgcn_readlane(v, 31),
              t2 = __builtin_amdgcn_readlane(v, 47);
    return v + (row > 0 ? t0 : 0) + (row > 1 ? t1 : 0) + (row > 2 ? t2 : 0);
}

__device__ __forceinline__ long long wave_sum_ll(long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block-wide exclusive scan of one int per thread (blockDim.x = 256); returns the
// exclusive prefix and writes the block total to *total.  Uses 4+1 ints of LDS.
__device__ __forceinline__ int block_excl_scan_256(int v, int* total, int* lds5) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int inc = wave_incl_scan(v);
    if (lane == 63) lds5[w] = inc;
    __syncthreads();
    int base = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (k < w) base += lds5[k];
    const int tot = lds5[0] + lds5[1] + lds5[2] + lds5[3];
    __syncthreads();
    *total = tot;
    return base + inc - v;
}

// ----------------------------------------------------------------------------- fused tables
// Creation tables written straight from the kernel rows (the TAB forms of the kernel passes).
struct TabOut {
    double dt;
    double* gamma;
    uint32_t* n0;
    uint32_t* thr;
    uint64_t* cdf;
    uint32_t* guide;  // NULL: no guide table
    int G;            // guide buckets
};

constexpr int TAB_GMAX = 256;  // guide buckets the fused epilogue supports

// Creation tables of one 2-D row (W entries, t = (my + P) n_m + (mx + P)) staged in LDS at Kr
// by the whole workgroup: the arithmetic of the table kernels.  Ascending positive sums by one
// thread (the order is the definition), then every thread converts its entries; the guide by
// binary search.  Every thread of the workgroup calls it; the row must be in place.
__device__ __forceinline__ void tab_row_block(double* Kr, int W, long r, const TabOut& tb, int* last_s) {
    __syncthreads();
    if (threadIdx.x == 0) {
        double C = 0.0;
        int last = -1;
        for (int t = 0; t < W; ++t) {
            const double k = Kr[t];
            if (k > 0.0) {
                C = C + k;
                last = t;
            }
            Kr[t] = C;
        }
        *last_s = last;
        const double p = C * tb.dt;
        const double fl = floor(p);
        tb.gamma[r] = C;
        tb.n0[r] = (uint32_t)fl;
        tb.thr[r] = (uint32_t)floor((p - fl) * 4294967296.0);
    }
    __syncthreads();
    const int last = *last_s;
    const double g = last >= 0 ? Kr[last] : 0.0;
    __syncthreads();  // every thread has read Kr[last] before entries are overwritten
    uint64_t* crow = tb.cdf + r * W;
    for (int t = threadIdx.x; t < W; t += blockDim.x) {
        uint64_t v;
        if (last < 0)
            v = 0;
        else if (t >= last)
            v = 1ull << 32;
        else
            v = (uint64_t)floor(Kr[t] / g * 4294967296.0);
        crow[t] = v;
        reinterpret_cast<uint64_t*>(Kr)[t] = v;
    }
    if (tb.guide != nullptr) {
        __syncthreads();
        const uint64_t* T = reinterpret_cast<const uint64_t*>(Kr);
        uint32_t* gout = tb.guide + r * (tb.G + 1);
        for (int k = threadIdx.x; k < tb.G; k += blockDim.x) {
            const uint64_t L = ((uint64_t)k << 32) / (uint64_t)tb.G;
            int lo = 0, hi = W - 1;  // first t with T[t] > L, at most W - 1
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (T[mid] > L)
                    hi = mid;
                else
                    lo = mid + 1;
            }
            gout[k] = (uint32_t)lo;
        }
        if (threadIdx.x == 0) gout[tb.G] = (uint32_t)(W - 1);
    }
}

}  // namespace wk
