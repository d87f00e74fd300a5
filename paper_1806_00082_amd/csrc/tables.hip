// Creation-rate tables of postulate II (Sec. 2.1, eq.(1) on the grid).
// Each row's positive part is summed in ascending m in FP64 by one lane (the order is the
// definition), so gamma, the integer creation thresholds and the CDF are the same numbers
// whatever the launch shape.  Rows up to TB_MAXW entries take one wave each: the row is
// staged in LDS with coalesced loads, one lane forms the running sums there, and the whole
// wave converts and stores the CDF; wider rows take one thread each.
#include "wk_internal.h"

namespace wk {

// Entry t (m = t - P) of a full row, read from either table layout.
template <typename KT>
__device__ __forceinline__ double row_entry(const KT* row, int layout, int P, int t) {
    if (layout == WK_FULL) return (double)row[t];
    if (t == 0) return -(double)row[P - 1];
    if (t < P) return -(double)row[P - 1 - t];
    if (t == P) return 0.0;
    return (double)row[t - P - 1];
}

template <typename KT>
__global__ void gamma_tables_kernel(const KT* __restrict__ K, int layout, int width, int row_len,
                                    int P, int n_rows, double dt, double* __restrict__ gamma,
                                    uint32_t* __restrict__ n0, uint32_t* __restrict__ thr,
                                    uint64_t* __restrict__ cdf) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    const KT* row = K + (long)r * row_len;
    double g = 0.0;
    int last = -1;
    for (int t = 0; t < width; ++t) {
        const double k = row_entry(row, layout, P, t);
        if (k > 0.0) {
            g = g + k;
            last = t;
        }
    }
    const double p = g * dt;
    const double fl = floor(p);
    gamma[r] = g;
    n0[r] = (uint32_t)fl;
    thr[r] = (uint32_t)floor((p - fl) * 4294967296.0);
    uint64_t* crow = cdf + (long)r * width;
    double C = 0.0;
    for (int t = 0; t < width; ++t) {
        const double k = row_entry(row, layout, P, t);
        if (k > 0.0) C = C + k;
        uint64_t v;
        if (last < 0)
            v = 0;
        else if (t >= last)
            v = 1ull << 32;
        else
            v = (uint64_t)floor(C / g * 4294967296.0);
        crow[t] = v;
    }
}

constexpr int TB_MAXW = 4096;  // widest row handled one wave per row (LDS: 8 bytes per entry)

template <typename KT>
__global__ __launch_bounds__(64) void gamma_tables_wave(const KT* __restrict__ K, int layout, int width,
                                                        int row_len, int P, int n_rows, double dt,
                                                        double* __restrict__ gamma,
                                                        uint32_t* __restrict__ n0,
                                                        uint32_t* __restrict__ thr,
                                                        uint64_t* __restrict__ cdf) {
    extern __shared__ double Cs[];  // [width]: the row, then its running positive sums
    __shared__ int last_s;
    const int r = blockIdx.x, lane = threadIdx.x;
    if (r >= n_rows) return;
    const KT* row = K + (long)r * row_len;
    for (int t = lane; t < width; t += 64) Cs[t] = row_entry(row, layout, P, t);
    __syncthreads();
    if (lane == 0) {
        double C = 0.0;
        int last = -1;
        for (int t = 0; t < width; ++t) {
            const double k = Cs[t];
            if (k > 0.0) {
                C = C + k;
                last = t;
            }
            Cs[t] = C;
        }
        last_s = last;
        const double g = C;
        const double p = g * dt;
        const double fl = floor(p);
        gamma[r] = g;
        n0[r] = (uint32_t)fl;
        thr[r] = (uint32_t)floor((p - fl) * 4294967296.0);
    }
    __syncthreads();
    const int last = last_s;
    const double g = last >= 0 ? Cs[last] : 0.0;
    uint64_t* crow = cdf + (long)r * width;
    for (int t = lane; t < width; t += 64) {
        uint64_t v;
        if (last < 0)
            v = 0;
        else if (t >= last)
            v = 1ull << 32;
        else
            v = (uint64_t)floor(Cs[t] / g * 4294967296.0);
        crow[t] = v;
    }
}

// Guide table of a CDF row for indexed search (Chen and Asau, 1974): for G buckets of the
// 32-bit uniforms, guide[k] = min{t : cdf[t] > floor(k 2^32 / G)} (k < G) and guide[G] =
// width - 1.  A draw u falls in bucket k = floor(u G / 2^32), and min{t : u < cdf[t]} lies in
// [guide[k], guide[k+1]], so the search visits a handful of entries instead of log2(width).
// One thread per row, one merge pass over the row.
__global__ void sampling_guide_kernel(const uint64_t* __restrict__ cdf, int n_rows, int width,
                                      int G, uint32_t* __restrict__ guide) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    const uint64_t* T = cdf + (long)r * width;
    uint32_t* out = guide + (long)r * (G + 1);
    int t = 0;
    for (int k = 0; k < G; ++k) {
        const uint64_t L = ((uint64_t)k << 32) / (uint64_t)G;
        while (t < width - 1 && T[t] <= L) ++t;
        out[k] = (uint32_t)t;
    }
    out[G] = (uint32_t)(width - 1);
}

// The same guide, one wave per row: the row is staged in LDS, each lane finds its buckets'
// entries by binary search (first t with cdf[t] > L, at most width - 1: the merge's result).
__global__ __launch_bounds__(64) void sampling_guide_wave(const uint64_t* __restrict__ cdf, int n_rows,
                                                          int width, int G, uint32_t* __restrict__ guide) {
    extern __shared__ uint64_t Ts[];  // [width]
    const int r = blockIdx.x, lane = threadIdx.x;
    if (r >= n_rows) return;
    const uint64_t* T = cdf + (long)r * width;
    for (int t = lane; t < width; t += 64) Ts[t] = T[t];
    __syncthreads();
    uint32_t* out = guide + (long)r * (G + 1);
    for (int k = lane; k < G; k += 64) {
        const uint64_t L = ((uint64_t)k << 32) / (uint64_t)G;
        int lo = 0, hi = width - 1;  // answer in [lo, hi]
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (Ts[mid] > L)
                hi = mid;
            else
                lo = mid + 1;
        }
        out[k] = (uint32_t)lo;
    }
    if (lane == 0) out[G] = (uint32_t)(width - 1);
}

}  // namespace wk

extern "C" int wk_sampling_guide(const uint64_t* cdf, int32_t n_rows, int32_t width,
                                 int32_t guide_len, uint32_t* guide, void* stream) {
    WK_REQUIRE(n_rows >= 0, "wk_sampling_guide: negative row count");
    WK_REQUIRE(width >= 1, "wk_sampling_guide: width must be positive");
    WK_REQUIRE(guide_len >= 1 && guide_len <= (1 << 20), "wk_sampling_guide: guide_len out of range");
    if (n_rows == 0) return WK_OK;
    WK_REQUIRE(cdf && guide, "wk_sampling_guide: NULL array");
    if (width <= wk::TB_MAXW) {
        hipLaunchKernelGGL(wk::sampling_guide_wave, dim3((unsigned)n_rows), dim3(64),
                           sizeof(uint64_t) * (size_t)width, wk::as_stream(stream), cdf, n_rows, width,
                           guide_len, guide);
    } else {
        dim3 grid((n_rows + 127) / 128), block(128);
        hipLaunchKernelGGL(wk::sampling_guide_kernel, grid, block, 0, wk::as_stream(stream), cdf, n_rows,
                           width, guide_len, guide);
    }
    return wk::check_launch("wk_sampling_guide");
}

extern "C" int wk_gamma_tables(const wk_mesh* mesh, const void* K, int32_t k_f64, int32_t layout,
                               int32_t n_rows, double dt, double* gamma, uint32_t* n0,
                               uint32_t* thr, uint64_t* cdf, void* stream) {
    WK_REQUIRE(mesh != nullptr, "wk_gamma_tables: mesh is NULL");
    WK_REQUIRE(mesh->dim == 1 || mesh->dim == 2, "wk_gamma_tables: dim must be 1 or 2");
    WK_REQUIRE(mesh->n_m >= 2 && mesh->n_m % 2 == 0, "wk_gamma_tables: n_m must be even");
    WK_REQUIRE(layout == WK_FULL || (layout == WK_HALF && mesh->dim == 1),
               "wk_gamma_tables: half layout is 1-D only");
    WK_REQUIRE(n_rows >= 0, "wk_gamma_tables: negative row count");
    WK_REQUIRE(dt >= 0.0, "wk_gamma_tables: dt must be >= 0");
    if (n_rows == 0) return WK_OK;
    WK_REQUIRE(K && gamma && n0 && thr && cdf, "wk_gamma_tables: NULL array");
    const int P = mesh->n_m / 2;
    const int width = mesh->dim == 1 ? mesh->n_m : mesh->n_m * mesh->n_m;
    const int row_len = layout == WK_HALF ? P : width;
    hipStream_t s = wk::as_stream(stream);
    if (width <= wk::TB_MAXW) {
        const size_t sh = sizeof(double) * (size_t)width;
        if (k_f64)
            hipLaunchKernelGGL(wk::gamma_tables_wave<double>, dim3((unsigned)n_rows), dim3(64), sh, s,
                               static_cast<const double*>(K), layout, width, row_len, P, n_rows, dt,
                               gamma, n0, thr, cdf);
        else
            hipLaunchKernelGGL(wk::gamma_tables_wave<float>, dim3((unsigned)n_rows), dim3(64), sh, s,
                               static_cast<const float*>(K), layout, width, row_len, P, n_rows, dt,
                               gamma, n0, thr, cdf);
        return wk::check_launch("wk_gamma_tables");
    }
    dim3 grid((n_rows + 127) / 128), block(128);
    if (k_f64)
        hipLaunchKernelGGL(wk::gamma_tables_kernel<double>, grid, block, 0, s,
                           static_cast<const double*>(K), layout, width, row_len, P, n_rows, dt,
                           gamma, n0, thr, cdf);
    else
        hipLaunchKernelGGL(wk::gamma_tables_kernel<float>, grid, block, 0, s,
                           static_cast<const float*>(K), layout, width, row_len, P, n_rows, dt,
                           gamma, n0, thr, cdf);
    return wk::check_launch("wk_gamma_tables");
}
