// Creation-rate tables of postulate II (Sec. 2.1, eq.(1) on the grid).
// One thread per table row sums max(K, 0) in ascending m in FP64, so gamma, the integer
// creation thresholds and the CDF are the same numbers whatever the launch shape.
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

}  // namespace wk

extern "C" int wk_sampling_guide(const uint64_t* cdf, int32_t n_rows, int32_t width,
                                 int32_t guide_len, uint32_t* guide, void* stream) {
    WK_REQUIRE(n_rows >= 0, "wk_sampling_guide: negative row count");
    WK_REQUIRE(width >= 1, "wk_sampling_guide: width must be positive");
    WK_REQUIRE(guide_len >= 1 && guide_len <= (1 << 20), "wk_sampling_guide: guide_len out of range");
    if (n_rows == 0) return WK_OK;
    WK_REQUIRE(cdf && guide, "wk_sampling_guide: NULL array");
    dim3 grid((n_rows + 127) / 128), block(128);
    hipLaunchKernelGGL(wk::sampling_guide_kernel, grid, block, 0, wk::as_stream(stream), cdf, n_rows,
                       width, guide_len, guide);
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
