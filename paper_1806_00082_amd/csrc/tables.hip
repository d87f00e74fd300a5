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

}  // namespace wk

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
