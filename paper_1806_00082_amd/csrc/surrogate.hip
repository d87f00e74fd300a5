// The trainable reduced-width kernel network of eq.(5) (Sec. 2.3) and its hand-written
// adjoint, plus the MSE gradient and SGD update of the training loop (Sec. 3).
//
//   Kh[r][t] = Pi(t) * sum_g A[r][g] Bm[g][t],                 m = t + 1, t < P
//   A[r][g]  = sum_p wV[p] V(clamp(i_r + o(g,p))),             o(g,p) = -P + N g + p
//   Bm[g][t] = W[g] sin(u_g m),  u_g = (2 pi / n_m) sum_p wT[p] o(g,p)
//   Pi(t)    = prod_{s < log2 N} cos(2^s pi m / n_m)
// A is a stride-N convolution of the potential (the f_V of Sec. 3) built per row tile in
// LDS; Bm and Pi are tiny (H x P, P) and are formed once per call by surr_prep.
#include <map>
#include <mutex>
#include <string>
#include <type_traits>

#include "lowp.h"
#include "wk_internal.h"

namespace wk {

constexpr int SU_THREADS = 256;
constexpr int SU_BM = 32;            // rows per workgroup of the backward
constexpr int SD_BM = 16;            // rows per workgroup (FP64 forward, backward tiles)
constexpr int SB_MAXBLK = 1024;      // workgroups of the backward (each loops over row tiles)
constexpr int SU_MAXH = 256;         // largest hidden width supported
constexpr int SU_MAXN = 64;          // largest group size supported

__device__ __forceinline__ double two_pi_over(int n_m) { return 6.283185307179586476925286766559 / (double)n_m; }

// Bm (H x Pn, zero padded) and Pi (Pn) in double and float.
__global__ void surr_prep(int n_m, int N, int H, int Pn, const float* __restrict__ wT,
                          const float* __restrict__ W, double* __restrict__ Bd,
                          float* __restrict__ Bf, double* __restrict__ Pid, float* __restrict__ Pif,
                          double* __restrict__ u_out) {
    const int P = n_m / 2;
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    int L = 0;
    while ((1 << L) < N) ++L;
    if (idx < (long)H * Pn) {
        const int g = (int)(idx / Pn), t = (int)(idx % Pn);
        double u = 0.0;
        for (int p = 0; p < N; ++p) u += (double)wT[p] * (two_pi_over(n_m) * (double)(-P + N * g + p));
        const double v = t < P ? (double)W[g] * sin(u * (double)(t + 1)) : 0.0;
        Bd[idx] = v;
        Bf[idx] = (float)v;
        if (t == 0) u_out[g] = u;
    }
    if (idx < Pn) {
        double pr = 1.0;
        if (idx < P)
            for (int s = 0; s < L; ++s)
                pr *= cospi((double)(1 << s) * (double)(idx + 1) / (double)n_m);
        else
            pr = 0.0;
        Pid[idx] = pr;
        Pif[idx] = (float)pr;
    }
}

template <int BM, typename T>
__device__ __forceinline__ void conv_rows(const double* __restrict__ V, int nx, long row0, long R,
                                          int n_cells, const int32_t* __restrict__ cells, int P,
                                          int N, int H, const float* __restrict__ wV, T* A,
                                          int lda, int* rcell, long* rbase) {
    __syncthreads();  // previous users of A / rcell are done
    for (int rr = threadIdx.x; rr < BM; rr += blockDim.x) {
        const long r = row0 + rr;
        int cell = -1;
        long base = 0;
        if (r < R) {
            const long b = r / n_cells;
            const int ci = (int)(r - b * n_cells);
            cell = cells ? cells[ci] : ci;
            if (cell < 0 || cell >= nx) cell = -2;
            base = b * (long)nx;
        }
        rcell[rr] = cell;
        rbase[rr] = base;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, nwv = blockDim.x >> 6;
    for (int rr = threadIdx.x >> 6; rr < BM; rr += nwv) {  // rows to waves, groups to lanes
        const int cell = rcell[rr];
        const double* Vb = V + rbase[rr];
        for (int g = lane; g < H; g += 64) {
            double a = cell == -2 ? __builtin_nan("") : 0.0;
            if (cell >= 0) {
                a = 0.0;
                for (int p = 0; p < N; ++p) {
                    const int l = min(max(cell - P + N * g + p, 0), nx - 1);
                    a += (double)wV[p] * Vb[l];
                }
            }
            A[rr * lda + g] = (T)a;
        }
    }
    __syncthreads();
}

// Reference-precision forward: FP64 FMAs, one thread per output.
__global__ __launch_bounds__(SU_THREADS) void surr_fwd_f64(
    const double* __restrict__ V, int nx, long R, int n_cells, const int32_t* __restrict__ cells,
    int P, int N, int H, int Pn, const float* __restrict__ wV, const double* __restrict__ Bd,
    const double* __restrict__ Pid, double* __restrict__ out) {
    extern __shared__ double smem_d[];
    __shared__ int rcell[SD_BM];
    __shared__ long rbase[SD_BM];
    double* A = smem_d;  // [SD_BM][H + 1]
    const long row0 = (long)blockIdx.x * SD_BM;
    conv_rows<SD_BM, double>(V, nx, row0, R, n_cells, cells, P, N, H, wV, A, H + 1, rcell, rbase);
    for (int e = threadIdx.x; e < SD_BM * P; e += blockDim.x) {
        const int rr = e / P, t = e - rr * P;
        const long r = row0 + rr;
        if (r >= R) continue;
        double acc = 0.0;
        for (int g = 0; g < H; ++g) acc += A[rr * (H + 1) + g] * Bd[(long)g * Pn + t];
        out[r * P + t] = Pid[t] * acc;
    }
}

// Bm transposed and zero padded to Hk (a multiple of 32), in FP32 and as BF16 bits, so that a
// lane's MFMA B fragment is contiguous: Bt[t][g] = Bm[g][t].
__global__ void surr_prep_t(int H, int Hk, int Pn, const float* __restrict__ Bf,
                            float* __restrict__ Btf, uint16_t* __restrict__ Btb) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)Pn * Hk) return;
    const int t = (int)(idx / Hk), g = (int)(idx % Hk);
    const float v = g < H ? Bf[(long)g * Pn + t] : 0.f;
    Btf[idx] = v;
    Btb[idx] = bf16_bits_f(v);
}

// Forward on MFMA (FP32: v_mfma_f32_16x16x4_f32; BF16: v_mfma_f32_16x16x32_bf16 with FP32
// sums), SF_BM rows per tile, workgroups looping over tiles.  When a tile is a run of
// consecutive cells of one potential (all cells evaluated), the potential window it needs
// (SF_BM + n_m values) is staged in LDS once and the stride-N convolution reads it there;
// otherwise (cell lists, tiles across potentials) rows gather their values from global
// memory.  A is kept in LDS in the MFMA input type.  The contraction index is permuted per
// lane group (lane group j of a 16 x 16 x 4 step s takes g = j Hk/4 + s; of a 16 x 16 x 32
// step s, g = j Hk/4 + 8 s + q), the same for A and B, so that a lane's fragments of
// consecutive steps are contiguous and load as 16-byte vectors.  Four waves split the
// column tiles; B fragments come from the transposed table.
constexpr int SF_BM = 64;

template <bool BF16>
__global__ __launch_bounds__(SU_THREADS) void surr_fwd_mfma(
    const double* __restrict__ V, int nx, long R, int n_cells, const int32_t* __restrict__ cells,
    int P, int N, int H, int Hk, int Pn, const float* __restrict__ wV,
    const float* __restrict__ Btf, const uint16_t* __restrict__ Btb,
    const float* __restrict__ Pif, float* __restrict__ out) {
    using AT = typename std::conditional<BF16, uint16_t, float>::type;
    extern __shared__ double smem_sf[];
    __shared__ int rcell[SF_BM];
    __shared__ long rbase[SF_BM];
    const int lda = BF16 ? Hk + 8 : Hk + 4;  // 16-byte aligned rows, bank-spread
    AT* A = reinterpret_cast<AT*>(smem_sf);                                  // [SF_BM][lda]
    double* Vw = smem_sf + (SF_BM * lda * (int)sizeof(AT) + 7) / 8;          // [SF_BM + 2P]
    float* Ag = reinterpret_cast<float*>(Vw);  // gather path: FP32 rows [SF_BM][Hk + 1]
    for (int e = threadIdx.x; e < SF_BM * lda; e += blockDim.x) A[e] = (AT)0;  // pads stay 0
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int kq = Hk / 4;  // contraction indices per lane group
    const long ntiles = (R + SF_BM - 1) / SF_BM;
    for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const long row0 = tile * SF_BM;
        const long rend = min(R, row0 + SF_BM);
        const bool run = cells == nullptr && n_cells == nx && row0 / nx == (rend - 1) / nx;
        __syncthreads();  // previous tile's users of A / Vw are done
        if (run) {
            const long b = row0 / nx;
            const int c0 = (int)(row0 - b * nx);
            const double* Vb = V + b * (long)nx;
            const int nw = SF_BM + 2 * P;
            for (int k = threadIdx.x; k < nw; k += blockDim.x)
                Vw[k] = Vb[min(max(c0 - P + k, 0), nx - 1)];
            __syncthreads();
            const int nrow = (int)(rend - row0);
            // rows to waves, groups to lanes (no index divisions)
            for (int rr = wave; rr < SF_BM; rr += 4)
                for (int g = lane; g < H; g += 64) {
                    double a = 0.0;
                    if (rr < nrow)
                        for (int p = 0; p < N; ++p) a += (double)wV[p] * Vw[rr + N * g + p];
                    A[rr * lda + g] = BF16 ? (AT)bf16_bits_f((float)a) : (AT)(float)a;
                }
        } else {
            conv_rows<SF_BM, float>(V, nx, row0, R, n_cells, cells, P, N, H, wV, Ag, Hk + 1, rcell,
                                    rbase);
            for (int rr = wave; rr < SF_BM; rr += 4)
                for (int g = lane; g < H; g += 64) {
                    const float a = Ag[rr * (Hk + 1) + g];
                    A[rr * lda + g] = BF16 ? (AT)bf16_bits_f(a) : (AT)a;
                }
        }
        __syncthreads();
        for (int ct = wave; ct * 16 < Pn; ct += 4) {
            f32x4 acc[SF_BM / 16];
#pragma unroll
            for (int tm = 0; tm < SF_BM / 16; ++tm) acc[tm] = f32x4{0.f, 0.f, 0.f, 0.f};
            const long brow = (long)(ct * 16 + lr) * Hk + lk * kq;
            if (BF16) {
                for (int s8 = 0; s8 < kq; s8 += 8) {
                    const bf16x8 bv = *reinterpret_cast<const bf16x8*>(Btb + brow + s8);
#pragma unroll
                    for (int tm = 0; tm < SF_BM / 16; ++tm) {
                        const bf16x8 av = *reinterpret_cast<const bf16x8*>(
                            reinterpret_cast<const uint16_t*>(A) + (tm * 16 + lr) * lda + lk * kq + s8);
                        acc[tm] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[tm], 0, 0, 0);
                    }
                }
            } else {
                for (int s4 = 0; s4 < kq; s4 += 4) {
                    const float4 bv = *reinterpret_cast<const float4*>(Btf + brow + s4);
#pragma unroll
                    for (int tm = 0; tm < SF_BM / 16; ++tm) {
                        const float4 av = *reinterpret_cast<const float4*>(
                            reinterpret_cast<const float*>(A) + (tm * 16 + lr) * lda + lk * kq + s4);
                        acc[tm] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, bv.x, acc[tm], 0, 0, 0);
                        acc[tm] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, bv.y, acc[tm], 0, 0, 0);
                        acc[tm] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, bv.z, acc[tm], 0, 0, 0);
                        acc[tm] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, bv.w, acc[tm], 0, 0, 0);
                    }
                }
            }
            const int t = ct * 16 + lr;
            if (t < P) {
                const float pi = Pif[t];
#pragma unroll
                for (int tm = 0; tm < SF_BM / 16; ++tm)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const long r = row0 + tm * 16 + 4 * lk + e;
                        if (r < R) out[r * P + t] = pi * acc[tm][e];
                    }
            }
        }
    }
}

// Forward with the whole transposed table Bt in LDS (used when it fits): persistent
// workgroups load Bt once, then per tile of SF_BM rows form A in LDS (as above), and each wave
// takes 16 rows: its A fragments for the whole contraction move into registers, and it sweeps
// the column tiles four at a time (four independent accumulators), B fragments from LDS.
// Natural contraction order per 16x16x32 step (g = 32 s + 8 (l / 16) + q); the FP32 form
// takes four 16x16x4 steps per 16-byte fragment (g = 16 s + 4 (l / 16) + q, step q).
template <bool BF16, int HK>
__global__ __launch_bounds__(SU_THREADS) void surr_fwd_lds(
    const double* __restrict__ V, int nx, long R, int n_cells, const int32_t* __restrict__ cells,
    int P, int N, int H, int Pn, const float* __restrict__ wV,
    const float* __restrict__ Btf, const uint16_t* __restrict__ Btb,
    const float* __restrict__ Pif, float* __restrict__ out) {
    using AT = typename std::conditional<BF16, uint16_t, float>::type;
    constexpr int LD = HK + (BF16 ? 8 : 4);    // row stride (elements): 16-byte rows, spread banks
    constexpr int NF = BF16 ? HK / 32 : HK / 16;  // 16-byte A fragments per lane
    extern __shared__ double smem_fl[];
    __shared__ int rcell[SF_BM];
    __shared__ long rbase[SF_BM];
    // column tiles padded to a multiple of four (zero rows of Bt, zero Pi): no per-tile guards
    const int Pn4 = (Pn + 63) / 64 * 64;
    AT* Bs = reinterpret_cast<AT*>(smem_fl);                               // [Pn4][LD]
    AT* As = Bs + (long)Pn4 * LD;                                          // [SF_BM][LD]
    float* Pis = reinterpret_cast<float*>(As + SF_BM * LD);                // [Pn4]
    double* Vw = smem_fl + ((long)(Pn4 + SF_BM) * LD * (long)sizeof(AT) + 4L * Pn4 + 7) / 8;  // [SF_BM + 2P]
    for (int e = threadIdx.x; e < Pn4 * HK; e += blockDim.x) {
        const int t = e / HK, g = e - t * HK;
        Bs[t * LD + g] = t < Pn ? (BF16 ? (AT)Btb[e] : (AT)Btf[e]) : (AT)0;
    }
    for (int t = threadIdx.x; t < Pn4; t += blockDim.x) Pis[t] = t < P ? Pif[t] : 0.f;
    for (int e = threadIdx.x; e < SF_BM * LD; e += blockDim.x) As[e] = (AT)0;  // pads stay 0
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int nct = Pn4 / 16;
    const long ntiles = (R + SF_BM - 1) / SF_BM;
    // a tile whose rows are consecutive cells of one potential reads a window of it; the next
    // tile's window is loaded into registers while this tile's products run (WPF values per
    // thread; wider windows are loaded in place)
    constexpr int WPF = 4;
    const int nwin = SF_BM + 2 * P;
    const bool pf = nwin <= WPF * SU_THREADS;
    auto is_run = [&](long row0) {
        const long rend = min(R, row0 + SF_BM);
        return cells == nullptr && n_cells == nx && row0 / nx == (rend - 1) / nx;
    };
    double wpf[WPF];
    auto fetch = [&](long row0) {
        const long b = row0 / nx;
        const int c0 = (int)(row0 - b * nx);
        const double* Vb = V + b * (long)nx;
#pragma unroll
        for (int i = 0; i < WPF; ++i) {
            const int k = threadIdx.x + i * SU_THREADS;
            if (k < nwin) wpf[i] = Vb[min(max(c0 - P + k, 0), nx - 1)];
        }
    };
    if (pf && blockIdx.x < ntiles && is_run((long)blockIdx.x * SF_BM)) fetch((long)blockIdx.x * SF_BM);
    for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const long row0 = tile * SF_BM;
        const long rend = min(R, row0 + SF_BM);
        const int nrow = (int)(rend - row0);
        const bool run = is_run(row0);
        __syncthreads();  // previous tile's readers of As / Vw are done
        if (run) {
            if (pf) {
#pragma unroll
                for (int i = 0; i < WPF; ++i) {
                    const int k = threadIdx.x + i * SU_THREADS;
                    if (k < nwin) Vw[k] = wpf[i];
                }
            } else {
                const long b = row0 / nx;
                const int c0 = (int)(row0 - b * nx);
                const double* Vb = V + b * (long)nx;
                for (int k = threadIdx.x; k < nwin; k += blockDim.x) Vw[k] = Vb[min(max(c0 - P + k, 0), nx - 1)];
            }
            __syncthreads();
            // rows to waves, groups to lanes (no index divisions)
            for (int rr = wave; rr < SF_BM; rr += 4)
                for (int g = lane; g < H; g += 64) {
                    double a = 0.0;
                    if (rr < nrow)
                        for (int p = 0; p < N; ++p) a += (double)wV[p] * Vw[rr + N * g + p];
                    As[rr * LD + g] = BF16 ? (AT)bf16_bits_f((float)a) : (AT)(float)a;
                }
        } else {
            for (int rr = threadIdx.x; rr < SF_BM; rr += blockDim.x) {
                const long r = row0 + rr;
                int cell = -1;
                long base = 0;
                if (r < R) {
                    const long b = r / n_cells;
                    const int ci = (int)(r - b * n_cells);
                    cell = cells ? cells[ci] : ci;
                    if (cell < 0 || cell >= nx) cell = -2;  // id outside the mesh: row of NaN
                    base = b * (long)nx;
                }
                rcell[rr] = cell;
                rbase[rr] = base;
            }
            __syncthreads();
            for (int rr = wave; rr < SF_BM; rr += 4) {
                const int cell = rcell[rr];
                const double* Vb = V + rbase[rr];
                for (int g = lane; g < H; g += 64) {
                    double a = cell == -2 ? __builtin_nan("") : 0.0;
                    if (cell >= 0)
                        for (int p = 0; p < N; ++p)
                            a += (double)wV[p] * Vb[min(max(cell - P + N * g + p, 0), nx - 1)];
                    As[rr * LD + g] = BF16 ? (AT)bf16_bits_f((float)a) : (AT)(float)a;
                }
            }
        }
        __syncthreads();
        // this wave's rows: 16 wave .. 16 wave + 15
        s16x8 afb[BF16 ? NF : 1];
        float4 aff[BF16 ? 1 : NF];
        const AT* arow = As + (wave * 16 + lr) * LD;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            if constexpr (BF16)
                afb[f] = *reinterpret_cast<const s16x8*>(arow + 32 * f + 8 * lk);
            else
                aff[f] = *reinterpret_cast<const float4*>(arow + 16 * f + 4 * lk);
        }
        {
            const long nt = tile + gridDim.x;
            if (pf && nt < ntiles && is_run(nt * SF_BM)) fetch(nt * SF_BM);
        }
        for (int ct0 = 0; ct0 < nct; ct0 += 4) {
            f32x4 acc[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                if constexpr (BF16) {
                    s16x8 bv[4];
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        bv[c] = *reinterpret_cast<const s16x8*>(Bs + ((ct0 + c) * 16 + lr) * LD + 32 * f + 8 * lk);
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            __builtin_bit_cast(bf16x8, afb[f]), __builtin_bit_cast(bf16x8, bv[c]), acc[c], 0, 0, 0);
                } else {
                    float4 bv[4];
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        bv[c] = *reinterpret_cast<const float4*>(Bs + ((ct0 + c) * 16 + lr) * LD + 16 * f + 4 * lk);
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(aff[f].x, bv[c].x, acc[c], 0, 0, 0);
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(aff[f].y, bv[c].y, acc[c], 0, 0, 0);
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(aff[f].z, bv[c].z, acc[c], 0, 0, 0);
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(aff[f].w, bv[c].w, acc[c], 0, 0, 0);
                }
            }
            float* orow = out + (row0 + wave * 16 + 4 * lk) * P + ct0 * 16 + lr;
            if (nrow == SF_BM && (ct0 + 4) * 16 <= P) {
                // whole group inside the table: no per-lane guards (stores issue back to back)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const float pi = Pis[(ct0 + c) * 16 + lr];
#pragma unroll
                    for (int e = 0; e < 4; ++e) orow[e * P + c * 16] = pi * acc[c][e];
                }
            } else {
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int t = (ct0 + c) * 16 + lr;
                    const float pi = Pis[t];
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (t < P && wave * 16 + 4 * lk + e < nrow) orow[e * P + c * 16] = pi * acc[c][e];
                }
            }
        }
    }
}

// LDS bytes of surr_fwd_lds for a shape, or 0 when it does not fit (then surr_fwd_mfma runs).
static size_t surr_fwd_lds_bytes(bool bf16, int Hk, int Pn, int P) {
    if (Hk != 32 && Hk != 64 && Hk != 128 && Hk != 256) return 0;
    const size_t es = bf16 ? 2 : 4, ld = (size_t)Hk + (bf16 ? 8 : 4);
    const size_t pn4 = ((size_t)Pn + 63) / 64 * 64;
    const size_t b = ((pn4 + SF_BM) * ld * es + 4 * pn4 + 7) / 8 * 8 + sizeof(double) * (SF_BM + 2 * (size_t)P);
    return b <= 150 * 1024 ? b : 0;
}

// ----------------------------------------------------------------------------- backward
// Per workgroup of SU_BM rows: Et = E * Pi (LDS), GA = Et Bm^T (LDS and, for dV, global),
// block partials of GB = A^T Et (H x P) and of dwV.  A fixed-order reduction over the
// workgroups then forms dW, du (-> dwT) and dwV.  dV is a gather over rows (all-cells only).
struct SurrWS {
    float* GBpart;    // [nblk][H][P]
    float* wVpart;    // [nblk][N]
    float* GA;        // [R][H]   (only when dV is requested)
    double* u;        // [H]
    double* du;       // [H]
    double* Bd;       // [H][Pn]
    float* Bf;        // [H][Pn]
    double* Pid;      // [Pn]
    float* Pif;       // [Pn]
};

__global__ __launch_bounds__(SU_THREADS) void surr_bwd_block(
    const double* __restrict__ V, int nx, long R, int n_cells, const int32_t* __restrict__ cells,
    int P, int N, int H, int Pn, const float* __restrict__ wV, const float* __restrict__ E,
    SurrWS w, int want_GA) {
    extern __shared__ float smem_f[];
    __shared__ int rcell[SD_BM];
    __shared__ long rbase[SD_BM];
    float* A = smem_f;                       // [SD_BM][H + 1]
    float* Et = A + SD_BM * (H + 1);         // [SD_BM][P + 1]
    float* GA = Et + SD_BM * (P + 1);        // [SD_BM][H + 1]
    float* gbp = w.GBpart + (long)blockIdx.x * H * P;   // this workgroup's private partials
    float* wvp = w.wVpart + (long)blockIdx.x * N;
    for (int e = threadIdx.x; e < H * P; e += blockDim.x) gbp[e] = 0.f;
    for (int p = threadIdx.x; p < N; p += blockDim.x) wvp[p] = 0.f;
    const long ntiles = (R + SD_BM - 1) / SD_BM;
    for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const long row0 = tile * SD_BM;
        conv_rows<SD_BM, float>(V, nx, row0, R, n_cells, cells, P, N, H, wV, A, H + 1, rcell, rbase);
        for (int e = threadIdx.x; e < SD_BM * P; e += blockDim.x) {
            const int rr = e / P, t = e - rr * P;
            const long r = row0 + rr;
            Et[rr * (P + 1) + t] = (r < R && rcell[rr] >= 0) ? E[r * P + t] * w.Pif[t] : 0.f;
        }
        __syncthreads();
        // GA = Et Bm^T
        for (int e = threadIdx.x; e < SD_BM * H; e += blockDim.x) {
            const int rr = e / H, g = e - rr * H;
            float acc = 0.f;
            for (int t = 0; t < P; ++t) acc = fmaf(Et[rr * (P + 1) + t], w.Bf[(long)g * Pn + t], acc);
            GA[rr * (H + 1) + g] = acc;
            const long r = row0 + rr;
            if (want_GA && r < R) w.GA[r * H + g] = acc;
        }
        __syncthreads();
        // GB partial += A^T Et over this tile (each entry owned by one thread)
        for (int e = threadIdx.x; e < H * P; e += blockDim.x) {
            const int g = e / P, t = e - g * P;
            float acc = gbp[e];
            for (int rr = 0; rr < SD_BM; ++rr)
                if (rcell[rr] >= 0) acc = fmaf(A[rr * (H + 1) + g], Et[rr * (P + 1) + t], acc);
            gbp[e] = acc;
        }
        // dwV partial += sum_rows sum_g GA[r][g] V(clamp(i + o(g,p)))  (one wave per tap)
        for (int p = threadIdx.x >> 6; p < N; p += SU_THREADS / 64) {
            float acc = 0.f;
            for (int e = threadIdx.x & 63; e < SD_BM * H; e += 64) {
                const int rr = e / H, g = e - rr * H;
                const int cell = rcell[rr];
                if (cell < 0) continue;
                const int l = min(max(cell - P + N * g + p, 0), nx - 1);
                acc = fmaf(GA[rr * (H + 1) + g], (float)V[rbase[rr] + l], acc);
            }
            for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
            if ((threadIdx.x & 63) == 0) wvp[p] += acc;
        }
    }
}

// The same partials on FP32 MFMA (v_mfma_f32_16x16x4_f32), for shapes whose tables fit in
// LDS.  Persistent workgroups over tiles of SBM rows; per tile, in LDS: Et = E Pi (row-major
// for GA, transposed for GB), A^T from the convolution, GA = Et Bm^T (Bm fragments from the
// L2-resident table).  GB += A^T Et accumulates in registers across the workgroup's tiles (16 x
// 16 tiles of GB dealt round-robin to the four waves), dwV in LDS; both are written to the
// workgroup's partial slots at the end, for the same fixed-order reductions as above.
// Operand layouts (16x16x4 f32): lane l holds A[l % 16][k], B[k][l % 16] with k = l / 16, and
// C[4 (l / 16) + e][l % 16]; four consecutive steps take k = 16 s + 4 (l / 16) + q (q < 4), the
// same for both operands, so each lane's operands are 16-byte LDS reads.
constexpr int SBM = 32;       // rows per tile
constexpr int SB_MAXT = 16;   // GB accumulator tiles per wave
constexpr int SB_JMAX = 2;    // GA column blocks per wave (H <= 128)
constexpr int SB_SMAX = 8;    // 16-wide contraction groups of GA (P <= 128)

__global__ __launch_bounds__(SU_THREADS, 2) void surr_bwd_mfma(
    const double* __restrict__ V, int nx, long R, int n_cells, const int32_t* __restrict__ cells,
    int P, int N, int H, int Pn, int Hp, int Pp, const float* __restrict__ wV,
    const float* __restrict__ E, SurrWS w, int want_GA) {
    extern __shared__ float smem_b[];
    __shared__ int rcell[SBM];
    __shared__ long rbase[SBM];
    const int LP = Pp + 4, LR = SBM + 4, LH = Hp + 4;
    float* EtR = smem_b;                      // [SBM][LP]  Et[r][t]
    float* EtT = EtR + SBM * LP;              // [Pp][LR]   Et[r][t] at [t][r]
    float* AsT = EtT + Pp * LR;               // [Hp][LR]   A[r][g] at [g][r]
    float* GAs = AsT + Hp * LR;               // [SBM][LH]  GA[r][g]
    float* dwv = GAs + SBM * LH;              // [N]
    double* Vw = reinterpret_cast<double*>(dwv + ((N + 1) / 2) * 2);   // [SBM + 2P]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    for (int p = threadIdx.x; p < N; p += blockDim.x) dwv[p] = 0.f;
    // Bm fragments of this wave's GA column blocks (g = 16 j + l % 16, t = 16 sg + 4 (l / 16) + q),
    // loaded once: zero past H and P
    float4 bfr[SB_JMAX][SB_SMAX];
#pragma unroll
    for (int jb = 0; jb < SB_JMAX; ++jb)
#pragma unroll
        for (int sg = 0; sg < SB_SMAX; ++sg) {
            const int g = 16 * (wave + 4 * jb) + lr;
            bfr[jb][sg] = (g < H && sg < Pp / 16)
                              ? *reinterpret_cast<const float4*>(w.Bf + (long)g * Pn + 16 * sg + 4 * lk)
                              : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    const int ngt = (Hp / 16) * (Pp / 16);    // GB tiles
    f32x4 gb[SB_MAXT];
#pragma unroll
    for (int k = 0; k < SB_MAXT; ++k) gb[k] = f32x4{0.f, 0.f, 0.f, 0.f};
    const long ntiles = (R + SBM - 1) / SBM;
    auto is_run = [&](long row0) {
        const long rend = min(R, row0 + SBM);
        return cells == nullptr && n_cells == nx && row0 / nx == (rend - 1) / nx;
    };
    for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const long row0 = tile * SBM;
        const bool run = is_run(row0);
        __syncthreads();  // the previous tile's readers are done
        for (int rr = threadIdx.x; rr < SBM; rr += blockDim.x) {
            const long r = row0 + rr;
            int cell = -1;
            long base = 0;
            if (r < R) {
                const long b = r / n_cells;
                const int ci = (int)(r - b * n_cells);
                cell = cells ? cells[ci] : ci;
                if (cell < 0 || cell >= nx) cell = -2;
                base = b * (long)nx;
            }
            rcell[rr] = cell;
            rbase[rr] = base;
        }
        if (run) {
            const long b = row0 / nx;
            const int c0 = (int)(row0 - b * nx);
            const double* Vb = V + b * (long)nx;
            for (int k = threadIdx.x; k < SBM + 2 * P; k += blockDim.x) Vw[k] = Vb[min(max(c0 - P + k, 0), nx - 1)];
        }
        __syncthreads();
        // Et (both layouts) and A^T; rows outside the mesh or past R contribute nothing.  Rows
        // go to waves, columns to lanes (no index divisions); a wave's eight rows of E are
        // loaded before any is stored (loads in flight).
        for (int t = lane; t < Pp; t += 64) {
            const float pi = t < P ? w.Pif[t] : 0.f;
            float v[SBM / 4];
#pragma unroll
            for (int q = 0; q < SBM / 4; ++q) {
                const int rr = wave + 4 * q;
                v[q] = (t < P && rcell[rr] >= 0) ? E[(row0 + rr) * P + t] * pi : 0.f;
            }
#pragma unroll
            for (int q = 0; q < SBM / 4; ++q) {
                const int rr = wave + 4 * q;
                EtR[rr * LP + t] = v[q];
                EtT[t * LR + rr] = v[q];
            }
        }
        for (int rr = wave; rr < SBM; rr += 4) {
            const int cell = rcell[rr];
            const double* Vb = V + rbase[rr];
            for (int g = lane; g < Hp; g += 64) {
                double a = 0.0;
                if (cell >= 0 && g < H) {
                    if (run) {
                        for (int p = 0; p < N; ++p) a += (double)wV[p] * Vw[rr + N * g + p];
                    } else {
                        for (int p = 0; p < N; ++p) a += (double)wV[p] * Vb[min(max(cell - P + N * g + p, 0), nx - 1)];
                    }
                }
                AsT[g * LR + rr] = (float)a;
            }
        }
        __syncthreads();
        // GA = Et Bm^T: (SBM x Pp) (Pp x Hp); wave w takes column blocks j = w, w + 4 (both
        // row blocks), with their Bm fragments held in registers for the whole workgroup
#pragma unroll
        for (int jb = 0; jb < SB_JMAX; ++jb) {
            const int j = wave + 4 * jb;
            if (j >= Hp / 16) break;
#pragma unroll
            for (int i = 0; i < SBM / 16; ++i) {
                f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
                const float* ar = EtR + (16 * i + lr) * LP + 4 * lk;
#pragma unroll
                for (int sg = 0; sg < SB_SMAX; ++sg) {
                    if (sg >= Pp / 16) break;
                    const float4 a = *reinterpret_cast<const float4*>(ar + 16 * sg);
                    const float4 b = bfr[jb][sg];
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, acc, 0, 0, 0);
                }
                const int g = 16 * j + lr;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int rr = 16 * i + 4 * lk + e;
                    GAs[rr * LH + g] = acc[e];
                    if (want_GA && g < H && row0 + rr < R) w.GA[(row0 + rr) * H + g] = acc[e];
                }
            }
        }
        // GB += A^T Et: (Hp x SBM) (SBM x Pp)
#pragma unroll
        for (int k = 0; k < SB_MAXT; ++k) {
            const int q = wave + 4 * k;
            if (q >= ngt) break;
            const int gi = q % (Hp / 16), tj = q / (Hp / 16);
            const float* ar = AsT + (16 * gi + lr) * LR + 4 * lk;
            const float* br = EtT + (16 * tj + lr) * LR + 4 * lk;
#pragma unroll
            for (int s = 0; s < SBM; s += 16) {
                const float4 a = *reinterpret_cast<const float4*>(ar + s);
                const float4 b = *reinterpret_cast<const float4*>(br + s);
                gb[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, gb[k], 0, 0, 0);
                gb[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, gb[k], 0, 0, 0);
                gb[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, gb[k], 0, 0, 0);
                gb[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, gb[k], 0, 0, 0);
            }
        }
        __syncthreads();  // GA complete
        // dwV += sum over rows and groups of GA[r][g] V(clamp(i_r + o(g,p))), one wave per tap;
        // branch-free (rows outside the mesh have GA = 0; the window path always reads inside
        // the window, the gathered path a clamped cell of the row's potential)
        for (int p = wave; p < N; p += 4) {
            float acc = 0.f;
            for (int rr = 0; rr < SBM; ++rr) {
                const int cell = max(rcell[rr], 0);
                const double* Vb = V + rbase[rr];
                for (int g = lane; g < H; g += 64) {
                    const float v = run ? (float)Vw[rr + N * g + p]
                                        : (float)Vb[min(max(cell - P + N * g + p, 0), nx - 1)];
                    acc = fmaf(GAs[rr * LH + g], v, acc);
                }
            }
            for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
            if (lane == 0) dwv[p] += acc;
        }
    }
    __syncthreads();
    float* gbp = w.GBpart + (long)blockIdx.x * H * P;
#pragma unroll
    for (int k = 0; k < SB_MAXT; ++k) {
        const int q = wave + 4 * k;
        if (q >= ngt) break;
        const int gi = q % (Hp / 16), tj = q / (Hp / 16);
        const int t = 16 * tj + lr;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int g = 16 * gi + 4 * lk + e;
            if (g < H && t < P) gbp[(long)g * P + t] = gb[k][e];
        }
    }
    for (int p = threadIdx.x; p < N; p += blockDim.x) w.wVpart[(long)blockIdx.x * N + p] = dwv[p];
}

// LDS bytes of surr_bwd_mfma, or 0 when the shape does not fit (then surr_bwd_block runs).
static size_t surr_bwd_mfma_bytes(int H, int P, int N) {
    const size_t Hp = ((size_t)H + 15) / 16 * 16, Pp = ((size_t)P + 15) / 16 * 16;
    if ((Hp / 16) * (Pp / 16) > 4 * (size_t)SB_MAXT || Hp > 64 * SB_JMAX || Pp > 16 * SB_SMAX) return 0;
    const size_t LP = Pp + 4, LR = SBM + 4, LH = Hp + 4;
    const size_t f = SBM * LP + Pp * LR + Hp * LR + SBM * LH + ((size_t)N + 1) / 2 * 2;
    const size_t b = 4 * f + 8 * (SBM + 2 * (size_t)P);
    return b <= 150 * 1024 ? b : 0;
}

__global__ void zero_grads(float* a, int na, float* b, int nb, float* c, int nc) {
    for (int i = threadIdx.x; i < na; i += blockDim.x) a[i] = 0.f;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) b[i] = 0.f;
    for (int i = threadIdx.x; i < nc; i += blockDim.x) c[i] = 0.f;
}

// Fixed-order sum of the block partials: 64 entries of GB per workgroup of 16 waves; wave j
// sums the partials k = j, j + 16, ... in ascending k, and the sixteen sums are added in wave
// order.
constexpr int RG_WAVES = 16;
__global__ __launch_bounds__(64 * RG_WAVES) void surr_bwd_reduce_gb(int nblk, int H, int P, SurrWS w) {
    __shared__ float part[RG_WAVES][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const long e = (long)blockIdx.x * 64 + lane;
    const long n = (long)H * P;
    float acc = 0.f;
    if (e < n)
        for (int k = wv; k < nblk; k += RG_WAVES) acc += w.GBpart[(long)k * n + e];
    part[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && e < n) {
        float t = part[0][lane];
#pragma unroll
        for (int j = 1; j < RG_WAVES; ++j) t += part[j][lane];
        w.GBpart[e] = t;
    }
}

// dW[g] = sum_t GB[g][t] sin(u_g m) and du[g] = sum_t GB[g][t] W[g] m cos(u_g m), m = t + 1:
// one workgroup per g, FP64 terms summed in a fixed tree order.
__global__ __launch_bounds__(256) void surr_bwd_params_g(int P, const float* __restrict__ W, SurrWS w,
                                                         float* __restrict__ dW, double* __restrict__ du) {
    __shared__ double red[2][4];
    const int g = blockIdx.x, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const double u = w.u[g];
    double a = 0.0, b = 0.0;
    for (int t = threadIdx.x; t < P; t += blockDim.x) {
        const double gbv = (double)w.GBpart[(long)g * P + t];
        const double m = (double)(t + 1);
        a += gbv * sin(u * m);
        b += gbv * (double)W[g] * m * cos(u * m);
    }
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
    }
    if (lane == 0) {
        red[0][wv] = a;
        red[1][wv] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        dW[g] = (float)(((red[0][0] + red[0][1]) + red[0][2]) + red[0][3]);
        du[g] = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
    }
}

// dwT[p] = sum_g du[g] (2 pi / n_m) o(g,p) and dwV[p] = sum of the workgroups' partials: one
// wave per tap p, lanes over g (resp. workgroups), fixed butterfly.
__global__ __launch_bounds__(64) void surr_bwd_params(int n_m, int N, int H, int nblk,
                                                      const double* __restrict__ du, SurrWS w,
                                                      float* __restrict__ dwV, float* __restrict__ dwT) {
    const int Pm = n_m / 2, p = blockIdx.x, lane = threadIdx.x;
    double a = 0.0, sv = 0.0;
    for (int g = lane; g < H; g += 64) a += du[g] * (two_pi_over(n_m) * (double)(-Pm + N * g + p));
    for (int k = lane; k < nblk; k += 64) sv += (double)w.wVpart[(long)k * N + p];
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        sv += __shfl_xor(sv, o, 64);
    }
    if (lane == 0) {
        dwT[p] = (float)a;
        dwV[p] = (float)sv;
    }
}

// dV[b][l] += sum over rows i of potential b, groups g and taps p with
// clamp(i + o(g,p)) = l of GA[i][g] wV[p]  (all-cells layout: row = b * nx + i).
__global__ void surr_bwd_dV(int B, int nx, int P, int N, int H, const float* __restrict__ wV,
                            const float* __restrict__ GA, double* __restrict__ dV) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)B * nx) return;
    const long b = idx / nx;
    const int l = (int)(idx - b * nx);
    const float* ga = GA + b * (long)nx * H;
    double acc = 0.0;
    for (int g = 0; g < H; ++g)
        for (int p = 0; p < N; ++p) {
            const int o = -P + N * g + p;
            if (l > 0 && l < nx - 1) {
                const int i = l - o;
                if (i >= 0 && i < nx) acc += (double)ga[(long)i * H + g] * (double)wV[p];
            } else {
                // edge cell: every row whose (clamped) tap lands here
                for (int i = 0; i < nx; ++i) {
                    const int q = min(max(i + o, 0), nx - 1);
                    if (q == l) acc += (double)ga[(long)i * H + g] * (double)wV[p];
                }
            }
        }
    dV[idx] += acc;
}

static int surr_check(const wk_mesh* mesh, int N, int* H) {
    WK_REQUIRE(mesh && mesh->dim == 1 && mesh->ny == 1 && mesh->nx > 0, "surrogate: 1-D meshes only");
    WK_REQUIRE(mesh->n_m >= 2 && mesh->n_m % 2 == 0, "surrogate: n_m must be even");
    WK_REQUIRE(N >= 1 && (N & (N - 1)) == 0 && mesh->n_m % N == 0 && N <= SU_MAXN,
               "surrogate: N must be a power of two dividing n_m");
    *H = mesh->n_m / N;
    WK_REQUIRE(*H <= SU_MAXH, "surrogate: hidden width too large");
    return WK_OK;
}

static long surr_nblk(long R) {
    const long t = (R + SD_BM - 1) / SD_BM;
    return t < SB_MAXBLK ? t : SB_MAXBLK;
}

static size_t surr_ws_bytes(int H, int P, int N, long R, bool with_GA) {
    const long nblk = surr_nblk(R);
    const int Pn = (P + 15) / 16 * 16;
    size_t b = 0;
    b += sizeof(float) * (size_t)nblk * H * P;
    b += sizeof(float) * (size_t)nblk * N;
    b += with_GA ? sizeof(float) * (size_t)R * H : 0;
    b += 2 * sizeof(double) * H + sizeof(double) * (size_t)H * Pn + sizeof(float) * (size_t)H * Pn;
    b += sizeof(double) * Pn + sizeof(float) * Pn;
    return b + 8 * 256;
}

static SurrWS surr_carve(void* ws, int H, int P, int N, long R, bool with_GA) {
    const long nblk = surr_nblk(R);
    const int Pn = (P + 15) / 16 * 16;
    char* p = static_cast<char*>(ws);
    auto take = [&](size_t n) {
        char* q = p;
        p += (n + 255) / 256 * 256;
        return q;
    };
    SurrWS w;
    w.GBpart = reinterpret_cast<float*>(take(sizeof(float) * (size_t)nblk * H * P));
    w.wVpart = reinterpret_cast<float*>(take(sizeof(float) * (size_t)nblk * N));
    w.GA = with_GA ? reinterpret_cast<float*>(take(sizeof(float) * (size_t)R * H)) : nullptr;
    w.u = reinterpret_cast<double*>(take(sizeof(double) * H));
    w.du = reinterpret_cast<double*>(take(sizeof(double) * H));
    w.Bd = reinterpret_cast<double*>(take(sizeof(double) * (size_t)H * Pn));
    w.Bf = reinterpret_cast<float*>(take(sizeof(float) * (size_t)H * Pn));
    w.Pid = reinterpret_cast<double*>(take(sizeof(double) * Pn));
    w.Pif = reinterpret_cast<float*>(take(sizeof(float) * Pn));
    return w;
}

// Scratch of the forward: the Bm / Pi tables of the prep kernel (the backward's prep section)
// followed by the transposed FP32 and BF16 copies of Bm.
static size_t surr_fwd_ws_bytes(int H, int P, int N) {
    const int Pn = (P + 15) / 16 * 16, Hk = (H + 31) / 32 * 32;
    const size_t prep = (surr_ws_bytes(H, P, N, 0, false) + 255) / 256 * 256;
    return prep + (size_t)Pn * Hk * (sizeof(float) + sizeof(uint16_t));
}

// Validation shared by the forward entry points; *H receives n_m / N.
int surr_fwd_check(const wk_mesh* mesh, int N, const float* wV, const float* wT, const float* W,
                   const double* V, int B, const int32_t* cells, int n_cells, int prec, void* K_out,
                   int* H) {
    int rc = surr_check(mesh, N, H);
    if (rc) return rc;
    WK_REQUIRE(B >= 0 && n_cells >= 0, "wk_surrogate_fwd: negative size");
    WK_REQUIRE(prec == WK_FP64 || prec == WK_FP32 || prec == WK_BF16,
               "wk_surrogate_fwd: prec must be WK_FP64, WK_FP32 or WK_BF16");
    if ((long)B * n_cells == 0) return WK_OK;
    WK_REQUIRE(cells != nullptr || n_cells == mesh->nx,
               "wk_surrogate_fwd: with cells == NULL, n_cells must be nx");
    WK_REQUIRE(wV && wT && W && V && K_out, "wk_surrogate_fwd: NULL array");
    return WK_OK;
}

size_t surr_fwd_scratch_bytes(const wk_mesh* mesh, int N) {
    int H;
    if (surr_check(mesh, N, &H) != WK_OK) return 0;
    return surr_fwd_ws_bytes(H, mesh->n_m / 2, N);
}

// The forward on validated arguments with `scratch` (surr_fwd_scratch_bytes bytes) as the
// prep tables' memory.
int surr_fwd_run(const wk_mesh* mesh, int N, int H, const float* wV, const float* wT, const float* W,
                 const double* V, int B, const int32_t* cells, int n_cells, int prec, void* K_out,
                 void* scratch, hipStream_t s) {
    if ((long)B * n_cells == 0) return WK_OK;
    const int P = mesh->n_m / 2, Pn = (P + 15) / 16 * 16;
    const long R = (long)B * n_cells;
    // prep tables, then the transposed copies of Bm
    const int Hk = (H + 31) / 32 * 32;
    const size_t prep = (surr_ws_bytes(H, P, N, 0, false) + 255) / 256 * 256;
    SurrWS w = surr_carve(scratch, H, P, N, 0, false);
    float* Btf = reinterpret_cast<float*>(static_cast<char*>(scratch) + prep);
    uint16_t* Btb = reinterpret_cast<uint16_t*>(Btf + (size_t)Pn * Hk);
    const long np = (long)H * Pn > Pn ? (long)H * Pn : Pn;
    hipLaunchKernelGGL(surr_prep, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, mesh->n_m, N,
                       H, Pn, wT, W, w.Bd, w.Bf, w.Pid, w.Pif, w.u);
    if (prec == WK_FP64) {
        const size_t sh = sizeof(double) * SD_BM * (H + 1);
        hipLaunchKernelGGL(surr_fwd_f64, dim3((unsigned)((R + SD_BM - 1) / SD_BM)), dim3(SU_THREADS), sh, s, V, mesh->nx, R, n_cells,
                           cells, P, N, H, Pn, wV, w.Bd, w.Pid, static_cast<double*>(K_out));
    } else {
        const long nt = (long)Pn * Hk;
        hipLaunchKernelGGL(surr_prep_t, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, H, Hk, Pn,
                           w.Bf, Btf, Btb);
        const long ntiles = (R + SF_BM - 1) / SF_BM;
        const bool bf = prec == WK_BF16;
        // the LDS-resident form only where two workgroups fit per CU (one per CU leaves each
        // tile's load, convolution and stores without overlap: slower than streaming Bt)
        size_t lds = surr_fwd_lds_bytes(bf, Hk, Pn, P);
        if (lds > 76 * 1024) lds = 0;
        if (lds) {
            const long per_cu = lds <= 50 * 1024 ? 3 : 2;
            const long g = 256 * per_cu;
            const dim3 gl((unsigned)(ntiles < g ? ntiles : g));
#define SURR_LDS(BFV, HKV)                                                                           \
    do {                                                                                             \
        auto* fn = surr_fwd_lds<BFV, HKV>;                                                           \
        if (lds > 64 * 1024 &&                                                                        \
            hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,        \
                                (int)lds) != hipSuccess)                                             \
            return fail(WK_EHIP, "wk_surrogate_fwd: cannot reserve LDS");                            \
        hipLaunchKernelGGL(fn, gl, dim3(SU_THREADS), lds, s, V, mesh->nx, R, n_cells, cells, P, N, H, \
                           Pn, wV, Btf, Btb, w.Pif, static_cast<float*>(K_out));                    \
    } while (0)
            if (bf) {
                if (Hk == 32) SURR_LDS(true, 32);
                else if (Hk == 64) SURR_LDS(true, 64);
                else if (Hk == 128) SURR_LDS(true, 128);
                else SURR_LDS(true, 256);
            } else {
                if (Hk == 32) SURR_LDS(false, 32);
                else if (Hk == 64) SURR_LDS(false, 64);
                else if (Hk == 128) SURR_LDS(false, 128);
                else SURR_LDS(false, 256);
            }
#undef SURR_LDS
            return check_launch("wk_surrogate_fwd");
        }
        const dim3 grid((unsigned)(ntiles < 4096 ? ntiles : 4096));
        // A [SF_BM][Hk + 8] (bf16) or [SF_BM][Hk + 4] (f32), then the potential window or,
        // for gathered rows, an FP32 staging copy of A
        const size_t a_bytes = prec == WK_BF16 ? sizeof(uint16_t) * SF_BM * (Hk + 8)
                                               : sizeof(float) * SF_BM * (Hk + 4);
        const size_t w_bytes = sizeof(double) * (SF_BM + 2 * P);
        const size_t g_bytes = sizeof(float) * SF_BM * (Hk + 1);
        const size_t sh = (a_bytes + 7) / 8 * 8 + (w_bytes > g_bytes ? w_bytes : g_bytes);
        if (prec == WK_BF16)
            hipLaunchKernelGGL(surr_fwd_mfma<true>, grid, dim3(SU_THREADS), sh, s, V, mesh->nx, R,
                               n_cells, cells, P, N, H, Hk, Pn, wV, Btf, Btb, w.Pif,
                               static_cast<float*>(K_out));
        else
            hipLaunchKernelGGL(surr_fwd_mfma<false>, grid, dim3(SU_THREADS), sh, s, V, mesh->nx, R,
                               n_cells, cells, P, N, H, Hk, Pn, wV, Btf, Btb, w.Pif,
                               static_cast<float*>(K_out));
    }
    return check_launch("wk_surrogate_fwd");
}
}  // namespace wk

using namespace wk;

extern "C" size_t wk_surrogate_fwd_workspace(const wk_mesh* mesh, int32_t N) {
    return surr_fwd_scratch_bytes(mesh, N);
}

extern "C" int wk_surrogate_fwd(const wk_mesh* mesh, int32_t N, const float* wV, const float* wT,
                                const float* W, const double* V, int32_t B,
                                const int32_t* cells, int32_t n_cells, int32_t prec, void* K_out,
                                void* ws, size_t ws_bytes, void* stream) {
    int H;
    int rc = surr_fwd_check(mesh, N, wV, wT, W, V, B, cells, n_cells, prec, K_out, &H);
    if (rc) return rc;
    if ((long)B * n_cells == 0) return WK_OK;
    WK_REQUIRE(ws && ws_bytes >= surr_fwd_scratch_bytes(mesh, N), "wk_surrogate_fwd: workspace too small");
    return surr_fwd_run(mesh, N, H, wV, wT, W, V, B, cells, n_cells, prec, K_out, ws, as_stream(stream));
}

extern "C" size_t wk_surrogate_workspace(const wk_mesh* mesh, int32_t N, int32_t B, int32_t n_cells) {
    int H;
    if (surr_check(mesh, N, &H) != WK_OK || B < 0 || n_cells < 0) return 0;
    return surr_ws_bytes(H, mesh->n_m / 2, N, (long)B * n_cells, true);
}

extern "C" int wk_surrogate_bwd(const wk_mesh* mesh, int32_t N, const float* wV, const float* wT,
                                const float* W, const double* V, int32_t B, const int32_t* cells,
                                int32_t n_cells, const float* E, float* dwV, float* dwT, float* dW,
                                double* dV, void* ws, size_t ws_bytes, void* stream) {
    int H;
    int rc = surr_check(mesh, N, &H);
    if (rc) return rc;
    WK_REQUIRE(B >= 0 && n_cells >= 0, "wk_surrogate_bwd: negative size");
    WK_REQUIRE(dwV && dwT && dW, "wk_surrogate_bwd: NULL gradient array");
    WK_REQUIRE(cells != nullptr || n_cells == mesh->nx,
               "wk_surrogate_bwd: with cells == NULL, n_cells must be nx");
    WK_REQUIRE(dV == nullptr || cells == nullptr, "wk_surrogate_bwd: dV needs the all-cells layout");
    const int P = mesh->n_m / 2, Pn = (P + 15) / 16 * 16;
    const long R = (long)B * n_cells;
    WK_REQUIRE(ws && ws_bytes >= surr_ws_bytes(H, P, N, R, true), "wk_surrogate_bwd: workspace too small");
    WK_REQUIRE(R == 0 || (wV && wT && W && V && E), "wk_surrogate_bwd: NULL array");
    hipStream_t s = as_stream(stream);
    SurrWS w = surr_carve(ws, H, P, N, R, true);
    const long np = (long)H * Pn;
    hipLaunchKernelGGL(surr_prep, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, mesh->n_m, N,
                       H, Pn, wT, W, w.Bd, w.Bf, w.Pid, w.Pif, w.u);
    long nblk = surr_nblk(R);
    const size_t lds = surr_bwd_mfma_bytes(H, P, N);
    if (nblk > 0 && lds) {
        // persistent workgroups (at most the partial slots the workspace holds)
        const long per_cu = lds <= 76 * 1024 ? 2 : 1;
        const long tiles = (R + SBM - 1) / SBM;
        nblk = min(nblk, min(tiles, 256 * per_cu));
        if (lds > 64 * 1024 &&
            hipFuncSetAttribute((const void*)surr_bwd_mfma, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds) != hipSuccess)
            return fail(WK_EHIP, "wk_surrogate_bwd: cannot reserve LDS");
        const int Hp = (H + 15) / 16 * 16, Pp = (P + 15) / 16 * 16;
        hipLaunchKernelGGL(surr_bwd_mfma, dim3((unsigned)nblk), dim3(SU_THREADS), lds, s, V, mesh->nx, R,
                           n_cells, cells, P, N, H, Pn, Hp, Pp, wV, E, w, dV ? 1 : 0);
    } else if (nblk > 0) {
        const size_t sh = sizeof(float) * SD_BM * (2 * (H + 1) + (P + 1));
        hipLaunchKernelGGL(surr_bwd_block, dim3((unsigned)nblk), dim3(SU_THREADS), sh, s, V,
                           mesh->nx, R, n_cells, cells, P, N, H, Pn, wV, E, w, dV ? 1 : 0);
    }
    if (nblk > 0) {
        hipLaunchKernelGGL(surr_bwd_reduce_gb, dim3((unsigned)(((long)H * P + 63) / 64)), dim3(64 * RG_WAVES),
                           0, s, (int)nblk, H, P, w);
        hipLaunchKernelGGL(surr_bwd_params_g, dim3((unsigned)H), dim3(256), 0, s, P, W, w, dW, w.du);
        hipLaunchKernelGGL(surr_bwd_params, dim3((unsigned)N), dim3(64), 0, s, mesh->n_m, N, H, (int)nblk, w.du,
                           w, dwV, dwT);
    } else {
        hipLaunchKernelGGL(zero_grads, dim3(1), dim3(256), 0, s, dwV, N, dwT, N, dW, H);
    }
    if (dV && R > 0)
        hipLaunchKernelGGL(surr_bwd_dV, dim3((unsigned)((R + 255) / 256)), dim3(256), 0, s, B,
                           mesh->nx, P, N, H, wV, w.GA, dV);
    return check_launch("wk_surrogate_bwd");
}

// ----------------------------------------------------------------------------- training ops
namespace wk {
__global__ void mse_partial(const float* __restrict__ Kh, const double* __restrict__ K, long n,
                            double inv_scale, float* __restrict__ E, double* __restrict__ part) {
    __shared__ double red[4];
    const double inv_n = 1.0 / (double)n;
    double acc = 0.0;
    // four elements per thread and step, their loads issued together
    const long stride = (long)gridDim.x * blockDim.x;
    for (long i0 = (long)blockIdx.x * blockDim.x + threadIdx.x; i0 < n; i0 += 4 * stride) {
        float kh[4];
        double k[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const long i = i0 + q * stride;
            kh[q] = i < n ? Kh[i] : 0.f;
            k[q] = i < n ? K[i] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const long i = i0 + q * stride;
            if (i < n) {
                const double d = ((double)kh[q] - k[q]) * inv_scale;
                acc += d * d;
                E[i] = (float)(2.0 * d * inv_scale * inv_n);
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// One wave: lane l sums the partials l, l + 64, ..., then a fixed butterfly (deterministic).
__global__ void mse_final(const double* __restrict__ part, int nb, long n, double* loss) {
    const int lane = threadIdx.x;
    double s = 0.0;
    for (int k = lane; k < nb; k += 64) s += part[k];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) loss[0] = s / (double)(n > 0 ? n : 1);
}

__global__ void sgd_kernel(float* w, const float* g, int n, float lr) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) w[i] = w[i] - lr * g[i];
}
}  // namespace wk

extern "C" int wk_mse_grad(const float* Kh, const double* K, int64_t count, double inv_scale,
                           float* E, double* loss, void* ws, size_t ws_bytes, void* stream) {
    WK_REQUIRE(count >= 0, "wk_mse_grad: negative count");
    WK_REQUIRE(loss && ws && ws_bytes >= 8 * 1024, "wk_mse_grad: NULL loss or small workspace");
    WK_REQUIRE(count == 0 || (Kh && K && E), "wk_mse_grad: NULL array");
    hipStream_t s = as_stream(stream);
    if (count == 0) {
        hipLaunchKernelGGL(mse_final, dim3(1), dim3(64), 0, s, static_cast<double*>(ws), 0, 1, loss);
        return check_launch("wk_mse_grad");
    }
    const int nb = 1024;
    hipLaunchKernelGGL(mse_partial, dim3(nb), dim3(256), 0, s, Kh, K, (long)count, inv_scale, E,
                       static_cast<double*>(ws));
    hipLaunchKernelGGL(mse_final, dim3(1), dim3(64), 0, s, static_cast<double*>(ws), nb, (long)count, loss);
    return check_launch("wk_mse_grad");
}

extern "C" int wk_sgd_update(float* w, const float* grad, int32_t n, float lr, void* stream) {
    WK_REQUIRE(n >= 0, "wk_sgd_update: negative size");
    if (n == 0) return WK_OK;
    WK_REQUIRE(w && grad, "wk_sgd_update: NULL array");
    hipLaunchKernelGGL(sgd_kernel, dim3((n + 255) / 256), dim3(256), 0, as_stream(stream), w, grad, n, lr);
    return check_launch("wk_sgd_update");
}

// ----------------------------------------------------------------------------- d = 2 forward
// eq.(5) in d = 2: the window of a cell on the periodic grid (o_a in [-P, P), the end point -P
// holding the mean of the two end values, where the d = 2 kernel has its half weights) grouped
// N x N; G[gy][gx] = W[g] sum_p wV[p] Vt(o(g, p)) is contracted like the d = 2 kernel, with
// sin(ux mx + uy my) = sin(ux mx) cos(uy my) + cos(ux mx) sin(uy my):
//   stage 1  T[gy][n] = sum_gx G[gy][gx] Bx[gx][n],  Bx = [sin(ux mx) | cos(ux mx)]
//   stage 2  Kh[my][mx] = Pi(mx) Pi(my) sum_k A2[my][k] T'[k][mx],  A2 = [cos(uy my) | sin(uy my)],
// both on v_mfma_f64_16x16x4; the trig operands depend on the weights and the lane only and are
// formed once per workgroup; workgroups loop over the requested cells.
namespace wk {
__device__ __forceinline__ double prefactor2(int L, int m, int n_m) {
    double pr = 1.0;
    for (int s = 0; s < L; ++s) pr *= cospi((double)(1 << s) * (double)m / (double)n_m);
    return pr;
}

template <int P, int N, bool TAB = false>
__global__ __launch_bounds__(256) void surr_fwd_2d_f64(
    const double* __restrict__ V, int nx, int ny, long R, int n_cells, const int32_t* __restrict__ cells,
    const float* __restrict__ wV, const float* __restrict__ wTx, const float* __restrict__ wTy,
    const float* __restrict__ W, double* __restrict__ out, TabOut tb) {
    constexpr int n_m = 2 * P, H = n_m / N, J = 2 * P + 1;
    constexpr int M1 = (H + 15) / 16 * 16, K1 = (H + 3) / 4 * 4, N1 = 2 * n_m;
    constexpr int NT1 = N1 / 16, MT1 = M1 / 16, NT1W = (NT1 + 3) / 4;
    constexpr int M2 = (n_m + 15) / 16 * 16, N2 = M2, K2 = 2 * K1, T2 = (M2 / 16) * (N2 / 16);
    static_assert(T2 <= 4, "one stage-2 tile per wave");
    int L = 0;
    while ((1 << L) < N) ++L;

    __shared__ double Wv[J][J + 1];
    __shared__ double Gs[M1][K1 + 1];
    __shared__ double Ts[K2][N2 + 1];
    __shared__ double ux[H], uy[H];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const double two_pi = 6.283185307179586476925286766559;
    for (int g = threadIdx.x; g < H; g += 256) {
        double a = 0.0, b = 0.0;
        for (int p = 0; p < N; ++p) {
            a += (double)wTx[p] * (two_pi * (double)(-P + N * g + p) / (double)n_m);
            b += (double)wTy[p] * (two_pi * (double)(-P + N * g + p) / (double)n_m);
        }
        ux[g] = a;
        uy[g] = b;
    }
    for (int e = threadIdx.x; e < K2 * (N2 + 1); e += 256) (&Ts[0][0])[e] = 0.0;
    __syncthreads();
    double b1[NT1W][K1 / 4];
#pragma unroll
    for (int q = 0; q < NT1W; ++q) {
        const int nt = wave + 4 * q;
#pragma unroll
        for (int ks = 0; ks < K1 / 4; ++ks) {
            const int gx = 4 * ks + lk, n = nt * 16 + lr;
            double v = 0.0;
            if (nt < NT1 && gx < H) {
                const int mx = (n < n_m ? n : n - n_m) - P;
                v = n < n_m ? sin(ux[gx] * (double)mx) : cos(ux[gx] * (double)mx);
            }
            b1[q][ks] = v;
        }
    }
    const int tm2 = wave / (N2 / 16), tn2 = wave % (N2 / 16);
    double a2[K2 / 4];
#pragma unroll
    for (int ks = 0; ks < K2 / 4; ++ks) {
        const int k = 4 * ks + lk, my_i = tm2 * 16 + lr;
        double v = 0.0;
        if (wave < T2 && my_i < n_m) {
            const int my = my_i - P, gy = k < K1 ? k : k - K1;
            if (gy < H) v = k < K1 ? cos(uy[gy] * (double)my) : sin(uy[gy] * (double)my);
        }
        a2[ks] = v;
    }
    for (long r = blockIdx.x; r < R; r += gridDim.x) {
        const long b = r / n_cells;
        const int ci = (int)(r - b * n_cells);
        int cell = cells ? cells[ci] : ci;
        const bool bad = cell < 0 || cell >= nx * ny;
        if (bad) cell = 0;
        const int cx = cell % nx, cy = cell / nx;
        const double* Vb = V + b * (long)nx * ny;
        __syncthreads();  // previous cell's LDS use is over
        for (int e = threadIdx.x; e < J * J; e += 256) {
            const int ty = e / J, tx = e - ty * J;
            const int yy = min(max(cy - P + ty, 0), ny - 1), xx = min(max(cx - P + tx, 0), nx - 1);
            Wv[ty][tx] = Vb[(long)yy * nx + xx];
        }
        __syncthreads();
        // G = W * (grouped, weighted window); window index o + P, the end point -P (index 0)
        // holds the mean with index 2P along that axis
        for (int e = threadIdx.x; e < M1 * K1; e += 256) {
            const int gy = e / K1, gx = e - gy * K1;
            double gv = 0.0;
            if (gy < H && gx < H) {
                double acc = 0.0;
                for (int py = 0; py < N; ++py) {
                    const int oy = N * gy + py;
                    for (int px = 0; px < N; ++px) {
                        const int ox = N * gx + px;
                        double v;
                        if (ox == 0 && oy == 0)
                            v = 0.25 * (((Wv[0][0] + Wv[0][2 * P]) + Wv[2 * P][0]) + Wv[2 * P][2 * P]);
                        else if (ox == 0)
                            v = 0.5 * (Wv[oy][0] + Wv[oy][2 * P]);
                        else if (oy == 0)
                            v = 0.5 * (Wv[0][ox] + Wv[2 * P][ox]);
                        else
                            v = Wv[oy][ox];
                        acc += (double)wV[py * N + px] * v;
                    }
                }
                gv = (double)W[gy * H + gx] * acc;
            }
            Gs[gy][gx] = bad ? __builtin_nan("") : gv;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NT1W; ++q) {
            const int nt = wave + 4 * q;
            if (nt >= NT1) continue;
#pragma unroll
            for (int mt = 0; mt < MT1; ++mt) {
                f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int ks = 0; ks < K1 / 4; ++ks)
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Gs[mt * 16 + lr][4 * ks + lk], b1[q][ks], acc, 0, 0, 0);
                const int n = nt * 16 + lr;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int gy = mt * 16 + lk + 4 * e;
                    if (gy >= K1) continue;
                    if (n < n_m)
                        Ts[gy][n] = acc[e];
                    else
                        Ts[K1 + gy][n - n_m] = acc[e];
                }
            }
        }
        __syncthreads();
        if (wave < T2) {
            f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
            const int mx_i = tn2 * 16 + lr;
#pragma unroll
            for (int ks = 0; ks < K2 / 4; ++ks)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[ks], Ts[4 * ks + lk][mx_i], acc, 0, 0, 0);
            // TAB: the row stays on chip, in the window tile (free once the groups are formed)
            double* o = TAB ? &Wv[0][0] : out + r * (long)n_m * n_m;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int my_i = tm2 * 16 + lk + 4 * e;
                if (my_i < n_m && mx_i < n_m)
                    o[my_i * n_m + mx_i] = prefactor2(L, mx_i - P, n_m) * prefactor2(L, my_i - P, n_m) * acc[e];
            }
        }
        if constexpr (TAB) {
            static_assert(J * (J + 1) >= n_m * n_m, "2-D row stage");
            __shared__ int last_s;
            tab_row_block(&Wv[0][0], n_m * n_m, r, tb, &last_s);
        }
    }
}
}  // namespace wk

namespace wk {
static int surr_2d_check(const wk_mesh* mesh, int N, int B, int n_cells, const int32_t* cells, const char* who) {
    if (!(mesh && mesh->dim == 2 && mesh->nx > 0 && mesh->ny > 0)) return fail(WK_EINVAL, std::string(who) + ": 2-D mesh needed");
    if (!(mesh->n_m == 8 || mesh->n_m == 16 || mesh->n_m == 32))
        return fail(WK_EINVAL, std::string(who) + ": n_m must be 8, 16 or 32");
    if (!(N >= 1 && (N & (N - 1)) == 0 && N <= 8 && N < mesh->n_m))
        return fail(WK_EINVAL, std::string(who) + ": N must be 1, 2, 4 or 8 and below n_m");
    if (B < 0 || n_cells < 0) return fail(WK_EINVAL, std::string(who) + ": negative size");
    if ((long)B * n_cells == 0) return WK_OK;
    if (!(cells != nullptr || n_cells == mesh->nx * mesh->ny))
        return fail(WK_EINVAL, std::string(who) + ": with cells == NULL, n_cells must be the number of cells");
    return WK_OK;
}

// eq.(5) in d = 2 on R = B n_cells rows: written out (TAB = false) or turned into the
// creation tables on chip (TAB).
template <bool TAB>
static int surr_2d_launch(const wk_mesh* mesh, int N, const float* wV, const float* wTx, const float* wTy,
                          const float* W, const double* V, int B, const int32_t* cells, int n_cells,
                          double* K_out, const TabOut& tb, hipStream_t s) {
    const long R = (long)B * n_cells;
    const unsigned grid = (unsigned)(R < 4096 ? R : 4096);
    const char* name = TAB ? "surr_tables_2d_f64" : "surr_fwd_2d_f64";
#define S2D(PP, NN)                                                                                       \
    WK_LAUNCH(name, (surr_fwd_2d_f64<PP, NN, TAB>), dim3(grid), dim3(256), 0, s, V, mesh->nx,             \
              mesh->ny, R, n_cells, cells, wV, wTx, wTy, W, K_out, tb)
#define S2D_N(PP)            \
    switch (N) {             \
        case 1: S2D(PP, 1); break; \
        case 2: S2D(PP, 2); break; \
        case 4: S2D(PP, 4); break; \
        default: S2D(PP, 8); break; \
    }
    if (mesh->n_m == 8) {
        S2D_N(4)
    } else if (mesh->n_m == 16) {
        S2D_N(8)
    } else {
        S2D_N(16)
    }
#undef S2D_N
#undef S2D
    return check_launch(name);
}
}  // namespace wk

extern "C" int wk_surrogate_fwd_2d(const wk_mesh* mesh, int32_t N, const float* wV, const float* wTx,
                                   const float* wTy, const float* W, const double* V, int32_t B,
                                   const int32_t* cells, int32_t n_cells, double* K_out, void* stream) {
    const int rc = wk::surr_2d_check(mesh, N, B, n_cells, cells, "wk_surrogate_fwd_2d");
    if (rc != WK_OK || (long)B * n_cells == 0) return rc;
    WK_REQUIRE(wV && wTx && wTy && W && V && K_out, "wk_surrogate_fwd_2d: NULL array");
    return wk::surr_2d_launch<false>(mesh, N, wV, wTx, wTy, W, V, B, cells, n_cells, K_out, wk::TabOut{},
                                     wk::as_stream(stream));
}

extern "C" int wk_surrogate_tables_2d(const wk_mesh* mesh, int32_t N, const float* wV, const float* wTx,
                                      const float* wTy, const float* W, const double* V, int32_t B,
                                      const int32_t* cells, int32_t n_cells, double dt, double* gamma,
                                      uint32_t* n0, uint32_t* thr, uint64_t* cdf, uint32_t* guide,
                                      int32_t guide_len, void* stream) {
    const int rc = wk::surr_2d_check(mesh, N, B, n_cells, cells, "wk_surrogate_tables_2d");
    if (rc != WK_OK || (long)B * n_cells == 0) return rc;
    WK_REQUIRE(dt >= 0.0, "wk_surrogate_tables_2d: dt must be >= 0");
    WK_REQUIRE(wV && wTx && wTy && W && V && gamma && n0 && thr && cdf, "wk_surrogate_tables_2d: NULL array");
    WK_REQUIRE(guide == nullptr || (guide_len >= 1 && guide_len <= wk::TAB_GMAX),
               "wk_surrogate_tables_2d: guide_len must lie in [1, 256]");
    const wk::TabOut tb{dt, gamma, n0, thr, cdf, guide, guide ? (int)guide_len : 0};
    return wk::surr_2d_launch<true>(mesh, N, wV, wTx, wTy, W, V, B, cells, n_cells, nullptr, tb,
                                    wk::as_stream(stream));
}

// ----------------------------------------------------------------------------- no-alloc forward
// Scratch of wk_surrogate_fwd_static: one file-scope device array per GPU.  In host code the
// array's name is a host-side stand-in, not a device address; the kernels only ever receive
// the address hipGetSymbolAddress returns for the current device, resolved once per device on
// the entry point's first call there.  Every call on a device shares that device's copy.
namespace wk {
constexpr size_t SURR_STATIC_BYTES = size_t(4) << 20;
static __device__ __align__(256) unsigned char scratch[SURR_STATIC_BYTES];

static void* static_scratch(int* err) {
    static std::mutex mu;
    static std::map<int, void*> addr;
    int dev = 0;
    *err = WK_OK;
    if (hipGetDevice(&dev) != hipSuccess) {
        *err = fail(WK_EHIP, "wk_surrogate_fwd_static: hipGetDevice failed");
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(dev);
    if (it != addr.end()) return it->second;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
        *err = fail(WK_EHIP, std::string("wk_surrogate_fwd_static: hipGetSymbolAddress: ") + hipGetErrorString(e));
        return nullptr;
    }
    addr[dev] = p;
    return p;
}
}  // namespace wk

extern "C" size_t wk_surrogate_fwd_static_max(void) { return wk::SURR_STATIC_BYTES; }

extern "C" int wk_surrogate_fwd_static(const wk_mesh* mesh, int32_t N, const float* wV, const float* wT,
                                       const float* W, const double* V, int32_t B,
                                       const int32_t* cells, int32_t n_cells, int32_t prec,
                                       void* K_out, void* stream) {
    int H;
    int rc = surr_fwd_check(mesh, N, wV, wT, W, V, B, cells, n_cells, prec, K_out, &H);
    if (rc) return rc;
    if ((long)B * n_cells == 0) return WK_OK;
    const size_t need = surr_fwd_scratch_bytes(mesh, N);
    if (need > SURR_STATIC_BYTES)
        return fail(WK_EINVAL, "wk_surrogate_fwd_static: n_m = " + std::to_string(mesh->n_m) + ", N = " +
                                   std::to_string(N) + " needs " + std::to_string(need) +
                                   " bytes of scratch, above the static " +
                                   std::to_string(SURR_STATIC_BYTES) + " (use wk_surrogate_fwd)");
    int err;
    void* ptr = static_scratch(&err);
    if (!ptr) return err;
    return surr_fwd_run(mesh, N, H, wV, wT, W, V, B, cells, n_cells, prec, K_out, ptr, as_stream(stream));
}
