// Wigner kernel of eq.(4) (Sec. 2.2) on requested cells as an MFMA contraction:
//   K[row][t] = c * sum_jj D[row][jj] * S[jj][t],  c = -2 / (hbar n_m),
//   D[row][jj] = V(i + jj + 1) - V(i - jj - 1)      (the potential difference operand),
//   S[jj][t]   = sin(2 pi (jj+1)(t+1) / n_m)        (the sine table, m = t + 1).
// D never exists in HBM: each workgroup builds its BM x BK slice in LDS from the potential
// (nearest-edge value outside the mesh); S comes from a per-device table (L2 resident).
#include "lowp.h"
#include "wk_internal.h"

namespace wk {

constexpr int KE_BK = 16;     // contraction depth staged per LDS tile (FP64)
constexpr int KE_THREADS = 256;
constexpr int KE_BM = 64;     // rows per workgroup
constexpr int KE_WIN = 64 + 2 * 512 + 8;   // LDS potential window (rows + 2P + 1), P <= 512

// Row r -> (offset of its potential in V, cell index) for the BM rows of a block, and
// whether the block's rows are consecutive cells of one potential (then they share one
// window of the potential, staged in LDS).
template <int BM>
__device__ __forceinline__ bool load_rows(long row0, long R, int n_cells, int nx, int P,
                                          const int32_t* __restrict__ cells, long* rbase,
                                          int* rcell) {
    for (int rr = threadIdx.x; rr < BM; rr += blockDim.x) {
        const long r = row0 + rr;
        long base = 0;
        int cell = -1;
        if (r < R) {
            const long b = r / n_cells;
            const int ci = (int)(r - b * n_cells);
            cell = cells ? cells[ci] : ci;
            if (cell < 0 || cell >= nx) cell = -2;  // id outside the mesh: row of NaN
            base = b * (long)nx;
        }
        rbase[rr] = base;
        rcell[rr] = cell;
    }
    return cells == nullptr && row0 + BM <= R && row0 / n_cells == (row0 + BM - 1) / n_cells &&
           BM + 2 * P + 1 <= KE_WIN;
}

// Potential window W[t] = V(c0 - P + t), t < BM + 2P + 1 (nearest-edge value outside).
template <int BM>
__device__ __forceinline__ void load_window(const double* __restrict__ V, long base, int c0, int nx,
                                            int P, double* Wv) {
    for (int t = threadIdx.x; t < BM + 2 * P + 1; t += blockDim.x)
        Wv[t] = V[base + min(max(c0 - P + t, 0), nx - 1)];
}

// D[rr][jj] = V(cell + jj + 1) - V(cell - jj - 1) for a row of the block (0 beyond P).
template <int BM>
__device__ __forceinline__ double d_elem(bool contig, const double* Wv, const double* __restrict__ V,
                                         const long* rbase, const int* rcell, int nx, int P, int rr,
                                         int j) {
    const int cell = rcell[rr];
    if (cell == -2) return __builtin_nan("");
    if (cell < 0 || j > P) return 0.0;
    if (contig) return Wv[rr + P + j] - Wv[rr + P - j];
    const double* Vb = V + rbase[rr];
    return Vb[min(cell + j, nx - 1)] - Vb[max(cell - j, 0)];
}


// Creation tables of nr rows staged in LDS (row q at lds + q SW holds the full row, entry t
// <-> m = t - P; grow(q) is its table row): exactly the arithmetic of the table kernels.  One
// lane per row sums the positive part in ascending m in FP64 (the order is the definition)
// and leaves the running sums in place, every lane converts them to the integer CDF, and
// (optionally) each bucket of the guide table is found by binary search over the CDF row.
// Lg holds the guide's bucket limits floor(k 2^32 / G); last_s one int per staged row.
template <typename GrowFn>
__device__ __forceinline__ void tab_rows(double* lds, int SW, int nr, GrowFn grow, int* last_s,
                                         const uint64_t* Lg, long R, int n_m, const TabOut& tb) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int q = threadIdx.x; q < nr; q += KE_THREADS) {  // one thread per row
        double* srow = lds + q * SW;
        double C = 0.0;
        int last = -1;
        for (int t = 0; t < n_m; ++t) {
            const double k = srow[t];
            if (k > 0.0) {
                C = C + k;
                last = t;
            }
            srow[t] = C;
        }
        last_s[q] = last;
        const long row = grow(q);
        if (row < R) {
            const double p = C * tb.dt;
            const double fl = floor(p);
            tb.gamma[row] = C;
            tb.n0[row] = (uint32_t)fl;
            tb.thr[row] = (uint32_t)floor((p - fl) * 4294967296.0);
        }
    }
    __syncthreads();
    // rows to waves, entries to lanes; each lane converts its own entries in place
    for (int q = wave; q < nr; q += KE_THREADS / 64) {
        const long row = grow(q);
        double* srow = lds + q * SW;
        const int last = last_s[q];
        const double g = last >= 0 ? srow[last] : 0.0;
        uint64_t* crow = tb.cdf + row * n_m;
        for (int t = lane; t < n_m; t += 64) {
            uint64_t v;
            if (last < 0)
                v = 0;
            else if (t >= last)
                v = 1ull << 32;
            else
                v = (uint64_t)floor(srow[t] / g * 4294967296.0);
            if (row < R) crow[t] = v;
            reinterpret_cast<uint64_t*>(srow)[t] = v;
        }
    }
    if (tb.guide == nullptr) return;
    __syncthreads();
    for (int q = wave; q < nr; q += KE_THREADS / 64) {
        const long row = grow(q);
        if (row >= R) continue;
        const uint64_t* T = reinterpret_cast<const uint64_t*>(lds + q * SW);
        uint32_t* gout = tb.guide + row * (tb.G + 1);
        for (int k = lane; k < tb.G; k += 64) {
            const uint64_t L = Lg[k];
            int lo = 0, hi = n_m - 1;  // first t with T[t] > L, at most n_m - 1
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (T[mid] > L)
                    hi = mid;
                else
                    lo = mid + 1;
            }
            gout[k] = (uint32_t)lo;
        }
        if (lane == 0) gout[tb.G] = (uint32_t)(n_m - 1);
    }
}

// Creation tables of eq.(1) from a workgroup's finished rows, which never leave the chip.
// The rows are staged in LDS as full rows, entry t <-> m = t - P, in groups of 8 (x WAVES_M)
// rows; the narrowest tiles (H <= 32) take as many groups per round as the operand tiles' LDS
// holds (three of four, 48 rows, at 80 momenta), the wider ones one group per round,
// with the values the kernel would have written (K(m) = c (O + E), K(P - m) = c (O - E),
// K(-m) = -K(m), K(0) = K(-P) = 0); then tab_rows.  One column block must hold every m of a
// row (H <= BN).
template <int WM, int WN, int WAVES_N>
__device__ __forceinline__ void tab_epilogue(const f64x4 (&acc)[2][WM][WN], double* lds, int lds_len,
                                             long row0, long R, int P, int n_m, int H, double c,
                                             const TabOut& tb) {
    constexpr int WAVES_M = 4 / WAVES_N;
    constexpr int SR = 8 * WAVES_M;   // rows of one (tm, eh) group: tile rows 8 eh + [0, 8) of
    constexpr int NG = 2 * WM;        // row tile tm in each wave row; NG groups per workgroup
    __shared__ int last_s[NG * SR];
    __shared__ uint64_t Lg[TAB_GMAX];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = wave / WAVES_N, wc = wave % WAVES_N;
    const int lr = lane & 15, lk = lane >> 4;
    const int SW = n_m + 1;  // odd row stride: the per-row lanes of the prefix hit distinct banks
    for (int k = threadIdx.x; k < tb.G; k += KE_THREADS) Lg[k] = ((uint64_t)k << 32) / (uint64_t)tb.G;
    // group gi = 2 tm + eh into staged rows slot SR + [0, SR): staged row slot SR + wr 8 + lk + 4 ee
    // holds tile row 8 eh + lk + 4 ee of row tile tm of wave row wr
    auto stage = [&](const int gi, const int slot) {
        const int tm = gi >> 1, eh = gi & 1;
#pragma unroll
        for (int tn = 0; tn < WN; ++tn) {
            const int t = (wc * WN + tn) * 16 + lr, m = t + 1;
#pragma unroll
            for (int ee = 0; ee < 2; ++ee) {
                double* srow = lds + (slot * SR + wr * 8 + lk + 4 * ee) * SW;
                if (t < H) {
                    const int e = 2 * eh + ee;
                    const double o = acc[0][tm][tn][e], ev = acc[1][tm][tn][e];
                    const double kp = c * (o + ev), km = c * (o - ev);
                    srow[P + m] = kp;
                    srow[P - m] = -kp;
                    if (2 * m < P) {
                        srow[2 * P - m] = km;
                        srow[m] = -km;
                    }
                }
                if (t == 0) {
                    srow[0] = 0.0;
                    srow[P] = 0.0;
                }
            }
        }
    };
    // tables of the nr staged rows of groups g0, g0 + 1, ...
    auto tables = [&](const int g0, const int nr) {
        auto grow = [&](int q) -> long {  // table row of staged row q
            const int gi = g0 + q / SR, qq = q % SR;
            return row0 + ((qq >> 3) * WM + (gi >> 1)) * 16 + 8 * (gi & 1) + (qq & 7);
        };
        tab_rows(lds, SW, nr, grow, last_s, Lg, R, n_m, tb);
    };
    if constexpr (WAVES_N == 4) {
        // the wider tiles (H > 32) hold one or two groups per round and are register bound:
        // straight-line rounds keep the accumulators' indices constant (and the occupancy)
#pragma unroll
        for (int gi = 0; gi < NG; ++gi) {
            __syncthreads();  // the previous round (or the contraction) is done with the LDS
            stage(gi, 0);
            __syncthreads();
            tables(gi, SR);
        }
    } else {
        // as many groups per round as the LDS holds (at least one: checked on the host)
        const int gpr = min(NG, lds_len / (SR * SW));
        for (int g0 = 0; g0 < NG; g0 += gpr) {  // uniform
            const int ng = min(gpr, NG - g0);
            __syncthreads();
#pragma unroll
            for (int gi = 0; gi < NG; ++gi)
                if (gi >= g0 && gi < g0 + ng) stage(gi, gi - g0);
            __syncthreads();
            tables(g0, ng * SR);
        }
    }
}

// FP64 path: v_mfma_f64_16x16x4_f64 on the folded sum.  With n_m = 2P the sine of eq.(4)
// obeys sin(2 pi j (P - m) / n_m) = -(-1)^j sin(2 pi j m / n_m), so splitting the sum over j
// into odd and even terms gives, for m = t + 1 <= H = floor(P / 2),
//   O[row][t] = sum_k So[k][t] D[row][2k + 1],   E[row][t] = sum_k Se[k][t] D[row][2k + 2],
//   K(m) = c (O + E),   K(P - m) = c (O - E),
// two H x H contractions per row in place of one (P - 1) x (P - 1): half the products
// (one radix-2 step of a fast sine transform; the tables obey the identity exactly, so the
// results differ from the direct sum by rounding order only).
// WAVES_N waves split the columns t, 4 / WAVES_N split the rows; each wave owns a
// (16 WM) x (16 WN) tile of both O and E.  Operand layouts (16x16x4 f64): lane l holds
// A[l % 16][l / 16], B[l / 16][l % 16], and C[l / 16 + 4 e][l % 16], e < 4.  The odd and even
// D tiles are double-buffered in LDS; the next chunk's tiles are built in four slices between
// the current chunk's sub-steps, and its sine fragments are loaded one chunk ahead.
template <int WM, int WN, int WAVES_N, bool TAB = false>
__global__ __launch_bounds__(KE_THREADS) void kernel_eval_f64(
    const double* __restrict__ V, int nx, long R, int n_cells, const int32_t* __restrict__ cells,
    int P, int n_m, int H, int Hk, int Hn, const double* __restrict__ So,
    const double* __restrict__ Se, double c, int layout, double* __restrict__ out, TabOut tb) {
    constexpr int WAVES_M = 4 / WAVES_N;
    constexpr int BM = 16 * WM * WAVES_M, BN = 16 * WN * WAVES_N, BK = KE_BK;
    static_assert(BM <= KE_BM, "row tile");
    __shared__ double Ds[2][2][BM][BK + 1];  // [buffer][0: odd j, 1: even j][row][k]
    __shared__ double Wv[KE_WIN];
    __shared__ long rbase[BM];
    __shared__ int rcell[BM];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = wave / WAVES_N, wc = wave % WAVES_N;
    const long row0 = (long)blockIdx.x * BM;
    const int col0 = blockIdx.y * BN;
    const int lr = lane & 15, lk = lane >> 4;

    const bool contig = load_rows<BM>(row0, R, n_cells, nx, P, cells, rbase, rcell);
    if (contig) load_window<BM>(V, (row0 / n_cells) * (long)nx, (int)(row0 % n_cells), nx, P, Wv);
    __syncthreads();

    // element e of a chunk's two tiles: part e / (BM BK), then row-major [BM][BK]; rows of
    // one window need no per-row lookups (offsets past P read the window at P, then give 0)
    auto put = [&](int e, int k0, int buf) {
        const int part = e / (BM * BK), rem = e - part * (BM * BK);
        const int rr = rem / BK, kk = rem - rr * BK;
        const int j = 2 * (k0 + kk) + 1 + part;
        double d;
        if (contig) {
            const int jc = min(j, P);
            d = Wv[rr + P + jc] - Wv[rr + P - jc];
            if (j > P) d = 0.0;
        } else {
            d = d_elem<BM>(false, Wv, V, rbase, rcell, nx, P, rr, j);
        }
        Ds[buf][part][rr][kk] = d;
    };

    f64x4 acc[2][WM][WN];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int a = 0; a < WM; ++a)
#pragma unroll
            for (int b = 0; b < WN; ++b) acc[p][a][b] = f64x4{0.0, 0.0, 0.0, 0.0};

    const long cw = (long)col0 + wc * WN * 16 + lr;
    const double* Sw[2] = {So + cw, Se + cw};
    // sine fragments: loaded one chunk ahead into bnext only (also before the loop), and
    // moved into bfrag at the top of each chunk, so that the loads of a chunk have a whole
    // chunk of products to arrive and no product waits on a load issued in its own chunk
    double bnext[2][BK / 4][WN];
    auto load_b = [&](int k0) {
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int ks = 0; ks < BK / 4; ++ks)
#pragma unroll
                for (int tn = 0; tn < WN; ++tn)
                    bnext[p][ks][tn] = Sw[p][(long)(k0 + 4 * ks + lk) * Hn + tn * 16];
    };
    load_b(0);
    for (int e = threadIdx.x; e < 2 * BM * BK; e += KE_THREADS) put(e, 0, 0);
    __syncthreads();
    __builtin_amdgcn_s_waitcnt(0);  // the prologue's loads have landed (see the 16-bit path)

    static_assert((2 * BM * BK) % (KE_THREADS * (BK / 4)) == 0, "build slices");
    constexpr int SLICE = 2 * BM * BK / (BK / 4);  // D elements per slice
    int buf = 0;
    for (int k0 = 0; k0 < Hk; k0 += BK) {
        const bool more = k0 + BK < Hk;
        double bfrag[2][BK / 4][WN];
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int ks = 0; ks < BK / 4; ++ks)
#pragma unroll
                for (int tn = 0; tn < WN; ++tn) bfrag[p][ks][tn] = bnext[p][ks][tn];
        if (more) load_b(k0 + BK);
        double afrag[2][WM], anext[2][WM];
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int tm = 0; tm < WM; ++tm) afrag[p][tm] = Ds[buf][p][(wr * WM + tm) * 16 + lr][lk];
#pragma unroll
        for (int ks = 0; ks < BK / 4; ++ks) {
            if (ks + 1 < BK / 4) {
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int tm = 0; tm < WM; ++tm)
                        anext[p][tm] = Ds[buf][p][(wr * WM + tm) * 16 + lr][4 * (ks + 1) + lk];
            }
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int tm = 0; tm < WM; ++tm)
#pragma unroll
                    for (int tn = 0; tn < WN; ++tn)
                        acc[p][tm][tn] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                            afrag[p][tm], bfrag[p][ks][tn], acc[p][tm][tn], 0, 0, 0);
            if (more)
                for (int e = ks * SLICE + threadIdx.x; e < (ks + 1) * SLICE; e += KE_THREADS)
                    put(e, k0 + BK, buf ^ 1);
            if (ks + 1 < BK / 4) {
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int tm = 0; tm < WM; ++tm) afrag[p][tm] = anext[p][tm];
            }
        }
        __syncthreads();
        buf ^= 1;
    }

    if constexpr (TAB) {
        tab_epilogue<WM, WN, WAVES_N>(acc, &Ds[0][0][0][0], 2 * 2 * BM * (BK + 1), row0, R, P, n_m,
                                      H, c, tb);
        return;
    }
#pragma unroll
    for (int tm = 0; tm < WM; ++tm) {
#pragma unroll
        for (int tn = 0; tn < WN; ++tn) {
            const int t = col0 + (wc * WN + tn) * 16 + lr, m = t + 1;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const long row = row0 + (wr * WM + tm) * 16 + lk + 4 * e;
                if (row >= R || t >= H) continue;
                const double o = acc[0][tm][tn][e], ev = acc[1][tm][tn][e];
                const double kp = c * (o + ev), km = c * (o - ev);
                const bool mirror = 2 * m < P;  // m = P / 2 (even P) is its own mirror
                if (layout == WK_HALF) {
                    double* h = out + row * P;  // entry m - 1 holds K(m), m = 1..P
                    h[m - 1] = kp;
                    if (mirror) h[P - m - 1] = km;
                    if (t == 0) h[P - 1] = 0.0;
                } else {
                    double* f = out + row * (long)n_m;  // entry P + m holds K(m), m = -P..P-1
                    f[P + m] = kp;
                    f[P - m] = -kp;
                    if (mirror) {
                        f[2 * P - m] = km;
                        f[m] = -km;
                    }
                    if (t == 0) {
                        f[0] = 0.0;
                        f[P] = 0.0;
                    }
                }
            }
        }
    }
}

// n_m = 2: every entry of eq.(4) is sin(pi j m) = 0.
__global__ void kernel_zero_f64(double* __restrict__ out, long n) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n) out[idx] = 0.0;
}

// Reduced-precision path: v_mfma_f32_16x16x32_{bf16,f16} with FP32 accumulation, on the same
// odd/even fold as the FP64 path (O and E accumulated separately, K(m) = c(O+E),
// K(P-m) = c(O-E)).  Layouts (16x16x32): lane l holds A[l % 16][8 (l / 16) + q],
// B[8 (l / 16) + q][l % 16] for q < 8, and C[4 (l / 16) + e][l % 16] for e < 4.  The potential
// differences are formed in FP64 and rounded to the 16-bit format (hi); the split forms also
// keep lo = d - hi, and sum hi*hi + hi*lo + lo*hi (the lo*lo term is below FP32 accumulation
// error).  The fold tables are read transposed, T[t][k], so each lane's eight B elements are
// one contiguous 16-byte load.
constexpr int LP_BK = 32;

template <int PREC>
struct LowpTraits;
template <>
struct LowpTraits<WK_BF16> {
    typedef bf16x8 vec;
    static constexpr bool split = false, half = false;
};
template <>
struct LowpTraits<WK_FP16> {
    typedef f16x8 vec;
    static constexpr bool split = false, half = true;
};
template <>
struct LowpTraits<WK_BF16X3> {
    typedef bf16x8 vec;
    static constexpr bool split = true, half = false;
};
template <>
struct LowpTraits<WK_FP16X3> {
    typedef f16x8 vec;
    static constexpr bool split = true, half = true;
};

template <bool HALF>
__device__ __forceinline__ f32x4 mfma16(const s16x8& a, const s16x8& b, f32x4 c) {
    if constexpr (HALF)
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                      __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// Creation tables from the 16-bit kernel's finished rows (the TAB form of kernel_eval_lowp),
// equal bit for bit to the table kernels run on the FP32 rows the kernel would have written:
// each entry is staged as that FP32 value (c (O + E), c (O - E) in FP32), widened to FP64.
// Accumulator layout of v_mfma_f32_16x16x32: lane l holds C[4 (l / 16) + e][l % 16], e < 4.
// Group gi = 2 tm + eh stages the tile rows 4 lk + 2 eh + ee (ee < 2) of row tile tm of every
// wave row: staged row wr 8 + 2 lk + ee.  One round per group (the LDS holds 8 WAVES_M rows
// of up to 4 BN + 3 entries); one column block holds every m of a row (H <= BN).
template <int WM, int WN, int WAVES_N>
__device__ __forceinline__ void tab_epilogue_lowp(const f32x4 (&acc)[2][WM][WN], double* lds, long row0,
                                                  long R, int P, int n_m, int H, float c,
                                                  const TabOut& tb) {
    constexpr int WAVES_M = 4 / WAVES_N;
    constexpr int SR = 8 * WAVES_M;
    constexpr int NG = 2 * WM;
    __shared__ int last_s[SR];
    __shared__ uint64_t Lg[TAB_GMAX];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = wave / WAVES_N, wc = wave % WAVES_N;
    const int lr = lane & 15, lk = lane >> 4;
    const int SW = n_m + 1;
    for (int k = threadIdx.x; k < tb.G; k += KE_THREADS) Lg[k] = ((uint64_t)k << 32) / (uint64_t)tb.G;
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
        const int tm = gi >> 1, eh = gi & 1;
        __syncthreads();  // the previous round (or the contraction) is done with the LDS
#pragma unroll
        for (int tn = 0; tn < WN; ++tn) {
            const int t = (wc * WN + tn) * 16 + lr, m = t + 1;
#pragma unroll
            for (int ee = 0; ee < 2; ++ee) {
                double* srow = lds + (wr * 8 + 2 * lk + ee) * SW;
                if (t < H) {
                    const int e = 2 * eh + ee;
                    const float o = acc[0][tm][tn][e], ev = acc[1][tm][tn][e];
                    const double kp = (double)(c * (o + ev)), km = (double)(c * (o - ev));
                    srow[P + m] = kp;
                    srow[P - m] = -kp;
                    if (2 * m < P) {
                        srow[2 * P - m] = km;
                        srow[m] = -km;
                    }
                }
                if (t == 0) {
                    srow[0] = 0.0;
                    srow[P] = 0.0;
                }
            }
        }
        __syncthreads();
        auto grow = [&](int q) -> long {  // q = wr 8 + 2 lk + ee -> tile row 4 lk + 2 eh + ee
            return row0 + ((q >> 3) * WM + tm) * 16 + 4 * ((q & 7) >> 1) + 2 * eh + (q & 1);
        };
        tab_rows(lds, SW, SR, grow, last_s, Lg, R, n_m, tb);
    }
}

template <int PREC, int WM, int WN, int WAVES_N, bool TAB = false>
__global__ __launch_bounds__(KE_THREADS) void kernel_eval_lowp(
    const double* __restrict__ V, int nx, long R, int n_cells, const int32_t* __restrict__ cells,
    int P, int n_m, int H, int Hk, const uint16_t* __restrict__ To_hi, const uint16_t* __restrict__ Te_hi,
    const uint16_t* __restrict__ To_lo, const uint16_t* __restrict__ Te_lo, float c, int layout,
    float* __restrict__ out, TabOut tb) {
    typedef LowpTraits<PREC> TR;
    constexpr int WAVES_M = 4 / WAVES_N;
    constexpr int BM = 16 * WM * WAVES_M, BN = 16 * WN * WAVES_N, BK = LP_BK, LD = BK + 8;
    constexpr int NS = TR::split ? 2 : 1;  // hi (and lo) tiles
    static_assert(BM == KE_BM, "row tile");
    // operand tiles [buffer][part][hi, lo][row][k] during the contraction; the same bytes stage
    // whole output rows afterwards (16 * WAVES_M rows of up to 2 BN + 4 floats)
    constexpr int OPS = 2 * 2 * NS * BM * LD * 2;
    constexpr int SP = 2 * BN + 4;
    constexpr int STG = 16 * WAVES_M * SP * 4;
    // TAB: rounds of 8 WAVES_M full FP64 rows of up to n_m + 1 = 4 BN + 3 entries (H <= BN)
    constexpr int TBS = TAB ? 8 * WAVES_M * (4 * BN + 3) * 8 : 0;
    constexpr int LDS1 = OPS > STG ? OPS : STG;
    __shared__ __attribute__((aligned(16))) char lds_ops[LDS1 > TBS ? LDS1 : TBS];
    auto Dt = reinterpret_cast<uint16_t(*)[2][NS][BM][LD]>(lds_ops);
    __shared__ double Wv[KE_WIN];
    __shared__ long rbase[BM];
    __shared__ int rcell[BM];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = wave / WAVES_N, wc = wave % WAVES_N;
    const long row0 = (long)blockIdx.x * BM;
    const int col0 = blockIdx.y * BN;
    const int lr = lane & 15, lk = lane >> 4;

    const bool contig = load_rows<BM>(row0, R, n_cells, nx, P, cells, rbase, rcell);
    if (contig) load_window<BM>(V, (row0 / n_cells) * (long)nx, (int)(row0 % n_cells), nx, P, Wv);
    __syncthreads();

    // group g of a step: part g / (BM BK/8), row g % BM, eight consecutive k; the 64 lanes of
    // a wave take 64 consecutive rows (window reads on distinct banks).  Offsets j = 2k+1+part.
    auto build = [&](int k0, int buf) {
        for (int g = threadIdx.x; g < 2 * BM * (BK / 8); g += KE_THREADS) {
            const int part = g / (BM * (BK / 8)), rem = g - part * (BM * (BK / 8));
            const int rr = rem % BM, kq = (rem / BM) * 8;
            const int j0 = 2 * (k0 + kq) + 1 + part;
            double d[8];
            if (contig && j0 + 14 <= P) {
                // one window, eight offsets in range: sixteen independent LDS reads
                const double* up = Wv + rr + P + j0;
                const double* dn = Wv + rr + P - j0;
#pragma unroll
                for (int q = 0; q < 8; ++q) d[q] = up[2 * q] - dn[-2 * q];
            } else if (contig) {  // offsets past P read the window at P, then give 0
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int j = j0 + 2 * q, jc = min(j, P);
                    const double v = Wv[rr + P + jc] - Wv[rr + P - jc];
                    d[q] = j > P ? 0.0 : v;
                }
            } else {
#pragma unroll
                for (int q = 0; q < 8; ++q) d[q] = d_elem<BM>(false, Wv, V, rbase, rcell, nx, P, rr, j0 + 2 * q);
            }
            // hi = round16(d); split forms also lo = round16(d - hi) (d - hi is exact in FP64)
            uint32_t hv[4], lv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                hv[q] = pack16<TR::half>(d[2 * q], d[2 * q + 1]);
                if constexpr (TR::split)
                    lv[q] = pack16<TR::half>(d[2 * q] - value16<TR::half>(hv[q] & 0xFFFFu),
                                             d[2 * q + 1] - value16<TR::half>(hv[q] >> 16));
            }
            *reinterpret_cast<uint4*>(&Dt[buf][part][0][rr][kq]) = make_uint4(hv[0], hv[1], hv[2], hv[3]);
            if constexpr (TR::split)
                *reinterpret_cast<uint4*>(&Dt[buf][part][NS - 1][rr][kq]) = make_uint4(lv[0], lv[1], lv[2], lv[3]);
        }
    };
    const uint16_t* Th[2] = {To_hi, Te_hi};
    const uint16_t* Tl[2] = {To_lo, Te_lo};
    auto load_b = [&](int k0, s16x8 (&bh)[2][WN], s16x8 (&bl)[2][WN]) {
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int tn = 0; tn < WN; ++tn) {
                const long off = (long)(col0 + (wc * WN + tn) * 16 + lr) * Hk + k0 + 8 * lk;
                bh[p][tn] = *reinterpret_cast<const s16x8*>(Th[p] + off);
                if constexpr (TR::split) bl[p][tn] = *reinterpret_cast<const s16x8*>(Tl[p] + off);
            }
    };

    f32x4 acc[2][WM][WN];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int a = 0; a < WM; ++a)
#pragma unroll
            for (int b = 0; b < WN; ++b) acc[p][a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

    // sine fragments are loaded one step ahead into nh / nl only and moved into bh / bl at
    // the top of each step (no product waits on a load issued in its own step)
    s16x8 nh[2][WN], nl[2][WN];
    load_b(0, nh, nl);
    build(0, 0);
    __syncthreads();
    // every load of the prologue has landed: without this the compiler's wait counting
    // merges them into the loop and makes each step's products wait on the next step's loads
    __builtin_amdgcn_s_waitcnt(0);
    int buf = 0;
    for (int k0 = 0; k0 < Hk; k0 += BK) {
        const bool more = k0 + BK < Hk;
        s16x8 bh[2][WN], bl[2][WN];
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int tn = 0; tn < WN; ++tn) {
                bh[p][tn] = nh[p][tn];
                if constexpr (TR::split) bl[p][tn] = nl[p][tn];
            }
        if (more) {
            load_b(k0 + BK, nh, nl);
            build(k0 + BK, buf ^ 1);
        }
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int tm = 0; tm < WM; ++tm) {
                const int rr = (wr * WM + tm) * 16 + lr;
                const s16x8 ah = *reinterpret_cast<const s16x8*>(&Dt[buf][p][0][rr][8 * lk]);
                s16x8 al;
                if constexpr (TR::split) al = *reinterpret_cast<const s16x8*>(&Dt[buf][p][NS - 1][rr][8 * lk]);
#pragma unroll
                for (int tn = 0; tn < WN; ++tn) {
                    acc[p][tm][tn] = mfma16<TR::half>(ah, bh[p][tn], acc[p][tm][tn]);
                    if constexpr (TR::split) {
                        acc[p][tm][tn] = mfma16<TR::half>(ah, bl[p][tn], acc[p][tm][tn]);
                        acc[p][tm][tn] = mfma16<TR::half>(al, bh[p][tn], acc[p][tm][tn]);
                    }
                }
            }
        __syncthreads();
        buf ^= 1;
    }

    if constexpr (TAB) {
        tab_epilogue_lowp<WM, WN, WAVES_N>(acc, reinterpret_cast<double*>(lds_ops), row0, R, P, n_m, H, c, tb);
        return;
    }
    if (layout == WK_HALF && gridDim.y == 1 && (P & 3) == 0 && P <= SP - 4) {
        // one column block holds every m of its rows: whole rows of the half table are staged
        // in LDS and leave in 16-byte stores (entry m - 1 holds K(m), m = 1..P)
        float* stg = reinterpret_cast<float*>(lds_ops);  // [16 * WAVES_M][SP]
        constexpr int SR = 16 * WAVES_M;
#pragma unroll
        for (int tm = 0; tm < WM; ++tm) {
#pragma unroll
            for (int tn = 0; tn < WN; ++tn) {
                const int t = (wc * WN + tn) * 16 + lr, m = t + 1;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    float* srow = stg + (wr * 16 + 4 * lk + e) * SP;
                    if (t < H) {
                        const float o = acc[0][tm][tn][e], ev = acc[1][tm][tn][e];
                        srow[m - 1] = c * (o + ev);
                        if (2 * m < P) srow[P - m - 1] = c * (o - ev);
                    }
                    if (t == 0) srow[P - 1] = 0.0f;
                }
            }
            __syncthreads();
            // local row q of the stage is global row row0 + ((q / 16) * WM + tm) * 16 + q % 16;
            // rows go to waves and their 16-byte pieces to lanes (no index division), and a
            // wave's LDS reads are all issued before its stores
            constexpr int NWV = KE_THREADS / 64, RPW = SR / NWV;
            static_assert(SR % NWV == 0, "stage rows per wave");
            float4 v[RPW];
            for (int c4 = 4 * lane; c4 < P; c4 += 256) {
#pragma unroll
                for (int i = 0; i < RPW; ++i)
                    v[i] = *reinterpret_cast<const float4*>(stg + (wave + NWV * i) * SP + c4);
#pragma unroll
                for (int i = 0; i < RPW; ++i) {
                    const int q = wave + NWV * i;
                    const long row = row0 + ((q >> 4) * WM + tm) * 16 + (q & 15);
                    if (row < R) *reinterpret_cast<float4*>(out + row * P + c4) = v[i];
                }
            }
            __syncthreads();
        }
        return;
    }
#pragma unroll
    for (int tm = 0; tm < WM; ++tm) {
#pragma unroll
        for (int tn = 0; tn < WN; ++tn) {
            const int t = col0 + (wc * WN + tn) * 16 + lr, m = t + 1;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const long row = row0 + (wr * WM + tm) * 16 + 4 * lk + e;
                if (row >= R || t >= H) continue;
                const float o = acc[0][tm][tn][e], ev = acc[1][tm][tn][e];
                const float kp = c * (o + ev), km = c * (o - ev);
                const bool mirror = 2 * m < P;
                if (layout == WK_HALF) {
                    float* h = out + row * P;
                    h[m - 1] = kp;
                    if (mirror) h[P - m - 1] = km;
                    if (t == 0) h[P - 1] = 0.0f;
                } else {
                    float* f = out + row * (long)n_m;
                    f[P + m] = kp;
                    f[P - m] = -kp;
                    if (mirror) {
                        f[2 * P - m] = km;
                        f[m] = -km;
                    }
                    if (t == 0) {
                        f[0] = 0.0f;
                        f[P] = 0.0f;
                    }
                }
            }
        }
    }
}

// n_m = 2 in reduced precision: every entry is zero.
__global__ void kernel_zero_f32(float* __restrict__ out, long n) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n) out[idx] = 0.0f;
}

static int round_up(int a, int b) { return (a + b - 1) / b * b; }

enum { CFG_SMALL = 0, CFG_MID = 1, CFG_LARGE = 2 };

// Folded FP64 tiles by H = floor(P / 2): 64 x 128 blocks of 64 x 32 wave tiles (both parts,
// sixteen accumulators) for H > 64, 64 x 64 for H in (32, 64], 64 x 32 below; one column block
// covers H <= 128 (P <= 257), so each difference is formed once per row.
static int fold_cfg(int H) { return H > 64 ? CFG_LARGE : (H > 32 ? CFG_MID : CFG_SMALL); }
static int fold_bn(int cfg) { return cfg == CFG_LARGE ? 128 : (cfg == CFG_MID ? 64 : 32); }
static int fold_bm(int cfg) { (void)cfg; return 64; }

int kernel_eval_1d_f64(const wk_mesh* mesh, const double* V, int B, const int32_t* cells,
                       int n_cells, int layout, double* out, hipStream_t stream) {
    const int n_m = mesh->n_m, P = n_m / 2, H = P / 2;
    const long R = (long)B * n_cells;
    if (R == 0) return WK_OK;
    if (H == 0) {
        const long n = R * (layout == WK_HALF ? P : n_m);
        hipLaunchKernelGGL(kernel_zero_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, out, n);
        return check_launch("kernel_zero_f64");
    }
    const int cfg = fold_cfg(H), BN = fold_bn(cfg), BM = fold_bm(cfg);
    const int Hk = round_up(H, KE_BK), Hn = round_up(H, BN);
    int err = WK_OK;
    const double* So = static_cast<const double*>(sine_table(n_m, SINE_ODD, Hk, Hn, &err));
    if (!So) return err;
    const double* Se = static_cast<const double*>(sine_table(n_m, SINE_EVEN, Hk, Hn, &err));
    if (!Se) return err;
    const double c = -2.0 / (mesh->hbar * (double)n_m);
    dim3 grid((unsigned)((R + BM - 1) / BM), (unsigned)(Hn / BN));
#define KE_LAUNCH_F64(WM, WN, WNV)                                                              \
    WK_LAUNCH("kernel_eval_f64", (kernel_eval_f64<WM, WN, WNV>), grid, dim3(KE_THREADS), 0, stream, V, \
                       mesh->nx, R, n_cells, cells, P, n_m, H, Hk, Hn, So, Se, c, layout, out, TabOut{})
    if (cfg == CFG_LARGE)
        KE_LAUNCH_F64(4, 2, 4);
    else if (cfg == CFG_MID)
        KE_LAUNCH_F64(4, 1, 4);
    else
        KE_LAUNCH_F64(2, 1, 2);
#undef KE_LAUNCH_F64
    return check_launch("kernel_eval_f64");
}

// eq.(4) rows straight into the creation tables (the TAB form of kernel_eval_f64): one column
// block must cover every m (H <= 128, n_m <= 514) and a round of staged rows must fit the
// operand tiles' LDS.
int kernel_tables_1d_f64(const wk_mesh* mesh, const double* V, int B, const int32_t* cells,
                         int n_cells, const TabOut& tb, hipStream_t stream) {
    const int n_m = mesh->n_m, P = n_m / 2, H = P / 2;
    const long R = (long)B * n_cells;
    if (R == 0) return WK_OK;
    WK_REQUIRE(n_m >= 4 && H <= 128, "wk_kernel_tables: n_m must lie in [4, 514]");
    WK_REQUIRE(tb.guide == nullptr || (tb.G >= 1 && tb.G <= TAB_GMAX),
               "wk_kernel_tables: guide_len must lie in [1, 256]");
    const int cfg = fold_cfg(H), BN = fold_bn(cfg), BM = fold_bm(cfg);
    const int waves_m = cfg == CFG_SMALL ? 2 : 1;
    WK_REQUIRE(8 * waves_m * (n_m + 1) <= 2 * 2 * BM * (KE_BK + 1), "wk_kernel_tables: row stage exceeds LDS");
    const int Hk = round_up(H, KE_BK), Hn = round_up(H, BN);
    int err = WK_OK;
    const double* So = static_cast<const double*>(sine_table(n_m, SINE_ODD, Hk, Hn, &err));
    if (!So) return err;
    const double* Se = static_cast<const double*>(sine_table(n_m, SINE_EVEN, Hk, Hn, &err));
    if (!Se) return err;
    const double c = -2.0 / (mesh->hbar * (double)n_m);
    dim3 grid((unsigned)((R + BM - 1) / BM), 1);
#define KT_LAUNCH_F64(WM, WN, WNV)                                                                 \
    WK_LAUNCH("kernel_tables_f64", (kernel_eval_f64<WM, WN, WNV, true>), grid, dim3(KE_THREADS), 0, \
              stream, V, mesh->nx, R, n_cells, cells, P, n_m, H, Hk, Hn, So, Se, c, WK_HALF,       \
              (double*)nullptr, tb)
    if (cfg == CFG_LARGE)
        KT_LAUNCH_F64(4, 2, 4);
    else if (cfg == CFG_MID)
        KT_LAUNCH_F64(4, 1, 4);
    else
        KT_LAUNCH_F64(2, 1, 2);
#undef KT_LAUNCH_F64
    return check_launch("kernel_tables_f64");
}

// 16-bit fold tiles by H: 64 x 128 blocks of 64 x 32 wave tiles (both parts) for H > 64,
// 64 x 64 for H in (32, 64], 64 x 32 below.
template <int PREC>
static void launch_lowp(int cfg, dim3 grid, hipStream_t stream, const double* V, int nx, long R,
                        int n_cells, const int32_t* cells, int P, int n_m, int H, int Hk,
                        const uint16_t* const* T, float c, int layout, float* out) {
#define KE_LAUNCH_LP(WM, WN, WNV)                                                                  \
    WK_LAUNCH("kernel_eval_lowp", (kernel_eval_lowp<PREC, WM, WN, WNV>), grid, dim3(KE_THREADS), 0, \
              stream, V, nx, R, n_cells, cells, P, n_m, H, Hk, T[0], T[1], T[2], T[3], c, layout, out, \
              TabOut{})
    if (cfg == CFG_LARGE)
        KE_LAUNCH_LP(4, 2, 4);
    else if (cfg == CFG_MID)
        KE_LAUNCH_LP(4, 1, 4);
    else
        KE_LAUNCH_LP(2, 1, 2);
#undef KE_LAUNCH_LP
}

int kernel_eval_1d_lowp(const wk_mesh* mesh, const double* V, int B, const int32_t* cells,
                        int n_cells, int prec, int layout, float* out, hipStream_t stream) {
    const int n_m = mesh->n_m, P = n_m / 2, H = P / 2;
    const long R = (long)B * n_cells;
    if (R == 0) return WK_OK;
    if (H == 0) {
        const long n = R * (layout == WK_HALF ? P : n_m);
        hipLaunchKernelGGL(kernel_zero_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, out, n);
        return check_launch("kernel_zero_f32");
    }
    const int cfg = fold_cfg(H), BN = fold_bn(cfg);
    const int Hk = round_up(H, LP_BK), Hn = round_up(H, BN);
    const bool half = prec == WK_FP16 || prec == WK_FP16X3;
    const bool split = prec == WK_BF16X3 || prec == WK_FP16X3;
    const int fh = half ? 3 : 1, fl = half ? 4 : 2;
    // transposed fold tables T[t][k] (Hn rows, Hk columns): odd hi, even hi, odd lo, even lo
    const int kinds[4] = {fh | SINE_ODD_T, fh | SINE_EVEN_T, fl | SINE_ODD_T, fl | SINE_EVEN_T};
    const uint16_t* T[4];
    int err = WK_OK;
    for (int i = 0; i < 4; ++i) {
        if (i >= 2 && !split) {
            T[i] = T[i - 2];
            continue;
        }
        T[i] = static_cast<const uint16_t*>(sine_table(n_m, kinds[i], Hn, Hk, &err));
        if (!T[i]) return err;
    }
    const float c = (float)(-2.0 / (mesh->hbar * (double)n_m));
    dim3 grid((unsigned)((R + KE_BM - 1) / KE_BM), (unsigned)(Hn / BN));
    switch (prec) {
        case WK_BF16:
            launch_lowp<WK_BF16>(cfg, grid, stream, V, mesh->nx, R, n_cells, cells, P, n_m, H, Hk, T, c, layout, out);
            break;
        case WK_FP16:
            launch_lowp<WK_FP16>(cfg, grid, stream, V, mesh->nx, R, n_cells, cells, P, n_m, H, Hk, T, c, layout, out);
            break;
        case WK_BF16X3:
            launch_lowp<WK_BF16X3>(cfg, grid, stream, V, mesh->nx, R, n_cells, cells, P, n_m, H, Hk, T, c, layout, out);
            break;
        default:
            launch_lowp<WK_FP16X3>(cfg, grid, stream, V, mesh->nx, R, n_cells, cells, P, n_m, H, Hk, T, c, layout, out);
            break;
    }
    return check_launch("kernel_eval_lowp");
}
// The 16-bit forms' rows straight into the creation tables (the TAB form of kernel_eval_lowp):
// the same tables as kernel_eval_1d_lowp's FP32 half rows given to the table kernels.  One
// column block must cover every m (H <= 128, n_m <= 514).
template <int PREC>
static void launch_lowp_tab(int cfg, dim3 grid, hipStream_t stream, const double* V, int nx, long R,
                            int n_cells, const int32_t* cells, int P, int n_m, int H, int Hk,
                            const uint16_t* const* T, float c, const TabOut& tb) {
#define KT_LAUNCH_LP(WM, WN, WNV)                                                                  \
    WK_LAUNCH("kernel_tables_lowp", (kernel_eval_lowp<PREC, WM, WN, WNV, true>), grid, dim3(KE_THREADS), \
              0, stream, V, nx, R, n_cells, cells, P, n_m, H, Hk, T[0], T[1], T[2], T[3], c, WK_HALF,   \
              (float*)nullptr, tb)
    if (cfg == CFG_LARGE)
        KT_LAUNCH_LP(4, 2, 4);
    else if (cfg == CFG_MID)
        KT_LAUNCH_LP(4, 1, 4);
    else
        KT_LAUNCH_LP(2, 1, 2);
#undef KT_LAUNCH_LP
}

int kernel_tables_1d_lowp(const wk_mesh* mesh, const double* V, int B, const int32_t* cells,
                          int n_cells, int prec, const TabOut& tb, hipStream_t stream) {
    const int n_m = mesh->n_m, P = n_m / 2, H = P / 2;
    const long R = (long)B * n_cells;
    if (R == 0) return WK_OK;
    WK_REQUIRE(n_m >= 4 && H <= 128, "wk_kernel_tables: n_m must lie in [4, 514]");
    WK_REQUIRE(tb.guide == nullptr || (tb.G >= 1 && tb.G <= TAB_GMAX),
               "wk_kernel_tables: guide_len must lie in [1, 256]");
    const int cfg = fold_cfg(H), BN = fold_bn(cfg);
    const int Hk = round_up(H, LP_BK), Hn = round_up(H, BN);
    const bool half = prec == WK_FP16 || prec == WK_FP16X3;
    const bool split = prec == WK_BF16X3 || prec == WK_FP16X3;
    const int fh = half ? 3 : 1, fl = half ? 4 : 2;
    const int kinds[4] = {fh | SINE_ODD_T, fh | SINE_EVEN_T, fl | SINE_ODD_T, fl | SINE_EVEN_T};
    const uint16_t* T[4];
    int err = WK_OK;
    for (int i = 0; i < 4; ++i) {
        if (i >= 2 && !split) {
            T[i] = T[i - 2];
            continue;
        }
        T[i] = static_cast<const uint16_t*>(sine_table(n_m, kinds[i], Hn, Hk, &err));
        if (!T[i]) return err;
    }
    const float c = (float)(-2.0 / (mesh->hbar * (double)n_m));
    dim3 grid((unsigned)((R + KE_BM - 1) / KE_BM), 1);
    switch (prec) {
        case WK_BF16:
            launch_lowp_tab<WK_BF16>(cfg, grid, stream, V, mesh->nx, R, n_cells, cells, P, n_m, H, Hk, T, c, tb);
            break;
        case WK_FP16:
            launch_lowp_tab<WK_FP16>(cfg, grid, stream, V, mesh->nx, R, n_cells, cells, P, n_m, H, Hk, T, c, tb);
            break;
        case WK_BF16X3:
            launch_lowp_tab<WK_BF16X3>(cfg, grid, stream, V, mesh->nx, R, n_cells, cells, P, n_m, H, Hk, T, c, tb);
            break;
        default:
            launch_lowp_tab<WK_FP16X3>(cfg, grid, stream, V, mesh->nx, R, n_cells, cells, P, n_m, H, Hk, T, c, tb);
            break;
    }
    return check_launch("kernel_tables_lowp");
}

int kernel_eval_2d(const wk_mesh* mesh, const double* V, int B, const int32_t* cells, int n_cells,
                   double* out, hipStream_t stream);
int kernel_eval_2d_16(const wk_mesh* mesh, const double* V, int B, const int32_t* cells, int n_cells,
                      int prec, float* out, hipStream_t stream);
int kernel_tables_2d(const wk_mesh* mesh, const double* V, int B, const int32_t* cells, int n_cells,
                     const TabOut& tb, hipStream_t stream);
int kernel_tables_2d_16(const wk_mesh* mesh, const double* V, int B, const int32_t* cells, int n_cells,
                        int prec, const TabOut& tb, hipStream_t stream);

}  // namespace wk

extern "C" int wk_kernel_eval(const wk_mesh* mesh, const double* V, int32_t B,
                              const int32_t* cells, int32_t n_cells, int32_t prec, int32_t layout,
                              void* K_out, void* stream) {
    WK_REQUIRE(mesh != nullptr, "wk_kernel_eval: mesh is NULL");
    WK_REQUIRE(mesh->dim == 1 || mesh->dim == 2, "wk_kernel_eval: dim must be 1 or 2");
    WK_REQUIRE(mesh->nx > 0 && mesh->ny > 0, "wk_kernel_eval: empty mesh");
    WK_REQUIRE(mesh->n_m >= 2 && (mesh->n_m % 2) == 0, "wk_kernel_eval: n_m must be even and >= 2");
    WK_REQUIRE(mesh->hbar > 0.0, "wk_kernel_eval: hbar must be positive");
    WK_REQUIRE(B >= 0 && n_cells >= 0, "wk_kernel_eval: negative size");
    WK_REQUIRE(layout == WK_FULL || layout == WK_HALF, "wk_kernel_eval: bad layout");
    if ((long)B * n_cells == 0) return WK_OK;
    const long ncell = (long)mesh->nx * mesh->ny;
    WK_REQUIRE(cells != nullptr || n_cells == ncell,
               "wk_kernel_eval: with cells == NULL, n_cells must be the number of cells");
    WK_REQUIRE(V != nullptr && K_out != nullptr, "wk_kernel_eval: NULL array");
    if (mesh->dim == 1) {
        WK_REQUIRE(mesh->ny == 1, "wk_kernel_eval: 1-D mesh needs ny == 1");
        if (prec == WK_FP64)
            return wk::kernel_eval_1d_f64(mesh, V, B, cells, n_cells, layout,
                                          static_cast<double*>(K_out), wk::as_stream(stream));
        if (prec >= WK_BF16 && prec <= WK_FP16X3)
            return wk::kernel_eval_1d_lowp(mesh, V, B, cells, n_cells, prec, layout,
                                           static_cast<float*>(K_out), wk::as_stream(stream));
        return wk::fail(WK_EINVAL, "wk_kernel_eval: unknown precision");
    }
    WK_REQUIRE(layout == WK_FULL, "wk_kernel_eval: 2-D tables are full");
    if (prec == WK_FP64)
        return wk::kernel_eval_2d(mesh, V, B, cells, n_cells, static_cast<double*>(K_out),
                                  wk::as_stream(stream));
    WK_REQUIRE(prec >= WK_BF16 && prec <= WK_FP16X3, "wk_kernel_eval: unknown precision");
    return wk::kernel_eval_2d_16(mesh, V, B, cells, n_cells, prec, static_cast<float*>(K_out),
                                 wk::as_stream(stream));
}

extern "C" int wk_kernel_tables(const wk_mesh* mesh, const double* V, int32_t B,
                                const int32_t* cells, int32_t n_cells, int32_t prec, double dt,
                                double* gamma, uint32_t* n0, uint32_t* thr, uint64_t* cdf,
                                uint32_t* guide, int32_t guide_len, void* stream) {
    WK_REQUIRE(mesh != nullptr, "wk_kernel_tables: mesh is NULL");
    WK_REQUIRE((mesh->dim == 1 && mesh->ny == 1) || mesh->dim == 2, "wk_kernel_tables: bad mesh");
    WK_REQUIRE(mesh->nx > 0 && mesh->ny > 0, "wk_kernel_tables: empty mesh");
    WK_REQUIRE(mesh->n_m >= 2 && (mesh->n_m % 2) == 0, "wk_kernel_tables: n_m must be even and >= 2");
    WK_REQUIRE(mesh->hbar > 0.0, "wk_kernel_tables: hbar must be positive");
    WK_REQUIRE(B >= 0 && n_cells >= 0, "wk_kernel_tables: negative size");
    WK_REQUIRE(dt >= 0.0, "wk_kernel_tables: dt must be >= 0");
    if ((long)B * n_cells == 0) return WK_OK;
    WK_REQUIRE(cells != nullptr || n_cells == (long)mesh->nx * mesh->ny,
               "wk_kernel_tables: with cells == NULL, n_cells must be the number of cells");
    WK_REQUIRE(V && gamma && n0 && thr && cdf, "wk_kernel_tables: NULL array");
    const wk::TabOut tb{dt, gamma, n0, thr, cdf, guide, guide ? (int)guide_len : 0};
    if (mesh->dim == 2) {
        if (prec == WK_FP64) return wk::kernel_tables_2d(mesh, V, B, cells, n_cells, tb, wk::as_stream(stream));
        WK_REQUIRE(prec >= WK_BF16 && prec <= WK_FP16X3, "wk_kernel_tables: unknown precision");
        return wk::kernel_tables_2d_16(mesh, V, B, cells, n_cells, prec, tb, wk::as_stream(stream));
    }
    if (prec == WK_FP64) return wk::kernel_tables_1d_f64(mesh, V, B, cells, n_cells, tb, wk::as_stream(stream));
    WK_REQUIRE(prec >= WK_BF16 && prec <= WK_FP16X3, "wk_kernel_tables: unknown precision");
    return wk::kernel_tables_1d_lowp(mesh, V, B, cells, n_cells, prec, tb, wk::as_stream(stream));
}

// ----------------------------------------------------------------------------- adjoint
// K is linear in V (eq.(4)), so dL/dV = (dK/dV)^T G, computed in three deterministic steps:
//   1. fold the table gradient onto the unique momenta: G1[r][t] = dL/dK(m = t + 1)
//      (full layout: G(m) - G(-m), and -G(-P) for m = P);
//   2. GD[r][jj] = c * sum_t G1[r][t] S[t][jj]  (MFMA on the odd/even fold below);
//   3. dV[b][l] += sum_r (GD[r][l - i_r] - GD[r][i_r - l]) over the rows r of potential b with
//      cell i_r (terms with offsets in [1, P] only), plus at the two edges the sums of every
//      term whose clamped index lands there (per-row tails, then a fixed-order sum).
// T = double (FP64 MFMA) or float (FP32 MFMA); dV is double either way.
namespace wk {

template <typename T> struct BwdMfma;
template <> struct BwdMfma<double> {
    typedef f64x4 acc_t;
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // output element e of a lane sits at row lane / 16 + 4 e of the 16 x 16 tile
    static __device__ __forceinline__ int row(int lk, int e) { return lk + 4 * e; }
};
template <> struct BwdMfma<float> {
    typedef f32x4 acc_t;
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // output element e of a lane sits at row 4 (lane / 16) + e of the 16 x 16 tile
    static __device__ __forceinline__ int row(int lk, int e) { return 4 * lk + e; }
};

// Step 2 on the odd/even fold (the transpose of the forward's): pairing m with P - m,
//   GD[r][2k]     = c sum_{m <= H} So[k][m - 1] (G1(m) + G1(P - m))     (j = 2k + 1 odd)
//   GD[r][2k + 1] = c sum_{m <= H} Se[k][m - 1] (G1(m) - G1(P - m))     (j = 2k + 2 even)
// (m = P / 2 taken once), two H x H products per row; the fold tables are read transposed,
// T[m - 1][k].  For odd P the column j = P (all sines zero) is written as 0.
template <typename T, int WM, int WN>
__global__ __launch_bounds__(KE_THREADS) void kernel_bwd_gemm(
    const T* __restrict__ G, long R, int P, int n_m, int layout, int H, int Hk, int Hn,
    const T* __restrict__ To, const T* __restrict__ Te, T c, T* __restrict__ GD) {
    typedef BwdMfma<T> MF;
    typedef typename MF::acc_t acc_t;
    constexpr int BM = 32 * WM, BN = 32 * WN, BK = KE_BK;
    __shared__ T As[2][BM][BK + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const long row0 = (long)blockIdx.x * BM;
    const int col0 = blockIdx.y * BN;
    const int lr = lane & 15, lk = lane >> 4;
    // dL/dK at momentum m (1 <= m <= P) of row r, from either layout
    auto g1 = [&](long r, int m) -> T {
        if (layout == WK_HALF) return G[r * P + (m - 1)];
        const T* gr = G + r * (long)n_m;
        return m < P ? gr[P + m] - gr[P - m] : -gr[0];
    };
    acc_t acc[2][WM][WN];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int a = 0; a < WM; ++a)
#pragma unroll
            for (int b = 0; b < WN; ++b) acc[p][a][b] = acc_t{0, 0, 0, 0};
    const long cw = (long)col0 + wc * WN * 16 + lr;
    const T* Tw[2] = {To + cw, Te + cw};
    for (int k0 = 0; k0 < Hk; k0 += BK) {
        T bfrag[2][BK / 4][WN];
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int ks = 0; ks < BK / 4; ++ks)
#pragma unroll
                for (int tn = 0; tn < WN; ++tn) bfrag[p][ks][tn] = Tw[p][(long)(k0 + 4 * ks + lk) * Hn + tn * 16];
        __syncthreads();
        for (int e = threadIdx.x; e < BM * BK; e += KE_THREADS) {
            const int rr = e / BK, kk = e - rr * BK;
            const long r = row0 + rr;
            const int m = k0 + kk + 1;
            T gp = 0, gm = 0;
            if (r < R && m <= H) {
                const T a = g1(r, m), b = 2 * m < P ? g1(r, P - m) : T(0);
                gp = a + b;
                gm = a - b;
            }
            As[0][rr][kk] = gp;
            As[1][rr][kk] = gm;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < BK / 4; ++ks) {
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                T afrag[WM];
#pragma unroll
                for (int tm = 0; tm < WM; ++tm) afrag[tm] = As[p][(wr * WM + tm) * 16 + lr][4 * ks + lk];
#pragma unroll
                for (int tm = 0; tm < WM; ++tm)
#pragma unroll
                    for (int tn = 0; tn < WN; ++tn)
                        acc[p][tm][tn] = MF::mma(afrag[tm], bfrag[p][ks][tn], acc[p][tm][tn]);
            }
        }
    }
#pragma unroll
    for (int tm = 0; tm < WM; ++tm)
#pragma unroll
        for (int tn = 0; tn < WN; ++tn) {
            const int k = col0 + (wc * WN + tn) * 16 + lr;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const long row = row0 + (wr * WM + tm) * 16 + MF::row(lk, e);
                if (row >= R) continue;
                if (k < H) {
                    GD[row * P + 2 * k] = c * acc[0][tm][tn][e];
                    GD[row * P + 2 * k + 1] = c * acc[1][tm][tn][e];
                }
                if ((P & 1) && k == 0) GD[row * P + P - 1] = T(0);
            }
        }
}

template <typename T>
__global__ void kernel_bwd_zero(T* __restrict__ out, long n) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n) out[idx] = T(0);
}

// Per row r (cell i): sums of GD over the offsets whose clamped index is an edge.  Only rows
// within P of an edge have such offsets (i >= nx - 1 - P for the upper edge, i <= P for the
// lower).  One wave per row reads it coalesced and adds with a fixed butterfly.
// All cells (cells == NULL): the rows are enumerated per potential, first 0..nlo-1
// (nlo = min(P, nx - 1) + 1), then the rest of [nx - 1 - P, nx - 1], and the tails are stored
// by cell.  Cell lists: one wave per row of the list; rows away from the edges (and ids outside
// the mesh) store zero tails.
__device__ __forceinline__ void edge_rows(int nx, int P, int* nlo, int* hi0, int* ne) {
    *nlo = min(P, nx - 1) + 1;
    *hi0 = max(*nlo, nx - 1 - P);
    *ne = *nlo + (nx - *hi0);
}

template <typename T>
__global__ __launch_bounds__(256) void kernel_bwd_tails(const T* __restrict__ GD, int B, int nx, int P,
                                                        const int32_t* __restrict__ cells, int n_cells,
                                                        T* __restrict__ tail_hi, T* __restrict__ tail_lo) {
    const int lane = threadIdx.x & 63;
    const long wid = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    long row;
    int i;
    if (cells == nullptr) {
        int nlo, hi0, ne;
        edge_rows(nx, P, &nlo, &hi0, &ne);
        const long b = wid / ne;
        if (b >= B) return;
        const int k = (int)(wid - b * ne);
        i = k < nlo ? k : hi0 + (k - nlo);
        row = b * nx + i;
    } else {
        if (wid >= (long)B * n_cells) return;
        row = wid;
        i = cells[wid % n_cells];
        if (i < 0 || i >= nx || (i > P && i < nx - 1 - P)) {
            if (lane == 0) {
                tail_hi[row] = T(0);
                tail_lo[row] = T(0);
            }
            return;
        }
    }
    const T* g = GD + row * (long)P;
    T hi = 0, lo = 0;
    for (int j = 1 + lane; j <= P; j += 64) {
        const T v = g[j - 1];
        if (i + j >= nx - 1) hi += v;  // V(i + j) clamps to (or is) cell nx - 1
        if (i - j <= 0) lo += v;       // V(i - j) clamps to (or is) cell 0
    }
    for (int o = 32; o > 0; o >>= 1) {
        hi += __shfl_xor(hi, o, 64);
        lo += __shfl_xor(lo, o, 64);
    }
    if (lane == 0) {
        tail_hi[row] = hi;
        tail_lo[row] = lo;
    }
}

// All cells: a workgroup takes 64 consecutive outputs l of one potential and walks the rows
// they need; its four waves take every fourth row.  At row i a wave's lanes read consecutive
// columns of GD (ascending for the terms GD[l - j][j - 1], descending for GD[l + j][j - 1]),
// so each load is one contiguous segment.  The four partial sums of an output are added in
// wave order, then the edge tails (fixed order).
template <typename T>
__global__ __launch_bounds__(256) void kernel_bwd_gather(const T* __restrict__ GD, int B, int nx, int P,
                                                         const T* __restrict__ tail_hi,
                                                         const T* __restrict__ tail_lo,
                                                         double* __restrict__ dV) {
    __shared__ T part[4][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const long wpp = (nx + 63) / 64;  // output groups per potential
    const long b = blockIdx.x / wpp;
    const int l0 = (int)(blockIdx.x - b * wpp) * 64, l = l0 + lane;
    const T* g = GD + b * (long)nx * P;
    T acc = 0;
    // rows i = l - j, j = 1..P (outputs l < nx - 1)
    const int i1 = min(l0 + 62, nx - 1);
#pragma unroll 4
    for (int i = max(l0 - P, 0) + wv; i <= i1; i += 4) {
        const int j = l - i;
        if (l < nx - 1 && j >= 1 && j <= P) acc += g[(long)i * P + (j - 1)];
    }
    // rows i = l + j, j = 1..P (outputs 0 < l < nx)
    const int i2 = min(l0 + 63 + P, nx - 1);
#pragma unroll 4
    for (int i = l0 + 1 + wv; i <= i2; i += 4) {
        const int j = i - l;
        if (l > 0 && l < nx && j >= 1 && j <= P) acc -= g[(long)i * P + (j - 1)];
    }
    part[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && l < nx) {
        T t = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
        // edge tails: only the rows within P of the edge have them (see kernel_bwd_tails)
        if (l == nx - 1)
            for (int i = max(0, nx - 1 - P); i < nx; ++i) t += tail_hi[b * nx + i];
        if (l == 0)
            for (int i = 0; i <= min(P, nx - 1); ++i) t -= tail_lo[b * nx + i];
        dV[b * (long)nx + l] += (double)t;
    }
}

// Cell lists: a workgroup takes 64 consecutive outputs l of one potential; its four waves take
// every fourth row of the potential's list (the cell id is wave-uniform).  Row r with cell i
// adds GD[r][l - i - 1] for l - i in [1, P] (l < nx - 1) and subtracts GD[r][i - l - 1] for
// i - l in [1, P] (l > 0): each a contiguous segment of the row across the lanes.  Rows whose
// window misses the group are skipped; ids outside the mesh contribute nothing.  Partial
// sums are added in wave order, then the tails of the rows in list order.
template <typename T>
__global__ __launch_bounds__(256) void kernel_bwd_gather_cells(
    const T* __restrict__ GD, int B, int nx, int P, const int32_t* __restrict__ cells, int n_cells,
    const T* __restrict__ tail_hi, const T* __restrict__ tail_lo, double* __restrict__ dV) {
    __shared__ T part[4][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const long wpp = (nx + 63) / 64;
    const long b = blockIdx.x / wpp;
    const int l0 = (int)(blockIdx.x - b * wpp) * 64, l = l0 + lane;
    const T* g = GD + b * (long)n_cells * P;
    T acc = 0;
    for (int r = wv; r < n_cells; r += 4) {
        const int i = cells[r];
        if (i < 0 || i >= nx || i + P < l0 || i - P > l0 + 63) continue;
        const T* gr = g + (long)r * P;
        const int jp = l - i, jm = i - l;
        if (l < nx - 1 && jp >= 1 && jp <= P) acc += gr[jp - 1];
        if (l > 0 && l < nx && jm >= 1 && jm <= P) acc -= gr[jm - 1];
    }
    part[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && l < nx) {
        T t = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
        const long r0 = b * (long)n_cells;
        if (l == nx - 1)
            for (int r = 0; r < n_cells; ++r) t += tail_hi[r0 + r];
        if (l == 0)
            for (int r = 0; r < n_cells; ++r) t -= tail_lo[r0 + r];
        dV[b * (long)nx + l] += (double)t;
    }
}

// Tile of the adjoint product: 2 x 2 waves of 32 x 32 (BN = 64 columns per block).
constexpr int BWD_WM = 2, BWD_WN = 2, BWD_BM = 32 * BWD_WM, BWD_BN = 32 * BWD_WN;

template <typename T>
static int kernel_bwd_run(const wk_mesh* mesh, const T* G, int B, const int32_t* cells, int n_cells,
                          int layout, double* dV, void* ws, hipStream_t s) {
    const int n_m = mesh->n_m, P = n_m / 2, H = P / 2, nx = mesh->nx;
    const long R = (long)B * n_cells;
    T* GD = static_cast<T*>(ws);
    T* th = GD + R * P;
    T* tl = th + R;
    const T c = (T)(-2.0 / (mesh->hbar * (double)n_m));
    const char* name = sizeof(T) == 8 ? "kernel_bwd_f64" : "kernel_bwd_f32";
    if (H == 0) {  // n_m = 2: every sine of eq.(4) is zero
        hipLaunchKernelGGL(kernel_bwd_zero<T>, dim3((unsigned)((R * P + 255) / 256)), dim3(256), 0, s, GD, R * P);
    } else {
        const int Hk = round_up(H, KE_BK), Hn = round_up(H, BWD_BN);
        const int fmt = sizeof(T) == 8 ? SINE_F64 : SINE_F32;
        int err = WK_OK;
        const T* To = static_cast<const T*>(sine_table(n_m, fmt | SINE_ODD_T, Hk, Hn, &err));
        if (!To) return err;
        const T* Te = static_cast<const T*>(sine_table(n_m, fmt | SINE_EVEN_T, Hk, Hn, &err));
        if (!Te) return err;
        WK_LAUNCH(name, (kernel_bwd_gemm<T, BWD_WM, BWD_WN>),
                  dim3((unsigned)((R + BWD_BM - 1) / BWD_BM), Hn / BWD_BN), dim3(KE_THREADS), 0, s, G, R, P,
                  n_m, layout, H, Hk, Hn, To, Te, c, GD);
    }
    const long groups = (long)B * ((nx + 63) / 64);
    if (cells == nullptr) {
        const int nlo = (P < nx - 1 ? P : nx - 1) + 1, hi0 = nlo > nx - 1 - P ? nlo : nx - 1 - P;
        const long erows = (long)B * (nlo + (nx - hi0));  // one wave each
        hipLaunchKernelGGL(kernel_bwd_tails<T>, dim3((unsigned)((erows + 3) / 4)), dim3(256), 0, s, GD, B, nx,
                           P, nullptr, n_cells, th, tl);
        hipLaunchKernelGGL(kernel_bwd_gather<T>, dim3((unsigned)groups), dim3(256), 0, s, GD, B, nx, P, th, tl, dV);
    } else {
        hipLaunchKernelGGL(kernel_bwd_tails<T>, dim3((unsigned)((R + 3) / 4)), dim3(256), 0, s, GD, B, nx, P,
                           cells, n_cells, th, tl);
        hipLaunchKernelGGL(kernel_bwd_gather_cells<T>, dim3((unsigned)groups), dim3(256), 0, s, GD, B, nx, P,
                           cells, n_cells, th, tl, dV);
    }
    return check_launch("wk_kernel_bwd");
}

}  // namespace wk

extern "C" size_t wk_kernel_bwd_workspace(const wk_mesh* mesh, int32_t B, int32_t n_cells, int32_t prec) {
    if (!mesh || mesh->n_m < 2 || B < 0 || n_cells < 0 || mesh->nx <= 0) return 0;
    if (prec != WK_FP64 && prec != WK_FP32) return 0;
    const size_t R = (size_t)B * n_cells, el = prec == WK_FP64 ? sizeof(double) : sizeof(float);
    return el * (R * (size_t)(mesh->n_m / 2) + 2 * R) + 256;
}

extern "C" int wk_kernel_bwd(const wk_mesh* mesh, const void* G, int32_t B, const int32_t* cells,
                             int32_t n_cells, int32_t prec, int32_t layout, double* dV, void* ws,
                             size_t ws_bytes, void* stream) {
    using namespace wk;
    WK_REQUIRE(mesh != nullptr, "wk_kernel_bwd: mesh is NULL");
    WK_REQUIRE(mesh->dim == 1 && mesh->ny == 1 && mesh->nx > 0, "wk_kernel_bwd: 1-D meshes only");
    WK_REQUIRE(mesh->n_m >= 2 && mesh->n_m % 2 == 0, "wk_kernel_bwd: n_m must be even");
    WK_REQUIRE(mesh->hbar > 0.0, "wk_kernel_bwd: hbar must be positive");
    WK_REQUIRE(layout == WK_FULL || layout == WK_HALF, "wk_kernel_bwd: bad layout");
    WK_REQUIRE(prec == WK_FP64 || prec == WK_FP32, "wk_kernel_bwd: prec must be WK_FP64 or WK_FP32");
    WK_REQUIRE(B >= 0 && n_cells >= 0, "wk_kernel_bwd: negative size");
    WK_REQUIRE(cells != nullptr || n_cells == mesh->nx,
               "wk_kernel_bwd: with cells == NULL, n_cells must be nx");
    if ((long)B * n_cells == 0) return WK_OK;
    WK_REQUIRE(G && dV && ws, "wk_kernel_bwd: NULL array");
    WK_REQUIRE(ws_bytes >= wk_kernel_bwd_workspace(mesh, B, n_cells, prec), "wk_kernel_bwd: workspace too small");
    hipStream_t s = as_stream(stream);
    if (prec == WK_FP64)
        return kernel_bwd_run<double>(mesh, static_cast<const double*>(G), B, cells, n_cells, layout, dV, ws, s);
    return kernel_bwd_run<float>(mesh, static_cast<const float*>(G), B, cells, n_cells, layout, dV, ws, s);
}

// ----------------------------------------------------------------------------- set-up
// The sine tables every 1-D contraction of this file reads for a given n_m (forward FP64 and
// fused tables, the 16-bit forms, the FP64 and FP32 adjoints), in the shapes they look up.
namespace wk {
static int prepare_1d(int n_m, hipStream_t s) {
    const int P = n_m / 2, H = P / 2;
    if (H == 0) return WK_OK;
    int rc;
    {   // forward FP64 and the fused tables
        const int Hk = round_up(H, KE_BK), Hn = round_up(H, fold_bn(fold_cfg(H)));
        if ((rc = sine_table_build(n_m, SINE_ODD, Hk, Hn, s))) return rc;
        if ((rc = sine_table_build(n_m, SINE_EVEN, Hk, Hn, s))) return rc;
    }
    {   // 16-bit forms: transposed hi / lo fold tables
        const int Hk = round_up(H, LP_BK), Hn = round_up(H, fold_bn(fold_cfg(H)));
        for (int fmt = 1; fmt <= 4; ++fmt) {
            if ((rc = sine_table_build(n_m, fmt | SINE_ODD_T, Hn, Hk, s))) return rc;
            if ((rc = sine_table_build(n_m, fmt | SINE_EVEN_T, Hn, Hk, s))) return rc;
        }
    }
    {   // adjoints
        const int Hk = round_up(H, KE_BK), Hn = round_up(H, BWD_BN);
        for (int fmt : {SINE_F64, SINE_F32}) {
            if ((rc = sine_table_build(n_m, fmt | SINE_ODD_T, Hk, Hn, s))) return rc;
            if ((rc = sine_table_build(n_m, fmt | SINE_EVEN_T, Hk, Hn, s))) return rc;
        }
    }
    return WK_OK;
}
}  // namespace wk

extern "C" int wk_prepare(const wk_mesh* mesh, void* stream) {
    using namespace wk;
    WK_REQUIRE(mesh != nullptr, "wk_prepare: mesh is NULL");
    WK_REQUIRE(mesh->n_m >= 2 && mesh->n_m % 2 == 0, "wk_prepare: n_m must be even and >= 2");
    if (mesh->dim == 2) return WK_OK;  // the 2-D contraction forms its trig operands in registers
    WK_REQUIRE(mesh->dim == 1, "wk_prepare: dim must be 1 or 2");
    return prepare_1d(mesh->n_m, as_stream(stream));
}

// ----------------------------------------------------------------------------- d = 2
// eq.(4) in two dimensions (half weight at |j_a| = P), separated with
// sin(a_x + a_y) = sin a_x cos a_y + cos a_x sin a_y:
//   stage 1  T[jy][n]  = sum_jx D[jy][jx] B1[jx][n],  B1 = [w sin(2 pi mx jx/n_m) | w cos(...)]
//   stage 2  K[my][mx] = c2 sum_k A2[my][k] T'[k][mx], A2 = [w cos(2 pi my jy/n_m) | w sin(...)],
//            T' = [T_sin ; T_cos] stacked along jy
// with D[jy][jx] = V(i + j) - V(i - j) formed in LDS from a (2P+1)^2 window of V, and
// c2 = -1/(hbar n_m^2).  Both stages run on v_mfma_f64_16x16x4; the trig operands depend only
// on (n_m, lane) and are computed once per workgroup into registers.  Workgroups loop over
// the requested cells.
namespace wk {

__device__ __forceinline__ double w_end(int j, int P) { return (j == P || j == -P) ? 0.5 : 1.0; }


template <int P, bool TAB = false>
__global__ __launch_bounds__(KE_THREADS) void kernel_eval_2d_f64(
    const double* __restrict__ V, int nx, int ny, long R, int n_cells,
    const int32_t* __restrict__ cells, double c2, double* __restrict__ out, TabOut tb) {
    constexpr int J = 2 * P + 1;                       // offsets per axis
    constexpr int M1 = (J + 15) / 16 * 16;             // stage-1 rows (jy), padded
    constexpr int K1 = (J + 3) / 4 * 4;                // stage-1 depth (jx), padded
    constexpr int N1 = (4 * P + 15) / 16 * 16;         // stage-1 columns: 2P sin + 2P cos
    constexpr int NT1 = N1 / 16, MT1 = M1 / 16;
    constexpr int M2 = (2 * P + 15) / 16 * 16;         // stage-2 rows (my)
    constexpr int N2 = M2;                             // stage-2 columns (mx)
    constexpr int K2 = 2 * K1;                         // stage-2 depth: sin block + cos block
    constexpr int NT1W = (NT1 + 3) / 4;                // stage-1 column tiles per wave
    constexpr int T2 = (M2 / 16) * (N2 / 16);          // stage-2 tiles
    const int n_m = 2 * P;

    __shared__ double Wv[J][J + 1];
    __shared__ double Ds[M1][K1 + 1];
    __shared__ double Ts[K2][N2 + 1];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;

    // trig operands in registers
    double b1[NT1W][K1 / 4];
#pragma unroll
    for (int q = 0; q < NT1W; ++q) {
        const int nt = wave + 4 * q;
#pragma unroll
        for (int ks = 0; ks < K1 / 4; ++ks) {
            const int jxi = 4 * ks + lk, n = nt * 16 + lr;
            double v = 0.0;
            if (nt < NT1 && jxi < J && n < 4 * P) {
                const int jx = jxi - P;
                const int mx = (n < 2 * P ? n : n - 2 * P) - P;
                const double w = w_end(jx, P);
                v = n < 2 * P ? w * sin_2pi_ratio((long)mx * jx, n_m) : w * cos_2pi_ratio((long)mx * jx, n_m);
            }
            b1[q][ks] = v;
        }
    }
    double a2[K2 / 4];
    const int tile2 = wave;                      // stage-2 tile of this wave (if any)
    const int tm2 = tile2 / (N2 / 16), tn2 = tile2 % (N2 / 16);
#pragma unroll
    for (int ks = 0; ks < K2 / 4; ++ks) {
        const int k = 4 * ks + lk, my_i = tm2 * 16 + lr;
        double v = 0.0;
        if (tile2 < T2 && my_i < 2 * P) {
            const int my = my_i - P;
            const int jyi = k < K1 ? k : k - K1;
            if (jyi < J) {
                const int jy = jyi - P;
                const double w = w_end(jy, P);
                v = k < K1 ? w * cos_2pi_ratio((long)my * jy, n_m) : w * sin_2pi_ratio((long)my * jy, n_m);
            }
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
        for (int e = threadIdx.x; e < J * J; e += KE_THREADS) {
            const int ty = e / J, tx = e - ty * J;
            const int yy = min(max(cy - P + ty, 0), ny - 1), xx = min(max(cx - P + tx, 0), nx - 1);
            Wv[ty][tx] = Vb[(long)yy * nx + xx];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < M1 * K1; e += KE_THREADS) {
            const int jyi = e / K1, jxi = e - jyi * K1;
            double d = 0.0;
            if (jyi < J && jxi < J) d = Wv[jyi][jxi] - Wv[J - 1 - jyi][J - 1 - jxi];
            Ds[jyi][jxi] = bad ? __builtin_nan("") : d;
        }
        __syncthreads();
        // stage 1 -> Ts (sin part rows 0..K1-1, cos part rows K1..2K1-1)
#pragma unroll
        for (int q = 0; q < NT1W; ++q) {
            const int nt = wave + 4 * q;
            if (nt >= NT1) continue;
#pragma unroll
            for (int mt = 0; mt < MT1; ++mt) {
                f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int ks = 0; ks < K1 / 4; ++ks)
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Ds[mt * 16 + lr][4 * ks + lk], b1[q][ks],
                                                             acc, 0, 0, 0);
                const int n = nt * 16 + lr;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int jyi = mt * 16 + lk + 4 * e;
                    if (jyi >= K1 || n >= 4 * P) continue;
                    if (n < 2 * P)
                        Ts[jyi][n] = acc[e];
                    else
                        Ts[K1 + jyi][n - 2 * P] = acc[e];
                }
            }
        }
        __syncthreads();
        if (tile2 < T2) {
            f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int ks = 0; ks < K2 / 4; ++ks) {
                const int k = 4 * ks + lk, mx_i = tn2 * 16 + lr;
                const double bv = mx_i < 2 * P ? Ts[k][mx_i] : 0.0;
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[ks], bv, acc, 0, 0, 0);
            }
            const int mx_i = tn2 * 16 + lr;
            // TAB: the row stays on chip, in the stage-1 operand tile (free after stage 1)
            double* o = TAB ? &Ds[0][0] : out + r * (long)n_m * n_m;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int my_i = tm2 * 16 + lk + 4 * e;
                if (my_i < 2 * P && mx_i < 2 * P) o[my_i * n_m + mx_i] = c2 * acc[e];
            }
        }
        if constexpr (TAB) {
            static_assert(M1 * (K1 + 1) >= 4 * P * P, "2-D row stage");
            __shared__ int last_s;
            tab_row_block(&Ds[0][0], 4 * P * P, r, tb, &last_s);
        }
    }
}

// d = 2 in 16-bit operands with FP32 sums (BF16 / FP16, and their hi/lo split forms): the same
// two stages on v_mfma_f32_16x16x32_{bf16,f16}.  Stage 1 contracts over jx: T[jy][n] =
// sum_jx D[jy][jx] B1[jx][n] (n < 2P: w sin, else w cos), D rounded from FP64 to 16 bits in
// LDS (hi, and for the split forms lo = round16(D - hi)); its FP32 result is rounded again
// (hi / lo) into a transposed tile Tt[mx][part * M1 + jy] (part 0: the sine columns, 1: the
// cosines), which stage 2 contracts over (part, jy) against A2[my][(part, jy)] = w cos / w sin.
// Split forms add the hi x lo and lo x hi products in both stages.  The trig operands depend on
// (n_m, lane) only and live in registers; workgroups loop over the requested cells.
template <int P, int PREC, bool TAB = false>
__global__ __launch_bounds__(KE_THREADS) void kernel_eval_2d_lowp(
    const double* __restrict__ V, int nx, int ny, long R, int n_cells,
    const int32_t* __restrict__ cells, float c2, float* __restrict__ out, TabOut tb) {
    typedef LowpTraits<PREC> TR;
    constexpr bool HALF = TR::half, SPLIT = TR::split;
    constexpr int NS = SPLIT ? 2 : 1;
    constexpr int J = 2 * P + 1;
    constexpr int M1 = (J + 15) / 16 * 16, K1 = (J + 31) / 32 * 32, N1 = 4 * P;
    constexpr int MT1 = M1 / 16, KS1 = K1 / 32, NT1 = N1 / 16, NT1W = (NT1 + 3) / 4;
    constexpr int K2 = 2 * M1, KS2 = K2 / 32;
    constexpr int M2 = (2 * P + 15) / 16 * 16, N2 = M2, T2 = (M2 / 16) * (N2 / 16);
    constexpr int LD1 = K1 + 8, LD2 = K2 + 8;  // 16-bit row strides (16-byte aligned rows)
    static_assert(N1 % 16 == 0 && K2 % 32 == 0, "2-D tile shapes");
    static_assert(T2 <= 4, "one stage-2 tile per wave");
    const int n_m = 2 * P;

    __shared__ double Wv[J][J + 1];
    __shared__ __attribute__((aligned(16))) uint16_t Ds[NS][M1][LD1];
    __shared__ __attribute__((aligned(16))) uint16_t Tt[NS][N2][LD2];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    // hi / lo 16-bit bits of a double (lo: the rounding remainder, exact in FP64)
    auto split16 = [&](double v, uint16_t* hi, uint16_t* lo) {
        const uint32_t h = pack16<HALF>(v, 0.0) & 0xFFFFu;
        *hi = (uint16_t)h;
        if constexpr (SPLIT) *lo = (uint16_t)(pack16<HALF>(v - value16<HALF>(h), 0.0) & 0xFFFFu);
    };
    // stage-1 B operand: lane holds B1[jx = 32 ks + 8 lk + i][n = 16 nt + lr], i < 8
    s16x8 b1[NT1W][KS1][NS];
#pragma unroll
    for (int q = 0; q < NT1W; ++q) {
        const int nt = wave + 4 * q;
#pragma unroll
        for (int ks = 0; ks < KS1; ++ks) {
            uint16_t h[8], l[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int jxi = 32 * ks + 8 * lk + i, n = nt * 16 + lr;
                double v = 0.0;
                if (nt < NT1 && jxi < J) {
                    const int jx = jxi - P, mx = (n < 2 * P ? n : n - 2 * P) - P;
                    const double w = w_end(jx, P);
                    v = n < 2 * P ? w * sin_2pi_ratio((long)mx * jx, n_m) : w * cos_2pi_ratio((long)mx * jx, n_m);
                }
                split16(v, &h[i], &l[i]);
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                b1[q][ks][0][i] = (short)h[i];
                if constexpr (SPLIT) b1[q][ks][NS - 1][i] = (short)l[i];
            }
        }
    }
    // stage-2 A operand: lane holds A2[my = 16 tm2 + lr][k = 32 ks + 8 lk + i], k = part M1 + jy
    const int tm2 = wave / (N2 / 16), tn2 = wave % (N2 / 16);
    s16x8 a2[KS2][NS];
#pragma unroll
    for (int ks = 0; ks < KS2; ++ks) {
        uint16_t h[8], l[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int k = 32 * ks + 8 * lk + i, my_i = tm2 * 16 + lr;
            const int part = k / M1, jyi = k - part * M1;
            double v = 0.0;
            if (wave < T2 && my_i < 2 * P && jyi < J) {
                const int my = my_i - P, jy = jyi - P;
                const double w = w_end(jy, P);
                v = part == 0 ? w * cos_2pi_ratio((long)my * jy, n_m) : w * sin_2pi_ratio((long)my * jy, n_m);
            }
            split16(v, &h[i], &l[i]);
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            a2[ks][0][i] = (short)h[i];
            if constexpr (SPLIT) a2[ks][NS - 1][i] = (short)l[i];
        }
    }
    // padding of the transposed tile (columns mx >= 2P) stays zero
    for (int e = threadIdx.x; e < NS * N2 * LD2; e += KE_THREADS) (&Tt[0][0][0])[e] = 0;

    for (long r = blockIdx.x; r < R; r += gridDim.x) {
        const long b = r / n_cells;
        const int ci = (int)(r - b * n_cells);
        int cell = cells ? cells[ci] : ci;
        const bool bad = cell < 0 || cell >= nx * ny;
        if (bad) cell = 0;
        const int cx = cell % nx, cy = cell / nx;
        const double* Vb = V + b * (long)nx * ny;
        __syncthreads();  // previous cell's LDS use is over
        for (int e = threadIdx.x; e < J * J; e += KE_THREADS) {
            const int ty = e / J, tx = e - ty * J;
            const int yy = min(max(cy - P + ty, 0), ny - 1), xx = min(max(cx - P + tx, 0), nx - 1);
            Wv[ty][tx] = Vb[(long)yy * nx + xx];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < M1 * K1; e += KE_THREADS) {
            const int jyi = e / K1, jxi = e - jyi * K1;
            double d = 0.0;
            if (jyi < J && jxi < J) d = Wv[jyi][jxi] - Wv[J - 1 - jyi][J - 1 - jxi];
            if (bad) d = __builtin_nan("");
            uint16_t h, l = 0;
            split16(d, &h, &l);
            Ds[0][jyi][jxi] = h;
            if constexpr (SPLIT) Ds[NS - 1][jyi][jxi] = l;
        }
        __syncthreads();
        // stage 1 -> Tt (rounded to 16 bits, transposed)
#pragma unroll
        for (int q = 0; q < NT1W; ++q) {
            const int nt = wave + 4 * q;
            if (nt >= NT1) continue;
#pragma unroll
            for (int mt = 0; mt < MT1; ++mt) {
                f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < KS1; ++ks) {
                    const s16x8 ah = *reinterpret_cast<const s16x8*>(&Ds[0][mt * 16 + lr][32 * ks + 8 * lk]);
                    acc = mfma16<HALF>(ah, b1[q][ks][0], acc);
                    if constexpr (SPLIT) {
                        const s16x8 al = *reinterpret_cast<const s16x8*>(&Ds[NS - 1][mt * 16 + lr][32 * ks + 8 * lk]);
                        acc = mfma16<HALF>(ah, b1[q][ks][NS - 1], acc);
                        acc = mfma16<HALF>(al, b1[q][ks][0], acc);
                    }
                }
                const int n = nt * 16 + lr, part = n < 2 * P ? 0 : 1, mx = n - part * 2 * P;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int jy = mt * 16 + 4 * lk + e;
                    uint16_t h, l = 0;
                    split16((double)acc[e], &h, &l);
                    Tt[0][mx][part * M1 + jy] = h;
                    if constexpr (SPLIT) Tt[NS - 1][mx][part * M1 + jy] = l;
                }
            }
        }
        __syncthreads();
        if (wave < T2) {
            f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < KS2; ++ks) {
                const s16x8 bh = *reinterpret_cast<const s16x8*>(&Tt[0][tn2 * 16 + lr][32 * ks + 8 * lk]);
                acc = mfma16<HALF>(a2[ks][0], bh, acc);
                if constexpr (SPLIT) {
                    const s16x8 bl = *reinterpret_cast<const s16x8*>(&Tt[NS - 1][tn2 * 16 + lr][32 * ks + 8 * lk]);
                    acc = mfma16<HALF>(a2[ks][0], bl, acc);
                    acc = mfma16<HALF>(a2[ks][NS - 1], bh, acc);
                }
            }
            const int mx_i = tn2 * 16 + lr;
            if constexpr (TAB) {
                // the row stays on chip as the FP32 values the kernel would store, widened to
                // FP64, in the window tile (free once the differences are formed)
                double* Kr = &Wv[0][0];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int my_i = tm2 * 16 + 4 * lk + e;
                    if (my_i < 2 * P && mx_i < 2 * P) Kr[my_i * n_m + mx_i] = (double)(c2 * acc[e]);
                }
            } else {
                float* o = out + r * (long)n_m * n_m;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int my_i = tm2 * 16 + 4 * lk + e;
                    if (my_i < 2 * P && mx_i < 2 * P) o[my_i * n_m + mx_i] = c2 * acc[e];
                }
            }
        }
        if constexpr (TAB) {
            static_assert(J * (J + 1) >= 4 * P * P, "2-D row stage");
            __shared__ int last_s;
            tab_row_block(&Wv[0][0], 4 * P * P, r, tb, &last_s);
        }
    }
}

template <int PREC, bool TAB = false>
static int launch_2d_lowp(const wk_mesh* mesh, const double* V, int B, const int32_t* cells, int n_cells,
                          float* out, const TabOut& tb, hipStream_t stream) {
    const long R = (long)B * n_cells;
    if (R == 0) return WK_OK;
    const float c2 = (float)(-1.0 / (mesh->hbar * (double)mesh->n_m * (double)mesh->n_m));
    const unsigned grid = (unsigned)(R < 4096 ? R : 4096);
    const char* name = TAB ? "kernel_tables_2d_lowp" : "kernel_eval_2d_lowp";
    switch (mesh->n_m) {
        case 8:
            WK_LAUNCH(name, (kernel_eval_2d_lowp<4, PREC, TAB>), dim3(grid), dim3(KE_THREADS), 0,
                      stream, V, mesh->nx, mesh->ny, R, n_cells, cells, c2, out, tb);
            break;
        case 16:
            WK_LAUNCH(name, (kernel_eval_2d_lowp<8, PREC, TAB>), dim3(grid), dim3(KE_THREADS), 0,
                      stream, V, mesh->nx, mesh->ny, R, n_cells, cells, c2, out, tb);
            break;
        case 32:
            WK_LAUNCH(name, (kernel_eval_2d_lowp<16, PREC, TAB>), dim3(grid), dim3(KE_THREADS), 0,
                      stream, V, mesh->nx, mesh->ny, R, n_cells, cells, c2, out, tb);
            break;
        default:
            return fail(WK_EINVAL, TAB ? "wk_kernel_tables: 2-D supports n_m = 8, 16 and 32"
                                       : "wk_kernel_eval: 2-D supports n_m = 8, 16 and 32");
    }
    return check_launch(name);
}

int kernel_eval_2d_16(const wk_mesh* mesh, const double* V, int B, const int32_t* cells, int n_cells,
                      int prec, float* out, hipStream_t stream) {
    switch (prec) {
        case WK_BF16: return launch_2d_lowp<WK_BF16>(mesh, V, B, cells, n_cells, out, TabOut{}, stream);
        case WK_FP16: return launch_2d_lowp<WK_FP16>(mesh, V, B, cells, n_cells, out, TabOut{}, stream);
        case WK_BF16X3: return launch_2d_lowp<WK_BF16X3>(mesh, V, B, cells, n_cells, out, TabOut{}, stream);
        case WK_FP16X3: return launch_2d_lowp<WK_FP16X3>(mesh, V, B, cells, n_cells, out, TabOut{}, stream);
        default: return fail(WK_EINVAL, "wk_kernel_eval: unknown precision");
    }
}

// The 2-D 16-bit forms' rows straight into the creation tables (the tables of the FP32 rows
// kernel_eval_2d_16 would write).
int kernel_tables_2d_16(const wk_mesh* mesh, const double* V, int B, const int32_t* cells, int n_cells,
                        int prec, const TabOut& tb, hipStream_t stream) {
    WK_REQUIRE(tb.guide == nullptr || (tb.G >= 1 && tb.G <= TAB_GMAX),
               "wk_kernel_tables: guide_len must lie in [1, 256]");
    switch (prec) {
        case WK_BF16: return launch_2d_lowp<WK_BF16, true>(mesh, V, B, cells, n_cells, nullptr, tb, stream);
        case WK_FP16: return launch_2d_lowp<WK_FP16, true>(mesh, V, B, cells, n_cells, nullptr, tb, stream);
        case WK_BF16X3: return launch_2d_lowp<WK_BF16X3, true>(mesh, V, B, cells, n_cells, nullptr, tb, stream);
        case WK_FP16X3: return launch_2d_lowp<WK_FP16X3, true>(mesh, V, B, cells, n_cells, nullptr, tb, stream);
        default: return fail(WK_EINVAL, "wk_kernel_tables: unknown precision");
    }
}

// d = 2 rows, written out (TAB = false) or turned into the creation tables on chip (TAB).
template <bool TAB>
static int launch_2d(const wk_mesh* mesh, const double* V, int B, const int32_t* cells, int n_cells,
                     double* out, const TabOut& tb, hipStream_t stream) {
    const long R = (long)B * n_cells;
    if (R == 0) return WK_OK;
    const double c2 = -1.0 / (mesh->hbar * (double)mesh->n_m * (double)mesh->n_m);
    const unsigned grid = (unsigned)(R < 4096 ? R : 4096);
    const char* name = TAB ? "kernel_tables_2d_f64" : "kernel_eval_2d_f64";
    switch (mesh->n_m) {
        case 8:
            WK_LAUNCH(name, (kernel_eval_2d_f64<4, TAB>), dim3(grid), dim3(KE_THREADS), 0, stream,
                      V, mesh->nx, mesh->ny, R, n_cells, cells, c2, out, tb);
            break;
        case 16:
            WK_LAUNCH(name, (kernel_eval_2d_f64<8, TAB>), dim3(grid), dim3(KE_THREADS), 0, stream,
                      V, mesh->nx, mesh->ny, R, n_cells, cells, c2, out, tb);
            break;
        case 32:
            WK_LAUNCH(name, (kernel_eval_2d_f64<16, TAB>), dim3(grid), dim3(KE_THREADS), 0, stream,
                      V, mesh->nx, mesh->ny, R, n_cells, cells, c2, out, tb);
            break;
        default:
            return fail(WK_EINVAL, TAB ? "wk_kernel_tables: 2-D supports n_m = 8, 16 and 32"
                                       : "wk_kernel_eval: 2-D supports n_m = 8, 16 and 32");
    }
    return check_launch(name);
}

int kernel_eval_2d(const wk_mesh* mesh, const double* V, int B, const int32_t* cells, int n_cells,
                   double* out, hipStream_t stream) {
    return launch_2d<false>(mesh, V, B, cells, n_cells, out, TabOut{}, stream);
}

int kernel_tables_2d(const wk_mesh* mesh, const double* V, int B, const int32_t* cells, int n_cells,
                     const TabOut& tb, hipStream_t stream) {
    WK_REQUIRE(tb.guide == nullptr || (tb.G >= 1 && tb.G <= TAB_GMAX),
               "wk_kernel_tables: guide_len must lie in [1, 256]");
    return launch_2d<true>(mesh, V, B, cells, n_cells, nullptr, tb, stream);
}

}  // namespace wk
