// Signed-particle passes (Sec. 2.1): pair creation + field-less drift + absorbing boundaries
// (sp_step), annihilation on the (cell, momentum) grid (sp_annihilate), initial placement
// (sp_init) and the rule-1 read-out (sp_density).
//
// Layout: struct-of-arrays in HBM, positions in cell units.  Every pass streams the
// arrays once or twice with coalesced accesses.  Ordered outputs (appended children,
// compacted survivors) use a fixed grid of PB workgroups, each owning one contiguous
// chunk of particle ids: pass 1 counts per chunk, a single workgroup scans the chunk
// counts, pass 2 re-derives the per-particle counts and scans them inside the workgroup.
// Output positions therefore depend only on the data, never on scheduling, and there
// are no floating-point atomics anywhere (integer atomics only for histogram counts).
#include <climits>

#include "wk_internal.h"

namespace wk {

constexpr int PB = 2048;    // workgroups of the chunked passes
constexpr int PT = 256;     // threads per workgroup

struct Geo {
    int dim, nx, ny, n_m, n_k, M_min, P, fb;
    long width;       // table entries per row (n_m or n_m^2)
    long n_bins;
    double vdt;
    uint64_t seed;
};

// Workspace (sp_workspace_size): int64 scalars[16] | int64 counts[PB] | int64 offs[PB] |
// int64 bpart[PB] | int64 boffs[PB] | int32 binoff[n_bins].
enum { SC_N_OLD = 0, SC_GO = 1, SC_TOTAL = 2, SC_KEPT = 3, SC_NBIN_TOTAL = 4 };

struct WS {
    long long* sc;
    long long* counts;
    long long* offs;
    long long* bpart;
    long long* boffs;
    int* binoff;
};

static WS carve(void* ws) {
    WS w;
    char* p = static_cast<char*>(ws);
    w.sc = reinterpret_cast<long long*>(p);
    w.counts = w.sc + 16;
    w.offs = w.counts + PB;
    w.bpart = w.offs + PB;
    w.boffs = w.bpart + PB;
    w.binoff = reinterpret_cast<int*>(w.boffs + PB);
    return w;
}

static size_t ws_bytes_for(long n_bins) {
    return sizeof(long long) * (16 + 4 * (size_t)PB) + sizeof(int) * (size_t)(n_bins + 1);
}

constexpr int IT = 4;          // particles per thread in the streaming passes
constexpr int TILE = PT * IT;  // particles per workgroup iteration

__device__ __forceinline__ void chunk_of(long n, long* lo, long* hi) {
    long chunk = (n + PB - 1) / PB;
    chunk = (chunk + TILE - 1) / TILE * TILE;
    *lo = (long)blockIdx.x * chunk;
    *hi = min(n, *lo + chunk);
    if (*lo > n) *lo = n;
}

template <typename T>
__device__ __forceinline__ int cell_index(T x, int n) {
    if (!(x >= (T)0) || !(x < (T)n)) return -1;
    return (int)x;  // x >= 0: truncation is floor
}

template <typename T>
__device__ __forceinline__ T cell_plus_frac(int c, uint32_t u, int fb) {
    const T frac = (T)(u >> (32 - fb)) * (T)ldexp(1.0, -fb);
    return (T)c + frac;
}

// Histogram bin of a particle, -1 when dead or outside the grid.
template <typename T, int DIM>
__device__ __forceinline__ long bin_val(const Geo& g, T x, T y, int m, int my, int8_t s) {
    if (s == 0) return -1;
    const int cx = cell_index<T>(x, g.nx);
    if (cx < 0) return -1;
    const int kx = m - g.M_min;
    if (kx < 0 || kx >= g.n_k) return -1;
    if (DIM == 1) return (long)cx * g.n_k + kx;
    const int cy = cell_index<T>(y, g.ny);
    if (cy < 0) return -1;
    const int ky = my - g.M_min;
    if (ky < 0 || ky >= g.n_k) return -1;
    return (((long)cy * g.nx + cx) * g.n_k + ky) * g.n_k + kx;
}

// Four consecutive particles (ids id .. id+3, id a multiple of 4) loaded with 16-byte
// (positions, int32 momenta), 8-byte (int16 momenta) and 4-byte (signs) accesses;
// slots at or beyond hi read as dead.
template <typename T, int DIM>
struct Part4 {
    T x[IT], y[IT];
    int m[IT], my[IT];
    int8_t s[IT];
};

__device__ __forceinline__ void ld4(const float* p, long i, float* v) {
    const float4 t = *reinterpret_cast<const float4*>(p + i);
    v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
}
__device__ __forceinline__ void ld4(const double* p, long i, double* v) {
    const double2 a = *reinterpret_cast<const double2*>(p + i);
    const double2 b = *reinterpret_cast<const double2*>(p + i + 2);
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
__device__ __forceinline__ void ld4(const int32_t* p, long i, int* v) {
    const int4 t = *reinterpret_cast<const int4*>(p + i);
    v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
}
__device__ __forceinline__ void ld4(const int16_t* p, long i, int* v) {
    const short4 t = *reinterpret_cast<const short4*>(p + i);
    v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
}
__device__ __forceinline__ void ld4(const int8_t* p, long i, int8_t* v) {
    const char4 t = *reinterpret_cast<const char4*>(p + i);
    v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
}
__device__ __forceinline__ void st4(float* p, long i, const float* v) {
    *reinterpret_cast<float4*>(p + i) = make_float4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void st4(double* p, long i, const double* v) {
    *reinterpret_cast<double2*>(p + i) = make_double2(v[0], v[1]);
    *reinterpret_cast<double2*>(p + i + 2) = make_double2(v[2], v[3]);
}

template <typename T, typename MT, int DIM>
__device__ __forceinline__ void load4(const T* x, const T* y, const MT* M, const MT* My,
                                      const int8_t* s, long id, long hi, Part4<T, DIM>& p) {
    if (id + IT <= hi) {
        ld4(x, id, p.x);
        ld4(M, id, p.m);
        ld4(s, id, p.s);
        if (DIM == 2) {
            ld4(y, id, p.y);
            ld4(My, id, p.my);
        }
    } else {
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const bool v = id + k < hi;
            p.x[k] = v ? x[id + k] : (T)0;
            p.m[k] = v ? (int)M[id + k] : 0;
            p.s[k] = v ? s[id + k] : (int8_t)0;
            p.y[k] = (DIM == 2 && v) ? y[id + k] : (T)0;
            p.my[k] = (DIM == 2 && v) ? (int)My[id + k] : 0;
        }
    }
    if (DIM == 1) {
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            p.y[k] = (T)0;
            p.my[k] = 0;
        }
    }
}

// Pairs created by particle id this step (postulate II with the integer tables).
template <typename T, int DIM>
__device__ __forceinline__ int pairs_of(const Geo& g, uint32_t id, uint32_t step, T px, T py,
                                        int8_t sv, const int32_t* __restrict__ cell_slot,
                                        const uint32_t* __restrict__ n0,
                                        const uint32_t* __restrict__ thr, int* slot, u32x4* w) {
    *slot = -1;
    if (sv == 0) return 0;
    const int cx = cell_index<T>(px, g.nx);
    if (cx < 0) return 0;
    int c = cx;
    if (DIM == 2) {
        const int cy = cell_index<T>(py, g.ny);
        if (cy < 0) return 0;
        c = cy * g.nx + cx;
    }
    const int sl = cell_slot[c];
    if (sl < 0) return 0;
    *slot = sl;
    *w = philox(id, step, 0u, TAG_CREATE, g.seed);
    return (int)n0[sl] + (w->v[0] < thr[sl] ? 1 : 0);
}

__device__ __forceinline__ int sample_cdf(const uint64_t* __restrict__ T, long width, uint32_t u) {
    // smallest t with u < T[t]; T is non-decreasing and ends at 2^32 > u
    long lo = 0, hi = width - 1;
    while (lo < hi) {
        const long mid = (lo + hi) >> 1;
        if ((uint64_t)u < T[mid])
            hi = mid;
        else
            lo = mid + 1;
    }
    return (int)lo;
}

// Field-less drift over one step, x <- fma(M, vdt, x) in the position precision.
__device__ __forceinline__ float drift(float x, int M, float vdt) { return fmaf((float)M, vdt, x); }
__device__ __forceinline__ double drift(double x, int M, double vdt) { return fma((double)M, vdt, x); }

template <typename T>
__device__ __forceinline__ bool inside(T x, int n) {
    return x >= (T)0 && x < (T)n;
}

// ----------------------------------------------------------------------------- sp_step
template <typename T, typename MT, int DIM>
__global__ __launch_bounds__(PT) void step_count(Geo g, uint32_t step, const int32_t* cell_slot,
                                                 const uint32_t* n0, const uint32_t* thr,
                                                 const T* x, const T* y, const MT* M,
                                                 const MT* My, const int8_t* s,
                                                 const long long* d_n, const long long* stats,
                                                 WS w) {
    __shared__ long long red[PT / 64];
    long long cnt = 0;
    if (stats[WK_ST_OVERFLOW] == 0) {
        long lo, hi;
        chunk_of(*d_n, &lo, &hi);
        for (long t0 = lo; t0 < hi; t0 += TILE) {
            const long id = t0 + IT * threadIdx.x;
            Part4<T, DIM> p;
            load4<T, MT, DIM>(x, y, M, My, s, id, hi, p);
#pragma unroll
            for (int k = 0; k < IT; ++k) {
                int slot;
                u32x4 r;
                cnt += pairs_of<T, DIM>(g, (uint32_t)(id + k), step, p.x[k], p.y[k], p.s[k],
                                        cell_slot, n0, thr, &slot, &r);
            }
        }
    }
    cnt = wave_sum_ll(cnt);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) w.counts[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Exclusive scan of PB int64 values by one workgroup of PT threads (PB / PT per thread).
__device__ void scan_pb(const long long* in, long long* out, long long* total) {
    __shared__ long long part[PT];
    constexpr int per = PB / PT;
    long long loc[per];
    long long s = 0;
    for (int k = 0; k < per; ++k) {
        loc[k] = in[threadIdx.x * per + k];
        s += loc[k];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long run = 0;
        for (int k = 0; k < PT; ++k) {
            long long v = part[k];
            part[k] = run;
            run += v;
        }
        *total = run;
    }
    __syncthreads();
    long long run = part[threadIdx.x];
    for (int k = 0; k < per; ++k) {
        out[threadIdx.x * per + k] = run;
        run += loc[k];
    }
}

__global__ __launch_bounds__(PT) void step_scan(long long* d_n, long long capacity,
                                                long long* stats, long long step, WS w) {
    __shared__ long long total;
    const bool sticky = stats[WK_ST_OVERFLOW] != 0;
    scan_pb(w.counts, w.offs, &total);
    if (threadIdx.x != 0) return;
    if (sticky) {
        w.sc[SC_GO] = 0;
        return;
    }
    const long long n = *d_n;
    const long long needed = n + 2 * total;
    if (needed > capacity) {
        stats[WK_ST_NEEDED] = needed;
        stats[WK_ST_OVERFLOW] = 1;
        stats[WK_ST_OVERFLOW_STEP] = step;
        w.sc[SC_GO] = 0;
        return;
    }
    w.sc[SC_N_OLD] = n;
    w.sc[SC_GO] = 1;
    stats[WK_ST_N] = needed;
    stats[WK_ST_PAIRS] = total;
    stats[WK_ST_CUM_STEPS] += 1;
    stats[WK_ST_CUM_N] += n;
    stats[WK_ST_CUM_PAIRS] += total;
    stats[WK_ST_ABS_X] = 0;
    stats[WK_ST_ABS_M] = 0;
    stats[WK_ST_NEEDED] = 0;
    *d_n = needed;
}

template <typename T, typename MT, int DIM>
__global__ __launch_bounds__(PT) void step_apply(Geo g, uint32_t step, const int32_t* cell_slot,
                                                 const uint32_t* n0, const uint32_t* thr,
                                                 const uint64_t* cdf, T* x, T* y, MT* M, MT* My,
                                                 int8_t* s, long long* stats, WS w) {
    __shared__ int lds5[5];
    __shared__ long long red[2][PT / 64];
    if (w.sc[SC_GO] == 0) return;
    const long n = (long)w.sc[SC_N_OLD];
    long lo, hi;
    chunk_of(n, &lo, &hi);
    long long run = w.offs[blockIdx.x];
    const T vdt = (T)g.vdt;
    long long abs_x = 0, abs_m = 0;
    auto absorbed = [&](T nx_, T ny_, int m, int my) -> int {
        bool outx = !inside<T>(nx_, g.nx);
        if (DIM == 2) outx = outx || !inside<T>(ny_, g.ny);
        bool outm = m < g.M_min || m >= g.M_min + g.n_k;
        if (DIM == 2) outm = outm || my < g.M_min || my >= g.M_min + g.n_k;
        return outx ? 1 : (outm ? 2 : 0);
    };
    for (long t0 = lo; t0 < hi; t0 += TILE) {  // uniform trip count in the workgroup
        const long id = t0 + IT * threadIdx.x;
        Part4<T, DIM> p;
        load4<T, MT, DIM>(x, y, M, My, s, id, hi, p);
        int slot[IT];
        u32x4 r[IT];
        int np[IT], npt = 0;
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            np[k] = pairs_of<T, DIM>(g, (uint32_t)(id + k), step, p.x[k], p.y[k], p.s[k], cell_slot,
                                     n0, thr, &slot[k], &r[k]);
            npt += np[k];
        }
        int tot;
        const int ex = block_excl_scan_256(npt, &tot, lds5);
        long o = n + 2 * (long)(run + ex);
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            for (int q = 0; q < np[k]; ++q) {
                uint32_t u;
                if (q < 3) {
                    u = q == 0 ? r[k].v[1] : (q == 1 ? r[k].v[2] : r[k].v[3]);
                } else {
                    const u32x4 r2 = philox((uint32_t)(id + k), step, (uint32_t)(1 + (q - 3) / 4),
                                            TAG_CREATE, g.seed);
                    const int wq = (q - 3) & 3;
                    u = wq == 0 ? r2.v[0] : (wq == 1 ? r2.v[1] : (wq == 2 ? r2.v[2] : r2.v[3]));
                }
                const int t = sample_cdf(cdf + (long)slot[k] * g.width, g.width, u);
                const int mx = (DIM == 1 ? t : t % g.n_m) - g.P;
                const int my = DIM == 1 ? 0 : t / g.n_m - g.P;
#pragma unroll
                for (int ch = 0; ch < 2; ++ch, ++o) {
                    const int sg = ch == 0 ? 1 : -1;
                    const int cm = p.m[k] + sg * mx, cmy = p.my[k] + sg * my;
                    const T cx = drift(p.x[k], cm, vdt);
                    const T cy = DIM == 2 ? drift(p.y[k], cmy, vdt) : (T)0;
                    const int a = absorbed(cx, cy, cm, cmy);
                    abs_x += a == 1;
                    abs_m += a == 2;
                    x[o] = cx;
                    M[o] = (MT)cm;
                    if (DIM == 2) {
                        y[o] = cy;
                        My[o] = (MT)cmy;
                    }
                    s[o] = a ? (int8_t)0 : (int8_t)(sg * p.s[k]);
                }
            }
        }
        // parents: drift in place, absorb
        T nxv[IT], nyv[IT];
        bool sdirty = false;
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            nxv[k] = p.x[k];
            nyv[k] = p.y[k];
            if (p.s[k] != 0) {
                nxv[k] = drift(p.x[k], p.m[k], vdt);
                if (DIM == 2) nyv[k] = drift(p.y[k], p.my[k], vdt);
                const int a = absorbed(nxv[k], nyv[k], p.m[k], p.my[k]);
                abs_x += a == 1;
                abs_m += a == 2;
                if (a) {
                    p.s[k] = 0;
                    sdirty = true;
                }
            }
        }
        if (id + IT <= hi) {
            st4(x, id, nxv);
            if (DIM == 2) st4(y, id, nyv);
            if (sdirty)
                *reinterpret_cast<char4*>(s + id) = make_char4(p.s[0], p.s[1], p.s[2], p.s[3]);
        } else {
#pragma unroll
            for (int k = 0; k < IT; ++k) {
                if (id + k < hi) {
                    x[id + k] = nxv[k];
                    if (DIM == 2) y[id + k] = nyv[k];
                    s[id + k] = p.s[k];
                }
            }
        }
        run += tot;
    }
    abs_x = wave_sum_ll(abs_x);
    abs_m = wave_sum_ll(abs_m);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = abs_x;
        red[1][threadIdx.x >> 6] = abs_m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const long long ax = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        const long long am = red[1][0] + red[1][1] + red[1][2] + red[1][3];
        if (ax) atomicAdd(reinterpret_cast<unsigned long long*>(&stats[WK_ST_ABS_X]), (unsigned long long)ax);
        if (am) atomicAdd(reinterpret_cast<unsigned long long*>(&stats[WK_ST_ABS_M]), (unsigned long long)am);
    }
}

// ----------------------------------------------------------------------------- bins
// Per-bin output counts: from caller counts (init) or |H+ - H-| of mixed bins (annihilation).
struct BinCount {
    const int32_t* counts;  // init mode
    const int32_t* hist;    // annihilation mode: [2][n_bins]
    long n_bins;
    __device__ __forceinline__ long operator()(long b) const {
        if (counts) return counts[b] > 0 ? counts[b] : 0;
        const int hp = hist[b], hm = hist[n_bins + b];
        if (hp > 0 && hm > 0) return hp > hm ? hp - hm : hm - hp;
        return 0;
    }
    __device__ __forceinline__ bool mixed(long b) const {
        return !counts && hist[b] > 0 && hist[n_bins + b] > 0;
    }
};

__device__ __forceinline__ void bin_chunk(long n_bins, long* lo, long* hi) {
    long chunk = (n_bins + PB - 1) / PB;
    *lo = min(n_bins, (long)blockIdx.x * chunk);
    *hi = min(n_bins, *lo + chunk);
}

__global__ __launch_bounds__(PT) void bins_reduce(BinCount bc, const long long* stats, WS w) {
    __shared__ long long red[2][PT / 64];
    long long c = 0, mixed = 0;
    if (stats[WK_ST_OVERFLOW] == 0) {
        long lo, hi;
        bin_chunk(bc.n_bins, &lo, &hi);
        for (long b = lo + threadIdx.x; b < hi; b += PT) {
            c += bc(b);
            mixed += bc.mixed(b) ? 1 : 0;
        }
    }
    c = wave_sum_ll(c);
    mixed = wave_sum_ll(mixed);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = c;
        red[1][threadIdx.x >> 6] = mixed;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        w.bpart[blockIdx.x] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        w.counts[blockIdx.x] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
}

// mode 0 (init): out count = total; mode 1 (annihilation): out count = kept + total.
__global__ __launch_bounds__(PT) void bins_scan(int mode, long long* d_n_out, long long capacity,
                                                long long* stats, WS w) {
    __shared__ long long total;
    __shared__ long long mixed_total;
    scan_pb(w.bpart, w.boffs, &total);
    __syncthreads();
    {
        __shared__ long long red[PT / 64];
        long long m = 0;
        for (int k = threadIdx.x; k < PB; k += PT) m += w.counts[k];
        m = wave_sum_ll(m);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
        __syncthreads();
        if (threadIdx.x == 0) mixed_total = red[0] + red[1] + red[2] + red[3];
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    if (stats[WK_ST_OVERFLOW] != 0) {
        w.sc[SC_GO] = 0;
        return;
    }
    const long long base = mode == 0 ? 0 : w.sc[SC_KEPT];
    const long long n_out = base + total;
    if (n_out > capacity) {
        stats[WK_ST_NEEDED] = n_out;
        stats[WK_ST_OVERFLOW] = 1;
        w.sc[SC_GO] = 0;
        return;
    }
    w.sc[SC_GO] = 1;
    w.sc[SC_NBIN_TOTAL] = total;
    stats[WK_ST_N] = n_out;
    if (mode == 1) {
        stats[WK_ST_KEPT] = base;
        stats[WK_ST_REGEN] = total;
        stats[WK_ST_MIXED] = mixed_total;
        stats[WK_ST_CUM_ANNIH_IN] += w.sc[SC_N_OLD];
        stats[WK_ST_CUM_KEPT] += base;
        stats[WK_ST_CUM_REGEN] += total;
    } else {
        stats[WK_ST_NEEDED] = 0;
    }
    *d_n_out = n_out;
}

__global__ __launch_bounds__(PT) void bins_downsweep(BinCount bc, int mode, WS w) {
    __shared__ int lds5[5];
    if (w.sc[SC_GO] == 0) return;
    long lo, hi;
    bin_chunk(bc.n_bins, &lo, &hi);
    long long run = w.boffs[blockIdx.x] + (mode == 0 ? 0 : w.sc[SC_KEPT]);
    for (long base = lo; base < hi; base += PT) {
        const long b = base + threadIdx.x;
        const int c = b < hi ? (int)bc(b) : 0;
        int tot;
        const int ex = block_excl_scan_256(c, &tot, lds5);
        if (b < hi) w.binoff[b] = (int)(run + ex);
        run += tot;
    }
}

// Particle slot o of the bin range -> its bin: the largest b in [lo, hi) with binoff[b] <= o.
__device__ __forceinline__ long find_bin(const int* binoff, long lo, long hi, long o) {
    while (lo < hi) {
        const long mid = (lo + hi) >> 1;
        if ((long)binoff[mid] <= o)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo - 1;
}

// Each workgroup fills a contiguous range of output slots; the bins covering the range are
// bracketed once per workgroup, so each slot searches only a few bins.
template <typename T, typename MT, int DIM>
__global__ __launch_bounds__(PT) void bins_place(Geo g, BinCount bc, int mode, uint32_t c1,
                                                 uint32_t tag, T* x, T* y, MT* M, MT* My,
                                                 int8_t* s, WS w) {
    __shared__ long brange[2];
    if (w.sc[SC_GO] == 0) return;
    const long base = mode == 0 ? 0 : (long)w.sc[SC_KEPT];
    const long total = (long)w.sc[SC_NBIN_TOTAL];
    const long chunk = (total + gridDim.x - 1) / gridDim.x;
    const long k_lo = min(total, (long)blockIdx.x * chunk), k_hi = min(total, k_lo + chunk);
    if (k_lo >= k_hi) return;
    if (threadIdx.x == 0) {
        brange[0] = find_bin(w.binoff, 0, g.n_bins, base + k_lo);
        brange[1] = find_bin(w.binoff, 0, g.n_bins, base + k_hi - 1) + 1;
    }
    __syncthreads();
    const long blo = brange[0], bhi = brange[1];
    for (long k = k_lo + threadIdx.x; k < k_hi; k += PT) {
        const long o = base + k;
        const long b = find_bin(w.binoff, blo, bhi, o);
        const long r = o - w.binoff[b];
        int8_t sign = 1;
        if (mode == 1) sign = bc.hist[b] > bc.hist[g.n_bins + b] ? 1 : -1;
        if (DIM == 1) {
            const int cx = (int)(b / g.n_k), kx = (int)(b % g.n_k);
            const u32x4 u = philox((uint32_t)b, c1, (uint32_t)(r >> 2), tag, g.seed);
            const int wq = (int)(r & 3);
            const uint32_t uw = wq == 0 ? u.v[0] : (wq == 1 ? u.v[1] : (wq == 2 ? u.v[2] : u.v[3]));
            x[o] = cell_plus_frac<T>(cx, uw, g.fb);
            M[o] = (MT)(g.M_min + kx);
        } else {
            const int kx = (int)(b % g.n_k), ky = (int)((b / g.n_k) % g.n_k);
            const long c = b / ((long)g.n_k * g.n_k);
            const int cx = (int)(c % g.nx), cy = (int)(c / g.nx);
            const u32x4 u = philox((uint32_t)b, c1, (uint32_t)(r >> 1), tag, g.seed);
            const bool odd = (r & 1) != 0;
            x[o] = cell_plus_frac<T>(cx, odd ? u.v[2] : u.v[0], g.fb);
            y[o] = cell_plus_frac<T>(cy, odd ? u.v[3] : u.v[1], g.fb);
            M[o] = (MT)(g.M_min + kx);
            My[o] = (MT)(g.M_min + ky);
        }
        s[o] = sign;
    }
}

// ----------------------------------------------------------------------------- annihilation
__global__ void fill_i32(int32_t* p, long n, int32_t v) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        p[i] = v;
}

// Signed histogram of rule 1.  Counters are shared by all XCDs, so every global update is a
// device-coherent atomic; the ensemble is close to bin-ordered (initial placement is
// bin-major, survivors keep their order, fresh particles are appended bin by bin), so the
// contiguous chunk a workgroup owns touches a narrow range of bins.  Each workgroup counts
// into an LDS window of HW bins starting just below the smallest bin of its first tile,
// then adds the non-zero window entries to the global histogram; particles outside the
// window (rare) go straight to global atomics, merged per run of equal keys in a wave.
constexpr int HW = 4096;

template <typename T, typename MT, int DIM>
__global__ __launch_bounds__(PT) void annih_hist(Geo g, const T* x, const T* y, const MT* M,
                                                 const MT* My, const int8_t* s,
                                                 const long long* d_n, int32_t* hist,
                                                 const long long* stats) {
    __shared__ int lh[2][HW];
    __shared__ long wmin[PT / 64];
    if (stats[WK_ST_OVERFLOW] != 0) return;
    long lo, hi;
    chunk_of((long)*d_n, &lo, &hi);
    const int lane = threadIdx.x & 63;
    for (int k = threadIdx.x; k < 2 * HW; k += PT) (&lh[0][0])[k] = 0;
    // window base: smallest bin of the first tile, less a quarter window
    long b0 = LONG_MAX;
    {
        Part4<T, DIM> p;
        load4<T, MT, DIM>(x, y, M, My, s, lo + IT * threadIdx.x, hi, p);
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const long b = bin_val<T, DIM>(g, p.x[k], p.y[k], p.m[k], p.my[k], p.s[k]);
            if (b >= 0) b0 = min(b0, b);
        }
    }
    for (int o = 32; o > 0; o >>= 1) b0 = min(b0, (long)__shfl_xor(b0, o, 64));
    if (lane == 0) wmin[threadIdx.x >> 6] = b0;
    __syncthreads();
    long base = min(min(wmin[0], wmin[1]), min(wmin[2], wmin[3]));
    base = base == LONG_MAX ? 0 : max(0L, base - HW / 4);
    for (long t0 = lo; t0 < hi; t0 += TILE) {
        const long id = t0 + IT * threadIdx.x;
        Part4<T, DIM> p;
        load4<T, MT, DIM>(x, y, M, My, s, id, hi, p);
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            uint32_t key = 0xFFFFFFFFu;    // out-of-window key (global path)
            const long b = bin_val<T, DIM>(g, p.x[k], p.y[k], p.m[k], p.my[k], p.s[k]);
            if (b >= 0) {
                const int sg = p.s[k] > 0 ? 0 : 1;
                if (b >= base && b < base + HW)
                    atomicAdd(&lh[sg][b - base], 1);
                else
                    key = (uint32_t)(2 * b + sg);
            }
            const uint32_t prev = __shfl_up(key, 1, 64);
            const bool head = lane == 0 || prev != key;
            const unsigned long long heads = __ballot(head);
            if (head && key != 0xFFFFFFFFu) {
                const unsigned long long above = lane == 63 ? 0ull : (heads >> (lane + 1));
                const int next = above ? lane + 1 + __builtin_ctzll(above) : 64;
                const long bb = (long)(key >> 1);
                atomicAdd(&hist[(key & 1u) ? g.n_bins + bb : bb], next - lane);
            }
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < HW; k += PT) {
        const long b = base + k;
        if (b >= g.n_bins) break;
        if (lh[0][k]) atomicAdd(&hist[b], lh[0][k]);
        if (lh[1][k]) atomicAdd(&hist[g.n_bins + b], lh[1][k]);
    }
}

__device__ __forceinline__ bool keeps_bin(long b, const int32_t* hist, long n_bins) {
    return b >= 0 && !(hist[b] > 0 && hist[n_bins + b] > 0);
}

template <typename T, typename MT, int DIM>
__global__ __launch_bounds__(PT) void annih_keep_count(Geo g, const T* x, const T* y,
                                                       const MT* M, const MT* My, const int8_t* s,
                                                       const long long* d_n, const int32_t* hist,
                                                       const long long* stats, WS w) {
    __shared__ long long red[PT / 64];
    long long c = 0;
    if (stats[WK_ST_OVERFLOW] == 0) {
        long lo, hi;
        chunk_of(*d_n, &lo, &hi);
        for (long t0 = lo; t0 < hi; t0 += TILE) {
            const long id = t0 + IT * threadIdx.x;
            Part4<T, DIM> p;
            load4<T, MT, DIM>(x, y, M, My, s, id, hi, p);
#pragma unroll
            for (int k = 0; k < IT; ++k)
                c += keeps_bin(bin_val<T, DIM>(g, p.x[k], p.y[k], p.m[k], p.my[k], p.s[k]), hist,
                               g.n_bins) ? 1 : 0;
        }
    }
    c = wave_sum_ll(c);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) w.counts[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(PT) void annih_keep_scan(const long long* d_n_in, WS w) {
    __shared__ long long total;
    scan_pb(w.counts, w.offs, &total);
    if (threadIdx.x == 0) {
        w.sc[SC_KEPT] = total;
        w.sc[SC_N_OLD] = *d_n_in;
    }
}

template <typename T, typename MT, int DIM>
__global__ __launch_bounds__(PT) void annih_keep_write(Geo g, const T* x, const T* y,
                                                       const MT* M, const MT* My, const int8_t* s,
                                                       const int32_t* hist, T* xo, T* yo, MT* Mo,
                                                       MT* Myo, int8_t* so, const long long* stats,
                                                       WS w) {
    __shared__ int lds5[5];
    if (stats[WK_ST_OVERFLOW] != 0) return;
    long lo, hi;
    chunk_of((long)w.sc[SC_N_OLD], &lo, &hi);
    long long run = w.offs[blockIdx.x];
    for (long t0 = lo; t0 < hi; t0 += TILE) {
        const long id = t0 + IT * threadIdx.x;
        Part4<T, DIM> p;
        load4<T, MT, DIM>(x, y, M, My, s, id, hi, p);
        bool kp[IT];
        int kt = 0;
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            kp[k] = keeps_bin(bin_val<T, DIM>(g, p.x[k], p.y[k], p.m[k], p.my[k], p.s[k]), hist, g.n_bins);
            kt += kp[k];
        }
        int tot;
        const int ex = block_excl_scan_256(kt, &tot, lds5);
        long o = run + ex;
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            if (!kp[k]) continue;
            xo[o] = p.x[k];
            Mo[o] = (MT)p.m[k];
            if (DIM == 2) {
                yo[o] = p.y[k];
                Myo[o] = (MT)p.my[k];
            }
            so[o] = p.s[k];
            ++o;
        }
        run += tot;
    }
}

__global__ void density_kernel(const int32_t* hist, long n_cells, long per_cell, long n_bins,
                               double inv_n0, double* rho) {
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    long long acc = 0;
    for (long k = 0; k < per_cell; ++k) {
        const long b = c * per_cell + k;
        acc += (long long)hist[b] - (long long)hist[n_bins + b];
    }
    rho[c] = (double)acc * inv_n0;
}


// ----------------------------------------------------------------------------- occupied cells
// occ[c] = 1 if the histogram holds any particle in cell c (one wave per cell).
__global__ void occupied_kernel(const int32_t* __restrict__ hist, long n_cells, long per_cell,
                                long n_bins, uint8_t* __restrict__ occ) {
    const long c = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (c >= n_cells) return;
    int o = 0;
    for (long k = lane; k < per_cell; k += 64) {
        const long b = c * per_cell + k;
        o |= (hist[b] | hist[n_bins + b]) != 0;
    }
    const unsigned long long any = __ballot(o);
    if (lane == 0) occ[c] = any != 0ull;
}

// Cells without a table row that lie within `margin` cells (per axis) of an occupied cell,
// compacted in ascending order by one workgroup (deterministic).
__global__ __launch_bounds__(1024) void cells_needed_kernel(const uint8_t* __restrict__ occ,
                                                           int dim, int nx, int ny, int margin,
                                                           const int32_t* __restrict__ cell_slot,
                                                           int32_t* __restrict__ new_cells,
                                                           long long* __restrict__ d_count) {
    __shared__ int wsum[16];
    const long n_cells = (long)nx * ny;
    const long per = (n_cells + 1023) / 1024;
    const long lo = min(n_cells, (long)threadIdx.x * per), hi = min(n_cells, lo + per);
    auto needed = [&](long c) -> int {
        if (cell_slot[c] >= 0) return 0;
        const int cx = (int)(c % nx), cy = (int)(c / nx);
        const int y0 = dim == 2 ? max(cy - margin, 0) : 0, y1 = dim == 2 ? min(cy + margin, ny - 1) : 0;
        for (int yy = y0; yy <= y1; ++yy)
            for (int xx = max(cx - margin, 0); xx <= min(cx + margin, nx - 1); ++xx)
                if (occ[(long)yy * nx + xx]) return 1;
        return 0;
    };
    int cnt = 0;
    for (long c = lo; c < hi; ++c) cnt += needed(c);
    // block exclusive scan of cnt over 1024 threads (16 waves)
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int inc = wave_incl_scan(cnt);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int base = 0, total = 0;
    for (int k = 0; k < 16; ++k) {
        if (k < w) base += wsum[k];
        total += wsum[k];
    }
    long o = base + inc - cnt;
    for (long c = lo; c < hi; ++c)
        if (needed(c)) new_cells[o++] = (int32_t)c;
    if (threadIdx.x == 0) *d_count = total;
}

__global__ void assign_slots_kernel(const int32_t* __restrict__ new_cells,
                                    const long long* __restrict__ d_count, int32_t first_row,
                                    int32_t* __restrict__ cell_slot) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < *d_count) cell_slot[new_cells[k]] = first_row + (int32_t)k;
}

// ----------------------------------------------------------------------------- host side
static int make_geo(const sp_geom* gm, Geo* g) {
    WK_REQUIRE(gm != nullptr, "particles: geometry is NULL");
    WK_REQUIRE(gm->dim == 1 || gm->dim == 2, "particles: dim must be 1 or 2");
    WK_REQUIRE(gm->nx > 0 && gm->ny > 0 && (gm->dim == 2 || gm->ny == 1), "particles: bad mesh");
    WK_REQUIRE(gm->n_m >= 2 && gm->n_m % 2 == 0, "particles: n_m must be even");
    WK_REQUIRE(gm->n_k > 0, "particles: n_k must be positive");
    WK_REQUIRE(gm->dim == 1 || (gm->M_min >= -32768 && gm->M_min + gm->n_k <= 32767),
               "particles: 2-D momenta must fit int16");
    g->dim = gm->dim;
    g->nx = gm->nx;
    g->ny = gm->ny;
    g->n_m = gm->n_m;
    g->n_k = gm->n_k;
    g->M_min = gm->M_min;
    g->P = gm->n_m / 2;
    g->fb = frac_bits_host(gm->nx > gm->ny ? gm->nx : gm->ny, gm->pos_f64);
    g->width = gm->dim == 1 ? gm->n_m : (long)gm->n_m * gm->n_m;
    g->n_bins = (long)gm->nx * gm->ny * gm->n_k * (gm->dim == 2 ? gm->n_k : 1);
    g->vdt = gm->vdt;
    g->seed = gm->seed;
    WK_REQUIRE(g->n_bins < (1L << 31), "particles: too many bins");
    WK_REQUIRE(g->fb >= 1, "particles: mesh too large for the position precision");
    return WK_OK;
}

static int check_particles(const sp_geom* gm, const sp_particles* p, const char* what) {
    WK_REQUIRE(p != nullptr, std::string(what) + ": particles is NULL");
    WK_REQUIRE(p->x && p->M && p->s && p->d_n, std::string(what) + ": NULL particle array");
    WK_REQUIRE(gm->dim == 1 || (p->y && p->My), std::string(what) + ": 2-D needs y and My");
    WK_REQUIRE(p->capacity >= 0 && p->capacity < (1LL << 31),
               std::string(what) + ": capacity must be < 2^31");
    return WK_OK;
}

template <typename T, typename MT, int DIM>
static void launch_step(const Geo& g, uint32_t step, const int32_t* cs, const uint32_t* n0,
                        const uint32_t* thr, const uint64_t* cdf, sp_particles* p,
                        long long* stats, long long st, WS w, hipStream_t s) {
    T* x = static_cast<T*>(p->x);
    T* y = static_cast<T*>(p->y);
    MT* M = static_cast<MT*>(p->M);
    MT* My = static_cast<MT*>(p->My);
    long long* d_n = reinterpret_cast<long long*>(p->d_n);
    WK_LAUNCH("step_count", (step_count<T, MT, DIM>), dim3(PB), dim3(PT), 0, s, g, step, cs, n0, thr, x,
                       y, M, My, p->s, d_n, stats, w);
    WK_LAUNCH("step_scan", step_scan, dim3(1), dim3(PT), 0, s, d_n, (long long)p->capacity, stats, st, w);
    WK_LAUNCH("step_apply", (step_apply<T, MT, DIM>), dim3(PB), dim3(PT), 0, s, g, step, cs, n0, thr,
                       cdf, x, y, M, My, p->s, stats, w);
}

template <typename T, typename MT, int DIM>
static void launch_annih(const Geo& g, uint32_t step, const sp_particles* in, sp_particles* out,
                         int32_t* hist, long long* stats, WS w, hipStream_t s) {
    const T* x = static_cast<const T*>(in->x);
    const T* y = static_cast<const T*>(in->y);
    const MT* M = static_cast<const MT*>(in->M);
    const MT* My = static_cast<const MT*>(in->My);
    const long long* d_n = reinterpret_cast<const long long*>(in->d_n);
    WK_LAUNCH("hist_clear", fill_i32, dim3(1024), dim3(256), 0, s, hist, 2 * g.n_bins, 0);
    WK_LAUNCH("annih_hist", (annih_hist<T, MT, DIM>), dim3(PB), dim3(PT), 0, s, g, x, y, M, My, in->s,
                       d_n, hist, stats);  // fixed grid: chunk_of() splits the ensemble
    WK_LAUNCH("annih_keep_count", (annih_keep_count<T, MT, DIM>), dim3(PB), dim3(PT), 0, s, g, x, y, M, My,
                       in->s, d_n, hist, stats, w);
    WK_LAUNCH("annih_keep_scan", annih_keep_scan, dim3(1), dim3(PT), 0, s, d_n, w);
    WK_LAUNCH("annih_keep_write", (annih_keep_write<T, MT, DIM>), dim3(PB), dim3(PT), 0, s, g, x, y, M, My,
                       in->s, hist, static_cast<T*>(out->x), static_cast<T*>(out->y),
                       static_cast<MT*>(out->M), static_cast<MT*>(out->My), out->s, stats, w);
    BinCount bc{nullptr, hist, g.n_bins};
    WK_LAUNCH("bins_reduce", bins_reduce, dim3(PB), dim3(PT), 0, s, bc, stats, w);
    WK_LAUNCH("bins_scan", bins_scan, dim3(1), dim3(PT), 0, s, 1,
                       reinterpret_cast<long long*>(out->d_n), (long long)out->capacity, stats, w);
    WK_LAUNCH("bins_downsweep", bins_downsweep, dim3(PB), dim3(PT), 0, s, bc, 1, w);
    WK_LAUNCH("bins_place", (bins_place<T, MT, DIM>), dim3(PB), dim3(PT), 0, s, g, bc, 1, step,
                       (uint32_t)TAG_ANNIH, static_cast<T*>(out->x), static_cast<T*>(out->y),
                       static_cast<MT*>(out->M), static_cast<MT*>(out->My), out->s, w);
}

template <typename T, typename MT, int DIM>
static void launch_init(const Geo& g, const int32_t* counts, sp_particles* out, long long* stats,
                        WS w, hipStream_t s) {
    BinCount bc{counts, nullptr, g.n_bins};
    WK_LAUNCH("bins_reduce", bins_reduce, dim3(PB), dim3(PT), 0, s, bc, stats, w);
    WK_LAUNCH("bins_scan", bins_scan, dim3(1), dim3(PT), 0, s, 0,
                       reinterpret_cast<long long*>(out->d_n), (long long)out->capacity, stats, w);
    WK_LAUNCH("bins_downsweep", bins_downsweep, dim3(PB), dim3(PT), 0, s, bc, 0, w);
    WK_LAUNCH("bins_place", (bins_place<T, MT, DIM>), dim3(PB), dim3(PT), 0, s, g, bc, 0, 0xFFFFFFFFu,
                       (uint32_t)TAG_INIT, static_cast<T*>(out->x), static_cast<T*>(out->y),
                       static_cast<MT*>(out->M), static_cast<MT*>(out->My), out->s, w);
}

}  // namespace wk

using namespace wk;

extern "C" size_t sp_workspace_size(const sp_geom* gm) {
    Geo g;
    if (make_geo(gm, &g) != WK_OK) return 0;
    return ws_bytes_for(g.n_bins);
}

#define WK_DISPATCH(gm, FN, ...)                                                      \
    do {                                                                             \
        if ((gm)->dim == 1) {                                                        \
            if ((gm)->pos_f64)                                                       \
                FN<double, int32_t, 1>(__VA_ARGS__);                                 \
            else                                                                     \
                FN<float, int32_t, 1>(__VA_ARGS__);                                  \
        } else {                                                                     \
            if ((gm)->pos_f64)                                                       \
                FN<double, int16_t, 2>(__VA_ARGS__);                                 \
            else                                                                     \
                FN<float, int16_t, 2>(__VA_ARGS__);                                  \
        }                                                                            \
    } while (0)

extern "C" int sp_init(const sp_geom* gm, const int32_t* bin_counts, sp_particles* out,
                       int64_t* d_stats, void* ws, size_t ws_bytes, void* stream) {
    Geo g;
    int rc = make_geo(gm, &g);
    if (rc) return rc;
    rc = check_particles(gm, out, "sp_init");
    if (rc) return rc;
    WK_REQUIRE(bin_counts && d_stats, "sp_init: NULL array");
    WK_REQUIRE(ws && ws_bytes >= ws_bytes_for(g.n_bins), "sp_init: workspace too small");
    WS w = carve(ws);
    WK_DISPATCH(gm, launch_init, g, bin_counts, out, reinterpret_cast<long long*>(d_stats), w,
                as_stream(stream));
    return check_launch("sp_init");
}

extern "C" int sp_step(const sp_geom* gm, const int32_t* cell_slot, const uint32_t* n0,
                       const uint32_t* thr, const uint64_t* cdf, sp_particles* p, int64_t step,
                       int64_t* d_stats, void* ws, size_t ws_bytes, void* stream) {
    Geo g;
    int rc = make_geo(gm, &g);
    if (rc) return rc;
    rc = check_particles(gm, p, "sp_step");
    if (rc) return rc;
    WK_REQUIRE(cell_slot && n0 && thr && cdf && d_stats, "sp_step: NULL array");
    WK_REQUIRE(step >= 0 && step < (1LL << 32), "sp_step: step must fit 32 bits");
    WK_REQUIRE(ws && ws_bytes >= ws_bytes_for(g.n_bins), "sp_step: workspace too small");
    WS w = carve(ws);
    WK_DISPATCH(gm, launch_step, g, (uint32_t)step, cell_slot, n0, thr, cdf, p,
                reinterpret_cast<long long*>(d_stats), (long long)step, w, as_stream(stream));
    return check_launch("sp_step");
}

extern "C" int sp_annihilate(const sp_geom* gm, const sp_particles* in, sp_particles* out,
                             int32_t* hist, int64_t step, int64_t* d_stats, void* ws,
                             size_t ws_bytes, void* stream) {
    Geo g;
    int rc = make_geo(gm, &g);
    if (rc) return rc;
    rc = check_particles(gm, in, "sp_annihilate(in)");
    if (rc) return rc;
    rc = check_particles(gm, out, "sp_annihilate(out)");
    if (rc) return rc;
    WK_REQUIRE(in->x != out->x && in->s != out->s, "sp_annihilate: in and out must differ");
    WK_REQUIRE(out->capacity >= in->capacity, "sp_annihilate: out capacity below in capacity");
    WK_REQUIRE(hist && d_stats, "sp_annihilate: NULL array");
    WK_REQUIRE(step >= 0 && step < (1LL << 32), "sp_annihilate: step must fit 32 bits");
    WK_REQUIRE(ws && ws_bytes >= ws_bytes_for(g.n_bins), "sp_annihilate: workspace too small");
    WS w = carve(ws);
    WK_DISPATCH(gm, launch_annih, g, (uint32_t)step, in, out, hist,
                reinterpret_cast<long long*>(d_stats), w, as_stream(stream));
    return check_launch("sp_annihilate");
}

extern "C" int sp_density(const sp_geom* gm, const int32_t* hist, double N0, double* rho,
                          void* stream) {
    Geo g;
    int rc = make_geo(gm, &g);
    if (rc) return rc;
    WK_REQUIRE(hist && rho, "sp_density: NULL array");
    WK_REQUIRE(N0 > 0, "sp_density: N0 must be positive");
    const long n_cells = (long)g.nx * g.ny;
    const long per = g.n_bins / n_cells;
    hipLaunchKernelGGL(density_kernel, dim3((unsigned)((n_cells + 255) / 256)), dim3(256), 0,
                       as_stream(stream), hist, n_cells, per, g.n_bins, 1.0 / N0, rho);
    return check_launch("sp_density");
}

extern "C" int sp_cells_to_evaluate(const sp_geom* gm, const int32_t* hist, int32_t margin,
                                    const int32_t* cell_slot, int32_t* new_cells, int64_t* d_count,
                                    void* ws, size_t ws_bytes, void* stream) {
    Geo g;
    int rc = make_geo(gm, &g);
    if (rc) return rc;
    WK_REQUIRE(hist && cell_slot && new_cells && d_count, "sp_cells_to_evaluate: NULL array");
    WK_REQUIRE(margin >= 0, "sp_cells_to_evaluate: negative margin");
    WK_REQUIRE(ws && ws_bytes >= ws_bytes_for(g.n_bins), "sp_cells_to_evaluate: workspace too small");
    const long n_cells = (long)g.nx * g.ny;
    uint8_t* occ = reinterpret_cast<uint8_t*>(carve(ws).binoff);  // n_cells <= n_bins bytes
    hipStream_t s = as_stream(stream);
    hipLaunchKernelGGL(occupied_kernel, dim3((unsigned)((n_cells * 64 + 255) / 256)), dim3(256), 0, s,
                       hist, n_cells, g.n_bins / n_cells, g.n_bins, occ);
    hipLaunchKernelGGL(cells_needed_kernel, dim3(1), dim3(1024), 0, s, occ, g.dim, g.nx, g.ny, margin,
                       cell_slot, new_cells, reinterpret_cast<long long*>(d_count));
    return check_launch("sp_cells_to_evaluate");
}

extern "C" int sp_assign_slots(const int32_t* new_cells, const int64_t* d_count, int32_t max_count,
                               int32_t first_row, int32_t* cell_slot, void* stream) {
    WK_REQUIRE(new_cells && d_count && cell_slot, "sp_assign_slots: NULL array");
    WK_REQUIRE(max_count >= 0 && first_row >= 0, "sp_assign_slots: negative size");
    if (max_count == 0) return WK_OK;
    hipLaunchKernelGGL(assign_slots_kernel, dim3((unsigned)((max_count + 255) / 256)), dim3(256), 0,
                       as_stream(stream), new_cells, reinterpret_cast<const long long*>(d_count),
                       first_row, cell_slot);
    return check_launch("sp_assign_slots");
}
