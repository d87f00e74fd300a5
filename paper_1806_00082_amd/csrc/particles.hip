// Signed-particle passes (Sec. 2.1): pair creation + field-less drift + absorbing boundaries
// (sp_step), annihilation on the (cell, momentum) grid (sp_annihilate), initial placement
// (sp_init) and the rule-1 read-out (sp_density).
//
// Layout: struct-of-arrays in HBM, positions in cell units.  Every pass streams the
// arrays once with coalesced accesses.  Ordered outputs (appended children, compacted
// survivors) use a fixed grid of PB workgroups (SB_MAX for sp_step on large buffers) whose
// waves each own one contiguous chunk of
// particle ids: a counting pass stores one count per wave and per workgroup, and every
// workgroup of the writing pass re-totals the PB workgroup counts (from L2) for its own
// offset and the capacity check; each wave then walks its chunk with wave-level scans only,
// no workgroup barriers.  Particles placed bin by bin (annihilation, initial state) are
// split into equal ranges of output slots over the placing workgroups, which find their
// bins through per-chunk counts.  Output positions therefore depend only on the data, never
// on scheduling, and there are no floating-point atomics anywhere (integer atomics only,
// for histogram counts).
//
// One time step is four launches: step_count (creation counts; clears the histogram),
// step_apply (children, drifted parents, absorption, and the signed histogram of the
// result), annih_count (survivors per wave chunk, particles to place per bin chunk) and
// annih_write (regenerated particles placed, then the survivors copied in order).
#include <climits>

#include "wk_internal.h"

namespace wk {

constexpr int PB = 2048;    // workgroups of the chunked passes
constexpr int PT = 256;     // threads per workgroup

struct Geo {
    int dim, nx, ny, n_m, n_k, M_min, P, fb;
    long width;       // table entries per row (n_m or n_m^2)
    long n_bins;
    long n_chunks;    // bin chunks of BC bins
    long gpb;         // bin chunks per bin workgroup (PB bin workgroups)
    int bshift;       // bins per block of the block map: 2^bshift (a multiple of BC)
    double vdt;
    uint64_t seed;
};

constexpr int BC = PT;      // bins per bin chunk
// The block map: one bit per block of consecutive bins (2^Geo::bshift bins, at least BC and
// as many as keep the blocks within BMW * 32), set by the histogram builders wherever they add
// counts.  The bin pass of the annihilation then reads only the histogram of marked blocks.
constexpr int BMW = 2048;
constexpr int WPB = PT / 64;  // waves per workgroup
constexpr int NW = PB * WPB;  // wave chunks of the ordered passes
// sp_step on large buffers: twice the chunk owners.  Per-chunk work varies (creation and
// scattered children concentrate where gamma is large) and the launch takes several
// residency rounds, so shorter chunks shorten the last round; on small ensembles the
// per-workgroup prologue costs more than that saves.  The host knows the buffer capacity,
// not the particle count (that stays on the device), so capacity sets the scale.
constexpr int SB_MAX = 2 * PB;
constexpr long long SB_LARGE = 1LL << 26;  // output capacity from which sp_step uses SB_MAX

constexpr int PLACE_BLOCKS = PB;  // workgroups placing regenerated / initial particles
constexpr int CT_MAX = 1024;       // cells of the LDS creation table (larger meshes: ctab)

constexpr int PLACE_WAVES = PLACE_BLOCKS * WPB;
// Placement work items: each bin chunk's particles to place, in pieces of at most PIECE slots.
constexpr int PIECE = 2048;

// Workspace (sp_workspace_size): int64 scalars[16] | int64 bcnt[SB_MAX] | int64 wcnt[SB_MAX WPB] |
// int64 bpart[PB] | int64 bmixed[PB] | int64 kpre[SB_MAX] | int64 bpre[PB] | int64 bitem[PB] |
// int64 ipre[PB] | int32 wstart[PLACE_WAVES] | int32 csum[n_chunks] | uint8 occ[n_cells] |
// uint8 occx[n_cells] | uint2 ctab[n_cells] (8-byte aligned) | uint32 mixbits[8 n_chunks]
// (16-byte aligned).
enum { SC_GO = 0, SC_PLACED = 1, SC_KEPT = 2, SC_ITEMS = 3, SC_KBITS = 4 };

struct WS {
    long long* sc;
    long long* bcnt;    // per workgroup of a counting pass: its count
    long long* wcnt;    // per wave of a counting pass: its count
    long long* bpart;   // per bin workgroup: particles to place
    long long* bmixed;  // per bin workgroup: mixed bins
    long long* kpre;    // exclusive prefix of the survivor counts (bcnt) of sp_annihilate
    long long* bpre;    // inclusive prefix of bpart
    long long* bitem;   // per bin workgroup: placement work items (pieces of its chunks)
    long long* ipre;    // inclusive prefix of bitem
    int* wstart;        // per placing wave: bin workgroup holding its first work item
    int* csum;          // per bin chunk: particles to place
    uint8_t* occ;
    uint2* ctab;        // meshes above CT_MAX cells: (n0, thr) per cell, gathered each step
    uint32_t* mixbits;  // one bit per bin: set when the bin holds both signs (annih_bins)
    uint32_t* blkmap;   // one bit per block of 2^bshift bins: set when the histogram builder
                        // added counts there (BMW words)
};

static long n_chunks_for(long n_bins) { return (n_bins + BC - 1) / BC; }

static WS carve(void* ws, long n_bins, long n_cells) {
    WS w;
    char* p = static_cast<char*>(ws);
    w.sc = reinterpret_cast<long long*>(p);
    w.bcnt = w.sc + 16;
    w.wcnt = w.bcnt + SB_MAX;
    w.bpart = w.wcnt + (size_t)SB_MAX * WPB;
    w.bmixed = w.bpart + PB;
    w.kpre = w.bmixed + PB;
    w.bpre = w.kpre + SB_MAX;
    w.bitem = w.bpre + PB;
    w.ipre = w.bitem + PB;
    w.wstart = reinterpret_cast<int*>(w.ipre + PB);
    w.csum = w.wstart + PLACE_WAVES;
    w.occ = reinterpret_cast<uint8_t*>(w.csum + (n_chunks_for(n_bins) + 1) / 2 * 2);
    const uintptr_t e = reinterpret_cast<uintptr_t>(w.occ) + 2 * (size_t)n_cells;
    w.ctab = reinterpret_cast<uint2*>((e + 7) & ~(uintptr_t)7);
    const uintptr_t f = reinterpret_cast<uintptr_t>(w.ctab) + sizeof(uint2) * (n_cells > CT_MAX ? (size_t)n_cells : 0);
    w.mixbits = reinterpret_cast<uint32_t*>((f + 15) & ~(uintptr_t)15);
    w.blkmap = w.mixbits + 8 * (size_t)n_chunks_for(n_bins);
    return w;
}

static size_t ws_bytes_for(long n_bins, long n_cells) {
    return sizeof(long long) * (16 + (size_t)SB_MAX * (2 + WPB) + 5 * (size_t)PB) +
           sizeof(int) * (size_t)(PLACE_WAVES + (n_chunks_for(n_bins) + 1) / 2 * 2) +
           2 * (size_t)n_cells +  // occupancy byte per cell, then its dilation along x
           8 + sizeof(uint2) * (n_cells > CT_MAX ? (size_t)n_cells : 0) +  // aligned ctab
           16 + sizeof(uint32_t) * 8 * (size_t)n_chunks_for(n_bins) +      // aligned mixbits
           sizeof(uint32_t) * BMW;                                          // block map
}

constexpr int IT = 4;          // particles per lane in the streaming passes
constexpr int WT = 64 * IT;    // particles per wave tile

// The 8 bits of b moved to bits 0, 4, 8, ..., 28.
__device__ __forceinline__ uint32_t spread4(uint32_t b) {
    b = (b | (b << 12)) & 0x000F000Fu;
    b = (b | (b << 6)) & 0x03030303u;
    b = (b | (b << 3)) & 0x11111111u;
    return b;
}

// Wave chunk `wv` of nw: a whole number of wave tiles, the last ones possibly empty.
__device__ __forceinline__ void wave_chunk(long n, long wv, long* lo, long* hi, long nw = NW) {
    long cs = (n + nw - 1) / nw;
    cs = (cs + WT - 1) / WT * WT;
    *lo = min(n, wv * cs);
    *hi = min(n, *lo + cs);
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

// Histogram bin of a particle, -1 when dead or outside the grid.  n_bins < 2^31 (checked on
// the host) and every partial sum below is at most the bin index: 32-bit arithmetic is exact.
template <typename T, int DIM>
__device__ __forceinline__ long bin_val(const Geo& g, T x, T y, int m, int my, int8_t s) {
    if (s == 0) return -1;
    const int cx = cell_index<T>(x, g.nx);
    if (cx < 0) return -1;
    const int kx = m - g.M_min;
    if (kx < 0 || kx >= g.n_k) return -1;
    if (DIM == 1) return (long)(cx * g.n_k + kx);
    const int cy = cell_index<T>(y, g.ny);
    if (cy < 0) return -1;
    const int ky = my - g.M_min;
    if (ky < 0 || ky >= g.n_k) return -1;
    return (long)(((cy * g.nx + cx) * g.n_k + ky) * g.n_k + kx);
}

// A particle's (bin, sign) key of the signed histogram: 2 bin + 1 for negative particles,
// HKEY_NONE when it has no bin (dead or outside the grid).  n_bins < 2^31.
constexpr uint32_t HKEY_NONE = 0xFFFFFFFFu;
__device__ __forceinline__ uint32_t hist_key(long b, int8_t s) {
    return b < 0 ? HKEY_NONE : 2u * (uint32_t)b + (s > 0 ? 0u : 1u);
}

// Four consecutive particles (ids id .. id+3, id a multiple of 4) loaded with 16-byte
// (positions, int32 momenta), 8-byte (int16 momenta) and 4-byte (int8 momenta, signs) accesses;
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
__device__ __forceinline__ void ld4(const int8_t* p, long i, int* v) {
    const char4 t = *reinterpret_cast<const char4*>(p + i);
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

__device__ __forceinline__ void st4(int32_t* p, long i, const int* v) {
    *reinterpret_cast<int4*>(p + i) = make_int4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void st4(int16_t* p, long i, const int* v) {
    *reinterpret_cast<short4*>(p + i) = make_short4((short)v[0], (short)v[1], (short)v[2], (short)v[3]);
}
__device__ __forceinline__ void st4(int8_t* p, long i, const int* v) {
    *reinterpret_cast<char4*>(p + i) = make_char4((signed char)v[0], (signed char)v[1], (signed char)v[2],
                                                  (signed char)v[3]);
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

// The same four particles as loaded, momenta and signs still packed in the words the loads
// return.  A prefetch of the next tile is carried across the loop in this form: unpacking
// (sign-extending) at the load would make the wave wait for the loads right there, while
// unpack() at the top of the next iteration waits only when the values are needed.
template <typename MT> struct Packed4;  // four MT in one load
template <> struct Packed4<int8_t> { using type = uint32_t; };
template <> struct Packed4<int16_t> { using type = uint2; };
template <> struct Packed4<int32_t> { using type = int4; };

template <typename T, typename MT, int DIM>
struct Raw4 {
    T x[IT], y[IT];
    typename Packed4<MT>::type m, my;
    uint32_t s;
};

template <typename T, typename MT, int DIM>
__device__ __forceinline__ void load4r(const T* x, const T* y, const MT* M, const MT* My,
                                       const int8_t* s, long id, long hi, Raw4<T, MT, DIM>& r) {
    using PW = typename Packed4<MT>::type;
    static_assert(sizeof(PW) == IT * sizeof(MT), "four momenta per packed word");
    if (id + IT <= hi) {
        ld4(x, id, r.x);
        r.m = *reinterpret_cast<const PW*>(M + id);
        r.s = *reinterpret_cast<const uint32_t*>(s + id);
        if (DIM == 2) {
            ld4(y, id, r.y);
            r.my = *reinterpret_cast<const PW*>(My + id);
        }
    } else {
        MT mm[IT], mmy[IT];
        int8_t ss[IT];
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const bool v = id + k < hi;
            r.x[k] = v ? x[id + k] : (T)0;
            mm[k] = v ? M[id + k] : (MT)0;
            ss[k] = v ? s[id + k] : (int8_t)0;
            r.y[k] = (DIM == 2 && v) ? y[id + k] : (T)0;
            mmy[k] = (DIM == 2 && v) ? My[id + k] : (MT)0;
        }
        __builtin_memcpy(&r.m, mm, sizeof(PW));
        __builtin_memcpy(&r.my, mmy, sizeof(PW));
        __builtin_memcpy(&r.s, ss, sizeof(uint32_t));
    }
    if (DIM == 1) {
#pragma unroll
        for (int k = 0; k < IT; ++k) r.y[k] = (T)0;
        __builtin_memset(&r.my, 0, sizeof(PW));
    }
}

// An empty asm statement that takes a register and gives it back: the compiler cannot look
// through it, so it keeps a packed word whole until this point instead of splitting it into
// bytes right after its load (which waits for the load there).
__device__ __forceinline__ void opaque(uint32_t& v) { asm volatile("" : "+v"(v)); }
__device__ __forceinline__ void opaque(uint2& v) {
    asm volatile("" : "+v"(v.x));
    asm volatile("" : "+v"(v.y));
}
__device__ __forceinline__ void opaque(int4& v) {
    asm volatile("" : "+v"(v.x));
    asm volatile("" : "+v"(v.y));
    asm volatile("" : "+v"(v.z));
    asm volatile("" : "+v"(v.w));
}

// Part4 of what load4r loaded: the same values load4 gives.
template <typename T, typename MT, int DIM>
__device__ __forceinline__ Part4<T, DIM> unpack(Raw4<T, MT, DIM> r) {
    Part4<T, DIM> p;
    opaque(r.m);
    opaque(r.s);
    if (DIM == 2) opaque(r.my);
    MT mm[IT], mmy[IT];
    int8_t ss[IT];
    __builtin_memcpy(mm, &r.m, sizeof(mm));
    __builtin_memcpy(mmy, &r.my, sizeof(mmy));
    __builtin_memcpy(ss, &r.s, sizeof(ss));
#pragma unroll
    for (int k = 0; k < IT; ++k) {
        p.x[k] = r.x[k];
        p.y[k] = r.y[k];
        p.m[k] = mm[k];
        p.my[k] = mmy[k];
        p.s[k] = ss[k];
    }
    return p;
}

// Histogram keys of four consecutive particles (id a multiple of 4); slots at or beyond hi
// read as HKEY_NONE.
__device__ __forceinline__ void load_keys4(const uint32_t* keys, long id, long hi, uint32_t* k4) {
    if (id + IT <= hi) {
        const uint4 t = *reinterpret_cast<const uint4*>(keys + id);
        k4[0] = t.x; k4[1] = t.y; k4[2] = t.z; k4[3] = t.w;
    } else {
#pragma unroll
        for (int k = 0; k < IT; ++k) k4[k] = id + k < hi ? keys[id + k] : HKEY_NONE;
    }
}

// Stores four consecutive particles (positions xv, yv; momenta and signs from p); slots at
// or beyond hi are left alone.
template <typename T, typename MT, int DIM>
__device__ __forceinline__ void store4(T* x, T* y, MT* M, MT* My, int8_t* s, long id, long hi,
                                       const T* xv, const T* yv, const Part4<T, DIM>& p) {
    if (id + IT <= hi) {
        st4(x, id, xv);
        st4(M, id, p.m);
        *reinterpret_cast<char4*>(s + id) = make_char4(p.s[0], p.s[1], p.s[2], p.s[3]);
        if (DIM == 2) {
            st4(y, id, yv);
            st4(My, id, p.my);
        }
    } else {
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            if (id + k < hi) {
                x[id + k] = xv[k];
                M[id + k] = (MT)p.m[k];
                s[id + k] = p.s[k];
                if (DIM == 2) {
                    y[id + k] = yv[k];
                    My[id + k] = (MT)p.my[k];
                }
            }
        }
    }
}

// Pair counts of four consecutive particles kept between the two passes of sp_step in the
// output buffer, which the second pass overwrites only after reading them: one byte per
// particle in the sign array, and for a count of 255 or more (byte 255) the full count in the
// first four bytes of the particle's position slot.
template <typename T>
__device__ __forceinline__ void store_np4(T* xo, int8_t* so, long id, long hi, const int* np) {
    uint8_t b[IT];
#pragma unroll
    for (int k = 0; k < IT; ++k) {
        b[k] = np[k] >= 255 ? (uint8_t)255 : (uint8_t)np[k];
        if (np[k] >= 255 && id + k < hi) *reinterpret_cast<int*>(xo + id + k) = np[k];
    }
    if (id + IT <= hi) {
        *reinterpret_cast<uchar4*>(so + id) = make_uchar4(b[0], b[1], b[2], b[3]);
    } else {
#pragma unroll
        for (int k = 0; k < IT; ++k)
            if (id + k < hi) so[id + k] = (int8_t)b[k];
    }
}
template <typename T>
__device__ __forceinline__ void load_np4(const T* xo, const int8_t* so, long id, long hi, int* np) {
    if (id + IT <= hi) {
        const uchar4 v = *reinterpret_cast<const uchar4*>(so + id);
        np[0] = v.x;
        np[1] = v.y;
        np[2] = v.z;
        np[3] = v.w;
    } else {
#pragma unroll
        for (int k = 0; k < IT; ++k) np[k] = id + k < hi ? (int)(uint8_t)so[id + k] : 0;
    }
#pragma unroll
    for (int k = 0; k < IT; ++k)
        if (np[k] == 255) np[k] = *reinterpret_cast<const int*>(xo + id + k);
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
    const uint32_t base = n0[sl], t = thr[sl];
    if (base == 0 && t == 0) return 0;  // no pair whatever u0 is: the draw is not needed
    *slot = sl;
    *w = philox(id, step, 0u, TAG_CREATE, g.seed);
    // 2^30 pairs already exceed any capacity (< 2^31): larger counts are reported as that
    if (base >= (1u << 30)) return 1 << 30;
    return (int)base + (w->v[0] < t ? 1 : 0);
}

// The cell of a live particle inside the mesh (the index into a cell-indexed table), else -1.
template <typename T, int DIM>
__device__ __forceinline__ int live_cell(const Geo& g, T px, T py, int8_t sv) {
    if (sv == 0) return -1;
    const int cx = cell_index<T>(px, g.nx);
    if (cx < 0) return -1;
    if (DIM == 1) return cx;
    const int cy = cell_index<T>(py, g.ny);
    return cy < 0 ? -1 : cy * g.nx + cx;
}

// Pair count of a live particle (postulate II) in a cell whose creation-table entry is
// e = (n0, thr): n0, plus one if the first Philox word of the particle's draw is below thr.
// The entry comes from a per-workgroup LDS table on small meshes, else from the cell-indexed
// table gathered each step (cells without a table row hold (0, 0): no pairs).
__device__ __forceinline__ int pairs_of_entry(const Geo& g, uint32_t id, uint32_t step, uint2 e) {
    if (e.x == 0 && e.y == 0) return 0;
    const u32x4 w = philox(id, step, 0u, TAG_CREATE, g.seed);
    if (e.x >= (1u << 30)) return 1 << 30;
    return (int)e.x + (w.v[0] < e.y ? 1 : 0);
}

// Smallest t with u < T[t] (T non-decreasing, ending at 2^32 > u), searched in [lo, hi]:
// the whole row, or the bucket of u given by the row's guide table (G buckets).
__device__ __forceinline__ int sample_cdf(const uint64_t* __restrict__ T,
                                          const uint32_t* __restrict__ guide, int G, long width,
                                          uint32_t u) {
    long lo = 0, hi = width - 1;
    if (guide != nullptr) {
        const uint32_t k = (uint32_t)(((uint64_t)u * (uint32_t)G) >> 32);
        lo = guide[k];
        hi = guide[k + 1];
    }
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

// ----------------------------------------------------------------------------- block utilities
__device__ __forceinline__ long long wave_incl_scan_ll(long long v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const long long t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// Sum over the wave of values in [0, 2^33), one per lane (all lanes active), exact: two 32-bit
// DPP scans, of the low 24 bits (sum below 2^30) and of the rest (below 2^15), instead of
// six rounds of 64-bit shuffles, each an LDS round trip.
__device__ __forceinline__ long long wave_sum_nonneg33(long long v) {
    const int lo = (int)(v & 0xFFFFFF), hi = (int)(v >> 24);
    const int slo = __builtin_amdgcn_readlane(wave_incl_scan(lo), 63);
    const int shi = __builtin_amdgcn_readlane(wave_incl_scan(hi), 63);
    return ((long long)shi << 24) + slo;
}

// Sum over the block of one int64 per thread (PT threads); the result is valid in every
// thread.
__device__ __forceinline__ long long block_sum_ll(long long v, long long* redw) {
    v = wave_sum_ll(v);
    if ((threadIdx.x & 63) == 0) redw[threadIdx.x >> 6] = v;
    __syncthreads();
    long long t = 0;
#pragma unroll
    for (int k = 0; k < WPB; ++k) t += redw[k];
    __syncthreads();
    return t;
}

// Block-wide exclusive scan of one int per thread (PT threads); returns the exclusive prefix
// and writes the block total to *total.  Uses WPB ints of LDS.
__device__ __forceinline__ int block_excl_scan_pt(int v, int* total, int* ldsw) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int inc = wave_incl_scan(v);
    if (lane == 63) ldsw[wv] = inc;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < WPB; ++k) {
        const int t = ldsw[k];
        base += k < wv ? t : 0;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return base + inc - v;
}

// Makes the LDS writes of every lane of the wave visible to the others (the waves of a
// workgroup run independently here, so no workgroup barrier).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// First index i in [0, n) with a[i] > key (a non-decreasing), n if none.
template <typename V, typename K>
__device__ __forceinline__ int upper_bound_lds(const V* a, int n, K key) {
    int l = 0, h = n;
    while (l < h) {
        const int mid = (l + h) >> 1;
        if (a[mid] > key)
            h = mid;
        else
            l = mid + 1;
    }
    return l;
}

// ----------------------------------------------------------------------------- chunk offsets
// A counting pass leaves one count per workgroup (bcnt) and per wave (wcnt) of its PB
// chunk-owning workgroups.  Each workgroup of the matching writing pass totals bcnt (PB
// values from L2) for the capacity check; a chunk owner (blockIdx.x < PB, own = true) also
// gets the offset of its calling wave's chunk in *wave_off (valid in every lane).
__device__ long long chunk_offsets(const WS& w, bool own, long long* wave_off, long long* redw,
                                   int nb = PB) {
    long long a = 0, p = 0;
    for (int k = threadIdx.x; k < nb; k += PT) {
        const long long v = w.bcnt[k];
        a += v;
        if (own && k < (int)blockIdx.x) p += v;
    }
    const long long total = block_sum_ll(a, redw);
    long long off = 0;
    if (own) {
        off = block_sum_ll(p, redw);
        const int wv = threadIdx.x >> 6;
        for (int j = 0; j < wv; ++j) off += w.wcnt[(long)blockIdx.x * WPB + j];
    }
    *wave_off = off;
    return total;
}

// Stores a wave's count (lane 0) and the workgroup's sum of its waves' counts (thread 0).
__device__ void store_counts(const WS& w, long long wave_count, long long* redw) {
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        w.wcnt[(long)blockIdx.x * WPB + wv] = wave_count;
        redw[wv] = wave_count;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        long long t = 0;
#pragma unroll
        for (int k = 0; k < WPB; ++k) t += redw[k];
        w.bcnt[blockIdx.x] = t;
    }
}

// ----------------------------------------------------------------------------- histogram window
// Signed histogram of rule 1.  Counters are shared by all XCDs, so a global update is a
// device-coherent atomic; the ensemble is close to bin-ordered (initial placement is
// bin-major, survivors keep their order, fresh particles are placed bin by bin, children
// follow their parents' order), so the particles of one workgroup touch a narrow range of
// bins, with long runs of one bin.  Each workgroup counts into an LDS window of W bins per
// sign starting a quarter window below the smallest bin of its first particles, one atomic
// per run of equal (bin, sign) among the 64 lanes of a wave, then adds the non-zero window
// entries to the global histogram; runs outside the window (rare) go straight to global
// atomics.
// HASH (the 2-D passes): drift along y moves a particle by nx n_k^2 bins, far outside any
// window of consecutive bins, yet a workgroup still touches only a few hundred distinct bins.
// The same LDS then holds a hash table of W (bin, sign) keys with their counts (linear
// probing, keys claimed by compare-and-swap), flushed once per workgroup; a key that finds
// no slot within HPROBE probes goes to the global histogram.  Integer sums: the histogram
// is the same whichever way a count travels.
template <int W, bool HASH = false, bool MARK = false>
struct HistWindow {
    int* lh;  // [2][W] in LDS: window counts per sign, or (HASH) keys then counts
    long base;
    int32_t* hist;
    long n_bins;
    uint32_t* bm;    // [BMW] in LDS: the workgroup's block map
    uint32_t* gmap;  // [BMW] the block map in the workspace (OR-ed in by flush)
    int bshift;

    __device__ __forceinline__ void mark(long b) {
        if constexpr (MARK) {
            const uint32_t k = (uint32_t)(b >> bshift);
            atomicOr(&bm[k >> 5], 1u << (k & 31u));
        }
    }

    static_assert(!HASH || (W & (W - 1)) == 0, "hash table size must be a power of two");
    // probes before a key gives up on the table: once it fills, long probes cost more LDS
    // round trips than the global atomic they avoid (4 measured best of 1, 2, 4, 8, 32)
    static constexpr int HPROBE = 4;
    static constexpr uint32_t EMPTY = 0xFFFFFFFFu;  // never a key: 2 b + 1 < 2^32 - 1

    static constexpr int LOG2W = __builtin_ctz(W);
    static constexpr int DPP_WAVE_SHR1 = 0x138;  // DPP control: lane i reads lane i - 1

    __device__ __forceinline__ void bump(long b, int sg, int cnt) {
        if constexpr (HASH) {
            uint32_t* keys = reinterpret_cast<uint32_t*>(lh);
            int* vals = lh + W;
            const uint32_t key = (uint32_t)(2 * b + sg);
            // Fibonacci hashing: the top bits of key * 2^32/phi depend on every bit of the key
            // (its low bits would depend only on the key's low bits: sign and momentum, so the
            // same momentum in different cells would always collide)
            uint32_t h = (key * 2654435761u) >> (32 - LOG2W);
#pragma unroll 1
            for (int p = 0; p < HPROBE; ++p) {
                // a slot's key never changes once claimed: a plain read settles hits and
                // foreign keys, and only an empty slot needs the compare-and-swap
                uint32_t cur = __atomic_load_n(&keys[h], __ATOMIC_RELAXED);
                if (cur == EMPTY) cur = atomicCAS(&keys[h], EMPTY, key);
                if (cur == EMPTY || cur == key) {
                    atomicAdd(&vals[h], cnt);
                    return;
                }
                h = (h + 1) & (uint32_t)(W - 1);
            }
            mark(b);
            atomicAdd(&hist[sg * n_bins + b], cnt);
        } else {
            const int k = (int)b - (int)base;  // bins and base are below 2^31
            if ((unsigned)k < (unsigned)W) {
                atomicAdd(&lh[sg * W + k], cnt);
            } else {
                mark(b);
                atomicAdd(&hist[sg * n_bins + b], cnt);
            }
        }
    }

    // one particle per lane (b < 0: none); all 64 lanes of the wave must call it together
    // (32-bit keys 2 b + sign: n_bins < 2^31, and EMPTY marks "no particle")
    __device__ __forceinline__ void add_wave(long b, int8_t sv) {
        const int lane = threadIdx.x & 63;
        const uint32_t key = b < 0 ? EMPTY : 2u * (uint32_t)b + (sv > 0 ? 0u : 1u);
        // the previous lane's key by a DPP wave shift (a VALU move; __shfl_up is an LDS
        // permute with its round trip); lane 0 gets EMPTY and is a head anyway
        const uint32_t prev = (uint32_t)__builtin_amdgcn_update_dpp((int)EMPTY, (int)key, DPP_WAVE_SHR1,
                                                                    0xf, 0xf, false);
        const bool head = lane == 0 || prev != key;
        const unsigned long long heads = __ballot(head);
        if (head && key != EMPTY) {
            const unsigned long long above = lane == 63 ? 0ull : (heads >> (lane + 1));
            const int next = above ? lane + 1 + __builtin_ctzll(above) : 64;
            bump((long)(key >> 1), (int)(key & 1u), next - lane);
        }
    }

    // one particle, any lane pattern
    __device__ __forceinline__ void add_one(long b, int8_t sv) {
        if (b >= 0) bump(b, sv > 0 ? 0 : 1, 1);
    }

    // smallest live bin among the block's candidates -> window base (uniform in the block)
    __device__ void init(long b_min_thread, long* wminw) {
        for (int k = threadIdx.x; k < 2 * W; k += PT) lh[k] = (HASH && k < W) ? (int)EMPTY : 0;
        if constexpr (MARK)
            for (int k = threadIdx.x; k < BMW; k += PT) bm[k] = 0u;
        long b0 = b_min_thread;
        for (int o = 32; o > 0; o >>= 1) b0 = min(b0, (long)__shfl_xor(b0, o, 64));
        if ((threadIdx.x & 63) == 0) wminw[threadIdx.x >> 6] = b0;
        __syncthreads();
        long m = wminw[0];
#pragma unroll
        for (int k = 1; k < WPB; ++k) m = min(m, wminw[k]);
        base = m == LONG_MAX ? 0 : max(0L, m - W / 4);
    }

    __device__ void flush() {
        __syncthreads();
        if constexpr (HASH) {
            const uint32_t* keys = reinterpret_cast<const uint32_t*>(lh);
            for (int k = threadIdx.x; k < W; k += PT) {
                const uint32_t key = keys[k];
                const int v = lh[W + k];
                if (key != EMPTY && v != 0) {
                    mark((long)(key >> 1));
                    atomicAdd(&hist[(long)(key & 1u) * n_bins + (long)(key >> 1)], v);
                }
            }
        } else {
            for (int k = threadIdx.x; k < W; k += PT) {
                const long b = base + k;
                if (b >= n_bins) break;
                if (lh[k] | lh[W + k]) mark(b);
                if (lh[k]) atomicAdd(&hist[b], lh[k]);
                if (lh[W + k]) atomicAdd(&hist[n_bins + b], lh[W + k]);
            }
        }
        if constexpr (MARK) {
            __syncthreads();
            for (int k = threadIdx.x; k < BMW; k += PT)
                if (bm[k]) atomicOr(&gmap[k], bm[k]);
        }
    }
};

// Smallest live bin among a lane's first particles of its wave chunk (LONG_MAX if none).
template <typename T, typename MT, int DIM>
__device__ long first_bin(const Geo& g, const T* x, const T* y, const MT* M, const MT* My,
                          const int8_t* s, long lo, long hi) {
    long b0 = LONG_MAX;
    Part4<T, DIM> p;
    load4<T, MT, DIM>(x, y, M, My, s, lo + IT * (threadIdx.x & 63), hi, p);
#pragma unroll
    for (int k = 0; k < IT; ++k) {
        const long b = bin_val<T, DIM>(g, p.x[k], p.y[k], p.m[k], p.my[k], p.s[k]);
        if (b >= 0) b0 = min(b0, b);
    }
    return b0;
}

// ----------------------------------------------------------------------------- sp_step
// Meshes above CT_MAX cells: (n0, thr) of every cell gathered through cell_slot into one
// cell-indexed table, so that a particle's creation test is one load instead of two
// dependent ones.
__global__ void cell_table_kernel(long n_cells, const int32_t* __restrict__ cell_slot,
                                  const uint32_t* __restrict__ n0, const uint32_t* __restrict__ thr,
                                  uint2* __restrict__ ctab) {
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    const int sl = cell_slot[c];
    ctab[c] = sl < 0 ? make_uint2(0u, 0u) : make_uint2(n0[sl], thr[sl]);
}

// Pass 1: pairs per wave chunk of `in`.  Also clears the histogram pass 2 accumulates into
// and the absorption counters; refuses an input count the buffers cannot hold.
template <typename T, typename MT, int DIM>
__global__ __launch_bounds__(PT) void step_count(Geo g, uint32_t step, const int32_t* cell_slot,
                                                 const uint32_t* n0, const uint32_t* thr,
                                                 const T* x, const T* y, const MT* M,
                                                 const MT* My, const int8_t* s,
                                                 const long long* d_n_in, long long cap_in,
                                                 T* xo, int8_t* so, long long cap_out,
                                                 int32_t* hist, int sparse, long long* stats,
                                                 long long st, WS w) {
    __shared__ long long red[PT / 64];
    __shared__ uint2 ct_lds[CT_MAX];
    if (stats[WK_ST_OVERFLOW] != 0) return;
    const long n = (long)*d_n_in;
    if (n < 0 || n > cap_in || n > cap_out) {  // refused: nothing is written
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            stats[WK_ST_NEEDED] = n > cap_in || n < 0 ? -1 : n;
            stats[WK_ST_OVERFLOW] = 1;
            stats[WK_ST_OVERFLOW_STEP] = st;
        }
        return;
    }
    if (hist != nullptr && DIM == 2 && sparse) {
        // the histogram is zero outside the blocks the map marks: clear those blocks and the
        // map; map word k and its 32 blocks belong to workgroup k mod gridDim.x alone
        for (long k = blockIdx.x; k < BMW; k += gridDim.x) {
            uint32_t bits = w.blkmap[k];  // the same value in every thread: uniform branches
            while (bits) {
                const int j = __builtin_ctz(bits);
                bits &= bits - 1u;
                const long b0 = (k * 32 + j) << g.bshift;
                const long b1 = min(b0 + (1L << g.bshift), g.n_bins);
                for (long b = b0 + threadIdx.x; b < b1; b += PT) {
                    hist[b] = 0;
                    hist[g.n_bins + b] = 0;
                }
            }
            __syncthreads();  // every thread has read word k
            if (threadIdx.x == 0) w.blkmap[k] = 0u;
        }
    } else if (hist != nullptr) {
        const long nh = 2 * g.n_bins;
        for (long k = (long)blockIdx.x * PT + threadIdx.x; k < nh; k += (long)gridDim.x * PT) hist[k] = 0;
        if (DIM == 2)
            for (long k = (long)blockIdx.x * PT + threadIdx.x; k < BMW; k += (long)gridDim.x * PT) w.blkmap[k] = 0u;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        stats[WK_ST_ABS_X] = 0;
        stats[WK_ST_ABS_M] = 0;
    }
    const long n_cells = (long)g.nx * g.ny;
    const uint2* ct = w.ctab;  // larger meshes: the cell-indexed table of cell_table_kernel
    if (n_cells <= CT_MAX) {  // (n0, thr) per cell in LDS
        for (int c = threadIdx.x; c < n_cells; c += PT) {
            const int sl = cell_slot[c];
            ct_lds[c] = sl < 0 ? make_uint2(0u, 0u) : make_uint2(n0[sl], thr[sl]);
        }
        __syncthreads();
        ct = ct_lds;
    }
    long lo, hi;
    wave_chunk(n, (long)blockIdx.x * WPB + (threadIdx.x >> 6), &lo, &hi, (long)gridDim.x * WPB);
    const int lane = threadIdx.x & 63;
    long long cnt = 0;
    // A particle's (n0, thr) entry depends on its position: the entries of a tile are requested
    // (unconditionally: a particle without a cell reads entry 0 and ignores it) before the
    // next tile's positions, and the draws follow.  (Taking two or four tiles per round trip
    // raised the registers and was slower.)
    Part4<T, DIM> nxt;  // the next wave tile's loads stay in flight during this one
    load4<T, MT, DIM>(x, y, M, My, s, lo + IT * lane, hi, nxt);
    for (long t0 = lo; t0 < hi; t0 += WT) {  // per wave, no workgroup barriers
        const long id = t0 + IT * lane;
        uint2 e[IT];
        int8_t sv[IT];
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int c = live_cell<T, DIM>(g, nxt.x[k], nxt.y[k], nxt.s[k]);
            sv[k] = c < 0 ? (int8_t)0 : nxt.s[k];
            e[k] = ct[c < 0 ? 0 : c];
        }
        load4<T, MT, DIM>(x, y, M, My, s, id + WT, hi, nxt);
        int np[IT];
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            np[k] = sv[k] == 0 ? 0 : pairs_of_entry(g, (uint32_t)(id + k), step, e[k]);
            cnt += np[k];
        }
        store_np4<T>(xo, so, id, hi, np);  // for pass 2
    }
    store_counts(w, wave_sum_ll(cnt), red);
}

// Pass 2, in -> out: every workgroup totals the counts (capacity check, its waves' offsets);
// each wave then walks its chunk: the drifted and absorbed parents go to their own index and
// (HIST) into the histogram, and every particle that creates pairs goes into a per-wave
// queue in LDS (id, slot of its first child); the pair counts come from pass 1 (kept in the
// output buffer).  Between tiles, once the queue could not take another tile, and
// at the end of the chunk, the wave drains it one particle per lane: the parent's draws are
// redone (same Philox counters), its pairs' momentum offsets sampled from its CDF row and its
// children written.  One chain of dependent table loads serves up to 64 creating particles,
// and the streaming loop draws nothing.
constexpr int HW_STEP = 2048;
constexpr int QN = 320;  // creator queue entries per wave: up to 64 waiting + a tile of 256

template <typename T, typename MT, int DIM, bool HIST>
__global__ __launch_bounds__(PT) void step_apply(Geo g, uint32_t step, const int32_t* cell_slot,
                                                 const uint32_t* n0, const uint32_t* thr,
                                                 const uint64_t* cdf, const uint32_t* guide,
                                                 int guide_len, const T* x, const T* y,
                                                 const MT* M, const MT* My, const int8_t* s,
                                                 const long long* d_n_in, T* xo, T* yo, MT* Mo,
                                                 MT* Myo, int8_t* so, long long* d_n_out,
                                                 long long cap_out, int32_t* hist, uint32_t* keys,
                                                 long long* stats, long long st, WS w) {
    __shared__ long long red[PT / 64];
    __shared__ long wmin[PT / 64];
    __shared__ int lh[HIST ? 2 * HW_STEP : 1];
    __shared__ uint32_t bmap[HIST && DIM == 2 ? BMW : 1];
    __shared__ uint32_t q_id[WPB][QN];
    __shared__ int q_o[WPB][QN];
    if (stats[WK_ST_OVERFLOW] != 0) return;
    const long n = (long)*d_n_in;
    long long run;
    const long long total = chunk_offsets(w, true, &run, red, (int)gridDim.x);  // grid = step_count's
    const long long needed = n + 2 * total;
    if (needed > cap_out) {  // the same decision in every workgroup
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            stats[WK_ST_NEEDED] = needed;
            stats[WK_ST_OVERFLOW] = 1;
            stats[WK_ST_OVERFLOW_STEP] = st;
        }
        return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        stats[WK_ST_N] = needed;
        stats[WK_ST_PAIRS] = total;
        stats[WK_ST_NEEDED] = 0;
        stats[WK_ST_CUM_STEPS] += 1;
        stats[WK_ST_CUM_N] += n;
        stats[WK_ST_CUM_PAIRS] += total;
        *d_n_out = needed;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    long lo, hi;
    wave_chunk(n, (long)blockIdx.x * WPB + wv, &lo, &hi, (long)gridDim.x * WPB);
    const T vdt = (T)g.vdt;
    long long abs_x = 0, abs_m = 0;
    HistWindow<HW_STEP, DIM == 2, DIM == 2> hw{lh, 0, hist, g.n_bins, bmap, w.blkmap, g.bshift};
    if (HIST) hw.init(first_bin<T, MT, DIM>(g, x, y, M, My, s, lo, hi), wmin);
    auto absorbed = [&](T nx_, T ny_, int m, int my) -> int {
        bool outx = !inside<T>(nx_, g.nx);
        if (DIM == 2) outx = outx || !inside<T>(ny_, g.ny);
        bool outm = m < g.M_min || m >= g.M_min + g.n_k;
        if (DIM == 2) outm = outm || my < g.M_min || my >= g.M_min + g.n_k;
        return outx ? 1 : (outm ? 2 : 0);
    };
    int qhead = 0, qlen = 0;  // uniform in the wave
    // children of the queued particles until at most `keep` remain, up to 64 at a time
    auto drain = [&](int keep) {
        wave_lds_sync();
        while (qlen > keep) {
            const int cnt = qlen < 64 ? qlen : 64;
            if (lane < cnt) {
                int e = qhead + lane;
                if (e >= QN) e -= QN;
                const long pid = (long)q_id[wv][e];
                long o = (long)q_o[wv][e];
                const T px = x[pid];
                const T py = DIM == 2 ? y[pid] : (T)0;
                const int pm = (int)M[pid];
                const int pmy = DIM == 2 ? (int)My[pid] : 0;
                const int8_t ps = s[pid];
                int row;
                u32x4 r;
                const int np = pairs_of<T, DIM>(g, (uint32_t)pid, step, px, py, ps, cell_slot, n0,
                                                thr, &row, &r);
                const uint64_t* crow = cdf + (long)row * g.width;
                const uint32_t* grow = guide ? guide + (long)row * (guide_len + 1) : nullptr;
                for (int q = 0; q < np; ++q) {
                    uint32_t u;
                    if (q < 3) {
                        u = q == 0 ? r.v[1] : (q == 1 ? r.v[2] : r.v[3]);
                    } else {
                        const u32x4 r2 = philox((uint32_t)pid, step, (uint32_t)(1 + (q - 3) / 4),
                                                TAG_CREATE, g.seed);
                        const int wq = (q - 3) & 3;
                        u = wq == 0 ? r2.v[0] : (wq == 1 ? r2.v[1] : (wq == 2 ? r2.v[2] : r2.v[3]));
                    }
                    const int t = sample_cdf(crow, grow, guide_len, g.width, u);
                    const int mx = (DIM == 1 ? t : t % g.n_m) - g.P;
                    const int my = DIM == 1 ? 0 : t / g.n_m - g.P;
#pragma unroll
                    for (int ch = 0; ch < 2; ++ch, ++o) {
                        const int sg = ch == 0 ? 1 : -1;
                        const int cm = pm + sg * mx, cmy = pmy + sg * my;
                        const T cx = drift(px, cm, vdt);
                        const T cy = DIM == 2 ? drift(py, cmy, vdt) : (T)0;
                        const int a = absorbed(cx, cy, cm, cmy);
                        abs_x += a == 1;
                        abs_m += a == 2;
                        const int8_t cs = a ? (int8_t)0 : (int8_t)(sg * ps);
                        if (o >= n && o < cap_out) {  // always true after the capacity check
                            xo[o] = cx;
                            Mo[o] = (MT)cm;
                            if (DIM == 2) {
                                yo[o] = cy;
                                Myo[o] = (MT)cmy;
                            }
                            so[o] = cs;
                        }
                        if (HIST) {
                            const long cb = bin_val<T, DIM>(g, cx, cy, cm, cmy, cs);
                            if (keys != nullptr && o >= n && o < cap_out) keys[o] = hist_key(cb, cs);
                            hw.add_one(cb, cs);
                        }
                    }
                }
            }
            qhead += cnt;
            if (qhead >= QN) qhead -= QN;
            qlen -= cnt;
        }
        wave_lds_sync();  // the entries are reused by later particles
    };
    Raw4<T, MT, DIM> nxt;  // the next wave tile's loads stay in flight during this one
    load4r<T, MT, DIM>(x, y, M, My, s, lo + IT * lane, hi, nxt);
    for (long t0 = lo; t0 < hi; t0 += WT) {  // per wave, no workgroup barriers
        const long id = t0 + IT * lane;
        Part4<T, DIM> p = unpack(nxt);
        load4r<T, MT, DIM>(x, y, M, My, s, id + WT, hi, nxt);
        int np[IT];
        load_np4<T>(xo, so, id, hi, np);  // left by pass 1 (before the parents overwrite it below)
        // after the capacity check all pairs of the step number below 2^30: 32-bit sums
        int npt = 0;
#pragma unroll
        for (int k = 0; k < IT; ++k) npt += np[k];
        const int inc = wave_incl_scan(npt);
        long o = n + 2 * (long)(run + (inc - npt));  // this lane's first child slot
        run += __shfl(inc, 63, 64);
        // queue the creating particles (at most WT per tile; room was left by the last drain)
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const bool has = np[k] > 0;
            const unsigned long long m = __ballot(has);
            if (has) {
                int e = qhead + qlen + __popcll(m & ((1ull << lane) - 1ull));
                if (e >= QN) e -= QN;
                q_id[wv][e] = (uint32_t)(id + k);
                q_o[wv][e] = (int)o;
            }
            qlen += __popcll(m);
            o += 2 * np[k];
        }
        // parents: drift, absorb, same index in `out` (n <= cap_out was checked)
        T nxv[IT], nyv[IT];
        uint32_t kk[IT];
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
                if (a) p.s[k] = 0;
            }
            if (HIST) {
                const long b = bin_val<T, DIM>(g, nxv[k], nyv[k], p.m[k], p.my[k], p.s[k]);
                kk[k] = hist_key(b, p.s[k]);
                hw.add_wave(b, p.s[k]);
            }
        }
        store4<T, MT, DIM>(xo, yo, Mo, Myo, so, id, hi, nxv, nyv, p);
        if (HIST && keys != nullptr) {
            if (id + IT <= hi) {
                *reinterpret_cast<uint4*>(keys + id) = make_uint4(kk[0], kk[1], kk[2], kk[3]);
            } else {
#pragma unroll
                for (int k = 0; k < IT; ++k)
                    if (id + k < hi) keys[id + k] = kk[k];
            }
        }
        if (qlen > QN - WT) drain(QN - WT);  // room for the next tile
    }
    drain(0);
    if (HIST) hw.flush();
    abs_x = block_sum_ll(abs_x, red);
    abs_m = block_sum_ll(abs_m, red);
    if (threadIdx.x == 0) {
        if (abs_x) atomicAdd(reinterpret_cast<unsigned long long*>(&stats[WK_ST_ABS_X]), (unsigned long long)abs_x);
        if (abs_m) atomicAdd(reinterpret_cast<unsigned long long*>(&stats[WK_ST_ABS_M]), (unsigned long long)abs_m);
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

// The mixed-bin bits of the bins a workgroup's particles fall in, copied to LDS (KWW words of
// 32 bins from a quarter window below the smallest bin of its waves' first tiles); the
// survivor test reads there and falls back to the global bitmap outside the window.
constexpr int KWW = 2048;

struct KeepWindow {
    const uint32_t* lw;  // [KWW] in LDS
    long base;           // first word of the window
    const uint32_t* bits;
    const uint8_t* flags;  // pair removal: per input particle, 1 = not annihilated (else NULL)

    // Particle `id` in bin b survives rule 2: its bin holds one sign, or (pair removal) it
    // has no partner of the other sign.
    __device__ __forceinline__ bool keeps(long b, long id) const {
        if (b < 0) return false;
        const long wd = b >> 5;
        const int k = (int)(wd - base);  // words are below 2^26
        const uint32_t word = (unsigned)k < (unsigned)KWW ? lw[k] : bits[wd];
        if (((word >> (b & 31)) & 1u) == 0u) return true;
        return flags != nullptr && flags[id] != 0;
    }
    // the bin holds both signs
    __device__ __forceinline__ bool mixed(long b) const {
        if (b < 0) return false;
        const long wd = b >> 5;
        const int k = (int)(wd - base);
        const uint32_t word = (unsigned)k < (unsigned)KWW ? lw[k] : bits[wd];
        return ((word >> (b & 31)) & 1u) != 0u;
    }
};

__device__ KeepWindow keep_window(long b_min_thread, uint32_t* lw, long* wminw, const uint32_t* bits,
                                  long n_words, const uint8_t* flags) {
    long b0 = b_min_thread;
    for (int o = 32; o > 0; o >>= 1) b0 = min(b0, (long)__shfl_xor(b0, o, 64));
    if ((threadIdx.x & 63) == 0) wminw[threadIdx.x >> 6] = b0;
    __syncthreads();
    long m = wminw[0];
#pragma unroll
    for (int k = 1; k < WPB; ++k) m = min(m, wminw[k]);
    const long base = m == LONG_MAX ? 0 : max(0L, (m >> 5) - KWW / 4);
    for (int k = threadIdx.x; k < KWW; k += PT) {
        const long wd = base + k;
        lw[k] = wd < n_words ? bits[wd] : 0u;
    }
    __syncthreads();
    return KeepWindow{lw, base, bits, flags};
}

// ----------------------------------------------------------------------------- annihilation
__global__ void fill_i32(int32_t* p, long n, int32_t v) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        p[i] = v;
}

// Stand-alone histogram pass (when sp_step did not build it), over the wave chunks.
constexpr int HW = 4096;

template <typename T, typename MT, int DIM>
__global__ __launch_bounds__(PT) void annih_hist(Geo g, const T* x, const T* y, const MT* M,
                                                 const MT* My, const int8_t* s,
                                                 const long long* d_n, long long cap_in,
                                                 int32_t* hist, uint32_t* blkmap,
                                                 const long long* stats) {
    __shared__ int lh[2 * HW];
    __shared__ uint32_t bmap[DIM == 2 ? BMW : 1];
    __shared__ long wmin[PT / 64];
    if (stats[WK_ST_OVERFLOW] != 0) return;
    const long n = (long)*d_n;
    if (n < 0 || n > cap_in) return;  // refused by annih_count
    long lo, hi;
    wave_chunk(n, (long)blockIdx.x * WPB + (threadIdx.x >> 6), &lo, &hi);
    HistWindow<HW, DIM == 2, DIM == 2> hw{lh, 0, hist, g.n_bins, bmap, blkmap, g.bshift};
    hw.init(first_bin<T, MT, DIM>(g, x, y, M, My, s, lo, hi), wmin);
    Raw4<T, MT, DIM> nxt;  // the next wave tile's loads stay in flight during this one
    load4r<T, MT, DIM>(x, y, M, My, s, lo + IT * (threadIdx.x & 63), hi, nxt);
    for (long t0 = lo; t0 < hi; t0 += WT) {
        const long id = t0 + IT * (threadIdx.x & 63);
        Part4<T, DIM> p = unpack(nxt);
        load4r<T, MT, DIM>(x, y, M, My, s, id + WT, hi, nxt);
#pragma unroll
        for (int k = 0; k < IT; ++k)
            hw.add_wave(bin_val<T, DIM>(g, p.x[k], p.y[k], p.m[k], p.my[k], p.s[k]), p.s[k]);
    }
    hw.flush();
}

// Counting pass of sp_annihilate over the particles: each wave counts the survivors (particles
// of bins holding one sign) of its chunk of `in`, reading the mixed-bin bits annih_bins left.
template <typename T, typename MT, int DIM>
__global__ __launch_bounds__(PT) void annih_count(Geo g, const T* x, const T* y, const MT* M,
                                                  const MT* My, const int8_t* s,
                                                  const long long* d_n_in, long long cap_in,
                                                  const uint8_t* flags, uint32_t* kbits,
                                                  const uint32_t* keys, long long* stats, WS w) {
    __shared__ long long red[PT / 64];
    __shared__ uint32_t lw[KWW];
    __shared__ long wmin[PT / 64];
    if (stats[WK_ST_OVERFLOW] != 0) return;
    const long n = (long)*d_n_in;
    if (n < 0 || n > cap_in) {  // refused: nothing is written
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            stats[WK_ST_NEEDED] = -1;
            stats[WK_ST_OVERFLOW] = 1;
        }
        return;
    }
    const int lane = threadIdx.x & 63;
    long lo, hi;
    wave_chunk(n, (long)blockIdx.x * WPB + (threadIdx.x >> 6), &lo, &hi, (long)gridDim.x * WPB);
    long long a = 0;
    // one keep bit per particle: word q of the tile (ids t0 + 32q .. t0 + 32q + 31, t0 a
    // multiple of 256) holds bit k of lane 8q + i at 4i + k, built from one ballot per k
    auto tile_done = [&](long t0, uint32_t nib) {
        a += __popc(nib);
        if (kbits != nullptr) {
            uint32_t word = 0;
#pragma unroll
            for (int k = 0; k < IT; ++k)
                word |= spread4((uint32_t)(__ballot((nib >> k) & 1u) >> (8 * (lane & 7))) & 0xFFu) << k;
            if (lane < 8) kbits[(t0 >> 5) + lane] = word;
        }
    };
    if (keys != nullptr && flags == nullptr) {
        // With the keys sp_step wrote for `in`, a particle's mixed-bin word is one load that
        // depends on one 4-byte load.  The wave takes KG tiles at a time: their keys were
        // loaded during the previous group, and the words of all KG tiles are loaded together,
        // so one round trip to the map serves KG tiles (4 measured best of 1, 2, 4, 8).  The
        // words come straight from the map, with no LDS window to fill first; a dead particle
        // or a slot past the chunk (HKEY_NONE) reads word 0 and ignores it.  The pair removal
        // (flags) never passes keys; it takes the window path below.
        constexpr int KG = 4;
        uint32_t knx[KG][IT];
#pragma unroll
        for (int u = 0; u < KG; ++u) load_keys4(keys, lo + u * WT + IT * lane, hi, knx[u]);
        for (long t0 = lo; t0 < hi; t0 += KG * WT) {  // per wave, no workgroup barriers
            uint32_t kc[KG][IT], wd[KG][IT];
#pragma unroll
            for (int u = 0; u < KG; ++u)
#pragma unroll
                for (int k = 0; k < IT; ++k) kc[u][k] = knx[u][k];
#pragma unroll
            for (int u = 0; u < KG; ++u)
#pragma unroll
                for (int k = 0; k < IT; ++k) wd[u][k] = w.mixbits[kc[u][k] == HKEY_NONE ? 0u : kc[u][k] >> 6];
#pragma unroll
            for (int u = 0; u < KG; ++u) load_keys4(keys, t0 + (KG + u) * WT + IT * lane, hi, knx[u]);
#pragma unroll
            for (int u = 0; u < KG; ++u) {
                if (t0 + u * WT >= hi) break;  // uniform in the wave
                uint32_t nib = 0;
#pragma unroll
                for (int k = 0; k < IT; ++k)  // survives rule 2: its bin holds one sign
                    nib |= kc[u][k] != HKEY_NONE && ((wd[u][k] >> ((kc[u][k] >> 1) & 31u)) & 1u) == 0u
                               ? 1u << k : 0u;
                tile_done(t0 + u * WT, nib);
            }
        }
    } else {
        const KeepWindow kw = keep_window(first_bin<T, MT, DIM>(g, x, y, M, My, s, lo, hi), lw, wmin,
                                          w.mixbits, 8 * g.n_chunks, flags);
        Raw4<T, MT, DIM> nxt;  // the next wave tile's loads stay in flight during this one
        load4r<T, MT, DIM>(x, y, M, My, s, lo + IT * lane, hi, nxt);
        for (long t0 = lo; t0 < hi; t0 += WT) {
            const long id = t0 + IT * lane;
            Part4<T, DIM> p = unpack(nxt);
            load4r<T, MT, DIM>(x, y, M, My, s, id + WT, hi, nxt);
            uint32_t nib = 0;
#pragma unroll
            for (int k = 0; k < IT; ++k)
                nib |= kw.keeps(bin_val<T, DIM>(g, p.x[k], p.y[k], p.m[k], p.my[k], p.s[k]), id + k) ? 1u << k : 0u;
            tile_done(t0, nib);
        }
    }
    store_counts(w, wave_sum_ll(a), red);
}

// Counting pass over the bins of sp_annihilate (histogram) and sp_init (per-bin counts): bin
// workgroup c owns g.gpb consecutive chunks of BC bins and its waves take every WPB-th chunk.
// Per chunk (lane l holds bins 4l .. 4l+3): the particles to place (csum), their placement
// work items, and, from the histogram, one bit per bin that holds both signs (mixbits, eight
// words per chunk).  Per bin workgroup: the particles to place (bpart), its mixed bins
// (bmixed) and work items (bitem).  place = 0 (pair removal): nothing is placed.
__global__ __launch_bounds__(PT) void annih_bins(Geo g, BinCount bc, int place, const long long* stats,
                                                 WS w, const uint32_t* marked) {
    __shared__ long long red[PT / 64];
    if (stats[WK_ST_OVERFLOW] != 0) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const long c = blockIdx.x;
    const long j0 = min(g.n_chunks, c * g.gpb), j1 = min(g.n_chunks, j0 + g.gpb);
    const bool vec = bc.counts == nullptr && (bc.n_bins & 3) == 0 &&  // 16-byte aligned rows
                     (reinterpret_cast<uintptr_t>(bc.hist) & 15) == 0;
    long long part = 0, mixed = 0, items = 0;
    for (long j = j0 + wv; j < j1; j += WPB) {  // per wave, no workgroup barriers
        const long b0 = j * BC + 4 * lane;
        int cnt[4];
        uint32_t mb = 0;
        // a block the histogram builder never added to holds only zeros (wave-uniform test)
        const long blk = (j * BC) >> g.bshift;
        if (marked != nullptr && ((marked[blk >> 5] >> (blk & 31)) & 1u) == 0u) {
#pragma unroll
            for (int k = 0; k < 4; ++k) cnt[k] = 0;
        } else if (vec && b0 + 3 < bc.n_bins) {
            const int4 hp = *reinterpret_cast<const int4*>(bc.hist + b0);
            const int4 hm = *reinterpret_cast<const int4*>(bc.hist + bc.n_bins + b0);
            const int a[4] = {hp.x, hp.y, hp.z, hp.w}, m[4] = {hm.x, hm.y, hm.z, hm.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const bool mx = a[k] > 0 && m[k] > 0;
                cnt[k] = mx ? (a[k] > m[k] ? a[k] - m[k] : m[k] - a[k]) : 0;
                mb |= mx ? 1u << k : 0u;
            }
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const long b = b0 + k;
                cnt[k] = b < g.n_bins ? (int)bc(b) : 0;
                mb |= (b < g.n_bins && bc.mixed(b)) ? 1u << k : 0u;
            }
        }
        // the chunk's particles to place; from a histogram every lane's sum is in [0, 2^33)
        const long long ls = (long long)cnt[0] + cnt[1] + cnt[2] + cnt[3];
        const long long t = !place ? 0 : bc.counts == nullptr ? wave_sum_nonneg33(ls) : wave_sum_ll(ls);
        mixed += __popc(mb);
        if (lane == 0) {
            w.csum[j] = (int)t;  // < 2^31 whenever the capacity check passes
            part += t;
            items += (t + PIECE - 1) / PIECE;
        }
        if (bc.counts == nullptr) {
            // word q of the chunk (bins 32q .. 32q+31) holds bit k of lane 8q + i at 4i + k
            uint32_t word = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                word |= spread4((uint32_t)(__ballot((mb >> k) & 1u) >> (8 * (lane & 7))) & 0xFFu) << k;
            if (lane < 8) w.mixbits[j * 8 + lane] = word;
        }
    }
    part = block_sum_ll(part, red);
    mixed = block_sum_ll(mixed, red);
    items = block_sum_ll(items, red);
    if (threadIdx.x == 0) {
        w.bpart[c] = part;
        w.bmixed[c] = mixed;
        w.bitem[c] = items;
    }
}

// One wave places the particles of one bin chunk (BC bins, chunk output count cnt_ch starting
// at output slot ch_start) that fall in the slot range [s_lo, s_hi).  Lane j reads bins
// 4j .. 4j+3 of the chunk; a wave scan of their counts gives every bin's first slot, which the
// lanes keep in the wave's LDS table with the bin's cell, momenta and sign; then consecutive
// lanes fill consecutive slots (coalesced stores), each taking its position from its Philox
// block (4 draws = 4 positions in 1-D, 2 x (x, y) in 2-D).  No workgroup barrier: the waves
// of a placing workgroup work on different chunks.  build = false: the table already holds
// this chunk (consecutive pieces of one chunk).
constexpr int PW_LDS = 6 * BC;  // ints per wave: inclusive offsets, x, kx, y, ky, sign
template <typename T, typename MT, int DIM>
__device__ void place_chunk_wave(const Geo& g, const BinCount& bc, int mode, uint32_t c1, uint32_t tag,
                                 long ch, long ch_start, long cnt_ch, long s_lo, long s_hi, T* xo,
                                 T* yo, MT* Mo, MT* Myo, int8_t* so, long long capacity, int* wl,
                                 bool build) {
    constexpr int Q = DIM == 1 ? 4 : 2;
    const int lane = threadIdx.x & 63;
    int* bo_in = wl;            // [BC] inclusive slot offsets
    int* m_x = wl + BC;         // [BC] cell x
    int* m_kx = wl + 2 * BC;    // [BC] momentum index x
    int* m_y = wl + 3 * BC;     // [BC] cell y (2-D)
    int* m_ky = wl + 4 * BC;    // [BC] momentum index y (2-D)
    int* m_s = wl + 5 * BC;     // [BC] sign
    if (build) {  // else the table holds this chunk already (the previous piece's)
        const long b0 = ch * BC + 4 * lane;
        int cnt[4], sg[4], tot4 = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const long b = b0 + k;
            cnt[k] = 0;
            sg[k] = 1;
            if (b < g.n_bins) {
                if (bc.counts) {
                    const int c = bc.counts[b];
                    cnt[k] = c > 0 ? c : 0;
                } else {
                    const int hp = bc.hist[b], hm = bc.hist[bc.n_bins + b];
                    if (hp > 0 && hm > 0) cnt[k] = hp > hm ? hp - hm : hm - hp;
                    sg[k] = hp > hm ? 1 : -1;
                }
            }
            tot4 += cnt[k];
        }
        int run = wave_incl_scan(tot4) - tot4;
        wave_lds_sync();  // the previous chunk's fill has read the table
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            run += cnt[k];
            const int j = 4 * lane + k;
            bo_in[j] = run;
            if (cnt[k] > 0) {
                // this bin's cell and momenta (32-bit index arithmetic: n_bins < 2^31)
                const uint32_t b32 = (uint32_t)(b0 + k), nk = (uint32_t)g.n_k;
                if (DIM == 1) {
                    const uint32_t cx = b32 / nk;
                    m_x[j] = (int)cx;
                    m_kx[j] = (int)(b32 - cx * nk);
                } else {
                    const uint32_t t = b32 / nk, cc = t / nk, cy = cc / (uint32_t)g.nx;
                    m_kx[j] = (int)(b32 - t * nk);
                    m_ky[j] = (int)(t - cc * nk);
                    m_x[j] = (int)(cc - cy * (uint32_t)g.nx);
                    m_y[j] = (int)cy;
                }
                m_s[j] = mode == 1 ? sg[k] : 1;
            }
        }
        wave_lds_sync();
    }
    const int lo_c = (int)(max(s_lo, ch_start) - ch_start);            // slots of this chunk
    const int hi_c = (int)(min(s_hi, ch_start + cnt_ch) - ch_start);   // to fill: [lo_c, hi_c)
    // A slot's bin is the first j with bo_in[j] > rel (bo_in[BC - 1] = cnt_ch exceeds every
    // slot).  The last offsets of the first 15 groups of 16 bins, read once (the same for
    // every lane), give a slot's group by compares; a search of its 16 entries follows: five
    // dependent LDS reads per slot instead of nine.
    static_assert(BC == 256, "16 groups of 16 bins");
    int cb[15];
#pragma unroll
    for (int i = 0; i < 15; ++i) cb[i] = __builtin_amdgcn_readfirstlane(bo_in[16 * i + 15]);
    for (int rel = lo_c + lane; rel < hi_c; rel += 64) {
        int gi = 0;
#pragma unroll
        for (int i = 0; i < 15; ++i) gi += cb[i] <= rel ? 1 : 0;
        const int j = 16 * gi + upper_bound_lds(bo_in + 16 * gi, 16, rel);
        const int r = rel - (j ? bo_in[j - 1] : 0);
        const long bb = ch * BC + j;
        const long o = ch_start + rel;
        if (o >= capacity) break;  // never taken after the capacity check
        const int8_t sign = (int8_t)m_s[j];
        const u32x4 u = philox((uint32_t)bb, c1, (uint32_t)(r / Q), tag, g.seed);
        const int e = r % Q;
        if (DIM == 1) {
            const uint32_t ue = e == 0 ? u.v[0] : (e == 1 ? u.v[1] : (e == 2 ? u.v[2] : u.v[3]));
            xo[o] = cell_plus_frac<T>(m_x[j], ue, g.fb);
            Mo[o] = (MT)(g.M_min + m_kx[j]);
        } else {
            xo[o] = cell_plus_frac<T>(m_x[j], e ? u.v[2] : u.v[0], g.fb);
            yo[o] = cell_plus_frac<T>(m_y[j], e ? u.v[3] : u.v[1], g.fb);
            Mo[o] = (MT)(g.M_min + m_kx[j]);
            Myo[o] = (MT)(g.M_min + m_ky[j]);
        }
        so[o] = sign;
    }
}

// Between the counting and the writing pass of sp_annihilate (mode 1) / sp_init (mode 0),
// one workgroup: prefix of the particles to place per bin workgroup (bpre, inclusive) and of
// the survivors per particle workgroup (kpre, exclusive), the capacity check, the counts
// and statistics, and for every placing workgroup the bin workgroup where its equal share of
// output slots starts.
constexpr int ST_THREADS = 1024;
static_assert(PB % ST_THREADS == 0 && SB_MAX % ST_THREADS == 0, "scans take whole threads' shares");

__global__ __launch_bounds__(ST_THREADS) void annih_scan(int mode, int place_blocks,
                                                         const long long* d_n_in,
                                                         long long* d_n_out, long long capacity,
                                                         long long kb_limit, int owners,
                                                         long long* stats, WS w) {
    __shared__ long long bp[PB];
    __shared__ long long part[ST_THREADS];
    __shared__ long long tot[2];
    if (stats[WK_ST_OVERFLOW] != 0) {
        if (threadIdx.x == 0) w.sc[SC_GO] = 0;
        return;
    }
    constexpr int PER_MAX = SB_MAX / ST_THREADS;
    constexpr int NWS = ST_THREADS / 64;
    // exclusive / inclusive scans of m values (PB, or the `owners` of the particle counts), per
    // thread m / ST_THREADS consecutive ones: thread sums scanned within each wave by shuffles,
    // then across the waves' totals
    auto scan = [&](const long long* in, long long* out_excl, long long* out_incl, long long* total,
                    int m) {
        const int per = m / ST_THREADS;
        long long loc[PER_MAX], acc = 0;
#pragma unroll
        for (int k = 0; k < PER_MAX; ++k) {
            loc[k] = k < per ? in[threadIdx.x * per + k] : 0;
            acc += loc[k];
        }
        const long long inc = wave_incl_scan_ll(acc);
        if ((threadIdx.x & 63) == 63) part[threadIdx.x >> 6] = inc;
        __syncthreads();
        long long base = 0;
        for (int k = 0; k < (int)(threadIdx.x >> 6); ++k) base += part[k];
        if (threadIdx.x == ST_THREADS - 1) {
            long long t = 0;
            for (int k = 0; k < NWS; ++k) t += part[k];
            part[NWS] = t;
        }
        __syncthreads();
        long long run = base + inc - acc;
#pragma unroll
        for (int k = 0; k < PER_MAX; ++k) {
            if (k >= per) break;
            if (out_excl) out_excl[threadIdx.x * per + k] = run;
            run += loc[k];
            if (out_incl) out_incl[threadIdx.x * per + k] = run;
        }
        if (threadIdx.x == 0) *total = part[NWS];
        __syncthreads();
    };
    scan(w.bpart, nullptr, bp, &tot[0], PB);
    if (mode == 1) {
        scan(w.bcnt, w.kpre, nullptr, &tot[1], owners);
    } else if (threadIdx.x == 0) {
        tot[1] = 0;
    }
    long long mx = 0;
    for (int k = threadIdx.x; k < PB; k += ST_THREADS) {
        w.bpre[k] = bp[k];
        mx += w.bmixed[k];
    }
    mx = wave_sum_ll(mx);
    __syncthreads();
    const long long placed = tot[0], kept = tot[1];
    // placement work items: prefix per bin workgroup, then every placing wave's first one
    __syncthreads();  // bp (the placed-particle prefix) has been copied out above
    __shared__ long long n_items;
    scan(w.bitem, nullptr, bp, &n_items, PB);
    for (int k = threadIdx.x; k < PB; k += ST_THREADS) w.ipre[k] = bp[k];
    const long long nw = (long long)place_blocks * WPB;
    const long long per_it = (n_items + nw - 1) / nw;
    for (int v = threadIdx.x; v < nw; v += ST_THREADS)
        w.wstart[v] = upper_bound_lds(bp, PB, (long long)min(n_items, (long long)v * per_it));
    // mixed-bin total: one value per wave, summed by thread 0
    __shared__ long long wmx[ST_THREADS / 64];
    if ((threadIdx.x & 63) == 0) wmx[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x != 0) return;
    long long mixed = 0;
    for (int k = 0; k < ST_THREADS / 64; ++k) mixed += wmx[k];
    const long long n_out = placed + kept;
    if (n_out > capacity) {
        stats[WK_ST_NEEDED] = n_out;
        stats[WK_ST_OVERFLOW] = 1;
        w.sc[SC_GO] = 0;
        return;
    }
    w.sc[SC_GO] = 1;
    w.sc[SC_PLACED] = placed;
    w.sc[SC_KEPT] = kept;
    w.sc[SC_ITEMS] = n_items;
    // the counting pass's keep bits sit past the output's positions when they fit there
    w.sc[SC_KBITS] = mode == 1 && kb_limit >= 0 && n_out <= kb_limit;
    stats[WK_ST_N] = n_out;
    stats[WK_ST_NEEDED] = 0;
    if (mode == 1) {
        const long long n_in = *d_n_in;
        stats[WK_ST_KEPT] = kept;
        stats[WK_ST_REGEN] = placed;
        stats[WK_ST_MIXED] = mixed;
        stats[WK_ST_CUM_ANNIH_IN] += n_in;
        stats[WK_ST_CUM_KEPT] += kept;
        stats[WK_ST_CUM_REGEN] += placed;
    }
    *d_n_out = n_out;
}

// Writing pass of sp_annihilate (mode 1) and sp_init (mode 0).  Output: the particles placed
// bin by bin (mixed bins' survivors of rule 2, or the initial state), then, in mode 1, the
// particles of single-sign bins in input order.  Workgroups below part_blocks copy their
// waves' survivors, in order, through an LDS stage; the place_blocks after them fill equal
// ranges of the placed particles' output slots bin chunk by bin chunk.
template <typename T, typename MT, int DIM>
__global__ __launch_bounds__(PT) void annih_write(Geo g, int part_blocks, int place_blocks,
                                                  BinCount bc, int mode, uint32_t c1,
                                                  uint32_t tag, const T* x, const T* y,
                                                  const MT* M, const MT* My, const int8_t* s,
                                                  const long long* d_n_in, T* xo, T* yo, MT* Mo,
                                                  MT* Myo, int8_t* so, long long capacity,
                                                  const uint8_t* flags, const uint32_t* kbits,
                                                  WS w) {
    constexpr int STAGE = WT * (DIM * (int)sizeof(T) + DIM * (int)sizeof(int) + 1);  // per wave
    constexpr int KEEP_LDS = WPB * STAGE + KWW * (int)sizeof(uint32_t);
    constexpr int PLACE_LDS = WPB * PW_LDS * (int)sizeof(int);
    __shared__ long wmin[PT / 64];
    // keepers: one stage per wave + histogram window; placers: chunk and bin prefix tables
    __shared__ __align__(16) char smem[KEEP_LDS > PLACE_LDS ? KEEP_LDS : PLACE_LDS];
    uint32_t* lw = reinterpret_cast<uint32_t*>(smem + WPB * STAGE);
    if (w.sc[SC_GO] == 0) return;
    const long long placed = w.sc[SC_PLACED];
    if ((int)blockIdx.x < part_blocks) {
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        // per-wave stage: the tile's survivors, compacted, then written out contiguously
        char* st = smem + wv * STAGE;
        T* sx = reinterpret_cast<T*>(st);
        T* sy = sx + (DIM == 2 ? WT : 0);
        int* sm = reinterpret_cast<int*>(sx + DIM * WT);
        int* smy = sm + (DIM == 2 ? WT : 0);
        int8_t* ssg = reinterpret_cast<int8_t*>(sm + DIM * WT);
        long lo, hi;
        wave_chunk((long)*d_n_in, (long)blockIdx.x * WPB + wv, &lo, &hi, (long)part_blocks * WPB);
        // with the counting pass's keep bits, a lane loads its four particles only when one of
        // them survives (particles of mixed bins, about half, are never read again); without
        // them the survivor test is redone from the positions and momenta
        const bool bits = kbits != nullptr && w.sc[SC_KBITS] != 0;
        KeepWindow kw{};
        if (!bits)
            kw = keep_window(first_bin<T, MT, DIM>(g, x, y, M, My, s, lo, hi), lw, wmin, w.mixbits,
                             8 * g.n_chunks, flags);
        // keep bits of lane `lane`'s four particles of the tile at t (t a multiple of 256)
        auto nib_at = [&](long t) -> uint32_t {
            return t < hi ? (kbits[(t >> 5) + (lane >> 3)] >> (4 * (lane & 7))) & 0xFu : 0u;
        };
        long long run = placed + w.kpre[blockIdx.x];
        for (int j = 0; j < wv; ++j) run += w.wcnt[(long)blockIdx.x * WPB + j];
        uint32_t nib_n = bits ? nib_at(lo) : 0xFu;  // the tile in flight, and the one after
        Part4<T, DIM> nxt;  // the next wave tile's loads stay in flight during this one
        if (nib_n) load4<T, MT, DIM>(x, y, M, My, s, lo + IT * lane, hi, nxt);
        uint32_t nib_nn = bits ? nib_at(lo + WT) : 0xFu;
        for (long t0 = lo; t0 < hi; t0 += WT) {  // per wave, no workgroup barriers
            const long id = t0 + IT * lane;
            Part4<T, DIM> p = nxt;
            const uint32_t nib = nib_n;
            nib_n = nib_nn;
            if (nib_n) load4<T, MT, DIM>(x, y, M, My, s, id + WT, hi, nxt);
            if (bits) nib_nn = nib_at(t0 + 2 * WT);
            bool kp[IT];
            int kt = 0;
#pragma unroll
            for (int k = 0; k < IT; ++k) {
                kp[k] = bits ? ((nib >> k) & 1u) != 0u
                             : kw.keeps(bin_val<T, DIM>(g, p.x[k], p.y[k], p.m[k], p.my[k], p.s[k]), id + k);
                kt += kp[k];
            }
            const int inc = wave_incl_scan(kt);
            const int tot = __shfl(inc, 63, 64);
            int e = inc - kt;
#pragma unroll
            for (int k = 0; k < IT; ++k) {
                if (!kp[k]) continue;
                sx[e] = p.x[k];
                sm[e] = p.m[k];
                if (DIM == 2) {
                    sy[e] = p.y[k];
                    smy[e] = p.my[k];
                }
                ssg[e] = p.s[k];
                ++e;
            }
            wave_lds_sync();
            for (int i = lane; i < tot; i += 64) {
                const long o = (long)run + i;
                if (o >= capacity) break;  // never taken after the capacity check
                xo[o] = sx[i];
                Mo[o] = (MT)sm[i];
                if (DIM == 2) {
                    yo[o] = sy[i];
                    Myo[o] = (MT)smy[i];
                }
                so[o] = ssg[i];
            }
            wave_lds_sync();  // the stage is rewritten by the next tile
            run += tot;
        }
        return;
    }
    // placing wave v: work items [it, it_hi) of the ones dealt out evenly by annih_scan, an
    // item being one piece of at most PIECE slots of one bin chunk.  The wave walks the bin
    // workgroups from its first item's on, 64 chunks at a time (wave scans of their counts and
    // item counts), and places each of its items on its own.
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long v = ((long)blockIdx.x - part_blocks) * WPB + wv;
    const long long n_items = w.sc[SC_ITEMS];
    const long long npw = (long long)place_blocks * WPB;
    const long long per = (n_items + npw - 1) / npw;
    long long it = min(n_items, (long long)v * per);
    const long long it_hi = min(n_items, it + per);
    if (it >= it_hi) return;
    int* wl = reinterpret_cast<int*>(smem) + wv * PW_LDS;
    long last_ch = -1;
    for (int c = w.wstart[v]; c < PB && it < it_hi;) {  // uniform per wave
        long long ib = c ? w.ipre[c - 1] : 0, sb = c ? w.bpre[c - 1] : 0;
        const long j0 = min(g.n_chunks, (long)c * g.gpb), j1 = min(g.n_chunks, j0 + g.gpb);
        for (long g0 = j0; g0 < j1 && it < it_hi; g0 += 64) {
            const long j = g0 + lane;
            const long long cnt = j < j1 ? (long long)w.csum[j] : 0;
            const long long itm = (cnt + PIECE - 1) / PIECE;
            const long long s_inc = wave_incl_scan_ll(cnt), i_inc = wave_incl_scan_ll(itm);
            const long long i_tot = __shfl(i_inc, 63, 64), s_tot = __shfl(s_inc, 63, 64);
            while (it < it_hi && it < ib + i_tot) {
                const long long rel = it - ib;
                const int l = __builtin_ctzll(__ballot(i_inc > rel));  // the chunk holding item `it`
                const long long i_ex = __shfl(i_inc - itm, l, 64);
                const long long s_ex = __shfl(s_inc - cnt, l, 64);
                const long long cn = __shfl(cnt, l, 64);
                const long ch = g0 + l;
                const long ch_start = (long)(sb + s_ex);
                const long p_lo = ch_start + (long)(rel - i_ex) * PIECE;
                const long p_hi = min(ch_start + (long)cn, p_lo + PIECE);
                place_chunk_wave<T, MT, DIM>(g, bc, mode, c1, tag, ch, ch_start, (long)cn, p_lo, p_hi, xo,
                                             yo, Mo, Myo, so, capacity, wl, ch != last_ch);
                last_ch = ch;
                ++it;
            }
            ib += i_tot;
            sb += s_tot;
        }
        // the next bin workgroup holding item `it` (skipping empty ones): first c' > c with
        // ipre[c'] > it
        int lo = c + 1, hi = PB;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (w.ipre[mid] > it)
                hi = mid;
            else
                lo = mid + 1;
        }
        c = lo;
    }
}

// ----------------------------------------------------------------------------- pair removal
// Rule 2 read literally (sp_annihilate_pairs): in each bin the k-th positive and the k-th
// negative particle (input order) annihilate, k < min(H+, H-).  The particles of mixed bins
// are listed in input order as (key = 2 bin + [s > 0], index), the list is sorted by key
// with a stable LSD radix sort (so each (bin, sign) segment keeps input order), a
// particle's rank is its distance from the start of its segment, and it survives iff its
// rank is at least min(H+, H-).  The survivors of all bins are then compacted in input
// order by the passes of sp_annihilate (nothing is placed).
constexpr int RB = PB;  // workgroups of the radix passes, each owning a contiguous range
constexpr int RBITS = 9;             // digit width of the radix passes
constexpr int RD = 1 << RBITS;       // digits per pass
constexpr int DPT = RD / PT;         // digits per thread in the per-digit loops
static_assert(RD % PT == 0, "digits per thread");

// Caller scratch of sp_annihilate_pairs: int64 sc[16] | int64 woff[NW] | uint32 cnt[RD RB] |
// uint32 off[RD RB] | uint32 dtot[RD] | uint32 dbase[RD] | uint32 keys[2][n_max] |
// uint32 vals[2][n_max] | uint8 flags[n_max].
struct PairScratch {
    long long* sc;     // sc[0]: number of listed particles
    long long* woff;   // per wave of the listing pass: first list slot
    uint32_t* cnt;     // radix digit counts [digit][block]
    uint32_t* off;     // their exclusive prefix within each digit
    uint32_t* dtot;    // per digit: its count over all blocks
    uint32_t* dbase;   // exclusive prefix of dtot
    uint32_t* keys[2];
    uint32_t* vals[2];
    uint8_t* flags;
};

static size_t pair_scratch_bytes(long n_max) {
    return sizeof(long long) * (16 + (size_t)NW) + 2 * sizeof(uint32_t) * RD * ((size_t)RB + 1) +
           4 * sizeof(uint32_t) * (size_t)n_max + (size_t)n_max + 64;
}

static PairScratch pair_carve(void* p, long n_max) {
    PairScratch q;
    q.sc = static_cast<long long*>(p);
    q.woff = q.sc + 16;
    q.cnt = reinterpret_cast<uint32_t*>(q.woff + NW);
    q.off = q.cnt + RD * RB;
    q.dtot = q.off + RD * RB;
    q.dbase = q.dtot + RD;
    q.keys[0] = q.dbase + RD;
    q.keys[1] = q.keys[0] + n_max;
    q.vals[0] = q.keys[1] + n_max;
    q.vals[1] = q.vals[0] + n_max;
    q.flags = reinterpret_cast<uint8_t*>(q.vals[1] + n_max);
    return q;
}

// Listing, pass 1: per wave, the particles of its chunk whose bin holds both signs.
template <typename T, typename MT, int DIM>
__global__ __launch_bounds__(PT) void pair_count(Geo g, const T* x, const T* y, const MT* M,
                                                 const MT* My, const int8_t* s,
                                                 const long long* d_n_in, long long cap_in,
                                                 long long* stats, WS w) {
    __shared__ long long red[PT / 64];
    __shared__ uint32_t lw[KWW];
    __shared__ long wmin[PT / 64];
    if (stats[WK_ST_OVERFLOW] != 0) return;
    const long n = (long)*d_n_in;
    if (n < 0 || n > cap_in) {  // refused: the later passes see the sticky flag and do nothing
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            stats[WK_ST_NEEDED] = -1;
            stats[WK_ST_OVERFLOW] = 1;
        }
        return;
    }
    long lo, hi;
    wave_chunk(n, (long)blockIdx.x * WPB + (threadIdx.x >> 6), &lo, &hi);
    const KeepWindow kw = keep_window(first_bin<T, MT, DIM>(g, x, y, M, My, s, lo, hi), lw, wmin,
                                      w.mixbits, 8 * g.n_chunks, nullptr);
    long long a = 0;
    Raw4<T, MT, DIM> nxt;
    load4r<T, MT, DIM>(x, y, M, My, s, lo + IT * (threadIdx.x & 63), hi, nxt);
    for (long t0 = lo; t0 < hi; t0 += WT) {
        const long id = t0 + IT * (threadIdx.x & 63);
        Part4<T, DIM> p = unpack(nxt);
        load4r<T, MT, DIM>(x, y, M, My, s, id + WT, hi, nxt);
#pragma unroll
        for (int k = 0; k < IT; ++k)
            a += kw.mixed(bin_val<T, DIM>(g, p.x[k], p.y[k], p.m[k], p.my[k], p.s[k])) ? 1 : 0;
    }
    store_counts(w, wave_sum_ll(a), red);
}

// Exclusive prefix of the listing pass's NW wave counts (one workgroup); sc[0] = the total.
__global__ __launch_bounds__(ST_THREADS) void pair_scan(const long long* stats, WS w, PairScratch q) {
    __shared__ long long part[ST_THREADS / 64 + 1];
    if (stats[WK_ST_OVERFLOW] != 0) {
        if (threadIdx.x == 0) q.sc[0] = 0;
        return;
    }
    constexpr int per = NW / ST_THREADS;
    long long loc[per], acc = 0;
    for (int k = 0; k < per; ++k) {
        loc[k] = w.wcnt[threadIdx.x * per + k];
        acc += loc[k];
    }
    const long long inc = wave_incl_scan_ll(acc);
    if ((threadIdx.x & 63) == 63) part[threadIdx.x >> 6] = inc;
    __syncthreads();
    long long run = inc - acc;
    for (int k = 0; k < (int)(threadIdx.x >> 6); ++k) run += part[k];
    for (int k = 0; k < per; ++k) {
        q.woff[threadIdx.x * per + k] = run;
        run += loc[k];
    }
    if (threadIdx.x == ST_THREADS - 1) q.sc[0] = run;
}

// Listing, pass 2: each wave writes its listed particles, in input order, from its offset.
template <typename T, typename MT, int DIM>
__global__ __launch_bounds__(PT) void pair_write(Geo g, const T* x, const T* y, const MT* M,
                                                 const MT* My, const int8_t* s,
                                                 const long long* d_n_in, long long cap_in,
                                                 const long long* stats, WS w, PairScratch q) {
    __shared__ uint32_t lw[KWW];
    __shared__ long wmin[PT / 64];
    if (stats[WK_ST_OVERFLOW] != 0) return;
    const long n = (long)*d_n_in;
    if (n < 0 || n > cap_in) return;
    const int lane = threadIdx.x & 63;
    long lo, hi;
    wave_chunk(n, (long)blockIdx.x * WPB + (threadIdx.x >> 6), &lo, &hi);
    const KeepWindow kw = keep_window(first_bin<T, MT, DIM>(g, x, y, M, My, s, lo, hi), lw, wmin,
                                      w.mixbits, 8 * g.n_chunks, nullptr);
    long long run = q.woff[(long)blockIdx.x * WPB + (threadIdx.x >> 6)];
    Raw4<T, MT, DIM> nxt;
    load4r<T, MT, DIM>(x, y, M, My, s, lo + IT * lane, hi, nxt);
    for (long t0 = lo; t0 < hi; t0 += WT) {
        const long id = t0 + IT * lane;
        Part4<T, DIM> p = unpack(nxt);
        load4r<T, MT, DIM>(x, y, M, My, s, id + WT, hi, nxt);
        // every keep flag starts at 0 (coalesced here); pair_flags sets those of the kept ones
        if (id + IT <= hi) {
            *reinterpret_cast<uchar4*>(q.flags + id) = make_uchar4(0, 0, 0, 0);
        } else {
#pragma unroll
            for (int k = 0; k < IT; ++k)
                if (id + k < hi) q.flags[id + k] = 0;
        }
        long b[IT];
        int c = 0;
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            b[k] = bin_val<T, DIM>(g, p.x[k], p.y[k], p.m[k], p.my[k], p.s[k]);
            if (!kw.mixed(b[k])) b[k] = -1;
            c += b[k] >= 0;
        }
        const int inc = wave_incl_scan(c);
        long long o = run + inc - c;
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            if (b[k] < 0) continue;
            q.keys[0][o] = (uint32_t)(2 * b[k] + (p.s[k] > 0 ? 1 : 0));
            q.vals[0][o] = (uint32_t)(id + k);
            ++o;
        }
        run += __shfl(inc, 63, 64);
    }
}

// The contiguous list range of radix block r: whole tiles of PT elements.
__device__ __forceinline__ void radix_range(long m, long r, long* lo, long* hi) {
    long c = (m + RB - 1) / RB;
    c = (c + PT - 1) / PT * PT;
    *lo = min(m, r * c);
    *hi = min(m, *lo + c);
}

// Radix pass, 1: digit counts of each block's range (LDS counters).
__global__ __launch_bounds__(PT) void radix_hist(const uint32_t* __restrict__ keys, int shift, PairScratch q) {
    __shared__ uint32_t h[RD];
#pragma unroll
    for (int j = 0; j < DPT; ++j) h[threadIdx.x + j * PT] = 0;
    __syncthreads();
    long lo, hi;
    radix_range(q.sc[0], blockIdx.x, &lo, &hi);
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    // one LDS update per distinct digit of a wave's 64 elements (a pass over few distinct
    // digits, like the top bits of the bin, would otherwise serialise on a few counters)
    for (long b0 = lo; b0 < hi; b0 += PT) {  // uniform
        const long e = b0 + threadIdx.x;
        const bool valid = e < hi;
        const uint32_t d = valid ? (keys[e] >> shift) & (uint32_t)(RD - 1) : 0u;
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < RBITS; ++bit) {
            const unsigned long long m = __ballot((d >> bit) & 1u);
            peers &= ((d >> bit) & 1u) ? m : ~m;
        }
        if (valid && (peers & below) == 0) atomicAdd(&h[d], (uint32_t)__popcll(peers));
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < DPT; ++j) q.cnt[(long)(threadIdx.x + j * PT) * RB + blockIdx.x] = h[threadIdx.x + j * PT];
}

// Radix pass, 2a: per digit (one workgroup each), the exclusive prefix of its RB block counts
// and its total.
__global__ __launch_bounds__(PT) void radix_scan_digits(PairScratch q) {
    __shared__ int ldsw[WPB];
    constexpr int per = RB / PT;
    const long base = (long)blockIdx.x * RB + (long)threadIdx.x * per;
    uint32_t loc[per], acc = 0;
#pragma unroll
    for (int k = 0; k < per; ++k) {
        loc[k] = q.cnt[base + k];
        acc += loc[k];
    }
    int tot;
    uint32_t run = (uint32_t)block_excl_scan_pt((int)acc, &tot, ldsw);  // counts < 2^31
#pragma unroll
    for (int k = 0; k < per; ++k) {
        q.off[base + k] = run;
        run += loc[k];
    }
    if (threadIdx.x == 0) q.dtot[blockIdx.x] = (uint32_t)tot;
}

// Radix pass, 2b: exclusive prefix of the RD digit totals (one workgroup; DPT consecutive
// digits per thread).
__global__ __launch_bounds__(PT) void radix_scan_totals(PairScratch q) {
    __shared__ int ldsw[WPB];
    uint32_t v[DPT], acc = 0;
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
        v[j] = q.dtot[threadIdx.x * DPT + j];
        acc += v[j];
    }
    int tot;
    uint32_t run = (uint32_t)block_excl_scan_pt((int)acc, &tot, ldsw);
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
        q.dbase[threadIdx.x * DPT + j] = run;
        run += v[j];
    }
}

// Radix pass, 3: stable scatter.  Block r walks its range in batches of RS_TILES tiles of PT
// elements (element b0 + k PT + thread of tile k).  An element's rank among the batch's
// elements of its digit is the tiles before it (running per-digit counts) plus the earlier
// elements of its own tile (the lanes of its wave with that digit, found with RBITS ballots,
// and the counts of the earlier waves).  The batch is then staged in LDS sorted by digit and
// written out in that order, so that consecutive threads fill consecutive slots of each
// digit's run (about RS_TILES elements per digit) instead of one scattered slot each.
constexpr int RS_TILES = 16;

__global__ __launch_bounds__(PT) void radix_scatter(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                    uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                    int shift, PairScratch q) {
    constexpr int NB = RS_TILES * PT;
    constexpr uint32_t DM = RD - 1;
    __shared__ uint32_t run[RD];      // next output slot of each digit
    __shared__ uint32_t bcnt[RD];     // the batch's running count of each digit
    __shared__ uint32_t boff[RD];     // exclusive prefix of the batch counts
    __shared__ uint32_t cw[WPB][RD];  // per wave: its count of each digit in the current tile
    __shared__ int ldsw[WPB];
    __shared__ uint32_t sk[NB], sv[NB];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
        const int dd = threadIdx.x + j * PT;
        run[dd] = q.dbase[dd] + q.off[(long)dd * RB + blockIdx.x];
#pragma unroll
        for (int k = 0; k < WPB; ++k) cw[k][dd] = 0;
    }
    long lo, hi;
    radix_range(q.sc[0], blockIdx.x, &lo, &hi);
    const unsigned long long below = (1ull << lane) - 1ull;
    for (long b0 = lo; b0 < hi; b0 += NB) {  // uniform
#pragma unroll
        for (int j = 0; j < DPT; ++j) bcnt[threadIdx.x + j * PT] = 0;
        uint32_t key[RS_TILES], val[RS_TILES], rk[RS_TILES];
#pragma unroll
        for (int k = 0; k < RS_TILES; ++k) {
            const long e = b0 + (long)k * PT + threadIdx.x;
            key[k] = e < hi ? kin[e] : 0u;
            val[k] = e < hi ? vin[e] : 0u;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < RS_TILES; ++k) {
            const bool valid = b0 + (long)k * PT + threadIdx.x < hi;
            const uint32_t d = (key[k] >> shift) & DM;
            unsigned long long peers = __ballot(valid);
#pragma unroll
            for (int bit = 0; bit < RBITS; ++bit) {
                const unsigned long long m = __ballot((d >> bit) & 1u);
                peers &= ((d >> bit) & 1u) ? m : ~m;
            }
            const int lower = __popcll(peers & below);
            if (valid && lower == 0) cw[wv][d] = (uint32_t)__popcll(peers);
            __syncthreads();
            rk[k] = 0;
            if (valid) {
                uint32_t r = bcnt[d] + (uint32_t)lower;
                for (int w = 0; w < wv; ++w) r += cw[w][d];
                rk[k] = r;
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < DPT; ++j) {
                const int dd = threadIdx.x + j * PT;
                uint32_t t = 0;
#pragma unroll
                for (int w = 0; w < WPB; ++w) {
                    t += cw[w][dd];
                    cw[w][dd] = 0;
                }
                bcnt[dd] += t;
            }
            __syncthreads();
        }
        {  // exclusive prefix of the batch counts, DPT consecutive digits per thread
            uint32_t v[DPT], acc = 0;
#pragma unroll
            for (int j = 0; j < DPT; ++j) {
                v[j] = bcnt[threadIdx.x * DPT + j];
                acc += v[j];
            }
            int tot;
            uint32_t r = (uint32_t)block_excl_scan_pt((int)acc, &tot, ldsw);
#pragma unroll
            for (int j = 0; j < DPT; ++j) {
                boff[threadIdx.x * DPT + j] = r;
                r += v[j];
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < RS_TILES; ++k) {
            if (b0 + (long)k * PT + threadIdx.x < hi) {
                const uint32_t pl = boff[(key[k] >> shift) & DM] + rk[k];
                sk[pl] = key[k];
                sv[pl] = val[k];
            }
        }
        __syncthreads();
        const int nb = (int)min((long)NB, hi - b0);
        for (int i = threadIdx.x; i < nb; i += PT) {
            const uint32_t kk = sk[i], d = (kk >> shift) & DM;
            const uint32_t pos = run[d] + (uint32_t)i - boff[d];
            kout[pos] = kk;
            vout[pos] = sv[i];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < DPT; ++j) run[threadIdx.x + j * PT] += bcnt[threadIdx.x + j * PT];
        __syncthreads();
    }
}

// Ranks and flags: position p of the sorted list holds key k; its rank is p minus the first
// position of k (a running maximum of the segment heads, started from a binary search at the
// wave's first position); a particle is kept when rank >= min(H+, H-) of its bin.  Only the
// kept ones are written (flags[index] = 1): pair_write has set every flag to 0, and far fewer
// particles survive a mixed bin than are listed, so most scattered byte writes are saved.
__global__ __launch_bounds__(PT) void pair_flags(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ vals,
                                                 const int32_t* __restrict__ hist, long n_bins, PairScratch q) {
    const int lane = threadIdx.x & 63;
    const long m = q.sc[0];
    long lo, hi;
    wave_chunk(m, (long)blockIdx.x * WPB + (threadIdx.x >> 6), &lo, &hi);
    if (lo >= hi) return;
    long start;  // first position of the key at lo
    {
        const uint32_t k0 = keys[lo];
        long a = 0, b = lo;
        while (a < b) {
            const long mid = (a + b) >> 1;
            if (keys[mid] < k0)
                a = mid + 1;
            else
                b = mid;
        }
        start = a;
    }
    for (long t0 = lo; t0 < hi; t0 += 64) {
        const long p = t0 + lane;
        const bool valid = p < hi;
        const uint32_t k = valid ? keys[p] : 0u;
        const bool head = valid && (p == 0 || keys[p - 1] != k);
        long hs = head ? p : -1;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const long t = __shfl_up(hs, o, 64);
            if (lane >= o) hs = max(hs, t);
        }
        const long st = max(start, hs);
        if (valid) {
            const long bin = (long)(k >> 1);
            const int hp = hist[bin], hm = hist[n_bins + bin];
            const long pairs = hp < hm ? hp : hm;
            if (p - st >= pairs) q.flags[vals[p]] = 1;
        }
        start = __shfl(st, 63, 64);
    }
}

// Chunk owners of the annihilation's particle passes: as for sp_step, twice as many on large
// buffers (the per-workgroup prologue amortised, the last residency round shorter).
static int annih_owners(const sp_particles* in) {
    return in->capacity >= SB_LARGE ? SB_MAX : PB;
}

// The counting pass's keep bits (one per input slot, in whole 256-particle tiles) go to the
// end of out->x, past every position the output can occupy when the output is short enough;
// annih_scan checks that against the output count and the writing pass uses them only then.
template <typename T>
static void keep_bits_region(const sp_particles* in, const sp_particles* out, uint32_t** kbits,
                             long long* kb_limit) {
    const size_t bytes = (size_t)((in->capacity + 255) / 256) * 8 * sizeof(uint32_t);
    const size_t end = (size_t)out->capacity * sizeof(T);
    if (bytes + 256 > end) {
        *kbits = nullptr;
        *kb_limit = -1;
        return;
    }
    const size_t off = (end - bytes) & ~(size_t)255;
    *kbits = reinterpret_cast<uint32_t*>(static_cast<char*>(out->x) + off);
    *kb_limit = (long long)(off / sizeof(T));
}

template <typename T, typename MT, int DIM>
static void launch_pairs(const Geo& g, const sp_particles* in, sp_particles* out, int32_t* hist,
                         int hist_ready, long long* stats, WS w, PairScratch q, int passes, hipStream_t s) {
    const T* x = static_cast<const T*>(in->x);
    const T* y = static_cast<const T*>(in->y);
    const MT* M = static_cast<const MT*>(in->M);
    const MT* My = static_cast<const MT*>(in->My);
    const long long* d_n = reinterpret_cast<const long long*>(in->d_n);
    const long long cap_in = (long long)in->capacity;
    if (!hist_ready) {
        WK_LAUNCH("hist_clear", fill_i32, dim3(1024), dim3(256), 0, s, hist, 2 * g.n_bins, 0);
        if (DIM == 2) {
            WK_LAUNCH("map_clear", fill_i32, dim3(BMW / 256), dim3(256), 0, s,
                      reinterpret_cast<int32_t*>(w.blkmap), (long)BMW, 0);
        }
        WK_LAUNCH("annih_hist", (annih_hist<T, MT, DIM>), dim3(PB), dim3(PT), 0, s, g, x, y, M, My,
                  in->s, d_n, cap_in, hist, w.blkmap, stats);
    }
    // the block map is valid when this call or the sp_step before it built the histogram (the
    // 2-D builders mark it; a 1-D histogram is small enough to read whole)
    const uint32_t* marked = hist_ready == 1 || DIM == 1 ? nullptr : w.blkmap;
    const BinCount bc{nullptr, hist, g.n_bins};
    WK_LAUNCH("annih_bins", annih_bins, dim3(PB), dim3(PT), 0, s, g, bc, 0, stats, w, marked);
    WK_LAUNCH("pair_count", (pair_count<T, MT, DIM>), dim3(PB), dim3(PT), 0, s, g, x, y, M, My, in->s,
              d_n, cap_in, stats, w);
    WK_LAUNCH("pair_scan", pair_scan, dim3(1), dim3(ST_THREADS), 0, s, stats, w, q);
    WK_LAUNCH("pair_write", (pair_write<T, MT, DIM>), dim3(PB), dim3(PT), 0, s, g, x, y, M, My, in->s,
              d_n, cap_in, stats, w, q);
    for (int k = 0; k < passes; ++k) {
        const int src = k & 1;
        WK_LAUNCH("radix_hist", radix_hist, dim3(RB), dim3(PT), 0, s, q.keys[src], RBITS * k, q);
        WK_LAUNCH("radix_scan", radix_scan_digits, dim3(RD), dim3(PT), 0, s, q);
        WK_LAUNCH("radix_totals", radix_scan_totals, dim3(1), dim3(PT), 0, s, q);
        WK_LAUNCH("radix_scatter", radix_scatter, dim3(RB), dim3(PT), 0, s, q.keys[src], q.vals[src],
                  q.keys[src ^ 1], q.vals[src ^ 1], RBITS * k, q);
    }
    WK_LAUNCH("pair_flags", pair_flags, dim3(PB), dim3(PT), 0, s, q.keys[passes & 1], q.vals[passes & 1], hist,
              g.n_bins, q);
    uint32_t* kbits;
    long long kb_limit;
    keep_bits_region<T>(in, out, &kbits, &kb_limit);
    const int own = annih_owners(in);
    WK_LAUNCH("annih_count", (annih_count<T, MT, DIM>), dim3(own), dim3(PT), 0, s, g, x, y, M, My, in->s,
              d_n, cap_in, (const uint8_t*)q.flags, kbits, (const uint32_t*)nullptr, stats, w);
    WK_LAUNCH("annih_scan", annih_scan, dim3(1), dim3(ST_THREADS), 0, s, 1, PLACE_BLOCKS, d_n,
              reinterpret_cast<long long*>(out->d_n), (long long)out->capacity, kb_limit, own, stats, w);
    WK_LAUNCH("annih_write", (annih_write<T, MT, DIM>), dim3(own + PLACE_BLOCKS), dim3(PT), 0, s, g,
              own, PLACE_BLOCKS, bc, 1, 0u, (uint32_t)TAG_ANNIH, x, y, M, My, in->s, d_n,
              static_cast<T*>(out->x), static_cast<T*>(out->y), static_cast<MT*>(out->M),
              static_cast<MT*>(out->My), out->s, (long long)out->capacity, (const uint8_t*)q.flags,
              (const uint32_t*)kbits, w);
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
                                long n_bins, const uint32_t* __restrict__ marked, int bshift,
                                uint8_t* __restrict__ occ) {
    const long c = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (c >= n_cells) return;
    if (marked != nullptr) {  // no marked block under the cell: its bins are all zero
        bool any = false;
        for (long k = (c * per_cell) >> bshift; k <= ((c + 1) * per_cell - 1) >> bshift && !any; ++k)
            any = ((marked[k >> 5] >> (k & 31)) & 1u) != 0u;
        if (!any) {
            if (lane == 0) occ[c] = 0;
            return;
        }
    }
    int o = 0;
    for (long k = lane; k < per_cell; k += 64) {
        const long b = c * per_cell + k;
        o |= (hist[b] | hist[n_bins + b]) != 0;
    }
    const unsigned long long any = __ballot(o);
    if (lane == 0) occ[c] = any != 0ull;
}

// Cells without a table row that lie within `margin` cells (per axis) of an occupied cell.
// The box test is separable: dilate the occupancy along x, then along y (one thread per cell
// each), then one workgroup compacts the flagged cells in ascending order (deterministic).
__global__ void dilate_x_kernel(const uint8_t* __restrict__ occ, int nx, long n_cells, int margin,
                                uint8_t* __restrict__ occx) {
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    const int cx = (int)(c % nx);
    const uint8_t* row = occ + (c - cx);
    int o = 0;
    for (int xx = max(cx - margin, 0); xx <= min(cx + margin, nx - 1) && !o; ++xx) o = row[xx];
    occx[c] = o != 0;
}

__global__ void need_kernel(const uint8_t* __restrict__ occx, int dim, int nx, int ny, int margin,
                            const int32_t* __restrict__ cell_slot, uint8_t* __restrict__ need) {
    const long n_cells = (long)nx * ny;
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    int o = 0;
    if (cell_slot[c] < 0) {
        const int cx = (int)(c % nx), cy = (int)(c / nx);
        const int y0 = dim == 2 ? max(cy - margin, 0) : 0, y1 = dim == 2 ? min(cy + margin, ny - 1) : 0;
        for (int yy = y0; yy <= y1 && !o; ++yy) o = occx[(long)yy * nx + cx];
    }
    need[c] = o != 0;
}

__global__ __launch_bounds__(1024) void cells_needed_kernel(const uint8_t* __restrict__ need,
                                                           long n_cells,
                                                           int32_t* __restrict__ new_cells,
                                                           long long* __restrict__ d_count) {
    __shared__ int wsum[16];
    const long per = (n_cells + 1023) / 1024;
    const long lo = min(n_cells, (long)threadIdx.x * per), hi = min(n_cells, lo + per);
    int cnt = 0;
    for (long c = lo; c < hi; ++c) cnt += need[c];
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
        if (need[c]) new_cells[o++] = (int32_t)c;
    if (threadIdx.x == 0) *d_count = total;
}

__global__ void assign_slots_kernel(const int32_t* __restrict__ new_cells,
                                    const long long* __restrict__ d_count, int32_t first_row,
                                    int32_t* __restrict__ cell_slot) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < *d_count) cell_slot[new_cells[k]] = first_row + (int32_t)k;
}

// ----------------------------------------------------------------------------- host side
// Bytes per stored momentum index (sp_geom.m_bytes, 0 = the default for the dimension).
static int m_bytes_of(const sp_geom* gm) {
    return gm->m_bytes ? gm->m_bytes : (gm->dim == 1 ? 4 : 2);
}

static int make_geo(const sp_geom* gm, Geo* g) {
    WK_REQUIRE(gm != nullptr, "particles: geometry is NULL");
    WK_REQUIRE(gm->dim == 1 || gm->dim == 2, "particles: dim must be 1 or 2");
    WK_REQUIRE(gm->nx > 0 && gm->ny > 0 && (gm->dim == 2 || gm->ny == 1), "particles: bad mesh");
    WK_REQUIRE(gm->n_m >= 2 && gm->n_m % 2 == 0, "particles: n_m must be even");
    WK_REQUIRE(gm->n_k > 0, "particles: n_k must be positive");
    const int mb = m_bytes_of(gm);
    WK_REQUIRE(mb == 1 || mb == 2 || (mb == 4 && gm->dim == 1),
               "particles: m_bytes must be 0, 1, 2 or (1-D) 4");
    {
        // stored momenta: the window and the children's offsets of up to n_m/2 either way
        const long lo = (long)gm->M_min - gm->n_m / 2, hi = (long)gm->M_min + gm->n_k - 1 + gm->n_m / 2;
        const long tmin = mb == 1 ? -128 : (mb == 2 ? -32768 : INT_MIN);
        const long tmax = mb == 1 ? 127 : (mb == 2 ? 32767 : INT_MAX);
        WK_REQUIRE(lo >= tmin && hi <= tmax, "particles: the momentum window (widened by n_m/2) "
                                             "does not fit the momentum type (m_bytes)");
    }
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
    g->n_chunks = n_chunks_for(g->n_bins);
    g->gpb = (g->n_chunks + PB - 1) / PB;
    g->bshift = __builtin_ctz(BC);
    while (((g->n_bins + (1L << g->bshift) - 1) >> g->bshift) > 32L * BMW) ++g->bshift;
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
                        const uint32_t* thr, const uint64_t* cdf, const uint32_t* guide,
                        int guide_len, const sp_particles* in, sp_particles* out, int32_t* hist,
                        int hist_mode, uint32_t* keys, long long* stats, long long st, WS w,
                        hipStream_t s) {
    const long long* d_n_in = reinterpret_cast<const long long*>(in->d_n);
    long long* d_n_out = reinterpret_cast<long long*>(out->d_n);
    const long long cap = (long long)out->capacity;
    const T* x = static_cast<const T*>(in->x);
    const T* y = static_cast<const T*>(in->y);
    const MT* M = static_cast<const MT*>(in->M);
    const MT* My = static_cast<const MT*>(in->My);
    T* xo = static_cast<T*>(out->x);
    T* yo = static_cast<T*>(out->y);
    MT* Mo = static_cast<MT*>(out->M);
    MT* Myo = static_cast<MT*>(out->My);
    const long n_cells = (long)g.nx * g.ny;
    if (n_cells > CT_MAX)
        WK_LAUNCH("cell_table", cell_table_kernel, dim3((unsigned)((n_cells + 255) / 256)), dim3(256), 0, s,
                  n_cells, cs, n0, thr, w.ctab);
    const unsigned sb = cap >= SB_LARGE ? SB_MAX : PB;  // chunk owners of both passes
    WK_LAUNCH("step_count", (step_count<T, MT, DIM>), dim3(sb), dim3(PT), 0, s, g, step, cs, n0, thr,
              x, y, M, My, in->s, d_n_in, (long long)in->capacity, xo, out->s, cap, hist, hist_mode,
              stats, st, w);
    if (hist)
        WK_LAUNCH("step_apply", (step_apply<T, MT, DIM, true>), dim3(sb), dim3(PT), 0, s, g, step, cs,
                  n0, thr, cdf, guide, guide_len, x, y, M, My, in->s, d_n_in, xo, yo, Mo, Myo,
                  out->s, d_n_out, cap, hist, keys, stats, st, w);
    else
        WK_LAUNCH("step_apply", (step_apply<T, MT, DIM, false>), dim3(sb), dim3(PT), 0, s, g, step, cs,
                  n0, thr, cdf, guide, guide_len, x, y, M, My, in->s, d_n_in, xo, yo, Mo, Myo,
                  out->s, d_n_out, cap, hist, (uint32_t*)nullptr, stats, st, w);
}

template <typename T, typename MT, int DIM>
static void launch_annih(const Geo& g, uint32_t step, const sp_particles* in, sp_particles* out,
                         int32_t* hist, int hist_ready, const uint32_t* keys, long long* stats, WS w,
                         hipStream_t s) {
    const T* x = static_cast<const T*>(in->x);
    const T* y = static_cast<const T*>(in->y);
    const MT* M = static_cast<const MT*>(in->M);
    const MT* My = static_cast<const MT*>(in->My);
    const long long* d_n = reinterpret_cast<const long long*>(in->d_n);
    const long long cap_in = (long long)in->capacity;
    if (!hist_ready) {
        WK_LAUNCH("hist_clear", fill_i32, dim3(1024), dim3(256), 0, s, hist, 2 * g.n_bins, 0);
        if (DIM == 2) {
            WK_LAUNCH("map_clear", fill_i32, dim3(BMW / 256), dim3(256), 0, s,
                      reinterpret_cast<int32_t*>(w.blkmap), (long)BMW, 0);
        }
        WK_LAUNCH("annih_hist", (annih_hist<T, MT, DIM>), dim3(PB), dim3(PT), 0, s, g, x, y, M, My,
                  in->s, d_n, cap_in, hist, w.blkmap, stats);
    }
    // the block map is valid when this call or the sp_step before it built the histogram (the
    // 2-D builders mark it; a 1-D histogram is small enough to read whole)
    const uint32_t* marked = hist_ready == 1 || DIM == 1 ? nullptr : w.blkmap;
    const BinCount bc{nullptr, hist, g.n_bins};
    long long* d_n_out = reinterpret_cast<long long*>(out->d_n);
    WK_LAUNCH("annih_bins", annih_bins, dim3(PB), dim3(PT), 0, s, g, bc, 1, stats, w, marked);
    uint32_t* kbits;
    long long kb_limit;
    keep_bits_region<T>(in, out, &kbits, &kb_limit);
    const int own = annih_owners(in);
    WK_LAUNCH("annih_count", (annih_count<T, MT, DIM>), dim3(own), dim3(PT), 0, s, g, x, y, M, My, in->s,
              d_n, cap_in, (const uint8_t*)nullptr, kbits, keys, stats, w);
    WK_LAUNCH("annih_scan", annih_scan, dim3(1), dim3(ST_THREADS), 0, s, 1, PLACE_BLOCKS, d_n,
              d_n_out, (long long)out->capacity, kb_limit, own, stats, w);
    WK_LAUNCH("annih_write", (annih_write<T, MT, DIM>), dim3(own + PLACE_BLOCKS), dim3(PT), 0, s, g,
              own, PLACE_BLOCKS, bc, 1, step, (uint32_t)TAG_ANNIH, x, y, M, My, in->s, d_n,
              static_cast<T*>(out->x), static_cast<T*>(out->y), static_cast<MT*>(out->M),
              static_cast<MT*>(out->My), out->s, (long long)out->capacity, (const uint8_t*)nullptr,
              (const uint32_t*)kbits, w);
}

template <typename T, typename MT, int DIM>
static void launch_init(const Geo& g, const int32_t* counts, sp_particles* out, long long* stats,
                        WS w, hipStream_t s) {
    const BinCount bc{counts, nullptr, g.n_bins};
    WK_LAUNCH("init_count", annih_bins, dim3(PB), dim3(PT), 0, s, g, bc, 1, stats, w,
              (const uint32_t*)nullptr);
    WK_LAUNCH("init_scan", annih_scan, dim3(1), dim3(ST_THREADS), 0, s, 0, PLACE_BLOCKS,
              (const long long*)nullptr, reinterpret_cast<long long*>(out->d_n),
              (long long)out->capacity, -1LL, PB, stats, w);
    WK_LAUNCH("init_write", (annih_write<T, MT, DIM>), dim3(PLACE_BLOCKS), dim3(PT), 0, s, g, 0,
              PLACE_BLOCKS, bc, 0, 0xFFFFFFFFu, (uint32_t)TAG_INIT, (const T*)nullptr,
              (const T*)nullptr, (const MT*)nullptr, (const MT*)nullptr, (const int8_t*)nullptr,
              (const long long*)nullptr, static_cast<T*>(out->x), static_cast<T*>(out->y),
              static_cast<MT*>(out->M), static_cast<MT*>(out->My), out->s,
              (long long)out->capacity, (const uint8_t*)nullptr, (const uint32_t*)nullptr, w);
}

}  // namespace wk

using namespace wk;

extern "C" size_t sp_workspace_size(const sp_geom* gm) {
    Geo g;
    if (make_geo(gm, &g) != WK_OK) return 0;
    return ws_bytes_for(g.n_bins, (long)g.nx * g.ny);
}

#define WK_DISPATCH_POS(gm, FN, MT, D, ...)                                          \
    do {                                                                             \
        if ((gm)->pos_f64)                                                           \
            FN<double, MT, D>(__VA_ARGS__);                                          \
        else                                                                         \
            FN<float, MT, D>(__VA_ARGS__);                                           \
    } while (0)

// make_geo has accepted gm (dimension and momentum width are consistent)
#define WK_DISPATCH(gm, FN, ...)                                                      \
    do {                                                                             \
        const int mb_ = m_bytes_of(gm);                                              \
        if ((gm)->dim == 1) {                                                        \
            if (mb_ == 4)                                                            \
                WK_DISPATCH_POS(gm, FN, int32_t, 1, __VA_ARGS__);                    \
            else if (mb_ == 2)                                                       \
                WK_DISPATCH_POS(gm, FN, int16_t, 1, __VA_ARGS__);                    \
            else                                                                     \
                WK_DISPATCH_POS(gm, FN, int8_t, 1, __VA_ARGS__);                     \
        } else {                                                                     \
            if (mb_ == 2)                                                            \
                WK_DISPATCH_POS(gm, FN, int16_t, 2, __VA_ARGS__);                    \
            else                                                                     \
                WK_DISPATCH_POS(gm, FN, int8_t, 2, __VA_ARGS__);                     \
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
    WK_REQUIRE(ws && ws_bytes >= ws_bytes_for(g.n_bins, (long)g.nx * g.ny), "sp_init: workspace too small");
    WS w = carve(ws, g.n_bins, (long)g.nx * g.ny);
    WK_DISPATCH(gm, launch_init, g, bin_counts, out, reinterpret_cast<long long*>(d_stats), w,
                as_stream(stream));
    return check_launch("sp_init");
}

extern "C" int sp_step(const sp_geom* gm, const int32_t* cell_slot, const uint32_t* n0,
                       const uint32_t* thr, const uint64_t* cdf, const uint32_t* guide,
                       int32_t guide_len, const sp_particles* in, sp_particles* out,
                       int32_t* hist, int32_t hist_mode, uint32_t* keys, int64_t step,
                       int64_t* d_stats, void* ws, size_t ws_bytes, void* stream) {
    Geo g;
    int rc = make_geo(gm, &g);
    if (rc) return rc;
    rc = check_particles(gm, in, "sp_step(in)");
    if (rc) return rc;
    rc = check_particles(gm, out, "sp_step(out)");
    if (rc) return rc;
    WK_REQUIRE(in->x != out->x && in->M != out->M && in->s != out->s && in->d_n != out->d_n,
               "sp_step: in and out must be different buffers");
    WK_REQUIRE(cell_slot && n0 && thr && cdf && d_stats, "sp_step: NULL array");
    WK_REQUIRE(hist_mode == 0 || hist_mode == 1, "sp_step: hist_mode must be 0 or 1");
    WK_REQUIRE(keys == nullptr || hist != nullptr, "sp_step: keys come with the histogram (hist != NULL)");
    WK_REQUIRE(keys == nullptr || (reinterpret_cast<uintptr_t>(keys) & 15) == 0,
               "sp_step: keys must be 16-byte aligned");
    WK_REQUIRE(step >= 0 && step < (1LL << 32), "sp_step: step must fit 32 bits");
    WK_REQUIRE(guide == nullptr || (guide_len >= 1 && guide_len <= (1 << 20)),
               "sp_step: guide_len out of range");
    WK_REQUIRE(ws && ws_bytes >= ws_bytes_for(g.n_bins, (long)g.nx * g.ny), "sp_step: workspace too small");
    WS w = carve(ws, g.n_bins, (long)g.nx * g.ny);
    WK_DISPATCH(gm, launch_step, g, (uint32_t)step, cell_slot, n0, thr, cdf, guide, guide_len, in,
                out, hist, (int)hist_mode, keys, reinterpret_cast<long long*>(d_stats), (long long)step,
                w, as_stream(stream));
    return check_launch("sp_step");
}

extern "C" int sp_annihilate(const sp_geom* gm, const sp_particles* in, sp_particles* out,
                             int32_t* hist, int32_t hist_ready, const uint32_t* keys, int64_t step,
                             int64_t* d_stats, void* ws, size_t ws_bytes, void* stream) {
    Geo g;
    int rc = make_geo(gm, &g);
    if (rc) return rc;
    rc = check_particles(gm, in, "sp_annihilate(in)");
    if (rc) return rc;
    rc = check_particles(gm, out, "sp_annihilate(out)");
    if (rc) return rc;
    WK_REQUIRE(in->x != out->x && in->M != out->M && in->s != out->s && in->d_n != out->d_n,
               "sp_annihilate: in and out must be different buffers");
    WK_REQUIRE(hist && d_stats, "sp_annihilate: NULL array");
    WK_REQUIRE(hist_ready >= 0 && hist_ready <= 2, "sp_annihilate: hist_ready must be 0, 1 or 2");
    WK_REQUIRE(keys == nullptr || (reinterpret_cast<uintptr_t>(keys) & 15) == 0,
               "sp_annihilate: keys must be 16-byte aligned");
    WK_REQUIRE(step >= 0 && step < (1LL << 32), "sp_annihilate: step must fit 32 bits");
    WK_REQUIRE(ws && ws_bytes >= ws_bytes_for(g.n_bins, (long)g.nx * g.ny), "sp_annihilate: workspace too small");
    WS w = carve(ws, g.n_bins, (long)g.nx * g.ny);
    WK_DISPATCH(gm, launch_annih, g, (uint32_t)step, in, out, hist, (int)hist_ready, keys,
                reinterpret_cast<long long*>(d_stats), w, as_stream(stream));
    return check_launch("sp_annihilate");
}

extern "C" size_t sp_pairs_scratch_size(const sp_geom* gm, int64_t n_max) {
    if (!gm || n_max < 0 || n_max >= (1LL << 31)) return 0;
    return pair_scratch_bytes((long)n_max);
}

extern "C" int sp_annihilate_pairs(const sp_geom* gm, const sp_particles* in, sp_particles* out,
                                   int32_t* hist, int32_t hist_ready, int64_t* d_stats, void* ws,
                                   size_t ws_bytes, void* scratch, size_t scratch_bytes, void* stream) {
    Geo g;
    int rc = make_geo(gm, &g);
    if (rc) return rc;
    rc = check_particles(gm, in, "sp_annihilate_pairs(in)");
    if (rc) return rc;
    rc = check_particles(gm, out, "sp_annihilate_pairs(out)");
    if (rc) return rc;
    WK_REQUIRE(in->x != out->x && in->M != out->M && in->s != out->s && in->d_n != out->d_n,
               "sp_annihilate_pairs: in and out must be different buffers");
    WK_REQUIRE(hist && d_stats, "sp_annihilate_pairs: NULL array");
    WK_REQUIRE(hist_ready >= 0 && hist_ready <= 2, "sp_annihilate_pairs: hist_ready must be 0, 1 or 2");
    WK_REQUIRE(2 * g.n_bins < (1L << 32), "sp_annihilate_pairs: too many bins for 32-bit keys");
    WK_REQUIRE(ws && ws_bytes >= ws_bytes_for(g.n_bins, (long)g.nx * g.ny),
               "sp_annihilate_pairs: workspace too small");
    WK_REQUIRE(scratch && scratch_bytes >= pair_scratch_bytes((long)in->capacity),
               "sp_annihilate_pairs: scratch smaller than sp_pairs_scratch_size(g, in->capacity)");
    int bits = 0;
    while ((1L << bits) < 2 * g.n_bins) ++bits;
    const int passes = (bits + RBITS - 1) / RBITS;
    WS w = carve(ws, g.n_bins, (long)g.nx * g.ny);
    const PairScratch q = pair_carve(scratch, (long)in->capacity);
    WK_DISPATCH(gm, launch_pairs, g, in, out, hist, (int)hist_ready,
                reinterpret_cast<long long*>(d_stats), w, q, passes, as_stream(stream));
    return check_launch("sp_annihilate_pairs");
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

extern "C" int sp_cells_to_evaluate(const sp_geom* gm, const int32_t* hist, int32_t hist_mode,
                                    int32_t margin, const int32_t* cell_slot, int32_t* new_cells,
                                    int64_t* d_count, void* ws, size_t ws_bytes, void* stream) {
    Geo g;
    int rc = make_geo(gm, &g);
    if (rc) return rc;
    WK_REQUIRE(hist && cell_slot && new_cells && d_count, "sp_cells_to_evaluate: NULL array");
    WK_REQUIRE(margin >= 0, "sp_cells_to_evaluate: negative margin");
    WK_REQUIRE(hist_mode == 0 || hist_mode == 1, "sp_cells_to_evaluate: hist_mode must be 0 or 1");
    WK_REQUIRE(ws && ws_bytes >= ws_bytes_for(g.n_bins, (long)g.nx * g.ny), "sp_cells_to_evaluate: workspace too small");
    const long n_cells = (long)g.nx * g.ny;
    const WS w = carve(ws, g.n_bins, (long)g.nx * g.ny);
    uint8_t* occ = w.occ;  // [n_cells] occupancy, then [n_cells] x-dilation
    uint8_t* occx = occ + n_cells;
    hipStream_t s = as_stream(stream);
    const dim3 cg((unsigned)((n_cells + 255) / 256));
    hipLaunchKernelGGL(occupied_kernel, dim3((unsigned)((n_cells * 64 + 255) / 256)), dim3(256), 0, s,
                       hist, n_cells, g.n_bins / n_cells, g.n_bins,
                       (const uint32_t*)(hist_mode == 1 && g.dim == 2 ? w.blkmap : nullptr), g.bshift, occ);
    hipLaunchKernelGGL(dilate_x_kernel, cg, dim3(256), 0, s, occ, g.nx, n_cells, margin, occx);
    hipLaunchKernelGGL(need_kernel, cg, dim3(256), 0, s, occx, g.dim, g.nx, g.ny, margin, cell_slot, occ);
    hipLaunchKernelGGL(cells_needed_kernel, dim3(1), dim3(1024), 0, s, occ, n_cells, new_cells,
                       reinterpret_cast<long long*>(d_count));
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
