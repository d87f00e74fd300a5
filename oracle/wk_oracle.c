/*
 * wk_oracle.c -- plain, slow, single-threaded CPU reference for the signed
 * particle Wigner Monte Carlo hot path of arXiv:1806.00082 (Sellier,
 * Leygonie, Marceau Caron).  TEST INFRASTRUCTURE ONLY: the product path never
 * includes, links or calls it.  Built with -O2 -ffp-contract=off, no
 * fast-math, so every floating-point operation is the one written here.
 *
 * Pins that tie this file to the paper and to mathematics live in the tests
 * (DST-I identity, Parseval, linear-potential closed form, brute force in
 * high precision, Philox known answers, invariants of the particle passes).
 *
 * Readings of the paper used here:
 *   - Delta p = pi*hbar/L_C (Sec. 2.2, the printed pi/(hbar L_C) has the
 *     wrong dimension); with L_C = n_m dx the argument of the sine in eq.(4)
 *     is 2*pi*j*m/n_m and the prefactor -dx/(hbar L_C) = -1/(hbar n_m).
 *   - V outside the mesh takes the nearest edge value.
 *   - d = 2: the same quadrature per axis with weight 1/2 on the end points
 *     |j_a| = P (the end points are the same point of the periodic grid).
 *   - Creation (postulate II): floor(gamma dt) pairs plus one more with
 *     probability frac(gamma dt); children at the parent's start-of-step
 *     position; then every particle drifts by dt; particles leaving the
 *     domain or the momentum window are absorbed.
 *   - Annihilation (rule 2) on the (cell, momentum) grid: particles in bins
 *     holding only one sign are kept unchanged, each bin holding both signs
 *     is replaced by |net| particles of the net sign, uniform in the cell.
 *     Storage order (a convention; the ensemble is a set): the fresh
 *     particles in ascending bin order first, then the kept ones in input
 *     order.
 */
#include "wk_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define TWO_PI 6.283185307179586476925286766559
#define PI_D 3.14159265358979323846264338327950

/* ---------------------------------------------------------------- Philox */
/* Philox4x32-10 as defined by Salmon, Moraes, Dror and Shaw, "Parallel
 * random numbers: as easy as 1, 2, 3" (SC'11): ten rounds of two 32x32->64
 * multiplications with the round keys bumped by the Weyl constants. */
static void mulhilo32(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo) {
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint32_t hi0, lo0, hi1, lo1;
        mulhilo32(0xD2511F53u, x0, &hi0, &lo0);
        mulhilo32(0xCD9E8D57u, x2, &hi1, &lo1);
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        x0 = y0;
        x1 = lo1;
        x2 = y2;
        x3 = lo0;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

/* Stream tags in the last counter word. */
enum { TAG_CREATE = 1, TAG_ANNIH = 2, TAG_INIT = 3 };

static void draw4(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t tag, uint32_t out[4]) {
    uint32_t ctr[4] = {c0, c1, c2, tag};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    oracle_philox4x32_10(ctr, key, out);
}

/* ---------------------------------------------------------------- kernel */
static double v1(const double* Vb, int nx, long i) {
    if (i < 0) i = 0;
    if (i >= nx) i = nx - 1;
    return Vb[i];
}

static double v2(const double* Vb, int nx, int ny, long ix, long iy) {
    if (ix < 0) ix = 0;
    if (ix >= nx) ix = nx - 1;
    if (iy < 0) iy = 0;
    if (iy >= ny) iy = ny - 1;
    return Vb[iy * (long)nx + ix];
}

static long mod_pos(long a, long n) {
    long r = a % n;
    return r < 0 ? r + n : r;
}

/* sin(2 pi k / n): the integer argument is reduced exactly to the first quarter
 * period with sin(2 pi - a) = -sin a and sin(pi - a) = sin a, so the zeros at
 * k = 0, n/2 and the oddness in k hold exactly. */
static double sin_frac(long k, long n) {
    long t = mod_pos(k, n);
    if (t == 0 || 2 * t == n) return 0.0;
    double sg = 1.0;
    if (2 * t > n) {
        t = n - t;
        sg = -1.0;
    }
    if (4 * t > n) return sg * sin(PI_D * (double)(n - 2 * t) / (double)n);
    return sg * sin(TWO_PI * (double)t / (double)n);
}

/* eq.(4): V_W(i;m) = -dx/(hbar L_C) sum_{j=-P..P} sin(2 pi j m / n_m) [V(i+j)-V(i-j)];
 * the summand is even in j and vanishes at j = 0, so it is 2x the sum over j = 1..P,
 * giving the constant weight -2 dx/(hbar L_C) = -2/(hbar n_m) of Sec. 2.2. */
int oracle_kernel_1d(int nx, int n_m, double hbar, const double* V, int B, const int32_t* cells,
                     int n_cells, double* K) {
    if (nx <= 0 || n_m <= 0 || (n_m & 1) || B < 0 || n_cells < 0 || hbar <= 0) return -1;
    const int P = n_m / 2;
    const double c = -2.0 / (hbar * (double)n_m);
    for (int b = 0; b < B; ++b) {
        const double* Vb = V + (long)b * nx;
        for (int r = 0; r < n_cells; ++r) {
            const long i = cells ? cells[r] : r;
            if (i < 0 || i >= nx) return -1;
            double* row = K + ((long)b * n_cells + r) * n_m;
            for (int t = 0; t < n_m; ++t) {
                const long m = t - P;
                double acc = 0.0;
                for (long j = 1; j <= P; ++j) {
                    const double d = v1(Vb, nx, i + j) - v1(Vb, nx, i - j);
                    acc += sin_frac(j * m, n_m) * d;
                }
                row[t] = c * acc;
            }
        }
    }
    return 0;
}

/* eq.(4) term by term, offsets -P..P inclusive, prefactor -1/(hbar n_m). */
int oracle_kernel_1d_literal(int nx, int n_m, double hbar, const double* V, int B,
                             const int32_t* cells, int n_cells, double* K) {
    if (nx <= 0 || n_m <= 0 || (n_m & 1) || B < 0 || n_cells < 0 || hbar <= 0) return -1;
    const int P = n_m / 2;
    const double pref = -1.0 / (hbar * (double)n_m);
    for (int b = 0; b < B; ++b) {
        const double* Vb = V + (long)b * nx;
        for (int r = 0; r < n_cells; ++r) {
            const long i = cells ? cells[r] : r;
            if (i < 0 || i >= nx) return -1;
            double* row = K + ((long)b * n_cells + r) * n_m;
            for (int t = 0; t < n_m; ++t) {
                const long m = t - P;
                double acc = 0.0;
                for (long j = -P; j <= P; ++j)
                    acc += sin_frac(j * m, n_m) * (v1(Vb, nx, i + j) - v1(Vb, nx, i - j));
                row[t] = pref * acc;
            }
        }
    }
    return 0;
}

/* d = 2: V_W(i;m) = -(dx^2/(hbar L_C^2)) sum_{j in [-P,P]^2} w_j sin(2 pi m.j / n_m)
 * [V(i+j) - V(i-j)], w_j = prod_a (1/2 if |j_a| = P else 1). */
int oracle_kernel_2d(int nx, int ny, int n_m, double hbar, const double* V, int B,
                     const int32_t* cells, int n_cells, double* K) {
    if (nx <= 0 || ny <= 0 || n_m <= 0 || (n_m & 1) || B < 0 || n_cells < 0 || hbar <= 0) return -1;
    const int P = n_m / 2;
    const double pref = -1.0 / (hbar * (double)n_m * (double)n_m);
    const long ncell = (long)nx * ny;
    for (int b = 0; b < B; ++b) {
        const double* Vb = V + (long)b * ncell;
        for (int r = 0; r < n_cells; ++r) {
            const long cid = cells ? cells[r] : r;
            if (cid < 0 || cid >= ncell) return -1;
            const long ix = cid % nx, iy = cid / nx;
            double* row = K + ((long)b * n_cells + r) * (long)n_m * n_m;
            for (int ty = 0; ty < n_m; ++ty) {
                for (int tx = 0; tx < n_m; ++tx) {
                    const long mx = tx - P, my = ty - P;
                    double acc = 0.0;
                    for (long jy = -P; jy <= P; ++jy) {
                        const double wy = (jy == -P || jy == P) ? 0.5 : 1.0;
                        for (long jx = -P; jx <= P; ++jx) {
                            const double wx = (jx == -P || jx == P) ? 0.5 : 1.0;
                            const double d = v2(Vb, nx, ny, ix + jx, iy + jy) -
                                             v2(Vb, nx, ny, ix - jx, iy - jy);
                            acc += (wx * wy) * sin_frac(mx * jx + my * jy, n_m) * d;
                        }
                    }
                    row[(long)ty * n_m + tx] = pref * acc;
                }
            }
        }
    }
    return 0;
}

/* Adjoint of the 1-D map V -> half table K[b][i][t] (m = t+1), all cells:
 * K = c sum_j sin(2 pi j m/n_m) (V[cl(i+j)] - V[cl(i-j)]) is linear in V. */
int oracle_kernel_bwd_1d(int nx, int n_m, double hbar, const double* G, int B,
                         const int32_t* cells, int n_cells, double* dV) {
    if (nx <= 0 || n_m <= 0 || (n_m & 1) || B < 0 || n_cells < 0 || hbar <= 0) return -1;
    if (!cells && n_cells != nx) return -1;
    const int P = n_m / 2;
    const double c = -2.0 / (hbar * (double)n_m);
    for (int b = 0; b < B; ++b) {
        double* dVb = dV + (long)b * nx;
        for (long r = 0; r < n_cells; ++r) {
            const long i = cells ? cells[r] : r;
            if (i < 0 || i >= nx) return -1;
            const double* g = G + ((long)b * n_cells + r) * P;
            for (long j = 1; j <= P; ++j) {
                double gd = 0.0;
                for (long t = 0; t < P; ++t) gd += g[t] * sin_frac(j * (t + 1), n_m);
                gd = c * gd;
                long lp = i + j, lm = i - j;
                if (lp >= nx) lp = nx - 1;
                if (lm < 0) lm = 0;
                dVb[lp] += gd;
                dVb[lm] -= gd;
            }
        }
    }
    return 0;
}

/* ---------------------------------------------------------------- tables */
/* gamma = sum of the positive part of the row in ascending m (eq.(1)),
 * p = gamma dt, n0 = floor(p), thr = floor(frac(p) 2^32); cdf[t] =
 * floor(C[t]/gamma 2^32) with C the running positive sum, and 2^32 from the
 * last positive entry on, so that min{t : u < cdf[t]} samples K+/gamma. */
int oracle_gamma_tables(int width, const double* K, int n_rows, double dt, double* gamma,
                        uint32_t* n0, uint32_t* thr, uint64_t* cdf) {
    if (width <= 0 || n_rows < 0 || !(dt >= 0)) return -1;
    for (int r = 0; r < n_rows; ++r) {
        const double* k = K + (long)r * width;
        double g = 0.0;
        int last = -1;
        for (int t = 0; t < width; ++t) {
            if (k[t] > 0.0) {
                g += k[t];
                last = t;
            }
        }
        const double p = g * dt;
        const double fl = floor(p);
        if (!(fl < 4294967296.0)) return -1;
        gamma[r] = g;
        n0[r] = (uint32_t)fl;
        thr[r] = (uint32_t)floor((p - fl) * 4294967296.0);
        double C = 0.0;
        for (int t = 0; t < width; ++t) {
            if (k[t] > 0.0) C += k[t];
            uint64_t v;
            if (last < 0)
                v = 0;
            else if (t >= last)
                v = 1ull << 32;
            else
                v = (uint64_t)floor(C / g * 4294967296.0);
            cdf[(long)r * width + t] = v;
        }
    }
    return 0;
}

/* ---------------------------------------------------------------- particles */
/* Fraction bits such that (cell + k 2^-fb) is exact in the position type. */
static int frac_bits(int n_max, int pos_f64) {
    int k = 0;
    while ((1L << k) < (long)n_max) ++k;
    int fb = (pos_f64 ? 53 : 24) - k;
    return fb > 32 ? 32 : fb;
}

static double frac_of(uint32_t u, int fb) { return ldexp((double)(u >> (32 - fb)), -fb); }

typedef struct {
    int dim, nx, ny, n_k, M_min, f64;
} pgeom;

static double get_pos(const void* a, int f64, int64_t i) {
    return f64 ? ((const double*)a)[i] : (double)((const float*)a)[i];
}
static void set_pos(void* a, int f64, int64_t i, double v) {
    if (f64)
        ((double*)a)[i] = v;
    else
        ((float*)a)[i] = (float)v; /* callers only store values exact in float */
}
static long get_mom(const void* a, int dim, int64_t i) {
    return dim == 1 ? (long)((const int32_t*)a)[i] : (long)((const int16_t*)a)[i];
}
static void set_mom(void* a, int dim, int64_t i, long v) {
    if (dim == 1)
        ((int32_t*)a)[i] = (int32_t)v;
    else
        ((int16_t*)a)[i] = (int16_t)v;
}

/* Cell index of a position given in cell units, -1 outside [0, n). */
static long cell_of(double x, int n) {
    if (!(x >= 0.0) || !(x < (double)n)) return -1;
    return (long)floor(x);
}

/* Histogram bin of particle id, -1 if dead or outside the grid. */
static long bin_of(const pgeom* g, int64_t id, const void* x, const void* y, const void* M,
                   const void* My, const int8_t* s) {
    if (s[id] == 0) return -1;
    long cx = cell_of(get_pos(x, g->f64, id), g->nx);
    if (cx < 0) return -1;
    long kx = get_mom(M, g->dim, id) - g->M_min;
    if (kx < 0 || kx >= g->n_k) return -1;
    if (g->dim == 1) return cx * g->n_k + kx;
    long cy = cell_of(get_pos(y, g->f64, id), g->ny);
    if (cy < 0) return -1;
    long ky = get_mom(My, g->dim, id) - g->M_min;
    if (ky < 0 || ky >= g->n_k) return -1;
    return ((cy * g->nx + cx) * g->n_k + ky) * g->n_k + kx;
}

/* Fill particle slot o with a particle of bin b drawn uniformly in its cell;
 * the r-th particle of the bin uses counter (b, c1, r/4 or r/2, tag). */
static void place_in_bin(const pgeom* g, uint64_t seed, uint32_t c1, uint32_t tag, long b, long r,
                         int8_t sign, int64_t o, void* x, void* y, void* M, void* My, int8_t* s) {
    uint32_t w[4];
    int fb = frac_bits(g->nx > g->ny ? g->nx : g->ny, g->f64);
    if (g->dim == 1) {
        long cx = b / g->n_k, kx = b % g->n_k;
        draw4(seed, (uint32_t)b, c1, (uint32_t)(r / 4), tag, w);
        set_pos(x, g->f64, o, (double)cx + frac_of(w[r % 4], fb));
        set_mom(M, 1, o, g->M_min + kx);
    } else {
        long kx = b % g->n_k, ky = (b / g->n_k) % g->n_k, c = b / ((long)g->n_k * g->n_k);
        long cx = c % g->nx, cy = c / g->nx;
        draw4(seed, (uint32_t)b, c1, (uint32_t)(r / 2), tag, w);
        set_pos(x, g->f64, o, (double)cx + frac_of(w[2 * (r % 2)], fb));
        set_pos(y, g->f64, o, (double)cy + frac_of(w[2 * (r % 2) + 1], fb));
        set_mom(M, 2, o, g->M_min + kx);
        set_mom(My, 2, o, g->M_min + ky);
    }
    s[o] = sign;
}

int64_t oracle_sp_init(int dim, int nx, int ny, int n_k, int M_min, int pos_f64, uint64_t seed,
                       const int32_t* bin_counts, void* x, void* y, void* M, void* My, int8_t* s,
                       int64_t capacity) {
    if ((dim != 1 && dim != 2) || nx <= 0 || n_k <= 0) return -1;
    if (dim == 1) ny = 1;
    pgeom g = {dim, nx, ny, n_k, M_min, pos_f64};
    long n_bins = (long)nx * ny * n_k * (dim == 2 ? n_k : 1);
    int64_t o = 0;
    for (long b = 0; b < n_bins; ++b) {
        if (bin_counts[b] < 0) return -1;
        if (o + bin_counts[b] > capacity) return -2;
        for (long r = 0; r < bin_counts[b]; ++r, ++o)
            place_in_bin(&g, seed, 0xFFFFFFFFu, TAG_INIT, b, r, 1, o, x, y, M, My, s);
    }
    return o;
}

/* Number of pairs particle id creates this step and its first Philox block. */
static long pairs_of(const pgeom* g, uint64_t seed, int64_t step, int64_t id, const void* x,
                     const void* y, const int8_t* s, const int32_t* cell_slot, const uint32_t* n0,
                     const uint32_t* thr, long* slot_out, uint32_t w[4]) {
    *slot_out = -1;
    if (s[id] == 0) return 0;
    long cx = cell_of(get_pos(x, g->f64, id), g->nx);
    if (cx < 0) return 0;
    long c = cx;
    if (g->dim == 2) {
        long cy = cell_of(get_pos(y, g->f64, id), g->ny);
        if (cy < 0) return 0;
        c = cy * g->nx + cx;
    }
    long slot = cell_slot[c];
    if (slot < 0) return 0;
    *slot_out = slot;
    draw4(seed, (uint32_t)id, (uint32_t)step, 0, TAG_CREATE, w);
    return (long)n0[slot] + (w[0] < thr[slot] ? 1 : 0);
}

int64_t oracle_sp_step(int dim, int nx, int ny, int n_m, int n_k, int M_min, int pos_f64,
                       double vdt, uint64_t seed, int64_t step, const int32_t* cell_slot,
                       const uint32_t* n0, const uint32_t* thr, const uint64_t* cdf, int64_t n,
                       void* x, void* y, void* M, void* My, int8_t* s, int64_t capacity,
                       int64_t* stats) {
    if ((dim != 1 && dim != 2) || nx <= 0 || n_m <= 0 || (n_m & 1) || n < 0) return -1;
    if (dim == 1) ny = 1;
    pgeom g = {dim, nx, ny, n_k, M_min, pos_f64};
    const int P = n_m / 2;
    const long width = dim == 1 ? n_m : (long)n_m * n_m;
    for (int k = 0; k < 8; ++k) stats[k] = 0;

    /* count the pairs first: nothing is written if they do not fit */
    int64_t total = 0;
    uint32_t w[4];
    long slot;
    for (int64_t id = 0; id < n; ++id)
        total += pairs_of(&g, seed, step, id, x, y, s, cell_slot, n0, thr, &slot, w);
    const int64_t needed = n + 2 * total;
    if (needed > capacity) {
        stats[ORACLE_ST_NEEDED] = needed;
        return -2;
    }

    /* creation at the start-of-step position, children appended in id order */
    int64_t o = n;
    for (int64_t id = 0; id < n; ++id) {
        long np = pairs_of(&g, seed, step, id, x, y, s, cell_slot, n0, thr, &slot, w);
        for (long k = 0; k < np; ++k) {
            uint32_t u;
            if (k < 3) {
                u = w[k + 1];
            } else {
                uint32_t w2[4];
                draw4(seed, (uint32_t)id, (uint32_t)step, (uint32_t)(1 + (k - 3) / 4), TAG_CREATE, w2);
                u = w2[(k - 3) % 4];
            }
            const uint64_t* T = cdf + slot * width;
            long t = 0;
            while (!((uint64_t)u < T[t])) ++t;
            const long mx = (dim == 1 ? t : t % n_m) - P;
            const long my = (dim == 1 ? 0 : t / n_m) - P;
            for (int child = 0; child < 2; ++child, ++o) {
                const long sg = child == 0 ? 1 : -1;
                set_pos(x, pos_f64, o, get_pos(x, pos_f64, id));
                set_mom(M, dim, o, get_mom(M, dim, id) + sg * mx);
                if (dim == 2) {
                    set_pos(y, pos_f64, o, get_pos(y, pos_f64, id));
                    set_mom(My, dim, o, get_mom(My, dim, id) + sg * my);
                }
                s[o] = (int8_t)(sg * s[id]);
            }
        }
    }

    /* field-less drift of every particle, then the absorbing boundaries */
    int64_t abs_x = 0, abs_m = 0;
    for (int64_t id = 0; id < needed; ++id) {
        if (s[id] == 0) continue;
        int out_x = 0;
        long mom[2] = {get_mom(M, dim, id), dim == 2 ? get_mom(My, dim, id) : 0};
        void* arr[2] = {x, y};
        int ncell[2] = {nx, ny};
        for (int a = 0; a < dim; ++a) {
            if (pos_f64) {
                double* p = (double*)arr[a];
                p[id] = fma((double)mom[a], vdt, p[id]);
                if (!(p[id] >= 0.0) || !(p[id] < (double)ncell[a])) out_x = 1;
            } else {
                float* p = (float*)arr[a];
                p[id] = fmaf((float)mom[a], (float)vdt, p[id]);
                if (!(p[id] >= 0.0f) || !(p[id] < (float)ncell[a])) out_x = 1;
            }
        }
        int out_m = 0;
        for (int a = 0; a < dim; ++a)
            if (mom[a] < M_min || mom[a] >= (long)M_min + n_k) out_m = 1;
        if (out_x) {
            s[id] = 0;
            ++abs_x;
        } else if (out_m) {
            s[id] = 0;
            ++abs_m;
        }
    }
    stats[ORACLE_ST_N] = needed;
    stats[ORACLE_ST_PAIRS] = total;
    stats[ORACLE_ST_ABS_X] = abs_x;
    stats[ORACLE_ST_ABS_M] = abs_m;
    return needed;
}

int64_t oracle_sp_annihilate(int dim, int nx, int ny, int n_k, int M_min, int pos_f64,
                             uint64_t seed, int64_t step, int64_t n, const void* x, const void* y,
                             const void* M, const void* My, const int8_t* s, void* xo, void* yo,
                             void* Mo, void* Myo, int8_t* so, int64_t capacity,
                             int32_t* hist_plus, int32_t* hist_minus, int64_t* stats) {
    if ((dim != 1 && dim != 2) || nx <= 0 || n_k <= 0 || n < 0) return -1;
    if (dim == 1) ny = 1;
    pgeom g = {dim, nx, ny, n_k, M_min, pos_f64};
    const long n_bins = (long)nx * ny * n_k * (dim == 2 ? n_k : 1);
    int32_t* hp = hist_plus ? hist_plus : (int32_t*)malloc(sizeof(int32_t) * n_bins);
    int32_t* hm = hist_minus ? hist_minus : (int32_t*)malloc(sizeof(int32_t) * n_bins);
    memset(hp, 0, sizeof(int32_t) * n_bins);
    memset(hm, 0, sizeof(int32_t) * n_bins);
    for (int k = 0; k < 8; ++k) stats[k] = 0;

    for (int64_t id = 0; id < n; ++id) {
        long b = bin_of(&g, id, x, y, M, My, s);
        if (b < 0) continue;
        if (s[id] > 0)
            hp[b]++;
        else
            hm[b]++;
    }
    int64_t o = 0, rc = 0, mixed = 0;
    /* mixed bins, ascending: |net| fresh particles of the net sign */
    for (long b = 0; b < n_bins && rc == 0; ++b) {
        if (!(hp[b] > 0 && hm[b] > 0)) continue;
        ++mixed;
        const long net = (long)hp[b] - (long)hm[b];
        const long cnt = net < 0 ? -net : net;
        if (o + cnt > capacity) {
            rc = -2;
            break;
        }
        for (long r = 0; r < cnt; ++r, ++o)
            place_in_bin(&g, seed, (uint32_t)step, TAG_ANNIH, b, r, net > 0 ? 1 : -1, o, xo, yo,
                         Mo, Myo, so);
    }
    const int64_t regen = o;
    /* then the particles of single-sign bins, unchanged and in input order */
    for (int64_t id = 0; id < n && rc == 0; ++id) {
        long b = bin_of(&g, id, x, y, M, My, s);
        if (b < 0 || (hp[b] > 0 && hm[b] > 0)) continue;
        if (o >= capacity) {
            rc = -2;
            break;
        }
        set_pos(xo, pos_f64, o, get_pos(x, pos_f64, id));
        set_mom(Mo, dim, o, get_mom(M, dim, id));
        if (dim == 2) {
            set_pos(yo, pos_f64, o, get_pos(y, pos_f64, id));
            set_mom(Myo, dim, o, get_mom(My, dim, id));
        }
        so[o++] = s[id];
    }
    if (!hist_plus) free(hp);
    if (!hist_minus) free(hm);
    if (rc) return rc;
    stats[ORACLE_ST_N] = o;
    stats[ORACLE_ST_ANNIH_KEPT] = o - regen;
    stats[ORACLE_ST_ANNIH_REGEN] = regen;
    stats[ORACLE_ST_MIXED] = mixed;
    return o;
}

/* ---------------------------------------------------------------- surrogate */
/* eq.(5) read with the offsets of a cell's window o in [-P, P) grouped N at a
 * time, o(g,p) = -P + N g + p, angle theta(o, m) = 2 pi o m / n_m (Sec. 2.3):
 *   Kh(i,m) = prod_{s < log2 N} cos(2^s pi m / n_m)
 *             * sum_g W_g (sum_p wV_p V(i+o(g,p))) sin(sum_p wT_p theta(o(g,p), m)). */
static int log2_exact(int N) {
    int L = 0;
    while ((1 << L) < N) ++L;
    return (1 << L) == N ? L : -1;
}

static double cos_prefactor(int L, long m, int n_m) {
    double pr = 1.0;
    for (int s = 0; s < L; ++s) pr *= cos(PI_D * (double)(1L << s) * (double)m / (double)n_m);
    return pr;
}

int oracle_surrogate_fwd(int nx, int n_m, int N, const double* wV, const double* wT,
                         const double* W, const double* V, int B, const int32_t* cells,
                         int n_cells, double* Kh) {
    const int L = log2_exact(N);
    if (nx <= 0 || n_m <= 0 || (n_m & 1) || N <= 0 || L < 0 || n_m % N || B < 0) return -1;
    const int P = n_m / 2, H = n_m / N;
    for (int b = 0; b < B; ++b) {
        const double* Vb = V + (long)b * nx;
        for (int r = 0; r < n_cells; ++r) {
            const long i = cells ? cells[r] : r;
            if (i < 0 || i >= nx) return -1;
            double* row = Kh + ((long)b * n_cells + r) * P;
            for (int t = 0; t < P; ++t) {
                const long m = t + 1;
                double acc = 0.0;
                for (int g = 0; g < H; ++g) {
                    double fV = 0.0, fT = 0.0;
                    for (int p = 0; p < N; ++p) {
                        const long o = -P + (long)N * g + p;
                        fV += wV[p] * v1(Vb, nx, i + o);
                        fT += wT[p] * (TWO_PI * (double)o * (double)m / (double)n_m);
                    }
                    acc += W[g] * fV * sin(fT);
                }
                row[t] = cos_prefactor(L, m, n_m) * acc;
            }
        }
    }
    return 0;
}

int oracle_surrogate_bwd(int nx, int n_m, int N, const double* wV, const double* wT,
                         const double* W, const double* V, int B, const int32_t* cells,
                         int n_cells, const double* E, double* dwV, double* dwT, double* dW,
                         double* dV) {
    const int L = log2_exact(N);
    if (nx <= 0 || n_m <= 0 || (n_m & 1) || N <= 0 || L < 0 || n_m % N || B < 0) return -1;
    const int P = n_m / 2, H = n_m / N;
    for (int p = 0; p < N; ++p) dwV[p] = dwT[p] = 0.0;
    for (int g = 0; g < H; ++g) dW[g] = 0.0;
    for (int b = 0; b < B; ++b) {
        const double* Vb = V + (long)b * nx;
        for (int r = 0; r < n_cells; ++r) {
            const long i = cells ? cells[r] : r;
            if (i < 0 || i >= nx) return -1;
            const double* e = E + ((long)b * n_cells + r) * P;
            for (int t = 0; t < P; ++t) {
                const long m = t + 1;
                const double ep = e[t] * cos_prefactor(L, m, n_m);
                for (int g = 0; g < H; ++g) {
                    double fV = 0.0, u = 0.0;
                    for (int p = 0; p < N; ++p) {
                        const long o = -P + (long)N * g + p;
                        fV += wV[p] * v1(Vb, nx, i + o);
                        u += wT[p] * (TWO_PI * (double)o / (double)n_m);
                    }
                    const double sn = sin(u * (double)m), cs = cos(u * (double)m);
                    dW[g] += ep * fV * sn;
                    const double dfV = ep * W[g] * sn;      /* d/d fV */
                    const double du = ep * W[g] * fV * cs * (double)m; /* d/d u_g */
                    for (int p = 0; p < N; ++p) {
                        const long o = -P + (long)N * g + p;
                        long l = i + o;
                        if (l < 0) l = 0;
                        if (l >= nx) l = nx - 1;
                        dwV[p] += dfV * Vb[l];
                        dwT[p] += du * (TWO_PI * (double)o / (double)n_m);
                        if (dV) dV[(long)b * nx + l] += dfV * wV[p];
                    }
                }
            }
        }
    }
    return 0;
}

/* ---------------------------------------------------------------- training (Sec. 3) */
/* Mean squared error of the network against labels, on targets scaled by inv_scale:
 *   loss = sum ((Kh - K) inv_scale)^2 / count,  E = dloss/dKh = 2 (Kh - K) inv_scale^2 / count. */
double oracle_mse_grad(const double* Kh, const double* K, int64_t count, double inv_scale,
                       double* E) {
    double loss = 0.0;
    const double s2 = inv_scale * inv_scale;
    for (int64_t k = 0; k < count; ++k) {
        const double d = Kh[k] - K[k];
        loss += d * d * s2;
        if (E) E[k] = 2.0 * d * s2 / (double)count;
    }
    return loss / (double)count;
}

/* One step of stochastic gradient descent on that loss over a batch of B potentials (all
 * cells), with the labels K [B][nx][P] given: forward of eq.(5), loss and its gradient, the
 * backward, then w <- w - lr g per group, with W stepped in units of c = -2/(hbar n_m), i.e.
 * W <- W - lr_W c^2 dL/dW.  Returns the loss before the step (negative on bad arguments). */
double oracle_sgd_step(int nx, int n_m, int N, double hbar, const double* V, int B,
                       const double* K, double inv_scale, double lr_V, double lr_T, double lr_W,
                       double* wV, double* wT, double* W) {
    if (nx <= 0 || n_m <= 0 || (n_m & 1) || N <= 0 || n_m % N || B <= 0 || hbar <= 0) return -1.0;
    const int P = n_m / 2, H = n_m / N;
    const int64_t count = (int64_t)B * nx * P;
    double* Kh = (double*)malloc(sizeof(double) * (size_t)count);
    double* E = (double*)malloc(sizeof(double) * (size_t)count);
    double* gV = (double*)malloc(sizeof(double) * (size_t)N);
    double* gT = (double*)malloc(sizeof(double) * (size_t)N);
    double* gW = (double*)malloc(sizeof(double) * (size_t)H);
    double loss = -1.0;
    if (Kh && E && gV && gT && gW &&
        oracle_surrogate_fwd(nx, n_m, N, wV, wT, W, V, B, NULL, nx, Kh) == 0) {
        loss = oracle_mse_grad(Kh, K, count, inv_scale, E);
        if (oracle_surrogate_bwd(nx, n_m, N, wV, wT, W, V, B, NULL, nx, E, gV, gT, gW, NULL) == 0) {
            const double c = -2.0 / (hbar * (double)n_m);
            for (int p = 0; p < N; ++p) {
                wV[p] -= lr_V * gV[p];
                wT[p] -= lr_T * gT[p];
            }
            for (int g = 0; g < H; ++g) W[g] -= lr_W * c * c * gW[g];
        } else {
            loss = -1.0;
        }
    }
    free(Kh);
    free(E);
    free(gV);
    free(gT);
    free(gW);
    return loss;
}

/* ---------------------------------------------------------------- rule 2, pair removal */
/* Rule 2 of Sec. 2.1 read literally: particles of opposite sign in the same (cell, momentum)
 * bin annihilate in pairs.  Within a bin the k-th positive particle in input order meets
 * the k-th negative one, k < min(H+, H-); those pairs are removed and every other live
 * particle is kept unchanged (its exact position), in input order.  Returns the number kept,
 * or -2 if capacity is too small; the histogram (H+, H-) of the input is left in
 * hist_plus / hist_minus when they are given. */
int64_t oracle_sp_annihilate_pairs(int dim, int nx, int ny, int n_k, int M_min, int pos_f64,
                                   int64_t n, const void* x, const void* y, const void* M,
                                   const void* My, const int8_t* s, void* xo, void* yo,
                                   void* Mo, void* Myo, int8_t* so, int64_t capacity,
                                   int32_t* hist_plus, int32_t* hist_minus, int64_t* stats) {
    if ((dim != 1 && dim != 2) || nx <= 0 || n_k <= 0 || n < 0) return -1;
    if (dim == 1) ny = 1;
    pgeom g = {dim, nx, ny, n_k, M_min, pos_f64};
    const long n_bins = (long)nx * ny * n_k * (dim == 2 ? n_k : 1);
    int32_t* hp = hist_plus ? hist_plus : (int32_t*)malloc(sizeof(int32_t) * n_bins);
    int32_t* hm = hist_minus ? hist_minus : (int32_t*)malloc(sizeof(int32_t) * n_bins);
    int32_t* seen_p = (int32_t*)calloc((size_t)n_bins, sizeof(int32_t));
    int32_t* seen_m = (int32_t*)calloc((size_t)n_bins, sizeof(int32_t));
    memset(hp, 0, sizeof(int32_t) * n_bins);
    memset(hm, 0, sizeof(int32_t) * n_bins);
    for (int k = 0; k < 8; ++k) stats[k] = 0;
    for (int64_t id = 0; id < n; ++id) {
        const long b = bin_of(&g, id, x, y, M, My, s);
        if (b < 0) continue;
        if (s[id] > 0)
            hp[b]++;
        else
            hm[b]++;
    }
    int64_t mixed = 0;
    for (long b = 0; b < n_bins; ++b)
        if (hp[b] > 0 && hm[b] > 0) ++mixed;
    int64_t o = 0, rc = 0;
    for (int64_t id = 0; id < n; ++id) {
        const long b = bin_of(&g, id, x, y, M, My, s);
        if (b < 0) continue;
        const int32_t pairs = hp[b] < hm[b] ? hp[b] : hm[b];
        const int32_t rank = s[id] > 0 ? seen_p[b]++ : seen_m[b]++;
        if (rank < pairs) continue; /* annihilated with its partner of the other sign */
        if (o >= capacity) {
            rc = -2;
            break;
        }
        set_pos(xo, pos_f64, o, get_pos(x, pos_f64, id));
        set_mom(Mo, dim, o, get_mom(M, dim, id));
        if (dim == 2) {
            set_pos(yo, pos_f64, o, get_pos(y, pos_f64, id));
            set_mom(Myo, dim, o, get_mom(My, dim, id));
        }
        so[o++] = s[id];
    }
    free(seen_p);
    free(seen_m);
    if (!hist_plus) free(hp);
    if (!hist_minus) free(hm);
    if (rc) return rc;
    stats[ORACLE_ST_N] = o;
    stats[ORACLE_ST_ANNIH_KEPT] = o;
    stats[ORACLE_ST_ANNIH_REGEN] = 0;
    stats[ORACLE_ST_MIXED] = mixed;
    return o;
}

/* ---------------------------------------------------------------- surrogate, d = 2 */
/* eq.(5) carried to d = 2 (the d-dimensional statement of Sec. 2.1): the offsets o of a cell's
 * window on the periodic grid, o_a in [-P, P) per axis, are grouped N x N, g = (gx, gy),
 * o(g, p) = (-P + N gx + px, -P + N gy + py);
 *   Kh(i; mx, my) = prod_s cos(2^s pi mx / n_m) prod_s cos(2^s pi my / n_m)
 *                   * sum_g W[gy H + gx] (sum_p wV[py N + px] Vt(i, o(g, p)))
 *                     * sin(ux(gx) mx + uy(gy) my),
 *   ux(gx) = (2 pi / n_m) sum_px wTx[px] (-P + N gx + px), uy likewise with wTy,
 * where Vt(i, o) = V(i + o) except at an end point o_a = -P of the periodic grid, where it is
 * the mean of V at i_a - P and i_a + P (both ends, per axis): the trapezoid half weights of
 * the d = 2 kernel.  With wV = 1, wT = 1/N, W = -2/(hbar n_m^2), N = 1 is that kernel
 * exactly.  Full table [B][n_cells][n_m][n_m] (ty, tx), (mx, my) = (tx - P, ty - P). */
static double vt2(const double* Vb, int nx, int ny, long ix, long iy, long ox, long oy, int P) {
    const int ex = ox == -P, ey = oy == -P;
    double s = 0.0;
    int k = 0;
    for (int a = 0; a <= ex; ++a)
        for (int b = 0; b <= ey; ++b) {
            const long dx = a ? P : ox, dy = b ? P : oy;
            s += v2(Vb, nx, ny, ix + dx, iy + dy);
            ++k;
        }
    return s / (double)k;
}

int oracle_surrogate_fwd_2d(int nx, int ny, int n_m, int N, const double* wV, const double* wTx,
                            const double* wTy, const double* W, const double* V, int B,
                            const int32_t* cells, int n_cells, double* Kh) {
    const int L = log2_exact(N);
    if (nx <= 0 || ny <= 0 || n_m <= 0 || (n_m & 1) || N <= 0 || L < 0 || n_m % N || B < 0) return -1;
    const int P = n_m / 2, H = n_m / N;
    const long ncell = (long)nx * ny;
    for (int b = 0; b < B; ++b) {
        const double* Vb = V + (long)b * ncell;
        for (int r = 0; r < n_cells; ++r) {
            const long cid = cells ? cells[r] : r;
            if (cid < 0 || cid >= ncell) return -1;
            const long ix = cid % nx, iy = cid / nx;
            double* row = Kh + ((long)b * n_cells + r) * (long)n_m * n_m;
            for (int ty = 0; ty < n_m; ++ty) {
                for (int tx = 0; tx < n_m; ++tx) {
                    const long mx = tx - P, my = ty - P;
                    double acc = 0.0;
                    for (int gy = 0; gy < H; ++gy) {
                        for (int gx = 0; gx < H; ++gx) {
                            double fV = 0.0, ux = 0.0, uy = 0.0;
                            for (int py = 0; py < N; ++py)
                                for (int px = 0; px < N; ++px)
                                    fV += wV[py * N + px] * vt2(Vb, nx, ny, ix, iy, -P + (long)N * gx + px,
                                                                -P + (long)N * gy + py, P);
                            for (int p = 0; p < N; ++p) {
                                ux += wTx[p] * (TWO_PI * (double)(-P + N * gx + p) / (double)n_m);
                                uy += wTy[p] * (TWO_PI * (double)(-P + N * gy + p) / (double)n_m);
                            }
                            acc += W[gy * H + gx] * fV * sin(ux * (double)mx + uy * (double)my);
                        }
                    }
                    row[(long)ty * n_m + tx] = cos_prefactor(L, mx, n_m) * cos_prefactor(L, my, n_m) * acc;
                }
            }
        }
    }
    return 0;
}
