/*
 * wk_oracle.h -- plain CPU reference of the signed-particle Wigner Monte Carlo
 * hot path (Sellier, Leygonie, Marceau Caron, "Combining neural networks and
 * signed particles to simulate quantum systems more efficiently, Part II",
 * arXiv:1806.00082).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code with the HIP library.
 *
 * Conventions (all arrays host memory, row-major, caller-owned):
 *   - 1-D mesh: nx cells, potential V[b][i] sampled at cell centres.
 *     2-D mesh: V[b][iy][ix].  Outside the mesh V is the nearest edge value.
 *   - n_m = L_C / dx pseudo-momenta per axis (even), P = n_m / 2,
 *     momentum index m in [-P, P), Delta k = pi / L_C.
 *   - Full 1-D table: K[row][t], m = t - P.  Full 2-D table: K[row][ty][tx].
 *     Half 1-D table: K[row][t], m = t + 1 (t in [0, P)).
 *   - Particle positions are in units of the cell width (cell c = floor(x)).
 *   - Return value >= 0 on success, negative on error.
 */
#ifndef WK_ORACLE_H
#define WK_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Philox4x32-10 block: out = Philox(ctr, key). */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* eq.(4) folded onto positive offsets, full table [B][n_cells][n_m]. */
int oracle_kernel_1d(int nx, int n_m, double hbar, const double* V, int B,
                     const int32_t* cells, int n_cells, double* K);
/* eq.(4) exactly as printed (offsets -P..P, both terms), full table. */
int oracle_kernel_1d_literal(int nx, int n_m, double hbar, const double* V, int B,
                             const int32_t* cells, int n_cells, double* K);
/* d = 2 form of eq.(4), direct double sum with half weights at |j_a| = P.
 * cells are flat ids iy*nx+ix; output [B][n_cells][n_m][n_m] (ty, tx). */
int oracle_kernel_2d(int nx, int ny, int n_m, double hbar, const double* V, int B,
                     const int32_t* cells, int n_cells, double* K);
/* Adjoint of V -> half table (1-D) on the requested cells (NULL = all, n_cells = nx):
 * G [B][n_cells][P]; dV[b][l] += sum_{r,t} G[b][r][t] dK(cells[r], t + 1)/dV[b][l]. */
int oracle_kernel_bwd_1d(int nx, int n_m, double hbar, const double* G, int B,
                         const int32_t* cells, int n_cells, double* dV);

/* eq.(1) on the grid and the integer sampling tables (width = entries per row). */
int oracle_gamma_tables(int width, const double* K, int n_rows, double dt,
                        double* gamma, uint32_t* n0, uint32_t* thr, uint64_t* cdf);

/* Particle passes.  pos_f64 selects double (1) or float (0) positions.
 * stats (int64[8]): see ORACLE_ST_* below. */
enum { ORACLE_ST_N = 0, ORACLE_ST_PAIRS = 1, ORACLE_ST_ABS_X = 2, ORACLE_ST_ABS_M = 3,
       ORACLE_ST_NEEDED = 4, ORACLE_ST_ANNIH_KEPT = 5, ORACLE_ST_ANNIH_REGEN = 6,
       ORACLE_ST_MIXED = 7 };

int64_t oracle_sp_init(int dim, int nx, int ny, int n_k, int M_min, int pos_f64, uint64_t seed,
                       const int32_t* bin_counts, void* x, void* y, void* M, void* My,
                       int8_t* s, int64_t capacity);

int64_t oracle_sp_step(int dim, int nx, int ny, int n_m, int n_k, int M_min, int pos_f64,
                       double vdt, uint64_t seed, int64_t step,
                       const int32_t* cell_slot, const uint32_t* n0, const uint32_t* thr,
                       const uint64_t* cdf, int64_t n, void* x, void* y, void* M, void* My,
                       int8_t* s, int64_t capacity, int64_t* stats);

int64_t oracle_sp_annihilate(int dim, int nx, int ny, int n_k, int M_min, int pos_f64,
                             uint64_t seed, int64_t step, int64_t n,
                             const void* x, const void* y, const void* M, const void* My,
                             const int8_t* s, void* xo, void* yo, void* Mo, void* Myo,
                             int8_t* so, int64_t capacity, int32_t* hist_plus,
                             int32_t* hist_minus, int64_t* stats);

/* Rule 2 as pair removal: in each bin the k-th positive and k-th negative particle (input
 * order) annihilate for k < min(H+, H-); the other live particles are kept unchanged, in
 * input order (no regeneration, exact positions). */
int64_t oracle_sp_annihilate_pairs(int dim, int nx, int ny, int n_k, int M_min, int pos_f64,
                                   int64_t n, const void* x, const void* y, const void* M,
                                   const void* My, const int8_t* s, void* xo, void* yo,
                                   void* Mo, void* Myo, int8_t* so, int64_t capacity,
                                   int32_t* hist_plus, int32_t* hist_minus, int64_t* stats);

/* eq.(5) with N-term groups; half table m = 1..P.  wV, wT: [N]; W: [n_m/N]. */
int oracle_surrogate_fwd(int nx, int n_m, int N, const double* wV, const double* wT,
                         const double* W, const double* V, int B, const int32_t* cells,
                         int n_cells, double* Kh);
/* Gradients of sum(E * Kh) w.r.t. wV, wT, W (overwritten) and V (accumulated, may be NULL). */
int oracle_surrogate_bwd(int nx, int n_m, int N, const double* wV, const double* wT,
                         const double* W, const double* V, int B, const int32_t* cells,
                         int n_cells, const double* E, double* dwV, double* dwT, double* dW,
                         double* dV);

/* eq.(5) in d = 2: offsets grouped N x N, angle weights per axis (wTx, wTy [N]), wV [N*N],
 * W [(n_m/N)^2]; the window value at an end point -P of the periodic grid is the mean of the
 * two end values (N = 1 with analytic weights is the d = 2 kernel).  Full table
 * [B][n_cells][n_m][n_m]. */
int oracle_surrogate_fwd_2d(int nx, int ny, int n_m, int N, const double* wV, const double* wTx,
                            const double* wTy, const double* W, const double* V, int B,
                            const int32_t* cells, int n_cells, double* Kh);

/* Training of Sec. 3.  MSE on targets scaled by inv_scale; returns the loss and writes
 * E = dloss/dKh (E may be NULL). */
double oracle_mse_grad(const double* Kh, const double* K, int64_t count, double inv_scale,
                       double* E);
/* One SGD step on a batch of B potentials (all cells) with labels K [B][nx][P]: updates wV,
 * wT (step lr_V, lr_T) and W (step lr_W in units of c = -2/(hbar n_m)) in place; returns the
 * loss before the step. */
double oracle_sgd_step(int nx, int n_m, int N, double hbar, const double* V, int B,
                       const double* K, double inv_scale, double lr_V, double lr_T, double lr_W,
                       double* wV, double* wT, double* W);

#ifdef __cplusplus
}
#endif
#endif
