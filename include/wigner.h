/*
 * wigner.h -- C ABI of libwigner.so, the MI355X (gfx950) hot path of the signed-particle
 * Wigner Monte Carlo method with a neural-network Wigner kernel (Sellier, Leygonie,
 * Marceau Caron, arXiv:1806.00082).
 *
 * General conventions
 *   - Every array argument is a DEVICE pointer owned by the caller; the library never
 *     frees caller memory.  Scalars and the small parameter structs are host values.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).  Every call
 *     only enqueues work on that stream and returns without synchronising.
 *   - Return value: WK_OK (0) or a negative code.  Arguments are validated on the host
 *     before anything is enqueued; on WK_EINVAL nothing is enqueued.  wk_last_error()
 *     returns a thread-local description of the last failure.
 *   - Set-up: wk_prepare(mesh) builds, per device and n_m, the read-only sine tables the
 *     1-D contractions read (device memory held until the process ends); it allocates and
 *     synchronises its stream, and must be called once per device and n_m before
 *     wk_kernel_eval, wk_kernel_tables or wk_kernel_bwd use that n_m in 1-D (they fail with
 *     WK_EINVAL otherwise).  No other call allocates memory or synchronises: scratch
 *     space is the caller's workspace argument.
 *   - Results are deterministic: identical inputs give bit-identical outputs.
 *
 * Mesh and tables (Sec. 2.2 of the paper)
 *   - 1-D: nx cells; V[b][i] is the potential (eV) at the centre of cell i of potential
 *     b.  2-D: V[b][iy][ix].  Outside the mesh V takes the nearest edge value.
 *   - n_m = L_C / dx pseudo-momenta per axis, even; P = n_m / 2; momentum index
 *     m in [-P, P) counts Delta k = pi / L_C (Delta p = pi hbar / L_C).
 *   - Full 1-D table  K[row][t], t in [0, n_m), m = t - P (n_m entries per row).
 *     Half 1-D table  K[row][t], t in [0, P),   m = t + 1 (V_W is odd in m:
 *     K(-m) = -K(m), K(0) = 0, and the full entry m = -P is -K(P)).
 *     Full 2-D table  K[row][ty][tx], (m_x, m_y) = (tx - P, ty - P).
 *   - Rows: row = b * n_cells + r for potential b and the r-th requested cell
 *     (cells[r], or r itself when cells is NULL).  Values are in 1/fs.
 *
 * Particles (Sec. 2.1)
 *   - Struct-of-arrays.  Positions are in units of the cell width (cell = floor(x)),
 *     float or double per sp_geom.pos_f64.  Momentum indices (1-D: M; 2-D: M on the x
 *     axis and My) are int32, int16 or int8 per sp_geom.m_bytes.  s is int8: +1 / -1,
 *     0 = absorbed (dropped by the next annihilation).
 *   - The particle count lives in device memory (*d_n) so a time loop needs no host
 *     synchronisation.
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by the 64-bit seed,
 *     counter (particle or bin id, step, block, stream tag); the stream of a particle
 *     depends only on its index at the start of the step, never on the launch shape.
 */
#ifndef WIGNER_H
#define WIGNER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WK_OK 0
#define WK_EINVAL (-1)     /* bad argument; nothing enqueued */
#define WK_ECAPACITY (-2)  /* particle buffer too small (see WK_ST_NEEDED) */
#define WK_EHIP (-3)       /* HIP runtime error (message in wk_last_error) */

#define WK_VERSION 4

/* Arithmetic of the kernel contraction. */
enum wk_prec {
    WK_FP64 = 0,    /* FP64 MFMA, FP64 output */
    WK_BF16 = 1,    /* BF16 operands, FP32 accumulate, FP32 output */
    WK_FP16 = 2,    /* FP16 operands, FP32 accumulate, FP32 output */
    WK_BF16X3 = 3,  /* hi/lo BF16 split, three products, FP32 accumulate and output */
    WK_FP16X3 = 4,  /* hi/lo FP16 split, three products, FP32 accumulate and output */
    WK_FP32 = 5     /* FP32 operands and arithmetic (wk_kernel_bwd, wk_surrogate_fwd) */
};

enum wk_layout { WK_FULL = 0, WK_HALF = 1 };

typedef struct wk_mesh {
    int32_t dim;   /* 1 or 2 */
    int32_t nx;    /* cells along x */
    int32_t ny;    /* cells along y (1 in 1-D) */
    int32_t n_m;   /* pseudo-momenta per axis = L_C / dx, even, >= 2 */
    double hbar;   /* reduced Planck constant in eV fs */
} wk_mesh;

typedef struct sp_geom {
    int32_t dim;      /* 1 or 2 */
    int32_t nx, ny;   /* cells per axis (ny = 1 in 1-D) */
    int32_t n_m;      /* width of the kernel tables per axis (as wk_mesh.n_m) */
    int32_t n_k;      /* particle momentum window per axis: [M_min, M_min + n_k) */
    int32_t M_min;
    int32_t pos_f64;  /* 1: double positions, 0: float positions */
    int32_t m_bytes;  /* bytes per stored momentum index: 4 = int32 (1-D only), 2 = int16,
                         1 = int8; 0 = the default (4 in 1-D, 2 in 2-D).  Every particle
                         buffer of a call uses that width.  The window widened by the
                         largest pair offset, [M_min - n_m/2, M_min + n_k - 1 + n_m/2],
                         must fit the type (children outside the window are stored, dead,
                         with their momenta); else WK_EINVAL. */
    double vdt;       /* drift per step per unit momentum index, in cells */
    uint64_t seed;    /* Philox key */
} sp_geom;

typedef struct sp_particles {
    void* x;          /* [capacity] float or double */
    void* y;          /* [capacity] (2-D only, else NULL) */
    void* M;          /* [capacity] momentum index (x axis), width per sp_geom.m_bytes */
    void* My;         /* [capacity] y-axis momentum index (2-D only, else NULL), same width */
    int8_t* s;        /* [capacity] */
    int64_t capacity; /* host value: number of slots */
    int64_t* d_n;     /* device int64: current number of particles */
} sp_particles;

/* d_stats: device int64[WK_ST_COUNT].  Each call overwrites only its own entries. */
enum wk_stat {
    WK_ST_N = 0,          /* particles after the call */
    WK_ST_PAIRS = 1,      /* pairs created (sp_step) */
    WK_ST_ABS_X = 2,      /* absorbed at the domain boundary (sp_step) */
    WK_ST_ABS_M = 3,      /* absorbed at the momentum window (sp_step) */
    WK_ST_NEEDED = 4,     /* capacity sp_step needed when it overflowed, else 0 */
    WK_ST_KEPT = 5,       /* particles of single-sign bins kept (sp_annihilate) */
    WK_ST_REGEN = 6,      /* particles regenerated in mixed bins (sp_annihilate) */
    WK_ST_MIXED = 7,      /* bins holding both signs (sp_annihilate) */
    WK_ST_OVERFLOW = 8,   /* sticky: 1 once an overflow happened; later particle calls
                             are then no-ops until the caller clears it */
    WK_ST_OVERFLOW_STEP = 9, /* step index of that overflow */
    /* running sums over calls (the caller zeroes them to start a measurement window) */
    WK_ST_CUM_STEPS = 10,    /* sp_step calls that ran */
    WK_ST_CUM_N = 11,        /* particles at the start of those steps */
    WK_ST_CUM_PAIRS = 12,    /* pairs they created */
    WK_ST_CUM_ANNIH_IN = 13, /* particles entering sp_annihilate */
    WK_ST_CUM_KEPT = 14,     /* particles it kept */
    WK_ST_CUM_REGEN = 15,    /* particles it regenerated */
    WK_ST_COUNT = 16
};

const char* wk_last_error(void);
int wk_version(void);

/* Per-kernel timing for measurement tools.  wk_trace_enable(max) creates 2*max events and
 * from then on brackets each library kernel launch (up to max launches) with events on the
 * launch stream; wk_trace_read(name) synchronises those events and returns the summed
 * duration (ms) and number of launches of kernel `name`; wk_trace_names() writes the
 * traced kernel names, one per line.  Host-side bookkeeping only; results are unchanged. */
int wk_trace_enable(int32_t max_launches);
int wk_trace_disable(void);
int wk_trace_read(const char* name, double* total_ms, int64_t* count);
int wk_trace_names(char* buf, size_t len);
/* Number of HIP devices visible (0 without a GPU); never fails. */
int wk_device_count(void);

/* ------------------------------------------------------------------ Wigner kernel
 * wk_prepare -- set-up for a mesh's n_m on the current device: builds the sine tables of
 * eq.(4) (S[j][m] = sin(2 pi j m / n_m) in the folded, transposed and 16-bit / FP32 forms
 * the 1-D contractions read).  Allocates device memory (kept until the process ends) and
 * synchronises `stream`; a repeated call for the same device and n_m does nothing.  Not
 * needed in 2-D.  Calls on several threads are serialised. */
int wk_prepare(const wk_mesh* mesh, void* stream);

/* wk_kernel_eval -- eq.(4) of Sec. 2.2 (the "N = 1" analytic network of Sec. 2.2):
 *   K(i, m) = -2/(hbar n_m) sum_{j=1..P} sin(2 pi j m / n_m) [V(i+j) - V(i-j)]
 * in 1-D, and its d = 2 form (weights 1/2 at |j_a| = P) in 2-D, evaluated only on the
 * requested cells (the point of the method: no table over the whole phase space).
 *   V       [B][nx] (1-D) or [B][ny][nx] (2-D), double.
 *   cells   [n_cells] int32 cell ids (2-D: iy * nx + ix), or NULL for all cells
 *           (then n_cells must be nx * ny).  An id outside the mesh gives a row of NaN.
 *   prec    enum wk_prec (WK_FP64 .. WK_FP16X3); 2-D supports n_m in {8, 16, 32}.
 *   layout  WK_FULL or WK_HALF (1-D only).
 *   K_out   [B * n_cells][n_m] (full), [B * n_cells][P] (half) or
 *           [B * n_cells][n_m][n_m] (2-D); double for WK_FP64, float otherwise.
 */
int wk_kernel_eval(const wk_mesh* mesh, const double* V, int32_t B, const int32_t* cells,
                   int32_t n_cells, int32_t prec, int32_t layout, void* K_out, void* stream);

/* wk_kernel_bwd -- adjoint of wk_kernel_eval (1-D) with respect to V, on the same rows:
 *   dV[b][l] += sum_{r,t} G[row][t] dK[row][t] / dV[b][l],   row = b * n_cells + r,
 * where K is eq.(4) on cell cells[r] (or r when cells is NULL; then n_cells = nx).  K is
 * linear in V, so this is the exact derivative for any V.
 *   G      [B * n_cells][n_m] (WK_FULL) or [B * n_cells][P] (WK_HALF): double for WK_FP64,
 *          float for WK_FP32 (the product then runs on FP32 MFMA, sums in FP32).
 *   cells  int32 ids in any order, repeats allowed; ids outside [0, nx) contribute nothing.
 *   dV     [B][nx] double, accumulated into (not overwritten).
 *   ws     workspace of wk_kernel_bwd_workspace(mesh, B, n_cells, prec) bytes.
 * Deterministic: fixed-order sums, no floating-point atomics. */
size_t wk_kernel_bwd_workspace(const wk_mesh* mesh, int32_t B, int32_t n_cells, int32_t prec);
int wk_kernel_bwd(const wk_mesh* mesh, const void* G, int32_t B, const int32_t* cells,
                  int32_t n_cells, int32_t prec, int32_t layout, double* dV, void* ws,
                  size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ creation tables
 * wk_gamma_tables -- eq.(1) on the grid and the integer sampling tables of postulate II:
 *   gamma[r] = sum over the row, in ascending m, of max(K, 0)       (FP64, sequential)
 *   p = gamma dt; n0[r] = floor(p); thr[r] = floor((p - n0) 2^32)
 *   cdf[r][t] = floor(C_t / gamma 2^32) with C_t the running positive sum, and 2^32
 *               from the last positive entry on (all 0 when gamma = 0).
 * A particle then creates n0 pairs plus one with probability thr / 2^32, each with
 * momentum offset index min{t : u < cdf[t]} for a uniform 32-bit u.
 *   K      [n_rows][width] full table (width = n_m in 1-D, n_m^2 in 2-D), or the 1-D
 *          half table when layout = WK_HALF; double (k_f64 = 1) or float (k_f64 = 0).
 *   gamma  [n_rows] double, n0/thr [n_rows] uint32, cdf [n_rows][width] uint64. */
int wk_gamma_tables(const wk_mesh* mesh, const void* K, int32_t k_f64, int32_t layout,
                    int32_t n_rows, double dt, double* gamma, uint32_t* n0, uint32_t* thr,
                    uint64_t* cdf, void* stream);

/* wk_sampling_guide -- guide table for the CDF search of sp_step (indexed search, Chen and
 * Asau 1974; an acceleration structure only: sampling results are unchanged):
 *   guide[r][k] = min{t : cdf[r][t] > floor(k 2^32 / guide_len)}  for k < guide_len,
 *   guide[r][guide_len] = width - 1.
 * A draw u then lies in bucket k = floor(u guide_len / 2^32) and its index
 * min{t : u < cdf[r][t]} in [guide[r][k], guide[r][k+1]].
 *   cdf   [n_rows][width] uint64 from wk_gamma_tables.
 *   guide [n_rows][guide_len + 1] uint32 (written). */
int wk_sampling_guide(const uint64_t* cdf, int32_t n_rows, int32_t width, int32_t guide_len,
                      uint32_t* guide, void* stream);

/* wk_kernel_tables -- eq.(4) on the requested cells and, from those rows, the creation tables
 * of eq.(1) and postulate II in one pass: the kernel rows exist only on chip, never in
 * device memory (the paper's point that the kernel need not be stored, Sec. 2.2).
 * The results are bit-identical to wk_kernel_eval in the same precision (any layout)
 * followed by wk_gamma_tables and wk_sampling_guide on the rows it would have written.
 *   V, B, cells, n_cells  as wk_kernel_eval; rows r = b * n_cells + i.
 *   prec   WK_FP64, or one of WK_BF16, WK_FP16, WK_BF16X3, WK_FP16X3 (the 16-bit
 *          contractions of wk_kernel_eval, whose FP32 rows feed the tables), 1-D and 2-D.
 *   dt     time step in fs (p = gamma dt).
 *   gamma  [R] double, n0/thr [R] uint32, cdf [R][width] uint64 (width = n_m in 1-D,
 *          n_m^2 in 2-D), as wk_gamma_tables.
 *   guide  NULL, or [R][guide_len + 1] uint32 as wk_sampling_guide, 1 <= guide_len <= 256.
 * Limits: 1-D 4 <= n_m <= 514, 2-D n_m in {8, 16, 32} (WK_EINVAL otherwise: use the
 * two-step form). */
int wk_kernel_tables(const wk_mesh* mesh, const double* V, int32_t B, const int32_t* cells,
                     int32_t n_cells, int32_t prec, double dt, double* gamma, uint32_t* n0,
                     uint32_t* thr, uint64_t* cdf, uint32_t* guide, int32_t guide_len,
                     void* stream);

/* ------------------------------------------------------------------ particles
 * sp_init -- place the particles of an initial Wigner function given per-bin counts
 * (eq.(6) turned into counts by the caller): for bins in ascending order, count[b]
 * particles of sign +1 with the bin's momentum and positions uniform in the bin's cell.
 * Bins: 1-D b = c * n_k + (M - M_min); 2-D b = ((cy*nx + cx)*n_k + (My-M_min))*n_k + (Mx-M_min).
 *   bin_counts [n_bins] int32 >= 0.  Writes *out->d_n.  WK_ECAPACITY (reported in
 *   d_stats[WK_ST_NEEDED], nothing written) if the total exceeds out->capacity.
 *   ws: sp_workspace_size() bytes. */
size_t sp_workspace_size(const sp_geom* g);
int sp_init(const sp_geom* g, const int32_t* bin_counts, sp_particles* out, int64_t* d_stats,
            void* ws, size_t ws_bytes, void* stream);

/* sp_step -- one time step dt of postulate II (Sec. 2.1) with absorbing boundaries
 * (Sec. 3), from `in` (n particles) to `out`:
 *   1. each particle (index id < n) in a cell with a table row creates
 *      n0 + [u0 < thr] pairs; pair k draws t_k = min{t : u < cdf[t]}, momentum offset
 *      m' = t_k - P (2-D: (t mod n_m - P, t / n_m - P)), and the children
 *      (x, M + m', +s), (x, M - m', -s) go to out at n + 2 * (pairs of lower ids) + 2k, 2k + 1;
 *   2. every particle drifts: x <- fma(M, vdt, x) in the position precision; the parent
 *      goes to out at its own index id;
 *   3. particles leaving [0, nx) (x [0, ny)) or the momentum window get s = 0.
 * Philox counter (id, step, 0, 1) gives u0 and the draws of pairs 0..2; pair k >= 3
 * uses counter (id, step, 1 + (k-3)/4, 1), word (k-3) mod 4.
 *   cell_slot [nx*ny] int32: table row of each cell, or -1 for no creation there.
 *   n0, thr, cdf: from wk_gamma_tables.
 *   guide NULL (plain binary search of the CDF row), or the rows' wk_sampling_guide table
 *         with guide_len buckets; the particles are the same either way.
 *   in, out  distinct buffers; *out->d_n receives n + 2 * pairs.
 *   hist  NULL, or [2][n_bins] int32 that receives the signed histogram of rule 1 (H+ then
 *         H-) of the particles after the step -- the input of the next sp_annihilate,
 *         which then need not build it (hist_ready = 1, or 2 with this same workspace).
 *   hist_mode  how `hist` is cleared first: 0 = every counter; 1 = a promise that the last
 *         call on this workspace that built a 2-D histogram (this step's own kind, or an
 *         annihilation with hist_ready = 0) built the one `hist` holds, unchanged since, so
 *         only the blocks of bins that call marked in the workspace hold counts and only
 *         they are cleared.  1-D histograms are always cleared whole.  Other values:
 *         WK_EINVAL.
 *   keys  NULL, or uint32 [out->capacity] (16-byte aligned; needs hist) that receives each
 *         output particle's histogram key: 2 * bin + 1 for a negative particle, 2 * bin for a
 *         positive one, 0xFFFFFFFF for a particle outside the grid or absorbed.  Handed to
 *         the next sp_annihilate, its counting pass reads them instead of the particles.
 * If out cannot hold n + 2 * pairs particles, d_stats[WK_ST_NEEDED] gets the required
 * capacity, the sticky WK_ST_OVERFLOW flag is set and `out` is invalid; `in` is never
 * written, and because the random stream is counter-based, re-running the step into a
 * larger buffer is bit-identical.
 * ws: sp_workspace_size() bytes (scratch between the launches of one call; calls sharing a
 * workspace must not overlap). */
int sp_step(const sp_geom* g, const int32_t* cell_slot, const uint32_t* n0, const uint32_t* thr,
            const uint64_t* cdf, const uint32_t* guide, int32_t guide_len,
            const sp_particles* in, sp_particles* out, int32_t* hist, int32_t hist_mode,
            uint32_t* keys, int64_t step, int64_t* d_stats, void* ws, size_t ws_bytes,
            void* stream);

/* sp_annihilate -- rule 2 of Sec. 2.1 on the (cell, momentum) grid, from `in` to `out`:
 * output = for each bin holding both signs, in ascending bin order, |H+ - H-| particles of
 * sign sgn(H+ - H-) with the bin's momentum and positions uniform in its cell (Philox
 * counter (bin, step, r/4, 2), word r mod 4 in 1-D; (bin, step, r/2, 2), words 2(r mod 2),
 * 2(r mod 2)+1 for x, y in 2-D), followed by the live particles of bins holding one sign
 * only, unchanged and in input order.
 *   hist [2][n_bins] int32, caller-owned: with hist_ready = 0 it is rebuilt here from
 *   `in`; with hist_ready = 1 it must already hold the histogram of `in` (as sp_step
 *   leaves it, or as the caller wrote it); hist_ready = 2 promises more: the last call on
 *   this same workspace that built a histogram (sp_step with hist, or an annihilation with
 *   hist_ready = 0) built this one, and `hist` is unchanged since.  That call also left in
 *   the workspace a map of the blocks of bins it added counts to, and the annihilation then
 *   reads only those blocks of the histogram (the rest are zero).  Any other value is
 *   refused (WK_EINVAL).  Either way `hist` is left holding H+ then H- of the input: the
 *   signed histogram of rule 1.
 *   keys  NULL, or the keys sp_step wrote for the particles of `in` (16-byte aligned),
 *   unchanged since: the survivor test then reads them instead of the particles.
 * If the output would exceed out->capacity, d_stats gets the needed size, the sticky
 * overflow flag is set and `out` is invalid (`in` is untouched).  The slots of `out` past
 * the output count serve as scratch during the call; their contents are unspecified. */
int sp_annihilate(const sp_geom* g, const sp_particles* in, sp_particles* out, int32_t* hist,
                  int32_t hist_ready, const uint32_t* keys, int64_t step, int64_t* d_stats,
                  void* ws, size_t ws_bytes, void* stream);

/* sp_annihilate_pairs -- rule 2 of Sec. 2.1 read literally, as pair removal: in each
 * (cell, momentum) bin the k-th positive and the k-th negative particle in input order
 * annihilate, for k < min(H+, H-); every other live particle of `in` is kept unchanged (its
 * exact position and momentum), in input order.  No random numbers; net sign per bin is
 * conserved and no bin holds both signs afterwards.  The output histogram equals that of
 * sp_annihilate (which regenerates |H+ - H-| particles of a mixed bin instead).
 *   hist, hist_ready, ws, d_stats as sp_annihilate (WK_ST_REGEN = 0; WK_ST_KEPT = output
 *   count), and as there the slots of `out` past the output count are scratch; out->capacity
 *   >= the input count always suffices.
 *   scratch  caller buffer of sp_pairs_scratch_size(g, in->capacity) bytes (the list of the
 *            particles of mixed bins and its radix-sort buffers, ~17 B per particle slot).
 * Requires 2 * n_bins < 2^32 (WK_EINVAL otherwise).  Calls sharing a workspace or scratch
 * must not overlap. */
size_t sp_pairs_scratch_size(const sp_geom* g, int64_t n_max);
int sp_annihilate_pairs(const sp_geom* g, const sp_particles* in, sp_particles* out, int32_t* hist,
                        int32_t hist_ready, int64_t* d_stats, void* ws, size_t ws_bytes,
                        void* scratch, size_t scratch_bytes, void* stream);

/* sp_density -- rule 1 read-out: rho[c] = sum_M (H+ - H-) / N0 (double [nx*ny]) from the
 * histogram sp_annihilate left in `hist`. */
int sp_density(const sp_geom* g, const int32_t* hist, double N0, double* rho, void* stream);

/* sp_cells_to_evaluate -- the cells that need kernel rows next (Sec. 2.2: the kernel is
 * evaluated only on the phase-space cells the particles occupy): every cell within `margin`
 * cells per axis of a cell holding particles in `hist` (from sp_annihilate) whose
 * cell_slot is still -1, written in ascending order to new_cells [nx*ny] (int32), their
 * number to *d_count (device int64).  ws: sp_workspace_size() bytes.  hist_mode as for
 * sp_step: 1 promises that `hist` is unchanged since the last 2-D histogram build on this
 * workspace, and the cells under no marked block are then not read (2-D). */
int sp_cells_to_evaluate(const sp_geom* g, const int32_t* hist, int32_t hist_mode, int32_t margin,
                         const int32_t* cell_slot, int32_t* new_cells, int64_t* d_count,
                         void* ws, size_t ws_bytes, void* stream);

/* sp_assign_slots -- cell_slot[new_cells[k]] = first_row + k for k < *d_count (device count,
 * at most max_count). */
int sp_assign_slots(const int32_t* new_cells, const int64_t* d_count, int32_t max_count,
                    int32_t first_row, int32_t* cell_slot, void* stream);

/* ------------------------------------------------------------------ learned kernel
 * wk_surrogate_fwd -- the trainable network of eq.(5), Sec. 2.3 (1-D), half table
 * m = 1..P:
 *   Kh(i, m) = prod_{s < log2 N} cos(2^s pi m / n_m)
 *              * sum_{g < n_m/N} W[g] A(i, g) sin(u_g m),
 *   A(i, g) = sum_{p < N} wV[p] V(i + o(g,p)),  u_g = (2 pi / n_m) sum_p wT[p] o(g,p),
 *   o(g, p) = -P + N g + p  (the window offsets of a cell grouped N at a time).
 * With wV = 1, wT = 1/N, W = -2/(hbar n_m): N = 1 is eq.(4) exactly, N = 2 the
 * barycentric form of Sec. 2.3.
 *   N power of two dividing n_m; wV, wT [N] and W [n_m/N] float (device).
 *   prec WK_FP64 (double out, reference arithmetic), WK_FP32 (FP32 MFMA; training) or
 *   WK_BF16 (bf16 products, FP32 accumulate); K_out [B*n_cells][P].
 *   ws   workspace of wk_surrogate_fwd_workspace(mesh, N) bytes (the per-call tables
 *        W[g] sin(u_g m) and the cos prefactor); calls sharing a workspace must not overlap. */
size_t wk_surrogate_fwd_workspace(const wk_mesh* mesh, int32_t N);
int wk_surrogate_fwd(const wk_mesh* mesh, int32_t N, const float* wV, const float* wT,
                     const float* W, const double* V, int32_t B, const int32_t* cells,
                     int32_t n_cells, int32_t prec, void* K_out, void* ws, size_t ws_bytes,
                     void* stream);

/* wk_surrogate_fwd_static -- wk_surrogate_fwd without a workspace argument, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and results as
 * wk_surrogate_fwd; its scratch is a library-owned device array of
 * wk_surrogate_fwd_static_max() bytes (4 MiB; every device the library runs on holds one
 * until the process ends), enough for every supported shape with n_m <= 1024.  Shapes whose scratch
 * (wk_surrogate_fwd_workspace) exceeds it fail with WK_EINVAL.  The call allocates
 * nothing; its first call on a device resolves that device's array address once.  Every
 * call on a GPU shares that GPU's array: calls that overlap on one GPU (two streams, two
 * threads) race and must be serialised by the caller. */
size_t wk_surrogate_fwd_static_max(void);
int wk_surrogate_fwd_static(const wk_mesh* mesh, int32_t N, const float* wV, const float* wT,
                            const float* W, const double* V, int32_t B, const int32_t* cells,
                            int32_t n_cells, int32_t prec, void* K_out, void* stream);

/* wk_surrogate_fwd_2d -- eq.(5) in d = 2 (FP64, forward only): the window of a cell on the
 * periodic grid (offsets o_a in [-P, P) per axis; at the end point -P the mean of the two
 * end values, where the d = 2 kernel of wk_kernel_eval has its half weights), grouped N x N:
 *   Kh(i; mx, my) = prod_s cos(2^s pi mx / n_m) prod_s cos(2^s pi my / n_m)
 *                   * sum_g W[gy H + gx] (sum_p wV[py N + px] Vt(i + o(g, p)))
 *                     * sin(ux(gx) mx + uy(gy) my),
 *   o(g, p) = (-P + N gx + px, -P + N gy + py), ux(gx) = (2 pi / n_m) sum_p wTx[p] (-P + N gx + p)
 *   (uy likewise with wTy), H = n_m / N.
 * With wV = 1, wT = 1/N, W = -2/(hbar n_m^2), N = 1 is the d = 2 kernel exactly.
 *   n_m in {8, 16, 32}; N in {1, 2, 4, 8}, N < n_m; wV [N*N], wTx, wTy [N], W [H*H] float.
 *   K_out [B * n_cells][n_m][n_m] double, (mx, my) = (tx - P, ty - P). */
int wk_surrogate_fwd_2d(const wk_mesh* mesh, int32_t N, const float* wV, const float* wTx,
                        const float* wTy, const float* W, const double* V, int32_t B,
                        const int32_t* cells, int32_t n_cells, double* K_out, void* stream);

/* wk_surrogate_tables_2d -- wk_surrogate_fwd_2d's rows turned straight into the creation tables
 * of eq.(1) and postulate II, the rows never in device memory (the learned kernel in the time
 * loop, Sec. 2.2 and Sec. 4).  Bit-identical to wk_surrogate_fwd_2d followed by
 * wk_gamma_tables (FP64 rows, 2-D) and wk_sampling_guide.
 *   mesh, N, wV, wTx, wTy, W, V, B, cells, n_cells  as wk_surrogate_fwd_2d.
 *   dt, gamma, n0, thr, cdf, guide, guide_len       as wk_kernel_tables (width n_m^2). */
int wk_surrogate_tables_2d(const wk_mesh* mesh, int32_t N, const float* wV, const float* wTx,
                           const float* wTy, const float* W, const double* V, int32_t B,
                           const int32_t* cells, int32_t n_cells, double dt, double* gamma,
                           uint32_t* n0, uint32_t* thr, uint64_t* cdf, uint32_t* guide,
                           int32_t guide_len, void* stream);

/* wk_surrogate_bwd -- gradients of L = sum E * Kh with respect to wV, wT, W (written,
 * float) and V (accumulated into dV [B][nx] double, may be NULL); E [B*n_cells][P] float.
 * Deterministic two-level reductions.  ws: wk_surrogate_workspace() bytes. */
size_t wk_surrogate_workspace(const wk_mesh* mesh, int32_t N, int32_t B, int32_t n_cells);
int wk_surrogate_bwd(const wk_mesh* mesh, int32_t N, const float* wV, const float* wT,
                     const float* W, const double* V, int32_t B, const int32_t* cells,
                     int32_t n_cells, const float* E, float* dwV, float* dwT, float* dW,
                     double* dV, void* ws, size_t ws_bytes, void* stream);

/* wk_mse_grad -- mean squared error of the training loop of Sec. 3, on targets scaled by
 * inv_scale (so that the loss is O(1) whatever the units): with n = count,
 *   loss[0] = sum ((Kh - K) inv_scale)^2 / n            (double, written)
 *   E       = 2 (Kh - K) inv_scale^2 / n = dloss/dKh     (float, written)
 * Kh float, K (labels) double; both [count].  ws: >= 8 KiB of device scratch. */
int wk_mse_grad(const float* Kh, const double* K, int64_t count, double inv_scale, float* E,
                double* loss, void* ws, size_t ws_bytes, void* stream);

/* wk_sgd_update -- w[k] -= lr * grad[k] for k < n (float). */
int wk_sgd_update(float* w, const float* grad, int32_t n, float lr, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* WIGNER_H */
