/*
 * libharp: reduced Macro-Basis-Function array solver with the HARP interaction
 * model (Bui-Van et al., "Fast and Accurate Simulation Technique for Large
 * Irregular Arrays", arXiv 1702.03781), for AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Every pointer named d_* is device memory owned by the caller; every
 * other pointer is host memory owned by the caller.  The library never
 * allocates device memory: calls that need scratch space take a workspace
 * (d_ws, ws_bytes) whose size a *_ws query returns.  All device work is
 * enqueued on the caller's stream and is asynchronous, except where a call
 * says it synchronises.  Argument errors are returned synchronously and
 * nothing is enqueued; numerical outcomes (domain counts, zero pivots,
 * refinement reports) are written to device arrays or, after a documented
 * synchronisation, to host reports.  Nothing throws across this interface.
 *
 * Matrices are column-major with interleaved complex storage (re, im), as
 * complex64 (HARP_C64) or complex128 (HARP_C128); "ld" is the leading
 * dimension in complex elements and "stride" the distance in complex elements
 * between consecutive matrices of a batch.
 *
 * Indexing of the reduced matrix (Section II-A): antenna m carries MBFs
 * T = 0..N_m-1; unknown (m, T) is row/column m * N_m + T.  Entry
 * Z[(m,T),(n,S)] is the reaction of testing MBF T on antenna m with source
 * MBF S on antenna n.
 */
#ifndef HARP_H
#define HARP_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HARP_OK = 0,
    HARP_E_ARG = -1,       /* invalid argument (size, pointer, layout, NaN input) */
    HARP_E_DOMAIN = -2,    /* a pair closer than the model's inner radius r_min */
    HARP_E_SINGULAR = -3,  /* exact zero pivot in the factorisation */
    HARP_E_NOCONV = -4,    /* refinement did not reach its tolerance */
    HARP_E_HIP = -5,       /* a HIP runtime call failed */
    HARP_E_WORKSPACE = -6  /* workspace missing or smaller than the *_ws query */
} harp_status;

typedef enum { HARP_C64 = 0, HARP_C128 = 1 } harp_dtype;

const char *harp_status_str(harp_status s);
/* Library version as major * 10000 + minor * 100 + patch. */
int32_t harp_version(void);

/* ------------------------------------------------------------------------ */
/* Element description                                                       */
/* ------------------------------------------------------------------------ */

/* One antenna type: n_mbf macro basis functions (the "primary and
 * secondaries" MBFs of Section II), each represented by n_samp point-dipole
 * samples.  d_samples is device memory, [n_mbf][n_samp][8] float64 records
 * (x, y, z, ux, uy, uz, a_re, a_im): position in metres relative to the
 * element reference point (which sits at (x_m, y_m, 0) in the array), unit
 * orientation, complex moment in A m.  wire_radius (m) regularises the
 * zero-distance (self) interaction.  The port of the element drives its MBFs
 * with weights w_T = moment of sample 0 of MBF T. */
typedef struct {
    int32_t n_mbf;
    int32_t n_samp;
    const double *d_samples;
    double wire_radius;
} harp_element;

/* ------------------------------------------------------------------------ */
/* HARP model (Section II-A/B, Eqs. 1-4)                                     */
/* ------------------------------------------------------------------------ */

/* A model is one device blob per element and frequency.  Layout (all offsets
 * in bytes from the blob start, each section 256-byte aligned):
 *   [0, 256)    header: uint32 magic 0x50524148, uint32 version 1,
 *               int32 n_mbf, n_samp, P, Q, n_alpha, n_t,
 *               float64 freq_hz, k, omega_mu, r_min, wire_radius,
 *               int64 off_coef, off_coef32, off_self, off_port, off_samples,
 *               total_bytes; zero padding.
 *   off_coef    complex128 C[T][S][p+P][q], p = -P..P, q = 0..Q
 *   off_coef32  complex64 rounding of C (read by the complex64 fill)
 *   off_self    complex128 Z_self[T][S] (zero-distance block)
 *   off_port    complex128 w[T]
 *   off_samples float64 [n_mbf][n_samp][8] copy of the element samples
 * The model evaluates, for a testing antenna at relative position
 * R = r (cos a, sin a) from the source antenna, t = r_min / r:
 *   Z_TS(r, a) = e^{-jkr} sum_{p=-P..P} e^{j p a} sum_{q=0..Q} C_pq t^q
 * which is Eq. (4) with the far-field term of Eq. (1) expanded on the same
 * Fourier basis and folded into q = 1 (1/r = t / r_min). */
size_t harp_model_bytes(int32_t n_mbf, int32_t n_samp, int32_t P, int32_t Q);

harp_status harp_fit_ws(int32_t n_mbf, int32_t n_samp, int32_t P, int32_t Q, int32_t n_alpha,
                        int32_t n_t, size_t *bytes);

/* Build the model of `elem` at freq_hz (Section II-A, Eqs. 1-3, with the
 * Section II-B improvements): exact FP64 reactions on the polar grid
 * a_i = 2 pi i / n_alpha, t_l = l / n_t (l = 1..n_t, r_l = r_min / t_l), the
 * remainder of Eq. (2) after the far field of Eq. (1), a DFT over a for
 * |p| <= P and a Householder least-squares fit over t (including B = 0 at
 * t = 0) for q = 0..Q; plus the zero-distance block with the thin-wire
 * reduced kernel and the port weights.
 * Requirements: n_alpha >= 2P + 1 and even, n_t >= Q, r_min > 0,
 * model_bytes >= harp_model_bytes(...), ws_bytes >= harp_fit_ws(...).
 * Asynchronous on `stream`. */
harp_status harp_fit(const harp_element *elem, double freq_hz, int32_t P, int32_t Q, double r_min,
                     int32_t n_alpha, int32_t n_t, void *d_model, size_t model_bytes, void *d_ws,
                     size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Reduced-matrix fill (Eq. 4)                                               */
/* ------------------------------------------------------------------------ */

/* Fill n_freq reduced matrices of order n = n_ant * n_mbf from n_freq models
 * stored model_stride bytes apart in d_models (all with the given n_mbf and
 * polynomial order Q, harmonic order P <= p_max).  For every ordered pair of
 * antennas m != n the N_m x N_m block is the model at R = (x_m - x_n,
 * y_m - y_n); diagonal blocks are Z_self; when ri > 0, blocks with r > ri
 * are zero (radius of influence, Section II-D).
 *   dtype HARP_C128: FP64 evaluation, d_Z complex128.
 *   dtype HARP_C64 : FP32 evaluation (distance and k r reduced in FP64),
 *                    d_Z complex64.
 *   d_Z32 != NULL: a second complex64 copy in d_Z32 (ld32, stride32): with
 *                    HARP_C128 the FP64 result rounded to complex64, with
 *                    HARP_C64 the same complex64 values as d_Z (so that one
 *                    copy can be factored in place while the other stays
 *                    the matrix a refinement residual is taken against).
 * d_info[f] (int32, device) receives the number of ordered pairs with
 * r < r_min (outside the model; their blocks hold the polynomial continued
 * beyond t = 1), or -1 if model f does not match n_mbf / Q / p_max.
 * Positions d_x, d_y: float64 [n_ant], metres.  Limits: n_mbf <= 64, Q in
 * [2, 8], and the coefficients of one source MBF must fit 64 KB:
 * n_mbf (2 p_max + 1)(Q + 1) x 16 bytes (complex128) or x 8 (complex64)
 * <= 65536; HARP_E_ARG otherwise.  Asynchronous. */
harp_status harp_fill(const void *d_models, int64_t model_stride, int32_t n_freq, int32_t n_mbf,
                      int32_t Q, int32_t p_max, const double *d_x, const double *d_y,
                      int32_t n_ant, double ri, harp_dtype dtype, void *d_Z, int64_t ldz,
                      int64_t stride_z, void *d_Z32, int64_t ld32, int64_t stride32,
                      int32_t *d_info, hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Batches of unequal layouts (many layouts and frequencies reusing one      */
/* model per element and frequency, Section II-D, Section III-C)            */
/* ------------------------------------------------------------------------ */

/* One system of a batch: the layout of n_ant antennas whose positions are
 * x[pos .. pos + n_ant), y[same), evaluated with model blob number `model`;
 * its ports are its first n_ports antennas (0: all n_ant). */
typedef struct {
    int32_t model;
    int32_t n_ant;
    int64_t pos;
    int32_t n_ports;
    int32_t reserved;  /* 0 */
} harp_system;

/* Grouping plan (host only, no device work).  The n_sys systems (antenna
 * counts n_ant[], host) are sorted by size (stable) and cut into contiguous
 * groups; each group is padded to the antenna count of its largest system
 * rounded up to a multiple of pad_multiple, with padded order
 * N = n_pad * n_mbf <= max_order, and holds at most max_batch systems.  The
 * cut minimises the modelled time sum over groups of
 * cost[0] + cost[1] N + cost[2] c N^3 (c systems in the group; cost == NULL
 * takes built-in defaults measured on MI355X).  Outputs (host, caller-owned):
 * order[n_sys] the system indices in group order, group_begin[n_groups + 1]
 * (capacity n_sys + 1) offsets into order, group_pad[n_groups] (capacity
 * n_sys) the padded antenna count, *n_groups.  HARP_E_ARG on a non-positive
 * count or a system whose padded order exceeds max_order. */
harp_status harp_batch_plan(const int32_t *n_ant, int32_t n_sys, int32_t n_mbf, int32_t pad_multiple,
                            int32_t max_order, int32_t max_batch, const double *cost, int32_t *order,
                            int32_t *group_begin, int32_t *group_pad, int32_t *n_groups);

/* harp_fill for a group of n_sys systems (d_sys, device, [n_sys]) padded to
 * n_ant_pad antennas: matrix s (order N = n_ant_pad * n_mbf) holds the Eq. (4)
 * fill of system s in its leading n x n block (n = its n_ant * n_mbf) and the
 * identity in the trailing N - n rows and columns (zeros elsewhere), so that
 * its LU and its solution for right-hand sides padded with zeros are those of
 * the layout, padded.  Model blobs d_models[0 .. n_models), n_pos positions in
 * d_x, d_y.  d_info[s] as for harp_fill, or -2 if descriptor s is out of range
 * (model index, n_ant not in [1, n_ant_pad], positions beyond n_pos; nothing
 * is written to that matrix).  Asynchronous. */
harp_status harp_fill_systems(const void *d_models, int64_t model_stride, int32_t n_models,
                              int32_t n_mbf, int32_t Q, int32_t p_max, const double *d_x,
                              const double *d_y, int64_t n_pos, const harp_system *d_sys,
                              int32_t n_sys, int32_t n_ant_pad, double ri, harp_dtype dtype, void *d_Z,
                              int64_t ldz, int64_t stride_z, void *d_Z32, int64_t ld32,
                              int64_t stride32, int32_t *d_info, hipStream_t stream);

/* harp_port_rhs for a padded group: B_s (complex128, N x n_ports_pad) holds
 * the unit excitation of the system's ports (its model's weights) in its
 * leading n x n_ports block (column j: e_j (x) w) and zeros elsewhere.  A
 * descriptor out of range, or with n_ports beyond n_ant or n_ports_pad, gives
 * zeros. */
harp_status harp_port_rhs_systems(const void *d_models, int64_t model_stride, int32_t n_models,
                                  int32_t n_mbf, const harp_system *d_sys, int32_t n_sys,
                                  int32_t n_ant_pad, int32_t n_ports_pad, void *d_B, int64_t ldb,
                                  int64_t stride_b, hipStream_t stream);

/* harp_port_admittance for a padded group: Y_s (complex128,
 * n_ant_pad x n_ports_pad) = W^T X_s (X_s: N x n_ports_pad) in its leading
 * n_ant x n_ports block (the currents at every port of the system for a unit
 * voltage at each of its excited ports), zeros elsewhere. */
harp_status harp_port_admittance_systems(const void *d_models, int64_t model_stride, int32_t n_models,
                                         int32_t n_mbf, const harp_system *d_sys, int32_t n_sys,
                                         int32_t n_ant_pad, int32_t n_ports_pad, const void *d_X,
                                         int64_t ldx, int64_t stride_x, void *d_Y, int64_t ldy,
                                         int64_t stride_y, hipStream_t stream);

/* Overlapping-subarray tessellation (Section II-D; host only, no device
 * work).  Flat-top regular hexagonal cells of circumradius r_in with centres
 * (ox + 1.5 r_in i, oy + sqrt(3) r_in (j + i / 2)), i, j integers, tile the
 * plane; each antenna (x[], y[], host, n_ant) belongs to the inner part of
 * the cell whose centre is nearest (ties: smallest (i, j)).  The subarray of a
 * cell is every antenna inside the concentric flat-top hexagon of
 * circumradius r_in + r_ext.  Only cells with at least one inner antenna are
 * returned, in (i, j) order.  Outputs (host, caller-owned): *n_cells,
 * *n_members; and when members != NULL: cell_begin[n_cells + 1] (offsets into
 * members), cell_inner[n_cells] (inner antennas of the cell, listed first in
 * ascending order, followed by the cell's other antennas in ascending order),
 * members[n_members], centers[2 n_cells] (x, y).  Call once with
 * members == NULL for the sizes.  HARP_E_ARG on r_in <= 0, r_ext < 0 or
 * non-finite input.  Cost O(n_ant x cells). */
harp_status harp_tessellate(const double *x, const double *y, int32_t n_ant, double r_in, double r_ext,
                            double ox, double oy, int32_t *n_cells, int64_t *n_members,
                            int64_t *cell_begin, int32_t *cell_inner, int32_t *members,
                            double *centers);

/* ------------------------------------------------------------------------ */
/* Ports (Sections I and II-C)                                               */
/* ------------------------------------------------------------------------ */

/* Unit-voltage excitation of every port: B = I_{n_ant} (x) w, complex128
 * n x n_ant per frequency (column j holds w on the rows of antenna j).
 * Asynchronous. */
harp_status harp_port_rhs(const void *d_models, int64_t model_stride, int32_t n_freq,
                          int32_t n_mbf, int32_t n_ant, void *d_B, int64_t ldb, int64_t stride_b,
                          hipStream_t stream);

/* Port admittances Y = W^T X (complex128, n_ant x n_ant per frequency):
 * Y_ij is the current at port i for a unit voltage at port j.  X is
 * complex128 n x n_ant (ldx, stride_x).  n_mbf <= 64 (HARP_E_ARG
 * otherwise).  Asynchronous. */
harp_status harp_port_admittance(const void *d_models, int64_t model_stride, int32_t n_freq,
                                 int32_t n_mbf, int32_t n_ant, const void *d_X, int64_t ldx,
                                 int64_t stride_x, void *d_Y, int64_t ldy, int64_t stride_y,
                                 hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Dense reduced solve (Section I: Gaussian elimination, one RHS per port)   */
/* ------------------------------------------------------------------------ */

/* Kernel tuning per matrix order (process-wide; set it before enqueueing
 * work, not while factorisations or solves are being enqueued on other
 * threads).  An entry applies to orders n <= max_order (entries ascending in
 * max_order); orders above the last entry, or every order with an empty
 * table, take the built-in defaults.  panel_width_c64 / _c128: columns per
 * panel launch of reduced_factor (complex64: 4, 8, or 16 up to order 2048;
 * complex128: 2, 4, or 8 up to order 2048); small_grid_wgs: GEMM launches of
 * the factorisation and the solves whose grid has fewer 64 x 64 tiles than
 * this use 32 x 32 tiles.  harp_set_tuning validates every entry (a width
 * without a launch configuration for the entry's orders is refused) and
 * replaces the table; n_entries = 0 restores the defaults (max 64 entries).
 * harp_default_tuning fills the built-in choice for order n. */
typedef struct {
    int32_t max_order;
    int32_t panel_width_c64;
    int32_t panel_width_c128;
    int32_t small_grid_wgs;
} harp_tuning_entry;

harp_status harp_set_tuning(const harp_tuning_entry *entries, int32_t n_entries);
harp_status harp_get_tuning(harp_tuning_entry *entries, int32_t capacity, int32_t *n_entries);
harp_status harp_default_tuning(int32_t n, harp_tuning_entry *entry);

/* Bytes of the factor auxiliary buffer of reduced_factor / reduced_solve. */
harp_status reduced_factor_ws(int32_t n, int32_t batch, harp_dtype dtype, size_t *bytes);

/* In-place LU factorisation with partial pivoting of `batch` n x n matrices
 * (complex64 or complex128, lda >= n, n <= 8192): blocked right-looking
 * elimination, pivot = first row maximising |Re| + |Im| in the column.  On
 * return the upper triangle holds U and the strict lower triangle the
 * multipliers of L; d_ipiv[b * n + i] (int32, device) is the row exchanged with
 * row i at step i.  The rows are grouped in solve groups of 256: the row
 * exchanges of a group are applied to the multipliers of that group but not to
 * those of earlier groups (the forward solve applies them group by group).
 * d_aux (device, reduced_factor_ws bytes, caller-owned) serves as scratch
 * during the elimination (each 64-column block's inverse unit-lower diagonal
 * block and row-exchange map) and on return holds the inverses of the
 * diagonal 256 x 256 blocks of L and U and each group's row permutation;
 * pass it unchanged to reduced_solve.  d_info[b] = 0, or i + 1 if
 * U(i, i) is exactly zero (the factorisation then continues; a solve with it
 * is meaningless).  Asynchronous. */
harp_status reduced_factor(int32_t n, int32_t batch, harp_dtype dtype, void *d_A, int64_t lda,
                           int64_t stride_a, int32_t *d_ipiv, int32_t *d_info, void *d_aux,
                           size_t aux_bytes, hipStream_t stream);

/* FP64 iterative refinement of a solve whose factors are complex64 (or
 * complex128).  d_report (optional, device, [batch] harp_refine_report,
 * caller-owned) receives the per-system report on the device. */
typedef struct {
    const void *d_Z;     /* matrices the residual is taken against (see z_complex64) */
    int64_t ldz;
    int64_t stride_z;
    double tol;          /* stop when ||B - Z X||_F <= tol ||Z||_F ||X||_F */
    int32_t max_iter;    /* maximum number of correction sweeps (>= 0) */
    void *d_report;      /* optional device copy of the report (NULL: none) */
    int32_t z_complex64; /* 0: d_Z is complex128; 1: d_Z is complex64, each
                            entry widened to FP64 as the residual reads it
                            (the refinement then converges to the solution
                            of that complex64 matrix).  With complex64
                            factors too, the check after the first
                            correction D (complex64, added to X in FP64)
                            updates the residual instead, R - Z D, with
                            complex64 products over at most 16 K slices
                            added in FP64; it counts as converged only when
                            ||R||_F plus the update's error bound
                            (sqrt(2) gamma_{2 Ks + 2} ||Z||_F ||D||_F, Ks
                            the slice length, plus the rounding of X + D)
                            meets the tolerance, and any later check is a
                            full FP64 residual again */
} harp_refine;

typedef struct {
    int32_t iters;       /* correction sweeps applied */
    int32_t converged;   /* 1 if the tolerance was met */
    double resid_rel;    /* last ||B - Z X||_F / (||Z||_F ||X||_F) as computed
                            (for an updated residual: without its bound) */
} harp_refine_report;

harp_status reduced_solve_ws(int32_t n, int32_t nrhs, int32_t batch, harp_dtype dtype,
                             int32_t refine, size_t *bytes);

/* Solve A X = B for `batch` systems with the factors (d_LU, d_ipiv, d_aux) of
 * reduced_factor (dtype as factored): per group of 256 rows, the group's row
 * exchanges, the inverse unit-lower block and the update of the rows below;
 * then per group backwards, the inverse upper block and the update of the rows
 * above, all products on the matrix cores.  B and X are complex128 (n x nrhs).
 * The first forward substitution leaves out the update products of right-hand
 * sides that are still exactly zero (their solution is zero above the first
 * non-zero row of P B: a port excitation touching only its own antenna's rows
 * skips most of them); the result is the same up to the sign of zeros.
 * With refine == NULL, X is the solve in the factor precision.  With refine !=
 * NULL: the residual R = B - Z X is formed in FP64 against refine->d_Z and
 * corrections are solved with the factors and added in FP64, until the
 * tolerance or max_iter sweeps.  The convergence test runs on the device: a
 * system that meets the tolerance (or exhausts max_iter) is skipped by every
 * later kernel.
 *   report != NULL (host, [batch]): the call synchronises the stream once
 *     after the first correction and once after each further sweep while some
 *     system still needs one, fills the report, and returns HARP_E_NOCONV if a
 *     system missed the tolerance.
 *   report == NULL: nothing synchronises (the call may be captured in a HIP
 *     graph); all max_iter sweeps are enqueued, converged systems skipping
 *     them; the report is left on the device (refine->d_report, when given)
 *     and the call returns HARP_OK.
 * Kernels of this call read and write d_ws; concurrent calls need separate
 * workspaces. */
harp_status reduced_solve(int32_t n, int32_t nrhs, int32_t batch, harp_dtype dtype,
                          const void *d_LU, int64_t lda, int64_t stride_lu, const int32_t *d_ipiv,
                          const void *d_aux, size_t aux_bytes, const void *d_B, int64_t ldb, int64_t stride_b, void *d_X, int64_t ldx,
                          int64_t stride_x, const harp_refine *refine,
                          harp_refine_report *report, void *d_ws, size_t ws_bytes,
                          hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture that must not call hipMalloc, tight serving loops, harnesses that
 * forbid allocation): reduced_solve without a workspace argument.  Its
 * scratch (the same layout reduced_solve_ws sizes) lives in a static device
 * array of reduced_solve_noalloc_max_bytes() bytes (64 MiB) that the library
 * holds on every GPU it runs on until the process ends; a call whose
 * reduced_solve_ws size exceeds it returns HARP_E_WORKSPACE and enqueues
 * nothing.  The call allocates nothing (no hipMalloc / hipFree); the first
 * call on a device looks up that device's copy of the array (the device of
 * the caller's stream must be current).  Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (different streams, threads or
 * graphs) race and must be serialised by the caller.  Results, report and
 * synchronisation behaviour are those of reduced_solve. */
size_t reduced_solve_noalloc_max_bytes(void);
harp_status reduced_solve_noalloc(int32_t n, int32_t nrhs, int32_t batch, harp_dtype dtype,
                                  const void *d_LU, int64_t lda, int64_t stride_lu,
                                  const int32_t *d_ipiv, const void *d_aux, size_t aux_bytes,
                                  const void *d_B, int64_t ldb, int64_t stride_b, void *d_X,
                                  int64_t ldx, int64_t stride_x, const harp_refine *refine,
                                  harp_refine_report *report, hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Embedded element patterns (Eqs. 5-6)                                      */
/* ------------------------------------------------------------------------ */

harp_status embedded_patterns_ws(int32_t n_mbf, int32_t n_ant, int32_t n_dir, size_t *bytes);

/* Eqs. (5)-(6): for each of n_ports coefficient columns of d_X (complex128,
 * n x n_ports, ld ldx; e.g. the solution for an excitation of each port) and
 * each direction (theta, phi) (float64 radians, device):
 *   E = -(j omega mu0 / 4 pi) sum_T F_T(u) sum_i X[i N_m + T] e^{jk(u_x x_i + u_y y_i)}
 * projected on theta-hat and phi-hat, with F_T the radiation vector of MBF T
 * (sum over its samples of a s_hat e^{+jk u . rho}; the model blob carries the
 * samples).  The far electric field is E e^{-jkr} / r.  d_E: complex128
 * [n_ports][n_dir][2] (theta, phi).  Needs a workspace of
 * embedded_patterns_ws(...) bytes.  Asynchronous. */
harp_status embedded_patterns(const void *d_model, int32_t n_mbf, const double *d_x,
                              const double *d_y, int32_t n_ant, const void *d_X, int64_t ldx,
                              int32_t n_ports, const double *d_theta, const double *d_phi,
                              int32_t n_dir, void *d_E, void *d_ws, size_t ws_bytes,
                              hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Adjoint with respect to the antenna positions (array synthesis)          */
/* ------------------------------------------------------------------------ */
/* Convention: a cotangent G of a complex output Z is the array with
 * dJ = Re sum conj(G) dZ for a real objective J (PyTorch's complex autograd
 * convention).  Position gradients are float64 [n_ant] and are accumulated
 * (+=) into the caller's arrays.  The solve's adjoint reuses the factors of
 * reduced_factor: Z is complex-symmetric (reciprocity), so Z^-H G =
 * conj(Z^-1 conj(G)). */

/* D = beta C + alpha A B for `batch` column-major complex matrices (complex64
 * or complex128, interleaved; alpha, beta real; D may alias C; C may be null
 * when beta = 0), on the matrix cores.  Strides in complex elements.
 * Asynchronous. */
harp_status harp_cgemm(harp_dtype dtype, int32_t M, int32_t N, int32_t K, int32_t batch, double alpha,
                       const void *d_A, int64_t lda, int64_t stride_a, const void *d_B, int64_t ldb,
                       int64_t stride_b, double beta, const void *d_C, int64_t ldc, int64_t stride_c,
                       void *d_D, int64_t ldd, int64_t stride_d, hipStream_t stream);

/* dst = op(src) for `batch` complex128 matrices of rows x cols (column-major,
 * leading dimensions lds / ldd, batch strides in elements): op transposes
 * when `transpose` != 0 (dst is then cols x rows) and conjugates when `conj`
 * != 0.  In place only without transposition.  Asynchronous. */
harp_status harp_cmatrix_copy(int32_t rows, int32_t cols, int32_t batch, const void *d_src, int64_t lds,
                              int64_t stride_src, void *d_dst, int64_t ldd, int64_t stride_dst,
                              int32_t transpose, int32_t conj, hipStream_t stream);

/* Cotangent of X through the port admittances Y = W^T X:
 * gX[(i,T), q] = conj(w_T) gY[i, q] (complex128; overwrites gX). */
harp_status harp_port_admittance_vjp(const void *d_models, int64_t model_stride, int32_t n_freq,
                                     int32_t n_mbf, int32_t n_ant, const void *d_gY, int64_t ldy,
                                     int64_t stride_y, void *d_gX, int64_t ldx, int64_t stride_x,
                                     hipStream_t stream);

/* Workspace bytes of harp_fill_vjp. */
harp_status harp_fill_vjp_ws(int32_t n_ant, size_t *bytes);

/* Eq. (4) differentiated with respect to the positions (Sections II-A/B: the
 * modified coordinates t = r_min / r and alpha of every pair): for one model
 * (one frequency), gx_i += Re sum_ab W_ab dZ_ab/dx_i and likewise for y, over
 * the ordered pairs with r <= ri (ri <= 0: all); W (complex128, n x n, ld ldw)
 * plays the role of conj of the cotangent of Z.  Q must equal the model's Q;
 * d_info (int32, device) is set to -1 when the model does not match.
 * Deterministic (fixed-order reductions).  Asynchronous. */
harp_status harp_fill_vjp(const void *d_model, int32_t n_mbf, int32_t Q, const double *d_x,
                          const double *d_y, int32_t n_ant, double ri, const void *d_W, int64_t ldw,
                          double *d_gx, double *d_gy, int32_t *d_info, void *d_ws, size_t ws_bytes,
                          hipStream_t stream);

/* Workspace bytes of embedded_patterns_vjp. */
harp_status embedded_patterns_vjp_ws(int32_t n_mbf, int32_t n_ant, int32_t n_dir, int32_t n_ports,
                                     size_t *bytes);

/* Eqs. (5)-(6) differentiated: for the cotangent gE of the patterns
 * (complex128 [n_ports][n_dir][2], as produced by embedded_patterns), adds
 * A^H gE to gX (complex128 n x n_ports, ld ldgx; A the pattern operator
 * E = A X) and the explicit dependence of the array phase on the positions
 * to gx, gy.  Asynchronous. */
harp_status embedded_patterns_vjp(const void *d_model, int32_t n_mbf, const double *d_x, const double *d_y,
                                  int32_t n_ant, const void *d_X, int64_t ldx, int32_t n_ports,
                                  const double *d_theta, const double *d_phi, int32_t n_dir,
                                  const void *d_gE, void *d_gX, int64_t ldgx, double *d_gx, double *d_gy,
                                  void *d_ws, size_t ws_bytes, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* HARP_H */
