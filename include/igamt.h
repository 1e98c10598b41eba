/*
 * igamt -- interpolation-and-lookup assembly of isogeometric stiffness matrices
 * for microstructured geometries built by spline composition, on AMD MI355X
 * (gfx950).  Method: Hirschler, Antolin, Buffa, "Fast and multiscale formation
 * of isogeometric matrices of microstructured geometric models".
 *
 * C ABI.  Plain pointers and sizes only.  Conventions for every entry point:
 *   - Return value: IGAMT_OK (0) or a negative igamt_status.  No C++ exception
 *     crosses the boundary.  igamt_last_error() returns a description of the
 *     last failure on the calling thread.
 *   - "host" pointers are read during the call only; the plan keeps copies.
 *   - "device" pointers are caller-owned device memory on the plan's device
 *     (the device current at the first device call on the plan); the library
 *     never frees them.
 *   - stream is a hipStream_t (NULL = the default stream).  Device work is
 *     queued asynchronously on it unless a function says it synchronises.
 *   - Index conventions (tile-local and global) are stated in each comment;
 *     "x fastest" means flat = i + n_x (j + n_y k).
 */
#ifndef IGAMT_H
#define IGAMT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t igamt_status;
#define IGAMT_OK            0
#define IGAMT_EINVAL       -1  /* invalid argument (knots, sizes, NaN, NULL) */
#define IGAMT_ENOMEM       -2  /* device or host allocation failed */
#define IGAMT_EDEGENERATE  -3  /* det J <= 0 (or not finite) at a fit/quadrature point */
#define IGAMT_EHIP         -4  /* a HIP runtime call failed */
#define IGAMT_ESHAPE       -5  /* buffer size does not match the plan */
#define IGAMT_EUNSUPPORTED -6  /* valid input outside what this build implements */
#define IGAMT_ESTATE       -7  /* call order violated (e.g. assemble before tables exist) */

/* Arithmetic of the contraction (eq. (58)).  The fit is FP64 in every mode.
 * F64     : FP64 operands, FP64 MFMA, FP64 output.
 * F32     : FP32 operands, FP32 MFMA, FP32 output.
 * BF16X3  : x = hi + lo in bfloat16 for table and coefficients, products
 *           hi*hi + hi*lo + lo*hi, FP32 accumulation and output.
 * F16X3   : the same in float16 with a power-of-two scale per table row and
 *           per coefficient column, FP32 accumulation and output.            */
typedef enum { IGAMT_F64 = 0, IGAMT_F32 = 1, IGAMT_BF16X3 = 2, IGAMT_F16X3 = 3 } igamt_precision;

typedef struct igamt_plan igamt_plan;

/* Trivariate B-spline or NURBS (eq. (1)-(4)).  host memory.
 * knots[k]: n_ctrl[k] + degree[k] + 1 values, clamped (first and last
 * degree+1 values equal), non-decreasing, spanning [0, 1].
 * ctrl: [n_ctrl[2]][n_ctrl[1]][n_ctrl[0]][3], x fastest.
 * weights: NULL for a B-spline; else [n_ctrl[2]][n_ctrl[1]][n_ctrl[0]]
 *   positive NURBS weights (rational basis w_i N_i / sum_j w_j N_j).  Accepted
 *   for the macro map by every entry point (the shape gradients differentiate
 *   with respect to the control points, weights fixed); the tile must be a
 *   B-spline (IGAMT_EUNSUPPORTED).                                            */
typedef struct {
  int32_t degree[3];
  int32_t n_ctrl[3];
  const double *knots[3];
  const double *ctrl;
  const double *weights;
} igamt_spline3d;

/* Tile grid and method parameters.
 * tiles[k]  : tiles per direction.  box_mode 0: tile i is the i-th non-empty
 *             knot span of the macro map (eq. (5)-(8)), so tiles[k] must equal
 *             the number of non-empty spans.  box_mode 1: uniform boxes of
 *             size 1/tiles[k] in the macro parameter domain.
 * q         : projection degree p_pi (eq. (21)), 0..6.
 * n_fit     : Gauss-Legendre samples per direction for the projection,
 *             >= q + 1 (q + 1 = interpolation at the Gauss nodes, which equals
 *             the discrete L2 projection of eq. (23)-(24) with that rule).
 * n_gauss   : Gauss-Legendre points per direction per micro element for the
 *             lookup table (eq. (52)), 1..8.
 * anisotropic, q_dir[3]: with anisotropic != 0, the projection degrees per
 *             direction (Section 3.3.4), each 0..6 (q is then ignored);
 *             n_pi = prod_k (q_k + 1) and n_fit >= max_k q_k + 1 (a
 *             least-squares fit in the directions of lower degree).  With
 *             anisotropic = 0, q in every direction and q_dir is not read.
 *             Every entry point takes plans whose degrees differ per direction. */
typedef struct {
  int32_t tiles[3];
  int32_t box_mode;
  int32_t q;
  int32_t n_fit;
  int32_t n_gauss;
  int32_t anisotropic;
  int32_t q_dir[3];
} igamt_plan_desc;

/* Sizes derived from a plan. */
typedef struct {
  int64_t n_tiles;        /* m_M */
  int64_t n_tiles_pad;    /* m_M rounded up to a multiple of 16 */
  int64_t n_pairs;        /* n_nz = |I_coo| (eq. (56)), rows of the table */
  int64_t n_cols;         /* 9 (q+1)^3, columns of the table (eq. (57)) */
  int64_t n_cols_pad;     /* n_cols rounded up to a multiple of 64 */
  int64_t n_tile_ctrl;    /* n_T */
  int64_t n_macro_ctrl;   /* macro control points */
  int64_t n_global_ctrl;  /* global control points after gluing tiles */
  int64_t n_dofs;         /* 3 n_global_ctrl */
  int64_t nnz;            /* CSR entries, both triangles */
} igamt_sizes;

const char *igamt_last_error(void);

/* --- plan (host integer setup; no device work) ---------------------------
 * Validates both splines and the descriptor, computes tile boxes, the pair
 * set I_coo (eq. (56): A <= B in tile-local x-fastest order, supports sharing
 * a micro element, sorted by (A, B)), the glued global numbering
 * G = (t_x (n_x-1) + i, t_y (n_y-1) + j, t_z (n_z-1) + k) x fastest, dof 3 G + a,
 * and the CSR structure (full symmetric, sorted columns).
 * Tile knots must have no repeated interior knot (IGAMT_EUNSUPPORTED), tile
 * boundary control points must sit at the identity (Greville) positions so
 * that tiles conform (IGAMT_EINVAL otherwise).  *out is owned by the caller
 * and released with igamt_plan_destroy.                                     */
igamt_status igamt_plan_create(const igamt_spline3d *macro, const igamt_spline3d *tile,
                               const igamt_plan_desc *desc, igamt_plan **out);
void igamt_plan_destroy(igamt_plan *plan);                       /* NULL-safe */
igamt_status igamt_plan_sizes(const igamt_plan *plan, igamt_sizes *out);
/* I_coo as host int32 [n_pairs][2]. */
igamt_status igamt_plan_pairs(const igamt_plan *plan, int32_t *pairs);
/* CSR structure into host buffers row_ptr int64 [n_dofs + 1], col_idx int32 [nnz]. */
igamt_status igamt_plan_csr(const igamt_plan *plan, int64_t *row_ptr, int32_t *col_idx);
/* The same CSR structure generated on the device (bit-identical). */
igamt_status igamt_plan_csr_device(igamt_plan *plan, int64_t *d_row_ptr, int32_t *d_col_idx, void *stream);

/* --- design updates (same topology) ------------------------------------------
 * New macro control points [n_ctrl z][y][x][3], from host (on_device = 0) or
 * device memory (on_device = 1).  The plan's device copy of the control points
 * is the current one: every kernel reads it, and nothing is uploaded again
 * from the host copy once the first call has placed the plan on the device (a
 * device-side set leaves the host copy behind, unused).  Host input must be
 * finite (IGAMT_EINVAL); device input is queued unchecked, and a non-finite
 * point shows up as a degenerate Jacobian (the flag igamt_check reports).     */
igamt_status igamt_set_macro_ctrl(igamt_plan *plan, const double *ctrl, int32_t on_device, void *stream);
/* New reference-tile control points (host), same knots; tables must be rebuilt.
 * Boundary points must stay at their Greville positions (IGAMT_EINVAL).       */
igamt_status igamt_set_tile_ctrl(igamt_plan *plan, const double *ctrl);
/* The same from device memory (double [n_z][n_y][n_x][3]), queued on the
 * stream; the boundary check runs on the device and a violation is reported
 * by the next igamt_check (IGAMT_EINVAL).                                     */
igamt_status igamt_set_tile_ctrl_device(igamt_plan *plan, const double *d_ctrl, void *stream);

/* --- lookup tables (eq. (52), (57)) ------------------------------------------
 * Table layout (row-major): table[p][9 C + 3 i + j], p = pair index, C =
 * c1 + (q+1)(c2 + (q+1) c3) the Bernstein index, i, j the derivative
 * directions.  tables_build integrates eq. (52) on the device in FP64 with
 * n_gauss points per direction per micro element.  tables_set / tables_get
 * copy a caller device buffer double [n_pairs][n_cols].  After build or set,
 * the FP32 and split BF16 / F16 copies used by the other precisions are
 * derived on the device.                                                      */
igamt_status igamt_tables_build(igamt_plan *plan, void *stream);
/* tables_build whose kernels do nothing unless *d_gate != 0 (int32 on the
 * device), so that a decision taken on the device (igamt_table_rows_check)
 * selects the exact table without a host round trip.  The plan must already
 * hold a table (built, set or reconstructed), which is kept when the gate is 0. */
igamt_status igamt_tables_build_gated(igamt_plan *plan, const int32_t *d_gate, void *stream);
igamt_status igamt_tables_set(igamt_plan *plan, const double *d_table, void *stream);
igamt_status igamt_tables_get(const igamt_plan *plan, double *d_out, void *stream);
/* Exact FP64 table rows for the listed pair indices (device int32 [n_rows]) into
 * d_out double [n_rows][n_cols]; used to estimate the error of a learned table. */
igamt_status igamt_tables_build_rows(igamt_plan *plan, const int32_t *d_rows, int32_t n_rows,
                                     double *d_out, void *stream);

/* --- the assembly path -----------------------------------------------------
 * Workspace sizes (bytes) for the stage buffers of a precision:
 *   coef  : the fitted coefficients in the contraction layout (below);
 *   blocks: per-tile stiffness blocks, [n_tiles][n_pairs][9] of double (F64)
 *           or float (other modes), entry [t][p][3 a + b] = K^(t)[(A,a),(B,b)]
 *           for (A, B) = pairs[p].                                             */
igamt_status igamt_workspace_bytes(const igamt_plan *plan, igamt_precision prec,
                                   int64_t *coef_bytes, int64_t *blocks_bytes);

/* Stage 1, the fit (Section 3.2.2, eq. (37), (42)): for every tile and every
 * Gauss sample, J = J_M(a + h xi) diag(h), F = J^-1, D = det J and
 * A_ij,ab = D (lam F_ia F_jb + mu (F_i . F_j) delta_ab + mu F_ib F_ja), then the
 * Bernstein coefficients <A_ij,ab>_C.  lam, mu from E, nu (3-D isotropic).
 * d_coef layout (element type by precision): column-major per tile,
 *   F64 : double [n_tiles_pad][9 (a,b)][n_cols_pad (9C+3i+j)]
 *   F32 : float  [same]
 *   BF16X3: hi then lo, each uint16 (bfloat16 bits) [same]
 *   F16X3 : hi then lo, each uint16 (float16 bits) [same], then float
 *           inv_scale [n_tiles_pad][9]; hi + lo = coefficient / inv_scale with
 *           inv_scale a power of two chosen per column.
 * Padding tiles and columns are written as zeros.  A det J <= 0 raises the
 * plan's degeneracy flag (reported by igamt_check).                          */
igamt_status igamt_fit(igamt_plan *plan, double E, double nu, igamt_precision prec,
                       void *d_coef, void *stream);
/* Stage 2, the contraction of eq. (58) on MFMA: blocks[t][p][ab] =
 * sum_k table[p][k] coef[t][ab][k].  Requires tables (ESTATE otherwise).     */
igamt_status igamt_contract(igamt_plan *plan, igamt_precision prec, const void *d_coef,
                            void *d_blocks, void *stream);
/* Ablations of the BF16 split contraction (precision study, not a production
 * path): on the coefficients igamt_fit writes for IGAMT_BF16X3 (hi and lo
 * planes), FP32 blocks as igamt_contract writes them, with
 *   products = 3: lo*hi + hi*lo + hi*hi (what IGAMT_BF16X3 computes);
 *   products = 2: the table split only, the coefficients rounded once to BF16
 *                 (lo*hi + hi*hi; the lo plane of the coefficients is ignored);
 *   products = 4: all four products (lo*lo added).
 * Requires tables (IGAMT_ESTATE) and a padded table width of 128 or 256
 * columns (q <= 2 isotropic; IGAMT_EUNSUPPORTED otherwise); IGAMT_EINVAL for
 * other product counts.                                                      */
igamt_status igamt_contract_products(igamt_plan *plan, int32_t products, const void *d_coef, void *d_blocks,
                                     void *stream);
/* Stage 3, deterministic scatter into the fixed CSR structure (step 4 of
 * Section 3.2.4): value(3 G_A + a, 3 G_B + b) = sum over the tiles that hold both
 * control points, in ascending tile index, of the block entry ((A,B) upper
 * pair: [p][3a+b]; lower: [p(B,A)][3b+a]).  d_values double (F64) or float. */
igamt_status igamt_scatter(igamt_plan *plan, igamt_precision prec, const void *d_blocks,
                           void *d_values, void *stream);
/* All three stages in turn on `stream`; d_workspace must hold coef_bytes +
 * blocks_bytes (256-byte aligned sub-buffers, coef first).  The result is
 * bitwise the same as the three stage calls.  Calls on one plan from
 * different streams must be ordered by the caller.                            */
igamt_status igamt_assemble(igamt_plan *plan, double E, double nu, igamt_precision prec,
                            void *d_values, void *d_workspace, void *stream);
/* Synchronises the stream and reports a degenerate tile seen since the last
 * check (IGAMT_EDEGENERATE, *bad_tile = smallest tile index) or IGAMT_OK.   */
igamt_status igamt_check(igamt_plan *plan, void *stream, int64_t *bad_tile);

/* --- sensitivities (Section 4.1.2, eq. (69)-(73)) ----------------------------
 * d(u^T K^pi u)/d m for every macro control point m (u fixed), FP64 fit and
 * fit-adjoint, contraction in FP64 (F64) or FP32 (F32).  Per tile the adjoint
 * field W = table^T U, U[p][ab] = m_p u_(A,a) u_(B,b) (m_p = 2 if A < B else 1),
 * is paired with dA/dm.  With u = K^-1 f and f independent of m, the
 * compliance gradient is minus this.  d_u double [n_dofs]; d_grad double
 * [n_macro_ctrl][3] (z, y, x order as ctrl); d_uKu double [1] (may be NULL).
 * d_workspace: igamt_grad_workspace_bytes.                                   */
igamt_status igamt_grad_workspace_bytes(const igamt_plan *plan, igamt_precision prec, int64_t *bytes);
igamt_status igamt_uKu_grad(igamt_plan *plan, double E, double nu, igamt_precision prec,
                            const double *d_u, double *d_grad, double *d_uKu,
                            void *d_workspace, void *stream);

/* Sparse matrix-vector product y = K x for the CSR produced above (support
 * routine: rigid-mode checks, iterative solves).  F64: double values/x/y;
 * F32: float.                                                                 */
igamt_status igamt_spmv(igamt_precision prec, int64_t n_rows, const int64_t *d_row_ptr,
                        const int32_t *d_col_idx, const void *d_values, const void *d_x,
                        void *d_y, void *stream);

/* --- learned tables ------------------------------------------------------------
 * POD basis of a set of tables (not in the paper; replaces one table build per
 * design of a parameterised tile family).  d_snap double [n_s][n_e] (n_e =
 * n_pairs * n_cols, row-major tables).  Computes the mean, the Gram matrix of
 * the centred snapshots (FP64, device), its eigenpairs (host: Householder
 * tridiagonalisation, then implicit QR steps with Wilkinson shifts; an
 * iteration that does not converge within 64 n_s steps returns
 * IGAMT_EDEGENERATE), and the r leading modes.  Outputs: d_mean float [n_e], d_basis float
 * [r][n_e] (orthonormal rows), h_sigma double [n_s] singular values
 * (descending), h_coeffs double [n_s][r] (may be NULL): the coefficients of
 * each centred snapshot in the basis (= V Sigma).  d_work double:
 * 17 n_s^2 + n_s r + n_e.  Synchronises the stream.                           */
igamt_status igamt_pod_build(const double *d_snap, int32_t n_s, int64_t n_e, int32_t r,
                             float *d_mean, float *d_basis, double *h_sigma, double *h_coeffs,
                             double *d_work, void *stream);
/* Table of a design from POD coefficients: table = mean + basis^T (scale c)
 * (FP32 mean/basis/coefficients d_coeffs [r], r <= 256, reconstructed in FP64
 * into the plan's table, then the precision copies are derived).             */
igamt_status igamt_table_from_pod(igamt_plan *plan, const float *d_mean, const float *d_basis,
                                  int32_t r, const float *d_coeffs, double coeff_scale, void *stream);
/* Relative Frobenius error of the plan's current table on listed rows against
 * exact rows (d_exact double [n_rows][n_cols]); result to d_err double [1].   */
igamt_status igamt_table_rows_error(const igamt_plan *plan, const int32_t *d_rows, int32_t n_rows,
                                    const double *d_exact, double *d_err, void *stream);
/* The same error, plus a decision for igamt_tables_build_gated: d_gate int32 [1]
 * is set to 0 when the error is <= tol and to 1 otherwise (also for NaN).    */
igamt_status igamt_table_rows_check(const igamt_plan *plan, const int32_t *d_rows, int32_t n_rows,
                                    const double *d_exact, double tol, double *d_err, int32_t *d_gate,
                                    void *stream);

/* Multilayer perceptron x -> GELU(x W1 + b1) -> ... -> x W_L + b_L (no
 * activation on the last layer), GELU(z) = 0.5 z (1 + erf(z / sqrt 2)).
 * Parameters are one flat float buffer [W1 (in x out, row-major), b1, W2, b2,
 * ...].  widths[0..n_layers] are the layer sizes.  Activations buffer d_act
 * float: batch * (sum of widths[1..n_layers]) pre-activations, written by
 * forward and read by backward.  All float32.                                 */
typedef struct {
  int32_t n_layers;
  int32_t widths[9];
  int32_t batch;
} igamt_mlp_desc;
int64_t igamt_mlp_n_params(const igamt_mlp_desc *desc);
igamt_status igamt_mlp_forward(const igamt_mlp_desc *desc, const float *d_params, const float *d_x,
                               float *d_act, float *d_y, void *stream);
/* Mean-squared error L = mean((y - t)^2) over batch x outputs; writes dL/dy
 * (float [batch][out]) and L (float [1]).                                    */
igamt_status igamt_mse_loss(const igamt_mlp_desc *desc, const float *d_y, const float *d_target,
                            float *d_dy, float *d_loss, void *stream);
/* Gradients of all parameters (flat, same layout as d_params) given dL/dy.
 * d_scratch float: 2 * batch * max(widths).                                  */
igamt_status igamt_mlp_backward(const igamt_mlp_desc *desc, const float *d_params, const float *d_x,
                                const float *d_act, const float *d_dy, float *d_grads,
                                float *d_scratch, void *stream);
/* Adam with bias correction, in place on d_params, d_m, d_v (float [n]). */
igamt_status igamt_adam_step(float *d_params, const float *d_grads, float *d_m, float *d_v, int64_t n,
                             float lr, float beta1, float beta2, float eps, int32_t step, void *stream);

/* The whole learned-table step for one design, queued on the stream with no host
 * synchronisation: MLP forward (desc->batch = 1, d_x the scaled parameters
 * [1][n_in], d_act / d_y its workspace and output [1][r]), POD reconstruction
 * into the plan's table (as igamt_table_from_pod with the MLP output as
 * coefficients), exact rebuild of the check rows (as igamt_tables_build_rows,
 * into d_exact_rows double [n_rows][n_cols]), their error and gate (as
 * igamt_table_rows_check), and the exact table in place of the learned one when
 * the gate is set (as igamt_tables_build_gated).  The tile control points of the
 * design must have been set before.                                           */
igamt_status igamt_table_learned(igamt_plan *plan, const igamt_mlp_desc *desc, const float *d_params,
                                 const float *d_x, float *d_act, float *d_y, const float *d_mean,
                                 const float *d_basis, double coeff_scale, const int32_t *d_rows,
                                 int32_t n_rows, double *d_exact_rows, double tol, double *d_err,
                                 int32_t *d_gate, void *stream);

/* --- load vector (Section 3.2.2-3.2.3, eq. (39)-(41), (44)-(45), (53)-(55)) --
 * External loads: a constant body force b (3 doubles, force per unit volume)
 * and a constant traction t_f on each of the six macro faces f = 2 d + side
 * (xi_d = 0 for side 0, xi_d = 1 for side 1; 18 doubles, force per unit area;
 * zeros where there is none).  Host arrays, read during the call.
 *
 * igamt_load_table_build: the lookup table of eq. (54)-(55) for the plan's tile,
 *   F[A][C][0] = int R_A N_C (volume) and F[A][C][1 + f] = int over tile face f
 *   of R_A N_C, kept on the device; rebuild after igamt_set_tile_ctrl.
 * igamt_load_table_get: copy it to d_out double [n_tile_ctrl][n_pi][7].
 * igamt_load_fit: the projection coefficients of bbar = b |det J_M| (eq. (40),
 *   (44)) and, on the macro faces a tile touches, of tbar_f = t_f times the
 *   face's area element (eq. (41), (45), (87)-(88)) into d_coef double
 *   [n_tiles][7][3][n_pi] (slot 0 the body, 1 + f face f; zero where a tile
 *   does not touch f).  A det J <= 0 at a sample raises the degeneracy flag.
 * igamt_load_gather: f[3 G + a] = sum over the tiles holding G, in ascending
 *   tile index, of sum_slot sum_C coef[t][slot][a][C] F[A][C][slot] (eq. (53)),
 *   into d_f double [n_dofs]; every entry is written, bitwise reproducibly.
 * igamt_load_assemble: fit then gather, with d_workspace of
 *   igamt_load_workspace_bytes holding the coefficients.                      */
igamt_status igamt_load_table_build(igamt_plan *plan, void *stream);
igamt_status igamt_load_table_get(const igamt_plan *plan, double *d_out, void *stream);
igamt_status igamt_load_workspace_bytes(const igamt_plan *plan, int64_t *bytes);
igamt_status igamt_load_fit(igamt_plan *plan, const double *body, const double *traction, double *d_coef,
                            void *stream);
igamt_status igamt_load_gather(igamt_plan *plan, const double *d_coef, double *d_f, void *stream);
igamt_status igamt_load_assemble(igamt_plan *plan, const double *body, const double *traction, double *d_f,
                                 void *d_workspace, void *stream);

/* Shape derivative of the external work (Section 4.1.2, eq. (69), through the
 * load projections of eq. (40)-(41), (44)-(45) and the lookup of eq. (53)):
 * d(u . f^pi)/d m for every macro control point m, u fixed, f^pi the load vector
 * igamt_load_assemble computes for the same body force and tractions (host
 * arrays as there).  Its body term carries |det J_M| and its face terms the face
 * area element, both of which move with m; with u = K^-1 f the compliance
 * c = f^T K^-1 f has dc/dm = 2 d(u . f)/dm - d(u^T K u)/dm.  FP64 throughout.
 * d_u double [n_dofs]; d_grad double [n_macro_ctrl][3] (z, y, x order as ctrl);
 * d_uf double [1] receives u . f^pi (may be NULL).  d_workspace:
 * igamt_uf_grad_workspace_bytes (per-tile local gradients and shares, reduced
 * over the tiles in a fixed order: bitwise reproducible).  Needs the load table
 * (igamt_load_table_build); IGAMT_ESTATE otherwise.  A det J <= 0 at a sample
 * raises the degeneracy flag.  NURBS maps: weights held fixed.               */
igamt_status igamt_uf_grad_workspace_bytes(const igamt_plan *plan, int64_t *bytes);
igamt_status igamt_uf_grad(igamt_plan *plan, const double *body, const double *traction, const double *d_u,
                           double *d_grad, double *d_uf, void *d_workspace, void *stream);

/* --- matrix-free product (Section 4.2, eq. (74)) ------------------------------
 * y = K u for the full symmetric stiffness matrix K (the CSR matrix igamt_assemble
 * would produce), as the sum over tiles of K^(t) u^(t) glued at shared control
 * points, without the global matrix.  d_u and d_y are double [n_dofs] (dof
 * 3 G + a) on the device; every entry of d_y is written.  The tile products
 * accumulate in FP64 from blocks in the precision's storage type (double for
 * IGAMT_F64, float otherwise); per dof, the tiles are summed in ascending tile
 * index: no atomics, bitwise reproducible.  Tiles with more control points than
 * the kernel's LDS holds (about 700 for FP64 blocks) give IGAMT_EUNSUPPORTED.
 *
 * igamt_linop_workspace_bytes: workspace of igamt_apply_blocks (slab_tiles = 0:
 *   the tile products, 24 n_tile_ctrl bytes per tile) or of igamt_linop
 *   (slab_tiles > 0, a multiple of 16: the tile products plus the blocks of one
 *   slab of slab_tiles tiles); IGAMT_EINVAL for other slab_tiles.
 * igamt_apply_blocks: from the tile blocks of igamt_contract in d_blocks
 *   [n_tiles][n_pairs][9] (the matrix is formed once, then applied many times).
 * igamt_linop: on the fly, from the table and the projection coefficients of
 *   igamt_fit (d_coef) only: per slab of slab_tiles tiles, the contraction of
 *   eq. (58) into the workspace, then the slab's tile products; the tile
 *   matrices of the whole mesh never exist at once.  Requires tables
 *   (IGAMT_ESTATE).  The result equals igamt_apply_blocks on the blocks of
 *   igamt_contract bit for bit, whatever the slab size.                       */
igamt_status igamt_linop_workspace_bytes(const igamt_plan *plan, igamt_precision prec, int64_t slab_tiles,
                                         int64_t *bytes);
igamt_status igamt_apply_blocks(igamt_plan *plan, igamt_precision prec, const void *d_blocks, const double *d_u,
                                double *d_y, void *d_workspace, void *stream);
igamt_status igamt_linop(igamt_plan *plan, igamt_precision prec, int64_t slab_tiles, const void *d_coef,
                         const double *d_u, double *d_y, void *d_workspace, void *stream);

/* --- Krylov solve (eq. (30) with the product of eq. (74), Section 4.2) ---------
 * K u = f with homogeneous Dirichlet conditions: d_fixed uint8 [n_dofs], 1 on
 * clamped dofs (u = 0 there), 0 on free ones; K_ff must be positive definite
 * (at least one clamped face).  Jacobi-preconditioned conjugate gradients on
 * the free dofs with the matrix-free product of igamt_apply_blocks (d_blocks as
 * there), until |f - K u|_f <= rtol |f|_f by the updated residual, or max_iter
 * iterations.  d_u double [n_dofs]: initial guess in, solution out (clamped
 * entries set to 0).  d_f double [n_dofs].  d_workspace of
 * igamt_pcg_workspace_bytes.  The call synchronises the stream once per
 * iteration (host stopping test).  *iterations = iterations done;
 * *rel_residual = |f - K u|_f / |f|_f recomputed from the final u (0 when f
 * vanishes on the free dofs, where u = 0 is returned).  Reductions run in a
 * fixed order: a solve is bitwise reproducible.  IGAMT_EINVAL for rtol <= 0,
 * max_iter < 0, or a search direction with p.Kp <= 0.                        */
igamt_status igamt_pcg_workspace_bytes(const igamt_plan *plan, int64_t *bytes);
igamt_status igamt_pcg(igamt_plan *plan, igamt_precision prec, const void *d_blocks, const double *d_f,
                       const uint8_t *d_fixed, double *d_u, double rtol, int32_t max_iter, void *d_workspace,
                       void *stream, int32_t *iterations, double *rel_residual);

/* --- volume and its shape sensitivity (Section 3.1, eq. (14)-(19), (25)-(26);
 *     Section 4.1.1, eq. (66)-(67)) -------------------------------------------
 * igamt_volume_table_build: the table t^h[C] = int |det J_T| (N_C o T) (eq. (18))
 *   by the stiffness table's micro-element Gauss points, its fold t_pi =
 *   M_pi^-1 t^h (eq. (26)), and the per-sample weights of the fit, kept on the
 *   device; rebuild after igamt_set_tile_ctrl.
 * igamt_volume_table_get: copy t^h and/or t_pi (either pointer may be NULL) to
 *   double [n_pi] device buffers.
 * igamt_volume: per tile V^(t) = t^h . d^(t) (eq. (17)), d^(t) the projection of
 *   det J_M^(t) (eq. (15), (23)) on the plan's fit samples, into d_tile_volumes
 *   double [n_tiles] (NULL: kept in the workspace); V = sum of the tile volumes
 *   in a fixed order into d_volume double [1]; if d_grad is not NULL, dV/dm
 *   (eq. (66) with the adjoint field of eq. (67), under the fit's Gauss rule:
 *   the exact derivative of the discrete V) into d_grad double
 *   [n_macro_ctrl][3] (control points x fastest).  d_workspace of
 *   igamt_volume_workspace_bytes.  det J_M <= 0 at a sample raises the
 *   degeneracy flag (igamt_check).  Requires the table (IGAMT_ESTATE).        */
igamt_status igamt_volume_table_build(igamt_plan *plan, void *stream);
igamt_status igamt_volume_table_get(const igamt_plan *plan, double *d_table, double *d_folded, void *stream);
igamt_status igamt_volume_workspace_bytes(const igamt_plan *plan, int64_t *bytes);
igamt_status igamt_volume(igamt_plan *plan, double *d_tile_volumes, double *d_volume, double *d_grad,
                          void *d_workspace, void *stream);

/* igamt_volume_noalloc: igamt_volume without a workspace and without any
 * allocation, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * tile volumes and local gradients go to a static device array of
 * IGAMT_VOLUME_SCRATCH_BYTES (32 MiB) that the library holds on every GPU it
 * runs on until the process ends: 8 n_tiles bytes (256-aligned), plus
 * 24 n_tiles Lx Ly Lz bytes with d_grad (L_k the macro control points a tile's
 * samples touch per direction: 27 at a degree-2 map on its knot spans, so
 * about 250 000 tiles without the gradient and 51 000 with it).  A plan that
 * needs more returns IGAMT_ESHAPE and queues nothing.  Same arguments, kernels
 * and results (bit for bit) as igamt_volume.  The volume table must be built
 * (IGAMT_ESTATE otherwise; the plan is then already on its device, so this
 * call sets nothing up).  Every call on one GPU shares that GPU's array, which
 * keeps the last call's contents (nothing in it needs to start at zero):
 * calls that overlap on one GPU (other streams, other plans) race and must be
 * ordered by the caller.                                                      */
#define IGAMT_VOLUME_SCRATCH_BYTES (32LL << 20)
igamt_status igamt_volume_noalloc(igamt_plan *plan, double *d_tile_volumes, double *d_volume, double *d_grad,
                                  void *stream);

/* --- projection error and adaptive degree (Section 3.2.2 after eq. (48);
 *     Section 3.3.1, eq. (59), (65)) --------------------------------------------
 * igamt_eproj: E_proj(q) = max over tiles and samples of |A - Pi_q A|_F / |A|_F
 *   (eq. (59)), A the macro field of eq. (37) for (E, nu), Pi_q its projection
 *   onto the degree-q Bernstein space fitted on q + 1 Gauss-Legendre nodes per
 *   direction, whatever the plan's own q; samples: the uniform grid
 *   k / (n_sample - 1), k = 0 .. n_sample - 1, per direction of every tile's
 *   box (2 <= n_sample <= 8; 0 <= q <= 6).  *e_proj on the host (the call
 *   synchronises the stream); d_tile_e double [n_tiles] receives the per-tile
 *   maxima if not NULL.  det J_M <= 0 raises the degeneracy flag.
 * igamt_select_q: eq. (65), the first q from the macro degree to q_max with
 *   E_proj(q) <= tol; *q_out = that q and *e_out its error, or *q_out = -1 and
 *   *e_out = E_proj(q_max) when none meets tol.  A plan for the chosen degree
 *   is then made with igamt_plan_create.                                       */
igamt_status igamt_eproj(igamt_plan *plan, double E, double nu, int32_t q, int32_t n_sample, double *d_tile_e,
                         double *e_proj, void *stream);
igamt_status igamt_select_q(igamt_plan *plan, double E, double nu, double tol, int32_t q_max, int32_t n_sample,
                            int32_t *q_out, double *e_out, void *stream);
/* Anisotropic forms (Section 3.3.4).  igamt_eproj_aniso: as igamt_eproj with
 * degrees q[3] per direction (host array), fitted on max_k q_k + 1 nodes per
 * direction.  igamt_select_q_aniso: from the macro degrees per direction, while
 * E_proj > tol raise by one the direction (below q_max) whose raise gives the
 * lowest E_proj (ties: the lowest direction); q_out[3] the degrees found (all
 * -1 when every direction reached q_max first) and *e_out their E_proj.      */
igamt_status igamt_eproj_aniso(igamt_plan *plan, double E, double nu, const int32_t *q, int32_t n_sample,
                               double *d_tile_e, double *e_proj, void *stream);
igamt_status igamt_select_q_aniso(igamt_plan *plan, double E, double nu, double tol, int32_t q_max,
                                  int32_t n_sample, int32_t *q_out, double *e_out, void *stream);

/* --- batches of designs ----------------------------------------------------
 * The same table steps for n_design designs of one tile family at once (same
 * knots, degree and pair set as the plan's reference tile, different control
 * points).  Tables of a batch are dense, d_tables double
 * [n_design][n_pairs][n_cols]; the plan's own table is not touched.  Tile
 * control points d_ctrl double [n_design][n_tile_ctrl][3] on the device; a
 * boundary point off its Greville position is reported by igamt_check, as for
 * igamt_set_tile_ctrl.  1 <= n_design <= 65535.  Scratch for the point records
 * of the batch is allocated on the first call and grown when a larger batch
 * needs it.
 *
 * Exact tables (eq. (52), as igamt_tables_build); with d_gate (int32
 * [n_design], may be NULL) design b is built only when d_gate[b] != 0 and its
 * table is left as it is otherwise.                                           */
igamt_status igamt_tables_build_batch(igamt_plan *plan, const double *d_ctrl, int32_t n_design,
                                      const int32_t *d_gate, double *d_tables, void *stream);
/* Exact rows of each design's table (as igamt_tables_build_rows) into d_out
 * double [n_design][n_rows][n_cols].                                          */
igamt_status igamt_tables_build_rows_batch(igamt_plan *plan, const double *d_ctrl, int32_t n_design,
                                           const int32_t *d_rows, int32_t n_rows, double *d_out, void *stream);
/* POD reconstruction of n_design tables, tables[b][e] = mean[e] + sum_k
 * basis[k][e] * coeff_scale * coeffs[b][k] (d_coeffs float [n_design][r]),
 * bit-identical per design to igamt_table_from_pod.  d_coef_work: double
 * scratch of igamt_pod_batch_work_doubles(r, n_design) elements.              */
igamt_status igamt_tables_from_pod_batch(const igamt_plan *plan, const float *d_mean, const float *d_basis,
                                         int32_t r, const float *d_coeffs, int32_t n_design, double coeff_scale,
                                         double *d_coef_work, double *d_tables, void *stream);
int64_t igamt_pod_batch_work_doubles(int32_t r, int32_t n_design);
/* Per-design error and gate (as igamt_table_rows_check) of batch tables against
 * exact rows d_exact double [n_design][n_rows][n_cols]; d_err double
 * [n_design], d_gate int32 [n_design].                                        */
igamt_status igamt_tables_rows_check_batch(const igamt_plan *plan, const double *d_tables, int32_t n_design,
                                           const int32_t *d_rows, int32_t n_rows, const double *d_exact,
                                           double tol, double *d_err, int32_t *d_gate, void *stream);
/* The learned path for a batch: MLP forward with desc->batch = n_design
 * designs (d_x float [n_design][n_in]), batched reconstruction into d_tables,
 * exact check rows, per-design error and gate, and exact tables in place of
 * the learned ones of the designs whose gate is set; nothing waits on the
 * host.  d_exact_rows double [n_design][n_rows][n_cols], d_err / d_gate
 * [n_design], d_coef_work as for igamt_tables_from_pod_batch.                 */
igamt_status igamt_tables_learned_batch(igamt_plan *plan, const igamt_mlp_desc *desc, const float *d_params,
                                        const float *d_x, float *d_act, float *d_y, const float *d_mean,
                                        const float *d_basis, double coeff_scale, const double *d_ctrl,
                                        const int32_t *d_rows, int32_t n_rows, double *d_exact_rows, double tol,
                                        double *d_err, int32_t *d_gate, double *d_coef_work, double *d_tables,
                                        void *stream);

#ifdef __cplusplus
}
#endif
#endif /* IGAMT_H */
