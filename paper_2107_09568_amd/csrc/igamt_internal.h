// Internal definitions shared by the host plan and the HIP kernels of libigamt.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/igamt.h"

namespace igamt {

constexpr int kMaxDegree = 6;      // spline degrees handled by the device evaluators
constexpr int kMaxQ = 6;           // projection degree
constexpr int kMaxFit = 8;         // fit samples per direction
constexpr int kMaxGauss = 8;       // table quadrature points per direction
constexpr int kTileGroup = 16;     // tiles per contraction column group (144 columns)
constexpr int kColPad = 64;        // table columns padded to a multiple of this
#ifndef IGAMT_SCATTER_CHUNK
#define IGAMT_SCATTER_CHUNK 512
#endif
constexpr int kScatterChunk = IGAMT_SCATTER_CHUNK;   // block records per scatter workgroup
constexpr int kDescWords = 12;                        // ints per scatter pair descriptor
constexpr int kRowPad = 128;       // table rows padded to a multiple of this
constexpr int kMaxTileControl = 16;   // tile control points per direction

void set_error(const std::string &msg);


// One direction of the glued 1-D structure: for every global index g its sorted
// neighbour list (g2) and, per neighbour, the tiles holding both (1 or 2) with
// the tile-local indices of g and g2.
struct Pair1D {
  int32_t g, g2, rank, ntile;
  int32_t tile[2], li[2], lj[2];
  int32_t pad[2];
};
static_assert(sizeof(Pair1D) == 48, "Pair1D layout");

struct Direction {
  int NG = 0;                        // global control points in this direction
  std::vector<Pair1D> pairs;         // sorted by (g, g2)
  std::vector<int32_t> off;          // [NG + 1] first entry of g
  std::vector<int64_t> pre;          // [NG + 1] exclusive prefix of neighbour counts
  std::vector<int32_t> lo;           // [NG] first neighbour of g (neighbours of g are lo .. lo + count - 1)
};

struct DevicePtrs {
  bool ready = false;
  int device = -1;
  double *macro_knots[3] = {nullptr, nullptr, nullptr};
  double *macro_ctrl = nullptr;
  double *macro_w = nullptr;         // NURBS weights of the macro map (null: B-spline)
  double *box_a[3] = {nullptr, nullptr, nullptr};
  double *box_h[3] = {nullptr, nullptr, nullptr};
  double *fit_x = nullptr;           // [n_fit] Gauss nodes on [0,1]
  double *fit_P = nullptr;           // [(q+1) * n_fit] 1-D projection matrix
  double *fit_P3 = nullptr;          // the three per-direction operators, concatenated
  double *tile_knots[3] = {nullptr, nullptr, nullptr};
  double *tile_ctrl = nullptr;
  double *tile_grev = nullptr;       // [n_x + n_y + n_z] Greville abscissae of the tile knots
  double *gauss_x = nullptr;         // [n_gauss] nodes on [0,1]
  double *gauss_w = nullptr;
  int32_t *pairs = nullptr;          // [n_pairs][2]
  int32_t *pair_lut = nullptr;       // [n_T][S_z][S_y][S_x] -> pair index or -1
  Pair1D *dir_pairs[3] = {nullptr, nullptr, nullptr};
  int32_t *dir_off[3] = {nullptr, nullptr, nullptr};
  int64_t *dir_pre[3] = {nullptr, nullptr, nullptr};
  int32_t *dir_lo[3] = {nullptr, nullptr, nullptr};
  int32_t *pair_desc = nullptr;      // [n_pairs][kDescWords] scatter descriptor of each pair
  int32_t *mirror_perm = nullptr;    // [chunks * kScatterChunk] per scatter chunk: records ordered by (B, A)
  int32_t *ctrl_lo[3] = {nullptr, nullptr, nullptr};     // per tile: first local macro ctrl index
  int32_t *ctrl_tiles_off[3] = {nullptr, nullptr, nullptr};  // per macro ctrl index: tiles touching it
  int32_t *ctrl_tiles[3] = {nullptr, nullptr, nullptr};      // (tile, local offset) pairs
  int32_t *flag = nullptr;           // smallest degenerate tile index (INT32_MAX = none)
  // tables
  double *table = nullptr;           // [Mp][Kp] FP64, zero padded
  double *table_t = nullptr;         // [transposed_rows][Mp] FP64 (transposed, zero padded, for the adjoint)
  float *table_f32 = nullptr;        // [Mp][Kp]
  float *table_t_f32 = nullptr;      // [transposed_rows][Mp]
  uint16_t *table_bf = nullptr;      // hi [Mp][Kp] then lo [Mp][Kp]
  uint16_t *table_h = nullptr;       // hi then lo, scaled rows
  float *table_h_scale = nullptr;    // [Mp] inverse row scale
  double *point_data = nullptr;      // table builder scratch
  double *batch_points = nullptr;    // point records of batched designs (grown on demand)
  double *load_table = nullptr;      // [nTt][npi][7] load-vector table (volume, six faces)
  // matrix-free tile product schedule (one allocation at apply_rec; the others point into it)
  int32_t *apply_rec = nullptr;      // [n_pairs] A | B << 16
  int32_t *apply_perm = nullptr;     // per chunk: slots sorted by destination row (16 bits each)
  int32_t *apply_seg = nullptr;      // per chunk: row | segment end << 16
  double *eproj_buf = nullptr;       // projection-error scratch: per-tile errors, nodes, operator, result
  double *volume_data = nullptr;     // volume table t^h [npi], folded table t_pi [npi], sample weights [n_fit^3]
};

}  // namespace igamt

struct igamt_plan {
  // macro map
  int pM[3], nM[3];
  std::vector<double> kM[3];
  std::vector<double> ctrlM;
  std::vector<double> wM;             // NURBS weights [nz][ny][nx] (empty: B-spline)
  // reference tile
  int pT[3], nT[3];
  std::vector<double> kT[3];
  std::vector<double> ctrlT;
  std::vector<double> grevT;           // Greville abscissae of the tile knots, x then y then z
  int eT[3];                          // micro elements per direction
  // descriptor
  int tiles[3], box_mode, q, n_fit, n_gauss;
  int qd[3];                          // projection degree per direction (all q unless anisotropic)
  bool aniso = false;                 // degrees differ per direction
  // derived sizes
  int64_t n_tiles, n_tiles_pad, n_groups;
  int npi, K, Kp;
  int64_t n_pairs, Mp, nTt;
  int S[3];                           // 2 pT + 1 per direction (pair LUT strides)
  std::vector<double> box_a[3], box_h[3];
  std::vector<int32_t> pairs;         // [n_pairs][2]
  std::vector<int32_t> pair_lut;      // [nTt][S2][S1][S0]
  // scatter descriptors, kDescWords per pair: w0 = a_x | a_y << 8 | a_z << 16 | flags << 24
  // (bits 0-2: a_d = b_d = 0, bits 3-5: a_d = b_d = n_d - 1, bit 6: A = B),
  // w1 = b_x | b_y << 8 | b_z << 16, w[1 + delta] = index of the same pair in the tile shifted by
  // delta = dx + 2 dy + 4 dz (delta = 1..7; -1 where the pair does not lie on those faces)
  std::vector<int32_t> pair_desc;
  std::vector<int32_t> mirror_perm;   // per scatter chunk of the pair list: local order by (B, A)
  igamt::Direction dir[3];
  int64_t n_global, nnz;
  // 1-D fit operator
  std::vector<double> fit_x, fit_w, fit_P;
  std::vector<double> fit_P3;         // per-direction operators, [(qd[0]+1) nf][(qd[1]+1) nf][(qd[2]+1) nf]
  std::vector<double> gauss_x, gauss_w;
  // macro control points touched by each tile (for the fit adjoint)
  int Lc[3];                          // local control points per direction (max over tiles)
  std::vector<int32_t> ctrl_lo[3];
  std::vector<int32_t> ctrl_tiles_off[3], ctrl_tiles[3];
  // state
  bool tables_ready = false;
  int64_t batch_points_cap = 0;       // doubles allocated in dev.batch_points
  bool load_table_ready = false;
  bool volume_ready = false;
  igamt::DevicePtrs dev;
};

namespace igamt {
// host helpers (plan.cpp)
void gauss_legendre01(int n, std::vector<double> &x, std::vector<double> &w);
// 1-D projection operator P ((q+1) x n, row-major) onto the degree-q Bernstein basis by the
// weighted discrete L2 fit at the points x with weights w (eq. (23)-(24)); false if singular
bool projection_1d(int q, const std::vector<double> &x, const std::vector<double> &w, std::vector<double> &P);
int find_span_host(const std::vector<double> &U, int n, int p, double x);
// device helpers (device.hip)
igamt_status ensure_device(igamt_plan *plan);
void free_device(igamt_plan *plan);
igamt_status upload_macro_ctrl(igamt_plan *plan, const double *ctrl, int on_device, void *stream);
// copies for the other precisions; with a gate, the kernels do nothing unless *gate != 0
igamt_status derive_table_copies(igamt_plan *plan, void *stream, const int32_t *gate = nullptr);
// point records of the tile's micro elements (w det J_T, Bernstein values, mapped gradients) into
// dev.point_data for the current tile control points (table.hip)
igamt_status table_point_records(igamt_plan *plan, void *stream, int64_t &stride);
// synchronous upload of the host tile control points
igamt_status upload_tile_ctrl(igamt_plan *plan);
// stage launchers (fit.hip, contract.hip, scatter.hip)
int64_t coef_bytes(const igamt_plan *plan, igamt_precision prec);
int64_t blocks_bytes(const igamt_plan *plan, igamt_precision prec);
// tile range [t0, t1) (t1 <= n_tiles_pad); t1 < 0 means all tiles
igamt_status launch_fit(igamt_plan *plan, double E, double nu, igamt_precision prec, void *d_coef, void *stream,
                        int64_t t0 = 0, int64_t t1 = -1);
// tile groups [g0, g1) of kTileGroup tiles; g1 < 0 means all groups
igamt_status launch_contract(igamt_plan *plan, igamt_precision prec, const void *d_coef, void *d_blocks,
                             void *stream, int64_t g0 = 0, int64_t g1 = -1);
// owner records of all tiles
igamt_status launch_scatter(igamt_plan *plan, igamt_precision prec, const void *d_blocks, void *d_values,
                            void *stream);
// C (rows x 9 n_tiles) = A (rows_pad x kdim, row-major) B (kdim per column, 9 n_tiles_pad columns),
// written as out[t][row][ab] for row < rows; FP64 or FP32 operands (contract.hip)
igamt_status launch_gemm_tiles(igamt_precision prec, const void *A, const void *B, void *out, int64_t rows,
                               int64_t rows_pad, int64_t kdim, int64_t n_tiles, int64_t n_groups, void *stream);
// fixed-order reductions of the shape gradients (adjoint.hip): per-tile local gradients
// [n_tiles][Lc2][Lc1][Lc0][3] summed per macro control point into grad [n_macro_ctrl][3]; and a
// one-workgroup sum of x [n] into out[0]
// Looks up this device's address of the static scratch of igamt_volume_noalloc (once per device,
// with that device current); called by ensure_device.
igamt_status volume_scratch_setup(int device);
igamt_status launch_grad_reduce(igamt_plan *plan, const double *local_grad, double *grad, void *stream);
igamt_status launch_sum(const double *x, int64_t n, double *out, void *stream);
// rows of the transposed table (table columns padded to a multiple of the contraction's row block)
inline int64_t transposed_rows(const igamt_plan *P) { return (P->Kp + 127) / 128 * 128; }
}  // namespace igamt
