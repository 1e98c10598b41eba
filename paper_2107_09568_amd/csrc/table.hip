// Micro-scale stiffness lookup table (Section 3.2.3, eq. (51)-(52), (57)):
//   table[p(A,B)][9C + 3i + j] = int_Omega_T d_i(R_A o T^-1) d_j(R_B o T^-1) N_C dxi
// pulled back to the tile parameter domain,
//   = sum_e sum_g w_g det J_T (J_T^-T grad R_A)_i (J_T^-T grad R_B)_j N_C(T^r(theta_g)),
// with n_gauss Gauss-Legendre points per direction on every micro element.
//
// Pass 1 (one thread per micro element x Gauss point) evaluates the tile map
// and stores, per point, w det J_T, the Bernstein values N_C(T^r(theta)) and the
// mapped gradients of the (p+1)^3 active functions.  Pass 2 (one wave per
// row and Bernstein index C) sums the nine (i, j) integrals over the micro
// elements shared by A and B and their points, in a fixed order, so the table
// is bitwise reproducible.
#include "device_common.h"

namespace igamt {

struct TableArgs {
  const double *knots[3];
  int nT[3], eT[3];
  const double *ctrl;
  const double *gx, *gw;
  int ng, qd[3], npi;    // projection degree per direction, n_pi = prod (qd + 1)
  int64_t stride;        // doubles per point record
  double *pts;
  int32_t *flag;
  const int32_t *gate;   // optional: do nothing unless gate[design] != 0
  int64_t ctrl_stride;   // batched designs (grid y): control points and point records per design
  int64_t pts_stride;
};

template <int PT>
__global__ __launch_bounds__(64) void table_points_kernel(TableArgs a) {
  if (a.gate && a.gate[blockIdx.y] == 0) return;
  const int G = a.ng * a.ng * a.ng;
  const int64_t id = (int64_t)blockIdx.x * 64 + threadIdx.x;
  const int64_t nE = (int64_t)a.eT[0] * a.eT[1] * a.eT[2];
  if (id >= nE * G) return;
  const int64_t e = id / G;
  const int g = (int)(id % G);
  const double *ctrl = a.ctrl + blockIdx.y * a.ctrl_stride;
  const int ei[3] = {(int)(e % a.eT[0]), (int)((e / a.eT[0]) % a.eT[1]), (int)(e / ((int64_t)a.eT[0] * a.eT[1]))};
  const int gi[3] = {g % a.ng, (g / a.ng) % a.ng, g / (a.ng * a.ng)};
  double N[3][PT + 1], dN[3][PT + 1];
  double w = 1.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int span = ei[k] + PT;
    const double lo = a.knots[k][span], hi = a.knots[k][span + 1];
    const double th = lo + (hi - lo) * a.gx[gi[k]];
    w *= (hi - lo) * a.gw[gi[k]];
    bspline_ders<PT>(a.knots[k], span, th, N[k], dN[k]);
  }
  // map value and Jacobian J[c][k] = dT_c / dtheta_k
  double X[3] = {0, 0, 0};
  double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int rz = 0; rz <= PT; ++rz)
    for (int ry = 0; ry <= PT; ++ry)
#pragma unroll
      for (int rx = 0; rx <= PT; ++rx) {
        const int64_t A = (ei[0] + rx) + (int64_t)a.nT[0] * ((ei[1] + ry) + (int64_t)a.nT[1] * (ei[2] + rz));
        const double *c = ctrl + 3 * A;
        const double R = N[0][rx] * N[1][ry] * N[2][rz];
        const double d0 = dN[0][rx] * N[1][ry] * N[2][rz];
        const double d1 = N[0][rx] * dN[1][ry] * N[2][rz];
        const double d2 = N[0][rx] * N[1][ry] * dN[2][rz];
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
          X[cc] += R * c[cc];
          J[cc][0] += c[cc] * d0;
          J[cc][1] += c[cc] * d1;
          J[cc][2] += c[cc] * d2;
        }
      }
  double F[3][3];
  const double D = inv3(J, F);
  if (!(D > 0.0) || !isfinite(D)) atomicMin(a.flag + 1, (int32_t)e);
  double *out = a.pts + blockIdx.y * a.pts_stride + id * a.stride;
  out[0] = w * D;
  double B[3][kMaxQ + 1];
#pragma unroll
  for (int k = 0; k < 3; ++k) bernstein(a.qd[k], X[k], B[k]);
  const int q1x = a.qd[0] + 1, q1y = a.qd[1] + 1;
  for (int C = 0; C < a.npi; ++C) out[1 + C] = B[0][C % q1x] * B[1][(C / q1x) % q1y] * B[2][C / (q1x * q1y)];
  double *gout = out + 1 + a.npi;
  int la = 0;
  for (int rz = 0; rz <= PT; ++rz)
    for (int ry = 0; ry <= PT; ++ry)
#pragma unroll
      for (int rx = 0; rx <= PT; ++rx, ++la) {
        const double d[3] = {dN[0][rx] * N[1][ry] * N[2][rz], N[0][rx] * dN[1][ry] * N[2][rz],
                             N[0][rx] * N[1][ry] * dN[2][rz]};
#pragma unroll
        for (int c = 0; c < 3; ++c) gout[3 * la + c] = F[0][c] * d[0] + F[1][c] * d[1] + F[2][c] * d[2];
      }
}

struct TableSumArgs {
  const int32_t *pairs;
  const int32_t *rows;   // optional row list
  int64_t n_rows;
  int64_t n_pairs;
  int nT[3], eT[3], pT;
  int ng, npi;
  int64_t stride;
  const double *pts;
  double *out;
  int64_t out_stride;    // doubles per output row
  const int32_t *gate;   // optional: do nothing unless gate[design] != 0
  int64_t pts_stride;    // batched designs (grid y): point records and output per design
  int64_t out_dstride;
};

// One wave per (row, C): the terms of the nine sums (i, j), one per (shared micro element, Gauss
// point), are split over the lanes (lane l takes terms l, l + 64, ... in ascending element and
// point order), then combined by a butterfly across the wave, whose every step adds the same two
// operands on both lanes: the order is fixed, so every entry is bitwise reproducible and the same
// whether the whole table or a row subset is built.
__global__ __launch_bounds__(256) void table_sum_kernel(TableSumArgs a) {
  if (a.gate && a.gate[blockIdx.y] == 0) return;
  const int lane = threadIdx.x & 63;
  const int64_t wv = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);   // (row, C), uniform per wave
  if (wv >= a.n_rows * a.npi) return;
  const int C = (int)(wv % a.npi);
  const int64_t row = wv / a.npi;
  const int64_t p = a.rows ? a.rows[row] : row;
  double *o = a.out + blockIdx.y * a.out_dstride + row * a.out_stride + 9 * C;
  if (p < 0 || p >= a.n_pairs) {  // invalid row index: flag the output instead of reading out of bounds
    if (lane < 9) o[lane] = __builtin_nan("");
    return;
  }
  const int A = a.pairs[2 * p], B = a.pairs[2 * p + 1];
  const int ai[3] = {A % a.nT[0], (A / a.nT[0]) % a.nT[1], A / (a.nT[0] * a.nT[1])};
  const int bi[3] = {B % a.nT[0], (B / a.nT[0]) % a.nT[1], B / (a.nT[0] * a.nT[1])};
  int lo[3], n[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    lo[k] = max(max(ai[k], bi[k]) - a.pT, 0);
    n[k] = max(0, min(min(ai[k], bi[k]), a.eT[k] - 1) - lo[k] + 1);
  }
  const int G = a.ng * a.ng * a.ng;
  const int p1 = a.pT + 1;
  const int nt = n[0] * n[1] * n[2] * G;
  const double *pts = a.pts + blockIdx.y * a.pts_stride;
  double acc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = 0.0;
  for (int t = lane; t < nt; t += 64) {
    const int sl = t / G, g = t - sl * G;
    const int ex = lo[0] + sl % n[0], ey = lo[1] + (sl / n[0]) % n[1], ez = lo[2] + sl / (n[0] * n[1]);
    const int64_t e = ex + (int64_t)a.eT[0] * (ey + (int64_t)a.eT[1] * ez);
    const int la = (ai[0] - ex) + p1 * ((ai[1] - ey) + p1 * (ai[2] - ez));
    const int lb = (bi[0] - ex) + p1 * ((bi[1] - ey) + p1 * (bi[2] - ez));
    const double *pd = pts + (e * G + g) * a.stride;
    const double wn = pd[0] * pd[1 + C];
    const double *gA = pd + 1 + a.npi + 3 * la, *gB = pd + 1 + a.npi + 3 * lb;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double ga = wn * gA[i];
#pragma unroll
      for (int j = 0; j < 3; ++j) acc[3 * i + j] += ga * gB[j];
    }
  }
#pragma unroll
  for (int k = 0; k < 9; ++k)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc[k] += __shfl_xor(acc[k], off);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 9; ++k) o[k] = acc[k];
  }
}

static __global__ void zero_f64(const int32_t *gate, double *p, int64_t n) {
  if (gate && *gate == 0) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

static igamt_status run_points(igamt_plan *P, hipStream_t s, int64_t &stride, const int32_t *gate) {
  const int G = P->n_gauss * P->n_gauss * P->n_gauss;
  const int64_t nE = (int64_t)P->eT[0] * P->eT[1] * P->eT[2];
  const int nact = (P->pT[0] + 1) * (P->pT[1] + 1) * (P->pT[2] + 1);
  stride = 1 + P->npi + 3 * nact;
  if (!P->dev.point_data) IGAMT_HIP(hipMalloc((void **)&P->dev.point_data, nE * G * stride * sizeof(double)));
  if (P->pT[0] != P->pT[1] || P->pT[0] != P->pT[2]) {
    set_error("reference tiles with different degrees per direction are not supported");
    return IGAMT_EUNSUPPORTED;
  }
  TableArgs a;
  for (int k = 0; k < 3; ++k) {
    a.knots[k] = P->dev.tile_knots[k];
    a.nT[k] = P->nT[k];
    a.eT[k] = P->eT[k];
  }
  a.ctrl = P->dev.tile_ctrl;
  a.gx = P->dev.gauss_x;
  a.gw = P->dev.gauss_w;
  a.ng = P->n_gauss;
  for (int k = 0; k < 3; ++k) a.qd[k] = P->qd[k];
  a.npi = P->npi;
  a.stride = stride;
  a.pts = P->dev.point_data;
  a.flag = P->dev.flag;
  a.gate = gate;
  a.ctrl_stride = 0;
  a.pts_stride = 0;
  const dim3 grid((unsigned)((nE * G + 63) / 64)), block(64);
  switch (P->pT[0]) {
    case 1: hipLaunchKernelGGL(table_points_kernel<1>, grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL(table_points_kernel<2>, grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL(table_points_kernel<3>, grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL(table_points_kernel<4>, grid, block, 0, s, a); break;
    case 5: hipLaunchKernelGGL(table_points_kernel<5>, grid, block, 0, s, a); break;
    case 6: hipLaunchKernelGGL(table_points_kernel<6>, grid, block, 0, s, a); break;
    default: set_error("unsupported tile degree"); return IGAMT_EUNSUPPORTED;
  }
  IGAMT_LAUNCH_CHECK();
  return IGAMT_OK;
}

igamt_status table_point_records(igamt_plan *P, void *stream, int64_t &stride) {
  return run_points(P, (hipStream_t)stream, stride, nullptr);
}

static TableSumArgs sum_args(const igamt_plan *P, int64_t stride) {
  TableSumArgs b;
  b.pairs = P->dev.pairs;
  b.rows = nullptr;
  b.gate = nullptr;
  b.pts_stride = 0;
  b.out_dstride = 0;
  b.n_rows = P->n_pairs;
  b.n_pairs = P->n_pairs;
  for (int k = 0; k < 3; ++k) {
    b.nT[k] = P->nT[k];
    b.eT[k] = P->eT[k];
  }
  b.pT = P->pT[0];
  b.ng = P->n_gauss;
  b.npi = P->npi;
  b.stride = stride;
  b.pts = P->dev.point_data;
  return b;
}

}  // namespace igamt

using namespace igamt;

static igamt_status build_tables(igamt_plan *P, void *stream, const int32_t *gate) {
  igamt_status st = ensure_device(P);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  int64_t stride = 0;
  if ((st = run_points(P, s, stride, gate))) return st;
  const int64_t MK = P->Mp * P->Kp;
  hipLaunchKernelGGL(zero_f64, dim3((unsigned)((MK + 255) / 256)), dim3(256), 0, s, gate, P->dev.table, MK);
  IGAMT_LAUNCH_CHECK();
  TableSumArgs b = sum_args(P, stride);
  b.out = P->dev.table;
  b.out_stride = P->Kp;
  b.gate = gate;
  const int64_t nw = P->n_pairs * P->npi;   // one wave per (row, C)
  hipLaunchKernelGGL(table_sum_kernel, dim3((unsigned)((nw + 3) / 4)), dim3(256), 0, s, b);
  IGAMT_LAUNCH_CHECK();
  return derive_table_copies(P, stream, gate);
}

extern "C" igamt_status igamt_tables_build(igamt_plan *P, void *stream) {
  if (!P) { set_error("NULL argument"); return IGAMT_EINVAL; }
  return build_tables(P, stream, nullptr);
}

extern "C" igamt_status igamt_tables_build_gated(igamt_plan *P, const int32_t *d_gate, void *stream) {
  if (!P || !d_gate) { set_error("NULL argument"); return IGAMT_EINVAL; }
  if (!P->tables_ready) { set_error("a gated build replaces an existing table: build or set one first"); return IGAMT_ESTATE; }
  return build_tables(P, stream, d_gate);
}

extern "C" igamt_status igamt_tables_build_rows(igamt_plan *P, const int32_t *d_rows, int32_t n_rows, double *d_out,
                                                void *stream) {
  if (!P || !d_rows || !d_out || n_rows <= 0) { set_error("invalid argument"); return IGAMT_EINVAL; }
  igamt_status st = ensure_device(P);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  int64_t stride = 0;
  if ((st = run_points(P, s, stride, nullptr))) return st;
  TableSumArgs b = sum_args(P, stride);
  b.rows = d_rows;
  b.n_rows = n_rows;
  b.out = d_out;
  b.out_stride = P->K;
  const int64_t nw = (int64_t)n_rows * P->npi;
  hipLaunchKernelGGL(table_sum_kernel, dim3((unsigned)((nw + 3) / 4)), dim3(256), 0, s, b);
  IGAMT_LAUNCH_CHECK();
  return IGAMT_OK;
}

// ---- batched designs -------------------------------------------------------------------
static __global__ void tile_boundary_batch_kernel(const double *__restrict__ ctrl, int64_t n_design, const double *grev,
                                                  int nx, int ny, int nz, int32_t *flag) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)nx * ny * nz;
  if (id >= n * n_design) return;
  const int64_t pt = id % n;
  const int i = (int)(pt % nx), j = (int)((pt / nx) % ny), k = (int)(pt / ((int64_t)nx * ny));
  if (!(i == 0 || j == 0 || k == 0 || i == nx - 1 || j == ny - 1 || k == nz - 1)) return;
  const double *c = ctrl + 3 * id;
  const double e = fabs(c[0] - grev[i]) + fabs(c[1] - grev[nx + j]) + fabs(c[2] - grev[nx + ny + k]);
  if (!(e <= 1e-12)) atomicMin(flag + 2, (int32_t)pt);
}

// Point records of n_design designs (tile control points d_ctrl [n_design][n_tile_ctrl][3])
// into dev.batch_points, grown on demand; designs with gate[b] == 0 are skipped.
static igamt_status run_points_batch(igamt_plan *P, hipStream_t s, const double *d_ctrl, int32_t n_design,
                                     const int32_t *gate, int64_t &stride, int64_t &per) {
  if (P->pT[0] != P->pT[1] || P->pT[0] != P->pT[2]) {
    set_error("reference tiles with different degrees per direction are not supported");
    return IGAMT_EUNSUPPORTED;
  }
  const int G = P->n_gauss * P->n_gauss * P->n_gauss;
  const int64_t nE = (int64_t)P->eT[0] * P->eT[1] * P->eT[2];
  const int nact = (P->pT[0] + 1) * (P->pT[1] + 1) * (P->pT[2] + 1);
  stride = 1 + P->npi + 3 * nact;
  per = nE * G * stride;
  if (P->batch_points_cap < per * n_design) {
    if (P->dev.batch_points) IGAMT_HIP(hipFree(P->dev.batch_points));
    P->dev.batch_points = nullptr;
    P->batch_points_cap = 0;
    IGAMT_HIP(hipMalloc((void **)&P->dev.batch_points, per * n_design * sizeof(double)));
    P->batch_points_cap = per * n_design;
  }
  hipLaunchKernelGGL(tile_boundary_batch_kernel, dim3((unsigned)((P->nTt * n_design + 255) / 256)), dim3(256), 0, s,
                     d_ctrl, (int64_t)n_design, P->dev.tile_grev, P->nT[0], P->nT[1], P->nT[2], P->dev.flag);
  IGAMT_LAUNCH_CHECK();
  TableArgs a;
  for (int k = 0; k < 3; ++k) {
    a.knots[k] = P->dev.tile_knots[k];
    a.nT[k] = P->nT[k];
    a.eT[k] = P->eT[k];
  }
  a.ctrl = d_ctrl;
  a.gx = P->dev.gauss_x;
  a.gw = P->dev.gauss_w;
  a.ng = P->n_gauss;
  for (int k = 0; k < 3; ++k) a.qd[k] = P->qd[k];
  a.npi = P->npi;
  a.stride = stride;
  a.pts = P->dev.batch_points;
  a.flag = P->dev.flag;
  a.gate = gate;
  a.ctrl_stride = 3 * P->nTt;
  a.pts_stride = per;
  const dim3 grid((unsigned)((nE * G + 63) / 64), (unsigned)n_design), block(64);
  switch (P->pT[0]) {
    case 1: hipLaunchKernelGGL(table_points_kernel<1>, grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL(table_points_kernel<2>, grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL(table_points_kernel<3>, grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL(table_points_kernel<4>, grid, block, 0, s, a); break;
    case 5: hipLaunchKernelGGL(table_points_kernel<5>, grid, block, 0, s, a); break;
    case 6: hipLaunchKernelGGL(table_points_kernel<6>, grid, block, 0, s, a); break;
    default: set_error("unsupported tile degree"); return IGAMT_EUNSUPPORTED;
  }
  IGAMT_LAUNCH_CHECK();
  return IGAMT_OK;
}

static igamt_status sum_batch(igamt_plan *P, hipStream_t s, int32_t n_design, const int32_t *gate,
                              const int32_t *d_rows, int32_t n_rows, double *d_out, int64_t stride, int64_t per) {
  TableSumArgs b = sum_args(P, stride);
  b.pts = P->dev.batch_points;
  b.pts_stride = per;
  b.gate = gate;
  b.rows = d_rows;
  b.n_rows = d_rows ? n_rows : P->n_pairs;
  b.out = d_out;
  b.out_stride = P->K;
  b.out_dstride = b.n_rows * P->K;
  const int64_t nw = b.n_rows * P->npi;
  hipLaunchKernelGGL(table_sum_kernel, dim3((unsigned)((nw + 3) / 4), (unsigned)n_design), dim3(256), 0, s, b);
  IGAMT_LAUNCH_CHECK();
  return IGAMT_OK;
}

extern "C" igamt_status igamt_tables_build_batch(igamt_plan *P, const double *d_ctrl, int32_t n_design,
                                                 const int32_t *d_gate, double *d_tables, void *stream) {
  if (!P || !d_ctrl || !d_tables || n_design <= 0 || n_design > 65535) {
    set_error("invalid argument");
    return IGAMT_EINVAL;
  }
  igamt_status st = ensure_device(P);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  int64_t stride = 0, per = 0;
  if ((st = run_points_batch(P, s, d_ctrl, n_design, d_gate, stride, per))) return st;
  return sum_batch(P, s, n_design, d_gate, nullptr, 0, d_tables, stride, per);
}

extern "C" igamt_status igamt_tables_build_rows_batch(igamt_plan *P, const double *d_ctrl, int32_t n_design,
                                                      const int32_t *d_rows, int32_t n_rows, double *d_out,
                                                      void *stream) {
  if (!P || !d_ctrl || !d_rows || !d_out || n_rows <= 0 || n_design <= 0 || n_design > 65535) {
    set_error("invalid argument");
    return IGAMT_EINVAL;
  }
  igamt_status st = ensure_device(P);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  int64_t stride = 0, per = 0;
  if ((st = run_points_batch(P, s, d_ctrl, n_design, nullptr, stride, per))) return st;
  return sum_batch(P, s, n_design, nullptr, d_rows, n_rows, d_out, stride, per);
}
