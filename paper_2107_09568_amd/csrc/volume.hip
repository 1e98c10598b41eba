// Volume of the microstructured geometry by interpolation and lookup, and its shape sensitivity
// (Section 3.1, eq. (14)-(19), (23)-(26); Section 4.1.1, eq. (66)-(67)).
//
// Table (eq. (18)): t^h[C] = int |det J_T| (N_C o T) dtheta, summed over the tile's micro
// elements and Gauss points (the stiffness table builder's point records) in a fixed order.
// Folded table (eq. (26)): t_pi = M_pi^-1 t^h, M_pi the Bernstein mass matrix of eq. (24), the
// Kronecker cube of the 1-D matrix int B_a B_b = C(q,a) C(q,b) / ((2q+1) C(2q,a+b)).
// Tile volume (eq. (17)): V^(t) = t^h . d^(t) with d^(t) = P D^(t), P the projection operator of
// eq. (23)-(24) (Kronecker cube of the plan's 1-D operator) and D^(t) = det J_M^(t) at the fit
// samples; folded into sample weights g = P^T t^h, V^(t) = g . D^(t).
// Sensitivity (eq. (66)-(67)): dV/dm = sum_t sum_s g_s dD_s/dm.  With the fit's n_fit-point Gauss
// rule, g_s = w_s v(xi_s), v = sum_C N_C t_pi[C] the adjoint field of eq. (67), so this is eq. (66)
// under that rule and the exact derivative of the discrete V.  With J = J_M(a + h xi) diag(h):
//   dD/dm_(i,c) = D sum_n (J^-1)[n][c] h_n d_n N_i.
// Per tile: one 64-thread workgroup; local gradients of the macro control points the tile's
// samples touch, then the fixed-order per-control-point reduction shared with the compliance
// sensitivity.  V = sum of the tile volumes in a fixed order: bitwise reproducible.
#include <cmath>
#include <mutex>
#include <vector>

#include "device_common.h"

namespace igamt {

// t^h[C] over the point records (w det J_T, N_C o T per micro element and Gauss point)
__global__ __launch_bounds__(64) void volume_table_kernel(const double *__restrict__ pts, int64_t stride,
                                                          int64_t n_rec, int npi, double *__restrict__ th) {
  const int C = blockIdx.x * 64 + threadIdx.x;
  if (C >= npi) return;
  double s = 0.0;
  for (int64_t r = 0; r < n_rec; ++r) {
    const double *pd = pts + r * stride;
    s += fabs(pd[0]) * pd[1 + C];
  }
  th[C] = s;
}

struct VolumeFoldArgs {
  double minv[3][(kMaxQ + 1) * (kMaxQ + 1)];   // inverse 1-D Bernstein mass matrix per direction
  const double *fP3;                            // per-direction 1-D projection operators [q1[k]][nf]
  int q1[3], nf;
  double *data;                                 // t^h [npi] in; t_pi [npi], g [nf^3] out
};

// t_pi = (Minv_x x Minv_y x Minv_z) t^h and g = (P_x x P_y x P_z)^T t^h
__global__ __launch_bounds__(256) void volume_fold_kernel(VolumeFoldArgs a) {
  const int qx = a.q1[0], qy = a.q1[1], qz = a.q1[2], npi = qx * qy * qz, nf = a.nf, ns = nf * nf * nf;
  const double *th = a.data;
  double *tpi = a.data + npi, *g = a.data + 2 * npi;
  const double *Px = a.fP3, *Py = Px + qx * nf, *Pz = Py + qy * nf;
  for (int C = threadIdx.x; C < npi; C += 256) {
    const int c[3] = {C % qx, (C / qx) % qy, C / (qx * qy)};
    double s = 0.0;
    for (int D = 0; D < npi; ++D) {
      const int d[3] = {D % qx, (D / qx) % qy, D / (qx * qy)};
      s += a.minv[0][c[0] * qx + d[0]] * a.minv[1][c[1] * qy + d[1]] * a.minv[2][c[2] * qz + d[2]] * th[D];
    }
    tpi[C] = s;
  }
  for (int S = threadIdx.x; S < ns; S += 256) {
    const int si[3] = {S % nf, (S / nf) % nf, S / (nf * nf)};
    double s = 0.0;
    for (int C = 0; C < npi; ++C) {
      const int c[3] = {C % qx, (C / qx) % qy, C / (qx * qy)};
      s += Px[c[0] * nf + si[0]] * Py[c[1] * nf + si[1]] * Pz[c[2] * nf + si[2]] * th[C];
    }
    g[S] = s;
  }
}

struct VolumeTileArgs {
  const double *knots[3];
  int nM[3];
  const double *ctrl;
  const double *wts;      // NURBS weights of the macro map, or null (B-spline)
  const double *box_a[3];
  const double *box_h[3];
  const int32_t *ctrl_lo[3];
  int tiles[3], Lc[3];
  const double *fx;
  const double *g;          // [nf^3] sample weights
  int nf;
  double *tile_vol;         // [n_tiles]
  double *local_grad;       // [n_tiles][Lz][Ly][Lx][3] or null
  int32_t *flag;
  int Lm;                   // max(Lc): row length of the 1-D factor tables
};

template <int P0, int P1, int P2>
__global__ __launch_bounds__(64) void volume_tile_kernel(VolumeTileArgs a) {
  constexpr int PMX = max3(P0, P1, P2);
  constexpr int PD[3] = {P0, P1, P2};
  extern __shared__ double GS[];    // [ns][9]: g_s D_s (J^-1)[n][c] h_n at [3 c + n]; NURBS: then WQ [ns][4]
  __shared__ double NB[3][kMaxFit][kMaxDegree + 1], DB[3][kMaxFit][kMaxDegree + 1];
  __shared__ int SP[3][kMaxFit];
  __shared__ double red[64];
  const int tid = threadIdx.x, nf = a.nf, ns = nf * nf * nf;
  const int64_t t = blockIdx.x;
  const int tt[3] = {(int)(t % a.tiles[0]), (int)((t / a.tiles[0]) % a.tiles[1]),
                     (int)(t / ((int64_t)a.tiles[0] * a.tiles[1]))};
  const double ax[3] = {a.box_a[0][tt[0]], a.box_a[1][tt[1]], a.box_a[2][tt[2]]};
  const double hx[3] = {a.box_h[0][tt[0]], a.box_h[1][tt[1]], a.box_h[2][tt[2]]};
  const bool grad = a.local_grad != nullptr;
  double *WQ = GS + ns * 9;   // NURBS: 1 / W and sum_n GS[c][n] d_n W / W^2 per sample
  for (int e = tid; e < 3 * nf; e += 64) {   // 1-D macro bases at the tile's sample abscissae
    const int k = e / nf, s = e % nf;
    const double x = ax[k] + hx[k] * a.fx[s];
    const int sp = find_span(a.knots[k], a.nM[k], PD[k], x);
    double N[PMX + 1], dN[PMX + 1];
    bspline_ders_dir<P0, P1, P2>(k, a.knots[k], sp, x, N, dN);
    SP[k][s] = sp;
    for (int r = 0; r <= PMX; ++r) { NB[k][s][r] = N[r]; DB[k][s][r] = dN[r]; }
  }
  __syncthreads();   // the basis tables are read by the sample loop and the local gradients
  double vol = 0.0;
  for (int s = tid; s < ns; s += 64) {
    const int si[3] = {s % nf, (s / nf) % nf, s / (nf * nf)};
    double J[3][3], N[3][PMX + 1], dN[3][PMX + 1];
    int span[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {   // the shared 1-D bases (the values spline_jacobian3 computes)
      span[k] = SP[k][si[k]];
#pragma unroll
      for (int r = 0; r <= PMX; ++r) {
        N[k][r] = NB[k][si[k]][r];
        dN[k][r] = DB[k][si[k]][r];
      }
    }
    spline_jacobian_sum<P0, P1, P2>(a.nM, a.ctrl, a.wts, span, N, dN, J);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int n = 0; n < 3; ++n) J[c][n] *= hx[n];
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double D = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    if (!(D > 0.0) || !isfinite(D)) atomicMin(a.flag, (int32_t)t);
    const double gs = a.g[s];
    vol += gs * D;
    if (grad) {
      // D (J^-1)[n][c] is the cofactor of J[c][n]
      double cof[3][3];
      cof[0][0] = c00; cof[0][1] = c01; cof[0][2] = c02;
      cof[1][0] = J[2][1] * J[0][2] - J[2][2] * J[0][1];
      cof[1][1] = J[2][2] * J[0][0] - J[2][0] * J[0][2];
      cof[1][2] = J[2][0] * J[0][1] - J[2][1] * J[0][0];
      cof[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
      cof[2][1] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
      cof[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int n = 0; n < 3; ++n) GS[s * 9 + 3 * c + n] = gs * cof[c][n] * hx[n];
      if (a.wts) rational_terms3<P0, P1, P2>(a.wts, a.nM, SP, NB, DB, si, GS + s * 9, WQ + s * 4);
    }
  }
  red[tid] = vol;
  __syncthreads();
  for (int w = 32; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) a.tile_vol[t] = red[0];
  if (!grad) return;
  // local control-point gradients: g[i][c] = sum_s sum_n GS[s][c][n] d_n N_i(s).  The basis is a
  // tensor product, so its factors are tabulated per direction: XV[k][s][l] = N_r(x_s) and
  // XD[k][s][l] = N_r'(x_s) with r = lo_k + l - (span_s - p), zero where l is outside the support
  // of the sample (such samples add an exact zero).
  const int L0 = a.Lc[0], L1 = a.Lc[1], L2 = a.Lc[2], Lm = a.Lm;
  const int lo[3] = {a.ctrl_lo[0][tt[0]], a.ctrl_lo[1][tt[1]], a.ctrl_lo[2][tt[2]]};
  double *XV = GS + ns * 13, *XD = XV + 3 * nf * Lm;   // [3][nf][Lm] each, after GS and WQ
  for (int e = tid; e < 3 * nf * Lm; e += 64) {
    const int k = e / (nf * Lm), rem = e - k * nf * Lm, sk = rem / Lm, l = rem - sk * Lm;
    const int r = lo[k] + l - (SP[k][sk] - PD[k]);
    const bool on = r >= 0 && r <= PD[k];
    const int rc = on ? r : 0;
    XV[e] = on ? NB[k][sk][rc] : 0.0;
    XD[e] = on ? DB[k][sk][rc] : 0.0;
  }
  __syncthreads();
  double *lg = a.local_grad + t * (int64_t)L0 * L1 * L2 * 3;
  for (int e = tid; e < L0 * L1 * L2 * 3; e += 64) {
    const int c = e % 3, li = e / 3;
    const int l[3] = {li % L0, (li / L0) % L1, li / (L0 * L1)};
    double gsum = 0.0;
    for (int s3 = 0; s3 < nf; ++s3) {
      const double v2 = XV[(2 * nf + s3) * Lm + l[2]], d2 = XD[(2 * nf + s3) * Lm + l[2]];
      for (int s2 = 0; s2 < nf; ++s2) {
        const double v1 = XV[(nf + s2) * Lm + l[1]], d1 = XD[(nf + s2) * Lm + l[1]];
        for (int s1 = 0; s1 < nf; ++s1) {
          const double v0 = XV[s1 * Lm + l[0]], d0 = XD[s1 * Lm + l[0]];
          const int s = (s3 * nf + s2) * nf + s1;
          const double *gc = GS + s * 9 + 3 * c;
          const double tb = gc[0] * d0 * v1 * v2 + gc[1] * v0 * d1 * v2 + gc[2] * v0 * v1 * d2;
          gsum += a.wts ? tb * WQ[s * 4] - v0 * v1 * v2 * WQ[s * 4 + 1 + c] : tb;
        }
      }
    }
    lg[e] = a.wts ? gsum * local_weight(a.wts, a.nM, lo, l)
                  : gsum;
  }
}

// inverse of the 1-D Bernstein mass matrix (Gauss-Jordan with partial pivoting, q + 1 <= 7)
static bool bernstein_mass_inverse(int q, double *inv) {
  const int n = q + 1;
  std::vector<double> m(n * n), r(n * n, 0.0);
  auto binom = [](int nn, int k) {
    double b = 1.0;
    for (int i = 1; i <= k; ++i) b = b * (nn - k + i) / i;
    return b;
  };
  for (int i = 0; i < n; ++i) {
    r[i * n + i] = 1.0;
    for (int j = 0; j < n; ++j) m[i * n + j] = binom(q, i) * binom(q, j) / ((2 * q + 1) * binom(2 * q, i + j));
  }
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int i = c + 1; i < n; ++i)
      if (std::fabs(m[i * n + c]) > std::fabs(m[piv * n + c])) piv = i;
    if (m[piv * n + c] == 0.0) return false;
    for (int j = 0; j < n; ++j) {
      std::swap(m[c * n + j], m[piv * n + j]);
      std::swap(r[c * n + j], r[piv * n + j]);
    }
    const double d = m[c * n + c];
    for (int j = 0; j < n; ++j) {
      m[c * n + j] /= d;
      r[c * n + j] /= d;
    }
    for (int i = 0; i < n; ++i)
      if (i != c) {
        const double f = m[i * n + c];
        for (int j = 0; j < n; ++j) {
          m[i * n + j] -= f * m[c * n + j];
          r[i * n + j] -= f * r[c * n + j];
        }
      }
  }
  for (int i = 0; i < n * n; ++i) inv[i] = r[i];
  return true;
}

}  // namespace igamt

using namespace igamt;

extern "C" igamt_status igamt_volume_table_build(igamt_plan *P, void *stream) {
  if (!P) { set_error("NULL argument"); return IGAMT_EINVAL; }
  igamt_status st = ensure_device(P);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  int64_t stride = 0;
  if ((st = table_point_records(P, s, stride))) return st;
  const int ns = P->n_fit * P->n_fit * P->n_fit;
  if (!P->dev.volume_data) IGAMT_HIP(hipMalloc((void **)&P->dev.volume_data, (2 * P->npi + ns) * sizeof(double)));
  const int64_t n_rec = (int64_t)P->eT[0] * P->eT[1] * P->eT[2] * P->n_gauss * P->n_gauss * P->n_gauss;
  hipLaunchKernelGGL(volume_table_kernel, dim3((unsigned)((P->npi + 63) / 64)), dim3(64), 0, s, P->dev.point_data,
                     stride, n_rec, P->npi, P->dev.volume_data);
  IGAMT_LAUNCH_CHECK();
  VolumeFoldArgs f;
  for (int k = 0; k < 3; ++k) {
    if (!bernstein_mass_inverse(P->qd[k], f.minv[k])) { set_error("singular Bernstein mass matrix"); return IGAMT_EINVAL; }
    f.q1[k] = P->qd[k] + 1;
  }
  f.fP3 = P->dev.fit_P3;
  f.nf = P->n_fit;
  f.data = P->dev.volume_data;
  hipLaunchKernelGGL(volume_fold_kernel, dim3(1), dim3(256), 0, s, f);
  IGAMT_LAUNCH_CHECK();
  P->volume_ready = true;
  return IGAMT_OK;
}

extern "C" igamt_status igamt_volume_table_get(const igamt_plan *P, double *d_table, double *d_folded, void *stream) {
  if (!P || (!d_table && !d_folded)) { set_error("NULL argument"); return IGAMT_EINVAL; }
  if (!P->dev.ready || !P->volume_ready) { set_error("volume table not built"); return IGAMT_ESTATE; }
  hipStream_t s = (hipStream_t)stream;
  if (d_table)
    IGAMT_HIP(hipMemcpyAsync(d_table, P->dev.volume_data, P->npi * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (d_folded)
    IGAMT_HIP(hipMemcpyAsync(d_folded, P->dev.volume_data + P->npi, P->npi * sizeof(double), hipMemcpyDeviceToDevice, s));
  return IGAMT_OK;
}

// ---- scratch of igamt_volume_noalloc ------------------------------------------------------
// One file-scope device array per GPU (the tile volumes, then the tiles' local control-point
// gradients), held until the process ends.  In host code `scratch` names a host-side stand-in, not
// a device address: every use goes through the per-device address looked up by
// volume_scratch_setup, which ensure_device calls once per device with that device current.
static __device__ __align__(256) unsigned char scratch[IGAMT_VOLUME_SCRATCH_BYTES];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

namespace igamt {
igamt_status volume_scratch_setup(int device) {
  if (device < 0 || device >= kMaxScratchDevices) { set_error("device index out of range"); return IGAMT_EINVAL; }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return IGAMT_OK;
  void *ptr = nullptr;
  IGAMT_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) { set_error("no device address for the volume scratch"); return IGAMT_EHIP; }
  g_scratch_ptr[device] = ptr;
  return IGAMT_OK;
}
}  // namespace igamt

static void *volume_scratch_ptr(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

static int64_t volume_local_bytes(const igamt_plan *P) {
  return align256(P->n_tiles * (int64_t)P->Lc[0] * P->Lc[1] * P->Lc[2] * 3 * sizeof(double));
}

extern "C" igamt_status igamt_volume_workspace_bytes(const igamt_plan *P, int64_t *bytes) {
  if (!P || !bytes) { set_error("NULL argument"); return IGAMT_EINVAL; }
  *bytes = align256(P->n_tiles * (int64_t)sizeof(double)) + volume_local_bytes(P);
  return IGAMT_OK;
}

// The tile kernel, the fixed-order volume sum and, with d_grad, the per-control-point reduction,
// with the tile volumes and local gradients in the workspace ws.
static igamt_status volume_run(igamt_plan *P, double *d_tile_volumes, double *d_volume, double *d_grad, void *d_workspace,
                               void *stream) {
  igamt_status st;
  hipStream_t s = (hipStream_t)stream;
  char *ws = (char *)d_workspace;
  double *tv = d_tile_volumes ? d_tile_volumes : (double *)ws;
  double *lg = (double *)(ws + align256(P->n_tiles * (int64_t)sizeof(double)));
  VolumeTileArgs a;
  for (int k = 0; k < 3; ++k) {
    a.knots[k] = P->dev.macro_knots[k];
    a.nM[k] = P->nM[k];
    a.box_a[k] = P->dev.box_a[k];
    a.box_h[k] = P->dev.box_h[k];
    a.ctrl_lo[k] = P->dev.ctrl_lo[k];
    a.tiles[k] = P->tiles[k];
    a.Lc[k] = P->Lc[k];
  }
  a.ctrl = P->dev.macro_ctrl;
  a.wts = P->dev.macro_w;
  a.fx = P->dev.fit_x;
  a.g = P->dev.volume_data + 2 * P->npi;
  a.nf = P->n_fit;
  a.tile_vol = tv;
  a.local_grad = d_grad ? lg : nullptr;
  a.flag = P->dev.flag;
  const int ns = P->n_fit * P->n_fit * P->n_fit;
  a.Lm = std::max(P->Lc[0], std::max(P->Lc[1], P->Lc[2]));
  const size_t shm = d_grad ? (size_t)(ns * (9 + 4) + 6 * (int64_t)P->n_fit * a.Lm) * sizeof(double) : 0;
  if (shm > 60 * 1024) { set_error("tile samples or macro control points per tile too many for the volume gradient"); return IGAMT_EUNSUPPORTED; }
  const dim3 grid((unsigned)P->n_tiles), block(64);
  switch (IGAMT_DEGREE_KEY(P->pM[0], P->pM[1], P->pM[2])) {
#define VOL_CASE(p0, p1, p2)                                                                              \
  case IGAMT_DEGREE_KEY(p0, p1, p2): hipLaunchKernelGGL((volume_tile_kernel<p0, p1, p2>), grid, block, shm, s, a); break;
    IGAMT_FOR_MACRO_DEGREES(VOL_CASE)
#undef VOL_CASE
    default: set_error("unsupported macro degrees (isotropic 1..6, or 1..3 per direction)"); return IGAMT_EUNSUPPORTED;
  }
  IGAMT_LAUNCH_CHECK();
  if ((st = launch_sum(tv, P->n_tiles, d_volume, stream))) return st;
  if (d_grad && (st = launch_grad_reduce(P, lg, d_grad, stream))) return st;
  return IGAMT_OK;
}

extern "C" igamt_status igamt_volume(igamt_plan *P, double *d_tile_volumes, double *d_volume, double *d_grad,
                                     void *d_workspace, void *stream) {
  if (!P || !d_volume || !d_workspace) { set_error("NULL argument"); return IGAMT_EINVAL; }
  igamt_status st = ensure_device(P);
  if (st) return st;
  if (!P->volume_ready) { set_error("volume table not built"); return IGAMT_ESTATE; }
  return volume_run(P, d_tile_volumes, d_volume, d_grad, d_workspace, stream);
}

extern "C" igamt_status igamt_volume_noalloc(igamt_plan *P, double *d_tile_volumes, double *d_volume, double *d_grad,
                                             void *stream) {
  if (!P || !d_volume) { set_error("NULL argument"); return IGAMT_EINVAL; }
  // the volume table exists, so the plan is already on its device: no set-up (and no allocation) here
  if (!P->dev.ready || !P->volume_ready) { set_error("volume table not built"); return IGAMT_ESTATE; }
  int cur = 0;
  IGAMT_HIP(hipGetDevice(&cur));
  if (cur != P->dev.device) { set_error("plan used on a different device than it was set up on"); return IGAMT_ESTATE; }
  const int64_t need = align256(P->n_tiles * (int64_t)sizeof(double)) + (d_grad ? volume_local_bytes(P) : 0);
  if (need > (int64_t)IGAMT_VOLUME_SCRATCH_BYTES) {
    set_error("igamt_volume_noalloc: the plan needs " + std::to_string(need) + " bytes of scratch (" +
              (d_grad ? std::string("tile volumes and local gradients") : std::string("tile volumes")) +
              "), the library's static scratch holds " + std::to_string((int64_t)IGAMT_VOLUME_SCRATCH_BYTES) +
              "; use igamt_volume with a workspace");
    return IGAMT_ESHAPE;
  }
  void *ws = volume_scratch_ptr(cur);
  if (!ws) { set_error("the volume scratch's device address could not be looked up on this device"); return IGAMT_EHIP; }
  return volume_run(P, d_tile_volumes, d_volume, d_grad, ws, stream);
}
