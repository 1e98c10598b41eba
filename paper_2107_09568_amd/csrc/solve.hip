// Krylov solve of the clamped system K u = f (eq. (30)) with the matrix-free product of eq. (74)
// (Section 4.2 points at Krylov methods with matrix-vector products only).
//
// Conjugate gradients with the Jacobi preconditioner.  Clamped dofs (homogeneous Dirichlet
// conditions, a caller's per-dof mask) are removed: every iterate, residual and search direction
// is zero there, and the product's entries there are ignored, so the iteration runs on K_ff.
//   r = f - K u,  z = D^-1 r,  p = z
//   repeat: alpha = (r.z) / (p.K p);  u += alpha p;  r -= alpha K p;  z = D^-1 r;
//           beta = (r.z)_new / (r.z);  p = z + beta p
// until |r| <= rtol |f_f|.  D is diag(K_ff), summed from the tiles' (A, A) blocks in ascending
// tile index.  Dot products reduce in a fixed order (fixed grid, fixed per-thread stride, fixed
// tree), so a solve is bitwise reproducible.  Scalars stay on the device; the host reads |r|^2
// once per iteration for the stopping test.
#include "device_common.h"

namespace igamt {

constexpr int kDotBlocks = 1024;
constexpr int kDotThreads = 256;

struct PcgScalars {
  double rz, rr, ff, alpha, beta, pap, rr_true;
};

// Fixed-order block sum of v into out (thread 0 returns it); s has kDotThreads doubles.
__device__ inline double block_sum(double v, double *s) {
  const int tid = threadIdx.x;
  s[tid] = v;
  __syncthreads();
  for (int w = kDotThreads / 2; w > 0; w >>= 1) {
    if (tid < w) s[tid] += s[tid + w];
    __syncthreads();
  }
  const double r = s[0];
  __syncthreads();
  return r;
}

template <typename BT>
__global__ __launch_bounds__(256) void pcg_diag_kernel(const BT *__restrict__ blocks, const int32_t *__restrict__ lut,
                                                       int64_t lut_stride, int64_t lut_center, int64_t n_pairs,
                                                       int nx, int ny, int nz, int tx_n, int ty_n, int tz_n,
                                                       int GX, int GY, int64_t n_dofs,
                                                       const uint8_t *__restrict__ fixed, double *__restrict__ dinv) {
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (id >= n_dofs) return;
  const int a = (int)(id % 3);
  const int64_t G = id / 3;
  const int g[3] = {(int)(G % GX), (int)((G / GX) % GY), (int)(G / ((int64_t)GX * GY))};
  const int n[3] = {nx, ny, nz}, tn[3] = {tx_n, ty_n, tz_n};
  int tlo[3], thi[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int m = n[k] - 1;
    thi[k] = min(g[k] / m, tn[k] - 1);
    tlo[k] = g[k] > 0 ? (g[k] - 1) / m : 0;
  }
  double d = 0.0;
  for (int tz = tlo[2]; tz <= thi[2]; ++tz)
    for (int ty = tlo[1]; ty <= thi[1]; ++ty)
      for (int tx = tlo[0]; tx <= thi[0]; ++tx) {
        const int64_t t = tx + (int64_t)tx_n * (ty + (int64_t)ty_n * tz);
        const int64_t A = (g[0] - tx * (nx - 1)) + (int64_t)nx * ((g[1] - ty * (ny - 1)) + (int64_t)ny * (g[2] - tz * (nz - 1)));
        const int32_t p = lut[A * lut_stride + lut_center];
        d += (double)blocks[(t * n_pairs + p) * 9 + 4 * a];
      }
  dinv[id] = fixed[id] ? 0.0 : 1.0 / d;
}

// r = f - Ku on free dofs, z = D^-1 r, p = z; partial sums of r.z, r.r, f.f (free dofs)
__global__ __launch_bounds__(kDotThreads) void pcg_init_kernel(int64_t n, const double *__restrict__ f,
                                                               const double *__restrict__ Ku,
                                                               const uint8_t *__restrict__ fixed,
                                                               const double *__restrict__ dinv, double *r, double *z,
                                                               double *p, double *partial) {
  __shared__ double s[kDotThreads];
  double rz = 0.0, rr = 0.0, ff = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kDotThreads + threadIdx.x; i < n; i += (int64_t)kDotBlocks * kDotThreads) {
    const bool fr = !fixed[i];
    const double ri = fr ? f[i] - Ku[i] : 0.0;
    const double zi = dinv[i] * ri;
    r[i] = ri;
    z[i] = zi;
    p[i] = zi;
    rz += ri * zi;
    rr += ri * ri;
    ff += fr ? f[i] * f[i] : 0.0;
  }
  rz = block_sum(rz, s);
  rr = block_sum(rr, s);
  ff = block_sum(ff, s);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = rz;
    partial[kDotBlocks + blockIdx.x] = rr;
    partial[2 * kDotBlocks + blockIdx.x] = ff;
  }
}

// partial sums of p.Kp (p vanishes on clamped dofs, so their Kp entries drop out)
__global__ __launch_bounds__(kDotThreads) void pcg_pap_kernel(int64_t n, const double *__restrict__ p,
                                                              const double *__restrict__ Ap, double *partial) {
  __shared__ double s[kDotThreads];
  double v = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kDotThreads + threadIdx.x; i < n; i += (int64_t)kDotBlocks * kDotThreads)
    v += p[i] * Ap[i];
  v = block_sum(v, s);
  if (threadIdx.x == 0) partial[blockIdx.x] = v;
}

// u += alpha p, r -= alpha Kp (free dofs), z = D^-1 r; partial sums of r.z and r.r
__global__ __launch_bounds__(kDotThreads) void pcg_update_kernel(int64_t n, const PcgScalars *__restrict__ sc,
                                                                 const double *__restrict__ p,
                                                                 const double *__restrict__ Ap,
                                                                 const uint8_t *__restrict__ fixed,
                                                                 const double *__restrict__ dinv, double *u,
                                                                 double *r, double *z, double *partial) {
  __shared__ double s[kDotThreads];
  const double alpha = sc->alpha;
  double rz = 0.0, rr = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kDotThreads + threadIdx.x; i < n; i += (int64_t)kDotBlocks * kDotThreads) {
    u[i] += alpha * p[i];
    const double ri = fixed[i] ? 0.0 : r[i] - alpha * Ap[i];
    const double zi = dinv[i] * ri;
    r[i] = ri;
    z[i] = zi;
    rz += ri * zi;
    rr += ri * ri;
  }
  rz = block_sum(rz, s);
  rr = block_sum(rr, s);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = rz;
    partial[kDotBlocks + blockIdx.x] = rr;
  }
}

// partial sums of |f - K u|^2 over free dofs
__global__ __launch_bounds__(kDotThreads) void pcg_resid_kernel(int64_t n, const double *__restrict__ f,
                                                                const double *__restrict__ Ku,
                                                                const uint8_t *__restrict__ fixed, double *partial) {
  __shared__ double s[kDotThreads];
  double v = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kDotThreads + threadIdx.x; i < n; i += (int64_t)kDotBlocks * kDotThreads) {
    const double ri = fixed[i] ? 0.0 : f[i] - Ku[i];
    v += ri * ri;
  }
  v = block_sum(v, s);
  if (threadIdx.x == 0) partial[blockIdx.x] = v;
}

__global__ __launch_bounds__(kDotThreads) void pcg_clear_fixed_kernel(int64_t n, const uint8_t *__restrict__ fixed,
                                                                      double *u) {
  for (int64_t i = (int64_t)blockIdx.x * kDotThreads + threadIdx.x; i < n; i += (int64_t)kDotBlocks * kDotThreads)
    if (fixed[i]) u[i] = 0.0;
}

__global__ __launch_bounds__(kDotThreads) void pcg_p_kernel(int64_t n, const PcgScalars *__restrict__ sc,
                                                            const double *__restrict__ z, double *p) {
  const double beta = sc->beta;
  for (int64_t i = (int64_t)blockIdx.x * kDotThreads + threadIdx.x; i < n; i += (int64_t)kDotBlocks * kDotThreads)
    p[i] = z[i] + beta * p[i];
}

enum PcgStage { kStageInit = 0, kStageAlpha = 1, kStageBeta = 2, kStageResid = 3 };

// One workgroup: the fixed-order totals of the partial sums, then the stage's scalar update.
__global__ __launch_bounds__(kDotThreads) void pcg_scalars_kernel(const double *__restrict__ partial, int n_vals,
                                                                  int stage, PcgScalars *sc) {
  __shared__ double s[kDotThreads];
  double tot[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < n_vals; ++k) {
    double v = 0.0;
    for (int b = threadIdx.x; b < kDotBlocks; b += kDotThreads) v += partial[k * kDotBlocks + b];
    tot[k] = block_sum(v, s);
  }
  if (threadIdx.x != 0) return;
  switch (stage) {
    case kStageInit:
      sc->rz = tot[0];
      sc->rr = tot[1];
      sc->ff = tot[2];
      break;
    case kStageAlpha:
      sc->pap = tot[0];
      sc->alpha = tot[0] > 0.0 ? sc->rz / tot[0] : 0.0;
      break;
    case kStageBeta:
      sc->beta = sc->rz > 0.0 ? tot[0] / sc->rz : 0.0;
      sc->rz = tot[0];
      sc->rr = tot[1];
      break;
    default:
      sc->rr_true = tot[0];
      break;
  }
}

}  // namespace igamt

using namespace igamt;

static int64_t pcg_vec_bytes(const igamt_plan *P) { return align256(3 * P->n_global * (int64_t)sizeof(double)); }

extern "C" igamt_status igamt_pcg_workspace_bytes(const igamt_plan *P, int64_t *bytes) {
  if (!P || !bytes) { set_error("NULL argument"); return IGAMT_EINVAL; }
  int64_t lin = 0;
  igamt_status st = igamt_linop_workspace_bytes(P, IGAMT_F64, 0, &lin);
  if (st) return st;
  *bytes = 5 * pcg_vec_bytes(P) + lin + align256(3 * kDotBlocks * sizeof(double)) + align256(sizeof(PcgScalars));
  return IGAMT_OK;
}

extern "C" igamt_status igamt_pcg(igamt_plan *P, igamt_precision prec, const void *d_blocks, const double *d_f,
                                  const uint8_t *d_fixed, double *d_u, double rtol, int32_t max_iter,
                                  void *d_workspace, void *stream, int32_t *iterations, double *rel_residual) {
  if (!P || !d_blocks || !d_f || !d_fixed || !d_u || !d_workspace || !iterations || !rel_residual) {
    set_error("NULL argument");
    return IGAMT_EINVAL;
  }
  if (prec < IGAMT_F64 || prec > IGAMT_F16X3) { set_error("unknown precision"); return IGAMT_EINVAL; }
  if (!(rtol > 0.0) || !std::isfinite(rtol) || max_iter < 0) {
    set_error("rtol must be positive and finite, max_iter non-negative");
    return IGAMT_EINVAL;
  }
  igamt_status st = ensure_device(P);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = 3 * P->n_global, vb = pcg_vec_bytes(P);
  char *ws = (char *)d_workspace;
  double *r = (double *)ws, *z = (double *)(ws + vb), *p = (double *)(ws + 2 * vb), *Ap = (double *)(ws + 3 * vb),
         *dinv = (double *)(ws + 4 * vb);
  int64_t lin = 0;
  if ((st = igamt_linop_workspace_bytes(P, prec, 0, &lin))) return st;
  void *ytile = ws + 5 * vb;
  double *partial = (double *)(ws + 5 * vb + lin);
  PcgScalars *sc = (PcgScalars *)(ws + 5 * vb + lin + align256(3 * kDotBlocks * sizeof(double)));
  // diagonal of K_ff from the tiles' (A, A) blocks
  const int64_t lut_stride = (int64_t)P->S[0] * P->S[1] * P->S[2];
  const int64_t lut_center = ((int64_t)P->pT[2] * P->S[1] + P->pT[1]) * P->S[0] + P->pT[0];
  const dim3 gd((unsigned)((n + 255) / 256));
  if (prec == IGAMT_F64)
    hipLaunchKernelGGL(pcg_diag_kernel<double>, gd, dim3(256), 0, s, (const double *)d_blocks, P->dev.pair_lut,
                       lut_stride, lut_center, P->n_pairs, P->nT[0], P->nT[1], P->nT[2], P->tiles[0], P->tiles[1],
                       P->tiles[2], P->dir[0].NG, P->dir[1].NG, n, d_fixed, dinv);
  else
    hipLaunchKernelGGL(pcg_diag_kernel<float>, gd, dim3(256), 0, s, (const float *)d_blocks, P->dev.pair_lut,
                       lut_stride, lut_center, P->n_pairs, P->nT[0], P->nT[1], P->nT[2], P->tiles[0], P->tiles[1],
                       P->tiles[2], P->dir[0].NG, P->dir[1].NG, n, d_fixed, dinv);
  IGAMT_LAUNCH_CHECK();
  const dim3 gdot(kDotBlocks), bdot(kDotThreads);
  PcgScalars h;
  auto read_scalars = [&]() -> igamt_status {
    IGAMT_HIP(hipMemcpyAsync(&h, sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, s));
    IGAMT_HIP(hipStreamSynchronize(s));
    return IGAMT_OK;
  };
  // r0 = f - K u0, with the clamped entries of u0 cleared first
  hipLaunchKernelGGL(pcg_clear_fixed_kernel, gdot, bdot, 0, s, n, d_fixed, d_u);
  if ((st = igamt_apply_blocks(P, prec, d_blocks, d_u, Ap, ytile, stream))) return st;
  hipLaunchKernelGGL(pcg_init_kernel, gdot, bdot, 0, s, n, d_f, Ap, d_fixed, dinv, r, z, p, partial);
  hipLaunchKernelGGL(pcg_scalars_kernel, dim3(1), bdot, 0, s, partial, 3, (int)kStageInit, sc);
  IGAMT_LAUNCH_CHECK();
  if ((st = read_scalars())) return st;
  const double fnorm = std::sqrt(h.ff);
  int it = 0;
  if (fnorm == 0.0) {   // no load on the free dofs: u = 0 there
    IGAMT_HIP(hipMemsetAsync(d_u, 0, n * sizeof(double), s));
    IGAMT_HIP(hipStreamSynchronize(s));
    *iterations = 0;
    *rel_residual = 0.0;
    return IGAMT_OK;
  }
  while (it < max_iter && std::sqrt(h.rr) > rtol * fnorm) {
    if ((st = igamt_apply_blocks(P, prec, d_blocks, p, Ap, ytile, stream))) return st;
    hipLaunchKernelGGL(pcg_pap_kernel, gdot, bdot, 0, s, n, p, Ap, partial);
    hipLaunchKernelGGL(pcg_scalars_kernel, dim3(1), bdot, 0, s, partial, 1, (int)kStageAlpha, sc);
    hipLaunchKernelGGL(pcg_update_kernel, gdot, bdot, 0, s, n, sc, p, Ap, d_fixed, dinv, d_u, r, z, partial);
    hipLaunchKernelGGL(pcg_scalars_kernel, dim3(1), bdot, 0, s, partial, 2, (int)kStageBeta, sc);
    hipLaunchKernelGGL(pcg_p_kernel, gdot, bdot, 0, s, n, sc, z, p);
    IGAMT_LAUNCH_CHECK();
    ++it;
    if ((st = read_scalars())) return st;
    if (!(h.pap > 0.0)) { set_error("K_ff is not positive definite on the search direction"); return IGAMT_EINVAL; }
  }
  // true residual of the result
  if ((st = igamt_apply_blocks(P, prec, d_blocks, d_u, Ap, ytile, stream))) return st;
  hipLaunchKernelGGL(pcg_resid_kernel, gdot, bdot, 0, s, n, d_f, Ap, d_fixed, partial);
  hipLaunchKernelGGL(pcg_scalars_kernel, dim3(1), bdot, 0, s, partial, 1, (int)kStageResid, sc);
  IGAMT_LAUNCH_CHECK();
  if ((st = read_scalars())) return st;
  *iterations = it;
  *rel_residual = std::sqrt(h.rr_true) / fnorm;
  return IGAMT_OK;
}
