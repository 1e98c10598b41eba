// Stage 1 of the assembly: macro-field fit (Section 3.2.2).
//
// One 64-thread workgroup per tile.  Every Gauss sample xi_s of the tile gets
// J = J_M(a + h xi_s) diag(h) (Cox-de Boor derivatives of the macro map),
// F = J^-1 and D = det J in FP64.  The projection coefficients
//   <A_ij,ab>_C = sum_s P[C, s] A_ij,ab(xi_s),  P = P1 (x) P1 (x) P1,
// (eq. (42) with the 1-D operator of eq. (23)-(24)) are applied sum-factorised,
// one direction at a time, for one component (a, b) of A at a time (its nine (i, j) blocks
// side by side, so that each coefficient row is written contiguously), with
//   A_ij,ab = D (lam F_ia F_jb + mu (F_i . F_j) delta_ab + mu F_ib F_ja),
// the Cartesian form of eq. (37) (F_i is row i of F).  The result is written in
// the column-major layout the contraction reads: coef[t][3a+b][9C+3i+j].
#include "device_common.h"

namespace igamt {

struct FitArgs {
  const double *knots[3];
  int nM[3];
  const double *ctrl;
  const double *wts;      // NURBS weights of the macro map, or null (B-spline)
  const double *box_a[3];
  const double *box_h[3];
  int tiles[3];
  int64_t n_tiles;
  const double *fx;
  const double *fP3;    // per-direction 1-D operators [(q1[0]) nf][(q1[1]) nf][(q1[2]) nf]
  int q1[3], nf, Kp, prec;
  bool tiled;           // split modes: coefficient planes in the tiled layout (split_coef_index)
  double lam, mu;
  double L3;            // product over directions of the largest row sum of |P_k| (F16X3 scale bound)
  void *out;
  int64_t plane;        // n_tiles_pad * 9 * Kp elements per stored plane
  int64_t t0;           // first tile of the launch
  int32_t *flag;
};

// coefficient (column col = 9 t + ab, k) of the stored planes in the contraction's precision
__device__ inline void store_coef(const FitArgs &a, int Kp, int64_t col, int k, double v, double scale) {
  if (a.prec == IGAMT_F64) {
    ((double *)a.out)[col * Kp + k] = v;
  } else if (a.prec == IGAMT_F32) {
    ((float *)a.out)[col * Kp + k] = (float)v;
  } else {
    const int64_t pos = split_coef_index(col, k, Kp, a.tiled);   // the split planes may be tiled
    uint16_t hi, lo;
    if (a.prec == IGAMT_BF16X3)
      split_bf16(v, hi, lo);
    else
      split_f16(v * scale, hi, lo);
    ((uint16_t *)a.out)[pos] = hi;
    ((uint16_t *)a.out)[a.plane + pos] = lo;
  }
}

// QC > 0: the projection degree is QC in every direction with QC + 1 fit nodes, known at compile
// time (every index division of the passes by a constant); QC = 0: degrees and nodes from the
// arguments.  Both compute the same sums in the same order.
template <int P0, int P1, int P2, int QC>
__global__ __launch_bounds__(64) void fit_kernel(FitArgs a) {
  constexpr int PMX = max3(P0, P1, P2);
  extern __shared__ double smem[];
  const int nf = QC ? QC + 1 : a.nf;
  const int q1x = QC ? QC + 1 : a.q1[0], q1y = QC ? QC + 1 : a.q1[1], q1z = QC ? QC + 1 : a.q1[2];
  const int Kp = QC ? (9 * (QC + 1) * (QC + 1) * (QC + 1) + kColPad - 1) / kColPad * kColPad : a.Kp;
  const int ns = nf * nf * nf;
  const int npi = q1x * q1y * q1z;
  double *FD = smem;              // [ns][10]
  double *buf0 = FD + ns * 10;    // [ns][9]
  double *buf1 = buf0 + ns * 9;   // [ns][9]
  __shared__ double Pm[3][(kMaxQ + 1) * kMaxFit];
  const int tid = threadIdx.x;
  const int64_t t = a.t0 + blockIdx.x;

  if (t >= a.n_tiles) {  // padding tile: zeros
    for (int e = tid; e < 9 * Kp; e += 64) store_coef(a, Kp, t * 9 + e / Kp, e % Kp, 0.0, 1.0);
    if (a.prec == IGAMT_F16X3 && tid < 9)
      ((float *)((uint16_t *)a.out + 2 * a.plane))[t * 9 + tid] = 1.0f;
    return;
  }
  for (int e = tid; e < q1x * nf; e += 64) Pm[0][e] = a.fP3[e];
  for (int e = tid; e < q1y * nf; e += 64) Pm[1][e] = a.fP3[q1x * nf + e];
  for (int e = tid; e < q1z * nf; e += 64) Pm[2][e] = a.fP3[(q1x + q1y) * nf + e];
  const int tx = (int)(t % a.tiles[0]);
  const int ty = (int)((t / a.tiles[0]) % a.tiles[1]);
  const int tz = (int)(t / ((int64_t)a.tiles[0] * a.tiles[1]));
  const double ax[3] = {a.box_a[0][tx], a.box_a[1][ty], a.box_a[2][tz]};
  const double hx[3] = {a.box_h[0][tx], a.box_h[1][ty], a.box_h[2][tz]};

  // Jacobians at the samples
  for (int s = tid; s < ns; s += 64) {
    const int si[3] = {s % nf, (s / nf) % nf, s / (nf * nf)};
    double N[3][PMX + 1], dN[3][PMX + 1];
    int span[3];
    const double xh[3] = {ax[0] + hx[0] * a.fx[si[0]], ax[1] + hx[1] * a.fx[si[1]], ax[2] + hx[2] * a.fx[si[2]]};
    double J[3][3];
    spline_jacobian3<P0, P1, P2, true>(a.knots, a.nM, a.ctrl, a.wts, xh, J, span, N, dN);
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
#pragma unroll
      for (int k = 0; k < 3; ++k) J[cc][k] *= hx[k];
    double F[3][3];
    const double D = inv3(J, F);
    if (!(D > 0.0) || !isfinite(D)) atomicMin(a.flag, (int32_t)t);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) FD[s * 10 + 3 * r + c] = F[r][c];
    FD[s * 10 + 9] = D;
  }
  __syncthreads();
  // F16X3: |coef| <= L_x L_y L_z max|A_ij,ab| with L_k the max row sum of |P_k| (a.L3)
  const double L3 = a.L3;

  // One component (a, b) of A at a time, its nine blocks (i, j) side by side: the last pass then
  // writes the coefficient row [ab][9 C + ij] contiguously (coalesced stores; each row's lines are
  // written once).
  for (int ab = 0; ab < 9; ++ab) {
    const int aa = ab / 3, bb = ab % 3;
    // A_ij,ab at every sample, buf0[s][ij]
    for (int e = tid; e < ns * 9; e += 64) {
      const int s = e / 9, ij = e % 9, i = ij / 3, j = ij % 3;
      const double *Fs = FD + s * 10;
      const double fij = Fs[3 * i] * Fs[3 * j] + Fs[3 * i + 1] * Fs[3 * j + 1] + Fs[3 * i + 2] * Fs[3 * j + 2];
      buf0[e] = Fs[9] * (a.lam * Fs[3 * i + aa] * Fs[3 * j + bb] + (aa == bb ? a.mu * fij : 0.0) +
                         a.mu * Fs[3 * i + bb] * Fs[3 * j + aa]);
    }
    __syncthreads();
    double sc = 1.0;
    if (a.prec == IGAMT_F16X3) {  // the column's scale from max |A_ij,ab| over the tile (one wave)
      double m = 0.0;
      for (int e = tid; e < ns * 9; e += 64) m = fmax(m, fabs(buf0[e]));
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
      sc = f16_scale_for(m * L3);
      if (tid == 0) ((float *)((uint16_t *)a.out + 2 * a.plane))[t * 9 + ab] = (float)(1.0 / sc);
    }
    // x direction: buf1[(s3, s2, c1)][ij]
    for (int e = tid; e < q1x * nf * nf * 9; e += 64) {
      const int ij = e % 9, r = e / 9, c1 = r % q1x, s23 = r / q1x;
      double v = 0.0;
      for (int s1 = 0; s1 < nf; ++s1) v += Pm[0][c1 * nf + s1] * buf0[(s23 * nf + s1) * 9 + ij];
      buf1[e] = v;
    }
    __syncthreads();
    // y direction: buf0[(s3, c2, c1)][ij]
    for (int e = tid; e < q1x * q1y * nf * 9; e += 64) {
      const int ij = e % 9, r = e / 9, c1 = r % q1x, c2 = (r / q1x) % q1y, s3 = r / (q1x * q1y);
      double v = 0.0;
      for (int s2 = 0; s2 < nf; ++s2) v += Pm[1][c2 * nf + s2] * buf1[(((s3 * nf + s2) * q1x) + c1) * 9 + ij];
      buf0[e] = v;
    }
    __syncthreads();
    // z direction and store: C = c1 + q1x (c2 + q1y c3), column k = 9 C + ij = e
    for (int e = tid; e < npi * 9; e += 64) {
      const int ij = e % 9, C = e / 9;
      const int c1 = C % q1x, c2 = (C / q1x) % q1y, c3 = C / (q1x * q1y);
      double v = 0.0;
      for (int s3 = 0; s3 < nf; ++s3) v += Pm[2][c3 * nf + s3] * buf0[(((s3 * q1y + c2) * q1x) + c1) * 9 + ij];
      store_coef(a, Kp, t * 9 + ab, e, v, sc);
    }
    __syncthreads();
  }
  // zero the padded columns
  const int K = 9 * npi;
  for (int e = tid; e < 9 * (Kp - K); e += 64) {
    const int ab = e / (Kp - K), k = K + e % (Kp - K);
    store_coef(a, Kp, t * 9 + ab, k, 0.0, 1.0);
  }
}

int64_t coef_elem_bytes(igamt_precision prec) {
  return prec == IGAMT_F64 ? 8 : prec == IGAMT_F32 ? 4 : 4;  // split modes: two 2-byte planes
}

int64_t coef_bytes(const igamt_plan *P, igamt_precision prec) {
  const int64_t plane = P->n_tiles_pad * 9 * P->Kp;
  int64_t b = plane * coef_elem_bytes(prec);
  if (prec == IGAMT_F16X3) b += P->n_tiles_pad * 9 * 4;
  return align256(b);
}

int64_t blocks_bytes(const igamt_plan *P, igamt_precision prec) {
  return align256(P->n_tiles * P->n_pairs * 9 * (prec == IGAMT_F64 ? 8 : 4));
}

igamt_status launch_fit(igamt_plan *P, double E, double nu, igamt_precision prec, void *d_coef, void *stream,
                        int64_t t0, int64_t t1) {
  if (t1 < 0) t1 = P->n_tiles_pad;
  if (t0 < 0 || t1 > P->n_tiles_pad || t0 >= t1) { set_error("invalid tile range"); return IGAMT_EINVAL; }
  if (!(E > 0.0) || !std::isfinite(E) || !(nu > -1.0 && nu < 0.5)) {
    set_error("material constants must satisfy E > 0 and -1 < nu < 0.5");
    return IGAMT_EINVAL;
  }
  FitArgs a;
  for (int k = 0; k < 3; ++k) {
    a.knots[k] = P->dev.macro_knots[k];
    a.nM[k] = P->nM[k];
    a.box_a[k] = P->dev.box_a[k];
    a.box_h[k] = P->dev.box_h[k];
    a.tiles[k] = P->tiles[k];
  }
  a.ctrl = P->dev.macro_ctrl;
  a.wts = P->dev.macro_w;
  a.n_tiles = P->n_tiles;
  a.fx = P->dev.fit_x;
  a.fP3 = P->dev.fit_P3;
  for (int k = 0; k < 3; ++k) a.q1[k] = P->qd[k] + 1;
  a.nf = P->n_fit;
  a.Kp = P->Kp;
  a.prec = prec;
  a.tiled = split_tiled(P->Kp);
  a.lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  a.mu = E / (2.0 * (1.0 + nu));
  a.L3 = 1.0;
  for (int k = 0, off = 0; k < 3; off += a.q1[k] * a.nf, ++k) {
    double L = 0.0;
    for (int c = 0; c < a.q1[k]; ++c) {
      double rs = 0.0;
      for (int s = 0; s < a.nf; ++s) rs += std::fabs(P->fit_P3[off + c * a.nf + s]);
      L = std::fmax(L, rs);
    }
    a.L3 *= L;
  }
  a.out = d_coef;
  a.plane = P->n_tiles_pad * 9 * (int64_t)P->Kp;
  a.flag = P->dev.flag;
  const size_t shm = (size_t)28 * P->n_fit * P->n_fit * P->n_fit * sizeof(double);
  a.t0 = t0;
  const dim3 grid((unsigned)(t1 - t0)), block(64);
  hipStream_t s = (hipStream_t)stream;
#define FIT_LAUNCH(p0, p1, p2, qc)                                                                    \
  do {                                                                                                \
    if (shm > 65536) IGAMT_HIP(hipFuncSetAttribute((const void *)fit_kernel<p0, p1, p2, qc>,          \
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm)); \
    hipLaunchKernelGGL((fit_kernel<p0, p1, p2, qc>), grid, block, shm, s, a);                         \
  } while (0)
  // isotropic macro map and projection degree q <= 3 on q + 1 nodes: the compile-time shape
  const int qc = (P->qd[0] == P->qd[1] && P->qd[0] == P->qd[2] && P->n_fit == P->qd[0] + 1 && P->qd[0] >= 1 &&
                  P->qd[0] <= 3) ? P->qd[0] : 0;
  switch (IGAMT_DEGREE_KEY(P->pM[0], P->pM[1], P->pM[2])) {
#define FIT_ISO(p)                                                                                    \
  case IGAMT_DEGREE_KEY(p, p, p):                                                                     \
    if (qc == 1) FIT_LAUNCH(p, p, p, 1);                                                              \
    else if (qc == 2) FIT_LAUNCH(p, p, p, 2);                                                         \
    else if (qc == 3) FIT_LAUNCH(p, p, p, 3);                                                         \
    else FIT_LAUNCH(p, p, p, 0);                                                                      \
    break;
#define FIT_CASE(p0, p1, p2)                                                                          \
  case IGAMT_DEGREE_KEY(p0, p1, p2): FIT_LAUNCH(p0, p1, p2, 0); break;
    FIT_ISO(1) FIT_ISO(2) FIT_ISO(3) FIT_ISO(4) FIT_ISO(5) FIT_ISO(6)
    IGAMT_FOR_ANISO_MACRO_DEGREES(FIT_CASE)
#undef FIT_CASE
#undef FIT_ISO
#undef FIT_LAUNCH
    default:
      set_error("unsupported macro degrees (isotropic 1..6, or 1..3 per direction)");
      return IGAMT_EUNSUPPORTED;
  }
  IGAMT_LAUNCH_CHECK();
  return IGAMT_OK;
}

}  // namespace igamt

using namespace igamt;

extern "C" igamt_status igamt_workspace_bytes(const igamt_plan *P, igamt_precision prec, int64_t *cb, int64_t *bb) {
  if (!P || !cb || !bb) { set_error("NULL argument"); return IGAMT_EINVAL; }
  if (prec < IGAMT_F64 || prec > IGAMT_F16X3) { set_error("unknown precision"); return IGAMT_EINVAL; }
  *cb = coef_bytes(P, prec);
  *bb = blocks_bytes(P, prec);
  return IGAMT_OK;
}

extern "C" igamt_status igamt_fit(igamt_plan *P, double E, double nu, igamt_precision prec, void *d_coef,
                                  void *stream) {
  if (!P || !d_coef) { set_error("NULL argument"); return IGAMT_EINVAL; }
  if (prec < IGAMT_F64 || prec > IGAMT_F16X3) { set_error("unknown precision"); return IGAMT_EINVAL; }
  igamt_status st = ensure_device(P);
  if (st) return st;
  return launch_fit(P, E, nu, prec, d_coef, stream);
}
