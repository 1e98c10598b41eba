// Stage 1 of the assembly: macro-field fit (Section 3.2.2).
//
// One 64-thread workgroup per tile.  Every Gauss sample xi_s of the tile gets
// J = J_M(a + h xi_s) diag(h) (Cox-de Boor derivatives of the macro map),
// F = J^-1 and D = det J in FP64.  The projection coefficients
//   <A_ij,ab>_C = sum_s P[C, s] A_ij,ab(xi_s),  P = P1 (x) P1 (x) P1,
// (eq. (42) with the 1-D operator of eq. (23)-(24)) are applied sum-factorised,
// one direction at a time, with
//   A_ij,ab = D (lam F_ia F_jb + mu (F_i . F_j) delta_ab + mu F_ib F_ja),
// the Cartesian form of eq. (37) (F_i is row i of F).  The result is written in
// the column-major layout the contraction reads: coef[t][3a+b][9C+3i+j] (the split modes' planes
// tiled where the contraction keeps the table in LDS).  Two kernels: fit_q_kernel for an isotropic
// map and degree q <= 3 on q + 1 nodes (compile-time shape, passes in registers), fit_kernel for
// every other shape (passes through LDS).
#include <cstring>

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


// J diag(h) from the macro map's parameter Jacobian J, its inverse and determinant into FDs[0..9];
// a tile whose map folds (D <= 0) is flagged.
__device__ inline void fit_store_inverse(const FitArgs &a, int64_t t, const double (&hx)[3], double (&J)[3][3],
                                         double *FDs) {
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
    for (int c = 0; c < 3; ++c) FDs[3 * r + c] = F[r][c];
  FDs[9] = D;
}

// Jacobian, inverse and determinant at the fit sample xi_s = (fx[s1], fx[s2], fx[s3]) of tile t, into
// FD[s][0..8] (F row-major) and FD[s][9] (D); a tile whose map folds (D <= 0) is flagged.
template <int P0, int P1, int P2>
__device__ inline void fit_sample_jacobian(const FitArgs &a, int64_t t, const double (&ax)[3], const double (&hx)[3],
                                           int s1, int s2, int s3, double *FDs) {
  constexpr int PMX = max3(P0, P1, P2);
  double N[3][PMX + 1], dN[3][PMX + 1];
  int span[3];
  const double xh[3] = {ax[0] + hx[0] * a.fx[s1], ax[1] + hx[1] * a.fx[s2], ax[2] + hx[2] * a.fx[s3]};
  double J[3][3];
  spline_jacobian3<P0, P1, P2, true>(a.knots, a.nM, a.ctrl, a.wts, xh, J, span, N, dN);
  fit_store_inverse(a, t, hx, J, FDs);
}

// General shapes: projection degrees and fit nodes from the arguments (q_k + 1 <= n_fit per
// direction), the passes through LDS, one component (a, b) of A at a time.
template <int P0, int P1, int P2>
__global__ __launch_bounds__(64) void fit_kernel(FitArgs a) {
  extern __shared__ double smem[];
  const int nf = a.nf;
  const int q1x = a.q1[0], q1y = a.q1[1], q1z = a.q1[2];
  const int Kp = a.Kp;
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
  for (int s = tid; s < ns; s += 64)
    fit_sample_jacobian<P0, P1, P2>(a, t, ax, hx, s % nf, (s / nf) % nf, s / (nf * nf), FD + s * 10);
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
      buf0[e] = 3 * i + aa <= 3 * j + bb ? elastic_density(Fs + 3 * i, Fs + 3 * j, Fs[9], aa, bb, a.lam, a.mu)
                                         : elastic_density(Fs + 3 * j, Fs + 3 * i, Fs[9], bb, aa, a.lam, a.mu);
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


// Projection degree Q in every direction on Q + 1 fit nodes (the interpolating case), with the
// shape known at compile time.  After the Jacobians, lane l < 45 takes one of the 45 index pairs
// (u, v) = (3 i + a, 3 j + b) with u <= v: it evaluates A_ij,ab at every sample, which is also
// A_ji,ba, and runs the three 1-D passes on them in registers (the same sums in the same order as
// the LDS passes of fit_kernel).  The results go into an LDS image of the tile's nine coefficient
// rows in the stored precision (entry (ab, 9 C + ij) from lane (u, v), entry (ba, 9 C + ji) from
// the same lane; FP64 in two passes of at most five rows), which the workgroup then writes out as
// 16-byte pieces, consecutive lanes on consecutive pieces.  F16X3: the column scale is the maximum
// of |A_ij,ab| over the column's lanes (an LDS atomic maximum on the bits of non-negative doubles),
// the same for (a, b) and (b, a).
template <int Q, int PREC>
struct FitShape {
  static constexpr int NF = Q + 1, NS = NF * NF * NF, K = 9 * NS;
  static constexpr int KP = (K + kColPad - 1) / kColPad * kColPad;
  static constexpr int ROWS = PREC == IGAMT_F64 ? 5 : 9;              // coefficient rows per LDS image
  static constexpr int STAGE = ROWS * KP * (PREC == IGAMT_F64 ? 8 : 4);  // bytes: values, or hi and lo planes
};

template <int P0, int P1, int P2, int Q, int PREC>
__global__ __launch_bounds__(64) void fit_q_kernel(FitArgs a) {
  using S = FitShape<Q, PREC>;
  constexpr int NF = S::NF, NS = S::NS, K = S::K, KP = S::KP;
  extern __shared__ __align__(16) unsigned char stage[];
  __shared__ double FD[NS * 10];
  __shared__ unsigned long long cmax[9];  // F16X3: bits of the column maxima (non-negative doubles)
  __shared__ double NB[3][NF][2][P0 + 1];   // per direction and node: B-spline values, derivatives
  __shared__ int SP[3][NF];                 // and spans
  static_assert(P0 == P1 && P1 == P2, "isotropic macro maps only");
  const int tid = threadIdx.x;
  const int64_t t = a.t0 + blockIdx.x;

  if (t >= a.n_tiles) {  // padding tile: zeros
    for (int e = tid; e < 9 * KP; e += 64) store_coef(a, KP, t * 9 + e / KP, e % KP, 0.0, 1.0);
    if (PREC == IGAMT_F16X3 && tid < 9) ((float *)((uint16_t *)a.out + 2 * a.plane))[t * 9 + tid] = 1.0f;
    return;
  }
  const int tx = (int)(t % a.tiles[0]);
  const int ty = (int)((t / a.tiles[0]) % a.tiles[1]);
  const int tz = (int)(t / ((int64_t)a.tiles[0] * a.tiles[1]));
  const double ax[3] = {a.box_a[0][tx], a.box_a[1][ty], a.box_a[2][tz]};
  const double hx[3] = {a.box_h[0][tx], a.box_h[1][ty], a.box_h[2][tz]};
  // the spans and 1-D basis values and derivatives at the Q + 1 nodes of each direction, one lane
  // each, shared by the samples (the values spline_jacobian3 would compute at every sample)
  if (tid < 3 * NF) {
    const int d = tid / NF, sn = tid % NF;
    const double x = (d == 0 ? ax[0] : d == 1 ? ax[1] : ax[2]) + (d == 0 ? hx[0] : d == 1 ? hx[1] : hx[2]) * a.fx[sn];
    const double *U = d == 0 ? a.knots[0] : d == 1 ? a.knots[1] : a.knots[2];
    const int sp = find_span(U, d == 0 ? a.nM[0] : d == 1 ? a.nM[1] : a.nM[2], P0, x);
    double N[P0 + 1], dN[P0 + 1];
    bspline_ders<P0>(U, sp, x, N, dN);
    SP[d][sn] = sp;
#pragma unroll
    for (int r = 0; r <= P0; ++r) {
      NB[d][sn][0][r] = N[r];
      NB[d][sn][1][r] = dN[r];
    }
  }
  if (PREC == IGAMT_F16X3 && tid < 9) cmax[tid] = 0;
  __syncthreads();
  if (tid < NS) {
    const int si[3] = {tid % NF, (tid / NF) % NF, tid / (NF * NF)};
    int span[3];
    double N[3][P0 + 1], dN[3][P0 + 1];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      span[k] = SP[k][si[k]];
#pragma unroll
      for (int r = 0; r <= P0; ++r) {
        N[k][r] = NB[k][si[k]][0][r];
        dN[k][r] = NB[k][si[k]][1][r];
      }
    }
    double J[3][3];
    spline_jacobian_sum<P0, P1, P2, (P0 > 3)>(a.nM, a.ctrl, a.wts, span, N, dN, J);
    fit_store_inverse(a, t, hx, J, FD + tid * 10);
  }

  // this lane's pair (u, v), u <= v (lanes 45..63 repeat pair 44 and store nothing)
  int u = 0, rem = min(tid, 44);
  while (rem >= 9 - u) { rem -= 9 - u; ++u; }
  const int v = u + rem;
  const int i = u / 3, aa = u % 3, j = v / 3, bb = v % 3;
  const bool act = tid < 45;
  // the 1-D operator, the same in every direction here (checked by the launcher), in scalar registers
  double P[NF][NF];
#pragma unroll
  for (int c = 0; c < NF; ++c)
#pragma unroll
    for (int s = 0; s < NF; ++s) P[c][s] = uniform_f64(a.fP3[c * NF + s]);
  __syncthreads();

  double val[NS];
  double m = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    val[s] = elastic_density(FD + s * 10 + 3 * i, FD + s * 10 + 3 * j, FD[s * 10 + 9], aa, bb, a.lam, a.mu);
    m = fmax(m, fabs(val[s]));
  }
  // x: (s3, s2, s1) -> (s3, s2, c1); y: (s3, s2, c1) -> (s3, c2, c1); z: (s3, c2, c1) -> (c3, c2, c1)
#pragma unroll
  for (int l = 0; l < NF * NF; ++l) {
    double o[NF];
#pragma unroll
    for (int c = 0; c < NF; ++c) {
      double w = 0.0;
#pragma unroll
      for (int s = 0; s < NF; ++s) w += P[c][s] * val[l * NF + s];
      o[c] = w;
    }
#pragma unroll
    for (int c = 0; c < NF; ++c) val[l * NF + c] = o[c];
  }
#pragma unroll
  for (int s3 = 0; s3 < NF; ++s3)
#pragma unroll
    for (int c1 = 0; c1 < NF; ++c1) {
      double o[NF];
#pragma unroll
      for (int c = 0; c < NF; ++c) {
        double w = 0.0;
#pragma unroll
        for (int s = 0; s < NF; ++s) w += P[c][s] * val[(s3 * NF + s) * NF + c1];
        o[c] = w;
      }
#pragma unroll
      for (int c = 0; c < NF; ++c) val[(s3 * NF + c) * NF + c1] = o[c];
    }
#pragma unroll
  for (int l = 0; l < NF * NF; ++l) {
    double o[NF];
#pragma unroll
    for (int c = 0; c < NF; ++c) {
      double w = 0.0;
#pragma unroll
      for (int s = 0; s < NF; ++s) w += P[c][s] * val[s * NF * NF + l];
      o[c] = w;
    }
#pragma unroll
    for (int c = 0; c < NF; ++c) val[c * NF * NF + l] = o[c];
  }

  double sc = 1.0;
  if (PREC == IGAMT_F16X3) {  // |coef| <= L_x L_y L_z max|A_ij,ab| with L_k the max row sum of |P_k|
    const int col = min(3 * aa + bb, 3 * bb + aa);  // (a, b) and (b, a) share the maximum
    if (act) atomicMax(&cmax[col], (unsigned long long)__double_as_longlong(m));
    __syncthreads();
    sc = f16_scale_for(__longlong_as_double((long long)cmax[col]) * a.L3);
    if (act && i == 0 && j == 0) {
      float *inv = (float *)((uint16_t *)a.out + 2 * a.plane) + t * 9;
      inv[3 * aa + bb] = (float)(1.0 / sc);
      inv[3 * bb + aa] = (float)(1.0 / sc);
    }
  }

  // LDS image of the nine rows in the stored precision
  auto put = [&](int r, int k, double x, double scale) {
    if (PREC == IGAMT_F64) {
      ((double *)stage)[r * KP + k] = x;
    } else if (PREC == IGAMT_F32) {
      ((float *)stage)[r * KP + k] = (float)x;
    } else {
      uint16_t hi, lo;
      if (PREC == IGAMT_BF16X3)
        split_bf16(x, hi, lo);
      else
        split_f16(x * scale, hi, lo);
      ((uint16_t *)stage)[r * KP + k] = hi;
      ((uint16_t *)stage)[9 * KP + r * KP + k] = lo;
    }
  };
  // FP64: the rows in two passes of at most five, which halves the image (and the LDS a workgroup holds)
  constexpr int RH = S::ROWS;
#pragma unroll
  for (int r0 = 0; r0 < 9; r0 += RH) {
    if (r0) __syncthreads();  // the previous pass's pieces are read out
    if (act) {
      const int r1 = 3 * aa + bb - r0, r2 = 3 * bb + aa - r0;
#pragma unroll
      for (int C = 0; C < NS; ++C) {
        if (r1 >= 0 && r1 < RH) put(r1, 9 * C + 3 * i + j, val[C], sc);
        if (u != v && r2 >= 0 && r2 < RH) put(r2, 9 * C + 3 * j + i, val[C], sc);
      }
    }
    const int nr = min(RH, 9 - r0);  // rows in this pass
    if constexpr (KP > K)
      for (int e = tid; e < nr * (KP - K); e += 64) put(e / (KP - K), K + e % (KP - K), 0.0, 1.0);
    __syncthreads();

    // 16-byte pieces: rows of doubles / floats, or runs of 8 split entries of one column
    if (PREC == IGAMT_F64 || PREC == IGAMT_F32) {
      constexpr int W = PREC == IGAMT_F64 ? 2 : 4;  // entries per piece
      for (int e = tid; e < nr * KP / W; e += 64) {
        const int r = e / (KP / W), k = (e % (KP / W)) * W;
        const uint4 x = *(const uint4 *)(stage + (r * KP + k) * (16 / W));
        *(uint4 *)((unsigned char *)a.out + ((t * 9 + r0 + r) * KP + k) * (16 / W)) = x;
      }
    } else {
      constexpr bool TILED = split_tiled(KP);
      for (int e = tid; e < 2 * 9 * KP / 8; e += 64) {
        // tiled: the columns of one 8-entry run adjacent in memory, so the row index runs fastest
        const int pl = e / (9 * KP / 8), f = e % (9 * KP / 8);
        const int r = TILED ? f % 9 : f / (KP / 8), k = (TILED ? f / 9 : f % (KP / 8)) * 8;
        const uint4 x = *(const uint4 *)((const uint16_t *)stage + pl * 9 * KP + r * KP + k);
        *(uint4 *)((uint16_t *)a.out + pl * a.plane + split_coef_index(t * 9 + r, k, KP, TILED)) = x;
      }
    }
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

template <int PM, int Q>
void launch_fit_q(const FitArgs &a, igamt_precision prec, dim3 grid, hipStream_t s) {
  switch (prec) {
    case IGAMT_F64:
      hipLaunchKernelGGL((fit_q_kernel<PM, PM, PM, Q, IGAMT_F64>), grid, dim3(64), (FitShape<Q, IGAMT_F64>::STAGE), s, a);
      break;
    case IGAMT_F32:
      hipLaunchKernelGGL((fit_q_kernel<PM, PM, PM, Q, IGAMT_F32>), grid, dim3(64), (FitShape<Q, IGAMT_F32>::STAGE), s, a);
      break;
    case IGAMT_BF16X3:
      hipLaunchKernelGGL((fit_q_kernel<PM, PM, PM, Q, IGAMT_BF16X3>), grid, dim3(64), (FitShape<Q, IGAMT_BF16X3>::STAGE), s,
                         a);
      break;
    default:
      hipLaunchKernelGGL((fit_q_kernel<PM, PM, PM, Q, IGAMT_F16X3>), grid, dim3(64), (FitShape<Q, IGAMT_F16X3>::STAGE), s,
                         a);
      break;
  }
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
#define FIT_LAUNCH(p0, p1, p2)                                                                        \
  do {                                                                                                \
    if (shm > 65536) IGAMT_HIP(hipFuncSetAttribute((const void *)fit_kernel<p0, p1, p2>,              \
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm)); \
    hipLaunchKernelGGL((fit_kernel<p0, p1, p2>), grid, block, shm, s, a);                             \
  } while (0)
  // isotropic macro map and projection degree q <= 3 on q + 1 nodes: the compile-time shape
  // and the same 1-D operator in every direction
  int qc = (P->qd[0] == P->qd[1] && P->qd[0] == P->qd[2] && P->n_fit == P->qd[0] + 1 && P->qd[0] >= 1 &&
            P->qd[0] <= 3) ? P->qd[0] : 0;
  if (qc) {
    const size_t n1 = (size_t)(qc + 1) * (qc + 1);
    if (std::memcmp(P->fit_P3.data(), P->fit_P3.data() + n1, n1 * sizeof(double)) != 0 ||
        std::memcmp(P->fit_P3.data(), P->fit_P3.data() + 2 * n1, n1 * sizeof(double)) != 0)
      qc = 0;
  }
  switch (IGAMT_DEGREE_KEY(P->pM[0], P->pM[1], P->pM[2])) {
#define FIT_ISO(p)                                                                                    \
  case IGAMT_DEGREE_KEY(p, p, p):                                                                     \
    if (qc == 1) launch_fit_q<p, 1>(a, prec, grid, s);                                                \
    else if (qc == 2) launch_fit_q<p, 2>(a, prec, grid, s);                                           \
    else if (qc == 3) launch_fit_q<p, 3>(a, prec, grid, s);                                           \
    else FIT_LAUNCH(p, p, p);                                                                         \
    break;
#define FIT_CASE(p0, p1, p2)                                                                          \
  case IGAMT_DEGREE_KEY(p0, p1, p2): FIT_LAUNCH(p0, p1, p2); break;
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
