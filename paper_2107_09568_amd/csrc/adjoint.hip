// Shape sensitivity of u^T K^pi u with respect to the macro control points
// (Section 4.1.2, eq. (69)-(73)), u fixed.
//
// Per tile t, with Coef^(t) the fitted coefficients (eq. (42)) and the table of
// eq. (57):
//   u^T K^(t) u = sum_{k,ab} Coef[k][ab] W[k][ab],
//   W = table^T U,  U[p][ab] = m_p u_(A,a) u_(B,b),  m_p = 2 if A < B else 1,
// W being the adjoint field of eq. (71)-(73): the lookup table contracted with
// products of the tile's displacement coefficients.  Then
//   Abar(xi_s) = P^T W                       (transpose of the projection)
//   (Fbar, Dbar) from Abar                   (adjoint of A = D G(F))
//   Jbar = -F^T Fbar F^T + Dbar D F^T        (F = J^-1, D = det J)
//   mbar_i += sum_n Jbar[c][n] h_n d_n N_i   (J = J_M(a + h xi) diag(h))
// Kernels: (1) the fit (FP64); (2) U from the gathered displacement, then the
// transposed contraction W = table^T U on the forward MFMA kernel (W stored
// [t][k][ab]); (3) the FP64 fit adjoint, one workgroup per tile, giving per-tile
// gradients of the macro control points the tile touches and the tile's share of
// u^T K u; (4) reductions over the tiles in a fixed order (bitwise reproducible).
#include "device_common.h"

namespace igamt {

// ---- (2) U, then W = table^T U on MFMA ------------------------------------------
// U is formed once per tile, stored like the coefficients of the forward product (one
// column per (tile, ab), contiguous over the pairs p), so that W = table^T U runs on the
// forward contraction kernel with the transposed table as its row operand.
struct UFormArgs {
  const int32_t *desc;    // [M][kDescWords] pair descriptors (local coordinates of A and B)
  const double *u;        // global displacement [3 n_global]
  void *U;                // [n_tiles_pad][9][Mp] (double or float)
  int64_t M, Mp, n_tiles, n_tiles_pad;
  int tiles[3], nT[3], NG[3];
};

template <typename E>
__global__ __launch_bounds__(256) void u_form_kernel(UFormArgs a) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t t = blockIdx.y;
  if (p >= a.Mp || t >= a.n_tiles_pad) return;
  double v[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) v[k] = 0.0;
  if (p < a.M && t < a.n_tiles) {
    const int32_t w0 = a.desc[kDescWords * p], w1 = a.desc[kDescWords * p + 1];
    const int ai[3] = {w0 & 255, (w0 >> 8) & 255, (w0 >> 16) & 255};
    const int bi[3] = {w1 & 255, (w1 >> 8) & 255, (w1 >> 16) & 255};
    const int tt[3] = {(int)(t % a.tiles[0]), (int)((t / a.tiles[0]) % a.tiles[1]),
                       (int)(t / ((int64_t)a.tiles[0] * a.tiles[1]))};
    int64_t GA = 0, GB = 0;
    for (int k = 2; k >= 0; --k) {
      GA = GA * a.NG[k] + tt[k] * (a.nT[k] - 1) + ai[k];
      GB = GB * a.NG[k] + tt[k] * (a.nT[k] - 1) + bi[k];
    }
    const double m = GA == GB ? 1.0 : 2.0;   // A < B pairs stand for both orders
    const double uA[3] = {a.u[3 * GA], a.u[3 * GA + 1], a.u[3 * GA + 2]};
    const double uB[3] = {a.u[3 * GB], a.u[3 * GB + 1], a.u[3 * GB + 2]};
#pragma unroll
    for (int aa = 0; aa < 3; ++aa)
#pragma unroll
      for (int bb = 0; bb < 3; ++bb) v[3 * aa + bb] = m * uA[aa] * uB[bb];
  }
  E *U = (E *)a.U;
#pragma unroll
  for (int k = 0; k < 9; ++k) U[(t * 9 + k) * a.Mp + p] = (E)v[k];
}

// ---- (3) fit adjoint ---------------------------------------------------------------
struct FitAdjArgs {
  const double *knots[3];
  int nM[3];
  const double *ctrl;
  const double *wts;      // NURBS weights of the macro map, or null (B-spline)
  const double *box_a[3];
  const double *box_h[3];
  const int32_t *ctrl_lo[3];
  int tiles[3], Lc[3];
  int64_t n_tiles;
  const double *fx;
  const double *fP3;      // per-direction 1-D projection operators [q1[k]][nf], concatenated
  int q1[3], nf, Kp;
  bool w_f64;
  double lam, mu;
  const double *coef;   // [n_tiles_pad][9][Kp] FP64
  const void *W;        // [n_tiles][Kp][9], double or float
  double *local_grad;   // [n_tiles][Lz][Ly][Lx][3]
  double *uKu_part;     // [n_tiles]
  int32_t *flag;
  int Lm;               // max(Lc): row length of the 1-D factor tables
  int64_t xt_off;       // doubles of dynamic LDS before the 1-D factor tables
};

constexpr int kFitAdjThreads = 256;   // threads per tile in the fit adjoint

// GJ (1 or 3): (i, j) blocks carried through the passes together (the same i, consecutive j)
template <int P0, int P1, int P2, int GJ>
__global__ __launch_bounds__(kFitAdjThreads) void fit_adjoint_kernel(FitAdjArgs a) {
  constexpr int PMX = max3(P0, P1, P2);
  constexpr int PD[3] = {P0, P1, P2};
  constexpr int NC = 9 * GJ;         // components per pass: (j, a, b)
  extern __shared__ double smem[];
  const int nf = a.nf, q1x = a.q1[0], q1y = a.q1[1], q1z = a.q1[2];
  const int ns = nf * nf * nf, npi = q1x * q1y * q1z;
  double *FD = smem;                 // [ns][10]  F, D
  double *FB = FD + ns * 10;         // [ns][10]  Fbar (before the factor D), Dbar
  double *buf0 = FB + ns * 10;       // [max(ns, npi)][NC]
  double *buf1 = buf0 + ns * NC;     // [ns][NC]
  __shared__ double Pm[3][(kMaxQ + 1) * kMaxFit];
  __shared__ double NB[3][kMaxFit][kMaxDegree + 1], DB[3][kMaxFit][kMaxDegree + 1];
  __shared__ int SP[3][kMaxFit];
  __shared__ double red[kFitAdjThreads];
  const int tid = threadIdx.x;
  const int64_t t = blockIdx.x;
  const int64_t tbase = t * 9 * (int64_t)a.Kp;
  for (int e = tid; e < q1x * nf; e += kFitAdjThreads) Pm[0][e] = a.fP3[e];
  for (int e = tid; e < q1y * nf; e += kFitAdjThreads) Pm[1][e] = a.fP3[q1x * nf + e];
  for (int e = tid; e < q1z * nf; e += kFitAdjThreads) Pm[2][e] = a.fP3[(q1x + q1y) * nf + e];
  const int tt[3] = {(int)(t % a.tiles[0]), (int)((t / a.tiles[0]) % a.tiles[1]),
                     (int)(t / ((int64_t)a.tiles[0] * a.tiles[1]))};
  const double ax[3] = {a.box_a[0][tt[0]], a.box_a[1][tt[1]], a.box_a[2][tt[2]]};
  const double hx[3] = {a.box_h[0][tt[0]], a.box_h[1][tt[1]], a.box_h[2][tt[2]]};
  // 1-D macro basis at the tile's sample abscissae (tensor grid)
  for (int e = tid; e < 3 * nf; e += kFitAdjThreads) {
    const int k = e / nf, s = e % nf;
    const double x = ax[k] + hx[k] * a.fx[s];
    const int sp = find_span(a.knots[k], a.nM[k], PD[k], x);
    double N[PMX + 1], dN[PMX + 1];
    bspline_ders_dir<P0, P1, P2>(k, a.knots[k], sp, x, N, dN);
    SP[k][s] = sp;
    for (int r = 0; r <= PMX; ++r) { NB[k][s][r] = N[r]; DB[k][s][r] = dN[r]; }
  }
  __syncthreads();   // the basis tables are read by the sample loop
  // F and D at the samples (from the shared 1-D bases: the values spline_jacobian3 computes); zero
  // the adjoint accumulators
  for (int s = tid; s < ns; s += kFitAdjThreads) {
    const int si[3] = {s % nf, (s / nf) % nf, s / (nf * nf)};
    double J[3][3], N[3][PMX + 1], dN[3][PMX + 1];
    int span[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
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
      for (int k = 0; k < 3; ++k) J[c][k] *= hx[k];
    double F[3][3];
    const double D = inv3(J, F);
    if (!(D > 0.0) || !isfinite(D)) atomicMin(a.flag, (int32_t)t);
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) FD[s * 10 + 3 * r + c] = F[r][c];
    FD[s * 10 + 9] = D;
    for (int k = 0; k < 10; ++k) FB[s * 10 + k] = 0.0;
  }
  // this tile's share of u^T K u (fixed-order block reduction)
  {
    // e = tid + 256 j in ascending j, four terms' loads issued before their products are added
    const int n9 = 9 * a.Kp;
    double part = 0.0;
    for (int e0 = 0; e0 < n9; e0 += 4 * kFitAdjThreads) {
      double cv[4], wv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + u * kFitAdjThreads + tid;
        const bool in = e < n9;
        const int ab = in ? e / a.Kp : 0, k = in ? e - ab * a.Kp : 0;
        const int64_t wi = (t * a.Kp + k) * 9 + ab;   // W is stored [t][k][ab]
        cv[u] = in ? a.coef[tbase + e] : 0.0;
        wv[u] = in ? (a.w_f64 ? ((const double *)a.W)[wi] : (double)((const float *)a.W)[wi]) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (e0 + u * kFitAdjThreads + tid < n9) part += cv[u] * wv[u];
    }
    red[tid] = part;
  }
  __syncthreads();
  for (int s = kFitAdjThreads / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) a.uKu_part[t] = red[0];

  for (int ij0 = 0; ij0 < 9; ij0 += GJ) {
    // W blocks of (ij0 .. ij0 + GJ - 1): buf0[C][jj 9 + ab], contiguous in W ([t][9 C + ij][ab])
    for (int e = tid; e < npi * NC; e += kFitAdjThreads) {
      const int C = e / NC, q = e - C * NC;
      const int64_t idx = (t * a.Kp + 9 * C + ij0) * 9 + q;
      buf0[e] = a.w_f64 ? ((const double *)a.W)[idx] : (double)((const float *)a.W)[idx];
    }
    __syncthreads();
    // transpose of the z pass: buf1[(s3, c2, c1)][q] = sum_c3 P[c3][s3] W[(c3, c2, c1)][q]
    for (int e = tid; e < nf * q1y * q1x * NC; e += kFitAdjThreads) {
      const int q = e % NC, r = e / NC, c1 = r % q1x, c2 = (r / q1x) % q1y, s3 = r / (q1x * q1y);
      double v = 0.0;
      for (int c3 = 0; c3 < q1z; ++c3) v += Pm[2][c3 * nf + s3] * buf0[((c3 * q1y + c2) * q1x + c1) * NC + q];
      buf1[e] = v;
    }
    __syncthreads();
    // transpose of the y pass: buf0[(s3, s2, c1)][q]
    for (int e = tid; e < nf * nf * q1x * NC; e += kFitAdjThreads) {
      const int q = e % NC, r = e / NC, c1 = r % q1x, s2 = (r / q1x) % nf, s3 = r / (q1x * nf);
      double v = 0.0;
      for (int c2 = 0; c2 < q1y; ++c2) v += Pm[1][c2 * nf + s2] * buf1[((s3 * q1y + c2) * q1x + c1) * NC + q];
      buf0[e] = v;
    }
    __syncthreads();
    // transpose of the x pass: buf1[(s3, s2, s1)][q] = Abar at sample s
    for (int e = tid; e < ns * NC; e += kFitAdjThreads) {
      const int q = e % NC, s = e / NC, s1 = s % nf, s23 = s / nf;
      double v = 0.0;
      for (int c1 = 0; c1 < q1x; ++c1) v += Pm[0][c1 * nf + s1] * buf0[(s23 * q1x + c1) * NC + q];
      buf1[e] = v;
    }
    __syncthreads();
    // accumulate the adjoint of A_ij = D G_ij(F) into (Fbar / D, Dbar), one sample per thread,
    // (i, j) in ascending order
    for (int s = tid; s < ns; s += kFitAdjThreads)
    for (int jj = 0; jj < GJ; ++jj) {
      const int i = (ij0 + jj) / 3, j = (ij0 + jj) % 3;
      const double *F = FD + s * 10;
      const double D = F[9];
      const double *Ab = buf1 + s * NC + 9 * jj;     // Abar_ij[a][b]
      double *fb = FB + s * 10;
      const double fij = F[3 * i] * F[3 * j] + F[3 * i + 1] * F[3 * j + 1] + F[3 * i + 2] * F[3 * j + 2];
      double T = 0.0, dbar = 0.0;
      for (int aa = 0; aa < 3; ++aa) {
        T += Ab[4 * aa];
        for (int bb = 0; bb < 3; ++bb) {
          const double g = a.lam * F[3 * i + aa] * F[3 * j + bb] + (aa == bb ? a.mu * fij : 0.0) +
                           a.mu * F[3 * i + bb] * F[3 * j + aa];
          dbar += Ab[3 * aa + bb] * g;
        }
      }
      fb[9] += dbar;
      for (int c = 0; c < 3; ++c) {
        double si = 0.0, sj = 0.0;
        for (int b = 0; b < 3; ++b) {
          // lambda terms: d/dF_ic of F_ia F_jb uses Abar[c][b] F_jb; d/dF_jc uses Abar[a][c] F_ia
          si += a.lam * Ab[3 * c + b] * F[3 * j + b] + a.mu * Ab[3 * b + c] * F[3 * j + b];
          sj += a.lam * Ab[3 * b + c] * F[3 * i + b] + a.mu * Ab[3 * c + b] * F[3 * i + b];
        }
        si += a.mu * T * F[3 * j + c];
        sj += a.mu * T * F[3 * i + c];
        fb[3 * i + c] += si;
        fb[3 * j + c] += sj;
      }
      (void)D;
    }
    __syncthreads();
  }
  // Jbar at each sample, scaled by h (stored over FB[s][0..8])
  for (int s = tid; s < ns; s += kFitAdjThreads) {
    const double *F = FD + s * 10;
    double *fb = FB + s * 10;
    const double D = F[9];
    double Fb[3][3];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) Fb[r][c] = D * fb[3 * r + c];   // Gbar = D Abar
    // M = F^T Fb F^T:  M[c][n] = sum_{r,m} F[r][c] Fb[r][m] F[n][m]
    double Jb[3][3];
    for (int c = 0; c < 3; ++c)
      for (int n = 0; n < 3; ++n) {
        double m = 0.0;
        for (int r = 0; r < 3; ++r)
          for (int q = 0; q < 3; ++q) m += F[3 * r + c] * Fb[r][q] * F[3 * n + q];
        Jb[c][n] = -m + fb[9] * D * F[3 * n + c];
      }
    for (int c = 0; c < 3; ++c)
      for (int n = 0; n < 3; ++n) fb[3 * c + n] = Jb[c][n] * hx[n];
  }
  __syncthreads();
  // NURBS: 1 / W and sum_n JbarH[c][n] d_n W / W^2 per sample (buf0 is free here)
  double *WQ = buf0;
  if (a.wts) {
    for (int s = tid; s < ns; s += kFitAdjThreads) {
      const int si[3] = {s % nf, (s / nf) % nf, s / (nf * nf)};
      rational_terms3<P0, P1, P2>(a.wts, a.nM, SP, NB, DB, si, FB + s * 10, WQ + s * 4);
    }
    __syncthreads();
  }
  // local control-point gradients: mbar[i][c] = sum_s sum_n JbarH[s][c][n] d_n R_i(s)
  // (R_i = N_i for a B-spline map; w_i (d_n N_i - N_i d_n W / W) / W for a NURBS map).  The basis
  // is a tensor product, so its factors are tabulated per direction: XV[k][s][l] = N_r(x_s) and
  // XD[k][s][l] = N_r'(x_s) with r = lo_k + l - (span_s - p), zero where l is outside the support
  // of the sample (such samples add an exact zero).
  const int L0 = a.Lc[0], L1 = a.Lc[1], L2 = a.Lc[2], Lm = a.Lm;
  const int lo[3] = {a.ctrl_lo[0][tt[0]], a.ctrl_lo[1][tt[1]], a.ctrl_lo[2][tt[2]]};
  double *XV = smem + a.xt_off, *XD = XV + 3 * nf * Lm;   // [3][nf][Lm] each
  for (int e = tid; e < 3 * nf * Lm; e += kFitAdjThreads) {
    const int k = e / (nf * Lm), rem = e - k * nf * Lm, sk = rem / Lm, l = rem - sk * Lm;
    const int r = lo[k] + l - (SP[k][sk] - PD[k]);
    const bool on = r >= 0 && r <= PD[k];
    const int rc = on ? r : 0;
    XV[e] = on ? NB[k][sk][rc] : 0.0;
    XD[e] = on ? DB[k][sk][rc] : 0.0;
  }
  __syncthreads();
  double *lg = a.local_grad + t * (int64_t)L0 * L1 * L2 * 3;
  for (int e = tid; e < L0 * L1 * L2 * 3; e += kFitAdjThreads) {
    const int c = e % 3, li = e / 3;
    const int l[3] = {li % L0, (li / L0) % L1, li / (L0 * L1)};
    double g = 0.0;
    for (int s3 = 0; s3 < nf; ++s3) {
      const double v2 = XV[(2 * nf + s3) * Lm + l[2]], d2 = XD[(2 * nf + s3) * Lm + l[2]];
      for (int s2 = 0; s2 < nf; ++s2) {
        const double v1 = XV[(nf + s2) * Lm + l[1]], d1 = XD[(nf + s2) * Lm + l[1]];
        for (int s1 = 0; s1 < nf; ++s1) {
          const double v0 = XV[s1 * Lm + l[0]], d0 = XD[s1 * Lm + l[0]];
          const int s = (s3 * nf + s2) * nf + s1;
          const double *jb = FB + s * 10 + 3 * c;
          const double tb = jb[0] * d0 * v1 * v2 + jb[1] * v0 * d1 * v2 + jb[2] * v0 * v1 * d2;
          g += a.wts ? tb * WQ[s * 4] - v0 * v1 * v2 * WQ[s * 4 + 1 + c] : tb;
        }
      }
    }
    lg[e] = a.wts ? g * local_weight(a.wts, a.nM, lo, l)
                  : g;
  }
}

// ---- (4) reductions ------------------------------------------------------------------
struct GradReduceArgs {
  const int32_t *off[3];
  const int32_t *lst[3];
  int nM[3], tiles[3], Lc[3];
  const double *local_grad;
  double *grad;
};

// One workgroup per macro control point: the (tile, local index) contributions are split
// over the threads in a fixed strided order and combined by a fixed tree, so the gradient is
// bitwise reproducible.
__global__ __launch_bounds__(256) void grad_reduce_kernel(GradReduceArgs a) {
  __shared__ double red[3][256];
  const int64_t m = blockIdx.x;
  const int tid = threadIdx.x;
  const int ix = (int)(m % a.nM[0]), iy = (int)((m / a.nM[0]) % a.nM[1]), iz = (int)(m / ((int64_t)a.nM[0] * a.nM[1]));
  const int ex0 = a.off[0][ix], nx = a.off[0][ix + 1] - ex0;
  const int ey0 = a.off[1][iy], ny = a.off[1][iy + 1] - ey0;
  const int ez0 = a.off[2][iz], nz = a.off[2][iz + 1] - ez0;
  double g[3] = {0.0, 0.0, 0.0};
  for (int f = tid; f < nx * ny * nz; f += 256) {
    const int ex = ex0 + f % nx, ey = ey0 + (f / nx) % ny, ez = ez0 + f / (nx * ny);
    const int64_t t = a.lst[0][2 * ex] + (int64_t)a.tiles[0] * (a.lst[1][2 * ey] + (int64_t)a.tiles[1] * a.lst[2][2 * ez]);
    const int lx = a.lst[0][2 * ex + 1], ly = a.lst[1][2 * ey + 1], lz = a.lst[2][2 * ez + 1];
    const double *src = a.local_grad + (((t * a.Lc[2] + lz) * a.Lc[1] + ly) * a.Lc[0] + lx) * 3;
#pragma unroll
    for (int c = 0; c < 3; ++c) g[c] += src[c];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) red[c][tid] = g[c];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s)
#pragma unroll
      for (int c = 0; c < 3; ++c) red[c][tid] += red[c][tid + s];
    __syncthreads();
  }
  if (tid < 3) a.grad[3 * m + tid] = red[tid][0];
}

__global__ __launch_bounds__(256) void sum_kernel(const double *x, int64_t n, double *out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += x[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

igamt_status launch_grad_reduce(igamt_plan *P, const double *local_grad, double *grad, void *stream) {
  GradReduceArgs g;
  for (int k = 0; k < 3; ++k) {
    g.off[k] = P->dev.ctrl_tiles_off[k];
    g.lst[k] = P->dev.ctrl_tiles[k];
    g.nM[k] = P->nM[k];
    g.tiles[k] = P->tiles[k];
    g.Lc[k] = P->Lc[k];
  }
  g.local_grad = local_grad;
  g.grad = grad;
  const int64_t n_ctrl = (int64_t)P->nM[0] * P->nM[1] * P->nM[2];
  hipLaunchKernelGGL(grad_reduce_kernel, dim3((unsigned)n_ctrl), dim3(256), 0, (hipStream_t)stream, g);
  IGAMT_LAUNCH_CHECK();
  return IGAMT_OK;
}

igamt_status launch_sum(const double *x, int64_t n, double *out, void *stream) {
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, x, n, out);
  IGAMT_LAUNCH_CHECK();
  return IGAMT_OK;
}

static int64_t grad_ws_layout(const igamt_plan *P, igamt_precision prec, int64_t off[6]) {
  const int64_t plane = P->n_tiles_pad * 9 * P->Kp;
  const int64_t eb = prec == IGAMT_F64 ? 8 : 4;
  off[0] = 0;                                                        // coef (FP64)
  off[1] = off[0] + align256(plane * 8);                             // W [n_tiles][Kp][9]
  off[2] = off[1] + align256(plane * eb);                            // local gradients
  off[3] = off[2] + align256(P->n_tiles * (int64_t)P->Lc[0] * P->Lc[1] * P->Lc[2] * 3 * 8);
  off[4] = off[3] + align256(P->n_tiles * 8);                        // uKu parts
  off[5] = off[4] + align256(P->n_tiles_pad * 9 * P->Mp * eb);       // U [n_tiles_pad][9][Mp]
  return off[5];
}

}  // namespace igamt

using namespace igamt;

extern "C" igamt_status igamt_grad_workspace_bytes(const igamt_plan *P, igamt_precision prec, int64_t *bytes) {
  if (!P || !bytes) { set_error("NULL argument"); return IGAMT_EINVAL; }
  if (prec != IGAMT_F64 && prec != IGAMT_F32) { set_error("gradient contraction runs in F64 or F32"); return IGAMT_EUNSUPPORTED; }
  int64_t off[6];
  *bytes = grad_ws_layout(P, prec, off);
  return IGAMT_OK;
}

extern "C" igamt_status igamt_uKu_grad(igamt_plan *P, double E, double nu, igamt_precision prec, const double *d_u,
                                       double *d_grad, double *d_uKu, void *d_workspace, void *stream) {
  if (!P || !d_u || !d_grad || !d_workspace) { set_error("NULL argument"); return IGAMT_EINVAL; }
  if (prec != IGAMT_F64 && prec != IGAMT_F32) { set_error("gradient contraction runs in F64 or F32"); return IGAMT_EUNSUPPORTED; }
  igamt_status st = ensure_device(P);
  if (st) return st;
  if (!P->tables_ready) { set_error("tables are not built or set"); return IGAMT_ESTATE; }
  hipStream_t s = (hipStream_t)stream;
  int64_t off[6];
  grad_ws_layout(P, prec, off);
  char *ws = (char *)d_workspace;
  double *coef = (double *)(ws + off[0]);
  void *W = ws + off[1];
  double *lg = (double *)(ws + off[2]);
  double *part = (double *)(ws + off[3]);
  void *U = ws + off[4];
  // (1) fit in FP64
  if ((st = launch_fit(P, E, nu, IGAMT_F64, coef, stream))) return st;
  // (2) U, then W = table^T U
  UFormArgs c;
  c.desc = P->dev.pair_desc;
  c.u = d_u;
  c.U = U;
  c.M = P->n_pairs;
  c.Mp = P->Mp;
  c.n_tiles = P->n_tiles;
  c.n_tiles_pad = P->n_tiles_pad;
  for (int k = 0; k < 3; ++k) {
    c.tiles[k] = P->tiles[k];
    c.nT[k] = P->nT[k];
    c.NG[k] = P->dir[k].NG;
  }
  const dim3 ugrid((unsigned)((P->Mp + 255) / 256), (unsigned)P->n_tiles_pad);
  if (prec == IGAMT_F64)
    hipLaunchKernelGGL(u_form_kernel<double>, ugrid, dim3(256), 0, s, c);
  else
    hipLaunchKernelGGL(u_form_kernel<float>, ugrid, dim3(256), 0, s, c);
  IGAMT_LAUNCH_CHECK();
  if ((st = launch_gemm_tiles(prec, prec == IGAMT_F64 ? (const void *)P->dev.table_t : (const void *)P->dev.table_t_f32,
                              U, W, P->Kp, transposed_rows(P), P->Mp, P->n_tiles, P->n_groups, stream)))
    return st;
  // (3) fit adjoint
  FitAdjArgs f;
  for (int k = 0; k < 3; ++k) {
    f.knots[k] = P->dev.macro_knots[k];
    f.nM[k] = P->nM[k];
    f.box_a[k] = P->dev.box_a[k];
    f.box_h[k] = P->dev.box_h[k];
    f.ctrl_lo[k] = P->dev.ctrl_lo[k];
    f.tiles[k] = P->tiles[k];
    f.Lc[k] = P->Lc[k];
  }
  f.ctrl = P->dev.macro_ctrl;
  f.wts = P->dev.macro_w;
  f.n_tiles = P->n_tiles;
  f.fx = P->dev.fit_x;
  f.fP3 = P->dev.fit_P3;
  for (int k = 0; k < 3; ++k) f.q1[k] = P->qd[k] + 1;
  f.nf = P->n_fit;
  f.Kp = P->Kp;
  f.w_f64 = prec == IGAMT_F64;
  f.lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  f.mu = E / (2.0 * (1.0 + nu));
  f.coef = coef;
  f.W = W;
  f.local_grad = lg;
  f.uKu_part = part;
  f.flag = P->dev.flag;
  const int ns = P->n_fit * P->n_fit * P->n_fit;
  f.Lm = std::max(P->Lc[0], std::max(P->Lc[1], P->Lc[2]));
  // three (i, j) blocks per pass where the buffers leave room for three workgroups per CU
  const int64_t nsp = std::max(ns, P->npi), xt = 6 * (int64_t)P->n_fit * f.Lm;
  const int gj = (20 + 2 * 27) * nsp + xt <= 6 * 1024 ? 3 : 1;
  f.xt_off = (20 + 2 * 9 * gj) * nsp;
  const size_t shm = (size_t)(f.xt_off + xt) * sizeof(double);
  if (shm > 150 * 1024) { set_error("tile samples or macro control points per tile too many for the fit adjoint"); return IGAMT_EUNSUPPORTED; }
  const dim3 fgrid((unsigned)P->n_tiles), fblock(kFitAdjThreads);
  switch (IGAMT_DEGREE_KEY(P->pM[0], P->pM[1], P->pM[2])) {
#define FA_LAUNCH(p0, p1, p2, g)                                                                        \
  do {                                                                                                  \
    if (shm > 65536) IGAMT_HIP(hipFuncSetAttribute((const void *)fit_adjoint_kernel<p0, p1, p2, g>,     \
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm)); \
    hipLaunchKernelGGL((fit_adjoint_kernel<p0, p1, p2, g>), fgrid, fblock, shm, s, f);                  \
  } while (0)
#define FA_CASE(p0, p1, p2)                                                                             \
  case IGAMT_DEGREE_KEY(p0, p1, p2):                                                                    \
    if (gj == 3) FA_LAUNCH(p0, p1, p2, 3); else FA_LAUNCH(p0, p1, p2, 1);                               \
    break;
    IGAMT_FOR_MACRO_DEGREES(FA_CASE)
#undef FA_CASE
#undef FA_LAUNCH
    default: set_error("unsupported macro degrees (isotropic 1..6, or 1..3 per direction)"); return IGAMT_EUNSUPPORTED;
  }
  IGAMT_LAUNCH_CHECK();
  // (4) reductions
  if ((st = launch_grad_reduce(P, lg, d_grad, stream))) return st;
  if (d_uKu && (st = launch_sum(part, P->n_tiles, d_uKu, stream))) return st;
  return IGAMT_OK;
}
