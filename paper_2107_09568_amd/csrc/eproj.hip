// Sampled projection error of the macro field and the adaptive projection degree
// (Section 3.2.2 after eq. (48); Section 3.3.1, eq. (59), (65)).
//
// E_proj(q) = max over tiles t and samples xi of |A(xi) - Pi_q A(xi)|_F / |A(xi)|_F, with A the
// macro field of eq. (37) (Cartesian form, as the fit) and Pi_q A its projection onto the degree-q
// Bernstein space from q + 1 Gauss-Legendre nodes per direction (the fit of eq. (42) at degree q).
// The samples are a uniform tensor grid with both ends, x_k = k / (n_s - 1), in box coordinates.
// Per tile one 256-thread workgroup: F = J^-1 and D = det J at the fit nodes and the samples (LDS;
// the macro map's 1-D bases are evaluated once per direction and node and shared by the points);
// for each (i, j) block of A, the nine components at the fit nodes, their coefficients by three 1-D
// passes (one operator per direction), their values at the samples by three 1-D Bernstein passes;
// per sample the squared Frobenius error and norm accumulate over the blocks.  The maxima are
// order-free, so the result is deterministic.  Eq. (65): the first q from the macro degree up
// whose E_proj meets the tolerance (a host loop over this kernel).
#include <algorithm>
#include <cmath>
#include <vector>

#include "device_common.h"

namespace igamt {

constexpr int kMaxSample = 8;   // samples per direction

struct EprojArgs {
  const double *knots[3];
  int nM[3];
  const double *ctrl;
  const double *wts;      // NURBS weights of the macro map, or null (B-spline)
  const double *box_a[3];
  const double *box_h[3];
  int tiles[3];
  const double *fx;       // [nf] fit nodes
  const double *fP;       // per-direction 1-D projection operators [q1[0]][nf], [q1[1]][nf], [q1[2]][nf]
  const double *sx;       // [n_s] sample coordinates
  int q1[3], nf, n_s;
  double lam, mu;
  double *tile_e;         // [n_tiles]
  int32_t *flag;
};

__device__ inline double field_component(const double *FD, int i, int j, int aa, int bb, double lam, double mu) {
  const double *Fi = FD + 3 * i, *Fj = FD + 3 * j;
  const double fij = Fi[0] * Fj[0] + Fi[1] * Fj[1] + Fi[2] * Fj[2];
  return FD[9] * (lam * Fi[aa] * Fj[bb] + (aa == bb ? mu * fij : 0.0) + mu * Fi[bb] * Fj[aa]);
}

// J diag(h) from the macro map's parameter Jacobian J: F = (J diag(h))^-1 and D = det(J diag(h)) into
// FD[0..9]; a tile whose map folds (D <= 0) is flagged.
__device__ inline void point_FD_store(const EprojArgs &a, const double (&hx)[3], double (&J)[3][3], double *FD,
                                      int64_t t) {
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int n = 0; n < 3; ++n) J[c][n] *= hx[n];
  double F[3][3];
  const double D = inv3(J, F);
  if (!(D > 0.0) || !isfinite(D)) atomicMin(a.flag, (int32_t)t);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) FD[3 * r + c] = F[r][c];
  FD[9] = D;
}

template <int P0, int P1, int P2>
__global__ __launch_bounds__(256) void eproj_kernel(EprojArgs a) {
  extern __shared__ double smem[];
  const int tid = threadIdx.x, nf = a.nf, ns1 = a.n_s, q1x = a.q1[0], q1y = a.q1[1], q1z = a.q1[2];
  const int nfit = nf * nf * nf, nsmp = ns1 * ns1 * ns1, npi = q1x * q1y * q1z;
  const int nbuf = 9 * max(nfit, nsmp);
  double *FDf = smem;                 // [nfit][10]
  double *FDs = FDf + nfit * 10;      // [nsmp][10]
  double *err2 = FDs + nsmp * 10;     // [nsmp]
  double *nrm2 = err2 + nsmp;         // [nsmp]
  double *b0 = nrm2 + nsmp;           // ping-pong buffers of the sum-factorised passes, [9][...]
  double *b1 = b0 + nbuf;
  __shared__ double Pm[3][(kMaxQ + 1) * kMaxFit];
  __shared__ double Bs[3][kMaxSample][kMaxQ + 1];
  __shared__ double red[256];
  const int64_t t = blockIdx.x;
  const int tt[3] = {(int)(t % a.tiles[0]), (int)((t / a.tiles[0]) % a.tiles[1]),
                     (int)(t / ((int64_t)a.tiles[0] * a.tiles[1]))};
  const double ax[3] = {a.box_a[0][tt[0]], a.box_a[1][tt[1]], a.box_a[2][tt[2]]};
  const double hx[3] = {a.box_h[0][tt[0]], a.box_h[1][tt[1]], a.box_h[2][tt[2]]};
  for (int k = 0, off = 0; k < 3; off += a.q1[k] * nf, ++k)
    for (int e = tid; e < a.q1[k] * nf; e += 256) Pm[k][e] = a.fP[off + e];
  for (int e = tid; e < 3 * ns1; e += 256) {
    const int k = e / ns1, m = e % ns1;
    double B[kMaxQ + 1];
    bernstein(a.q1[k] - 1, a.sx[m], B);
    for (int c = 0; c < a.q1[k]; ++c) Bs[k][m][c] = B[c];
  }
  // the spans and 1-D B-spline values and derivatives of the macro map at the fit nodes and the
  // samples of each direction, one thread each, shared by the points (the values spline_jacobian3
  // would compute at every point)
  constexpr int PMX = max3(P0, P1, P2);
  __shared__ double NB[3][kMaxFit + kMaxSample][2][PMX + 1];
  __shared__ int SP[3][kMaxFit + kMaxSample];
  const int n1 = nf + ns1;
  if (tid < 3 * n1) {
    const int d = tid / n1, m = tid - d * n1;
    const double x = (d == 0 ? ax[0] : d == 1 ? ax[1] : ax[2]) +
                     (d == 0 ? hx[0] : d == 1 ? hx[1] : hx[2]) * (m < nf ? a.fx[m] : a.sx[m - nf]);
    constexpr int PD[3] = {P0, P1, P2};
    const int sp = find_span(a.knots[d], a.nM[d], d == 0 ? PD[0] : d == 1 ? PD[1] : PD[2], x);
    double N[PMX + 1], dN[PMX + 1];
    bspline_ders_dir<P0, P1, P2>(d, a.knots[d], sp, x, N, dN);
    SP[d][m] = sp;
#pragma unroll
    for (int r = 0; r <= PMX; ++r) {
      NB[d][m][0][r] = N[r];
      NB[d][m][1][r] = dN[r];
    }
  }
  __syncthreads();
  auto point = [&](int m0, int m1, int m2, double *FD) {
    const int mi[3] = {m0, m1, m2};
    int span[3];
    double N[3][PMX + 1], dN[3][PMX + 1];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      span[k] = SP[k][mi[k]];
#pragma unroll
      for (int r = 0; r <= PMX; ++r) {
        N[k][r] = NB[k][mi[k]][0][r];
        dN[k][r] = NB[k][mi[k]][1][r];
      }
    }
    double J[3][3];
    spline_jacobian_sum<P0, P1, P2, true>(a.nM, a.ctrl, a.wts, span, N, dN, J);
    point_FD_store(a, hx, J, FD, t);
  };
  for (int s = tid; s < nfit; s += 256) point(s % nf, (s / nf) % nf, s / (nf * nf), FDf + s * 10);
  for (int k = tid; k < nsmp; k += 256) {
    point(nf + k % ns1, nf + (k / ns1) % ns1, nf + k / (ns1 * ns1), FDs + k * 10);
    err2[k] = 0.0;
    nrm2[k] = 0.0;
  }
  __syncthreads();
  for (int ij = 0; ij < 9; ++ij) {
    const int i = ij / 3, j = ij % 3;
    // the nine components A_ij,ab at the fit nodes: b0[ab][s], s = s1 + nf (s2 + nf s3)
    for (int e = tid; e < 9 * nfit; e += 256) {
      const int ab = e / nfit, sp = e % nfit;
      b0[e] = field_component(FDf + sp * 10, i, j, ab / 3, ab % 3, a.lam, a.mu);
    }
    __syncthreads();
    // projection, one direction at a time: x: b1[ab][(s3, s2), c1]
    for (int e = tid; e < 9 * nf * nf * q1x; e += 256) {
      const int c1 = e % q1x, r = e / q1x, s23 = r % (nf * nf), ab = r / (nf * nf);
      const double *src = b0 + (int64_t)ab * nfit + s23 * nf;
      double v = 0.0;
      for (int s1 = 0; s1 < nf; ++s1) v += Pm[0][c1 * nf + s1] * src[s1];
      b1[e] = v;
    }
    __syncthreads();
    // y: b0[ab][s3, c2, c1]
    for (int e = tid; e < 9 * nf * q1y * q1x; e += 256) {
      const int c1 = e % q1x, c2 = (e / q1x) % q1y, r = e / (q1x * q1y), s3 = r % nf, ab = r / nf;
      double v = 0.0;
      for (int s2 = 0; s2 < nf; ++s2) v += Pm[1][c2 * nf + s2] * b1[((int64_t)(ab * nf + s3) * nf + s2) * q1x + c1];
      b0[e] = v;
    }
    __syncthreads();
    // z: b1[ab][C], C = c1 + q1x (c2 + q1y c3): the coefficients of the nine components
    for (int e = tid; e < 9 * npi; e += 256) {
      const int C = e % npi, ab = e / npi, c12 = C % (q1x * q1y), c3 = C / (q1x * q1y);
      double v = 0.0;
      for (int s3 = 0; s3 < nf; ++s3) v += Pm[2][c3 * nf + s3] * b0[((int64_t)ab * nf + s3) * q1x * q1y + c12];
      b1[e] = v;
    }
    __syncthreads();
    // evaluation at the samples, one direction at a time: x: b0[ab][(c3, c2), k0]
    for (int e = tid; e < 9 * q1z * q1y * ns1; e += 256) {
      const int k0 = e % ns1, r = e / ns1, c23 = r % (q1y * q1z), ab = r / (q1y * q1z);
      const double *src = b1 + (int64_t)ab * npi + c23 * q1x;
      double v = 0.0;
      for (int c1 = 0; c1 < q1x; ++c1) v += Bs[0][k0][c1] * src[c1];
      b0[e] = v;
    }
    __syncthreads();
    // y: b1[ab][c3, k1, k0]
    for (int e = tid; e < 9 * q1z * ns1 * ns1; e += 256) {
      const int k0 = e % ns1, k1 = (e / ns1) % ns1, r = e / (ns1 * ns1), c3 = r % q1z, ab = r / q1z;
      double v = 0.0;
      for (int c2 = 0; c2 < q1y; ++c2) v += Bs[1][k1][c2] * b0[((int64_t)(ab * q1z + c3) * q1y + c2) * ns1 + k0];
      b1[e] = v;
    }
    __syncthreads();
    // z and the per-sample error: thread per sample k = k0 + ns1 (k1 + ns1 k2)
    for (int k = tid; k < nsmp; k += 256) {
      const int k01 = k % (ns1 * ns1), k2 = k / (ns1 * ns1);
      double e2 = 0.0, n2 = 0.0;
      for (int ab = 0; ab < 9; ++ab) {
        double pr = 0.0;
        for (int c3 = 0; c3 < q1z; ++c3) pr += Bs[2][k2][c3] * b1[((int64_t)ab * q1z + c3) * ns1 * ns1 + k01];
        const double ex = field_component(FDs + k * 10, i, j, ab / 3, ab % 3, a.lam, a.mu);
        e2 += (ex - pr) * (ex - pr);
        n2 += ex * ex;
      }
      err2[k] += e2;
      nrm2[k] += n2;
    }
    __syncthreads();
  }
  double m = 0.0;
  for (int k = tid; k < nsmp; k += 256) m = fmax(m, sqrt(err2[k] / nrm2[k]));
  red[tid] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
    __syncthreads();
  }
  if (tid == 0) a.tile_e[t] = red[0];
}

// Isotropic macro map of degree PM and projection degree Q on Q + 1 nodes (the interpolating
// case), with the shape known at compile time.  One 128-thread workgroup per tile.  After F and D at
// the fit nodes and the samples (1-D bases shared as above), lane l < 45 takes one of the 45 index
// pairs (u, v) = (3 i + a, 3 j + b), u <= v: it evaluates A_ij,ab (= A_ji,ba) at the fit nodes and
// projects it with three 1-D passes in registers (as the fit does), into LDS.  Then one thread per
// sample: the tensor Bernstein weights of its sample in registers, and over the 45 pairs the exact
// value, the projected one and their squared difference, counted twice for u < v (the (j, i) block
// holds the same entries).
constexpr int kEprojQThreads = 128;

template <int PM, int Q>
__global__ __launch_bounds__(kEprojQThreads) void eproj_q_kernel(EprojArgs a) {
  constexpr int NF = Q + 1, NFIT = NF * NF * NF;
  extern __shared__ double smem[];
  const int tid = threadIdx.x, ns1 = a.n_s, nsmp = ns1 * ns1 * ns1;
  double *FDf = smem;               // [NFIT][10]
  double *FDs = FDf + NFIT * 10;    // [nsmp][10]
  double *cf = FDs + nsmp * 10;     // [45][NFIT] coefficients of the 45 pairs
  __shared__ double NB[3][kMaxFit + kMaxSample][2][PM + 1];
  __shared__ int SP[3][kMaxFit + kMaxSample];
  __shared__ double Bs[3][kMaxSample][Q + 1];
  __shared__ double red[kEprojQThreads / 64];
  const int64_t t = blockIdx.x;
  const int tt[3] = {(int)(t % a.tiles[0]), (int)((t / a.tiles[0]) % a.tiles[1]),
                     (int)(t / ((int64_t)a.tiles[0] * a.tiles[1]))};
  const double ax[3] = {a.box_a[0][tt[0]], a.box_a[1][tt[1]], a.box_a[2][tt[2]]};
  const double hx[3] = {a.box_h[0][tt[0]], a.box_h[1][tt[1]], a.box_h[2][tt[2]]};
  const int n1 = NF + ns1;
  for (int e = tid; e < 3 * n1; e += kEprojQThreads) {
    const int d = e / n1, m = e - d * n1;
    const double x = (d == 0 ? ax[0] : d == 1 ? ax[1] : ax[2]) +
                     (d == 0 ? hx[0] : d == 1 ? hx[1] : hx[2]) * (m < NF ? a.fx[m] : a.sx[m - NF]);
    const int sp = find_span(a.knots[d], a.nM[d], PM, x);
    double N[PM + 1], dN[PM + 1];
    bspline_ders<PM>(a.knots[d], sp, x, N, dN);
    SP[d][m] = sp;
#pragma unroll
    for (int r = 0; r <= PM; ++r) {
      NB[d][m][0][r] = N[r];
      NB[d][m][1][r] = dN[r];
    }
  }
  for (int e = tid; e < 3 * ns1; e += kEprojQThreads) {
    const int k = e / ns1, m = e % ns1;
    double B[kMaxQ + 1];
    bernstein(Q, a.sx[m], B);
#pragma unroll
    for (int c = 0; c <= Q; ++c) Bs[k][m][c] = B[c];
  }
  __syncthreads();
  for (int e = tid; e < NFIT + nsmp; e += kEprojQThreads) {
    int mi[3];
    double *FD;
    if (e < NFIT) {
      mi[0] = e % NF, mi[1] = (e / NF) % NF, mi[2] = e / (NF * NF);
      FD = FDf + e * 10;
    } else {
      const int k = e - NFIT;
      mi[0] = NF + k % ns1, mi[1] = NF + (k / ns1) % ns1, mi[2] = NF + k / (ns1 * ns1);
      FD = FDs + k * 10;
    }
    int span[3];
    double N[3][PM + 1], dN[3][PM + 1];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      span[k] = SP[k][mi[k]];
#pragma unroll
      for (int r = 0; r <= PM; ++r) {
        N[k][r] = NB[k][mi[k]][0][r];
        dN[k][r] = NB[k][mi[k]][1][r];
      }
    }
    double J[3][3];
    spline_jacobian_sum<PM, PM, PM, true>(a.nM, a.ctrl, a.wts, span, N, dN, J);
    point_FD_store(a, hx, J, FD, t);
  }
  __syncthreads();

  // the 45 pairs' projection coefficients
  if (tid < 45) {
    int u = 0, rem = tid;
    while (rem >= 9 - u) { rem -= 9 - u; ++u; }
    const int v = u + rem;
    const int i = u / 3, aa = u % 3, j = v / 3, bb = v % 3;
    double P[NF][NF];   // the 1-D operator, the same in every direction here (checked by the launcher)
#pragma unroll
    for (int c = 0; c < NF; ++c)
#pragma unroll
      for (int q = 0; q < NF; ++q) P[c][q] = uniform_f64(a.fP[c * NF + q]);
    double val[NFIT];
#pragma unroll
    for (int q = 0; q < NFIT; ++q)
      val[q] = elastic_density(FDf + q * 10 + 3 * i, FDf + q * 10 + 3 * j, FDf[q * 10 + 9], aa, bb, a.lam, a.mu);
#pragma unroll
    for (int l = 0; l < NF * NF; ++l) {   // x
      double o[NF];
#pragma unroll
      for (int c = 0; c < NF; ++c) {
        double w = 0.0;
#pragma unroll
        for (int q = 0; q < NF; ++q) w += P[c][q] * val[l * NF + q];
        o[c] = w;
      }
#pragma unroll
      for (int c = 0; c < NF; ++c) val[l * NF + c] = o[c];
    }
#pragma unroll
    for (int s3 = 0; s3 < NF; ++s3)   // y
#pragma unroll
      for (int c1 = 0; c1 < NF; ++c1) {
        double o[NF];
#pragma unroll
        for (int c = 0; c < NF; ++c) {
          double w = 0.0;
#pragma unroll
          for (int q = 0; q < NF; ++q) w += P[c][q] * val[(s3 * NF + q) * NF + c1];
          o[c] = w;
        }
#pragma unroll
        for (int c = 0; c < NF; ++c) val[(s3 * NF + c) * NF + c1] = o[c];
      }
#pragma unroll
    for (int l = 0; l < NF * NF; ++l) {   // z
      double o[NF];
#pragma unroll
      for (int c = 0; c < NF; ++c) {
        double w = 0.0;
#pragma unroll
        for (int q = 0; q < NF; ++q) w += P[c][q] * val[q * NF * NF + l];
        o[c] = w;
      }
#pragma unroll
      for (int c = 0; c < NF; ++c) val[c * NF * NF + l] = o[c];
    }
#pragma unroll
    for (int C = 0; C < NFIT; ++C) cf[tid * NFIT + C] = val[C];
  }
  __syncthreads();

  // one thread per sample
  double m = 0.0;
  for (int k = tid; k < nsmp; k += kEprojQThreads) {
    const int k0 = k % ns1, k1 = (k / ns1) % ns1, k2 = k / (ns1 * ns1);
    double W[NFIT];
#pragma unroll
    for (int C = 0; C < NFIT; ++C) W[C] = Bs[0][k0][C % NF] * Bs[1][k1][(C / NF) % NF] * Bs[2][k2][C / (NF * NF)];
    const double *F = FDs + k * 10;
    double e2 = 0.0, n2 = 0.0;
    int u = 0, v = 0;   // the pair of index l, row-major over u <= v
#pragma unroll 1
    for (int l = 0; l < 45; ++l) {
      const double ex = elastic_density(F + 3 * (u / 3), F + 3 * (v / 3), F[9], u % 3, v % 3, a.lam, a.mu);
      double pr = 0.0;
#pragma unroll
      for (int C = 0; C < NFIT; ++C) pr += cf[l * NFIT + C] * W[C];
      const double d = ex - pr, w = u == v ? 1.0 : 2.0;
      e2 += w * d * d;
      n2 += w * ex * ex;
      if (++v == 9) v = ++u;
    }
    m = fmax(m, sqrt(e2 / n2));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((tid & 63) == 0) red[tid >> 6] = m;
  __syncthreads();
  if (tid == 0) {
    double r = red[0];
    for (int w = 1; w < kEprojQThreads / 64; ++w) r = fmax(r, red[w]);
    a.tile_e[t] = r;
  }
}

__global__ __launch_bounds__(256) void max_kernel(const double *x, int64_t n, double *out) {
  __shared__ double red[256];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) m = fmax(m, x[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + k]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// scratch layout (doubles): [0, n_tiles) per-tile errors; then fit nodes [kMaxFit], operators
// [3 (kMaxQ+1) kMaxFit], samples [kMaxSample], result [1]
static int64_t eproj_buf_doubles(const igamt_plan *P) {
  return P->n_tiles + kMaxFit + 3 * (kMaxQ + 1) * kMaxFit + kMaxSample + 1;
}

// E_proj for degrees q[3], fitted on max_k q_k + 1 Gauss-Legendre nodes per direction
static igamt_status eproj_run(igamt_plan *P, double E, double nu, const int (&q)[3], int n_s, double *d_tile_e,
                              double *e_out, hipStream_t s) {
  if (!P->dev.eproj_buf) IGAMT_HIP(hipMalloc((void **)&P->dev.eproj_buf, eproj_buf_doubles(P) * sizeof(double)));
  double *buf = P->dev.eproj_buf;
  double *d_fx = buf + P->n_tiles, *d_fP = d_fx + kMaxFit, *d_sx = d_fP + 3 * (kMaxQ + 1) * kMaxFit,
         *d_res = d_sx + kMaxSample;
  const int nf = std::max(q[0], std::max(q[1], q[2])) + 1;
  std::vector<double> fx, fw, fP, sx(n_s);
  gauss_legendre01(nf, fx, fw);
  for (int k = 0; k < 3; ++k) {
    std::vector<double> Pk;
    if (!projection_1d(q[k], fx, fw, Pk)) { set_error("singular projection matrix"); return IGAMT_EINVAL; }
    fP.insert(fP.end(), Pk.begin(), Pk.end());
  }
  for (int k = 0; k < n_s; ++k) sx[k] = (double)k / (n_s - 1);
  IGAMT_HIP(hipMemcpyAsync(d_fx, fx.data(), nf * sizeof(double), hipMemcpyHostToDevice, s));
  IGAMT_HIP(hipMemcpyAsync(d_fP, fP.data(), fP.size() * sizeof(double), hipMemcpyHostToDevice, s));
  IGAMT_HIP(hipMemcpyAsync(d_sx, sx.data(), n_s * sizeof(double), hipMemcpyHostToDevice, s));
  EprojArgs a;
  for (int k = 0; k < 3; ++k) {
    a.knots[k] = P->dev.macro_knots[k];
    a.nM[k] = P->nM[k];
    a.box_a[k] = P->dev.box_a[k];
    a.box_h[k] = P->dev.box_h[k];
    a.tiles[k] = P->tiles[k];
  }
  a.ctrl = P->dev.macro_ctrl;
  a.wts = P->dev.macro_w;
  a.fx = d_fx;
  a.fP = d_fP;
  a.sx = d_sx;
  for (int k = 0; k < 3; ++k) a.q1[k] = q[k] + 1;
  a.nf = nf;
  a.n_s = n_s;
  a.lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  a.mu = E / (2.0 * (1.0 + nu));
  a.tile_e = d_tile_e ? d_tile_e : buf;
  a.flag = P->dev.flag;
  const int nfit = nf * nf * nf, nsmp = n_s * n_s * n_s;
  // isotropic macro map and degree q <= 3: the compile-time shape
  if (P->pM[0] == P->pM[1] && P->pM[0] == P->pM[2] && q[0] == q[1] && q[0] == q[2] && q[0] >= 1 && q[0] <= 3) {
    const size_t shmq = (size_t)(10 * nfit + 10 * nsmp + 45 * nfit) * sizeof(double);
    const dim3 gq((unsigned)P->n_tiles), bq(kEprojQThreads);
    switch (P->pM[0] * 8 + q[0]) {
#define EPQ_CASE(pm, qq)                                                                                  \
  case pm * 8 + qq:                                                                                       \
    if (shmq > 65536)                                                                                     \
      IGAMT_HIP(hipFuncSetAttribute((const void *)eproj_q_kernel<pm, qq>,                                 \
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmq));              \
    hipLaunchKernelGGL((eproj_q_kernel<pm, qq>), gq, bq, shmq, s, a);                                     \
    break;
#define EPQ_DEG(pm) EPQ_CASE(pm, 1) EPQ_CASE(pm, 2) EPQ_CASE(pm, 3)
      EPQ_DEG(1) EPQ_DEG(2) EPQ_DEG(3) EPQ_DEG(4) EPQ_DEG(5) EPQ_DEG(6)
#undef EPQ_DEG
#undef EPQ_CASE
      default: set_error("unsupported macro degree"); return IGAMT_EUNSUPPORTED;
    }
    IGAMT_LAUNCH_CHECK();
    hipLaunchKernelGGL(max_kernel, dim3(1), dim3(256), 0, s, a.tile_e, P->n_tiles, d_res);
    IGAMT_LAUNCH_CHECK();
    IGAMT_HIP(hipMemcpyAsync(e_out, d_res, sizeof(double), hipMemcpyDeviceToHost, s));
    IGAMT_HIP(hipStreamSynchronize(s));   // the host vectors above and *e_out are used until here
    return IGAMT_OK;
  }
  const size_t shm = (size_t)(10 * nfit + 10 * nsmp + 2 * nsmp + 2 * 9 * std::max(nfit, nsmp)) * sizeof(double);
  const dim3 grid((unsigned)P->n_tiles), block(256);
  switch (IGAMT_DEGREE_KEY(P->pM[0], P->pM[1], P->pM[2])) {
#define EP_CASE(p0, p1, p2)                                                                               \
  case IGAMT_DEGREE_KEY(p0, p1, p2):                                                                      \
    if (shm > 65536)                                                                                      \
      IGAMT_HIP(hipFuncSetAttribute((const void *)eproj_kernel<p0, p1, p2>,                               \
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));               \
    hipLaunchKernelGGL((eproj_kernel<p0, p1, p2>), grid, block, shm, s, a);                               \
    break;
    IGAMT_FOR_MACRO_DEGREES(EP_CASE)
#undef EP_CASE
    default: set_error("unsupported macro degrees (isotropic 1..6, or 1..3 per direction)"); return IGAMT_EUNSUPPORTED;
  }
  IGAMT_LAUNCH_CHECK();
  hipLaunchKernelGGL(max_kernel, dim3(1), dim3(256), 0, s, a.tile_e, P->n_tiles, d_res);
  IGAMT_LAUNCH_CHECK();
  IGAMT_HIP(hipMemcpyAsync(e_out, d_res, sizeof(double), hipMemcpyDeviceToHost, s));
  IGAMT_HIP(hipStreamSynchronize(s));   // the host vectors above and *e_out are used until here
  return IGAMT_OK;
}

static igamt_status eproj_checks(igamt_plan *P, double E, double nu, int n_s) {
  if (!(E > 0.0) || !std::isfinite(E) || !(nu > -1.0 && nu < 0.5)) {
    set_error("E must be positive and -1 < nu < 0.5");
    return IGAMT_EINVAL;
  }
  if (n_s < 2 || n_s > kMaxSample) { set_error("samples per direction must be in [2, 8]"); return IGAMT_EINVAL; }
  return ensure_device(P);
}

}  // namespace igamt

using namespace igamt;

extern "C" igamt_status igamt_eproj(igamt_plan *P, double E, double nu, int32_t q, int32_t n_sample,
                                    double *d_tile_e, double *e_proj, void *stream) {
  const int32_t qd[3] = {q, q, q};
  return igamt_eproj_aniso(P, E, nu, qd, n_sample, d_tile_e, e_proj, stream);
}

extern "C" igamt_status igamt_eproj_aniso(igamt_plan *P, double E, double nu, const int32_t *q, int32_t n_sample,
                                          double *d_tile_e, double *e_proj, void *stream) {
  if (!P || !e_proj || !q) { set_error("NULL argument"); return IGAMT_EINVAL; }
  for (int k = 0; k < 3; ++k)
    if (q[k] < 0 || q[k] > kMaxQ) { set_error("projection degrees must be in [0, 6]"); return IGAMT_EINVAL; }
  igamt_status st = eproj_checks(P, E, nu, n_sample);
  if (st) return st;
  const int qd[3] = {q[0], q[1], q[2]};
  return eproj_run(P, E, nu, qd, n_sample, d_tile_e, e_proj, (hipStream_t)stream);
}

extern "C" igamt_status igamt_select_q(igamt_plan *P, double E, double nu, double tol, int32_t q_max,
                                       int32_t n_sample, int32_t *q_out, double *e_out, void *stream) {
  if (!P || !q_out || !e_out) { set_error("NULL argument"); return IGAMT_EINVAL; }
  if (!(tol >= 0.0) || !std::isfinite(tol)) { set_error("tolerance must be finite and non-negative"); return IGAMT_EINVAL; }
  igamt_status st = eproj_checks(P, E, nu, n_sample);
  if (st) return st;
  const int q0 = std::max(P->pM[0], std::max(P->pM[1], P->pM[2]));   // the macro degree (largest direction)
  if (q_max < q0 || q_max > kMaxQ) { set_error("q_max must be in [macro degree, 6]"); return IGAMT_EINVAL; }
  double e = 0.0;
  for (int q = q0; q <= q_max; ++q) {
    const int qd[3] = {q, q, q};
    if ((st = eproj_run(P, E, nu, qd, n_sample, nullptr, &e, (hipStream_t)stream))) return st;
    if (e <= tol) {
      *q_out = q;
      *e_out = e;
      return IGAMT_OK;
    }
  }
  *q_out = -1;
  *e_out = e;
  return IGAMT_OK;
}

extern "C" igamt_status igamt_select_q_aniso(igamt_plan *P, double E, double nu, double tol, int32_t q_max,
                                             int32_t n_sample, int32_t *q_out, double *e_out, void *stream) {
  if (!P || !q_out || !e_out) { set_error("NULL argument"); return IGAMT_EINVAL; }
  if (!(tol >= 0.0) || !std::isfinite(tol)) { set_error("tolerance must be finite and non-negative"); return IGAMT_EINVAL; }
  igamt_status st = eproj_checks(P, E, nu, n_sample);
  if (st) return st;
  if (q_max < std::max(P->pM[0], std::max(P->pM[1], P->pM[2])) || q_max > kMaxQ) {
    set_error("q_max must be in [largest macro degree, 6]");
    return IGAMT_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  int q[3] = {P->pM[0], P->pM[1], P->pM[2]};
  double e = 0.0;
  if ((st = eproj_run(P, E, nu, q, n_sample, nullptr, &e, s))) return st;
  while (e > tol) {   // raise the direction whose raise lowers E_proj most (ties: lowest index)
    int best = -1;
    double be = 0.0;
    for (int k = 0; k < 3; ++k) {
      if (q[k] >= q_max) continue;
      int trial[3] = {q[0], q[1], q[2]};
      ++trial[k];
      double et = 0.0;
      if ((st = eproj_run(P, E, nu, trial, n_sample, nullptr, &et, s))) return st;
      if (best < 0 || et < be) {
        best = k;
        be = et;
      }
    }
    if (best < 0) {
      for (int k = 0; k < 3; ++k) q_out[k] = -1;
      *e_out = e;
      return IGAMT_OK;
    }
    ++q[best];
    e = be;
  }
  for (int k = 0; k < 3; ++k) q_out[k] = q[k];
  *e_out = e;
  return IGAMT_OK;
}
