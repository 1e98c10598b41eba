// Learned lookup tables (not part of the paper, which precomputes one table per
// reference tile): a POD basis of the tables of a parameterised tile family and
// a small MLP from design parameters to POD coefficients.
//
//  * POD: mean, Gram matrix of the centred snapshots (FP64, device, summed over
//    fixed slices in a fixed order), symmetric eigenproblem on the host (cyclic
//    Jacobi), modes Phi_k = X_c v_k / sigma_k, and the snapshot coefficients
//    Phi^T X_c = V Sigma, which follow from G V = V Lambda without another pass.
//  * Reconstruction of a design's table T = mean + sum_k c_k Phi_k straight into
//    the plan's FP64 table, and a row-subset relative error against exact rows.
//  * MLP x -> GELU(x W1 + b1) -> ... -> x W_L + b_L with hand-written forward,
//    backward (deterministic reductions over the batch), mean-squared-error and
//    Adam kernels, all FP32.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <vector>

#include <limits>

#include "device_common.h"

namespace igamt {

// ---- POD -------------------------------------------------------------------------
__global__ __launch_bounds__(256) void column_mean_kernel(const double *__restrict__ X, int n_s, int64_t n_e,
                                                          double *__restrict__ mean) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n_e) return;
  double s = 0.0;
  for (int i = 0; i < n_s; ++i) s += X[(int64_t)i * n_e + e];
  mean[e] = s / n_s;
}

// Partial Gram matrices: block (bi, bj, slice) computes the 32x32 tile
// sum_{e in slice} (X_i[e] - m[e]) (X_j[e] - m[e]) for i in bi, j in bj (bi <= bj).
constexpr int GT = 32, GE = 64;
__global__ __launch_bounds__(256) void gram_kernel(const double *__restrict__ X, const double *__restrict__ mean,
                                                   int n_s, int64_t n_e, int n_slices, int nb,
                                                   double *__restrict__ part) {
  __shared__ double Xi[GT][GE + 1], Xj[GT][GE + 1];
  int b = blockIdx.x;
  const int slice = b % n_slices;
  b /= n_slices;
  int bi = 0;
  while (b >= nb - bi) { b -= nb - bi; ++bi; }
  const int bj = bi + b;
  const int64_t e_lo = n_e * slice / n_slices, e_hi = n_e * (slice + 1) / n_slices;
  const int tid = threadIdx.x;
  const int ti = tid / 16, tj = tid % 16;   // each thread: rows 2ti, 2ti+1; cols 2tj, 2tj+1
  double acc[2][2] = {{0, 0}, {0, 0}};
  for (int64_t e0 = e_lo; e0 < e_hi; e0 += GE) {
    __syncthreads();
    for (int idx = tid; idx < GT * GE; idx += 256) {
      const int r = idx / GE, c = idx % GE;
      const int64_t e = e0 + c;
      const int i = bi * GT + r, j = bj * GT + r;
      const double m = e < e_hi ? mean[e] : 0.0;
      Xi[r][c] = (e < e_hi && i < n_s) ? X[(int64_t)i * n_e + e] - m : 0.0;
      Xj[r][c] = (e < e_hi && j < n_s) ? X[(int64_t)j * n_e + e] - m : 0.0;
    }
    __syncthreads();
    for (int c = 0; c < GE; ++c) {
      const double a0 = Xi[2 * ti][c], a1 = Xi[2 * ti + 1][c];
      const double b0 = Xj[2 * tj][c], b1 = Xj[2 * tj + 1][c];
      acc[0][0] += a0 * b0; acc[0][1] += a0 * b1;
      acc[1][0] += a1 * b0; acc[1][1] += a1 * b1;
    }
  }
  double *out = part + (int64_t)slice * n_s * n_s;
  for (int u = 0; u < 2; ++u)
    for (int v = 0; v < 2; ++v) {
      const int i = bi * GT + 2 * ti + u, j = bj * GT + 2 * tj + v;
      if (i < n_s && j < n_s) out[(int64_t)i * n_s + j] = acc[u][v];
    }
}

__global__ void gram_sum_kernel(const double *__restrict__ part, int n_s, int n_slices, double *__restrict__ G) {
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (id >= (int64_t)n_s * n_s) return;
  const int i = (int)(id / n_s), j = (int)(id % n_s);
  if (i > j) return;
  double s = 0.0;
  for (int k = 0; k < n_slices; ++k) s += part[(int64_t)k * n_s * n_s + id];
  G[id] = s;
  G[(int64_t)j * n_s + i] = s;
}

// basis[k][e] = sum_i (X_i[e] - m[e]) V[i][k] / sigma_k, mean -> float
__global__ __launch_bounds__(256) void pod_basis_kernel(const double *__restrict__ X, const double *__restrict__ mean,
                                                        const double *__restrict__ Vs, int n_s, int64_t n_e, int r,
                                                        float *__restrict__ basis, float *__restrict__ mean_f) {
  extern __shared__ double vs[];   // [n_s][16] columns k0..k0+15 of V / sigma
  const int k0 = blockIdx.y * 16;
  for (int idx = threadIdx.x; idx < n_s * 16; idx += 256) {
    const int i = idx / 16, k = k0 + idx % 16;
    vs[idx] = k < r ? Vs[(int64_t)i * r + k] : 0.0;
  }
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n_e) return;
  const double m = mean[e];
  if (blockIdx.y == 0) mean_f[e] = (float)m;
  double acc[16];
  for (int k = 0; k < 16; ++k) acc[k] = 0.0;
  for (int i = 0; i < n_s; ++i) {
    const double x = X[(int64_t)i * n_e + e] - m;
    for (int k = 0; k < 16; ++k) acc[k] += x * vs[i * 16 + k];
  }
  for (int k = 0; k < 16; ++k)
    if (k0 + k < r) basis[(int64_t)(k0 + k) * n_e + e] = (float)acc[k];
}

// Symmetric eigen-decomposition (row-major A, n x n): Householder reduction to tridiagonal
// form T = Q^T A Q, then implicit symmetric QR steps with the Wilkinson shift on T, each step a
// chase of the bulge by Givens rotations that are also applied to Q (the method of Golub and
// Van Loan, Matrix Computations, sections 8.3.1-8.3.3).  On return A's diagonal holds the
// eigenvalues and V's columns (V[i n + k]) the eigenvectors.  Returns false if the QR steps hit
// their cap (64 n) before every off-diagonal entry was deflated.
static bool sym_eigen(std::vector<double> &A, int n, std::vector<double> &V) {
  auto at = [&](int i, int j) -> double & { return A[(size_t)i * n + j]; };
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  std::vector<double> v(n), pv(n), w(n);
  // 1. Householder: column k below the subdiagonal is annihilated by H = I - beta v v^T
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;   // length of the reflected part (indices k+1 .. n-1)
    double nx = 0.0;
    for (int i = 0; i < m; ++i) nx += at(k + 1 + i, k) * at(k + 1 + i, k);
    nx = std::sqrt(nx);
    if (nx == 0.0) continue;
    const double x0 = at(k + 1, k);
    const double alpha = x0 >= 0.0 ? -nx : nx;
    for (int i = 0; i < m; ++i) v[i] = at(k + 1 + i, k);
    v[0] -= alpha;
    double vv = 0.0;
    for (int i = 0; i < m; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    const double beta = 2.0 / vv;
    // trailing block: A <- A - v w^T - w v^T with p = beta A v, w = p - (beta/2)(p.v) v
    for (int i = 0; i < m; ++i) {
      double acc = 0.0;
      for (int j = 0; j < m; ++j) acc += at(k + 1 + i, k + 1 + j) * v[j];
      pv[i] = beta * acc;
    }
    double pvv = 0.0;
    for (int i = 0; i < m; ++i) pvv += pv[i] * v[i];
    const double kk = 0.5 * beta * pvv;
    for (int i = 0; i < m; ++i) w[i] = pv[i] - kk * v[i];
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) at(k + 1 + i, k + 1 + j) -= v[i] * w[j] + w[i] * v[j];
    at(k + 1, k) = at(k, k + 1) = alpha;
    for (int i = 1; i < m; ++i) at(k + 1 + i, k) = at(k, k + 1 + i) = 0.0;
    // Q <- Q H on columns k+1 .. n-1
    for (int r = 0; r < n; ++r) {
      double t = 0.0;
      for (int j = 0; j < m; ++j) t += V[(size_t)r * n + k + 1 + j] * v[j];
      t *= beta;
      for (int j = 0; j < m; ++j) V[(size_t)r * n + k + 1 + j] -= t * v[j];
    }
  }
  std::vector<double> d(n), e(n > 1 ? n - 1 : 1, 0.0);
  for (int i = 0; i < n; ++i) d[i] = at(i, i);
  for (int i = 0; i + 1 < n; ++i) e[i] = at(i + 1, i);
  // 2. implicit symmetric QR with Wilkinson shift on (d, e)
  const double eps = std::numeric_limits<double>::epsilon();
  int hi = n - 1, iters = 0;
  while (hi > 0 && iters < 64 * n) {
    if (std::fabs(e[hi - 1]) <= eps * (std::fabs(d[hi - 1]) + std::fabs(d[hi]))) {
      e[hi - 1] = 0.0;
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && std::fabs(e[lo - 1]) > eps * (std::fabs(d[lo - 1]) + std::fabs(d[lo]))) --lo;
    ++iters;
    const double dl = 0.5 * (d[hi - 1] - d[hi]), bl = e[hi - 1];
    const double mu = d[hi] - bl * bl / (dl + (dl >= 0.0 ? 1.0 : -1.0) * std::hypot(dl, bl));
    double x = d[lo] - mu, z = e[lo];
    for (int k = lo; k < hi; ++k) {
      const double r = std::hypot(x, z);
      const double c = r == 0.0 ? 1.0 : x / r, s = r == 0.0 ? 0.0 : z / r;
      if (k > lo) e[k - 1] = r;   // (k-1, k) after zeroing the bulge at (k-1, k+1)
      const double ak = d[k], ak1 = d[k + 1], bk = e[k];
      d[k] = c * c * ak + 2.0 * c * s * bk + s * s * ak1;
      d[k + 1] = s * s * ak - 2.0 * c * s * bk + c * c * ak1;
      e[k] = c * s * (ak1 - ak) + (c * c - s * s) * bk;
      if (k + 1 < hi) {
        x = e[k];
        z = s * e[k + 1];        // new bulge at (k, k+2)
        e[k + 1] = c * e[k + 1];
      }
      for (int i = 0; i < n; ++i) {  // Q <- Q R^T on columns k, k+1
        const double qk = V[(size_t)i * n + k], qk1 = V[(size_t)i * n + k + 1];
        V[(size_t)i * n + k] = c * qk + s * qk1;
        V[(size_t)i * n + k + 1] = -s * qk + c * qk1;
      }
    }
  }
  for (int i = 0; i < n; ++i) at(i, i) = d[i];
  return hi == 0;
}

// table[p][k] = mean[e] + sum_r basis[r][e] c[r], e = p * K + k
__global__ __launch_bounds__(256) void pod_reconstruct_kernel(const float *__restrict__ mean,
                                                              const float *__restrict__ basis, int r,
                                                              const float *__restrict__ c, double scale, int64_t n_e,
                                                              int K, int64_t Kp, double *__restrict__ table) {
  __shared__ double cs[256];
  for (int i = threadIdx.x; i < r; i += 256) cs[i] = scale * (double)c[i];
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n_e) return;
  double v = mean[e];
  for (int k = 0; k < r; ++k) v += (double)basis[(int64_t)k * n_e + e] * cs[k];   // same form as the batch kernel
  const int64_t p = e / K, col = e - p * K;
  table[p * Kp + col] = v;
}

// Scaled coefficients of a batch, transposed and padded: cd[k][b] = scale * c[b][k] for b < B,
// 0 for B <= b < Bp.
__global__ __launch_bounds__(256) void pod_coeffs_kernel(const float *__restrict__ c, int B, int Bp, int r,
                                                         double scale, double *__restrict__ cd) {
  const int id = blockIdx.x * 256 + threadIdx.x;
  if (id >= r * Bp) return;
  const int k = id / Bp, b = id - k * Bp;
  cd[id] = b < B ? scale * (double)c[(int64_t)b * r + k] : 0.0;
}

// tables[b][e] = mean[e] + sum_k basis[k][e] cd[k][b] for a group of DB designs per thread:
// every basis value is loaded once per group and the coefficients, uniform over the
// workgroup, come through scalar loads.  The per-design sum runs over k in ascending order,
// exactly as the one-design kernel, so both give the same table bit for bit.
template <int DB>
__global__ __launch_bounds__(256) void pod_reconstruct_batch_kernel(const float *__restrict__ mean,
                                                                    const float *__restrict__ basis, int r,
                                                                    const double *__restrict__ cd, int B, int Bp,
                                                                    int n_groups, int64_t n_e,
                                                                    double *__restrict__ tables) {
  const int g = blockIdx.x % n_groups;
  const int64_t e = (int64_t)(blockIdx.x / n_groups) * 256 + threadIdx.x;
  if (e >= n_e) return;
  const double m = mean[e];
  double v[DB];
#pragma unroll
  for (int d = 0; d < DB; ++d) v[d] = m;
  const double *cg = cd + g * DB;
  for (int k = 0; k < r; ++k) {
    const double x = (double)basis[(int64_t)k * n_e + e];
    const double *ck = cg + (int64_t)k * Bp;
#pragma unroll
    for (int d = 0; d < DB; ++d) v[d] += x * ck[d];
  }
#pragma unroll
  for (int d = 0; d < DB; ++d)
    if (g * DB + d < B) tables[(int64_t)(g * DB + d) * n_e + e] = v[d];
}

// Relative Frobenius error of listed table rows against exact rows; one workgroup per design
// (grid x), with per-design strides of the table and of the exact rows.  Each thread keeps four
// partial sums (elements i, i + T, i + 2T, i + 3T of every stride of 4T), combined in a fixed
// order and then over a fixed tree, so the error is bitwise reproducible.
constexpr int kRowsErrThreads = 1024;
__global__ __launch_bounds__(kRowsErrThreads) void rows_error_kernel(const double *__restrict__ table, int64_t Kp,
                                                                     int K, const int32_t *__restrict__ rows,
                                                                     int n_rows, int64_t n_pairs,
                                                                     const double *__restrict__ exact,
                                                                     double *__restrict__ err, double tol,
                                                                     int32_t *__restrict__ gate,
                                                                     int64_t table_dstride) {
  constexpr int T = kRowsErrThreads;
  __shared__ double num[T], den[T];
  table += blockIdx.x * table_dstride;
  exact += (int64_t)blockIdx.x * n_rows * K;
  const int n = n_rows * K;   // the host checks that it fits an int
  // element i0 + u T goes to partial sum u mod 4, in ascending i0; 16 elements' loads are issued
  // together (the table row of an element is known only after its row index has arrived)
  double a[4] = {0.0, 0.0, 0.0, 0.0}, b[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i0 = threadIdx.x; i0 < n; i0 += 16 * T) {
    double x[16], y[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int i = i0 + u * T;
      x[u] = y[u] = 0.0;
      if (i < n) {
        const int rr = (int)((unsigned)i / (unsigned)K), c = i - rr * K;
        const int64_t p = rows[rr];
        x[u] = exact[i];
        y[u] = (p >= 0 && p < n_pairs) ? table[p * Kp + c] : __builtin_nan("");
      }
    }
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (i0 + u * T < n) {
        a[u & 3] += (y[u] - x[u]) * (y[u] - x[u]);
        b[u & 3] += x[u] * x[u];
      }
  }
  num[threadIdx.x] = (a[0] + a[1]) + (a[2] + a[3]);
  den[threadIdx.x] = (b[0] + b[1]) + (b[2] + b[3]);
  __syncthreads();
  for (int s = T / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) { num[threadIdx.x] += num[threadIdx.x + s]; den[threadIdx.x] += den[threadIdx.x + s]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double e = sqrt(num[0] / den[0]);
    err[blockIdx.x] = e;
    if (gate) gate[blockIdx.x] = e <= tol ? 0 : 1;   // NaN (bad row, empty reference) also asks for the exact table
  }
}

// ---- MLP -----------------------------------------------------------------------------
__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// Z[b][o] = bias[o] + sum_i H[b][i] W[i][o], H = x (layer 0) or GELU(previous Z).  One workgroup
// per batch row and block of outputs: the row's inputs (through GELU) are computed once into LDS,
// then every thread sums its output in ascending i.
constexpr int kMlpMaxWidth = 4096;
// Forward pass of all layers, one workgroup per batch row; a layer's inputs (x, then GELU of the
// previous layer's pre-activations) sit in LDS.  Output o of layer l is bias[o] + sum_i h[i] W[i][o],
// summed over i in order (unrolled so that the weight loads are in flight together); Z_l is stored
// for the backward pass, and the last layer's Z is also y.
struct MlpLayout {
  int n_layers, widths[9];
  int64_t w_off[8], z_off[8];   // offsets of W_l in the parameters and of Z_l in the activations
};
__global__ __launch_bounds__(256) void mlp_forward_kernel(MlpLayout m, const float *__restrict__ params,
                                                          const float *__restrict__ x, float *__restrict__ act,
                                                          float *__restrict__ y) {
  __shared__ float hs[2][kMlpMaxWidth];
  const int b = blockIdx.x;
  for (int i = threadIdx.x; i < m.widths[0]; i += blockDim.x) hs[0][i] = x[(int64_t)b * m.widths[0] + i];
  __syncthreads();
  int cur = 0;
  for (int l = 0; l < m.n_layers; ++l) {
    const int fi = m.widths[l], fo = m.widths[l + 1];
    const float *W = params + m.w_off[l], *bias = W + (int64_t)fi * fo;
    float *Z = act + m.z_off[l] + (int64_t)b * fo;
    const float *h = hs[cur];
    for (int o = threadIdx.x; o < fo; o += blockDim.x) {
      float z = bias[o];
      const float *w = W + o;
      int i = 0;
      for (; i + 16 <= fi; i += 16) {
        float wv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) wv[u] = w[(int64_t)(i + u) * fo];
#pragma unroll
        for (int u = 0; u < 16; ++u) z += h[i + u] * wv[u];
      }
      for (; i < fi; ++i) z += h[i] * w[(int64_t)i * fo];
      Z[o] = z;
      if (l == m.n_layers - 1) y[(int64_t)b * fo + o] = z;
      hs[cur ^ 1][o] = gelu(z);
    }
    __syncthreads();
    cur ^= 1;
  }
}

// dZ = dH * GELU'(Z) (or dY unchanged for the output layer)
__global__ void mlp_dz(const float *__restrict__ dH, const float *__restrict__ Z, int64_t n, int apply,
                       float *__restrict__ dZ) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  dZ[i] = apply ? dH[i] * gelu_grad(Z[i]) : dH[i];
}

// dW[i][o] = sum_b H[b][i] dZ[b][o]; db[o] = sum_b dZ[b][o]  (batch order fixed)
__global__ __launch_bounds__(256) void mlp_dw(const float *__restrict__ in, int in_gelu, const float *__restrict__ dZ,
                                              int batch, int fi, int fo, float *__restrict__ dW,
                                              float *__restrict__ db) {
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (id >= (int64_t)(fi + 1) * fo) return;
  const int i = (int)(id / fo), o = (int)(id % fo);
  float s = 0.0f;
  if (i < fi) {
    for (int b = 0; b < batch; ++b) {
      const float h = in[(int64_t)b * fi + i];
      s += (in_gelu ? gelu(h) : h) * dZ[(int64_t)b * fo + o];
    }
    dW[(int64_t)i * fo + o] = s;
  } else {
    for (int b = 0; b < batch; ++b) s += dZ[(int64_t)b * fo + o];
    db[o] = s;
  }
}

// dH[b][i] = sum_o dZ[b][o] W[i][o]
__global__ __launch_bounds__(256) void mlp_dh(const float *__restrict__ dZ, const float *__restrict__ W, int batch,
                                              int fi, int fo, float *__restrict__ dH) {
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (id >= (int64_t)batch * fi) return;
  const int b = (int)(id / fi), i = (int)(id % fi);
  float s = 0.0f;
  for (int o = 0; o < fo; ++o) s += dZ[(int64_t)b * fo + o] * W[(int64_t)i * fo + o];
  dH[id] = s;
}

__global__ __launch_bounds__(256) void mse_kernel(const float *__restrict__ y, const float *__restrict__ t, int64_t n,
                                                  float *__restrict__ dy, float *__restrict__ loss) {
  __shared__ float red[256];
  float s = 0.0f;
  const float scale = 2.0f / (float)n;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const float d = y[i] - t[i];
    dy[i] = scale * d;
    s += d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = red[0] / (float)n;
}

__global__ void adam_kernel(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

static bool mlp_ok(const igamt_mlp_desc *d) {
  if (!d || d->n_layers < 1 || d->n_layers > 8 || d->batch < 1) return false;
  for (int l = 0; l <= d->n_layers; ++l)
    if (d->widths[l] < 1 || d->widths[l] > kMlpMaxWidth) return false;
  return true;
}

static int64_t param_offset(const igamt_mlp_desc *d, int layer) {   // offset of W_layer (0-based layer)
  int64_t off = 0;
  for (int l = 0; l < layer; ++l) off += (int64_t)d->widths[l] * d->widths[l + 1] + d->widths[l + 1];
  return off;
}

static int64_t act_offset(const igamt_mlp_desc *d, int layer) {     // offset of Z_layer in the activations
  int64_t off = 0;
  for (int l = 0; l < layer; ++l) off += (int64_t)d->batch * d->widths[l + 1];
  return off;
}

static unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace igamt

using namespace igamt;

extern "C" igamt_status igamt_pod_build(const double *d_snap, int32_t n_s, int64_t n_e, int32_t r, float *d_mean,
                                        float *d_basis, double *h_sigma, double *h_coeffs, double *d_work,
                                        void *stream) {
  if (!d_snap || !d_mean || !d_basis || !h_sigma || !d_work || n_s < 2 || n_e < 1 || r < 1 || r > n_s) {
    set_error("invalid POD arguments");
    return IGAMT_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  // workspace: G (n_s^2) | V Sigma^-1 (n_s r) | mean (n_e) | partial Grams (n_slices n_s^2)
  const int n_slices = 16;
  double *G = d_work;
  double *Vs = G + (int64_t)n_s * n_s;
  double *mean = Vs + (int64_t)n_s * r;
  double *part = mean + n_e;
  hipLaunchKernelGGL(column_mean_kernel, dim3(blocks_for(n_e)), dim3(256), 0, s, d_snap, n_s, n_e, mean);
  IGAMT_LAUNCH_CHECK();
  const int nb = (n_s + GT - 1) / GT;
  const int n_pairs = nb * (nb + 1) / 2;
  hipLaunchKernelGGL(gram_kernel, dim3((unsigned)(n_pairs * n_slices)), dim3(256), 0, s, d_snap, mean, n_s, n_e,
                     n_slices, nb, part);
  IGAMT_LAUNCH_CHECK();
  hipLaunchKernelGGL(gram_sum_kernel, dim3(blocks_for((int64_t)n_s * n_s)), dim3(256), 0, s, part, n_s, n_slices, G);
  IGAMT_LAUNCH_CHECK();
  std::vector<double> A((size_t)n_s * n_s), V;
  IGAMT_HIP(hipMemcpyAsync(A.data(), G, A.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  IGAMT_HIP(hipStreamSynchronize(s));
  if (!sym_eigen(A, n_s, V)) {
    set_error("POD: the symmetric QR iteration did not converge within its step cap");
    return IGAMT_EDEGENERATE;
  }
  std::vector<int> order(n_s);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(),
            [&](int a, int b) { return A[(size_t)a * n_s + a] > A[(size_t)b * n_s + b]; });
  std::vector<double> vs((size_t)n_s * r);
  for (int k = 0; k < n_s; ++k) h_sigma[k] = std::sqrt(std::max(A[(size_t)order[k] * n_s + order[k]], 0.0));
  for (int k = 0; k < r; ++k) {
    if (!(h_sigma[k] > 0.0)) { set_error("POD rank exceeds the rank of the snapshots"); return IGAMT_EINVAL; }
    // sign convention: largest-magnitude entry of each eigenvector positive
    int im = 0;
    for (int i = 1; i < n_s; ++i)
      if (std::fabs(V[(size_t)i * n_s + order[k]]) > std::fabs(V[(size_t)im * n_s + order[k]])) im = i;
    const double sg = V[(size_t)im * n_s + order[k]] < 0 ? -1.0 : 1.0;
    for (int i = 0; i < n_s; ++i) {
      vs[(size_t)i * r + k] = sg * V[(size_t)i * n_s + order[k]] / h_sigma[k];
      if (h_coeffs) h_coeffs[(size_t)i * r + k] = sg * V[(size_t)i * n_s + order[k]] * h_sigma[k];
    }
  }
  IGAMT_HIP(hipMemcpyAsync(Vs, vs.data(), vs.size() * sizeof(double), hipMemcpyHostToDevice, s));
  const size_t shm = (size_t)n_s * 16 * sizeof(double);
  if (shm > 65536) IGAMT_HIP(hipFuncSetAttribute((const void *)pod_basis_kernel,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
  hipLaunchKernelGGL(pod_basis_kernel, dim3(blocks_for(n_e), (unsigned)((r + 15) / 16)), dim3(256), shm, s, d_snap,
                     mean, Vs, n_s, n_e, r, d_basis, d_mean);
  IGAMT_LAUNCH_CHECK();
  IGAMT_HIP(hipStreamSynchronize(s));
  return IGAMT_OK;
}

extern "C" igamt_status igamt_table_from_pod(igamt_plan *P, const float *d_mean, const float *d_basis, int32_t r,
                                             const float *d_coeffs, double coeff_scale, void *stream) {
  if (!P || !d_mean || !d_basis || !d_coeffs || r < 1 || r > 256) { set_error("invalid argument"); return IGAMT_EINVAL; }
  igamt_status st = ensure_device(P);
  if (st) return st;
  const int64_t n_e = P->n_pairs * P->K;
  hipLaunchKernelGGL(pod_reconstruct_kernel, dim3(blocks_for(n_e)), dim3(256), 0, (hipStream_t)stream, d_mean,
                     d_basis, r, d_coeffs, coeff_scale, n_e, P->K, (int64_t)P->Kp, P->dev.table);
  IGAMT_LAUNCH_CHECK();
  return derive_table_copies(P, stream);
}

extern "C" igamt_status igamt_table_rows_error(const igamt_plan *P, const int32_t *d_rows, int32_t n_rows,
                                               const double *d_exact, double *d_err, void *stream) {
  if (!P || !d_rows || !d_exact || !d_err || n_rows < 1) { set_error("invalid argument"); return IGAMT_EINVAL; }
  if ((int64_t)n_rows * P->K > INT32_MAX) { set_error("too many check rows"); return IGAMT_EINVAL; }
  if (!P->dev.ready || !P->tables_ready) { set_error("tables not built"); return IGAMT_ESTATE; }
  hipLaunchKernelGGL(rows_error_kernel, dim3(1), dim3(kRowsErrThreads), 0, (hipStream_t)stream, P->dev.table, (int64_t)P->Kp,
                     P->K, d_rows, n_rows, P->n_pairs, d_exact, d_err, 0.0, nullptr, 0);
  IGAMT_LAUNCH_CHECK();
  return IGAMT_OK;
}

extern "C" igamt_status igamt_table_rows_check(const igamt_plan *P, const int32_t *d_rows, int32_t n_rows,
                                               const double *d_exact, double tol, double *d_err, int32_t *d_gate,
                                               void *stream) {
  if (!P || !d_rows || !d_exact || !d_err || !d_gate || n_rows < 1 || !(tol >= 0.0)) {
    set_error("invalid argument");
    return IGAMT_EINVAL;
  }
  if ((int64_t)n_rows * P->K > INT32_MAX) { set_error("too many check rows"); return IGAMT_EINVAL; }
  if (!P->dev.ready || !P->tables_ready) { set_error("tables not built"); return IGAMT_ESTATE; }
  hipLaunchKernelGGL(rows_error_kernel, dim3(1), dim3(kRowsErrThreads), 0, (hipStream_t)stream, P->dev.table, (int64_t)P->Kp,
                     P->K, d_rows, n_rows, P->n_pairs, d_exact, d_err, tol, d_gate, 0);
  IGAMT_LAUNCH_CHECK();
  return IGAMT_OK;
}

extern "C" int64_t igamt_mlp_n_params(const igamt_mlp_desc *d) {
  if (!mlp_ok(d)) return -1;
  return param_offset(d, d->n_layers);
}

extern "C" igamt_status igamt_mlp_forward(const igamt_mlp_desc *d, const float *d_params, const float *d_x,
                                          float *d_act, float *d_y, void *stream) {
  if (!mlp_ok(d) || !d_params || !d_x || !d_act || !d_y) { set_error("invalid MLP arguments"); return IGAMT_EINVAL; }
  MlpLayout m;
  m.n_layers = d->n_layers;
  for (int l = 0; l <= d->n_layers; ++l) m.widths[l] = d->widths[l];
  for (int l = 0; l < d->n_layers; ++l) {
    m.w_off[l] = param_offset(d, l);
    m.z_off[l] = act_offset(d, l);
  }
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)d->batch), dim3(256), 0, (hipStream_t)stream, m, d_params, d_x,
                     d_act, d_y);
  IGAMT_LAUNCH_CHECK();
  return IGAMT_OK;
}

extern "C" igamt_status igamt_mse_loss(const igamt_mlp_desc *d, const float *d_y, const float *d_target, float *d_dy,
                                       float *d_loss, void *stream) {
  if (!mlp_ok(d) || !d_y || !d_target || !d_dy || !d_loss) { set_error("invalid arguments"); return IGAMT_EINVAL; }
  const int64_t n = (int64_t)d->batch * d->widths[d->n_layers];
  hipLaunchKernelGGL(mse_kernel, dim3(1), dim3(256), 0, (hipStream_t)stream, d_y, d_target, n, d_dy, d_loss);
  IGAMT_LAUNCH_CHECK();
  return IGAMT_OK;
}

extern "C" igamt_status igamt_mlp_backward(const igamt_mlp_desc *d, const float *d_params, const float *d_x,
                                           const float *d_act, const float *d_dy, float *d_grads, float *d_scratch,
                                           void *stream) {
  if (!mlp_ok(d) || !d_params || !d_x || !d_act || !d_dy || !d_grads || !d_scratch) {
    set_error("invalid MLP arguments");
    return IGAMT_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  int wmax = 0;
  for (int l = 0; l <= d->n_layers; ++l) wmax = std::max(wmax, d->widths[l]);
  float *dZ = d_scratch;
  float *dH = d_scratch + (int64_t)d->batch * wmax;
  for (int l = d->n_layers - 1; l >= 0; --l) {
    const int fi = d->widths[l], fo = d->widths[l + 1];
    const int64_t n = (int64_t)d->batch * fo;
    const float *Z = d_act + act_offset(d, l);
    const float *upstream = l == d->n_layers - 1 ? d_dy : dH;
    hipLaunchKernelGGL(mlp_dz, dim3(blocks_for(n)), dim3(256), 0, s, upstream, Z, n, l == d->n_layers - 1 ? 0 : 1, dZ);
    IGAMT_LAUNCH_CHECK();
    const float *W = d_params + param_offset(d, l);
    float *gW = d_grads + param_offset(d, l);
    float *gb = gW + (int64_t)fi * fo;
    const float *in = l == 0 ? d_x : d_act + act_offset(d, l - 1);
    hipLaunchKernelGGL(mlp_dw, dim3(blocks_for((int64_t)(fi + 1) * fo)), dim3(256), 0, s, in, l > 0 ? 1 : 0, dZ,
                       d->batch, fi, fo, gW, gb);
    IGAMT_LAUNCH_CHECK();
    if (l > 0) {
      hipLaunchKernelGGL(mlp_dh, dim3(blocks_for((int64_t)d->batch * fi)), dim3(256), 0, s, dZ, W, d->batch, fi, fo,
                         dH);
      IGAMT_LAUNCH_CHECK();
    }
  }
  return IGAMT_OK;
}

extern "C" igamt_status igamt_adam_step(float *d_params, const float *d_grads, float *d_m, float *d_v, int64_t n,
                                        float lr, float beta1, float beta2, float eps, int32_t step, void *stream) {
  if (!d_params || !d_grads || !d_m || !d_v || n < 0 || step < 1) { set_error("invalid Adam arguments"); return IGAMT_EINVAL; }
  if (n == 0) return IGAMT_OK;
  const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, d_params, d_grads, d_m, d_v,
                     n, lr, beta1, beta2, eps, c1, c2);
  IGAMT_LAUNCH_CHECK();
  return IGAMT_OK;
}

extern "C" igamt_status igamt_tables_build_rows(igamt_plan *P, const int32_t *d_rows, int32_t n_rows, double *d_out,
                                                void *stream);
extern "C" igamt_status igamt_tables_build_gated(igamt_plan *P, const int32_t *d_gate, void *stream);

extern "C" igamt_status igamt_table_learned(igamt_plan *P, const igamt_mlp_desc *mlp, const float *d_params,
                                            const float *d_x, float *d_act, float *d_y, const float *d_mean,
                                            const float *d_basis, double coeff_scale, const int32_t *d_rows,
                                            int32_t n_rows, double *d_exact_rows, double tol, double *d_err,
                                            int32_t *d_gate, void *stream) {
  if (!P || !mlp || !d_params || !d_x || !d_act || !d_y || !d_mean || !d_basis || !d_rows || !d_exact_rows ||
      !d_err || !d_gate) {
    set_error("NULL argument");
    return IGAMT_EINVAL;
  }
  if (mlp->batch != 1) { set_error("the learned table path predicts one design (batch 1)"); return IGAMT_EINVAL; }
  igamt_status st;
  if ((st = igamt_mlp_forward(mlp, d_params, d_x, d_act, d_y, stream))) return st;
  if ((st = igamt_table_from_pod(P, d_mean, d_basis, mlp->widths[mlp->n_layers], d_y, coeff_scale, stream))) return st;
  if ((st = igamt_tables_build_rows(P, d_rows, n_rows, d_exact_rows, stream))) return st;
  if ((st = igamt_table_rows_check(P, d_rows, n_rows, d_exact_rows, tol, d_err, d_gate, stream))) return st;
  return igamt_tables_build_gated(P, d_gate, stream);
}

// ---- batches of designs ------------------------------------------------------------------
static constexpr int kPodGroup = 16;   // designs per thread in the batched reconstruction

extern "C" igamt_status igamt_tables_from_pod_batch(const igamt_plan *P, const float *d_mean, const float *d_basis,
                                                    int32_t r, const float *d_coeffs, int32_t n_design,
                                                    double coeff_scale, double *d_coef_work, double *d_tables,
                                                    void *stream) {
  if (!P || !d_mean || !d_basis || !d_coeffs || !d_coef_work || !d_tables || r < 1 || r > 256 || n_design < 1) {
    set_error("invalid argument");
    return IGAMT_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  const int n_groups = (n_design + kPodGroup - 1) / kPodGroup, Bp = n_groups * kPodGroup;
  const int64_t n_e = P->n_pairs * P->K;
  hipLaunchKernelGGL(pod_coeffs_kernel, dim3(blocks_for((int64_t)r * Bp)), dim3(256), 0, s, d_coeffs, n_design, Bp, r,
                     coeff_scale, d_coef_work);
  IGAMT_LAUNCH_CHECK();
  const int64_t nb = (int64_t)blocks_for(n_e) * n_groups;
  if (nb > 0x7fffffffLL) { set_error("batch too large for one launch"); return IGAMT_EINVAL; }
  hipLaunchKernelGGL(pod_reconstruct_batch_kernel<kPodGroup>, dim3((unsigned)nb), dim3(256), 0, s, d_mean, d_basis,
                     r, d_coef_work, n_design, Bp, n_groups, n_e, d_tables);
  IGAMT_LAUNCH_CHECK();
  return IGAMT_OK;
}

extern "C" int64_t igamt_pod_batch_work_doubles(int32_t r, int32_t n_design) {
  if (r < 1 || n_design < 1) return -1;
  return (int64_t)r * ((n_design + kPodGroup - 1) / kPodGroup) * kPodGroup;
}

extern "C" igamt_status igamt_tables_rows_check_batch(const igamt_plan *P, const double *d_tables, int32_t n_design,
                                                      const int32_t *d_rows, int32_t n_rows, const double *d_exact,
                                                      double tol, double *d_err, int32_t *d_gate, void *stream) {
  if (!P || !d_tables || !d_rows || !d_exact || !d_err || !d_gate || n_rows < 1 || n_design < 1 ||
      !(tol >= 0.0)) {
    set_error("invalid argument");
    return IGAMT_EINVAL;
  }
  if ((int64_t)n_rows * P->K > INT32_MAX) { set_error("too many check rows"); return IGAMT_EINVAL; }
  hipLaunchKernelGGL(rows_error_kernel, dim3((unsigned)n_design), dim3(kRowsErrThreads), 0, (hipStream_t)stream, d_tables,
                     (int64_t)P->K, P->K, d_rows, n_rows, P->n_pairs, d_exact, d_err, tol, d_gate,
                     P->n_pairs * P->K);
  IGAMT_LAUNCH_CHECK();
  return IGAMT_OK;
}

extern "C" igamt_status igamt_tables_build_batch(igamt_plan *P, const double *d_ctrl, int32_t n_design,
                                                 const int32_t *d_gate, double *d_tables, void *stream);
extern "C" igamt_status igamt_tables_build_rows_batch(igamt_plan *P, const double *d_ctrl, int32_t n_design,
                                                      const int32_t *d_rows, int32_t n_rows, double *d_out,
                                                      void *stream);

extern "C" igamt_status igamt_tables_learned_batch(igamt_plan *P, const igamt_mlp_desc *mlp, const float *d_params,
                                                   const float *d_x, float *d_act, float *d_y, const float *d_mean,
                                                   const float *d_basis, double coeff_scale, const double *d_ctrl,
                                                   const int32_t *d_rows, int32_t n_rows, double *d_exact_rows,
                                                   double tol, double *d_err, int32_t *d_gate, double *d_coef_work,
                                                   double *d_tables, void *stream) {
  if (!P || !mlp || !d_params || !d_x || !d_act || !d_y || !d_mean || !d_basis || !d_ctrl || !d_rows ||
      !d_exact_rows || !d_err || !d_gate || !d_coef_work || !d_tables) {
    set_error("NULL argument");
    return IGAMT_EINVAL;
  }
  const int32_t B = mlp->batch;
  igamt_status st;
  if ((st = igamt_mlp_forward(mlp, d_params, d_x, d_act, d_y, stream))) return st;
  if ((st = igamt_tables_from_pod_batch(P, d_mean, d_basis, mlp->widths[mlp->n_layers], d_y, B, coeff_scale,
                                        d_coef_work, d_tables, stream)))
    return st;
  if ((st = igamt_tables_build_rows_batch(P, d_ctrl, B, d_rows, n_rows, d_exact_rows, stream))) return st;
  if ((st = igamt_tables_rows_check_batch(P, d_tables, B, d_rows, n_rows, d_exact_rows, tol, d_err, d_gate, stream)))
    return st;
  return igamt_tables_build_batch(P, d_ctrl, B, d_gate, d_tables, stream);
}
