// Device helpers for the libigamt kernels: B-spline and Bernstein evaluation,
// 3x3 algebra, precision conversions and error-checking macros.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>
#include <string>
#include <type_traits>

#include "igamt_internal.h"

#define IGAMT_HIP(call)                                                              \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess) {                                                          \
      igamt::set_error(std::string(#call) + ": " + hipGetErrorString(e_));           \
      return IGAMT_EHIP;                                                             \
    }                                                                                \
  } while (0)

#define IGAMT_LAUNCH_CHECK()                                                         \
  do {                                                                               \
    hipError_t e_ = hipGetLastError();                                               \
    if (e_ != hipSuccess) {                                                          \
      igamt::set_error(std::string("kernel launch: ") + hipGetErrorString(e_));      \
      return IGAMT_EHIP;                                                             \
    }                                                                                \
  } while (0)

namespace igamt {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// Knot span containing x: the largest i in [p, n-1] with U[i] <= x (x = 1 goes
// to the last non-empty span).  U has n + p + 1 entries.
// Wait for this wave's LDS operations, then synchronise the workgroup.  Unlike __syncthreads this
// does not wait for outstanding global loads or stores (register prefetches stay in flight, stores
// drain in the background); it orders LDS accesses only.
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

__device__ inline int find_span(const double *__restrict__ U, int n, int p, double x) {
  if (x >= U[n]) return n - 1;
  if (x <= U[p]) return p;
  int lo = p, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (x < U[mid]) hi = mid; else lo = mid;
  }
  return lo;
}

// Values N[r] and first derivatives dN[r] of the P+1 B-splines that are non-zero
// on span `span` (global index span - P + r), by the triangular Cox-de Boor
// recursion over the degrees 0..P.
template <int P>
__device__ inline void bspline_ders(const double *__restrict__ U, int span, double x,
                                    double (&N)[P + 1], double (&dN)[P + 1]) {
  double V[P + 1];
  double Vp[P + 1];
#pragma unroll
  for (int r = 0; r <= P; ++r) { V[r] = 0.0; Vp[r] = 0.0; }
  V[0] = 1.0;
#pragma unroll
  for (int k = 1; k <= P; ++k) {
#pragma unroll
    for (int r = 0; r <= P; ++r) Vp[r] = V[r];
#pragma unroll
    for (int r = 0; r <= k; ++r) {
      double v = 0.0;
      if (r >= 1) {
        const double den = U[span + r] - U[span - k + r];
        if (den > 0.0) v += (x - U[span - k + r]) / den * Vp[r - 1];
      }
      if (r <= k - 1) {
        const double den = U[span + r + 1] - U[span - k + r + 1];
        if (den > 0.0) v += (U[span + r + 1] - x) / den * Vp[r];
      }
      V[r] = v;
    }
  }
#pragma unroll
  for (int r = 0; r <= P; ++r) {
    double d = 0.0;
    if (r >= 1) {
      const double den = U[span + r] - U[span - P + r];
      if (den > 0.0) d += Vp[r - 1] / den;
    }
    if (r <= P - 1) {
      const double den = U[span + r + 1] - U[span - P + r + 1];
      if (den > 0.0) d -= Vp[r] / den;
    }
    N[r] = V[r];
    dN[r] = P * d;
  }
}

// Bernstein polynomials of degree q at x (runtime q <= kMaxQ).
__device__ inline void bernstein(int q, double x, double *B) {
  // B^q_c = C(q,c) x^c (1-x)^(q-c), built by the de Casteljau-type recursion
  // B^k_c = (1-x) B^{k-1}_c + x B^{k-1}_{c-1}.
  B[0] = 1.0;
  for (int k = 1; k <= q; ++k) {
    B[k] = x * B[k - 1];
    for (int c = k - 1; c >= 1; --c) B[c] = (1.0 - x) * B[c] + x * B[c - 1];
    B[0] = (1.0 - x) * B[0];
  }
}

__device__ inline double det3(const double (&J)[3][3]) {
  return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
         J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
         J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

// F = J^-1 by cofactors; returns det J.
__device__ inline double inv3(const double (&J)[3][3], double (&F)[3][3]) {
  const double D = det3(J);
  const double r = 1.0 / D;
  F[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) * r;
  F[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * r;
  F[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * r;
  F[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) * r;
  F[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * r;
  F[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * r;
  F[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) * r;
  F[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * r;
  F[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * r;
  return D;
}

// Round-to-nearest-even float -> bfloat16 bits (finite inputs).
__device__ inline uint16_t f32_to_bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf16_bits_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

__device__ inline uint16_t f32_to_f16_bits(float f) {
  // an empty asm keeps the compiler from merging a preceding double -> float rounding into one
  // double -> half rounding, which it expands into a long integer sequence; this way the two
  // roundings stay as written, each one hardware conversion
  asm("" : "+v"(f));
  _Float16 h = (_Float16)f;
  return *reinterpret_cast<uint16_t *>(&h);
}
__device__ inline float f16_bits_to_f32(uint16_t b) {
  _Float16 h = *reinterpret_cast<_Float16 *>(&b);
  return (float)h;
}

// x ~ hi + lo with both parts representable in bfloat16.
__device__ inline void split_bf16(double x, uint16_t &hi, uint16_t &lo) {
  hi = f32_to_bf16_bits((float)x);
  lo = f32_to_bf16_bits((float)(x - (double)bf16_bits_to_f32(hi)));
}
__device__ inline void split_f16(double x, uint16_t &hi, uint16_t &lo) {
  hi = f32_to_f16_bits((float)x);
  lo = f32_to_f16_bits((float)(x - (double)f16_bits_to_f32(hi)));
}

// Power-of-two scale that maps a magnitude bound to about 2^14 (float16 range).
__device__ inline double f16_scale_for(double bound) {
  if (!(bound > 0.0)) return 1.0;
  int e;
  frexp(bound, &e);           // bound = m 2^e, m in [0.5, 1)
  return ldexp(1.0, 14 - e);  // bound * scale < 2^14
}

// A_ij,ab at one sample from the rows F_i, F_j of F = J^-1 and D = det J (the Cartesian form of
// eq. (37)).  The elasticity tensor's symmetry gives A_ij,ab = A_ji,ba; callers pass (i, a) and
// (j, b) ordered so that 3 i + a <= 3 j + b, and the two entries come out bit-identical.
__device__ inline double elastic_density(const double *Fi, const double *Fj, double D, int aa, int bb, double lam,
                                         double mu) {
  const double fij = Fi[0] * Fj[0] + Fi[1] * Fj[1] + Fi[2] * Fj[2];
  return D * (lam * Fi[aa] * Fj[bb] + (aa == bb ? mu * fij : 0.0) + mu * Fi[bb] * Fj[aa]);
}

// a wave-uniform double moved to scalar registers
__device__ inline double uniform_f64(double x) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b), hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

constexpr int max3(int a, int b, int c) { return a > b ? (a > c ? a : c) : (b > c ? b : c); }

// Values and first derivatives of the B-splines of degree PD[k] non-zero on span `span` of direction
// k (a run-time direction, compile-time degrees), padded with zeros to PMX + 1 entries.
template <int P0, int P1, int P2>
__device__ inline void bspline_ders_dir(int k, const double *__restrict__ U, int span, double x,
                                        double (&N)[max3(P0, P1, P2) + 1], double (&dN)[max3(P0, P1, P2) + 1]) {
  constexpr int PMX = max3(P0, P1, P2);
#pragma unroll
  for (int r = 0; r <= PMX; ++r) N[r] = dN[r] = 0.0;
  if (k == 0) {
    double a[P0 + 1], b[P0 + 1];
    bspline_ders<P0>(U, span, x, a, b);
#pragma unroll
    for (int r = 0; r <= P0; ++r) { N[r] = a[r]; dN[r] = b[r]; }
  } else if (k == 1) {
    double a[P1 + 1], b[P1 + 1];
    bspline_ders<P1>(U, span, x, a, b);
#pragma unroll
    for (int r = 0; r <= P1; ++r) { N[r] = a[r]; dN[r] = b[r]; }
  } else {
    double a[P2 + 1], b[P2 + 1];
    bspline_ders<P2>(U, span, x, a, b);
#pragma unroll
    for (int r = 0; r <= P2; ++r) { N[r] = a[r]; dN[r] = b[r]; }
  }
}

// The tensor sum of spline_jacobian3 (below) from given spans and 1-D basis values and derivatives.
template <int P0, int P1, int P2, bool ROLL_X = false>
__device__ inline void spline_jacobian_sum(const int *n, const double *__restrict__ ctrl, const double *__restrict__ w,
                                           const int (&span)[3], const double (&N)[3][max3(P0, P1, P2) + 1],
                                           const double (&dN)[3][max3(P0, P1, P2) + 1], double (&J)[3][3]) {
  double A[3] = {0.0, 0.0, 0.0}, W = 0.0, dW[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int c = 0; c < 3; ++c) J[c][0] = J[c][1] = J[c][2] = 0.0;
#pragma unroll 1
  for (int rz = 0; rz <= P2; ++rz) {
    const int iz = span[2] - P2 + rz;
#pragma unroll 1
    for (int ry = 0; ry <= P1; ++ry) {
      const int iy = span[1] - P1 + ry;
      const double wyz = N[1][ry] * N[2][rz];
      const double dy = dN[1][ry] * N[2][rz];
      const double dz = N[1][ry] * dN[2][rz];
      auto point = [&](int rx) {
        const int ix = span[0] - P0 + rx;
        const int64_t id = ix + (int64_t)n[0] * (iy + (int64_t)n[1] * iz);
        const double *c = ctrl + 3 * id;
        const double wi = w ? w[id] : 1.0;
        const double v = N[0][rx] * wyz * wi;
        const double g0 = dN[0][rx] * wyz * wi, g1 = N[0][rx] * dy * wi, g2 = N[0][rx] * dz * wi;
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
          A[cc] += c[cc] * v;
          J[cc][0] += c[cc] * g0;
          J[cc][1] += c[cc] * g1;
          J[cc][2] += c[cc] * g2;
        }
        W += v;
        dW[0] += g0;
        dW[1] += g1;
        dW[2] += g2;
      };
      if constexpr (ROLL_X) {
#pragma unroll 1
        for (int rx = 0; rx <= P0; ++rx) point(rx);
      } else {
#pragma unroll
        for (int rx = 0; rx <= P0; ++rx) point(rx);
      }
    }
  }
  if (w) {
    const double r = 1.0 / W;
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      const double M = A[cc] * r;
#pragma unroll
      for (int k = 0; k < 3; ++k) J[cc][k] = (J[cc][k] - M * dW[k]) * r;
    }
  }
}

// Jacobian of the trivariate spline map with control points ctrl ([n2][n1][n0][3], x fastest) at
// parameter x, degree P0, P1, P2 in the three directions; also returns the spans and the 1-D basis
// values and derivatives used (N[k][r], r <= Pk; zero above).  w: NULL for a B-spline map, else the
// NURBS weights ([n2][n1][n0]); the map is then A / W with A = sum w_i N_i P_i, W = sum w_i N_i, and
// dM/dx_k = (dA/dx_k - M dW/dx_k) / W.  ROLL_X keeps the innermost (x) control-point loop rolled
// too: fewer registers (more waves per SIMD) for kernels whose occupancy the Jacobian limits, the
// same sums in the same order.
template <int P0, int P1, int P2, bool ROLL_X = false>
__device__ inline void spline_jacobian3(const double *const *knots, const int *n, const double *__restrict__ ctrl,
                                        const double *__restrict__ w, const double (&x)[3], double (&J)[3][3],
                                        int (&span)[3], double (&N)[3][max3(P0, P1, P2) + 1],
                                        double (&dN)[3][max3(P0, P1, P2) + 1]) {
  constexpr int PD[3] = {P0, P1, P2};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    span[k] = find_span(knots[k], n[k], PD[k], x[k]);
    bspline_ders_dir<P0, P1, P2>(k, knots[k], span[k], x[k], N[k], dN[k]);
  }
  spline_jacobian_sum<P0, P1, P2, ROLL_X>(n, ctrl, w, span, N, dN, J);
}

// The same with one degree P in every direction.
template <int P, bool ROLL_X = false>
__device__ inline void spline_jacobian(const double *const *knots, const int *n, const double *__restrict__ ctrl,
                                       const double *__restrict__ w, const double (&x)[3], double (&J)[3][3],
                                       int (&span)[3], double (&N)[3][P + 1], double (&dN)[3][P + 1]) {
  spline_jacobian3<P, P, P, ROLL_X>(knots, n, ctrl, w, x, J, span, N, dN);
}

// NURBS control-point derivatives at one sample of a tensor grid: from the 1-D B-spline values NB
// and derivatives DB at the sample's abscissae si (spans SP), W = sum w N and d_n W; then with
// G[c][n] the sample's weights of d_n R_i (R_i = w_i N_i / W, d_n R_i = w_i (d_n N_i - N_i d_n W / W) / W):
// out[0] = 1 / W, out[1 + c] = sum_n G[c][n] d_n W / W^2.  Degrees P0, P1, P2 per direction.
template <int P0, int P1, int P2, int MF, int MD>
__device__ inline void rational_terms3(const double *__restrict__ wts, const int *nM, const int (&SP)[3][MF],
                                       const double (&NB)[3][MF][MD], const double (&DB)[3][MF][MD],
                                       const int (&si)[3], const double *G, double *out) {
  double W = 0.0, dW[3] = {0.0, 0.0, 0.0};
  for (int rz = 0; rz <= P2; ++rz)
    for (int ry = 0; ry <= P1; ++ry)
      for (int rx = 0; rx <= P0; ++rx) {
        const int ix = SP[0][si[0]] - P0 + rx, iy = SP[1][si[1]] - P1 + ry, iz = SP[2][si[2]] - P2 + rz;
        const double wi = wts[ix + (int64_t)nM[0] * (iy + (int64_t)nM[1] * iz)];
        const double nx = NB[0][si[0]][rx], ny = NB[1][si[1]][ry], nz = NB[2][si[2]][rz];
        W += wi * nx * ny * nz;
        dW[0] += wi * DB[0][si[0]][rx] * ny * nz;
        dW[1] += wi * nx * DB[1][si[1]][ry] * nz;
        dW[2] += wi * nx * ny * DB[2][si[2]][rz];
      }
  const double r = 1.0 / W;
  out[0] = r;
  for (int c = 0; c < 3; ++c) out[1 + c] = (G[3 * c] * dW[0] + G[3 * c + 1] * dW[1] + G[3 * c + 2] * dW[2]) * r * r;
}

// NURBS weight of the tile-local macro control point lo + l, or 0 where lo + l lies past the net (a
// tile whose samples meet fewer spans than the widest tile: no sample lies in such a point's
// support, so its local gradient is an exact zero anyway).
__device__ inline double local_weight(const double *__restrict__ w, const int *nM, const int (&lo)[3], const int (&l)[3]) {
  const int i0 = lo[0] + l[0], i1 = lo[1] + l[1], i2 = lo[2] + l[2];
  if (i0 >= nM[0] || i1 >= nM[1] || i2 >= nM[2]) return 0.0;
  return w[i0 + (int64_t)nM[0] * (i1 + (int64_t)nM[1] * i2)];
}

// The split modes (BF16X3, F16X3) contract with the table resident in LDS when the padded table
// width is 128 or 256 columns (q <= 2 isotropic); their coefficient planes are then stored tiled:
// the 16 columns x 32 k of one MFMA fragment contiguous, lane (l16, kq) at (kq 16 + l16) 8, i.e.
// element (col, k) at ((col / 16) (Kp / 32) + k / 32) 512 + ((k % 32) / 8 16 + col % 16) 8 + k % 8.
// Other widths keep the column-major layout col Kp + k.
__host__ __device__ constexpr bool split_tiled(int64_t Kp) { return Kp == 128 || Kp == 256; }
__host__ __device__ inline int64_t split_coef_index(int64_t col, int64_t k, int64_t Kp, bool tiled) {
  if (!tiled) return col * Kp + k;
  return ((col >> 4) * (Kp >> 5) + (k >> 5)) * 512 + ((((k & 31) >> 3) << 4) + (col & 15)) * 8 + (k & 7);
}

// Macro-map degrees (per direction) the kernels are instantiated for: every isotropic degree 1..6,
// and every combination of degrees 1..3 that differs between directions.  X(p0, p1, p2) per entry;
// IGAMT_DEGREE_KEY gives the switch key of a degree triple.
#define IGAMT_DEGREE_KEY(a, b, c) ((a) * 64 + (b) * 8 + (c))
#define IGAMT_FOR_MACRO_DEGREES(X) \
  X(1, 1, 1) X(2, 2, 2) X(3, 3, 3) X(4, 4, 4) X(5, 5, 5) X(6, 6, 6) IGAMT_FOR_ANISO_MACRO_DEGREES(X)
#define IGAMT_FOR_ANISO_MACRO_DEGREES(X) \
  X(1, 1, 2) X(1, 1, 3) X(1, 2, 1) X(1, 2, 2) X(1, 2, 3) X(1, 3, 1) X(1, 3, 2) X(1, 3, 3) \
  X(2, 1, 1) X(2, 1, 2) X(2, 1, 3) X(2, 2, 1) X(2, 2, 3) X(2, 3, 1) X(2, 3, 2) X(2, 3, 3) \
  X(3, 1, 1) X(3, 1, 2) X(3, 1, 3) X(3, 2, 1) X(3, 2, 2) X(3, 2, 3) X(3, 3, 1) X(3, 3, 2)

__host__ __device__ inline int64_t align256(int64_t b) { return (b + 255) / 256 * 256; }

}  // namespace igamt
