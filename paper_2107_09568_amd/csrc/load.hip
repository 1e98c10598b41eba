// Load vector of the multiscale assembly (Section 3.2.2-3.2.3, eq. (39)-(41), (44)-(45),
// (53)-(55); Appendix A.1, eq. (85)-(88)).
//
// Table (eq. (54)-(55)), per tile control point A and Bernstein index C, seven slots:
//   F[A][C][0]     = int R_A(theta) N_C(T^r(theta)) det J_T(theta) dtheta     (volume)
//   F[A][C][1 + f] = int over tile face f of R_A N_C dGamma                     (faces)
// pulled back to the tile parameter domain; faces f = 2 d + side (side 0: theta_d = 0).  The
// tile's boundary control points sit at the identity positions, so T^r is the identity on its
// faces and dGamma is the unit-square measure.  The volume slot reuses the point records of the
// stiffness table builder (w det J_T and N_C at every micro element's Gauss points).
//
// Fit, per tile (box coordinates xi in [0,1]^3, J = J_M(a + h xi) diag(h)):
//   body:     bbar(xi) = b |det J|, projected onto Q_q (eq. (40), (44));
//   traction: on every macro face f the tile's box touches, tbar_f = t_f |J e_u x J e_v|
//             (the area element of eq. (87)-(88) for a face xi_d = const), projected onto the
//             face's (q+1)^2 Bernstein functions (eq. (41), (45)).
// The projections are the 1-D operator of eq. (23)-(24) applied per direction (the 2-D and 3-D
// operators are its Kronecker products).  Coefficients: coef[t][slot][a][C], slot 0 the body,
// 1 + f the faces (zero where the tile does not touch face f).
//
// Gather (eq. (53) and the conforming gluing): one thread per global dof 3 G + a sums, over the
// tiles holding G in ascending tile index, sum_slot sum_C coef[t][slot][a][C] F[A][C][slot]
// (slots of faces the tile does not touch skipped); no atomics, bitwise reproducible.
#include "device_common.h"

namespace igamt {

constexpr int kLoadSlots = 7;

struct LoadTableArgs {
  const double *knots[3];
  int nT[3], eT[3];
  const double *gx, *gw;
  int ng, qd[3], npi;        // projection degree per direction
  int64_t stride;            // doubles per point record
  const double *pts;         // point records of the table builder
  double *table;             // [nTt][npi][7]
};

template <int PT>
__global__ __launch_bounds__(64) void load_table_kernel(LoadTableArgs a) {
  const int64_t id = (int64_t)blockIdx.x * 64 + threadIdx.x;
  const int64_t nTt = (int64_t)a.nT[0] * a.nT[1] * a.nT[2];
  if (id >= nTt * a.npi) return;
  const int C = (int)(id % a.npi);
  const int64_t A = id / a.npi;
  const int ai[3] = {(int)(A % a.nT[0]), (int)((A / a.nT[0]) % a.nT[1]), (int)(A / ((int64_t)a.nT[0] * a.nT[1]))};
  const int q1x = a.qd[0] + 1, q1y = a.qd[1] + 1;
  const int ci[3] = {C % q1x, (C / q1x) % q1y, C / (q1x * q1y)};
  const int G = a.ng * a.ng * a.ng;
  double *out = a.table + id * kLoadSlots;
  // volume: the micro elements in the support of R_A, Gauss points in ascending order
  int lo[3], hi[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    lo[k] = max(ai[k] - PT, 0);
    hi[k] = min(ai[k], a.eT[k] - 1);
  }
  double vol = 0.0;
  for (int ez = lo[2]; ez <= hi[2]; ++ez)
    for (int ey = lo[1]; ey <= hi[1]; ++ey)
      for (int ex = lo[0]; ex <= hi[0]; ++ex) {
        const int e[3] = {ex, ey, ez};
        const int64_t el = ex + (int64_t)a.eT[0] * (ey + (int64_t)a.eT[1] * ez);
        for (int g = 0; g < G; ++g) {
          const int gi[3] = {g % a.ng, (g / a.ng) % a.ng, g / (a.ng * a.ng)};
          double R = 1.0;
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            const int span = e[k] + PT;
            const double l = a.knots[k][span], h = a.knots[k][span + 1];
            double N[PT + 1], dN[PT + 1];
            bspline_ders<PT>(a.knots[k], span, l + (h - l) * a.gx[gi[k]], N, dN);
            R *= N[ai[k] - e[k]];
          }
          const double *pd = a.pts + (el * G + g) * a.stride;
          vol += pd[0] * pd[1 + C] * R;
        }
      }
  out[0] = vol;
  // faces: A on face f, C in I_f; R_A and N_C are products of 1-D functions on the face
  for (int f = 0; f < 6; ++f) {
    const int d = f >> 1, side = f & 1;
    const int u = d == 0 ? 1 : 0, v = d == 2 ? 1 : 2;
    double s = 0.0;
    if (ai[d] == (side ? a.nT[d] - 1 : 0) && ci[d] == (side ? a.qd[d] : 0)) {
      for (int ev = max(ai[v] - PT, 0); ev <= min(ai[v], a.eT[v] - 1); ++ev)
        for (int eu = max(ai[u] - PT, 0); eu <= min(ai[u], a.eT[u] - 1); ++eu)
          for (int gv = 0; gv < a.ng; ++gv)
            for (int gu = 0; gu < a.ng; ++gu) {
              double val = 1.0, wt = 1.0;
              const int ee[2] = {eu, ev}, gg[2] = {gu, gv}, kk[2] = {u, v};
#pragma unroll
              for (int m = 0; m < 2; ++m) {
                const int k = kk[m], span = ee[m] + PT;
                const double l = a.knots[k][span], h = a.knots[k][span + 1];
                const double th = l + (h - l) * a.gx[gg[m]];
                double N[PT + 1], dN[PT + 1];
                bspline_ders<PT>(a.knots[k], span, th, N, dN);
                double B[kMaxQ + 1];
                bernstein(a.qd[k], th, B);
                val *= N[ai[k] - ee[m]] * B[ci[k]];
                wt *= (h - l) * a.gw[gg[m]];
              }
              s += wt * val;   // the end functions are 1 on the face, as are their Bernstein partners
            }
    }
    out[1 + f] = s;
  }
}

struct LoadFitArgs {
  const double *knots[3];
  int nM[3];
  const double *ctrl;
  const double *wts;      // NURBS weights of the macro map, or null (B-spline)
  const double *box_a[3];
  const double *box_h[3];
  int tiles[3];
  int64_t n_tiles;
  const double *fx;
  const double *fP3;         // per-direction 1-D projection operators [qd[k]+1][n_fit], concatenated
  int qd[3], nf, npi;
  double body[3];
  double traction[6][3];
  double *coef;              // [n_tiles][7][3][npi]
  int32_t *flag;
};

template <int P0, int P1, int P2>
__global__ __launch_bounds__(64) void load_fit_kernel(LoadFitArgs a) {
  constexpr int PMX = max3(P0, P1, P2);
  constexpr int PD[3] = {P0, P1, P2};
  __shared__ double vals[kMaxFit * kMaxFit * kMaxFit];   // |det J| at the body samples / face areas
  const int64_t t = blockIdx.x;
  const int tid = threadIdx.x;
  const int nf = a.nf, npi = a.npi;
  const int q1[3] = {a.qd[0] + 1, a.qd[1] + 1, a.qd[2] + 1};
  const double *Pk[3] = {a.fP3, a.fP3 + q1[0] * nf, a.fP3 + (q1[0] + q1[1]) * nf};
  const int tt[3] = {(int)(t % a.tiles[0]), (int)((t / a.tiles[0]) % a.tiles[1]),
                     (int)(t / ((int64_t)a.tiles[0] * a.tiles[1]))};
  const double ax[3] = {a.box_a[0][tt[0]], a.box_a[1][tt[1]], a.box_a[2][tt[2]]};
  const double hx[3] = {a.box_h[0][tt[0]], a.box_h[1][tt[1]], a.box_h[2][tt[2]]};
  double *co = a.coef + t * (int64_t)kLoadSlots * 3 * npi;
  // body samples: the spans and 1-D B-spline values and derivatives at the nodes of each direction,
  // one thread each, shared by the samples (the values spline_jacobian3 would compute per sample)
  __shared__ double NB[3][kMaxFit][2][PMX + 1];
  __shared__ int SP[3][kMaxFit];
  if (tid < 3 * nf) {
    const int d = tid / nf, m = tid - d * nf;
    const double x = (d == 0 ? ax[0] : d == 1 ? ax[1] : ax[2]) + (d == 0 ? hx[0] : d == 1 ? hx[1] : hx[2]) * a.fx[m];
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
  const int ns = nf * nf * nf;
  for (int s = tid; s < ns; s += 64) {
    const int si[3] = {s % nf, (s / nf) % nf, s / (nf * nf)};
    double J[3][3], N[3][PMX + 1], dN[3][PMX + 1];
    int span[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      span[k] = SP[k][si[k]];
#pragma unroll
      for (int r = 0; r <= PMX; ++r) {
        N[k][r] = NB[k][si[k]][0][r];
        dN[k][r] = NB[k][si[k]][1][r];
      }
    }
    spline_jacobian_sum<P0, P1, P2, true>(a.nM, a.ctrl, a.wts, span, N, dN, J);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int k = 0; k < 3; ++k) J[c][k] *= hx[k];
    const double D = det3(J);
    if (!(D > 0.0) || !isfinite(D)) atomicMin(a.flag, (int32_t)t);
    vals[s] = fabs(D);
  }
  __syncthreads();
  for (int e = tid; e < 3 * npi; e += 64) {
    const int comp = e / npi, C = e - comp * npi;
    const int c1 = C % q1[0], c2 = (C / q1[0]) % q1[1], c3 = C / (q1[0] * q1[1]);
    double v = 0.0;
    for (int s3 = 0, s = 0; s3 < nf; ++s3)   // s = s1 + nf (s2 + nf s3), ascending
      for (int s2 = 0; s2 < nf; ++s2)
        for (int s1 = 0; s1 < nf; ++s1, ++s)
          v += Pk[0][c1 * nf + s1] * Pk[1][c2 * nf + s2] * Pk[2][c3 * nf + s3] * vals[s];
    co[e] = a.body[comp] * v;
  }
  // faces
  for (int f = 0; f < 6; ++f) {
    const int d = f >> 1, side = f & 1;
    const int u = d == 0 ? 1 : 0, v = d == 2 ? 1 : 2;
    double *cf = co + (int64_t)(1 + f) * 3 * npi;
    const bool touched = tt[d] == (side ? a.tiles[d] - 1 : 0);
    __syncthreads();   // vals is reused
    if (touched) {
      for (int s = tid; s < nf * nf; s += 64) {
        const int su = s % nf, sv = s / nf;
        double xh[3];
        xh[d] = ax[d] + hx[d] * side;
        xh[u] = ax[u] + hx[u] * a.fx[su];
        xh[v] = ax[v] + hx[v] * a.fx[sv];
        double J[3][3], N[3][PMX + 1], dN[3][PMX + 1];
        int span[3];
        spline_jacobian3<P0, P1, P2, true>(a.knots, a.nM, a.ctrl, a.wts, xh, J, span, N, dN);
        const double gu[3] = {J[0][u] * hx[u], J[1][u] * hx[u], J[2][u] * hx[u]};
        const double gv[3] = {J[0][v] * hx[v], J[1][v] * hx[v], J[2][v] * hx[v]};
        const double n0 = gu[1] * gv[2] - gu[2] * gv[1], n1 = gu[2] * gv[0] - gu[0] * gv[2],
                     n2 = gu[0] * gv[1] - gu[1] * gv[0];
        vals[s] = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
      }
    }
    __syncthreads();
    for (int e = tid; e < 3 * npi; e += 64) {
      const int comp = e / npi, C = e - comp * npi;
      const int c[3] = {C % q1[0], (C / q1[0]) % q1[1], C / (q1[0] * q1[1])};
      double r = 0.0;
      if (touched && c[d] == (side ? a.qd[d] : 0)) {
        for (int sv = 0, s = 0; sv < nf; ++sv)   // s = su + nf sv, ascending
          for (int su = 0; su < nf; ++su, ++s) r += Pk[u][c[u] * nf + su] * Pk[v][c[v] * nf + sv] * vals[s];
        r *= a.traction[f][comp];
      }
      cf[e] = r;
    }
  }
}

struct LoadGatherArgs {
  const double *table;       // [nTt][npi][7]
  const double *coef;        // [n_tiles][7][3][npi]
  int nT[3], tiles[3], npi;
  int64_t n_global;
  int GX, GY;
  double *f;                 // [3 n_global]
};

__global__ __launch_bounds__(256) void load_gather_kernel(LoadGatherArgs a) {
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (id >= 3 * a.n_global) return;
  const int comp = (int)(id % 3);
  const int64_t G = id / 3;
  const int g[3] = {(int)(G % a.GX), (int)((G / a.GX) % a.GY), (int)(G / ((int64_t)a.GX * a.GY))};
  int tlo[3], thi[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int m = a.nT[k] - 1;   // tile t holds global indices t m .. t m + m along k
    thi[k] = min(g[k] / m, a.tiles[k] - 1);
    tlo[k] = g[k] > 0 ? (g[k] - 1) / m : 0;
  }
  double sum = 0.0;
  for (int tz = tlo[2]; tz <= thi[2]; ++tz)
    for (int ty = tlo[1]; ty <= thi[1]; ++ty)
      for (int tx = tlo[0]; tx <= thi[0]; ++tx) {
        const int tt[3] = {tx, ty, tz};
        const int64_t t = tx + (int64_t)a.tiles[0] * (ty + (int64_t)a.tiles[1] * tz);
        const int li[3] = {g[0] - tx * (a.nT[0] - 1), g[1] - ty * (a.nT[1] - 1), g[2] - tz * (a.nT[2] - 1)};
        const int64_t A = li[0] + (int64_t)a.nT[0] * (li[1] + (int64_t)a.nT[1] * li[2]);
        const double *tb = a.table + A * a.npi * kLoadSlots;
        const double *co = a.coef + t * (int64_t)kLoadSlots * 3 * a.npi + (int64_t)comp * a.npi;
        for (int slot = 0; slot < kLoadSlots; ++slot) {
          if (slot > 0) {
            const int f = slot - 1, d = f >> 1, side = f & 1;
            if (tt[d] != (side ? a.tiles[d] - 1 : 0)) continue;   // the tile does not touch face f
          }
          const double *cs = co + (int64_t)slot * 3 * a.npi;
          // unrolled so that the loads run ahead of the (sequential, fixed-order) sum
#pragma unroll 9
          for (int C = 0; C < a.npi; ++C) sum += cs[C] * tb[C * kLoadSlots + slot];
        }
      }
  a.f[id] = sum;
}

// ---- shape derivative of the external work u . f^pi (eq. (69) through eq. (40)-(41), (44)-(45)) ----
// For a fixed vector u, per tile t:
//   y[slot][C] = sum_A (l_slot . u_A) F[A][C][slot]      (l_0 = b, l_(1+f) = t_f: the lookup's adjoint)
//   body:  gbar[s] = sum_C P3[C][s] y[0][C],  d(u.f)/dJs = gbar[s] d|det Js|/dJs = gbar[s] sign(D) cof(Js)
//   face f (normal d, in-face axes u, v): abar[s] = sum_(cu,cv) Pu[cu][su] Pv[cv][sv] y[1+f][C(cu,cv)],
//          with n = g_u x g_v (g_k = Js e_k) and area = |n|:
//          d area/d g_u = (g_v x n) / area,  d area/d g_v = (n x g_u) / area
// (Js = J_M(a + h xi) diag(h)); the chain through Js = J_M diag(h) scales column n by h_n, and
// dJ_M[c][n]/dm_(i,c) = d_n R_i(x) gives the tile's local control-point gradients over the body
// samples and the face samples, reduced over the tiles in a fixed order afterwards.
// u . f^(t) itself is sum_s gbar[s] |D_s| + sum_faces sum_s abar[s] area_s.
struct LoadAdjArgs {
  const double *knots[3];
  int nM[3];
  const double *ctrl;
  const double *wts;         // NURBS weights of the macro map, or null (B-spline)
  const double *box_a[3];
  const double *box_h[3];
  const int32_t *ctrl_lo[3];
  int tiles[3], Lc[3], Lm;
  int nT[3], NG[3];
  const double *fx;
  const double *fP3;         // per-direction 1-D projection operators [qd[k]+1][n_fit], concatenated
  int qd[3], nf, npi;
  double body[3];
  double traction[6][3];
  const double *table;       // [nTt][npi][7]
  const double *u;           // [3 n_global]
  double *local_grad;        // [n_tiles][Lz][Ly][Lx][3]
  double *uf_part;           // [n_tiles]
  int32_t *flag;
};

constexpr int kLoadAdjThreads = 64;
constexpr int kAbsc = kMaxFit + 2;   // per direction: the n_fit nodes, then the box ends 0 and 1

__host__ __device__ inline int64_t load_adj_lds_doubles(int nTt, int npi, int nf, int Lm) {
  const int64_t S = (int64_t)nf * nf * nf + 6 * (int64_t)nf * nf;
  return (int64_t)kLoadSlots * nTt + (int64_t)kLoadSlots * npi + S * (1 + 9 + 4) + 2 * 3 * (int64_t)(nf + 2) * Lm +
         kLoadAdjThreads;
}

template <int P0, int P1, int P2>
__global__ __launch_bounds__(kLoadAdjThreads) void load_adjoint_kernel(LoadAdjArgs a) {
  constexpr int PMX = max3(P0, P1, P2);
  constexpr int PD[3] = {P0, P1, P2};
  extern __shared__ double smem[];
  __shared__ double NB[3][kAbsc][kMaxDegree + 1], DB[3][kAbsc][kMaxDegree + 1];
  __shared__ int SP[3][kAbsc];
  const int tid = threadIdx.x;
  const int64_t t = blockIdx.x;
  const int nf = a.nf, npi = a.npi, Lm = a.Lm;
  const int nTt = a.nT[0] * a.nT[1] * a.nT[2];
  const int ns = nf * nf * nf, S = ns + 6 * nf * nf;
  double *UB = smem;                       // [7][nTt]  l_slot . u_A
  double *Y = UB + kLoadSlots * nTt;       // [7][npi]
  double *SV = Y + kLoadSlots * npi;       // [S]       gbar / abar per sample
  double *JH = SV + S;                     // [S][9]    d(u.f)/dJ_M per sample (columns scaled by h)
  double *WQ = JH + 9 * S;                 // [S][4]    NURBS terms
  double *XV = WQ + 4 * S;                 // [3][nf+2][Lm]
  double *XD = XV + 3 * (nf + 2) * Lm;     // [3][nf+2][Lm]
  double *RED = XD + 3 * (nf + 2) * Lm;    // [64]
  const int q1[3] = {a.qd[0] + 1, a.qd[1] + 1, a.qd[2] + 1};
  const double *Pk[3] = {a.fP3, a.fP3 + q1[0] * nf, a.fP3 + (q1[0] + q1[1]) * nf};
  const int tt[3] = {(int)(t % a.tiles[0]), (int)((t / a.tiles[0]) % a.tiles[1]),
                     (int)(t / ((int64_t)a.tiles[0] * a.tiles[1]))};
  const double ax[3] = {a.box_a[0][tt[0]], a.box_a[1][tt[1]], a.box_a[2][tt[2]]};
  const double hx[3] = {a.box_h[0][tt[0]], a.box_h[1][tt[1]], a.box_h[2][tt[2]]};
  int tmask = 0;   // bit f: the tile touches macro face f
#pragma unroll
  for (int f = 0; f < 6; ++f) tmask |= (tt[f >> 1] == ((f & 1) ? a.tiles[f >> 1] - 1 : 0)) << f;
  auto touched = [&](int f) { return (tmask >> f) & 1; };
  // 1-D macro basis at the abscissae of every direction: the fit nodes, then the box ends
  for (int e = tid; e < 3 * (nf + 2); e += kLoadAdjThreads) {
    const int k = e / (nf + 2), s = e % (nf + 2);
    const double xi = s < nf ? a.fx[s] : (double)(s - nf);
    const double x = ax[k] + hx[k] * xi;
    const int sp = find_span(a.knots[k], a.nM[k], PD[k], x);
    double N[PMX + 1], dN[PMX + 1];
    bspline_ders_dir<P0, P1, P2>(k, a.knots[k], sp, x, N, dN);
    SP[k][s] = sp;
    for (int r = 0; r <= PMX; ++r) { NB[k][s][r] = N[r]; DB[k][s][r] = dN[r]; }
  }
  // the loads paired with the tile's displacement
  for (int A = tid; A < nTt; A += kLoadAdjThreads) {
    const int ai[3] = {A % a.nT[0], (A / a.nT[0]) % a.nT[1], A / (a.nT[0] * a.nT[1])};
    const int64_t G = (tt[0] * (a.nT[0] - 1) + ai[0]) +
                      (int64_t)a.NG[0] * ((tt[1] * (a.nT[1] - 1) + ai[1]) + (int64_t)a.NG[1] * (tt[2] * (a.nT[2] - 1) + ai[2]));
    const double uA[3] = {a.u[3 * G], a.u[3 * G + 1], a.u[3 * G + 2]};
    UB[A] = a.body[0] * uA[0] + a.body[1] * uA[1] + a.body[2] * uA[2];
    for (int f = 0; f < 6; ++f)
      UB[(1 + f) * nTt + A] = a.traction[f][0] * uA[0] + a.traction[f][1] * uA[1] + a.traction[f][2] * uA[2];
  }
  __syncthreads();
  // y[slot][C] = sum_A UB[slot][A] F[A][C][slot] (A ascending)
  for (int e = tid; e < kLoadSlots * npi; e += kLoadAdjThreads) {
    const int slot = e / npi, C = e - slot * npi;
    double v = 0.0;
    if (slot == 0 || touched(slot - 1))
      for (int A = 0; A < nTt; ++A) v += UB[slot * nTt + A] * a.table[((int64_t)A * npi + C) * kLoadSlots + slot];
    Y[e] = v;
  }
  __syncthreads();
  double part = 0.0;
  // body samples
  for (int s = tid; s < ns; s += kLoadAdjThreads) {
    const int si[3] = {s % nf, (s / nf) % nf, s / (nf * nf)};
    double gbar = 0.0;
    for (int c3 = 0, C = 0; c3 < q1[2]; ++c3)
      for (int c2 = 0; c2 < q1[1]; ++c2)
        for (int c1 = 0; c1 < q1[0]; ++c1, ++C)
          gbar += Pk[0][c1 * nf + si[0]] * Pk[1][c2 * nf + si[1]] * Pk[2][c3 * nf + si[2]] * Y[C];
    const double xh[3] = {ax[0] + hx[0] * a.fx[si[0]], ax[1] + hx[1] * a.fx[si[1]], ax[2] + hx[2] * a.fx[si[2]]};
    double J[3][3], N[3][PMX + 1], dN[3][PMX + 1];
    int span[3];
    spline_jacobian3<P0, P1, P2, true>(a.knots, a.nM, a.ctrl, a.wts, xh, J, span, N, dN);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int k = 0; k < 3; ++k) J[c][k] *= hx[k];
    const double D = det3(J);
    if (!(D > 0.0) || !isfinite(D)) atomicMin(a.flag, (int32_t)t);
    const double sg = D < 0.0 ? -1.0 : 1.0;
    // cofactors: d det / dJ[c][n]
    const double cof[3][3] = {{J[1][1] * J[2][2] - J[1][2] * J[2][1], J[1][2] * J[2][0] - J[1][0] * J[2][2],
                               J[1][0] * J[2][1] - J[1][1] * J[2][0]},
                              {J[0][2] * J[2][1] - J[0][1] * J[2][2], J[0][0] * J[2][2] - J[0][2] * J[2][0],
                               J[0][1] * J[2][0] - J[0][0] * J[2][1]},
                              {J[0][1] * J[1][2] - J[0][2] * J[1][1], J[0][2] * J[1][0] - J[0][0] * J[1][2],
                               J[0][0] * J[1][1] - J[0][1] * J[1][0]}};
    SV[s] = gbar;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int n = 0; n < 3; ++n) JH[s * 9 + 3 * c + n] = gbar * sg * cof[c][n] * hx[n];
    part += gbar * fabs(D);
  }
  // face samples of the touched faces
  for (int f = 0; f < 6; ++f) {
    if (!touched(f)) continue;
    const int d = f >> 1, side = f & 1;
    const int u = d == 0 ? 1 : 0, v = d == 2 ? 1 : 2;
    const double *yf = Y + (1 + f) * npi;
    for (int sl = tid; sl < nf * nf; sl += kLoadAdjThreads) {
      const int su = sl % nf, sv = sl / nf, s = ns + f * nf * nf + sl;
      double abar = 0.0;
      for (int cv = 0; cv < q1[v]; ++cv)
        for (int cu = 0; cu < q1[u]; ++cu) {
          int c[3];
          c[d] = side ? a.qd[d] : 0;
          c[u] = cu;
          c[v] = cv;
          abar += Pk[u][cu * nf + su] * Pk[v][cv * nf + sv] * yf[c[0] + q1[0] * (c[1] + q1[1] * c[2])];
        }
      double xh[3];
      xh[d] = ax[d] + hx[d] * side;
      xh[u] = ax[u] + hx[u] * a.fx[su];
      xh[v] = ax[v] + hx[v] * a.fx[sv];
      double J[3][3], N[3][PMX + 1], dN[3][PMX + 1];
      int span[3];
      spline_jacobian3<P0, P1, P2, true>(a.knots, a.nM, a.ctrl, a.wts, xh, J, span, N, dN);
      const double gu[3] = {J[0][u] * hx[u], J[1][u] * hx[u], J[2][u] * hx[u]};
      const double gv[3] = {J[0][v] * hx[v], J[1][v] * hx[v], J[2][v] * hx[v]};
      const double n[3] = {gu[1] * gv[2] - gu[2] * gv[1], gu[2] * gv[0] - gu[0] * gv[2], gu[0] * gv[1] - gu[1] * gv[0]};
      const double area = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      const double r = area > 0.0 ? abar / area : 0.0;
      // (g_v x n) and (n x g_u)
      const double du[3] = {gv[1] * n[2] - gv[2] * n[1], gv[2] * n[0] - gv[0] * n[2], gv[0] * n[1] - gv[1] * n[0]};
      const double dv[3] = {n[1] * gu[2] - n[2] * gu[1], n[2] * gu[0] - n[0] * gu[2], n[0] * gu[1] - n[1] * gu[0]};
      SV[s] = abar;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        JH[s * 9 + 3 * c + d] = 0.0;
        JH[s * 9 + 3 * c + u] = r * du[c] * hx[u];
        JH[s * 9 + 3 * c + v] = r * dv[c] * hx[v];
      }
      part += abar * area;
    }
  }
  RED[tid] = part;
  __syncthreads();
  for (int w = kLoadAdjThreads / 2; w > 0; w >>= 1) {
    if (tid < w) RED[tid] += RED[tid + w];
    __syncthreads();
  }
  if (tid == 0) a.uf_part[t] = RED[0];
  // NURBS: 1 / W and sum_n JH[c][n] d_n W / W^2 per sample
  auto sample_index = [&](int s, int (&si)[3]) {
    if (s < ns) {
      si[0] = s % nf; si[1] = (s / nf) % nf; si[2] = s / (nf * nf);
    } else {
      const int f = (s - ns) / (nf * nf), sl = (s - ns) - f * nf * nf, d = f >> 1;
      const int u = d == 0 ? 1 : 0, v = d == 2 ? 1 : 2;
      si[d] = nf + (f & 1);
      si[u] = sl % nf;
      si[v] = sl / nf;
    }
  };
  if (a.wts) {
    for (int s = tid; s < S; s += kLoadAdjThreads) {
      if (s >= ns && !touched((s - ns) / (nf * nf))) continue;
      int si[3];
      sample_index(s, si);
      rational_terms3<P0, P1, P2>(a.wts, a.nM, SP, NB, DB, si, JH + s * 9, WQ + s * 4);
    }
  }
  // per-direction factor tables: XV[k][s][l] = N_r(x_s), XD = N_r'(x_s), r the local function l's
  // index on the sample's span (zero outside its support)
  const int L0 = a.Lc[0], L1 = a.Lc[1], L2 = a.Lc[2];
  const int lo[3] = {a.ctrl_lo[0][tt[0]], a.ctrl_lo[1][tt[1]], a.ctrl_lo[2][tt[2]]};
  for (int e = tid; e < 3 * (nf + 2) * Lm; e += kLoadAdjThreads) {
    const int k = e / ((nf + 2) * Lm), rem = e - k * (nf + 2) * Lm, sk = rem / Lm, l = rem - sk * Lm;
    const int r = lo[k] + l - (SP[k][sk] - PD[k]);
    const bool on = r >= 0 && r <= PD[k];
    const int rc = on ? r : 0;
    XV[e] = on ? NB[k][sk][rc] : 0.0;
    XD[e] = on ? DB[k][sk][rc] : 0.0;
  }
  __syncthreads();
  double *lg = a.local_grad + t * (int64_t)L0 * L1 * L2 * 3;
  const int na = nf + 2;
  for (int e = tid; e < L0 * L1 * L2 * 3; e += kLoadAdjThreads) {
    const int c = e % 3, li = e / 3;
    const int l[3] = {li % L0, (li / L0) % L1, li / (L0 * L1)};
    auto term = [&](int s, const int (&si)[3]) {
      const double v0 = XV[(0 * na + si[0]) * Lm + l[0]], d0 = XD[(0 * na + si[0]) * Lm + l[0]];
      const double v1 = XV[(1 * na + si[1]) * Lm + l[1]], d1 = XD[(1 * na + si[1]) * Lm + l[1]];
      const double v2 = XV[(2 * na + si[2]) * Lm + l[2]], d2 = XD[(2 * na + si[2]) * Lm + l[2]];
      const double *jb = JH + s * 9 + 3 * c;
      const double tb = jb[0] * d0 * v1 * v2 + jb[1] * v0 * d1 * v2 + jb[2] * v0 * v1 * d2;
      return a.wts ? tb * WQ[s * 4] - v0 * v1 * v2 * WQ[s * 4 + 1 + c] : tb;
    };
    double g = 0.0;
    for (int s = 0; s < S; ++s) {
      if (s >= ns && !touched((s - ns) / (nf * nf))) { s += nf * nf - 1; continue; }
      int si[3];
      sample_index(s, si);
      g += term(s, si);
    }
    lg[e] = a.wts ? g * local_weight(a.wts, a.nM, lo, l)
                  : g;
  }
}

}  // namespace igamt

using namespace igamt;

static igamt_status load_fit_launch(igamt_plan *P, const double *body, const double *traction, double *d_coef,
                                    hipStream_t s) {
  LoadFitArgs a;
  for (int k = 0; k < 3; ++k) {
    a.knots[k] = P->dev.macro_knots[k];
    a.nM[k] = P->nM[k];
    a.box_a[k] = P->dev.box_a[k];
    a.box_h[k] = P->dev.box_h[k];
    a.tiles[k] = P->tiles[k];
    a.body[k] = body[k];
  }
  for (int f = 0; f < 6; ++f)
    for (int k = 0; k < 3; ++k) a.traction[f][k] = traction[3 * f + k];
  a.ctrl = P->dev.macro_ctrl;
  a.wts = P->dev.macro_w;
  a.n_tiles = P->n_tiles;
  a.fx = P->dev.fit_x;
  a.fP3 = P->dev.fit_P3;
  for (int k = 0; k < 3; ++k) a.qd[k] = P->qd[k];
  a.nf = P->n_fit;
  a.npi = P->npi;
  a.coef = d_coef;
  a.flag = P->dev.flag;
  const dim3 grid((unsigned)P->n_tiles), block(64);
  switch (IGAMT_DEGREE_KEY(P->pM[0], P->pM[1], P->pM[2])) {
#define LF_CASE(p0, p1, p2)                                                                               \
  case IGAMT_DEGREE_KEY(p0, p1, p2): hipLaunchKernelGGL((load_fit_kernel<p0, p1, p2>), grid, block, 0, s, a); break;
    IGAMT_FOR_MACRO_DEGREES(LF_CASE)
#undef LF_CASE
    default: set_error("unsupported macro degrees (isotropic 1..6, or 1..3 per direction)"); return IGAMT_EUNSUPPORTED;
  }
  IGAMT_LAUNCH_CHECK();
  return IGAMT_OK;
}

static bool finite_loads(const double *body, const double *traction) {
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(body[k])) return false;
  for (int k = 0; k < 18; ++k)
    if (!std::isfinite(traction[k])) return false;
  return true;
}

extern "C" igamt_status igamt_load_table_build(igamt_plan *P, void *stream) {
  if (!P) { set_error("NULL argument"); return IGAMT_EINVAL; }
  igamt_status st = ensure_device(P);
  if (st) return st;
  if (P->pT[0] != P->pT[1] || P->pT[0] != P->pT[2]) {
    set_error("reference tiles with different degrees per direction are not supported");
    return IGAMT_EUNSUPPORTED;
  }
  hipStream_t s = (hipStream_t)stream;
  int64_t stride = 0;
  if ((st = table_point_records(P, s, stride))) return st;
  if (!P->dev.load_table) IGAMT_HIP(hipMalloc((void **)&P->dev.load_table, P->nTt * P->npi * kLoadSlots * sizeof(double)));
  LoadTableArgs a;
  for (int k = 0; k < 3; ++k) {
    a.knots[k] = P->dev.tile_knots[k];
    a.nT[k] = P->nT[k];
    a.eT[k] = P->eT[k];
  }
  a.gx = P->dev.gauss_x;
  a.gw = P->dev.gauss_w;
  a.ng = P->n_gauss;
  for (int k = 0; k < 3; ++k) a.qd[k] = P->qd[k];
  a.npi = P->npi;
  a.stride = stride;
  a.pts = P->dev.point_data;
  a.table = P->dev.load_table;
  const dim3 grid((unsigned)((P->nTt * P->npi + 63) / 64)), block(64);
  switch (P->pT[0]) {
    case 1: hipLaunchKernelGGL(load_table_kernel<1>, grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL(load_table_kernel<2>, grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL(load_table_kernel<3>, grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL(load_table_kernel<4>, grid, block, 0, s, a); break;
    case 5: hipLaunchKernelGGL(load_table_kernel<5>, grid, block, 0, s, a); break;
    case 6: hipLaunchKernelGGL(load_table_kernel<6>, grid, block, 0, s, a); break;
    default: set_error("unsupported tile degree"); return IGAMT_EUNSUPPORTED;
  }
  IGAMT_LAUNCH_CHECK();
  P->load_table_ready = true;
  return IGAMT_OK;
}

extern "C" igamt_status igamt_load_table_get(const igamt_plan *P, double *d_out, void *stream) {
  if (!P || !d_out) { set_error("NULL argument"); return IGAMT_EINVAL; }
  if (!P->dev.ready || !P->load_table_ready) { set_error("load table not built"); return IGAMT_ESTATE; }
  IGAMT_HIP(hipMemcpyAsync(d_out, P->dev.load_table, P->nTt * P->npi * kLoadSlots * sizeof(double),
                           hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return IGAMT_OK;
}

extern "C" igamt_status igamt_load_workspace_bytes(const igamt_plan *P, int64_t *bytes) {
  if (!P || !bytes) { set_error("NULL argument"); return IGAMT_EINVAL; }
  *bytes = align256(P->n_tiles * kLoadSlots * 3 * P->npi * (int64_t)sizeof(double));
  return IGAMT_OK;
}

extern "C" igamt_status igamt_load_fit(igamt_plan *P, const double *body, const double *traction, double *d_coef,
                                       void *stream) {
  if (!P || !body || !traction || !d_coef) { set_error("NULL argument"); return IGAMT_EINVAL; }
  if (!finite_loads(body, traction)) { set_error("non-finite body force or traction"); return IGAMT_EINVAL; }
  igamt_status st = ensure_device(P);
  if (st) return st;
  return load_fit_launch(P, body, traction, d_coef, (hipStream_t)stream);
}

extern "C" igamt_status igamt_load_gather(igamt_plan *P, const double *d_coef, double *d_f, void *stream) {
  if (!P || !d_coef || !d_f) { set_error("NULL argument"); return IGAMT_EINVAL; }
  igamt_status st = ensure_device(P);
  if (st) return st;
  if (!P->load_table_ready) { set_error("load table not built"); return IGAMT_ESTATE; }
  LoadGatherArgs a;
  a.table = P->dev.load_table;
  a.coef = d_coef;
  for (int k = 0; k < 3; ++k) {
    a.nT[k] = P->nT[k];
    a.tiles[k] = P->tiles[k];
  }
  a.npi = P->npi;
  a.n_global = P->n_global;
  a.GX = P->dir[0].NG;
  a.GY = P->dir[1].NG;
  a.f = d_f;
  hipLaunchKernelGGL(load_gather_kernel, dim3((unsigned)((3 * P->n_global + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, a);
  IGAMT_LAUNCH_CHECK();
  return IGAMT_OK;
}

extern "C" igamt_status igamt_load_assemble(igamt_plan *P, const double *body, const double *traction, double *d_f,
                                            void *d_workspace, void *stream) {
  if (!P || !body || !traction || !d_f || !d_workspace) { set_error("NULL argument"); return IGAMT_EINVAL; }
  igamt_status st;
  if ((st = igamt_load_fit(P, body, traction, (double *)d_workspace, stream))) return st;
  return igamt_load_gather(P, (const double *)d_workspace, d_f, stream);
}

static int64_t uf_grad_ws_layout(const igamt_plan *P, int64_t off[3]) {
  off[0] = 0;                                                                                   // local gradients
  off[1] = off[0] + align256(P->n_tiles * (int64_t)P->Lc[0] * P->Lc[1] * P->Lc[2] * 3 * sizeof(double));
  off[2] = off[1] + align256(P->n_tiles * (int64_t)sizeof(double));                             // tile shares
  return off[2];
}

extern "C" igamt_status igamt_uf_grad_workspace_bytes(const igamt_plan *P, int64_t *bytes) {
  if (!P || !bytes) { set_error("NULL argument"); return IGAMT_EINVAL; }
  int64_t off[3];
  *bytes = uf_grad_ws_layout(P, off);
  return IGAMT_OK;
}

extern "C" igamt_status igamt_uf_grad(igamt_plan *P, const double *body, const double *traction, const double *d_u,
                                      double *d_grad, double *d_uf, void *d_workspace, void *stream) {
  if (!P || !body || !traction || !d_u || !d_grad || !d_workspace) { set_error("NULL argument"); return IGAMT_EINVAL; }
  if (!finite_loads(body, traction)) { set_error("non-finite body force or traction"); return IGAMT_EINVAL; }
  igamt_status st = ensure_device(P);
  if (st) return st;
  if (!P->load_table_ready) { set_error("load table not built"); return IGAMT_ESTATE; }
  hipStream_t s = (hipStream_t)stream;
  int64_t off[3];
  uf_grad_ws_layout(P, off);
  char *ws = (char *)d_workspace;
  LoadAdjArgs a;
  for (int k = 0; k < 3; ++k) {
    a.knots[k] = P->dev.macro_knots[k];
    a.nM[k] = P->nM[k];
    a.box_a[k] = P->dev.box_a[k];
    a.box_h[k] = P->dev.box_h[k];
    a.ctrl_lo[k] = P->dev.ctrl_lo[k];
    a.tiles[k] = P->tiles[k];
    a.Lc[k] = P->Lc[k];
    a.nT[k] = P->nT[k];
    a.NG[k] = P->dir[k].NG;
    a.qd[k] = P->qd[k];
    a.body[k] = body[k];
  }
  for (int f = 0; f < 6; ++f)
    for (int k = 0; k < 3; ++k) a.traction[f][k] = traction[3 * f + k];
  a.Lm = std::max(P->Lc[0], std::max(P->Lc[1], P->Lc[2]));
  a.ctrl = P->dev.macro_ctrl;
  a.wts = P->dev.macro_w;
  a.fx = P->dev.fit_x;
  a.fP3 = P->dev.fit_P3;
  a.nf = P->n_fit;
  a.npi = P->npi;
  a.table = P->dev.load_table;
  a.u = d_u;
  a.local_grad = (double *)(ws + off[0]);
  a.uf_part = (double *)(ws + off[1]);
  a.flag = P->dev.flag;
  const size_t shm = (size_t)load_adj_lds_doubles((int)P->nTt, P->npi, P->n_fit, a.Lm) * sizeof(double);
  if (shm > 150 * 1024) { set_error("tile control points or fit samples too many for the load adjoint"); return IGAMT_EUNSUPPORTED; }
  const dim3 grid((unsigned)P->n_tiles), block(kLoadAdjThreads);
  switch (IGAMT_DEGREE_KEY(P->pM[0], P->pM[1], P->pM[2])) {
#define LA_CASE(p0, p1, p2)                                                                             \
  case IGAMT_DEGREE_KEY(p0, p1, p2):                                                                    \
    if (shm > 65536) IGAMT_HIP(hipFuncSetAttribute((const void *)load_adjoint_kernel<p0, p1, p2>,       \
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm)); \
    hipLaunchKernelGGL((load_adjoint_kernel<p0, p1, p2>), grid, block, shm, s, a);                      \
    break;
    IGAMT_FOR_MACRO_DEGREES(LA_CASE)
#undef LA_CASE
    default: set_error("unsupported macro degrees (isotropic 1..6, or 1..3 per direction)"); return IGAMT_EUNSUPPORTED;
  }
  IGAMT_LAUNCH_CHECK();
  if ((st = launch_grad_reduce(P, (const double *)(ws + off[0]), d_grad, stream))) return st;
  if (d_uf && (st = launch_sum((const double *)(ws + off[1]), P->n_tiles, d_uf, stream))) return st;
  return IGAMT_OK;
}
