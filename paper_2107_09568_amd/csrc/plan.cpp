// Host side of libigamt: validation and the integer set-up of a plan.
//
// Everything here is integer work or tiny dense algebra done once per
// topology: tile boxes (eq. (5)-(8)), the pair set I_coo (eq. (56)), the glued
// numbering of tile control points, the CSR structure of K, the 1-D Gauss rule
// and the 1-D projection operator of eq. (23)-(24).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "igamt_internal.h"

namespace igamt {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

// Gauss-Legendre rule on [0, 1]: Newton iteration on the Legendre polynomial
// P_n from the usual cosine initial guesses, weights 2 / ((1 - x^2) P_n'(x)^2)
// on [-1, 1], then the affine map to [0, 1].  Nodes ascending.
void gauss_legendre01(int n, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
    }
    x[i] = 0.5 * (1.0 - z);   // cos guesses are descending in z; 1 - z ascending
    w[i] = 1.0 / ((1.0 - z * z) * dp * dp);   // 2/((1-z^2)P'^2) halved for [0,1]
  }
}

int find_span_host(const std::vector<double> &U, int n, int p, double x) {
  if (x >= U[n]) return n - 1;
  if (x <= U[p]) return p;
  int lo = p, hi = n;
  while (hi - lo > 1) {
    int mid = (lo + hi) / 2;
    if (x < U[mid]) hi = mid; else lo = mid;
  }
  return lo;
}

static double binom(int n, int k) {
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// Solve (V^T W V) P = V^T W for the 1-D projection operator P ((q+1) x n).
bool projection_1d(int q, const std::vector<double> &x, const std::vector<double> &w, std::vector<double> &P) {
  const int m = q + 1, n = (int)x.size();
  std::vector<double> V(n * m);
  for (int s = 0; s < n; ++s)
    for (int c = 0; c < m; ++c)
      V[s * m + c] = binom(q, c) * std::pow(x[s], c) * std::pow(1.0 - x[s], q - c);
  std::vector<double> M(m * m, 0.0), R(m * n, 0.0);
  for (int a = 0; a < m; ++a)
    for (int b = 0; b < m; ++b)
      for (int s = 0; s < n; ++s) M[a * m + b] += V[s * m + a] * w[s] * V[s * m + b];
  for (int a = 0; a < m; ++a)
    for (int s = 0; s < n; ++s) R[a * n + s] = V[s * m + a] * w[s];
  // Gaussian elimination with partial pivoting on [M | R]
  for (int col = 0; col < m; ++col) {
    int piv = col;
    for (int r = col + 1; r < m; ++r)
      if (std::fabs(M[r * m + col]) > std::fabs(M[piv * m + col])) piv = r;
    if (std::fabs(M[piv * m + col]) < 1e-300) return false;
    if (piv != col) {
      for (int c = 0; c < m; ++c) std::swap(M[col * m + c], M[piv * m + c]);
      for (int c = 0; c < n; ++c) std::swap(R[col * n + c], R[piv * n + c]);
    }
    for (int r = 0; r < m; ++r) {
      if (r == col) continue;
      double f = M[r * m + col] / M[col * m + col];
      for (int c = 0; c < m; ++c) M[r * m + c] -= f * M[col * m + c];
      for (int c = 0; c < n; ++c) R[r * n + c] -= f * R[col * n + c];
    }
  }
  P.assign(m * n, 0.0);
  for (int a = 0; a < m; ++a)
    for (int s = 0; s < n; ++s) P[a * n + s] = R[a * n + s] / M[a * m + a];
  return true;
}

static igamt_status check_spline(const igamt_spline3d *s, const char *what, int *p, int *n,
                                 std::vector<double> *k, std::vector<double> &ctrl) {
  if (!s || !s->ctrl) { set_error(std::string(what) + ": NULL spline"); return IGAMT_EINVAL; }
  int64_t total = 1;
  for (int d = 0; d < 3; ++d) {
    p[d] = s->degree[d];
    n[d] = s->n_ctrl[d];
    if (p[d] < 1 || p[d] > kMaxDegree) {
      set_error(std::string(what) + ": degree must be in 1..6");
      return p[d] < 1 ? IGAMT_EINVAL : IGAMT_EUNSUPPORTED;
    }
    if (n[d] < p[d] + 1) { set_error(std::string(what) + ": need n_ctrl >= degree + 1"); return IGAMT_EINVAL; }
    if (!s->knots[d]) { set_error(std::string(what) + ": NULL knots"); return IGAMT_EINVAL; }
    const int nk = n[d] + p[d] + 1;
    k[d].assign(s->knots[d], s->knots[d] + nk);
    for (int i = 0; i < nk; ++i)
      if (!std::isfinite(k[d][i])) { set_error(std::string(what) + ": non-finite knot"); return IGAMT_EINVAL; }
    for (int i = 0; i + 1 < nk; ++i)
      if (k[d][i + 1] < k[d][i]) { set_error(std::string(what) + ": knots decrease"); return IGAMT_EINVAL; }
    for (int i = 0; i <= p[d]; ++i)
      if (k[d][i] != 0.0 || k[d][nk - 1 - i] != 1.0) {
        set_error(std::string(what) + ": knots must be clamped on [0, 1]");
        return IGAMT_EINVAL;
      }
    total *= n[d];
  }
  ctrl.assign(s->ctrl, s->ctrl + 3 * total);
  for (double v : ctrl)
    if (!std::isfinite(v)) { set_error(std::string(what) + ": non-finite control point"); return IGAMT_EINVAL; }
  return IGAMT_OK;
}

static std::vector<double> greville(const std::vector<double> &U, int p, int n) {
  std::vector<double> g(n);
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int j = 1; j <= p; ++j) s += U[i + j];
    g[i] = s / p;
  }
  return g;
}

static bool overlap1d(int i, int j, int p, int e) {
  // basis functions i, j of a clamped knot vector without repeated interior knots
  // are non-zero on elements [i - p, i] (clipped to [0, e - 1]); do they share one?
  int lo = std::max(std::max(i, j) - p, 0);
  int hi = std::min(std::min(i, j), e - 1);
  return lo <= hi;
}

}  // namespace igamt

using namespace igamt;

extern "C" const char *igamt_last_error(void) { return g_last_error.c_str(); }

static igamt_status build_plan(igamt_plan *P, const igamt_spline3d *macro, const igamt_spline3d *tile,
                               const igamt_plan_desc *desc) {
  igamt_status st = check_spline(macro, "macro", P->pM, P->nM, P->kM, P->ctrlM);
  if (st) return st;
  st = check_spline(tile, "tile", P->pT, P->nT, P->kT, P->ctrlT);
  if (st) return st;
  P->wM.clear();
  if (macro->weights) {   // NURBS macro map: positive, finite weights
    P->wM.assign(macro->weights, macro->weights + P->ctrlM.size() / 3);
    for (double v : P->wM)
      if (!(v > 0.0) || !std::isfinite(v)) { set_error("macro: NURBS weights must be positive and finite"); return IGAMT_EINVAL; }
  }
  if (tile->weights) {
    set_error("NURBS reference tiles are not supported (the tile is a B-spline)");
    return IGAMT_EUNSUPPORTED;
  }
  if (!desc) { set_error("NULL descriptor"); return IGAMT_EINVAL; }
  // tile knots: no repeated interior knots; elements per direction
  for (int d = 0; d < 3; ++d) {
    const auto &U = P->kT[d];
    const int p = P->pT[d], n = P->nT[d];
    for (int i = p + 1; i <= n; ++i)
      if (!(U[i] > U[i - 1])) {
        set_error("tile knots with repeated interior knots are not supported");
        return IGAMT_EUNSUPPORTED;
      }
    P->eT[d] = n - p;
    if (n > kMaxTileControl) {   // the scatter keeps a tile's slice of the 1-D tables in LDS
      set_error("tiles with more than 16 control points per direction are not supported");
      return IGAMT_EUNSUPPORTED;
    }
  }
  // tile boundary control points at the identity (Greville) positions
  {
    std::vector<double> g[3];
    for (int d = 0; d < 3; ++d) g[d] = greville(P->kT[d], P->pT[d], P->nT[d]);
    P->grevT.clear();
    for (int d = 0; d < 3; ++d) P->grevT.insert(P->grevT.end(), g[d].begin(), g[d].end());
    for (int k = 0; k < P->nT[2]; ++k)
      for (int j = 0; j < P->nT[1]; ++j)
        for (int i = 0; i < P->nT[0]; ++i) {
          bool bnd = i == 0 || j == 0 || k == 0 || i == P->nT[0] - 1 || j == P->nT[1] - 1 || k == P->nT[2] - 1;
          if (!bnd) continue;
          const double *c = &P->ctrlT[3 * (i + P->nT[0] * (j + P->nT[1] * k))];
          double e = std::fabs(c[0] - g[0][i]) + std::fabs(c[1] - g[1][j]) + std::fabs(c[2] - g[2][k]);
          if (e > 1e-12) {
            set_error("tile boundary control points must sit at the identity (Greville) positions");
            return IGAMT_EINVAL;
          }
        }
  }
  for (int d = 0; d < 3; ++d) P->tiles[d] = desc->tiles[d];
  P->box_mode = desc->box_mode;
  P->q = desc->q;
  P->n_fit = desc->n_fit;
  P->n_gauss = desc->n_gauss;
  int qmax = 0;
  for (int k = 0; k < 3; ++k) {
    P->qd[k] = desc->anisotropic ? desc->q_dir[k] : desc->q;
    if (P->qd[k] < 0 || P->qd[k] > kMaxQ) { set_error("projection degrees must be in 0..6"); return IGAMT_EUNSUPPORTED; }
    qmax = std::max(qmax, P->qd[k]);
  }
  P->aniso = P->qd[0] != P->qd[1] || P->qd[1] != P->qd[2];
  P->q = P->aniso ? qmax : P->qd[0];   // the isotropic degree (largest one when anisotropic)
  if (P->n_fit < qmax + 1 || P->n_fit > kMaxFit) { set_error("n_fit must be in max(q)+1..8"); return IGAMT_EINVAL; }
  if (P->n_gauss < 1 || P->n_gauss > kMaxGauss) { set_error("n_gauss must be in 1..8"); return IGAMT_EINVAL; }
  if (P->box_mode != 0 && P->box_mode != 1) { set_error("box_mode must be 0 or 1"); return IGAMT_EINVAL; }
  // tile boxes
  for (int d = 0; d < 3; ++d) {
    if (P->tiles[d] < 1) { set_error("tiles must be >= 1"); return IGAMT_EINVAL; }
    P->box_a[d].clear();
    P->box_h[d].clear();
    if (P->box_mode == 0) {
      const auto &U = P->kM[d];
      for (size_t i = 0; i + 1 < U.size(); ++i)
        if (U[i + 1] > U[i]) { P->box_a[d].push_back(U[i]); P->box_h[d].push_back(U[i + 1] - U[i]); }
      if ((int)P->box_a[d].size() != P->tiles[d]) {
        set_error("box_mode 0: tiles per direction must equal the number of macro knot spans");
        return IGAMT_EINVAL;
      }
    } else {
      for (int t = 0; t < P->tiles[d]; ++t) {
        P->box_a[d].push_back((double)t / P->tiles[d]);
        P->box_h[d].push_back(1.0 / P->tiles[d]);
      }
    }
  }
  P->n_tiles = (int64_t)P->tiles[0] * P->tiles[1] * P->tiles[2];
  P->n_tiles_pad = (P->n_tiles + kTileGroup - 1) / kTileGroup * kTileGroup;
  P->n_groups = P->n_tiles_pad / kTileGroup;
  P->npi = (P->qd[0] + 1) * (P->qd[1] + 1) * (P->qd[2] + 1);
  P->K = 9 * P->npi;
  P->Kp = (P->K + kColPad - 1) / kColPad * kColPad;
  P->nTt = (int64_t)P->nT[0] * P->nT[1] * P->nT[2];
  // pair set I_coo, sorted by (A, B), and the offset lookup table
  for (int d = 0; d < 3; ++d) P->S[d] = 2 * P->pT[d] + 1;
  P->pairs.clear();
  const int64_t lut_stride = (int64_t)P->S[0] * P->S[1] * P->S[2];
  P->pair_lut.assign(P->nTt * lut_stride, -1);
  for (int64_t A = 0; A < P->nTt; ++A) {
    const int ai = (int)(A % P->nT[0]), aj = (int)((A / P->nT[0]) % P->nT[1]), ak = (int)(A / ((int64_t)P->nT[0] * P->nT[1]));
    for (int64_t B = A; B < P->nTt; ++B) {
      const int bi = (int)(B % P->nT[0]), bj = (int)((B / P->nT[0]) % P->nT[1]), bk = (int)(B / ((int64_t)P->nT[0] * P->nT[1]));
      if (!overlap1d(ai, bi, P->pT[0], P->eT[0]) || !overlap1d(aj, bj, P->pT[1], P->eT[1]) ||
          !overlap1d(ak, bk, P->pT[2], P->eT[2]))
        continue;
      const int64_t idx = (int64_t)P->pairs.size() / 2;
      P->pairs.push_back((int32_t)A);
      P->pairs.push_back((int32_t)B);
      const int dx = bi - ai + P->pT[0], dy = bj - aj + P->pT[1], dz = bk - ak + P->pT[2];
      P->pair_lut[A * lut_stride + ((int64_t)dz * P->S[1] + dy) * P->S[0] + dx] = (int32_t)idx;
    }
  }
  P->n_pairs = (int64_t)P->pairs.size() / 2;
  P->Mp = (P->n_pairs + kRowPad - 1) / kRowPad * kRowPad;
  // scatter descriptors (see igamt_internal.h)
  {
    const int nx = P->nT[0], ny = P->nT[1];
    P->pair_desc.assign(igamt::kDescWords * P->n_pairs, -1);
    for (int64_t p = 0; p < P->n_pairs; ++p) {
      const int A = P->pairs[2 * p], B = P->pairs[2 * p + 1];
      const int ai[3] = {A % nx, (A / nx) % ny, A / (nx * ny)};
      const int bi[3] = {B % nx, (B / nx) % ny, B / (nx * ny)};
      int flags = A == B ? 64 : 0, hi = 0;
      for (int d = 0; d < 3; ++d) {
        if (ai[d] == 0 && bi[d] == 0) flags |= 1 << d;
        if (ai[d] == P->nT[d] - 1 && bi[d] == P->nT[d] - 1) { flags |= 8 << d; hi |= 1 << d; }
      }
      int32_t *w = &P->pair_desc[igamt::kDescWords * p];
      w[0] = ai[0] | ai[1] << 8 | ai[2] << 16 | flags << 24;
      w[1] = bi[0] | bi[1] << 8 | bi[2] << 16;
      const int off = ((bi[2] - ai[2] + P->pT[2]) * P->S[1] + (bi[1] - ai[1] + P->pT[1])) * P->S[0] +
                      (bi[0] - ai[0] + P->pT[0]);
      for (int delta = 1; delta < 8; ++delta) {
        if (delta & ~hi) continue;
        const int dx = delta & 1, dy = (delta >> 1) & 1, dz = delta >> 2;
        const int A2 = A - dx * (nx - 1) - nx * (dy * (ny - 1) + ny * dz * (P->nT[2] - 1));
        const int32_t q = P->pair_lut[(int64_t)A2 * lut_stride + off];
        if (q < 0) { set_error("internal: shifted pair missing"); return IGAMT_EINVAL; }
        w[1 + delta] = q;
      }
    }
  }
  // scatter chunks of kScatterChunk consecutive pairs: each chunk's records ordered by (B, A), the
  // order in which the transposed blocks are written (consecutive A of one B are adjacent in row G_B)
  {
    const int64_t C = igamt::kScatterChunk;
    const int64_t chunks = (P->n_pairs + C - 1) / C;
    P->mirror_perm.assign(chunks * C, 0);
    for (int64_t c = 0; c < chunks; ++c) {
      const int64_t p0 = c * C, n = std::min<int64_t>(C, P->n_pairs - p0);
      int32_t *perm = &P->mirror_perm[c * C];
      for (int64_t i = 0; i < C; ++i) perm[i] = i < n ? (int32_t)i : 0;
      std::stable_sort(perm, perm + n, [&](int32_t x, int32_t y) {
        const int32_t bx = P->pairs[2 * (p0 + x) + 1], by = P->pairs[2 * (p0 + y) + 1];
        if (bx != by) return bx < by;
        return P->pairs[2 * (p0 + x)] < P->pairs[2 * (p0 + y)];
      });
    }
  }
  // glued 1-D structure per direction
  for (int d = 0; d < 3; ++d) {
    Direction &D = P->dir[d];
    const int n = P->nT[d], p = P->pT[d], e = P->eT[d], T = P->tiles[d];
    D.NG = T * (n - 1) + 1;
    D.pairs.clear();
    D.off.assign(D.NG + 1, 0);
    D.pre.assign(D.NG + 1, 0);
    D.lo.assign(D.NG, 0);
    for (int g = 0; g < D.NG; ++g) {
      D.off[g] = (int32_t)D.pairs.size();
      std::vector<Pair1D> lst;
      for (int t = 0; t < T; ++t) {
        const int base = t * (n - 1);
        if (g < base || g > base + n - 1) continue;
        const int i = g - base;
        for (int j = 0; j < n; ++j) {
          if (!overlap1d(i, j, p, e)) continue;
          const int g2 = base + j;
          Pair1D *hit = nullptr;
          for (auto &q : lst)
            if (q.g2 == g2) hit = &q;
          if (!hit) {
            Pair1D q{};
            q.g = g; q.g2 = g2; q.ntile = 0;
            q.tile[0] = q.tile[1] = -1;
            lst.push_back(q);
            hit = &lst.back();
          }
          hit->tile[hit->ntile] = t;
          hit->li[hit->ntile] = i;
          hit->lj[hit->ntile] = j;
          hit->ntile++;
        }
      }
      std::sort(lst.begin(), lst.end(), [](const Pair1D &a, const Pair1D &b) { return a.g2 < b.g2; });
      for (size_t r = 0; r < lst.size(); ++r) {
        lst[r].rank = (int32_t)r;
        D.pairs.push_back(lst[r]);
        if (lst[r].g2 != lst[0].g2 + (int)r) {   // the scatter computes ranks as g2 - first neighbour
          set_error("1-D neighbour sets must be contiguous (repeated interior tile knots?)");
          return IGAMT_EUNSUPPORTED;
        }
      }
      D.lo[g] = lst.empty() ? g : lst[0].g2;
      D.pre[g + 1] = D.pre[g] + (int64_t)lst.size();
    }
    D.off[D.NG] = (int32_t)D.pairs.size();
  }
  P->n_global = (int64_t)P->dir[0].NG * P->dir[1].NG * P->dir[2].NG;
  P->nnz = 9 * P->dir[0].pre[P->dir[0].NG] * P->dir[1].pre[P->dir[1].NG] * P->dir[2].pre[P->dir[2].NG];
  // Gauss rules and the 1-D projection operator
  gauss_legendre01(P->n_fit, P->fit_x, P->fit_w);
  gauss_legendre01(P->n_gauss, P->gauss_x, P->gauss_w);
  if (!projection_1d(P->q, P->fit_x, P->fit_w, P->fit_P)) { set_error("singular projection matrix"); return IGAMT_EINVAL; }
  P->fit_P3.clear();
  for (int k = 0; k < 3; ++k) {
    std::vector<double> Pk;
    if (!projection_1d(P->qd[k], P->fit_x, P->fit_w, Pk)) { set_error("singular projection matrix"); return IGAMT_EINVAL; }
    P->fit_P3.insert(P->fit_P3.end(), Pk.begin(), Pk.end());
  }
  // macro control points touched by each tile's samples, and the reverse map
  for (int d = 0; d < 3; ++d) {
    const int p = P->pM[d], n = P->nM[d], T = P->tiles[d];
    P->ctrl_lo[d].assign(T, 0);
    std::vector<int> cnt(T);
    int L = 0;
    for (int t = 0; t < T; ++t) {
      int smin = 1 << 30, smax = -1;
      for (int s = 0; s < P->n_fit; ++s) {
        const int sp = find_span_host(P->kM[d], n, p, P->box_a[d][t] + P->box_h[d][t] * P->fit_x[s]);
        smin = std::min(smin, sp);
        smax = std::max(smax, sp);
      }
      // tiles on a macro face also take samples on that face (the traction's area element)
      if (t == 0) smin = std::min(smin, find_span_host(P->kM[d], n, p, P->box_a[d][t]));
      if (t == T - 1) smax = std::max(smax, find_span_host(P->kM[d], n, p, P->box_a[d][t] + P->box_h[d][t]));
      P->ctrl_lo[d][t] = smin - p;
      cnt[t] = smax - smin + p + 1;
      L = std::max(L, cnt[t]);
    }
    P->Lc[d] = L;
    P->ctrl_tiles_off[d].assign(n + 1, 0);
    P->ctrl_tiles[d].clear();
    for (int i = 0; i < n; ++i) {
      P->ctrl_tiles_off[d][i] = (int32_t)P->ctrl_tiles[d].size() / 2;
      for (int t = 0; t < T; ++t)
        if (i >= P->ctrl_lo[d][t] && i < P->ctrl_lo[d][t] + cnt[t]) {
          P->ctrl_tiles[d].push_back(t);
          P->ctrl_tiles[d].push_back(i - P->ctrl_lo[d][t]);
        }
    }
    P->ctrl_tiles_off[d][n] = (int32_t)P->ctrl_tiles[d].size() / 2;
  }
  return IGAMT_OK;
}

extern "C" igamt_status igamt_plan_create(const igamt_spline3d *macro, const igamt_spline3d *tile,
                                          const igamt_plan_desc *desc, igamt_plan **out) {
  if (!out) { set_error("NULL output pointer"); return IGAMT_EINVAL; }
  *out = nullptr;
  igamt_plan *P = new (std::nothrow) igamt_plan();
  if (!P) { set_error("host allocation failed"); return IGAMT_ENOMEM; }
  igamt_status st;
  try {
    st = build_plan(P, macro, tile, desc);
  } catch (const std::bad_alloc &) {
    set_error("host allocation failed");
    st = IGAMT_ENOMEM;
  }
  if (st != IGAMT_OK) { delete P; return st; }
  *out = P;
  return IGAMT_OK;
}

extern "C" void igamt_plan_destroy(igamt_plan *plan) {
  if (!plan) return;
  free_device(plan);
  delete plan;
}

extern "C" igamt_status igamt_plan_sizes(const igamt_plan *P, igamt_sizes *o) {
  if (!P || !o) { set_error("NULL argument"); return IGAMT_EINVAL; }
  o->n_tiles = P->n_tiles;
  o->n_tiles_pad = P->n_tiles_pad;
  o->n_pairs = P->n_pairs;
  o->n_cols = P->K;
  o->n_cols_pad = P->Kp;
  o->n_tile_ctrl = P->nTt;
  o->n_macro_ctrl = (int64_t)P->nM[0] * P->nM[1] * P->nM[2];
  o->n_global_ctrl = P->n_global;
  o->n_dofs = 3 * P->n_global;
  o->nnz = P->nnz;
  return IGAMT_OK;
}

extern "C" igamt_status igamt_plan_pairs(const igamt_plan *P, int32_t *pairs) {
  if (!P || !pairs) { set_error("NULL argument"); return IGAMT_EINVAL; }
  std::memcpy(pairs, P->pairs.data(), P->pairs.size() * sizeof(int32_t));
  return IGAMT_OK;
}

extern "C" igamt_status igamt_plan_csr(const igamt_plan *P, int64_t *row_ptr, int32_t *col_idx) {
  if (!P || !row_ptr || !col_idx) { set_error("NULL argument"); return IGAMT_EINVAL; }
  const Direction &X = P->dir[0], &Y = P->dir[1], &Z = P->dir[2];
  const int64_t SX = X.pre[X.NG], SY = Y.pre[Y.NG];
  for (int gz = 0; gz < Z.NG; ++gz)
    for (int gy = 0; gy < Y.NG; ++gy)
      for (int gx = 0; gx < X.NG; ++gx) {
        const int64_t G = gx + (int64_t)X.NG * (gy + (int64_t)Y.NG * gz);
        const int64_t cx = X.pre[gx + 1] - X.pre[gx], cy = Y.pre[gy + 1] - Y.pre[gy], cz = Z.pre[gz + 1] - Z.pre[gz];
        const int64_t nnb = cx * cy * cz;
        const int64_t before = Z.pre[gz] * SY * SX + cz * (Y.pre[gy] * SX + cy * X.pre[gx]);
        for (int a = 0; a < 3; ++a) {
          int64_t pos = 9 * before + 3 * a * nnb;
          row_ptr[3 * G + a] = pos;
          for (int64_t kz = 0; kz < cz; ++kz) {
            const int gz2 = Z.pairs[Z.off[gz] + kz].g2;
            for (int64_t ky = 0; ky < cy; ++ky) {
              const int gy2 = Y.pairs[Y.off[gy] + ky].g2;
              for (int64_t kx = 0; kx < cx; ++kx) {
                const int gx2 = X.pairs[X.off[gx] + kx].g2;
                const int64_t G2 = gx2 + (int64_t)X.NG * (gy2 + (int64_t)Y.NG * gz2);
                for (int b = 0; b < 3; ++b) col_idx[pos++] = (int32_t)(3 * G2 + b);
              }
            }
          }
        }
      }
  row_ptr[3 * P->n_global] = P->nnz;
  return IGAMT_OK;
}

extern "C" igamt_status igamt_set_tile_ctrl(igamt_plan *P, const double *ctrl) {
  if (!P || !ctrl) { set_error("NULL argument"); return IGAMT_EINVAL; }
  std::vector<double> c(ctrl, ctrl + 3 * P->nTt);
  for (double v : c)
    if (!std::isfinite(v)) { set_error("non-finite tile control point"); return IGAMT_EINVAL; }
  // boundary must stay at the identity
  std::vector<double> g[3];
  for (int d = 0; d < 3; ++d) g[d] = greville(P->kT[d], P->pT[d], P->nT[d]);
  for (int k = 0; k < P->nT[2]; ++k)
    for (int j = 0; j < P->nT[1]; ++j)
      for (int i = 0; i < P->nT[0]; ++i) {
        bool bnd = i == 0 || j == 0 || k == 0 || i == P->nT[0] - 1 || j == P->nT[1] - 1 || k == P->nT[2] - 1;
        if (!bnd) continue;
        const double *q = &c[3 * (i + P->nT[0] * (j + P->nT[1] * k))];
        if (std::fabs(q[0] - g[0][i]) + std::fabs(q[1] - g[1][j]) + std::fabs(q[2] - g[2][k]) > 1e-12) {
          set_error("tile boundary control points must sit at the identity (Greville) positions");
          return IGAMT_EINVAL;
        }
      }
  P->ctrlT = c;
  P->tables_ready = false;
  P->load_table_ready = false;
  P->volume_ready = false;
  if (P->dev.ready) return upload_tile_ctrl(P);
  return IGAMT_OK;
}
