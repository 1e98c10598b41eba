// Matrix-free product K u of the multiscale operator (Section 4.2, eq. (74)).
//
// K u = sum over tiles t of the tile product K^(t) u^(t), glued at the shared control points.
// The tile matrix K^(t) is available as the n_pairs upper 3x3 blocks the contraction of eq. (58)
// writes, blocks[t][p][3 a + b] for the pair p = (A, B), A <= B:
//   (K^(t) u^(t))[A][a] = sum_{p = (A, B)} sum_b K_p[a][b] u[B][b]
//                       + sum_{p = (B, A), B < A} sum_b K_p[b][a] u[B][b].
// Two entry points:
//   igamt_apply_blocks   from stored blocks of all tiles (one contraction, many products);
//   igamt_linop          on the fly, as the paper describes it: only the table and the projection
//                        coefficients are kept; the blocks of one slab of tiles at a time are
//                        contracted into a bounded workspace and applied at once, so the whole
//                        set of tile matrices never exists.  A slab of a few hundred tiles fits
//                        the device's last-level cache between its contraction and its product.
//
// Tile product kernel: one workgroup of 256 threads per tile.  The tile's displacements u^(t)
// go to LDS; the block records stream through LDS in chunks of kApplyChunk records (coalesced
// loads, the next chunk's loads in flight while the current one is used).  Per chunk, thread j
// forms record j's two 3-vectors K_p u_B (for row A) and K_p^T u_A (for row B, A != B); then the
// thread owning row A adds, in ascending record order, its upper records of the chunk and its
// mirror records (pairs (B, A)) of the chunk.  The per-row order is fixed by the plan: no atomics,
// bitwise reproducible.  Tile results go to ytile[t][3 A + a]; a gather then sums, per global dof,
// over the tiles holding it in ascending tile index.
#include <algorithm>

#include "device_common.h"

namespace igamt {

constexpr int kApplyChunk = 256;        // block records per chunk (one per thread)
constexpr int kApplyThreads = 256;
constexpr int kApplyLdsMax = 64 * 1024;

// Dynamic LDS of the tile product kernel for block element type of `eb` bytes.
inline int64_t apply_lds_bytes(int64_t nTt, int eb) {
  return (int64_t)kApplyChunk * 9 * eb + (int64_t)kApplyChunk * 6 * 8 + 6 * nTt * 8;
}

struct ApplyArgs {
  const void *blocks;         // [t1 - t0][n_pairs][9] (tile t at t - t0)
  const double *u;            // [3 n_global]
  double *ytile;              // [n_tiles][3 nTt]
  const int32_t *rec;         // [n_pairs] A | B << 16
  const int32_t *row_off;     // [nTt + 1] first record of row A
  const int32_t *mirror_p;    // records (B, A), B < A, grouped by A, ascending
  const int32_t *mirror_chunk;// [(n_chunks + 1) * nTt] first mirror entry of A at or after chunk c
  int64_t n_pairs, t0;
  int nTt, n_chunks;
  int nT[3], tiles[3];
  int GX, GY;
};

template <typename BT>
__global__ __launch_bounds__(kApplyThreads) void tile_apply_kernel(ApplyArgs a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  BT *kb = (BT *)lds_raw;                                                   // [kApplyChunk][9]
  double *upc = (double *)(lds_raw + (size_t)kApplyChunk * 9 * sizeof(BT));  // [kApplyChunk][3]
  double *loc = upc + kApplyChunk * 3;                                      // [kApplyChunk][3]
  double *us = loc + kApplyChunk * 3;                                       // [3 nTt]
  double *ys = us + 3 * a.nTt;                                              // [3 nTt]
  const int tid = threadIdx.x;
  const int64_t t = a.t0 + blockIdx.x;
  const int tt[3] = {(int)(t % a.tiles[0]), (int)((t / a.tiles[0]) % a.tiles[1]),
                     (int)(t / ((int64_t)a.tiles[0] * a.tiles[1]))};
  const BT *blk = (const BT *)a.blocks + (int64_t)blockIdx.x * a.n_pairs * 9;
  // chunk 0 loads in flight while u^(t) is gathered
  BT reg[9];
  int32_t rec_next = 0;
  auto load_chunk = [&](int c) {
    const int64_t c0 = (int64_t)c * kApplyChunk;
    const int64_t n = min((int64_t)kApplyChunk, a.n_pairs - c0) * 9;
    const BT *src = blk + c0 * 9;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int64_t e = tid + (int64_t)i * kApplyThreads;
      reg[i] = e < n ? src[e] : BT(0);
    }
    rec_next = c0 + tid < a.n_pairs ? a.rec[c0 + tid] : 0;
  };
  load_chunk(0);
  for (int i = tid; i < 3 * a.nTt; i += kApplyThreads) {
    const int A = i / 3, comp = i - 3 * A;
    const int l[3] = {A % a.nT[0], (A / a.nT[0]) % a.nT[1], A / (a.nT[0] * a.nT[1])};
    const int64_t G = (tt[0] * (a.nT[0] - 1) + l[0]) +
                      (int64_t)a.GX * ((tt[1] * (a.nT[1] - 1) + l[1]) + (int64_t)a.GY * (tt[2] * (a.nT[2] - 1) + l[2]));
    us[i] = a.u[3 * G + comp];
    ys[i] = 0.0;
  }
  for (int c = 0; c < a.n_chunks; ++c) {
    const int64_t c0 = (int64_t)c * kApplyChunk;
#pragma unroll
    for (int i = 0; i < 9; ++i) kb[tid + i * kApplyThreads] = reg[i];
    const int32_t rc = rec_next;
    lds_barrier();
    if (c + 1 < a.n_chunks) load_chunk(c + 1);
    if (c0 + tid < a.n_pairs) {
      const int A = rc & 0xffff, B = rc >> 16;
      double K[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) K[i] = (double)kb[tid * 9 + i];
      const double uB0 = us[3 * B], uB1 = us[3 * B + 1], uB2 = us[3 * B + 2];
      upc[3 * tid + 0] = K[0] * uB0 + K[1] * uB1 + K[2] * uB2;
      upc[3 * tid + 1] = K[3] * uB0 + K[4] * uB1 + K[5] * uB2;
      upc[3 * tid + 2] = K[6] * uB0 + K[7] * uB1 + K[8] * uB2;
      if (A != B) {
        const double uA0 = us[3 * A], uA1 = us[3 * A + 1], uA2 = us[3 * A + 2];
        loc[3 * tid + 0] = K[0] * uA0 + K[3] * uA1 + K[6] * uA2;
        loc[3 * tid + 1] = K[1] * uA0 + K[4] * uA1 + K[7] * uA2;
        loc[3 * tid + 2] = K[2] * uA0 + K[5] * uA1 + K[8] * uA2;
      }
    }
    lds_barrier();
    const int64_t c1 = min(c0 + kApplyChunk, a.n_pairs);
    for (int A = tid; A < a.nTt; A += kApplyThreads) {
      double y0 = ys[3 * A], y1 = ys[3 * A + 1], y2 = ys[3 * A + 2];
      const int64_t p0 = max((int64_t)a.row_off[A], c0), p1 = min((int64_t)a.row_off[A + 1], c1);
      for (int64_t p = p0; p < p1; ++p) {
        const int j = (int)(p - c0);
        y0 += upc[3 * j];
        y1 += upc[3 * j + 1];
        y2 += upc[3 * j + 2];
      }
      const int m0 = a.mirror_chunk[(int64_t)c * a.nTt + A], m1 = a.mirror_chunk[(int64_t)(c + 1) * a.nTt + A];
      for (int m = m0; m < m1; ++m) {
        const int j = (int)(a.mirror_p[m] - c0);
        y0 += loc[3 * j];
        y1 += loc[3 * j + 1];
        y2 += loc[3 * j + 2];
      }
      ys[3 * A] = y0;
      ys[3 * A + 1] = y1;
      ys[3 * A + 2] = y2;
    }
    lds_barrier();
  }
  double *out = a.ytile + t * 3 * a.nTt;
  for (int i = tid; i < 3 * a.nTt; i += kApplyThreads) out[i] = ys[i];
}

struct ApplyGatherArgs {
  const double *ytile;        // [n_tiles][3 nTt]
  int nT[3], tiles[3], nTt;
  int64_t n_global;
  int GX, GY;
  double *y;                  // [3 n_global]
};

__global__ __launch_bounds__(256) void apply_gather_kernel(ApplyGatherArgs a) {
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
        const int64_t t = tx + (int64_t)a.tiles[0] * (ty + (int64_t)a.tiles[1] * tz);
        const int li[3] = {g[0] - tx * (a.nT[0] - 1), g[1] - ty * (a.nT[1] - 1), g[2] - tz * (a.nT[2] - 1)};
        const int64_t A = li[0] + (int64_t)a.nT[0] * (li[1] + (int64_t)a.nT[1] * li[2]);
        sum += a.ytile[t * 3 * a.nTt + 3 * A + comp];
      }
  a.y[id] = sum;
}

// Record descriptors and the row and mirror schedules of the tile product (built once per plan
// from the pair list; they do not depend on the tile's control points).
static igamt_status ensure_apply_schedule(igamt_plan *P) {
  if (P->dev.apply_rec) return IGAMT_OK;
  const int64_t np = P->n_pairs, nTt = P->nTt;
  const int n_chunks = (int)((np + kApplyChunk - 1) / kApplyChunk);
  std::vector<int32_t> rec(np), row_off(nTt + 1, 0), mcount(nTt + 1, 0);
  for (int64_t p = 0; p < np; ++p) {
    const int A = P->pairs[2 * p], B = P->pairs[2 * p + 1];
    rec[p] = A | B << 16;
    ++row_off[A + 1];
    if (A != B) ++mcount[B + 1];
  }
  for (int64_t A = 0; A < nTt; ++A) {
    row_off[A + 1] += row_off[A];
    mcount[A + 1] += mcount[A];
  }
  std::vector<int32_t> mirror(std::max<int64_t>(mcount[nTt], 1)), fill(mcount.begin(), mcount.end() - 1);
  for (int64_t p = 0; p < np; ++p) {   // ascending p within each row's mirror list
    const int A = P->pairs[2 * p], B = P->pairs[2 * p + 1];
    if (A != B) mirror[fill[B]++] = (int32_t)p;
  }
  std::vector<int32_t> mchunk((int64_t)(n_chunks + 1) * nTt);
  for (int64_t A = 0; A < nTt; ++A) {
    int m = mcount[A];
    for (int c = 0; c <= n_chunks; ++c) {
      const int64_t c0 = (int64_t)c * kApplyChunk;
      while (m < mcount[A + 1] && mirror[m] < c0) ++m;
      mchunk[(int64_t)c * nTt + A] = m;
    }
  }
  std::vector<int32_t> all;
  all.reserve(rec.size() + row_off.size() + mirror.size() + mchunk.size());
  all.insert(all.end(), rec.begin(), rec.end());
  all.insert(all.end(), row_off.begin(), row_off.end());
  all.insert(all.end(), mirror.begin(), mirror.end());
  all.insert(all.end(), mchunk.begin(), mchunk.end());
  int32_t *d = nullptr;
  IGAMT_HIP(hipMalloc((void **)&d, all.size() * sizeof(int32_t)));
  if (hipMemcpy(d, all.data(), all.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    set_error("upload of the tile product schedule failed");
    return IGAMT_EHIP;
  }
  P->dev.apply_rec = d;
  P->dev.apply_row_off = d + rec.size();
  P->dev.apply_mirror = P->dev.apply_row_off + row_off.size();
  P->dev.apply_mirror_chunk = P->dev.apply_mirror + mirror.size();
  return IGAMT_OK;
}

static int64_t ytile_bytes(const igamt_plan *P) { return align256(P->n_tiles * 3 * P->nTt * (int64_t)sizeof(double)); }

static int64_t slab_bytes(const igamt_plan *P, igamt_precision prec, int64_t slab_tiles) {
  return align256(slab_tiles * P->n_pairs * 9 * (prec == IGAMT_F64 ? 8 : 4));
}

static igamt_status check_apply_plan(const igamt_plan *P, igamt_precision prec) {
  if (prec < IGAMT_F64 || prec > IGAMT_F16X3) { set_error("unknown precision"); return IGAMT_EINVAL; }
  if (apply_lds_bytes(P->nTt, prec == IGAMT_F64 ? 8 : 4) > kApplyLdsMax || P->nTt > 0xffff) {
    set_error("tile too large for the matrix-free product (its displacements do not fit the LDS)");
    return IGAMT_EUNSUPPORTED;
  }
  return IGAMT_OK;
}

// Tile products of tiles [t0, t1) from blocks (tile t at t - t0) into ytile.
static igamt_status launch_tile_apply(igamt_plan *P, igamt_precision prec, const void *blocks, const double *u,
                                      double *ytile, int64_t t0, int64_t t1, hipStream_t s) {
  ApplyArgs a;
  a.blocks = blocks;
  a.u = u;
  a.ytile = ytile;
  a.rec = P->dev.apply_rec;
  a.row_off = P->dev.apply_row_off;
  a.mirror_p = P->dev.apply_mirror;
  a.mirror_chunk = P->dev.apply_mirror_chunk;
  a.n_pairs = P->n_pairs;
  a.t0 = t0;
  a.nTt = (int)P->nTt;
  a.n_chunks = (int)((P->n_pairs + kApplyChunk - 1) / kApplyChunk);
  for (int k = 0; k < 3; ++k) {
    a.nT[k] = P->nT[k];
    a.tiles[k] = P->tiles[k];
  }
  a.GX = P->dir[0].NG;
  a.GY = P->dir[1].NG;
  const dim3 grid((unsigned)(t1 - t0)), block(kApplyThreads);
  if (prec == IGAMT_F64)
    hipLaunchKernelGGL(tile_apply_kernel<double>, grid, block, (size_t)apply_lds_bytes(P->nTt, 8), s, a);
  else
    hipLaunchKernelGGL(tile_apply_kernel<float>, grid, block, (size_t)apply_lds_bytes(P->nTt, 4), s, a);
  IGAMT_LAUNCH_CHECK();
  return IGAMT_OK;
}

static igamt_status launch_apply_gather(igamt_plan *P, const double *ytile, double *y, hipStream_t s) {
  ApplyGatherArgs a;
  a.ytile = ytile;
  for (int k = 0; k < 3; ++k) {
    a.nT[k] = P->nT[k];
    a.tiles[k] = P->tiles[k];
  }
  a.nTt = (int)P->nTt;
  a.n_global = P->n_global;
  a.GX = P->dir[0].NG;
  a.GY = P->dir[1].NG;
  a.y = y;
  hipLaunchKernelGGL(apply_gather_kernel, dim3((unsigned)((3 * P->n_global + 255) / 256)), dim3(256), 0, s, a);
  IGAMT_LAUNCH_CHECK();
  return IGAMT_OK;
}

}  // namespace igamt

using namespace igamt;

extern "C" igamt_status igamt_linop_workspace_bytes(const igamt_plan *P, igamt_precision prec, int64_t slab_tiles,
                                                    int64_t *bytes) {
  if (!P || !bytes) { set_error("NULL argument"); return IGAMT_EINVAL; }
  if (prec < IGAMT_F64 || prec > IGAMT_F16X3) { set_error("unknown precision"); return IGAMT_EINVAL; }
  if (slab_tiles < 0 || (slab_tiles > 0 && slab_tiles % kTileGroup != 0)) {
    set_error("slab_tiles must be 0 or a positive multiple of 16");
    return IGAMT_EINVAL;
  }
  *bytes = ytile_bytes(P) + (slab_tiles > 0 ? slab_bytes(P, prec, std::min(slab_tiles, P->n_tiles_pad)) : 0);
  return IGAMT_OK;
}

extern "C" igamt_status igamt_apply_blocks(igamt_plan *P, igamt_precision prec, const void *d_blocks,
                                           const double *d_u, double *d_y, void *d_workspace, void *stream) {
  if (!P || !d_blocks || !d_u || !d_y || !d_workspace) { set_error("NULL argument"); return IGAMT_EINVAL; }
  igamt_status st = check_apply_plan(P, prec);
  if (st) return st;
  if ((st = ensure_device(P))) return st;
  if ((st = ensure_apply_schedule(P))) return st;
  hipStream_t s = (hipStream_t)stream;
  double *ytile = (double *)d_workspace;
  if ((st = launch_tile_apply(P, prec, d_blocks, d_u, ytile, 0, P->n_tiles, s))) return st;
  return launch_apply_gather(P, ytile, d_y, s);
}

extern "C" igamt_status igamt_linop(igamt_plan *P, igamt_precision prec, int64_t slab_tiles, const void *d_coef,
                                    const double *d_u, double *d_y, void *d_workspace, void *stream) {
  if (!P || !d_coef || !d_u || !d_y || !d_workspace) { set_error("NULL argument"); return IGAMT_EINVAL; }
  if (slab_tiles <= 0 || slab_tiles % kTileGroup != 0) {
    set_error("slab_tiles must be a positive multiple of 16");
    return IGAMT_EINVAL;
  }
  igamt_status st = check_apply_plan(P, prec);
  if (st) return st;
  if ((st = ensure_device(P))) return st;
  if (!P->tables_ready) { set_error("tables are not built or set"); return IGAMT_ESTATE; }
  if ((st = ensure_apply_schedule(P))) return st;
  hipStream_t s = (hipStream_t)stream;
  double *ytile = (double *)d_workspace;
  char *slab = (char *)d_workspace + ytile_bytes(P);
  const int64_t tile_bytes = P->n_pairs * 9 * (prec == IGAMT_F64 ? 8 : 4);
  const int64_t groups = slab_tiles / kTileGroup;
  for (int64_t g0 = 0; g0 < P->n_groups; g0 += groups) {
    const int64_t g1 = std::min(g0 + groups, P->n_groups);
    const int64_t t0 = g0 * kTileGroup, t1 = std::min(g1 * kTileGroup, P->n_tiles);
    if (t0 >= t1) break;
    // the contraction addresses its output by absolute tile index; shift the base so that tile t0
    // lands at the start of the slab (only tiles t0 .. t1 - 1 are written)
    void *base = (void *)((uintptr_t)slab - (uintptr_t)(t0 * tile_bytes));
    if ((st = launch_contract(P, prec, d_coef, base, stream, g0, g1))) return st;
    if ((st = launch_tile_apply(P, prec, slab, d_u, ytile, t0, t1, s))) return st;
  }
  return launch_apply_gather(P, ytile, d_y, s);
}
