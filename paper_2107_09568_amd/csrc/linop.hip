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
// forms record j's two 3-vectors K_p u_B (for row A) and K_p^T u_A (for row B, A != B), and the
// wave sums the K_p u_B of each row's run of consecutive records (segmented scan); then the
// chunk's program, built once per plan, sums them per destination row: a list of the chunk's
// 3-vector slots sorted by (row, kind, record) and, per row present, the end of its segment in
// that list (one thread per segment; at most one segment per row and chunk).  The program is
// prefetched with the blocks, so the row sums use LDS only.  Rows add their chunk sums in
// ascending chunk order: no atomics, bitwise reproducible.  Tile results go to ytile[t][3 A + a];
// a gather then sums, per global dof, over the tiles holding it in ascending tile index.
#include <algorithm>

#include "device_common.h"

namespace igamt {

constexpr int kApplyChunk = 256;        // block records per chunk (one per thread)
constexpr int kApplyThreads = 256;
constexpr int kApplyLdsMax = 64 * 1024;
static_assert(kApplyChunk == kApplyThreads && kApplyChunk % 64 == 0, "one record per thread, whole waves");
static_assert(kApplyChunk * 9 == 2 * (4 * kApplyThreads + 128), "16-byte units of a chunk: 4.5 per thread");

// Dynamic LDS of the tile product kernel for block element type of `eb` bytes.
inline int64_t apply_lds_bytes(int64_t nTt, int eb) {
  return (int64_t)kApplyChunk * 9 * eb + (int64_t)kApplyChunk * 6 * 8 + (int64_t)kApplyChunk * (2 * (2 + 4) + 4) +
         6 * nTt * 8;
}

struct ApplyArgs {
  const void *blocks;         // [t1 - t0][n_pairs][9] (tile t at t - t0)
  const double *u;            // [3 n_global]
  double *ytile;              // [n_tiles][3 nTt]
  const int32_t *rec;         // [n_pairs] A | B << 16
  const int32_t *perm;        // [n_chunks][kApplyChunk]: two 16-bit slots each (slot s < kApplyChunk:
                              // K_p u_B of record c0 + s, else K_p^T u_A of record c0 + s - kApplyChunk)
  const int32_t *seg;         // [n_chunks][2 kApplyChunk]: row | end << 16 (row 0xffff: unused)
  int64_t n_pairs, t0;
  int nTt, n_chunks;
  int nT[3], tiles[3];
  int GX, GY;
};

typedef double dbl2 __attribute__((ext_vector_type(2)));

// V16: FP64 blocks moved in 16-byte units (4.5 per thread and chunk: four, then a fifth on the
// first 128 threads, clamped on the others so that every thread issues the same loads); needs a
// 16-byte aligned tile base, i.e. an even pair count.  Otherwise one element per load.
template <typename BT, bool V16>
__global__ __launch_bounds__(kApplyThreads) void tile_apply_kernel(ApplyArgs a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  BT *kb = (BT *)lds_raw;                                                    // [kApplyChunk][9]
  double *vals = (double *)(lds_raw + (size_t)kApplyChunk * 9 * sizeof(BT)); // [2 kApplyChunk][3]
  double *us = vals + kApplyChunk * 6;                                       // [3 nTt]
  double *ys = us + 3 * a.nTt;                                               // [3 nTt]
  int32_t *segs = (int32_t *)(ys + 3 * a.nTt);                               // [2 kApplyChunk]
  uint16_t *perm = (uint16_t *)(segs + 2 * kApplyChunk);                     // [2 kApplyChunk]
  int32_t *recs = (int32_t *)(perm + 2 * kApplyChunk);                       // [kApplyChunk]
  const int tid = threadIdx.x;
  const int64_t t = a.t0 + blockIdx.x;
  const int tt[3] = {(int)(t % a.tiles[0]), (int)((t / a.tiles[0]) % a.tiles[1]),
                     (int)(t / ((int64_t)a.tiles[0] * a.tiles[1]))};
  const BT *blk = (const BT *)a.blocks + (int64_t)blockIdx.x * a.n_pairs * 9;
  // Register prefetch, two chunks ahead in two alternating sets: a chunk's block entries, record
  // descriptors and program.  Loads past the last chunk re-read the last chunk (clamped addresses,
  // so every set always issues the same loads); their data is never used.
  struct Pref {
    BT r[9];
    dbl2 v[5];
    int32_t rec, perm, seg0, seg1;
  };
  auto load = [&](Pref &f, int c) {
    const int cc = min(c, a.n_chunks - 1);
    const int64_t c0 = (int64_t)cc * kApplyChunk;
    const int64_t n = min((int64_t)kApplyChunk, a.n_pairs - c0) * 9;
    const BT *src = blk + c0 * 9;
    f.rec = a.rec[min(c0 + tid, a.n_pairs - 1)];
    f.perm = a.perm[(int64_t)cc * kApplyChunk + tid];
    f.seg0 = a.seg[(int64_t)cc * 2 * kApplyChunk + tid];
    f.seg1 = a.seg[(int64_t)cc * 2 * kApplyChunk + kApplyThreads + tid];
    if constexpr (V16) {
      const dbl2 *src2 = (const dbl2 *)src;
      const int64_t nu = n / 2;   // n is even: an even number of records per chunk
#pragma unroll
      for (int i = 0; i < 4; ++i) f.v[i] = src2[min(tid + (int64_t)i * kApplyThreads, nu - 1)];
      f.v[4] = src2[min((int64_t)4 * kApplyThreads + (tid & 127), nu - 1)];
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) f.r[i] = src[min(tid + (int64_t)i * kApplyThreads, n - 1)];
    }
  };
  Pref f0, f1;
  load(f0, 0);
  load(f1, 1);
  for (int i = tid; i < 3 * a.nTt; i += kApplyThreads) {
    const int A = i / 3, comp = i - 3 * A;
    const int l[3] = {A % a.nT[0], (A / a.nT[0]) % a.nT[1], A / (a.nT[0] * a.nT[1])};
    const int64_t G = (tt[0] * (a.nT[0] - 1) + l[0]) +
                      (int64_t)a.GX * ((tt[1] * (a.nT[1] - 1) + l[1]) + (int64_t)a.GY * (tt[2] * (a.nT[2] - 1) + l[2]));
    us[i] = a.u[3 * G + comp];
    ys[i] = 0.0;
  }
  // one chunk from set f, then the load of chunk c + 2 into f
  auto step = [&](Pref &f, int c) {
    const int64_t c0 = (int64_t)c * kApplyChunk;
    if constexpr (V16) {
      dbl2 *kb2 = (dbl2 *)kb;
#pragma unroll
      for (int i = 0; i < 4; ++i) kb2[tid + i * kApplyThreads] = f.v[i];
      if (tid < 128) kb2[4 * kApplyThreads + tid] = f.v[4];
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) kb[tid + i * kApplyThreads] = f.r[i];
    }
    ((int32_t *)perm)[tid] = f.perm;
    segs[tid] = f.seg0;
    segs[kApplyThreads + tid] = f.seg1;
    recs[tid] = f.rec;   // through LDS: no register of f stays live across its reload
    lds_barrier();
    load(f, c + 2);
    const int32_t rc = recs[tid];
    {
      const bool valid = c0 + tid < a.n_pairs;
      const int A = valid ? rc & 0xffff : 0xffff, B = valid ? rc >> 16 : 0;
      double K[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) K[i] = valid ? (double)kb[tid * 9 + i] : 0.0;
      const double uB0 = us[3 * B], uB1 = us[3 * B + 1], uB2 = us[3 * B + 2];
      double up0 = K[0] * uB0 + K[1] * uB1 + K[2] * uB2;
      double up1 = K[3] * uB0 + K[4] * uB1 + K[5] * uB2;
      double up2 = K[6] * uB0 + K[7] * uB1 + K[8] * uB2;
      if (valid && A != B) {
        const double uA0 = us[3 * A], uA1 = us[3 * A + 1], uA2 = us[3 * A + 2];
        double *lo = vals + 3 * (kApplyChunk + tid);
        lo[0] = K[0] * uA0 + K[3] * uA1 + K[6] * uA2;
        lo[1] = K[1] * uA0 + K[4] * uA1 + K[7] * uA2;
        lo[2] = K[2] * uA0 + K[5] * uA1 + K[8] * uA2;
      }
      // a row's upper records are consecutive: inclusive scan of K_p u_B over the wave, segmented
      // by row (offsets 1, 2, ..., 32); the last lane of each row's run in the wave holds the run's
      // sum, and the chunk's program lists exactly those lanes
      const int lane = tid & 63;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int Ad = __shfl_up(A, d, 64);
        const double t0 = __shfl_up(up0, d, 64), t1 = __shfl_up(up1, d, 64), t2 = __shfl_up(up2, d, 64);
        if (lane >= d && Ad == A) {
          up0 += t0;
          up1 += t1;
          up2 += t2;
        }
      }
      const int An = __shfl_down(A, 1, 64);
      if (valid && (lane == 63 || An != A)) {
        double *up = vals + 3 * tid;
        up[0] = up0;
        up[1] = up1;
        up[2] = up2;
      }
    }
    lds_barrier();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = tid + h * kApplyThreads;
      const int32_t sg = segs[i];
      const int row = sg & 0xffff;
      if (c < a.n_chunks && row != 0xffff) {
        const int end = sg >> 16, start = i > 0 ? segs[i - 1] >> 16 : 0;
        // two independent partial sums (entries start + 2 m + r go to partial r), added at the end
        double y[2][3] = {};
        int k = start;
        for (; k + 2 <= end; k += 2) {
          const double *v0 = vals + 3 * perm[k], *v1 = vals + 3 * perm[k + 1];
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            y[0][d] += v0[d];
            y[1][d] += v1[d];
          }
        }
        if (k < end) {
          const double *v = vals + 3 * perm[k];
#pragma unroll
          for (int d = 0; d < 3; ++d) y[0][d] += v[d];
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) ys[3 * row + d] += y[0][d] + y[1][d];
      }
    }
    lds_barrier();
  };
  // both steps unconditional (the same loads on every path); with an odd number of chunks the
  // last step is empty: no valid record, no row sums
  for (int c = 0; c < a.n_chunks; c += 2) {
    step(f0, c);
    step(f1, c + 1);
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

// Record descriptors and the per-chunk row-sum programs of the tile product (built once per plan
// from the pair list; they do not depend on the tile's control points).
static igamt_status ensure_apply_schedule(igamt_plan *P) {
  if (P->dev.apply_rec) return IGAMT_OK;
  const int64_t np = P->n_pairs;
  const int n_chunks = (int)((np + kApplyChunk - 1) / kApplyChunk);
  std::vector<int32_t> rec(np);
  std::vector<uint16_t> perm((int64_t)n_chunks * 2 * kApplyChunk, 0);
  std::vector<int32_t> seg((int64_t)n_chunks * 2 * kApplyChunk, 0xffff);
  for (int64_t p = 0; p < np; ++p) rec[p] = P->pairs[2 * p] | P->pairs[2 * p + 1] << 16;
  struct Entry { int32_t row, kind, p, slot; };
  std::vector<Entry> ent;
  for (int c = 0; c < n_chunks; ++c) {
    const int64_t c0 = (int64_t)c * kApplyChunk, c1 = std::min(c0 + kApplyChunk, np);
    ent.clear();
    for (int64_t p = c0; p < c1; ++p) {
      const int A = P->pairs[2 * p], B = P->pairs[2 * p + 1];
      // upper records: only the last record of the row's run within its wave (kernel-side scan)
      const bool run_end = (p - c0) % 64 == 63 || p + 1 == c1 || P->pairs[2 * (p + 1)] != A;
      if (run_end) ent.push_back({A, 0, (int32_t)p, (int32_t)(p - c0)});
      if (A != B) ent.push_back({B, 1, (int32_t)p, (int32_t)(kApplyChunk + p - c0)});
    }
    std::sort(ent.begin(), ent.end(), [](const Entry &x, const Entry &y) {
      return x.row != y.row ? x.row < y.row : x.kind != y.kind ? x.kind < y.kind : x.p < y.p;
    });
    uint16_t *pc = &perm[(int64_t)c * 2 * kApplyChunk];
    int32_t *sc = &seg[(int64_t)c * 2 * kApplyChunk];
    int ns = 0;
    for (size_t k = 0; k < ent.size(); ++k) {
      pc[k] = (uint16_t)ent[k].slot;
      if (k + 1 == ent.size() || ent[k + 1].row != ent[k].row) sc[ns++] = ent[k].row | (int32_t)(k + 1) << 16;
    }
    for (int i = ns; i < 2 * kApplyChunk; ++i) sc[i] = 0xffff | (int32_t)ent.size() << 16;
  }
  const size_t n_words = rec.size() + perm.size() / 2 + seg.size();
  int32_t *d = nullptr;
  IGAMT_HIP(hipMalloc((void **)&d, n_words * sizeof(int32_t)));
  bool ok = hipMemcpy(d, rec.data(), rec.size() * 4, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(d + rec.size(), perm.data(), perm.size() * 2, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(d + rec.size() + perm.size() / 2, seg.data(), seg.size() * 4, hipMemcpyHostToDevice) ==
                hipSuccess;
  if (!ok) {
    (void)hipFree(d);
    set_error("upload of the tile product schedule failed");
    return IGAMT_EHIP;
  }
  P->dev.apply_rec = d;
  P->dev.apply_perm = d + rec.size();
  P->dev.apply_seg = P->dev.apply_perm + perm.size() / 2;
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
  a.perm = P->dev.apply_perm;
  a.seg = P->dev.apply_seg;
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
    if (P->n_pairs % 2 == 0 && (uintptr_t)blocks % 16 == 0)
      hipLaunchKernelGGL((tile_apply_kernel<double, true>), grid, block, (size_t)apply_lds_bytes(P->nTt, 8), s, a);
    else
      hipLaunchKernelGGL((tile_apply_kernel<double, false>), grid, block, (size_t)apply_lds_bytes(P->nTt, 8), s, a);
  else
    hipLaunchKernelGGL((tile_apply_kernel<float, false>), grid, block, (size_t)apply_lds_bytes(P->nTt, 4), s, a);
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
