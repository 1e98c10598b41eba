// Stage 3 of the assembly: deterministic scatter of the tile blocks into the
// fixed CSR structure (step 4 of Section 3.2.4).
//
// A workgroup takes kScatterChunk (512) consecutive block records of one tile (pairs p = (A, B),
// A <= B tile-local), loads them into LDS with coalesced loads, and gives one
// thread to each record.
// The record's global pair {G_A, G_B} may be shared with neighbouring tiles:
// per direction d, the 1-D pair (a_d, b_d) is shared with tile t_d - 1 when
// a_d = b_d = 0 and with tile t_d + 1 when a_d = b_d = n_d - 1, and the shared
// tiles hold it with the local indices shifted by n_d - 1 (the pair offset is
// unchanged, so no transposition arises).  The record of the lowest tile
// index owns the global pair: every other record is skipped, the owner
// sums the contributions in ascending tile index (its own first) and writes the
// 3x3 block at (G_A, G_B) and its transpose at (G_B, G_A).  Every CSR value is
// written exactly once, every record is read once (by its owner), no atomics
// are needed, and the result is bitwise reproducible.  The stores go through the
// LDS copy with a word-level lane mapping so that consecutive lanes write
// consecutive words of each contiguous run of blocks in a CSR row.
//
// CSR addressing needs no search: the three rows of G are contiguous and hold
// 9 nnb(G) values, with nnb(G) = c_x c_y c_z the product of the 1-D neighbour
// counts; their offset is 9 sum_{G' < G} nnb(G'), a combination of 1-D prefix
// sums; and the rank of G' among the neighbours of G (x fastest) follows from
// the first 1-D neighbour of each coordinate of G.
//
// Work items (tile, record chunk) are split into eight contiguous ranges,
// one per XCD, so that the records of a tile and of its neighbours (whose rows
// share cache lines) are handled by one L2.
#include "device_common.h"

namespace igamt {

constexpr int kScatterThreads = kScatterChunk;

constexpr int kMaxTileN = kMaxTileControl;   // tile control points per direction the LDS slices hold

struct ScatterArgs {
  const int32_t *desc;       // [M][kDescWords] pair descriptors
  const int64_t *pre[3];     // [NG + 1] prefix sums of 1-D neighbour counts
  const int32_t *lo[3];      // [NG] first 1-D neighbour
  const int32_t *mirror_perm;  // per chunk: record order for the transposed blocks
  int nT[3], tiles[3];
  int chunks;                // record chunks per tile
  int64_t M, n_tiles, per_xcd, SX, SY;
  const void *blocks;        // [n_tiles][M][9]
  void *values;              // [nnz]
};

template <typename T>
__global__ __launch_bounds__(kScatterThreads) void scatter_kernel(ScatterArgs a) {
  constexpr int NT = kScatterThreads;
  __shared__ T vals[NT * 9];          // the chunk's records, then the owners' sums
  __shared__ int64_t row0[NT][2];     // first value of the block in row 0 of G_A / of G_B (-1: none)
  __shared__ int32_t nnb[NT][2];      // neighbour counts of G_A / G_B
  __shared__ int64_t sp[3][kMaxTileN];  // the tile's slice of the 1-D tables: prefix sums,
  __shared__ int32_t sc[3][kMaxTileN];  // neighbour counts and first neighbours
  __shared__ int32_t sl[3][kMaxTileN];
  const int64_t w = blockIdx.x;
  const int64_t item = (w & 7) * a.per_xcd + (w >> 3);
  const int64_t tile = item / a.chunks;
  if (tile >= a.n_tiles) return;
  const int chunk = (int)(item - tile * a.chunks);
  const int64_t p0 = (int64_t)chunk * NT;
  const int nrec = (int)min((int64_t)NT, a.M - p0);
  const int tid = threadIdx.x;
  const T *blk = (const T *)a.blocks;
  const int tt[3] = {(int)(tile % a.tiles[0]), (int)((tile / a.tiles[0]) % a.tiles[1]),
                     (int)(tile / ((int64_t)a.tiles[0] * a.tiles[1]))};

  // 1. independent loads, all issued before the first wait: the pair descriptor, the tile's
  //    slices of the 1-D tables, and the chunk's records (contiguous, coalesced)
  const int4 *dp = (const int4 *)(a.desc + kDescWords * (p0 + min(tid, nrec - 1)));
  const int4 d0 = dp[0], d1 = dp[1];
  // (loads are unconditional, with clamped indices, so that none waits for another)
  // (no run-time index into the argument block: that would be a dependent load)
  const int sd = min(tid / kMaxTileN, 2);
  const int n_d = sd == 0 ? a.nT[0] : sd == 1 ? a.nT[1] : a.nT[2];
  const int t_d = sd == 0 ? tt[0] : sd == 1 ? tt[1] : tt[2];
  const int si = min(tid - sd * kMaxTileN, n_d - 1);
  const bool slicer = tid < 3 * kMaxTileN && tid - sd * kMaxTileN < n_d;
  const int64_t *pre_d = sd == 0 ? a.pre[0] : sd == 1 ? a.pre[1] : a.pre[2];
  const int32_t *lo_d = sd == 0 ? a.lo[0] : sd == 1 ? a.lo[1] : a.lo[2];
  const int g = t_d * (n_d - 1) + si;
  const int64_t s_pre = pre_d[g], s_pre1 = pre_d[g + 1];
  const int32_t s_lo = lo_d[g];
  {
    const T *src = blk + (tile * a.M + p0) * 9;
    const int last = nrec * 9 - 1;
    T r[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) r[k] = src[min(k * NT + tid, last)];
    __builtin_amdgcn_sched_barrier(0);   // keep every load above ahead of the first wait
#pragma unroll
    for (int k = 0; k < 9; ++k) vals[k * NT + tid] = r[k];
  }
  if (slicer) {
    sp[sd][si] = s_pre;
    sc[sd][si] = (int32_t)(s_pre1 - s_pre);
    sl[sd][si] = s_lo;
  }

  // 2. one thread per record: ownership, and the first record of a higher tile sharing the
  //    global pair is requested before the barrier
  const int flags = (d0.x >> 24) & 127;
  const int ai[3] = {d0.x & 255, (d0.x >> 8) & 255, (d0.x >> 16) & 255};
  const int bi[3] = {d0.y & 255, (d0.y >> 8) & 255, (d0.y >> 16) & 255};
  bool owner = tid < nrec;
  int up = 0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if ((flags >> d) & 1 && tt[d] > 0) owner = false;                          // a lower tile owns it
    if ((flags >> (3 + d)) & 1 && tt[d] < a.tiles[d] - 1) up |= 1 << d;       // higher tiles share it
  }
  if (!owner) up = 0;
  const int sh[8] = {-1, d0.z, d0.w, d1.x, d1.y, d1.z, d1.w, -1};
  const int d7 = up == 7 ? a.desc[kDescWords * (p0 + tid) + 8] : -1;
  T nb[9];
  const int first = up & -up;                     // lowest shift: 1, 2 or 4
  if (up) {
    const int64_t t2 = tile + (first & 1) + (int64_t)a.tiles[0] * (((first >> 1) & 1) + (int64_t)a.tiles[1] * (first >> 2));
    const T *src = blk + (t2 * a.M + sh[first]) * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) nb[k] = src[k];
  }
  __syncthreads();

  if (owner) {
    if (up) {
      T v[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) v[k] = vals[tid * 9 + k] + nb[k];
      // further sharing tiles (edges and corners of the tile grid's faces) in ascending tile
      // index = ascending delta = dx + 2 dy + 4 dz
      for (int delta = first + 1; delta < 8; ++delta) {
        if (delta & ~up) continue;
        const int dx = delta & 1, dy = (delta >> 1) & 1, dz = delta >> 2;
        const int64_t t2 = tile + dx + (int64_t)a.tiles[0] * (dy + (int64_t)a.tiles[1] * dz);
        const T *src = blk + (t2 * a.M + (delta == 7 ? d7 : sh[delta])) * 9;
#pragma unroll
        for (int k = 0; k < 9; ++k) v[k] += src[k];
      }
#pragma unroll
      for (int k = 0; k < 9; ++k) vals[tid * 9 + k] = v[k];
    }
    {
      const int64_t base = 9 * (sp[2][ai[2]] * a.SY * a.SX + sc[2][ai[2]] * (sp[1][ai[1]] * a.SX +
                                (int64_t)sc[1][ai[1]] * sp[0][ai[0]]));
      const int64_t rank = ((int64_t)(bi[2] + tt[2] * (a.nT[2] - 1) - sl[2][ai[2]]) * sc[1][ai[1]] +
                            (bi[1] + tt[1] * (a.nT[1] - 1) - sl[1][ai[1]])) * sc[0][ai[0]] +
                           (bi[0] + tt[0] * (a.nT[0] - 1) - sl[0][ai[0]]);
      row0[tid][0] = base + 3 * rank;
      nnb[tid][0] = sc[0][ai[0]] * sc[1][ai[1]] * sc[2][ai[2]];
    }
    if (!(flags & 64)) {
      const int64_t base = 9 * (sp[2][bi[2]] * a.SY * a.SX + sc[2][bi[2]] * (sp[1][bi[1]] * a.SX +
                                (int64_t)sc[1][bi[1]] * sp[0][bi[0]]));
      const int64_t rank = ((int64_t)(ai[2] + tt[2] * (a.nT[2] - 1) - sl[2][bi[2]]) * sc[1][bi[1]] +
                            (ai[1] + tt[1] * (a.nT[1] - 1) - sl[1][bi[1]])) * sc[0][bi[0]] +
                           (ai[0] + tt[0] * (a.nT[0] - 1) - sl[0][bi[0]]);
      row0[tid][1] = base + 3 * rank;
      nnb[tid][1] = sc[0][bi[0]] * sc[1][bi[1]] * sc[2][bi[2]];
    } else {
      row0[tid][1] = -1;
    }
  } else if (tid < nrec) {
    row0[tid][0] = row0[tid][1] = -1;
  }
  __syncthreads();

  // 3. stores, lane q -> (row r, piece i, word c) with c fastest, so that consecutive lanes write
  //    consecutive words wherever consecutive pieces are adjacent in the row:
  //    blocks at (G_A, G_B) in record order (for one A, consecutive B are adjacent in row G_A),
  //    transposed blocks at (G_B, G_A) in (B, A) order (for one B, consecutive A are adjacent).
  T *out = (T *)a.values;
  const int32_t *perm = a.mirror_perm + p0;
#pragma unroll
  for (int it = 0; it < 9; ++it) {
    const int q = it * NT + tid;
    const int r = q / (3 * NT), i = (q - r * 3 * NT) / 3, c = q % 3;
    if (i < nrec && row0[i][0] >= 0) out[row0[i][0] + 3 * r * (int64_t)nnb[i][0] + c] = vals[i * 9 + 3 * r + c];
  }
#pragma unroll
  for (int it = 0; it < 9; ++it) {
    const int q = it * NT + tid;
    const int r = q / (3 * NT), i = (q - r * 3 * NT) / 3, c = q % 3;
    if (i < nrec) {
      const int j = perm[i];
      if (row0[j][1] >= 0) out[row0[j][1] + 3 * r * (int64_t)nnb[j][1] + c] = vals[j * 9 + 3 * c + r];
    }
  }
}

igamt_status launch_scatter(igamt_plan *P, igamt_precision prec, const void *d_blocks, void *d_values, void *stream) {
  ScatterArgs a;
  for (int k = 0; k < 3; ++k) {
    if (P->nT[k] > kMaxTileN || P->nT[k] > 255) {
      set_error("tile too large for the scatter kernel");
      return IGAMT_EUNSUPPORTED;
    }
    a.pre[k] = P->dev.dir_pre[k];
    a.lo[k] = P->dev.dir_lo[k];
    a.nT[k] = P->nT[k];
    a.tiles[k] = P->tiles[k];
  }
  a.desc = P->dev.pair_desc;
  a.mirror_perm = P->dev.mirror_perm;
  a.M = P->n_pairs;
  a.n_tiles = P->n_tiles;
  a.chunks = (int)((P->n_pairs + kScatterThreads - 1) / kScatterThreads);
  const int64_t items = P->n_tiles * a.chunks;
  a.per_xcd = (items + 7) / 8;
  a.SX = P->dir[0].pre[P->dir[0].NG];
  a.SY = P->dir[1].pre[P->dir[1].NG];
  a.blocks = d_blocks;
  a.values = d_values;
  if (8 * a.per_xcd > INT32_MAX) { set_error("too many scatter work items"); return IGAMT_EUNSUPPORTED; }
  const dim3 grid((unsigned)(8 * a.per_xcd)), block(kScatterThreads);
  hipStream_t s = (hipStream_t)stream;
  if (prec == IGAMT_F64)
    hipLaunchKernelGGL(scatter_kernel<double>, grid, block, 0, s, a);
  else
    hipLaunchKernelGGL(scatter_kernel<float>, grid, block, 0, s, a);
  IGAMT_LAUNCH_CHECK();
  return IGAMT_OK;
}

}  // namespace igamt

using namespace igamt;

extern "C" igamt_status igamt_scatter(igamt_plan *P, igamt_precision prec, const void *d_blocks, void *d_values,
                                      void *stream) {
  if (!P || !d_blocks || !d_values) { set_error("NULL argument"); return IGAMT_EINVAL; }
  if (prec < IGAMT_F64 || prec > IGAMT_F16X3) { set_error("unknown precision"); return IGAMT_EINVAL; }
  igamt_status st = ensure_device(P);
  if (st) return st;
  return launch_scatter(P, prec, d_blocks, d_values, stream);
}
