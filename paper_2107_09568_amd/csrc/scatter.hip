// Stage 3 of the assembly: deterministic scatter of the tile blocks into the
// fixed CSR structure (step 4 of Section 3.2.4).
//
// The three CSR rows of a global control point G_A are contiguous (9 nnb(G_A)
// values: rows a = 0, 1, 2, each listing the neighbours G_B in ascending order
// with b = 0, 1, 2).  Every control point is owned by one tile (the tile whose
// local indices in [0, n-2] hold it; the last tile of a direction also owns the
// closing layer).  One workgroup per tile: the work items are the (G_A, rank of
// G_B) pairs of the owned points, flattened in CSR order, one 3x3 slot block per
// lane, so consecutive lanes store consecutive column triples of the same rows.
// The tile's 1-D neighbour entries and the row offsets of its points are staged
// in LDS first.  For each slot block the contributing tiles (1, 2, 4 or 8:
// products of the per-direction contributor lists) are summed in ascending tile
// index, so the result is bitwise reproducible and no atomics are used.  Tiles
// are handed out in an XCD-aware order (consecutive tiles on one XCD), so the
// blocks of a tile's neighbours are usually still in that XCD's L2.
#include <algorithm>

#include "device_common.h"

namespace igamt {

struct ScatterArgs {
  const Pair1D *p[3];
  const int32_t *off[3];
  const int64_t *pre[3];
  int NG[3];
  int tiles[3];
  int nT[3];
  int pT[3];
  int S[3];
  const int32_t *lut;
  int64_t M, n_tiles, per_xcd;
  int max_entries;   // LDS capacity for one direction's owned 1-D entries
  int max_own;       // LDS capacity for owned control points
  const void *blocks;
  void *values;
};

template <typename T>
__global__ __launch_bounds__(256) void scatter_kernel(ScatterArgs a) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  Pair1D *ent = (Pair1D *)smem;                                   // [3][max_entries]
  int64_t *rowbase = (int64_t *)(ent + 3 * a.max_entries);        // [max_own] 9 * before(G)
  int32_t *pref = (int32_t *)(rowbase + a.max_own);               // [max_own + 1] prefix of nnb
  int32_t *offl = pref + a.max_own + 1;                           // [3][max_own + 1] local entry offsets

  const int64_t w = blockIdx.x;
  const int64_t tile = (w & 7) * a.per_xcd + (w >> 3);
  if (tile >= a.n_tiles) return;
  const int tt[3] = {(int)(tile % a.tiles[0]), (int)((tile / a.tiles[0]) % a.tiles[1]),
                     (int)(tile / ((int64_t)a.tiles[0] * a.tiles[1]))};
  int g0[3], cnt[3], e0[3], ne[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    g0[k] = tt[k] * (a.nT[k] - 1);
    cnt[k] = a.nT[k] - 1 + (tt[k] == a.tiles[k] - 1 ? 1 : 0);
    e0[k] = a.off[k][g0[k]];
    ne[k] = a.off[k][g0[k] + cnt[k]] - e0[k];
  }
  const int n_own = cnt[0] * cnt[1] * cnt[2];
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    for (int i = tid; i < ne[k]; i += 256) ent[k * a.max_entries + i] = a.p[k][e0[k] + i];
    for (int i = tid; i <= cnt[k]; i += 256) offl[k * (a.max_own + 1) + i] = a.off[k][g0[k] + i] - e0[k];
  }
  const int64_t SX = a.pre[0][a.NG[0]], SY = a.pre[1][a.NG[1]];
  for (int o = tid; o < n_own; o += 256) {
    const int gx = g0[0] + o % cnt[0], gy = g0[1] + (o / cnt[0]) % cnt[1], gz = g0[2] + o / (cnt[0] * cnt[1]);
    const int64_t cy = a.pre[1][gy + 1] - a.pre[1][gy], cz = a.pre[2][gz + 1] - a.pre[2][gz];
    const int64_t cx = a.pre[0][gx + 1] - a.pre[0][gx];
    rowbase[o] = 9 * (a.pre[2][gz] * SY * SX + cz * (a.pre[1][gy] * SX + cy * a.pre[0][gx]));
    pref[o + 1] = (int32_t)(cx * cy * cz);
  }
  __syncthreads();
  if (tid == 0) {
    pref[0] = 0;
    for (int o = 0; o < n_own; ++o) pref[o + 1] += pref[o];
  }
  __syncthreads();

  const int64_t S3 = (int64_t)a.S[0] * a.S[1] * a.S[2];
  const T *blk = (const T *)a.blocks;
  T *out = (T *)a.values;
  const int W = pref[n_own];
  const Pair1D *EX = ent, *EY = ent + a.max_entries, *EZ = ent + 2 * a.max_entries;
  const int32_t *OX = offl, *OY = offl + (a.max_own + 1), *OZ = offl + 2 * (a.max_own + 1);
  for (int i = tid; i < W; i += 256) {
    int lo = 0, hi = n_own;          // pref[lo] <= i < pref[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (pref[mid] <= i) lo = mid; else hi = mid;
    }
    const int o = lo, rank = i - pref[o];
    const int ox = o % cnt[0], oy = (o / cnt[0]) % cnt[1], oz = o / (cnt[0] * cnt[1]);
    const int cx = OX[ox + 1] - OX[ox], cy = OY[oy + 1] - OY[oy];
    const int nnb = pref[o + 1] - pref[o];
    const int kx = rank % cx, r2 = rank / cx;
    const int ky = r2 % cy, kz = r2 / cy;
    const Pair1D &X = EX[OX[ox] + kx], &Y = EY[OY[oy] + ky], &Z = EZ[OZ[oz] + kz];
    T v[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) v[k] = (T)0;
    for (int iz = 0; iz < Z.ntile; ++iz)
      for (int iy = 0; iy < Y.ntile; ++iy)
        for (int ix = 0; ix < X.ntile; ++ix) {
          const int64_t t = X.tile[ix] + (int64_t)a.tiles[0] * (Y.tile[iy] + (int64_t)a.tiles[1] * Z.tile[iz]);
          const int A = X.li[ix] + a.nT[0] * (Y.li[iy] + a.nT[1] * Z.li[iz]);
          const int B = X.lj[ix] + a.nT[0] * (Y.lj[iy] + a.nT[1] * Z.lj[iz]);
          if (A <= B) {
            const int d = ((Z.lj[iz] - Z.li[iz] + a.pT[2]) * a.S[1] + (Y.lj[iy] - Y.li[iy] + a.pT[1])) * a.S[0] +
                          (X.lj[ix] - X.li[ix] + a.pT[0]);
            const T *src = blk + (t * a.M + a.lut[A * S3 + d]) * 9;
#pragma unroll
            for (int k = 0; k < 9; ++k) v[k] += src[k];
          } else {
            const int d = ((Z.li[iz] - Z.lj[iz] + a.pT[2]) * a.S[1] + (Y.li[iy] - Y.lj[iy] + a.pT[1])) * a.S[0] +
                          (X.li[ix] - X.lj[ix] + a.pT[0]);
            const T *src = blk + (t * a.M + a.lut[B * S3 + d]) * 9;
#pragma unroll
            for (int aa = 0; aa < 3; ++aa)
#pragma unroll
              for (int bb = 0; bb < 3; ++bb) v[3 * aa + bb] += src[3 * bb + aa];
          }
        }
    T *dst = out + rowbase[o] + 3 * rank;
#pragma unroll
    for (int aa = 0; aa < 3; ++aa)
#pragma unroll
      for (int bb = 0; bb < 3; ++bb) dst[3 * aa * nnb + bb] = v[3 * aa + bb];
  }
}

static size_t scatter_lds(int max_entries, int max_own) {
  return (size_t)3 * max_entries * sizeof(Pair1D) + (size_t)max_own * 8 + (size_t)(max_own + 1) * 4 +
         (size_t)3 * (max_own + 1) * 4;
}

igamt_status launch_scatter(igamt_plan *P, igamt_precision prec, const void *d_blocks, void *d_values, void *stream) {
  ScatterArgs a;
  int max_entries = 0, max_own = 1;
  for (int k = 0; k < 3; ++k) {
    a.p[k] = P->dev.dir_pairs[k];
    a.off[k] = P->dev.dir_off[k];
    a.pre[k] = P->dev.dir_pre[k];
    a.NG[k] = P->dir[k].NG;
    a.tiles[k] = P->tiles[k];
    a.nT[k] = P->nT[k];
    a.pT[k] = P->pT[k];
    a.S[k] = P->S[k];
    // largest owned range (the last tile owns n points) and its 1-D entries
    const int n = P->nT[k];
    int m = 0;
    for (int t = 0; t < P->tiles[k]; ++t) {
      const int g0 = t * (n - 1), c = n - 1 + (t == P->tiles[k] - 1 ? 1 : 0);
      m = std::max(m, P->dir[k].off[g0 + c] - P->dir[k].off[g0]);
    }
    max_entries = std::max(max_entries, m);
    max_own *= n;
  }
  a.max_entries = max_entries;
  a.max_own = max_own;
  a.lut = P->dev.pair_lut;
  a.M = P->n_pairs;
  a.n_tiles = P->n_tiles;
  a.per_xcd = (P->n_tiles + 7) / 8;
  a.blocks = d_blocks;
  a.values = d_values;
  const size_t shm = scatter_lds(max_entries, max_own);
  if (shm > 160 * 1024) { set_error("tile too large for the scatter kernel's LDS staging"); return IGAMT_EUNSUPPORTED; }
  const dim3 grid((unsigned)(8 * a.per_xcd)), block(256);
  hipStream_t s = (hipStream_t)stream;
  if (prec == IGAMT_F64) {
    if (shm > 65536) IGAMT_HIP(hipFuncSetAttribute((const void *)scatter_kernel<double>,
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    hipLaunchKernelGGL(scatter_kernel<double>, grid, block, shm, s, a);
  } else {
    if (shm > 65536) IGAMT_HIP(hipFuncSetAttribute((const void *)scatter_kernel<float>,
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    hipLaunchKernelGGL(scatter_kernel<float>, grid, block, shm, s, a);
  }
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
