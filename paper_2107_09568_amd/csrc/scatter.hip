// Stage 3 of the assembly: deterministic scatter of the tile blocks into the
// fixed CSR structure (step 4 of Section 3.2.4).
//
// The three CSR rows of a global control point G_A are contiguous (9 nnb(G_A)
// values: rows a = 0, 1, 2, each listing the neighbours G_B in ascending order
// with b = 0, 1, 2).  Every control point is owned by one tile (the tile whose
// local indices in [0, n-2] hold it; the last tile of a direction also owns the
// closing layer).  One workgroup per tile loops over the tile's owned x-lines
// of control points; for each line
//  1. it stages in LDS the tile's block records that the line's rows read: the
//     pairs (A, B) with A in the line (one contiguous range, pairs being sorted
//     by A) and the pairs (B, A) with A in the line and B < A (a fixed list), so
//     every record of the tile is fetched once as an "upper" record and once as
//     a "lower" one, the second time usually from L2; the line's rows of the
//     slot table are staged with them;
//  2. lanes sweep the (G_A, rank of G_B) slot blocks of the line's rows in CSR
//     order, so stores are coalesced; contributions of the own tile come from
//     LDS, those of neighbouring tiles (control points on shared faces) from
//     global memory, always summed in ascending tile index.
// The result is bitwise reproducible and no atomics are used.  Tiles are
// handed out XCD-aware (consecutive tiles on one XCD share neighbours' blocks).
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
  const int32_t *lut;        // pair index of (A, B), A <= B
  const int32_t *slot;       // staging slot of (A, B) in A's x-line
  const int32_t *line_up;
  const int32_t *lo_off;
  const int32_t *lo_p;
  int64_t M, n_tiles, per_xcd;
  int n_lines;               // x-lines per tile (n_y n_z)
  int max_records;           // LDS staging capacity (records)
  int max_x_entries;         // LDS capacity for the owned x-range's 1-D entries
  const void *blocks;
  void *values;
};

template <typename T>
__global__ __launch_bounds__(256) void scatter_kernel(ScatterArgs a) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int64_t w = blockIdx.x;
  const int64_t tile = (w & 7) * a.per_xcd + (w >> 3);
  if (tile >= a.n_tiles) return;
  const int tt[3] = {(int)(tile % a.tiles[0]), (int)((tile / a.tiles[0]) % a.tiles[1]),
                     (int)(tile / ((int64_t)a.tiles[0] * a.tiles[1]))};
  int cnt[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) cnt[k] = a.nT[k] - 1 + (tt[k] == a.tiles[k] - 1 ? 1 : 0);
  const int64_t S3 = (int64_t)a.S[0] * a.S[1] * a.S[2];

  T *stage = (T *)smem;                                                       // [max_records][9]
  int32_t *SL = (int32_t *)(smem + (size_t)a.max_records * 9 * sizeof(T));   // [n_x][S3] slot rows of the line
  Pair1D *EX = (Pair1D *)(SL + a.nT[0] * S3);                                 // owned x-range entries
  Pair1D *EY = EX + a.max_x_entries;                                          // entries of gy
  Pair1D *EZ = EY + 2 * a.pT[1] + 1;                                          // entries of gz
  int32_t *OX = (int32_t *)(EZ + 2 * a.pT[2] + 1);                            // [cnt_x + 1] local offsets
  int64_t *RB = (int64_t *)(((uintptr_t)(OX + a.nT[0] + 1) + 7) & ~(uintptr_t)7);   // [cnt_x] row bases
  int32_t *PF = (int32_t *)(RB + a.nT[0]);                                    // [cnt_x + 1] prefix of nnb

  const int tid = threadIdx.x;
  const T *blk = (const T *)a.blocks;
  T *out = (T *)a.values;
  const int gx0 = tt[0] * (a.nT[0] - 1);
  const int ex0 = a.off[0][gx0], nex = a.off[0][gx0 + cnt[0]] - ex0;
  for (int i = tid; i < nex; i += 256) EX[i] = a.p[0][ex0 + i];
  for (int o = tid; o <= cnt[0]; o += 256) OX[o] = a.off[0][gx0 + o] - ex0;
  const int64_t SX = a.pre[0][a.NG[0]], SY = a.pre[1][a.NG[1]];

  for (int lz = 0; lz < cnt[2]; ++lz)
    for (int ly = 0; ly < cnt[1]; ++ly) {
      const int line = ly + a.nT[1] * lz;
      const int up_lo = a.line_up[2 * line], n_up = a.line_up[2 * line + 1] - up_lo;
      const int lo0 = a.lo_off[line], n_lo = a.lo_off[line + 1] - lo0;
      const int gy = tt[1] * (a.nT[1] - 1) + ly, gz = tt[2] * (a.nT[2] - 1) + lz;
      const int ey0 = a.off[1][gy], cy = a.off[1][gy + 1] - ey0;
      const int ez0 = a.off[2][gz], cz = a.off[2][gz + 1] - ez0;
      __syncthreads();   // previous line done with the staging buffers
      {  // stage the line's records, slot rows and 1-D entries; loads are issued in batches
         // of 8 per thread before any LDS store so that many requests are in flight
        const T *src = blk + ((int64_t)tile * a.M + up_lo) * 9;
        const int nu = n_up * 9;
        for (int b0 = 0; b0 < nu; b0 += 256 * 8) {
          T r[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int e = b0 + u * 256 + tid;
            r[u] = e < nu ? src[e] : (T)0;
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int e = b0 + u * 256 + tid;
            if (e < nu) stage[e] = r[u];
          }
        }
        const int nl = n_lo * 9;
        const T *tb = blk + (int64_t)tile * a.M * 9;
        for (int b0 = 0; b0 < nl; b0 += 256 * 8) {
          int32_t q[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int e = b0 + u * 256 + tid;
            q[u] = e < nl ? a.lo_p[lo0 + e / 9] : 0;
          }
          T r[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int e = b0 + u * 256 + tid;
            r[u] = e < nl ? tb[(int64_t)q[u] * 9 + (e - 9 * (e / 9))] : (T)0;
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int e = b0 + u * 256 + tid;
            if (e < nl) stage[(n_up + e / 9) * 9 + (e - 9 * (e / 9))] = r[u];
          }
        }
        const int32_t *sl = a.slot + (int64_t)line * a.nT[0] * S3;
        const int ns = a.nT[0] * (int)S3;
        for (int b0 = 0; b0 < ns; b0 += 256 * 4) {
          int32_t r[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int e = b0 + u * 256 + tid;
            r[u] = e < ns ? sl[e] : 0;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int e = b0 + u * 256 + tid;
            if (e < ns) SL[e] = r[u];
          }
        }
        if (tid < cy) EY[tid] = a.p[1][ey0 + tid];
        if (tid >= 64 && tid - 64 < cz) EZ[tid - 64] = a.p[2][ez0 + tid - 64];
        if (tid >= 128 && tid - 128 < cnt[0]) {
          const int o = tid - 128;
          const int gx = gx0 + o;
          const int64_t cx = a.pre[0][gx + 1] - a.pre[0][gx];
          RB[o] = 9 * (a.pre[2][gz] * SY * SX + (int64_t)cz * (a.pre[1][gy] * SX + (int64_t)cy * a.pre[0][gx]));
          PF[o + 1] = (int32_t)(cx * cy * cz);
        }
      }
      __syncthreads();
      if (tid == 0) {
        PF[0] = 0;
        for (int o = 0; o < cnt[0]; ++o) PF[o + 1] += PF[o];
      }
      __syncthreads();
      const int W = PF[cnt[0]];
      for (int i = tid; i < W; i += 256) {
        int o = 0;
        while (PF[o + 1] <= i) ++o;
        const int rank = i - PF[o];
        const int cx = OX[o + 1] - OX[o];
        const int nnb = PF[o + 1] - PF[o];
        const int kx = rank % cx, r2 = rank / cx;
        const int ky = r2 % cy, kz = r2 / cy;
        const Pair1D &X = EX[OX[o] + kx], &Y = EY[ky], &Z = EZ[kz];
        T v[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) v[k] = (T)0;
        for (int iz = 0; iz < Z.ntile; ++iz)
          for (int iy = 0; iy < Y.ntile; ++iy)
            for (int ix = 0; ix < X.ntile; ++ix) {
              const int64_t t = X.tile[ix] + (int64_t)a.tiles[0] * (Y.tile[iy] + (int64_t)a.tiles[1] * Z.tile[iz]);
              const int A = X.li[ix] + a.nT[0] * (Y.li[iy] + a.nT[1] * Z.li[iz]);
              const int B = X.lj[ix] + a.nT[0] * (Y.lj[iy] + a.nT[1] * Z.lj[iz]);
              const int dAB = ((Z.lj[iz] - Z.li[iz] + a.pT[2]) * a.S[1] + (Y.lj[iy] - Y.li[iy] + a.pT[1])) * a.S[0] +
                              (X.lj[ix] - X.li[ix] + a.pT[0]);
              const T *src;
              if (t == tile) {
                src = stage + (int64_t)SL[X.li[ix] * S3 + dAB] * 9;   // own tile: A lies in this x-line
              } else if (A <= B) {
                src = blk + (t * a.M + a.lut[A * S3 + dAB]) * 9;
              } else {
                const int dBA = ((Z.li[iz] - Z.lj[iz] + a.pT[2]) * a.S[1] + (Y.li[iy] - Y.lj[iy] + a.pT[1])) * a.S[0] +
                                (X.li[ix] - X.lj[ix] + a.pT[0]);
                src = blk + (t * a.M + a.lut[B * S3 + dBA]) * 9;
              }
              if (A <= B) {
#pragma unroll
                for (int k = 0; k < 9; ++k) v[k] += src[k];
              } else {
#pragma unroll
                for (int aa = 0; aa < 3; ++aa)
#pragma unroll
                  for (int bb = 0; bb < 3; ++bb) v[3 * aa + bb] += src[3 * bb + aa];
              }
            }
        T *dst = out + RB[o] + 3 * rank;
#pragma unroll
        for (int aa = 0; aa < 3; ++aa)
#pragma unroll
          for (int bb = 0; bb < 3; ++bb) dst[3 * aa * nnb + bb] = v[3 * aa + bb];
      }
    }
}

static size_t scatter_lds(const igamt_plan *P, size_t elem, int max_x_entries) {
  size_t b = (size_t)P->max_line_records * 9 * elem;
  b += (size_t)P->nT[0] * P->S[0] * P->S[1] * P->S[2] * 4;
  b += (size_t)(max_x_entries + 2 * P->pT[1] + 1 + 2 * P->pT[2] + 1) * sizeof(Pair1D);
  b += (size_t)(P->nT[0] + 1) * 4 + 8;
  b += (size_t)P->nT[0] * 8 + (size_t)(P->nT[0] + 1) * 4;
  return b + 64;
}

igamt_status launch_scatter(igamt_plan *P, igamt_precision prec, const void *d_blocks, void *d_values, void *stream) {
  ScatterArgs a;
  int max_x_entries = 0;
  for (int k = 0; k < 3; ++k) {
    a.p[k] = P->dev.dir_pairs[k];
    a.off[k] = P->dev.dir_off[k];
    a.pre[k] = P->dev.dir_pre[k];
    a.NG[k] = P->dir[k].NG;
    a.tiles[k] = P->tiles[k];
    a.nT[k] = P->nT[k];
    a.pT[k] = P->pT[k];
    a.S[k] = P->S[k];
  }
  {
    const int n = P->nT[0];
    for (int t = 0; t < P->tiles[0]; ++t) {
      const int g0 = t * (n - 1), c = n - 1 + (t == P->tiles[0] - 1 ? 1 : 0);
      max_x_entries = std::max(max_x_entries, P->dir[0].off[g0 + c] - P->dir[0].off[g0]);
    }
  }
  a.lut = P->dev.pair_lut;
  a.slot = P->dev.slot_lut;
  a.line_up = P->dev.line_up;
  a.lo_off = P->dev.line_lo_off;
  a.lo_p = P->dev.line_lo_p;
  a.M = P->n_pairs;
  a.n_tiles = P->n_tiles;
  a.n_lines = P->nT[1] * P->nT[2];
  a.per_xcd = (P->n_tiles + 7) / 8;
  a.max_records = P->max_line_records;
  a.max_x_entries = max_x_entries;
  a.blocks = d_blocks;
  a.values = d_values;
  const size_t elem = prec == IGAMT_F64 ? 8 : 4;
  const size_t shm = scatter_lds(P, elem, max_x_entries);
  if (shm > 160 * 1024 || P->nT[0] > 128) {
    set_error("tile too large for the scatter kernel's LDS staging");
    return IGAMT_EUNSUPPORTED;
  }
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
