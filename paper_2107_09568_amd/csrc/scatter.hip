// Stage 3 of the assembly: deterministic scatter of the tile blocks into the
// fixed CSR structure (step 4 of Section 3.2.4).
//
// The CSR slots of a pair of global control points (G_A, G_B) form the tensor
// product of three 1-D neighbour lists (one per direction), so one thread per
// (x-entry, y-entry, z-entry) of those lists owns the 3x3 slots of one
// (G_A, G_B) pair.  The contributing tiles (1, 2, 4 or 8) are the products of
// the 1-D contributors; they are visited in ascending tile index, so the sum is
// bitwise reproducible and no atomics are used.  Row start and column rank
// follow from 1-D prefix sums, so no index is read from memory.
#include "device_common.h"

namespace igamt {

struct ScatterArgs {
  const Pair1D *p[3];
  const int64_t *pre[3];
  int64_t E[3];
  int NG[3];
  int tiles[3];
  int nT[3];
  int pT[3];
  int S[3];
  const int32_t *lut;
  int64_t M;
  const void *blocks;
  void *values;
};

template <typename T>
__global__ __launch_bounds__(256) void scatter_kernel(ScatterArgs a) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t total = a.E[0] * a.E[1] * a.E[2];
  if (idx >= total) return;
  const int64_t ex = idx % a.E[0];
  const int64_t r = idx / a.E[0];
  const int64_t ey = r % a.E[1], ez = r / a.E[1];
  const Pair1D X = a.p[0][ex], Y = a.p[1][ey], Z = a.p[2][ez];
  const int64_t SX = a.pre[0][a.NG[0]], SY = a.pre[1][a.NG[1]];
  const int64_t cx = a.pre[0][X.g + 1] - a.pre[0][X.g];
  const int64_t cy = a.pre[1][Y.g + 1] - a.pre[1][Y.g];
  const int64_t cz = a.pre[2][Z.g + 1] - a.pre[2][Z.g];
  const int64_t nnb = cx * cy * cz;
  const int64_t before = a.pre[2][Z.g] * SY * SX + cz * (a.pre[1][Y.g] * SX + cy * a.pre[0][X.g]);
  const int64_t rank = ((int64_t)Z.rank * cy + Y.rank) * cx + X.rank;
  const int64_t base = 9 * before + 3 * rank;
  const int64_t S3 = (int64_t)a.S[0] * a.S[1] * a.S[2];
  const T *blk = (const T *)a.blocks;

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
          const int64_t p = a.lut[A * S3 + d];
          const T *src = blk + (t * a.M + p) * 9;
#pragma unroll
          for (int k = 0; k < 9; ++k) v[k] += src[k];
        } else {
          const int d = ((Z.li[iz] - Z.lj[iz] + a.pT[2]) * a.S[1] + (Y.li[iy] - Y.lj[iy] + a.pT[1])) * a.S[0] +
                        (X.li[ix] - X.lj[ix] + a.pT[0]);
          const int64_t p = a.lut[B * S3 + d];
          const T *src = blk + (t * a.M + p) * 9;
#pragma unroll
          for (int aa = 0; aa < 3; ++aa)
#pragma unroll
            for (int bb = 0; bb < 3; ++bb) v[3 * aa + bb] += src[3 * bb + aa];
        }
      }
  T *out = (T *)a.values;
#pragma unroll
  for (int aa = 0; aa < 3; ++aa)
#pragma unroll
    for (int bb = 0; bb < 3; ++bb) out[base + 3 * aa * nnb + bb] = v[3 * aa + bb];
}

igamt_status launch_scatter(igamt_plan *P, igamt_precision prec, const void *d_blocks, void *d_values, void *stream) {
  ScatterArgs a;
  for (int k = 0; k < 3; ++k) {
    a.p[k] = P->dev.dir_pairs[k];
    a.pre[k] = P->dev.dir_pre[k];
    a.E[k] = (int64_t)P->dir[k].pairs.size();
    a.NG[k] = P->dir[k].NG;
    a.tiles[k] = P->tiles[k];
    a.nT[k] = P->nT[k];
    a.pT[k] = P->pT[k];
    a.S[k] = P->S[k];
  }
  a.lut = P->dev.pair_lut;
  a.M = P->n_pairs;
  a.blocks = d_blocks;
  a.values = d_values;
  const int64_t total = a.E[0] * a.E[1] * a.E[2];
  const dim3 grid((unsigned)((total + 255) / 256)), block(256);
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
