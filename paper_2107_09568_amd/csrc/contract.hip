// Stage 2 of the assembly: the single matrix product of eq. (58),
//   blocks[t][p][ab] = sum_k table[p][k] coef[t][ab][k],
// i.e. C (n_pairs x 9 m_M) = A (n_pairs x K) B (K x 9 m_M), on gfx950 MFMA.
//
// Layout: A row-major [Mp][Kp] and B column-major [n_tiles_pad*9][Kp], so both
// operands are contiguous along k.  A workgroup (4 waves) owns 128 table rows x
// one group of 16 tiles (144 columns); each wave owns 32 rows x 144 columns
// (2 x 9 MFMA 16x16 blocks).  B chunks of 256 bytes per column are staged in
// LDS through registers (next chunk loaded while the current one is consumed);
// each wave reads its A rows straight from global memory (they are not shared
// between waves).  Within a lane group the k index is permuted so that every
// lane loads contiguous k values with one vector load; A and B use the same
// permutation, so the sum over k is unchanged.
//
// Work order is XCD-aware: consecutive workgroups of one XCD take all row
// blocks of one column group, so a column group is fetched from HBM once and
// reused from that XCD's L2 while the whole table stays resident in the
// last-level cache.
#include "device_common.h"

namespace igamt {

constexpr int BM = 128;                 // table rows per workgroup
constexpr int BN = 144;                 // columns per workgroup (16 tiles x 9)
constexpr int CHUNK_BYTES = 256;        // bytes of one B column staged per chunk
constexpr int LDS_ROW = CHUNK_BYTES + 16;

struct ContractArgs {
  const void *A;          // table (hi plane for split modes)
  const void *A2;         // lo plane (split modes)
  const float *Ascale;    // F16X3 inverse row scales
  const void *B;          // coefficients (hi plane)
  const void *B2;         // lo plane
  const float *Bscale;    // F16X3 inverse column scales [n_tiles_pad][9]
  void *out;              // [n_tiles][M][9]
  int64_t M, Kp, n_tiles;
  int n_mblk, n_groups;
};

template <int MODE>
struct Mode;
template <>
struct Mode<IGAMT_F64> {
  using E = double;                      // stored element
  using O = double;
  using Acc = d4;
  static constexpr int KCH = 32;         // k per chunk (256 B of doubles)
  static constexpr int KSTEP = 16;       // k consumed per lane-load step
};
template <>
struct Mode<IGAMT_F32> {
  using E = float;
  using O = float;
  using Acc = f4;
  static constexpr int KCH = 64;
  static constexpr int KSTEP = 16;
};
template <>
struct Mode<IGAMT_BF16X3> {
  using E = uint16_t;
  using O = float;
  using Acc = f4;
  static constexpr int KCH = 64;         // 128 B hi + 128 B lo per column
  static constexpr int KSTEP = 32;
};
template <>
struct Mode<IGAMT_F16X3> {
  using E = uint16_t;
  using O = float;
  using Acc = f4;
  static constexpr int KCH = 64;
  static constexpr int KSTEP = 32;
};

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int MODE>
__device__ inline void load_chunk_regs(const ContractArgs &a, int64_t grp, int64_t k0, int tid, u32x4 (&r)[9]) {
  // 144 columns x 16 pieces of 16 B = 2304 pieces, 9 per thread
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int pc = tid + 256 * i;
    const int n = pc >> 4, j = pc & 15;
    const int64_t col = grp * BN + n;
    if constexpr (MODE == IGAMT_F64 || MODE == IGAMT_F32) {
      using E = typename Mode<MODE>::E;
      const char *src = (const char *)((const E *)a.B + col * a.Kp + k0) + 16 * j;
      r[i] = *(const u32x4 *)src;
    } else {
      const uint16_t *plane = (j < 8) ? (const uint16_t *)a.B : (const uint16_t *)a.B2;
      const char *src = (const char *)(plane + col * a.Kp + k0) + 16 * (j & 7);
      r[i] = *(const u32x4 *)src;
    }
  }
}

__device__ inline void store_chunk_lds(char *lds, int tid, const u32x4 (&r)[9]) {
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int pc = tid + 256 * i;
    const int n = pc >> 4, j = pc & 15;
    *(u32x4 *)(lds + n * LDS_ROW + 16 * j) = r[i];
  }
}

template <int MODE>
__global__ __launch_bounds__(256, 1) void contract_kernel(ContractArgs a) {
  using M_ = Mode<MODE>;
  using Acc = typename M_::Acc;
  using O = typename M_::O;
  __shared__ __attribute__((aligned(16))) char lds[BN * LDS_ROW];

  const int wg = blockIdx.x;
  const int xcd = wg & 7, local = wg >> 3;
  const int64_t grp = (int64_t)(local / a.n_mblk) * 8 + xcd;
  const int mb = local % a.n_mblk;
  if (grp >= a.n_groups) return;

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int l16 = lane & 15, kq = lane >> 4;
  const int64_t row0 = (int64_t)mb * BM + wave * 32;

  Acc acc[2][9];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 9; ++ni) acc[mi][ni] = Acc{0, 0, 0, 0};

  u32x4 pre[9];
  load_chunk_regs<MODE>(a, grp, 0, tid, pre);

  for (int64_t k0 = 0; k0 < a.Kp; k0 += M_::KCH) {
    __syncthreads();
    store_chunk_lds(lds, tid, pre);
    __syncthreads();
    if (k0 + M_::KCH < a.Kp) load_chunk_regs<MODE>(a, grp, k0 + M_::KCH, tid, pre);

#pragma unroll
    for (int ks = 0; ks < M_::KCH; ks += M_::KSTEP) {
      // All fragments of the k-step are loaded first; MFMAs are then issued so that
      // consecutive instructions update different accumulators (18 apart).
      if constexpr (MODE == IGAMT_F64 || MODE == IGAMT_F32) {
        using E = typename Mode<MODE>::E;
        E av[2][4], bv[9][4];
#pragma unroll
        for (int mi = 0; mi < 2; ++mi) {
          const E *src = (const E *)a.A + (row0 + mi * 16 + l16) * a.Kp + k0 + ks + 4 * kq;
#pragma unroll
          for (int s = 0; s < 4; ++s) av[mi][s] = src[s];
        }
#pragma unroll
        for (int ni = 0; ni < 9; ++ni) {
          const E *bp = (const E *)(lds + (ni * 16 + l16) * LDS_ROW) + ks + 4 * kq;
#pragma unroll
          for (int s = 0; s < 4; ++s) bv[ni][s] = bp[s];
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int ni = 0; ni < 9; ++ni) {
              if constexpr (MODE == IGAMT_F64)
                acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[mi][s], bv[ni][s], acc[mi][ni], 0, 0, 0);
              else
                acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[mi][s], bv[ni][s], acc[mi][ni], 0, 0, 0);
            }
      } else {
        // split modes: lane holds 8 consecutive k (16 B) of hi and lo; products lo*hi, hi*lo, hi*hi
        using V8 = typename std::conditional<MODE == IGAMT_BF16X3, bf16x8, f16x8>::type;
        V8 ah[2], al[2], bh[9], bl[9];
#pragma unroll
        for (int mi = 0; mi < 2; ++mi) {
          const int64_t off = (row0 + mi * 16 + l16) * a.Kp + k0 + ks + 8 * kq;
          ah[mi] = *(const V8 *)((const uint16_t *)a.A + off);
          al[mi] = *(const V8 *)((const uint16_t *)a.A2 + off);
        }
#pragma unroll
        for (int ni = 0; ni < 9; ++ni) {
          const char *bp = lds + (ni * 16 + l16) * LDS_ROW + (ks + 8 * kq) * 2;
          bh[ni] = *(const V8 *)bp;
          bl[ni] = *(const V8 *)(bp + 128);
        }
#pragma unroll
        for (int pr = 0; pr < 3; ++pr)
#pragma unroll
          for (int mi = 0; mi < 2; ++mi)
#pragma unroll
            for (int ni = 0; ni < 9; ++ni) {
              const V8 &x = pr == 0 ? al[mi] : ah[mi];
              const V8 &y = pr == 1 ? bl[ni] : bh[ni];
              if constexpr (MODE == IGAMT_BF16X3)
                acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, acc[mi][ni], 0, 0, 0);
              else
                acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_f16(x, y, acc[mi][ni], 0, 0, 0);
            }
      }
    }
  }

  // Epilogue.  Lane holds C[row][col l16] of each 16x16 block with row = 4 kq + r for the
  // FP32-accumulating instructions and row = kq + 4 r for the FP64 one (measured layouts).
  // The wave's 32 x 144 tile is transposed through LDS so that each tile's 32 rows x 9 values
  // (contiguous in the block array) are written as whole cache lines.
  O *out = (O *)a.out;
  O *stage = (O *)lds;
  constexpr int PER_ROUND = (int)(sizeof(lds) / (32 * 144 * sizeof(O)));   // waves staged per round
  for (int w0 = 0; w0 < 4; w0 += PER_ROUND) {
    __syncthreads();
    if (wave >= w0 && wave < w0 + PER_ROUND) {
      O *ws = stage + (wave - w0) * 32 * 144;
#pragma unroll
      for (int ni = 0; ni < 9; ++ni) {
        const int n = ni * 16 + l16;
        const int tl = n / 9, ab = n - 9 * tl;
        float cs = 1.0f;
        if constexpr (MODE == IGAMT_F16X3) cs = a.Bscale[(grp * 16 + tl) * 9 + ab];
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int ml = mi * 16 + (MODE == IGAMT_F64 ? kq + 4 * r : 4 * kq + r);
            O v = (O)acc[mi][ni][r];
            if constexpr (MODE == IGAMT_F16X3) v = v * (a.Ascale[mb * BM + wave * 32 + ml] * cs);
            ws[(tl * 32 + ml) * 9 + ab] = v;
          }
      }
    }
    __syncthreads();
    for (int wv = w0; wv < w0 + PER_ROUND && wv < 4; ++wv) {
      const O *ws = stage + (wv - w0) * 32 * 144;
      const int64_t r0 = (int64_t)mb * BM + wv * 32;
      const int rows = (int)min((int64_t)32, a.M - r0);
      if (rows <= 0) continue;
      for (int e = tid; e < 16 * 288; e += 256) {
        const int tl = e / 288, j = e - 288 * tl;
        const int64_t t = grp * 16 + tl;
        if (t < a.n_tiles && j < rows * 9) out[(t * a.M + r0) * 9 + j] = ws[tl * 288 + j];
      }
    }
  }
}

igamt_status launch_contract(igamt_plan *P, igamt_precision prec, const void *d_coef, void *d_blocks, void *stream) {
  if (!P->tables_ready) { set_error("tables are not built or set"); return IGAMT_ESTATE; }
  ContractArgs a;
  const int64_t MK = P->Mp * P->Kp;
  const int64_t plane = P->n_tiles_pad * 9 * P->Kp;
  a.M = P->n_pairs;
  a.Kp = P->Kp;
  a.n_tiles = P->n_tiles;
  a.n_mblk = (int)(P->Mp / BM);
  a.n_groups = (int)P->n_groups;
  a.out = d_blocks;
  a.A2 = nullptr;
  a.B2 = nullptr;
  a.Ascale = nullptr;
  a.Bscale = nullptr;
  a.B = d_coef;
  switch (prec) {
    case IGAMT_F64: a.A = P->dev.table; break;
    case IGAMT_F32: a.A = P->dev.table_f32; break;
    case IGAMT_BF16X3:
      a.A = P->dev.table_bf;
      a.A2 = P->dev.table_bf + MK;
      a.B2 = (const uint16_t *)d_coef + plane;
      break;
    case IGAMT_F16X3:
      a.A = P->dev.table_h;
      a.A2 = P->dev.table_h + MK;
      a.Ascale = P->dev.table_h_scale;
      a.B2 = (const uint16_t *)d_coef + plane;
      a.Bscale = (const float *)((const uint16_t *)d_coef + 2 * plane);
      break;
    default: set_error("unknown precision"); return IGAMT_EINVAL;
  }
  const int64_t groups8 = (P->n_groups + 7) / 8 * 8;
  const dim3 grid((unsigned)(a.n_mblk * groups8)), block(256);
  hipStream_t s = (hipStream_t)stream;
  switch (prec) {
    case IGAMT_F64: hipLaunchKernelGGL(contract_kernel<IGAMT_F64>, grid, block, 0, s, a); break;
    case IGAMT_F32: hipLaunchKernelGGL(contract_kernel<IGAMT_F32>, grid, block, 0, s, a); break;
    case IGAMT_BF16X3: hipLaunchKernelGGL(contract_kernel<IGAMT_BF16X3>, grid, block, 0, s, a); break;
    case IGAMT_F16X3: hipLaunchKernelGGL(contract_kernel<IGAMT_F16X3>, grid, block, 0, s, a); break;
  }
  IGAMT_LAUNCH_CHECK();
  return IGAMT_OK;
}

}  // namespace igamt

using namespace igamt;

extern "C" igamt_status igamt_contract(igamt_plan *P, igamt_precision prec, const void *d_coef, void *d_blocks,
                                       void *stream) {
  if (!P || !d_coef || !d_blocks) { set_error("NULL argument"); return IGAMT_EINVAL; }
  if (prec < IGAMT_F64 || prec > IGAMT_F16X3) { set_error("unknown precision"); return IGAMT_EINVAL; }
  igamt_status st = ensure_device(P);
  if (st) return st;
  return launch_contract(P, prec, d_coef, d_blocks, stream);
}

extern "C" igamt_status igamt_assemble(igamt_plan *P, double E, double nu, igamt_precision prec, void *d_values,
                                       void *d_workspace, void *stream) {
  if (!P || !d_values || !d_workspace) { set_error("NULL argument"); return IGAMT_EINVAL; }
  if (prec < IGAMT_F64 || prec > IGAMT_F16X3) { set_error("unknown precision"); return IGAMT_EINVAL; }
  igamt_status st = ensure_device(P);
  if (st) return st;
  if (!P->tables_ready) { set_error("tables are not built or set"); return IGAMT_ESTATE; }
  char *ws = (char *)d_workspace;
  void *coef = ws;
  void *blocks = ws + coef_bytes(P, prec);
  if ((st = launch_fit(P, E, nu, prec, coef, stream))) return st;
  if ((st = launch_contract(P, prec, coef, blocks, stream))) return st;
  return launch_scatter(P, prec, blocks, d_values, stream);
}
