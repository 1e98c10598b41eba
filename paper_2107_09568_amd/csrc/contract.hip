// Stage 2 of the assembly: the single matrix product of eq. (58),
//   blocks[t][p][ab] = sum_k table[p][k] coef[t][ab][k],
// i.e. C (n_pairs x 9 m_M) = A (n_pairs x K) B (K x 9 m_M), on gfx950 MFMA.
//
// Layout: A row-major [Mp][Kp] and B column-major [n_tiles_pad*9][Kp], so both
// operands are contiguous along k.  A workgroup owns 128 table rows x one group
// of 16 tiles (144 columns).  Its waves split the rows: each wave owns WM 16-row
// blocks x 144 columns (WM x 9 MFMA 16x16 blocks), WM = 1 with 8 waves for FP64,
// WM = 2 with 4 waves (two workgroups per CU) for FP32 and the split modes.  Every
// shape keeps a wave within the 256 registers that leave the accumulators in
// VGPRs: the FP64 MFMA runs about 2.3x slower, the BF16 one about 1.4x slower,
// when it accumulates in AGPRs.
//
// B chunks (64 k values per column) are staged in LDS through registers, one chunk
// ahead, into alternating buffers; each wave reads its A rows straight from
// global memory one k-step ahead (they are not shared between waves).  Within a
// lane group the k index is permuted so that every lane loads contiguous k
// values with one vector load; A and B use the same permutation, so the sum over
// k is unchanged.
//
// Work order is XCD-aware: consecutive workgroups of one XCD take all row
// blocks of one column group, so a column group is fetched from HBM once and
// reused from that XCD's L2 while the whole table stays resident in the
// last-level cache.
#include <algorithm>
#include <atomic>
#include <numeric>

#include "device_common.h"

namespace igamt {

constexpr int BN = 144;                 // columns per workgroup (16 tiles x 9)
#ifndef NW_F64
#define NW_F64 8
#endif
#ifndef KCH_F64
#define KCH_F64 32
#endif

struct ContractArgs {
  const void *A;          // table (hi plane for split modes)
  const void *A2;         // lo plane (split modes)
  const float *Ascale;    // F16X3 inverse row scales
  const void *B;          // coefficients (hi plane)
  const void *B2;         // lo plane
  const float *Bscale;    // F16X3 inverse column scales [n_tiles_pad][9]
  void *out;              // [n_tiles][M][9]
  int64_t M, Kp, n_tiles;
  int n_mblk, n_groups;  // row blocks; groups of this launch
  int64_t grp0;          // first group of this launch
};

template <int MODE>
struct Mode;
template <>
struct Mode<IGAMT_F64> {
  using E = double;                      // stored element
  using O = double;
  using Acc = d4;
  static constexpr int KCH = KCH_F64;    // k per staged chunk (256 B of doubles per column)
  static constexpr int KSTEP = 16;       // k consumed per lane-load step
  static constexpr int WM = 1;           // 16-row blocks per wave
  static constexpr int NW = NW_F64;      // waves per workgroup
};
template <>
struct Mode<IGAMT_F32> {
  using E = float;
  using O = float;
  using Acc = f4;
  static constexpr int KCH = 64;
  static constexpr int KSTEP = 16;
  static constexpr int WM = 2;
  static constexpr int NW = 4;
};
template <>
struct Mode<IGAMT_BF16X3> {
  using E = uint16_t;
  using O = float;
  using Acc = f4;
  static constexpr int KCH = 64;         // 128 B hi + 128 B lo per column
  static constexpr int KSTEP = 32;
  static constexpr int WM = 2;
  static constexpr int NW = 4;
};
template <>
struct Mode<IGAMT_F16X3> {
  using E = uint16_t;
  using O = float;
  using Acc = f4;
  static constexpr int KCH = 64;
  static constexpr int KSTEP = 32;
  static constexpr int WM = 2;
  static constexpr int NW = 4;
};
template <int MODE>
constexpr int kWaves = Mode<MODE>::NW;                // waves per workgroup
template <int MODE>
constexpr int kMinGroups = MODE != IGAMT_F64 ? 2 : 1;   // workgroups per CU
template <int MODE>
constexpr int kBM = 16 * Mode<MODE>::WM * Mode<MODE>::NW;   // table rows per workgroup
template <int MODE>
constexpr bool kPersist = MODE == IGAMT_F64;   // one workgroup per CU: a persistent loop over items
#ifndef IGAMT_SUPER
#define IGAMT_SUPER 8
#endif
constexpr int kSuper = IGAMT_SUPER;            // column groups per super-group of the item order
template <int MODE>
constexpr int kChunkBytes =   // bytes of one B column per staged chunk (split modes: hi then lo half)
    Mode<MODE>::KCH * ((MODE == IGAMT_F64 || MODE == IGAMT_F32) ? (int)sizeof(typename Mode<MODE>::E) : 4);
template <int MODE>
constexpr int kLdsRow = kChunkBytes<MODE> + 16;   // padded LDS row of one column
template <int MODE>
constexpr int kPpc = kChunkBytes<MODE> / 16;      // 16-byte pieces per column
template <int MODE>
constexpr int kPieces = BN * kPpc<MODE>;          // 16-byte pieces of one staged chunk
template <int MODE>
constexpr int kPre = (kPieces<MODE> + 64 * kWaves<MODE> - 1) / (64 * kWaves<MODE>);   // staged pieces per thread

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int MODE>
__device__ inline void load_chunk_regs(const ContractArgs &a, int64_t grp, int64_t k0, int tid, u32x4 (&r)[kPre<MODE>]) {
  // 144 columns x 16 pieces of 16 B; a piece index past the chunk re-reads the first column (unused)
  constexpr int NT = 64 * kWaves<MODE>;
#pragma unroll
  for (int i = 0; i < kPre<MODE>; ++i) {
    int pc = tid + NT * i;
    if (kPieces<MODE> % NT != 0 && pc >= kPieces<MODE>) pc = tid % kPpc<MODE>;
    const int n = pc / kPpc<MODE>, j = pc % kPpc<MODE>;
    const int64_t col = grp * BN + n;
    if constexpr (MODE == IGAMT_F64 || MODE == IGAMT_F32) {
      using E = typename Mode<MODE>::E;
      const char *src = (const char *)((const E *)a.B + col * a.Kp + k0) + 16 * j;
      r[i] = *(const u32x4 *)src;
    } else {
      constexpr int H = kPpc<MODE> / 2;   // pieces of the hi half
      const uint16_t *plane = (j < H) ? (const uint16_t *)a.B : (const uint16_t *)a.B2;
      const char *src = (const char *)(plane + col * a.Kp + k0) + 16 * (j % H);
      r[i] = *(const u32x4 *)src;
    }
  }
}

template <int MODE>
__device__ inline void store_chunk_lds(char *lds, int tid, const u32x4 (&r)[kPre<MODE>]) {
  constexpr int NT = 64 * kWaves<MODE>;
#pragma unroll
  for (int i = 0; i < kPre<MODE>; ++i) {
    const int pc = tid + NT * i;
    if (kPieces<MODE> % NT != 0 && pc >= kPieces<MODE>) break;
    const int n = pc / kPpc<MODE>, j = pc % kPpc<MODE>;
    *(u32x4 *)(lds + n * kLdsRow<MODE> + 16 * j) = r[i];
  }
}


// Operand fragments of one k-step of one wave: 2 row blocks of A (global) and 9 column blocks of B (LDS).
template <int MODE, bool SPLIT = (MODE == IGAMT_BF16X3 || MODE == IGAMT_F16X3)>
struct Frag;
template <int MODE>
struct Frag<MODE, false> {
  // A is prefetched a k-step ahead; B fragments are read from LDS inside mma (FP64 one k-slice
  // ahead): two whole fragment sets do not fit the register file next to the accumulators.
  using E = typename Mode<MODE>::E;
  static constexpr int WM = Mode<MODE>::WM;
  E av[WM][4];
  __device__ inline void load_a(const ContractArgs &a, int64_t row0, int l16, int kq, int64_t k) {
#pragma unroll
    for (int mi = 0; mi < WM; ++mi) {
      const E *src = (const E *)a.A + (row0 + mi * 16 + l16) * a.Kp + k + 4 * kq;
#pragma unroll
      for (int s = 0; s < 4; ++s) av[mi][s] = src[s];
    }
  }
  // consecutive MFMAs update different accumulators (9 or 18 apart)
  __device__ inline void mma(typename Mode<MODE>::Acc (&acc)[WM][9], const char *buf, int l16, int kq, int kk) const {
    if constexpr (MODE == IGAMT_F64) {
      // one 8-byte read per column block and k-slice, the next slice's reads issued before this
      // slice's MFMAs (16-byte reads of two slices at once avoid the bank conflicts of these reads,
      // 4 lanes on each bank pair, but lose the look-ahead: 9.05-9.15 against 8.95 ms)
      E b[2][9];
#pragma unroll
      for (int ni = 0; ni < 9; ++ni) b[0][ni] = *((const E *)(buf + (ni * 16 + l16) * kLdsRow<MODE>) + kk + 4 * kq);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        if (s + 1 < 4) {
#pragma unroll
          for (int ni = 0; ni < 9; ++ni)
            b[(s + 1) & 1][ni] = *((const E *)(buf + (ni * 16 + l16) * kLdsRow<MODE>) + kk + 4 * kq + s + 1);
        }
#pragma unroll
        for (int mi = 0; mi < WM; ++mi)
#pragma unroll
          for (int ni = 0; ni < 9; ++ni)
            acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[mi][s], b[s & 1][ni], acc[mi][ni], 0, 0, 0);
      }
    } else {
      // FP32: lane (l16, kq) takes the four k = kk + 4 kq + s in one 16-byte read per column block;
      // with the 16-byte row padding a quarter wave (l16 = 0..15) reads 16 different 4-bank groups,
      // so the reads are free of bank conflicts (4-byte reads put 4 lanes on each bank)
      typedef float f4v __attribute__((ext_vector_type(4)));
      f4v b[9];
#pragma unroll
      for (int ni = 0; ni < 9; ++ni) b[ni] = *(const f4v *)((const E *)(buf + (ni * 16 + l16) * kLdsRow<MODE>) + kk + 4 * kq);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int mi = 0; mi < WM; ++mi)
#pragma unroll
          for (int ni = 0; ni < 9; ++ni)
            acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[mi][s], b[ni][s], acc[mi][ni], 0, 0, 0);
    }
  }
};
template <int MODE>
struct Frag<MODE, true> {
  // Split modes: lane holds 8 consecutive k (16 B) of the hi and lo planes; products lo*hi, hi*lo,
  // hi*hi.  Only the A fragment is prefetched a k-step ahead; B fragments are read from LDS two
  // column blocks at a time inside mma (the next pair while the current pair's MFMAs run), which
  // keeps a wave within the 256 registers that leave the accumulators in VGPRs.
  using V8 = typename std::conditional<MODE == IGAMT_BF16X3, bf16x8, f16x8>::type;
  static constexpr int WM = Mode<MODE>::WM;
  V8 ah[WM], al[WM];
  __device__ inline void load_a(const ContractArgs &a, int64_t row0, int l16, int kq, int64_t k) {
#pragma unroll
    for (int mi = 0; mi < WM; ++mi) {
      const int64_t off = (row0 + mi * 16 + l16) * a.Kp + k + 8 * kq;
      ah[mi] = *(const V8 *)((const uint16_t *)a.A + off);
      al[mi] = *(const V8 *)((const uint16_t *)a.A2 + off);
    }
  }
  __device__ static inline void read_pair(const char *buf, int l16, int kq, int kk, int n0, V8 (&h)[2], V8 (&l)[2]) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int ni = min(n0 + q, 8);
      const char *bp = buf + (ni * 16 + l16) * kLdsRow<MODE> + (kk + 8 * kq) * 2;
      h[q] = *(const V8 *)bp;
      l[q] = *(const V8 *)(bp + kChunkBytes<MODE> / 2);
    }
  }
  __device__ inline void mma(f4 (&acc)[WM][9], const char *buf, int l16, int kq, int kk) const {
    V8 bh[2][2], bl[2][2];
    read_pair(buf, l16, kq, kk, 0, bh[0], bl[0]);
#pragma unroll
    for (int pi = 0; pi < 5; ++pi) {
      if (pi + 1 < 5) read_pair(buf, l16, kq, kk, 2 * (pi + 1), bh[(pi + 1) & 1], bl[(pi + 1) & 1]);
#pragma unroll
      for (int pr = 0; pr < 3; ++pr)
#pragma unroll
        for (int mi = 0; mi < WM; ++mi)
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const int ni = 2 * pi + q;
            if (ni < 9) {
              const V8 &x = pr == 0 ? al[mi] : ah[mi];
              const V8 &y = pr == 1 ? bl[pi & 1][q] : bh[pi & 1][q];
              if constexpr (MODE == IGAMT_BF16X3)
                acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, acc[mi][ni], 0, 0, 0);
              else
                acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_f16(x, y, acc[mi][ni], 0, 0, 0);
            }
          }
    }
  }
};

template <int MODE>
__global__ __launch_bounds__(64 * kWaves<MODE>, kMinGroups<MODE>) void contract_kernel(ContractArgs a) {
  using M_ = Mode<MODE>;
  constexpr int WM = M_::WM;
  using Acc = typename M_::Acc;
  using O = typename M_::O;
  constexpr int BUF = BN * kLdsRow<MODE>;
  constexpr int SPC = M_::KCH / M_::KSTEP;       // k-steps per staged chunk
  __shared__ __attribute__((aligned(16))) char lds[2 * BUF];

  // Work items (row block mb, column group grp): the column groups grp0 + 8 j + x belong to XCD x
  // and are visited in the order below.  Workgroup w runs items
  // l = w / 8, w / 8 + S, w / 8 + 2 S, ... of XCD w % 8 (S = workgroups per XCD): one item each
  // when the grid covers all items, or a persistent loop over items (FP64, one workgroup per CU),
  // where the first B chunks and A fragment of the next item are loaded during the last k-steps
  // of the current one and the epilogue's stores, so the item boundary costs no load latency.
  const int wg = blockIdx.x;
  const int xcd = wg & 7, slot = wg >> 3, n_slots = (int)(gridDim.x >> 3);
  const int64_t groups_x = a.n_groups > xcd ? (a.n_groups - xcd + 7) / 8 : 0;   // groups of this XCD
  const int64_t n_local = groups_x * a.n_mblk;
  int64_t l = slot;
  if (l >= n_local) return;

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int l16 = lane & 15, kq = lane >> 4;
  constexpr int BM = kBM<MODE>;
  const int n_chunks = (int)(a.Kp / M_::KCH);
  // Items of an XCD in super-groups of kSuper column groups: row block after row block, each over
  // the super-group's column groups, so that the XCD's L2 holds the B columns of the super-group
  // and the A rows of the few row blocks in flight at once (instead of the whole table streaming
  // through it for every column group).
  auto item_grp = [&](int64_t li) {
    const int64_t sg = li / (kSuper * a.n_mblk), rem = li - sg * kSuper * a.n_mblk;
    const int64_t width = min((int64_t)kSuper, groups_x - sg * kSuper);
    return a.grp0 + (sg * kSuper + rem % width) * 8 + xcd;
  };
  auto item_mb = [&](int64_t li) {
    const int64_t sg = li / (kSuper * a.n_mblk), rem = li - sg * kSuper * a.n_mblk;
    const int64_t width = min((int64_t)kSuper, groups_x - sg * kSuper);
    return (int)(rem / width);
  };

  // Software pipeline: B chunks go global -> registers -> LDS one chunk ahead into alternating
  // buffers (one barrier per chunk); the A fragment of k-step t+1 is loaded while the MFMAs of
  // k-step t run.  The chunk stream runs on across items: chunk c of an item sits in buffer
  // (c + par) & 1, where par flips after every item when the chunk count is odd.
  using F = Frag<MODE>;
  u32x4 pre[kPre<MODE>];
  F f[2];
  int64_t grp = item_grp(l);
  int mb = item_mb(l);
  int par = 0;
  load_chunk_regs<MODE>(a, grp, 0, tid, pre);
  store_chunk_lds<MODE>(lds, tid, pre);
  if (n_chunks > 1) load_chunk_regs<MODE>(a, grp, M_::KCH, tid, pre);
  f[0].load_a(a, (int64_t)mb * BM + wave * 16 * WM, l16, kq, 0);

  constexpr int NW = kWaves<MODE>, WR = 16 * WM, NT = 64 * NW;
  for (;;) {
    const int64_t row0 = (int64_t)mb * BM + wave * 16 * WM;
    const int64_t ln = l + n_slots;
    const bool has_next = kPersist<MODE> && ln < n_local;
    const int64_t grp_n = has_next ? item_grp(ln) : grp;
    const int64_t row0_n = has_next ? (int64_t)item_mb(ln) * BM + wave * 16 * WM : row0;

    Acc acc[WM][9];
#pragma unroll
    for (int mi = 0; mi < WM; ++mi)
#pragma unroll
      for (int ni = 0; ni < 9; ++ni) acc[mi][ni] = Acc{0, 0, 0, 0};

    // The loop body has no data-dependent branches (the compiler then tracks the outstanding
    // loads exactly): past the last chunk the prefetches read the next item's first chunks and A
    // fragment, or, after the last item, re-read the last chunk (unused).
    const int64_t k_last = a.Kp - M_::KSTEP;
    for (int c = 0; c < n_chunks; ++c) {
      const char *cur = lds + ((c + par) & 1) * BUF;
      char *nxt = lds + ((c + 1 + par) & 1) * BUF;
      const bool into_next = c + 2 >= n_chunks && has_next;
      const int64_t g2 = into_next ? grp_n : grp;
      const int64_t c2 = (int64_t)(into_next ? c + 2 - n_chunks : min(c + 2, n_chunks - 1)) * M_::KCH;
      // chunk c is visible and every wave has finished reading chunk c-1, whose buffer is refilled
      lds_barrier();
      store_chunk_lds<MODE>(nxt, tid, pre);
      load_chunk_regs<MODE>(a, g2, c2, tid, pre);
#pragma unroll
      for (int s = 0; s < SPC; ++s) {
        const int64_t k = (int64_t)c * M_::KCH + s * M_::KSTEP;
        F &now = f[s & 1], &next = f[(s + 1) & 1];
        if (s + 1 < SPC) {
          next.load_a(a, row0, l16, kq, k + M_::KSTEP);
        } else {
          const bool last = c + 1 == n_chunks;
          next.load_a(a, last ? row0_n : row0, l16, kq, last ? (has_next ? 0 : k_last) : k + M_::KSTEP);
        }
        // keep the prefetches ahead of this k-step's MFMAs (the scheduler would otherwise sink
        // them towards their first use in the next k-step)
        __builtin_amdgcn_sched_barrier(0);
        now.mma(acc, cur, l16, kq, s * M_::KSTEP);
      }
      if constexpr (SPC % 2 == 1) f[0] = f[1];
    }

    // Epilogue.  Lane holds C[row][col l16] of each 16x16 block with row = 4 kq + r for the
    // FP32-accumulating instructions and row = kq + 4 r for the FP64 one (measured layouts).
    // The waves' tiles are transposed through LDS (in the item loop only through the buffer of
    // the last chunk: the other one already holds the next item's first chunk), several
    // consecutive waves per round, so that each tile's rows x 9 values (contiguous in the block
    // array) are written as whole lines.
    constexpr int STAGE = kPersist<MODE> ? BUF : 2 * BUF;   // LDS bytes the epilogue may use
    constexpr int PER_ROUND = (int)(STAGE / (WR * 144 * sizeof(O))) < NW ? (int)(STAGE / (WR * 144 * sizeof(O))) : NW;
    constexpr int RR = PER_ROUND * WR;   // rows per round
    static_assert(PER_ROUND >= 1 && NW % PER_ROUND == 0, "epilogue rounds");
    O *out = (O *)a.out;
    O *stage = (O *)(kPersist<MODE> ? lds + ((n_chunks - 1 + par) & 1) * BUF : lds);
#pragma unroll 1
    for (int w0 = 0; w0 < NW; w0 += PER_ROUND) {
      // LDS-only barriers: the stage is the only shared data, and a full __syncthreads would also
      // wait for the previous round's global stores and the next item's prefetches
      lds_barrier();
      if (wave >= w0 && wave < w0 + PER_ROUND) {
        const int rbase = (wave - w0) * WR;
#pragma unroll
        for (int ni = 0; ni < 9; ++ni) {
          const int n = ni * 16 + l16;
          const int tl = n / 9, ab = n - 9 * tl;
          float cs = 1.0f;
          if constexpr (MODE == IGAMT_F16X3) cs = a.Bscale[(grp * 16 + tl) * 9 + ab];
#pragma unroll
          for (int mi = 0; mi < WM; ++mi)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int ml = mi * 16 + (MODE == IGAMT_F64 ? kq + 4 * r : 4 * kq + r);
              O v = (O)acc[mi][ni][r];
              if constexpr (MODE == IGAMT_F16X3) v = v * (a.Ascale[mb * BM + wave * WR + ml] * cs);
              stage[(tl * RR + rbase + ml) * 9 + ab] = v;
            }
        }
      }
      lds_barrier();
      const int64_t r0 = (int64_t)mb * BM + w0 * WR;
      const int rows = (int)min((int64_t)RR, a.M - r0);
      if (rows > 0) {
        if constexpr (kPersist<MODE>) {
          // a fixed number of stores per thread, so that the next item's prefetches (issued before
          // them) are waited for with an exact count instead of after every store has completed
          constexpr int PER_T = (16 * RR * 9 + NT - 1) / NT;
          O *base = out + (grp * 16 * a.M + r0) * 9;                     // tile grp * 16, row r0
          const int n_tl = (int)min((int64_t)16, a.n_tiles - grp * 16);   // tiles of this group
          const int tstride = (int)(a.M * 9);
#pragma unroll
          for (int it = 0; it < PER_T; ++it) {
            const int e = tid + it * NT;
            const int tl = e / (RR * 9), jj = e - RR * 9 * tl;
            if (e < 16 * RR * 9 && tl < n_tl && jj < rows * 9) base[tl * tstride + jj] = stage[e];
          }
        } else {
          for (int e = tid; e < 16 * RR * 9; e += NT) {
            const int tl = e / (RR * 9), jj = e - RR * 9 * tl;
            const int64_t t = grp * 16 + tl;
            if (t < a.n_tiles && jj < rows * 9) out[(t * a.M + r0) * 9 + jj] = stage[tl * RR * 9 + jj];
          }
        }
      }
    }
    if (!has_next) break;
    l = ln;
    grp = grp_n;
    mb = item_mb(ln);
    par ^= n_chunks & 1;
  }
}

// ---- split modes with the table resident in LDS ------------------------------------------------
// The split products need three MFMAs per operand pair, so their operands must reach the matrix
// cores at three times the FP32 rate.  This variant keeps a block of 112 table rows (hi and lo
// planes, all k) in LDS for the whole life of a workgroup (one per CU), and streams the
// coefficient columns straight from global memory into each wave's registers, a few k-steps
// ahead: the table is read from L2 once per workgroup instead of once per column group, there is
// no barrier after the table is staged, and every wave runs its own loop over passes of
// 16 NCB columns.  The coefficient planes are stored tiled for it (split_coef_index): the 16
// columns x 32 k of one MFMA fragment are 1 KB in lane order, so each fragment is one coalesced
// 16-byte load per lane.  Per k-step (32 k) a wave issues 7 x NCB x P MFMAs (P = 2, 3 or 4
// products) against 14 LDS fragment reads and NCB or 2 NCB global fragment loads.  Workgroups of
// one XCD take every row block of one eighth of the columns, so each coefficient column is
// fetched into that XCD's L2 once and read there by all row blocks.
//   PROD = 3: lo*hi + hi*lo + hi*hi (the split mode); 2: lo*hi + hi*hi with the coefficients' lo
//   plane ignored (table split only); 4: lo*lo + lo*hi + hi*lo + hi*hi.
constexpr int kSplitRB16 = 7;                          // 16-row blocks per workgroup
constexpr int kSplitRows = 16 * kSplitRB16;            // 112 table rows
#ifndef IGAMT_SPLIT_WAVES
#define IGAMT_SPLIT_WAVES 12
#endif
#ifndef IGAMT_SPLIT_NCB
#define IGAMT_SPLIT_NCB 2
#endif
#ifndef IGAMT_SPLIT_NPF
#define IGAMT_SPLIT_NPF 2
#endif
constexpr int kSplitWaves = IGAMT_SPLIT_WAVES;         // waves per workgroup
constexpr int kSplitNCB = IGAMT_SPLIT_NCB;             // 16-column blocks per wave and pass
constexpr int kSplitNPF = IGAMT_SPLIT_NPF;             // k-steps of coefficient fragments in flight
constexpr int kSplitWC = 16 * kSplitNCB;               // columns per wave and pass
constexpr int kStageCol = 20;                          // words per column of a wave's epilogue stage

struct SplitArgs {
  const float *Af, *Bf;      // FP32: table [Mp][Kp] and coefficients [9 n_tiles_pad][Kp]
  const uint16_t *Ah, *Al;   // table planes [Mp][Kp]
  const float *Ascale;       // F16X3 inverse row scales [Mp]
  const uint16_t *Bh, *Bl;   // coefficient planes, tiled (split_coef_index)
  const float *Bscale;       // F16X3 inverse column scales [n_tiles_pad * 9]
  float *out;                // [n_tiles][M][9], addressed by absolute tile index
  int64_t M, Mp, Kp;
  int64_t c_lo, c_hi;        // columns of this launch (tile groups of a slab, or all)
  int64_t ncol_pad;          // coefficient columns in memory (9 n_tiles_pad, a multiple of 16)
  int n_rblk, n_split;       // row blocks; column splits (a multiple of 8)
  int row_bytes;             // LDS bytes of one table row of one plane (2 Kp + 16)
};

// the two table planes, the row block's 112 inverse row scales (F16X3), then one epilogue stage of
// 32 columns x 16 rows per wave
__host__ __device__ inline int64_t split_lds_bytes(int64_t Kp) {
  return 2 * kSplitRows * (2 * Kp + 16) + 4 * kSplitRows + 4 * kSplitWaves * 32 * kStageCol;
}

template <int MODE, int KS, int PROD>
__global__ __launch_bounds__(64 * kSplitWaves, 1) void contract_split_kernel(SplitArgs a) {
  using V8 = typename std::conditional<MODE == IGAMT_BF16X3, bf16x8, f16x8>::type;
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const int wg = blockIdx.x, xcd = wg & 7, slot = wg >> 3;
  const int rb = slot % a.n_rblk, s = (slot / a.n_rblk) * 8 + xcd;
  if (s >= a.n_split) return;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, l16 = lane & 15, kq = lane >> 4;
  const int64_t row0 = (int64_t)rb * kSplitRows;
  constexpr int64_t Kp = 32 * KS;
  constexpr int RB = 64 * KS + 16;   // LDS bytes of one table row of one plane (= a.row_bytes)
  // columns of split s, in whole 16-column units
  const int64_t units = (a.c_hi - a.c_lo + 15) / 16;
  const int64_t c0 = a.c_lo + 16 * (units * s / a.n_split);
  const int64_t c1 = min(a.c_hi, a.c_lo + 16 * (units * (s + 1) / a.n_split));
  if (c1 <= c0) return;
  // stage the row block's two table planes (rows past Mp read as zero)
  {
    constexpr int ppr = (int)(Kp / 8);   // 16-byte pieces per row and plane
    for (int i = tid; i < 2 * kSplitRows * ppr; i += 64 * kSplitWaves) {
      const int plane = i / (kSplitRows * ppr), rem = i - plane * kSplitRows * ppr;
      const int r = rem / ppr, j = rem - r * ppr;
      u32x4 v = {0u, 0u, 0u, 0u};
      if (row0 + r < a.Mp) v = *(const u32x4 *)((plane ? a.Al : a.Ah) + (row0 + r) * Kp + 8 * j);
      *(u32x4 *)(lds + (plane * kSplitRows + r) * RB + 16 * j) = v;
    }
  }
  float *rscale = (float *)(lds + 2 * kSplitRows * RB);
  float *stage = rscale + kSplitRows + wave * 32 * kStageCol;   // this wave's epilogue stage (32 columns)
  if constexpr (MODE == IGAMT_F16X3)
    for (int r = tid; r < kSplitRows; r += 64 * kSplitWaves) rscale[r] = row0 + r < a.Mp ? a.Ascale[row0 + r] : 0.0f;
  __syncthreads();
  constexpr int64_t PER_PASS = kSplitWC * kSplitWaves;
  const int n_pass = (int)((c1 - c0 + PER_PASS - 1) / PER_PASS);
  // A fragment of row block r, k-step ks, plane pl: lane (l16, kq) holds row 16 r + l16, k 32 ks + 8 kq .. + 7;
  // every fragment is one of two base addresses plus an immediate offset
  const char *a_hi = lds + l16 * RB + 16 * kq;
  const char *a_lo = a_hi + kSplitRows * RB;
  auto a_frag = [&](int pl, int r, int ks) -> V8 {
    return *(const V8 *)((pl ? a_lo : a_hi) + 16 * r * RB + 64 * ks);
  };
  // coefficient fragments: lane (l16, kq) holds column l16 of block cb, k 32 ks + 8 kq .. + 7, which
  // the tiled planes store at lane * 8 within the fragment's 512 elements
  V8 bh[kSplitNPF][kSplitNCB], bl[kSplitNPF][kSplitNCB];
  auto load_b = [&](int slot_, int p, int ks) {
#pragma unroll
    for (int cb = 0; cb < kSplitNCB; ++cb) {
      int64_t col = c0 + p * PER_PASS + wave * kSplitWC + 16 * cb;
      col = min(col, a.ncol_pad - 16);   // past the range: a valid fragment, its result is not stored
      const int64_t off = ((col >> 4) * KS + ks) * 512 + 8 * lane;
      bh[slot_][cb] = *(const V8 *)(a.Bh + off);
      if constexpr (PROD != 2) bl[slot_][cb] = *(const V8 *)(a.Bl + off);
    }
  };
#pragma unroll
  for (int i = 0; i < kSplitNPF; ++i) load_b(i, i / KS, i % KS);
  f4 acc[kSplitRB16][kSplitNCB];
#pragma unroll
  for (int r = 0; r < kSplitRB16; ++r)
#pragma unroll
    for (int cb = 0; cb < kSplitNCB; ++cb) acc[r][cb] = f4{0.f, 0.f, 0.f, 0.f};
  auto mma = [&](const V8 &x, const V8 &y, f4 &c) {
    if constexpr (MODE == IGAMT_BF16X3)
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, c, 0, 0, 0);
    else
      c = __builtin_amdgcn_mfma_f32_16x16x32_f16(x, y, c, 0, 0, 0);
  };
  for (int p = 0; p < n_pass; ++p) {
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      // keep each k-step's fragment reads within the k-step (hoisted, they would hold every
      // k-step's fragments in registers at once)
      __builtin_amdgcn_sched_barrier(0);
      const int sl = ks % kSplitNPF;
      // row blocks in pairs, the next pair's fragments read while this pair's MFMAs run
      V8 ah[2][2], al[2][2];
      ah[0][0] = a_frag(0, 0, ks);
      al[0][0] = a_frag(1, 0, ks);
      ah[0][1] = a_frag(0, 1, ks);
      al[0][1] = a_frag(1, 1, ks);
#pragma unroll
      for (int rp = 0; rp < (kSplitRB16 + 1) / 2; ++rp) {
        const int cur = rp & 1, nx = cur ^ 1;
        if (rp + 1 < (kSplitRB16 + 1) / 2) {
          const int r2 = 2 * (rp + 1);
          ah[nx][0] = a_frag(0, r2, ks);
          al[nx][0] = a_frag(1, r2, ks);
          if (r2 + 1 < kSplitRB16) {
            ah[nx][1] = a_frag(0, r2 + 1, ks);
            al[nx][1] = a_frag(1, r2 + 1, ks);
          }
        }
        const int nr = 2 * rp + 1 < kSplitRB16 ? 2 : 1;
        if constexpr (PROD == 4) {
#pragma unroll
          for (int q = 0; q < 2; ++q)
            if (q < nr)
#pragma unroll
              for (int cb = 0; cb < kSplitNCB; ++cb) mma(al[cur][q], bl[sl][cb], acc[2 * rp + q][cb]);
        }
#pragma unroll
        for (int q = 0; q < 2; ++q)
          if (q < nr)
#pragma unroll
            for (int cb = 0; cb < kSplitNCB; ++cb) mma(al[cur][q], bh[sl][cb], acc[2 * rp + q][cb]);
        if constexpr (PROD != 2) {
#pragma unroll
          for (int q = 0; q < 2; ++q)
            if (q < nr)
#pragma unroll
              for (int cb = 0; cb < kSplitNCB; ++cb) mma(ah[cur][q], bl[sl][cb], acc[2 * rp + q][cb]);
        }
#pragma unroll
        for (int q = 0; q < 2; ++q)
          if (q < nr)
#pragma unroll
            for (int cb = 0; cb < kSplitNCB; ++cb) mma(ah[cur][q], bh[sl][cb], acc[2 * rp + q][cb]);
      }
      // refill this slot with the fragments kSplitNPF k-steps ahead (the next pass past the last),
      // after the last MFMA that reads it, so the loads can take the slot's registers
      __builtin_amdgcn_sched_barrier(0);
      const int kn = ks + kSplitNPF;
      load_b(sl, p + kn / KS, kn % KS);
    }
    // Epilogue through the wave's LDS stage, 32 columns (two column blocks) and one 16-row block at
    // a time.  Lane (l16, kq) holds C[4 kq + j][16 cb + l16]; the 16 x 32 values are written column
    // by column, then read back in the order of their addresses in the block array -- tile part,
    // row, ab, where a tile part is the run of the 32 columns that belong to one tile -- so that
    // consecutive lanes store consecutive words.  Element e = lane + 64 i of that order is fixed for
    // the 32 columns: its stage index and its block-array offset at row block 0 (row block r adds
    // 16 rows, 144 words).
#pragma unroll
    for (int h = 0; h < kSplitNCB / 2; ++h) {
      const int64_t cw = c0 + p * PER_PASS + wave * kSplitWC + 32 * h;
      const int64_t t0 = cw / 9;
      float *obase = a.out + (t0 * a.M + row0) * 9;   // tile t0, row row0
      int spk[8];    // stage index | row within the block << 16
      int goff[8];   // offset from obase at row block 0, or -1 past the column range
      {
        const int ab0 = (int)(cw - 9 * t0);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int e = lane + 64 * i;
          int base = 0, colo = 0, abs = ab0, k = min(9 - ab0, 32), t = 0;
#pragma unroll
          for (int j = 0; j < 4; ++j) {   // at most five parts (1 + 9 + 9 + 9 + 4 columns)
            if (e >= base + 16 * k) {
              base += 16 * k;
              colo += k;
              abs = 0;
              ++t;
              k = min(9, 32 - colo);
            }
          }
          const int local = e - base;
          const int rr = (int)((float)local / (float)k);   // exact: local < 144, k <= 9
          const int ab = abs + local - rr * k;
          const int cl = colo + ab - abs;
          spk[i] = (cl * kStageCol + rr) | (rr << 16);
          goff[i] = cw + cl < c1 ? (int)(((int64_t)t * a.M + rr) * 9 + ab) : -1;
        }
      }
      float cs[2] = {1.0f, 1.0f};
      if constexpr (MODE == IGAMT_F16X3)
#pragma unroll
        for (int c = 0; c < 2; ++c) cs[c] = cw + 16 * c + l16 < c1 ? a.Bscale[cw + 16 * c + l16] : 0.0f;
#pragma unroll
      for (int r = 0; r < kSplitRB16; ++r) {
        f4 rs = f4{1.f, 1.f, 1.f, 1.f};
        if constexpr (MODE == IGAMT_F16X3) rs = *(const f4 *)(rscale + 16 * r + 4 * kq);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          f4 v = acc[r][2 * h + c];
          if constexpr (MODE == IGAMT_F16X3)
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = v[j] * (rs[j] * cs[c]);
          *(f4 *)(stage + (16 * c + l16) * kStageCol + 4 * kq) = v;
          acc[r][2 * h + c] = f4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int i = 0; i < 8; ++i)
          if (goff[i] >= 0 && row0 + 16 * r + (spk[i] >> 16) < a.M) obase[goff[i] + 144 * r] = stage[spk[i] & 0xffff];
      }
    }
  }
}

// ---- split modes (and FP32) with the table resident in registers -----------------------------
// The LDS-resident variant above shares every coefficient column among the 112 table rows one CU
// holds, so each column crosses that CU's L1 once per 112 rows, and that stream bounds it.  Here
// each of the workgroup's 8 waves keeps 32 table rows (hi and lo planes, all k: 128 registers per
// lane for K = 256) in registers for its whole life, 256 rows per CU, and the columns pass through
// LDS once per workgroup: chunks of 32 columns (both planes, all k; 16 KB per plane, contiguous in
// the tiled layout) are loaded by the whole workgroup one chunk ahead into alternating LDS buffers,
// one barrier per chunk, and every wave reads each B fragment from LDS once for its 2 x 3 MFMAs
// (two row tiles, three products).  A chunk's epilogue runs during the next chunk's first k-steps
// (its accumulators are kept aside), so its stage traffic and stores overlap that chunk's MFMAs.
// Workgroups of one XCD take every row block of their column splits, so each column is fetched
// into that XCD's L2 once.  FP32 (K = 128 or 256) runs the same kernel: its table rows are FP32 (the
// same 128 registers per lane), its coefficient chunks plain columns padded in LDS, and each k-step
// of 32 issues 32 v_mfma_f32_16x16x4f32 per wave, so the epilogue hides under far more MFMA time.
#ifndef IGAMT_SPLIT_REG
#define IGAMT_SPLIT_REG 1
#endif
#ifndef IGAMT_F32_REG
#define IGAMT_F32_REG 1   // FP32 (K = 128 or 256) on this kernel too, the table as FP32 in registers
#endif
constexpr int kRegWaves = 8;                             // waves per workgroup
constexpr int kRegRT = 2;                                // 16-row tiles per wave
constexpr int kRegRows = 16 * kRegRT * kRegWaves;        // 256 table rows per workgroup
constexpr int kRegCols = 32;                             // columns per chunk (two column blocks)
constexpr int kRegStageCol = 36;                         // words per column of a wave's stage (32 rows + pad)

// bytes of one B chunk buffer: the split modes' two planes (2 bytes per element, the tiled layout),
// or FP32 columns of Kp floats padded by 16 bytes (so that the 16-byte fragment reads of a quarter
// wave fall on 16 different 4-bank groups)
__host__ __device__ constexpr int64_t reg_chunk_buf_bytes(bool f32, int64_t Kp) {
  return f32 ? kRegCols * (4 * Kp + 16) : 2 * kRegCols * Kp * 2;
}
// two B chunk buffers, one epilogue stage of 32 columns x 32 rows per wave, then each wave's 32
// inverse row scales (F16X3)
__host__ __device__ inline int64_t split_reg_lds_bytes(bool f32, int64_t Kp) {
  return 2 * reg_chunk_buf_bytes(f32, Kp) + 4 * kRegWaves * 32 * kRegStageCol + 4 * kRegWaves * 32;
}

template <int MODE, int KS, int PROD>
__global__ __launch_bounds__(64 * kRegWaves, 1) void contract_split_reg_kernel(SplitArgs a) {
  using V8 = typename std::conditional<MODE == IGAMT_BF16X3, bf16x8, f16x8>::type;
  typedef float f4v __attribute__((ext_vector_type(4)));
  constexpr bool F32 = MODE == IGAMT_F32;
  extern __shared__ __attribute__((aligned(16))) char lds[];
  constexpr int64_t Kp = 32 * KS;
  constexpr int CHUNK = kRegCols * (int)Kp * 2;          // bytes of one plane of one chunk (split modes)
  constexpr int BUFB = (int)reg_chunk_buf_bytes(F32, Kp);   // bytes of one chunk buffer
  constexpr int COLB = 4 * (int)Kp + 16;                 // FP32: bytes of one padded column in LDS
  // Persistent: the workgroups of one XCD (blockIdx.x mod 8) take the units (row block rb, column
  // split s = 8 j + xcd) of their XCD in turn, rb fastest, so that the row blocks of a column split
  // run at about the same time on one L2 and read its coefficients once.
  const int wg = blockIdx.x, xcd = wg & 7, slot = wg >> 3, per_xcd = (int)(gridDim.x >> 3);
  const int n_unit = a.n_rblk * (a.n_split / 8);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, l16 = lane & 15, kq = lane >> 4;
  const int64_t n16 = (a.c_hi - a.c_lo + 15) / 16;   // 16-column blocks of the launch
  int64_t row0 = 0, c0 = 0, c1 = 0;                  // this wave's first row; the unit's columns
  float *stage = (float *)(lds + 2 * BUFB) + wave * 32 * kRegStageCol;   // [32 columns][32 rows + pad]

  // the chunk's two planes: 2 column blocks x KS k-steps x 512 elements, contiguous per block
  constexpr int PIECES = CHUNK / 16;                     // 16-byte pieces per plane
  constexpr int NPRE = 2 * PIECES / (64 * kRegWaves);    // pieces per thread, both planes
  static_assert(2 * PIECES % (64 * kRegWaves) == 0, "chunk pieces must divide over the workgroup");
  u32x4 pre[NPRE];
  // (FP32: the same number of 16-byte pieces, Kp / 4 per column; thread tid takes column tid / 16,
  // pieces tid % 16 + 16 i, so that its pieces share one base address)
  static_assert(!F32 || Kp / 4 == 16 * NPRE, "FP32 chunk pieces per thread");
  auto load_chunk = [&](int c) {
#pragma unroll
    for (int i = 0; i < NPRE; ++i) {
      const int e = tid + i * 64 * kRegWaves;
      if constexpr (F32) {
        const int64_t col = min(c0 + (int64_t)c * kRegCols + (tid >> 4), a.ncol_pad - 1);   // past the range: not stored
        pre[i] = *(const u32x4 *)(a.Bf + col * Kp + 4 * (tid & 15) + 64 * i);
      } else {
        const int pl = e / PIECES, j = e - pl * PIECES;
        const int cb = j / (KS * 64), jj = j - cb * KS * 64;   // column block, piece within it
        int64_t col = c0 + (int64_t)c * kRegCols + 16 * cb;
        col = min(col, a.ncol_pad - 16);   // past the range: a valid block, its result is not stored
        pre[i] = *(const u32x4 *)((pl ? a.Bl : a.Bh) + (col >> 4) * KS * 512 + 8 * jj);
      }
    }
  };
  auto store_chunk = [&](int buf) {
#pragma unroll
    for (int i = 0; i < NPRE; ++i) {
      const int e = tid + i * 64 * kRegWaves;
      if constexpr (F32) {
        *(u32x4 *)(lds + buf * BUFB + (tid >> 4) * COLB + 16 * (tid & 15) + 256 * i) = pre[i];
      } else {
        const int pl = e / PIECES, j = e - pl * PIECES;
        *(u32x4 *)(lds + buf * BUFB + pl * CHUNK + 16 * j) = pre[i];
      }
    }
  };

  // this wave's table rows (loaded per unit): lane (l16, kq) holds row 16 rt + l16, k 32 ks + 8 kq .. + 7
  // (FP32: af, k 16 s + 4 kq .. + 3 of each 16-k block s; the unused set takes no registers)
  V8 ah[kRegRT][KS], al[kRegRT][KS];
  f4v af[kRegRT][2 * KS];
  // F16X3: the inverse row scales of the wave's 32 rows, in LDS after the stage
  float *rsl = (float *)(lds + 2 * BUFB) + kRegWaves * 32 * kRegStageCol + 32 * wave;
  auto mma = [&](const V8 &x, const V8 &y, f4 &c) {
    if constexpr (MODE == IGAMT_BF16X3)
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, c, 0, 0, 0);
    else
      c = __builtin_amdgcn_mfma_f32_16x16x32_f16(x, y, c, 0, 0, 0);
  };

  // Epilogue map: the 32 x 16 values of a chunk's row tile in block-array address order -- tile
  // part, row, ab, where a tile part is the run of the chunk's columns that belong to one tile -- so
  // that consecutive lanes store consecutive words.  It depends on the chunk only through the ab of
  // its first column (ab0).  Element e = lane + 64 i of map ab0: espk = its stage index (column cl,
  // row rr) | rr << 11, egoff = its offset in the block array from the chunk's first tile at the
  // wave's first row; each lane's eight entries are contiguous.
  __shared__ __attribute__((aligned(16))) uint16_t espk[9][64][8];
  __shared__ __attribute__((aligned(16))) int egoff[9][64][8];
  for (int idx = tid; idx < 9 * 512; idx += 64 * kRegWaves) {
    const int ab0 = idx >> 9, e = idx & 511;
    int base = 0, colo = 0, abs = ab0, k = min(9 - ab0, 32), t = 0;
    for (int j = 0; j < 4; ++j) {   // at most five parts (1 + 9 + 9 + 9 + 4 columns)
      if (e >= base + 16 * k) {
        base += 16 * k;
        colo += k;
        abs = 0;
        ++t;
        k = min(9, 32 - colo);
      }
    }
    const int local = e - base, rr = local / k, ab = abs + local - rr * k, cl = colo + ab - abs;
    espk[ab0][e & 63][e >> 6] = (uint16_t)((cl * kRegStageCol + rr) | rr << 11);
    egoff[ab0][e & 63][e >> 6] = (int)(((int64_t)t * a.M + rr) * 9 + ab);
  }

  // The previous chunk's epilogue, in three steps: (1) its accumulators (scaled) into the stage and
  // its map entries into registers, (2) the stage read back in map order, (3) the stores.
  f4 pacc[kRegRT][2];
  float pcs[2] = {1.0f, 1.0f};
  int64_t pcw = 0;
  int spk[8], goff[8];
  float v[kRegRT][8];
  auto epi1 = [&]() {
#pragma unroll
    for (int rt = 0; rt < kRegRT; ++rt)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        f4 x = pacc[rt][q];
        if constexpr (MODE == IGAMT_F16X3) {
          const f4 rs = *(const f4 *)(rsl + 16 * rt + 4 * kq);
#pragma unroll
          for (int j = 0; j < 4; ++j) x[j] = x[j] * (rs[j] * pcs[q]);
        }
        *(f4 *)(stage + (16 * q + l16) * kRegStageCol + 16 * rt + 4 * kq) = x;
      }
    const int ab0 = (int)(pcw - 9 * (pcw / 9));
    const u32x4 sp = *(const u32x4 *)&espk[ab0][lane][0];
    const u32x4 g0 = *(const u32x4 *)&egoff[ab0][lane][0], g1 = *(const u32x4 *)&egoff[ab0][lane][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      spk[2 * i] = (int)(sp[i] & 0xffffu);
      spk[2 * i + 1] = (int)(sp[i] >> 16);
      goff[i] = (int)g0[i];
      goff[4 + i] = (int)g1[i];
    }
  };
  auto epi2 = [&]() {
#pragma unroll
    for (int rt = 0; rt < kRegRT; ++rt)
#pragma unroll
      for (int i = 0; i < 8; ++i) v[rt][i] = stage[(spk[i] & 2047) + 16 * rt];
  };
  // part p of 4 (PARTS = 4: a quarter of the stores each), or all of them (p < 0); a chunk past the
  // column range or a row block past M takes the checked stores at once
  auto epi3 = [&](int p) {
    float *obase = a.out + ((pcw / 9) * a.M + row0) * 9;
    if (pcw + kRegCols <= c1 && row0 + 16 * kRegRT <= a.M) {
#pragma unroll
      for (int rt = 0; rt < kRegRT; ++rt)
#pragma unroll
        for (int i = 0; i < 8; ++i)
          if (p < 0 || p == rt * 2 + i / 4) obase[goff[i] + 144 * rt] = v[rt][i];
    } else if (p <= 0) {
      const int ncl = (int)min((int64_t)kRegCols, c1 - pcw);   // columns of the chunk in range
#pragma unroll
      for (int rt = 0; rt < kRegRT; ++rt)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int rr = spk[i] >> 11, cl = (spk[i] & 2047) / kRegStageCol;
          if (cl < ncl && row0 + 16 * rt + rr < a.M) obase[goff[i] + 144 * rt] = v[rt][i];
        }
    }
  };

  for (int u = slot; u < n_unit; u += per_xcd) {
  const int rb = u % a.n_rblk, s = (u / a.n_rblk) * 8 + xcd;
  row0 = (int64_t)rb * kRegRows + 32 * wave;
  c0 = a.c_lo + 16 * (n16 * s / a.n_split);
  c1 = min(a.c_hi, a.c_lo + 16 * (n16 * (s + 1) / a.n_split));
  if (c1 <= c0) continue;   // the same for every wave of the workgroup
  const int n_chunk = (int)((c1 - c0 + kRegCols - 1) / kRegCols);
#pragma unroll
  for (int rt = 0; rt < kRegRT; ++rt) {
    const int64_t r = row0 + 16 * rt + l16;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      if constexpr (F32) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
          af[rt][2 * ks + h] = r < a.Mp ? *(const f4v *)(a.Af + r * Kp + 32 * ks + 16 * h + 4 * kq) : f4v{};
      } else {
        const int64_t off = r * Kp + 32 * ks + 8 * kq;
        if (r < a.Mp) {
          ah[rt][ks] = *(const V8 *)(a.Ah + off);
          al[rt][ks] = *(const V8 *)(a.Al + off);
        } else {
          ah[rt][ks] = V8{};
          al[rt][ks] = V8{};
        }
      }
    }
  }
  // (the wave's last epilogue of the previous unit has read its scales: LDS accesses of one wave
  // complete in order)
  if constexpr (MODE == IGAMT_F16X3)
    if (lane < 32) rsl[lane] = row0 + lane < a.Mp ? a.Ascale[row0 + lane] : 0.0f;

  // Chunk c + 1 is loaded into registers during chunk c - 1 and written to LDS at the end of chunk
  // c, before the loads of chunk c + 2 are issued.
  load_chunk(0);
  __syncthreads();   // every wave is done with the previous unit's chunk buffers
  store_chunk(0);
  if (n_chunk > 1) load_chunk(1);
  for (int c = 0; c < n_chunk; ++c) {
    __syncthreads();   // chunk c is in its buffer; every wave is done with the other one
    const char *bh_base = lds + (c & 1) * BUFB + 16 * lane;
    const char *bl_base = bh_base + CHUNK;
    const char *bf_base = lds + (c & 1) * BUFB + l16 * COLB + 16 * kq;   // FP32: column l16, k 4 kq
    const int64_t cw = c0 + (int64_t)c * kRegCols;
    float cs[2] = {1.0f, 1.0f};
    if constexpr (MODE == IGAMT_F16X3)
#pragma unroll
      for (int q = 0; q < 2; ++q) cs[q] = cw + 16 * q + l16 < c1 ? a.Bscale[cw + 16 * q + l16] : 0.0f;
    f4 acc[kRegRT][2];
#pragma unroll
    for (int rt = 0; rt < kRegRT; ++rt) acc[rt][0] = acc[rt][1] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      if constexpr (F32) {
        // two 16-k blocks; lane (l16, kq) holds k = 16 s + 4 kq + t of column l16, the t-th MFMA
        // of a block takes k-slice {16 s + 4 kq + t : kq} (A holds the same k)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          f4v b[2];
#pragma unroll
          for (int cb = 0; cb < 2; ++cb) b[cb] = *(const f4v *)(bf_base + cb * 16 * COLB + (32 * ks + 16 * h) * 4);
#pragma unroll
          for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int rt = 0; rt < kRegRT; ++rt)
#pragma unroll
              for (int cb = 0; cb < 2; ++cb)
                acc[rt][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[rt][2 * ks + h][t], b[cb][t], acc[rt][cb], 0, 0, 0);
        }
      } else {
      V8 bh[2], bl[2];
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        bh[cb] = *(const V8 *)(bh_base + (cb * KS + ks) * 1024);
        if constexpr (PROD != 2) bl[cb] = *(const V8 *)(bl_base + (cb * KS + ks) * 1024);
      }
      if constexpr (PROD == 4)
#pragma unroll
        for (int rt = 0; rt < kRegRT; ++rt)
#pragma unroll
          for (int cb = 0; cb < 2; ++cb) mma(al[rt][ks], bl[cb], acc[rt][cb]);
#pragma unroll
      for (int rt = 0; rt < kRegRT; ++rt)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) mma(al[rt][ks], bh[cb], acc[rt][cb]);
      if constexpr (PROD != 2)
#pragma unroll
        for (int rt = 0; rt < kRegRT; ++rt)
#pragma unroll
          for (int cb = 0; cb < 2; ++cb) mma(ah[rt][ks], bl[cb], acc[rt][cb]);
#pragma unroll
      for (int rt = 0; rt < kRegRT; ++rt)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) mma(ah[rt][ks], bh[cb], acc[rt][cb]);
      }
      // the previous chunk's epilogue, one step per k-step, between this chunk's MFMAs
      if (c > 0) {
        if (ks == 0) epi1();
        if (ks == (KS > 2 ? 1 : 0)) epi2();
        if constexpr (KS >= 6) {
          if (ks >= 2 && ks < 6) epi3(ks - 2);
        } else if (ks == KS - 1) {
          epi3(-1);
        }
      }
    }
    if (c + 1 < n_chunk) store_chunk((c + 1) & 1);   // the other buffer: read by no wave since the barrier
    if (c + 2 < n_chunk) load_chunk(c + 2);
#pragma unroll
    for (int rt = 0; rt < kRegRT; ++rt) pacc[rt][0] = acc[rt][0], pacc[rt][1] = acc[rt][1];
    pcs[0] = cs[0];
    pcs[1] = cs[1];
    pcw = cw;
  }
  epi1();
  epi2();
  epi3(-1);
  }
}

// compute units of the current device, queried once per device
static int device_cus() {
  static std::atomic<int> cus[64];   // 0: not yet queried
  int dev = 0;
  (void)hipGetDevice(&dev);
  int n = cus[dev & 63].load(std::memory_order_relaxed);
  if (n == 0) {
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cus[dev & 63].store(n, std::memory_order_relaxed);
  }
  return n;
}

static igamt_status launch_contract_split(igamt_plan *P, igamt_precision prec, int prod, const void *d_coef,
                                          void *d_blocks, hipStream_t s, int64_t g0, int64_t g1) {
  SplitArgs a;
  const int64_t MK = P->Mp * P->Kp;
  const int64_t plane = P->n_tiles_pad * 9 * P->Kp;
  const bool bf = prec == IGAMT_BF16X3;
  const bool f32 = prec == IGAMT_F32;   // FP32 with the table in registers (not split)
  a.Af = f32 ? P->dev.table_f32 : nullptr;
  a.Bf = f32 ? (const float *)d_coef : nullptr;
  a.Ah = f32 ? nullptr : bf ? P->dev.table_bf : P->dev.table_h;
  a.Al = f32 ? nullptr : a.Ah + MK;
  a.Ascale = f32 || bf ? nullptr : P->dev.table_h_scale;
  a.Bh = f32 ? nullptr : (const uint16_t *)d_coef;
  a.Bl = f32 ? nullptr : a.Bh + plane;
  a.Bscale = f32 || bf ? nullptr : (const float *)(a.Bh + 2 * plane);
  a.out = (float *)d_blocks;
  a.M = P->n_pairs;
  a.Mp = P->Mp;
  a.Kp = P->Kp;
  a.c_lo = g0 * BN;
  a.c_hi = std::min(g1 * BN, 9 * P->n_tiles);
  a.ncol_pad = 9 * P->n_tiles_pad;
  const int rows = IGAMT_SPLIT_REG ? kRegRows : kSplitRows;
  a.n_rblk = (int)((P->Mp + rows - 1) / rows);
  a.row_bytes = (int)(2 * P->Kp + 16);
  unsigned n_wg;
  if (IGAMT_SPLIT_REG) {
    // one workgroup per CU; per XCD, n_rblk x R units over its G workgroups with R = G / gcd(n_rblk, G)
    // (every workgroup takes the same number of units), fewer splits where units would fall below
    // 8 chunks of columns
    const int G = std::max(1, device_cus() / 8);
    int R = G / std::gcd(a.n_rblk, G);
    const int64_t cols = a.c_hi - a.c_lo;
    while (R > 1 && cols / (8 * R) < 8 * kRegCols) R /= 2;
    a.n_split = 8 * R;
    n_wg = (unsigned)(8 * std::min<int64_t>(G, (int64_t)a.n_rblk * R));
  } else {
    a.n_split = 8 * std::max(1, 32 / a.n_rblk);
    n_wg = (unsigned)(a.n_rblk * a.n_split);
  }
  const size_t shm = (size_t)(IGAMT_SPLIT_REG ? split_reg_lds_bytes(f32, P->Kp) : split_lds_bytes(P->Kp));
  const dim3 grid(n_wg), block(64 * (IGAMT_SPLIT_REG ? kRegWaves : kSplitWaves));
#if IGAMT_SPLIT_REG
#define SPLIT_KERNEL contract_split_reg_kernel
#else
#define SPLIT_KERNEL contract_split_kernel
#endif
#define SPLIT_LAUNCH(M_, KS_, PR_)                                                                       \
  do {                                                                                                 \
    IGAMT_HIP(hipFuncSetAttribute((const void *)SPLIT_KERNEL<M_, KS_, PR_>,                            \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));              \
    hipLaunchKernelGGL((SPLIT_KERNEL<M_, KS_, PR_>), grid, block, shm, s, a);                          \
  } while (0)
  const int ks = (int)(P->Kp / 32);
#if IGAMT_SPLIT_REG
  if (f32) {
    if (ks == 8) SPLIT_LAUNCH(IGAMT_F32, 8, 3);
    else SPLIT_LAUNCH(IGAMT_F32, 4, 3);
  } else
#endif
  if (bf) {
    if (ks == 8) {
      if (prod == 3) SPLIT_LAUNCH(IGAMT_BF16X3, 8, 3);
      else if (prod == 2) SPLIT_LAUNCH(IGAMT_BF16X3, 8, 2);
      else SPLIT_LAUNCH(IGAMT_BF16X3, 8, 4);
    } else {
      if (prod == 3) SPLIT_LAUNCH(IGAMT_BF16X3, 4, 3);
      else if (prod == 2) SPLIT_LAUNCH(IGAMT_BF16X3, 4, 2);
      else SPLIT_LAUNCH(IGAMT_BF16X3, 4, 4);
    }
  } else {
    if (ks == 8) SPLIT_LAUNCH(IGAMT_F16X3, 8, 3);
    else SPLIT_LAUNCH(IGAMT_F16X3, 4, 3);
  }
#undef SPLIT_LAUNCH
#undef SPLIT_KERNEL
  IGAMT_LAUNCH_CHECK();
  return IGAMT_OK;
}

// Grid of the contraction: 8 x (items of the busiest XCD) workgroups, one item each, or for
// FP64 (one workgroup per CU) a persistent grid of one workgroup per CU, each looping over items.
static unsigned contract_grid(igamt_precision prec, const ContractArgs &a) {
  const int64_t items_x = (int64_t)(a.n_groups + 7) / 8 * a.n_mblk;
  int64_t slots = items_x;
  if (prec == IGAMT_F64 && kPersist<IGAMT_F64> && a.Kp / Mode<IGAMT_F64>::KCH >= 2)   // two chunks per item
    slots = std::min<int64_t>(items_x, std::max(1, device_cus() / 8));
  return (unsigned)(8 * slots);
}

igamt_status launch_contract(igamt_plan *P, igamt_precision prec, const void *d_coef, void *d_blocks, void *stream,
                             int64_t g0, int64_t g1) {
  if (g1 < 0) g1 = P->n_groups;
  if (g0 < 0 || g1 > P->n_groups || g0 >= g1) { set_error("invalid tile group range"); return IGAMT_EINVAL; }
  if (!P->tables_ready) { set_error("tables are not built or set"); return IGAMT_ESTATE; }
  ContractArgs a;
  const int64_t MK = P->Mp * P->Kp;
  const int64_t plane = P->n_tiles_pad * 9 * P->Kp;
  a.M = P->n_pairs;
  a.Kp = P->Kp;
  a.n_tiles = P->n_tiles;
  a.n_groups = (int)(g1 - g0);
  a.grp0 = g0;
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
  if ((prec == IGAMT_BF16X3 || prec == IGAMT_F16X3 || (prec == IGAMT_F32 && IGAMT_SPLIT_REG && IGAMT_F32_REG)) &&
      split_tiled(P->Kp))
    return launch_contract_split(P, prec, 3, d_coef, d_blocks, (hipStream_t)stream, g0, g1);
  const int bm = prec == IGAMT_F64 ? kBM<IGAMT_F64> : prec == IGAMT_F32 ? kBM<IGAMT_F32> : kBM<IGAMT_BF16X3>;
  if (P->Mp % bm != 0) { set_error("padded table rows are not a multiple of the row block"); return IGAMT_EINVAL; }
  a.n_mblk = (int)(P->Mp / bm);
  const dim3 grid(contract_grid(prec, a));
  hipStream_t s = (hipStream_t)stream;
  switch (prec) {
    case IGAMT_F64: hipLaunchKernelGGL(contract_kernel<IGAMT_F64>, grid, dim3(64 * kWaves<IGAMT_F64>), 0, s, a); break;
    case IGAMT_F32: hipLaunchKernelGGL(contract_kernel<IGAMT_F32>, grid, dim3(64 * kWaves<IGAMT_F32>), 0, s, a); break;
    case IGAMT_BF16X3:
      hipLaunchKernelGGL(contract_kernel<IGAMT_BF16X3>, grid, dim3(64 * kWaves<IGAMT_BF16X3>), 0, s, a);
      break;
    case IGAMT_F16X3:
      hipLaunchKernelGGL(contract_kernel<IGAMT_F16X3>, grid, dim3(64 * kWaves<IGAMT_F16X3>), 0, s, a);
      break;
  }
  IGAMT_LAUNCH_CHECK();
  return IGAMT_OK;
}

igamt_status launch_gemm_tiles(igamt_precision prec, const void *A, const void *B, void *out, int64_t rows,
                               int64_t rows_pad, int64_t kdim, int64_t n_tiles, int64_t n_groups, void *stream) {
  if (prec != IGAMT_F64 && prec != IGAMT_F32) { set_error("tile GEMM runs in F64 or F32"); return IGAMT_EUNSUPPORTED; }
  const int bm = prec == IGAMT_F64 ? kBM<IGAMT_F64> : kBM<IGAMT_F32>;
  const int kch = prec == IGAMT_F64 ? Mode<IGAMT_F64>::KCH : Mode<IGAMT_F32>::KCH;
  if (rows_pad % bm != 0 || kdim % kch != 0 || rows > rows_pad) {
    set_error("tile GEMM operands are not padded to the kernel's blocks");
    return IGAMT_EINVAL;
  }
  ContractArgs a;
  a.A = A;
  a.A2 = nullptr;
  a.Ascale = nullptr;
  a.B = B;
  a.B2 = nullptr;
  a.Bscale = nullptr;
  a.out = out;
  a.M = rows;
  a.Kp = kdim;
  a.n_tiles = n_tiles;
  a.n_mblk = (int)(rows_pad / bm);
  a.n_groups = (int)n_groups;
  a.grp0 = 0;
  const dim3 grid(contract_grid(prec, a));
  hipStream_t s = (hipStream_t)stream;
  if (prec == IGAMT_F64)
    hipLaunchKernelGGL(contract_kernel<IGAMT_F64>, grid, dim3(64 * kWaves<IGAMT_F64>), 0, s, a);
  else
    hipLaunchKernelGGL(contract_kernel<IGAMT_F32>, grid, dim3(64 * kWaves<IGAMT_F32>), 0, s, a);
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

extern "C" igamt_status igamt_contract_products(igamt_plan *P, int32_t products, const void *d_coef, void *d_blocks,
                                                void *stream) {
  if (!P || !d_coef || !d_blocks) { set_error("NULL argument"); return IGAMT_EINVAL; }
  if (products < 2 || products > 4) { set_error("products must be 2, 3 or 4"); return IGAMT_EINVAL; }
  igamt_status st = ensure_device(P);
  if (st) return st;
  if (!P->tables_ready) { set_error("tables are not built or set"); return IGAMT_ESTATE; }
  if (!split_tiled(P->Kp)) {
    set_error("the product ablations run for padded table widths of 128 or 256 columns");
    return IGAMT_EUNSUPPORTED;
  }
  return launch_contract_split(P, IGAMT_BF16X3, products, d_coef, d_blocks, (hipStream_t)stream, 0, P->n_groups);
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
  // The three stages in turn on the caller's stream.  (Running the scatter of one slab of tiles
  // beside the contraction of the next on a second stream gains nothing: the FP64 contraction
  // holds every CU's registers, and the scatter needs most CUs to reach its speed.)
  if ((st = launch_fit(P, E, nu, prec, coef, stream))) return st;
  if ((st = launch_contract(P, prec, coef, blocks, stream))) return st;
  return launch_scatter(P, prec, blocks, d_values, stream);
}
