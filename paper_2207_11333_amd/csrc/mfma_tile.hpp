// Shared pieces of the MFMA GEMMs (gemm_nt.hip, gemm_tn.hip): operand types
// per precision, the XCD-aware tile order and the LDS tile multiply-accumulate
// (whole, or as per-chunk fragment reads and products for loops pipelined
// by hand).
//
// MFMA GEMMs of the message, update and head-free linears (steps S1, S3 and
// their adjoints S6, S8).
//
// Two forms:
//  * gemm_nt:  C = act(sum_seg diag(scale_seg) A_seg B_seg^T + bias).  The
//    K dimension is a list of segments so that the update input
//    [h || A || s+ A || s- A] and the adjoint input [du || s+ du || s- du]
//    are read in place and scaled while being staged, never materialised.
//    512-thread workgroups (8 wave64s in a 2x4 grid) on 64 x 128 tiles,
//    operands staged through LDS in [row][k] order (k contiguous); small
//    grids with long K ranges double-buffer the LDS tiles.
//  * gemm_tn:  P[z] = X^T Yv over a fixed chunk z of the node rows (split-K),
//    reduced afterwards in the fixed order z = 0, 1, ...: weight gradients
//    are deterministic and need no atomics.  256-thread workgroups (4
//    wave64s in a 2x2 grid) on 64 x 64 tiles; FP32 keeps the node-row tiles
//    k-major in LDS, BF16 transposes them to [row][k] while staging.
// Precision 0 runs v_mfma_f32_16x16x4_f32 on FP32 operands; precision 1
// rounds operands to BF16 (RNE, v_cvt_pk_bf16_f32) while staging and runs
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation.  Weights in BF16 mode come
// as a hi + lo pair of BF16 arrays (two MFMAs per tile): a weight's rounding
// error is the same for every node, so unlike the activations' it does not
// average out and it dominates the output error of deep stacks.
//
// MFMA lane layout (16x16 output block, wave64): lane l supplies row
// (l % 16) of A and column (l % 16) of B for the k-slots of lane group
// l / 16, and receives D[4 (l / 16) + v][l % 16] in accumulator v.  The
// FP32 form consumes one k per lane group per instruction; a lane reads four
// consecutive k with one 16-byte LDS load and issues four instructions, so
// the k-slot of group g in instruction s is k = 4 g + s.  A and B use the same
// assignment, so the sum over all k is unchanged.
#pragma once
#include "common.hpp"

#include <type_traits>
#include <utility>

namespace hgnn {

namespace {

template <int PREC> struct Prec;
template <> struct Prec<0> {
  using T = float;
  static constexpr int BK = 64;   // k per LDS tile
  static constexpr int PAD = 4;   // elements of row padding (16 bytes)
};
template <> struct Prec<1> {
  using T = __bf16;
  static constexpr int BK = 64;
  static constexpr int PAD = 8;
};

template <int V> using IC = std::integral_constant<int, V>;

// Map the dispatch order (round-robin over the 8 XCDs) to output tiles so that
// each XCD receives a contiguous range of tiles: the N tiles of one M tile,
// which share A rows, then share that XCD's L2.  A bijection on [0, T).
// (Measured: mapping whole node ranges to XCDs across kernels is slower.)
__device__ __forceinline__ int xcd_tile(int bid, int T) {
  constexpr int X = 8;
  const int xcd = bid % X, local = bid / X;
  const int per = T / X, rem = T % X;
  return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

// Split-K grids of the weight-gradient GEMMs: a group is output tiles of one
// chunk of rows, which read that chunk's rows of X and Y.  Groups are dealt
// to the 8 XCDs in turn, each group whole on one XCD, so what its tiles
// share is fetched from HBM once and then served by that XCD's L2 (spread
// over the XCDs, every tile fetched its part again).  bid -> (group grp,
// tile j of the group); grp = -1 for the padding blocks of the last round.
__host__ __device__ inline int tn_group_rows(int chunks, int mtiles) {
  // a whole chunk (every row tile) when the chunks deal evenly to the XCDs,
  // else one row tile of a chunk (its column tiles, which share X): few
  // large groups dealt unevenly leave XCDs idle.  Measured at 40k rows:
  // message weight gradient (24 chunks) 86 -> 82 us with whole chunks,
  // update weight gradient (30 chunks) 155 -> 177 us.
  return chunks % 8 == 0 ? mtiles : 1;
}
__device__ __forceinline__ void xcd_group(int bid, int ngroups, int gsize, int &grp, int &j) {
  constexpr int X = 8;
  const int x = bid % X, l = bid / X;
  const int gi = l / gsize;
  j = l - gi * gsize;
  grp = gi * X + x;
  if (grp >= ngroups) grp = -1;
}
inline int xcd_group_grid(int ngroups, int gsize) { return 8 * ((ngroups + 7) / 8) * gsize; }

// Bucketed tiles: bucket q's rows [brow[q], brow[q + 1]) of the
// (degree, id)-ordered rows are cut into ceil(n_q / T) tiles of T rows,
// bucket after bucket.  Lane q of the wave takes bucket q (lanes past nb see
// empty buckets), so the walk costs one round of loads and a wave scan rather
// than a dependent load per bucket.  total() is the tile count; find() gives,
// for tile `want`, the bucket bq (-1 past the last tile), the tile's first
// row r0 and the bucket's end r1, the same in every lane.
struct BucketWalk {
  int lo, hi, nt, incl, T;
  __device__ __forceinline__ BucketWalk(const int *__restrict__ brow, int nb, int T_) : T(T_) {
    const int lane = threadIdx.x & 63;
    const int q = min(lane, kMaxBuckets - 1);
    lo = brow[min(q, nb)];
    hi = brow[min(q + 1, nb)];
    nt = lane < kMaxBuckets ? (hi - lo + T - 1) / T : 0;
    incl = nt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(incl, o, 64);
      if (lane >= o) incl += t;
    }
  }
  __device__ __forceinline__ void find(int want, int &bq, int &r0, int &r1) const {
    const int first = incl - nt;
    const unsigned long long hit = __ballot(nt > 0 && want >= first && want < incl);
    bq = hit ? __ffsll((long long)hit) - 1 : -1;
    const int src = bq < 0 ? 0 : bq;
    // wave-uniform results: keep them in scalar registers
    r0 = __builtin_amdgcn_readfirstlane(__shfl(lo, src, 64) + (want - __shfl(first, src, 64)) * T);
    r1 = __builtin_amdgcn_readfirstlane(__shfl(hi, src, 64));
    bq = __builtin_amdgcn_readfirstlane(bq);
  }
  __device__ __forceinline__ int total() const {
    return __builtin_amdgcn_readfirstlane(__shfl(incl, 63, 64));
  }
};

__device__ __forceinline__ void store4(float *dst, f4 v) {
  *reinterpret_cast<f4 *>(dst) = v;
}
__device__ __forceinline__ void store4(__bf16 *dst, f4 v) {
  bf16x4 b;
  b[0] = (__bf16)v[0];
  b[1] = (__bf16)v[1];
  b[2] = (__bf16)v[2];
  b[3] = (__bf16)v[3];
  *reinterpret_cast<bf16x4 *>(dst) = b;
}
__device__ __forceinline__ void store1(float *dst, float v) { *dst = v; }
__device__ __forceinline__ void store1(__bf16 *dst, float v) { *dst = (__bf16)v; }

// One K chunk of a wave's operands: FP32 16 k (four per lane, one 16-byte
// LDS read per 16-row block), BF16 32 k (eight per lane).
template <int PREC> struct Frag;
template <> struct Frag<0> {
  using V = f4;
  static constexpr int KC = 16;
};
template <> struct Frag<1> {
  using V = bf16x8;
  static constexpr int KC = 32;
};

// Read the A and B fragments of the K chunk starting at kc.
template <int PREC, int TM, int TN, int LDA>
__device__ __forceinline__ void read_frags(const typename Prec<PREC>::T *As,
                                           const typename Prec<PREC>::T *Bs, int wm0, int wn0,
                                           int kc, typename Frag<PREC>::V (&a)[TM],
                                           typename Frag<PREC>::V (&b)[TN]) {
  using V = typename Frag<PREC>::V;
  constexpr int PER = PREC == 0 ? 4 : 8; // k per lane group
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int i = 0; i < TM; ++i)
    a[i] = *reinterpret_cast<const V *>(As + (wm0 + i * 16 + r) * LDA + kc + PER * g);
#pragma unroll
  for (int j = 0; j < TN; ++j)
    b[j] = *reinterpret_cast<const V *>(Bs + (wn0 + j * 16 + r) * LDA + kc + PER * g);
}

// Multiply-accumulate one K chunk: FP32 issues four k-slots s per 16-byte
// read, each over every (i, j) block; BF16 one instruction per block.
template <int PREC, int TM, int TN>
__device__ __forceinline__ void mma_frags(const typename Frag<PREC>::V (&a)[TM],
                                          const typename Frag<PREC>::V (&b)[TN],
                                          f4 (&acc)[TM][TN]) {
  if constexpr (PREC == 0) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][s], b[j][s], acc[i][j], 0, 0, 0);
  } else {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  }
}

// Multiply-accumulate one BK-deep LDS tile into the wave's accumulators:
// read_frags then mma_frags per K chunk, written out (the same order).
template <int PREC, int TM, int TN, int LDA, int BK>
__device__ __forceinline__ void mma_tile(const typename Prec<PREC>::T *As,
                                         const typename Prec<PREC>::T *Bs,
                                         int wm0, int wn0, f4 (&acc)[TM][TN]) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  if constexpr (PREC == 0) {
#pragma unroll
    for (int kc = 0; kc < BK; kc += 16) {
      f4 a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i)
        a[i] = *reinterpret_cast<const f4 *>(As + (wm0 + i * 16 + r) * LDA + kc + 4 * g);
#pragma unroll
      for (int j = 0; j < TN; ++j)
        b[j] = *reinterpret_cast<const f4 *>(Bs + (wn0 + j * 16 + r) * LDA + kc + 4 * g);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][s], b[j][s], acc[i][j], 0, 0, 0);
    }
  } else {
#pragma unroll
    for (int kc = 0; kc < BK; kc += 32) {
      bf16x8 a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i)
        a[i] = *reinterpret_cast<const bf16x8 *>(As + (wm0 + i * 16 + r) * LDA + kc + 8 * g);
#pragma unroll
      for (int j = 0; j < TN; ++j)
        b[j] = *reinterpret_cast<const bf16x8 *>(Bs + (wn0 + j * 16 + r) * LDA + kc + 8 * g);
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
}

// Call f(IC<0>{}), ..., f(IC<N-1>{}) in order.
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F &f, std::integer_sequence<int, I...>) {
  (f(IC<I>{}), ...);
}
template <int N, typename F> __device__ __forceinline__ void static_for(F &&f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}


inline int cdiv(long long a, int b) { return (int)((a + b - 1) / b); }

} // namespace

} // namespace hgnn
