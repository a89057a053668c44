// MFMA GEMMs of the message, update and head-free linears (steps S1, S3 and
// their adjoints S6, S8).
//
// Two forms, both tiled for 256-thread workgroups (4 wave64s in a 2x2 grid)
// with operands staged through LDS in [row][k] order (k contiguous):
//  * gemm_nt:  C = act(sum_seg diag(scale_seg) A_seg B_seg^T + bias).  The
//    K dimension is a list of segments so that the update input
//    [h || A || s+ A || s- A] and the adjoint input [du || s+ du || s- du]
//    are read in place and scaled while being staged, never materialised.
//  * gemm_tn:  P[z] = X^T Yv over a fixed chunk z of the node rows (split-K),
//    reduced afterwards in a fixed order: weight gradients are deterministic
//    and need no atomics.
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
#include "common.hpp"

#include <type_traits>

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

// Multiply-accumulate one BK-deep LDS tile into the wave's accumulators.
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

// --------------------------------------------------------------------------
// NT form
// --------------------------------------------------------------------------
// TAG only distinguishes launch sites in profiles (1: the update linear).
// Waves form a 2 x WGN grid over the BM x BN tile (NTH = 128 WGN threads).
template <int PREC, int BM, int BN, bool SPLIT, int TAG, int WGN>
__global__ void __launch_bounds__(128 * WGN)
k_gemm_nt(const Dims *__restrict__ dims, const GemmNT g, int ntiles_n) {
  using P = Prec<PREC>;
  using T = typename P::T;
  constexpr int NTH = 128 * WGN;
  constexpr int BK = P::BK, LDA = BK + P::PAD;
  constexpr int WM = BM / 2, WN = BN / WGN, TM = WM / 16, TN = WN / 16;
  // A tile: BM x BK floats loaded as float4 -> NA vectors per thread
  constexpr int NA = BM * BK / 4 / NTH;
  // B tile: BN x BK elements loaded 16 bytes at a time
  constexpr int BVEC = (PREC == 0) ? 4 : 8;
  constexpr int NB = BN * BK / BVEC / NTH;
  static_assert(NA >= 1 && NB >= 1, "tile too small for 256 threads");
  __shared__ __attribute__((aligned(16))) T As[BM * LDA];
  __shared__ __attribute__((aligned(16))) T Bs[BN * LDA];
  __shared__ __attribute__((aligned(16))) T Bl[SPLIT ? BN * LDA : 1];

  const int M = g.M_fixed >= 0 ? g.M_fixed : dims->N;
  const int mtiles = (M + BM - 1) / BM;
  const int z = blockIdx.y;
  if ((int)blockIdx.x >= mtiles * ntiles_n) return;
  const int tile = xcd_tile(blockIdx.x, mtiles * ntiles_n);
  const int m0 = (tile / ntiles_n) * BM, n0 = (tile % ntiles_n) * BN;
  const int tid = threadIdx.x, wid = tid >> 6;
  const int wm0 = (wid / WGN) * WM, wn0 = (wid % WGN) * WN;

  // K tiles over all segments: cum[s] = first tile of segment s
  int cum[kMaxSeg + 1];
  cum[0] = 0;
#pragma unroll
  for (int q = 0; q < kMaxSeg; ++q)
    cum[q + 1] = cum[q] + (q < g.nseg && g.seg[q].k > 0 ? (g.seg[q].k + BK - 1) / BK : 0);
  // this split's contiguous range of K tiles [t_lo, t_lo + KT)
  const int KT_all = cum[kMaxSeg];
  const int t_lo = (int)((long long)KT_all * z / g.splits);
  const int KT = (int)((long long)KT_all * (z + 1) / g.splits) - t_lo;

  f4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  const T *Bg = reinterpret_cast<const T *>(g.B);
  const T *Blg = reinterpret_cast<const T *>(g.B_lo);
  // two register stages: tiles t and t+1 are in flight while t-1 computes.
  // Loads are unconditional from clamped (in-bounds) addresses and masked
  // by a select, so no branch forces the compiler to drain the load queue.
  f4 ra[2][NA], rb[2][NB], rl[2][SPLIT ? NB : 1];
  float rs[2][NA];
  int a_row[NA], a_col[NA];
  bool a_ok[NA];
#pragma unroll
  for (int j = 0; j < NA; ++j) {
    const int v = tid + j * NTH;
    const int m = m0 + v / (BK / 4);
    a_ok[j] = m < M;
    a_row[j] = min(m, M - 1);
    a_col[j] = (v % (BK / 4)) * 4;
  }
  int b_row[NB], b_col[NB];
  bool b_ok[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int v = tid + j * NTH;
    const int n = n0 + v / (BK / BVEC);
    b_ok[j] = n < g.Ncols;
    b_row[j] = min(n, g.Ncols - 1);
    b_col[j] = (v % (BK / BVEC)) * BVEC;
  }

  auto load = [&](auto st, int t) {
    constexpr int S = decltype(st)::value;
    t = t_lo + min(t, KT - 1);
    int q = 0;
#pragma unroll
    for (int u = 1; u < kMaxSeg; ++u) q += (t >= cum[u]) ? 1 : 0;
    const float *aptr = g.seg[q].ptr;
    const float *scale = g.seg[q].scale;
    const int lda = g.seg[q].ld, ks = g.seg[q].k, boff = g.seg[q].boff;
    const int k0 = (t - cum[q]) * BK;
    const float *sbase = scale ? scale : aptr;
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int k = k0 + a_col[j];
      const f4 val = *reinterpret_cast<const f4 *>(aptr + (size_t)a_row[j] * lda + min(k, ks - 4));
      ra[S][j] = (a_ok[j] && k < ks) ? val : f4{0.f, 0.f, 0.f, 0.f};
      rs[S][j] = sbase[a_row[j]];
    }
    if (!scale) {
#pragma unroll
      for (int j = 0; j < NA; ++j) rs[S][j] = 1.0f;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int k = k0 + b_col[j];
      const size_t off = (size_t)b_row[j] * g.ldb + boff + min(k, ks - BVEC);
      const bool ok = b_ok[j] && k < ks;
      const f4 val = *reinterpret_cast<const f4 *>(Bg + off);
      rb[S][j] = ok ? val : f4{0.f, 0.f, 0.f, 0.f};
      if constexpr (SPLIT) {
        const f4 vlo = *reinterpret_cast<const f4 *>(Blg + off);
        rl[S][j] = ok ? vlo : f4{0.f, 0.f, 0.f, 0.f};
      }
    }
  };
  auto stash = [&](auto st) {
    constexpr int S = decltype(st)::value;
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int v = tid + j * NTH;
      const int r = v / (BK / 4), c = (v % (BK / 4)) * 4;
      store4(As + r * LDA + c, ra[S][j] * rs[S][j]);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int v = tid + j * NTH;
      const int r = v / (BK / BVEC), c = (v % (BK / BVEC)) * BVEC;
      *reinterpret_cast<f4 *>(Bs + r * LDA + c) = rb[S][j]; // 16 raw bytes
      if constexpr (SPLIT) *reinterpret_cast<f4 *>(Bl + r * LDA + c) = rl[S][j];
    }
  };
  auto step = [&](auto st, int t) {
    __syncthreads();
    stash(st);
    __syncthreads();
    load(st, t + 2);
    mma_tile<PREC, TM, TN, LDA, BK>(As, Bs, wm0, wn0, acc);
    if constexpr (SPLIT) mma_tile<PREC, TM, TN, LDA, BK>(As, Bl, wm0, wn0, acc);
  };

  if (KT > 0) load(IC<0>{}, 0);
  if (KT > 1) load(IC<1>{}, 1);
  for (int t = 0; t < KT; t += 2) {
    step(IC<0>{}, t);
    if (t + 1 >= KT) break;
    step(IC<1>{}, t + 1);
  }

  const int lane = tid & 63;
  const int cr = 4 * (lane >> 4), cc = lane & 15;
  if (g.splits > 1) {
    float *Pz = g.P + (size_t)z * M * g.Ncols;
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int n = n0 + wn0 + j * 16 + cc;
      if (n >= g.Ncols) continue;
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int m = m0 + wm0 + i * 16 + cr + v;
          if (m < M) Pz[(size_t)m * g.Ncols + n] = acc[i][j][v];
        }
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int n = n0 + wn0 + j * 16 + cc;
    if (n >= g.Ncols) continue;
    const float bias = g.bias ? g.bias[n] : 0.f;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm0 + i * 16 + cr + v;
        if (m < M) {
          float o = acc[i][j][v] + bias;
          if (g.relu) o = o > 0.f ? o : 0.f;
          if (g.mask && !(g.mask[(size_t)m * g.ldc + n] > 0.f)) o = 0.f;
          g.C[(size_t)m * g.ldc + n] = o;
        }
      }
    }
  }
}

// --------------------------------------------------------------------------
// TN form (split-K weight gradients)
// --------------------------------------------------------------------------
template <int PREC, int BM, int BN>
__global__ void __launch_bounds__(256)
k_gemm_tn(const Dims *__restrict__ dims, const GemmTN g, int ntiles_n) {
  using P = Prec<PREC>;
  using T = typename P::T;
  constexpr int BK = P::BK / 2, LDA = BK + P::PAD;
  constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 16, TN = WN / 16;
  constexpr int NA = BM * BK / 4 / 256;
  constexpr int NB = BN * BK / 4 / 256;
  __shared__ __attribute__((aligned(16))) T As[BM * LDA];
  __shared__ __attribute__((aligned(16))) T Bs[BN * LDA];

  const int rows = dims->N;
  const int mtiles = (g.M + BM - 1) / BM;
  const int T2 = mtiles * ntiles_n;
  const int tile = xcd_tile(blockIdx.x % T2, T2);
  const int z = blockIdx.x / T2;
  const int m0 = (tile / ntiles_n) * BM, n0 = (tile % ntiles_n) * BN;
  int chunk = (rows + g.splits - 1) / g.splits;
  chunk = (chunk + BK - 1) / BK * BK;
  const int i_lo = z * chunk;
  const int i_hi = min(rows, i_lo + chunk);
  const int KT = i_hi > i_lo ? (i_hi - i_lo + BK - 1) / BK : 0;
  const int tid = threadIdx.x, wid = tid >> 6;
  const int wm0 = (wid >> 1) * WM, wn0 = (wid & 1) * WN;

  f4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  // Per-thread column pointers are fixed over the K loop (only the row i
  // moves); loads are unconditional from clamped rows and masked by select.
  f4 ra[2][NA], rb[2][NB];
  float rsc[2][NB];
  int a_il[NA], a_m[NA];
  bool a_ok[NA];
#pragma unroll
  for (int j = 0; j < NA; ++j) {
    const int v = tid + j * 256;
    a_il[j] = v / (BM / 4);
    const int m = m0 + (v % (BM / 4)) * 4;
    a_ok[j] = m < g.M;
    a_m[j] = min(m, g.M - 4);
  }
  const float *b_ptr[NB];
  const float *b_sptr[NB]; // row scales, or the operand itself when unscaled
  int b_ld[NB], b_il[NB], b_sstride[NB];
  bool b_ok[NB], b_has_scale[NB], b_ones[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int v = tid + j * 256;
    b_il[j] = v / (BN / 4);
    int n = n0 + (v % (BN / 4)) * 4;
    b_ok[j] = n < g.Ncols;
    n = min(n, g.Ncols - 4);
    int q = 0;
    while (q + 1 < g.nseg && n >= g.seg[q].ncols) { n -= g.seg[q].ncols; ++q; }
    // a constant segment reads nothing: point it at X (valid rows) and select
    b_ones[j] = g.seg[q].ptr == nullptr;
    b_ptr[j] = b_ones[j] ? g.X : g.seg[q].ptr + n;
    b_ld[j] = b_ones[j] ? g.ldx : g.seg[q].ld;
    b_has_scale[j] = g.seg[q].scale != nullptr;
    b_sptr[j] = b_has_scale[j] ? g.seg[q].scale : b_ptr[j];
    b_sstride[j] = b_has_scale[j] ? 1 : b_ld[j];
    if (b_ones[j]) b_ok[j] = b_ok[j] && n == 0;
  }
  const int i_last = max(i_hi - 1, 0);
  auto load = [&](auto st, int t) {
    constexpr int S = decltype(st)::value;
    const int i0 = i_lo + t * BK;
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int i = i0 + a_il[j];
      const f4 val = *reinterpret_cast<const f4 *>(g.X + (size_t)min(i, i_last) * g.ldx + a_m[j]);
      ra[S][j] = (a_ok[j] && i < i_hi) ? val : f4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int i = i0 + b_il[j];
      const int ic = min(i, i_last);
      f4 val = *reinterpret_cast<const f4 *>(b_ptr[j] + (size_t)ic * b_ld[j]);
      const float sv = b_sptr[j][(size_t)ic * b_sstride[j]];
      const float sc = b_has_scale[j] ? sv : 1.0f;
      if (b_ones[j]) val = f4{1.f, 0.f, 0.f, 0.f};
      rb[S][j] = (b_ok[j] && i < i_hi) ? val : f4{0.f, 0.f, 0.f, 0.f};
      rsc[S][j] = sc;
    }
  };
  auto stash = [&](auto st) {
    constexpr int S = decltype(st)::value;
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int v = tid + j * 256;
      const int il = v / (BM / 4), mc = (v % (BM / 4)) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) store1(As + (mc + e) * LDA + il, ra[S][j][e]);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int v = tid + j * 256;
      const int il = v / (BN / 4), nc = (v % (BN / 4)) * 4;
      const f4 val = rb[S][j] * rsc[S][j];
#pragma unroll
      for (int e = 0; e < 4; ++e) store1(Bs + (nc + e) * LDA + il, val[e]);
    }
  };
  auto step = [&](auto st, int t) {
    __syncthreads();
    stash(st);
    __syncthreads();
    load(st, min(t + 2, KT - 1));
    mma_tile<PREC, TM, TN, LDA, BK>(As, Bs, wm0, wn0, acc);
  };

  if (KT > 0) load(IC<0>{}, 0);
  if (KT > 1) load(IC<1>{}, 1);
  for (int t = 0; t < KT; t += 2) {
    step(IC<0>{}, t);
    if (t + 1 >= KT) break;
    step(IC<1>{}, t + 1);
  }

  const int lane = tid & 63;
  const int cr = 4 * (lane >> 4), cc = lane & 15;
  float *Pz = g.P + (size_t)z * g.M * g.Ncols;
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int n = n0 + wn0 + j * 16 + cc;
    if (n >= g.Ncols) continue;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm0 + i * 16 + cr + v;
        if (m < g.M) Pz[(size_t)m * g.Ncols + n] = acc[i][j][v];
      }
  }
}

// Ordered sum over split partials: 4 lanes per output each add a contiguous
// quarter of the splits in order, then the quarters are added in order
// (a fixed association, so the result is deterministic).
__device__ __forceinline__ float ordered_split_sum(const float *__restrict__ P, int splits,
                                                  long long stride, long long t, int q) {
  const int per = (splits + 3) / 4;
  const int z0 = q * per, z1 = min(splits, z0 + per);
  float s = 0.f;
  for (int z = z0; z < z1; ++z) s += P[(size_t)z * stride + t];
  const int lane = threadIdx.x & 63;
  const float s1 = __shfl(s, (lane & ~3) + 1, 64);
  const float s2 = __shfl(s, (lane & ~3) + 2, 64);
  const float s3 = __shfl(s, (lane & ~3) + 3, 64);
  const float s0 = __shfl(s, lane & ~3, 64);
  return ((s0 + s1) + s2) + s3;
}

// NT split-K: C = act(sum_z P[z] + bias) (* mask), z in order.
__global__ void __launch_bounds__(256)
k_reduce_nt(const Dims *__restrict__ dims, const GemmNT g) {
  const int M = g.M_fixed >= 0 ? g.M_fixed : dims->N;
  const long long gt = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long t = gt >> 2;
  const int q = (int)(gt & 3);
  const long long total = (long long)M * g.Ncols;
  const long long tc = t < total ? t : total - 1;
  float s = ordered_split_sum(g.P, g.splits, total, tc, q);
  if (t >= total || q != 0) return;
  const int m = (int)(t / g.Ncols), n = (int)(t % g.Ncols);
  if (g.bias) s += g.bias[n];
  if (g.relu) s = s > 0.f ? s : 0.f;
  if (g.mask && !(g.mask[(size_t)m * g.ldc + n] > 0.f)) s = 0.f;
  g.C[(size_t)m * g.ldc + n] = s;
}

// Sum the split-K partials in order and scatter them into the packed
// gradient layout (routes: see ReduceMap).
__global__ void __launch_bounds__(256) k_reduce_map(const ReduceMap r) {
  const long long gt = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long t = gt >> 2;
  const int q = (int)(gt & 3);
  const long long total = (long long)r.M * r.Ncols;
  const long long tc = t < total ? t : total - 1;
  const float s = ordered_split_sum(r.P, r.splits, total, tc, q);
  if (t >= total || q != 0) return;
  const int m = (int)(t / r.Ncols), c = (int)(t % r.Ncols);
  for (int k = 0; k < r.nroute; ++k) {
    const ReduceRoute &ro = r.route[k];
    if (m < ro.r0 || m >= ro.r1) continue;
    const int u = m - ro.r0;
    if (c < r.main_cols) {
      if (!ro.main) return;
      int oc;
      if (c < r.F) oc = c;
      else if (c < r.Fp) return;
      else oc = c - (r.Fp - r.F);
      ro.main[(size_t)u * ro.main_ld + ro.main_coloff + oc] = s;
    } else if (c == r.main_cols && ro.ones) {
      ro.ones[(size_t)(u % ro.ones_split) * ro.ones_stride + u / ro.ones_split] = s;
    }
    return;
  }
}

inline int cdiv(long long a, int b) { return (int)((a + b - 1) / b); }

constexpr int kNtWGN = 4; // 8 waves per workgroup

template <int PREC, int BM, int BN, int TAG>
hipError_t run_nt(const Dims *dims, int capM, const GemmNT &g, hipStream_t s,
                  hipEvent_t ev0, hipEvent_t ev1) {
  const int nt = cdiv(g.Ncols, BN);
  dim3 grid(cdiv(capM, BM) * nt, g.splits);
  if (ev0) (void)hipEventRecord(ev0, s);
  if (PREC == 1 && g.B_lo)
    k_gemm_nt<PREC, BM, BN, true, TAG, kNtWGN><<<grid, 128 * kNtWGN, 0, s>>>(dims, g, nt);
  else
    k_gemm_nt<PREC, BM, BN, false, TAG, kNtWGN><<<grid, 128 * kNtWGN, 0, s>>>(dims, g, nt);
  if (ev1) (void)hipEventRecord(ev1, s);
  if (g.splits > 1)
    k_reduce_nt<<<cdiv(4LL * capM * g.Ncols, 256), 256, 0, s>>>(dims, g);
  return hipGetLastError();
}

// Output tiles are 64 rows x 128 columns: one tile spans the whole hidden
// width, so each weight tile is staged once per 64 rows.  When the tiles
// alone cannot cover the 256 CUs, K is split (at least three K tiles per
// split, at most 8 splits).  Measured: more splits lose to their partial
// traffic at these sizes.
constexpr int kNtBM = 64, kNtBN = 128;

int nt_ktiles(int Ktot, int precision) {
  const int BK = precision ? Prec<1>::BK : Prec<0>::BK;
  return (Ktot + BK - 1) / BK;
}

} // namespace

int nt_splits(int capM, int Ncols, int Ktot, int precision) {
  const int tiles = cdiv(capM, kNtBM) * cdiv(Ncols, kNtBN);
  const int kt = nt_ktiles(Ktot, precision);
  int sp = 256 / (tiles > 0 ? tiles : 1);
  if (sp > kt / 3) sp = kt / 3;
  if (sp > 8) sp = 8;
  return sp < 1 ? 1 : sp;
}

// Upper bound of splits x capM x Ncols over every shape: a split is taken
// only while the tiles number fewer than 256, and then splits x tiles <= 256,
// so splits x capM x Ncols <= 256 x 64 x 128 floats.
size_t nt_partial_floats(int, int, int, int) { return (size_t)256 * kNtBM * kNtBN; }

hipError_t launch_gemm_nt(const Dims *dims, int capM, GemmNT g, int precision,
                          float *partials, hipStream_t s, int tag, hipEvent_t ev0,
                          hipEvent_t ev1) {
  if (capM <= 0 || g.Ncols <= 0) return hipSuccess;
  int Ktot = 0;
  for (int q = 0; q < g.nseg; ++q) Ktot += g.seg[q].k > 0 ? ((g.seg[q].k + 15) / 16) * 16 : 0;
  // segment tiles are counted per segment; bound the split by the sum
  int kt = 0;
  for (int q = 0; q < g.nseg; ++q)
    if (g.seg[q].k > 0) kt += nt_ktiles(g.seg[q].k, precision);
  g.splits = nt_splits(capM, g.Ncols, Ktot, precision);
  if (g.splits > kt / 2) g.splits = kt / 2 > 0 ? kt / 2 : 1;
  g.P = partials;
  if (g.splits > 1 && !partials) g.splits = 1;
  while (g.splits > 1 && (size_t)g.splits * capM * g.Ncols > nt_partial_floats(0, 0, 0, 0))
    --g.splits;
  if (tag == 1) {
    if (precision == 0) return run_nt<0, kNtBM, kNtBN, 1>(dims, capM, g, s, ev0, ev1);
    return run_nt<1, kNtBM, kNtBN, 1>(dims, capM, g, s, ev0, ev1);
  }
  if (precision == 0) return run_nt<0, kNtBM, kNtBN, 0>(dims, capM, g, s, ev0, ev1);
  return run_nt<1, kNtBM, kNtBN, 0>(dims, capM, g, s, ev0, ev1);
}

hipError_t launch_gemm_tn(const Dims *dims, const GemmTN &g, int precision,
                          hipStream_t s) {
  if (g.M <= 0 || g.Ncols <= 0) return hipSuccess;
  const int nt = cdiv(g.Ncols, 64);
  const int grid = cdiv(g.M, 64) * nt * g.splits;
  if (precision == 0)
    k_gemm_tn<0, 64, 64><<<grid, 256, 0, s>>>(dims, g, nt);
  else
    k_gemm_tn<1, 64, 64><<<grid, 256, 0, s>>>(dims, g, nt);
  return hipGetLastError();
}

namespace {
// Plain float4 copy used to calibrate the HBM byte counters.
__global__ void __launch_bounds__(256) k_calib_copy(const f4 *__restrict__ src,
                                                    f4 *__restrict__ dst, long long n4) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n4) dst[i] = src[i];
}
} // namespace

hipError_t launch_calib_copy(const float *src, float *dst, long long n, hipStream_t s) {
  const long long n4 = n / 4;
  if (n4 <= 0) return hipSuccess;
  k_calib_copy<<<cdiv(n4, 256), 256, 0, s>>>(reinterpret_cast<const f4 *>(src),
                                             reinterpret_cast<f4 *>(dst), n4);
  return hipGetLastError();
}

hipError_t launch_reduce_map(const ReduceMap &r, hipStream_t s) {
  const long long total = (long long)r.M * r.Ncols;
  if (total <= 0) return hipSuccess;
  k_reduce_map<<<cdiv(4 * total, 256), 256, 0, s>>>(r);
  return hipGetLastError();
}

} // namespace hgnn
