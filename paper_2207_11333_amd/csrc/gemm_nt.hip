// NT-form MFMA GEMM (steps S1, S3 and the input-gradient products of S6 and
// S8); split-K partials are added by reduce.hip.  Shared tile code:
// mfma_tile.hpp.
#include "mfma_tile.hpp"

namespace hgnn {

namespace {

// --------------------------------------------------------------------------
// NT form
// --------------------------------------------------------------------------
// TAG only distinguishes launch sites in profiles (1: the update linear).
// Waves form a 2 x WGN grid over the BM x BN tile (NTH = 128 WGN threads).
template <int PREC, int BM, int BN, bool SPLIT, int TAG, int WGN>
// FP32: four waves per SIMD (the compiler fits the kernel in 128 registers;
// measured 1.7% faster end to end).  BF16: five, which holds the kernel to
// 96 registers (one spilled).  Left to itself the compiler takes 125, and
// the weight-gradient GEMM that runs beside this kernel on the second stream
// then slows by 40% on the 8-layer hidden-256 workload (measured 63k vs 75k
// graphs/s end to end).
__global__ void __launch_bounds__(128 * WGN, PREC == 0 ? 4 : 5)
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
  // interleaved trailing segments (three: the host accepts no other count):
  // tiles from il_start on cycle through them
  const int il_first = g.nseg - 3;
  int il_start = 0x7fffffff;
  if (g.ileave_n == 3) {
#pragma unroll
    for (int q = 0; q < kMaxSeg; ++q)
      if (q == il_first) il_start = cum[q];
  }

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
    int kt = t - cum[q];
    if (t >= il_start) {
      const unsigned r = (unsigned)(t - il_start);
      kt = (int)(r / 3u);
      q = il_first + (int)(r - 3u * (unsigned)kt);
    }
    const float *aptr = g.seg[q].ptr;
    const float *scale = g.seg[q].scale;
    const int lda = g.seg[q].ld, ks = g.seg[q].k, boff = g.seg[q].boff;
    const int k0 = kt * BK;
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
          if (g.addend) o += g.addend[(size_t)m * g.ld_add + n];
          if (g.relu) o = o > 0.f ? o : 0.f;
          if (g.mask && !(g.mask[(size_t)m * g.ldc + n] > 0.f)) o = 0.f;
          g.C[(size_t)m * g.ldc + n] = o;
        }
      }
    }
  }
}

constexpr int kNtWGN = 4; // 8 waves per workgroup

template <int PREC, int BM, int BN, int TAG>
hipError_t run_nt(const Dims *dims, int capM, const GemmNT &g, hipStream_t s,
                  hipEvent_t ev0, hipEvent_t ev1) {
  const int nt = cdiv(g.Ncols, BN);
  dim3 grid(cdiv(capM, BM) * nt, g.splits);
  // A non-null event pair is stamped with the GEMM kernel's own start and end.
  const dim3 block(128 * kNtWGN);
  const GemmNT ga = g;
  // the hi + lo weight form exists only for BF16 (no FP32 instance of it)
  bool split_weights = false;
  if constexpr (PREC == 1) split_weights = g.B_lo != nullptr;
  if (split_weights) {
    if constexpr (PREC == 1)
      hipExtLaunchKernelGGL(k_gemm_nt<PREC, BM, BN, true, TAG, kNtWGN>, grid, block, 0, s, ev0,
                            ev1, 0, dims, ga, nt);
  } else {
    hipExtLaunchKernelGGL(k_gemm_nt<PREC, BM, BN, false, TAG, kNtWGN>, grid, block, 0, s, ev0,
                          ev1, 0, dims, ga, nt);
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && g.splits > 1) e = launch_reduce_nt(dims, capM, g, s);
  return e;
}

// Output tiles are 64 rows x 128 columns: one tile spans the whole hidden
// width, so each weight tile is staged once per 64 rows.  When the tiles
// alone cannot cover the 256 CUs, K is split (at least two K tiles per
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
  if (sp > kt / 2) sp = kt / 2;
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
  if (g.ileave_n != 0) {
    if (g.ileave_n != 3 || g.nseg < 3) return hipErrorInvalidValue;
    for (int q = g.nseg - 2; q < g.nseg; ++q)
      if (g.seg[q].k != g.seg[g.nseg - 3].k) return hipErrorInvalidValue;
  }
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

} // namespace hgnn
