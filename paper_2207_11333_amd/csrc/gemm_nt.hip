// NT-form MFMA GEMM (steps S1, S3 and the input-gradient products of S6 and
// S8); split-K partials are added by reduce.hip.  Shared tile code:
// mfma_tile.hpp.
#include "mfma_tile.hpp"

namespace hgnn {

namespace {

// --------------------------------------------------------------------------
// NT form
// --------------------------------------------------------------------------
// TAG only distinguishes launch sites in profiles: 1 the update linear (S3),
// 2 the message linear (S1), 3 the aggregate-input gradient (S6), 4 the
// layer-input gradient (S6 + S8), 0 the others.
// Waves form a 2 x WGN grid over the BM x BN tile (NTH = 128 WGN threads).
// DB doubles the LDS tiles: tile t+1 is staged while tile t computes, with one
// barrier per K step.  It needs 102 KB of LDS (FP32), so it is taken only
// where the grid holds at most one workgroup per CU anyway and each K split
// runs at least four K tiles (launch_gemm_nt).
// SCALE: some segment has per-row scales (the concatenated update and
// aggregate-input forms); without it no scale is loaded or applied.
template <int PREC, int BM, int BN, bool SPLIT, int TAG, int WGN, bool DB, bool SCALE>
// FP32: four waves per SIMD (the compiler fits the kernel in 128 registers;
// measured 1.7% faster end to end).  BF16: five, which holds the kernel to
// 96 registers (one spilled).  Left to itself the compiler takes 125, and
// the weight-gradient GEMM that runs beside this kernel on the second stream
// then slows by 40% on the 8-layer hidden-256 workload (measured 63k vs 75k
// graphs/s end to end).  DB: two, all that its LDS allows.
__global__ void __launch_bounds__(128 * WGN, (DB || BM * BN > 8192) ? 2 : 4)
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
  static_assert(NA >= 1 && NB >= 1, "tile too small for the workgroup");
  // With DB the second buffer is a separate set of arrays, so the compiler
  // can tell the stash into one buffer from the reads of the other.
  __shared__ __attribute__((aligned(16))) T As[BM * LDA];
  __shared__ __attribute__((aligned(16))) T Bs[BN * LDA];
  __shared__ __attribute__((aligned(16))) T Bl[SPLIT ? BN * LDA : 1];
  __shared__ __attribute__((aligned(16))) T As1[DB ? BM * LDA : 1];
  __shared__ __attribute__((aligned(16))) T Bs1[DB ? BN * LDA : 1];
  __shared__ __attribute__((aligned(16))) T Bl1[DB && SPLIT ? BN * LDA : 1];

  const int M = g.M_fixed >= 0 ? g.M_fixed : dims->N;
  // Row tiles: plain, or per degree bucket over the permuted rows (each
  // bucket's last tile may be partial).  The tile covers rows [m0, m_hi) of
  // the (permuted) row order and multiplies with bucket q's weights.
  int mtiles = (M + BM - 1) / BM;
  const int z = blockIdx.y;
  int mt, n0, m0, m_hi = M, bq = 0;
  if (g.perm) {
    const BucketWalk bw(g.brow, g.nb, BM);
    mtiles = bw.total();
    if ((int)blockIdx.x >= mtiles * ntiles_n) return;
    const int tile = xcd_tile(blockIdx.x, mtiles * ntiles_n);
    mt = tile / ntiles_n;
    n0 = (tile % ntiles_n) * BN;
    bw.find(mt, bq, m0, m_hi);
  } else {
    if ((int)blockIdx.x >= mtiles * ntiles_n) return;
    const int tile = xcd_tile(blockIdx.x, mtiles * ntiles_n);
    mt = tile / ntiles_n;
    n0 = (tile % ntiles_n) * BN;
    m0 = mt * BM;
  }
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

  const T *Bg = reinterpret_cast<const T *>(g.B) + (size_t)bq * g.bstride;
  const T *Blg = g.B_lo ? reinterpret_cast<const T *>(g.B_lo) + (size_t)bq * g.bstride : nullptr;
  // two register stages: tiles t and t+1 are in flight while t-1 computes.
  // Loads are unconditional from clamped (in-bounds) addresses.  The stages
  // keep the raw values and the row/column masks are applied only when a
  // stage is written to LDS: a select right after the load makes the
  // compiler wait for that load at once, so no load would overlap the
  // products of the step that issued it.
  // Rows and columns past the matrix read clamped (valid) rows: their
  // products land only in outputs that are never stored, so they need no
  // mask.  Only the K tail of a segment's last tile is zeroed, from klim (the
  // segment's k left at the tile's start, uniform), when it is below BK.
  f4 ra[2][NA], rb[2][NB], rl[2][SPLIT ? NB : 1];
  float rs[2][SCALE ? NA : 1];
  int klim[2];
  bool hs[2]; // the stage's segment has a row scale (SCALE only)
  int a_row[NA], a_col[NA];
#pragma unroll
  for (int j = 0; j < NA; ++j) {
    const int v = tid + j * NTH;
    const int m = m0 + v / (BK / 4);
    a_row[j] = min(m, m_hi - 1);
    if (g.perm) a_row[j] = g.perm[a_row[j]];
    a_col[j] = (v % (BK / 4)) * 4;
  }
  int b_row[NB], b_col[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int v = tid + j * NTH;
    const int n = n0 + v / (BK / BVEC);
    b_row[j] = min(n, g.Ncols - 1);
    b_col[j] = (v % (BK / BVEC)) * BVEC;
  }

  // Segment and K offset of tile t (of this split's range).
  auto locate = [&](int t, int &q, int &kt) {
    t = t_lo + min(t, KT - 1);
    q = 0;
#pragma unroll
    for (int u = 1; u < kMaxSeg; ++u) q += (t >= cum[u]) ? 1 : 0;
    kt = t - cum[q];
    if constexpr (DB) {
      // selects, not a branch: the loop body stays one block
      const unsigned r = (unsigned)(t - il_start);
      const int kt_il = (int)(r / 3u);
      const bool il = t >= il_start;
      q = il ? il_first + (int)(r - 3u * (unsigned)kt_il) : q;
      kt = il ? kt_il : kt;
    } else if (t >= il_start) {
      const unsigned r = (unsigned)(t - il_start);
      kt = (int)(r / 3u);
      q = il_first + (int)(r - 3u * (unsigned)kt);
    }
  };
  // Loads of tile t into stage S; the stage keeps the raw values, the bits of
  // the K-tail and edge masks and whether the segment has a row scale, all
  // applied when it is stashed.
  auto dload = [&](auto st, int t) {
    constexpr int S = decltype(st)::value;
    int q, kt;
    locate(t, q, kt);
    const float *aptr = g.seg[q].ptr;
    const float *scale = g.seg[q].scale;
    const int lda = g.seg[q].ld, ks = g.seg[q].k, boff = g.seg[q].boff;
    const int k0 = kt * BK;
    const float *sbase = scale ? scale : aptr; // a readable word either way
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int k = k0 + a_col[j];
      ra[S][j] = *reinterpret_cast<const f4 *>(aptr + (size_t)a_row[j] * lda + min(k, ks - 4));
      if constexpr (SCALE) rs[S][j] = sbase[a_row[j]];
    }
    klim[S] = ks - k0;
    hs[S] = scale != nullptr;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int k = k0 + b_col[j];
      const size_t off = (size_t)b_row[j] * g.ldb + boff + min(k, ks - BVEC);
      rb[S][j] = *reinterpret_cast<const f4 *>(Bg + off);
      if constexpr (SPLIT) rl[S][j] = *reinterpret_cast<const f4 *>(Blg + off);
    }
  };
  // register stage S goes to LDS buffer b (b = S when DB, else 0)
  auto stash_a = [&](auto st, auto buf) {
    constexpr int S = decltype(st)::value;
    T *Ad = decltype(buf)::value ? As1 : As;
    const f4 zero = {0.f, 0.f, 0.f, 0.f};
    // a uniform branch: only a segment's last, partial K tile pays for masks
    if (klim[S] >= BK) {
#pragma unroll
      for (int j = 0; j < NA; ++j) {
        const int v = tid + j * NTH;
        const int r = v / (BK / 4), c = (v % (BK / 4)) * 4;
        f4 x = ra[S][j];
        if constexpr (SCALE) x = x * (hs[S] ? rs[S][j] : 1.0f);
        store4(Ad + r * LDA + c, x);
      }
    } else {
#pragma unroll
      for (int j = 0; j < NA; ++j) {
        const int v = tid + j * NTH;
        const int r = v / (BK / 4), c = (v % (BK / 4)) * 4;
        f4 x = ra[S][j];
        if constexpr (SCALE) x = x * (hs[S] ? rs[S][j] : 1.0f);
        store4(Ad + r * LDA + c, c < klim[S] ? x : zero);
      }
    }
  };
  auto stash_b = [&](auto st, auto buf) {
    constexpr int S = decltype(st)::value;
    T *Bd = decltype(buf)::value ? Bs1 : Bs, *Ld = decltype(buf)::value ? Bl1 : Bl;
    const f4 zero = {0.f, 0.f, 0.f, 0.f};
    if (klim[S] >= BK) {
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const int v = tid + j * NTH;
        const int r = v / (BK / BVEC), c = (v % (BK / BVEC)) * BVEC;
        *reinterpret_cast<f4 *>(Bd + r * LDA + c) = rb[S][j]; // 16 raw bytes
        if constexpr (SPLIT) *reinterpret_cast<f4 *>(Ld + r * LDA + c) = rl[S][j];
      }
    } else {
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const int v = tid + j * NTH;
        const int r = v / (BK / BVEC), c = (v % (BK / BVEC)) * BVEC;
        const bool ok = c < klim[S];
        *reinterpret_cast<f4 *>(Bd + r * LDA + c) = ok ? rb[S][j] : zero;
        if constexpr (SPLIT) *reinterpret_cast<f4 *>(Ld + r * LDA + c) = ok ? rl[S][j] : zero;
      }
    }
  };
  auto stash = [&](auto st, auto buf) {
    stash_a(st, buf);
    stash_b(st, buf);
  };
  auto mma = [&](auto buf) {
    constexpr int b = decltype(buf)::value;
    const T *Ad = b ? As1 : As, *Bd = b ? Bs1 : Bs;
    mma_tile<PREC, TM, TN, LDA, BK>(Ad, Bd, wm0, wn0, acc);
    if constexpr (SPLIT) mma_tile<PREC, TM, TN, LDA, BK>(Ad, b ? Bl1 : Bl, wm0, wn0, acc);
  };
  // single buffer: the tile is staged between two barriers, then computed
  // (several workgroups share a CU here and cover each other's waits).
  // FP32 skips the clamped reloads past the range (a short K range, as in
  // the message linear's two K tiles, otherwise loads twice what it uses);
  // BF16 keeps them, since the branch makes its hi + lo form spill.
  auto step = [&](auto st, int t) {
    __syncthreads();
    stash(st, IC<0>{});
    __syncthreads();
    if (PREC == 1 || t + 2 < KT) dload(st, t + 2);
    mma(IC<0>{});
  };
  // double buffer, on entry: LDS buffer S holds tile t, register stage 1-S
  // holds tile t+1.  Stage S is free (its tile is in LDS) and takes tile t+2;
  // tile t+1 goes to the other buffer, last read by tile t-1's products,
  // which the previous step's barrier has retired.  With one workgroup per
  // CU nothing else covers a wave's waits, so the step is pipelined by hand
  // in chunks of MFMAs (one K chunk of one weight half each, in the order
  // mma_tile uses: the same sums in the same order as the single buffer,
  // bitwise equal for the non-negative finite row scales used here):
  // chunk c reads chunk c+1's fragments, the first chunk also issues tile
  // t+2's loads and the last ones write tile t+1 to LDS.  Scheduling
  // barriers between chunks keep the compiler from regrouping them.
  constexpr int KC = Frag<PREC>::KC, NKC = BK / KC, NCH = NKC * (SPLIT ? 2 : 1);
  constexpr int CH_SA = NCH >= 3 ? NCH - 2 : NCH - 1; // chunk that stashes A
  auto dstep = [&](auto st, int t) {
    constexpr int S = decltype(st)::value;
    const T *Ad = S ? As1 : As, *Bd = S ? Bs1 : Bs, *Ld = S ? Bl1 : Bl;
    typename Frag<PREC>::V fa[2][TM], fb[2][TN];
    read_frags<PREC, TM, TN, LDA>(Ad, Bd, wm0, wn0, 0, fa[0], fb[0]);
    static_for<NCH>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      if constexpr (c + 1 < NCH) {
        constexpr int n = c + 1;
        read_frags<PREC, TM, TN, LDA>(Ad, n >= NKC ? Ld : Bd, wm0, wn0, (n % NKC) * KC,
                                      fa[n & 1], fb[n & 1]);
      }
      if constexpr (c == 0) dload(st, t + 2);
      if constexpr (c == CH_SA) stash_a(IC<1 - S>{}, IC<1 - S>{});
      if constexpr (c == NCH - 1) stash_b(IC<1 - S>{}, IC<1 - S>{});
      mma_frags<PREC, TM, TN>(fa[c & 1], fb[c & 1], acc);
      __builtin_amdgcn_sched_barrier(0);
    });
    __syncthreads();
  };

  if constexpr (DB) {
    // tiles past the range clamp to its last one (KT = 1: tile 0 again)
    if (KT > 0) {
      dload(IC<0>{}, 0);
      dload(IC<1>{}, 1);
      stash(IC<0>{}, IC<0>{});
    }
    // drain tile 1's loads once here: otherwise the compiler carries their
    // pending register writes into the loop head and waits there every step
    __builtin_amdgcn_s_waitcnt(0x0f70); // vmcnt(0)
    __syncthreads();
    // pairs of steps, then an odd last tile: no branch inside the loop body
    int t = 0;
    for (; t + 1 < KT; t += 2) {
      dstep(IC<0>{}, t);
      dstep(IC<1>{}, t + 1);
    }
    if (t < KT) dstep(IC<0>{}, t);
  } else {
    if (KT > 0) dload(IC<0>{}, 0);
    if (KT > 1) dload(IC<1>{}, 1);
    for (int t = 0; t < KT; t += 2) {
      step(IC<0>{}, t);
      if (t + 1 >= KT) break;
      step(IC<1>{}, t + 1);
    }
  }

  // Epilogue.  The rows of this lane's outputs (and, bucketed, their nodes)
  // are fetched once, from clamped indices and without a branch, so their
  // loads are in flight together; only the stores are predicated.
  const int lane = tid & 63;
  const int cr = 4 * (lane >> 4), cc = lane & 15;
  int node[TM][4];
  bool rok[TM][4];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = m0 + wm0 + i * 16 + cr + v;
      rok[i][v] = r < m_hi;
      const int rr = min(r, m_hi - 1);
      node[i][v] = g.perm ? g.perm[rr] : rr;
    }
  if (g.splits > 1) {
    float *Pz = g.P + (size_t)z * M * g.Ncols;
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int n = n0 + wn0 + j * 16 + cc;
      if (n >= g.Ncols) continue;
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (rok[i][v]) Pz[(size_t)node[i][v] * g.Ncols + n] = acc[i][j][v];
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int n = n0 + wn0 + j * 16 + cc;
    const bool nok = n < g.Ncols;
    const int nc = min(n, g.Ncols - 1);
    const float bias = g.bias ? g.bias[nc] : 0.f;
    float o[TM][4];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) o[i][v] = acc[i][j][v] + bias;
    if (g.addend) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) o[i][v] += g.addend[(size_t)node[i][v] * g.ld_add + nc];
    }
    if (g.relu) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) o[i][v] = o[i][v] > 0.f ? o[i][v] : 0.f;
    }
    if (g.mask) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (!(g.mask[(size_t)node[i][v] * g.ldc + nc] > 0.f)) o[i][v] = 0.f;
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (nok && rok[i][v]) {
          g.C[(size_t)node[i][v] * g.ldc + n] = o[i][v];
          if (g.Cb) g.Cb[(size_t)node[i][v] * g.ldcb + n] = (__bf16)o[i][v];
        }
  }
}

constexpr int kNtWGN = 4; // 8 waves per workgroup
// The double-buffered form: grids of at most this many workgroups (one per
// CU) whose splits each run at least kNtDbMinKt K tiles.  Shorter K ranges
// leave it little to overlap, and its LDS and registers then mostly slow the
// weight-gradient GEMM beside it on the second stream.
constexpr long long kNtDbMaxGrid = 256;
constexpr int kNtDbMinKt = 4;

template <int PREC, int BM, int BN, int TAG, bool SCALE>
hipError_t run_nt(const Dims *dims, int capM, const GemmNT &g, bool db, hipStream_t s,
                  hipEvent_t ev0, hipEvent_t ev1) {
  const int nt = cdiv(g.Ncols, BN);
  // bucketed rows: each bucket's last tile may be partial
  dim3 grid((cdiv(capM, BM) + (g.perm ? g.nb : 0)) * nt, g.splits);
  // A non-null event pair is stamped with the GEMM kernel's own start and end.
  const dim3 block(128 * kNtWGN);
  const GemmNT ga = g;
  // the hi + lo weight form exists only for BF16 (no FP32 instance of it)
  bool split_weights = false;
  if constexpr (PREC == 1) split_weights = g.B_lo != nullptr;
  if (split_weights) {
    if constexpr (PREC == 1) {
      if (db)
        hipExtLaunchKernelGGL(k_gemm_nt<PREC, BM, BN, true, TAG, kNtWGN, true, SCALE>, grid,
                              block, 0, s, ev0, ev1, 0, dims, ga, nt);
      else
        hipExtLaunchKernelGGL(k_gemm_nt<PREC, BM, BN, true, TAG, kNtWGN, false, SCALE>, grid,
                              block, 0, s, ev0, ev1, 0, dims, ga, nt);
    }
  } else if (db) {
    hipExtLaunchKernelGGL(k_gemm_nt<PREC, BM, BN, false, TAG, kNtWGN, true, SCALE>, grid,
                          block, 0, s, ev0, ev1, 0, dims, ga, nt);
  } else {
    hipExtLaunchKernelGGL(k_gemm_nt<PREC, BM, BN, false, TAG, kNtWGN, false, SCALE>, grid,
                          block, 0, s, ev0, ev1, 0, dims, ga, nt);
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
  // BF16 products are never split: at 4.5k rows every site (message,
  // update, aggregate-input and layer-input gradients) is fastest unsplit,
  // in the double-buffered form where it applies (update 16.9 -> 14.7 us,
  // layer-input gradient 12.1 -> 10.8 us)
  if (precision == 1) g.splits = 1;
  if (g.max_splits > 0 && g.splits > g.max_splits) g.splits = g.max_splits;
  if (g.Cb) g.splits = 1; // the split reduction writes no BF16 copy
  g.P = partials;
  if (g.splits > 1 && !partials) g.splits = 1;
  while (g.splits > 1 && (size_t)g.splits * capM * g.Ncols > nt_partial_floats(0, 0, 0, 0))
    --g.splits;
  const long long grid =
      (long long)(cdiv(capM, kNtBM) + (g.perm ? g.nb : 0)) * cdiv(g.Ncols, kNtBN) * g.splits;
  const bool db = grid <= kNtDbMaxGrid && kt >= kNtDbMinKt * g.splits;
  // one instantiation per launch site, so that profiles name the site; row
  // scales occur only in the concatenated update and aggregate-input forms
  bool scaled = false;
  for (int q = 0; q < g.nseg; ++q) scaled = scaled || g.seg[q].scale != nullptr;
  if (scaled && tag != 1 && tag != 3) return hipErrorInvalidValue;
  switch (tag) {
#define HGNN_NT_RUN(T, SC)                                                                     \
  (precision == 0 ? run_nt<0, kNtBM, kNtBN, T, SC>(dims, capM, g, db, s, ev0, ev1)              \
                  : run_nt<1, kNtBM, kNtBN, T, SC>(dims, capM, g, db, s, ev0, ev1))
  case 1: return scaled ? HGNN_NT_RUN(1, true) : HGNN_NT_RUN(1, false);
  case 2: return HGNN_NT_RUN(2, false);
  case 3: return scaled ? HGNN_NT_RUN(3, true) : HGNN_NT_RUN(3, false);
  case 4: return HGNN_NT_RUN(4, false);
  default: return HGNN_NT_RUN(0, false);
#undef HGNN_NT_RUN
  }
}

} // namespace hgnn
