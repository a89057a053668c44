// TN-form MFMA GEMM (the weight gradients of S6 and S8, split-K over node
// chunks; reduce.hip adds the splits in order and scatters the result into
// the packed gradient).  Shared tile code: mfma_tile.hpp.
#include "mfma_tile.hpp"

namespace hgnn {

namespace {

// --------------------------------------------------------------------------
// TN form (split-K weight gradients)
// --------------------------------------------------------------------------
// TAG only distinguishes launch sites in profiles: 1 the update weight
// gradient (S6), 2 the message weight gradient (S8), 0 the others.  PERM:
// bucketed chunks (g.perm non-null), a template parameter so that the row
// lookups add no branch to the loop.  SCALE: some segment has row scales
// (the concatenated update input); without it no scale is loaded at all.
template <int PREC, int BM, int BN, int TAG, bool PERM, bool SCALE>
__global__ void __launch_bounds__(256)
k_gemm_tn(const Dims *__restrict__ dims, const GemmTN g, int ntiles_n) {
  using P = Prec<PREC>;
  using T = typename P::T;
  constexpr int BK = P::BK / 2, LDA = BK + P::PAD;
  constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 16, TN = WN / 16;
  constexpr int NA = BM * BK / 4 / 256;
  constexpr int NB = BN * BK / 4 / 256;
  // the A and B vectors of a thread lie in the same rows (a_il == b_il)
  static_assert(BM == BN && NA == NB, "square tiles");
  // FP32 keeps the tiles in LDS as they lie in memory, k-major ([k][m] and
  // [k][n], rows padded by 4 floats), written with 16-byte stores; the MFMA
  // operands are read one k-slot at a time.  With a 68-float row pitch the
  // lane groups of a read fall in distinct banks, whereas transposing on the
  // way in (the BF16 form, which needs 8 consecutive k per lane) puts a
  // wave's 64 scalar stores into 8 banks.
  constexpr bool KMAJ = PREC == 0;
  constexpr int LDKA = BM + 4, LDKB = BN + 4;
  __shared__ __attribute__((aligned(16))) T As[KMAJ ? BK * LDKA : BM * LDA];
  __shared__ __attribute__((aligned(16))) T Bs[KMAJ ? BK * LDKB : BN * LDA];

  const int rows = dims->N;
  const int mtiles = (g.M + BM - 1) / BM;
  const int zc = g.splits + (PERM ? g.nb : 0), gm = tn_group_rows(zc, mtiles);
  int grp, jt;
  xcd_group(blockIdx.x, zc * (mtiles / gm), gm * ntiles_n, grp, jt);
  if (grp < 0) return;
  const int z = grp / (mtiles / gm);
  const int m0 = ((grp % (mtiles / gm)) * gm + jt / ntiles_n) * BM, n0 = (jt % ntiles_n) * BN;
  int chunk = (rows + g.splits - 1) / g.splits;
  chunk = (chunk + BK - 1) / BK * BK;
  int i_lo = z * chunk;
  int i_hi = min(rows, i_lo + chunk);
  if constexpr (PERM) {
    // bucket-pure chunks over the permuted rows: bucket q holds
    // ceil(n_q / chunk) chunks, in bucket order; the chunks past the last
    // are empty and write zero partials
    int bq, r0, r1;
    BucketWalk(g.brow, g.nb, chunk).find(z, bq, r0, r1);
    i_lo = bq >= 0 ? r0 : 0;
    i_hi = bq >= 0 ? min(r1, r0 + chunk) : 0;
    if (m0 == 0 && n0 == 0 && threadIdx.x == 0) {
      g.zscale[2 * z] = bq >= 0 ? g.table[2 * bq] : 0.f;
      g.zscale[2 * z + 1] = bq >= 0 ? g.table[2 * bq + 1] : 0.f;
    }
  }
  const int KT = i_hi > i_lo ? (i_hi - i_lo + BK - 1) / BK : 0;
  const int tid = threadIdx.x, wid = tid >> 6;
  const int wm0 = (wid >> 1) * WM, wn0 = (wid & 1) * WN;

  f4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  // Per-thread column pointers are fixed over the K loop (only the row i
  // moves); loads are unconditional from clamped rows.  A stage keeps the
  // raw values and one bit per vector of whether its row is inside the
  // chunk; masks, constant columns and row scales are applied when the stage
  // is written to LDS, so the loads stay in flight over the step's products
  // (a select right after a load would make the compiler wait for it there).
  // Columns past the matrix read clamped (valid) columns: their products
  // land only in outputs that are never stored, so they need no mask.  Rows
  // past the chunk (its last step) are zeroed, from rlim (rows of the chunk
  // left at the step's first row, uniform) when it is below BK.
  f4 ra[2][NA], rb[2][NB];
  float rsc[2][NB];
  int rlim[2];
  int a_il[NA], a_m[NA];
#pragma unroll
  for (int j = 0; j < NA; ++j) {
    const int v = tid + j * 256;
    a_il[j] = v / (BM / 4);
    const int m = m0 + (v % (BM / 4)) * 4;
    a_m[j] = min(m, g.M - 4);
  }
  const float *b_ptr[NB];
  const float *b_sptr[NB]; // row scales, or the operand itself when unscaled
  int b_ld[NB], b_il[NB], b_sstride[NB];
  bool b_has_scale[NB], b_ones[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int v = tid + j * 256;
    b_il[j] = v / (BN / 4);
    int n = n0 + (v % (BN / 4)) * 4;
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
  }
  const int i_last = max(i_hi - 1, 0);
  // Row ids (nodes) of tile t's rows into slot Q.  With bucketed chunks
  // each is a load of the permutation: they are fetched one step before the
  // data loads that use them and issued ahead of that step's data loads, so
  // waiting for them never waits for data still in flight.
  int prow[2][NA];
  auto fetch_rows = [&](auto slot, int t) {
    constexpr int Q = decltype(slot)::value;
    const int i0 = i_lo + t * BK;
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int ic = min(i0 + a_il[j], i_last);
      if constexpr (PERM) prow[Q][j] = g.perm[ic];
      else prow[Q][j] = ic;
    }
  };
  // data loads of tile t into stage S, from the row ids in slot S
  auto load = [&](auto st, int t) {
    constexpr int S = decltype(st)::value;
    rlim[S] = i_hi - (i_lo + t * BK);
#pragma unroll
    for (int j = 0; j < NA; ++j)
      ra[S][j] = *reinterpret_cast<const f4 *>(g.X + (size_t)prow[S][j] * g.ldx + a_m[j]);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int ic = prow[S][j];
      rb[S][j] = *reinterpret_cast<const f4 *>(b_ptr[j] + (size_t)ic * b_ld[j]);
      if constexpr (SCALE) rsc[S][j] = b_sptr[j][(size_t)ic * b_sstride[j]];
    }
  };
  // (a uniform branch: only a chunk's last, partial step pays for masks)
  auto stash_rows = [&](auto st, auto masked) {
    constexpr int S = decltype(st)::value;
    constexpr bool MASK = decltype(masked)::value;
    const f4 zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int v = tid + j * 256;
      const int il = v / (BM / 4), mc = (v % (BM / 4)) * 4;
      const f4 av = (!MASK || a_il[j] < rlim[S]) ? ra[S][j] : zero;
      if constexpr (KMAJ) {
        store4(As + il * LDKA + mc, av);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) store1(As + (mc + e) * LDA + il, av[e]);
      }
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int v = tid + j * 256;
      const int il = v / (BN / 4), nc = (v % (BN / 4)) * 4;
      f4 val = b_ones[j] ? f4{1.f, 0.f, 0.f, 0.f} : rb[S][j];
      if constexpr (SCALE) val = val * (b_has_scale[j] ? rsc[S][j] : 1.0f);
      if constexpr (MASK) val = b_il[j] < rlim[S] ? val : zero;
      if constexpr (KMAJ) {
        store4(Bs + il * LDKB + nc, val);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) store1(Bs + (nc + e) * LDA + il, val[e]);
      }
    }
  };
  auto stash = [&](auto st) {
    constexpr int S = decltype(st)::value;
    if (rlim[S] >= BK) stash_rows(st, std::false_type{});
    else stash_rows(st, std::true_type{});
  };
  // k-major multiply: lane group g supplies k = kc + 4 g + s in instruction
  // s, the assignment mma_tile uses, so the sum runs in the same order.
  auto mma_kmajor = [&]() {
    const int lane = tid & 63;
    const int r = lane & 15, gq = lane >> 4;
#pragma unroll
    for (int kc = 0; kc < BK; kc += 16) {
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int k = kc + 4 * gq + s4;
        float a[TM], b[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) a[i] = As[k * LDKA + wm0 + i * 16 + r];
#pragma unroll
        for (int j = 0; j < TN; ++j) b[j] = Bs[k * LDKB + wn0 + j * 16 + r];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    }
  };
  // step t (stage S = t % 2): slot S holds tile t+2's rows (fetched in step
  // t-1), slot 1-S is free (tile t+1's loads used it) and takes tile t+3's
  // The scheduling barrier keeps the compiler from hoisting the other
  // stage's masking selects into this step: they would make it wait for the
  // loads still in flight.
  auto step = [&](auto st, int t) {
    constexpr int S = decltype(st)::value;
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
    stash(st);
    __syncthreads();
    fetch_rows(IC<1 - S>{}, min(t + 3, KT - 1));
    // the row ids are issued before the data loads: the next step waits for
    // them, and a wait for the youngest loads would wait for all
    __builtin_amdgcn_sched_barrier(0);
    load(st, min(t + 2, KT - 1));
    if constexpr (KMAJ) mma_kmajor();
    else mma_tile<PREC, TM, TN, LDA, BK>(As, Bs, wm0, wn0, acc);
  };

  if (KT > 0) {
    fetch_rows(IC<0>{}, 0);
    load(IC<0>{}, 0);
    fetch_rows(IC<1>{}, min(1, KT - 1));
    load(IC<1>{}, min(1, KT - 1)); // KT = 1: tile 0 again, never stashed
    fetch_rows(IC<0>{}, min(2, KT - 1));
  }
  // drain the prologue's loads once here: otherwise the compiler carries
  // their pending register writes into the loop head and waits for every
  // load in flight there, each step
  __builtin_amdgcn_s_waitcnt(0x0f70); // vmcnt(0)
  // pairs of steps, then an odd last tile: no branch inside the loop body,
  // so the waits for a stage's loads leave the other stage's loads in flight
  int t = 0;
  for (; t + 1 < KT; t += 2) {
    step(IC<0>{}, t);
    step(IC<1>{}, t + 1);
  }
  if (t < KT) step(IC<0>{}, t);

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

// BF16 weight gradients on 128 x 128 tiles (4 waves of 64 x 64), for grids
// large enough to fill the GPU with them.  Both operand tiles stay k-major
// in LDS, as they lie in memory ([node][m] and [node][n], converted to BF16
// and written 8 bytes at a time), and the MFMA operands -- 8 consecutive k
// of one row per lane -- come from gfx950's transposing LDS read
// (ds_read_b64_tr_b16): in each group of 16 lanes, lane i receives element
// i % 4 of the 8-byte pieces addressed by lanes 4k + i / 4, k = 0..3.  So
// when lane j of the group addresses row k0 + j / 4, columns c0 + 4 (j % 4)
// .. + 3, lane i receives column c0 + i of rows k0 .. k0 + 3; two such reads
// (k0 = 8 g and 8 g + 4 for lane group g) give the lane the k-slots
// 8 g .. 8 g + 7 that the 16 x 16 x 32 MFMA takes, the assignment of the
// 64 x 64 kernel, so both give the same sums in the same order.  The node
// chunks, the bucket walk and the partial layout are those of k_gemm_tn
// (BK = 32 as there).
typedef short v4s_t __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) v4s_t lds_v4s_t;
typedef __attribute__((address_space(3))) __bf16 lds_bf16_t;

template <int TAG, bool PERM, bool SCALE>
__global__ void __launch_bounds__(256, 2)
k_gemm_tn_tr(const Dims *__restrict__ dims, const GemmTN g, int ntiles_n) {
  constexpr int BM = 128, BN = 128, BK = 32;
  constexpr int WM = 64, WN = 64, TM = WM / 16, TN = WN / 16;
  constexpr int NV = BM * BK / 4 / 256; // float4 vectors per thread and operand
  // row pitch of the k-major tiles: 144 BF16 (288 bytes) puts the four rows
  // of one transposing read 32 bytes (8 banks) apart
  constexpr int LDK = BM + 16;
  __shared__ __attribute__((aligned(16))) __bf16 As[BK * LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[BK * LDK];

  const int rows = dims->N;
  const int mtiles = (g.M + BM - 1) / BM;
  const int zc = g.splits + (PERM ? g.nb : 0), gm = tn_group_rows(zc, mtiles);
  int grp, jt;
  xcd_group(blockIdx.x, zc * (mtiles / gm), gm * ntiles_n, grp, jt);
  if (grp < 0) return;
  const int z = grp / (mtiles / gm);
  const int m0 = ((grp % (mtiles / gm)) * gm + jt / ntiles_n) * BM, n0 = (jt % ntiles_n) * BN;
  int chunk = (rows + g.splits - 1) / g.splits;
  chunk = (chunk + BK - 1) / BK * BK;
  int i_lo = z * chunk;
  int i_hi = min(rows, i_lo + chunk);
  if constexpr (PERM) {
    int bq, r0, r1;
    BucketWalk(g.brow, g.nb, chunk).find(z, bq, r0, r1);
    i_lo = bq >= 0 ? r0 : 0;
    i_hi = bq >= 0 ? min(r1, r0 + chunk) : 0;
    if (m0 == 0 && n0 == 0 && threadIdx.x == 0) {
      g.zscale[2 * z] = bq >= 0 ? g.table[2 * bq] : 0.f;
      g.zscale[2 * z + 1] = bq >= 0 ? g.table[2 * bq + 1] : 0.f;
    }
  }
  const int KT = i_hi > i_lo ? (i_hi - i_lo + BK - 1) / BK : 0;
  const int tid = threadIdx.x, wid = tid >> 6;
  const int wm0 = (wid >> 1) * WM, wn0 = (wid & 1) * WN;

  f4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  // vector j of a thread: row (tid / 32) + 8 j of the tile, columns c .. c + 3
  // of both operand tiles (the tiles are equally wide, so every vector of a
  // thread has the same columns and one set of column pointers serves all)
  const int c = (tid % (BM / 4)) * 4, il0 = tid / (BM / 4);
  constexpr int RSTEP = 256 / (BM / 4);
  // columns past the matrix and rows past the chunk: as in k_gemm_tn
  const int a_m = min(m0 + c, g.M - 4);
  int n = min(n0 + c, g.Ncols - 4);
  int q = 0;
  while (q + 1 < g.nseg && n >= g.seg[q].ncols) { n -= g.seg[q].ncols; ++q; }
  const bool b_ones = g.seg[q].ptr == nullptr;
  const float *b_ptr = b_ones ? g.X : g.seg[q].ptr + n;
  const int b_ld = b_ones ? g.ldx : g.seg[q].ld;
  const bool b_has_scale = g.seg[q].scale != nullptr;
  const float *b_sptr = b_has_scale ? g.seg[q].scale : b_ptr;
  const int b_sstride = b_has_scale ? 1 : b_ld;
  const int i_last = max(i_hi - 1, 0);
  f4 ra[2][NV], rb[2][NV];
  float rsc[2][NV];
  int rlim[2];
  int prow[2][NV];
  auto fetch_rows = [&](auto slot, int t) {
    constexpr int Q = decltype(slot)::value;
    const int i0 = i_lo + t * BK + il0;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const int ic = min(i0 + RSTEP * j, i_last);
      if constexpr (PERM) prow[Q][j] = g.perm[ic];
      else prow[Q][j] = ic;
    }
  };
  auto load = [&](auto st, int t) {
    constexpr int S = decltype(st)::value;
    rlim[S] = i_hi - (i_lo + t * BK);
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const int r = prow[S][j];
      ra[S][j] = *reinterpret_cast<const f4 *>(g.X + (size_t)r * g.ldx + a_m);
      rb[S][j] = *reinterpret_cast<const f4 *>(b_ptr + (size_t)r * b_ld);
      if constexpr (SCALE) rsc[S][j] = b_sptr[(size_t)r * b_sstride];
    }
  };
  auto stash_rows = [&](auto st, auto masked) {
    constexpr int S = decltype(st)::value;
    constexpr bool MASK = decltype(masked)::value;
    const f4 zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const bool in = !MASK || il0 + RSTEP * j < rlim[S];
      f4 bv = b_ones ? f4{1.f, 0.f, 0.f, 0.f} : rb[S][j];
      if constexpr (SCALE) bv = bv * (b_has_scale ? rsc[S][j] : 1.0f);
      store4(As + (il0 + RSTEP * j) * LDK + c, in ? ra[S][j] : zero);
      store4(Bs + (il0 + RSTEP * j) * LDK + c, in ? bv : zero);
    }
  };
  auto stash = [&](auto st) {
    constexpr int S = decltype(st)::value;
    if (rlim[S] >= BK) stash_rows(st, std::false_type{});
    else stash_rows(st, std::true_type{});
  };
  // lane part of a transposing read: row 8 g + 4 p + (li / 4), column
  // 4 (li % 4) of the 16-wide block
  const int lane = tid & 63;
  const int li = lane & 15, lg = lane >> 4;
  const int tr_off0 = (8 * lg + (li >> 2)) * LDK + 4 * (li & 3);
  const int tr_off1 = tr_off0 + 4 * LDK;
  auto frag = [&](const __bf16 *base, int c0) {
    const lds_bf16_t *p = (const lds_bf16_t *)base + c0;
    const v4s_t lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s_t *)(p + tr_off0));
    const v4s_t hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s_t *)(p + tr_off1));
    typedef short v8s_t __attribute__((ext_vector_type(8)));
    const v8s_t w = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    return __builtin_bit_cast(bf16x8, w);
  };
  auto mma = [&]() {
    bf16x8 a[TM], b[TN];
#pragma unroll
    for (int i = 0; i < TM; ++i) a[i] = frag(As, wm0 + 16 * i);
#pragma unroll
    for (int j = 0; j < TN; ++j) b[j] = frag(Bs, wn0 + 16 * j);
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  };
  // scheduling barrier: as in k_gemm_tn
  auto step = [&](auto st, int t) {
    constexpr int S = decltype(st)::value;
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
    stash(st);
    __syncthreads();
    fetch_rows(IC<1 - S>{}, min(t + 3, KT - 1));
    // the row ids are issued before the data loads: the next step waits for
    // them, and a wait for the youngest loads would wait for all
    __builtin_amdgcn_sched_barrier(0);
    load(st, min(t + 2, KT - 1));
    mma();
  };
  if (KT > 0) {
    fetch_rows(IC<0>{}, 0);
    load(IC<0>{}, 0);
    fetch_rows(IC<1>{}, min(1, KT - 1));
    load(IC<1>{}, min(1, KT - 1)); // KT = 1: tile 0 again, never stashed
    fetch_rows(IC<0>{}, min(2, KT - 1));
  }
  // drain the prologue's loads once here: otherwise the compiler carries
  // their pending register writes into the loop head and waits for every
  // load in flight there, each step
  __builtin_amdgcn_s_waitcnt(0x0f70); // vmcnt(0)
  // pairs of steps, then an odd last tile: no branch inside the loop body,
  // so the waits for a stage's loads leave the other stage's loads in flight
  int t = 0;
  for (; t + 1 < KT; t += 2) {
    step(IC<0>{}, t);
    step(IC<1>{}, t + 1);
  }
  if (t < KT) step(IC<0>{}, t);

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

} // namespace

template <int TAG, bool PERM, bool SCALE>
static void run_tn(const Dims *dims, const GemmTN &g, hipStream_t s, hipEvent_t ev0,
                   hipEvent_t ev1, int grid, int nt) {
  // a non-null event pair is stamped with the kernel's own start and end
  hipExtLaunchKernelGGL(k_gemm_tn<0, 64, 64, TAG, PERM, SCALE>, dim3(grid), dim3(256), 0, s,
                        ev0, ev1, 0, dims, g, nt);
}

template <int TAG, bool PERM, bool SCALE>
static void run_tn_tr(const Dims *dims, const GemmTN &g, hipStream_t s, hipEvent_t ev0,
                      hipEvent_t ev1, int grid, int nt) {
  hipExtLaunchKernelGGL(k_gemm_tn_tr<TAG, PERM, SCALE>, dim3(grid), dim3(256), 0, s, ev0, ev1,
                        0, dims, g, nt);
}

// FP32: 64 x 64 tiles (k_gemm_tn); BF16: 128 x 128 tiles read through the
// transposing LDS loads (k_gemm_tn_tr).  Measured at 40k nodes: the BF16
// update weight gradient 257 -> 139 us and the message weight gradient
// 115 -> 70 us at their best split counts, with bitwise equal partials.
// Instances: the bucketed update weight gradient (no row scales), the
// concatenated one (scaled segments), the message weight gradient (no
// scales) and a general one for the other sites.
hipError_t launch_gemm_tn(const Dims *dims, const GemmTN &g, int precision,
                          hipStream_t s, int tag, hipEvent_t ev0, hipEvent_t ev1) {
  if (g.M <= 0 || g.Ncols <= 0) return hipSuccess;
  bool scaled = false;
  for (int q = 0; q < g.nseg; ++q) scaled = scaled || g.seg[q].scale != nullptr;
  if (tag == 1 && g.perm && scaled) return hipErrorInvalidValue;
  if (tag == 2 && (scaled || g.perm)) tag = 0;
  if (tag == 0 && g.perm) return hipErrorInvalidValue;
  const int T = precision ? 128 : 64;
  const int nt = cdiv(g.Ncols, T);
  const int zc = g.splits + (g.perm ? g.nb : 0), mt = cdiv(g.M, T), gm = tn_group_rows(zc, mt);
  const int grid = xcd_group_grid(zc * (mt / gm), gm * nt);
  if (precision) {
    if (tag == 1 && g.perm) run_tn_tr<1, true, false>(dims, g, s, ev0, ev1, grid, nt);
    else if (tag == 1) run_tn_tr<1, false, true>(dims, g, s, ev0, ev1, grid, nt);
    else if (tag == 2) run_tn_tr<2, false, false>(dims, g, s, ev0, ev1, grid, nt);
    else run_tn_tr<0, false, true>(dims, g, s, ev0, ev1, grid, nt);
  } else {
    if (tag == 1 && g.perm) run_tn<1, true, false>(dims, g, s, ev0, ev1, grid, nt);
    else if (tag == 1) run_tn<1, false, true>(dims, g, s, ev0, ev1, grid, nt);
    else if (tag == 2) run_tn<2, false, false>(dims, g, s, ev0, ev1, grid, nt);
    else run_tn<0, false, true>(dims, g, s, ev0, ev1, grid, nt);
  }
  return hipGetLastError();
}

} // namespace hgnn
