// NT-form MFMA GEMM with its operand tiles copied from HBM straight into LDS
// (steps S1, S3 and the layer-input gradient of S6 + S8).
//
// Every A segment is in the product's own precision in HBM: FP32 as it lies,
// or for BF16 a copy its producer wrote (RNE-rounded, the rounding the
// register-staged kernel applies while staging).  A K tile then needs no
// conversion and goes from HBM to LDS by gfx950's LDS-DMA loads
// (global_load_lds_dwordx4: 16 bytes per lane, written to LDS in lane order),
// never through registers, which are left to the products.
//
// LDS rows are 128 bytes: one K tile holds 32 FP32 or 64 BF16 of k.  Chunk c
// (16 bytes) of row r is stored at 16 (c ^ (r & 7)), so the eight rows read by
// eight adjacent lanes of a fragment load fall in distinct banks (the LDS
// bank-conflict counter reads 0).  A DMA instruction fills 8 rows: lane L
// writes row L / 8, position L % 8, so it loads logical chunk (L % 8) ^ (L / 8)
// of that row.  The loads of a tile (A rows, weight rows, BF16 weight low
// halves) are dealt to the waves in turn, the same number to each.
//
// Pipeline: three LDS stages; tiles t + 1 and t + 2 are in flight while tile t
// computes.  Each wave counts its own DMA loads (vmcnt) and one plain
// s_barrier per tile (the fence of __syncthreads would wait for every load in
// flight) makes every wave's loads visible and frees the stage read by the
// previous tile.  The barrier sits before the tile's last products, which
// cover the next tile's fragment reads.
//
// Measured: a wave's LDS-DMA loads are served about one at a time, so the copy
// rate grows with the waves that issue them (a streaming test: four waves per
// CU about 8 TB/s from L2, sixteen about 25, whatever the number of loads each
// keeps in flight); every configuration runs eight waves.  Two tile shapes:
// 128 x 128 (waves of 64 x 32) for grids that fill the GPU, 64 x 64 (waves of
// 32 x 16) for smaller ones, whose time is set by how many tiles run at once
// (update linear, BF16, alone: 80 against 105 us for the register-staged
// kernel at 40k rows; 9.7 against 14.3 us at 4.5k rows with 64 x 64 tiles).
//
// Products and their order per output are those of the register-staged
// kernel when it runs unsplit (FP32: per 16 k, four k-slots of
// v_mfma_f32_16x16x4_f32; BF16: per 64 k, weight hi over k 0-31 and 32-63,
// then lo over the same), so outputs are bitwise equal to its unsplit form.
#include "mfma_tile.hpp"

namespace hgnn {

namespace {

typedef __attribute__((address_space(3))) void lds_t;

constexpr int kQRow = 128; // bytes per LDS row (one K tile)
constexpr int kQStages = 3;
constexpr int kQWGM = 2, kQWGN = 4; // waves of a workgroup

// s_waitcnt immediate for vmcnt(n) with lgkmcnt(0) (expcnt left alone)
template <int N> struct WaitVm {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  static constexpr int value = 0x0070 | (N & 15) | ((N >> 4) << 14);
};

// PREC 0: FP32 operands and weights; 1: BF16 operands, weights as hi + lo.
// BM x BN tile, WGM x WGN waves.
template <int PREC, int BM, int BN, int WGM, int WGN, int TAG>
__global__ void __launch_bounds__(64 * WGM * WGN, 1)
k_gemm_ntb(const Dims *__restrict__ dims, const GemmNTB g, int ntiles_n) {
  using T = typename Prec<PREC>::T;
  constexpr bool SPLIT = PREC == 1;
  constexpr int EPC = 16 / (int)sizeof(T);   // elements per 16-byte chunk
  constexpr int BKE = kQRow / (int)sizeof(T); // k per K tile
  constexpr int NW = WGM * WGN, WM = BM / WGM, WN = BN / WGN, TM = WM / 16, TN = WN / 16;
  constexpr int IA = BM / 8, IB = BN / 8, IT = IA + IB * (SPLIT ? 2 : 1);
  static_assert(IT % NW == 0 && TM >= 1 && TN >= 1, "tile shape");
  constexpr int DMA = IT / NW; // DMA loads per wave per K tile
  constexpr int SA = BM * kQRow, SB = BN * kQRow, STAGE = SA + SB * (SPLIT ? 2 : 1);
  __shared__ __attribute__((aligned(1024))) char smem[kQStages * STAGE];

  const int M = g.M_fixed >= 0 ? g.M_fixed : dims->N;
  int mtiles = (M + BM - 1) / BM;
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
  const int tid = threadIdx.x, w = tid >> 6, L = tid & 63;
  const int wm0 = (w / WGN) * WM, wn0 = (w % WGN) * WN;

  // K tiles over the segments: segment q holds tiles [cum[q], cum[q + 1])
  int cum[kMaxSeg + 1];
  cum[0] = 0;
#pragma unroll
  for (int q = 0; q < kMaxSeg; ++q) cum[q + 1] = cum[q] + (q < g.nseg ? g.seg[q].k / BKE : 0);
  const int KT = cum[kMaxSeg];

  // DMA load u of this wave is load w + NW u of the tile: A rows, then weight
  // rows, then (BF16) weight low halves, 8 rows each.  Rows and columns past
  // the matrix read clamped (valid) rows, whose products land only in
  // outputs that are never stored.
  const int dr = L >> 3;
  const int dk = EPC * ((L & 7) ^ dr); // first k of the chunk this lane loads
  int rowi[DMA], kind[DMA], ldsoff[DMA];
#pragma unroll
  for (int u = 0; u < DMA; ++u) {
    const int gi = w + NW * u;
    if (gi < IA) {
      kind[u] = 0;
      const int m = min(m0 + 8 * gi + dr, m_hi - 1);
      rowi[u] = g.perm ? g.perm[m] : m;
      ldsoff[u] = 8 * gi * kQRow;
    } else {
      const int bi = gi - IA, half = bi / IB, bb = bi - half * IB;
      kind[u] = 1 + half;
      rowi[u] = min(n0 + 8 * bb + dr, g.Ncols - 1);
      ldsoff[u] = SA + half * SB + 8 * bb * kQRow;
    }
  }
  const T *Bq = static_cast<const T *>(g.B) + (size_t)bq * g.bstride;
  const T *Lq = SPLIT ? static_cast<const T *>(g.B_lo) + (size_t)bq * g.bstride : Bq;

  // the loads of K tile t into the stage at byte offset st
  auto issue = [&](int t, int st) {
    int q = 0;
#pragma unroll
    for (int u = 1; u < kMaxSeg; ++u) q += (t >= cum[u]) ? 1 : 0;
    const int k0 = (t - cum[q]) * BKE;
    const T *ap = static_cast<const T *>(g.seg[q].ptr) + k0 + dk;
    const int lda = g.seg[q].ld;
    const size_t bo = (size_t)g.seg[q].boff + k0 + dk;
#pragma unroll
    for (int u = 0; u < DMA; ++u) {
      const T *src = kind[u] == 0 ? ap + (size_t)rowi[u] * lda
                                  : (kind[u] == 1 ? Bq : Lq) + (size_t)rowi[u] * g.ldb + bo;
      // the builtin takes a non-const pointer: without the cast the host pass
      // drops the kernel templates (their launch handles stay undefined)
      __builtin_amdgcn_global_load_lds((void *)src, (lds_t *)(smem + st + ldsoff[u]), 16, 0, 0);
    }
  };

  // fragment reads: lane (r = L % 16, group L / 16) takes row r of each
  // 16-row block and logical chunk 4 c + L / 16 of the tile's two halves c
  // (BF16: 8 k per lane of a 32-deep MFMA; FP32: 4 k, the k-slots of four
  // 4-deep MFMAs)
  using V = typename Frag<PREC>::V;
  const int fr = L & 15;
  const int p0 = (L >> 4) ^ (fr & 7);
  const int offA0 = (wm0 + fr) * kQRow + 16 * p0, offA1 = (wm0 + fr) * kQRow + 16 * (p0 ^ 4);
  const int offB0 = SA + (wn0 + fr) * kQRow + 16 * p0;
  const int offB1 = SA + (wn0 + fr) * kQRow + 16 * (p0 ^ 4);
  V fa[2][2][TM], fb[2][2][TN], fl[2][2][SPLIT ? TN : 1]; // [set][half][block]
  auto read = [&](auto set, int st) {
    constexpr int S = decltype(set)::value;
    const char *base = smem + st;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      fa[S][0][i] = *reinterpret_cast<const V *>(base + offA0 + 16 * i * kQRow);
      fa[S][1][i] = *reinterpret_cast<const V *>(base + offA1 + 16 * i * kQRow);
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      fb[S][0][j] = *reinterpret_cast<const V *>(base + offB0 + 16 * j * kQRow);
      fb[S][1][j] = *reinterpret_cast<const V *>(base + offB1 + 16 * j * kQRow);
    }
    if constexpr (SPLIT) {
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        fl[S][0][j] = *reinterpret_cast<const V *>(base + SB + offB0 + 16 * j * kQRow);
        fl[S][1][j] = *reinterpret_cast<const V *>(base + SB + offB1 + 16 * j * kQRow);
      }
    }
  };

  f4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  auto mm = [&](const V (&a)[TM], const V (&b)[TN]) { mma_frags<PREC, TM, TN>(a, b, acc); };
  auto next = [](int st) { return st == (kQStages - 1) * STAGE ? 0 : st + STAGE; };

  // tile t (register set S, LDS stage st): its first products; then, if a
  // tile follows, wait for it, refill this stage with tile t + 3 and read
  // tile t + 1's fragments; then the last products
  auto step = [&](auto set, int t, int st) {
    constexpr int S = decltype(set)::value;
    mm(fa[S][0], fb[S][0]);
    if constexpr (SPLIT) {
      mm(fa[S][1], fb[S][1]);
      mm(fa[S][0], fl[S][0]);
    }
    __builtin_amdgcn_sched_barrier(0);
    if (t + 1 < KT) {
      if (t + 2 < KT) __builtin_amdgcn_s_waitcnt(WaitVm<DMA>::value);
      else __builtin_amdgcn_s_waitcnt(WaitVm<0>::value);
      __builtin_amdgcn_s_barrier();
      __builtin_amdgcn_sched_barrier(0);
      if (t + 3 < KT) issue(t + 3, st);
      read(IC<1 - S>{}, next(st));
    }
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (SPLIT) mm(fa[S][1], fl[S][1]);
    else mm(fa[S][1], fb[S][1]);
  };

  issue(0, 0);
  if (KT > 1) issue(1, STAGE);
  if (KT > 2) issue(2, 2 * STAGE);
  if (KT > 2) __builtin_amdgcn_s_waitcnt(WaitVm<2 * DMA>::value);
  else if (KT > 1) __builtin_amdgcn_s_waitcnt(WaitVm<DMA>::value);
  else __builtin_amdgcn_s_waitcnt(WaitVm<0>::value);
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_sched_barrier(0);
  read(IC<0>{}, 0);
  int st = 0;
  for (int t = 0; t < KT; t += 2) {
    step(IC<0>{}, t, st);
    st = next(st);
    if (t + 1 >= KT) break;
    step(IC<1>{}, t + 1, st);
    st = next(st);
  }

  // Epilogue (as the register-staged kernel's): lane (cr = 4 (L / 16),
  // cc = L % 16) holds rows wm0 + 16 i + cr + v, columns wn0 + 16 j + cc; the
  // rows' nodes are fetched once, from clamped indices, without a branch.
  const int cr = 4 * (L >> 4), cc = L & 15;
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

inline bool al16(const void *p) { return ((uintptr_t)p & 15) == 0; }

// the large tile when its grid fills every CU at least once
bool large_tiles(int capM, const GemmNTB &g) {
  return (long long)(cdiv(capM, 128) + (g.perm ? g.nb : 0)) * cdiv(g.Ncols, 128) >= 256;
}

} // namespace

bool gemm_ntb_ok(const GemmNTB &g, int precision) {
  const int bke = precision ? 64 : 32, esz = precision ? 2 : 4;
  if (g.nseg < 1 || g.nseg > kMaxSeg || !g.B || !g.C || g.Ncols <= 0) return false;
  if ((precision == 1) != (g.B_lo != nullptr) || (precision == 0 && g.Cb)) return false;
  if ((g.ldb * esz) % 16 || !al16(g.B) || (g.B_lo && !al16(g.B_lo))) return false;
  if (g.perm && (!g.brow || g.nb < 1 || (g.bstride * esz) % 16)) return false;
  for (int q = 0; q < g.nseg; ++q) {
    const SegB &s = g.seg[q];
    if (!s.ptr || !al16(s.ptr) || s.k <= 0 || s.k % bke || (s.ld * esz) % 16 ||
        (s.boff * esz) % 16)
      return false;
  }
  return true;
}

hipError_t launch_gemm_ntb(const Dims *dims, int capM, const GemmNTB &g, int precision,
                           hipStream_t s, int tag, hipEvent_t ev0, hipEvent_t ev1) {
  if (capM <= 0) return hipSuccess;
  if (!gemm_ntb_ok(g, precision)) return hipErrorInvalidValue;
  const int B = large_tiles(capM, g) ? 128 : 64;
  const int nt = cdiv(g.Ncols, B);
  // bucketed rows: each bucket's last tile may be partial
  const dim3 grid((cdiv(capM, B) + (g.perm ? g.nb : 0)) * nt), block(64 * kQWGM * kQWGN);
  const int key = precision * 1000 + B * 10 + tag;
  switch (key) {
#define HGNN_NTB(P, BB, T)                                                                     \
  case P * 1000 + BB * 10 + T:                                                                 \
    hipExtLaunchKernelGGL(k_gemm_ntb<P, BB, BB, kQWGM, kQWGN, T>, grid, block, 0, s, ev0, ev1,  \
                          0, dims, g, nt);                                                     \
    break;
#define HGNN_NTB_TAGS(P, BB) HGNN_NTB(P, BB, 0) HGNN_NTB(P, BB, 1) HGNN_NTB(P, BB, 2) HGNN_NTB(P, BB, 4)
    HGNN_NTB_TAGS(0, 64)
    HGNN_NTB_TAGS(0, 128)
    HGNN_NTB_TAGS(1, 64)
    HGNN_NTB_TAGS(1, 128)
#undef HGNN_NTB_TAGS
#undef HGNN_NTB
  default:
    return hipErrorInvalidValue; // a tag without an instance
  }
  return hipGetLastError();
}

} // namespace hgnn
