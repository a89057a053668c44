// NT-form MFMA GEMM on BF16 operands (steps S1, S3 and the layer-input
// gradient of S6 + S8 in BF16 mode, when their inputs have BF16 copies).
//
// Every A segment is already BF16 in HBM (its producer wrote the RNE-rounded
// copy), so a K tile needs no conversion: it is copied from HBM to LDS by
// the LDS-DMA loads of gfx950 (global_load_lds_dwordx4: 16 bytes per lane,
// written to LDS in lane order), never passing through registers, which are
// left to the products: 128 x 128 tiles, eight waves in a 2 x 4 grid, each
// wave 64 x 32 of output (4 x 2 MFMA blocks).  Measured: a wave's LDS-DMA
// loads are served about one at a time, so the copy rate grows with the
// waves that issue them (four waves per CU reach about 8 TB/s from L2,
// sixteen about 25); eight waves of 64 x 32 beat four of 64 x 64 (update
// linear at 40k rows: 80 against 96 us, the register-staged kernel 105).
//
// Pipeline: three LDS stages of one 64-deep K tile each (A, weight hi, weight
// lo: 48 KB); tiles t + 1 and t + 2 are in flight while tile t computes.
// Each wave counts its own DMA loads (vmcnt) and one barrier per tile makes
// every wave's loads visible and frees the stage read by the previous tile
// (a plain s_barrier: the fence of __syncthreads would wait for every load
// in flight).  The barrier sits before the tile's last quarter of MFMAs,
// which covers the next tile's fragment reads.
//
// LDS rows are 128 bytes (64 BF16 of k): chunk c (8 k) of row r is stored at
// 16 (c ^ (r & 7)), so the eight rows read by eight adjacent lanes of a
// fragment load fall in distinct banks.  A DMA instruction fills 8 rows:
// lane L writes row L / 8, position L % 8, so it loads logical chunk
// (L % 8) ^ (L / 8) of that row.
//
// Products and their order are those of the register-staged kernel's BF16
// hi + lo form on the same operand values (per 64-deep K tile: weight hi over
// k 0-31, hi over 32-63, lo over 0-31, lo over 32-63), so the outputs are
// bitwise equal to it.
#include "mfma_tile.hpp"

namespace hgnn {

namespace {

typedef __attribute__((address_space(3))) void lds_t;

constexpr int kQBM = 128, kQBN = 128, kQBK = 64;
constexpr int kQRow = kQBK * 2;              // bytes per LDS row
constexpr int kQA = kQBM * kQRow;            // A tile bytes
constexpr int kQB = kQBN * kQRow;            // one weight half's tile bytes
constexpr int kQStage = kQA + 2 * kQB;       // 48 KB
constexpr int kQStages = 3;

// s_waitcnt immediate for vmcnt(n) with lgkmcnt(0) (expcnt left alone)
template <int N> struct WaitVm {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  static constexpr int value = 0x0070 | (N & 15) | ((N >> 4) << 14);
};

// WGM x WGN waves, each (128 / WGM) x (128 / WGN) of output.
template <int TAG, int WGM, int WGN>
__global__ void __launch_bounds__(64 * WGM * WGN, 1)
k_gemm_ntb(const Dims *__restrict__ dims, const GemmNTB g, int ntiles_n) {
  constexpr int NW = WGM * WGN, WM = kQBM / WGM, WN = kQBN / WGN, TM = WM / 16, TN = WN / 16;
  constexpr int RPW = kQBM / NW;   // rows of each operand tile one wave loads
  constexpr int JD = RPW / 8;      // DMA loads per wave per operand tile
  constexpr int DMA = 3 * JD;      // per wave per K tile
  static_assert(kQBM == kQBN && RPW % 8 == 0 && TM >= 1 && TN >= 1, "tile shape");
  __shared__ __attribute__((aligned(1024))) char smem[kQStages * kQStage];

  const int M = g.M_fixed >= 0 ? g.M_fixed : dims->N;
  int mtiles = (M + kQBM - 1) / kQBM;
  int mt, n0, m0, m_hi = M, bq = 0;
  if (g.perm) {
    const BucketWalk bw(g.brow, g.nb, kQBM);
    mtiles = bw.total();
    if ((int)blockIdx.x >= mtiles * ntiles_n) return;
    const int tile = xcd_tile(blockIdx.x, mtiles * ntiles_n);
    mt = tile / ntiles_n;
    n0 = (tile % ntiles_n) * kQBN;
    bw.find(mt, bq, m0, m_hi);
  } else {
    if ((int)blockIdx.x >= mtiles * ntiles_n) return;
    const int tile = xcd_tile(blockIdx.x, mtiles * ntiles_n);
    mt = tile / ntiles_n;
    n0 = (tile % ntiles_n) * kQBN;
    m0 = mt * kQBM;
  }
  const int tid = threadIdx.x, w = tid >> 6, L = tid & 63;
  const int wm0 = (w / WGN) * WM, wn0 = (w % WGN) * WN;

  // K tiles over the segments: segment q holds tiles [cum[q], cum[q + 1])
  int cum[kMaxSeg + 1];
  cum[0] = 0;
#pragma unroll
  for (int q = 0; q < kMaxSeg; ++q) cum[q + 1] = cum[q] + (q < g.nseg ? g.seg[q].k / kQBK : 0);
  const int KT = cum[kMaxSeg];

  // DMA roles: wave w fills rows RPW w .. RPW (w + 1) - 1 of each tile, 8 per load;
  // rows and columns past the matrix read clamped (valid) rows, whose
  // products land only in outputs that are never stored
  const int dr = L >> 3;
  const int dk = 8 * ((L & 7) ^ dr); // first k of the chunk this lane loads
  int anode[JD], bcol[JD];
#pragma unroll
  for (int j = 0; j < JD; ++j) {
    const int m = min(m0 + RPW * w + 8 * j + dr, m_hi - 1);
    anode[j] = g.perm ? g.perm[m] : m;
    bcol[j] = min(n0 + RPW * w + 8 * j + dr, g.Ncols - 1);
  }
  const __bf16 *Bq = g.B + (size_t)bq * g.bstride;
  const __bf16 *Lq = g.B_lo + (size_t)bq * g.bstride;
  char *const wa = smem + RPW * w * kQRow; // this wave's rows of stage 0

  // the loads of K tile t into the stage at byte offset st
  auto issue = [&](int t, int st) {
    int q = 0;
#pragma unroll
    for (int u = 1; u < kMaxSeg; ++u) q += (t >= cum[u]) ? 1 : 0;
    const int k0 = (t - cum[q]) * kQBK;
    const __bf16 *ap = g.seg[q].ptr + k0 + dk;
    const int lda = g.seg[q].ld;
    const size_t bo = (size_t)g.seg[q].boff + k0 + dk;
#pragma unroll
    for (int j = 0; j < JD; ++j)
      __builtin_amdgcn_global_load_lds(ap + (size_t)anode[j] * lda,
                                       (lds_t *)(wa + st + 8 * j * kQRow), 16, 0, 0);
#pragma unroll
    for (int j = 0; j < JD; ++j)
      __builtin_amdgcn_global_load_lds(Bq + (size_t)bcol[j] * g.ldb + bo,
                                       (lds_t *)(wa + st + kQA + 8 * j * kQRow), 16, 0, 0);
#pragma unroll
    for (int j = 0; j < JD; ++j)
      __builtin_amdgcn_global_load_lds(Lq + (size_t)bcol[j] * g.ldb + bo,
                                       (lds_t *)(wa + st + kQA + kQB + 8 * j * kQRow), 16, 0, 0);
  };

  // fragment reads: lane (r = L % 16, group L / 16) takes row r of each
  // 16-row block, logical chunk 4 c + L / 16 (k 32 c + 8 (L / 16) ..)
  const int fr = L & 15;
  const int p0 = (L >> 4) ^ (fr & 7);
  const int offA0 = (wm0 + fr) * kQRow + 16 * p0, offA1 = (wm0 + fr) * kQRow + 16 * (p0 ^ 4);
  const int offB0 = kQA + (wn0 + fr) * kQRow + 16 * p0;
  const int offB1 = kQA + (wn0 + fr) * kQRow + 16 * (p0 ^ 4);
  bf16x8 fa[2][2][TM], fb[2][2][TN], fl[2][2][TN]; // [register set][k chunk][block]
  auto read = [&](auto set, int st) {
    constexpr int S = decltype(set)::value;
    const char *base = smem + st;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      fa[S][0][i] = *reinterpret_cast<const bf16x8 *>(base + offA0 + 16 * i * kQRow);
      fa[S][1][i] = *reinterpret_cast<const bf16x8 *>(base + offA1 + 16 * i * kQRow);
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      fb[S][0][j] = *reinterpret_cast<const bf16x8 *>(base + offB0 + 16 * j * kQRow);
      fb[S][1][j] = *reinterpret_cast<const bf16x8 *>(base + offB1 + 16 * j * kQRow);
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      fl[S][0][j] = *reinterpret_cast<const bf16x8 *>(base + kQB + offB0 + 16 * j * kQRow);
      fl[S][1][j] = *reinterpret_cast<const bf16x8 *>(base + kQB + offB1 + 16 * j * kQRow);
    }
  };

  f4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  auto mm = [&](const bf16x8 (&a)[TM], const bf16x8 (&b)[TN]) {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  };
  auto next = [](int st) { return st == (kQStages - 1) * kQStage ? 0 : st + kQStage; };

  // tile t (register set S, LDS stage st): three quarters of its products;
  // then, if a tile follows, wait for it, refill this stage with tile t + 3
  // and read tile t + 1's fragments; then the last quarter
  auto step = [&](auto set, int t, int st) {
    constexpr int S = decltype(set)::value;
    mm(fa[S][0], fb[S][0]);
    mm(fa[S][1], fb[S][1]);
    mm(fa[S][0], fl[S][0]);
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
    mm(fa[S][1], fl[S][1]);
  };

  issue(0, 0);
  if (KT > 1) issue(1, kQStage);
  if (KT > 2) issue(2, 2 * kQStage);
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
  // cc = L % 16) holds rows wm0 + 16 i + cr + v, columns wn0 + 16 j + cc.
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

constexpr int kQWGM = 2, kQWGN = 4; // waves of a workgroup

inline bool al16(const void *p) { return ((uintptr_t)p & 15) == 0; }

} // namespace

bool gemm_ntb_ok(const GemmNTB &g) {
  if (g.nseg < 1 || g.nseg > kMaxSeg || !g.B || !g.B_lo || !g.C || g.Ncols <= 0) return false;
  if (g.ldb % 8 || !al16(g.B) || !al16(g.B_lo) || (g.perm && (!g.brow || g.nb < 1))) return false;
  if (g.perm && g.bstride % 8) return false;
  for (int q = 0; q < g.nseg; ++q) {
    const SegB &s = g.seg[q];
    if (!s.ptr || !al16(s.ptr) || s.k <= 0 || s.k % kQBK || s.ld % 8 || s.boff % 8) return false;
  }
  return true;
}

hipError_t launch_gemm_ntb(const Dims *dims, int capM, const GemmNTB &g, hipStream_t s, int tag,
                           hipEvent_t ev0, hipEvent_t ev1) {
  if (capM <= 0) return hipSuccess;
  if (!gemm_ntb_ok(g)) return hipErrorInvalidValue;
  const int nt = cdiv(g.Ncols, kQBN);
  // bucketed rows: each bucket's last tile may be partial
  const dim3 grid((cdiv(capM, kQBM) + (g.perm ? g.nb : 0)) * nt);
  switch (tag) {
#define HGNN_NTB(T)                                                                              \
  hipExtLaunchKernelGGL(k_gemm_ntb<T, kQWGM, kQWGN>, grid, dim3(64 * kQWGM * kQWGN), 0, s, ev0,   \
                        ev1, 0, dims, g, nt);                                                    \
  break
  case 1: HGNN_NTB(1);
  case 2: HGNN_NTB(2);
  case 4: HGNN_NTB(4);
  default: HGNN_NTB(0);
#undef HGNN_NTB
  }
  return hipGetLastError();
}

} // namespace hgnn
