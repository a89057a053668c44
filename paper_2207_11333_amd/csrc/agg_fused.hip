// Step S6's aggregate-input gradient fused into step S7's aggregation
// adjoint, for degree-bucketed models.
//
// dA = du W_eff(d) (one [4H, H] weight per in-degree bucket) is needed only
// by the adjoint of the same node, four values per feature (the gradients of
// its mean, min, max and std aggregates).  A workgroup takes 64 rows of one
// bucket (the (degree, id) order) and 32 features c0 .. c0 + 31: it forms the
// 64 x 128 block of dA with those features' four aggregator columns on the
// matrix cores, keeps it in LDS, and runs the adjoint of its 64 nodes for
// those features from there.  dA never reaches HBM (at 40k nodes and H = 256
// that is 166 MB written and read again per layer), and the two launches
// become one.
//
// The product is the NT GEMM's (gemm_nt.hip): the same 64 x 128 tile, 8
// waves in a 2 x 4 grid, 64-deep K steps, the same staging and the same
// MFMA order over K, so dA is bitwise the NT GEMM's.  Tile column
// j * 32 + f is dA column j H + c0 + f (wave column j holds aggregator j).
// The adjoint is node_adjoint's (agg_msg.hpp), as in k_aggregate_bwd, with
// its loads split off: the node id is fetched with the product's first
// operand tiles, and after the product the CSR bounds, source ids and the
// rows they gather are loaded before the dA block goes through LDS, so they
// are in flight meanwhile.  The CSR bounds and source ids are not fetched
// earlier: held over the K loop they raise the register count past what two
// workgroups per CU allow, which costs more than they save.
#include "mfma_tile.hpp"
#include "agg_msg.hpp"

namespace hgnn {

namespace {

constexpr int kFusedFC = 32; // features per workgroup
constexpr int kFusedBM = 64; // rows per workgroup

template <int PREC, int FE, bool SPLIT>
__global__ void __launch_bounds__(512, 2)
k_agg_bwd_fused(const AggBwdFused a) {
  using P = Prec<PREC>;
  using T = typename P::T;
  constexpr int BM = kFusedBM, BN = 4 * kFusedFC, WGN = 4, NTH = 128 * WGN;
  constexpr int BK = P::BK, LDA = BK + P::PAD;
  constexpr int WM = BM / 2, WN = BN / WGN, TM = WM / 16, TN = WN / 16;
  constexpr int NA = BM * BK / 4 / NTH;
  constexpr int BVEC = (PREC == 0) ? 4 : 8;
  constexpr int NB = BN * BK / BVEC / NTH;
  static_assert(NA >= 1 && NB >= 1 && WN == kFusedFC, "tile shape");
  // LDS: the operand tiles of the product, then (reusing them) the dA block
  constexpr int LDD = BN + 4; // floats per row of the dA block
  constexpr int kBytesAB = (BM + BN * (SPLIT ? 2 : 1)) * LDA * (int)sizeof(T);
  constexpr int kBytesD = BM * LDD * 4;
  __shared__ __attribute__((aligned(16))) char smem[kBytesAB > kBytesD ? kBytesAB : kBytesD];
  T *As = reinterpret_cast<T *>(smem);
  T *Bs = As + BM * LDA;
  T *Bl = Bs + BN * LDA;
  float *sD = reinterpret_cast<float *>(smem);

  const int H = a.H, K = a.H;
  const int nch = H / kFusedFC;
  const BucketWalk bw(a.brow, a.nb, BM);
  const int mtiles = bw.total();
  if ((int)blockIdx.x >= mtiles * nch) return;
  // the feature chunks of one row tile are adjacent, so they share an XCD
  const int tile = xcd_tile(blockIdx.x, mtiles * nch);
  const int mt = tile / nch, c0 = (tile % nch) * kFusedFC;
  int bq, m0, m_hi;
  bw.find(mt, bq, m0, m_hi);
  const int tid = threadIdx.x, wid = tid >> 6;
  const int wm0 = (wid / WGN) * WM, wn0 = (wid % WGN) * WN;
  // this thread's node in the adjoint (rows past the bucket's end repeat its
  // last node and write nothing), fetched beside the product's operands
  const int r = tid >> 3, q4 = 4 * (tid & 7);
  const int node = a.perm[min(m0 + r, m_hi - 1)];

  f4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  const T *Bg = reinterpret_cast<const T *>(a.B) + (size_t)bq * a.bstride;
  const T *Blg = SPLIT ? reinterpret_cast<const T *>(a.B_lo) + (size_t)bq * a.bstride : nullptr;
  // per-thread rows and columns, fixed over K (rows from clamped indices)
  int a_row[NA], a_col[NA];
  bool a_ok[NA];
#pragma unroll
  for (int j = 0; j < NA; ++j) {
    const int v = tid + j * NTH;
    const int m = m0 + v / (BK / 4);
    a_ok[j] = m < m_hi;
    a_row[j] = a.perm[min(m, m_hi - 1)];
    a_col[j] = (v % (BK / 4)) * 4;
  }
  int b_row[NB], b_col[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int v = tid + j * NTH;
    const int tc = v / (BK / BVEC); // tile column: aggregator tc / 32, feature tc % 32
    b_row[j] = (tc / kFusedFC) * H + c0 + tc % kFusedFC;
    b_col[j] = (v % (BK / BVEC)) * BVEC;
  }
  const int KT = (K + BK - 1) / BK;
  // two register stages keeping raw loads; masks applied when stashed (the
  // NT GEMM's scheme: loads stay in flight over the step's products)
  f4 ra[2][NA], rb[2][NB], rl[2][SPLIT ? NB : 1];
  unsigned am[2], bmk[2];
  auto dload = [&](auto st, int t) {
    constexpr int S = decltype(st)::value;
    const int k0 = min(t, KT - 1) * BK;
    unsigned mk = 0;
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int k = k0 + a_col[j];
      ra[S][j] = *reinterpret_cast<const f4 *>(a.du + (size_t)a_row[j] * H + min(k, K - 4));
      mk |= (a_ok[j] && k < K) ? 1u << j : 0u;
    }
    am[S] = mk;
    mk = 0;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int k = k0 + b_col[j];
      const size_t off = (size_t)b_row[j] * K + min(k, K - BVEC);
      rb[S][j] = *reinterpret_cast<const f4 *>(Bg + off);
      if constexpr (SPLIT) rl[S][j] = *reinterpret_cast<const f4 *>(Blg + off);
      mk |= (k < K) ? 1u << j : 0u;
    }
    bmk[S] = mk;
  };
  auto stash = [&](auto st) {
    constexpr int S = decltype(st)::value;
    const f4 zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int v = tid + j * NTH;
      const int r = v / (BK / 4), c = (v % (BK / 4)) * 4;
      store4(As + r * LDA + c, (am[S] >> j & 1u) ? ra[S][j] : zero);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int v = tid + j * NTH;
      const int r = v / (BK / BVEC), c = (v % (BK / BVEC)) * BVEC;
      const bool ok = bmk[S] >> j & 1u;
      *reinterpret_cast<f4 *>(Bs + r * LDA + c) = ok ? rb[S][j] : zero; // 16 raw bytes
      if constexpr (SPLIT) *reinterpret_cast<f4 *>(Bl + r * LDA + c) = ok ? rl[S][j] : zero;
    }
  };
  auto step = [&](auto st, int t) {
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
    stash(st);
    __syncthreads();
    if (t + 2 < KT) dload(st, t + 2);
    mma_tile<PREC, TM, TN, LDA, BK>(As, Bs, wm0, wn0, acc);
    if constexpr (SPLIT) mma_tile<PREC, TM, TN, LDA, BK>(As, Bl, wm0, wn0, acc);
  };
  dload(IC<0>{}, 0);
  if (KT > 1) dload(IC<1>{}, 1);
  __builtin_amdgcn_s_waitcnt(0x0f70); // vmcnt(0): see the TN GEMMs
  int t = 0;
  for (; t + 1 < KT; t += 2) {
    step(IC<0>{}, t);
    step(IC<1>{}, t + 1);
  }
  if (t < KT) step(IC<0>{}, t);
  // the adjoint's operands that do not depend on dA are in flight while the
  // block goes through LDS
  const int lo = a.rowptr[node], deg = a.rowptr[node + 1] - lo;
  int src[kCache];
  if (deg > 0) fetch_sources(a.csr_src, lo, deg, src);
  AdjIn in;
  adj_load<FE>(in, node, lo, deg, src, c0 + q4, H, a.PQ, a.csr_e, a.WeT, a.bm, a.A, a.args);

  // the dA block into LDS, over the operand tiles once every wave is done
  __syncthreads();
  {
    const int lane = tid & 63;
    const int cr = 4 * (lane >> 4), cc = lane & 15;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          sD[(wm0 + i * 16 + cr + v) * LDD + wn0 + j * 16 + cc] = acc[i][j][v];
  }
  __syncthreads();

  // adjoint: thread (row r, features c0 + 4 q .. + 3)
  if (m0 + r >= m_hi) return;
  const float *d = sD + r * LDD + q4;
  adj_finish<FE>(in, node, c0 + q4, H, a.PQ, a.csr_src, a.csr_e,
                 *reinterpret_cast<const f4 *>(d), *reinterpret_cast<const f4 *>(d + kFusedFC),
                 *reinterpret_cast<const f4 *>(d + 2 * kFusedFC),
                 *reinterpret_cast<const f4 *>(d + 3 * kFusedFC), a.dm, a.D, a.ldD);
}

template <int PREC, bool SPLIT>
void run_fused(int grid, const AggBwdFused &a, int Fe, hipStream_t s, hipEvent_t ev0,
               hipEvent_t ev1) {
#define HGNN_FUSED(FE)                                                                      \
  hipExtLaunchKernelGGL(k_agg_bwd_fused<PREC, FE, SPLIT>, dim3(grid), dim3(512), 0, s, ev0, \
                        ev1, 0, a)
  switch (Fe) {
  case 0: HGNN_FUSED(0); break;
  case 1: HGNN_FUSED(1); break;
  case 2: HGNN_FUSED(2); break;
  case 3: HGNN_FUSED(3); break;
  default: HGNN_FUSED(4); break;
  }
#undef HGNN_FUSED
}

} // namespace

bool agg_bwd_fused_ok(int H, int nb) { return nb > 0 && H % kFusedFC == 0; }

hipError_t launch_agg_bwd_fused(int capN, const AggBwdFused &a, int precision, int Fe,
                                hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if (capN <= 0) return hipSuccess;
  if (!agg_bwd_fused_ok(a.H, a.nb) || Fe > 4 || (precision == 1) != (a.B_lo != nullptr))
    return hipErrorInvalidValue;
  // every bucket's last row tile may be partial
  const int grid = (cdiv(capN, kFusedBM) + a.nb) * (a.H / kFusedFC);
  if (precision == 1) run_fused<1, true>(grid, a, Fe, s, ev0, ev1);
  else run_fused<0, false>(grid, a, Fe, s, ev0, ev1);
  return hipGetLastError();
}

} // namespace hgnn
