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

namespace hgnn {

namespace {

template <int PREC> struct Prec;
template <> struct Prec<0> {
  using T = float;
  static constexpr int BK = 32;   // k per LDS tile
  static constexpr int PAD = 4;   // elements of row padding (16 bytes)
};
template <> struct Prec<1> {
  using T = __bf16;
  static constexpr int BK = 64;
  static constexpr int PAD = 8;
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

// Multiply-accumulate one BK-deep LDS tile into the wave's accumulators.
template <int PREC, int TM, int TN, int LDA>
__device__ __forceinline__ void mma_tile(const typename Prec<PREC>::T *As,
                                         const typename Prec<PREC>::T *Bs,
                                         int wm0, int wn0, f4 (&acc)[TM][TN]) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  if constexpr (PREC == 0) {
#pragma unroll
    for (int kc = 0; kc < Prec<0>::BK; kc += 16) {
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
    for (int kc = 0; kc < Prec<1>::BK; kc += 32) {
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
template <int PREC, int BM, int BN, bool SPLIT>
__global__ void __launch_bounds__(256)
k_gemm_nt(const Dims *__restrict__ dims, const GemmNT g) {
  using P = Prec<PREC>;
  using T = typename P::T;
  constexpr int BK = P::BK, LDA = BK + P::PAD;
  constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 16, TN = WN / 16;
  // A tile: BM x BK floats loaded as float4 -> NA vectors per thread
  constexpr int NA = BM * BK / 4 / 256;
  // B tile: BN x BK elements loaded 16 bytes at a time
  constexpr int BVEC = (PREC == 0) ? 4 : 8;
  constexpr int NB = BN * BK / BVEC / 256;
  static_assert(NA >= 1 && NB >= 1, "tile too small for 256 threads");
  __shared__ __attribute__((aligned(16))) T As[BM * LDA];
  __shared__ __attribute__((aligned(16))) T Bs[BN * LDA];
  __shared__ __attribute__((aligned(16))) T Bl[SPLIT ? BN * LDA : 1];

  const int M = g.M_fixed >= 0 ? g.M_fixed : dims->N;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  if (m0 >= M) return;
  const int tid = threadIdx.x, wid = tid >> 6;
  const int wm0 = (wid >> 1) * WM, wn0 = (wid & 1) * WN;

  f4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  const T *Bg = reinterpret_cast<const T *>(g.B);
  const T *Blg = reinterpret_cast<const T *>(g.B_lo);
  f4 ra[NA];
  f4 rb[NB]; // raw 16-byte B vectors (FP32 or BF16) kept as f4 bit patterns
  f4 rl[SPLIT ? NB : 1];

  auto load = [&](int sidx, int k0) {
    const SegA &sg = g.seg[sidx];
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int v = tid + j * 256;
      const int r = v / (BK / 4), c = (v % (BK / 4)) * 4;
      const int m = m0 + r, k = k0 + c;
      f4 val = f4{0.f, 0.f, 0.f, 0.f};
      if (m < M && k < sg.k) {
        val = *reinterpret_cast<const f4 *>(sg.ptr + (size_t)m * sg.ld + k);
        if (sg.scale) {
          const float s = sg.scale[m];
          val *= s;
        }
      }
      ra[j] = val;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int v = tid + j * 256;
      const int r = v / (BK / BVEC), c = (v % (BK / BVEC)) * BVEC;
      const int n = n0 + r, k = k0 + c;
      f4 val = f4{0.f, 0.f, 0.f, 0.f}, vlo = val;
      if (n < g.Ncols && k < sg.k) {
        val = *reinterpret_cast<const f4 *>(Bg + (size_t)n * g.ldb + sg.boff + k);
        if constexpr (SPLIT)
          vlo = *reinterpret_cast<const f4 *>(Blg + (size_t)n * g.ldb + sg.boff + k);
      }
      rb[j] = val;
      if constexpr (SPLIT) rl[j] = vlo;
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int v = tid + j * 256;
      const int r = v / (BK / 4), c = (v % (BK / 4)) * 4;
      store4(As + r * LDA + c, ra[j]);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int v = tid + j * 256;
      const int r = v / (BK / BVEC), c = (v % (BK / BVEC)) * BVEC;
      *reinterpret_cast<f4 *>(Bs + r * LDA + c) = rb[j]; // 16 raw bytes
      if constexpr (SPLIT) *reinterpret_cast<f4 *>(Bl + r * LDA + c) = rl[j];
    }
  };

  int sidx = 0, k0 = 0;
  // skip empty segments
  while (sidx < g.nseg && g.seg[sidx].k <= 0) ++sidx;
  if (sidx < g.nseg) {
    load(sidx, k0);
    while (true) {
      __syncthreads();
      stash();
      __syncthreads();
      // advance to the next tile and prefetch it while this one computes
      int ns = sidx, nk = k0 + BK;
      if (nk >= g.seg[ns].k) {
        ++ns;
        nk = 0;
        while (ns < g.nseg && g.seg[ns].k <= 0) ++ns;
      }
      const bool more = ns < g.nseg;
      if (more) load(ns, nk);
      mma_tile<PREC, TM, TN, LDA>(As, Bs, wm0, wn0, acc);
      if constexpr (SPLIT) mma_tile<PREC, TM, TN, LDA>(As, Bl, wm0, wn0, acc);
      if (!more) break;
      sidx = ns;
      k0 = nk;
    }
  }

  const int lane = tid & 63;
  const int cr = 4 * (lane >> 4), cc = lane & 15;
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
k_gemm_tn(const Dims *__restrict__ dims, const GemmTN g) {
  using P = Prec<PREC>;
  using T = typename P::T;
  constexpr int BK = P::BK, LDA = BK + P::PAD;
  constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 16, TN = WN / 16;
  constexpr int NA = BM * BK / 4 / 256;
  constexpr int NB = BN * BK / 4 / 256;
  __shared__ __attribute__((aligned(16))) T As[BM * LDA];
  __shared__ __attribute__((aligned(16))) T Bs[BN * LDA];

  const int rows = dims->N;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN, z = blockIdx.z;
  int chunk = (rows + g.splits - 1) / g.splits;
  chunk = (chunk + BK - 1) / BK * BK;
  const int i_lo = z * chunk;
  const int i_hi = min(rows, i_lo + chunk);
  const int tid = threadIdx.x, wid = tid >> 6;
  const int wm0 = (wid >> 1) * WM, wn0 = (wid & 1) * WN;

  f4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  f4 ra[NA], rb[NB];
  auto load = [&](int i0) {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int v = tid + j * 256;
      const int il = v / (BM / 4), mc = (v % (BM / 4)) * 4;
      const int i = i0 + il, m = m0 + mc;
      f4 val = f4{0.f, 0.f, 0.f, 0.f};
      if (i < i_hi && m < g.M) val = *reinterpret_cast<const f4 *>(g.X + (size_t)i * g.ldx + m);
      ra[j] = val;
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int v = tid + j * 256;
      const int il = v / (BN / 4), nc = (v % (BN / 4)) * 4;
      const int i = i0 + il;
      int n = n0 + nc;
      f4 val = f4{0.f, 0.f, 0.f, 0.f};
      if (i < i_hi && n < g.Ncols) {
        int s = 0;
        while (s + 1 < g.nseg && n >= g.seg[s].ncols) { n -= g.seg[s].ncols; ++s; }
        const SegY &sg = g.seg[s];
        val = *reinterpret_cast<const f4 *>(sg.ptr + (size_t)i * sg.ld + n);
        if (sg.scale) val *= sg.scale[i];
      }
      rb[j] = val;
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int v = tid + j * 256;
      const int il = v / (BM / 4), mc = (v % (BM / 4)) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) store1(As + (mc + e) * LDA + il, ra[j][e]);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int v = tid + j * 256;
      const int il = v / (BN / 4), nc = (v % (BN / 4)) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) store1(Bs + (nc + e) * LDA + il, rb[j][e]);
    }
  };

  if (i_lo < i_hi) {
    int i0 = i_lo;
    load(i0);
    while (true) {
      __syncthreads();
      stash();
      __syncthreads();
      const int ni = i0 + BK;
      const bool more = ni < i_hi;
      if (more) load(ni);
      mma_tile<PREC, TM, TN, LDA>(As, Bs, wm0, wn0, acc);
      if (!more) break;
      i0 = ni;
    }
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

// Sum the split-K partials in order z = 0..splits-1 and scatter them into the
// packed gradient layout.
__global__ void k_reduce_map(const ReduceMap r) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = (long long)r.M * r.Ncols;
  if (t >= total) return;
  const int m = (int)(t / r.Ncols), c = (int)(t % r.Ncols);
  int oc;
  if (c < r.F) oc = c;
  else if (c < r.Fp) return;
  else oc = c - (r.Fp - r.F);
  float s = 0.f;
  for (int z = 0; z < r.splits; ++z) s += r.P[(size_t)z * total + t];
  r.out[(size_t)(m % r.rsplit) * r.ldo + (size_t)(m / r.rsplit) * r.rcoloff + oc] = s;
}

inline int cdiv(long long a, int b) { return (int)((a + b - 1) / b); }

template <int PREC, int BM, int BN>
hipError_t run_nt(const Dims *dims, int capM, const GemmNT &g, hipStream_t s) {
  dim3 grid(cdiv(capM, BM), cdiv(g.Ncols, BN));
  if (PREC == 1 && g.B_lo)
    k_gemm_nt<PREC, BM, BN, true><<<grid, 256, 0, s>>>(dims, g);
  else
    k_gemm_nt<PREC, BM, BN, false><<<grid, 256, 0, s>>>(dims, g);
  return hipGetLastError();
}

} // namespace

hipError_t launch_gemm_nt(const Dims *dims, int capM, const GemmNT &g,
                          int precision, hipStream_t s) {
  if (capM <= 0 || g.Ncols <= 0) return hipSuccess;
  // Small node counts leave most of the 256 CUs idle with 64-row tiles.
  const long long tiles64 = (long long)cdiv(capM, 64) * cdiv(g.Ncols, 64);
  const bool small = tiles64 < 512;
  if (precision == 0)
    return small ? run_nt<0, 32, 64>(dims, capM, g, s) : run_nt<0, 64, 64>(dims, capM, g, s);
  return small ? run_nt<1, 32, 64>(dims, capM, g, s) : run_nt<1, 64, 64>(dims, capM, g, s);
}

hipError_t launch_gemm_tn(const Dims *dims, const GemmTN &g, int precision,
                          hipStream_t s) {
  if (g.M <= 0 || g.Ncols <= 0) return hipSuccess;
  dim3 grid(cdiv(g.M, 64), cdiv(g.Ncols, 64), g.splits);
  if (precision == 0)
    k_gemm_tn<0, 64, 64><<<grid, 256, 0, s>>>(dims, g);
  else
    k_gemm_tn<1, 64, 64><<<grid, 256, 0, s>>>(dims, g);
  return hipGetLastError();
}

hipError_t launch_reduce_map(const ReduceMap &r, hipStream_t s) {
  const long long total = (long long)r.M * r.Ncols;
  if (total <= 0) return hipSuccess;
  k_reduce_map<<<cdiv(total, 256), 256, 0, s>>>(r);
  return hipGetLastError();
}

} // namespace hgnn
