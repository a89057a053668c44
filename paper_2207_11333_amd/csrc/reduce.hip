// Ordered split-K reductions of the MFMA GEMMs (gemm_nt.hip, gemm_tn.hip):
// the partial sums P[z] are added in the fixed order z = 0, 1, ... so the
// result does not depend on scheduling.  One thread owns four consecutive
// outputs (every Ncols here is a multiple of 4) and issues the 16-byte loads
// of up to kBatch splits before adding them, so they are in flight together.
#include "common.hpp"

namespace hgnn {

namespace {

inline int cdiv(long long a, int b) { return (int)((a + b - 1) / b); }

constexpr int kBatch = 4;

__device__ __forceinline__ f4 ordered_sum(const float *__restrict__ src, int splits,
                                          long long stride) {
  f4 sum = *reinterpret_cast<const f4 *>(src);
  for (int z0 = 1; z0 < splits; z0 += kBatch) {
    f4 v[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int z = min(z0 + u, splits - 1);
      v[u] = *reinterpret_cast<const f4 *>(src + z * stride);
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
      if (z0 + u < splits) sum += v[u];
  }
  return sum;
}

// NT: C = act(sum_z P[z] + bias) (* mask).
__global__ void __launch_bounds__(256)
k_reduce_nt(const Dims *__restrict__ dims, const GemmNT g) {
  const int M = g.M_fixed >= 0 ? g.M_fixed : dims->N;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = (long long)M * g.Ncols;
  if (4 * t >= total) return;
  f4 sum = ordered_sum(g.P + 4 * t, g.splits, total);
  const int m = (int)(4 * t / g.Ncols), n = (int)(4 * t % g.Ncols);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    float o = sum[e] + (g.bias ? g.bias[n + e] : 0.f);
    if (g.relu) o = o > 0.f ? o : 0.f;
    if (g.mask && !(g.mask[(size_t)m * g.ldc + n + e] > 0.f)) o = 0.f;
    sum[e] = o;
  }
  *reinterpret_cast<f4 *>(g.C + (size_t)m * g.ldc + n) = sum;
}

// TN: sum, then scatter into the packed gradient layout (routes: see ReduceMap).
__global__ void __launch_bounds__(256) k_reduce_map(const ReduceMap r) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = (long long)r.M * r.Ncols;
  if (4 * t >= total) return;
  const f4 sum = ordered_sum(r.P + 4 * t, r.splits, total);
  const int m = (int)(4 * t / r.Ncols), c0 = (int)(4 * t % r.Ncols);
  for (int k = 0; k < r.nroute; ++k) {
    const ReduceRoute &ro = r.route[k];
    if (m < ro.r0 || m >= ro.r1) continue;
    const int u = m - ro.r0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int c = c0 + e;
      if (c < r.main_cols) {
        if (!ro.main || (c >= r.F && c < r.Fp)) continue;
        const int oc = c < r.F ? c : c - (r.Fp - r.F);
        ro.main[(size_t)u * ro.main_ld + ro.main_coloff + oc] = sum[e];
      } else if (c == r.main_cols && ro.ones) {
        ro.ones[(size_t)(u % ro.ones_split) * ro.ones_stride + u / ro.ones_split] = sum[e];
      }
    }
    return;
  }
}

} // namespace

hipError_t launch_reduce_nt(const Dims *dims, int capM, const GemmNT &g, hipStream_t s) {
  const long long total = (long long)capM * g.Ncols;
  if (total <= 0) return hipSuccess;
  k_reduce_nt<<<cdiv(total / 4, 256), 256, 0, s>>>(dims, g);
  return hipGetLastError();
}

hipError_t launch_reduce_map(const ReduceMap &r, hipStream_t s) {
  const long long total = (long long)r.M * r.Ncols;
  if (total <= 0) return hipSuccess;
  k_reduce_map<<<cdiv(total / 4, 256), 256, 0, s>>>(r);
  return hipGetLastError();
}

} // namespace hgnn
