// Ordered split-K reductions of the MFMA GEMMs (gemm_nt.hip, gemm_tn.hip):
// the partial sums P[z] are added in a fixed order, so the result does not
// depend on scheduling.  Each output float4 (every Ncols here is a multiple
// of 4) is owned by a group of G adjacent lanes: lane g adds the contiguous
// splits [g per, (g + 1) per) in order, issuing all of its 16-byte loads
// before adding them, and the G lane sums are combined by a fixed pairwise
// tree of wave shuffles.  G grows with the split count so that no lane waits
// on more than kPerLane loads.
#include "common.hpp"

namespace hgnn {

namespace {

inline int cdiv(long long a, int b) { return (int)((a + b - 1) / b); }

constexpr int kPerLane = 4;

template <int G>
__device__ __forceinline__ f4 ordered_sum(const float *__restrict__ src, int splits,
                                          long long stride, int g) {
  const int per = (splits + G - 1) / G;
  const int z_lo = g * per, z_hi = min(splits, z_lo + per);
  f4 sum = f4{0.f, 0.f, 0.f, 0.f};
  for (int z0 = z_lo; z0 < z_hi; z0 += kPerLane) {
    f4 v[kPerLane];
#pragma unroll
    for (int u = 0; u < kPerLane; ++u) {
      const int z = min(z0 + u, splits - 1);
      v[u] = *reinterpret_cast<const f4 *>(src + z * stride);
    }
#pragma unroll
    for (int u = 0; u < kPerLane; ++u)
      if (z0 + u < z_hi) sum += v[u];
  }
#pragma unroll
  for (int off = 1; off < G; off <<= 1) {
#pragma unroll
    for (int e = 0; e < 4; ++e) sum[e] += __shfl_down(sum[e], off, G);
  }
  return sum;
}

int pick_group(int splits) {
  int G = 1;
  while (G < 16 && G * kPerLane < splits) G <<= 1;
  return G;
}

// NT: C = act(sum_z P[z] + bias) (* mask).
template <int G>
__global__ void __launch_bounds__(256)
k_reduce_nt(const Dims *__restrict__ dims, const GemmNT g) {
  const int M = g.M_fixed >= 0 ? g.M_fixed : dims->N;
  const long long gt = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long t = gt / G;
  const long long total = (long long)M * g.Ncols;
  // lanes past the end still take part in their group's shuffles
  const bool live = 4 * t < total;
  f4 sum = ordered_sum<G>(g.P + (live ? 4 * t : 0), g.splits, total, (int)(gt % G));
  if (!live || gt % G != 0) return;
  const int m = (int)(4 * t / g.Ncols), n = (int)(4 * t % g.Ncols);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    float o = sum[e] + (g.bias ? g.bias[n + e] : 0.f);
    if (g.addend) o += g.addend[(size_t)m * g.ld_add + n + e];
    if (g.relu) o = o > 0.f ? o : 0.f;
    if (g.mask && !(g.mask[(size_t)m * g.ldc + n + e] > 0.f)) o = 0.f;
    sum[e] = o;
  }
  *reinterpret_cast<f4 *>(g.C + (size_t)m * g.ldc + n) = sum;
}

// TN: sum, then scatter into the packed gradient layout (routes: see ReduceMap).
template <int G>
__global__ void __launch_bounds__(256) k_reduce_map(const ReduceMap r) {
  const long long gt = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long t = gt / G;
  const long long total = (long long)r.M * r.Ncols;
  const bool live = 4 * t < total;
  const f4 sum = ordered_sum<G>(r.P + (live ? 4 * t : 0), r.splits, total, (int)(gt % G));
  if (!live || gt % G != 0) return;
  const int m = (int)(4 * t / r.Ncols), c0 = (int)(4 * t % r.Ncols);
  for (int k = 0; k < r.nroute; ++k) {
    const ReduceRoute &ro = r.route[k];
    if (m < ro.r0 || m >= ro.r1) continue;
    const int u = m - ro.r0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int c = c0 + e;
      if (c < r.main_cols) {
        if (!ro.main) continue;
        const int nb = r.npad > 1 ? r.npad : 1;
        int oc;
        if (c < nb * r.Fp) {
          const int blk = c / r.Fp, w = c - blk * r.Fp;
          if (w >= r.F) continue;
          oc = blk * r.F + w;
        } else {
          oc = c - nb * (r.Fp - r.F);
        }
        ro.main[(size_t)u * ro.main_ld + ro.main_coloff + oc] = sum[e];
      } else if (c == r.main_cols && ro.ones) {
        ro.ones[(size_t)(u % ro.ones_split) * ro.ones_stride + u / ro.ones_split] = sum[e];
      }
    }
    return;
  }
}

// Bucketed update weight gradient: the chunks of one bucket share its
// scalers, so sum_z P[z] gives the h block, W_0 and the bias, and the
// s+ and s- weighted sums give W_+ and W_-.  Same lane grouping and order
// as ordered_sum.
template <int G>
__global__ void __launch_bounds__(256) k_reduce_upd(const ReduceUpd r) {
  const long long gt = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long t = gt / G;
  const long long total = (long long)r.M * r.Ncols;
  const bool live = 4 * t < total;
  const float *src = r.P + (live ? 4 * t : 0);
  const int g = (int)(gt % G);
  const int per = (r.Z + G - 1) / G;
  const int z_lo = g * per, z_hi = min(r.Z, z_lo + per);
  f4 s0 = f4{0.f, 0.f, 0.f, 0.f}, s1 = s0, s2 = s0;
  for (int z0 = z_lo; z0 < z_hi; z0 += kPerLane) {
    f4 v[kPerLane];
    float a[kPerLane], b[kPerLane];
#pragma unroll
    for (int u = 0; u < kPerLane; ++u) {
      const int z = min(z0 + u, r.Z - 1);
      v[u] = *reinterpret_cast<const f4 *>(src + z * total);
      a[u] = r.zscale[2 * z];
      b[u] = r.zscale[2 * z + 1];
    }
#pragma unroll
    for (int u = 0; u < kPerLane; ++u)
      if (z0 + u < z_hi) {
        s0 += v[u];
        s1 += a[u] * v[u];
        s2 += b[u] * v[u];
      }
  }
#pragma unroll
  for (int off = 1; off < G; off <<= 1) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      s0[e] += __shfl_down(s0[e], off, G);
      s1[e] += __shfl_down(s1[e], off, G);
      s2[e] += __shfl_down(s2[e], off, G);
    }
  }
  if (!live || g != 0) return;
  const int m = (int)(4 * t / r.Ncols), c0 = (int)(4 * t % r.Ncols);
  const int H = r.H, ldp = r.F + 12 * H;
  float *row = r.dWp + (size_t)m * ldp;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int c = c0 + e;
    if (c < r.Fp) {
      if (c < r.F) row[c] = s0[e];
    } else if (c < r.Fp + 4 * H) {
      const int cc = c - r.Fp;
      row[r.F + cc] = s0[e];
      row[r.F + 4 * H + cc] = s1[e];
      row[r.F + 8 * H + cc] = s2[e];
    } else if (c == r.Fp + 4 * H) {
      r.dbp[m] = s0[e];
    }
  }
}

// Column sums of X [N rows, C columns] over fixed row chunks: chunk z of
// Z covers rows [z R, (z + 1) R), R = ceil(N / Z), and is one workgroup.
// Its threads split into RP row lanes of one 16-byte column group each: lane
// rl adds rows lo + rl, lo + rl + RP, ... in order, and the lanes' sums are
// added in lane order through LDS (a fixed order, so the result does not
// depend on timing).  The partials are written as P[z][c][0..3] =
// {sum, 0, 0, 0}: the layout of a weight-gradient GEMM's sum column, so that
// launch_reduce_map adds them.
constexpr int kColsumThreads = 1024;

__global__ void __launch_bounds__(kColsumThreads)
k_colsum(const Dims *__restrict__ dims, const float *__restrict__ X, int ldx, int C, int Z,
         float *__restrict__ P) {
  __shared__ f4 part[kColsumThreads];
  // thread (row lane rl, 16-byte column group cg): the workgroup reads RP
  // rows of up to 256 column groups at a time, four such passes in flight
  const int CG = C >> 2, g0 = blockIdx.y * 256;
  const int cgb = min(CG - g0, 256), RP = kColsumThreads / cgb;
  const int t = threadIdx.x, rl = t / cgb, cg = g0 + t % cgb;
  const int N = dims->N, z = blockIdx.x;
  const int R = (N + Z - 1) / Z;
  const int lo = min(z * R, N), hi = min(lo + R, N);
  f4 sum = {0.f, 0.f, 0.f, 0.f};
  if (rl < RP) {
    const float *base = X + 4 * cg;
    int i = lo + rl;
    for (; i + 3 * RP < hi; i += 4 * RP) {
      f4 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = *reinterpret_cast<const f4 *>(base + (size_t)(i + u * RP) * ldx);
#pragma unroll
      for (int u = 0; u < 4; ++u) sum += v[u];
    }
    for (; i < hi; i += RP) sum += *reinterpret_cast<const f4 *>(base + (size_t)i * ldx);
  }
  part[t] = sum;
  __syncthreads();
  if (rl != 0) return;
  // the row lanes' sums in lane order
  for (int k = 1; k < RP; ++k) sum += part[t + k * cgb];
#pragma unroll
  for (int e = 0; e < 4; ++e)
    *reinterpret_cast<f4 *>(P + ((size_t)z * C + 4 * cg + e) * 4) = f4{sum[e], 0.f, 0.f, 0.f};
}

// Several reductions in one launch (the weight gradients of one layer): job
// j takes grid[j] workgroups; each job's lane groups are G[j] lanes wide (a
// runtime width: the shuffle tree reads lanes up to G - 1 above, and only a
// group's first lane, which sums its own group, writes).  The bodies are
// k_reduce_upd's and k_reduce_map's, so each output is the same sum in the
// same order as in those kernels.
__device__ __forceinline__ float tree_sum(float v, int G) {
  for (int off = 1; off < G; off <<= 1) v += __shfl_down(v, off, 64);
  return v;
}

__device__ __forceinline__ void job_upd(const ReduceUpd &r, long long gt, int G) {
  const long long t = gt / G;
  const long long total = (long long)r.M * r.Ncols;
  const bool live = 4 * t < total;
  const float *src = r.P + (live ? 4 * t : 0);
  const int g = (int)(gt % G);
  const int per = (r.Z + G - 1) / G;
  const int z_lo = g * per, z_hi = min(r.Z, z_lo + per);
  f4 s0 = f4{0.f, 0.f, 0.f, 0.f}, s1 = s0, s2 = s0;
  for (int z0 = z_lo; z0 < z_hi; z0 += kPerLane) {
    f4 v[kPerLane];
    float a[kPerLane], b[kPerLane];
#pragma unroll
    for (int u = 0; u < kPerLane; ++u) {
      const int z = min(z0 + u, r.Z - 1);
      v[u] = *reinterpret_cast<const f4 *>(src + z * total);
      a[u] = r.zscale[2 * z];
      b[u] = r.zscale[2 * z + 1];
    }
#pragma unroll
    for (int u = 0; u < kPerLane; ++u)
      if (z0 + u < z_hi) {
        s0 += v[u];
        s1 += a[u] * v[u];
        s2 += b[u] * v[u];
      }
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    s0[e] = tree_sum(s0[e], G);
    s1[e] = tree_sum(s1[e], G);
    s2[e] = tree_sum(s2[e], G);
  }
  if (!live || g != 0) return;
  const int m = (int)(4 * t / r.Ncols), c0 = (int)(4 * t % r.Ncols);
  const int H = r.H, ldp = r.F + 12 * H;
  float *row = r.dWp + (size_t)m * ldp;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int c = c0 + e;
    if (c < r.Fp) {
      if (c < r.F) row[c] = s0[e];
    } else if (c < r.Fp + 4 * H) {
      const int cc = c - r.Fp;
      row[r.F + cc] = s0[e];
      row[r.F + 4 * H + cc] = s1[e];
      row[r.F + 8 * H + cc] = s2[e];
    } else if (c == r.Fp + 4 * H) {
      r.dbp[m] = s0[e];
    }
  }
}

__device__ __forceinline__ void job_map(const ReduceMap &r, long long gt, int G) {
  const long long t = gt / G;
  const long long total = (long long)r.M * r.Ncols;
  const bool live = 4 * t < total;
  const float *src = r.P + (live ? 4 * t : 0);
  const int g = (int)(gt % G);
  const int per = (r.splits + G - 1) / G;
  const int z_lo = g * per, z_hi = min(r.splits, z_lo + per);
  f4 sum = f4{0.f, 0.f, 0.f, 0.f};
  for (int z0 = z_lo; z0 < z_hi; z0 += kPerLane) {
    f4 v[kPerLane];
#pragma unroll
    for (int u = 0; u < kPerLane; ++u) {
      const int z = min(z0 + u, r.splits - 1);
      v[u] = *reinterpret_cast<const f4 *>(src + z * total);
    }
#pragma unroll
    for (int u = 0; u < kPerLane; ++u)
      if (z0 + u < z_hi) sum += v[u];
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) sum[e] = tree_sum(sum[e], G);
  if (!live || g != 0) return;
  const int m = (int)(4 * t / r.Ncols), c0 = (int)(4 * t % r.Ncols);
  for (int k = 0; k < r.nroute; ++k) {
    const ReduceRoute &ro = r.route[k];
    if (m < ro.r0 || m >= ro.r1) continue;
    const int u = m - ro.r0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int c = c0 + e;
      if (c < r.main_cols) {
        if (!ro.main) continue;
        const int nb = r.npad > 1 ? r.npad : 1;
        int oc;
        if (c < nb * r.Fp) {
          const int blk = c / r.Fp, w = c - blk * r.Fp;
          if (w >= r.F) continue;
          oc = blk * r.F + w;
        } else {
          oc = c - nb * (r.Fp - r.F);
        }
        ro.main[(size_t)u * ro.main_ld + ro.main_coloff + oc] = sum[e];
      } else if (c == r.main_cols && ro.ones) {
        ro.ones[(size_t)(u % ro.ones_split) * ro.ones_stride + u / ro.ones_split] = sum[e];
      }
    }
    return;
  }
}

__global__ void __launch_bounds__(256) k_reduce_jobs(const ReduceJobs j) {
  int b = blockIdx.x, k = 0;
  while (k + 1 < j.njobs && b >= j.grid[k]) b -= j.grid[k++];
  const long long gt = (long long)b * blockDim.x + threadIdx.x;
  if (j.upd[k]) job_upd(j.u, gt, j.G[k]);
  else job_map(j.m[k], gt, j.G[k]);
}

} // namespace

hipError_t launch_colsum(const Dims *dims, const float *X, int ldx, int C, int Z, float *P,
                         hipStream_t s) {
  if (C <= 0 || Z <= 0) return hipSuccess;
  // whole 16-byte column groups
  if (C % 4 || ldx % 4 || reinterpret_cast<uintptr_t>(X) % 16) return hipErrorInvalidValue;
  k_colsum<<<dim3(Z, cdiv(C / 4, 256)), kColsumThreads, 0, s>>>(dims, X, ldx, C, Z, P);
  return hipGetLastError();
}

hipError_t launch_reduce_upd(const ReduceUpd &r, hipStream_t s) {
  const long long total = (long long)r.M * r.Ncols;
  if (total <= 0) return hipSuccess;
  const int G = pick_group(r.Z);
  const int grid = cdiv(total / 4 * G, 256);
  switch (G) {
  case 1: k_reduce_upd<1><<<grid, 256, 0, s>>>(r); break;
  case 2: k_reduce_upd<2><<<grid, 256, 0, s>>>(r); break;
  case 4: k_reduce_upd<4><<<grid, 256, 0, s>>>(r); break;
  case 8: k_reduce_upd<8><<<grid, 256, 0, s>>>(r); break;
  default: k_reduce_upd<16><<<grid, 256, 0, s>>>(r); break;
  }
  return hipGetLastError();
}

hipError_t launch_reduce_nt(const Dims *dims, int capM, const GemmNT &g, hipStream_t s) {
  const long long total = (long long)capM * g.Ncols;
  if (total <= 0) return hipSuccess;
  const int G = pick_group(g.splits);
  const int grid = cdiv(total / 4 * G, 256);
  switch (G) {
  case 1: k_reduce_nt<1><<<grid, 256, 0, s>>>(dims, g); break;
  case 2: k_reduce_nt<2><<<grid, 256, 0, s>>>(dims, g); break;
  case 4: k_reduce_nt<4><<<grid, 256, 0, s>>>(dims, g); break;
  case 8: k_reduce_nt<8><<<grid, 256, 0, s>>>(dims, g); break;
  default: k_reduce_nt<16><<<grid, 256, 0, s>>>(dims, g); break;
  }
  return hipGetLastError();
}

hipError_t launch_reduce_map(const ReduceMap &r, hipStream_t s) {
  const long long total = (long long)r.M * r.Ncols;
  if (total <= 0) return hipSuccess;
  const int G = pick_group(r.splits);
  const int grid = cdiv(total / 4 * G, 256);
  switch (G) {
  case 1: k_reduce_map<1><<<grid, 256, 0, s>>>(r); break;
  case 2: k_reduce_map<2><<<grid, 256, 0, s>>>(r); break;
  case 4: k_reduce_map<4><<<grid, 256, 0, s>>>(r); break;
  case 8: k_reduce_map<8><<<grid, 256, 0, s>>>(r); break;
  default: k_reduce_map<16><<<grid, 256, 0, s>>>(r); break;
  }
  return hipGetLastError();
}

hipError_t launch_reduce_jobs(ReduceJobs j, hipStream_t s) {
  int total = 0;
  for (int k = 0; k < j.njobs; ++k) {
    const long long n = j.upd[k] ? (long long)j.u.M * j.u.Ncols : (long long)j.m[k].M * j.m[k].Ncols;
    j.G[k] = pick_group(j.upd[k] ? j.u.Z : j.m[k].splits);
    j.grid[k] = n > 0 ? cdiv(n / 4 * j.G[k], 256) : 0;
    total += j.grid[k];
  }
  if (total <= 0) return hipSuccess;
  k_reduce_jobs<<<total, 256, 0, s>>>(j);
  return hipGetLastError();
}

} // namespace hgnn
