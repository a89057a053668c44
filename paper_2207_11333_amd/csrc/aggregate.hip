// Steps S2 and S7: the PNA segmented aggregation over each node's in-edges
// and its adjoint.
//
// Forward: for node i and feature c, over the in-edges k of i (CSR order,
// i.e. by (source, edge id)), the message m_k = P_i + Q_{src(k)} + e_k w_e + b
// (the decomposed message linear: P = h W_dst^T, Q = h W_src^T computed by
// one GEMM) is reduced to mean, min, max and std = sqrt(mean((m - mean)^2)
// + eps) (two passes).  Strict comparisons keep the first extremum in CSR
// order; its segment offset is stored as a byte for the backward pass.
// One thread owns four consecutive features of one node (16-byte loads of
// the gathered Q rows, coalesced across the H/4 threads of the node).
//
// Adjoint: dm_k = dmean/d + [k = argmin] dmin + [k = argmax] dmax
//               + dstd (m_k - mean) / (d std), with m_k recomputed.  The
// per-edge dm is stored in CSR order; D_in[i] = sum over in-edges (same
// pass) and D_out[j] = sum over the out-edges of j through the by-source
// transpose (second kernel): fixed summation orders, no atomics.
#include "agg_msg.hpp"

namespace hgnn {

namespace {

inline int cdiv(long long a, int b) { return (int)((a + b - 1) / b); }

template <int FE>
__global__ void __launch_bounds__(256)
k_aggregate(const Dims *__restrict__ dims, int H, const float *__restrict__ PQ,
            const int *__restrict__ rowptr, const int *__restrict__ csr_src,
            const float *__restrict__ csr_e, const float *__restrict__ WeT,
            const float *__restrict__ bmv, float *__restrict__ A,
            uint8_t *__restrict__ args, float eps, __bf16 *__restrict__ Ab) {
  const int tpn = H >> 2;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = (int)(t / tpn), c = (int)(t % tpn) * 4;
  if (i >= dims->N) return;
  const int lo = rowptr[i], hi = rowptr[i + 1], d = hi - lo;
  f4 mu = {0.f, 0.f, 0.f, 0.f}, mn = mu, mx = mu, sd = mu;
  uint32_t amin = 0, amax = 0;
  if (d > 0) {
    f4 we[4];
#pragma unroll
    for (int f = 0; f < FE; ++f)
      we[f] = *reinterpret_cast<const f4 *>(WeT + (size_t)f * H + c);
    const f4 bm = *reinterpret_cast<const f4 *>(bmv + c);
    const f4 p = *reinterpret_cast<const f4 *>(PQ + (size_t)i * 2 * H + c);
    f4 cache[kCache];
    float ev[kCache][4];
    const int dc = gather_messages<FE>(PQ, H, c, p, bm, we, csr_src, csr_e, lo, d, cache, ev);
    f4 sum = cache[0];
    mn = cache[0];
    mx = cache[0];
    int imn[4] = {0, 0, 0, 0}, imx[4] = {0, 0, 0, 0};
    auto visit = [&](const f4 &m, int o) {
      sum += m;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (m[e] < mn[e]) { mn[e] = m[e]; imn[e] = o; }
        if (m[e] > mx[e]) { mx[e] = m[e]; imx[e] = o; }
      }
    };
#pragma unroll
    for (int o = 1; o < kCache; ++o)
      if (o < dc) visit(cache[o], o);
    for (int o = kCache; o < d; ++o)
      visit(message<FE>(PQ, H, csr_src[lo + o], c, p, bm, we, csr_e, lo + o), o);
    const float fd = (float)d;
    mu = sum / fd;
    f4 ss = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int o = 0; o < kCache; ++o)
      if (o < dc) {
        const f4 dv = cache[o] - mu;
        ss += dv * dv;
      }
    for (int o = kCache; o < d; ++o) {
      const f4 dv = message<FE>(PQ, H, csr_src[lo + o], c, p, bm, we, csr_e, lo + o) - mu;
      ss += dv * dv;
    }
    const f4 var = ss / fd;
#pragma unroll
    for (int e = 0; e < 4; ++e) sd[e] = sqrtf(var[e] + eps);
    amin = (uint32_t)imn[0] | ((uint32_t)imn[1] << 8) | ((uint32_t)imn[2] << 16) |
           ((uint32_t)imn[3] << 24);
    amax = (uint32_t)imx[0] | ((uint32_t)imx[1] << 8) | ((uint32_t)imx[2] << 16) |
           ((uint32_t)imx[3] << 24);
  }
  float *Ai = A + (size_t)i * 4 * H;
  *reinterpret_cast<f4 *>(Ai + c) = mu;
  *reinterpret_cast<f4 *>(Ai + H + c) = mn;
  *reinterpret_cast<f4 *>(Ai + 2 * H + c) = mx;
  *reinterpret_cast<f4 *>(Ai + 3 * H + c) = sd;
  if (Ab) { // the BF16 copy read by the BF16 update linear (RNE, as its staging rounds)
    __bf16 *Bi = Ab + (size_t)i * 4 * H;
    const f4 v[4] = {mu, mn, mx, sd};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      bf16x4 b;
#pragma unroll
      for (int e = 0; e < 4; ++e) b[e] = (__bf16)v[j][e];
      *reinterpret_cast<bf16x4 *>(Bi + j * H + c) = b;
    }
  }
  if (args) {
    uint8_t *ai = args + (size_t)i * 2 * H;
    *reinterpret_cast<uint32_t *>(ai + c) = amin;
    *reinterpret_cast<uint32_t *>(ai + H + c) = amax;
  }
}

template <int FE>
__global__ void __launch_bounds__(256)
k_aggregate_bwd(const Dims *__restrict__ dims, int H, const float *__restrict__ PQ,
                const int *__restrict__ rowptr, const int *__restrict__ csr_src,
                const float *__restrict__ csr_e, const float *__restrict__ WeT,
                const float *__restrict__ bmv, const float *__restrict__ A,
                const uint8_t *__restrict__ args, const float *__restrict__ dA,
                float *__restrict__ dm, float *__restrict__ D, int ldD) {
  const int tpn = H >> 2;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = (int)(t / tpn), c = (int)(t % tpn) * 4;
  if (i >= dims->N) return;
  const float *dAi = dA + (size_t)i * 4 * H;
  const f4 dmu = *reinterpret_cast<const f4 *>(dAi + c);
  const f4 dmn = *reinterpret_cast<const f4 *>(dAi + H + c);
  const f4 dmx = *reinterpret_cast<const f4 *>(dAi + 2 * H + c);
  const f4 dsd = *reinterpret_cast<const f4 *>(dAi + 3 * H + c);
  node_adjoint<FE>(i, c, H, PQ, rowptr, csr_src, csr_e, WeT, bmv, A, args, dmu, dmn, dmx, dsd,
                   dm, D, ldD);
}

__global__ void __launch_bounds__(256)
k_transpose_sum(const Dims *__restrict__ dims, int H, const int *__restrict__ srcptr,
                const int *__restrict__ t2csr, const float *__restrict__ dm,
                float *__restrict__ D, int ldD) {
  const int tpn = H >> 2;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = (int)(t / tpn), c = (int)(t % tpn) * 4;
  if (j >= dims->N) return;
  const int lo = srcptr[j], hi = srcptr[j + 1], d = hi - lo;
  f4 s = {0.f, 0.f, 0.f, 0.f};
  if (d > 0) {
    int pos[kCache];
#pragma unroll
    for (int o = 0; o < kCache; ++o) pos[o] = t2csr[lo + min(o, d - 1)];
    f4 v[kCache];
#pragma unroll
    for (int o = 0; o < kCache; ++o) v[o] = *reinterpret_cast<const f4 *>(dm + (size_t)pos[o] * H + c);
#pragma unroll
    for (int o = 0; o < kCache; ++o)
      if (o < d) s += v[o];
    for (int p = lo + kCache; p < hi; ++p)
      s += *reinterpret_cast<const f4 *>(dm + (size_t)t2csr[p] * H + c);
  }
  *reinterpret_cast<f4 *>(D + (size_t)j * ldD + H + c) = s;
}

__global__ void __launch_bounds__(256)
k_relu_mask(const Dims *__restrict__ dims, int H, const float *__restrict__ dh,
            const float *__restrict__ hout, float *__restrict__ du) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long n4 = (long long)dims->N * H / 4;
  if (t >= n4) return;
  const f4 g = reinterpret_cast<const f4 *>(dh)[t];
  const f4 h = reinterpret_cast<const f4 *>(hout)[t];
  f4 o;
#pragma unroll
  for (int e = 0; e < 4; ++e) o[e] = h[e] > 0.f ? g[e] : 0.f;
  reinterpret_cast<f4 *>(du)[t] = o;
}

} // namespace

// A non-null event pair is stamped with the kernel's own start and end
// (hipExtLaunchKernelGGL), so its elapsed time is the kernel's duration.
hipError_t launch_aggregate(const Dims *dims, int capN, int H, int Fe,
                            const float *PQ, const int *rowptr, const int *csr_src,
                            const float *csr_e, const float *WeT,
                            const float *bm, float *A, uint8_t *args, float eps,
                            hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, __bf16 *Ab) {
  if (capN <= 0) return hipSuccess;
  const dim3 grid(cdiv((long long)capN * (H / 4), 256));
#define HGNN_AGG(FE)                                                                      \
  hipExtLaunchKernelGGL(k_aggregate<FE>, grid, dim3(256), 0, s, ev0, ev1, 0, dims, H, PQ,  \
                        rowptr, csr_src, csr_e, WeT, bm, A, args, eps, Ab)
  switch (Fe) {
  case 0: HGNN_AGG(0); break;
  case 1: HGNN_AGG(1); break;
  case 2: HGNN_AGG(2); break;
  case 3: HGNN_AGG(3); break;
  default: HGNN_AGG(4); break;
  }
#undef HGNN_AGG
  return hipGetLastError();
}

hipError_t launch_aggregate_bwd(const Dims *dims, int capN, int H, int Fe,
                                const float *PQ, const int *rowptr,
                                const int *csr_src, const float *csr_e,
                                const float *WeT, const float *bm,
                                const float *A, const uint8_t *args,
                                const float *dA, float *dm, float *D, int ldD,
                                hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if (capN <= 0) return hipSuccess;
  const dim3 grid(cdiv((long long)capN * (H / 4), 256));
#define HGNN_AGG_BWD(FE)                                                                  \
  hipExtLaunchKernelGGL(k_aggregate_bwd<FE>, grid, dim3(256), 0, s, ev0, ev1, 0, dims, H,  \
                        PQ, rowptr, csr_src, csr_e, WeT, bm, A, args, dA, dm, D, ldD)
  switch (Fe) {
  case 0: HGNN_AGG_BWD(0); break;
  case 1: HGNN_AGG_BWD(1); break;
  case 2: HGNN_AGG_BWD(2); break;
  case 3: HGNN_AGG_BWD(3); break;
  default: HGNN_AGG_BWD(4); break;
  }
#undef HGNN_AGG_BWD
  return hipGetLastError();
}

hipError_t launch_transpose_sum(const Dims *dims, int capN, int H, const int *srcptr,
                                const int *t2csr, const float *dm, float *D, int ldD,
                                hipStream_t s) {
  if (capN <= 0) return hipSuccess;
  k_transpose_sum<<<cdiv((long long)capN * (H / 4), 256), 256, 0, s>>>(dims, H, srcptr,
                                                                       t2csr, dm, D, ldD);
  return hipGetLastError();
}

hipError_t launch_relu_mask(const Dims *dims, int capN, int H, const float *dh,
                            const float *hout, float *du, hipStream_t s) {
  if (capN <= 0) return hipSuccess;
  k_relu_mask<<<cdiv((long long)capN * H / 4, 256), 256, 0, s>>>(dims, H, dh, hout, du);
  return hipGetLastError();
}

} // namespace hgnn
