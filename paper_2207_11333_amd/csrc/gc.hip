// The other GC layer kinds HydraGNN provides (named in Section 2 of the
// paper): GraphSAGE with the mean aggregator and CGCNN's gated edge
// convolution.  Both run on the destination-sorted CSR of csr.hip and the
// MFMA GEMMs of gemm_nt.hip / gemm_tn.hip; this file holds their
// neighbourhood kernels and the staging of their weights into GEMM layouts.
//
//  GraphSAGE:  M_i = mean of h_j over in-edges j -> i (0 without in-edges),
//              h'_i = ReLU(W_self h_i + W_nbr M_i + b).
//  CGCNN:      z = [h_i || h_j || e_ij], f = W_f z + b_f, s = W_s z + b_s,
//              h'_i = ReLU(h_i + sum over in-edges sigmoid(f) * softplus(s)),
//              after a linear embedding of the atom features.
//
// One thread per (node, 4 features); a node's in-edges are visited in CSR
// order, so every sum has a fixed order and results are reproducible.
#include "common.hpp"

namespace hgnn {

namespace {

inline int cdiv(long long a, int b) { return (int)((a + b - 1) / b); }

constexpr int kBatch = 4; // in-edges whose loads are issued together

__device__ __forceinline__ f4 ld4(const float *p) { return *reinterpret_cast<const f4 *>(p); }
__device__ __forceinline__ void st4(float *p, f4 v) { *reinterpret_cast<f4 *>(p) = v; }

// sigmoid and softplus in forms that neither overflow nor lose small values,
// on the hardware exponential, logarithm and reciprocal (__expf, __logf,
// v_rcp_f32: a few ulp).  Both start from e = exp(-|x|) in (0, 1]:
//   sigmoid(x)  = 1 / (1 + e) for x >= 0, e / (1 + e) otherwise;
//   softplus(x) = max(x, 0) + log1p(e), with log1p(e) = log(u) e / (u - 1),
//                 u = 1 + e rounded (Kahan's correction, Goldberg 1991,
//                 Theorem 4: u - 1 is exact, and the factor e / (u - 1)
//                 cancels the rounding of u); log1p(e) = e when u rounds to 1.
__device__ __forceinline__ float neg_abs_exp(float x) { return __expf(-fabsf(x)); }
__device__ __forceinline__ float sigm_e(float x, float e) {
  const float r = __builtin_amdgcn_rcpf(1.0f + e);
  return x >= 0.f ? r : e * r;
}
__device__ __forceinline__ float softp_e(float x, float e) {
  const float u = 1.0f + e;
  const float lp = u == 1.0f ? e : __logf(u) * (e * __builtin_amdgcn_rcpf(u - 1.0f));
  return fmaxf(x, 0.f) + lp;
}

// ---- GraphSAGE ------------------------------------------------------------

// M[i, :] = mean of h[j, :] over the in-edges of i (F columns, F % 4 == 0).
__global__ void __launch_bounds__(256)
k_sage_mean(const Dims *__restrict__ dims, int F, const int *__restrict__ rowptr,
            const int *__restrict__ csr_src, const float *__restrict__ h, int ldh,
            float *__restrict__ M) {
  const int tpn = F >> 2;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = (int)(t / tpn), c = (int)(t % tpn) * 4;
  if (i >= dims->N) return;
  const int lo = rowptr[i], hi = rowptr[i + 1];
  f4 s = {0.f, 0.f, 0.f, 0.f};
  // kBatch in-edges at a time: their ids, then their rows, are in flight
  // together (clamped to the last in-edge, masked after)
  for (int p0 = lo; p0 < hi; p0 += kBatch) {
    int j[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) j[u] = csr_src[min(p0 + u, hi - 1)];
    f4 v[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) v[u] = ld4(h + (size_t)j[u] * ldh + c);
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
      if (p0 + u < hi) s += v[u];
  }
  if (hi > lo) {
    const float d = (float)(hi - lo);
#pragma unroll
    for (int e = 0; e < 4; ++e) s[e] = s[e] / d;
  }
  st4(M + (size_t)i * F + c, s);
}

// dh_in[j] = G[j, 0:F] + sum over out-edges j -> i of G[i, F:2F] / deg(i),
// zeroed where mask <= 0 (the ReLU adjoint of the layer that produced h_in).
__global__ void __launch_bounds__(256)
k_sage_scatter(const Dims *__restrict__ dims, int F, const int *__restrict__ srcptr,
               const int *__restrict__ t2csr, const int *__restrict__ csr_dst,
               const int *__restrict__ rowptr, const float *__restrict__ G,
               const float *__restrict__ mask, float *__restrict__ dh) {
  const int tpn = F >> 2;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = (int)(t / tpn), c = (int)(t % tpn) * 4;
  if (j >= dims->N) return;
  const size_t ldg = 2 * (size_t)F;
  f4 s = ld4(G + (size_t)j * ldg + c);
  const int lo = srcptr[j], hi = srcptr[j + 1];
  for (int q0 = lo; q0 < hi; q0 += kBatch) {
    int i[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) i[u] = csr_dst[t2csr[min(q0 + u, hi - 1)]];
    f4 g[kBatch];
    float d[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      g[u] = ld4(G + (size_t)i[u] * ldg + F + c);
      d[u] = (float)(rowptr[i[u] + 1] - rowptr[i[u]]);
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
      if (q0 + u < hi) {
#pragma unroll
        for (int e = 0; e < 4; ++e) s[e] += g[u][e] / d[u];
      }
  }
  if (mask) {
    const f4 m = ld4(mask + (size_t)j * F + c);
#pragma unroll
    for (int e = 0; e < 4; ++e) s[e] = m[e] > 0.f ? s[e] : 0.f;
  }
  st4(dh + (size_t)j * F + c, s);
}

// ---- CGCNN ----------------------------------------------------------------
// PQ [N, 4H] = [P_f | P_s | Q_f | Q_s]: the destination (P) and source (Q)
// parts of the filter and core linears; weT [Fe, 2H] their edge-feature
// columns; b [2H] their biases.

// edge-feature columns of the filter and core linears for FE features
template <int FE> struct EdgeTerms {
  f4 wf[FE > 0 ? FE : 1], ws[FE > 0 ? FE : 1];
};

// Filter and core pre-activations of in-edges p0 .. p0 + kBatch - 1 (clamped
// to the last in-edge hi - 1; the caller masks the extra ones): all source
// ids first, then all gathered rows, so the loads are in flight together.
template <int FE>
__device__ __forceinline__ void gate_batch(const float *__restrict__ PQ, int H,
                                           const int *__restrict__ csr_src,
                                           const float *__restrict__ csr_e, int p0, int hi,
                                           f4 Pf, f4 Ps, const EdgeTerms<FE> &w, f4 (&f)[kBatch],
                                           f4 (&s)[kBatch]) {
  int j[kBatch];
#pragma unroll
  for (int u = 0; u < kBatch; ++u) j[u] = csr_src[min(p0 + u, hi - 1)];
#pragma unroll
  for (int u = 0; u < kBatch; ++u) {
    const size_t r = (size_t)j[u] * 4 * H;
    f[u] = Pf + ld4(PQ + r + 2 * H);
    s[u] = Ps + ld4(PQ + r + 3 * H);
  }
#pragma unroll
  for (int k = 0; k < FE; ++k) {
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const float ev = csr_e[(size_t)min(p0 + u, hi - 1) * FE + k];
      f[u] += w.wf[k] * ev;
      s[u] += w.ws[k] * ev;
    }
  }
}

// FE (the edge-feature count, 0..4) is a template parameter so that the
// per-feature arrays are sized exactly and indexed by constants.
template <int FE>
__global__ void __launch_bounds__(256)
k_cg_aggregate(const Dims *__restrict__ dims, int H, const int *__restrict__ rowptr,
               const int *__restrict__ csr_src, const float *__restrict__ csr_e,
               const float *__restrict__ PQ, const float *__restrict__ weT,
               const float *__restrict__ b, const float *__restrict__ h_in,
               float *__restrict__ h_out) {
  const int tpn = H >> 2;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = (int)(t / tpn), c = (int)(t % tpn) * 4;
  if (i >= dims->N) return;
  EdgeTerms<FE> w;
#pragma unroll
  for (int k = 0; k < FE; ++k) {
    w.wf[k] = ld4(weT + (size_t)k * 2 * H + c);
    w.ws[k] = ld4(weT + (size_t)k * 2 * H + H + c);
  }
  const size_t r = (size_t)i * 4 * H;
  const f4 Pf = ld4(PQ + r + c) + ld4(b + c), Ps = ld4(PQ + r + H + c) + ld4(b + H + c);
  f4 acc = {0.f, 0.f, 0.f, 0.f};
  const int lo = rowptr[i], hi = rowptr[i + 1];
  for (int p0 = lo; p0 < hi; p0 += kBatch) {
    f4 f[kBatch], s[kBatch];
    gate_batch<FE>(PQ + c, H, csr_src, csr_e, p0, hi, Pf, Ps, w, f, s);
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
      if (p0 + u < hi) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float ef = neg_abs_exp(f[u][e]), es = neg_abs_exp(s[u][e]);
          acc[e] += sigm_e(f[u][e], ef) * softp_e(s[u][e], es);
        }
      }
  }
  const f4 u = ld4(h_in + (size_t)i * H + c) + acc;
  f4 o;
#pragma unroll
  for (int e = 0; e < 4; ++e) o[e] = u[e] > 0.f ? u[e] : 0.f;
  st4(h_out + (size_t)i * H + c, o);
}

// From du = dL/du (the layer's ReLU adjoint applied): per in-edge the
// pre-activation gradients dm = [df | ds] [E, 2H], and per node
// D[i] = [sum dm (2H) | (D_out, written by the transpose) | sum dm e_k (Fe x 2H)].
template <int FE>
__global__ void __launch_bounds__(256)
k_cg_aggregate_bwd(const Dims *__restrict__ dims, int H, const int *__restrict__ rowptr,
                   const int *__restrict__ csr_src, const float *__restrict__ csr_e,
                   const float *__restrict__ PQ, const float *__restrict__ weT,
                   const float *__restrict__ b, const float *__restrict__ du,
                   float *__restrict__ dm, float *__restrict__ D, int ldD) {
  const int tpn = H >> 2;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = (int)(t / tpn), c = (int)(t % tpn) * 4;
  if (i >= dims->N) return;
  EdgeTerms<FE> w;
#pragma unroll
  for (int k = 0; k < FE; ++k) {
    w.wf[k] = ld4(weT + (size_t)k * 2 * H + c);
    w.ws[k] = ld4(weT + (size_t)k * 2 * H + H + c);
  }
  const size_t r = (size_t)i * 4 * H;
  const f4 Pf = ld4(PQ + r + c) + ld4(b + c), Ps = ld4(PQ + r + H + c) + ld4(b + H + c);
  const f4 g = ld4(du + (size_t)i * H + c);
  const f4 z = {0.f, 0.f, 0.f, 0.f};
  f4 sf_in = z, ss_in = z, ef[FE > 0 ? FE : 1], es[FE > 0 ? FE : 1];
#pragma unroll
  for (int k = 0; k < (FE > 0 ? FE : 1); ++k) ef[k] = es[k] = z;
  const int lo = rowptr[i], hi = rowptr[i + 1];
  for (int p0 = lo; p0 < hi; p0 += kBatch) {
    f4 f[kBatch], s[kBatch];
    gate_batch<FE>(PQ + c, H, csr_src, csr_e, p0, hi, Pf, Ps, w, f, s);
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      if (p0 + u >= hi) break;
      const int p = p0 + u;
      f4 df, ds;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float ef = neg_abs_exp(f[u][e]), es = neg_abs_exp(s[u][e]);
        const float a = sigm_e(f[u][e], ef);
        df[e] = g[e] * softp_e(s[u][e], es) * a * (1.0f - a);
        ds[e] = g[e] * a * sigm_e(s[u][e], es);
      }
      st4(dm + (size_t)p * 2 * H + c, df);
      st4(dm + (size_t)p * 2 * H + H + c, ds);
      sf_in += df;
      ss_in += ds;
#pragma unroll
      for (int k = 0; k < FE; ++k) {
        const float ev = csr_e[(size_t)p * FE + k];
        ef[k] += df * ev;
        es[k] += ds * ev;
      }
    }
  }
  float *Di = D + (size_t)i * ldD;
  st4(Di + c, sf_in);
  st4(Di + H + c, ss_in);
#pragma unroll
  for (int k = 0; k < FE; ++k) {
    st4(Di + 4 * H + (size_t)k * 2 * H + c, ef[k]);
    st4(Di + 4 * H + (size_t)k * 2 * H + H + c, es[k]);
  }
}

// ---- weight staging ---------------------------------------------------------
// Job y copies a rows x cols block: dst[r * ld + c] = src[r * rs + c * cs]
// for r < vrows and c < vcols, 0 elsewhere; as FP32 or as a BF16 hi + lo pair.
__global__ void __launch_bounds__(256)
k_gc_stage(const GcStageJob *__restrict__ jobs, long long *bump) {
  const GcStageJob &j = jobs[blockIdx.y];
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (bump && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *bump += 1;
  if (t >= (long long)j.rows * j.cols) return;
  const int r = (int)(t / j.cols), c = (int)(t % j.cols);
  const float v = (r < j.vrows && c < j.vcols) ? j.src[r * j.rs + c * j.cs] : 0.f;
  const size_t o = (size_t)r * j.ld + c;
  if (j.bf16) {
    const __bf16 hi = (__bf16)v;
    reinterpret_cast<__bf16 *>(j.hi)[o] = hi;
    reinterpret_cast<__bf16 *>(j.lo)[o] = (__bf16)(v - (float)hi);
  } else {
    reinterpret_cast<float *>(j.hi)[o] = v;
  }
}

} // namespace

hipError_t launch_sage_mean(const Dims *dims, int capN, int F, const int *rowptr,
                            const int *csr_src, const float *h, int ldh, float *M,
                            hipStream_t s) {
  if (capN <= 0) return hipSuccess;
  if (F % 4 || ldh % 4) return hipErrorInvalidValue;
  k_sage_mean<<<cdiv((long long)capN * (F / 4), 256), 256, 0, s>>>(dims, F, rowptr, csr_src,
                                                                   h, ldh, M);
  return hipGetLastError();
}

hipError_t launch_sage_scatter(const Dims *dims, int capN, int F, const int *srcptr,
                               const int *t2csr, const int *csr_dst, const int *rowptr,
                               const float *G, const float *mask, float *dh, hipStream_t s) {
  if (capN <= 0) return hipSuccess;
  if (F % 4) return hipErrorInvalidValue;
  k_sage_scatter<<<cdiv((long long)capN * (F / 4), 256), 256, 0, s>>>(
      dims, F, srcptr, t2csr, csr_dst, rowptr, G, mask, dh);
  return hipGetLastError();
}

hipError_t launch_cg_aggregate(const Dims *dims, int capN, int H, int Fe, const int *rowptr,
                               const int *csr_src, const float *csr_e, const float *PQ,
                               const float *weT, const float *b, const float *h_in,
                               float *h_out, hipStream_t s) {
  if (capN <= 0) return hipSuccess;
  if (H % 4 || Fe < 0 || Fe > kMaxFe) return hipErrorInvalidValue;
  const int grid = cdiv((long long)capN * (H / 4), 256);
#define HGNN_CG_FWD(FE)                                                                    \
  k_cg_aggregate<FE><<<grid, 256, 0, s>>>(dims, H, rowptr, csr_src, csr_e, PQ, weT, b, h_in, \
                                          h_out)
  switch (Fe) {
  case 0: HGNN_CG_FWD(0); break;
  case 1: HGNN_CG_FWD(1); break;
  case 2: HGNN_CG_FWD(2); break;
  case 3: HGNN_CG_FWD(3); break;
  default: HGNN_CG_FWD(4); break;
  }
#undef HGNN_CG_FWD
  return hipGetLastError();
}

hipError_t launch_cg_aggregate_bwd(const Dims *dims, int capN, int H, int Fe,
                                   const int *rowptr, const int *csr_src, const float *csr_e,
                                   const float *PQ, const float *weT, const float *b,
                                   const float *du, float *dm, float *D, int ldD,
                                   hipStream_t s) {
  if (capN <= 0) return hipSuccess;
  if (H % 4 || Fe < 0 || Fe > kMaxFe || ldD % 4) return hipErrorInvalidValue;
  const int grid = cdiv((long long)capN * (H / 4), 256);
#define HGNN_CG_BWD(FE)                                                                    \
  k_cg_aggregate_bwd<FE><<<grid, 256, 0, s>>>(dims, H, rowptr, csr_src, csr_e, PQ, weT, b, du, \
                                              dm, D, ldD)
  switch (Fe) {
  case 0: HGNN_CG_BWD(0); break;
  case 1: HGNN_CG_BWD(1); break;
  case 2: HGNN_CG_BWD(2); break;
  case 3: HGNN_CG_BWD(3); break;
  default: HGNN_CG_BWD(4); break;
  }
#undef HGNN_CG_BWD
  return hipGetLastError();
}

hipError_t launch_gc_stage(const GcStageJob *jobs, int njobs, long long max_elems,
                           long long *bump, hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  const dim3 grid(cdiv(max_elems > 0 ? max_elems : 1, 256), njobs);
  k_gc_stage<<<grid, 256, 0, s>>>(jobs, bump);
  return hipGetLastError();
}

} // namespace hgnn
