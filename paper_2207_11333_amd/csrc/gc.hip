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

__device__ __forceinline__ f4 ld4(const float *p) { return *reinterpret_cast<const f4 *>(p); }
__device__ __forceinline__ void st4(float *p, f4 v) { *reinterpret_cast<f4 *>(p) = v; }

// sigmoid and softplus in forms that neither overflow nor lose small values
__device__ __forceinline__ float sigm(float x) {
  const float e = expf(-fabsf(x));
  return x >= 0.f ? 1.0f / (1.0f + e) : e / (1.0f + e);
}
__device__ __forceinline__ float softp(float x) {
  return fmaxf(x, 0.f) + log1pf(expf(-fabsf(x)));
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
#pragma unroll 4
  for (int p = lo; p < hi; ++p) s += ld4(h + (size_t)csr_src[p] * ldh + c);
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
  for (int q = lo; q < hi; ++q) {
    const int i = csr_dst[t2csr[q]];
    const float d = (float)(rowptr[i + 1] - rowptr[i]);
    const f4 g = ld4(G + (size_t)i * ldg + F + c);
#pragma unroll
    for (int e = 0; e < 4; ++e) s[e] += g[e] / d;
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

struct EdgeTerms {
  f4 wf[kMaxFe], ws[kMaxFe];
};

__device__ __forceinline__ void gate_pre(const float *__restrict__ PQ, int H, int Fe, int j,
                                         const float *__restrict__ csr_e, int p, f4 Pf, f4 Ps,
                                         const EdgeTerms &w, f4 &f, f4 &s) {
  const size_t r = (size_t)j * 4 * H;
  f = Pf + ld4(PQ + r + 2 * H);
  s = Ps + ld4(PQ + r + 3 * H);
  for (int k = 0; k < Fe; ++k) {
    const float ev = csr_e[(size_t)p * Fe + k];
    f += w.wf[k] * ev;
    s += w.ws[k] * ev;
  }
}

__global__ void __launch_bounds__(256)
k_cg_aggregate(const Dims *__restrict__ dims, int H, int Fe, const int *__restrict__ rowptr,
               const int *__restrict__ csr_src, const float *__restrict__ csr_e,
               const float *__restrict__ PQ, const float *__restrict__ weT,
               const float *__restrict__ b, const float *__restrict__ h_in,
               float *__restrict__ h_out) {
  const int tpn = H >> 2;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = (int)(t / tpn), c = (int)(t % tpn) * 4;
  if (i >= dims->N) return;
  EdgeTerms w;
  for (int k = 0; k < Fe; ++k) {
    w.wf[k] = ld4(weT + (size_t)k * 2 * H + c);
    w.ws[k] = ld4(weT + (size_t)k * 2 * H + H + c);
  }
  const size_t r = (size_t)i * 4 * H;
  const f4 Pf = ld4(PQ + r + c) + ld4(b + c), Ps = ld4(PQ + r + H + c) + ld4(b + H + c);
  f4 acc = {0.f, 0.f, 0.f, 0.f};
  const int lo = rowptr[i], hi = rowptr[i + 1];
  for (int p = lo; p < hi; ++p) {
    f4 f, s;
    gate_pre(PQ + c, H, Fe, csr_src[p], csr_e, p, Pf, Ps, w, f, s);
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[e] += sigm(f[e]) * softp(s[e]);
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
__global__ void __launch_bounds__(256)
k_cg_aggregate_bwd(const Dims *__restrict__ dims, int H, int Fe, const int *__restrict__ rowptr,
                   const int *__restrict__ csr_src, const float *__restrict__ csr_e,
                   const float *__restrict__ PQ, const float *__restrict__ weT,
                   const float *__restrict__ b, const float *__restrict__ du,
                   float *__restrict__ dm, float *__restrict__ D, int ldD) {
  const int tpn = H >> 2;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = (int)(t / tpn), c = (int)(t % tpn) * 4;
  if (i >= dims->N) return;
  EdgeTerms w;
  for (int k = 0; k < Fe; ++k) {
    w.wf[k] = ld4(weT + (size_t)k * 2 * H + c);
    w.ws[k] = ld4(weT + (size_t)k * 2 * H + H + c);
  }
  const size_t r = (size_t)i * 4 * H;
  const f4 Pf = ld4(PQ + r + c) + ld4(b + c), Ps = ld4(PQ + r + H + c) + ld4(b + H + c);
  const f4 g = ld4(du + (size_t)i * H + c);
  const f4 z = {0.f, 0.f, 0.f, 0.f};
  f4 sf_in = z, ss_in = z, ef[kMaxFe], es[kMaxFe];
  for (int k = 0; k < kMaxFe; ++k) ef[k] = es[k] = z;
  const int lo = rowptr[i], hi = rowptr[i + 1];
  for (int p = lo; p < hi; ++p) {
    f4 f, s;
    gate_pre(PQ + c, H, Fe, csr_src[p], csr_e, p, Pf, Ps, w, f, s);
    f4 df, ds;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float a = sigm(f[e]);
      df[e] = g[e] * softp(s[e]) * a * (1.0f - a);
      ds[e] = g[e] * a * sigm(s[e]);
    }
    st4(dm + (size_t)p * 2 * H + c, df);
    st4(dm + (size_t)p * 2 * H + H + c, ds);
    sf_in += df;
    ss_in += ds;
    for (int k = 0; k < Fe; ++k) {
      const float ev = csr_e[(size_t)p * Fe + k];
      ef[k] += df * ev;
      es[k] += ds * ev;
    }
  }
  float *Di = D + (size_t)i * ldD;
  st4(Di + c, sf_in);
  st4(Di + H + c, ss_in);
  for (int k = 0; k < Fe; ++k) {
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
  k_cg_aggregate<<<cdiv((long long)capN * (H / 4), 256), 256, 0, s>>>(
      dims, H, Fe, rowptr, csr_src, csr_e, PQ, weT, b, h_in, h_out);
  return hipGetLastError();
}

hipError_t launch_cg_aggregate_bwd(const Dims *dims, int capN, int H, int Fe,
                                   const int *rowptr, const int *csr_src, const float *csr_e,
                                   const float *PQ, const float *weT, const float *b,
                                   const float *du, float *dm, float *D, int ldD,
                                   hipStream_t s) {
  if (capN <= 0) return hipSuccess;
  if (H % 4 || Fe < 0 || Fe > kMaxFe || ldD % 4) return hipErrorInvalidValue;
  k_cg_aggregate_bwd<<<cdiv((long long)capN * (H / 4), 256), 256, 0, s>>>(
      dims, H, Fe, rowptr, csr_src, csr_e, PQ, weT, b, du, dm, D, ldD);
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
