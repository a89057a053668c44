// Message recomputation shared by the aggregation (aggregate.hip) and the
// fused aggregation adjoint (agg_fused.hip): m_k = P_i + Q_src(k) + e_k w_e + b
// for four consecutive features, with up to kCache in-edges of a node
// fetched together.
#pragma once
#include "common.hpp"

namespace hgnn {

namespace {

constexpr int kCache = 4; // messages kept in registers per thread

template <int FE>
__device__ __forceinline__ f4 message(const float *__restrict__ PQ, int H, int s,
                                      int c, f4 p, f4 bm, const f4 (&we)[4],
                                      const float *__restrict__ csr_e, int q) {
  f4 m = p + *reinterpret_cast<const f4 *>(PQ + (size_t)s * 2 * H + H + c);
#pragma unroll
  for (int f = 0; f < FE; ++f) m += csr_e[(size_t)q * FE + f] * we[f];
  return m + bm;
}

// Up to kCache in-edges of a node are fetched together: all source ids,
// then all gathered Q rows, so a node costs three dependent memory latencies
// (rowptr, ids, rows) whatever its degree up to kCache; the loads are from
// clamped indices and masked, so no branch serialises them.
template <int FE>
__device__ __forceinline__ int gather_messages(const float *__restrict__ PQ, int H, int c,
                                               f4 p, f4 bm, const f4 (&we)[4],
                                               const int *__restrict__ csr_src,
                                               const float *__restrict__ csr_e, int lo,
                                               int d, f4 (&m)[kCache], float (&ev)[kCache][4]) {
  int src[kCache];
#pragma unroll
  for (int o = 0; o < kCache; ++o) src[o] = csr_src[lo + min(o, d - 1)];
#pragma unroll
  for (int o = 0; o < kCache; ++o) {
    const int q = lo + min(o, d - 1);
#pragma unroll
    for (int f = 0; f < FE; ++f) ev[o][f] = csr_e[(size_t)q * FE + f];
  }
  f4 qr[kCache];
#pragma unroll
  for (int o = 0; o < kCache; ++o)
    qr[o] = *reinterpret_cast<const f4 *>(PQ + (size_t)src[o] * 2 * H + H + c);
#pragma unroll
  for (int o = 0; o < kCache; ++o) {
    f4 v = p + qr[o];
#pragma unroll
    for (int f = 0; f < FE; ++f) v += ev[o][f] * we[f];
    m[o] = v + bm;
  }
  return min(d, kCache);
}

// The aggregation adjoint of node i, features c .. c + 3, given its gradients
// dmu, dmn, dmx, dsd with respect to the mean, min, max and std aggregates:
// dm_k = dmu/d + [k = argmin] dmn + [k = argmax] dmx + dsd (m_k - mean)/(d std)
// for its in-edges k (messages recomputed), written per edge in CSR order,
// with D_in (their sum) and De (their edge-feature-weighted sums) into the
// node's row of D.
template <int FE>
__device__ __forceinline__ void node_adjoint(int i, int c, int H, const float *__restrict__ PQ,
                                             const int *__restrict__ rowptr,
                                             const int *__restrict__ csr_src,
                                             const float *__restrict__ csr_e,
                                             const float *__restrict__ WeT,
                                             const float *__restrict__ bmv,
                                             const float *__restrict__ A,
                                             const uint8_t *__restrict__ args, f4 dmu, f4 dmn,
                                             f4 dmx, f4 dsd, float *__restrict__ dm,
                                             float *__restrict__ D, int ldD) {
  const int lo = rowptr[i], hi = rowptr[i + 1], d = hi - lo;
  f4 din = {0.f, 0.f, 0.f, 0.f};
  f4 de[4] = {din, din, din, din};
  if (d > 0) {
    f4 we[4];
#pragma unroll
    for (int f = 0; f < FE; ++f)
      we[f] = *reinterpret_cast<const f4 *>(WeT + (size_t)f * H + c);
    const f4 bm = *reinterpret_cast<const f4 *>(bmv + c);
    const f4 p = *reinterpret_cast<const f4 *>(PQ + (size_t)i * 2 * H + c);
    const float *Ai = A + (size_t)i * 4 * H;
    const f4 mu = *reinterpret_cast<const f4 *>(Ai + c);
    const f4 sd = *reinterpret_cast<const f4 *>(Ai + 3 * H + c);
    const uint32_t amin = *reinterpret_cast<const uint32_t *>(args + (size_t)i * 2 * H + c);
    const uint32_t amax = *reinterpret_cast<const uint32_t *>(args + (size_t)i * 2 * H + H + c);
    f4 cache[kCache];
    float ev[kCache][4];
    const int dc = gather_messages<FE>(PQ, H, c, p, bm, we, csr_src, csr_e, lo, d, cache, ev);
    const float fd = (float)d;
    const f4 base = dmu / fd;
    const f4 coef = dsd / (fd * sd);
    auto emit = [&](const f4 &m, int o, const float *e) {
      f4 g = base + coef * (m - mu);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if ((int)((amin >> (8 * k)) & 0xff) == o) g[k] += dmn[k];
        if ((int)((amax >> (8 * k)) & 0xff) == o) g[k] += dmx[k];
      }
      *reinterpret_cast<f4 *>(dm + (size_t)(lo + o) * H + c) = g;
      din += g;
#pragma unroll
      for (int f = 0; f < FE; ++f) de[f] += g * e[f];
    };
#pragma unroll
    for (int o = 0; o < kCache; ++o)
      if (o < dc) emit(cache[o], o, ev[o]);
    for (int o = kCache; o < d; ++o) {
      const int q = lo + o;
      float e[4];
#pragma unroll
      for (int f = 0; f < FE; ++f) e[f] = csr_e[(size_t)q * FE + f];
      emit(message<FE>(PQ, H, csr_src[q], c, p, bm, we, csr_e, q), o, e);
    }
  }
  float *Di = D + (size_t)i * ldD;
  *reinterpret_cast<f4 *>(Di + c) = din;
#pragma unroll
  for (int f = 0; f < FE; ++f) *reinterpret_cast<f4 *>(Di + (2 + f) * H + c) = de[f];
}

} // namespace

} // namespace hgnn
