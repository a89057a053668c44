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

// The source ids of up to kCache in-edges of a node (lo, degree d > 0), from
// clamped indices so that no branch serialises the loads.
__device__ __forceinline__ void fetch_sources(const int *__restrict__ csr_src, int lo, int d,
                                              int (&src)[kCache]) {
#pragma unroll
  for (int o = 0; o < kCache; ++o) src[o] = csr_src[lo + min(o, d - 1)];
}

// The gathered Q rows and edge features of those edges.
template <int FE>
__device__ __forceinline__ void load_rows(const float *__restrict__ PQ, int H, int c,
                                          const int (&src)[kCache],
                                          const float *__restrict__ csr_e, int lo, int d,
                                          f4 (&qr)[kCache], float (&ev)[kCache][4]) {
#pragma unroll
  for (int o = 0; o < kCache; ++o) {
    const int q = lo + min(o, d - 1);
#pragma unroll
    for (int f = 0; f < FE; ++f) ev[o][f] = csr_e[(size_t)q * FE + f];
  }
#pragma unroll
  for (int o = 0; o < kCache; ++o)
    qr[o] = *reinterpret_cast<const f4 *>(PQ + (size_t)src[o] * 2 * H + H + c);
}

// Messages from the loaded rows, in the order of message().
template <int FE>
__device__ __forceinline__ void form_messages(f4 p, f4 bm, const f4 (&we)[4],
                                              const f4 (&qr)[kCache],
                                              const float (&ev)[kCache][4], f4 (&m)[kCache]) {
#pragma unroll
  for (int o = 0; o < kCache; ++o) {
    f4 v = p + qr[o];
#pragma unroll
    for (int f = 0; f < FE; ++f) v += ev[o][f] * we[f];
    m[o] = v + bm;
  }
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
  fetch_sources(csr_src, lo, d, src);
  f4 qr[kCache];
  load_rows<FE>(PQ, H, c, src, csr_e, lo, d, qr, ev);
  form_messages<FE>(p, bm, we, qr, ev, m);
  return min(d, kCache);
}

// The operands of node i's aggregation adjoint at features c .. c + 3 that
// do not depend on its aggregate gradients (loaded only for d > 0).
struct AdjIn {
  int lo, d;
  f4 p, bm, mu, sd;
  f4 we[4];
  uint32_t amin, amax;
  f4 qr[kCache];
  float ev[kCache][4];
};

template <int FE>
__device__ __forceinline__ void adj_load(AdjIn &n, int i, int lo, int d,
                                         const int (&src)[kCache], int c, int H,
                                         const float *__restrict__ PQ,
                                         const float *__restrict__ csr_e,
                                         const float *__restrict__ WeT,
                                         const float *__restrict__ bmv,
                                         const float *__restrict__ A,
                                         const uint8_t *__restrict__ args) {
  n.lo = lo;
  n.d = d;
  if (d > 0) {
#pragma unroll
    for (int f = 0; f < FE; ++f)
      n.we[f] = *reinterpret_cast<const f4 *>(WeT + (size_t)f * H + c);
    n.bm = *reinterpret_cast<const f4 *>(bmv + c);
    n.p = *reinterpret_cast<const f4 *>(PQ + (size_t)i * 2 * H + c);
    const float *Ai = A + (size_t)i * 4 * H;
    n.mu = *reinterpret_cast<const f4 *>(Ai + c);
    n.sd = *reinterpret_cast<const f4 *>(Ai + 3 * H + c);
    n.amin = *reinterpret_cast<const uint32_t *>(args + (size_t)i * 2 * H + c);
    n.amax = *reinterpret_cast<const uint32_t *>(args + (size_t)i * 2 * H + H + c);
    load_rows<FE>(PQ, H, c, src, csr_e, lo, d, n.qr, n.ev);
  }
}

// The aggregation adjoint of node i, features c .. c + 3, given its gradients
// dmu, dmn, dmx, dsd with respect to the mean, min, max and std aggregates:
// dm_k = dmu/d + [k = argmin] dmn + [k = argmax] dmx + dsd (m_k - mean)/(d std)
// for its in-edges k (messages recomputed), written per edge in CSR order,
// with D_in (their sum) and De (their edge-feature-weighted sums) into the
// node's row of D.  Edges past the first kCache are loaded here.
template <int FE>
__device__ __forceinline__ void adj_finish(const AdjIn &n, int i, int c, int H,
                                           const float *__restrict__ PQ,
                                           const int *__restrict__ csr_src,
                                           const float *__restrict__ csr_e, f4 dmu, f4 dmn,
                                           f4 dmx, f4 dsd, float *__restrict__ dm,
                                           float *__restrict__ D, int ldD) {
  const int lo = n.lo, d = n.d;
  f4 din = {0.f, 0.f, 0.f, 0.f};
  f4 de[4] = {din, din, din, din};
  if (d > 0) {
    f4 cache[kCache];
    form_messages<FE>(n.p, n.bm, n.we, n.qr, n.ev, cache);
    const int dc = min(d, kCache);
    const float fd = (float)d;
    const f4 base = dmu / fd;
    const f4 coef = dsd / (fd * n.sd);
    auto emit = [&](const f4 &m, int o, const float *e) {
      f4 g = base + coef * (m - n.mu);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if ((int)((n.amin >> (8 * k)) & 0xff) == o) g[k] += dmn[k];
        if ((int)((n.amax >> (8 * k)) & 0xff) == o) g[k] += dmx[k];
      }
      *reinterpret_cast<f4 *>(dm + (size_t)(lo + o) * H + c) = g;
      din += g;
#pragma unroll
      for (int f = 0; f < FE; ++f) de[f] += g * e[f];
    };
#pragma unroll
    for (int o = 0; o < kCache; ++o)
      if (o < dc) emit(cache[o], o, n.ev[o]);
    for (int o = kCache; o < d; ++o) {
      const int q = lo + o;
      float e[4];
#pragma unroll
      for (int f = 0; f < FE; ++f) e[f] = csr_e[(size_t)q * FE + f];
      emit(message<FE>(PQ, H, csr_src[q], c, n.p, n.bm, n.we, csr_e, q), o, e);
    }
  }
  float *Di = D + (size_t)i * ldD;
  *reinterpret_cast<f4 *>(Di + c) = din;
#pragma unroll
  for (int f = 0; f < FE; ++f) *reinterpret_cast<f4 *>(Di + (2 + f) * H + c) = de[f];
}

// Both halves, for a node whose aggregate gradients are at hand.
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
  const int lo = rowptr[i], d = rowptr[i + 1] - lo;
  int src[kCache];
  if (d > 0) fetch_sources(csr_src, lo, d, src);
  AdjIn n;
  adj_load<FE>(n, i, lo, d, src, c, H, PQ, csr_e, WeT, bmv, A, args);
  adj_finish<FE>(n, i, c, H, PQ, csr_src, csr_e, dmu, dmn, dmx, dsd, dm, D, ldD);
}

} // namespace

} // namespace hgnn
