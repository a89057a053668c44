// Steps S4 and S5: global mean pooling over each graph's nodes (Section 3.1),
// the fully connected head Linear(H,H)-ReLU-Linear(H,1), the MSE loss
// (Section 3.2) and their adjoint; generalised to several graph-level heads
// and to node-level heads (HydraGNN's multi-headed outputs) with a weighted
// sum of the heads' losses.  One workgroup per graph; every reduction
// runs in a fixed order, so results are deterministic and a graph's
// prediction does not depend on the other graphs of the batch.
#include "common.hpp"

namespace hgnn {

namespace {

inline int cdiv(long long a, int b) { return (int)((a + b - 1) / b); }
constexpr int kHeadThreads = 256;
// the graph part of the head adjoint: one workgroup per graph, whose time is
// the latency of its dg = W1^T dq sums (split into P = threads / H ordered
// partial ranges) and of its nodes' stores; 512 threads halve the ranges
// (C1 step 184.5k -> 185.9k graphs/s)
constexpr int kHeadBwdThreads = 512;
constexpr int kMaxGraphHeads = 8;

// Node range of graph b, clamped to [0, N] so that an unvalidated malformed
// graph_ptr (reported through the error word) never leads out of bounds.
__device__ __forceinline__ void graph_range(const int *gptr, int b, int N, int &lo, int &hi) {
  lo = min(max(gptr[b], 0), N);
  hi = min(max(gptr[b + 1], lo), N);
}

// Fixed-shape tree reduction over a workgroup of NT threads (deterministic).
template <int NT = kHeadThreads>
__device__ float block_sum(float v, float *red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const float r = red[0];
  __syncthreads();
  return r;
}

// Graph head t of Tg (blockIdx.y): head weights at wh + t (H^2 + 2H + 1) as
// W1 [H, H], b1 [H], w2 [H], b2 [1]; q of head t at q + (t B + b) H; the
// prediction goes to pred[b Tg + t].  W1T (nullable): the staged transposes
// [Tg][H][H] of the W1s, read along the threads' outputs (coalesced); the
// sums run over k in the same order either way.
// 512 threads: thread (p, c) takes feature c and the p-th of P = 512 / H
// ranges of the graph's nodes (pooling) and of k (the W1 product); the P
// partial sums are added in order through LDS.  One thread per feature left
// half of a 256-thread workgroup idle at H = 128 and walked all H rows of W1
// in one chain.
constexpr int kHeadFwdThreads = 512;

__global__ void __launch_bounds__(kHeadFwdThreads)
k_head_forward(const Dims *__restrict__ dims, int H, int Tg, const int *__restrict__ gptr,
               const float *__restrict__ h, const float *__restrict__ wh,
               const float *__restrict__ W1T, float *__restrict__ g, float *__restrict__ q,
               float *__restrict__ pred, float *__restrict__ pred2) {
  __shared__ float gs[512];
  __shared__ float red[kHeadFwdThreads];
  const int b = blockIdx.x, t = blockIdx.y;
  const int B = dims->B;
  if (b >= B) return;
  const float *W1 = wh + (size_t)t * (H * H + 2 * H + 1);
  const float *b1 = W1 + H * H, *w2 = b1 + H, *b2 = w2 + H;
  int lo, hi;
  graph_range(gptr, b, dims->N, lo, hi);
  const float inv_n = 1.0f / (float)(hi - lo);
  const int P = kHeadFwdThreads / H; // H <= 512
  const int tid = threadIdx.x, c = tid % H, p = tid / H;
  const bool act = p < P;
  // pooling: nodes lo + p R .. of this range
  {
    const int R = (hi - lo + P - 1) / P;
    const int i0 = min(lo + p * R, hi), i1 = min(i0 + R, hi);
    float s = 0.f;
    if (act) {
#pragma unroll 8
      for (int i = i0; i < i1; ++i) s += h[(size_t)i * H + c];
    }
    red[tid] = s;
  }
  __syncthreads();
  if (p == 0) {
    float s = red[c];
    for (int k = 1; k < P; ++k) s += red[k * H + c];
    const float gv = s * inv_n;
    gs[c] = gv;
    if (t == 0) g[(size_t)b * H + c] = gv;
  }
  __syncthreads();
  // the W1 product over k = p RK ..
  {
    const int RK = (H + P - 1) / P;
    const int k0 = min(p * RK, H), k1 = min(k0 + RK, H);
    float s = 0.f;
    if (act) {
      if (W1T) {
        const float *W1Tt = W1T + (size_t)t * H * H;
#pragma unroll 8
        for (int k = k0; k < k1; ++k) s += W1Tt[(size_t)k * H + c] * gs[k];
      } else {
        const float *row = W1 + (size_t)c * H;
#pragma unroll 8
        for (int k = k0; k < k1; ++k) s += row[k] * gs[k];
      }
    }
    __syncthreads(); // every read of red above is done
    red[tid] = s;
  }
  __syncthreads();
  float part = 0.f;
  if (p == 0) {
    float s = b1[c];
    for (int k = 0; k < P; ++k) s += red[k * H + c];
    const float qv = s > 0.f ? s : 0.f;
    q[((size_t)t * B + b) * H + c] = qv;
    part = w2[c] * qv;
  }
  __syncthreads();
  const float y = block_sum<kHeadFwdThreads>(part, red) + b2[0];
  if (threadIdx.x == 0) {
    pred[(size_t)b * Tg + t] = y;
    if (pred2) pred2[(size_t)b * Tg + t] = y;
  }
}

// loss = sum_t gw_t mean_b (pred - y)^2 + sum_s nw_s mean_i (z - z_target)^2,
// each mean a fixed-order workgroup sum (weights default to 1).
__global__ void __launch_bounds__(kHeadThreads)
k_loss(const Dims *__restrict__ dims, int Tg, const float *__restrict__ pred,
       const float *__restrict__ t, const float *__restrict__ gw, int Tn,
       const float *__restrict__ z, const float *__restrict__ zt,
       const float *__restrict__ nw, float *__restrict__ loss) {
  __shared__ float red[kHeadThreads];
  const int B = dims->B, N = dims->N;
  float acc = 0.f;
  for (int k = 0; k < Tg; ++k) {
    float s = 0.f;
    for (int b = threadIdx.x; b < B; b += kHeadThreads) {
      const float d = pred[(size_t)b * Tg + k] - t[(size_t)b * Tg + k];
      s += d * d;
    }
    acc += (gw ? gw[k] : 1.0f) * (block_sum(s, red) / (float)B);
  }
  for (int k = 0; k < Tn; ++k) {
    float s = 0.f;
    for (int i = threadIdx.x; i < N; i += kHeadThreads) {
      const float d = z[(size_t)i * Tn + k] - zt[(size_t)i * Tn + k];
      s += d * d;
    }
    acc += (nw ? nw[k] : 1.0f) * (block_sum(s, red) / (float)N);
  }
  if (threadIdx.x == 0) *loss = acc;
}

// Per graph, for every graph head t: dy, dq_t = dy w2_t * [q_t > 0]; then
// dg = sum_t W1_t^T dq_t and dh_i = dg / n_b (+ add_i, the node heads' share),
// masked by relu_of > 0 when given.  The sums over c are split into P
// contiguous ranges (P = 256 / H threads per output when H < 256) whose
// partials are added in range order.
__global__ void __launch_bounds__(kHeadBwdThreads)
k_head_bwd_graph(const Dims *__restrict__ dims, int H, int Tg, const int *__restrict__ gptr,
                 const float *__restrict__ wh, const float *__restrict__ q,
                 const float *__restrict__ pred, const float *__restrict__ target,
                 const float *__restrict__ dpred, const float *__restrict__ gw,
                 float *__restrict__ dy, float *__restrict__ dq, float *__restrict__ dh,
                 const float *__restrict__ relu_of, const float *__restrict__ add) {
  __shared__ float dqs[kMaxGraphHeads * 512];
  __shared__ float red[kHeadBwdThreads];
  __shared__ float dgs[512];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int B = dims->B;
  if (b >= B) return;
  const size_t HS = (size_t)H * H + 2 * H + 1;
  for (int t = 0; t < Tg; ++t) {
    const size_t o = (size_t)b * Tg + t;
    const float dyb = dpred ? dpred[o]
                            : (2.0f * (pred[o] - target[o]) / (float)B) * (gw ? gw[t] : 1.0f);
    if (tid == 0) dy[o] = dyb;
    const float *w2 = wh + t * HS + H * H + H;
    const float *qt = q + ((size_t)t * B + b) * H;
    float *dqt = dq + ((size_t)t * B + b) * H;
    for (int c = tid; c < H; c += kHeadBwdThreads) {
      const float v = qt[c] > 0.f ? dyb * w2[c] : 0.f;
      dqs[t * H + c] = v;
      dqt[c] = v;
    }
  }
  __syncthreads();
  if (H < kHeadBwdThreads) {
    const int P = kHeadBwdThreads / H;
    if (tid < P * H) {
      const int k = tid % H, p = tid / H;
      const int c0 = (p * H) / P, c1 = ((p + 1) * H) / P;
      float s = 0.f;
      for (int t = 0; t < Tg; ++t) {
        const float *W1 = wh + t * HS;
#pragma unroll 8
        for (int c = c0; c < c1; ++c) s += W1[(size_t)c * H + k] * dqs[t * H + c];
      }
      red[tid] = s;
    }
    __syncthreads();
    if (tid < H) {
      float s = red[tid];
      for (int p = 1; p < P; ++p) s += red[p * H + tid];
      dgs[tid] = s;
    }
  } else {
    for (int k = tid; k < H; k += kHeadBwdThreads) {
      float s = 0.f;
      for (int t = 0; t < Tg; ++t) {
        const float *W1 = wh + t * HS;
#pragma unroll 8
        for (int c = 0; c < H; ++c) s += W1[(size_t)c * H + k] * dqs[t * H + c];
      }
      dgs[k] = s;
    }
  }
  __syncthreads();
  int lo, hi;
  graph_range(gptr, b, dims->N, lo, hi);
  const float inv_n = 1.0f / (float)(hi - lo);
  const long long n = (long long)(hi - lo) * H;
  for (long long idx = tid; idx < n; idx += kHeadBwdThreads) {
    const int k = (int)(idx % H);
    const size_t at = (size_t)lo * H + idx;
    float o = dgs[k] * inv_n;
    if (add) o += add[at];
    // fold in the ReLU adjoint of the layer that produced h
    if (relu_of && !(relu_of[at] > 0.f)) o = 0.f;
    dh[at] = o;
  }
}

// Head weight gradients, each a fixed-order sum over the graphs.
// Output layout (packed): dW1 [H, H], db1 [H], dw2 [H], db2 [1].  A
// workgroup owns 32 outputs; its 8 thread groups sum interleaved graphs and
// the 8 partial sums are added in a fixed order.
constexpr int kHeadOut = 32, kHeadParts = 8;

__global__ void __launch_bounds__(256)
k_head_bwd_weights(const Dims *__restrict__ dims, int H, int Tg, const float *__restrict__ g,
                   const float *__restrict__ qall, const float *__restrict__ dyall,
                   const float *__restrict__ dqall, float *__restrict__ outall) {
  __shared__ float red[kHeadParts][kHeadOut];
  const int o = threadIdx.x % kHeadOut, p = threadIdx.x / kHeadOut;
  const int t = blockIdx.x * kHeadOut + o;
  const int B = dims->B;
  const int n1 = H * H, total = n1 + 2 * H + 1;
  // graph head blockIdx.y: its q, dq, dy column and output block
  const int hd = blockIdx.y;
  const float *q = qall + (size_t)hd * B * H, *dq = dqall + (size_t)hd * B * H;
  float *out = outall + (size_t)hd * total;
  struct Col {
    const float *p;
    int s;
    __device__ float operator[](int b) const { return p[(size_t)b * s]; }
  } dy{dyall + hd, Tg};
  float s = 0.f;
  if (t < n1) {
    const int c = t / H, k = t % H;
    for (int b = p; b < B; b += kHeadParts) s += dq[(size_t)b * H + c] * g[(size_t)b * H + k];
  } else if (t < n1 + H) {
    const int c = t - n1;
    for (int b = p; b < B; b += kHeadParts) s += dq[(size_t)b * H + c];
  } else if (t < n1 + 2 * H) {
    const int c = t - n1 - H;
    for (int b = p; b < B; b += kHeadParts) s += dy[b] * q[(size_t)b * H + c];
  } else if (t < total) {
    for (int b = p; b < B; b += kHeadParts) s += dy[b];
  }
  red[p][o] = s;
  __syncthreads();
  if (p == 0 && t < total) {
    float acc = red[0][o];
    for (int j = 1; j < kHeadParts; ++j) acc += red[j][o];
    out[t] = acc;
  }
}

// The same gradients for large batches, in two launches.  The graphs are
// split into Z chunks of R = ceil(B / Z); k_head_w_part writes every
// output's sum over each chunk (P [Tg][Z][n], n = H^2 + 2H + 1) and
// k_head_w_sum adds the chunks in order.  dW1: a workgroup takes a 16 x 64
// block of (c, k) and walks its chunk 64 graphs at a time, the rows of dq
// and g staged in LDS (thread: one c, four k); db1, dw2 and db2 take one more
// workgroup per chunk (thread: one c, the chunk's graphs in order).  The
// one-pass kernel above reads each g and dq value once per output.
constexpr int kHeadChunks = 16, kHeadTC = 16, kHeadTK = 64, kHeadRows = 64;
constexpr int kHeadChunkedMinB = 512;

__global__ void __launch_bounds__(256)
k_head_w_part(const Dims *__restrict__ dims, int H, int Tg, int Z, const float *__restrict__ g,
              const float *__restrict__ qall, const float *__restrict__ dyall,
              const float *__restrict__ dqall, float *__restrict__ Pall) {
  __shared__ float sdq[kHeadRows][kHeadTC];
  __shared__ f4 sg[kHeadRows][kHeadTK / 4];
  const int B = dims->B, n1 = H * H, n = n1 + 2 * H + 1;
  const int hd = blockIdx.z, z = blockIdx.y;
  const float *q = qall + (size_t)hd * B * H, *dq = dqall + (size_t)hd * B * H;
  float *P = Pall + ((size_t)hd * Z + z) * n;
  const int R = (B + Z - 1) / Z, b_lo = min(z * R, B), b_hi = min(b_lo + R, B);
  const int ntk = (H + kHeadTK - 1) / kHeadTK, tiles = (H / kHeadTC) * ntk;
  const int t = threadIdx.x;
  if ((int)blockIdx.x == tiles) { // db1, dw2, db2 over this chunk
    for (int c = t; c < H; c += 256) {
      float s1 = 0.f, s2 = 0.f;
      for (int b = b_lo; b < b_hi; ++b) {
        s1 += dq[(size_t)b * H + c];
        s2 += dyall[(size_t)b * Tg + hd] * q[(size_t)b * H + c];
      }
      P[n1 + c] = s1;
      P[n1 + H + c] = s2;
    }
    if (t == 0) {
      float s3 = 0.f;
      for (int b = b_lo; b < b_hi; ++b) s3 += dyall[(size_t)b * Tg + hd];
      P[n1 + 2 * H] = s3;
    }
    return;
  }
  const int c0 = (blockIdx.x / ntk) * kHeadTC, k0 = (blockIdx.x % ntk) * kHeadTK;
  const int ci = t / (kHeadTK / 4), kq = t % (kHeadTK / 4);
  const int kk = k0 + 4 * kq; // first k of this thread (H is a multiple of 16)
  f4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int r0 = b_lo; r0 < b_hi; r0 += kHeadRows) {
    const int nr = min(kHeadRows, b_hi - r0);
    __syncthreads();
    // stage rows r0 .. r0 + nr - 1: dq[., c0 .. c0 + 15], g[., k0 .. k0 + 63]
    for (int e = t; e < kHeadRows * kHeadTC; e += 256) {
      const int r = e / kHeadTC, cc = e % kHeadTC;
      sdq[r][cc] = r < nr ? dq[(size_t)(r0 + r) * H + c0 + cc] : 0.f;
    }
    for (int e = t; e < kHeadRows * (kHeadTK / 4); e += 256) {
      const int r = e / (kHeadTK / 4), kc = e % (kHeadTK / 4), k = k0 + 4 * kc;
      sg[r][kc] = (r < nr && k < H) ? *reinterpret_cast<const f4 *>(g + (size_t)(r0 + r) * H + k)
                                    : f4{0.f, 0.f, 0.f, 0.f};
    }
    __syncthreads();
    for (int r = 0; r < nr; ++r) acc += sdq[r][ci] * sg[r][kq];
  }
  if (kk < H) *reinterpret_cast<f4 *>(P + (size_t)(c0 + ci) * H + kk) = acc;
}

__global__ void __launch_bounds__(256)
k_head_w_sum(int H, int Z, const float *__restrict__ Pall, float *__restrict__ outall) {
  const int n = H * H + 2 * H + 1, hd = blockIdx.y;
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  const float *P = Pall + (size_t)hd * Z * n + t;
  float s = 0.f;
  for (int z = 0; z < Z; ++z) s += P[(size_t)z * n];
  outall[(size_t)hd * n + t] = s;
}

// ---- node-level heads (Tn of them; head s at wn + s (H^2 + 2H + 1)) ------
// Their hidden layer Q_s = ReLU(h W1_s^T + b1_s) [N, H] comes from the NT
// GEMM (Q_s at Qn + s capN H); these kernels do the rest.

// 16-byte-aligned copies of W1_s for the GEMMs: W1n [Tn][H][H] as stored and
// W1nT [H][Tn H] with W1nT[n][s H + c] = W1_s[c][n].
__global__ void __launch_bounds__(256)
k_stage_node_heads(int H, int Tn, const float *__restrict__ wn, float *__restrict__ W1n,
                   float *__restrict__ W1nT) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long n = (long long)Tn * H * H;
  if (t >= n) return;
  const int sh = (int)(t / ((long long)H * H)), r = (int)((t / H) % H), k = (int)(t % H);
  const float v = wn[(size_t)sh * (H * H + 2 * H + 1) + (size_t)r * H + k];
  W1n[t] = v;
  W1nT[(size_t)k * Tn * H + (size_t)sh * H + r] = v;
}

// z[i, s] = w2_s . Q_s[i] + b2_s (one thread per node and head).
__global__ void __launch_bounds__(256)
k_node_head_out(const Dims *__restrict__ dims, int H, int Tn, size_t capN,
                const float *__restrict__ Qn, const float *__restrict__ wn,
                float *__restrict__ z, float *__restrict__ z2) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int N = dims->N;
  if (t >= (long long)N * Tn) return;
  const int i = (int)(t / Tn), sh = (int)(t % Tn);
  const float *w2 = wn + (size_t)sh * (H * H + 2 * H + 1) + H * H + H;
  const float *q = Qn + (size_t)sh * capN * H + (size_t)i * H;
  float acc = w2[H];
#pragma unroll 8
  for (int c = 0; c < H; ++c) acc += w2[c] * q[c];
  z[t] = acc;
  if (z2) z2[t] = acc;
}

// e[i, s] = 2 nw_s (z - z_target) / N and dQ_s[i, c] = e w2_s[c] [Q_s[i, c] > 0].
__global__ void __launch_bounds__(256)
k_node_head_err(const Dims *__restrict__ dims, int H, int Tn, size_t capN,
                const float *__restrict__ Qn, const float *__restrict__ wn,
                const float *__restrict__ z, const float *__restrict__ zt,
                const float *__restrict__ nw, float *__restrict__ e, float *__restrict__ dQ) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int N = dims->N;
  if (t >= (long long)N * Tn * H) return;
  const int c = (int)(t % H);
  const long long is = t / H;
  const int i = (int)(is / Tn), sh = (int)(is % Tn);
  const float ev = (2.0f * (z[is] - zt[is]) / (float)N) * (nw ? nw[sh] : 1.0f);
  if (c == 0) e[is] = ev;
  const size_t o = (size_t)sh * capN * H + (size_t)i * H + c;
  const float w2 = wn[(size_t)sh * (H * H + 2 * H + 1) + H * H + H + c];
  dQ[o] = Qn[o] > 0.f ? ev * w2 : 0.f;
}

// dw2_s[c] = sum_i e[i, s] Q_s[i, c] and db2_s = sum_i e[i, s] (column c = H),
// in a fixed order: the nodes are cut into kNodeChunks contiguous chunks
// (blockIdx.x), each chunk's sum goes to part[s][chunk][c], and
// k_node_head_small_sum adds the chunks in order.
constexpr int kNodeChunks = 128;

__global__ void __launch_bounds__(256)
k_node_head_small(const Dims *__restrict__ dims, int H, int Tn, size_t capN,
                  const float *__restrict__ Qn, const float *__restrict__ e,
                  float *__restrict__ part) {
  const int r = blockIdx.x, sh = blockIdx.y;
  const int N = dims->N;
  const int rows = (N + kNodeChunks - 1) / kNodeChunks;
  const int i0 = min(r * rows, N), i1 = min(i0 + rows, N);
  const float *Q = Qn + (size_t)sh * capN * H;
  float *out = part + ((size_t)sh * kNodeChunks + r) * (H + 1);
  for (int c = threadIdx.x; c <= H; c += 256) {
    float s = 0.f;
    if (c < H)
      for (int i = i0; i < i1; ++i) s += e[(size_t)i * Tn + sh] * Q[(size_t)i * H + c];
    else
      for (int i = i0; i < i1; ++i) s += e[(size_t)i * Tn + sh];
    out[c] = s;
  }
}

__global__ void __launch_bounds__(256)
k_node_head_small_sum(int H, const float *__restrict__ part, float *__restrict__ gwn) {
  const int sh = blockIdx.x;
  const float *p = part + (size_t)sh * kNodeChunks * (H + 1);
  float *dw2 = gwn + (size_t)sh * (H * H + 2 * H + 1) + H * H + H;
  for (int c = threadIdx.x; c <= H; c += 256) {
    float s = 0.f;
    for (int r = 0; r < kNodeChunks; ++r) s += p[(size_t)r * (H + 1) + c];
    dw2[c] = s;
  }
}

} // namespace

hipError_t launch_stage_node_heads(int H, int Tn, const float *wn, float *W1n, float *W1nT,
                                   hipStream_t s) {
  const long long n = (long long)Tn * H * H;
  if (n <= 0) return hipSuccess;
  k_stage_node_heads<<<cdiv(n, 256), 256, 0, s>>>(H, Tn, wn, W1n, W1nT);
  return hipGetLastError();
}

hipError_t launch_node_head_out(const Dims *dims, int capN, int H, int Tn, const float *Qn,
                                const float *wn, float *z, float *z2, hipStream_t s) {
  if (capN <= 0 || Tn <= 0) return hipSuccess;
  k_node_head_out<<<cdiv((long long)capN * Tn, 256), 256, 0, s>>>(dims, H, Tn, (size_t)capN,
                                                                  Qn, wn, z, z2);
  return hipGetLastError();
}

hipError_t launch_node_head_err(const Dims *dims, int capN, int H, int Tn, const float *Qn,
                                const float *wn, const float *z, const float *zt,
                                const float *nw, float *e, float *dQ, hipStream_t s) {
  if (capN <= 0 || Tn <= 0) return hipSuccess;
  k_node_head_err<<<cdiv((long long)capN * Tn * H, 256), 256, 0, s>>>(
      dims, H, Tn, (size_t)capN, Qn, wn, z, zt, nw, e, dQ);
  return hipGetLastError();
}

size_t node_head_small_floats(int H, int Tn) { return (size_t)Tn * kNodeChunks * (H + 1); }

hipError_t launch_node_head_small(const Dims *dims, int capN, int H, int Tn, const float *Qn,
                                  const float *e, float *part, float *gwn, hipStream_t s) {
  if (Tn <= 0) return hipSuccess;
  k_node_head_small<<<dim3(kNodeChunks, Tn), 256, 0, s>>>(dims, H, Tn, (size_t)capN, Qn, e,
                                                          part);
  k_node_head_small_sum<<<Tn, 256, 0, s>>>(H, part, gwn);
  return hipGetLastError();
}

hipError_t launch_head_forward(const Dims *dims, int capB, int H, int Tg, const int *graph_ptr,
                               const float *h, const float *wh, const float *W1T, float *g,
                               float *q, float *pred, float *pred2, hipStream_t s) {
  if (capB <= 0) return hipSuccess;
  if (Tg < 1 || Tg > kMaxGraphHeads || H < 1 || H > 512) return hipErrorInvalidValue;
  k_head_forward<<<dim3(capB, Tg), kHeadFwdThreads, 0, s>>>(dims, H, Tg, graph_ptr, h, wh, W1T,
                                                             g, q, pred, pred2);
  return hipGetLastError();
}

// W1T[t][k][c] = W1_t[c][k] for the Tg graph heads, through 32 x 32 LDS tiles.
__global__ void __launch_bounds__(256)
k_stage_head_t(const float *__restrict__ wh, int H, float *__restrict__ W1T) {
  __shared__ float tl[32][33];
  const int t = blockIdx.z;
  const float *W1 = wh + (size_t)t * (H * H + 2 * H + 1);
  float *out = W1T + (size_t)t * H * H;
  const int c0 = blockIdx.y * 32, k0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int c = c0 + r, k = k0 + tx;
    tl[r][tx] = (c < H && k < H) ? W1[(size_t)c * H + k] : 0.f;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int k = k0 + r, c = c0 + tx;
    if (k < H && c < H) out[(size_t)k * H + c] = tl[tx][r];
  }
}

hipError_t launch_stage_head_t(const float *wh, int H, int Tg, float *W1T, hipStream_t s) {
  const dim3 grid(cdiv(H, 32), cdiv(H, 32), Tg);
  k_stage_head_t<<<grid, 256, 0, s>>>(wh, H, W1T);
  return hipGetLastError();
}

hipError_t launch_loss(const Dims *dims, int Tg, const float *pred, const float *t,
                       const float *gw, int Tn, const float *z, const float *zt,
                       const float *nw, float *loss, hipStream_t s) {
  k_loss<<<1, kHeadThreads, 0, s>>>(dims, Tg, pred, t, gw, Tn, z, zt, nw, loss);
  return hipGetLastError();
}

hipError_t launch_head_backward(const Dims *dims, int capB, int H, int Tg, const int *graph_ptr,
                                const float *wh, const float *g, const float *q,
                                const float *pred, const float *target, const float *dpred,
                                const float *gw, float *dy, float *dq, float *dh,
                                float *dw_head, const float *relu_of, const float *add,
                                float *part, hipStream_t s) {
  if (capB <= 0) return hipSuccess;
  if (Tg < 1 || Tg > kMaxGraphHeads || H > 512) return hipErrorInvalidValue;
  k_head_bwd_graph<<<capB, kHeadBwdThreads, 0, s>>>(dims, H, Tg, graph_ptr, wh, q, pred, target,
                                                 dpred, gw, dy, dq, dh, relu_of, add);
  const int n = H * H + 2 * H + 1;
  if (part && capB >= kHeadChunkedMinB && H % 16 == 0) {
    const int Z = std::min(kHeadChunks, cdiv(capB, kHeadRows));
    const int tiles = (H / kHeadTC) * cdiv(H, kHeadTK);
    k_head_w_part<<<dim3(tiles + 1, Z, Tg), 256, 0, s>>>(dims, H, Tg, Z, g, q, dy, dq, part);
    k_head_w_sum<<<dim3(cdiv(n, 256), Tg), 256, 0, s>>>(H, Z, part, dw_head);
  } else {
    k_head_bwd_weights<<<dim3(cdiv(n, kHeadOut), Tg), 256, 0, s>>>(dims, H, Tg, g, q, dy, dq,
                                                                   dw_head);
  }
  return hipGetLastError();
}

size_t head_partial_floats(int H, int Tg) {
  return (size_t)Tg * kHeadChunks * ((size_t)H * H + 2 * H + 1);
}

} // namespace hgnn
