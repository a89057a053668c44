// Steps S4 and S5: global mean pooling over each graph's nodes (Section 3.1),
// the fully connected head Linear(H,H)-ReLU-Linear(H,1), the MSE loss
// (Section 3.2) and their adjoint.  One workgroup per graph; every reduction
// runs in a fixed order, so results are deterministic and a graph's
// prediction does not depend on the other graphs of the batch.
#include "common.hpp"

namespace hgnn {

namespace {

inline int cdiv(long long a, int b) { return (int)((a + b - 1) / b); }
constexpr int kHeadThreads = 256;

// Node range of graph b, clamped to [0, N] so that an unvalidated malformed
// graph_ptr (reported through the error word) never leads out of bounds.
__device__ __forceinline__ void graph_range(const int *gptr, int b, int N, int &lo, int &hi) {
  lo = min(max(gptr[b], 0), N);
  hi = min(max(gptr[b + 1], lo), N);
}

// Fixed-shape tree reduction over the workgroup (deterministic).
__device__ float block_sum(float v, float *red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int s = kHeadThreads / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const float r = red[0];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(kHeadThreads)
k_head_forward(const Dims *__restrict__ dims, int H, const int *__restrict__ gptr,
               const float *__restrict__ h, const float *__restrict__ W1,
               const float *__restrict__ b1, const float *__restrict__ w2,
               const float *__restrict__ b2, float *__restrict__ g,
               float *__restrict__ q, float *__restrict__ pred,
               float *__restrict__ pred2) {
  __shared__ float gs[512];
  __shared__ float red[kHeadThreads];
  const int b = blockIdx.x;
  if (b >= dims->B) return;
  int lo, hi;
  graph_range(gptr, b, dims->N, lo, hi);
  const float inv_n = 1.0f / (float)(hi - lo);
  for (int c = threadIdx.x; c < H; c += kHeadThreads) {
    float s = 0.f;
    for (int i = lo; i < hi; ++i) s += h[(size_t)i * H + c];
    const float gv = s * inv_n;
    gs[c] = gv;
    g[(size_t)b * H + c] = gv;
  }
  __syncthreads();
  float part = 0.f;
  for (int c = threadIdx.x; c < H; c += kHeadThreads) {
    float s = b1[c];
    const float *row = W1 + (size_t)c * H;
    for (int k = 0; k < H; ++k) s += row[k] * gs[k];
    const float qv = s > 0.f ? s : 0.f;
    q[(size_t)b * H + c] = qv;
    part += w2[c] * qv;
  }
  const float y = block_sum(part, red) + b2[0];
  if (threadIdx.x == 0) {
    pred[b] = y;
    if (pred2) pred2[b] = y;
  }
}

__global__ void __launch_bounds__(kHeadThreads)
k_loss(const Dims *__restrict__ dims, const float *__restrict__ pred,
       const float *__restrict__ t, float *__restrict__ loss) {
  __shared__ float red[kHeadThreads];
  const int B = dims->B;
  float s = 0.f;
  for (int b = threadIdx.x; b < B; b += kHeadThreads) {
    const float d = pred[b] - t[b];
    s += d * d;
  }
  const float tot = block_sum(s, red);
  if (threadIdx.x == 0) *loss = tot / (float)B;
}

// Per graph: dy, dq = dy w2 * [q > 0], dg = W1^T dq, dh_i = dg / n_b.
__global__ void __launch_bounds__(kHeadThreads)
k_head_bwd_graph(const Dims *__restrict__ dims, int H, const int *__restrict__ gptr,
                 const float *__restrict__ W1, const float *__restrict__ w2,
                 const float *__restrict__ q, const float *__restrict__ pred,
                 const float *__restrict__ target, const float *__restrict__ dpred,
                 float *__restrict__ dy, float *__restrict__ dq, float *__restrict__ dh,
                 const float *__restrict__ relu_of) {
  __shared__ float dqs[512];
  const int b = blockIdx.x;
  const int B = dims->B;
  if (b >= B) return;
  const float dyb = dpred ? dpred[b] : 2.0f * (pred[b] - target[b]) / (float)B;
  if (threadIdx.x == 0) dy[b] = dyb;
  for (int c = threadIdx.x; c < H; c += kHeadThreads) {
    const float v = q[(size_t)b * H + c] > 0.f ? dyb * w2[c] : 0.f;
    dqs[c] = v;
    dq[(size_t)b * H + c] = v;
  }
  __syncthreads();
  int lo, hi;
  graph_range(gptr, b, dims->N, lo, hi);
  const float inv_n = 1.0f / (float)(hi - lo);
  for (int k = threadIdx.x; k < H; k += kHeadThreads) {
    float s = 0.f;
    for (int c = 0; c < H; ++c) s += W1[(size_t)c * H + k] * dqs[c];
    const float v = s * inv_n;
    if (relu_of) // fold in the ReLU adjoint of the layer that produced h
      for (int i = lo; i < hi; ++i) dh[(size_t)i * H + k] = relu_of[(size_t)i * H + k] > 0.f ? v : 0.f;
    else
      for (int i = lo; i < hi; ++i) dh[(size_t)i * H + k] = v;
  }
}

// Head weight gradients, each a fixed-order sum over the graphs.
// Output layout (packed): dW1 [H, H], db1 [H], dw2 [H], db2 [1].  A
// workgroup owns 32 outputs; its 8 thread groups sum interleaved graphs and
// the 8 partial sums are added in a fixed order.
constexpr int kHeadOut = 32, kHeadParts = 8;

__global__ void __launch_bounds__(256)
k_head_bwd_weights(const Dims *__restrict__ dims, int H, const float *__restrict__ g,
                   const float *__restrict__ q, const float *__restrict__ dy,
                   const float *__restrict__ dq, float *__restrict__ out) {
  __shared__ float red[kHeadParts][kHeadOut];
  const int o = threadIdx.x % kHeadOut, p = threadIdx.x / kHeadOut;
  const int t = blockIdx.x * kHeadOut + o;
  const int B = dims->B;
  const int n1 = H * H, total = n1 + 2 * H + 1;
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

} // namespace

hipError_t launch_head_forward(const Dims *dims, int capB, int H, const int *graph_ptr,
                               const float *h, const float *W1, const float *b1,
                               const float *w2, const float *b2, float *g, float *q,
                               float *pred, float *pred2, hipStream_t s) {
  if (capB <= 0) return hipSuccess;
  k_head_forward<<<capB, kHeadThreads, 0, s>>>(dims, H, graph_ptr, h, W1, b1, w2, b2, g,
                                               q, pred, pred2);
  return hipGetLastError();
}

hipError_t launch_loss(const Dims *dims, const float *pred, const float *t, float *loss,
                       hipStream_t s) {
  k_loss<<<1, kHeadThreads, 0, s>>>(dims, pred, t, loss);
  return hipGetLastError();
}

hipError_t launch_head_backward(const Dims *dims, int capB, int H, const int *graph_ptr,
                                const float *W1, const float *w2, const float *g,
                                const float *q, const float *pred, const float *target,
                                const float *dpred, float *dy, float *dq, float *dh,
                                float *dw_head, const float *relu_of, hipStream_t s) {
  if (capB <= 0) return hipSuccess;
  k_head_bwd_graph<<<capB, kHeadThreads, 0, s>>>(dims, H, graph_ptr, W1, w2, q, pred,
                                                 target, dpred, dy, dq, dh, relu_of);
  const int n = H * H + 2 * H + 1;
  k_head_bwd_weights<<<cdiv(n, kHeadOut), 256, 0, s>>>(dims, H, g, q, dy, dq, dw_head);
  return hipGetLastError();
}

} // namespace hgnn
