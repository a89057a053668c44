// Step S0: batch validation and the destination-sorted CSR.
//
// Edges of a batch of molecular graphs (Table 1 layout: edge_index (2, E),
// row 0 source, row 1 destination) are grouped by destination and, within a
// destination, ordered by (source id, edge id).  The by-source transpose
// lists, for every node, the CSR positions of its out-edges in ascending
// order; the aggregation adjoint uses it to sum per-edge gradients by source
// without atomics.  Atomic counters only place edges into their segment; a
// per-segment sort then fixes the order, so every integer output is
// deterministic and independent of the COO edge order.
#include "common.hpp"

namespace hgnn {

namespace {

__global__ void k_set_dims(Dims *d, int B, int N, int E, int *err) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (d) {
      d->B = B;
      d->N = N;
      d->E = E;
      d->pad = 0;
    }
    if (err) *err = 0;
  }
}

// node -> graph id by binary search over graph_ptr; zero the counters;
// check graph_ptr.
__global__ void k_csr_init(const Dims *__restrict__ dims,
                           const int *__restrict__ graph_ptr,
                           int *__restrict__ node_graph, int *__restrict__ cnt_in,
                           int *__restrict__ cnt_out, int *__restrict__ err,
                           const float *__restrict__ x, int F, float *__restrict__ xpad,
                           int Fp) {
  const int B = dims->B, N = dims->N;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < B) {
    if (graph_ptr[i + 1] <= graph_ptr[i]) atomicOr(err, ERR_GRAPH_PTR);
  }
  if (i == 0) {
    if (graph_ptr[0] != 0 || graph_ptr[B] != N) atomicOr(err, ERR_GRAPH_PTR);
  }
  if (i < N) {
    int lo = 0, hi = B; // find last b with graph_ptr[b] <= i
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (graph_ptr[mid] <= i) lo = mid; else hi = mid;
    }
    node_graph[i] = lo;
    cnt_in[i] = 0;
    cnt_out[i] = 0;
    if (x) { // the first layer's input, zero-padded from F to Fp columns
      bool finite = true;
      for (int c = 0; c < Fp; ++c) {
        const float v = c < F ? x[(size_t)i * F + c] : 0.f;
        finite = finite && isfinite(v);
        xpad[(size_t)i * Fp + c] = v;
      }
      if (!finite) atomicOr(err, ERR_NONFINITE);
    }
  }
}

__device__ __forceinline__ bool edge_ok(int s, int d, int N,
                                        const int *__restrict__ node_graph) {
  return s >= 0 && s < N && d >= 0 && d < N && node_graph[s] == node_graph[d];
}

__global__ void k_csr_count(const Dims *__restrict__ dims,
                            const int *__restrict__ ei,
                            const int *__restrict__ node_graph,
                            int *__restrict__ cnt_in, int *__restrict__ cnt_out,
                            int *__restrict__ err) {
  const int N = dims->N, E = dims->E;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= E) return;
  const int s = ei[k], d = ei[E + k];
  if (s < 0 || s >= N || d < 0 || d >= N) {
    atomicOr(err, ERR_EDGE_RANGE);
    return;
  }
  if (node_graph[s] != node_graph[d]) {
    atomicOr(err, ERR_EDGE_CROSS);
    return;
  }
  atomicAdd(&cnt_in[d], 1);
  atomicAdd(&cnt_out[s], 1);
}

// Exclusive scans of both degree counters (rowptr, srcptr) over all nodes in
// three passes, no workgroup waiting on another: per block of kScanNodes
// nodes the counter sums and the node count of every degree bucket
// (k_scan_count); one workgroup turns those into block offsets and bucket
// offsets (k_scan_top); every block then scans its own nodes again, adds its
// offsets and writes rowptr, srcptr, degrees, scalers and, with degree
// buckets, each node's place in the (degree, node id) order (k_scan_apply).
constexpr int kScanTop = 1024;

__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

__device__ __forceinline__ int bucket_of(int d, int max_degree) {
  return d < max_degree ? d : max_degree; // clamped: a bad degree is flagged elsewhere
}

__global__ void __launch_bounds__(256)
k_scan_count(const Dims *__restrict__ dims, const int *__restrict__ cnt_in,
             const int *__restrict__ cnt_out, int max_degree, int nb,
             int *__restrict__ scan) {
  __shared__ int s_b[kMaxBuckets];
  __shared__ int s_w[2][4];
  const int N = dims->N;
  const int base = blockIdx.x * kScanNodes;
  if (base >= N) return;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  if (tid < kMaxBuckets) s_b[tid] = 0;
  __syncthreads();
  int si = 0, so = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int i = base + 4 * tid + j;
    if (i < N) {
      const int vi = cnt_in[i];
      si += vi;
      so += cnt_out[i];
      if (nb) atomicAdd(&s_b[bucket_of(vi, max_degree)], 1); // an order-free count
    }
  }
  si = wave_incl_scan(si);
  so = wave_incl_scan(so);
  if (lane == 63) {
    s_w[0][wid] = si;
    s_w[1][wid] = so;
  }
  __syncthreads();
  int *rec = scan + (size_t)blockIdx.x * kScanRec;
  if (tid == 0) {
    rec[0] = s_w[0][0] + s_w[0][1] + s_w[0][2] + s_w[0][3];
    rec[1] = s_w[1][0] + s_w[1][1] + s_w[1][2] + s_w[1][3];
  }
  if (tid < nb) rec[2 + tid] = s_b[tid];
}

// One workgroup: each column of the block records becomes its exclusive
// prefix over the blocks; the bucket columns then get their bucket's first
// row added (brow[q] = nodes of lower degree).
__global__ void __launch_bounds__(kScanTop)
k_scan_top(const Dims *__restrict__ dims, int nb, int *__restrict__ scan,
           int *__restrict__ brow, int *__restrict__ rowptr, int *__restrict__ srcptr) {
  __shared__ int wsum[kScanTop / 64];
  __shared__ int carry;
  __shared__ int tot[kScanRec];
  __shared__ int s_brow[kMaxBuckets + 1];
  const int N = dims->N;
  const int nblk = (N + kScanNodes - 1) / kScanNodes;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  constexpr int nw = kScanTop / 64;
  for (int c = 0; c < 2 + nb; ++c) {
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int b0 = 0; b0 < nblk; b0 += kScanTop) {
      const int k = b0 + tid;
      const int v = k < nblk ? scan[(size_t)k * kScanRec + c] : 0;
      const int inc = wave_incl_scan(v);
      if (lane == 63) wsum[wid] = inc;
      __syncthreads();
      if (wid == 0) {
        int a = lane < nw ? wsum[lane] : 0;
        a = wave_incl_scan(a);
        if (lane < nw) wsum[lane] = a;
      }
      __syncthreads();
      const int excl = carry + (wid ? wsum[wid - 1] : 0) + inc - v;
      if (k < nblk) scan[(size_t)k * kScanRec + c] = excl;
      __syncthreads();
      if (tid == kScanTop - 1) carry = excl + v;
      __syncthreads();
    }
    if (tid == 0) tot[c] = carry;
    __syncthreads();
  }
  if (tid == 0) {
    rowptr[N] = tot[0];
    srcptr[N] = tot[1];
    int a = 0;
    for (int q = 0; q < nb; ++q) {
      s_brow[q] = a;
      a += tot[2 + q];
    }
    s_brow[nb] = a;
  }
  __syncthreads();
  if (nb == 0) return;
  if (tid <= nb) brow[tid] = s_brow[tid];
  for (int k = tid; k < nblk; k += kScanTop)
    for (int q = 0; q < nb; ++q) scan[(size_t)k * kScanRec + 2 + q] += s_brow[q];
}

// Per block: its own exclusive scans plus the block offsets.  A node's place
// among the nodes of its degree bucket counts the block's earlier nodes of
// that bucket (earlier waves, earlier lanes, then the lane's own earlier
// nodes), so the permutation is stable in node id.
__global__ void __launch_bounds__(256)
k_scan_apply(const Dims *__restrict__ dims, int *__restrict__ cnt_in,
             int *__restrict__ cnt_out, const int *__restrict__ scan,
             const float *__restrict__ table, int max_degree, int nb,
             int *__restrict__ rowptr, int *__restrict__ srcptr, int *__restrict__ deg,
             float *__restrict__ sp, float *__restrict__ sm, int *__restrict__ perm,
             int *__restrict__ err) {
  __shared__ int s_w[2][4];
  __shared__ int s_bw[4][kMaxBuckets];
  const int N = dims->N;
  const int base = blockIdx.x * kScanNodes;
  if (base >= N) return;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int *rec = scan + (size_t)blockIdx.x * kScanRec;
  int vi[4], vo[4], bq[4];
  int si = 0, so = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int i = base + 4 * tid + j;
    vi[j] = i < N ? cnt_in[i] : 0;
    vo[j] = i < N ? cnt_out[i] : 0;
    bq[j] = i < N ? bucket_of(vi[j], max_degree) : -1;
    si += vi[j];
    so += vo[j];
  }
  const int ii = wave_incl_scan(si), io = wave_incl_scan(so);
  if (lane == 63) {
    s_w[0][wid] = ii;
    s_w[1][wid] = io;
  }
  // bucket ranks inside the wave: per bucket, the lane's count and the
  // exclusive sum over lower lanes
  int pos[4] = {0, 0, 0, 0};
  for (int q = 0; q < nb; ++q) {
    int cq = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) cq += bq[j] == q ? 1 : 0;
    const int inc = wave_incl_scan(cq);
    if (lane == 63) s_bw[wid][q] = inc;
    int run = inc - cq;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (bq[j] == q) pos[j] = run++;
  }
  __syncthreads();
  int ei_ = rec[0], eo_ = rec[1];
  for (int w = 0; w < wid; ++w) {
    ei_ += s_w[0][w];
    eo_ += s_w[1][w];
  }
  ei_ += ii - si;
  eo_ += io - so;
  int bad = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int i = base + 4 * tid + j;
    if (i < N) {
      rowptr[i] = ei_;
      srcptr[i] = eo_;
      deg[i] = vi[j];
      const int dc = bucket_of(vi[j], max_degree);
      sp[i] = table[2 * dc];
      sm[i] = table[2 * dc + 1];
      if (vi[j] > max_degree || vo[j] > max_degree) bad = 1;
      cnt_in[i] = 0;
      cnt_out[i] = 0;
      if (nb) {
        const int q = bq[j];
        int p = rec[2 + q] + pos[j];
        for (int w = 0; w < wid; ++w) p += s_bw[w][q];
        perm[p] = i;
      }
    }
    ei_ += vi[j];
    eo_ += vo[j];
  }
  if (bad) atomicOr(err, ERR_DEGREE);
}

__global__ void k_csr_fill(const Dims *__restrict__ dims,
                           const int *__restrict__ ei,
                           const int *__restrict__ node_graph,
                           const int *__restrict__ rowptr,
                           const int *__restrict__ srcptr,
                           int *__restrict__ cnt_in, int *__restrict__ cnt_out,
                           int *__restrict__ csr_eid, int *__restrict__ tmp_out) {
  const int N = dims->N, E = dims->E;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= E) return;
  const int s = ei[k], d = ei[E + k];
  if (!edge_ok(s, d, N, node_graph)) return;
  csr_eid[rowptr[d] + atomicAdd(&cnt_in[d], 1)] = k;
  tmp_out[srcptr[s] + atomicAdd(&cnt_out[s], 1)] = k;
}

// Per destination: order the segment by (source, edge id); write csr_src,
// the inverse map and the edge attributes in CSR order.
__global__ void k_csr_sort_in(const Dims *__restrict__ dims,
                              const int *__restrict__ ei,
                              const int *__restrict__ rowptr,
                              int *__restrict__ csr_eid, int *__restrict__ csr_src,
                              int *__restrict__ csr_dst, int *__restrict__ csr_pos,
                              const float *__restrict__ edge_attr, int Fe,
                              float *__restrict__ csr_e, int max_degree,
                              int *__restrict__ err) {
  const int N = dims->N;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int lo = rowptr[i], hi = rowptr[i + 1];
  if (hi - lo <= max_degree) {
    for (int a = lo + 1; a < hi; ++a) { // insertion sort by (src, eid)
      const int ka = csr_eid[a];
      const int sa = ei[ka];
      int b = a - 1;
      while (b >= lo) {
        const int kb = csr_eid[b];
        const int sb = ei[kb];
        if (sb < sa || (sb == sa && kb < ka)) break;
        csr_eid[b + 1] = kb;
        --b;
      }
      csr_eid[b + 1] = ka;
    }
  }
  bool finite = true;
  for (int q = lo; q < hi; ++q) {
    const int k = csr_eid[q];
    csr_src[q] = ei[k];
    csr_dst[q] = i;
    csr_pos[k] = q;
    for (int f = 0; f < Fe; ++f) {
      const float v = edge_attr[(size_t)k * Fe + f];
      finite = finite && isfinite(v);
      csr_e[(size_t)q * Fe + f] = v;
    }
  }
  if (!finite) atomicOr(err, ERR_NONFINITE);
}

// Per source: CSR positions of its out-edges, ascending.
__global__ void k_csr_sort_out(const Dims *__restrict__ dims,
                               const int *__restrict__ srcptr,
                               const int *__restrict__ tmp_out,
                               const int *__restrict__ csr_pos,
                               int *__restrict__ t2csr, int max_degree) {
  const int N = dims->N;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const int lo = srcptr[j], hi = srcptr[j + 1];
  for (int p = lo; p < hi; ++p) t2csr[p] = csr_pos[tmp_out[p]];
  if (hi - lo > max_degree) return;
  for (int a = lo + 1; a < hi; ++a) {
    const int va = t2csr[a];
    int b = a - 1;
    while (b >= lo && t2csr[b] > va) {
      t2csr[b + 1] = t2csr[b];
      --b;
    }
    t2csr[b + 1] = va;
  }
}

__global__ void k_pad_copy(const Dims *__restrict__ dims, const float *__restrict__ x,
                           int F, float *__restrict__ xp, int Fp) {
  const int N = dims->N;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = (int)(t / Fp), c = (int)(t % Fp);
  if (i >= N) return;
  xp[t] = c < F ? x[(size_t)i * F + c] : 0.0f;
}

inline int cdiv(long long a, int b) { return (int)((a + b - 1) / b); }

} // namespace

hipError_t launch_set_dims(Dims *d, int B, int N, int E, int *err, hipStream_t s) {
  k_set_dims<<<1, 64, 0, s>>>(d, B, N, E, err);
  return hipGetLastError();
}

hipError_t launch_csr_build(const Dims *dims, int capB, int capN, int capE,
                            const int *graph_ptr, const int *edge_index,
                            const float *edge_attr, int Fe, int max_degree,
                            const float *table, const CsrBufs &c, bool clear_err,
                            const float *x, int F, float *xpad, int Fp, hipStream_t s) {
  if (clear_err) k_set_dims<<<1, 64, 0, s>>>(nullptr, 0, 0, 0, c.err);
  const int nb = capN > capB ? capN : capB;
  k_csr_init<<<cdiv(nb > 0 ? nb : 1, 256), 256, 0, s>>>(dims, graph_ptr, c.node_graph,
                                                        c.cnt_in, c.cnt_out, c.err, x, F,
                                                        xpad, Fp);
  if (capE > 0)
    k_csr_count<<<cdiv(capE, 256), 256, 0, s>>>(dims, edge_index, c.node_graph,
                                                c.cnt_in, c.cnt_out, c.err);
  {
    const int nsb = cdiv(capN > 0 ? capN : 1, kScanNodes);
    k_scan_count<<<nsb, 256, 0, s>>>(dims, c.cnt_in, c.cnt_out, max_degree, c.nb, c.scan);
    k_scan_top<<<1, kScanTop, 0, s>>>(dims, c.nb, c.scan, c.brow, c.rowptr, c.srcptr);
    k_scan_apply<<<nsb, 256, 0, s>>>(dims, c.cnt_in, c.cnt_out, c.scan, table, max_degree,
                                     c.nb, c.rowptr, c.srcptr, c.deg, c.sp, c.sm, c.perm,
                                     c.err);
  }
  if (capE > 0)
    k_csr_fill<<<cdiv(capE, 256), 256, 0, s>>>(dims, edge_index, c.node_graph, c.rowptr,
                                               c.srcptr, c.cnt_in, c.cnt_out, c.csr_eid,
                                               c.tmp_out);
  if (capN > 0) {
    k_csr_sort_in<<<cdiv(capN, 128), 128, 0, s>>>(dims, edge_index, c.rowptr, c.csr_eid,
                                                  c.csr_src, c.csr_dst, c.csr_pos, edge_attr, Fe,
                                                  c.csr_e, max_degree, c.err);
    k_csr_sort_out<<<cdiv(capN, 128), 128, 0, s>>>(dims, c.srcptr, c.tmp_out, c.csr_pos,
                                                   c.t2csr, max_degree);
  }
  return hipGetLastError();
}

hipError_t launch_pad_copy(const Dims *dims, int capN, const float *x, int F,
                           float *xp, int Fp, hipStream_t s) {
  if (capN <= 0) return hipSuccess;
  k_pad_copy<<<cdiv((long long)capN * Fp, 256), 256, 0, s>>>(dims, x, F, xp, Fp);
  return hipGetLastError();
}

} // namespace hgnn
