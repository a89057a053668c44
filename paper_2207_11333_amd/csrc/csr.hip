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

// node -> graph id by binary search over graph_ptr (staged in LDS when it
// fits, so the search costs no dependent global loads); zero the counters;
// check graph_ptr; the first layer's input zero-padded from F to Fp columns.
// Thread t covers node t and the four padded-input columns 4 (t % (Fp/4)) ..
// of row t / (Fp/4), so the grid spreads the copy over many CUs.
constexpr int kInitThreads = 256;
constexpr int kGraphPtrLds = 4096;

__global__ void __launch_bounds__(kInitThreads)
k_csr_init(const Dims *__restrict__ dims, const int *__restrict__ graph_ptr,
           int *__restrict__ node_graph, int *__restrict__ cnt_in, int *__restrict__ cnt_out,
           int *__restrict__ err, const float *__restrict__ x, int F,
           float *__restrict__ xpad, int Fp) {
  __shared__ int s_gp[kGraphPtrLds];
  const int B = dims->B, N = dims->N;
  const int i = blockIdx.x * kInitThreads + threadIdx.x;
  // only workgroups holding nodes search (the condition is uniform per block)
  const bool staged = B + 1 <= kGraphPtrLds && (int)blockIdx.x * kInitThreads < N;
  if (staged)
    for (int k = threadIdx.x; k <= B; k += kInitThreads) s_gp[k] = graph_ptr[k];
  __syncthreads();
  if (i < B) {
    if (graph_ptr[i + 1] <= graph_ptr[i]) atomicOr(err, ERR_GRAPH_PTR);
  }
  if (i == 0) {
    if (graph_ptr[0] != 0 || graph_ptr[B] != N) atomicOr(err, ERR_GRAPH_PTR);
  }
  if (i < N) {
    // last b with graph_ptr[b] <= i (two loops, so that each reads its own
    // address space: LDS reads rather than generic ones)
    int lo = 0, hi = B;
    if (staged) {
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s_gp[mid] <= i) lo = mid; else hi = mid;
      }
    } else {
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (graph_ptr[mid] <= i) lo = mid; else hi = mid;
      }
    }
    node_graph[i] = lo;
    cnt_in[i] = 0;
    cnt_out[i] = 0;
  }
  const int q = Fp >> 2; // 16-byte groups per padded row
  if (x && i < N * q) {
    const int r = i / q, c0 = (i - r * q) * 4;
    const float *xr = x + (size_t)r * F;
    f4 v;
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = c0 + k < F ? xr[c0 + k] : 0.f;
    if (!(isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]) && isfinite(v[3])))
      atomicOr(err, ERR_NONFINITE);
    *reinterpret_cast<f4 *>(xpad + (size_t)r * Fp + c0) = v;
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
// nodes (one per thread) the counter sums and the node count of every degree
// bucket (k_scan_count); one workgroup, a wave per column, turns those into
// block offsets and bucket offsets (k_scan_top); every block then scans its
// own nodes again, adds its offsets and writes rowptr, srcptr, degrees,
// scalers and, with degree buckets, each node's place in the (degree, node
// id) order (k_scan_apply).
constexpr int kScanTop = 1024;
static_assert(kScanNodes == 256, "one node per thread of a 256-thread block");

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

__global__ void __launch_bounds__(kScanNodes)
k_scan_count(const Dims *__restrict__ dims, const int *__restrict__ cnt_in,
             const int *__restrict__ cnt_out, int max_degree, int nb,
             int *__restrict__ scan) {
  __shared__ int s_w[2 + kMaxBuckets][kScanNodes / 64];
  const int N = dims->N;
  const int base = blockIdx.x * kScanNodes;
  if (base >= N) return;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int i = base + tid;
  const int vi = i < N ? cnt_in[i] : 0, vo = i < N ? cnt_out[i] : 0;
  const int bq = i < N ? bucket_of(vi, max_degree) : -1;
  const int si = wave_incl_scan(vi), so = wave_incl_scan(vo);
  if (lane == 63) {
    s_w[0][wid] = si;
    s_w[1][wid] = so;
  }
  for (int q = 0; q < nb; ++q) {
    const unsigned long long m = __ballot(bq == q);
    if (lane == 0) s_w[2 + q][wid] = __popcll(m);
  }
  __syncthreads();
  int *rec = scan + (size_t)blockIdx.x * kScanRec;
  if (tid < 2 + nb) rec[tid] = s_w[tid][0] + s_w[tid][1] + s_w[tid][2] + s_w[tid][3];
}

// One workgroup; wave c scans column c of the block records (c < 2 + nb)
// over the blocks, 64 at a time with a carry.  The column totals give
// rowptr[N], srcptr[N] and the first row of every degree bucket (brow[q] =
// nodes of lower degree), which k_scan_apply adds to the bucket columns.
__global__ void __launch_bounds__(kScanTop)
k_scan_top(const Dims *__restrict__ dims, int nb, int *__restrict__ scan,
           int *__restrict__ brow, int *__restrict__ rowptr, int *__restrict__ srcptr) {
  __shared__ int tot[kScanRec];
  const int N = dims->N;
  const int nblk = (N + kScanNodes - 1) / kScanNodes;
  const int ncol = 2 + nb;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int c = wid; c < ncol; c += kScanTop / 64) {
    int carry = 0;
    for (int b0 = 0; b0 < nblk; b0 += 64) {
      const int k = b0 + lane;
      int *cell = scan + (size_t)k * kScanRec + c;
      const int v = k < nblk ? *cell : 0;
      const int inc = wave_incl_scan(v);
      if (k < nblk) *cell = carry + inc - v;
      carry += __shfl(inc, 63, 64);
    }
    if (lane == 0) tot[c] = carry;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    rowptr[N] = tot[0];
    srcptr[N] = tot[1];
    if (nb) {
      int a = 0;
      for (int q = 0; q < nb; ++q) {
        brow[q] = a;
        a += tot[2 + q];
      }
      brow[nb] = a;
    }
  }
}

// Per block: its own exclusive scans plus the block offsets.  A node's place
// among the nodes of its degree bucket counts the block's earlier nodes of
// that bucket (earlier waves, then earlier lanes of its wave), so the
// permutation is stable in node id.
//
// fused (at most kScanFuse blocks): k_scan_top is not run; each block sums
// the raw block records itself (a wave per column: the records of earlier
// blocks and of all blocks), and block 0 writes rowptr[N], srcptr[N] and the
// bucket bounds.  One dependent launch fewer on the step's critical path.
constexpr int kScanFuse = 256;

__global__ void __launch_bounds__(kScanNodes)
k_scan_apply(const Dims *__restrict__ dims, int *__restrict__ cnt_in,
             int *__restrict__ cnt_out, const int *__restrict__ scan,
             const float *__restrict__ table, int max_degree, int nb,
             int *__restrict__ rowptr, int *__restrict__ srcptr, int *__restrict__ deg,
             float *__restrict__ sp, float *__restrict__ sm, int *__restrict__ perm,
             int *__restrict__ brow, int *__restrict__ err, int fused) {
  __shared__ int s_w[2][kScanNodes / 64];
  __shared__ int s_bw[kScanNodes / 64][kMaxBuckets];
  __shared__ int s_off[kScanRec], s_tot[kScanRec];
  const int N = dims->N;
  const int base = blockIdx.x * kScanNodes;
  if (base >= N) return;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int *rec = scan + (size_t)blockIdx.x * kScanRec;
  if (fused) {
    const int nblk = (N + kScanNodes - 1) / kScanNodes;
    for (int c = wid; c < 2 + nb; c += kScanNodes / 64) {
      int before = 0, total = 0;
      for (int k = lane; k < nblk; k += 64) {
        const int v = scan[(size_t)k * kScanRec + c];
        total += v;
        before += k < (int)blockIdx.x ? v : 0;
      }
      for (int o = 32; o > 0; o >>= 1) {
        before += __shfl_xor(before, o, 64);
        total += __shfl_xor(total, o, 64);
      }
      if (lane == 0) {
        s_off[c] = before;
        s_tot[c] = total;
      }
    }
  }
  const int i = base + tid;
  const int vi = i < N ? cnt_in[i] : 0, vo = i < N ? cnt_out[i] : 0;
  const int bq = i < N ? bucket_of(vi, max_degree) : -1;
  const int ii = wave_incl_scan(vi), io = wave_incl_scan(vo);
  if (lane == 63) {
    s_w[0][wid] = ii;
    s_w[1][wid] = io;
  }
  // rank among the wave's earlier lanes of the same bucket
  const unsigned long long below = (1ull << lane) - 1ull;
  int pos = 0;
  for (int q = 0; q < nb; ++q) {
    const unsigned long long m = __ballot(bq == q);
    if (lane == 0) s_bw[wid][q] = __popcll(m);
    if (bq == q) pos = __popcll(m & below);
  }
  __syncthreads();
  if (fused && blockIdx.x == 0 && tid == 0) {
    rowptr[N] = s_tot[0];
    srcptr[N] = s_tot[1];
    if (nb) {
      int a = 0;
      for (int q = 0; q < nb; ++q) {
        brow[q] = a;
        a += s_tot[2 + q];
      }
      brow[nb] = a;
    }
  }
  if (i >= N) return;
  const int r0 = fused ? s_off[0] : rec[0], r1 = fused ? s_off[1] : rec[1];
  int ei_ = r0 + ii - vi, eo_ = r1 + io - vo;
  for (int w = 0; w < wid; ++w) {
    ei_ += s_w[0][w];
    eo_ += s_w[1][w];
  }
  rowptr[i] = ei_;
  srcptr[i] = eo_;
  deg[i] = vi;
  sp[i] = table[2 * bq];
  sm[i] = table[2 * bq + 1];
  cnt_in[i] = 0;
  cnt_out[i] = 0;
  if (nb) {
    int p = pos;
    if (fused) {
      p += s_off[2 + bq];
      for (int q = 0; q < bq; ++q) p += s_tot[2 + q]; // the bucket's first row
    } else {
      p += brow[bq] + rec[2 + bq];
    }
    for (int w = 0; w < wid; ++w) p += s_bw[w][bq];
    perm[p] = i;
  }
  if (vi > max_degree || vo > max_degree) atomicOr(err, ERR_DEGREE);
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

// Segments of at most kRegSort entries (every molecular graph's) are
// sorted in registers: their entries are loaded at once and put in order by
// a fixed network of compare-exchanges, so a segment costs a few rounds of
// independent loads.  Longer segments take an insertion sort in place.
constexpr int kRegSort = 8;

template <typename K> __device__ __forceinline__ void cswap(K &a, K &b) {
  const K lo = a < b ? a : b, hi = a < b ? b : a;
  a = lo;
  b = hi;
}

// odd-even transposition sort of kRegSort keys (ascending)
template <typename K> __device__ __forceinline__ void sort_regs(K (&v)[kRegSort]) {
#pragma unroll
  for (int pass = 0; pass < kRegSort; ++pass)
#pragma unroll
    for (int a = pass & 1; a + 1 < kRegSort; a += 2) cswap(v[a], v[a + 1]);
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
  const int lo = rowptr[i], hi = rowptr[i + 1], n = hi - lo;
  if (n <= kRegSort) {
    // key = source << 32 | edge id; empty slots sort last
    unsigned long long key[kRegSort];
    int k[kRegSort];
#pragma unroll
    for (int a = 0; a < kRegSort; ++a) k[a] = a < n ? csr_eid[lo + a] : 0;
#pragma unroll
    for (int a = 0; a < kRegSort; ++a)
      key[a] = a < n ? ((unsigned long long)(unsigned)ei[k[a]] << 32) | (unsigned)k[a]
                     : ~0ull;
    sort_regs(key);
    bool finite = true;
#pragma unroll
    for (int a = 0; a < kRegSort; ++a)
      if (a < n) {
        const int ka = (int)(unsigned)(key[a] & 0xffffffffu);
        csr_eid[lo + a] = ka;
        csr_src[lo + a] = (int)(key[a] >> 32);
        csr_dst[lo + a] = i;
        csr_pos[ka] = lo + a;
        for (int f = 0; f < Fe; ++f) {
          const float v = edge_attr[(size_t)ka * Fe + f];
          finite = finite && isfinite(v);
          csr_e[(size_t)(lo + a) * Fe + f] = v;
        }
      }
    if (!finite) atomicOr(err, ERR_NONFINITE);
    return;
  }
  if (n <= max_degree) {
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
  for (int q = lo; q < hi; ++q) {
    const int k = csr_eid[q];
    csr_src[q] = ei[k];
    csr_dst[q] = i;
    csr_pos[k] = q;
  }
  bool finite = true;
  for (int q = lo; q < hi; ++q) {
    const int k = csr_eid[q];
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
  const int lo = srcptr[j], hi = srcptr[j + 1], n = hi - lo;
  if (n <= kRegSort) {
    int k[kRegSort];
    unsigned v[kRegSort];
#pragma unroll
    for (int a = 0; a < kRegSort; ++a) k[a] = a < n ? tmp_out[lo + a] : 0;
#pragma unroll
    for (int a = 0; a < kRegSort; ++a) v[a] = a < n ? (unsigned)csr_pos[k[a]] : ~0u;
    sort_regs(v);
#pragma unroll
    for (int a = 0; a < kRegSort; ++a)
      if (a < n) t2csr[lo + a] = (int)v[a];
    return;
  }
  for (int p = lo; p < hi; ++p) t2csr[p] = csr_pos[tmp_out[p]];
  if (n > max_degree) return;
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
  // Fp is a multiple of 16 (whole 16-byte groups per padded row)
  if (x && Fp % 16) return hipErrorInvalidValue;
  long long nt = capN > capB ? capN : capB;
  if (x && (long long)capN * (Fp / 4) > nt) nt = (long long)capN * (Fp / 4);
  k_csr_init<<<cdiv(nt > 0 ? nt : 1, kInitThreads), kInitThreads, 0, s>>>(
      dims, graph_ptr, c.node_graph, c.cnt_in, c.cnt_out, c.err, x, F, xpad, Fp);
  if (capE > 0)
    k_csr_count<<<cdiv(capE, 256), 256, 0, s>>>(dims, edge_index, c.node_graph,
                                                c.cnt_in, c.cnt_out, c.err);
  {
    const int nsb = cdiv(capN > 0 ? capN : 1, kScanNodes);
    const int fused = nsb <= kScanFuse;
    k_scan_count<<<nsb, 256, 0, s>>>(dims, c.cnt_in, c.cnt_out, max_degree, c.nb, c.scan);
    if (!fused)
      k_scan_top<<<1, kScanTop, 0, s>>>(dims, c.nb, c.scan, c.brow, c.rowptr, c.srcptr);
    k_scan_apply<<<nsb, 256, 0, s>>>(dims, c.cnt_in, c.cnt_out, c.scan, table, max_degree,
                                     c.nb, c.rowptr, c.srcptr, c.deg, c.sp, c.sm, c.perm,
                                     c.brow, c.err, fused);
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
