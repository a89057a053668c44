// Internal declarations shared by the HIP translation units of libhgnn.
// Every kernel here is written for gfx950 (CDNA4): 64-wide wavefronts,
// MFMA matrix cores, 160 KB LDS per CU.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

#include <string>

namespace hgnn {

// Device-side sizes of the batch being processed.  Kernels read the live
// sizes from here so that one launch (or one captured HIP graph) serves any
// batch up to the capacity its grid was sized for.
struct Dims {
  int32_t B, N, E, pad;
};

// Error-word bits raised by the CSR builder (device side).
enum : int32_t {
  ERR_EDGE_RANGE = 1,   // edge endpoint outside [0, N)
  ERR_EDGE_CROSS = 2,   // edge joins two graphs
  ERR_DEGREE = 4,       // in- or out-degree above max_degree
  ERR_GRAPH_PTR = 8,    // graph_ptr not 0..N or a graph without nodes
  ERR_NONFINITE = 16,   // a NaN or infinity in x or edge_attr
};

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------------
// GEMM descriptors.  Up to four K segments, each a row-major operand with
// its own leading dimension and an optional per-row scale.  Used for the
// "virtual" operands [h || A || s+ A || s- A] and [du || s+ du || s- du]
// that are never materialised.
// ------------------------------------------------------------------------
constexpr int kMaxSeg = 5;

// Degree buckets of the update linear.  The PNA scalers of a node depend on
// its in-degree d alone, so [A || s+ A || s- A] W^T = A W_eff(d)^T with
// W_eff(d) = W_0 + s+(d) W_+ + s-(d) W_- (one [H, 4H] matrix per degree).
// Nodes are grouped by degree (a stable permutation built with the CSR) and
// every row tile or node chunk of the update GEMMs holds one degree only, so
// the K range of the update linear and of its input gradient shrinks from
// F + 12H to F + 4H and from 3H to H.  Models whose max_degree + 1 exceeds
// kMaxBuckets keep the concatenated form.
constexpr int kMaxBuckets = 16;
// ints per block record of the multi-block CSR scan: the in- and out-degree
// sums and one count per bucket
constexpr int kScanRec = 2 + kMaxBuckets;
constexpr int kScanNodes = 256; // nodes per block of that scan

struct SegA {
  const float *ptr;   // [rows, ld] row-major, k-contiguous
  const float *scale; // per-row scale or nullptr
  int ld;             // leading dimension (floats)
  int k;              // segment length (multiple of 4)
  int boff;           // column offset of this segment inside the B rows
};

// C[m, n] = act( sum_seg sum_k scale_s[m] A_s[m, k] * B[n, boff_s + k] + bias[n] )
// for m < dims->N (or M_fixed when >= 0) and n < Ncols.
struct GemmNT {
  SegA seg[kMaxSeg];
  int nseg;
  const void *B;   // [Ncols, ldb] (float or bf16 per precision), k-contiguous
  const void *B_lo; // BF16 only: low halves of B (hi + lo split) or nullptr
  int ldb;
  int Ncols;
  const float *bias; // [Ncols] or nullptr
  int relu;
  float *C;
  int ldc;
  int M_fixed;       // -1: M = dims->N
  // split-K: with splits > 1 each split writes raw partial sums to
  // P[z][m][n] (splits x capM x Ncols) and a second kernel adds them in
  // order z = 0..splits-1 and applies bias and ReLU.
  int splits;
  float *P;
  int max_splits;    // > 0: cap on the split count chosen by the launcher
  // optional: zero C[m, n] where mask[m * ldc + n] <= 0 (ReLU adjoint of the
  // layer that produced `mask`)
  const float *mask;
  // optional: added to the product before bias/ReLU: C = act(A B^T + bias + addend)
  const float *addend;
  int ld_add;
  // 3: the last three segments read the same rows (equal k, differing only
  // in scale and boff) and their K tiles are taken interleaved -- tile j of
  // each in turn -- so a workgroup rereads a tile while it is still cached
  // instead of streaming the operand once per segment.  0: in order.
  int ileave_n;
  // Degree-bucketed rows (perm non-null): row tiles are taken per bucket q
  // over the permuted rows [brow[q], brow[q+1]) (brow [nb + 1], device);
  // a row r reads and writes node perm[r]; bucket q multiplies with
  // B + q * bstride (and B_lo + q * bstride).
  const int *perm;
  const int *brow;
  int nb;
  long long bstride;
  // optional: a BF16 copy of C (the stored values rounded, RNE) for the
  // consumers that read it in BF16; the product is then not split
  __bf16 *Cb;
  int ldcb;
};

// LDS-DMA NT form (gemm_ntb.hip): C = act(sum_seg A_seg B_seg^T + bias) with
// every A segment in the product's precision in HBM (FP32 as it lies, BF16 as
// a copy written by its producer) and every segment length a multiple of the
// K tile (32 FP32 or 64 BF16), so that whole K tiles are copied from HBM to
// LDS without passing through registers.  Same products, in the same order,
// as GemmNT's unsplit form on the same values: the outputs are bitwise equal.
// No split-K, row scales, interleave or addend.
struct SegB {
  const void *ptr; // [rows, ld] row-major, k-contiguous, 16-byte aligned rows
  int ld;          // leading dimension (elements; rows 16-byte multiples)
  int k;           // segment length (multiple of the K tile)
  int boff;        // column offset of this segment inside the B rows
};
struct GemmNTB {
  SegB seg[kMaxSeg];
  int nseg;
  const void *B, *B_lo;   // [Ncols, ldb] weights (FP32, or BF16 hi and lo halves)
  int ldb;
  long long bstride;      // per-bucket weight stride (bucketed rows)
  const int *perm, *brow; // degree-bucketed rows as in GemmNT, or nullptr
  int nb;
  int Ncols;
  const float *bias;
  int relu;
  const float *mask; // as in GemmNT
  float *C;
  int ldc;
  __bf16 *Cb; // BF16 only: optional BF16 copy of C (the same values rounded), or nullptr
  int ldcb;
  int M_fixed;
};
bool gemm_ntb_ok(const GemmNTB &g, int precision);
hipError_t launch_gemm_ntb(const Dims *dims, int capM, const GemmNTB &g, int precision,
                           hipStream_t s, int tag, hipEvent_t ev0, hipEvent_t ev1);

// Weight-gradient form, reduction over rows i (nodes):
// P[z][m, n] = sum_{i in chunk z} X[i, m] * Yv[i, n]
// where Yv = [seg0 || seg1 || ...] with per-row (per-i) scales.
struct SegY {
  const float *ptr;   // nullptr: a constant segment [1, 0, 0, 0] (4 columns), which
                      // turns the GEMM's last output column into sum_i X[i, m]
  const float *scale;
  int ld;
  int ncols;  // multiple of 4
};

struct GemmTN {
  const float *X;  // [rows, ldx], column m
  int ldx;
  int M;           // output rows (columns of X), multiple of 16
  SegY seg[kMaxSeg];
  int nseg;
  int Ncols;       // total columns of Yv
  float *P;        // partials [splits (+ nb), M, Ncols]
  int splits;
  // Degree-bucketed chunks (perm non-null): the node chunks are taken per
  // bucket over the permuted rows (as in GemmNT), nb more partials than
  // splits; chunk z writes zscale[2 z] = s+(q), zscale[2 z + 1] = s-(q) of
  // its bucket q from the scaler table (0, 0 for an empty chunk).
  const int *perm;
  const int *brow;
  int nb;
  const float *table;
  float *zscale;
};

// Ordered reduction of the bucketed update weight gradient: P has Z
// partials of [M = H, Ncols = Fp + 4H + 4] (columns: h block, A block, the
// sum column, padding); the A block gives W_0, W_+ and W_- as the plain and
// the s+, s- weighted sums over the chunks.
struct ReduceUpd {
  const float *P;
  const float *zscale; // [Z][2]
  int Z, M, Ncols, F, Fp, H;
  float *dWp;          // [H, F + 12H] packed
  float *dbp;          // [H]
};

// Scatter of reduced partials into the packed gradient vector.  Columns
// [0, main_cols) are the weight columns; the first npad blocks of Fp columns
// hold F real columns each (the rest is skipped), later columns shift down
// by npad (Fp - F); column main_cols is the sum column (from a constant-one
// segment); later columns are padding.  Up to three row ranges
// route rows m in [r0, r1) (local row u = m - r0):
//   weight columns -> main[u * main_ld + main_coloff + cmap(c)] (main may be null)
//   sum column     -> ones[(u % ones_split) * ones_stride + u / ones_split] (or null)
struct ReduceRoute {
  int r0, r1;
  float *main;
  int main_ld, main_coloff;
  float *ones;
  int ones_stride, ones_split;
};
struct ReduceMap {
  const float *P;
  int splits, M, Ncols;
  int main_cols, F, Fp;
  // number of leading Fp-wide column blocks padded from F (0 counts as 1):
  // block b, column w < F maps to b F + w; later columns shift by npad (Fp - F)
  int npad;
  ReduceRoute route[3];
  int nroute;
};

// ------------------------------------------------------------------------
// launchers (each returns hipGetLastError() of its launch)
// ------------------------------------------------------------------------

// csr.hip
struct CsrBufs {
  int *rowptr, *csr_src, *csr_eid, *deg, *srcptr, *t2csr, *node_graph;
  int *csr_dst;       // destination of each CSR position
  int *cnt_in, *cnt_out, *tmp_out, *csr_pos;
  float *csr_e;       // [E, Fe] edge attributes in CSR order
  float *sp, *sm;     // per-node degree scalers
  int *err;           // error word
  // degree buckets (nb > 0): perm [N] nodes in (degree, id) order, brow
  // [nb + 1] bucket offsets into perm; scan [kScanRec per block] scratch of
  // the multi-block scan
  int *perm, *brow, *scan;
  int nb;
};
// sets the batch sizes; also zeroes *err when err is non-null
hipError_t launch_set_dims(Dims *d, int B, int N, int E, int *err, hipStream_t s);
// clear_err: zero the error word first (else the caller has).  x non-null:
// also write the first layer's input zero-padded to Fp columns into xpad.
hipError_t launch_csr_build(const Dims *dims, int capB, int capN, int capE,
                            const int *graph_ptr, const int *edge_index,
                            const float *edge_attr, int Fe, int max_degree,
                            const float *scaler_table, const CsrBufs &c, bool clear_err,
                            const float *x, int F, float *xpad, int Fp, hipStream_t s);
hipError_t launch_pad_copy(const Dims *dims, int capN, const float *x, int F,
                           float *xp, int Fp, hipStream_t s);

// gemm.hip
// Picks the tile shape and the split count from the capacity capM and the
// shape; g.splits/g.P are set here (P must hold nt_partial_floats()).
// tag names the launch site's instantiation (1 update, 2 message, 3
// aggregate-input gradient, 4 layer-input gradient); ev0/ev1 (optional)
// bracket the GEMM kernel alone (not the split-K reduction).
hipError_t launch_gemm_nt(const Dims *dims, int capM, GemmNT g, int precision,
                          float *partials, hipStream_t s, int tag = 0,
                          hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t launch_calib_copy(const float *src, float *dst, long long n, hipStream_t s);

// Split count launch_gemm_nt will use, and the partial buffer it needs.
int nt_splits(int capM, int Ncols, int Ktot, int precision);
size_t nt_partial_floats(int capM, int Ncols, int Ktot, int precision);
// Grid capacity: g.splits chunks, plus g.nb when bucketed.
// tag names the launch site in profiles (1 update, 2 message weight gradient)
hipError_t launch_gemm_tn(const Dims *dims, const GemmTN &g, int precision,
                          hipStream_t s, int tag = 0, hipEvent_t ev0 = nullptr,
                          hipEvent_t ev1 = nullptr);
// reduce.hip
hipError_t launch_reduce_map(const ReduceMap &r, hipStream_t s);
hipError_t launch_reduce_upd(const ReduceUpd &r, hipStream_t s);
// Up to three reductions in one launch (a layer's weight gradients): job k
// is the ReduceUpd u when upd[k], else m[k]; the launcher fills G and grid.
// At most one job is a ReduceUpd.
struct ReduceJobs {
  int njobs;
  bool upd[3];
  ReduceUpd u;
  ReduceMap m[3];
  int G[3], grid[3];
};
hipError_t launch_reduce_jobs(ReduceJobs j, hipStream_t s);
// Column sums of X [dims->N, C] (leading dimension ldx) over Z fixed row
// chunks into P [Z][C][4] (sum in element 0, zeros after): partials in the
// layout of a weight-gradient GEMM's sum column, for launch_reduce_map.
hipError_t launch_colsum(const Dims *dims, const float *X, int ldx, int C, int Z, float *P,
                         hipStream_t s);
hipError_t launch_reduce_nt(const Dims *dims, int capM, const GemmNT &g, hipStream_t s);

// aggregate.hip
hipError_t launch_aggregate(const Dims *dims, int capN, int H, int Fe,
                            const float *PQ, const int *rowptr,
                            const int *csr_src, const float *csr_e,
                            const float *WeT, const float *bm,
                            float *A, uint8_t *args, float eps, hipStream_t s,
                            hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                            __bf16 *Ab = nullptr); // optional BF16 copy of A
hipError_t launch_relu_mask(const Dims *dims, int capN, int H,
                            const float *dh, const float *hout, float *du,
                            hipStream_t s);
// D = [D_in | D_out | De] per node, leading dimension ldD = (2 + Fe) H.
hipError_t launch_aggregate_bwd(const Dims *dims, int capN, int H, int Fe,
                                const float *PQ, const int *rowptr,
                                const int *csr_src, const float *csr_e,
                                const float *WeT, const float *bm,
                                const float *A, const uint8_t *args,
                                const float *dA, float *dm, float *D, int ldD,
                                hipStream_t s, hipEvent_t ev0 = nullptr,
                                hipEvent_t ev1 = nullptr);
// The aggregate-input gradient dA = du W_eff(d) fused into the aggregation
// adjoint (agg_fused.hip), for degree-bucketed models with H a multiple of
// 32: dA is formed per 64-row, 32-feature block in LDS and never stored.
struct AggBwdFused {
  int H, nb;
  const float *du;         // [N, H]
  const void *B, *B_lo;    // per bucket [4H, H] (FP32, or BF16 hi and lo), bstride apart
  long long bstride;
  const int *perm, *brow;  // the (degree, id) row order and its bucket bounds
  const float *PQ;         // [N, 2H] message halves
  const int *rowptr, *csr_src;
  const float *csr_e, *WeT, *bm, *A;
  const uint8_t *args;
  float *dm, *D;           // per-edge dm [E, H]; D rows [N, ldD] (D_in and De written)
  int ldD;
};
bool agg_bwd_fused_ok(int H, int nb);
hipError_t launch_agg_bwd_fused(int capN, const AggBwdFused &a, int precision, int Fe,
                                hipStream_t s, hipEvent_t ev0 = nullptr,
                                hipEvent_t ev1 = nullptr);
hipError_t launch_transpose_sum(const Dims *dims, int capN, int H,
                                const int *srcptr, const int *t2csr,
                                const float *dm, float *D, int ldD, hipStream_t s);
// head.hip
// Graph heads (Tg, packed head after head: W1 [H,H], b1, w2, b2): pooled
// embedding g [B, H], q [Tg][B][H], predictions pred (and pred2 if non-null)
// [B, Tg].
// W1T (nullable): the staged transposes of the heads' W1 (launch_stage_head_t)
hipError_t launch_head_forward(const Dims *dims, int capB, int H, int Tg,
                               const int *graph_ptr, const float *h, const float *wh,
                               const float *W1T, float *g, float *q, float *pred, float *pred2,
                               hipStream_t s);
hipError_t launch_stage_head_t(const float *wh, int H, int Tg, float *W1T, hipStream_t s);
// loss = sum_t gw_t mean_b (pred - t)^2 + sum_s nw_s mean_i (z - zt)^2
// (gw, nw nullable: weight 1).
hipError_t launch_loss(const Dims *dims, int Tg, const float *pred, const float *t,
                       const float *gw, int Tn, const float *z, const float *zt,
                       const float *nw, float *loss, hipStream_t s);
// dw_head receives, per graph head, [dW1 (H*H), db1 (H), dw2 (H), db2 (1)].
// relu_of (nullable): write dh masked by relu_of > 0 (the ReLU adjoint of the
// layer whose output was pooled); add (nullable) [N, H] is added to dh first.
hipError_t launch_head_backward(const Dims *dims, int capB, int H, int Tg,
                                const int *graph_ptr, const float *wh, const float *g,
                                const float *q, const float *pred, const float *target,
                                const float *dpred, const float *gw, float *dy, float *dq,
                                float *dh, float *dw_head, const float *relu_of,
                                const float *add, float *part, hipStream_t s);
// part (nullable): scratch of head_partial_floats(H, Tg) floats; with it,
// batches of 512 graphs or more take the head weight gradients in chunks.
size_t head_partial_floats(int H, int Tg);
// Node heads (Tn): aligned weight copies, outputs, errors and small gradients.
hipError_t launch_stage_node_heads(int H, int Tn, const float *wn, float *W1n, float *W1nT,
                                   hipStream_t s);
hipError_t launch_node_head_out(const Dims *dims, int capN, int H, int Tn, const float *Qn,
                                const float *wn, float *z, float *z2, hipStream_t s);
hipError_t launch_node_head_err(const Dims *dims, int capN, int H, int Tn, const float *Qn,
                                const float *wn, const float *z, const float *zt,
                                const float *nw, float *e, float *dQ, hipStream_t s);
// dw2/db2 of every node head; part holds node_head_small_floats(H, Tn) floats.
size_t node_head_small_floats(int H, int Tn);
hipError_t launch_node_head_small(const Dims *dims, int capN, int H, int Tn, const float *Qn,
                                  const float *e, float *part, float *gwn, hipStream_t s);
// adam.hip
hipError_t launch_adamw(float *theta, const float *g, float *m, float *v, int64_t n,
                        float lr, double b1, double b2, float eps, float wd,
                        const long long *step, hipStream_t s);
// Destinations of the four GEMM-layout weight copies of a layer; lo[] is
// used only for BF16 copies (the low half of a hi + lo split).
struct StageOut {
  void *hi[4];
  void *lo[4];
  float *weT; // [Fe, H] edge-feature columns of W^m, contiguous per feature (FP32)
};
// per-layer staging sources and destinations, kept in device memory
struct StageDesc {
  const float *Wm, *Wp;
  int F, Fp;
  StageOut o;
};
// nb > 0: the update-linear copies are per degree bucket (W_eff from the
// scaler table, see kMaxBuckets), else concatenated.
hipError_t launch_stage_all(const StageDesc *tab, int L, int maxFp, int H, int Fe,
                            int nb, const float *table, int to_bf16, long long *bump,
                            hipStream_t s);
hipError_t launch_stage_layer(const float *Wm, const float *Wp, int F, int Fp,
                              int H, int Fe, int nb, const float *table, const StageOut &o,
                              int to_bf16, hipStream_t s);
hipError_t launch_fill(float *p, int64_t n, float v, hipStream_t s);
// p[off + t] for t < n: bound * U[-1, 1) from SplitMix64(seed) at index off + t
hipError_t launch_init_uniform(float *p, int64_t off, int64_t n, float bound, uint64_t seed,
                               hipStream_t s);

// gc.hip: GraphSAGE and CGCNN layer kinds
constexpr int kMaxFe = 4;
hipError_t launch_sage_mean(const Dims *dims, int capN, int F, const int *rowptr,
                            const int *csr_src, const float *h, int ldh, float *M,
                            hipStream_t s);
// G [N, 2F] = du [W_self | W_nbr]; dh = G_self + neighbour scatter, masked
hipError_t launch_sage_scatter(const Dims *dims, int capN, int F, const int *srcptr,
                               const int *t2csr, const int *csr_dst, const int *rowptr,
                               const float *G, const float *mask, float *dh, hipStream_t s);
hipError_t launch_cg_aggregate(const Dims *dims, int capN, int H, int Fe, const int *rowptr,
                               const int *csr_src, const float *csr_e, const float *PQ,
                               const float *weT, const float *b, const float *h_in,
                               float *h_out, hipStream_t s);
hipError_t launch_cg_aggregate_bwd(const Dims *dims, int capN, int H, int Fe,
                                   const int *rowptr, const int *csr_src, const float *csr_e,
                                   const float *PQ, const float *weT, const float *b,
                                   const float *du, float *dm, float *D, int ldD,
                                   hipStream_t s);
// One block copy of a weight staging: dst[r ld + c] = src[r rs + c cs] inside
// the valid vrows x vcols corner, 0 outside; BF16 hi + lo when bf16.
struct GcStageJob {
  const float *src;
  long long rs, cs;
  int rows, cols, vrows, vcols;
  void *hi, *lo;
  int ld, bf16;
};
hipError_t launch_gc_stage(const GcStageJob *jobs, int njobs, long long max_elems,
                           long long *bump, hipStream_t s);

} // namespace hgnn
