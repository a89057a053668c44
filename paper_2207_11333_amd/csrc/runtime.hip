// Context, buffer management and the training-path C-ABI (hgnn.h).
//
// One pass of the hot path per batch: S0 CSR build, then per layer S1
// message linear (one GEMM producing P = h W_dst^T and Q = h W_src^T), S2
// segmented aggregation and S3 update linear + ReLU, then S4 pooling + head
// + loss; the backward pass runs S5 head adjoint and per layer (last first)
// S6 update adjoint, S7 aggregation adjoint and S8 message adjoint; S9 is
// the AdamW step.  Everything runs asynchronously on the caller's stream.
#include "runtime.hpp"

#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

using namespace hgnn;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

inline int ru(int a, int b) { return (a + b - 1) / b * b; }

} // namespace

namespace hgnn {

int set_error(int code, const std::string &msg) { return fail(code, msg); }

int hip_fail(hgnn_ctx *c, hipError_t e, const char *what) {
  if (c) c->sticky = 1;
  return fail(HGNN_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Test-only failure injection (hgnn_debug_fail_after): the n-th layer call
// from now reports a launch failure instead of launching, which puts the
// context into HGNN_ESTATE exactly as a real device failure would.
static int injected_failure(hgnn_ctx *c) {
  if (c->fail_after > 0 && --c->fail_after == 0)
    return hip_fail(c, hipErrorLaunchFailure, "injected failure (hgnn_debug_fail_after)");
  return 0;
}

static void dfree(void *&p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

template <typename T> static hipError_t dalloc(T *&p, size_t count) {
  void *q = nullptr;
  const size_t bytes = count * sizeof(T) < 256 ? 256 : count * sizeof(T);
  hipError_t e = hipMalloc(&q, bytes);
  p = reinterpret_cast<T *>(q);
  return e;
}

// Batches of at least this many nodes take the De rows of the message
// weight gradient apart (two more launches save a third of its products;
// measured: a gain at 40k nodes, a loss at 4.5k, where the launches lie on
// the critical path of the backward pass).
constexpr int kSplitDeRows = 16384;
// Row chunks of the De column sums (at 40k rows: about 320 rows per chunk;
// the sums then cost about as much as reading De once)
constexpr int kColsumChunks = 128;

// Split count of a weight-gradient GEMM (GEMM and ordered reduction timed
// together at 4.5k and 40k nodes).  FP32 (64 x 64 tiles): about 512
// workgroups (the update and message weight gradients at 4.5k nodes: 26
// and 19 us, against 28 and 21 us at 1024).  BF16 (128 x 128 tiles,
// gemm_tn.hip): about 384 workgroups, at most 24 splits (swept again after
// the loads were kept in flight: the update weight gradient at 4.5k nodes
// 17.4 us at 24 splits, 19.5 us at 32; the message weight gradient equal).
int tn_splits(int M, int Ncols, int precision) {
  const int T = precision ? 128 : 64;
  const int tiles = ((M + T - 1) / T) * ((Ncols + T - 1) / T);
  const int target = precision ? 384 : 512;
  int s = (target + tiles - 1) / tiles;
  if (s < 1) s = 1;
  if (s > (precision ? 24 : 64)) s = precision ? 24 : 64;
  return s;
}

void free_work(Exec &ex) {
  Work &w = ex.w;
  void **ptrs[] = {(void **)&w.csr.rowptr, (void **)&w.csr.csr_src, (void **)&w.csr.csr_eid,
                   (void **)&w.csr.deg, (void **)&w.csr.srcptr, (void **)&w.csr.t2csr,
                   (void **)&w.csr.node_graph, (void **)&w.csr.cnt_in,
                   (void **)&w.csr.cnt_out, (void **)&w.csr.tmp_out,
                   (void **)&w.csr.csr_pos, (void **)&w.csr.csr_e, (void **)&w.csr.sp,
                   (void **)&w.csr.sm, (void **)&w.xpad, (void **)&w.g, (void **)&w.q,
                   (void **)&w.ypred, (void **)&w.dy, (void **)&w.dq, (void **)&w.du,
                   (void **)&w.dA, (void **)&w.dm, (void **)&w.D, (void **)&w.D2, (void **)&w.dh0,
                   (void **)&w.dh1, (void **)&w.ntpart, (void **)&w.zn, (void **)&w.Qn,
                   (void **)&w.dQn, (void **)&w.en, (void **)&w.dhn,
                   (void **)&w.csr.csr_dst, (void **)&w.csr.perm, (void **)&w.csr.brow,
                   (void **)&w.csr.scan, (void **)&w.h0, (void **)&w.gcG,
                   (void **)&w.gcD, (void **)&w.gcdm, (void **)&w.gcD1};
  for (void **p : ptrs) dfree(*p);
  for (auto &p : w.gcA) dfree(reinterpret_cast<void *&>(p));
  w.gcA.clear();
  for (auto &p : w.hbuf) dfree(reinterpret_cast<void *&>(p));
  for (auto &p : w.hbuf_b) dfree(reinterpret_cast<void *&>(p));
  w.hbuf_b.clear();
  dfree(reinterpret_cast<void *&>(w.Ab));
  for (auto &p : w.PQ) dfree(reinterpret_cast<void *&>(p));
  for (auto &p : w.A) dfree(reinterpret_cast<void *&>(p));
  for (auto &p : w.args) dfree(reinterpret_cast<void *&>(p));
  w.hbuf.clear();
  w.PQ.clear();
  w.A.clear();
  w.args.clear();
  w.capB = w.capN = w.capE = 0;
}

// The BF16 linears of layers 1.. read BF16 copies of their inputs, written by
// the producers (update linear, aggregation), so that whole K tiles go from
// HBM to LDS untouched (gemm_ntb.hip): BF16 PNA models with degree buckets
// and a hidden width that whole 64-deep K tiles cover.
static bool bf16_copies(const hgnn_ctx *c) {
  return c->kind == HGNN_GC_PNA && c->prec == 1 && c->nb > 0 && c->H % 64 == 0;
}

// Every capacity-sized buffer of an Exec, with its element count: the one
// table used both to allocate and to price a batch for HBM admission.
template <typename F>
static bool for_each_buffer(const hgnn_ctx *c, Work &w, int capB, int capN, int capE,
                            bool inference, F &&f) {
  const int H = c->H, L = c->L, Fe = c->Fe > 0 ? c->Fe : 1;
  const int nstore = (c->recompute || inference) ? 1 : L;
  const int nh = inference ? 2 : L;
  bool ok = true;
  ok = ok && f(w.csr.rowptr, (size_t)capN + 1) && f(w.csr.srcptr, (size_t)capN + 1);
  ok = ok && f(w.csr.csr_src, (size_t)capE) && f(w.csr.csr_eid, (size_t)capE) &&
       f(w.csr.t2csr, (size_t)capE) && f(w.csr.tmp_out, (size_t)capE) &&
       f(w.csr.csr_pos, (size_t)capE) && f(w.csr.csr_dst, (size_t)capE);
  ok = ok && f(w.csr.deg, (size_t)capN) && f(w.csr.node_graph, (size_t)capN) &&
       f(w.csr.cnt_in, (size_t)capN) && f(w.csr.cnt_out, (size_t)capN);
  ok = ok && f(w.csr.csr_e, (size_t)capE * Fe) && f(w.csr.sp, (size_t)capN) &&
       f(w.csr.sm, (size_t)capN) && f(w.xpad, (size_t)capN * c->F0p);
  // degree buckets of the update linear (PNA models) and the scan records
  w.csr.nb = c->kind == HGNN_GC_PNA ? c->nb : 0;
  ok = ok && f(w.csr.scan, (size_t)((capN + kScanNodes - 1) / kScanNodes) * kScanRec);
  if (w.csr.nb) ok = ok && f(w.csr.perm, (size_t)capN) && f(w.csr.brow, (size_t)kMaxBuckets + 1);
  if (w.hbuf.size() != (size_t)nh) w.hbuf.assign(nh, nullptr);
  for (int l = 0; l < nh && ok; ++l) ok = f(w.hbuf[l], (size_t)capN * H);
  const bool shadows = !inference && bf16_copies(c);
  if (w.hbuf_b.size() != (size_t)(shadows ? nh : 0)) w.hbuf_b.assign(shadows ? nh : 0, nullptr);
  for (int l = 0; l < (int)w.hbuf_b.size() && ok; ++l) ok = f(w.hbuf_b[l], (size_t)capN * H);
  if (shadows) ok = ok && f(w.Ab, (size_t)capN * 4 * H);
  const bool pna = c->kind == HGNN_GC_PNA;
  if (pna) {
    if (w.PQ.size() != (size_t)nstore) {
      w.PQ.assign(nstore, nullptr);
      w.A.assign(nstore, nullptr);
      w.args.assign(nstore, nullptr);
    }
    // the arg decisions are read only by the backward pass
    for (int l = 0; l < nstore && ok; ++l)
      ok = f(w.PQ[l], (size_t)capN * 2 * H) && f(w.A[l], (size_t)capN * 4 * H) &&
           (inference || f(w.args[l], (size_t)capN * 2 * H));
  } else {
    if (w.gcA.size() != (size_t)L) w.gcA.assign(L, nullptr);
    for (int l = 0; l < L && ok; ++l) {
      const size_t width = c->kind == HGNN_GC_SAGE ? (size_t)c->ld[l].Fp : 4 * (size_t)H;
      ok = f(w.gcA[l], (size_t)capN * width);
    }
    if (c->kind == HGNN_GC_CGCNN) ok = ok && f(w.h0, (size_t)capN * H);
  }
  const int Tg = c->Tg, Tn = c->Tn;
  ok = ok && f(w.g, (size_t)capB * H) && f(w.q, (size_t)Tg * capB * H) &&
       f(w.ypred, (size_t)capB * Tg);
  if (Tn > 0) ok = ok && f(w.zn, (size_t)capN * Tn) && f(w.Qn, (size_t)Tn * capN * H);
  {
    const size_t np = nt_partial_floats(capN, H, 12 * H, c->prec);
    ok = ok && f(w.ntpart, np);
  }
  if (!inference) {
    ok = ok && f(w.dq, (size_t)Tg * capB * H) && f(w.dy, (size_t)capB * Tg);
    if (Tn > 0)
      ok = ok && f(w.dQn, (size_t)Tn * capN * H) && f(w.en, (size_t)capN * Tn) &&
           f(w.dhn, (size_t)capN * H);
    ok = ok && f(w.du, (size_t)capN * H) && f(w.dh0, (size_t)capN * H) &&
         f(w.dh1, (size_t)capN * H);
    if (pna) {
      // dA is stored only when the adjoint does not form it itself
      if (!agg_bwd_fused_ok(H, c->nb)) ok = ok && f(w.dA, (size_t)capN * 4 * H);
      ok = ok && f(w.dm, (size_t)capE * H) && f(w.D, (size_t)capN * (2 + c->Fe) * H);
      if (!c->recompute) ok = ok && f(w.D2, (size_t)capN * (2 + c->Fe) * H);
    }
    else if (c->kind == HGNN_GC_SAGE)
      ok = ok && f(w.gcG, (size_t)capN * 2 * H);
    else
      ok = ok && f(w.gcD, (size_t)capN * (4 + 2 * c->Fe) * H) &&
           f(w.gcD1, (size_t)capN * (4 + 2 * c->Fe) * H) && f(w.gcdm, (size_t)capE * 2 * H);
  }
  return ok;
}

size_t work_bytes(const hgnn_ctx *c, int B, int N, int E, bool inference_only) {
  Work tmp;
  size_t bytes = 0;
  for_each_buffer(c, tmp, B, N, E, inference_only, [&](auto &p, size_t n) {
    const size_t b = n * sizeof(*p);
    bytes += (b < 256 ? 256 : (b + 255) / 256 * 256);
    return true;
  });
  return bytes;
}

size_t carve_work(const hgnn_ctx *c, Exec &ex, int B, int N, int E, char *base,
                  size_t bytes) {
  Work &w = ex.w;
  size_t off = 0;
  const bool ok = for_each_buffer(c, w, B, N, E, /*inference=*/true, [&](auto &p, size_t n) {
    const size_t b = n * sizeof(*p);
    const size_t step = b < 256 ? 256 : (b + 255) / 256 * 256;
    if (off + step > bytes) return false;
    p = reinterpret_cast<std::remove_reference_t<decltype(p)>>(base + off);
    off += step;
    return true;
  });
  if (!ok) return 0;
  w.capB = B;
  w.capN = N;
  w.capE = E;
  w.stored_layer = -1;
  return off;
}

int ensure_work(hgnn_ctx *c, Exec &ex, int B, int N, int E) {
  Work &w = ex.w;
  if (B <= w.capB && N <= w.capN && E <= w.capE) return HGNN_OK;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(c, e, "hipDeviceSynchronize");
  const int capB = B > w.capB ? B : w.capB;
  const int capN = N > w.capN ? N : w.capN;
  const int capE = E > w.capE ? E : w.capE;
  free_work(ex);
  const bool ok = for_each_buffer(c, w, capB, capN, capE, ex.inference_only,
                                  [&](auto &p, size_t n) { return dalloc(p, n) == hipSuccess; });
  if (!ok) {
    free_work(ex);
    return fail(HGNN_ENOMEM, "hipMalloc failed for the batch workspace");
  }
  w.capB = capB;
  w.capN = capN;
  w.capE = capE;
  w.stored_layer = -1;
  return HGNN_OK;
}

static StageOut stage_out(hgnn_ctx *c, int l) {
  StageOut o{};
  o.hi[0] = c->Wds[l];
  o.hi[1] = c->Wpp[l];
  o.hi[2] = c->WpTA[l];
  o.hi[3] = c->WhdsT[l];
  if (c->prec) {
    o.lo[0] = c->Wds_lo[l];
    o.lo[1] = c->Wpp_lo[l];
    o.lo[2] = c->WpTA_lo[l];
    o.lo[3] = c->WhdsT_lo[l];
  }
  o.weT = static_cast<float *>(c->WeT[l]);
  return o;
}

int stage_all(hgnn_ctx *c, hipStream_t s) {
  long long *bump_step = c->bump_pending ? c->step_dev : nullptr;
  c->bump_pending = false;
  hipError_t e = launch_stage_head_t(c->params + c->off_head, c->H, c->Tg, c->W1T, s);
  if (e != hipSuccess) return hip_fail(c, e, "stage head weights");
  if (c->kind != HGNN_GC_PNA) {
    e = launch_gc_stage(c->gc_jobs, c->gc_njobs, c->gc_max_elems, bump_step, s);
    if (e != hipSuccess) return hip_fail(c, e, "stage weights");
    c->staged_from_params = true;
    return HGNN_OK;
  }
  int maxFp = 0;
  for (const LayerDesc &d : c->ld) maxFp = std::max(maxFp, d.Fp);
  e = launch_stage_all(c->stage_tab, c->L, maxFp, c->H, c->Fe, c->nb, c->table, c->prec,
                       bump_step, s);
  if (e != hipSuccess) return hip_fail(c, e, "stage weights");
  c->staged_from_params = true;
  return HGNN_OK;
}

static int stage_layer_from(hgnn_ctx *c, int l, const float *wl, hipStream_t s) {
  const LayerDesc &d = c->ld[l];
  hipError_t e = launch_stage_layer(wl + (d.oWm - d.off), wl + (d.oWp - d.off), d.F, d.Fp,
                                    c->H, c->Fe, c->nb, c->table, stage_out(c, l), c->prec, s);
  if (e != hipSuccess) return hip_fail(c, e, "stage layer weights");
  c->staged_from_params = false;
  return HGNN_OK;
}

int check_batch_host(hgnn_ctx *c, const hgnn_batch *b) {
  if (!b) return fail(HGNN_EINVAL, "batch is NULL");
  if (b->num_graphs < 1) return fail(HGNN_EINVAL, "num_graphs must be >= 1");
  if (b->num_nodes < b->num_graphs)
    return fail(HGNN_EINVAL, "num_nodes must be >= num_graphs (no empty graph)");
  if (b->num_edges < 0) return fail(HGNN_EINVAL, "num_edges must be >= 0");
  if (!b->graph_ptr || !b->x) return fail(HGNN_EINVAL, "graph_ptr and x are required");
  if (b->num_edges > 0 && !b->edge_index) return fail(HGNN_EINVAL, "edge_index is NULL");
  if ((c->Fe > 0) != (b->edge_attr != nullptr) && b->num_edges > 0)
    return fail(HGNN_EINVAL, "edge_attr must be given iff edge_feat > 0");
  if ((long long)b->num_nodes * c->F0p >= (1LL << 31) ||
      (long long)b->num_edges * c->H >= (1LL << 40))
    return fail(HGNN_EINVAL, "batch too large");
  return HGNN_OK;
}

std::string decode_err(int bits) {
  std::string m = "malformed batch:";
  if (bits & ERR_GRAPH_PTR) m += " graph_ptr does not run from 0 to num_nodes or a graph is empty;";
  if (bits & ERR_EDGE_RANGE) m += " edge endpoint out of range;";
  if (bits & ERR_EDGE_CROSS) m += " edge crosses graphs;";
  if (bits & ERR_DEGREE) m += " node degree above max_degree;";
  if (bits & ERR_NONFINITE) m += " non-finite value in x or edge_attr;";
  return m;
}

int prepare(hgnn_ctx *c, Exec &ex, const hgnn_batch *b, int flags, hipStream_t s) {
  int rc = check_batch_host(c, b);
  if (rc) return rc;
  rc = ensure_work(c, ex, b->num_graphs, b->num_nodes, b->num_edges);
  if (rc) return rc;
  Work &w = ex.w;
  // the first layer's padded input is written once here, while the CSR is
  // built; the batch's arrays are read at prepare time only
  hipError_t e;
  {
    TimedLaunch tl(c, ex, SITE_CSR, s);
    e = launch_set_dims(ex.dims, b->num_graphs, b->num_nodes, b->num_edges, w.csr.err, s);
    if (e == hipSuccess)
      e = launch_csr_build(ex.dims, b->num_graphs, b->num_nodes, b->num_edges, b->graph_ptr,
                           b->edge_index, b->edge_attr, c->Fe, c->maxd, c->table, w.csr,
                           /*clear_err=*/false, b->x, c->F0, w.xpad, c->F0p, s);
  }
  if (e != hipSuccess) return hip_fail(c, e, "csr build");
  ex.x_padded = true;
  ex.B = b->num_graphs;
  ex.N = b->num_nodes;
  ex.E = b->num_edges;
  ex.graph_ptr = b->graph_ptr;
  ex.xin = b->x;
  ex.target = b->y;
  ex.prepared = true;
  ++ex.generation;
  w.stored_layer = -1;
  if (flags & HGNN_VALIDATE) {
    int bits = 0;
    e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipMemcpy(&bits, w.csr.err, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "validate");
    if (bits) return fail(HGNN_EINVAL, decode_err(bits));
  }
  return HGNN_OK;
}

// Layer l's S2 (aggregation) from its messages' P|Q.
static int aggregate_into(hgnn_ctx *c, Exec &ex, int l, const float *wl, const float *PQ,
                          float *A, uint8_t *args, __bf16 *Ab, hipStream_t s) {
  const LayerDesc &d = c->ld[l];
  Work &w = ex.w;
  const float *bm = wl + (d.obm - d.off);
  hipError_t e;
  {
    TimedLaunch tl(c, ex, SITE_AGGREGATE, s, /*manual=*/true);
    e = launch_aggregate(ex.dims, ex.N, c->H, c->Fe, PQ, w.csr.rowptr, w.csr.csr_src,
                         w.csr.csr_e, static_cast<const float *>(c->WeT[l]), bm, A, args,
                         (float)c->cfg.std_eps, s, tl.start(), tl.stop(), Ab);
  }
  if (e != hipSuccess) return hip_fail(c, e, "aggregate");
  return HGNN_OK;
}

// The BF16 copy of layer l's input when the context holds one: the input is
// the previous layer's output buffer, written together with its copy.
static bool copies_on(const Exec &ex) { return !ex.w.hbuf_b.empty(); }
static const __bf16 *input_copy(const Exec &ex, int l, const float *h_in) {
  const Work &w = ex.w;
  return (copies_on(ex) && l > 0 && (size_t)l <= w.hbuf_b.size() && h_in == w.hbuf[l - 1])
             ? w.hbuf_b[l - 1]
             : nullptr;
}

// Layer l: S1 (P|Q GEMM), S2 (aggregation) into the given buffers.
// hb: BF16 copy of hin (or null); Ab: where to write the BF16 copy of A (or null).
static int message_and_aggregate(hgnn_ctx *c, Exec &ex, int l, const float *wl, const float *hin,
                                 int ldh, float *PQ, float *A, uint8_t *args,
                                 hipStream_t s, const __bf16 *hb = nullptr,
                                 __bf16 *Ab = nullptr) {
  const LayerDesc &d = c->ld[l];
  const int H = c->H;
  Work &w = ex.w;
  // the LDS-DMA form where it applies: FP32 on the input as it lies, BF16 on
  // its copy
  GemmNTB q{};
  q.nseg = 1;
  q.seg[0] = c->prec ? SegB{hb, H, d.Fp, 0} : SegB{hin, ldh, d.Fp, 0};
  q.B = c->Wds[l];
  q.B_lo = c->prec ? c->Wds_lo[l] : nullptr;
  q.ldb = d.Fp;
  q.Ncols = 2 * H;
  q.C = PQ;
  q.ldc = 2 * H;
  q.M_fixed = -1;
  if (q.seg[0].ptr && gemm_ntb_ok(q, c->prec)) {
    hipError_t e;
    {
      TimedLaunch tl(c, ex, SITE_MESSAGE_GEMM, s, /*manual=*/true);
      e = launch_gemm_ntb(ex.dims, ex.N, q, c->prec, s, /*tag=*/2, tl.start(), tl.stop());
    }
    if (e != hipSuccess) return hip_fail(c, e, "message GEMM");
    return aggregate_into(c, ex, l, wl, PQ, A, args, Ab, s);
  }
  GemmNT g{};
  g.nseg = 1;
  g.seg[0] = SegA{hin, nullptr, ldh, d.Fp, 0};
  g.B = c->Wds[l];
  g.B_lo = c->prec ? c->Wds_lo[l] : nullptr;
  g.ldb = d.Fp;
  g.Ncols = 2 * H;
  g.C = PQ;
  g.ldc = 2 * H;
  g.M_fixed = -1;
  hipError_t e;
  {
    TimedLaunch tl(c, ex, SITE_MESSAGE_GEMM, s, /*manual=*/true);
    e = launch_gemm_nt(ex.dims, ex.N, g, c->prec, w.ntpart, s, /*tag=*/2, tl.start(), tl.stop());
  }
  if (e != hipSuccess) return hip_fail(c, e, "message GEMM");
  return aggregate_into(c, ex, l, wl, PQ, A, args, Ab, s);
}

static const float *layer_input(hgnn_ctx *c, Exec &ex, int l, const float *h_in, int *ldh,
                                hipStream_t s, int *rc) {
  *rc = HGNN_OK;
  if (l == 0) {
    if (!(ex.x_padded && h_in == ex.xin)) {
      hipError_t e = launch_pad_copy(ex.dims, ex.N, h_in, c->F0, ex.w.xpad, c->F0p, s);
      if (e != hipSuccess) *rc = hip_fail(c, e, "pad input");
    }
    *ldh = c->F0p;
    return ex.w.xpad;
  }
  *ldh = c->H;
  return h_in;
}

int layer_forward(hgnn_ctx *c, Exec &ex, int l, const float *wl, const float *h_in, float *h_out,
                  hipStream_t s) {
  if (int rc = injected_failure(c)) return rc;
  const LayerDesc &d = c->ld[l];
  const int H = c->H;
  Work &w = ex.w;
  int rc, ldh;
  const float *hin = layer_input(c, ex, l, h_in, &ldh, s, &rc);
  if (rc) return rc;
  const int slot = (c->recompute || ex.inference_only) ? 0 : l;
  // BF16 copies: of this layer's input (layers 1..), of its aggregates (for
  // the update linear) and of its output (for the next layer)
  const __bf16 *hb = input_copy(ex, l, h_in);
  __bf16 *hb_out =
      (copies_on(ex) && (size_t)l < w.hbuf_b.size() && h_out == w.hbuf[l]) ? w.hbuf_b[l] : nullptr;
  rc = message_and_aggregate(c, ex, l, wl, hin, ldh, w.PQ[slot], w.A[slot],
                             ex.inference_only ? nullptr : w.args[slot], s, hb,
                             hb ? w.Ab : nullptr);
  if (rc) return rc;
  w.stored_layer = l;
  float *A = w.A[slot];
  // u = [h || A] [W_h | W_eff(d)]^T per bucket in the LDS-DMA form where it
  // applies: FP32 on the inputs as they lie, BF16 on their copies
  GemmNTB q{};
  if (c->nb) {
    q.nseg = 2;
    if (c->prec) {
      q.seg[0] = SegB{hb, H, d.Fp, 0};
      q.seg[1] = SegB{hb ? w.Ab : nullptr, 4 * H, 4 * H, d.Fp};
    } else {
      q.seg[0] = SegB{hin, ldh, d.Fp, 0};
      q.seg[1] = SegB{A, 4 * H, 4 * H, d.Fp};
    }
    q.B = c->Wpp[l];
    q.B_lo = c->prec ? c->Wpp_lo[l] : nullptr;
    q.ldb = d.Fp + 4 * H;
    q.bstride = (long long)H * q.ldb;
    q.perm = w.csr.perm;
    q.brow = w.csr.brow;
    q.nb = c->nb;
    q.Ncols = H;
    q.bias = wl + (d.obp - d.off);
    q.relu = 1;
    q.C = h_out;
    q.ldc = H;
    q.Cb = hb_out;
    q.ldcb = H;
    q.M_fixed = -1;
  }
  if (c->nb && q.seg[0].ptr && q.seg[1].ptr && gemm_ntb_ok(q, c->prec)) {
    hipError_t e;
    {
      TimedLaunch tl(c, ex, SITE_UPDATE_GEMM, s, /*manual=*/true);
      e = launch_gemm_ntb(ex.dims, ex.N, q, c->prec, s, /*tag=*/1, tl.start(), tl.stop());
    }
    if (e != hipSuccess) return hip_fail(c, e, "update GEMM");
    return HGNN_OK;
  }
  GemmNT g{};
  g.Cb = hb_out;
  g.ldcb = H;
  if (c->nb) {
    // degree buckets: u = [h || A] [W_h | W_eff(d)]^T per bucket of rows
    g.nseg = 2;
    g.seg[0] = SegA{hin, nullptr, ldh, d.Fp, 0};
    g.seg[1] = SegA{A, nullptr, 4 * H, 4 * H, d.Fp};
    g.ldb = d.Fp + 4 * H;
    g.perm = w.csr.perm;
    g.brow = w.csr.brow;
    g.nb = c->nb;
    g.bstride = (long long)H * g.ldb;
  } else {
    g.nseg = 4;
    g.seg[0] = SegA{hin, nullptr, ldh, d.Fp, 0};
    g.seg[1] = SegA{A, nullptr, 4 * H, 4 * H, d.Fp};
    g.seg[2] = SegA{A, w.csr.sp, 4 * H, 4 * H, d.Fp + 4 * H};
    g.seg[3] = SegA{A, w.csr.sm, 4 * H, 4 * H, d.Fp + 8 * H};
    g.ileave_n = 3;
    g.ldb = d.Fp + 12 * H;
  }
  g.B = c->Wpp[l];
  g.B_lo = c->prec ? c->Wpp_lo[l] : nullptr;
  g.Ncols = H;
  g.bias = wl + (d.obp - d.off);
  g.relu = 1;
  g.C = h_out;
  g.ldc = H;
  g.M_fixed = -1;
  hipError_t e;
  {
    TimedLaunch tl(c, ex, SITE_UPDATE_GEMM, s, /*manual=*/true);
    hipEvent_t e0 = tl.start(), e1 = tl.stop();
    e = launch_gemm_nt(ex.dims, ex.N, g, c->prec, w.ntpart, s, /*tag=*/1, e0, e1);
  }
  if (e != hipSuccess) return hip_fail(c, e, "update GEMM");
  return HGNN_OK;
}

// dh_out_masked: dh_out already carries this layer's ReLU adjoint (it is du).
// mask_dh_in: fold the previous layer's ReLU adjoint (h_in > 0) into dh_in.
// defer_join: leave the main stream's wait for this layer's weight-gradient
// work to the later layer_backward calls, which take it just before the
// first launch that overwrites a buffer it reads: the next layer's input
// gradient GEMM (this layer's du) and, with the second D buffer, the
// aggregation adjoint two layers on (with one D buffer, the next one's).
// Not with recomputation, which rewrites the stored A and PQ at the start of
// the next layer.
int layer_backward(hgnn_ctx *c, Exec &ex, int l, const float *wl, const float *h_in,
                   const float *h_out, const float *dh_out, float *dh_in, float *dwl,
                   hipStream_t s, bool dh_out_masked = false, bool mask_dh_in = false,
                   bool defer_join = false) {
  if (int rc = injected_failure(c)) return rc;
  const LayerDesc &d = c->ld[l];
  const int H = c->H, Fe = c->Fe, ldD = (2 + Fe) * H;
  Work &w = ex.w;
  int rc, ldh;
  const float *hin = layer_input(c, ex, l, h_in, &ldh, s, &rc);
  if (rc) return rc;
  const int slot = c->recompute ? 0 : l;
  if (c->recompute && w.stored_layer != l) { // S10: re-run S1/S2 for this layer
    rc = message_and_aggregate(c, ex, l, wl, hin, ldh, w.PQ[0], w.A[0], w.args[0], s,
                               input_copy(ex, l, h_in));
    if (rc) return rc;
    w.stored_layer = l;
  }
  float *PQ = w.PQ[slot], *A = w.A[slot];
  const uint8_t *args = w.args[slot];
  // D of this layer: odd layers use the second buffer when it exists (no
  // recomputation), so that writing it need not wait for the previous
  // layer's weight gradients, which read the other one
  float *Dl = (l & 1) && w.D2 ? w.D2 : w.D;
  const float *bm = wl + (d.obm - d.off);
  float *dWm = dwl + (d.oWm - d.off), *dbm = dwl + (d.obm - d.off);
  float *dWp = dwl + (d.oWp - d.off), *dbp = dwl + (d.obp - d.off);
  hipError_t e = hipSuccess;
  const float *du = dh_out;
  if (!dh_out_masked) {
    e = launch_relu_mask(ex.dims, ex.N, H, dh_out, h_out, w.du, s);
    if (e != hipSuccess) return hip_fail(c, e, "relu mask");
    du = w.du;
  }
  // fork: the weight gradients run on the aux stream
  hipStream_t a = c->aux;
  e = hipEventRecord(c->fork_ev[0], s);
  if (e == hipSuccess) e = hipStreamWaitEvent(a, c->fork_ev[0], 0);
  if (e != hipSuccess) return hip_fail(c, e, "fork");
  // S6: dW^p = du^T [h || A || s+ A || s- A]; with degree buckets
  // du^T [h || A] per bucket-pure chunk, the scalers applied by the
  // reduction.  Its partial sums stay in part_u until the message weight
  // gradient's are in part too: one launch reduces both.
  ReduceJobs red{};
  if (c->nb) {
    GemmTN t{};
    t.X = du;
    t.ldx = H;
    t.M = H;
    t.seg[0] = SegY{hin, nullptr, ldh, d.Fp};
    t.seg[1] = SegY{A, nullptr, 4 * H, 4 * H};
    t.seg[2] = SegY{nullptr, nullptr, 0, 4}; // sum column: db^p
    t.nseg = 3;
    t.Ncols = d.Fp + 4 * H + 4;
    t.P = c->part_u;
    t.splits = d.split_p;
    t.perm = w.csr.perm;
    t.brow = w.csr.brow;
    t.nb = c->nb;
    t.table = c->table;
    t.zscale = c->zscale;
    {
      TimedLaunch tl(c, ex, SITE_UPDATE_WGRAD, a, /*manual=*/true);
      e = launch_gemm_tn(ex.dims, t, c->prec, a, /*tag=*/1, tl.start(), tl.stop());
    }
    if (e != hipSuccess) return hip_fail(c, e, "update weight gradient");
    red.upd[0] = true;
    ReduceUpd &r = red.u;
    r.P = c->part_u;
    r.zscale = c->zscale;
    r.Z = d.split_p + c->nb;
    r.M = H;
    r.Ncols = t.Ncols;
    r.F = d.F;
    r.Fp = d.Fp;
    r.H = H;
    r.dWp = dWp;
    r.dbp = dbp;
  } else {
    GemmTN t{};
    t.X = du;
    t.ldx = H;
    t.M = H;
    t.nseg = 4;
    t.seg[0] = SegY{hin, nullptr, ldh, d.Fp};
    t.seg[1] = SegY{A, nullptr, 4 * H, 4 * H};
    t.seg[2] = SegY{A, w.csr.sp, 4 * H, 4 * H};
    t.seg[3] = SegY{A, w.csr.sm, 4 * H, 4 * H};
    t.seg[4] = SegY{nullptr, nullptr, 0, 4}; // sum column: db^p
    t.nseg = 5;
    t.Ncols = d.Fp + 12 * H + 4;
    t.P = c->part_u;
    t.splits = d.split_p;
    {
      TimedLaunch tl(c, ex, SITE_UPDATE_WGRAD, a, /*manual=*/true);
      e = launch_gemm_tn(ex.dims, t, c->prec, a, /*tag=*/1, tl.start(), tl.stop());
    }
    if (e != hipSuccess) return hip_fail(c, e, "update weight gradient");
    ReduceMap &r = red.m[0];
    r.P = c->part_u;
    r.splits = d.split_p;
    r.M = H;
    r.Ncols = d.Fp + 12 * H + 4;
    r.main_cols = d.Fp + 12 * H;
    r.F = d.F;
    r.Fp = d.Fp;
    r.route[0] = ReduceRoute{0, H, dWp, d.F + 12 * H, 0, dbp, 1, H};
    r.nroute = 1;
  }
  red.njobs = 1;
  // S6 + S7.  With degree buckets: dA = du W_eff(d) formed per row and
  // feature block inside the aggregation adjoint (one launch, dA not
  // stored).  Otherwise dA = [du || s+ du || s- du] [W0; W+; W-] by the NT
  // GEMM, then the adjoint.
  const bool fused = c->nb && agg_bwd_fused_ok(H, c->nb);
  if (!fused) {
    GemmNT g{};
    if (c->nb) {
      g.nseg = 1;
      g.seg[0] = SegA{du, nullptr, H, H, 0};
      g.ldb = H;
      g.perm = w.csr.perm;
      g.brow = w.csr.brow;
      g.nb = c->nb;
      g.bstride = (long long)4 * H * H;
    } else {
      g.nseg = 3;
      g.seg[0] = SegA{du, nullptr, H, H, 0};
      g.seg[1] = SegA{du, w.csr.sp, H, H, H};
      g.seg[2] = SegA{du, w.csr.sm, H, H, 2 * H};
      g.ileave_n = 3;
      g.ldb = 3 * H;
    }
    g.B = c->WpTA[l];
    g.B_lo = c->prec ? c->WpTA_lo[l] : nullptr;
    g.Ncols = 4 * H;
    g.C = w.dA;
    g.ldc = 4 * H;
    g.M_fixed = -1;
    {
      TimedLaunch tl(c, ex, SITE_AGG_INPUT_GEMM, s, /*manual=*/true);
      e = launch_gemm_nt(ex.dims, ex.N, g, c->prec, w.ntpart, s, /*tag=*/3, tl.start(),
                         tl.stop());
    }
    if (e != hipSuccess) return hip_fail(c, e, "aggregate-input gradient GEMM");
  }
  // the weight gradients of the last layer that read this D (l + 2, or l + 1
  // with a single D) must be done before it is rewritten
  {
    const int k = w.D2 ? (l & 1) : -1;
    for (int q = 0; q < 2; ++q)
      if ((k < 0 || q == k) && c->pjoin_pending[q]) {
        c->pjoin_pending[q] = false;
        e = hipStreamWaitEvent(s, c->pjoin_ev[q], 0);
        if (e != hipSuccess) return hip_fail(c, e, "join");
      }
  }
  // S7: per-edge dm, D_in, De; then D_out through the transpose
  if (fused) {
    AggBwdFused f{};
    f.H = H;
    f.nb = c->nb;
    f.du = du;
    f.B = c->WpTA[l];
    f.B_lo = c->prec ? c->WpTA_lo[l] : nullptr;
    f.bstride = (long long)4 * H * H;
    f.perm = w.csr.perm;
    f.brow = w.csr.brow;
    f.PQ = PQ;
    f.rowptr = w.csr.rowptr;
    f.csr_src = w.csr.csr_src;
    f.csr_e = w.csr.csr_e;
    f.WeT = static_cast<const float *>(c->WeT[l]);
    f.bm = bm;
    f.A = A;
    f.args = args;
    f.dm = w.dm;
    f.D = Dl;
    f.ldD = ldD;
    TimedLaunch tl(c, ex, SITE_AGGREGATE_BWD, s, /*manual=*/true);
    e = launch_agg_bwd_fused(ex.N, f, c->prec, Fe, s, tl.start(), tl.stop());
  } else {
    TimedLaunch tl(c, ex, SITE_AGGREGATE_BWD, s, /*manual=*/true);
    e = launch_aggregate_bwd(ex.dims, ex.N, H, Fe, PQ, w.csr.rowptr, w.csr.csr_src,
                             w.csr.csr_e, static_cast<const float *>(c->WeT[l]), bm, A, args, w.dA,
                             w.dm, Dl, ldD, s, tl.start(), tl.stop());
  }
  if (e == hipSuccess)
    e = launch_transpose_sum(ex.dims, ex.N, H, w.csr.srcptr, w.csr.t2csr, w.dm, Dl, ldD, s);
  if (e != hipSuccess) return hip_fail(c, e, "aggregation adjoint");
  // second fork: D = [D_in | D_out | De] is ready
  e = hipEventRecord(c->fork_ev[1], s);
  if (e == hipSuccess) e = hipStreamWaitEvent(a, c->fork_ev[1], 0);
  if (e != hipSuccess) return hip_fail(c, e, "fork");
  // S8: [dW_dst | dW_src] = [D_in | D_out]^T h, db^m = sum_i D_in, and the
  // edge-feature columns sum_i De_i = sum_k dm_k e_k (the sum column of the
  // De rows, whose product with h is not needed: for large batches those
  // rows get a GEMM of their own with the sum column alone)
  const bool split_de = Fe > 0 && ex.N >= kSplitDeRows;
  {
    GemmTN t{};
    t.X = Dl;
    t.ldx = ldD;
    t.M = split_de ? 2 * H : ldD;
    t.nseg = 2;
    t.seg[0] = SegY{hin, nullptr, ldh, d.Fp};
    t.seg[1] = SegY{nullptr, nullptr, 0, 4}; // sum column: db^m and the e_k weights
    t.Ncols = d.Fp + 4;
    t.P = c->part;
    t.splits = split_de ? d.split_m2 : d.split_m;
    {
      TimedLaunch tl(c, ex, SITE_MESSAGE_WGRAD, a, /*manual=*/true);
      e = launch_gemm_tn(ex.dims, t, c->prec, a, /*tag=*/2, tl.start(), tl.stop());
    }
    const int ldm = 2 * d.F + Fe;
    {
      ReduceMap &r = red.m[red.njobs++];
      r.P = c->part;
      r.splits = t.splits;
      r.M = t.M;
      r.Ncols = d.Fp + 4;
      r.main_cols = d.Fp;
      r.F = d.F;
      r.Fp = d.Fp;
      r.route[0] = ReduceRoute{0, H, dWm, ldm, 0, dbm, 1, H};               // D_in
      r.route[1] = ReduceRoute{H, 2 * H, dWm, ldm, d.F, nullptr, 0, 1};      // D_out
      r.route[2] = ReduceRoute{2 * H, ldD, nullptr, 0, 0, dWm + 2 * d.F, ldm, H}; // De
      r.nroute = (Fe > 0 && !split_de) ? 3 : 2;
    }
    // column sums of De over kColsumChunks row chunks, after the GEMM's
    // partials in the same buffer
    float *pcol = c->part + (size_t)t.splits * t.M * t.Ncols;
    if (e == hipSuccess && split_de) {
      e = launch_colsum(ex.dims, Dl + 2 * H, ldD, Fe * H, kColsumChunks, pcol, a);
      ReduceMap &r = red.m[red.njobs++];
      r.P = pcol;
      r.splits = kColsumChunks;
      r.M = Fe * H;
      r.Ncols = 4;
      r.main_cols = 0;
      r.F = 0;
      r.Fp = 0;
      r.route[0] = ReduceRoute{0, Fe * H, nullptr, 0, 0, dWm + 2 * d.F, ldm, H}; // De
      r.nroute = 1;
    }
    if (e == hipSuccess) e = launch_reduce_jobs(red, a);
    if (e != hipSuccess) return hip_fail(c, e, "weight gradients");
  }
  // S6 + S8 input gradient: dh = [du || D_in || D_out] [W_h; W_dst; W_src]
  if (dh_in) {
    // it rewrites the du that the previous layer's weight gradients read
    const int k = (l + 1) & 1;
    if (c->pjoin_pending[k]) {
      c->pjoin_pending[k] = false;
      e = hipStreamWaitEvent(s, c->pjoin_ev[k], 0);
      if (e != hipSuccess) return hip_fail(c, e, "join");
    }
    const float *mask = (mask_dh_in && l > 0) ? h_in : nullptr;
    // the LDS-DMA form where it applies (FP32: on the inputs as they lie)
    GemmNTB q{};
    q.nseg = 3;
    q.seg[0] = SegB{du, H, H, 0};
    q.seg[1] = SegB{Dl, ldD, H, H};
    q.seg[2] = SegB{Dl + H, ldD, H, 2 * H};
    q.B = c->WhdsT[l];
    q.ldb = 3 * H;
    q.Ncols = d.F;
    q.C = dh_in;
    q.ldc = d.F;
    q.M_fixed = -1;
    q.mask = mask;
    if (c->prec == 0 && gemm_ntb_ok(q, 0)) {
      TimedLaunch tl(c, ex, SITE_INPUT_GEMM, s, /*manual=*/true);
      e = launch_gemm_ntb(ex.dims, ex.N, q, 0, s, /*tag=*/4, tl.start(), tl.stop());
    } else {
      GemmNT g{};
      g.nseg = 3;
      g.seg[0] = SegA{du, nullptr, H, H, 0};
      g.seg[1] = SegA{Dl, nullptr, ldD, H, H};
      g.seg[2] = SegA{Dl + H, nullptr, ldD, H, 2 * H};
      g.B = c->WhdsT[l];
      g.B_lo = c->prec ? c->WhdsT_lo[l] : nullptr;
      g.ldb = 3 * H;
      g.Ncols = d.F;
      g.C = dh_in;
      g.ldc = d.F;
      g.M_fixed = -1;
      g.mask = mask;
      TimedLaunch tl(c, ex, SITE_INPUT_GEMM, s, /*manual=*/true);
      e = launch_gemm_nt(ex.dims, ex.N, g, c->prec, w.ntpart, s, /*tag=*/4, tl.start(),
                         tl.stop());
    }
    if (e != hipSuccess) return hip_fail(c, e, "input gradient GEMM");
  }
  // join now, or leave it to the launches above of the next layers
  e = hipEventRecord(c->pjoin_ev[l & 1], a);
  if (e == hipSuccess && !defer_join) e = hipStreamWaitEvent(s, c->pjoin_ev[l & 1], 0);
  if (e != hipSuccess) return hip_fail(c, e, "join");
  // a join covers every earlier record (the aux stream runs in order)
  if (!defer_join) c->pjoin_pending[0] = c->pjoin_pending[1] = false;
  else c->pjoin_pending[l & 1] = true;
  return HGNN_OK;
}

// Graph heads (and, in the fused path, node heads) and the weighted loss.
int head_forward(hgnn_ctx *c, Exec &ex, const float *wh, const float *h, const float *target,
                 float *pred, float *loss, hipStream_t s, float *pred_node,
                 const float *ynode) {
  const int H = c->H, Tn = c->Tn;
  Work &w = ex.w;
  // the staged W1 transposes describe the context's own head weights
  const float *W1T = (wh == c->params + c->off_head && c->staged_from_params) ? c->W1T : nullptr;
  hipError_t e = launch_head_forward(ex.dims, ex.B, H, c->Tg, ex.graph_ptr, h, wh, W1T, w.g,
                                     w.q, w.ypred, pred, s);
  if (e == hipSuccess && Tn > 0) {
    const float *wn = c->params + c->off_node;
    e = launch_stage_node_heads(H, Tn, wn, c->W1n, c->W1nT, s);
    for (int k = 0; k < Tn && e == hipSuccess; ++k) {
      GemmNT g{};
      g.nseg = 1;
      g.seg[0] = SegA{h, nullptr, H, H, 0};
      g.B = c->W1n + (size_t)k * H * H;
      g.ldb = H;
      g.Ncols = H;
      g.bias = wn + (size_t)k * node_head_size(H) + (size_t)H * H;
      g.relu = 1;
      g.C = w.Qn + (size_t)k * ex.N * H;
      g.ldc = H;
      g.M_fixed = -1;
      e = launch_gemm_nt(ex.dims, ex.N, g, /*precision=*/0, w.ntpart, s);
    }
    if (e == hipSuccess) e = launch_node_head_out(ex.dims, ex.N, H, Tn, w.Qn, wn, w.zn,
                                                  pred_node, s);
  }
  if (e == hipSuccess && loss && target)
    e = launch_loss(ex.dims, c->Tg, w.ypred, target, c->gw_dev, Tn, w.zn, ynode, c->nw_dev,
                    loss, s);
  if (e != hipSuccess) return hip_fail(c, e, "head forward");
  return HGNN_OK;
}

// Node heads' adjoint (fused path): their weight gradients and their share
// of dL/dh (into w.dhn).  h: the last layer's output.
static int node_heads_backward(hgnn_ctx *c, Exec &ex, const float *h, hipStream_t s) {
  const int H = c->H, Tn = c->Tn;
  Work &w = ex.w;
  const float *wn = c->params + c->off_node;
  float *gwn = c->grads + c->off_node;
  hipError_t e = launch_node_head_err(ex.dims, ex.N, H, Tn, w.Qn, wn, w.zn, ex.ynode,
                                      c->nw_dev, w.en, w.dQn, s);
  for (int k = 0; k < Tn && e == hipSuccess; ++k) {
    float *dW1 = gwn + (size_t)k * node_head_size(H);
    GemmTN t{};
    t.X = w.dQn + (size_t)k * ex.N * H;
    t.ldx = H;
    t.M = H;
    t.seg[0] = SegY{h, nullptr, H, H};
    t.seg[1] = SegY{nullptr, nullptr, 0, 4}; // sum column: db1
    t.nseg = 2;
    t.Ncols = H + 4;
    t.P = c->part;
    t.splits = c->split_node;
    e = launch_gemm_tn(ex.dims, t, /*precision=*/0, s);
    if (e == hipSuccess) {
      ReduceMap r{};
      r.P = c->part;
      r.splits = c->split_node;
      r.M = H;
      r.Ncols = H + 4;
      r.main_cols = H;
      r.F = H;
      r.Fp = H;
      r.route[0] = ReduceRoute{0, H, dW1, H, 0, dW1 + (size_t)H * H, 1, H};
      r.nroute = 1;
      e = launch_reduce_map(r, s);
    }
  }
  if (e == hipSuccess) e = launch_node_head_small(ex.dims, ex.N, H, Tn, w.Qn, w.en, c->nh_part, gwn, s);
  if (e == hipSuccess) {
    GemmNT g{};
    g.nseg = Tn;
    for (int k = 0; k < Tn; ++k)
      g.seg[k] = SegA{w.dQn + (size_t)k * ex.N * H, nullptr, H, H, k * H};
    g.B = c->W1nT;
    g.ldb = Tn * H;
    g.Ncols = H;
    g.C = w.dhn;
    g.ldc = H;
    g.M_fixed = -1;
    e = launch_gemm_nt(ex.dims, ex.N, g, /*precision=*/0, w.ntpart, s);
  }
  if (e != hipSuccess) return hip_fail(c, e, "node heads backward");
  return HGNN_OK;
}

int head_backward(hgnn_ctx *c, Exec &ex, const float *wh, const float *target, const float *dpred,
                  float *dh, float *dwh, hipStream_t s, const float *relu_of = nullptr,
                  const float *h_last = nullptr) {
  const int H = c->H;
  Work &w = ex.w;
  const float *add = nullptr;
  if (c->Tn > 0) {
    int rc = node_heads_backward(c, ex, h_last, s);
    if (rc) return rc;
    add = w.dhn;
  }
  hipError_t e = launch_head_backward(ex.dims, ex.B, H, c->Tg, ex.graph_ptr, wh, w.g, w.q,
                                      w.ypred, target, dpred, c->gw_dev, w.dy, w.dq, dh, dwh,
                                      relu_of, add, c->part, s);
  if (e != hipSuccess) return hip_fail(c, e, "head backward");
  return HGNN_OK;
}

// ---- GraphSAGE and CGCNN layer kinds ---------------------------------------

// The block copies that refresh their GEMM-layout weights (one launch).
static std::vector<GcStageJob> gc_stage_jobs(hgnn_ctx *c) {
  std::vector<GcStageJob> jobs;
  const int H = c->H, bf = c->prec;
  const size_t esz = bf ? 2 : 4;
  auto at = [&](void *base, size_t elems) {
    return base ? static_cast<void *>(static_cast<uint8_t *>(base) + esz * elems) : nullptr;
  };
  auto job = [&](const float *src, long long rs, long long cs, int rows, int cols, int vrows,
                 int vcols, void *hi, void *lo, int ld, int to_bf16) {
    jobs.push_back(GcStageJob{src, rs, cs, rows, cols, vrows, vcols, hi, lo, ld, to_bf16});
  };
  for (int l = 0; l < c->L; ++l) {
    const LayerDesc &d = c->ld[l];
    const float *W = c->params + d.oWm;
    void *g1 = c->Wg1[l], *g2 = c->Wg2[l];
    void *g1l = bf ? c->Wg1_lo[l] : nullptr, *g2l = bf ? c->Wg2_lo[l] : nullptr;
    if (c->kind == HGNN_GC_SAGE) {
      const int F = d.F, Fp = d.Fp;
      // Wg1 [H, 2Fp] = [W_self | W_nbr], each half zero-padded from F to Fp
      job(W, 2 * F, 1, H, Fp, H, F, g1, g1l, 2 * Fp, bf);
      job(W + F, 2 * F, 1, H, Fp, H, F, at(g1, Fp), at(g1l, Fp), 2 * Fp, bf);
      // Wg2 [2Fp, H] = [W_self^T; W_nbr^T], rows past F zero
      job(W, 1, 2 * F, Fp, H, F, H, g2, g2l, H, bf);
      job(W + F, 1, 2 * F, Fp, H, F, H, at(g2, (size_t)Fp * H), at(g2l, (size_t)Fp * H), H, bf);
    } else {
      const int ldw = 2 * H + c->Fe;
      // Wg1 [4H, H] = [W[:, 0:H]; W[:, H:2H]] (destination rows, then source rows)
      job(W, ldw, 1, 2 * H, H, 2 * H, H, g1, g1l, H, bf);
      job(W + H, ldw, 1, 2 * H, H, 2 * H, H, at(g1, (size_t)2 * H * H),
          at(g1l, (size_t)2 * H * H), H, bf);
      // Wg2 [H, 4H]: row n = [W[:, n] | W[:, H + n]]
      job(W, 1, ldw, H, 2 * H, H, 2 * H, g2, g2l, 4 * H, bf);
      job(W + H, 1, ldw, H, 2 * H, H, 2 * H, at(g2, 2 * H), at(g2l, 2 * H), 4 * H, bf);
      // edge-feature columns, FP32 in both precisions: weT[k, r] = W[r, 2H + k]
      if (c->Fe > 0)
        job(W + 2 * H, 1, ldw, c->Fe, 2 * H, c->Fe, 2 * H, c->WeT[l], nullptr, 2 * H, 0);
    }
  }
  if (c->kind == HGNN_GC_CGCNN)
    job(c->params + c->off_emb, c->F0, 1, H, c->F0p, H, c->F0, c->Wemb, c->Wemb_lo, c->F0p, bf);
  return jobs;
}

static void fork_to_aux(hgnn_ctx *c, int k, hipStream_t s, hipError_t &e) {
  if (e == hipSuccess) e = hipEventRecord(c->fork_ev[k], s);
  if (e == hipSuccess) e = hipStreamWaitEvent(c->aux, c->fork_ev[k], 0);
}

static void join_aux(hgnn_ctx *c, hipStream_t s, hipError_t &e) {
  if (e == hipSuccess) e = hipEventRecord(c->join_ev, c->aux);
  if (e == hipSuccess) e = hipStreamWaitEvent(s, c->join_ev, 0);
}

// Forward of the GC stack; *last receives the last layer's output.
static int gc_forward(hgnn_ctx *c, Exec &ex, hipStream_t s, const float **last) {
  Work &w = ex.w;
  const int H = c->H;
  hipError_t e = hipSuccess;
  const float *h = w.xpad;
  int ldh = c->F0p;
  if (c->kind == HGNN_GC_CGCNN) { // h0 = x W_emb^T + b_emb
    GemmNT g{};
    g.nseg = 1;
    g.seg[0] = SegA{w.xpad, nullptr, c->F0p, c->F0p, 0};
    g.B = c->Wemb;
    g.B_lo = c->prec ? c->Wemb_lo : nullptr;
    g.ldb = c->F0p;
    g.Ncols = H;
    g.bias = c->params + c->off_emb + (size_t)H * c->F0;
    g.C = w.h0;
    g.ldc = H;
    g.M_fixed = -1;
    e = launch_gemm_nt(ex.dims, ex.N, g, c->prec, w.ntpart, s);
    if (e != hipSuccess) return hip_fail(c, e, "embedding GEMM");
    h = w.h0;
    ldh = H;
  }
  for (int l = 0; l < c->L; ++l) {
    if (int rc = injected_failure(c)) return rc;
    const LayerDesc &d = c->ld[l];
    const float *b = c->params + d.obm;
    if (c->kind == HGNN_GC_SAGE) {
      e = launch_sage_mean(ex.dims, ex.N, d.Fp, w.csr.rowptr, w.csr.csr_src, h, ldh, w.gcA[l],
                           s);
      if (e != hipSuccess) return hip_fail(c, e, "neighbour mean");
      GemmNT g{};
      g.nseg = 2;
      g.seg[0] = SegA{h, nullptr, ldh, d.Fp, 0};
      g.seg[1] = SegA{w.gcA[l], nullptr, d.Fp, d.Fp, d.Fp};
      g.B = c->Wg1[l];
      g.B_lo = c->prec ? c->Wg1_lo[l] : nullptr;
      g.ldb = 2 * d.Fp;
      g.Ncols = H;
      g.bias = b;
      g.relu = 1;
      g.C = w.hbuf[l];
      g.ldc = H;
      g.M_fixed = -1;
      {
        TimedLaunch tl(c, ex, SITE_UPDATE_GEMM, s, /*manual=*/true);
        hipEvent_t e0 = tl.start(), e1 = tl.stop();
        e = launch_gemm_nt(ex.dims, ex.N, g, c->prec, w.ntpart, s, /*tag=*/1, e0, e1);
      }
      if (e != hipSuccess) return hip_fail(c, e, "GraphSAGE GEMM");
    } else {
      GemmNT g{};
      g.nseg = 1;
      g.seg[0] = SegA{h, nullptr, ldh, H, 0};
      g.B = c->Wg1[l];
      g.B_lo = c->prec ? c->Wg1_lo[l] : nullptr;
      g.ldb = H;
      g.Ncols = 4 * H;
      g.C = w.gcA[l];
      g.ldc = 4 * H;
      g.M_fixed = -1;
      e = launch_gemm_nt(ex.dims, ex.N, g, c->prec, w.ntpart, s);
      if (e != hipSuccess) return hip_fail(c, e, "CGCNN gate GEMM");
      {
        TimedLaunch tl(c, ex, SITE_AGGREGATE, s);
        e = launch_cg_aggregate(ex.dims, ex.N, H, c->Fe, w.csr.rowptr, w.csr.csr_src,
                                w.csr.csr_e, w.gcA[l], static_cast<const float *>(c->WeT[l]),
                                b, h, w.hbuf[l], s);
      }
      if (e != hipSuccess) return hip_fail(c, e, "CGCNN aggregation");
    }
    h = w.hbuf[l];
    ldh = H;
  }
  *last = h;
  return HGNN_OK;
}

// Backward of the GC stack from cur = dL/du of the last layer (its ReLU
// adjoint applied); nxt is the second [N, H] buffer of the ping-pong.
// The main stream waits for a layer's weight-gradient stream (join_ev) only
// at the next layer's first launch that overwrites a buffer those GEMMs read:
// GraphSAGE's neighbour scatter (it rewrites this layer's du) and CGCNN's
// input-gradient GEMM (CGCNN's D alternates between two buffers by layer
// parity, so the next layer's aggregation adjoint leaves this layer's D
// alone).  Layer 0 joins at once.
static void wait_pending_join(hgnn_ctx *c, hipStream_t s, hipError_t &e) {
  if (e == hipSuccess && c->join_pending) {
    c->join_pending = false;
    e = hipStreamWaitEvent(s, c->join_ev, 0);
  }
}

static int gc_backward(hgnn_ctx *c, Exec &ex, float *cur, float *nxt, hipStream_t s) {
  Work &w = ex.w;
  const int H = c->H, Fe = c->Fe;
  hipError_t e = hipSuccess;
  wait_pending_join(c, s, e); // left by a backward that failed part-way
  if (e != hipSuccess) return hip_fail(c, e, "join");
  for (int l = c->L - 1; l >= 0; --l) {
    if (int rc = injected_failure(c)) return rc;
    const LayerDesc &d = c->ld[l];
    float *dW = c->grads + d.oWm, *db = c->grads + d.obm;
    const float *hin = l ? w.hbuf[l - 1] : (c->kind == HGNN_GC_CGCNN ? w.h0 : w.xpad);
    const int ldh = l ? H : (c->kind == HGNN_GC_CGCNN ? H : c->F0p);
    const float *du = cur;
    if (c->kind == HGNN_GC_SAGE) {
      fork_to_aux(c, 0, s, e);
      if (e != hipSuccess) return hip_fail(c, e, "fork");
      // dW = du^T [h || M], db = sum du
      GemmTN t{};
      t.X = du;
      t.ldx = H;
      t.M = H;
      t.seg[0] = SegY{hin, nullptr, ldh, d.Fp};
      t.seg[1] = SegY{w.gcA[l], nullptr, d.Fp, d.Fp};
      t.seg[2] = SegY{nullptr, nullptr, 0, 4};
      t.nseg = 3;
      t.Ncols = 2 * d.Fp + 4;
      t.P = c->part;
      t.splits = d.split_p;
      {
        TimedLaunch tl(c, ex, SITE_UPDATE_WGRAD, c->aux);
        e = launch_gemm_tn(ex.dims, t, c->prec, c->aux);
      }
      if (e == hipSuccess) {
        ReduceMap r{};
        r.P = c->part;
        r.splits = d.split_p;
        r.M = H;
        r.Ncols = 2 * d.Fp + 4;
        r.main_cols = 2 * d.Fp;
        r.F = d.F;
        r.Fp = d.Fp;
        r.npad = 2;
        r.route[0] = ReduceRoute{0, H, dW, 2 * d.F, 0, db, 1, H};
        r.nroute = 1;
        e = launch_reduce_map(r, c->aux);
      }
      if (e != hipSuccess) return hip_fail(c, e, "GraphSAGE weight gradient");
      if (l > 0) { // G = du [W_self | W_nbr]; dh_in = G_self + neighbour scatter
        GemmNT g{};
        g.nseg = 1;
        g.seg[0] = SegA{du, nullptr, H, H, 0};
        g.B = c->Wg2[l];
        g.B_lo = c->prec ? c->Wg2_lo[l] : nullptr;
        g.ldb = H;
        g.Ncols = 2 * H;
        g.C = w.gcG;
        g.ldc = 2 * H;
        g.M_fixed = -1;
        e = launch_gemm_nt(ex.dims, ex.N, g, c->prec, w.ntpart, s);
        wait_pending_join(c, s, e);
        if (e == hipSuccess)
          e = launch_sage_scatter(ex.dims, ex.N, H, w.csr.srcptr, w.csr.t2csr, w.csr.csr_dst,
                                  w.csr.rowptr, w.gcG, hin, nxt, s);
        if (e != hipSuccess) return hip_fail(c, e, "GraphSAGE input gradient");
      }
    } else {
      const int ldD = (4 + 2 * Fe) * H;
      float *gcD = (l & 1) ? w.gcD1 : w.gcD;
      {
        TimedLaunch tl(c, ex, SITE_AGGREGATE_BWD, s);
        e = launch_cg_aggregate_bwd(ex.dims, ex.N, H, Fe, w.csr.rowptr, w.csr.csr_src,
                                    w.csr.csr_e, w.gcA[l], static_cast<const float *>(c->WeT[l]),
                                    c->params + d.obm, du, w.gcdm, gcD, ldD, s);
      }
      if (e == hipSuccess)
        e = launch_transpose_sum(ex.dims, ex.N, 2 * H, w.csr.srcptr, w.csr.t2csr, w.gcdm, gcD,
                                 ldD, s);
      if (e != hipSuccess) return hip_fail(c, e, "CGCNN aggregation adjoint");
      fork_to_aux(c, 0, s, e);
      if (e != hipSuccess) return hip_fail(c, e, "fork");
      // [dW_dst | dW_src] = [D_in | D_out]^T h; db and the edge columns from
      // the constant-one column
      GemmTN t{};
      t.X = gcD;
      t.ldx = ldD;
      t.M = ldD;
      t.seg[0] = SegY{hin, nullptr, ldh, H};
      t.seg[1] = SegY{nullptr, nullptr, 0, 4};
      t.nseg = 2;
      t.Ncols = H + 4;
      t.P = c->part;
      t.splits = d.split_p;
      {
        TimedLaunch tl(c, ex, SITE_UPDATE_WGRAD, c->aux);
        e = launch_gemm_tn(ex.dims, t, c->prec, c->aux);
      }
      if (e == hipSuccess) {
        const int ldw = 2 * H + Fe;
        ReduceMap r{};
        r.P = c->part;
        r.splits = d.split_p;
        r.M = ldD;
        r.Ncols = H + 4;
        r.main_cols = H;
        r.F = H;
        r.Fp = H;
        r.route[0] = ReduceRoute{0, 2 * H, dW, ldw, 0, db, 1, 2 * H};
        r.route[1] = ReduceRoute{2 * H, 4 * H, dW, ldw, H, nullptr, 0, 1};
        r.route[2] = ReduceRoute{4 * H, ldD, nullptr, 0, 0, dW + 2 * H, ldw, 2 * H};
        r.nroute = Fe > 0 ? 3 : 2;
        e = launch_reduce_map(r, c->aux);
      }
      if (e != hipSuccess) return hip_fail(c, e, "CGCNN weight gradient");
      // dh_in = du (residual) + [D_in | D_out] [W_dst; W_src], masked by the
      // ReLU of the layer below (the embedding below layer 0 has none)
      GemmNT g{};
      g.nseg = 2;
      g.seg[0] = SegA{gcD, nullptr, ldD, 2 * H, 0};
      g.seg[1] = SegA{gcD + 2 * H, nullptr, ldD, 2 * H, 2 * H};
      g.B = c->Wg2[l];
      g.B_lo = c->prec ? c->Wg2_lo[l] : nullptr;
      g.ldb = 4 * H;
      g.Ncols = H;
      g.addend = du;
      g.ld_add = H;
      g.mask = l ? hin : nullptr;
      g.C = nxt;
      g.ldc = H;
      g.M_fixed = -1;
      wait_pending_join(c, s, e);
      if (e != hipSuccess) return hip_fail(c, e, "join");
      {
        TimedLaunch tl(c, ex, SITE_INPUT_GEMM, s);
        e = launch_gemm_nt(ex.dims, ex.N, g, c->prec, w.ntpart, s);
      }
      if (e != hipSuccess) return hip_fail(c, e, "CGCNN input gradient");
    }
    if (l > 0) { // deferred to the next layer
      if (e == hipSuccess) e = hipEventRecord(c->join_ev, c->aux);
      c->join_pending = e == hipSuccess;
    } else {
      wait_pending_join(c, s, e);
      join_aux(c, s, e);
    }
    if (e != hipSuccess) return hip_fail(c, e, "join");
    std::swap(cur, nxt);
  }
  if (c->kind == HGNN_GC_CGCNN) { // embedding: dW_emb = dh0^T x, db_emb = sum dh0
    GemmTN t{};
    t.X = cur;
    t.ldx = H;
    t.M = H;
    t.seg[0] = SegY{w.xpad, nullptr, c->F0p, c->F0p};
    t.seg[1] = SegY{nullptr, nullptr, 0, 4};
    t.nseg = 2;
    t.Ncols = c->F0p + 4;
    t.P = c->part;
    t.splits = c->split_emb;
    e = launch_gemm_tn(ex.dims, t, c->prec, s);
    if (e == hipSuccess) {
      float *dWe = c->grads + c->off_emb;
      ReduceMap r{};
      r.P = c->part;
      r.splits = c->split_emb;
      r.M = H;
      r.Ncols = c->F0p + 4;
      r.main_cols = c->F0p;
      r.F = c->F0;
      r.Fp = c->F0p;
      r.route[0] = ReduceRoute{0, H, dWe, c->F0, 0, dWe + (size_t)H * c->F0, 1, H};
      r.nroute = 1;
      e = launch_reduce_map(r, s);
    }
    if (e != hipSuccess) return hip_fail(c, e, "embedding weight gradient");
  }
  return HGNN_OK;
}

static int create_ctx(const hgnn_config *cfg, int kind, const hgnn_heads *heads,
                      hgnn_ctx **out);

} // namespace hgnn

// ===========================================================================
// C-ABI
// ===========================================================================

#define HGNN_GUARD(c)                                                                  \
  do {                                                                                 \
    if (!(c)) return fail(HGNN_EINVAL, "context is NULL");                             \
    if ((c)->sticky) return fail(HGNN_ESTATE, "context failed earlier; restore state"); \
    hipError_t e_ = hipSetDevice((c)->dev);                                            \
    if (e_ != hipSuccess) return hip_fail((c), e_, "hipSetDevice");                    \
  } while (0)

extern "C" {

const char *hgnn_last_error(void) { return g_err.c_str(); }

int hgnn_create(const hgnn_config *cfg, const float *init_params, uint64_t seed, void *stream,
                hgnn_ctx **out) {
  int rc = hgnn_create_multitask(cfg, nullptr, out);
  if (rc) return rc;
  rc = init_params ? hgnn_set_params(*out, init_params, stream)
                   : hgnn_init_params(*out, seed, stream);
  if (rc) {
    hgnn_destroy(*out);
    *out = nullptr;
  }
  return rc;
}

int hgnn_create_multitask(const hgnn_config *cfg, const hgnn_heads *heads, hgnn_ctx **out) {
  return create_ctx(cfg, HGNN_GC_PNA, heads, out);
}

int hgnn_create_gc(const hgnn_config *cfg, int32_t kind, const hgnn_heads *heads,
                   hgnn_ctx **out) {
  if (kind != HGNN_GC_PNA && kind != HGNN_GC_SAGE && kind != HGNN_GC_CGCNN) {
    if (out) *out = nullptr;
    return fail(HGNN_EINVAL, "kind must be HGNN_GC_PNA, HGNN_GC_SAGE or HGNN_GC_CGCNN");
  }
  return create_ctx(cfg, kind, heads, out);
}

} // extern "C"

namespace hgnn {

static int create_ctx(const hgnn_config *cfg, int kind, const hgnn_heads *heads,
                      hgnn_ctx **out) {
  if (!cfg || !out) return fail(HGNN_EINVAL, "cfg and out are required");
  *out = nullptr;
  const bool pna = kind == HGNN_GC_PNA;
  const int Tg = heads ? heads->graph_heads : 1, Tn = heads ? heads->node_heads : 0;
  if (Tg < 1 || Tg > 8) return fail(HGNN_EINVAL, "graph_heads must be in 1..8");
  if (Tn < 0 || Tn > 4) return fail(HGNN_EINVAL, "node_heads must be in 0..4");
  std::vector<float> gw(Tg, 1.0f), nw(Tn, 1.0f);
  for (int k = 0; heads && heads->graph_weights && k < Tg; ++k) gw[k] = heads->graph_weights[k];
  for (int k = 0; heads && heads->node_weights && k < Tn; ++k) nw[k] = heads->node_weights[k];
  for (float v : gw)
    if (!(v >= 0.f) || !std::isfinite(v)) return fail(HGNN_EINVAL, "loss weights must be >= 0");
  for (float v : nw)
    if (!(v >= 0.f) || !std::isfinite(v)) return fail(HGNN_EINVAL, "loss weights must be >= 0");
  if (cfg->num_layers < 1 || cfg->num_layers > 64)
    return fail(HGNN_EINVAL, "num_layers must be in 1..64");
  if (cfg->hidden < 16 || cfg->hidden > 512 || cfg->hidden % 16)
    return fail(HGNN_EINVAL, "hidden must be a multiple of 16 in 16..512");
  if (cfg->node_feat < 1 || cfg->node_feat > 4096)
    return fail(HGNN_EINVAL, "node_feat must be in 1..4096");
  if (cfg->edge_feat < 0 || cfg->edge_feat > 4)
    return fail(HGNN_EINVAL, "edge_feat must be in 0..4");
  if (cfg->max_degree < 1 || cfg->max_degree > 255)
    return fail(HGNN_EINVAL, "max_degree must be in 1..255");
  if (cfg->precision != HGNN_PREC_FP32 && cfg->precision != HGNN_PREC_BF16)
    return fail(HGNN_EINVAL, "precision must be HGNN_PREC_FP32 or HGNN_PREC_BF16");
  if (cfg->recompute != 0 && cfg->recompute != 1)
    return fail(HGNN_EINVAL, "recompute must be 0 or 1");
  if (!pna && cfg->recompute) return fail(HGNN_EINVAL, "recompute is PNA-only");
  if (pna && (!(cfg->delta > 0.0) || !std::isfinite(cfg->delta)))
    return fail(HGNN_EINVAL, "delta must be positive and finite");
  if (!(cfg->std_eps >= 0.0) || !std::isfinite(cfg->std_eps))
    return fail(HGNN_EINVAL, "std_eps must be >= 0");

  hgnn_ctx *c = new (std::nothrow) hgnn_ctx();
  if (!c) return fail(HGNN_ENOMEM, "host allocation failed");
  c->cfg = *cfg;
  c->L = cfg->num_layers;
  c->H = cfg->hidden;
  c->F0 = cfg->node_feat;
  c->F0p = ru(cfg->node_feat, 16);
  c->Fe = cfg->edge_feat;
  c->maxd = cfg->max_degree;
  c->prec = cfg->precision;
  c->recompute = cfg->recompute;
  c->kind = kind;
  const int H = c->H;
  int64_t off = 0;
  size_t part_max = 0, part_u_max = 0;
  if (kind == HGNN_GC_SAGE) {
    for (int l = 0; l < c->L; ++l) {
      LayerDesc d{};
      d.F = l == 0 ? c->F0 : H;
      d.Fp = l == 0 ? c->F0p : H;
      d.off = d.oWm = off;
      off += (int64_t)H * 2 * d.F;
      d.obm = off;
      off += H;
      d.size = off - d.off;
      d.split_p = tn_splits(H, 2 * d.Fp + 4, cfg->precision);
      part_max = std::max(part_max, (size_t)d.split_p * H * (2 * d.Fp + 4));
      c->ld.push_back(d);
    }
  } else if (kind == HGNN_GC_CGCNN) {
    c->off_emb = 0;
    off += (int64_t)H * c->F0 + H;
    c->split_emb = tn_splits(H, c->F0p + 4, cfg->precision);
    part_max = std::max(part_max, (size_t)c->split_emb * H * (c->F0p + 4));
    const int ldD = (4 + 2 * c->Fe) * H;
    for (int l = 0; l < c->L; ++l) {
      LayerDesc d{};
      d.F = d.Fp = H;
      d.off = d.oWm = off;
      off += (int64_t)2 * H * (2 * H + c->Fe);
      d.obm = off;
      off += 2 * H;
      d.size = off - d.off;
      d.split_p = tn_splits(ldD, H + 4, cfg->precision);
      part_max = std::max(part_max, (size_t)d.split_p * ldD * (H + 4));
      c->ld.push_back(d);
    }
  }
  c->nb = (pna && c->maxd + 1 <= kMaxBuckets) ? c->maxd + 1 : 0;
  int zmax = 0; // chunks of the bucketed update weight gradient
  for (int l = 0; pna && l < c->L; ++l) {
    LayerDesc d;
    d.F = l == 0 ? c->F0 : H;
    d.Fp = l == 0 ? c->F0p : H;
    d.off = off;
    d.oWm = off;
    off += (int64_t)H * (2 * d.F + c->Fe);
    d.obm = off;
    off += H;
    d.oWp = off;
    off += (int64_t)H * (d.F + 12 * H);
    d.obp = off;
    off += H;
    d.size = off - d.off;
    // the update weight gradient's columns: [h | A | s+ A | s- A | sum] or,
    // with degree buckets, [h | A | sum] over nb more (bucket-pure) chunks
    const int wcols = d.Fp + (c->nb ? 4 : 12) * H + 4;
    d.split_p = tn_splits(H, wcols, cfg->precision);
    // message weight gradient: [D_in | D_out | De]^T [h | 1] in one GEMM, or
    // for large batches [D_in | D_out]^T [h | 1] and the column sums of De
    // apart (the De^T h block is not needed; see kSplitDeRows)
    d.split_m = tn_splits((2 + c->Fe) * H, d.Fp + 4, cfg->precision);
    d.split_m2 = tn_splits(2 * H, d.Fp + 4, cfg->precision);

    zmax = std::max(zmax, d.split_p + c->nb);
    // the update weight gradient's partials have a buffer of their own: they
    // are reduced together with the message weight gradient's
    part_u_max = std::max(part_u_max, (size_t)(d.split_p + c->nb) * H * wcols);
    const size_t b = std::max((size_t)d.split_m * (2 + c->Fe) * H * (d.Fp + 4),
                              (size_t)d.split_m2 * 2 * H * (d.Fp + 4) +
                                  (size_t)kColsumChunks * c->Fe * H * 4);
    part_max = std::max(part_max, b);
    c->ld.push_back(d);
  }
  c->Tg = Tg;
  c->Tn = Tn;
  // the head weight gradients' chunk partials (large batches) use part too
  part_max = std::max(part_max, head_partial_floats(H, Tg));
  c->cfg.reserved = Tg + 256 * Tn + 65536 * kind; // part of the checkpoint's identity
  // tensors of the packed vector, for the seeded initialisation
  if (kind == HGNN_GC_CGCNN) {
    c->init_tab.push_back(InitTensor{0, H, c->F0, false});
    c->init_tab.push_back(InitTensor{(int64_t)H * c->F0, H, 1, true});
  }
  for (const LayerDesc &d : c->ld) {
    if (kind == HGNN_GC_PNA) {
      c->init_tab.push_back(InitTensor{d.oWm, H, 2 * d.F + c->Fe, false});
      c->init_tab.push_back(InitTensor{d.obm, H, 1, true});
      c->init_tab.push_back(InitTensor{d.oWp, H, d.F + 12 * H, false});
      c->init_tab.push_back(InitTensor{d.obp, H, 1, true});
    } else if (kind == HGNN_GC_SAGE) {
      c->init_tab.push_back(InitTensor{d.oWm, H, 2 * d.F, false});
      c->init_tab.push_back(InitTensor{d.obm, H, 1, true});
    } else {
      c->init_tab.push_back(InitTensor{d.oWm, 2 * H, 2 * H + c->Fe, false});
      c->init_tab.push_back(InitTensor{d.obm, 2 * H, 1, true});
    }
  }
  for (int t = 0; t < Tg + Tn; ++t) {
    const int64_t o = off + (int64_t)t * node_head_size(H);
    c->init_tab.push_back(InitTensor{o, H, H, false});
    c->init_tab.push_back(InitTensor{o + (int64_t)H * H, H, 1, true});
    c->init_tab.push_back(InitTensor{o + (int64_t)H * H + H, 1, H, false});
    c->init_tab.push_back(InitTensor{o + (int64_t)H * H + 2 * H, 1, 1, true});
  }
  c->off_head = off;
  off += (int64_t)Tg * node_head_size(H);
  c->off_node = off;
  off += (int64_t)Tn * node_head_size(H);
  c->P = off;
  if (Tn > 0) {
    c->split_node = tn_splits(H, H + 4, 0);
    part_max = std::max(part_max, (size_t)c->split_node * H * (H + 4));
  }

  hipError_t e = hipGetDevice(&c->dev);
  int ndev = 0;
  if (e == hipSuccess) e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev < 1) {
    delete c;
    return fail(HGNN_EDEVICE, std::string("no HIP device: ") + hipGetErrorString(e));
  }
  // the allocation-free forward's workspace: this device's scratch array,
  // looked up once per device; its pointer vectors are sized here so that
  // carving the workspace allocates nothing on the host either
  if (int rc = noalloc_init(c->dev)) {
    delete c;
    return rc;
  }
  c->na.inference_only = true;
  c->na.w.hbuf.assign(2, nullptr);
  c->na.w.PQ.assign(1, nullptr);
  c->na.w.A.assign(1, nullptr);
  c->na.w.args.assign(1, nullptr);
#define HGNN_CALLOC(p, n)                                                               \
  do {                                                                                 \
    if (dalloc(p, (size_t)(n)) != hipSuccess) {                                         \
      hgnn_destroy(c);                                                                 \
      return fail(HGNN_ENOMEM, std::string("hipMalloc failed for ") + #p);             \
    }                                                                                  \
  } while (0)
  HGNN_CALLOC(c->params, c->P);
  HGNN_CALLOC(c->grads, c->P);
  HGNN_CALLOC(c->adam_m, c->P);
  HGNN_CALLOC(c->adam_v, c->P);
  HGNN_CALLOC(c->step_dev, 1);
  HGNN_CALLOC(c->table, 2 * (c->maxd + 1));
  HGNN_CALLOC(c->ex.dims, 1);
  HGNN_CALLOC(c->ex.w.csr.err, 1);
  HGNN_CALLOC(c->part, part_max);
  if (part_u_max) HGNN_CALLOC(c->part_u, part_u_max);
  if (c->nb) HGNN_CALLOC(c->zscale, 2 * (size_t)zmax);
  HGNN_CALLOC(c->gw_dev, Tg);
  HGNN_CALLOC(c->W1T, (size_t)Tg * H * H);
  if (Tn > 0) {
    HGNN_CALLOC(c->nw_dev, Tn);
    HGNN_CALLOC(c->W1n, (size_t)Tn * H * H);
    HGNN_CALLOC(c->W1nT, (size_t)Tn * H * H);
    HGNN_CALLOC(c->nh_part, node_head_small_floats(H, Tn));
  }
  if (hipMemcpy(c->gw_dev, gw.data(), Tg * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      (Tn > 0 && hipMemcpy(c->nw_dev, nw.data(), Tn * sizeof(float), hipMemcpyHostToDevice) !=
                     hipSuccess)) {
    hgnn_destroy(c);
    return fail(HGNN_EDEVICE, "copying the loss weights failed");
  }
  const size_t esz = c->prec ? 2 : 4;
  if (!pna) {
    // GEMM-layout copies: forward operand Wg1, input-gradient operand Wg2
    // (SAGE: [H, 2Fp] and [2Fp, H]; CGCNN: [4H, H] and [H, 4H]), the CGCNN
    // edge-feature weights [Fe, 2H] (FP32) and embedding [H, F0p]
    for (int l = 0; l < c->L; ++l) {
      const LayerDesc &d = c->ld[l];
      const size_t n = kind == HGNN_GC_SAGE ? (size_t)2 * H * d.Fp : (size_t)4 * H * H;
      uint8_t *p;
      HGNN_CALLOC(p, esz * n);
      c->Wg1.push_back(p);
      HGNN_CALLOC(p, esz * n);
      c->Wg2.push_back(p);
      if (c->prec) {
        HGNN_CALLOC(p, esz * n);
        c->Wg1_lo.push_back(p);
        HGNN_CALLOC(p, esz * n);
        c->Wg2_lo.push_back(p);
      }
      float *we = nullptr;
      if (kind == HGNN_GC_CGCNN && c->Fe > 0) HGNN_CALLOC(we, (size_t)c->Fe * 2 * H);
      c->WeT.push_back(we);
    }
    if (kind == HGNN_GC_CGCNN) {
      uint8_t *p;
      HGNN_CALLOC(p, esz * H * c->F0p);
      c->Wemb = p;
      if (c->prec) {
        HGNN_CALLOC(p, esz * H * c->F0p);
        c->Wemb_lo = p;
      }
    }
    std::vector<GcStageJob> jobs = gc_stage_jobs(c);
    c->gc_njobs = (int)jobs.size();
    c->gc_max_elems = 0;
    for (const GcStageJob &j : jobs)
      c->gc_max_elems = std::max(c->gc_max_elems, (long long)j.rows * j.cols);
    HGNN_CALLOC(c->gc_jobs, jobs.size());
    if (hipMemcpy(c->gc_jobs, jobs.data(), jobs.size() * sizeof(GcStageJob),
                  hipMemcpyHostToDevice) != hipSuccess) {
      hgnn_destroy(c);
      return fail(HGNN_EDEVICE, "copying the staging table failed");
    }
  }
  for (int l = 0; pna && l < c->L; ++l) {
    const LayerDesc &d = c->ld[l];
    // bucketed: the update copies hold one [W_h | W_eff(q)] and one
    // W_eff(q)^T per degree bucket q
    const size_t nbk = c->nb ? (size_t)c->nb : 1;
    const size_t n[4] = {(size_t)2 * H * d.Fp,
                         c->nb ? nbk * H * (d.Fp + 4 * H) : (size_t)H * (d.Fp + 12 * H),
                         c->nb ? nbk * 4 * H * H : (size_t)12 * H * H, (size_t)3 * H * d.Fp};
    std::vector<void *> *hi[4] = {&c->Wds, &c->Wpp, &c->WpTA, &c->WhdsT};
    std::vector<void *> *lo[4] = {&c->Wds_lo, &c->Wpp_lo, &c->WpTA_lo, &c->WhdsT_lo};
    for (int k = 0; k < 4; ++k) {
      uint8_t *p;
      HGNN_CALLOC(p, esz * n[k]);
      hi[k]->push_back(p);
      if (c->prec) {
        HGNN_CALLOC(p, esz * n[k]);
        lo[k]->push_back(p);
      }
    }
    float *we = nullptr;
    if (c->Fe > 0) HGNN_CALLOC(we, (size_t)c->Fe * H);
    c->WeT.push_back(we);
  }
  if (pna) {
    std::vector<StageDesc> tab(c->L);
    for (int l = 0; l < c->L; ++l) {
      const LayerDesc &d = c->ld[l];
      tab[l] = StageDesc{c->params + d.oWm, c->params + d.oWp, d.F, d.Fp, stage_out(c, l)};
    }
    HGNN_CALLOC(c->stage_tab, c->L);
    if (hipMemcpy(c->stage_tab, tab.data(), tab.size() * sizeof(StageDesc),
                  hipMemcpyHostToDevice) != hipSuccess) {
      hgnn_destroy(c);
      return fail(HGNN_EDEVICE, "copying the staging table failed");
    }
  }
#undef HGNN_CALLOC
  // Degree-scaler table: s+(d) = ln(d+1)/delta, s-(d) = delta/ln(d+1) in FP64,
  // rounded once to FP32; d = 0 maps to 0 (the aggregates are 0 there).
  std::vector<float> tab(2 * (c->maxd + 1));
  for (int d = 0; d <= c->maxd; ++d) {
    const double lg = std::log((double)d + 1.0);
    tab[2 * d] = d ? (float)(lg / cfg->delta) : 0.f;
    tab[2 * d + 1] = d ? (float)(cfg->delta / lg) : 0.f;
  }
  e = hipMemcpy(c->table, tab.data(), tab.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(c->params, 0, c->P * sizeof(float));
  if (e == hipSuccess) e = hipMemset(c->grads, 0, c->P * sizeof(float));
  if (e == hipSuccess) e = hipMemset(c->adam_m, 0, c->P * sizeof(float));
  if (e == hipSuccess) e = hipMemset(c->adam_v, 0, c->P * sizeof(float));
  if (e == hipSuccess) e = hipMemset(c->step_dev, 0, sizeof(long long));
  if (e == hipSuccess) e = hipMemset(c->ex.w.csr.err, 0, sizeof(int));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    hgnn_destroy(c);
    return fail(HGNN_EDEVICE, std::string("context init: ") + hipGetErrorString(e));
  }
  if (hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->fork_ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->fork_ev[1], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->stage_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->pjoin_ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->pjoin_ev[1], hipEventDisableTiming) != hipSuccess) {
    hgnn_destroy(c);
    return fail(HGNN_EDEVICE, "stream/event creation failed");
  }
  if (stage_all(c, nullptr) || hipDeviceSynchronize() != hipSuccess) {
    hgnn_destroy(c);
    return fail(HGNN_EDEVICE, "initial weight staging failed");
  }
  *out = c;
  return HGNN_OK;
}

} // namespace hgnn

extern "C" {

void hgnn_destroy(hgnn_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->dev);
  serve_shutdown(c);
  (void)hipDeviceSynchronize();
  free_work(c->ex);
  for (hipEvent_t ev : c->timer.ev) (void)hipEventDestroy(ev);
  c->timer.ev.clear();
  for (hipEvent_t ev : {c->fork_ev[0], c->fork_ev[1], c->join_ev, c->stage_ev, c->pjoin_ev[0],
                        c->pjoin_ev[1]})
    if (ev) (void)hipEventDestroy(ev);
  if (c->aux) (void)hipStreamDestroy(c->aux);
  void **ptrs[] = {(void **)&c->params, (void **)&c->grads, (void **)&c->adam_m,
                   (void **)&c->adam_v, (void **)&c->step_dev, (void **)&c->stage_tab,
                   (void **)&c->gw_dev, (void **)&c->nw_dev, (void **)&c->W1n,
                   (void **)&c->W1nT, (void **)&c->nh_part,
                   (void **)&c->table, (void **)&c->ex.dims, (void **)&c->ex.w.csr.err,
                   (void **)&c->part, (void **)&c->part_u, (void **)&c->zscale, (void **)&c->W1T};
  for (void **p : ptrs) dfree(*p);
  for (auto *v : {&c->Wds, &c->Wpp, &c->WpTA, &c->WhdsT, &c->Wds_lo, &c->Wpp_lo, &c->WpTA_lo,
                  &c->WhdsT_lo, &c->WeT, &c->Wg1, &c->Wg1_lo, &c->Wg2, &c->Wg2_lo})
    for (auto &p : *v) dfree(reinterpret_cast<void *&>(p));
  for (void **p : {(void **)&c->Wemb, (void **)&c->Wemb_lo, (void **)&c->gc_jobs}) dfree(*p);
  delete c;
}

int hgnn_num_params(const hgnn_ctx *c, int64_t *out) {
  if (!c || !out) return fail(HGNN_EINVAL, "ctx and out are required");
  *out = c->P;
  return HGNN_OK;
}

int hgnn_set_params(hgnn_ctx *c, const float *src, void *stream) {
  HGNN_GUARD(c);
  if (!src) return fail(HGNN_EINVAL, "params_dev is NULL");
  hipStream_t s = (hipStream_t)stream;
  if (src != c->params) {
    hipError_t e =
        hipMemcpyAsync(c->params, src, c->P * sizeof(float), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(c, e, "copy params");
  }
  return stage_all(c, s);
}

int hgnn_init_params(hgnn_ctx *c, uint64_t seed, void *stream) {
  HGNN_GUARD(c);
  hipStream_t s = (hipStream_t)stream;
  for (const InitTensor &t : c->init_tab) {
    const int64_t n = (int64_t)t.rows * t.cols;
    const float bound = t.bias ? 0.1f : (float)std::sqrt(6.0 / ((double)t.rows + t.cols));
    hipError_t e = launch_init_uniform(c->params, t.off, n, bound, seed, s);
    if (e != hipSuccess) return hip_fail(c, e, "init params");
  }
  return stage_all(c, s);
}

int hgnn_op_generation(const hgnn_ctx *c, int64_t *out) {
  if (!c || !out) return fail(HGNN_EINVAL, "ctx and out are required");
  *out = c->ex.generation;
  return HGNN_OK;
}

int hgnn_debug_fail_after(hgnn_ctx *c, int32_t n) {
  if (!c || n < 0) return fail(HGNN_EINVAL, "context is NULL or n < 0");
  c->fail_after = n;
  return HGNN_OK;
}

int hgnn_param_views(hgnn_ctx *c, float **params, float **grads) {
  if (!c) return fail(HGNN_EINVAL, "context is NULL");
  if (params) *params = c->params;
  if (grads) *grads = c->grads;
  return HGNN_OK;
}

int hgnn_get_params(hgnn_ctx *c, float *dst, void *stream) {
  HGNN_GUARD(c);
  if (!dst) return fail(HGNN_EINVAL, "params_dev is NULL");
  hipError_t e = hipMemcpyAsync(dst, c->params, c->P * sizeof(float), hipMemcpyDeviceToDevice,
                                (hipStream_t)stream);
  return e == hipSuccess ? HGNN_OK : hip_fail(c, e, "copy params");
}

int hgnn_get_grads(hgnn_ctx *c, float *dst, void *stream) {
  HGNN_GUARD(c);
  if (!dst) return fail(HGNN_EINVAL, "grads_dev is NULL");
  hipError_t e = hipMemcpyAsync(dst, c->grads, c->P * sizeof(float), hipMemcpyDeviceToDevice,
                                (hipStream_t)stream);
  return e == hipSuccess ? HGNN_OK : hip_fail(c, e, "copy grads");
}

int hgnn_check(hgnn_ctx *c, void *stream) {
  HGNN_GUARD(c);
  int bits = 0;
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e == hipSuccess) e = hipMemcpy(&bits, c->ex.w.csr.err, sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(c, e, "check");
  if (bits) return fail(HGNN_EINVAL, decode_err(bits));
  return HGNN_OK;
}

int hgnn_forward(hgnn_ctx *c, const hgnn_batch *b, float *pred, float *loss, int32_t flags,
                 void *stream) {
  HGNN_GUARD(c);
  if (c->Tn > 0) return fail(HGNN_EINVAL, "node heads present: use hgnn_forward_multitask");
  return hgnn_forward_multitask(c, b, nullptr, pred, nullptr, loss, flags, stream);
}

int hgnn_forward_multitask(hgnn_ctx *c, const hgnn_batch *b, const float *y_node,
                           float *pred, float *pred_node, float *loss, int32_t flags,
                           void *stream) {
  HGNN_GUARD(c);
  if (!pred || !b) return fail(HGNN_EINVAL, "batch and pred_dev are required");
  if (c->Tn > 0 && !pred_node) return fail(HGNN_EINVAL, "pred_node_dev is NULL");
  if (loss && (!b->y || (c->Tn > 0 && !y_node)))
    return fail(HGNN_EINVAL, "loss requested without targets");
  hipStream_t s = (hipStream_t)stream;
  Exec &ex = c->ex;
  // Weights changed since they were last staged (an AdamW step): refresh the
  // copies on the aux stream while this batch's CSR is built on s.
  int rc = HGNN_OK;
  const bool fork = !c->staged_from_params;
  if (fork) {
    hipError_t e = hipEventRecord(c->fork_ev[0], s);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->aux, c->fork_ev[0], 0);
    if (e != hipSuccess) return hip_fail(c, e, "fork");
    if ((rc = stage_all(c, c->aux))) return rc;
    if (hipError_t e = hipEventRecord(c->stage_ev, c->aux); e != hipSuccess)
      return hip_fail(c, e, "fork");
  }
  rc = prepare(c, ex, b, flags, s);
  if (fork) { // joined whether or not the batch was accepted
    if (hipError_t e = hipStreamWaitEvent(s, c->stage_ev, 0); e != hipSuccess)
      return hip_fail(c, e, "join");
  }
  if (rc) return rc;
  ex.ynode = y_node;
  const float *h = b->x;
  if (c->kind != HGNN_GC_PNA) {
    rc = gc_forward(c, ex, s, &h);
    if (rc) return rc;
  } else {
    for (int l = 0; l < c->L; ++l) {
      rc = layer_forward(c, ex, l, c->params + c->ld[l].off, h, c->ex.w.hbuf[l], s);
      if (rc) return rc;
      h = c->ex.w.hbuf[l];
    }
  }
  return head_forward(c, ex, c->params + c->off_head, h, b->y, pred, loss, s, pred_node,
                      y_node);
}

int hgnn_backward(hgnn_ctx *c, const float *dpred, void *stream) {
  HGNN_GUARD(c);
  if (!c->ex.prepared) return fail(HGNN_EINVAL, "no forward to differentiate");
  if (!dpred && !c->ex.target) return fail(HGNN_EINVAL, "no targets and no dpred");
  if (dpred && (c->Tg != 1 || c->Tn != 0))
    return fail(HGNN_EINVAL, "dpred_dev needs a single graph head and no node head");
  if (c->Tn > 0 && !c->ex.ynode) return fail(HGNN_EINVAL, "no node targets in the forward");
  if (!c->staged_from_params) return fail(HGNN_EINVAL, "weights changed since the forward");
  hipStream_t s = (hipStream_t)stream;
  Work &w = c->ex.w;
  float *cur = w.dh0, *nxt = w.dh1;
  // the head adjoint already applies the last layer's ReLU adjoint, and each
  // input gradient GEMM applies the one below it
  int rc = head_backward(c, c->ex, c->params + c->off_head, c->ex.target, dpred, cur,
                         c->grads + c->off_head, s, w.hbuf[c->L - 1], w.hbuf[c->L - 1]);
  if (rc) return rc;
  if (c->kind != HGNN_GC_PNA) return gc_backward(c, c->ex, cur, nxt, s);
  if (c->join_pending) { // left by a backward that failed part-way
    c->join_pending = false;
    if (hipError_t e = hipStreamWaitEvent(s, c->join_ev, 0); e != hipSuccess)
      return hip_fail(c, e, "join");
  }
  for (int q = 0; q < 2; ++q)
    if (c->pjoin_pending[q]) {
      c->pjoin_pending[q] = false;
      if (hipError_t e = hipStreamWaitEvent(s, c->pjoin_ev[q], 0); e != hipSuccess)
        return hip_fail(c, e, "join");
    }
  for (int l = c->L - 1; l >= 0; --l) {
    const float *h_in = l ? w.hbuf[l - 1] : c->ex.xin;
    // the last call (l = 0) joins, which orders all weight-gradient work
    rc = layer_backward(c, c->ex, l, c->params + c->ld[l].off, h_in, w.hbuf[l], cur,
                        l ? nxt : nullptr, c->grads + c->ld[l].off, s,
                        /*dh_out_masked=*/true, /*mask_dh_in=*/true,
                        /*defer_join=*/l > 0 && !c->recompute);
    if (rc) return rc;
    std::swap(cur, nxt);
  }
  return HGNN_OK;
}

int hgnn_adam_step(hgnn_ctx *c, float lr, float beta1, float beta2, float eps, float wd,
                   void *stream) {
  HGNN_GUARD(c);
  if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
      !(eps > 0.f) || !(wd >= 0.f))
    return fail(HGNN_EINVAL, "bad AdamW hyperparameters");
  hipStream_t s = (hipStream_t)stream;
  // a previous step's counter advance has not run yet (no forward since):
  // run it before this step reads the counter
  if (c->bump_pending)
    if (int rc = stage_all(c, s)) return rc;
  hipError_t e = launch_adamw(c->params, c->grads, c->adam_m, c->adam_v, c->P, lr,
                              (double)beta1, (double)beta2, eps, wd, c->step_dev, s);
  if (e != hipSuccess) return hip_fail(c, e, "adamw");
  // the weight copies are refreshed, and the counter advanced, by the next
  // forward (on the aux stream, beside its CSR build) or staging call
  c->staged_from_params = false;
  c->bump_pending = true;
  return HGNN_OK;
}

// ---- checkpoint -----------------------------------------------------------
namespace {
struct StateHeader {
  char magic[8];
  hgnn_config cfg;
  int64_t P;
  int64_t step;
};
} // namespace

int hgnn_get_state(hgnn_ctx *c, void *buf, size_t *bytes) {
  if (!c || !bytes) return fail(HGNN_EINVAL, "ctx and bytes are required");
  const size_t need = sizeof(StateHeader) + 3 * (size_t)c->P * sizeof(float);
  if (!buf) {
    *bytes = need;
    return HGNN_OK;
  }
  if (*bytes < need) return fail(HGNN_EINVAL, "state buffer too small");
  HGNN_GUARD(c);
  StateHeader h{};
  std::memcpy(h.magic, "HGNNST01", 8);
  h.cfg = c->cfg;
  h.P = c->P;
  long long step = 0;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(&step, c->step_dev, sizeof(step), hipMemcpyDeviceToHost);
  h.step = step + (c->bump_pending ? 1 : 0); // an AdamW step's advance not yet run
  char *p = reinterpret_cast<char *>(buf);
  std::memcpy(p, &h, sizeof(h));
  p += sizeof(h);
  const size_t n = (size_t)c->P * sizeof(float);
  if (e == hipSuccess) e = hipMemcpy(p, c->params, n, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(p + n, c->adam_m, n, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(p + 2 * n, c->adam_v, n, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(c, e, "get_state");
  *bytes = need;
  return HGNN_OK;
}

int hgnn_set_state(hgnn_ctx *c, const void *buf, size_t bytes) {
  if (!c || !buf) return fail(HGNN_EINVAL, "ctx and buf are required");
  StateHeader h;
  if (bytes < sizeof(h)) return fail(HGNN_EINVAL, "state buffer too small");
  std::memcpy(&h, buf, sizeof(h));
  if (std::memcmp(h.magic, "HGNNST01", 8) != 0) return fail(HGNN_EINVAL, "not an hgnn state");
  if (h.P != c->P || h.cfg.reserved != c->cfg.reserved ||
      h.cfg.num_layers != c->cfg.num_layers || h.cfg.hidden != c->cfg.hidden ||
      h.cfg.node_feat != c->cfg.node_feat || h.cfg.edge_feat != c->cfg.edge_feat)
    return fail(HGNN_EINVAL, "state belongs to a different model shape");
  const size_t n = (size_t)c->P * sizeof(float);
  if (bytes < sizeof(h) + 3 * n) return fail(HGNN_EINVAL, "state buffer truncated");
  (void)hipSetDevice(c->dev);
  hipError_t e = hipDeviceSynchronize();
  c->join_pending = false; // the synchronisation retired any deferred join
  c->pjoin_pending[0] = c->pjoin_pending[1] = false;
  if (e != hipSuccess) (void)hipGetLastError(); // clear a sticky launch error if possible
  const char *p = reinterpret_cast<const char *>(buf) + sizeof(h);
  long long step = h.step;
  e = hipMemcpy(c->params, p, n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->adam_m, p + n, n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->adam_v, p + 2 * n, n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->step_dev, &step, sizeof(step), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(c, e, "set_state");
  c->sticky = 0;
  c->bump_pending = false; // the stored counter already counts every step
  int rc = stage_all(c, nullptr);
  if (rc) return rc;
  e = hipDeviceSynchronize();
  return e == hipSuccess ? HGNN_OK : hip_fail(c, e, "set_state sync");
}

// ---- per-operation entries -------------------------------------------------

int hgnn_op_prepare(hgnn_ctx *c, const hgnn_batch *b, int32_t flags, void *stream) {
  HGNN_GUARD(c);
  return prepare(c, c->ex, b, flags, (hipStream_t)stream);
}

int hgnn_op_layer_forward(hgnn_ctx *c, int32_t l, const float *wl, const float *h_in,
                          float *h_out, void *stream) {
  HGNN_GUARD(c);
  if (c->kind != HGNN_GC_PNA) return fail(HGNN_EINVAL, "per-operation layer entries are PNA-only");
  if (!c->ex.prepared) return fail(HGNN_EINVAL, "call hgnn_op_prepare first");
  if (l < 0 || l >= c->L) return fail(HGNN_EINVAL, "layer out of range");
  if (!wl || !h_in || !h_out) return fail(HGNN_EINVAL, "NULL buffer");
  hipStream_t s = (hipStream_t)stream;
  int rc = stage_layer_from(c, l, wl, s);
  if (rc) return rc;
  return layer_forward(c, c->ex, l, wl, h_in, h_out, s);
}

static int check_generation(const hgnn_ctx *c, int64_t generation) {
  if (generation != c->ex.generation)
    return fail(HGNN_EINVAL, "the batch changed since this forward (generation " +
                                 std::to_string(generation) + ", now " +
                                 std::to_string(c->ex.generation) + "): run the forward again");
  return HGNN_OK;
}

int hgnn_op_layer_backward(hgnn_ctx *c, int64_t generation, int32_t l, const float *wl,
                           const float *h_in, const float *h_out, const float *dh_out,
                           float *dh_in, float *dwl, void *stream) {
  HGNN_GUARD(c);
  if (c->kind != HGNN_GC_PNA) return fail(HGNN_EINVAL, "per-operation layer entries are PNA-only");
  if (!c->ex.prepared) return fail(HGNN_EINVAL, "call hgnn_op_prepare first");
  if (int rc = check_generation(c, generation)) return rc;
  if (l < 0 || l >= c->L) return fail(HGNN_EINVAL, "layer out of range");
  if (!wl || !h_in || !h_out || !dh_out || !dwl) return fail(HGNN_EINVAL, "NULL buffer");
  hipStream_t s = (hipStream_t)stream;
  int rc = stage_layer_from(c, l, wl, s);
  if (rc) return rc;
  return layer_backward(c, c->ex, l, wl, h_in, h_out, dh_out, dh_in, dwl, s);
}

int hgnn_op_head_forward(hgnn_ctx *c, const float *wh, const float *h, const float *target,
                         float *pred, float *loss, void *stream) {
  HGNN_GUARD(c);
  if (!c->ex.prepared) return fail(HGNN_EINVAL, "call hgnn_op_prepare first");
  if (!wh || !h || !pred) return fail(HGNN_EINVAL, "NULL buffer");
  if (loss && !target) return fail(HGNN_EINVAL, "loss requested without targets");
  if (c->Tg != 1 || c->Tn != 0)
    return fail(HGNN_EINVAL, "the per-operation head entries take one graph head only");
  return head_forward(c, c->ex, wh, h, target, pred, loss, (hipStream_t)stream);
}

int hgnn_op_head_backward(hgnn_ctx *c, int64_t generation, const float *wh, const float *h,
                          const float *target, const float *dpred, float *dh, float *dwh,
                          void *stream) {
  HGNN_GUARD(c);
  (void)h;
  if (!c->ex.prepared) return fail(HGNN_EINVAL, "call hgnn_op_prepare first");
  if (int rc = check_generation(c, generation)) return rc;
  if (!wh || !dh || !dwh) return fail(HGNN_EINVAL, "NULL buffer");
  if (!dpred && !target) return fail(HGNN_EINVAL, "need dpred or targets");
  if (c->Tg != 1 || c->Tn != 0)
    return fail(HGNN_EINVAL, "the per-operation head entries take one graph head only");
  return head_backward(c, c->ex, wh, target, dpred, dh, dwh, (hipStream_t)stream);
}

int hgnn_timer_start(hgnn_ctx *c, int32_t site, int32_t max_launches) {
  HGNN_GUARD(c);
  if (site < 0 || site >= SITE_COUNT || max_launches < 0 || max_launches > 1 << 16)
    return fail(HGNN_EINVAL, "bad timer site or launch count");
  SiteTimer &t = c->timer;
  hipError_t e = hipDeviceSynchronize();
  for (hipEvent_t ev : t.ev) (void)hipEventDestroy(ev);
  t.ev.clear();
  t.used = 0;
  t.site = SITE_NONE;
  if (e != hipSuccess) return hip_fail(c, e, "timer sync");
  for (int i = 0; i < 2 * max_launches; ++i) {
    hipEvent_t ev;
    e = hipEventCreate(&ev);
    if (e != hipSuccess) return hip_fail(c, e, "hipEventCreate");
    t.ev.push_back(ev);
  }
  t.site = site;
  return HGNN_OK;
}

int hgnn_timer_read(hgnn_ctx *c, double *total_ms, int32_t *launches) {
  HGNN_GUARD(c);
  if (!total_ms || !launches) return fail(HGNN_EINVAL, "NULL output");
  SiteTimer &t = c->timer;
  double tot = 0.0;
  for (int i = 0; i + 1 < t.used; i += 2) {
    hipError_t e = hipEventSynchronize(t.ev[i + 1]);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.ev[i], t.ev[i + 1]);
    if (e != hipSuccess) return hip_fail(c, e, "timer read");
    tot += ms;
  }
  *total_ms = tot;
  *launches = t.used / 2;
  t.site = SITE_NONE;
  return HGNN_OK;
}

int hgnn_calib_copy(const float *src, float *dst, int64_t n, void *stream) {
  if (!src || !dst || n < 0 || n % 4) return fail(HGNN_EINVAL, "bad copy arguments");
  hipError_t e = launch_calib_copy(src, dst, n, (hipStream_t)stream);
  return e == hipSuccess ? HGNN_OK : fail(HGNN_EDEVICE, hipGetErrorString(e));
}

int hgnn_op_fetch(hgnn_ctx *c, int32_t which, int32_t layer, void *dst, size_t cap,
                  void *stream) {
  HGNN_GUARD(c);
  if (!c->ex.prepared) return fail(HGNN_EINVAL, "nothing prepared");
  if (!dst) return fail(HGNN_EINVAL, "dst is NULL");
  Work &w = c->ex.w;
  const int N = c->ex.N, E = c->ex.E, H = c->H, B = c->ex.B;
  const void *src = nullptr;
  size_t bytes = 0;
  switch (which) {
  case 0: src = w.csr.rowptr; bytes = (N + 1) * 4; break;
  case 1: src = w.csr.csr_src; bytes = (size_t)E * 4; break;
  case 2: src = w.csr.csr_eid; bytes = (size_t)E * 4; break;
  case 3: src = w.csr.deg; bytes = (size_t)N * 4; break;
  case 4: src = w.csr.srcptr; bytes = (N + 1) * 4; break;
  case 5: src = w.csr.t2csr; bytes = (size_t)E * 4; break;
  case 6: src = w.csr.node_graph; bytes = (size_t)N * 4; break;
  case 7:
  case 8: {
    if (c->kind != HGNN_GC_PNA) return fail(HGNN_EINVAL, "fetch ids 7 and 8 are PNA-only");
    if (layer < 0 || layer >= c->L) return fail(HGNN_EINVAL, "layer out of range");
    int slot = layer;
    if (c->recompute) {
      if (w.stored_layer != layer) return fail(HGNN_EINVAL, "layer not stored (recompute on)");
      slot = 0;
    }
    if (which == 7) { src = w.A[slot]; bytes = (size_t)N * 4 * H * 4; }
    else { src = w.args[slot]; bytes = (size_t)N * 2 * H; }
    break;
  }
  case 9: // q of graph head `layer`
    if (layer < 0 || layer >= c->Tg) return fail(HGNN_EINVAL, "graph head out of range");
    src = w.q + (size_t)layer * B * H;
    bytes = (size_t)B * H * 4;
    break;
  case 12: // hidden layer of node head `layer`
    if (layer < 0 || layer >= c->Tn) return fail(HGNN_EINVAL, "node head out of range");
    src = w.Qn + (size_t)layer * N * H;
    bytes = (size_t)N * H * 4;
    break;
  case 10: src = w.g; bytes = (size_t)B * H * 4; break;
  case 11:
    if (layer < 0 || layer >= c->L) return fail(HGNN_EINVAL, "layer out of range");
    src = w.hbuf[layer];
    bytes = (size_t)N * H * 4;
    break;
  default: return fail(HGNN_EINVAL, "unknown fetch id");
  }
  if (cap < bytes) return fail(HGNN_EINVAL, "destination too small");
  if (bytes == 0) return HGNN_OK;
  hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream);
  return e == hipSuccess ? HGNN_OK : hip_fail(c, e, "fetch");
}

} // extern "C"
