// Context layout shared by the training runtime and the serving scheduler.
#pragma once

#include "common.hpp"
#include "hgnn.h"

#include <string>
#include <vector>

namespace hgnn {


struct LayerDesc {
  int F, Fp;                       // input width and its padding to 16
  int64_t off, oWm, obm, oWp, obp; // offsets into the packed vector
  int64_t size;
  int split_p, split_m;            // split-K counts of the two weight gradients
  int split_m2;                    // message weight gradient without the De rows
};

// Capacity-sized device buffers of one batch.
struct Work {
  int capB = 0, capN = 0, capE = 0;
  CsrBufs csr{};
  float *xpad = nullptr;                 // [N, F0p] padded layer-0 input
  std::vector<float *> hbuf;             // [L] layer outputs [N, H]
  // BF16 copies of the layer outputs [L][N, H] and of one layer's aggregates
  // [N, 4H], read by the BF16 linears (gemm_ntb.hip); training batches of
  // bucketed BF16 PNA models only (empty / null otherwise)
  std::vector<__bf16 *> hbuf_b;
  __bf16 *Ab = nullptr;
  std::vector<float *> PQ, A;            // [L] (or 1 with recompute)
  std::vector<uint8_t *> args;
  int stored_layer = -1;                 // layer held by the shared slot
  float *g = nullptr, *q = nullptr, *ypred = nullptr, *dy = nullptr, *dq = nullptr;
  float *du = nullptr, *dA = nullptr, *dm = nullptr;
  float *D = nullptr;                    // [N, (2 + Fe) H] = [D_in | D_out | De]
  float *D2 = nullptr;                   // odd layers' D (deferred joins, no recompute)
  float *dh0 = nullptr, *dh1 = nullptr;
  float *ntpart = nullptr;               // split-K partials of the NT GEMMs
  // node heads: outputs [N, Tn], hidden [Tn][N][H], its adjoint, errors
  // [N, Tn], and their share of dL/dh [N, H]
  float *zn = nullptr, *Qn = nullptr, *dQn = nullptr, *en = nullptr, *dhn = nullptr;
  // GraphSAGE / CGCNN: per layer the neighbour means M [N, Fp] (SAGE) or the
  // gate halves PQ [N, 4H] (CGCNN); the CGCNN embedding h0 [N, H]; SAGE's
  // input-gradient product G [N, 2H]; CGCNN's D [N, (4 + 2Fe) H] and per-edge
  // gate gradients dm [E, 2H]
  std::vector<float *> gcA;
  float *h0 = nullptr, *gcG = nullptr, *gcD = nullptr, *gcdm = nullptr;
  float *gcD1 = nullptr; // CGCNN: D of odd layers (even layers use gcD)
};

// Batch-local execution state: device size header, CSR, activations and
// workspaces of one batch.  The training path owns one; every serving lane
// owns another, so lanes run concurrently against the shared weights.
struct Exec {
  Work w;
  Dims *dims = nullptr;
  int B = 0, N = 0, E = 0;
  const int *graph_ptr = nullptr;
  const float *xin = nullptr, *target = nullptr;
  const float *ynode = nullptr;  // node-level targets [N, Tn] of the last forward
  bool prepared = false;
  int64_t generation = 0;       // advanced by every prepare (new batch state)
  bool x_padded = false;        // w.xpad holds xin, zero-padded (written at prepare)
  bool inference_only = false;  // no backward buffers, two rotating h slots
};

struct Server;

// One tensor of the packed parameter vector, for the seeded initialisation:
// weights [rows, cols] are Xavier-uniform, biases U(-0.1, 0.1).
struct InitTensor {
  int64_t off;
  int rows, cols;
  bool bias;
};

// packed size of one head: W1 [H, H], b1 [H], w2 [H], b2 [1]
inline size_t node_head_size(int H) { return (size_t)H * H + 2 * (size_t)H + 1; }

// Launch sites that the opt-in event timer can bracket.
enum Site : int {
  SITE_NONE = 0,
  SITE_MESSAGE_GEMM = 1,   // S1
  SITE_AGGREGATE = 2,      // S2
  SITE_UPDATE_GEMM = 3,    // S3
  SITE_UPDATE_WGRAD = 4,   // S6 weight gradient (split-K GEMM)
  SITE_AGG_INPUT_GEMM = 5, // S6 gradient of the aggregates
  SITE_AGGREGATE_BWD = 6,  // S7 per-edge adjoint
  SITE_INPUT_GEMM = 7,     // S6+S8 input gradient
  SITE_MESSAGE_WGRAD = 8,  // S8 weight gradient (split-K GEMM)
  SITE_CSR = 9,            // S0 CSR build (all of its launches)
  SITE_COUNT = 10
};

struct SiteTimer {
  int site = SITE_NONE;
  std::vector<hipEvent_t> ev; // pairs
  int used = 0;
};

} // namespace hgnn

struct hgnn_ctx {
  hgnn_config cfg{};
  int dev = 0;
  int kind = HGNN_GC_PNA; // GC layer kind
  int L = 0, H = 0, F0 = 0, F0p = 0, Fe = 0, maxd = 0, prec = 0, recompute = 0;
  // degree buckets of the update linear: max_degree + 1 when that is at most
  // kMaxBuckets (PNA), else 0 (the concatenated form)
  int nb = 0;
  int64_t P = 0, off_head = 0;
  std::vector<hgnn::LayerDesc> ld;
  std::vector<hgnn::InitTensor> init_tab; // packing order
  float *params = nullptr, *grads = nullptr, *adam_m = nullptr, *adam_v = nullptr;
  long long *step_dev = nullptr;
  hgnn::StageDesc *stage_tab = nullptr; // device table for the one-launch weight staging
  // heads: Tg graph-level (packed from off_head), Tn node-level (from
  // off_node); loss weights on the device (null = all 1); aligned node-head
  // weight copies for the GEMMs
  int Tg = 1, Tn = 0;
  int64_t off_node = 0;
  int split_node = 1; // split-K count of a node head's weight-gradient GEMM
  float *gw_dev = nullptr, *nw_dev = nullptr;
  float *W1n = nullptr, *W1nT = nullptr;
  float *nh_part = nullptr; // node heads' per-chunk dw2/db2 partials
  float *table = nullptr;
  std::vector<void *> Wds, Wpp, WpTA, WhdsT; // GEMM-layout weight copies per layer
  std::vector<void *> Wds_lo, Wpp_lo, WpTA_lo, WhdsT_lo; // BF16 low halves
  std::vector<void *> WeT; // per layer [Fe, H] (CGCNN [Fe, 2H]) edge-feature weights (FP32)
  // GraphSAGE / CGCNN GEMM-layout copies per layer (forward B operand and
  // input-gradient B operand; BF16 low halves), the CGCNN embedding, and the
  // one-launch staging table that refreshes them
  std::vector<void *> Wg1, Wg1_lo, Wg2, Wg2_lo;
  void *Wemb = nullptr, *Wemb_lo = nullptr;
  int64_t off_emb = 0;
  int split_emb = 1;
  hgnn::GcStageJob *gc_jobs = nullptr;
  int gc_njobs = 0;
  long long gc_max_elems = 0;
  bool staged_from_params = false;
  float *part = nullptr;
  float *part_u = nullptr; // the update weight gradient's split-K partials
  float *zscale = nullptr; // per-chunk scalers of the bucketed update weight gradient
  float *W1T = nullptr;    // graph heads' W1 transposed [Tg][H][H] (staged with the layers)
  hgnn::Exec ex; // the training path's batch state
  // batch state of hgnn_forward_noalloc: its buffers are carved from the
  // device's scratch array (noalloc.hip) and never freed
  hgnn::Exec na;
  int sticky = 0;
  int fail_after = 0; // test-only failure injection (hgnn_debug_fail_after)
  hgnn::Server *server = nullptr;
  hgnn::SiteTimer timer;
  // The backward pass runs the weight-gradient GEMMs on this stream,
  // concurrently with the input-gradient chain (event fork/join).
  hipStream_t aux = nullptr;
  hipEvent_t fork_ev[2] = {nullptr, nullptr}, join_ev = nullptr;
  // the main stream has not yet waited for join_ev (a deferred layer join)
  bool join_pending = false;
  // The weight copies are refreshed on the aux stream while the next batch's
  // CSR is built (stage_ev marks the end); AdamW's step counter is advanced
  // by that refresh, which is pending after an AdamW step until it runs.
  hipEvent_t stage_ev = nullptr;
  bool bump_pending = false;
  // PNA backward: the end of layer l's weight-gradient work (aux) is marked
  // by pjoin_ev[l & 1]; the main stream waits for it before the first of its
  // launches that overwrites what that work reads (layer l - 2's aggregation
  // adjoint rewrites D of the same parity, layer l - 1's input gradient GEMM
  // rewrites layer l's du)
  hipEvent_t pjoin_ev[2] = {nullptr, nullptr};
  bool pjoin_pending[2] = {false, false};
};

namespace hgnn {

int set_error(int code, const std::string &msg);
int hip_fail(hgnn_ctx *c, hipError_t e, const char *what);
std::string decode_err(int bits);
void serve_shutdown(hgnn_ctx *c);

// forward-path building blocks shared by training and serving
int ensure_work(hgnn_ctx *c, Exec &ex, int B, int N, int E);
// Point every inference buffer of ex into [base, base + bytes) (256-byte
// aligned pieces, nothing allocated): the bytes used, 0 if they do not fit.
size_t carve_work(const hgnn_ctx *c, Exec &ex, int B, int N, int E, char *base,
                  size_t bytes);
int check_batch_host(hgnn_ctx *c, const hgnn_batch *b);
// Look up this device's scratch array of the allocation-free forward (once
// per device; the device must be current).
int noalloc_init(int dev);
void free_work(Exec &ex);
size_t work_bytes(const hgnn_ctx *c, int B, int N, int E, bool inference_only);
int layer_forward(hgnn_ctx *c, Exec &ex, int l, const float *wl, const float *h_in,
                  float *h_out, hipStream_t s);
// graph heads, node heads (fused path: pred_node/ynode), weighted loss
int head_forward(hgnn_ctx *c, Exec &ex, const float *wh, const float *h,
                 const float *target, float *pred, float *loss, hipStream_t s,
                 float *pred_node = nullptr, const float *ynode = nullptr);
// Refresh every layer's GEMM-layout weight copies from the parameters in one
// launch; AdamW's step counter is advanced by it when an AdamW step left that
// pending (bump_pending).
int stage_all(hgnn_ctx *c, hipStream_t s);

// Records an event pair around one launch when the timer watches `site`.
// Only the training path's launches are timed (serving lanes never are).
// RAII form: the pair brackets everything launched in the scope.  Manual
// form: start()/stop() hand the pair to a launcher that binds it to one
// kernel's dispatch, so the pair measures that kernel's duration alone.
struct TimedLaunch {
  hgnn_ctx *c;
  hipStream_t s;
  bool on, manual;
  TimedLaunch(hgnn_ctx *c_, const Exec &ex, int site, hipStream_t s_, bool manual_ = false)
      : c(c_), s(s_), on(false), manual(manual_) {
    SiteTimer &t = c->timer;
    if (&ex == &c->ex && t.site == site && t.used + 2 <= (int)t.ev.size()) {
      on = true;
      if (!manual) (void)hipEventRecord(t.ev[t.used], s);
    }
  }
  ~TimedLaunch() {
    if (on) {
      SiteTimer &t = c->timer;
      if (!manual) (void)hipEventRecord(t.ev[t.used + 1], s);
      t.used += 2;
    }
  }
  hipEvent_t start() const { return on ? c->timer.ev[c->timer.used] : nullptr; }
  hipEvent_t stop() const { return on ? c->timer.ev[c->timer.used + 1] : nullptr; }
};

} // namespace hgnn
