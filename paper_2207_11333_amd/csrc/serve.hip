// Step S11: serving with continuous batching.
//
// The paper motivates the surrogate as a fast screen for molecules streamed
// from design workflows (Section 1, Fig. 1).  Requests (each a packed batch
// of molecules, host arrays) are validated and copied into a queue by
// hgnn_serve_submit.  A scheduler thread keeps `lanes` slots; each lane owns
// a stream, device buffers sized to the lane capacity, pinned staging and an
// inference-only execution state, while the weights stay resident and
// shared.  Whenever a lane is free, the scheduler takes queued requests in
// order while they fit the lane, copies them into the lane's staging and
// launches: a packing kernel (request-local ids -> batch-global ids), the CSR
// build, the layers and the pooled head, as a captured HIP graph of the
// smallest capacity bucket that holds the batch (kernels read the live sizes
// from the device header the packing kernel writes).  Lanes run
// concurrently, so a request that arrives while others are on the GPU starts
// as soon as a lane frees up.  The number of lanes is bounded by the HBM
// budget: lanes x lane footprint <= budget.
#include "runtime.hpp"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

namespace hgnn {

namespace {

inline int cdiv(long long a, int b) { return (int)((a + b - 1) / b); }

// Staging layout (int32 words; floats reinterpreted), fixed per lane so that
// the captured graphs see fixed device addresses:
//   header[16]: B, N, E, R
//   req[3 * capB]: per request b_off, n_off, e_off
//   gp[capB]: request-local start node of each graph
//   src[capE], dst[capE]: request-local edge endpoints
//   x[capN * F0], ea[capE * Fe]
struct StageLayout {
  size_t off_req, off_gp, off_src, off_dst, off_x, off_ea, words;
  StageLayout(int capB, int capN, int capE, int F0, int Fe) {
    auto al = [](size_t v) { return (v + 3) / 4 * 4; };
    off_req = 16;
    off_gp = al(off_req + 3 * (size_t)capB);
    off_src = al(off_gp + (size_t)capB);
    off_dst = al(off_src + (size_t)capE);
    off_x = al(off_dst + (size_t)capE);
    off_ea = al(off_x + (size_t)capN * F0);
    words = al(off_ea + (size_t)capE * (Fe > 0 ? Fe : 1));
  }
};

// K10: request-local ids -> batch-global ids, and the device size header.
__global__ void k_serve_pack(const int32_t *__restrict__ st, int off_req, int off_gp,
                             int off_src, int off_dst, Dims *__restrict__ dims,
                             int32_t *__restrict__ graph_ptr, int32_t *__restrict__ ei) {
  const int B = st[0], N = st[1], E = st[2], R = st[3];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t *req = st + off_req;
  if (t == 0) {
    dims->B = B;
    dims->N = N;
    dims->E = E;
    dims->pad = 0;
    graph_ptr[B] = N;
  }
  if (t < B) {
    int lo = 0, hi = R; // last r with b_off[r] <= t
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (req[3 * mid] <= t) lo = mid; else hi = mid;
    }
    graph_ptr[t] = st[off_gp + t] + req[3 * lo + 1];
  }
  if (t < E) {
    int lo = 0, hi = R; // last r with e_off[r] <= t
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (req[3 * mid + 2] <= t) lo = mid; else hi = mid;
    }
    const int n_off = req[3 * lo + 1];
    ei[t] = st[off_src + t] + n_off;
    ei[E + t] = st[off_dst + t] + n_off;
  }
}

struct Req {
  uint64_t ticket = 0;
  int B = 0, N = 0, E = 0;
  std::vector<int32_t> gp, src, dst;
  std::vector<float> x, ea, pred;
  int state = 0; // 0 queued, 1 running, 2 done, 3 failed
  std::string err;
};

struct Bucket {
  int B, N, E;
};

struct Lane {
  Exec ex;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  int32_t *d_stage = nullptr, *h_stage = nullptr;
  int32_t *d_graph_ptr = nullptr, *d_ei = nullptr;
  float *d_pred = nullptr, *h_out = nullptr; // h_out: B preds then the error word
  std::vector<Req *> reqs;
  size_t bytes = 0;
  bool busy = false;
  std::vector<hipGraphExec_t> graphs;
  std::vector<int> graph_state; // 0 not captured, 1 ready, -1 capture failed
};

} // namespace

struct Server {
  hgnn_ctx *c = nullptr;
  hgnn_serve_config cfg{};
  StageLayout lay{1, 1, 1, 1, 0};
  std::vector<std::unique_ptr<Lane>> lanes;
  std::vector<Bucket> buckets;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Req *> queue;
  std::unordered_map<uint64_t, Req *> tickets;
  uint64_t next_ticket = 1;
  std::thread th;
  std::atomic<bool> stop{false};
  int64_t inflight = 0;
  hgnn_serve_stats stats{};
  size_t lane_bytes = 0;
};

namespace {

size_t input_bytes(const hgnn_ctx *c, int B, int N, int E) {
  return 4 * ((size_t)B + 1 + 2 * (size_t)E + (size_t)N * c->F0 + (size_t)E * c->Fe) + 4 * (size_t)B;
}

// Launch one batch on a lane: pack, CSR, layers, head (bucket-sized grids).
int run_batch(Server &S, Lane &ln, const Bucket &bk) {
  hgnn_ctx *c = S.c;
  Exec &ex = ln.ex;
  hipStream_t s = ln.stream;
  ex.B = bk.B;
  ex.N = bk.N;
  ex.E = bk.E;
  ex.graph_ptr = ln.d_graph_ptr;
  const int n = std::max(bk.B, bk.E);
  k_serve_pack<<<cdiv(n > 0 ? n : 1, 256), 256, 0, s>>>(
      ln.d_stage, (int)S.lay.off_req, (int)S.lay.off_gp, (int)S.lay.off_src,
      (int)S.lay.off_dst, ex.dims, ln.d_graph_ptr, ln.d_ei);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(c, e, "serve pack");
  const float *x = reinterpret_cast<const float *>(ln.d_stage + S.lay.off_x);
  const float *ea = c->Fe ? reinterpret_cast<const float *>(ln.d_stage + S.lay.off_ea) : nullptr;
  e = launch_csr_build(ex.dims, bk.B, bk.N, bk.E, ln.d_graph_ptr, ln.d_ei, ea, c->Fe, c->maxd,
                       c->table, ex.w.csr, /*clear_err=*/true, nullptr, 0, nullptr, 0, s);
  if (e != hipSuccess) return hip_fail(c, e, "serve csr build");
  const float *h = x;
  for (int l = 0; l < c->L; ++l) {
    float *out = ex.w.hbuf[l & 1];
    int rc = layer_forward(c, ex, l, c->params + c->ld[l].off, h, out, s);
    if (rc) return rc;
    h = out;
  }
  return head_forward(c, ex, c->params + c->off_head, h, nullptr, ln.d_pred, nullptr, s);
}

int launch_lane(Server &S, Lane &ln, int nb, int nn, int ne) {
  hgnn_ctx *c = S.c;
  // smallest bucket that holds the batch
  size_t bi = 0;
  while (bi + 1 < S.buckets.size() &&
         (nb > S.buckets[bi].B || nn > S.buckets[bi].N || ne > S.buckets[bi].E))
    ++bi;
  const Bucket &bk = S.buckets[bi];
  hipStream_t s = ln.stream;
  // host -> device: the used parts of the staging regions
  const int R = (int)ln.reqs.size();
  auto cp = [&](size_t off, size_t words) {
    if (!words) return hipSuccess;
    return hipMemcpyAsync(ln.d_stage + off, ln.h_stage + off, words * 4, hipMemcpyHostToDevice, s);
  };
  hipError_t e = cp(0, 16);
  if (e == hipSuccess) e = cp(S.lay.off_req, 3 * (size_t)R);
  if (e == hipSuccess) e = cp(S.lay.off_gp, nb);
  if (e == hipSuccess) e = cp(S.lay.off_src, ne);
  if (e == hipSuccess) e = cp(S.lay.off_dst, ne);
  if (e == hipSuccess) e = cp(S.lay.off_x, (size_t)nn * c->F0);
  if (e == hipSuccess && c->Fe) e = cp(S.lay.off_ea, (size_t)ne * c->Fe);
  if (e != hipSuccess) return hip_fail(c, e, "serve upload");
  int rc = HGNN_OK;
  bool launched = false;
  if (S.cfg.use_graphs) {
    if (ln.graph_state[bi] == 0) {
      hipGraph_t gr = nullptr;
      e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        rc = run_batch(S, ln, bk);
        hipError_t e2 = hipStreamEndCapture(s, &gr);
        if (rc == HGNN_OK && e2 == hipSuccess && gr) {
          e2 = hipGraphInstantiate(&ln.graphs[bi], gr, nullptr, nullptr, 0);
          ln.graph_state[bi] = e2 == hipSuccess ? 1 : -1;
        } else {
          ln.graph_state[bi] = -1;
        }
        if (gr) (void)hipGraphDestroy(gr);
        (void)hipGetLastError();
        if (rc != HGNN_OK) c->sticky = 0; // a failed capture is not a device failure
      } else {
        ln.graph_state[bi] = -1;
        (void)hipGetLastError();
      }
    }
    if (ln.graph_state[bi] == 1) {
      e = hipGraphLaunch(ln.graphs[bi], s);
      if (e != hipSuccess) return hip_fail(c, e, "hipGraphLaunch");
      launched = true;
      S.stats.graph_replays++;
    }
  }
  if (!launched) {
    rc = run_batch(S, ln, bk);
    if (rc) return rc;
  }
  // predictions, then the batch's error word in the slot after the largest bucket
  e = hipMemcpyAsync(ln.h_out, ln.d_pred, (size_t)nb * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ln.h_out + S.buckets.back().B, ln.ex.w.csr.err, 4,
                       hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipEventRecord(ln.done, s);
  if (e != hipSuccess) return hip_fail(c, e, "serve download");
  return HGNN_OK;
}

void finish_lane(Server &S, Lane &ln, bool ok, const std::string &why) {
  int err_bits = 0;
  const int capB = S.buckets.back().B;
  std::memcpy(&err_bits, ln.h_out + capB, 4);
  std::lock_guard<std::mutex> g(S.mu);
  int off = 0;
  for (Req *r : ln.reqs) {
    if (ok && !err_bits) {
      r->pred.assign(ln.h_out + off, ln.h_out + off + r->B);
      r->state = 2;
    } else {
      r->state = 3;
      r->err = ok ? decode_err(err_bits) : why;
    }
    off += r->B;
    S.stats.completed++;
  }
  S.inflight -= (int64_t)ln.bytes;
  ln.reqs.clear();
  ln.bytes = 0;
  ln.busy = false;
}

void scheduler(Server *Sp) {
  Server &S = *Sp;
  hgnn_ctx *c = S.c;
  (void)hipSetDevice(c->dev);
  const Bucket top = S.buckets.back();
  while (true) {
    bool progress = false;
    for (auto &lp : S.lanes) {
      Lane &ln = *lp;
      if (!ln.busy) continue;
      hipError_t q = hipEventQuery(ln.done);
      if (q == hipSuccess) {
        // the error word sits after the bucket's predictions
        finish_lane(S, ln, true, "");
        progress = true;
      } else if (q != hipErrorNotReady) {
        finish_lane(S, ln, false, std::string("device failure: ") + hipGetErrorString(q));
        progress = true;
      }
    }
    for (auto &lp : S.lanes) {
      Lane &ln = *lp;
      if (ln.busy) continue;
      int nb = 0, nn = 0, ne = 0;
      {
        std::lock_guard<std::mutex> g(S.mu);
        while (!S.queue.empty()) {
          Req *r = S.queue.front();
          if (nb + r->B > top.B || nn + r->N > top.N || ne + r->E > top.E) break;
          const size_t bytes = work_bytes(c, nb + r->B, nn + r->N, ne + r->E, true) +
                               input_bytes(c, nb + r->B, nn + r->N, ne + r->E);
          if ((int64_t)(S.inflight + bytes) > S.cfg.hbm_budget_bytes && !ln.reqs.empty()) break;
          S.queue.pop_front();
          r->state = 1;
          ln.reqs.push_back(r);
          nb += r->B;
          nn += r->N;
          ne += r->E;
        }
      }
      if (ln.reqs.empty()) break;
      // pack requests into the lane's pinned staging
      int32_t *h = ln.h_stage;
      h[0] = nb;
      h[1] = nn;
      h[2] = ne;
      h[3] = (int)ln.reqs.size();
      int bo = 0, no = 0, eo = 0, ri = 0;
      float *hx = reinterpret_cast<float *>(h + S.lay.off_x);
      float *hea = reinterpret_cast<float *>(h + S.lay.off_ea);
      for (Req *r : ln.reqs) {
        h[S.lay.off_req + 3 * ri] = bo;
        h[S.lay.off_req + 3 * ri + 1] = no;
        h[S.lay.off_req + 3 * ri + 2] = eo;
        std::memcpy(h + S.lay.off_gp + bo, r->gp.data(), (size_t)r->B * 4);
        std::memcpy(h + S.lay.off_src + eo, r->src.data(), (size_t)r->E * 4);
        std::memcpy(h + S.lay.off_dst + eo, r->dst.data(), (size_t)r->E * 4);
        std::memcpy(hx + (size_t)no * c->F0, r->x.data(), r->x.size() * 4);
        if (c->Fe) std::memcpy(hea + (size_t)eo * c->Fe, r->ea.data(), r->ea.size() * 4);
        bo += r->B;
        no += r->N;
        eo += r->E;
        ++ri;
      }
      ln.bytes = work_bytes(c, nb, nn, ne, true) + input_bytes(c, nb, nn, ne);
      {
        std::lock_guard<std::mutex> g(S.mu);
        S.inflight += (int64_t)ln.bytes;
        S.stats.peak_inflight_bytes = std::max<int64_t>(S.stats.peak_inflight_bytes, S.inflight);
        S.stats.batches++;
      }
      ln.busy = true;
      const int rc = launch_lane(S, ln, nb, nn, ne);
      if (rc != HGNN_OK) finish_lane(S, ln, false, hgnn_last_error());
      progress = true;
    }
    {
      std::unique_lock<std::mutex> g(S.mu);
      bool any_busy = false;
      for (auto &lp : S.lanes) any_busy |= lp->busy;
      if (!S.queue.empty() && !progress) {
        bool all_busy = true;
        for (auto &lp : S.lanes) all_busy &= lp->busy;
        if (all_busy) S.stats.admission_waits++;
      }
      if (S.stop && S.queue.empty() && !any_busy) break;
      if (!progress) {
        if (any_busy)
          S.cv.wait_for(g, std::chrono::microseconds(20));
        else
          S.cv.wait_for(g, std::chrono::milliseconds(2),
                        [&] { return S.stop.load() || !S.queue.empty(); });
      }
    }
  }
}

void destroy_lane(Lane &ln) {
  for (size_t i = 0; i < ln.graphs.size(); ++i)
    if (ln.graph_state[i] == 1) (void)hipGraphExecDestroy(ln.graphs[i]);
  free_work(ln.ex);
  if (ln.ex.dims) (void)hipFree(ln.ex.dims);
  if (ln.ex.w.csr.err) (void)hipFree(ln.ex.w.csr.err);
  if (ln.d_stage) (void)hipFree(ln.d_stage);
  if (ln.d_graph_ptr) (void)hipFree(ln.d_graph_ptr);
  if (ln.d_ei) (void)hipFree(ln.d_ei);
  if (ln.d_pred) (void)hipFree(ln.d_pred);
  if (ln.h_stage) (void)hipHostFree(ln.h_stage);
  if (ln.h_out) (void)hipHostFree(ln.h_out);
  if (ln.done) (void)hipEventDestroy(ln.done);
  if (ln.stream) (void)hipStreamDestroy(ln.stream);
}

// Host-side validation of one request (Table 1 layout, request-local ids).
std::string check_request(const hgnn_ctx *c, const hgnn_batch *r) {
  if (r->num_graphs < 1 || r->num_nodes < r->num_graphs || r->num_edges < 0)
    return "request sizes invalid";
  if (!r->graph_ptr || !r->x || (r->num_edges > 0 && !r->edge_index) ||
      (c->Fe > 0 && r->num_edges > 0 && !r->edge_attr))
    return "request pointer missing";
  const int B = r->num_graphs, N = r->num_nodes, E = r->num_edges;
  if (r->graph_ptr[0] != 0 || r->graph_ptr[B] != N) return "graph_ptr must run from 0 to N";
  std::vector<int> ng(N), din(N, 0), dout(N, 0);
  for (int b = 0; b < B; ++b) {
    if (r->graph_ptr[b + 1] <= r->graph_ptr[b]) return "empty graph in request";
    for (int i = r->graph_ptr[b]; i < r->graph_ptr[b + 1]; ++i) ng[i] = b;
  }
  for (int k = 0; k < E; ++k) {
    const int s = r->edge_index[k], d = r->edge_index[E + k];
    if (s < 0 || s >= N || d < 0 || d >= N) return "edge endpoint out of range";
    if (ng[s] != ng[d]) return "edge crosses graphs";
    if (++din[d] > c->maxd || ++dout[s] > c->maxd) return "degree above max_degree";
  }
  // Content is checked here as well: a batch shares one device error word,
  // so a non-finite value found on the device would fail every request
  // packed beside this one.
  const size_t nx = (size_t)N * c->F0;
  for (size_t i = 0; i < nx; ++i)
    if (!std::isfinite(r->x[i])) return "non-finite value in x";
  if (c->Fe > 0 && E > 0) {
    const size_t ne = (size_t)E * c->Fe;
    for (size_t i = 0; i < ne; ++i)
      if (!std::isfinite(r->edge_attr[i])) return "non-finite value in edge_attr";
  }
  return "";
}

} // namespace

void serve_shutdown(hgnn_ctx *c) {
  if (!c || !c->server) return;
  Server *S = c->server;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  if (S->th.joinable()) S->th.join();
  (void)hipDeviceSynchronize();
  for (auto &lp : S->lanes) destroy_lane(*lp);
  for (auto &kv : S->tickets) delete kv.second;
  delete S;
  c->server = nullptr;
}

} // namespace hgnn

using namespace hgnn;

extern "C" {

int hgnn_serve_start(hgnn_ctx *c, const hgnn_serve_config *cfg) {
  if (!c || !cfg) return set_error(HGNN_EINVAL, "ctx and cfg are required");
  if (c->sticky) return set_error(HGNN_ESTATE, "context failed earlier; restore state");
  if (c->server) return set_error(HGNN_EINVAL, "serving already started");
  if (c->Tg != 1 || c->Tn != 0)
    return set_error(HGNN_EINVAL, "serving takes a model with one graph head and no node head");
  if (c->kind != HGNN_GC_PNA) return set_error(HGNN_EINVAL, "serving takes PNA models only");
  if (cfg->max_batch_nodes < 16 || cfg->max_batch_graphs < 1 || cfg->max_batch_edges < 0 ||
      cfg->num_lanes < 1 || cfg->num_lanes > 64 || cfg->queue_capacity < 1 ||
      cfg->hbm_budget_bytes <= 0)
    return set_error(HGNN_EINVAL, "bad serve config");
  hipError_t e = hipSetDevice(c->dev);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  std::unique_ptr<Server> S(new Server());
  S->c = c;
  S->cfg = *cfg;
  const int capB = cfg->max_batch_graphs, capN = cfg->max_batch_nodes;
  const int capE = std::max(cfg->max_batch_edges, 1);
  S->lay = StageLayout(capB, capN, capE, c->F0, c->Fe);
  // capacity buckets: 1/8, 1/4, 1/2 and all of the lane capacity
  for (int d : {8, 4, 2, 1})
    S->buckets.push_back(Bucket{std::max(1, capB / d), std::max(16, capN / d),
                                std::max(1, capE / d)});
  S->lane_bytes = work_bytes(c, capB, capN, capE, true) + S->lay.words * 4 +
                  4 * ((size_t)capB + 1 + 2 * (size_t)capE + (size_t)capB + 16);
  const int fit = (int)std::min<int64_t>(cfg->num_lanes, cfg->hbm_budget_bytes / (int64_t)S->lane_bytes);
  if (fit < 1)
    return set_error(HGNN_EINVAL, "HBM budget is below the footprint of one lane (" +
                                      std::to_string(S->lane_bytes) + " bytes)");
  if (!c->staged_from_params) {
    int rc = stage_all(c, nullptr);
    if (rc) return rc;
  }
  for (int i = 0; i < fit; ++i) {
    std::unique_ptr<Lane> ln(new Lane());
    ln->ex.inference_only = true;
    bool ok = hipStreamCreateWithFlags(&ln->stream, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&ln->done, hipEventDisableTiming) == hipSuccess &&
              hipMalloc((void **)&ln->ex.dims, sizeof(Dims)) == hipSuccess &&
              hipMalloc((void **)&ln->ex.w.csr.err, 256) == hipSuccess &&
              hipMalloc((void **)&ln->d_stage, S->lay.words * 4) == hipSuccess &&
              hipMalloc((void **)&ln->d_graph_ptr, 4 * ((size_t)capB + 1)) == hipSuccess &&
              hipMalloc((void **)&ln->d_ei, 8 * (size_t)capE) == hipSuccess &&
              hipMalloc((void **)&ln->d_pred, 4 * (size_t)capB) == hipSuccess &&
              hipHostMalloc((void **)&ln->h_stage, S->lay.words * 4, hipHostMallocDefault) ==
                  hipSuccess &&
              hipHostMalloc((void **)&ln->h_out, 4 * ((size_t)capB + 4), hipHostMallocDefault) ==
                  hipSuccess;
    if (ok) ok = ensure_work(c, ln->ex, capB, capN, capE) == HGNN_OK;
    if (!ok) {
      destroy_lane(*ln);
      for (auto &lp : S->lanes) destroy_lane(*lp);
      return set_error(HGNN_ENOMEM, "serve lane allocation failed");
    }
    std::memset(ln->h_stage, 0, S->lay.words * 4);
    ln->graphs.assign(S->buckets.size(), nullptr);
    ln->graph_state.assign(S->buckets.size(), 0);
    S->lanes.push_back(std::move(ln));
  }
  e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    for (auto &lp : S->lanes) destroy_lane(*lp);
    return hip_fail(c, e, "serve start");
  }
  S->stats.lanes = (int64_t)S->lanes.size();
  S->stats.lane_bytes = (int64_t)S->lane_bytes;
  Server *raw = S.release();
  c->server = raw;
  raw->th = std::thread(scheduler, raw);
  return HGNN_OK;
}

int hgnn_serve_submit(hgnn_ctx *c, const hgnn_batch *r, uint64_t *ticket) {
  if (!c || !r || !ticket) return set_error(HGNN_EINVAL, "ctx, request and ticket are required");
  Server *S = c->server;
  if (!S) return set_error(HGNN_EINVAL, "serving not started");
  const Bucket &top = S->buckets.back();
  if (r->num_graphs > top.B || r->num_nodes > top.N || r->num_edges > top.E)
    return set_error(HGNN_EAGAIN, "request larger than a lane");
  const std::string why = check_request(c, r);
  if (!why.empty()) return set_error(HGNN_EINVAL, "malformed request: " + why);
  std::unique_ptr<Req> q(new Req());
  q->B = r->num_graphs;
  q->N = r->num_nodes;
  q->E = r->num_edges;
  q->gp.assign(r->graph_ptr, r->graph_ptr + q->B);
  if (q->E) {
    q->src.assign(r->edge_index, r->edge_index + q->E);
    q->dst.assign(r->edge_index + q->E, r->edge_index + 2 * (size_t)q->E);
    if (c->Fe) q->ea.assign(r->edge_attr, r->edge_attr + (size_t)q->E * c->Fe);
  }
  q->x.assign(r->x, r->x + (size_t)q->N * c->F0);
  {
    std::lock_guard<std::mutex> g(S->mu);
    if ((int)S->queue.size() >= S->cfg.queue_capacity)
      return set_error(HGNN_EAGAIN, "serve queue full");
    q->ticket = S->next_ticket++;
    *ticket = q->ticket;
    S->tickets[q->ticket] = q.get();
    S->queue.push_back(q.release());
    S->stats.submitted++;
  }
  S->cv.notify_all();
  return HGNN_OK;
}

int hgnn_serve_poll(hgnn_ctx *c, uint64_t ticket, float *pred, int32_t *done) {
  if (!c || !done) return set_error(HGNN_EINVAL, "ctx and done are required");
  Server *S = c->server;
  if (!S) return set_error(HGNN_EINVAL, "serving not started");
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->tickets.find(ticket);
  if (it == S->tickets.end()) return set_error(HGNN_EINVAL, "unknown ticket");
  Req *r = it->second;
  if (r->state == 2) {
    if (pred) std::memcpy(pred, r->pred.data(), r->pred.size() * 4);
    *done = 1;
    S->tickets.erase(it);
    delete r;
    return HGNN_OK;
  }
  if (r->state == 3) {
    const std::string msg = "request failed: " + r->err;
    S->tickets.erase(it);
    delete r;
    *done = 1;
    return set_error(HGNN_EINVAL, msg);
  }
  *done = 0;
  return HGNN_OK;
}

int hgnn_serve_stats_get(hgnn_ctx *c, hgnn_serve_stats *out) {
  if (!c || !out) return set_error(HGNN_EINVAL, "ctx and out are required");
  Server *S = c->server;
  if (!S) return set_error(HGNN_EINVAL, "serving not started");
  std::lock_guard<std::mutex> g(S->mu);
  *out = S->stats;
  return HGNN_OK;
}

int hgnn_serve_stop(hgnn_ctx *c) {
  if (!c) return set_error(HGNN_EINVAL, "ctx is NULL");
  serve_shutdown(c);
  return HGNN_OK;
}

} // extern "C"
