/*
 * hgnn.h - C-ABI of the MI355X (gfx950) PNA-style GCNN hot path.
 *
 * The library trains and serves the graph-convolutional surrogate of Choi et
 * al., "Scalable training of graph convolutional neural networks for fast and
 * accurate predictions of HOMO-LUMO gap in molecules": a stack of PNA graph
 * convolution layers (Section 3.1; 6 layers in Section 5.1), global mean
 * pooling (Section 3.1), fully connected layers (Sections 3.1-3.2), the MSE
 * loss, the backward phase and the AdamW optimiser step (Section 3.2, Section
 * 5.1).  Graphs come in the layout of Table 1: x (#nodes, #node features),
 * edge_index (2, #edges) with row 0 the source and row 1 the destination,
 * edge_attr (#edges, #edge features) and one graph-level target per graph.
 *
 * Layer definition (the paper names PNA without defining it; this is the
 * reading the library implements), for layer l with input width F:
 *   m_k   = W^m [h_dst(k) || h_src(k) || e_k] + b^m                   (H wide)
 *   A_i   = [mean || min || max || std] of m_k over in-edges of node i,
 *           std = sqrt(population variance + std_eps)
 *   s+_i  = ln(d_i + 1) / delta,  s-_i = delta / ln(d_i + 1)   (0 if d_i = 0)
 *   h'_i  = ReLU(W^p [h_i || A_i || s+_i A_i || s-_i A_i] + b^p)
 * then g_b = mean of h over graph b, y_b = w2 ReLU(W1 g_b + b1) + b2 and
 * loss = mean over graphs of (y_b - t_b)^2.  A min/max gradient goes to the
 * first in-edge in (source id, edge id) order that attains the extremum.
 *
 * Parameter packing (interchange and checkpoint order, row-major [out, in]):
 * per layer W^m [H, 2F+Fe], b^m [H], W^p [H, F+12H], b^p [H]; then W1 [H, H],
 * b1 [H], w2 [1, H], b2 [1].  F = node_feat for the first layer, H after.
 *
 * Conventions
 *  - Every pointer argument named *_dev is device memory; *_host is host
 *    memory.  Streams are hipStream_t passed as void* (NULL = default stream).
 *  - All calls are asynchronous on the given stream unless stated otherwise.
 *    The caller keeps every buffer it passes alive until that stream work is
 *    done.  The context owns its parameters, gradients, optimiser moments,
 *    CSR arrays, activation store and workspaces.
 *  - Status: 0 on success, a negative HGNN_E* code otherwise; nothing aborts.
 *    hgnn_last_error() returns a thread-local message for the last failure.
 *    Size and pointer checks are done on the host and return HGNN_EINVAL
 *    synchronously.  Content checks (edge endpoint out of range, edge across
 *    graphs, in- or out-degree above max_degree, empty graph, a NaN or
 *    infinity in x or edge_attr) are done on the device and set the
 *    context's error word: with HGNN_VALIDATE the call synchronises and
 *    returns HGNN_EINVAL; otherwise hgnn_check() reports it.
 *    A failed HIP call puts the context in HGNN_ESTATE until hgnn_set_state.
 *  - Gradients overwrite (never accumulate) and refer to the last forward.
 *  - Train calls on one context are not thread-safe; serve calls are.
 *  - Indices are int32: num_nodes and num_edges must be below 2^31.
 */
#ifndef HGNN_H
#define HGNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HGNN_OK = 0,
  HGNN_EINVAL = -1,  /* bad argument or malformed batch */
  HGNN_ENOMEM = -2,  /* device or host allocation failed */
  HGNN_EDEVICE = -3, /* a HIP call failed (no device, launch failure) */
  HGNN_EAGAIN = -4,  /* serving: queue full or request above the budget */
  HGNN_ESTATE = -5   /* context unusable after a device failure */
};

enum { HGNN_VALIDATE = 1 }; /* forward flag: synchronise and check content */
enum { HGNN_PREC_FP32 = 0, HGNN_PREC_BF16 = 1 };
/* GC layer kinds (Section 2 names PNA, CGCNN and GraphSAGE as the kinds
 * HydraGNN implements; the paper's runs use PNA). */
enum { HGNN_GC_PNA = 0, HGNN_GC_SAGE = 1, HGNN_GC_CGCNN = 2 };

typedef struct hgnn_ctx hgnn_ctx;

typedef struct {
  int32_t num_layers; /* L >= 1 */
  int32_t hidden;     /* H: multiple of 16, 16..512 */
  int32_t node_feat;  /* F0 >= 1 */
  int32_t edge_feat;  /* Fe in 0..4 */
  int32_t max_degree; /* 1..255; in- and out-degree bound of every node */
  int32_t precision;  /* HGNN_PREC_FP32: FP32 linears; HGNN_PREC_BF16: linear
                         operands rounded to BF16 (RNE), FP32 accumulation;
                         aggregation, scalers, pooling and loss stay FP32 */
  int32_t recompute;  /* 1: keep only layer inputs; the backward pass re-runs
                         the message linear and the aggregation per layer */
  int32_t reserved;
  double delta;       /* PNA degree normaliser (mean ln(d+1) of a calibration
                         set); a model constant, never recomputed per batch */
  double std_eps;     /* added to the variance inside the std aggregator */
} hgnn_config;

typedef struct {
  int32_t num_graphs, num_nodes, num_edges; /* B >= 1, N >= B, E >= 0 */
  int32_t reserved;
  const int32_t *graph_ptr; /* [B+1]; graph b owns nodes [ptr[b], ptr[b+1]) */
  const float *x;           /* [N, node_feat] */
  const int32_t *edge_index;/* [2, E]: row 0 sources, row 1 destinations,
                               global node ids; any order */
  const float *edge_attr;   /* [E, edge_feat], NULL iff edge_feat == 0 */
  const float *y;           /* [B] targets, or NULL when no loss is wanted */
} hgnn_batch;

/* ---- context ------------------------------------------------------------ */

/* Validate cfg, select the current HIP device, allocate the context and set
 * the parameters (the trainable weights of the layers, pooling head and loss
 * of Sections 3.1-3.2): from init_params_dev (device [P] in packing order,
 * copied; the caller keeps ownership) or, when it is NULL, by
 * hgnn_init_params(seed).  The parameter work runs on `stream`.  *out is NULL
 * after any failure.  EINVAL for a bad config (checked before any device
 * call), EDEVICE/ENOMEM otherwise. */
int hgnn_create(const hgnn_config *cfg, const float *init_params_dev, uint64_t seed,
                void *stream, hgnn_ctx **out);
/* Seeded initialisation of the packed parameters on the device, in packing
 * order: weights [rows, cols] Xavier-uniform with bound sqrt(6/(rows+cols)),
 * biases with bound 0.1.  Element j (index into the packed vector) takes
 * bound * k * 2^-23, k = (z >> 40) - 2^23, z the j-th output of SplitMix64
 * from `seed` (Steele, Lea and Flood, 2014): z = mix(seed + (j + 1) *
 * 0x9E3779B97F4A7C15) with mix(z) = z ^= z >> 30, z *= 0xBF58476D1CE4E5B9,
 * z ^= z >> 27, z *= 0x94D049BB133111EB, z ^= z >> 31 -- a counter
 * generator, reproducible on the host bit for bit.  Moments and the step
 * count are left as they are; the GEMM copies are refreshed. */
int hgnn_init_params(hgnn_ctx *ctx, uint64_t seed, void *stream);

/* Multitask heads (HydraGNN's multi-headed outputs; the paper's model has one
 * graph-level head, which is what hgnn_create builds).  graph_heads Tg in 1..8
 * graph-level heads on the pooled embedding, node_heads Tn in 0..4
 * node-level heads on every node's last-layer embedding, each head
 * Linear(H,H)-ReLU-Linear(H,1).  Loss = sum_t graph_weights[t] mean_b
 * (y[b,t] - Y[b,t])^2 + sum_s node_weights[s] mean_i (z[i,s] - Z[i,s])^2
 * (weight arrays are host memory, >= 0, NULL = all 1).  Packed parameters:
 * the layers, then the Tg graph heads, then the Tn node heads, each head
 * W1 [H,H], b1 [H], w2 [1,H], b2 [1].  Such a model is trained through
 * hgnn_forward_multitask, hgnn_backward (no dpred) and hgnn_adam_step;
 * serving and the per-operation head entries take single-head models only.
 * The config's `reserved` field records (Tg, Tn) and is part of a
 * checkpoint's identity. */
typedef struct {
  int32_t graph_heads, node_heads;
  int32_t reserved[2];
  const float *graph_weights; /* host [graph_heads] or NULL */
  const float *node_weights;  /* host [node_heads] or NULL */
} hgnn_heads;
int hgnn_create_multitask(const hgnn_config *cfg, const hgnn_heads *heads,
                          hgnn_ctx **out);

/* A model whose GC layers are of another kind (heads NULL: one graph head).
 * HGNN_GC_PNA is hgnn_create_multitask.  The others (cfg->delta is unused;
 * recompute must be 0; serving and the per-operation layer entries reject
 * them; hgnn_op_fetch ids 7 and 8 are PNA-only):
 *  HGNN_GC_SAGE   GraphSAGE, mean aggregator (Hamilton et al., 2017):
 *                 M_i = mean of h_j over the in-edges j -> i (0 without
 *                 in-edges), h'_i = ReLU(W_self h_i + W_nbr M_i + b).
 *                 Packed per layer: W [H, 2F] = [W_self | W_nbr], b [H].
 *  HGNN_GC_CGCNN  CGCNN (Xie and Grossman, 2018): h0 = W_emb x + b_emb, then
 *                 per layer, for every in-edge j -> i with z = [h_i || h_j ||
 *                 e_ij]: f = W_f z + b_f, s = W_s z + b_s, and h'_i =
 *                 ReLU(h_i + sum sigmoid(f) * softplus(s)).  Packed: W_emb
 *                 [H, F0], b_emb [H], then per layer W [2H, 2H + Fe] (rows
 *                 0..H-1 the filter f, H..2H-1 the core s) and b [2H].
 * Every layer ends in ReLU; batch normalisation is not applied.  The heads
 * follow the layers as for PNA.  The kind is part of a checkpoint's
 * identity (recorded in the config's `reserved` field). */
int hgnn_create_gc(const hgnn_config *cfg, int32_t kind, const hgnn_heads *heads,
                   hgnn_ctx **out);
void hgnn_destroy(hgnn_ctx *ctx); /* synchronises; NULL is ignored */
int hgnn_num_params(const hgnn_ctx *ctx, int64_t *out);
/* Copy the packed parameters in (device [P]) and refresh the internal GEMM
 * copies (padded, transposed, BF16 when precision is BF16).  Given the
 * context's own parameter vector (from hgnn_param_views) it copies nothing
 * and only refreshes the copies. */
int hgnn_set_params(hgnn_ctx *ctx, const float *params_dev, void *stream);
int hgnn_get_params(hgnn_ctx *ctx, float *params_dev, void *stream);
int hgnn_get_grads(hgnn_ctx *ctx, float *grads_dev, void *stream);
/* The context's own packed parameter and gradient vectors (device [P] each,
 * owned by the context, valid until hgnn_destroy; either output may be
 * NULL).  Gradients are rewritten by every hgnn_backward.  Parameters written
 * through the pointer reach the layers only after hgnn_set_params(ctx,
 * *params, stream); until then the forward pass uses the previous values. */
int hgnn_param_views(hgnn_ctx *ctx, float **params_dev, float **grads_dev);
/* Test hook for the failure path: the n-th layer call (forward or backward,
 * any layer kind) from now on returns HGNN_EDEVICE without launching, as a
 * failed launch would, and the context stays in HGNN_ESTATE until
 * hgnn_set_state.  n = 0 disables it.  For tests of callers' recovery. */
int hgnn_debug_fail_after(hgnn_ctx *ctx, int32_t n);
/* Synchronise the stream and report the device error word (EINVAL with a
 * message naming the first failed check) or a sticky ESTATE. */
int hgnn_check(hgnn_ctx *ctx, void *stream);

/* ---- training path (Section 3.2: forward, backward, optimiser) ---------- */

/* Build the CSR of the batch and run every layer, the pooling and the head.
 * pred_dev [B] receives y; loss_dev [1] (optional, needs batch->y) the MSE.
 * The context keeps what the backward pass needs (and a pointer to batch
 * buffers: keep them alive until hgnn_backward is done). */
int hgnn_forward(hgnn_ctx *ctx, const hgnn_batch *batch, float *pred_dev,
                 float *loss_dev, int32_t flags, void *stream);
/* Forward of a multitask model: batch->y is [B, Tg] (row-major), y_node_dev
 * [N, Tn] (device; NULL when no loss is wanted), pred_dev [B, Tg],
 * pred_node_dev [N, Tn] (required when Tn > 0).  The targets must stay
 * valid until hgnn_backward.  hgnn_forward is this call with Tn = 0. */
int hgnn_forward_multitask(hgnn_ctx *ctx, const hgnn_batch *batch,
                           const float *y_node_dev, float *pred_dev,
                           float *pred_node_dev, float *loss_dev, int32_t flags,
                           void *stream);
/* Gradients of the loss of the last forward (dpred_dev == NULL, needs
 * batch->y) or of sum(dpred * y) (dpred_dev [B]) into the context's packed
 * gradient vector. */
int hgnn_backward(hgnn_ctx *ctx, const float *dpred_dev, void *stream);
/* One AdamW step (decoupled decay, bias-corrected, step count kept by the
 * context starting at 1) on the packed parameters with the current
 * gradients (Section 5.1 trains with AdamW).  The internal GEMM copies of the
 * weights are refreshed by the next call that needs them (the next forward
 * does it on a second stream, beside its CSR build). */
int hgnn_adam_step(hgnn_ctx *ctx, float lr, float beta1, float beta2,
                   float eps, float weight_decay, void *stream);

/* ---- allocation-free inference forward ---------------------------------- */
/* For callers that cannot allocate device memory: code under HIP stream
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The forward
 * pass of hgnn_forward (same kernels; no activations are kept for a backward
 * pass) for a PNA model without node heads, whose whole batch workspace (size
 * header, error word, CSR, padded input, two rotating layer outputs, one
 * layer's messages and aggregates, head buffers, split-K partials) lies in one
 * static device array of the library: hgnn_noalloc_max_bytes() = 64 MiB,
 * held by each GPU the library runs on until the process ends.  The call
 * allocates nothing, on the device or the host, outside its error paths.
 * pred_dev [B] and loss_dev [1] (optional, needs batch->y) as in
 * hgnn_forward; flags as there (HGNN_VALIDATE synchronises).  EINVAL, with
 * nothing launched, when the batch needs more than the array holds
 * (hgnn_noalloc_bytes gives the need: 27.6 MB for 128 molecules of 4.5k atoms
 * at H = 128, 6 layers).  The array is shared by every call on one GPU
 * and keeps the last call's contents: calls that overlap on one GPU race,
 * whatever their context or stream.  The context's training state (the last
 * hgnn_forward, the gradients) is left alone. */
int hgnn_forward_noalloc(hgnn_ctx *ctx, const hgnn_batch *batch, float *pred_dev,
                         float *loss_dev, int32_t flags, void *stream);
/* Workspace bytes hgnn_forward_noalloc needs for a batch of these sizes. */
int hgnn_noalloc_bytes(const hgnn_ctx *ctx, int32_t num_graphs, int32_t num_nodes,
                       int32_t num_edges, int64_t *out);
int64_t hgnn_noalloc_max_bytes(void);

/* ---- checkpoint --------------------------------------------------------- */

/* Serialise config, step count, parameters and AdamW moments into a host
 * buffer.  With buf_host == NULL only *bytes is set.  Synchronises. */
int hgnn_get_state(hgnn_ctx *ctx, void *buf_host, size_t *bytes);
/* Restore a state written by hgnn_get_state for the same config; clears
 * HGNN_ESTATE.  Synchronises. */
int hgnn_set_state(hgnn_ctx *ctx, const void *buf_host, size_t bytes);

/* ---- per-operation entries (used by the autograd bindings) -------------- */
/* The forward pass of Section 3.1 (message passing, pooling, FC head) and the
 * backward phase of Section 3.2, one step at a time with explicit buffers.
 * w_layer_dev points at one layer's packed slice [W^m, b^m, W^p, b^p];
 * w_head_dev at [W1, b1, w2, b2]; dw_* receive gradients in the same
 * packing (overwritten).  A backward entry differentiates the forward of the
 * batch prepared last: it takes the generation that hgnn_op_generation
 * returned after that prepare and returns EINVAL, writing nothing, if
 * another batch has been prepared since (a second forward before the first
 * one's backward). */

/* Step S0 (Table 1 layout in; node degree for the PNA scalers, Section 3.1):
 * validate sizes, copy x into the padded layer-0 input and build the
 * destination-sorted CSR, its by-source transpose and the per-node scalers.
 * Advances the context's batch generation. */
int hgnn_op_prepare(hgnn_ctx *ctx, const hgnn_batch *batch, int32_t flags,
                    void *stream);
/* The batch generation: a count of prepares (hgnn_forward prepares too). */
int hgnn_op_generation(const hgnn_ctx *ctx, int64_t *out);
/* Layer l forward (one PNA graph convolution, Section 3.1): h_out_dev [N, H]
 * from h_in_dev [N, F_l].  Stores the layer's messages, aggregates and arg
 * decisions (unless recompute is on). */
int hgnn_op_layer_forward(hgnn_ctx *ctx, int32_t layer,
                          const float *w_layer_dev, const float *h_in_dev,
                          float *h_out_dev, void *stream);
/* Layer l backward (Section 3.2): from dh_out_dev [N, H] (gradient w.r.t.
 * h_out) write dw_layer_dev and, when dh_in_dev is not NULL, dh_in_dev
 * [N, F_l]. */
int hgnn_op_layer_backward(hgnn_ctx *ctx, int64_t generation, int32_t layer,
                           const float *w_layer_dev, const float *h_in_dev,
                           const float *h_out_dev, const float *dh_out_dev,
                           float *dh_in_dev, float *dw_layer_dev, void *stream);
/* Global mean pooling + FC head (Section 3.1), + the MSE loss (Section 3.2)
 * when target_dev and loss_dev are given.  pred_dev [B]. */
int hgnn_op_head_forward(hgnn_ctx *ctx, const float *w_head_dev,
                         const float *h_dev, const float *target_dev,
                         float *pred_dev, float *loss_dev, void *stream);
/* Head adjoint (Section 3.2): dpred_dev [B], or the MSE gradient from
 * target_dev when dpred_dev is NULL.  Writes dh_dev [N, H] and dw_head_dev. */
int hgnn_op_head_backward(hgnn_ctx *ctx, int64_t generation, const float *w_head_dev,
                          const float *h_dev, const float *target_dev,
                          const float *dpred_dev, float *dh_dev,
                          float *dw_head_dev, void *stream);

/* Inspection of stored results (parity tests).  which:
 *   0 rowptr [N+1]  1 csr_src [E]  2 csr_eid [E]  3 deg [N]
 *   4 srcptr [N+1]  5 t2csr [E]    6 node_graph [N]          (int32)
 *   7 aggregates A of `layer` [N, 4H] (float32)
 *   8 arg decisions of `layer` [N, 2H] (uint8: argmin offsets then argmax)
 *   9 hidden activations ReLU(W1 g + b1) of graph head `layer` [B, H] (float32)
 *  10 pooled features g [B, H] (float32)
 *  11 output of `layer` from the last hgnn_forward [N, H] (float32)
 *  12 hidden activations ReLU(W1 h + b1) of node head `layer` [N, H] (float32)
 * Copies into dst_dev (capacity bytes); EINVAL if too small or not stored. */
int hgnn_op_fetch(hgnn_ctx *ctx, int32_t which, int32_t layer, void *dst_dev,
                  size_t capacity, void *stream);

/* ---- measurement -------------------------------------------------------- */

/* Opt-in kernel timer: bracket every launch of one launch site with a pair of
 * HIP events recorded on that launch's stream, for up to max_launches
 * launches.  Sites: 1 message GEMM, 2 aggregation, 3 update GEMM, 4 update
 * weight-gradient GEMM, 5 aggregate-gradient GEMM, 6 aggregation adjoint,
 * 7 input-gradient GEMM, 8 message weight-gradient GEMM (these time the
 * kernel alone, not a split-K reduction after it), 9 the CSR build of a
 * training-path forward (all of its launches).  For GraphSAGE models site 3 is the layer GEMM and
 * 4 its weight gradient; for CGCNN models 2 is the gated aggregation, 4 the
 * layer weight gradient, 6 the aggregation adjoint and 7 the input-gradient
 * GEMM.  Synchronises the device. */
int hgnn_timer_start(hgnn_ctx *ctx, int32_t site, int32_t max_launches);
/* Sum of the bracketed durations (ms) and the number of launches; stops the
 * timer.  Waits for the recorded events. */
int hgnn_timer_read(hgnn_ctx *ctx, double *total_ms, int32_t *launches);
/* Plain copy of n floats (n a multiple of 4, both device, 16-byte aligned):
 * a kernel of known traffic for calibrating hardware byte counters. */
int hgnn_calib_copy(const float *src_dev, float *dst_dev, int64_t n, void *stream);

/* ---- serving (continuous batching of inference requests) --------------- */
/* The use the paper gives the surrogate (Section 1, Fig. 1): a fast screen of
 * molecules streamed from design workflows, one predicted HOMO-LUMO gap per
 * molecule.  Requests of any number of molecules are queued, packed into
 * batches that the forward pass of Section 3.1 runs on the GPU (no loss), and
 * their predictions handed back per request.  A request's predictions do not
 * depend on what it was batched with. */

typedef struct {
  int64_t hbm_budget_bytes; /* admission budget for in-flight batches */
  int32_t max_batch_nodes;  /* node capacity of the largest packed batch */
  int32_t max_batch_edges;  /* edge capacity of the largest packed batch */
  int32_t max_batch_graphs; /* graph capacity of the largest packed batch */
  int32_t num_lanes;        /* batches in flight at once (own stream each) */
  int32_t queue_capacity;   /* pending requests before submit says EAGAIN */
  int32_t use_graphs;       /* 1: replay captured HIP graphs per bucket */
} hgnn_serve_config;

typedef struct {
  int64_t submitted, completed, batches, graph_replays, admission_waits;
  int64_t peak_inflight_bytes;
  int64_t lanes;      /* lanes that fit the budget */
  int64_t lane_bytes; /* device footprint of one lane */
} hgnn_serve_stats;

/* Start the scheduler thread; the weights stay resident and are shared. */
int hgnn_serve_start(hgnn_ctx *ctx, const hgnn_serve_config *cfg);
/* Copy a request (host arrays, y ignored) into the queue; returns a ticket.
 * EAGAIN when the queue is full or the request alone exceeds a lane. */
int hgnn_serve_submit(hgnn_ctx *ctx, const hgnn_batch *request_host,
                      uint64_t *ticket);
/* *done = 1 and pred_host [B_request] filled once finished (the ticket is
 * then released); *done = 0 while pending.  EINVAL for an unknown ticket or
 * a request that failed validation. */
int hgnn_serve_poll(hgnn_ctx *ctx, uint64_t ticket, float *pred_host,
                    int32_t *done);
int hgnn_serve_stats_get(hgnn_ctx *ctx, hgnn_serve_stats *out);
/* Drain in-flight work and stop the thread. */
int hgnn_serve_stop(hgnn_ctx *ctx);

/* ---- packed graph store (Section 3.3: I/O; Table 1: graph layout) ------ */
/* A binary file of batches in the Table 1 layout, one contiguous record per
 * batch (graph_ptr, x, edge_index, edge_attr, y), read by host threads into
 * pinned buffers and copied to the device on the store's own stream, so the
 * copy of the next batch overlaps the caller's compute.  File format: a
 * 64-byte header ("HGNNSTR1", version 1, num_batches, node_feat, edge_feat,
 * has_y, index offset), an index of {offset, bytes, B, N, E} per batch, and
 * 4096-aligned records whose sections start 256-byte aligned in the order
 * graph_ptr i32 [B+1], x f32 [N, F], edge_index i32 [2, E], edge_attr f32
 * [E, Fe], y f32 [B].  The writer is paper_2207_11333_amd/graphstore.py. */
typedef struct hgnn_store hgnn_store;

typedef struct {
  int32_t num_batches, node_feat, edge_feat, has_y;
  int32_t max_graphs, max_nodes, max_edges, reserved;
  int64_t max_record_bytes;
} hgnn_store_info;

/* Open a store on the current device: io_threads (1..64) reader threads,
 * host_slots (2..64) pinned record buffers, two device record buffers.
 * EINVAL for a missing or malformed file, ENOMEM when buffers fail. */
int hgnn_store_open(const char *path, int32_t io_threads, int32_t host_slots,
                    hgnn_store **out);
int hgnn_store_info_get(const hgnn_store *store, hgnn_store_info *info);
/* The next batch in file order, cycling over the file: fills *out with
 * device pointers (owned by the store) and *index (may be NULL) with its
 * position in the file.  `stream` is made to wait for the batch's copy; the
 * pointers stay valid for all work enqueued on that stream until the next
 * call, which releases them.  Blocks while the batch is still being read.
 * EINVAL after a read error, EDEVICE when a HIP call fails. */
int hgnn_store_next(hgnn_store *store, void *stream, hgnn_batch *out,
                    int64_t *index);
/* Stop the readers, wait for copies in flight, free everything. */
int hgnn_store_close(hgnn_store *store);

const char *hgnn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HGNN_H */
