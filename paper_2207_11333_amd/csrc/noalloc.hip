// Allocation-free inference forward (hgnn_forward_noalloc): the forward pass
// of hgnn_forward without the stored activations, for callers that cannot
// allocate device memory (code under stream capture, tight serving loops).
//
// Its whole batch workspace -- the size header, the error word, the CSR
// arrays, the padded input, two rotating layer outputs, one layer's messages
// and aggregates, the head buffers and the split-K partials of the GEMMs --
// is carved from one file-scope device array per GPU.  Host code never passes
// the array's name to a kernel (in host code it names a host-side stand-in):
// its device address is looked up once per device with hipGetSymbolAddress
// and only that pointer is used.  Every call on one GPU shares the array and
// it keeps the last call's contents; calls that overlap on one GPU (any
// context, any stream) race.  Nothing in the workspace needs to start at
// zero: the size header and the error word are written first by every call
// and the CSR build clears its own counters.
#include "runtime.hpp"

#include <mutex>
#include <string>

namespace hgnn {

namespace {

constexpr size_t kNoAllocScratchBytes = size_t(64) << 20; // 64 MiB per GPU
constexpr size_t kHeaderBytes = 512; // Dims at 0, the error word at 256
constexpr int kMaxDevices = 64;

std::mutex g_mu;
char *g_ptr[kMaxDevices] = {}; // the array's device address, per device

} // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

int noalloc_init(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return set_error(HGNN_EDEVICE, "device id out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[dev]) return HGNN_OK;
  void *p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return set_error(HGNN_EDEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") +
                                       hipGetErrorString(e));
  g_ptr[dev] = static_cast<char *>(p);
  return HGNN_OK;
}

} // namespace hgnn

using namespace hgnn;

extern "C" {

int64_t hgnn_noalloc_max_bytes(void) { return (int64_t)kNoAllocScratchBytes; }

int hgnn_noalloc_bytes(const hgnn_ctx *c, int32_t num_graphs, int32_t num_nodes,
                       int32_t num_edges, int64_t *out) {
  if (!c || !out) return set_error(HGNN_EINVAL, "ctx and out are required");
  if (num_graphs < 1 || num_nodes < num_graphs || num_edges < 0)
    return set_error(HGNN_EINVAL, "bad batch sizes");
  *out = (int64_t)(kHeaderBytes + work_bytes(c, num_graphs, num_nodes, num_edges, true));
  return HGNN_OK;
}

int hgnn_forward_noalloc(hgnn_ctx *c, const hgnn_batch *b, float *pred, float *loss,
                         int32_t flags, void *stream) {
  if (!c) return set_error(HGNN_EINVAL, "context is NULL");
  if (c->sticky) return set_error(HGNN_ESTATE, "context failed earlier; restore state");
  hipError_t e = hipSetDevice(c->dev);
  if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  if (c->kind != HGNN_GC_PNA || c->Tn != 0)
    return set_error(HGNN_EINVAL, "the allocation-free forward takes PNA models without node heads");
  if (!b || !pred) return set_error(HGNN_EINVAL, "batch and pred_dev are required");
  if (loss && !b->y) return set_error(HGNN_EINVAL, "loss requested without targets");
  if (int rc = check_batch_host(c, b)) return rc;
  char *base = c->dev < kMaxDevices ? g_ptr[c->dev] : nullptr;
  if (!base) return set_error(HGNN_EDEVICE, "scratch array not set up on this device");
  Exec &ex = c->na;
  if (carve_work(c, ex, b->num_graphs, b->num_nodes, b->num_edges, base + kHeaderBytes,
                 kNoAllocScratchBytes - kHeaderBytes) == 0) {
    const size_t need =
        kHeaderBytes + work_bytes(c, b->num_graphs, b->num_nodes, b->num_edges, true);
    return set_error(HGNN_EINVAL, "batch needs " + std::to_string(need) +
                                      " bytes of workspace; the allocation-free forward holds " +
                                      std::to_string(kNoAllocScratchBytes));
  }
  ex.dims = reinterpret_cast<Dims *>(base);
  ex.w.csr.err = reinterpret_cast<int *>(base + 256);
  hipStream_t s = (hipStream_t)stream;
  Work &w = ex.w;
  e = launch_set_dims(ex.dims, b->num_graphs, b->num_nodes, b->num_edges, w.csr.err, s);
  if (e == hipSuccess)
    e = launch_csr_build(ex.dims, b->num_graphs, b->num_nodes, b->num_edges, b->graph_ptr,
                         b->edge_index, b->edge_attr, c->Fe, c->maxd, c->table, w.csr,
                         /*clear_err=*/false, b->x, c->F0, w.xpad, c->F0p, s);
  if (e != hipSuccess) return hip_fail(c, e, "csr build");
  ex.B = b->num_graphs;
  ex.N = b->num_nodes;
  ex.E = b->num_edges;
  ex.graph_ptr = b->graph_ptr;
  ex.xin = b->x;
  ex.target = b->y;
  ex.x_padded = true;
  ex.prepared = true;
  if (flags & HGNN_VALIDATE) {
    int bits = 0;
    e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipMemcpy(&bits, w.csr.err, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "validate");
    if (bits) return set_error(HGNN_EINVAL, decode_err(bits));
  }
  if (!c->staged_from_params)
    if (int rc = stage_all(c, s)) return rc;
  const float *h = b->x;
  for (int l = 0; l < c->L; ++l) {
    float *out = w.hbuf[l & 1];
    if (int rc = layer_forward(c, ex, l, c->params + c->ld[l].off, h, out, s)) return rc;
    h = out;
  }
  return head_forward(c, ex, c->params + c->off_head, h, b->y, pred, loss, s);
}

} // extern "C"
