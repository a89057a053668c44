// Packed graph store and its pinned-memory reader (the I/O path of
// Section 3.3: graphs kept in the Table 1 layout in one binary file, read in
// parallel and handed to training without per-graph work).
//
// File (little endian):
//   header, 64 bytes: magic "HGNNSTR1", u32 version (1), u32 num_batches,
//     u32 node_feat, u32 edge_feat, u32 has_y, u32 reserved[3],
//     u64 index_offset, u64 reserved[2]
//   index at index_offset: num_batches entries of
//     { u64 offset, u64 bytes, i32 B, i32 N, i32 E, i32 reserved }
//   one record per batch at `offset` (4096-aligned), sections in this order,
//   each starting 256-byte aligned from the record start:
//     graph_ptr i32 [B+1] | x f32 [N, F] | edge_index i32 [2, E] |
//     edge_attr f32 [E, Fe] | y f32 [B] (only when has_y)
//
// Reader: io_threads host threads read whole records with pread into
// host_slots pinned buffers, in file order and cycling over the file (one
// pass = one epoch).  hgnn_store_next copies a record to one of two device
// buffers with a single asynchronous copy on the store's own stream, makes
// the caller's stream wait for it, and starts the copy of the following
// record into the other device buffer, so that copy overlaps the caller's
// compute.  A device buffer is reused only after the caller's stream has
// passed the point where the batch was released (the next call).
#include "common.hpp"
#include "hgnn.h"

#include <atomic>
#include <condition_variable>
#include <cstring>
#include <fcntl.h>
#include <mutex>
#include <string>
#include <thread>
#include <unistd.h>
#include <vector>

namespace hgnn {
int set_error(int code, const std::string &msg);
}

namespace {

struct StoreHeader {
  char magic[8];
  uint32_t version, num_batches, node_feat, edge_feat, has_y, reserved[3];
  uint64_t index_offset, reserved2[2];
};
static_assert(sizeof(StoreHeader) == 64, "header layout");

struct StoreEntry {
  uint64_t offset, bytes;
  int32_t B, N, E, reserved;
};
static_assert(sizeof(StoreEntry) == 32, "index layout");

inline uint64_t align256(uint64_t v) { return (v + 255) & ~uint64_t(255); }

struct Sections {
  uint64_t gp, x, ei, ea, y, end;
};

Sections sections(int B, int N, int E, int F, int Fe, bool has_y) {
  Sections s{};
  s.gp = 0;
  s.x = align256(4ull * (B + 1));
  s.ei = s.x + align256(4ull * N * F);
  s.ea = s.ei + align256(8ull * E);
  s.y = s.ea + align256(4ull * E * Fe);
  s.end = s.y + (has_y ? align256(4ull * B) : 0);
  return s;
}

struct HostSlot {
  void *buf = nullptr;
  long long expect = 0;     // sequence number this slot holds next
  bool ready = false;       // holds record `expect`, read complete
  bool copying = false;     // a device copy from it may still be running
  hipEvent_t copied = nullptr;
};

struct DevSlot {
  uint8_t *buf = nullptr;
  long long seq = -1;       // sequence number whose copy was issued into it
  hipEvent_t copied = nullptr, released = nullptr;
  bool released_recorded = false;
};

} // namespace

struct hgnn_store {
  int fd = -1;
  StoreHeader hdr{};
  std::vector<StoreEntry> index;
  uint64_t max_bytes = 0;
  int32_t max_B = 0, max_N = 0, max_E = 0;
  int dev = 0;
  std::vector<HostSlot> host;
  DevSlot devs[2];
  hipStream_t copy = nullptr;
  std::vector<std::thread> threads;
  std::mutex mu;
  std::condition_variable cv;
  std::atomic<long long> next_read{0};
  bool stop = false;
  std::string io_error;
  long long consumed = 0;     // calls of hgnn_store_next so far
  hipStream_t last_stream = nullptr;
};

namespace {

int fail(int code, const std::string &m) { return hgnn::set_error(code, m); }

void reader(hgnn_store *s) {
  const int P = (int)s->host.size();
  const long long nb = (long long)s->index.size();
  for (;;) {
    const long long j = s->next_read.fetch_add(1);
    HostSlot &h = s->host[j % P];
    bool wait_copy = false;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv.wait(lk, [&] { return s->stop || (!h.ready && h.expect == j); });
      if (s->stop) return;
      wait_copy = h.copying;
    }
    if (wait_copy) {
      (void)hipSetDevice(s->dev);
      hipError_t e = hipEventSynchronize(h.copied);
      std::lock_guard<std::mutex> lk(s->mu);
      h.copying = false;
      if (e != hipSuccess && s->io_error.empty())
        s->io_error = std::string("store copy failed: ") + hipGetErrorString(e);
    }
    const StoreEntry &en = s->index[j % nb];
    uint64_t done = 0;
    bool ok = true;
    while (done < en.bytes) {
      const ssize_t r = pread(s->fd, (uint8_t *)h.buf + done, en.bytes - done,
                              (off_t)(en.offset + done));
      if (r <= 0) { ok = false; break; }
      done += (uint64_t)r;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (!ok && s->io_error.empty()) s->io_error = "short read from the graph store";
    h.ready = true;
    s->cv.notify_all();
  }
}

// Issue the device copy of record `seq` if its host slot is ready (or wait for
// it when `block`); returns 1 when issued, 0 when deferred, <0 on error.
int issue_copy(hgnn_store *s, long long seq, bool block) {
  const int P = (int)s->host.size();
  HostSlot &h = s->host[seq % P];
  DevSlot &d = s->devs[seq % 2];
  {
    std::unique_lock<std::mutex> lk(s->mu);
    if (block)
      s->cv.wait(lk, [&] { return !s->io_error.empty() || (h.ready && h.expect == seq); });
    if (!s->io_error.empty()) return fail(HGNN_EINVAL, s->io_error);
    if (!(h.ready && h.expect == seq)) return 0;
  }
  const StoreEntry &en = s->index[seq % (long long)s->index.size()];
  hipError_t e = hipSuccess;
  if (d.released_recorded) e = hipStreamWaitEvent(s->copy, d.released, 0);
  if (e == hipSuccess) e = hipMemcpyAsync(d.buf, h.buf, en.bytes, hipMemcpyHostToDevice, s->copy);
  if (e == hipSuccess) e = hipEventRecord(d.copied, s->copy);
  if (e == hipSuccess) e = hipEventRecord(h.copied, s->copy);
  if (e != hipSuccess) return fail(HGNN_EDEVICE, std::string("store copy: ") + hipGetErrorString(e));
  d.seq = seq;
  d.released_recorded = false;
  std::lock_guard<std::mutex> lk(s->mu);
  h.ready = false;
  h.copying = true;
  h.expect = seq + P;
  s->cv.notify_all();
  return 1;
}

void shutdown(hgnn_store *s) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  for (auto &t : s->threads) t.join();
  s->threads.clear();
  if (s->copy) (void)hipStreamSynchronize(s->copy);
  for (auto &h : s->host) {
    if (h.buf) (void)hipHostFree(h.buf);
    if (h.copied) (void)hipEventDestroy(h.copied);
  }
  for (auto &d : s->devs) {
    if (d.buf) (void)hipFree(d.buf);
    if (d.copied) (void)hipEventDestroy(d.copied);
    if (d.released) (void)hipEventDestroy(d.released);
  }
  if (s->copy) (void)hipStreamDestroy(s->copy);
  if (s->fd >= 0) close(s->fd);
}

} // namespace

extern "C" {

int hgnn_store_open(const char *path, int32_t io_threads, int32_t host_slots,
                    hgnn_store **out) {
  if (!path || !out) return fail(HGNN_EINVAL, "path and out are required");
  if (io_threads < 1 || io_threads > 64) return fail(HGNN_EINVAL, "io_threads must be in 1..64");
  if (host_slots < 2 || host_slots > 64) return fail(HGNN_EINVAL, "host_slots must be in 2..64");
  *out = nullptr;
  hgnn_store *s = new hgnn_store();
  s->fd = open(path, O_RDONLY);
  if (s->fd < 0) {
    delete s;
    return fail(HGNN_EINVAL, std::string("cannot open graph store ") + path);
  }
  auto bad = [&](const std::string &m) {
    shutdown(s);
    delete s;
    return fail(HGNN_EINVAL, std::string("graph store ") + path + ": " + m);
  };
  if (pread(s->fd, &s->hdr, sizeof(s->hdr), 0) != (ssize_t)sizeof(s->hdr)) return bad("no header");
  if (std::memcmp(s->hdr.magic, "HGNNSTR1", 8) != 0 || s->hdr.version != 1)
    return bad("not a version-1 graph store");
  const uint32_t nb = s->hdr.num_batches;
  if (nb < 1 || s->hdr.node_feat < 1 || s->hdr.edge_feat > 4 || s->hdr.has_y > 1)
    return bad("bad header fields");
  s->index.resize(nb);
  const ssize_t ib = (ssize_t)(sizeof(StoreEntry) * nb);
  if (pread(s->fd, s->index.data(), ib, (off_t)s->hdr.index_offset) != ib)
    return bad("truncated index");
  for (const StoreEntry &en : s->index) {
    if (en.B < 1 || en.N < en.B || en.E < 0) return bad("bad batch sizes in the index");
    const Sections sc = sections(en.B, en.N, en.E, (int)s->hdr.node_feat, (int)s->hdr.edge_feat,
                                 s->hdr.has_y != 0);
    if (en.bytes != sc.end) return bad("record size does not match its sizes");
    s->max_bytes = std::max<uint64_t>(s->max_bytes, en.bytes);
    s->max_B = std::max(s->max_B, en.B);
    s->max_N = std::max(s->max_N, en.N);
    s->max_E = std::max(s->max_E, en.E);
  }
  hipError_t e = hipGetDevice(&s->dev);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking);
  s->host.resize(host_slots);
  for (int i = 0; i < host_slots && e == hipSuccess; ++i) {
    s->host[i].expect = i;
    e = hipHostMalloc(&s->host[i].buf, s->max_bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->host[i].copied, hipEventDisableTiming);
  }
  for (int i = 0; i < 2 && e == hipSuccess; ++i) {
    e = hipMalloc(&s->devs[i].buf, s->max_bytes);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->devs[i].copied, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->devs[i].released, hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    shutdown(s);
    delete s;
    return fail(HGNN_ENOMEM, std::string("graph store buffers: ") + hipGetErrorString(e));
  }
  for (int i = 0; i < io_threads; ++i) s->threads.emplace_back(reader, s);
  *out = s;
  return HGNN_OK;
}

int hgnn_store_info_get(const hgnn_store *s, hgnn_store_info *info) {
  if (!s || !info) return fail(HGNN_EINVAL, "store and info are required");
  info->num_batches = (int32_t)s->index.size();
  info->node_feat = (int32_t)s->hdr.node_feat;
  info->edge_feat = (int32_t)s->hdr.edge_feat;
  info->has_y = (int32_t)s->hdr.has_y;
  info->max_graphs = s->max_B;
  info->max_nodes = s->max_N;
  info->max_edges = s->max_E;
  info->reserved = 0;
  info->max_record_bytes = (int64_t)s->max_bytes;
  return HGNN_OK;
}

int hgnn_store_next(hgnn_store *s, void *stream, hgnn_batch *out, int64_t *index) {
  if (!s || !out) return fail(HGNN_EINVAL, "store and out are required");
  hipError_t e = hipSetDevice(s->dev);
  if (e != hipSuccess) return fail(HGNN_EDEVICE, hipGetErrorString(e));
  hipStream_t st = (hipStream_t)stream;
  const long long k = s->consumed;
  // release the previous batch's device buffer once the caller's stream has
  // done everything enqueued for it so far
  if (k > 0) {
    DevSlot &prev = s->devs[(k - 1) % 2];
    e = hipEventRecord(prev.released, s->last_stream);
    if (e != hipSuccess) return fail(HGNN_EDEVICE, hipGetErrorString(e));
    prev.released_recorded = true;
  }
  DevSlot &d = s->devs[k % 2];
  if (d.seq != k) {
    int rc = issue_copy(s, k, /*block=*/true);
    if (rc < 0) return rc;
  }
  e = hipStreamWaitEvent(st, d.copied, 0);
  if (e != hipSuccess) return fail(HGNN_EDEVICE, hipGetErrorString(e));
  // start the next record's copy now if it has been read (else at the next call)
  {
    int rc = issue_copy(s, k + 1, /*block=*/false);
    if (rc < 0) return rc;
  }
  const StoreEntry &en = s->index[k % (long long)s->index.size()];
  const Sections sc = sections(en.B, en.N, en.E, (int)s->hdr.node_feat, (int)s->hdr.edge_feat,
                               s->hdr.has_y != 0);
  out->num_graphs = en.B;
  out->num_nodes = en.N;
  out->num_edges = en.E;
  out->reserved = 0;
  out->graph_ptr = reinterpret_cast<const int32_t *>(d.buf + sc.gp);
  out->x = reinterpret_cast<const float *>(d.buf + sc.x);
  out->edge_index = reinterpret_cast<const int32_t *>(d.buf + sc.ei);
  out->edge_attr = s->hdr.edge_feat ? reinterpret_cast<const float *>(d.buf + sc.ea) : nullptr;
  out->y = s->hdr.has_y ? reinterpret_cast<const float *>(d.buf + sc.y) : nullptr;
  if (index) *index = k % (long long)s->index.size();
  s->last_stream = st;
  s->consumed = k + 1;
  return HGNN_OK;
}

int hgnn_store_close(hgnn_store *s) {
  if (!s) return HGNN_OK;
  shutdown(s);
  delete s;
  return HGNN_OK;
}

} // extern "C"
