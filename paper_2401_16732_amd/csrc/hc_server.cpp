// Serving loop: continuous batching of HE-convolution requests on one GPU.
//
// A request is one image through every convolution layer of one network.
// The server owns an HBM arena; a request is admitted (FIFO) when its
// footprint - per layer the input ciphertexts, the mask, c0_ext and c1_out
// for one image - fits, and its inputs are then copied into the arena. Each
// scheduler step groups the next layer of every admitted request whose
// previous layer has finished by (network, layer), and launches each group of
// at most 16 images as one batched forward NTT -> multiply-accumulate ->
// masked inverse NTT on one of the server's streams. Layers of one request run
// in order (in the protocol the client answers between layers); requests that
// arrive while others are running join the groups of the layer they are at.
// Weights and twiddles stay resident in their layers and context.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <unordered_map>
#include <vector>

#include "../../include/hc.h"
#include "hc_internal.h"
#include "hc_objects.h"

using hc::fail;
using hc::hip_fail;

namespace {

#define SV_HIP(call)                                  \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return hip_fail(e_, #call); \
  } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator over the arena (offsets), coalescing on free.
class Arena {
 public:
  void reset(size_t bytes) {
    free_.clear();
    free_[0] = bytes;
    total_ = bytes;
    used_ = 0;
  }
  bool alloc(size_t bytes, size_t *off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t total() const { return total_; }

 private:
  std::map<size_t, size_t> free_;
  size_t total_ = 0, used_ = 0;
};

struct NetPlan {
  std::vector<const hc_layer *> layers;
  // per layer byte offsets inside a request block
  std::vector<size_t> off_in, off_mask, off_c0, off_c1, in_bytes, mask_bytes;
  size_t bytes = 0;
  size_t ws_bytes = 0;  // workspace for a group of max_batch images of the largest layer
};

struct Request {
  uint64_t id = 0;
  uint32_t net = 0;
  std::vector<const uint32_t *> src_in, src_mask;
  size_t off = 0;
  bool admitted = false, done = false;
  uint32_t next = 0;      // next layer to launch
  int group = -1;         // event slot of the layer in flight, or -1
  int ready = -1;         // event slot of the input copy, or -1 once observed
};

}  // namespace

struct hc_server {
  hc_ctx *ctx = nullptr;
  hc_server_config cfg{};
  std::vector<NetPlan> nets;
  char *arena = nullptr;
  Arena alloc;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Request> reqs;
  uint64_t next_id = 1;
  std::vector<hipStream_t> streams;
  hipStream_t copy = nullptr;
  std::vector<char *> ws;
  size_t ws_each = 0;
  uint32_t rr = 0;
  std::vector<hipEvent_t> events;
  std::vector<int> ev_refs;
  std::vector<int> ev_free;
  std::vector<uint64_t> completed;
  std::vector<int> inflight;  // event slots of launched groups not yet seen complete
  hc_server_stats st{};
};

namespace {

int ev_get(hc_server *s) {
  if (s->ev_free.empty()) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return -1;
    s->events.push_back(e);
    s->ev_refs.push_back(0);
    return (int)s->events.size() - 1;
  }
  int k = s->ev_free.back();
  s->ev_free.pop_back();
  return k;
}
void ev_unref(hc_server *s, int k) {
  if (--s->ev_refs[k] == 0) s->ev_free.push_back(k);
}

hc_status ensure_workspace(hc_server *s, size_t need) {
  if (need <= s->ws_each) return HC_OK;
  for (auto st : s->streams) SV_HIP(hipStreamSynchronize(st));  // old workspaces may still be in use
  for (char *p : s->ws) {
    if (p) SV_HIP(hipFree(p));
  }
  s->ws.assign(s->streams.size(), nullptr);
  for (auto &p : s->ws) {
    if (hipMalloc((void **)&p, need) != hipSuccess) return fail(HC_ENOMEM, "server workspace allocation");
  }
  s->ws_each = need;
  return HC_OK;
}

hc_status admit(hc_server *s, Request &r) {
  const NetPlan &np = s->nets[r.net];
  size_t off;
  if (!s->alloc.alloc(np.bytes, &off)) return HC_ENOMEM;  // not an error: stays queued
  r.off = off;
  char *base = s->arena + off;
  for (size_t k = 0; k < np.layers.size(); ++k) {
    SV_HIP(hipMemcpyAsync(base + np.off_in[k], r.src_in[k], np.in_bytes[k], hipMemcpyDefault, s->copy));
    SV_HIP(hipMemcpyAsync(base + np.off_mask[k], r.src_mask[k], np.mask_bytes[k], hipMemcpyDefault, s->copy));
  }
  int ev = ev_get(s);
  if (ev < 0) return fail(HC_EDEVICE, "event creation");
  SV_HIP(hipEventRecord(s->events[ev], s->copy));
  s->ev_refs[ev] = 1;
  r.ready = ev;
  r.admitted = true;
  s->st.admitted++;
  return HC_OK;
}

}  // namespace

extern "C" {

hc_status hc_server_create(hc_ctx *ctx, const hc_server_config *cfg, hc_server **out) {
  if (!ctx || !cfg || !out) return fail(HC_EINVAL, "null argument");
  *out = nullptr;
  if (cfg->max_batch < 1 || cfg->max_batch > hc::kMaxTab) return fail(HC_EUNSUPPORTED, "max_batch must be in [1, 16]");
  if (cfg->streams < 1 || cfg->streams > 8) return fail(HC_EUNSUPPORTED, "streams must be in [1, 8]");
  if (cfg->max_inflight && cfg->max_inflight < cfg->streams)
    return fail(HC_EINVAL, "max_inflight must be 0 or at least the number of streams");
  if (cfg->arena_bytes < kAlign) return fail(HC_EINVAL, "arena too small");
  hc::DeviceGuard dg(ctx->device);
  hc_server *s = new (std::nothrow) hc_server;
  if (!s) return fail(HC_ENOMEM, "host allocation");
  s->ctx = ctx;
  s->cfg = *cfg;
  if (hipMalloc((void **)&s->arena, cfg->arena_bytes) != hipSuccess) {
    delete s;
    return fail(HC_ENOMEM, "server arena allocation");
  }
  s->alloc.reset(cfg->arena_bytes);
  s->streams.assign(cfg->streams, nullptr);
  hipError_t e = hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking);
  for (auto &st : s->streams)
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (e != hipSuccess) {
    hc_server_destroy(s);
    return hip_fail(e, "server streams");
  }
  s->ws.assign(cfg->streams, nullptr);
  *out = s;
  return HC_OK;
}

hc_status hc_server_add_net(hc_server *s, const hc_layer *const *layers, uint32_t n, uint32_t *net_id) {
  if (!s || !layers || !net_id || n == 0) return fail(HC_EINVAL, "null argument");
  NetPlan np;
  size_t off = 0, ws = 0;
  const hc_ctx &c = *s->ctx;
  for (uint32_t k = 0; k < n; ++k) {
    const hc_layer *ly = layers[k];
    if (!ly) return fail(HC_EINVAL, "null layer");
    if (ly->ctx != s->ctx) return fail(HC_ESTATE, "layer belongs to another context");
    const hc_layout &lo = ly->lay;
    const size_t in_b = (size_t)lo.in_cts * 2 * c.L * c.N * 4;
    const size_t mask_b = (size_t)ly->shape.c_out * lo.ho * lo.wo * 4;
    const size_t c0_b = (size_t)ly->shape.c_out * c.L * lo.ho * lo.wo * 4;
    const size_t c1_b = (size_t)lo.out_cts * c.L * c.N * 4;
    np.layers.push_back(ly);
    np.off_in.push_back(off), off += align_up(in_b);
    np.off_mask.push_back(off), off += align_up(mask_b);
    np.off_c0.push_back(off), off += align_up(c0_b);
    np.off_c1.push_back(off), off += align_up(c1_b);
    np.in_bytes.push_back(in_b);
    np.mask_bytes.push_back(mask_b);
    const hc::Shapes sh = hc::shapes_for(c, s->cfg.max_batch);
    if (!hc::mac_offsets_fit(ly->geom, sh.mac)) return fail(HC_EUNSUPPORTED, "layer too large for the MAC tile");
    ws = std::max(ws, hc::ws_bytes_for(ly, s->cfg.max_batch, true));
  }
  np.bytes = off;
  np.ws_bytes = ws;
  if (np.bytes > s->alloc.total()) return fail(HC_EINVAL, "one request of this network exceeds the arena");
  hc::DeviceGuard dg(s->ctx->device);
  hc_status st = ensure_workspace(s, ws);
  if (st != HC_OK) return st;
  s->nets.push_back(std::move(np));
  *net_id = (uint32_t)s->nets.size() - 1;
  return HC_OK;
}

hc_status hc_server_request_bytes(const hc_server *s, uint32_t net, size_t *bytes) {
  if (!s || !bytes || net >= s->nets.size()) return fail(HC_EINVAL, "bad argument");
  *bytes = s->nets[net].bytes;
  return HC_OK;
}

hc_status hc_server_submit(hc_server *s, uint32_t net, const uint32_t *const *ct_in, const uint32_t *const *mask,
                           uint64_t *req_id) {
  if (!s || !ct_in || !mask || !req_id || net >= s->nets.size()) return fail(HC_EINVAL, "bad argument");
  const NetPlan &np = s->nets[net];
  Request r;
  r.id = s->next_id++;
  r.net = net;
  for (size_t k = 0; k < np.layers.size(); ++k) {
    if (!ct_in[k] || !mask[k]) return fail(HC_EINVAL, "null input buffer");
    r.src_in.push_back(ct_in[k]);
    r.src_mask.push_back(mask[k]);
  }
  const uint64_t id = r.id;
  s->reqs.emplace(id, std::move(r));
  s->queue.push_back(id);
  *req_id = id;
  s->st.submitted++;
  return HC_OK;
}

hc_status hc_server_step(hc_server *s) {
  if (!s) return fail(HC_EINVAL, "null server");
  hc::DeviceGuard dg(s->ctx->device);
  // 1. retire finished layers
  for (auto &kv : s->reqs) {
    Request &r = kv.second;
    if (r.ready >= 0) {
      hipError_t q = hipEventQuery(s->events[r.ready]);
      if (q == hipSuccess) {
        ev_unref(s, r.ready);
        r.ready = -1;
      } else if (q != hipErrorNotReady) {
        return hip_fail(q, "input copy");
      }
    }
    if (r.group >= 0) {
      hipError_t q = hipEventQuery(s->events[r.group]);
      if (q == hipSuccess) {
        ev_unref(s, r.group);
        r.group = -1;
        if (++r.next == s->nets[r.net].layers.size()) {
          r.done = true;
          s->completed.push_back(r.id);
          s->st.completed++;
        }
      } else if (q != hipErrorNotReady) {
        return hip_fail(q, "layer group");
      }
    }
  }
  for (size_t k = 0; k < s->inflight.size();) {
    hipError_t q = hipEventQuery(s->events[s->inflight[k]]);
    if (q == hipSuccess) {
      ev_unref(s, s->inflight[k]);
      s->inflight[k] = s->inflight.back();
      s->inflight.pop_back();
    } else if (q != hipErrorNotReady) {
      return hip_fail(q, "layer group");
    } else {
      ++k;
    }
  }
  // 2. admission, first come first served
  while (!s->queue.empty()) {
    Request &r = s->reqs.at(s->queue.front());
    hc_status a = admit(s, r);
    if (a == HC_ENOMEM) break;
    if (a != HC_OK) return a;
    s->queue.pop_front();
  }
  // 3. group the next layer of every ready request by (network, layer); chunks
  // of at most max_batch images, largest first, then the oldest request first
  std::map<std::pair<uint32_t, uint32_t>, std::vector<Request *>> groups;
  for (auto &kv : s->reqs) {
    Request &r = kv.second;
    if (!r.admitted || r.done || r.group >= 0 || r.ready >= 0) continue;
    groups[{r.net, r.next}].push_back(&r);
  }
  struct Chunk {
    uint32_t net, layer;
    std::vector<Request *> reqs;
  };
  std::vector<Chunk> chunks;
  for (auto &g : groups) {
    std::vector<Request *> &v = g.second;
    std::sort(v.begin(), v.end(), [](const Request *a, const Request *b) { return a->id < b->id; });
    for (size_t at = 0; at < v.size(); at += s->cfg.max_batch) {
      const size_t B = std::min<size_t>(s->cfg.max_batch, v.size() - at);
      chunks.push_back({g.first.first, g.first.second, std::vector<Request *>(v.begin() + at, v.begin() + at + B)});
    }
  }
  std::sort(chunks.begin(), chunks.end(), [](const Chunk &a, const Chunk &b) {
    if (a.reqs.size() != b.reqs.size()) return a.reqs.size() > b.reqs.size();
    return a.reqs.front()->id < b.reqs.front()->id;
  });
  for (Chunk &ch : chunks) {
    if (s->cfg.max_inflight && s->inflight.size() >= s->cfg.max_inflight) break;
    const NetPlan &np = s->nets[ch.net];
    const uint32_t k = ch.layer;
    const hc_layer *ly = np.layers[k];
    const uint32_t B = (uint32_t)ch.reqs.size();
    const uint32_t *in[hc::kMaxTab];
    const uint32_t *mk[hc::kMaxTab];
    uint32_t *c0[hc::kMaxTab];
    uint32_t *c1[hc::kMaxTab];
    for (uint32_t b = 0; b < B; ++b) {
      char *base = s->arena + ch.reqs[b]->off;
      in[b] = (const uint32_t *)(base + np.off_in[k]);
      mk[b] = (const uint32_t *)(base + np.off_mask[k]);
      c0[b] = (uint32_t *)(base + np.off_c0[k]);
      c1[b] = (uint32_t *)(base + np.off_c1[k]);
    }
    const uint32_t si = s->rr++ % (uint32_t)s->streams.size();
    if (B == 1 && ly->direct_one) {
      // a lone image on a layer where the coefficient-domain conv is faster (same bits)
      SV_HIP(hc::launch_conv_direct(ly->geom, in[0], ly->d_wt, ly->wt_rows, mk[0], c0[0], c1[0], 1,
                                    hc::direct_consts(*ly->ctx), ly->ctx->consts, s->streams[si]));
      s->st.direct_groups++;
    } else {
      hc_status cs = hc::enqueue_conv_gather(ly, B, in, mk, c0, c1, s->ws[si], s->streams[si]);
      if (cs != HC_OK) return cs;
    }
    int ev = ev_get(s);
    if (ev < 0) return fail(HC_EDEVICE, "event creation");
    SV_HIP(hipEventRecord(s->events[ev], s->streams[si]));
    s->ev_refs[ev] = (int)B + 1;  // the group's requests and the in-flight list
    s->inflight.push_back(ev);
    for (uint32_t b = 0; b < B; ++b) ch.reqs[b]->group = ev;
    s->st.groups++;
    s->st.images += B;
  }
  return HC_OK;
}

hc_status hc_server_poll(hc_server *s, uint64_t *ids, uint32_t cap, uint32_t *n) {
  if (!s || !n || (cap && !ids)) return fail(HC_EINVAL, "null argument");
  const uint32_t m = (uint32_t)std::min<size_t>(cap, s->completed.size());
  for (uint32_t i = 0; i < m; ++i) ids[i] = s->completed[i];
  s->completed.erase(s->completed.begin(), s->completed.begin() + m);
  *n = m;
  return HC_OK;
}

hc_status hc_server_outputs(const hc_server *s, uint64_t id, uint32_t layer, uint32_t **c0_ext, uint32_t **c1_out) {
  if (!s || !c0_ext || !c1_out) return fail(HC_EINVAL, "null argument");
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return fail(HC_EINVAL, "unknown request");
  const Request &r = it->second;
  if (!r.admitted) return fail(HC_ESTATE, "request not admitted yet");
  const NetPlan &np = s->nets[r.net];
  if (layer >= np.layers.size()) return fail(HC_EINVAL, "layer out of range");
  *c0_ext = (uint32_t *)(s->arena + r.off + np.off_c0[layer]);
  *c1_out = (uint32_t *)(s->arena + r.off + np.off_c1[layer]);
  return HC_OK;
}

hc_status hc_server_release(hc_server *s, uint64_t id) {
  if (!s) return fail(HC_EINVAL, "null server");
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return fail(HC_EINVAL, "unknown request");
  if (!it->second.done) return fail(HC_ESTATE, "request still running");
  s->alloc.release(it->second.off, s->nets[it->second.net].bytes);
  s->reqs.erase(it);
  return HC_OK;
}

hc_status hc_server_get_stats(const hc_server *s, hc_server_stats *out) {
  if (!s || !out) return fail(HC_EINVAL, "null argument");
  *out = s->st;
  out->queued = s->queue.size();
  out->arena_used = s->alloc.used();
  out->arena_bytes = s->alloc.total();
  return HC_OK;
}

hc_status hc_server_sync(hc_server *s) {
  if (!s) return fail(HC_EINVAL, "null server");
  hc::DeviceGuard dg(s->ctx->device);
  SV_HIP(hipStreamSynchronize(s->copy));
  for (auto st : s->streams) SV_HIP(hipStreamSynchronize(st));
  return HC_OK;
}

void hc_server_destroy(hc_server *s) {
  if (!s) return;
  hc::DeviceGuard dg(s->ctx->device);
  if (s->copy) (void)hipStreamSynchronize(s->copy);
  for (auto st : s->streams)
    if (st) (void)hipStreamSynchronize(st);
  for (auto st : s->streams)
    if (st) (void)hipStreamDestroy(st);
  if (s->copy) (void)hipStreamDestroy(s->copy);
  for (auto e : s->events) (void)hipEventDestroy(e);
  for (char *p : s->ws)
    if (p) (void)hipFree(p);
  if (s->arena) (void)hipFree(s->arena);
  delete s;
}

}  // extern "C"
