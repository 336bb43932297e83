// Trigger serving loop: continuous batching of events of any size over a
// fixed set of device-resident slots (see the declarations for the contract).
//
// A slot is one stream (default priority) with everything an event needs
// already allocated: a plan per grid kind (constant tables and scratch), one
// accumulator and peak list of the largest kind, the cluster outputs, and
// pinned host staging for the hits in and the results out.  An event runs
// on a free slot as: 4 copies of the hits and their count to the device, the
// device part (vote, peaks, refinement and vertex transform, copy of the
// results to the pinned output), and an event marker.  The device part is a
// HIP graph per kind captured once: every kernel takes the hit count from
// device memory, bounded by max_hits, so one graph serves any event size.
// Graphs hold no memset nodes (all clearing is done by kernels).
//
// Host side: submit copies the hits into the slot's pinned input (or, when
// every slot is busy, into a FIFO entry), poll finds finished slots by
// querying their markers, copies the results out and starts the next queued
// events on free slots.  Admission: the slot count is the largest that fits
// the HBM budget; an optional work budget bounds the hit-columns in flight
// (strict FIFO, an event runs alone when nothing else does); the FIFO is
// bounded, and beyond it events are shed.
#include <string.h>
#include <time.h>

#include <deque>
#include <new>
#include <vector>

#include "ht_internal.h"

// layouts the Python binding mirrors
static_assert(sizeof(ht_server_kind) == 112, "ht_server_kind layout");
static_assert(sizeof(ht_server_cfg) == 504, "ht_server_cfg layout");
static_assert(sizeof(ht_server_out) == 56, "ht_server_out layout");
static_assert(sizeof(ht_server_result) == 88, "ht_server_result layout");

namespace {

double now_s() {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

struct Job {
  int32_t kind = 0, n_hits = 0;
  uint64_t tag = 0;
  ht_server_out out{};
  double t_submit = 0.0;
  std::vector<float> r, phi;       // queued events only
  std::vector<uint8_t> layer;
};

// pinned result block of a slot, copied back by the device part
struct HostOut {
  int32_t counts[8];
  int32_t n_peaks;
  int32_t pad[7];
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t start = nullptr, done = nullptr;
  ht_plan* plan[HT_SERVER_MAX_KINDS] = {};
  hipGraph_t graph[HT_SERVER_MAX_KINDS] = {};
  hipGraphExec_t exec[HT_SERVER_MAX_KINDS] = {};
  // device
  int32_t* d_nhits = nullptr;
  float* d_r = nullptr;
  float* d_phi = nullptr;
  uint8_t* d_layer = nullptr;
  int32_t* d_acc = nullptr;
  ht_peak* d_peaks = nullptr;
  int32_t* d_npeaks = nullptr;
  int32_t* d_hit_owner = nullptr;
  ht_track* d_tracks = nullptr;
  ht_object* d_objects = nullptr;
  int32_t* d_members = nullptr;
  int32_t* d_counts = nullptr;
  // pinned host
  int32_t* h_nhits = nullptr;
  float* h_r = nullptr;
  float* h_phi = nullptr;
  uint8_t* h_layer = nullptr;
  HostOut* h_out = nullptr;
  int32_t* h_hit_owner = nullptr;
  ht_track* h_tracks = nullptr;
  ht_object* h_objects = nullptr;
  int32_t* h_members = nullptr;
  // state
  bool busy = false;
  int64_t work = 0;  // hit-columns of the running event
  Job job;
  double t_start = 0.0;
  int status = HT_OK;
};

}  // namespace

struct ht_server {
  ht_server_cfg cfg;
  std::vector<Slot> slots;
  std::deque<Job> queue;
  int64_t slot_bytes = 0;
  int64_t in_flight = 0;  // hit-columns of the running events
};

namespace {

template <typename T>
int dev_alloc(T** p, size_t n, int64_t* bytes) {
  *p = nullptr;
  if (n == 0) n = 1;
  if (hipMalloc((void**)p, n * sizeof(T)) != hipSuccess) {
    *p = nullptr;
    return HT_ENOMEM;
  }
  *bytes += (int64_t)(n * sizeof(T));
  return HT_OK;
}

template <typename T>
int host_alloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  if (hipHostMalloc((void**)p, n * sizeof(T), hipHostMallocDefault) != hipSuccess) {
    *p = nullptr;
    return HT_ENOMEM;
  }
  return HT_OK;
}

void free_slot(Slot& s) {
  for (int k = 0; k < HT_SERVER_MAX_KINDS; ++k) {
    if (s.exec[k]) (void)hipGraphExecDestroy(s.exec[k]);
    if (s.graph[k]) (void)hipGraphDestroy(s.graph[k]);
    if (s.plan[k]) ht_plan_destroy(s.plan[k]);
    s.exec[k] = nullptr;
    s.graph[k] = nullptr;
    s.plan[k] = nullptr;
  }
  void* dptrs[] = {s.d_nhits, s.d_r, s.d_phi, s.d_layer, s.d_acc, s.d_peaks, s.d_npeaks,
                   s.d_hit_owner, s.d_tracks, s.d_objects, s.d_members, s.d_counts};
  for (void* q : dptrs)
    if (q) (void)hipFree(q);
  void* hptrs[] = {s.h_nhits, s.h_r, s.h_phi, s.h_layer, s.h_out, s.h_hit_owner, s.h_tracks,
                   s.h_objects, s.h_members};
  for (void* q : hptrs)
    if (q) (void)hipHostFree(q);
  if (s.start) (void)hipEventDestroy(s.start);
  if (s.done) (void)hipEventDestroy(s.done);
  if (s.stream) (void)hipStreamDestroy(s.stream);
  s = Slot();
}

// The device part of one event of kind k on slot s (captured into a graph,
// or launched directly).  Copies back fixed-size result blocks.
int device_part(const ht_server_cfg& c, Slot& s, int k) {
  const ht_server_kind& K = c.kinds[k];
  const ht::Plan& P = *s.plan[k];
  int rc = ht::launch_vote(P, s.d_r, s.d_phi, c.max_hits, s.d_acc, nullptr, s.stream, s.d_nhits);
  if (rc != HT_OK) return rc;
  rc = ht::launch_peaks(P, s.d_acc, K.min_votes, s.d_peaks, K.peak_cap, s.d_npeaks, s.stream);
  if (rc != HT_OK) return rc;
  ht_cluster_out o;
  o.hit_owner = s.d_hit_owner;
  o.tracks = s.d_tracks;
  o.track_cap = c.track_cap;
  o.objects = s.d_objects;
  o.object_cap = c.object_cap;
  o.members = s.d_members;
  o.member_cap = c.member_cap;
  o.vacc = nullptr;
  o.counts = s.d_counts;
  o.work = nullptr;
  rc = ht::launch_assoc(P, s.d_r, s.d_phi, s.d_layer, c.max_hits, s.d_peaks, s.d_npeaks,
                        K.peak_cap, s.d_acc, K.cluster, o, s.stream, s.d_nhits);
  if (rc != HT_OK) return rc;
  const hipMemcpyKind d2h = hipMemcpyDeviceToHost;
  HT_CHECK(hipMemcpyAsync(s.h_out->counts, s.d_counts, 8 * sizeof(int32_t), d2h, s.stream));
  HT_CHECK(hipMemcpyAsync(&s.h_out->n_peaks, s.d_npeaks, sizeof(int32_t), d2h, s.stream));
  HT_CHECK(hipMemcpyAsync(s.h_hit_owner, s.d_hit_owner, (size_t)c.max_hits * sizeof(int32_t), d2h,
                          s.stream));
  if (c.track_cap > 0)
    HT_CHECK(hipMemcpyAsync(s.h_tracks, s.d_tracks, (size_t)c.track_cap * sizeof(ht_track), d2h,
                            s.stream));
  if (c.object_cap > 0)
    HT_CHECK(hipMemcpyAsync(s.h_objects, s.d_objects, (size_t)c.object_cap * sizeof(ht_object),
                            d2h, s.stream));
  if (c.member_cap > 0)
    HT_CHECK(hipMemcpyAsync(s.h_members, s.d_members, (size_t)c.member_cap * sizeof(int32_t),
                            d2h, s.stream));
  return HT_OK;
}

int make_slot(const ht_server_cfg& c, Slot& s, int64_t* bytes) {
  *bytes = 0;
  HT_CHECK(hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking));
  HT_CHECK(hipEventCreate(&s.start));
  HT_CHECK(hipEventCreate(&s.done));
  int64_t max_cells = 0, max_peaks = 0;
  int rc = HT_OK;
  for (int k = 0; k < c.n_kinds && rc == HT_OK; ++k) {
    const ht_server_kind& K = c.kinds[k];
    ht_limits lim;
    lim.max_hits = c.max_hits;
    lim.max_peaks = K.peak_cap;
    lim.max_member_cap = K.cluster.member_cap;
    lim.max_tracks = c.track_cap > 0 ? c.track_cap : 1;
    lim.max_vertex_cells = K.cluster.n_rho * K.cluster.n_theta;
    lim.max_n_rho = K.cluster.n_rho;
    rc = ht_plan_create(&K.grid, &lim, &s.plan[k]);
    if (rc == HT_OK) rc = ht::check_cluster(*s.plan[k], K.cluster, c.max_hits, K.peak_cap, c.track_cap);
    if (s.plan[k]) *bytes += s.plan[k]->dev_bytes;  // what the plan allocated
    const int64_t cells = (int64_t)K.grid.n_phi * K.grid.n_qpt * K.grid.n_d0;
    if (cells > max_cells) max_cells = cells;
    if (K.peak_cap > max_peaks) max_peaks = K.peak_cap;
  }
  const size_t nh = (size_t)c.max_hits;
  if (rc == HT_OK) rc = dev_alloc(&s.d_nhits, 64, bytes);
  if (rc == HT_OK) rc = dev_alloc(&s.d_r, nh, bytes);
  if (rc == HT_OK) rc = dev_alloc(&s.d_phi, nh, bytes);
  if (rc == HT_OK) rc = dev_alloc(&s.d_layer, nh, bytes);
  if (rc == HT_OK) rc = dev_alloc(&s.d_acc, (size_t)max_cells, bytes);
  if (rc == HT_OK) rc = dev_alloc(&s.d_peaks, (size_t)max_peaks, bytes);
  if (rc == HT_OK) rc = dev_alloc(&s.d_npeaks, 64, bytes);
  if (rc == HT_OK) rc = dev_alloc(&s.d_hit_owner, nh, bytes);
  if (rc == HT_OK) rc = dev_alloc(&s.d_tracks, (size_t)c.track_cap, bytes);
  if (rc == HT_OK) rc = dev_alloc(&s.d_objects, (size_t)c.object_cap, bytes);
  if (rc == HT_OK) rc = dev_alloc(&s.d_members, (size_t)c.member_cap, bytes);
  if (rc == HT_OK) rc = dev_alloc(&s.d_counts, 64, bytes);
  if (rc == HT_OK) rc = host_alloc(&s.h_nhits, 64);
  if (rc == HT_OK) rc = host_alloc(&s.h_r, nh);
  if (rc == HT_OK) rc = host_alloc(&s.h_phi, nh);
  if (rc == HT_OK) rc = host_alloc(&s.h_layer, nh);
  if (rc == HT_OK) rc = host_alloc(&s.h_out, 1);
  if (rc == HT_OK) rc = host_alloc(&s.h_hit_owner, nh);
  if (rc == HT_OK) rc = host_alloc(&s.h_tracks, (size_t)c.track_cap);
  if (rc == HT_OK) rc = host_alloc(&s.h_objects, (size_t)c.object_cap);
  if (rc == HT_OK) rc = host_alloc(&s.h_members, (size_t)c.member_cap);
  if (rc != HT_OK) return rc;
  if (c.use_graphs) {
    for (int k = 0; k < c.n_kinds; ++k) {
      HT_CHECK(hipStreamBeginCapture(s.stream, hipStreamCaptureModeThreadLocal));
      const int drc = device_part(c, s, k);
      hipGraph_t g = nullptr;
      const hipError_t erc = hipStreamEndCapture(s.stream, &g);
      if (drc != HT_OK) {
        if (g) (void)hipGraphDestroy(g);
        return drc;
      }
      if (erc != hipSuccess || !g) return HT_EDEVICE;
      s.graph[k] = g;
      HT_CHECK(hipGraphInstantiate(&s.exec[k], g, nullptr, nullptr, 0));
    }
  }
  return HT_OK;
}

// start job j on slot s (inputs already in the slot's pinned buffers)
void start(const ht_server_cfg& c, Slot& s, Job&& j) {
  s.job = std::move(j);
  s.busy = true;
  s.t_start = now_s();
  const size_t n = (size_t)s.job.n_hits;
  const hipMemcpyKind h2d = hipMemcpyHostToDevice;
  *s.h_nhits = s.job.n_hits;
  int rc = HT_OK;
  if (hipEventRecord(s.start, s.stream) != hipSuccess ||
      hipMemcpyAsync(s.d_nhits, s.h_nhits, sizeof(int32_t), h2d, s.stream) != hipSuccess ||
      (n && (hipMemcpyAsync(s.d_r, s.h_r, n * sizeof(float), h2d, s.stream) != hipSuccess ||
             hipMemcpyAsync(s.d_phi, s.h_phi, n * sizeof(float), h2d, s.stream) != hipSuccess ||
             hipMemcpyAsync(s.d_layer, s.h_layer, n, h2d, s.stream) != hipSuccess)))
    rc = HT_EDEVICE;
  if (rc == HT_OK) {
    if (c.use_graphs)
      rc = hipGraphLaunch(s.exec[s.job.kind], s.stream) == hipSuccess ? HT_OK : HT_EDEVICE;
    else
      rc = device_part(c, s, s.job.kind);
  }
  if (hipEventRecord(s.done, s.stream) != hipSuccess && rc == HT_OK) rc = HT_EDEVICE;
  s.status = rc;
}

void stage_inputs(Slot& s, const float* r, const float* phi, const uint8_t* layer, int32_t n) {
  if (n > 0) {
    memcpy(s.h_r, r, (size_t)n * sizeof(float));
    memcpy(s.h_phi, phi, (size_t)n * sizeof(float));
    memcpy(s.h_layer, layer, (size_t)n);
  }
}

void finish(const ht_server_cfg& c, Slot& s, ht_server_result* res) {
  const Job& j = s.job;
  res->tag = j.tag;
  res->kind = j.kind;
  res->n_hits = j.n_hits;
  res->status = s.status;
  res->n_peaks = s.h_out->n_peaks;
  memcpy(res->counts, s.h_out->counts, sizeof(res->counts));
  res->t_submit = j.t_submit;
  res->t_start = s.t_start;
  res->t_done = now_s();
  float ms = 0.0f;
  res->device_ms = hipEventElapsedTime(&ms, s.start, s.done) == hipSuccess ? (double)ms : -1.0;
  const ht_server_out& o = j.out;
  if (o.tracks && o.track_cap > 0) {
    int32_t n = s.h_out->counts[1];
    n = n < o.track_cap ? n : o.track_cap;
    n = n < c.track_cap ? n : c.track_cap;
    if (n > 0) memcpy(o.tracks, s.h_tracks, (size_t)n * sizeof(ht_track));
  }
  if (o.hit_owner && j.n_hits > 0) memcpy(o.hit_owner, s.h_hit_owner, (size_t)j.n_hits * sizeof(int32_t));
  if (o.objects && o.object_cap > 0) {
    int32_t n = s.h_out->counts[2];
    n = n < o.object_cap ? n : o.object_cap;
    n = n < c.object_cap ? n : c.object_cap;
    if (n > 0) memcpy(o.objects, s.h_objects, (size_t)n * sizeof(ht_object));
  }
  if (o.members && o.member_cap > 0) {
    int32_t n = s.h_out->counts[3];
    n = n < o.member_cap ? n : o.member_cap;
    n = n < c.member_cap ? n : c.member_cap;
    if (n > 0) memcpy(o.members, s.h_members, (size_t)n * sizeof(int32_t));
  }
  s.busy = false;
}

// an event's work: hits times the columns of its kind's grid
int64_t job_work(const ht_server_cfg& c, const Job& j) {
  const ht_grid& g = c.kinds[j.kind].grid;
  return (int64_t)j.n_hits * g.n_qpt * g.n_d0;
}

// whether an event of work w may start now (a slot being free aside)
bool fits(const ht_server* srv, int64_t w) {
  const int64_t b = srv->cfg.work_budget;
  return b <= 0 || srv->in_flight == 0 || srv->in_flight + w <= b;
}

Slot* free_slot_of(ht_server* srv) {
  for (Slot& s : srv->slots)
    if (!s.busy) return &s;
  return nullptr;
}

void run(ht_server* srv, Slot& s, Job&& j) {
  s.work = job_work(srv->cfg, j);
  srv->in_flight += s.work;
  start(srv->cfg, s, std::move(j));
}

bool cfg_ok(const ht_server_cfg& c) {
  if (c.n_kinds < 1 || c.n_kinds > HT_SERVER_MAX_KINDS) return false;
  if (c.max_hits < 1 || c.max_hits > 65535 || c.track_cap < 0 || c.object_cap < 0 ||
      c.member_cap < 0 || c.max_slots < 1 || c.queue_cap < 0 || c.hbm_budget <= 0 ||
      c.work_budget < 0)
    return false;
  for (int k = 0; k < c.n_kinds; ++k)
    if (c.kinds[k].peak_cap < 1) return false;
  return true;
}

}  // namespace

extern "C" {

int ht_server_create(const ht_server_cfg* cfg, ht_server** out) {
  if (!out) return HT_EINVAL;
  *out = nullptr;
  if (!cfg || !cfg_ok(*cfg)) return HT_EINVAL;
  ht_server* srv = new (std::nothrow) ht_server();
  if (!srv) return HT_ENOMEM;
  srv->cfg = *cfg;
  srv->slots.reserve((size_t)cfg->max_slots);
  int rc = HT_OK;
  int64_t used = 0;
  while ((int)srv->slots.size() < cfg->max_slots) {
    Slot s;
    int64_t bytes = 0;
    rc = make_slot(*cfg, s, &bytes);
    if (rc != HT_OK || used + bytes > cfg->hbm_budget) {
      free_slot(s);
      if (rc == HT_OK || rc == HT_ENOMEM) rc = HT_OK;  // the budget or the device is full
      break;
    }
    used += bytes;
    srv->slot_bytes = bytes;
    srv->slots.push_back(s);
  }
  if (rc == HT_OK && srv->slots.empty()) rc = HT_ENOMEM;
  if (rc != HT_OK) {
    for (Slot& s : srv->slots) free_slot(s);
    delete srv;
    return rc;
  }
  *out = srv;
  return HT_OK;
}

int ht_server_destroy(ht_server* srv) {
  if (!srv) return HT_EINVAL;
  for (Slot& s : srv->slots) {
    if (s.stream) (void)hipStreamSynchronize(s.stream);
    free_slot(s);
  }
  delete srv;
  return HT_OK;
}

int ht_server_info(const ht_server* srv, int32_t* n_slots, int64_t* slot_bytes) {
  if (!srv || !n_slots || !slot_bytes) return HT_EINVAL;
  *n_slots = (int32_t)srv->slots.size();
  *slot_bytes = srv->slot_bytes;
  return HT_OK;
}

int ht_server_submit(ht_server* srv, int32_t kind, const float* r, const float* phi,
                     const uint8_t* layer, int32_t n_hits, const ht_server_out* out,
                     uint64_t tag) {
  if (!srv || kind < 0 || kind >= srv->cfg.n_kinds || n_hits < 0) return HT_EINVAL;
  if (n_hits > 0 && (!r || !phi || !layer)) return HT_EINVAL;
  if (n_hits > srv->cfg.max_hits) return HT_EUNSUPPORTED;
  Job j;
  j.kind = kind;
  j.n_hits = n_hits;
  j.tag = tag;
  if (out) j.out = *out;
  j.t_submit = now_s();
  if (srv->queue.empty() && fits(srv, job_work(srv->cfg, j))) {
    if (Slot* s = free_slot_of(srv)) {
      stage_inputs(*s, r, phi, layer, n_hits);
      run(srv, *s, std::move(j));
      return HT_OK;
    }
  }
  if ((int32_t)srv->queue.size() >= srv->cfg.queue_cap) return HT_EBUSY;
  j.r.assign(r, r + n_hits);
  j.phi.assign(phi, phi + n_hits);
  j.layer.assign(layer, layer + n_hits);
  srv->queue.push_back(std::move(j));
  return HT_OK;
}

int ht_server_poll(ht_server* srv, ht_server_result* results, int32_t max, int32_t wait,
                   int32_t* n_results) {
  if (!srv || !n_results || max < 0 || (max > 0 && !results)) return HT_EINVAL;
  *n_results = 0;
  for (;;) {
    bool pending = false;
    for (Slot& s : srv->slots) {
      if (!s.busy) continue;
      pending = true;
      if (*n_results >= max) continue;
      const hipError_t q = hipEventQuery(s.done);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) s.status = HT_EDEVICE;
      finish(srv->cfg, s, &results[(*n_results)++]);
      srv->in_flight -= s.work;
      s.work = 0;
    }
    // start waiting events in FIFO order while a slot and the budget allow
    while (!srv->queue.empty() && fits(srv, job_work(srv->cfg, srv->queue.front()))) {
      Slot* s = free_slot_of(srv);
      if (!s) break;
      Job j = std::move(srv->queue.front());
      srv->queue.pop_front();
      stage_inputs(*s, j.r.data(), j.phi.data(), j.layer.data(), j.n_hits);
      j.r.clear();
      j.phi.clear();
      j.layer.clear();
      run(srv, *s, std::move(j));
      pending = true;
    }
    if (!wait || *n_results > 0 || !pending || *n_results >= max) break;
  }
  return HT_OK;
}

}  // extern "C"
