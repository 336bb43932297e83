// Trigger serving loop: continuous batching of events of any size over a
// fixed set of device-resident slots (see the declarations for the contract).
//
// A slot is one stream (default priority) with room for a batch of up to
// batch_max events.  Each event place of a slot has everything an event needs
// already allocated: a plan per grid kind (constant tables and scratch), one
// accumulator and peak list of the largest kind, the learned filter's logits,
// kept list and workspace when a kind has a filter, the cluster outputs, and
// pinned host staging for the hits in and the results out.  Place 0 takes
// events of up to max_hits hits, the others up to batch_max_hits.  A batch of
// nb events of one kind runs as: 4 copies per event of the hits and their
// count to the device, the device part (one launch of the vote, of each peak
// finder stage and of each assoc_cluster kernel for the whole batch, the
// filter's launches per event, copies of the results to the pinned outputs),
// and an event marker.  The device part is a HIP graph per kind and batch
// size captured once: every kernel takes the hit counts from device memory,
// bounded by the places' hit bound, so one graph serves any event sizes.
// Graphs hold no memset nodes (all clearing is done by kernels).
//
// Host side: submit copies the hits into a free slot's pinned input when
// nothing waits (the event starts at once, alone), else into a FIFO entry;
// poll finds finished slots by querying their markers, copies the results
// out and starts the waiting events on free slots, oldest first, each joined
// by later small events of its kind while it is small itself (batches form
// only under load, so an idle server adds no latency).  Admission: the slot
// count is the largest that fits the HBM budget; an optional work budget
// bounds the hit-columns in flight (a batch runs alone when nothing else
// does); the FIFO is bounded, and beyond it events are shed.
#include <string.h>
#include <time.h>

#include <deque>
#include <new>
#include <vector>

#include "ht_internal.h"

// layouts the Python binding mirrors
static_assert(sizeof(ht_server_kind) == 128, "ht_server_kind layout");
static_assert(sizeof(ht_server_cfg) == 576, "ht_server_cfg layout");
static_assert(sizeof(ht_server_out) == 56, "ht_server_out layout");
static_assert(sizeof(ht_server_result) == 96, "ht_server_result layout");

namespace {

constexpr int kKinds = HT_SERVER_MAX_KINDS;
constexpr int kBatch = HT_MAX_BATCH;

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

// pinned result block of an event place, copied back by the device part
struct HostOut {
  int32_t counts[8];
  int32_t n_peaks;
  int32_t n_kept;
  int32_t pad[6];
};

// one event place of a slot
struct Place {
  ht_plan* plan[kKinds] = {};
  int32_t max_hits = 0;  // hit bound of the place
  // device
  int32_t* d_nhits = nullptr;
  float* d_r = nullptr;
  float* d_phi = nullptr;
  uint8_t* d_layer = nullptr;
  int32_t* d_acc = nullptr;
  ht_peak* d_peaks = nullptr;
  int32_t* d_npeaks = nullptr;
  float* d_logits = nullptr;  // learned filter (kinds with parameters only)
  char* d_ws = nullptr;
  ht_peak* d_kept = nullptr;
  int32_t* d_nkept = nullptr;
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
  Job job;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t start = nullptr, done = nullptr;
  hipGraph_t graph[kKinds][kBatch] = {};
  hipGraphExec_t exec[kKinds][kBatch] = {};
  Place place[kBatch];
  int n_places = 0;
  // state
  bool busy = false;
  int nb = 0;        // events of the running batch
  int kind = 0;
  int64_t work = 0;  // hit-columns of the running batch
  double t_start = 0.0;
  int status = HT_OK;
};

}  // namespace

struct ht_server {
  ht_server_cfg cfg;
  int batch_max = 1;       // events per batch at most
  int32_t batch_hits = 0;  // hit bound of the places after the first
  float* d_params[kKinds] = {};  // the kinds' filter parameters on the device
  std::vector<Slot> slots;
  std::deque<Job> queue;
  int64_t slot_bytes = 0;
  int64_t in_flight = 0;  // hit-columns of the running batches
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

void free_place(Place& u) {
  for (int k = 0; k < kKinds; ++k) {
    if (u.plan[k]) ht_plan_destroy(u.plan[k]);
    u.plan[k] = nullptr;
  }
  void* dptrs[] = {u.d_nhits,  u.d_r,     u.d_phi,       u.d_layer,  u.d_acc,
                   u.d_peaks,  u.d_npeaks, u.d_logits,   u.d_ws,     u.d_kept,
                   u.d_nkept,  u.d_hit_owner, u.d_tracks, u.d_objects, u.d_members,
                   u.d_counts};
  for (void* q : dptrs)
    if (q) (void)hipFree(q);
  void* hptrs[] = {u.h_nhits, u.h_r,       u.h_phi,    u.h_layer,  u.h_out,
                   u.h_hit_owner, u.h_tracks, u.h_objects, u.h_members};
  for (void* q : hptrs)
    if (q) (void)hipHostFree(q);
  u = Place();
}

void free_slot(Slot& s) {
  for (int k = 0; k < kKinds; ++k)
    for (int b = 0; b < kBatch; ++b) {
      if (s.exec[k][b]) (void)hipGraphExecDestroy(s.exec[k][b]);
      if (s.graph[k][b]) (void)hipGraphDestroy(s.graph[k][b]);
    }
  for (int b = 0; b < kBatch; ++b) free_place(s.place[b]);
  if (s.start) (void)hipEventDestroy(s.start);
  if (s.done) (void)hipEventDestroy(s.done);
  if (s.stream) (void)hipStreamDestroy(s.stream);
  s = Slot();
}

// The device part of a batch of nb events of kind k on slot s (captured into
// a graph, or launched directly).  Copies back fixed-size result blocks.
int device_part(const ht_server* srv, Slot& s, int k, int nb) {
  const ht_server_cfg& c = srv->cfg;
  const ht_server_kind& K = c.kinds[k];
  const float* params = srv->d_params[k];
  // a batch of one runs on place 0 at its full bound; larger batches hold
  // small events only
  const int32_t nmax = nb == 1 ? s.place[0].max_hits : srv->batch_hits;
  const ht::Plan* plans[kBatch];
  const float* r[kBatch];
  const float* phi[kBatch];
  const int32_t* nd[kBatch];
  int32_t* acc[kBatch];
  const int32_t* cacc[kBatch];
  ht_peak* pk[kBatch];
  int32_t* nf[kBatch];
  for (int b = 0; b < nb; ++b) {
    Place& u = s.place[b];
    plans[b] = u.plan[k];
    r[b] = u.d_r;
    phi[b] = u.d_phi;
    nd[b] = u.d_nhits;
    acc[b] = u.d_acc;
    cacc[b] = u.d_acc;
    pk[b] = u.d_peaks;
    nf[b] = u.d_npeaks;
  }
  int rc = ht::launch_vote_batch(*plans[0], nb, r, phi, nd, nmax, acc, s.stream);
  if (rc != HT_OK) return rc;
  rc = ht::launch_peaks_batch(nb, plans, cacc, K.min_votes, pk, K.peak_cap, nf, s.stream);
  if (rc != HT_OK) return rc;
  ht::AssocEvent ae[kBatch];
  for (int b = 0; b < nb; ++b) {
    Place& u = s.place[b];
    const ht_peak* use = u.d_peaks;
    const int32_t* n_use = u.d_npeaks;
    if (params) {
      rc = ht::launch_cnn_score(*plans[b], params, u.d_acc, u.d_peaks, u.d_npeaks, K.peak_cap,
                                u.d_logits, u.d_ws, s.stream);
      if (rc == HT_OK)
        rc = ht::launch_cnn_keep(*plans[b], u.d_logits, u.d_peaks, u.d_npeaks, K.peak_cap,
                                 K.cnn_threshold, u.d_kept, K.peak_cap, u.d_nkept, s.stream);
      if (rc != HT_OK) return rc;
      use = u.d_kept;
      n_use = u.d_nkept;
    }
    ht_cluster_out o;
    o.hit_owner = u.d_hit_owner;
    o.tracks = u.d_tracks;
    o.track_cap = c.track_cap;
    o.objects = u.d_objects;
    o.object_cap = c.object_cap;
    o.members = u.d_members;
    o.member_cap = c.member_cap;
    o.vacc = nullptr;
    o.counts = u.d_counts;
    o.work = nullptr;
    ae[b] = ht::AssocEvent{plans[b], u.d_r, u.d_phi, u.d_layer, u.d_nhits, use, n_use,
                           u.d_acc, o};
  }
  rc = ht::launch_assoc_batch(nb, ae, nmax, K.peak_cap, K.cluster, s.stream);
  if (rc != HT_OK) return rc;
  const hipMemcpyKind d2h = hipMemcpyDeviceToHost;
  for (int b = 0; b < nb; ++b) {
    Place& u = s.place[b];
    HT_CHECK(hipMemcpyAsync(u.h_out->counts, u.d_counts, 8 * sizeof(int32_t), d2h, s.stream));
    HT_CHECK(hipMemcpyAsync(&u.h_out->n_peaks, u.d_npeaks, sizeof(int32_t), d2h, s.stream));
    HT_CHECK(hipMemcpyAsync(&u.h_out->n_kept, params ? u.d_nkept : u.d_npeaks, sizeof(int32_t),
                            d2h, s.stream));
    HT_CHECK(hipMemcpyAsync(u.h_hit_owner, u.d_hit_owner, (size_t)nmax * sizeof(int32_t), d2h,
                            s.stream));
    if (c.track_cap > 0)
      HT_CHECK(hipMemcpyAsync(u.h_tracks, u.d_tracks, (size_t)c.track_cap * sizeof(ht_track), d2h,
                              s.stream));
    if (c.object_cap > 0)
      HT_CHECK(hipMemcpyAsync(u.h_objects, u.d_objects, (size_t)c.object_cap * sizeof(ht_object),
                              d2h, s.stream));
    if (c.member_cap > 0)
      HT_CHECK(hipMemcpyAsync(u.h_members, u.d_members, (size_t)c.member_cap * sizeof(int32_t),
                              d2h, s.stream));
  }
  return HT_OK;
}

// one event place: plans for every kind and the buffers, for events of at
// most nh hits
int make_place(const ht_server* srv, Place& u, int32_t nh, int64_t* bytes) {
  const ht_server_cfg& c = srv->cfg;
  u.max_hits = nh;
  int64_t max_cells = 0, max_peaks = 0, filter_peaks = 0;
  int rc = HT_OK;
  for (int k = 0; k < c.n_kinds && rc == HT_OK; ++k) {
    const ht_server_kind& K = c.kinds[k];
    ht_limits lim;
    lim.max_hits = nh;
    lim.max_peaks = K.peak_cap;
    lim.max_member_cap = K.cluster.member_cap;
    lim.max_tracks = c.track_cap > 0 ? c.track_cap : 1;
    lim.max_vertex_cells = K.cluster.n_rho * K.cluster.n_theta;
    lim.max_n_rho = K.cluster.n_rho;
    rc = ht_plan_create(&K.grid, &lim, &u.plan[k]);
    if (rc == HT_OK) rc = ht::check_cluster(*u.plan[k], K.cluster, nh, K.peak_cap, c.track_cap);
    if (u.plan[k]) *bytes += u.plan[k]->dev_bytes;  // what the plan allocated
    const int64_t cells = (int64_t)K.grid.n_phi * K.grid.n_qpt * K.grid.n_d0;
    if (cells > max_cells) max_cells = cells;
    if (K.peak_cap > max_peaks) max_peaks = K.peak_cap;
    if (K.cnn_params && K.peak_cap > filter_peaks) filter_peaks = K.peak_cap;
  }
  const size_t n = (size_t)nh;
  if (rc == HT_OK) rc = dev_alloc(&u.d_nhits, 64, bytes);
  if (rc == HT_OK) rc = dev_alloc(&u.d_r, n, bytes);
  if (rc == HT_OK) rc = dev_alloc(&u.d_phi, n, bytes);
  if (rc == HT_OK) rc = dev_alloc(&u.d_layer, n, bytes);
  if (rc == HT_OK) rc = dev_alloc(&u.d_acc, (size_t)max_cells, bytes);
  if (rc == HT_OK) rc = dev_alloc(&u.d_peaks, (size_t)max_peaks, bytes);
  if (rc == HT_OK) rc = dev_alloc(&u.d_npeaks, 64, bytes);
  if (rc == HT_OK && filter_peaks > 0) {
    rc = dev_alloc(&u.d_logits, (size_t)filter_peaks, bytes);
    if (rc == HT_OK)
      rc = dev_alloc(&u.d_ws, ht::cnn_workspace_bytes((int32_t)filter_peaks, 0), bytes);
    if (rc == HT_OK) rc = dev_alloc(&u.d_kept, (size_t)filter_peaks, bytes);
    if (rc == HT_OK) rc = dev_alloc(&u.d_nkept, 64, bytes);
  }
  if (rc == HT_OK) rc = dev_alloc(&u.d_hit_owner, n, bytes);
  if (rc == HT_OK) rc = dev_alloc(&u.d_tracks, (size_t)c.track_cap, bytes);
  if (rc == HT_OK) rc = dev_alloc(&u.d_objects, (size_t)c.object_cap, bytes);
  if (rc == HT_OK) rc = dev_alloc(&u.d_members, (size_t)c.member_cap, bytes);
  if (rc == HT_OK) rc = dev_alloc(&u.d_counts, 64, bytes);
  if (rc == HT_OK) rc = host_alloc(&u.h_nhits, 64);
  if (rc == HT_OK) rc = host_alloc(&u.h_r, n);
  if (rc == HT_OK) rc = host_alloc(&u.h_phi, n);
  if (rc == HT_OK) rc = host_alloc(&u.h_layer, n);
  if (rc == HT_OK) rc = host_alloc(&u.h_out, 1);
  if (rc == HT_OK) rc = host_alloc(&u.h_hit_owner, n);
  if (rc == HT_OK) rc = host_alloc(&u.h_tracks, (size_t)c.track_cap);
  if (rc == HT_OK) rc = host_alloc(&u.h_objects, (size_t)c.object_cap);
  if (rc == HT_OK) rc = host_alloc(&u.h_members, (size_t)c.member_cap);
  return rc;
}

int make_slot(const ht_server* srv, Slot& s, int64_t* bytes) {
  const ht_server_cfg& c = srv->cfg;
  *bytes = 0;
  HT_CHECK(hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking));
  HT_CHECK(hipEventCreate(&s.start));
  HT_CHECK(hipEventCreate(&s.done));
  for (int b = 0; b < srv->batch_max; ++b) {
    const int rc = make_place(srv, s.place[b], b == 0 ? c.max_hits : srv->batch_hits, bytes);
    s.n_places = b + 1;
    if (rc != HT_OK) return rc;
  }
  if (c.use_graphs) {
    for (int k = 0; k < c.n_kinds; ++k)
      for (int nb = 1; nb <= srv->batch_max; ++nb) {
        HT_CHECK(hipStreamBeginCapture(s.stream, hipStreamCaptureModeThreadLocal));
        const int drc = device_part(srv, s, k, nb);
        hipGraph_t g = nullptr;
        const hipError_t erc = hipStreamEndCapture(s.stream, &g);
        if (drc != HT_OK) {
          if (g) (void)hipGraphDestroy(g);
          return drc;
        }
        if (erc != hipSuccess || !g) return HT_EDEVICE;
        s.graph[k][nb - 1] = g;
        HT_CHECK(hipGraphInstantiate(&s.exec[k][nb - 1], g, nullptr, nullptr, 0));
      }
  }
  return HT_OK;
}

void stage_inputs(Place& u, const float* r, const float* phi, const uint8_t* layer, int32_t n) {
  if (n > 0) {
    memcpy(u.h_r, r, (size_t)n * sizeof(float));
    memcpy(u.h_phi, phi, (size_t)n * sizeof(float));
    memcpy(u.h_layer, layer, (size_t)n);
  }
}

// start the batch already staged in the first s.nb places of slot s
void start(const ht_server* srv, Slot& s) {
  s.busy = true;
  s.t_start = now_s();
  const hipMemcpyKind h2d = hipMemcpyHostToDevice;
  int rc = hipEventRecord(s.start, s.stream) == hipSuccess ? HT_OK : HT_EDEVICE;
  for (int b = 0; b < s.nb && rc == HT_OK; ++b) {
    Place& u = s.place[b];
    const size_t n = (size_t)u.job.n_hits;
    *u.h_nhits = u.job.n_hits;
    if (hipMemcpyAsync(u.d_nhits, u.h_nhits, sizeof(int32_t), h2d, s.stream) != hipSuccess ||
        (n && (hipMemcpyAsync(u.d_r, u.h_r, n * sizeof(float), h2d, s.stream) != hipSuccess ||
               hipMemcpyAsync(u.d_phi, u.h_phi, n * sizeof(float), h2d, s.stream) != hipSuccess ||
               hipMemcpyAsync(u.d_layer, u.h_layer, n, h2d, s.stream) != hipSuccess)))
      rc = HT_EDEVICE;
  }
  if (rc == HT_OK) {
    if (srv->cfg.use_graphs)
      rc = hipGraphLaunch(s.exec[s.kind][s.nb - 1], s.stream) == hipSuccess ? HT_OK : HT_EDEVICE;
    else
      rc = device_part(srv, s, s.kind, s.nb);
  }
  if (hipEventRecord(s.done, s.stream) != hipSuccess && rc == HT_OK) rc = HT_EDEVICE;
  s.status = rc;
}

void finish_one(const ht_server_cfg& c, const Slot& s, const Place& u, double t_done, double ms,
                ht_server_result* res) {
  const Job& j = u.job;
  res->tag = j.tag;
  res->kind = j.kind;
  res->n_hits = j.n_hits;
  res->status = s.status;
  res->n_peaks = u.h_out->n_peaks;
  res->n_kept = u.h_out->n_kept;
  res->batch = s.nb;
  memcpy(res->counts, u.h_out->counts, sizeof(res->counts));
  res->t_submit = j.t_submit;
  res->t_start = s.t_start;
  res->t_done = t_done;
  res->device_ms = ms;
  const ht_server_out& o = j.out;
  if (o.tracks && o.track_cap > 0) {
    int32_t n = u.h_out->counts[1];
    n = n < o.track_cap ? n : o.track_cap;
    n = n < c.track_cap ? n : c.track_cap;
    if (n > 0) memcpy(o.tracks, u.h_tracks, (size_t)n * sizeof(ht_track));
  }
  if (o.hit_owner && j.n_hits > 0)
    memcpy(o.hit_owner, u.h_hit_owner, (size_t)j.n_hits * sizeof(int32_t));
  if (o.objects && o.object_cap > 0) {
    int32_t n = u.h_out->counts[2];
    n = n < o.object_cap ? n : o.object_cap;
    n = n < c.object_cap ? n : c.object_cap;
    if (n > 0) memcpy(o.objects, u.h_objects, (size_t)n * sizeof(ht_object));
  }
  if (o.members && o.member_cap > 0) {
    int32_t n = u.h_out->counts[3];
    n = n < o.member_cap ? n : o.member_cap;
    n = n < c.member_cap ? n : c.member_cap;
    if (n > 0) memcpy(o.members, u.h_members, (size_t)n * sizeof(int32_t));
  }
}

void finish(const ht_server_cfg& c, Slot& s, ht_server_result* res) {
  const double t = now_s();
  float ms = 0.0f;
  const double dms = hipEventElapsedTime(&ms, s.start, s.done) == hipSuccess ? (double)ms : -1.0;
  for (int b = 0; b < s.nb; ++b) finish_one(c, s, s.place[b], t, dms, &res[b]);
  for (int b = 0; b < s.nb; ++b) s.place[b].job = Job();
  s.busy = false;
  s.nb = 0;
}

// an event's work: hits times the columns of its kind's grid
int64_t job_work(const ht_server_cfg& c, const Job& j) {
  const ht_grid& g = c.kinds[j.kind].grid;
  return (int64_t)j.n_hits * g.n_qpt * g.n_d0;
}

// whether work w may start now (a slot being free aside)
bool fits(const ht_server* srv, int64_t w) {
  const int64_t b = srv->cfg.work_budget;
  return b <= 0 || srv->in_flight == 0 || srv->in_flight + w <= b;
}

// whether a batch may grow to work w (within the budget even when nothing
// else runs: only a single event may exceed it)
bool joins(const ht_server* srv, int64_t w) {
  const int64_t b = srv->cfg.work_budget;
  return b <= 0 || srv->in_flight + w <= b;
}

Slot* free_slot_of(ht_server* srv) {
  for (Slot& s : srv->slots)
    if (!s.busy) return &s;
  return nullptr;
}

// place job j as event b of slot s (its hits already staged there)
void seat(ht_server* srv, Slot& s, int b, Job&& j) {
  s.work += job_work(srv->cfg, j);
  s.place[b].job = std::move(j);
  s.place[b].job.r.clear();
  s.place[b].job.phi.clear();
  s.place[b].job.layer.clear();
  s.nb = b + 1;
}

void launch(ht_server* srv, Slot& s) {
  srv->in_flight += s.work;
  start(srv, s);
}

// the oldest waiting event and up to batch_max - 1 later small ones of its
// kind onto free slot s, while the work budget allows
void start_waiting(ht_server* srv, Slot& s) {
  Job first = std::move(srv->queue.front());
  srv->queue.pop_front();
  s.kind = first.kind;
  s.work = 0;
  const bool small = srv->batch_max > 1 && first.n_hits <= srv->batch_hits;
  const int kind = first.kind;
  stage_inputs(s.place[0], first.r.data(), first.phi.data(), first.layer.data(), first.n_hits);
  seat(srv, s, 0, std::move(first));
  if (small) {
    for (auto it = srv->queue.begin(); it != srv->queue.end() && s.nb < srv->batch_max;) {
      if (it->kind != kind || it->n_hits > srv->batch_hits ||
          !joins(srv, s.work + job_work(srv->cfg, *it))) {
        ++it;
        continue;
      }
      stage_inputs(s.place[s.nb], it->r.data(), it->phi.data(), it->layer.data(), it->n_hits);
      seat(srv, s, s.nb, std::move(*it));
      it = srv->queue.erase(it);
    }
  }
  launch(srv, s);
}

bool cfg_ok(const ht_server_cfg& c) {
  if (c.n_kinds < 1 || c.n_kinds > kKinds) return false;
  if (c.max_hits < 1 || c.max_hits > 65535 || c.track_cap < 0 || c.object_cap < 0 ||
      c.member_cap < 0 || c.max_slots < 1 || c.queue_cap < 0 || c.hbm_budget <= 0 ||
      c.work_budget < 0 || c.batch_max < 0 || c.batch_max > kBatch || c.reserved != 0)
    return false;
  if (c.batch_max > 1 && (c.batch_max_hits < 1 || c.batch_max_hits > c.max_hits)) return false;
  for (int k = 0; k < c.n_kinds; ++k) {
    const ht_server_kind& K = c.kinds[k];
    if (K.peak_cap < 1 || K.reserved != 0) return false;
    if (K.cnn_params && !(K.cnn_threshold == K.cnn_threshold)) return false;  // NaN
  }
  return true;
}

void free_server(ht_server* srv) {
  for (Slot& s : srv->slots) {
    if (s.stream) (void)hipStreamSynchronize(s.stream);
    free_slot(s);
  }
  for (int k = 0; k < kKinds; ++k)
    if (srv->d_params[k]) (void)hipFree(srv->d_params[k]);
  delete srv;
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
  srv->batch_max = cfg->batch_max > 1 ? cfg->batch_max : 1;
  srv->batch_hits = srv->batch_max > 1 ? cfg->batch_max_hits : cfg->max_hits;
  int rc = HT_OK;
  int64_t used = 0;
  // the filters' parameters: one device copy per kind, shared by the slots
  for (int k = 0; k < cfg->n_kinds && rc == HT_OK; ++k) {
    if (!cfg->kinds[k].cnn_params) continue;
    rc = dev_alloc(&srv->d_params[k], HT_CNN_PARAMS, &used);
    if (rc == HT_OK &&
        hipMemcpy(srv->d_params[k], cfg->kinds[k].cnn_params, HT_CNN_PARAMS * sizeof(float),
                  hipMemcpyHostToDevice) != hipSuccess)
      rc = HT_EDEVICE;
  }
  srv->slots.reserve((size_t)cfg->max_slots);
  while (rc == HT_OK && (int)srv->slots.size() < cfg->max_slots) {
    Slot s;
    int64_t bytes = 0;
    rc = make_slot(srv, s, &bytes);
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
    free_server(srv);
    return rc;
  }
  *out = srv;
  return HT_OK;
}

int ht_server_destroy(ht_server* srv) {
  if (!srv) return HT_EINVAL;
  free_server(srv);
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
      s->kind = kind;
      s->work = 0;
      stage_inputs(s->place[0], r, phi, layer, n_hits);
      seat(srv, *s, 0, std::move(j));
      launch(srv, *s);
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
  if (max > 0 && max < srv->batch_max) return HT_EINVAL;
  *n_results = 0;
  for (;;) {
    bool pending = false;
    for (Slot& s : srv->slots) {
      if (!s.busy) continue;
      pending = true;
      if (*n_results + s.nb > max) continue;
      const hipError_t q = hipEventQuery(s.done);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) s.status = HT_EDEVICE;
      const int nb = s.nb;
      srv->in_flight -= s.work;
      s.work = 0;
      finish(srv->cfg, s, &results[*n_results]);
      *n_results += nb;
    }
    // start waiting events, oldest first, while a slot and the budget allow
    while (!srv->queue.empty() && fits(srv, job_work(srv->cfg, srv->queue.front()))) {
      Slot* s = free_slot_of(srv);
      if (!s) break;
      start_waiting(srv, *s);
      pending = true;
    }
    if (!wait || *n_results > 0 || !pending || *n_results >= max) break;
  }
  return HT_OK;
}

}  // extern "C"
