// C-ABI entry points, argument validation and plan construction.
#include <math.h>
#include <string.h>

#include <new>
#include <vector>

#include "ht_internal.h"

namespace {

using ht::Plan;

bool grid_ok(const ht_grid* g) {
  if (!g) return false;
  if (g->n_phi < 4 || g->n_qpt < 1 || g->n_d0 < 1) return false;
  if ((int64_t)g->n_phi * g->n_qpt * g->n_d0 > 0x7fffffffLL) return false;
  if (!(g->bfield > 0.0f)) return false;
  if (!(g->qpt_hi >= g->qpt_lo) || !(g->d0_hi >= g->d0_lo)) return false;
  if (!isfinite(g->qpt_lo) || !isfinite(g->qpt_hi) || !isfinite(g->d0_lo) ||
      !isfinite(g->d0_hi) || !isfinite(g->bfield))
    return false;
  return true;
}

// Bin-centre constants, float64 then one rounding to float32:
//   kappa_j = -c_B q/pT_j, d0_k, KAP = kappa_j, Q = kappa_j d0_k^2 + 2 d0_k,
//   T = 0.5 / (1 + kappa_j d0_k).
double qpt_centre(const ht_grid& g, int j) {
  return (double)g.qpt_lo +
         ((double)j + 0.5) * ((double)g.qpt_hi - (double)g.qpt_lo) / (double)g.n_qpt;
}
double kappa_centre(const ht_grid& g, int j) {
  const double cb = ht::kCLight * (double)g.bfield;
  return -cb * qpt_centre(g, j);
}
double d0_centre(const ht_grid& g, int k) {
  return (double)g.d0_lo +
         ((double)k + 0.5) * ((double)g.d0_hi - (double)g.d0_lo) / (double)g.n_d0;
}
// cell edges (band vote): edge j of q/pT and edge k of d0, j, k = 0 .. n
double qpt_edge(const ht_grid& g, int j) {
  return (double)g.qpt_lo + (double)j * ((double)g.qpt_hi - (double)g.qpt_lo) / (double)g.n_qpt;
}
double d0_edge(const ht_grid& g, int k) {
  return (double)g.d0_lo + (double)k * ((double)g.d0_hi - (double)g.d0_lo) / (double)g.n_d0;
}

// device allocation of n elements for the plan; the plan's byte count adds
// each allocation rounded up to 4 KiB (an upper bound of what it takes)
template <typename T>
int dalloc(Plan* plan, T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  if (hipMalloc((void**)p, n * sizeof(T)) != hipSuccess) {
    *p = nullptr;
    return HT_ENOMEM;
  }
  plan->dev_bytes += (int64_t)((n * sizeof(T) + 4095) / 4096 * 4096);
  return HT_OK;
}

void free_plan(Plan* p) {
  void* ptrs[] = {p->d_kap,       p->d_kapc,      p->d_d0c,       p->d_q,         p->d_t,        p->d_bits,      p->d_tile_cnt,
                  p->d_tile_off,  p->d_pbits,     p->d_col_first, p->d_hx,       p->d_hy,
                  p->d_hq,        p->d_hitB,      p->d_mcount,    p->d_mem,      p->d_cstat,
                  p->d_cgeo,      p->d_chit,      p->d_cnl,      p->d_owner_key, p->d_ctile_cnt,
                  p->d_ctile_off, p->d_trk_peak,  p->d_arc0,     p->d_arcn,     p->d_arci0,    p->d_arcin,      p->d_tunit,      p->d_vacc,
                  p->d_obj_cnt,   p->d_vtile,     p->d_scalars,  p->d_ckl,       p->d_ckh,
                  p->d_cql,       p->d_ctl,       p->d_cqh,      p->d_cth,      p->d_spread,
                  p->d_cls,       p->d_bkt,       p->d_bkt_off,  p->d_hkey,     p->d_shit,
                  p->d_sphi};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
}

}  // namespace

namespace ht {
int check_cluster(const Plan& p, const ht_cluster_cfg& c, int32_t n_hits, int32_t peak_cap,
                  int32_t track_cap) {
  if (c.win_bins < 0 || c.min_layers < 3 || c.min_layers > HT_MAX_LAYERS || c.seed_k < 1 ||
      c.member_cap < 1 || !(c.road_sigmas > 0.0f) || !(c.box_margin >= 0.0f) ||
      c.fit_iters < 0 || c.n_rho < 1 || c.n_theta < 4 || !(c.rho_hi > c.rho_lo) ||
      !(c.rho_lo > 0.0f) || !(c.sigma_rphi > 0.0f) || !isfinite(c.rho_hi) ||
      !isfinite(c.bh_max_isotropy) || !isfinite(c.road_sigmas) || !isfinite(c.box_margin) ||
      !(c.vtx_min_d0 >= 0.0f) || !isfinite(c.vtx_min_d0) || c.fit_kind < 0 || c.fit_kind > 1 ||
      c.vtx_two_branch < 0 || c.vtx_two_branch > 1)
    return HT_EINVAL;
  if (c.seed_k > 4 || n_hits > p.lim.max_hits || peak_cap > p.lim.max_peaks ||
      c.member_cap > p.lim.max_member_cap || track_cap > p.lim.max_tracks ||
      (int64_t)c.n_rho * c.n_theta > p.lim.max_vertex_cells || c.n_rho > p.lim.max_n_rho)
    return HT_EUNSUPPORTED;
  return HT_OK;
}
}  // namespace ht

extern "C" {

const char* ht_strerror(int status) {
  switch (status) {
    case HT_OK: return "ok";
    case HT_EINVAL: return "invalid argument";
    case HT_ENOMEM: return "device allocation failed";
    case HT_EDEVICE: return "HIP runtime error";
    case HT_EUNSUPPORTED: return "unsupported size (beyond the library's limits)";
    case HT_EBUSY: return "every slot busy and the queue full";
    default: return "unknown status";
  }
}

int ht_plan_create(const ht_grid* grid, const ht_limits* lim, ht_plan** out) {
  if (!out) return HT_EINVAL;
  *out = nullptr;
  if (!grid_ok(grid) || !lim) return HT_EINVAL;
  if (lim->max_hits < 0 || lim->max_peaks < 0 || lim->max_member_cap < 0 || lim->max_tracks < 0 ||
      lim->max_vertex_cells < 0 || lim->max_n_rho < 0)
    return HT_EINVAL;
  if (lim->max_hits > 65535 || lim->max_peaks > (1 << 26) || grid->n_phi > 1024)
    return HT_EUNSUPPORTED;
  int dev = 0;
  HT_CHECK(hipGetDevice(&dev));
  ht_plan* p = new (std::nothrow) ht_plan();
  if (!p) return HT_ENOMEM;
  memset(static_cast<Plan*>(p), 0, sizeof(Plan));
  p->grid = *grid;
  p->lim = *lim;
  p->device = dev;
  const ht_grid& g = *grid;
  p->n_cells = (int64_t)g.n_phi * g.n_qpt * g.n_d0;
  p->n_tiles = (int32_t)((p->n_cells + 255) / 256);
  p->phi_lo = (float)(-ht::kPi);
  p->invw = (float)((double)g.n_phi / (2.0 * ht::kPi));

  const size_t ncol = (size_t)g.n_qpt * g.n_d0;
  float* hk = new (std::nothrow) float[g.n_qpt];
  float* hq = new (std::nothrow) float[ncol];
  float* ht_ = new (std::nothrow) float[ncol];
  double* hkc = new (std::nothrow) double[g.n_qpt];
  double* hdc = new (std::nothrow) double[g.n_d0];
  int rc = (hk && hq && ht_ && hkc && hdc) ? HT_OK : HT_ENOMEM;
  if (rc == HT_OK) {
    for (int j = 0; j < g.n_qpt; ++j) hkc[j] = kappa_centre(g, j);
    for (int k = 0; k < g.n_d0; ++k) hdc[k] = d0_centre(g, k);
    for (int j = 0; j < g.n_qpt; ++j) hk[j] = (float)kappa_centre(g, j);
    for (int k = 0; k < g.n_d0; ++k) {
      const double d0 = d0_centre(g, k);
      for (int j = 0; j < g.n_qpt; ++j) {
        const double kap = kappa_centre(g, j);
        hq[(size_t)k * g.n_qpt + j] = (float)(kap * d0 * d0 + 2.0 * d0);
        ht_[(size_t)k * g.n_qpt + j] = (float)(0.5 / (1.0 + kap * d0));
      }
    }
  }
  const size_t nh = (size_t)lim->max_hits;
  const size_t np = (size_t)lim->max_peaks;
  const size_t words = (size_t)p->n_tiles * 8 + 2;
  const int64_t ctiles = ((int64_t)np + 255) / 256;
  if (rc == HT_OK) rc = dalloc(p, &p->d_kap, (size_t)g.n_qpt);
  if (rc == HT_OK) rc = dalloc(p, &p->d_kapc, (size_t)g.n_qpt);
  if (rc == HT_OK) rc = dalloc(p, &p->d_d0c, (size_t)g.n_d0);
  if (rc == HT_OK) rc = dalloc(p, &p->d_q, ncol);
  if (rc == HT_OK) rc = dalloc(p, &p->d_t, ncol);
  // peak ballots: 256 bits per 256-cell tile, or per 1024-cell tile of four-cell lanes
  if (rc == HT_OK) rc = dalloc(p, &p->d_bits, (size_t)((p->n_tiles + 3) / 4) * 32 + 2);
  if (rc == HT_OK) rc = dalloc(p, &p->d_tile_cnt, (size_t)p->n_tiles);
  if (rc == HT_OK) rc = dalloc(p, &p->d_tile_off, (size_t)p->n_tiles);
  if (rc == HT_OK) rc = dalloc(p, &p->d_pbits, words);
  if (rc == HT_OK) rc = dalloc(p, &p->d_col_first, ncol);
  if (rc == HT_OK) rc = dalloc(p, &p->d_hx, nh);
  if (rc == HT_OK) rc = dalloc(p, &p->d_hy, nh);
  if (rc == HT_OK) rc = dalloc(p, &p->d_hq, nh);
  if (rc == HT_OK) rc = dalloc(p, &p->d_hitB, nh);
  if (rc == HT_OK) rc = dalloc(p, &p->d_mcount, np);
  if (rc == HT_OK) rc = dalloc(p, &p->d_mem, np * (size_t)lim->max_member_cap);
  if (rc == HT_OK) rc = dalloc(p, &p->d_cstat, np);
  if (rc == HT_OK) rc = dalloc(p, &p->d_cgeo, np * 5);
  if (rc == HT_OK) rc = dalloc(p, &p->d_chit, np * HT_MAX_LAYERS);
  if (rc == HT_OK) rc = dalloc(p, &p->d_cnl, np);
  if (rc == HT_OK) rc = dalloc(p, &p->d_owner_key, nh);
  if (rc == HT_OK) rc = dalloc(p, &p->d_ctile_cnt, (size_t)ctiles);
  if (rc == HT_OK) rc = dalloc(p, &p->d_ctile_off, (size_t)ctiles);
  if (rc == HT_OK) rc = dalloc(p, &p->d_trk_peak, (size_t)lim->max_tracks);
  if (rc == HT_OK) rc = dalloc(p, &p->d_arc0, (size_t)lim->max_tracks * lim->max_n_rho);
  if (rc == HT_OK) rc = dalloc(p, &p->d_arcn, (size_t)lim->max_tracks * lim->max_n_rho);
  if (rc == HT_OK) rc = dalloc(p, &p->d_arci0, (size_t)lim->max_tracks * lim->max_n_rho);
  if (rc == HT_OK) rc = dalloc(p, &p->d_arcin, (size_t)lim->max_tracks * lim->max_n_rho);
  if (rc == HT_OK) rc = dalloc(p, &p->d_tunit, (size_t)lim->max_tracks);
  if (rc == HT_OK) rc = dalloc(p, &p->d_vacc, (size_t)lim->max_vertex_cells);
  if (rc == HT_OK) rc = dalloc(p, &p->d_obj_cnt, (size_t)lim->max_vertex_cells);
  if (rc == HT_OK) rc = dalloc(p, &p->d_vtile, (size_t)lim->max_vertex_cells / 1024 + 1);
  if (rc == HT_OK) rc = dalloc(p, &p->d_scalars, 16);
  if (rc == HT_OK) rc = dalloc(p, &p->d_spread, ht::kSpreadWords);
  if (rc == HT_OK) rc = dalloc(p, &p->d_cls, (size_t)ht::kClsSlots);
  if (rc == HT_OK) rc = dalloc(p, &p->d_bkt, (size_t)ht::kBucketKeys);
  if (rc == HT_OK) rc = dalloc(p, &p->d_bkt_off, (size_t)ht::kBucketKeys + 1);
  if (rc == HT_OK) rc = dalloc(p, &p->d_hkey, nh);
  if (rc == HT_OK) rc = dalloc(p, &p->d_shit, nh);
  if (rc == HT_OK) rc = dalloc(p, &p->d_sphi, nh);
  // band-vote corner tables: (smallest kappa, lower d0 edge) and (largest
  // kappa, upper d0 edge) of every column
  if (rc == HT_OK) rc = dalloc(p, &p->d_ckl, (size_t)g.n_qpt);
  if (rc == HT_OK) rc = dalloc(p, &p->d_ckh, (size_t)g.n_qpt);
  if (rc == HT_OK) rc = dalloc(p, &p->d_cql, ncol);
  if (rc == HT_OK) rc = dalloc(p, &p->d_ctl, ncol);
  if (rc == HT_OK) rc = dalloc(p, &p->d_cqh, ncol);
  if (rc == HT_OK) rc = dalloc(p, &p->d_cth, ncol);
  if (rc == HT_OK) {
    std::vector<float> ckl(g.n_qpt), ckh(g.n_qpt), cql(ncol), ctl(ncol), cqh(ncol), cth(ncol);
    const double cb = ht::kCLight * (double)g.bfield;
    for (int j = 0; j < g.n_qpt; ++j) {
      ckl[j] = (float)(-cb * qpt_edge(g, j + 1));
      ckh[j] = (float)(-cb * qpt_edge(g, j));
    }
    for (int k = 0; k < g.n_d0; ++k) {
      const double dlo = d0_edge(g, k), dhi = d0_edge(g, k + 1);
      for (int j = 0; j < g.n_qpt; ++j) {
        const double klo = -cb * qpt_edge(g, j + 1), khi = -cb * qpt_edge(g, j);
        const size_t c = (size_t)k * g.n_qpt + j;
        cql[c] = (float)(klo * dlo * dlo + 2.0 * dlo);
        ctl[c] = (float)(0.5 / (1.0 + klo * dlo));
        cqh[c] = (float)(khi * dhi * dhi + 2.0 * dhi);
        cth[c] = (float)(0.5 / (1.0 + khi * dhi));
      }
    }
    if (hipMemcpy(p->d_ckl, ckl.data(), 4 * (size_t)g.n_qpt, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_ckh, ckh.data(), 4 * (size_t)g.n_qpt, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_cql, cql.data(), 4 * ncol, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_ctl, ctl.data(), 4 * ncol, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_cqh, cqh.data(), 4 * ncol, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_cth, cth.data(), 4 * ncol, hipMemcpyHostToDevice) != hipSuccess)
      rc = HT_EDEVICE;
  }
  if (rc == HT_OK &&
      (hipMemcpy(p->d_kap, hk, sizeof(float) * g.n_qpt, hipMemcpyHostToDevice) != hipSuccess ||
       hipMemcpy(p->d_q, hq, sizeof(float) * ncol, hipMemcpyHostToDevice) != hipSuccess ||
       hipMemcpy(p->d_t, ht_, sizeof(float) * ncol, hipMemcpyHostToDevice) != hipSuccess ||
       hipMemcpy(p->d_kapc, hkc, sizeof(double) * g.n_qpt, hipMemcpyHostToDevice) != hipSuccess ||
       hipMemcpy(p->d_d0c, hdc, sizeof(double) * g.n_d0, hipMemcpyHostToDevice) != hipSuccess))
    rc = HT_EDEVICE;
  if (rc == HT_OK) rc = ht::vote_init(g.n_phi);
  if (rc == HT_OK) rc = ht::cell_vote_init(g.n_phi);
  if (rc == HT_OK) rc = ht::peaks_init(g.n_phi);
  delete[] hk;
  delete[] hq;
  delete[] ht_;
  delete[] hkc;
  delete[] hdc;
  if (rc != HT_OK) {
    free_plan(p);
    delete p;
    return rc;
  }
  *out = p;
  return HT_OK;
}

void ht_plan_destroy(ht_plan* p) {
  if (!p) return;
  int cur = 0;
  if (hipGetDevice(&cur) == hipSuccess && cur != p->device) (void)hipSetDevice(p->device);
  (void)ht_profile_end(p);
  free_plan(p);
  if (cur != p->device) (void)hipSetDevice(cur);
  delete p;
}

int hough_vote(const ht_plan* p, const float* r, const float* phi, int32_t n_hits, int32_t* acc,
               unsigned long long* n_votes, void* stream) {
  if (!p || !acc || n_hits < 0 || (n_hits > 0 && (!r || !phi))) return HT_EINVAL;
  if (n_hits > 65535 || n_hits > p->lim.max_hits) return HT_EUNSUPPORTED;
  return ht::launch_vote(*p, r, phi, n_hits, acc, n_votes, (hipStream_t)stream);
}

int hough_vote_n(const ht_plan* p, const float* r, const float* phi, int32_t n_hits_max,
                 const int32_t* n_hits_dev, int32_t* acc, unsigned long long* n_votes,
                 void* stream) {
  if (!n_hits_dev) return HT_EINVAL;
  if (!p || !acc || n_hits_max < 0 || (n_hits_max > 0 && (!r || !phi))) return HT_EINVAL;
  if (n_hits_max > 65535 || n_hits_max > p->lim.max_hits) return HT_EUNSUPPORTED;
  return ht::launch_vote(*p, r, phi, n_hits_max, acc, n_votes, (hipStream_t)stream, n_hits_dev);
}

int hough_vote_cell(const ht_plan* p, const float* r, const float* phi, int32_t n_hits,
                    int32_t* acc, unsigned long long* n_votes, void* stream) {
  if (!p || !acc || n_hits < 0 || (n_hits > 0 && (!r || !phi))) return HT_EINVAL;
  if (n_hits > 65535 || n_hits > p->lim.max_hits) return HT_EUNSUPPORTED;
  return ht::launch_cell_vote(*p, r, phi, n_hits, acc, n_votes, (hipStream_t)stream);
}

int hough_peaks(const ht_plan* p, const int32_t* acc, int32_t min_votes, ht_peak* out,
                int32_t capacity, int32_t* n_found, void* stream) {
  if (!p || !acc || !n_found || capacity < 0 || (capacity > 0 && !out)) return HT_EINVAL;
  return ht::launch_peaks(*p, acc, min_votes, out, capacity, n_found, (hipStream_t)stream);
}

int hough_peaks_noalloc(const ht_grid* grid, const int32_t* acc, int32_t min_votes, ht_peak* out,
                        int32_t capacity, int32_t* n_found, void* stream) {
  if (!grid_ok(grid) || !acc || !n_found || capacity < 0 || (capacity > 0 && !out))
    return HT_EINVAL;
  if ((int64_t)grid->n_phi * grid->n_qpt * grid->n_d0 > ht::noalloc_max_cells())
    return HT_EUNSUPPORTED;
  return ht::launch_peaks_noalloc(*grid, acc, min_votes, out, capacity, n_found,
                                  (hipStream_t)stream);
}

int assoc_cluster(const ht_plan* p, const float* r, const float* phi, const uint8_t* layer,
                  int32_t n_hits, const ht_peak* peaks, const int32_t* n_peaks, int32_t peak_cap,
                  const int32_t* acc, const ht_cluster_cfg* cfg, const ht_cluster_out* out,
                  void* stream) {
  if (!p || !cfg || !out || !n_peaks || n_hits < 0 || peak_cap < 0) return HT_EINVAL;
  if (n_hits > 0 && (!r || !phi || !layer || !out->hit_owner)) return HT_EINVAL;
  if (peak_cap > 0 && !peaks) return HT_EINVAL;
  if (!out->counts || out->track_cap < 0 || out->object_cap < 0 || out->member_cap < 0)
    return HT_EINVAL;
  if ((out->track_cap > 0 && !out->tracks) || (out->object_cap > 0 && !out->objects) ||
      (out->member_cap > 0 && !out->members))
    return HT_EINVAL;
  const int rc = ht::check_cluster(*p, *cfg, n_hits, peak_cap, out->track_cap);
  if (rc != HT_OK) return rc;
  return ht::launch_assoc(*p, r, phi, layer, n_hits, peaks, n_peaks, peak_cap, acc, *cfg, *out,
                          (hipStream_t)stream);
}

int hough_batch(int32_t nb, const ht_batch_event* ev, int32_t n_hits_max, int32_t min_votes,
                int32_t peak_cap, const ht_cluster_cfg* cfg, void* stream) {
  if (!ev || !cfg || nb < 1 || n_hits_max < 0 || peak_cap < 0) return HT_EINVAL;
  if (nb > HT_MAX_BATCH) return HT_EUNSUPPORTED;
  if (n_hits_max > 65535) return HT_EUNSUPPORTED;
  const ht::Plan* plans[HT_MAX_BATCH];
  const float* r[HT_MAX_BATCH];
  const float* phi[HT_MAX_BATCH];
  const int32_t* ndev[HT_MAX_BATCH];
  int32_t* acc[HT_MAX_BATCH];
  const int32_t* cacc[HT_MAX_BATCH];
  ht_peak* out[HT_MAX_BATCH];
  int32_t* nf[HT_MAX_BATCH];
  ht::AssocEvent ae[HT_MAX_BATCH];
  for (int b = 0; b < nb; ++b) {
    const ht_batch_event& e = ev[b];
    if (!e.plan || !e.n_hits_dev || !e.acc || !e.n_peaks || (peak_cap > 0 && !e.peaks))
      return HT_EINVAL;
    if (n_hits_max > 0 && (!e.r || !e.phi || !e.layer || !e.out.hit_owner)) return HT_EINVAL;
    if (!e.out.counts || e.out.track_cap != ev[0].out.track_cap ||
        e.out.object_cap != ev[0].out.object_cap || e.out.member_cap != ev[0].out.member_cap ||
        e.out.track_cap < 0 || e.out.object_cap < 0 || e.out.member_cap < 0)
      return HT_EINVAL;
    if ((e.out.track_cap > 0 && !e.out.tracks) || (e.out.object_cap > 0 && !e.out.objects) ||
        (e.out.member_cap > 0 && !e.out.members))
      return HT_EINVAL;
    if (memcmp(&e.plan->grid, &ev[0].plan->grid, sizeof(ht_grid)) != 0) return HT_EINVAL;
    if (n_hits_max > e.plan->lim.max_hits) return HT_EUNSUPPORTED;
    const int rc = ht::check_cluster(*e.plan, *cfg, n_hits_max, peak_cap, e.out.track_cap);
    if (rc != HT_OK) return rc;
    plans[b] = e.plan;
    r[b] = e.r;
    phi[b] = e.phi;
    ndev[b] = e.n_hits_dev;
    acc[b] = e.acc;
    cacc[b] = e.acc;
    out[b] = e.peaks;
    nf[b] = e.n_peaks;
    ae[b] = ht::AssocEvent{e.plan, e.r, e.phi, e.layer, e.n_hits_dev, e.peaks, e.n_peaks,
                           e.acc, e.out};
  }
  hipStream_t s = (hipStream_t)stream;
  int rc = ht::launch_vote_batch(*plans[0], nb, r, phi, ndev, n_hits_max, acc, s);
  if (rc == HT_OK) rc = ht::launch_peaks_batch(nb, plans, cacc, min_votes, out, peak_cap, nf, s);
  if (rc == HT_OK) rc = ht::launch_assoc_batch(nb, ae, n_hits_max, peak_cap, *cfg, s);
  return rc;
}

int ht_compact_hits(const float* r, const float* phi, const uint8_t* layer, int32_t n_hits,
                    const int32_t* hit_owner, float* out_r, float* out_phi, uint8_t* out_layer,
                    int32_t* out_index, int32_t* n_out, void* stream) {
  if (n_hits < 0 || !n_out) return HT_EINVAL;
  if (n_hits > 0 && (!r || !phi || !layer || !hit_owner || !out_r || !out_phi || !out_layer ||
                     !out_index))
    return HT_EINVAL;
  if (n_hits > 65535) return HT_EUNSUPPORTED;
  return ht::launch_compact(r, phi, layer, hit_owner, n_hits, out_r, out_phi, out_layer,
                            out_index, n_out, (hipStream_t)stream);
}

int ht_remap_track_hits(ht_track* tracks, int32_t track_cap, const int32_t* counts,
                        const int32_t* index, int32_t n_index, void* stream) {
  if (track_cap < 0 || n_index < 0 || !counts || (track_cap > 0 && !tracks) ||
      (n_index > 0 && !index))
    return HT_EINVAL;
  if (track_cap == 0) return HT_OK;
  return ht::launch_remap(tracks, track_cap, counts, index, n_index, (hipStream_t)stream);
}

int assoc_cluster_n(const ht_plan* p, const float* r, const float* phi, const uint8_t* layer,
                    int32_t n_hits_max, const int32_t* n_hits_dev, const ht_peak* peaks,
                    const int32_t* n_peaks, int32_t peak_cap, const int32_t* acc,
                    const ht_cluster_cfg* cfg, const ht_cluster_out* out, void* stream) {
  if (!n_hits_dev) return HT_EINVAL;
  if (!p || !cfg || !out || !n_peaks || n_hits_max < 0 || peak_cap < 0) return HT_EINVAL;
  if (n_hits_max > 0 && (!r || !phi || !layer || !out->hit_owner)) return HT_EINVAL;
  if (peak_cap > 0 && !peaks) return HT_EINVAL;
  if (!out->counts || out->track_cap < 0 || out->object_cap < 0 || out->member_cap < 0)
    return HT_EINVAL;
  if ((out->track_cap > 0 && !out->tracks) || (out->object_cap > 0 && !out->objects) ||
      (out->member_cap > 0 && !out->members))
    return HT_EINVAL;
  const int rc = ht::check_cluster(*p, *cfg, n_hits_max, peak_cap, out->track_cap);
  if (rc != HT_OK) return rc;
  return ht::launch_assoc(*p, r, phi, layer, n_hits_max, peaks, n_peaks, peak_cap, acc, *cfg,
                          *out, (hipStream_t)stream, n_hits_dev);
}

int ht_asin_f32(const float* u, float* out, int64_t n, void* stream) {
  if (n < 0 || (n > 0 && (!u || !out))) return HT_EINVAL;
  if (n > ((int64_t)1 << 38)) return HT_EUNSUPPORTED;  // grid limit
  return ht::launch_asin(u, out, n, (hipStream_t)stream);
}

int ht_sqrt_f64(const double* x, double* out, int64_t n, void* stream) {
  if (n < 0 || (n > 0 && (!x || !out))) return HT_EINVAL;
  if (n > ((int64_t)1 << 38)) return HT_EUNSUPPORTED;  // grid limit
  return ht::launch_sqrt(x, out, n, (hipStream_t)stream);
}

size_t ht_cnn_workspace_bytes(int32_t max_windows, int32_t training) {
  return ht::cnn_workspace_bytes(max_windows, training);
}

int ht_cnn_windows(const ht_plan* p, const int32_t* acc, const ht_peak* peaks,
                   const int32_t* n_peaks, int32_t cap, uint16_t* win, void* stream) {
  if (!p || !acc || !n_peaks || cap < 0 || (cap > 0 && (!peaks || !win))) return HT_EINVAL;
  if (cap > p->lim.max_peaks) return HT_EUNSUPPORTED;
  if (cap == 0) return HT_OK;
  return ht::launch_cnn_windows(*p, acc, peaks, n_peaks, cap, win, (hipStream_t)stream);
}

int ht_cnn_forward(const float* params, const uint16_t* win, const int32_t* n_dev, int32_t n_max,
                   float* logits, void* ws, size_t ws_bytes, void* stream) {
  if (!params || n_max < 0 || (n_max > 0 && (!win || !logits)) || !ws) return HT_EINVAL;
  if (ws_bytes < ht::cnn_workspace_bytes(n_max, 0)) return HT_EINVAL;
  if (n_max > (1 << 26)) return HT_EUNSUPPORTED;
  if (n_max == 0) return HT_OK;
  return ht::launch_cnn_forward(params, win, n_dev, n_max, logits, ws, (hipStream_t)stream);
}

int ht_cnn_score(const ht_plan* p, const float* params, const int32_t* acc, const ht_peak* peaks,
                 const int32_t* n_peaks, int32_t cap, float* logits, void* ws, size_t ws_bytes,
                 void* stream) {
  if (!p || !params || !acc || !n_peaks || cap < 0 || (cap > 0 && (!peaks || !logits)) || !ws)
    return HT_EINVAL;
  if (ws_bytes < ht::cnn_workspace_bytes(cap, 0)) return HT_EINVAL;
  if (cap > p->lim.max_peaks) return HT_EUNSUPPORTED;
  if (cap == 0) return HT_OK;
  return ht::launch_cnn_score(*p, params, acc, peaks, n_peaks, cap, logits, ws,
                              (hipStream_t)stream);
}

int ht_cnn_train_step(float* params, float* mom, const uint16_t* win, const float* labels,
                      int32_t n, float lr, float momentum, float pos_weight, float* loss,
                      void* ws, size_t ws_bytes, void* stream) {
  if (!params || !mom || !loss || !ws || n < 1 || !win || !labels) return HT_EINVAL;
  if (!(lr >= 0.0f) || !(momentum >= 0.0f) || !(pos_weight > 0.0f)) return HT_EINVAL;
  if (ws_bytes < ht::cnn_workspace_bytes(n, 1)) return HT_EINVAL;
  if (n > (1 << 24)) return HT_EUNSUPPORTED;
  return ht::launch_cnn_train(params, mom, win, labels, n, lr, momentum, pos_weight, loss, ws,
                              (hipStream_t)stream);
}

int ht_cnn_keep(const ht_plan* p, const float* logits, const ht_peak* peaks,
                const int32_t* n_peaks, int32_t cap, float threshold, ht_peak* out,
                int32_t out_cap, int32_t* n_out, void* stream) {
  if (!p || !n_peaks || !n_out || cap < 0 || out_cap < 0) return HT_EINVAL;
  if ((cap > 0 && (!logits || !peaks)) || (out_cap > 0 && !out)) return HT_EINVAL;
  if (cap > p->lim.max_peaks) return HT_EUNSUPPORTED;
  return ht::launch_cnn_keep(*p, logits, peaks, n_peaks, cap, threshold, out, out_cap, n_out,
                             (hipStream_t)stream);
}

int ht_profile_begin(ht_plan* p, int32_t depth) {
  if (!p || depth < 1 || depth > 65536) return HT_EINVAL;
  int rc = ht_profile_end(p);
  if (rc != HT_OK) return rc;
  const size_t n = (size_t)HT_STAGES * depth * 2;
  hipEvent_t* ev = new (std::nothrow) hipEvent_t[n];
  if (!ev) return HT_ENOMEM;
  for (size_t e = 0; e < n; ++e) {
    if (hipEventCreate(&ev[e]) != hipSuccess) {
      for (size_t f = 0; f < e; ++f) (void)hipEventDestroy(ev[f]);
      delete[] ev;
      return HT_ENOMEM;
    }
  }
  p->prof_ev = ev;
  for (int st = 0; st < HT_STAGES; ++st) p->prof_used[st] = 0;
  p->prof_depth = depth;
  return HT_OK;
}

int ht_profile_read(ht_plan* p, double* ms, int64_t* launches) {
  if (!p || !ms || !launches) return HT_EINVAL;
  if (p->prof_depth == 0) return HT_OK;
  int rc = HT_OK;
  for (int st = 0; st < HT_STAGES; ++st) {
    for (int u = 0; u < p->prof_used[st]; ++u) {
      hipEvent_t* pair = p->prof_ev + ((size_t)st * p->prof_depth + u) * 2;
      float t = 0.0f;
      if (hipEventSynchronize(pair[1]) != hipSuccess ||
          hipEventElapsedTime(&t, pair[0], pair[1]) != hipSuccess) {
        rc = HT_EDEVICE;
        continue;
      }
      ms[st] += (double)t;
      launches[st] += 1;
    }
    p->prof_used[st] = 0;
  }
  return rc;
}

int ht_profile_end(ht_plan* p) {
  if (!p) return HT_EINVAL;
  if (p->prof_ev) {
    if (hipDeviceSynchronize() != hipSuccess) return HT_EDEVICE;
    const size_t n = (size_t)HT_STAGES * p->prof_depth * 2;
    for (size_t e = 0; e < n; ++e) (void)hipEventDestroy(p->prof_ev[e]);
    delete[] p->prof_ev;
  }
  p->prof_ev = nullptr;
  p->prof_depth = 0;
  for (int st = 0; st < HT_STAGES; ++st) p->prof_used[st] = 0;
  return HT_OK;
}

}  // extern "C"
