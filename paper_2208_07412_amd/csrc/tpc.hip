// libtpcreco: host side of the C ABI declared in include/tpc.h.
//
// A context owns the parameter block, the status word and the scratch; each
// tpc_* call checks its host arguments and enqueues kernels on the context's
// stream.  No call synchronises except tpc_sync, and nothing inside a launch
// sequence allocates or uses hipMemset, so a sequence can be captured into a
// HIP graph.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>

#include "common.hpp"
#include "k_cluster.hpp"
#include "k_links.hpp"
#include "k_track.hpp"
#include "k_qc.hpp"
#include "k_zspage.hpp"
#include "k_compress.hpp"
#include "k_merge.hpp"

namespace {

// Clusterizer tile shapes compiled into the library (window in time bins,
// windows per workgroup); the smallest window sizes the window-count scratch.
constexpr uint32_t kMinWin = 8;

struct Geometry {
  int32_t np[NROW], xfx[NROW], pfx[NROW];
};

// Row r at x = 85 + 160 r / 151 cm with round(66 + 72 r / 151) pads of pitch
// 2 x tan(10 deg) / n; fixed-point values in 2^-16 cm.
Geometry make_geometry() {
  Geometry g;
  for (int r = 0; r < NROW; ++r) {
    g.np[r] = (int32_t)((2 * (66 * 151 + 72 * r) + 151) / (2 * 151));
    const int64_t num = (int64_t)(85 * 151 + 160 * r) * 65536;
    g.xfx[r] = (int32_t)((2 * num + 151) / (2 * 151));
    const double x = 85.0 + r * 160.0 / 151.0;
    g.pfx[r] = (int32_t)std::floor(2.0 * x * std::tan(M_PI / 18.0) / g.np[r] * 65536.0 + 0.5);
  }
  return g;
}

uint32_t ceil_div(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

}  // namespace

struct tpc_ctx {
  hipStream_t stream = nullptr;
  int device = 0;
  tpc_params par;
  tpc_sizes max;
  DevParams* d_par = nullptr;
  DevStatus* d_st = nullptr;
  // scratch
  uint32_t* zblk = nullptr;   // sample block index
  uint32_t* cblk = nullptr;   // cluster block index (hit grid)
  uint32_t* win = nullptr;    // clusterizer window counts / offsets
  uint32_t* cl_list = nullptr;  // chunks the streaming peak pass handed back
  ClusterRec* crec = nullptr;  // raw cluster records, indexed like the samples
  void* bsum = nullptr;       // scan block sums (u64)
  unsigned long long* tot64 = nullptr;
  uint32_t* tot32 = nullptr;
  uint16_t* chain_len = nullptr;  // per listed chain start
  uint32_t* cand = nullptr;       // chain starts, ascending
  uint8_t* start_flag = nullptr;  // 1 where a chain starts (per cluster)
  int32_t* f_hits = nullptr;
  float* f_state = nullptr;
  uint16_t* f_nhits = nullptr;
  uint16_t* f_range = nullptr;
  uint8_t* f_ok = nullptr;
  uint32_t* f_pts = nullptr;   // per tracklet: middle and end cluster, unit-row of the start
  uint8_t* f_key = nullptr;    // per tracklet: estimated rows of the next following pass
  uint32_t* f_perm = nullptr;  // tracklets in the order a following pass takes them
  uint32_t* f_bins = nullptr;  // counts, then first positions, per (work estimate, block)
  uint8_t* f_krow = nullptr;
  ulonglong4* f_work = nullptr;  // per-wave work counters of the following
  uint32_t* f_qnext = nullptr;   // per-group queue counters of the following's refill mode
  int n_cu = 0;                  // compute units of the device
  int2* pos = nullptr;           // packed cluster positions
  uint32_t* owner = nullptr;
  uint16_t* nkept = nullptr;
  float *r_par = nullptr, *r_cov = nullptr, *r_chi2 = nullptr;
  uint8_t *r_row = nullptr, *r_flags = nullptr;
  uint32_t* trk_index = nullptr;
  uint32_t* hit_off = nullptr;
  uint32_t* qc_part = nullptr;   // per-workgroup QC histograms
  uint32_t* zp_off = nullptr;    // output offset of each raw ZS page
  uint32_t *cm_a = nullptr, *cm_b = nullptr;  // compression: lengths / counts, offsets
  uint64_t* cm_res = nullptr;  // compression: the hits' residual codes
  unsigned long long* cm_tot = nullptr;       // compression: bit totals
  uint32_t* cm_info = nullptr;                // compression: sizes of the stream
  // merging: per-segment ends, cells, union-find, member sort
  uint32_t *mg_fs = nullptr, *mg_cell = nullptr, *mg_cnt = nullptr, *mg_off = nullptr,
           *mg_cur = nullptr, *mg_ends = nullptr, *mg_parent = nullptr, *mg_key = nullptr,
           *mg_idx = nullptr, *mg_skey = nullptr, *mg_sidx = nullptr;
  uint8_t* mg_sector = nullptr;
  double *mg_C = nullptr, *mg_tgl = nullptr, *mg_e = nullptr, *mg_cs18 = nullptr;
  double *mg_pk = nullptr, *mg_hxy = nullptr;  // ends' gate data in cell order; hit positions
  size_t bsum_cap = 0;
  tpc_tuning tune;
  // stage timing (measurement only)
  static constexpr int kProfCap = 64;
  bool prof_on = false;
  bool count_work = false;  // following work counters (measurement)
  bool prof_events = false;
  hipEvent_t prof_ev[TPC_PROF_STAGES][2][kProfCap];
  uint32_t prof_n[TPC_PROF_STAGES] = {};
};

namespace {

struct Layout {
  size_t off = 0;
  template <typename T>
  size_t add(size_t n) {
    off = (off + 255) & ~(size_t)255;
    const size_t o = off;
    off += n * sizeof(T);
    return o;
  }
};

struct Plan {
  size_t zblk, cblk, win, cl_list, crec, bsum, tot64, tot32, chain_len, cand, start_flag, f_hits, f_state, f_nhits, f_range, f_ok, f_pts, f_key, f_perm, f_bins, f_krow, f_work, f_qnext, pos,
      owner, nkept, r_par, r_cov, r_chi2, r_row, r_flags, trk_index, qc_part, zp_off, cm_a, cm_b, cm_res, cm_tot, cm_info, mg_fs,
      mg_cell, mg_cnt, mg_off, mg_cur, mg_ends, mg_parent, mg_key, mg_idx, mg_skey, mg_sidx,
      mg_sector, mg_C, mg_tgl, mg_e, mg_cs18, mg_pk, mg_hxy, hit_off, par, st, total;
  size_t bsum_cap;
  uint32_t nblk, nblk_s, nwin;
};

// Most raw ZS pages one call may decode: far more than any packing of
// max_samples needs (a full page holds over 1,500 samples).
uint64_t max_pages(const tpc_sizes& m) {
  return (uint64_t)m.max_samples / 16 + (uint64_t)NROW * m.max_units;
}

// Records of a compressed stream: one per track, one per (unit,row).
uint64_t cm_records(const tpc_sizes& m) {
  return (uint64_t)m.max_tracklets + (uint64_t)NROW * m.max_units + 2;
}

// Drift cells of the merging grid per (frame-side, sector) and the cells.
uint32_t mg_nzb(uint32_t n_time_bins) { return (uint32_t)((n_time_bins / 2.0 + 2.0) / MG_ZBIN) + 2; }
uint64_t mg_cells(const tpc_sizes& m) {
  return (uint64_t)((m.max_units + 35) / 36) * 2 * MG_NXY * MG_NXY * mg_nzb(m.max_time_bins) + 1;
}

Plan plan_for(const tpc_sizes& m) {
  Plan p;
  Layout L;
  const uint64_t nur = (uint64_t)m.max_units * NROW;
  p.nblk = ceil_div(m.max_time_bins, 1u << CG_BSHIFT);
  p.nblk_s = ceil_div(m.max_time_bins, 1u << CL_BSHIFT);
  p.nwin = ceil_div(m.max_time_bins, kMinWin);
  uint64_t nscan = nur * p.nwin;
  if (m.max_clusters > nscan) nscan = m.max_clusters;
  if (m.max_tracklets > nscan) nscan = m.max_tracklets;
  if (max_pages(m) > nscan) nscan = max_pages(m);
  if (cm_records(m) > nscan) nscan = cm_records(m);
  if (mg_cells(m) > nscan) nscan = mg_cells(m);
  if (256ull * (ceil_div(m.max_tracklets, SORT_BLOCK) + XCD_GROUPS - 1) > nscan)
    nscan = 256ull * (ceil_div(m.max_tracklets, SORT_BLOCK) + XCD_GROUPS - 1);
  p.bsum_cap = ceil_div(nscan, SCAN_TILE) + 1;
  const uint64_t mc = m.max_clusters > 0 ? m.max_clusters : 1;
  const uint64_t mt = m.max_tracklets > 0 ? m.max_tracklets : 1;
  p.zblk = L.add<uint32_t>(nur * (p.nblk_s + 1));
  p.cblk = L.add<uint32_t>(nur * (p.nblk + 1));
  p.win = L.add<uint32_t>(nur * p.nwin);
  p.cl_list = L.add<uint32_t>(1 + nur * (p.nwin / 4 + 1));  // chunks handed back
  p.crec = L.add<ClusterRec>(m.max_samples > 0 ? m.max_samples : 1);
  p.bsum = L.add<unsigned long long>(p.bsum_cap);
  p.tot64 = L.add<unsigned long long>(1);
  p.tot32 = L.add<uint32_t>(2);
  p.chain_len = L.add<uint16_t>(mc / 2 + 1);
  p.cand = L.add<uint32_t>(mc / 2 + 1);
  p.start_flag = L.add<uint8_t>(mc);
  p.f_hits = L.add<int32_t>(mt * NROW);
  p.f_state = L.add<float>(mt * 6);
  p.f_nhits = L.add<uint16_t>(mt);
  p.f_range = L.add<uint16_t>(mt);
  p.f_ok = L.add<uint8_t>(mt);
  p.f_pts = L.add<uint32_t>(mt * 3);
  p.f_key = L.add<uint8_t>(mt);
  p.f_perm = L.add<uint32_t>(mt);
  p.f_bins = L.add<uint32_t>(256 * (ceil_div(mt, SORT_BLOCK) + XCD_GROUPS - 1));
  p.f_krow = L.add<uint8_t>(mt * NROW);
  p.f_work = L.add<ulonglong4>(2 * (mt / 64 + 4 * XCD_GROUPS + 8));  // two passes
  p.f_qnext = L.add<uint32_t>(2 * XCD_GROUPS);  // queue counters of the refill mode
  p.pos = L.add<int2>(mc);
  p.owner = L.add<uint32_t>(mc);
  p.nkept = L.add<uint16_t>(mt);
  p.r_par = L.add<float>(mt * 5);
  p.r_cov = L.add<float>(mt * 15);
  p.r_chi2 = L.add<float>(mt);
  p.r_row = L.add<uint8_t>(mt);
  p.r_flags = L.add<uint8_t>(mt);
  p.trk_index = L.add<uint32_t>(mt);
  p.hit_off = L.add<uint32_t>(mt);
  p.qc_part = L.add<uint32_t>((uint64_t)QC_WG * QC_BINS);
  p.zp_off = L.add<uint32_t>(max_pages(m) + 1);
  p.cm_a = L.add<uint32_t>(cm_records(m));
  p.cm_b = L.add<uint32_t>(cm_records(m));
  p.cm_res = L.add<unsigned long long>(2 * mc);  // two residual codes per hit
  p.cm_tot = L.add<unsigned long long>(2);
  p.cm_info = L.add<uint32_t>(8);
  p.mg_fs = L.add<uint32_t>(mt);
  p.mg_cell = L.add<uint32_t>(2 * mt);
  p.mg_cnt = L.add<uint32_t>(mg_cells(m));
  p.mg_off = L.add<uint32_t>(mg_cells(m) + 1);
  p.mg_cur = L.add<uint32_t>(mg_cells(m) + 1);
  p.mg_ends = L.add<uint32_t>(2 * mt);
  p.mg_parent = L.add<uint32_t>(mt);
  p.mg_key = L.add<uint32_t>(mt);
  p.mg_idx = L.add<uint32_t>(mt);
  p.mg_skey = L.add<uint32_t>(mt);
  p.mg_sidx = L.add<uint32_t>(mt);
  p.mg_sector = L.add<uint8_t>(mt);
  p.mg_C = L.add<double>(mt);
  p.mg_tgl = L.add<double>(mt);
  p.mg_e = L.add<double>(10 * mt);
  p.mg_cs18 = L.add<double>(36);
  p.mg_pk = L.add<double>(6 * mt);
  p.mg_hxy = L.add<double>(2 * mc);
  p.par = L.add<DevParams>(1);
  p.st = L.add<DevStatus>(1);
  p.total = (L.off + 255) & ~(size_t)255;
  return p;
}

DevParams make_dev_params(const tpc_params& p) {
  DevParams d;
  std::memset(&d, 0, sizeof d);
  const Geometry g = make_geometry();
  for (int r = 0; r < NROW; ++r) {
    d.np[r] = g.np[r];
    d.xfx[r] = g.xfx[r];
    d.pfx[r] = g.pfx[r];
    d.xd[r] = g.xfx[r] / 65536.0;
    d.hwd[r] = (double)((int64_t)g.np[r] * g.pfx[r]) / 131072.0;
    d.vyd[r] = p.sigma_y[r] * p.sigma_y[r];
    d.vzd[r] = p.sigma_z[r] * p.sigma_z[r];
    d.x[r] = (float)d.xd[r];
    d.hw[r] = (float)d.hwd[r];
    d.vy[r] = (float)d.vyd[r];
    d.vz[r] = (float)d.vzd[r];
  }
  d.qmax_min = p.qmax_min;
  d.min_tracklet = p.min_tracklet;
  d.max_miss = p.max_miss;
  d.min_track_hits = p.min_track_hits;
  d.win_y = p.win_y;
  d.win_z = p.win_z;
  d.s_max = p.s_max;
  d.chi2_max_d = p.chi2_max;
  d.snp_max_d = p.snp_max;
  d.bz_b_d = p.bz_b;
  d.c0_snp2_d = p.c0_snp * p.c0_snp;
  d.c0_tgl2_d = p.c0_tgl * p.c0_tgl;
  d.c0_qpt2_d = p.c0_qpt * p.c0_qpt;
  d.qpt_clamp_d = p.qpt_clamp;
  d.edge_margin_d = p.edge_margin;
  d.chi2_max = (float)p.chi2_max;
  d.snp_max = (float)p.snp_max;
  d.bz_b = (float)p.bz_b;
  d.c0_snp2 = (float)d.c0_snp2_d;
  d.c0_tgl2 = (float)d.c0_tgl2_d;
  d.c0_qpt2 = (float)d.c0_qpt2_d;
  d.qpt_clamp = (float)p.qpt_clamp;
  d.edge_margin = (float)p.edge_margin;
  d.lowpt_qpt = (float)p.lowpt_qpt;
  const double c0r[5] = {p.c0r_y, p.c0r_z, p.c0r_snp, p.c0r_tgl, p.c0r_qpt};
  for (int i = 0; i < 5; ++i) {
    d.c0r2_d[i] = c0r[i] * c0r[i];
    d.c0r2[i] = (float)d.c0r2_d[i];
  }
  d.refit_snp_max_d = p.refit_snp_max;
  d.refit_snp_max = (float)p.refit_snp_max;
  d.validate = p.validate;
  d.force_fallback = p.force_fallback;
  return d;
}

#define HIP_OK(x)                        \
  do {                                   \
    if ((x) != hipSuccess) return TPC_ERR_HIP; \
  } while (0)

int launch_ok() { return hipGetLastError() == hipSuccess ? TPC_OK : TPC_ERR_HIP; }

uint32_t grid_for(uint64_t n, uint32_t block, uint32_t cap = 1u << 20) {
  uint64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (uint32_t)g;
}

// Grid caps of the grid-stride kernels of the track stages, whose grids are
// sized by buffer capacity (the counts are known only on the device): a
// workgroup with nothing to do still costs its dispatch, and in the refit its
// copy of the parameter block into LDS.  Measured on a 2 ms Pb-Pb slice
// (buffers for 2.2x its clusters and 6.6x its tracklets), uncapped against
// capped: hit grid + tracklets + track output 0.77 -> 0.70 ms at 16384
// workgroups; claim and keep (a wave per 4 tracklets) 0.88 -> 0.78 ms at
// 65536 (1.02 at 16384, 1.10 at 32768: they want a wave per group); refit
// (one-wave workgroups) 0.71 -> 0.60 ms at 4096.
constexpr uint32_t kCapStream = 16384;
constexpr uint32_t kCapClaim = 65536;
constexpr uint32_t kCapRefit = 4096;

// Records a pair of events around one stage when stage timing is on.
struct StageTimer {
  tpc_ctx* c;
  int id;
  bool on;
  StageTimer(tpc_ctx* ctx, int stage) : c(ctx), id(stage) {
    on = c->prof_on && c->prof_n[id] < tpc_ctx::kProfCap;
    if (on) (void)hipEventRecord(c->prof_ev[id][0][c->prof_n[id]], c->stream);
  }
  ~StageTimer() {
    if (on) {
      (void)hipEventRecord(c->prof_ev[id][1][c->prof_n[id]], c->stream);
      ++c->prof_n[id];
    }
  }
};

template <typename T, class Get, class Emit>
void run_scan(tpc_ctx* c, Get get, Emit emit, const uint32_t* n_dev, uint32_t n_cap, T* total,
              uint32_t* total32) {
  uint32_t nb = ceil_div(n_cap, SCAN_TILE);
  if (nb < 1) nb = 1;
  T* bs = reinterpret_cast<T*>(c->bsum);
  k_scan_reduce<T, Get><<<nb, SCAN_BLOCK, 0, c->stream>>>(get, n_dev, n_cap, bs, c->d_st);
  k_scan_blocks<T><<<1, 1024, 0, c->stream>>>(bs, nb, total, total32, c->d_st);
  k_scan_down<T, Get, Emit><<<nb, SCAN_BLOCK, 0, c->stream>>>(get, emit, n_dev, n_cap, bs, c->d_st);
}

// The total alone (the reduce half of run_scan).
template <typename T, typename Get>
void run_count(tpc_ctx* c, Get get, const uint32_t* n_dev, uint32_t n_cap, uint32_t* total32) {
  uint32_t nb = ceil_div(n_cap, SCAN_TILE);
  if (nb < 1) nb = 1;
  T* bs = reinterpret_cast<T*>(c->bsum);
  k_scan_reduce<T, Get><<<nb, SCAN_BLOCK, 0, c->stream>>>(get, n_dev, n_cap, bs, c->d_st);
  k_scan_blocks<T><<<1, 1024, 0, c->stream>>>(bs, nb, (T*)nullptr, total32, c->d_st);
}

struct GetU32 {
  const uint32_t* a;
  __device__ uint32_t operator()(uint32_t i) const { return a[i]; }
};
struct EmitU32 {
  uint32_t* out;
  __device__ void operator()(uint32_t i, uint32_t pre, uint32_t) const { out[i] = pre; }
};

ZsArgs zs_args(const tpc_zs_input* in) {
  return ZsArgs{in->pad, in->time, in->adc, in->row_start, in->n_samples, in->n_units,
                in->n_time_bins};
}

ClusterView cluster_view(tpc_ctx* c, const tpc_clusters* cl) {
  return ClusterView{cl->y_fx,        cl->z_fx,        c->pos,       cl->ptime,
                     cl->crow_start, cl->n_clusters, cl->capacity};
}

FollowOut follow_out(tpc_ctx* c) {
  return FollowOut{c->f_hits, c->f_state, c->f_nhits, c->f_range, c->f_ok, c->f_krow};
}

RefitOut refit_out(tpc_ctx* c) {
  return RefitOut{c->r_par, c->r_cov, c->r_chi2, c->r_row, c->r_flags};
}

// ------------------------------------------------------------- validation
int check_units(tpc_ctx* c, uint32_t n_units, uint32_t n_time_bins) {
  if (n_units == 0 || n_units > c->max.max_units) return TPC_ERR_ARG;
  if (n_time_bins == 0 || n_time_bins > c->max.max_time_bins) return TPC_ERR_ARG;
  return TPC_OK;
}

int check_input(tpc_ctx* c, const tpc_zs_input* in) {
  if (!in) return TPC_ERR_ARG;
  if (in->n_samples > c->max.max_samples) return TPC_ERR_ARG;
  if (check_units(c, in->n_units, in->n_time_bins)) return TPC_ERR_ARG;
  if (!in->row_start) return TPC_ERR_ARG;
  if (in->n_samples && (!in->pad || !in->time || !in->adc)) return TPC_ERR_ARG;
  return TPC_OK;
}

int check_clusters(tpc_ctx* c, const tpc_clusters* cl, bool full) {
  if (!cl) return TPC_ERR_ARG;
  if (check_units(c, cl->n_units, cl->n_time_bins)) return TPC_ERR_ARG;
  if (!cl->n_clusters || !cl->crow_start || !cl->y_fx || !cl->z_fx || !cl->ptime)
    return TPC_ERR_ARG;
  if (cl->capacity > c->max.max_clusters) return TPC_ERR_ARG;
  if (full && (!cl->dpad || !cl->dtime || !cl->s2pad || !cl->s2time || !cl->qtot || !cl->qmax ||
               !cl->ppad || !cl->flags))
    return TPC_ERR_ARG;
  const bool any_m = cl->sp || cl->st || cl->spp || cl->stt || cl->nsamp;
  const bool all_m = cl->sp && cl->st && cl->spp && cl->stt && cl->nsamp;
  if (any_m && !all_m) return TPC_ERR_ARG;
  return TPC_OK;
}

int check_links(tpc_ctx* c, const tpc_clusters* cl, const tpc_links* l, bool clean) {
  if (!l || !l->down || !l->up) return TPC_ERR_ARG;
  if (clean && (!l->downc || !l->upc)) return TPC_ERR_ARG;
  if (l->capacity < cl->capacity) return TPC_ERR_ARG;
  (void)c;
  return TPC_OK;
}

int check_tracklets(tpc_ctx* c, const tpc_tracklets* t) {
  if (!t || !t->n_tracklets || !t->start || !t->len) return TPC_ERR_ARG;
  if (t->capacity > c->max.max_tracklets) return TPC_ERR_ARG;
  return TPC_OK;
}

int check_tracks(const tpc_tracks* t) {
  if (!t || !t->n_tracks || !t->n_hits || !t->tracklet || !t->par || !t->cov || !t->chi2 ||
      !t->ndf || !t->row || !t->flags || !t->z_anchor || !t->hit_start || !t->hits ||
      !t->cluster_track)
    return TPC_ERR_ARG;
  return TPC_OK;
}

// ------------------------------------------------------------- stages
template <int W, int K>
void launch_cluster(tpc_ctx* c, const ZsArgs& za, uint32_t nblk_s, uint32_t n_ur,
                    const ClusterOut& co, uint32_t* n_clusters, uint32_t capacity,
                    uint32_t* crow_start) {
  // samples prefetched into registers: 64 per step (3 steps cover the larger
  // windows of the denser rows)
  constexpr int PRE = W == 8 ? 1 : 3;
  hipStream_t s = c->stream;
  const uint32_t nwin = ceil_div(za.n_time_bins, W);
  const uint32_t nchunk = ceil_div(nwin, K);
  const uint32_t ngrid = n_ur * nchunk;
  const uint32_t nwt = n_ur * nwin;
  {
    StageTimer tm(c, 1);
    if (c->tune.cl_mode == 2) {
      // windows shared by two waves (W >= 24, checked by tpc_set_tuning)
      if constexpr (W >= 24)
        k_cluster_peaks_mw<W, K, 2, 2><<<ngrid, 128, 0, s>>>(za, c->zblk, nblk_s, nwin, nchunk,
                                                             n_ur, c->win, c->crec,
                                                             co.sample_label, c->d_par, c->d_st);
    } else {
      if (c->tune.cl_mode == 1) {
        // streaming pass, then the windowed pass over the chunks it handed back
        k_fill<uint32_t><<<1, 64, 0, s>>>(c->cl_list, 0u, 1);
        k_cluster_stream<W, K><<<ngrid, 64, 0, s>>>(za, c->zblk, nblk_s, nwin, nchunk, n_ur,
                                                    c->win, c->crec, co.sample_label, c->cl_list,
                                                    c->d_par, c->d_st);
        k_cluster_peaks_list<W, K, PRE><<<ngrid < 2048 ? ngrid : 2048, 64, 0, s>>>(
            za, c->zblk, nblk_s, nwin, nchunk, n_ur, c->win, c->crec, co.sample_label,
            c->cl_list, c->d_par, c->d_st);
      } else {
        k_cluster_peaks<W, K, PRE><<<ngrid, 64, 0, s>>>(za, c->zblk, nblk_s, nwin, nchunk, n_ur,
                                                         c->win, c->crec, co.sample_label,
                                                         c->d_par, c->d_st);
      }
    }
  }
  {
    StageTimer tm(c, 2);
    run_scan<uint32_t>(c, GetU32{c->win}, EmitU32{c->win}, nullptr, nwt, (uint32_t*)nullptr,
                       n_clusters);
    k_crow_start<<<grid_for(n_ur + 1, 256), 256, 0, s>>>(c->win, nwin, n_ur, n_clusters, capacity,
                                                         crow_start, c->d_st);
  }
  {
    StageTimer tm(c, 3);
    k_cluster_output<W><<<grid_for(nwt, 256), 256, 0, s>>>(c->win, n_clusters, nwin, n_ur, c->zblk,
                                                        nblk_s, za.n_samples, c->crec, co,
                                                        c->d_par, c->d_st);
  }
}

int stage_cluster(tpc_ctx* c, const tpc_zs_input* in, tpc_clusters* out) {
  const uint32_t n_ur = in->n_units * NROW;
  const uint32_t nblk_s = ceil_div(in->n_time_bins, 1u << CL_BSHIFT);
  hipStream_t s = c->stream;
  {
    StageTimer tm(c, 0);
    k_block_index<false><<<n_ur * BI_PARTS, 256, 0, s>>>(in->time, in->pad, in->adc, in->row_start,
                                                         n_ur,
                                              nblk_s,
                                              CL_BSHIFT, in->n_time_bins, in->n_samples, c->zblk,
                                              c->d_par, c->d_st, 1);
  }
  ClusterOut co{out->capacity, out->y_fx, out->z_fx, out->dpad, out->dtime, out->s2pad, out->s2time,
                out->qtot, out->qmax, out->ppad, out->ptime, out->flags, out->sp, out->st,
                out->spp, out->stt, out->nsamp, out->sample_label};
  const ZsArgs za = zs_args(in);
  const int w = c->tune.cl_window, k = c->tune.cl_chunk;
  auto run = [&](auto W, auto K) {
    launch_cluster<decltype(W)::value, decltype(K)::value>(c, za, nblk_s, n_ur, co, out->n_clusters,
                                                           out->capacity, out->crow_start);
  };
  using I16 = std::integral_constant<int, 16>;
  using I32 = std::integral_constant<int, 32>;
  using I4 = std::integral_constant<int, 4>;
  using I8 = std::integral_constant<int, 8>;
  using I16k = std::integral_constant<int, 16>;
  using I8w = std::integral_constant<int, 8>;
  if (w == 8 && k == 4) run(I8w{}, I4{});
  else if (w == 8 && k == 8) run(I8w{}, I8{});
  else if (w == 8 && k == 16) run(I8w{}, I16k{});
  else if (w == 16 && k == 4) run(I16{}, I4{});
  else if (w == 16 && k == 8) run(I16{}, I8{});
  else if (w == 16 && k == 16) run(I16{}, I16k{});
  else if (w == 20 && k == 8) run(std::integral_constant<int, 20>{}, I8{});
  else if (w == 24 && k == 8) run(std::integral_constant<int, 24>{}, I8{});
  else if (w == 32 && k == 4) run(I32{}, I4{});
  else if (w == 32 && k == 8) run(I32{}, I8{});
  else run(I32{}, I16k{});
  if (out->sample_label)
    k_sample_label<<<n_ur, 256, 0, s>>>(za, out->crow_start, out->ppad, out->ptime, n_ur,
                                        out->sample_label, c->d_st);
  return launch_ok();
}

int stage_grid(tpc_ctx* c, const tpc_clusters* cl) {
  const uint32_t n_ur = cl->n_units * NROW;
  const uint32_t nblk = ceil_div(cl->n_time_bins, 1u << CG_BSHIFT);
  StageTimer tm(c, 4);
  k_block_index<true><<<n_ur, 256, 0, c->stream>>>(cl->ptime, cl->ppad, nullptr, cl->crow_start,
                                                   n_ur, nblk,
                                             CG_BSHIFT,
                                             cl->n_time_bins, cl->capacity, c->cblk, c->d_par,
                                             c->d_st, 0);
  k_pack_pos<<<grid_for(cl->capacity, 256, kCapStream), 256, 0, c->stream>>>(cl->y_fx, cl->z_fx, cl->n_clusters,
                                                                 cl->capacity, c->pos, c->d_st);
  return launch_ok();
}

int stage_neighbours(tpc_ctx* c, const tpc_clusters* cl, tpc_links* l) {
  const uint32_t n_ur = cl->n_units * NROW;
  const uint32_t nblk = ceil_div(cl->n_time_bins, 1u << CG_BSHIFT);
  StageTimer tm(c, 5);
  k_neighbours<<<n_ur * NB_PARTS, 256, 0, c->stream>>>(cluster_view(c, cl), c->cblk, nblk, n_ur, l->down, l->up,
                                            c->d_par, c->d_st);
  return launch_ok();
}

int stage_tracklets(tpc_ctx* c, const tpc_clusters* cl, tpc_links* l, tpc_tracklets* t) {
  hipStream_t s = c->stream;
  const uint32_t cap = cl->capacity;
  const uint32_t g = grid_for(cap, 256, kCapStream);
  StageTimer tm(c, 6);
  k_ca_clean<<<g, 256, 0, s>>>(l->down, l->up, l->downc, l->upc, c->start_flag, cl->n_clusters, cap,
                               c->d_st);
  // chain starts (at most one per two clusters: chains are disjoint and have
  // at least two), their chain lengths, then the tracklets in start order
  const uint32_t capc = cap / 2 + 1;
  run_scan<uint32_t>(c, GetStart{c->start_flag}, EmitStart{c->cand, capc}, cl->n_clusters, cap,
                     (uint32_t*)nullptr, c->tot32);
  k_chain_len<<<grid_for(capc, 256, kCapStream), 256, 0, s>>>(c->cand, c->tot32, capc, l->upc, cl->n_clusters,
                                                  cap, c->chain_len, c->d_par, c->d_st);
  run_scan<uint32_t>(c, GetKeepLen{c->chain_len},
                     EmitTracklet{c->cand, c->chain_len, t->start, t->len, t->capacity}, c->tot32,
                     capc, (uint32_t*)nullptr, c->tot32 + 1);
  k_tracklet_count<<<1, 1, 0, s>>>(c->tot32 + 1, t->capacity, t->n_tracklets, c->d_st);
  return launch_ok();
}

int stage_fit(tpc_ctx* c, const tpc_clusters* cl, const tpc_links* l, const tpc_tracklets* t,
              tpc_tracks* tr) {
  hipStream_t s = c->stream;
  const uint32_t n_ur = cl->n_units * NROW;
  const uint32_t nblk = ceil_div(cl->n_time_bins, 1u << CG_BSHIFT);
  const uint32_t tcap = t->capacity;
  const uint32_t ccap = cl->capacity;
  const ClusterView cv = cluster_view(c, cl);
  const FollowOut fo = follow_out(c);
  const RefitOut ro = refit_out(c);
  const uint32_t g64 = grid_for(tcap, 64, kCapRefit);
  const uint32_t gw = grid_for(tcap, 32, kCapClaim);
  // f_perm = the tracklets sorted by f_key, largest first (stable)
  const uint32_t nsb = ceil_div(tcap, SORT_BLOCK);
  // ngrp groups sorted each on its own (the following: one group per XCD)
  auto sort_by_key = [&](uint32_t ngrp) {
    const uint32_t nb = nsb + ngrp - 1;
    k_sort_work<false><<<nb, 256, 0, s>>>(c->f_key, t->n_tracklets, tcap, ngrp, c->f_bins,
                                          c->f_perm, c->d_st);
    run_scan<uint32_t>(c, GetU32{c->f_bins}, EmitU32{c->f_bins}, (const uint32_t*)nullptr,
                       256 * nb, (uint32_t*)nullptr, (uint32_t*)nullptr);
    k_sort_work<true><<<nb, 256, 0, s>>>(c->f_key, t->n_tracklets, tcap, ngrp, c->f_bins,
                                         c->f_perm, c->d_st);
  };
  // per-call counters of the fit stage
  k_fill<uint32_t><<<1, 64, 0, s>>>(&c->d_st->n_fallback, 0u, 5);
  {
    StageTimer tm(c, 6);  // the tracklets' seed points belong to tracklet building
    k_tracklet_points<<<grid_for(tcap, 256, kCapStream), 256, 0, s>>>(cv, n_ur, l->upc, t->start, t->len,
                                                           t->n_tracklets, tcap, c->f_pts,
                                                           c->f_key, c->d_st);
  }
  {
    StageTimer tm(c, 7);
    const int fb = c->tune.follow_block;
    const uint32_t ng = XCD_GROUPS;
    const uint32_t gf = ceil_div(grid_for(tcap, fb), ng) * ng;
    const uint32_t nwf = gf * (uint32_t)(fb / 64);  // waves per following launch
    const bool split = c->tune.follow_mode != 1;
    auto launch = [&](auto Bc, auto Cc) {
      constexpr int Bv = decltype(Bc)::value;
      constexpr bool Cv = decltype(Cc)::value;
      if (c->tune.follow_mode == 2) {
        // lane refill: a grid of the resident workgroups (a multiple of ng),
        // each pass over the tracklets sorted by the most rows it can take
        k_fill<uint32_t><<<1, 64, 0, s>>>(c->f_qnext, 0u, 2 * ng);
        // waves beyond the resident grid leave their work counters untouched
        if (Cv)
          k_fill<unsigned long long><<<grid_for(8 * nwf, 256), 256, 0, s>>>(
              reinterpret_cast<unsigned long long*>(c->f_work), 0ull, 8 * nwf);
        // resident workgroups per compute unit of each pass kernel, queried
        // once per process (a property of the kernel, not of the call), at
        // most FOLLOW_Q_WAVES_PER_CU waves
        auto occupancy = [](const void* fn) {
          int per_cu = 0;
          if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, Bv, 0) != hipSuccess ||
              per_cu < 1)
            per_cu = 1;
          return per_cu;
        };
        static const int occ_a = occupancy((const void*)k_follow_q<Bv, FP_A, Cv>);
        static const int occ_b = occupancy((const void*)k_follow_q<Bv, FP_B, Cv>);
        auto grid_q = [&](int per_cu) {
          const int cap = FOLLOW_Q_WAVES_PER_CU / (Bv / 64);
          if (per_cu > cap) per_cu = cap;
          const uint32_t gq = ceil_div((uint32_t)(per_cu * c->n_cu), ng) * ng;
          return gq < gf ? gq : gf;
        };
        const uint32_t refill = FOLLOW_REFILL;
        sort_by_key(ng);
        k_follow_q<Bv, FP_A, Cv><<<grid_q(occ_a), Bv, 0, s>>>(
            cv, c->cblk, nblk, l->upc, t->start, t->len, c->f_pts, c->f_perm, c->f_bins, ng,
            c->f_qnext, refill, c->f_key, t->n_tracklets, tcap, fo, c->f_work, c->d_par, c->d_st);
        sort_by_key(ng);
        k_follow_q<Bv, FP_B, Cv><<<grid_q(occ_b), Bv, 0, s>>>(
            cv, c->cblk, nblk, l->upc, t->start, t->len, c->f_pts, c->f_perm, c->f_bins, ng,
            c->f_qnext + ng, refill, c->f_key, t->n_tracklets, tcap, fo, c->f_work + nwf, c->d_par,
            c->d_st);
        return;
      }
      if (split) {
        // pass A, then pass B, each over the tracklets sorted by the most rows
        // the pass can take (the key k_tracklet_points, then pass A, leaves)
        for (int pass = 0; pass < 2; ++pass) {
          sort_by_key(ng);
          if (pass == 0)
            k_follow<Bv, FP_A, Cv><<<gf, Bv, 0, s>>>(cv, c->cblk, nblk, l->upc, t->start, t->len,
                                                     c->f_pts, c->f_perm, c->f_bins, ng, c->f_key,
                                                     t->n_tracklets, tcap, fo, c->f_work, c->d_par,
                                                     c->d_st);
          else
            k_follow<Bv, FP_B, Cv><<<gf, Bv, 0, s>>>(cv, c->cblk, nblk, l->upc, t->start, t->len,
                                                     c->f_pts, c->f_perm, c->f_bins, ng, c->f_key,
                                                     t->n_tracklets, tcap, fo, c->f_work + nwf,
                                                     c->d_par, c->d_st);
        }
      } else {
        k_follow<Bv, FP_AB, Cv><<<gf, Bv, 0, s>>>(cv, c->cblk, nblk, l->upc, t->start, t->len,
                                                  c->f_pts, nullptr, nullptr, 1u, c->f_key,
                                                  t->n_tracklets, tcap, fo, c->f_work, c->d_par,
                                                  c->d_st);
      }
    };
    using B64 = std::integral_constant<int, 64>;
    using B128 = std::integral_constant<int, 128>;
    using B256 = std::integral_constant<int, 256>;
    using Cnt = std::true_type;
    using NoCnt = std::false_type;
    const bool cnt = c->count_work;
    if (fb == 256) cnt ? launch(B256{}, Cnt{}) : launch(B256{}, NoCnt{});
    else if (fb == 128) cnt ? launch(B128{}, Cnt{}) : launch(B128{}, NoCnt{});
    else cnt ? launch(B64{}, Cnt{}) : launch(B64{}, NoCnt{});
    if (cnt) k_work_sum<<<1, 1024, 0, s>>>(c->f_work, (split ? 2 : 1) * nwf, c->d_st);
  }
  {
    StageTimer tm(c, 8);
    k_fill_dev<uint32_t><<<grid_for(ccap, 256, kCapStream), 256, 0, s>>>(c->owner, 0u,
                                                                        cl->n_clusters, ccap);
    // one wave per tracklet, about 8 tracklets per wave
    k_claim<false><<<gw, 256, 0, s>>>(fo, t->n_tracklets, tcap, c->owner, ccap, c->d_par, c->d_st);
    k_claim<true><<<gw, 256, 0, s>>>(fo, t->n_tracklets, tcap, c->owner, ccap, c->d_par, c->d_st);
    k_keep<<<gw, 256, 0, s>>>(fo, t->n_tracklets, tcap, c->owner, ccap, c->nkept, c->f_key,
                              c->d_par, c->d_st);
  }
  {
    StageTimer tm(c, 9);
    // tracks by kept hits: lanes of a wave refit equally long tracks (one
    // group: per-XCD groups made the refit slower, 1.04 -> 1.06 ms)
    const uint32_t ng = 1;
    sort_by_key(ng);
    // at most refit_waves one-wave workgroups per CU (160 KB of LDS shared):
    // the rest of each workgroup's share is reserved, not used
    const int rw = c->tune.refit_waves;
    const size_t lds_pad = rw ? (size_t)(160 << 10) / rw - sizeof(DevParams) - 256 : 0;
    k_refit<<<ceil_div(g64, ng) * ng, 64, lds_pad, s>>>(cv, t->start, fo, t->n_tracklets, tcap,
                                                        c->nkept, c->f_perm, c->f_bins, ng, ro,
                                                        c->d_par, c->d_st);
  }
  {
    StageTimer tm(c, 10);
    // the tracks the refit redid in FP64, counted for the status (a reduction,
    // not one same-address atomic per track)
    run_count<uint32_t>(c, GetToFp64{ro.flags}, t->n_tracklets, tcap, &c->d_st->n_fp64_redo);
  }
  StageTimer tm(c, 11);
  run_scan<unsigned long long>(c, GetTrackPair{c->nkept, ro}, EmitTrackPair{c->trk_index, c->hit_off, c->f_perm, tcap},
                               t->n_tracklets, tcap, c->tot64, (uint32_t*)nullptr);
  TrackOut to{tr->capacity, tr->hit_capacity, tr->tracklet, tr->par, tr->cov, tr->chi2, tr->ndf,
              tr->row, tr->flags, tr->z_anchor, tr->hit_start, tr->hits, tr->cluster_track};
  k_track_totals<<<1, 1, 0, s>>>(c->tot64, to, tr->n_tracks, tr->n_hits, c->d_st);
  // tracklets of the tracks listed in f_perm (free after the refit)
  k_track_emit<<<grid_for(tcap, 256, kCapStream), 256, 0, s>>>(cv, t->start, fo, c->f_perm, c->nkept, ro,
                                                    c->hit_off, to, c->d_st);
  k_cluster_track<<<grid_for(ccap, 256, kCapStream), 256, 0, s>>>(c->owner, c->trk_index, cl->n_clusters, ccap,
                                                      tcap, tr->cluster_track, c->d_st);
  if (tr->follow_hits)
    k_follow_export<<<grid_for((uint64_t)tcap * NROW, 256), 256, 0, s>>>(fo, t->n_tracklets, tcap,
                                                                          tr->follow_hits, c->d_st);
  return launch_ok();
}

}  // namespace

// =================================================================== ABI
extern "C" {

int tpc_params_default(tpc_params* p, double noise_sigma) {
  if (!p || !(noise_sigma > 0)) return TPC_ERR_ARG;
  std::memset(p, 0, sizeof *p);
  p->qmax_min = (int32_t)std::floor(5.0 * noise_sigma + 0.5);
  p->min_tracklet = 5;
  p->max_miss = 6;
  p->min_track_hits = 15;
  p->win_y = 163840;
  p->win_z = 163840;
  p->s_max = (int64_t)1 << 32;
  p->chi2_max = 16.0;
  p->snp_max = 0.95;
  p->bz_b = 0.299792458e-3 * 5.0;
  p->c0_snp = 0.1;
  p->c0_tgl = 0.1;
  p->c0_qpt = 10.0;
  p->qpt_clamp = 20.0;
  p->edge_margin = 1.0;
  p->lowpt_qpt = 5.0;
  p->c0r_y = 5.0;
  p->c0r_z = 5.0;
  p->c0r_snp = 0.5;
  p->c0r_tgl = 0.5;
  p->c0r_qpt = 10.0;
  p->refit_snp_max = 0.999;
  for (int r = 0; r < NROW; ++r) {
    p->sigma_y[r] = 0.06;
    p->sigma_z[r] = 0.05;
  }
  return TPC_OK;
}

int tpc_geometry(int32_t* npads, int32_t* x_fx, int32_t* pitch_fx) {
  const Geometry g = make_geometry();
  for (int r = 0; r < NROW; ++r) {
    if (npads) npads[r] = g.np[r];
    if (x_fx) x_fx[r] = g.xfx[r];
    if (pitch_fx) pitch_fx[r] = g.pfx[r];
  }
  return TPC_OK;
}

// Bounds a context supports: time bins within 16 bits, tracklet ids within
// 24 bits, and the cluster positions and the cluster grid within the 32-bit
// byte offsets of the following's buffer loads.
bool sizes_ok(const tpc_sizes& m) {
  if (m.max_units == 0 || m.max_time_bins == 0 || m.max_time_bins > 65000 ||
      m.max_tracklets > (1u << 24))
    return false;
  const uint64_t grid = (uint64_t)m.max_units * NROW * (ceil_div(m.max_time_bins, 1u << CG_BSHIFT) + 1);
  return (uint64_t)m.max_clusters * 8 < (1ull << 32) && grid * 4 < (1ull << 32);
}

int tpc_workspace_size(const tpc_sizes* max, size_t* bytes) {
  if (!max || !bytes) return TPC_ERR_ARG;
  if (!sizes_ok(*max)) return TPC_ERR_ARG;
  *bytes = plan_for(*max).total;
  return TPC_OK;
}

int tpc_create(tpc_ctx** out, const tpc_params* p, const tpc_sizes* max, void* hip_stream) {
  if (!out || !p || !max) return TPC_ERR_ARG;
  *out = nullptr;
  if (!sizes_ok(*max)) return TPC_ERR_ARG;
  if (p->min_tracklet < 3 || p->min_tracklet > NROW || p->min_track_hits < 3 || p->max_miss < 1 ||
      p->qmax_min < 1 || !(p->chi2_max > 0) || !(p->snp_max > 0 && p->snp_max < 1) ||
      p->win_y < 0 || p->win_z < 0 || p->s_max < 0)
    return TPC_ERR_ARG;
  for (int r = 0; r < NROW; ++r)
    if (!(p->sigma_y[r] > 0) || !(p->sigma_z[r] > 0)) return TPC_ERR_ARG;
  tpc_ctx* c = new (std::nothrow) tpc_ctx();
  if (!c) return TPC_ERR_STATE;
  c->stream = (hipStream_t)hip_stream;
  c->par = *p;
  c->max = *max;
  if (hipGetDevice(&c->device) != hipSuccess ||
      hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, c->device) !=
          hipSuccess) {
    delete c;
    return TPC_ERR_HIP;
  }
  const Plan pl = plan_for(*max);
  char* base = nullptr;
  if (hipMalloc(&base, pl.total) != hipSuccess) {
    delete c;
    return TPC_ERR_HIP;
  }
  c->zblk = (uint32_t*)(base + pl.zblk);
  c->cblk = (uint32_t*)(base + pl.cblk);
  c->win = (uint32_t*)(base + pl.win);
  c->cl_list = (uint32_t*)(base + pl.cl_list);
  c->crec = (ClusterRec*)(base + pl.crec);
  c->bsum = base + pl.bsum;
  c->tot64 = (unsigned long long*)(base + pl.tot64);
  c->tot32 = (uint32_t*)(base + pl.tot32);
  c->chain_len = (uint16_t*)(base + pl.chain_len);
  c->cand = (uint32_t*)(base + pl.cand);
  c->start_flag = (uint8_t*)(base + pl.start_flag);
  c->f_hits = (int32_t*)(base + pl.f_hits);
  c->f_state = (float*)(base + pl.f_state);
  c->f_nhits = (uint16_t*)(base + pl.f_nhits);
  c->f_range = (uint16_t*)(base + pl.f_range);
  c->f_ok = (uint8_t*)(base + pl.f_ok);
  c->f_pts = (uint32_t*)(base + pl.f_pts);
  c->f_key = (uint8_t*)(base + pl.f_key);
  c->f_perm = (uint32_t*)(base + pl.f_perm);
  c->f_bins = (uint32_t*)(base + pl.f_bins);
  c->f_krow = (uint8_t*)(base + pl.f_krow);
  c->f_work = (ulonglong4*)(base + pl.f_work);
  c->f_qnext = (uint32_t*)(base + pl.f_qnext);
  c->pos = (int2*)(base + pl.pos);
  c->owner = (uint32_t*)(base + pl.owner);
  c->nkept = (uint16_t*)(base + pl.nkept);
  c->r_par = (float*)(base + pl.r_par);
  c->r_cov = (float*)(base + pl.r_cov);
  c->r_chi2 = (float*)(base + pl.r_chi2);
  c->r_row = (uint8_t*)(base + pl.r_row);
  c->r_flags = (uint8_t*)(base + pl.r_flags);
  c->trk_index = (uint32_t*)(base + pl.trk_index);
  c->hit_off = (uint32_t*)(base + pl.hit_off);
  c->qc_part = (uint32_t*)(base + pl.qc_part);
  c->zp_off = (uint32_t*)(base + pl.zp_off);
  c->cm_a = (uint32_t*)(base + pl.cm_a);
  c->cm_b = (uint32_t*)(base + pl.cm_b);
  c->cm_res = (uint64_t*)(base + pl.cm_res);
  c->cm_tot = (unsigned long long*)(base + pl.cm_tot);
  c->cm_info = (uint32_t*)(base + pl.cm_info);
  c->mg_fs = (uint32_t*)(base + pl.mg_fs);
  c->mg_cell = (uint32_t*)(base + pl.mg_cell);
  c->mg_cnt = (uint32_t*)(base + pl.mg_cnt);
  c->mg_off = (uint32_t*)(base + pl.mg_off);
  c->mg_cur = (uint32_t*)(base + pl.mg_cur);
  c->mg_ends = (uint32_t*)(base + pl.mg_ends);
  c->mg_parent = (uint32_t*)(base + pl.mg_parent);
  c->mg_key = (uint32_t*)(base + pl.mg_key);
  c->mg_idx = (uint32_t*)(base + pl.mg_idx);
  c->mg_skey = (uint32_t*)(base + pl.mg_skey);
  c->mg_sidx = (uint32_t*)(base + pl.mg_sidx);
  c->mg_sector = (uint8_t*)(base + pl.mg_sector);
  c->mg_C = (double*)(base + pl.mg_C);
  c->mg_tgl = (double*)(base + pl.mg_tgl);
  c->mg_e = (double*)(base + pl.mg_e);
  c->mg_cs18 = (double*)(base + pl.mg_cs18);
  c->mg_pk = (double*)(base + pl.mg_pk);
  c->mg_hxy = (double*)(base + pl.mg_hxy);
  c->d_par = (DevParams*)(base + pl.par);
  c->d_st = (DevStatus*)(base + pl.st);
  c->bsum_cap = pl.bsum_cap;
  tpc_tuning_default(&c->tune);
  const DevParams dp = make_dev_params(*p);
  DevStatus ds;
  std::memset(&ds, 0, sizeof ds);
  // sector azimuths ((s + 0.5) 20 deg) for the merging's global frame
  double cs18[36];
  for (int k = 0; k < 18; ++k) {
    const double a = ((double)k + 0.5) * 20.0 * M_PI / 180.0;
    cs18[2 * k] = std::cos(a);
    cs18[2 * k + 1] = std::sin(a);
  }
  if (hipMemcpy(c->mg_cs18, cs18, sizeof cs18, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_par, &dp, sizeof dp, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_st, &ds, sizeof ds, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(base);
    delete c;
    return TPC_ERR_HIP;
  }
  *out = c;
  return TPC_OK;
}

int tpc_destroy(tpc_ctx* c) {
  if (!c) return TPC_ERR_ARG;
  (void)hipStreamSynchronize(c->stream);
  if (c->prof_events)
    for (int i = 0; i < TPC_PROF_STAGES; ++i)
      for (int j = 0; j < 2; ++j)
        for (int k = 0; k < tpc_ctx::kProfCap; ++k) (void)hipEventDestroy(c->prof_ev[i][j][k]);
  // zblk is the base of the single scratch allocation
  (void)hipFree(c->zblk);
  delete c;
  return TPC_OK;
}

int tpc_decode_zs_pages(tpc_ctx* c, const uint32_t* pages, uint32_t n_pages, tpc_zs_soa* out) {
  if (!c || !out || !out->n_samples || !out->row_start || (n_pages && !pages)) return TPC_ERR_ARG;
  if ((uintptr_t)pages & 15) return TPC_ERR_ARG;  // each page is loaded in 16-byte words
  if (check_units(c, out->n_units, out->n_time_bins)) return TPC_ERR_ARG;
  if (out->capacity && (!out->pad || !out->time || !out->adc)) return TPC_ERR_ARG;
  if (n_pages > max_pages(c->max)) return TPC_ERR_ARG;
  hipStream_t s = c->stream;
  const uint32_t n_ur = out->n_units * NROW;
  StageTimer tm(c, 12);
  if (n_pages == 0) {
    k_fill<uint32_t><<<grid_for(n_ur + 1, 256), 256, 0, s>>>(out->row_start, 0u, n_ur + 1);
    k_fill<uint32_t><<<1, 64, 0, s>>>(out->n_samples, 0u, 1);
    return launch_ok();
  }
  run_scan<uint32_t>(c, GetPageSamples{pages, out->n_units}, EmitPageOffset{c->zp_off}, nullptr,
                     n_pages, (uint32_t*)nullptr, c->tot32);
  // pages per workgroup in turn (a 2 ms Pb-Pb slice's 86,836 pages: 1.18 ms
  // with 4096 workgroups, 1.11 with 16384, 1.13 with one per page)
  const uint32_t g = n_pages < 16384 ? n_pages : 16384;
  k_zs_decode<<<g, ZSP_BLOCK, 0, s>>>(pages, n_pages, out->n_units, out->n_time_bins, c->zp_off,
                                      out->capacity, out->pad, out->time, out->adc, c->d_par,
                                      c->d_st);
  k_zs_rows<<<grid_for((uint64_t)n_pages + 1, 256), 256, 0, s>>>(
      pages, n_pages, out->n_units, c->zp_off, c->tot32, out->capacity, out->row_start,
      out->n_samples, c->d_st);
  return launch_ok();
}

namespace {
int64_t cm_b30(const tpc_ctx* c) { return (int64_t)llrint(c->par.bz_b * 1073741824.0); }
}  // namespace

int tpc_compress(tpc_ctx* c, const tpc_clusters* cl, const tpc_tracks* tr, tpc_compressed* out) {
  if (!c || check_clusters(c, cl, true) || !tr || !out || !out->stream || !out->n_words ||
      out->capacity == 0)
    return TPC_ERR_ARG;
  if (!tr->par || !tr->row || !tr->z_anchor || !tr->hit_start || !tr->hits ||
      !tr->cluster_track || !tr->n_tracks || tr->capacity > c->max.max_tracklets)
    return TPC_ERR_ARG;
  hipStream_t s = c->stream;
  const uint32_t n_ur = cl->n_units * NROW;
  StageTimer tm(c, 13);
  const CmClusters cv{cl->crow_start, cl->y_fx, cl->z_fx, cl->qtot, cl->qmax, cl->flags,
                      cl->n_clusters, cl->capacity, n_ur};
  const CmTracks tv{tr->par, tr->row, tr->z_anchor, tr->hit_start, tr->hits, tr->cluster_track,
                    tr->n_tracks, tr->capacity, tr->hit_capacity};
  const int64_t b30 = cm_b30(c);
  if (out->res_hist) k_fill<uint32_t><<<1, 256, 0, s>>>(out->res_hist, 0u, 256);
  // the hits' residual codes, cached between the two track passes
  const uint32_t res_cap = (uint32_t)c->max.max_clusters;
  k_cm_track_bits<<<grid_for(tr->capacity, 4, kCapStream), 256, 0, s>>>(
      cv, tv, b30, c->d_par, c->cm_a, out->res_hist, c->cm_res, res_cap, c->d_st);
  k_cm_row_bits<<<grid_for(n_ur, 4, 4096), 256, 0, s>>>(cv, tr->cluster_track, c->cm_b, c->d_st);
  run_scan<unsigned long long>(c, CmGetU32{c->cm_a}, CmEmitTrack{out->stream, out->capacity},
                               tr->n_tracks, tr->capacity, c->cm_tot, (uint32_t*)nullptr);
  run_scan<unsigned long long>(
      c, CmGetU32{c->cm_b},
      CmEmitRow{out->stream, out->capacity, tr->n_tracks, tr->capacity, c->cm_tot}, nullptr, n_ur,
      c->cm_tot + 1, (uint32_t*)nullptr);
  k_cm_finish<<<1, 1, 0, s>>>(out->stream, out->capacity, cl->n_units, tr->n_tracks, tr->capacity,
                              tr->hit_start, cl->n_clusters, cl->capacity, c->cm_tot,
                              out->n_words, c->cm_info, c->d_st);
  k_cm_clear<<<grid_for(out->capacity, 256, 2048), 256, 0, s>>>(out->stream, c->cm_info, c->d_st);
  k_cm_track_write<<<grid_for(tr->capacity, 4, kCapStream), 256, 0, s>>>(
      cv, tv, b30, c->d_par, out->stream, c->cm_info, c->cm_res, res_cap, c->d_st);
  k_cm_row_write<<<grid_for(n_ur, 4, 4096), 256, 0, s>>>(cv, tr->cluster_track, out->stream,
                                                         tr->n_tracks, tr->capacity, c->cm_info,
                                                         c->d_st);
  return launch_ok();
}

int tpc_decompress(tpc_ctx* c, const uint32_t* stream, uint32_t stream_words,
                   tpc_decoded_clusters* out) {
  if (!c || !stream || !out || !out->n_clusters || !out->unit || !out->row || !out->y_fx ||
      !out->z_fx || !out->qtot || !out->qmax || !out->flags || !out->track)
    return TPC_ERR_ARG;
  hipStream_t s = c->stream;
  StageTimer tm(c, 14);
  const uint32_t max_rec = (uint32_t)cm_records(c->max);
  k_cm_dec_header<<<1, 1, 0, s>>>(stream, stream_words, c->max.max_units, c->max.max_tracklets,
                                  out->capacity, out->n_clusters, c->cm_info, c->d_st);
  k_cm_dec_counts<<<grid_for(max_rec, 256, 4096), 256, 0, s>>>(stream, c->cm_info, c->cm_a,
                                                               c->d_st);
  run_scan<unsigned long long>(c, CmGetU32{c->cm_a}, CmEmitOff{c->cm_b}, c->cm_info + 5, max_rec,
                               c->cm_tot, (uint32_t*)nullptr);
  const CmDecOut o{out->capacity, out->unit, out->row, out->y_fx, out->z_fx,
                   out->qtot, out->qmax, out->flags, out->track};
  k_cm_dec_tracks<<<grid_for(c->max.max_tracklets, 256, 4096), 256, 0, s>>>(
      stream, c->cm_info, c->cm_b, cm_b30(c), c->d_par, o, c->d_st);
  k_cm_dec_rows<<<grid_for((uint64_t)c->max.max_units * NROW, 4, 4096), 256, 0, s>>>(
      stream, c->cm_info, c->cm_b, c->cm_tot, o, c->d_st);
  return launch_ok();
}

struct MgEmitOff {
  uint32_t *off, *cur;
  __device__ void operator()(uint32_t i, uint32_t pre, uint32_t) const {
    off[i] = pre;
    cur[i] = pre;
  }
};

int tpc_merge_tracks(tpc_ctx* c, const tpc_clusters* cl, const tpc_tracks* tr, tpc_merged* out) {
  if (!c || check_clusters(c, cl, false) || !tr || !out || !out->n_merged || !out->label ||
      !out->near_tie || !out->fit)
    return TPC_ERR_ARG;
  if (!tr->par || !tr->row || !tr->hit_start || !tr->hits || !tr->n_tracks ||
      tr->capacity > c->max.max_tracklets || out->capacity < tr->capacity || tr->capacity == 0)
    return TPC_ERR_ARG;
  hipStream_t s = c->stream;
  StageTimer tm(c, 15);
  const uint32_t cap = tr->capacity, n_ur = cl->n_units * NROW;
  // hit positions are kept for at most max_clusters hits (a track set holds
  // each cluster at most once)
  const uint32_t hit_bound =
      tr->hit_capacity < c->max.max_clusters ? tr->hit_capacity : c->max.max_clusters;
  const uint32_t nzb = mg_nzb(cl->n_time_bins);
  const uint32_t n_cells = ((cl->n_units + 35) / 36) * 2 * MG_NXY * MG_NXY * nzb;
  const MgSegs S{c->mg_fs, c->mg_sector, c->mg_C, c->mg_tgl, c->mg_e};
  k_fill<uint32_t><<<grid_for(n_cells, 256, 4096), 256, 0, s>>>(c->mg_cnt, 0u, n_cells);
  k_fill<double><<<grid_for((uint64_t)out->capacity * TPC_MERGE_FIT, 256, 4096), 256, 0, s>>>(
      out->fit, 0.0, out->capacity * TPC_MERGE_FIT);
  k_mg_init<<<grid_for(cap, 256, 4096), 256, 0, s>>>(c->mg_parent, out->near_tie, c->mg_idx, cap,
                                                     c->d_st);
  k_mg_segments<<<grid_for(cap, 256, 4096), 256, 0, s>>>(
      cl->crow_start, n_ur, cl->y_fx, cl->z_fx, cl->n_clusters, cl->capacity, tr->par, tr->row,
      tr->hit_start, tr->hits, tr->hit_capacity, tr->n_tracks, cap, c->mg_cs18, c->par.bz_b, nzb,
      S, c->mg_cell, c->mg_cnt, c->d_par, c->d_st);
  run_scan<uint32_t>(c, GetU32{c->mg_cnt}, MgEmitOff{c->mg_off, c->mg_cur}, nullptr, n_cells,
                     (uint32_t*)nullptr, c->tot32);
  k_mg_total<<<1, 1, 0, s>>>(c->mg_off, c->tot32, n_cells, c->d_st);
  k_mg_fill_cells<<<grid_for(2 * (uint64_t)cap, 256, 4096), 256, 0, s>>>(
      c->mg_cell, tr->n_tracks, cap, c->mg_cur, c->mg_ends, c->d_st);
  k_mg_pack<<<grid_for(2 * (uint64_t)cap, 256, 4096), 256, 0, s>>>(c->mg_ends, c->tot32, c->mg_e,
                                                                   c->mg_pk, c->d_st);
  k_mg_pairs<<<grid_for(2 * (uint64_t)cap, 256, 8192), 256, 0, s>>>(
      S, nzb, c->tot32, c->mg_off, c->mg_ends, c->mg_cell, c->mg_pk, c->mg_parent, out->near_tie,
      c->d_st);
  k_mg_hits<<<grid_for(hit_bound, 256, 16384), 256, 0, s>>>(
      cl->crow_start, n_ur, cl->y_fx, cl->n_clusters, cl->capacity, tr->hit_start, tr->hits,
      hit_bound, tr->n_tracks, cap, c->mg_cs18, c->mg_hxy, c->d_par, c->d_st);
  k_mg_labels<<<grid_for(cap, 256, 4096), 256, 0, s>>>(c->mg_parent, tr->n_tracks, cap, out->label,
                                                       c->mg_key, c->d_st);
  // members grouped by component in ascending index: labels are below 2^24
  {
    const uint32_t nb = ceil_div(cap, MG_SORT_BLOCK);
    uint32_t *ki = c->mg_key, *vi = c->mg_idx, *ko = c->mg_skey, *vo = c->mg_sidx;
    for (int shift = 0; shift < 24; shift += 8) {
      k_mg_rsort<false><<<nb, 256, 0, s>>>(ki, vi, tr->n_tracks, cap, shift, c->f_bins, ko, vo,
                                           c->d_st);
      run_scan<uint32_t>(c, GetU32{c->f_bins}, EmitU32{c->f_bins}, nullptr, 256 * nb,
                         (uint32_t*)nullptr, c->tot32 + 1);
      k_mg_rsort<true><<<nb, 256, 0, s>>>(ki, vi, tr->n_tracks, cap, shift, c->f_bins, ko, vo,
                                          c->d_st);
      uint32_t* t = ki;
      ki = ko;
      ko = t;
      t = vi;
      vi = vo;
      vo = t;
    }
    // three passes: the result is in (mg_skey, mg_sidx)
  }
  k_mg_fit<<<grid_for(cap, 64, 16384), 64, 0, s>>>(c->mg_skey, c->mg_sidx, tr->n_tracks, cap,
                                                   cl->z_fx, tr->hit_start, tr->hits, hit_bound,
                                                   c->mg_hxy, out->fit, c->d_st);
  run_count<uint32_t>(c, MgIsRoot{out->label}, tr->n_tracks, cap, out->n_merged);
  return launch_ok();
}

int tpc_cluster(tpc_ctx* c, const tpc_zs_input* in, tpc_clusters* out) {
  if (!c || check_input(c, in) || check_clusters(c, out, true)) return TPC_ERR_ARG;
  if (out->n_units != in->n_units || out->n_time_bins != in->n_time_bins) return TPC_ERR_ARG;
  return stage_cluster(c, in, out);
}

int tpc_find_neighbours(tpc_ctx* c, const tpc_clusters* cl, tpc_links* l) {
  if (!c || check_clusters(c, cl, false) || check_links(c, cl, l, false)) return TPC_ERR_ARG;
  int rc = stage_grid(c, cl);
  if (rc) return rc;
  return stage_neighbours(c, cl, l);
}

int tpc_build_tracklets(tpc_ctx* c, const tpc_clusters* cl, tpc_links* l, tpc_tracklets* t) {
  if (!c || check_clusters(c, cl, false) || check_links(c, cl, l, true) || check_tracklets(c, t))
    return TPC_ERR_ARG;
  return stage_tracklets(c, cl, l, t);
}

int tpc_fit_tracks(tpc_ctx* c, const tpc_clusters* cl, const tpc_links* l, const tpc_tracklets* t,
                   tpc_tracks* tr) {
  if (!c || check_clusters(c, cl, false) || check_links(c, cl, l, true) || check_tracklets(c, t) ||
      check_tracks(tr))
    return TPC_ERR_ARG;
  int rc = stage_grid(c, cl);
  if (rc) return rc;
  return stage_fit(c, cl, l, t, tr);
}

static_assert(QC_BINS == TPC_QC_BINS && QC_QTOT == TPC_QC_QTOT && QC_QMAX == TPC_QC_QMAX &&
                  QC_NHITS == TPC_QC_NHITS && QC_ATTACH == TPC_QC_ATTACH,
              "QC histogram layout");

int tpc_qc_histograms(tpc_ctx* c, const tpc_clusters* cl, const tpc_tracks* tr, uint32_t* hist) {
  if (!c || !cl || !tr || !hist || !cl->n_clusters || !cl->qtot || !cl->qmax || !tr->n_tracks ||
      !tr->hit_start || !tr->cluster_track)
    return TPC_ERR_ARG;
  k_qc_fill<<<QC_WG, 256, 0, c->stream>>>(cl->qtot, cl->qmax, tr->cluster_track, cl->n_clusters,
                                          cl->capacity, tr->hit_start, tr->n_tracks,
                                          tr->capacity, c->qc_part, c->d_st);
  k_qc_sum<<<QC_BINS, 256, 0, c->stream>>>(c->qc_part, QC_WG, hist);
  return launch_ok();
}

// Allocation-free QC histograms.  The per-workgroup partial histograms live in
// a file-scope device array (one copy per GPU, held until the process ends)
// instead of a context's scratch.  One partial histogram per QC_NA_ITEMS
// entries of the larger capacity, at most QC_NA_WG of them.
namespace {
constexpr uint32_t QC_NA_WG = 1024;
constexpr uint32_t QC_NA_ITEMS = 65536;
constexpr int kMaxDevices = 64;
static_assert(TPC_QC_NOALLOC_MAX == (uint64_t)QC_NA_WG * QC_NA_ITEMS, "no-alloc QC limit");
}  // namespace

static __device__ __align__(256) uint32_t scratch[(size_t)QC_NA_WG * QC_BINS];

namespace {
std::mutex g_scratch_mu;
uint32_t* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's copy of `scratch`, resolved once per device
// with that device current.  The array's name in host code is a host-side
// stand-in, never a device address, so kernels only ever get this pointer.
int noalloc_scratch(uint32_t** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return TPC_ERR_HIP;
  if (dev < 0 || dev >= kMaxDevices) return TPC_ERR_STATE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return TPC_ERR_HIP;
    g_scratch_ptr[dev] = (uint32_t*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return TPC_OK;
}
}  // namespace

int tpc_qc_histograms_noalloc(const tpc_clusters* cl, const tpc_tracks* tr, uint32_t* hist,
                              void* hip_stream) {
  if (!cl || !tr || !hist || !cl->n_clusters || !cl->qtot || !cl->qmax || !tr->n_tracks ||
      !tr->hit_start || !tr->cluster_track)
    return TPC_ERR_ARG;
  const uint64_t items = cl->capacity > tr->capacity ? cl->capacity : tr->capacity;
  if (items > TPC_QC_NOALLOC_MAX) {
    std::fprintf(stderr,
                 "tpc_qc_histograms_noalloc: capacity %llu exceeds the limit of %llu entries "
                 "(fixed scratch of %u partial histograms)\n",
                 (unsigned long long)items, (unsigned long long)TPC_QC_NOALLOC_MAX, QC_NA_WG);
    return TPC_ERR_CAPACITY;
  }
  uint32_t* part = nullptr;
  const int rc = noalloc_scratch(&part);
  if (rc) return rc;
  uint32_t nwg = ceil_div(items, QC_NA_ITEMS);
  if (nwg == 0) nwg = 1;
  hipStream_t s = (hipStream_t)hip_stream;
  // every workgroup overwrites its whole partial histogram: nothing to clear
  k_qc_fill<<<nwg, 256, 0, s>>>(cl->qtot, cl->qmax, tr->cluster_track, cl->n_clusters,
                                cl->capacity, tr->hit_start, tr->n_tracks, tr->capacity, part,
                                nullptr);
  k_qc_sum<<<QC_BINS, 256, 0, s>>>(part, nwg, hist);
  return launch_ok();
}

int tpc_process_timeframe(tpc_ctx* c, const tpc_zs_input* in, tpc_clusters* cl, tpc_links* l,
                          tpc_tracklets* t, tpc_tracks* tr) {
  if (!c || check_input(c, in) || check_clusters(c, cl, true) || check_links(c, cl, l, true) ||
      check_tracklets(c, t) || check_tracks(tr))
    return TPC_ERR_ARG;
  if (cl->n_units != in->n_units || cl->n_time_bins != in->n_time_bins) return TPC_ERR_ARG;
  int rc = stage_cluster(c, in, cl);
  if (!rc) rc = stage_grid(c, cl);
  if (!rc) rc = stage_neighbours(c, cl, l);
  if (!rc) rc = stage_tracklets(c, cl, l, t);
  if (!rc) rc = stage_fit(c, cl, l, t, tr);
  return rc;
}

int tpc_sync(tpc_ctx* c, tpc_counts* counts) {
  if (!c) return TPC_ERR_ARG;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return TPC_ERR_HIP;
  DevStatus ds;
  if (hipMemcpy(&ds, c->d_st, sizeof ds, hipMemcpyDeviceToHost) != hipSuccess) return TPC_ERR_HIP;
  if (counts) {
    std::memset(counts, 0, sizeof *counts);
    counts->status = ds.status;
    counts->required = ds.required;
    counts->n_clusters = ds.n_clusters;
    counts->n_tracklets = ds.n_tracklets;
    counts->n_tracks = ds.n_tracks;
    counts->n_hits = ds.n_hits;
    counts->n_fallback = ds.n_fallback;
    counts->n_fallback_fail = ds.n_fallback_fail;
    counts->n_not_pd = ds.n_not_pd;
    counts->n_refit_fail = ds.n_refit_fail;
    counts->overflow = ds.overflow;
    for (int k = 0; k < 4; ++k) counts->required_by[k] = ds.req[k];
    counts->follow_steps = ds.f_steps;
    counts->follow_candidates = ds.f_cands;
    counts->follow_updates = ds.f_upds;
    counts->follow_lane_slots = ds.f_slots;
  }
  DevStatus zero;
  std::memset(&zero, 0, sizeof zero);
  if (hipMemcpy(c->d_st, &zero, sizeof zero, hipMemcpyHostToDevice) != hipSuccess)
    return TPC_ERR_HIP;
  return ds.status;
}

void* tpc_stream(tpc_ctx* c) { return c ? (void*)c->stream : nullptr; }

int tpc_profile_enable(tpc_ctx* c, int on) {
  if (!c || on < 0 || on > 3) return TPC_ERR_ARG;
  c->count_work = (on & 2) != 0;
  on &= 1;
  if (on && !c->prof_events) {
    for (int i = 0; i < TPC_PROF_STAGES; ++i)
      for (int j = 0; j < 2; ++j)
        for (int k = 0; k < tpc_ctx::kProfCap; ++k)
          if (hipEventCreate(&c->prof_ev[i][j][k]) != hipSuccess) return TPC_ERR_HIP;
    c->prof_events = true;
  }
  c->prof_on = on != 0;
  return TPC_OK;
}

int tpc_profile_read(tpc_ctx* c, double* ms, uint32_t* launches) {
  if (!c || !ms || !launches) return TPC_ERR_ARG;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return TPC_ERR_HIP;
  for (int i = 0; i < TPC_PROF_STAGES; ++i) {
    double acc = 0;
    for (uint32_t k = 0; k < c->prof_n[i]; ++k) {
      float t = 0;
      if (hipEventElapsedTime(&t, c->prof_ev[i][0][k], c->prof_ev[i][1][k]) != hipSuccess)
        return TPC_ERR_HIP;
      acc += t;
    }
    ms[i] = acc;
    launches[i] = c->prof_n[i];
    c->prof_n[i] = 0;
  }
  return TPC_OK;
}

const char* tpc_profile_stage_name(int i) {
  static const char* names[TPC_PROF_STAGES] = {
      "sample_index", "cluster_peaks", "cluster_scan", "cluster_output", "cluster_grid",
      "neighbours", "tracklets", "following", "resolution", "refit", "fp64_count",
      "track_output", "zs_decode", "compress", "decompress", "merge"};
  return (i >= 0 && i < TPC_PROF_STAGES) ? names[i] : "unknown";
}

int tpc_tuning_default(tpc_tuning* t) {
  if (!t) return TPC_ERR_ARG;
  t->cl_window = 32;
  t->cl_chunk = 8;
  t->follow_block = 64;
  t->follow_mode = 2;
  t->refit_waves = 6;
  t->cl_mode = 2;
  return TPC_OK;
}

int tpc_set_tuning(tpc_ctx* c, const tpc_tuning* t) {
  if (!c || !t) return TPC_ERR_ARG;
  if (t->cl_window != 8 && t->cl_window != 16 && t->cl_window != 20 && t->cl_window != 24 &&
      t->cl_window != 32)
    return TPC_ERR_ARG;
  if ((t->cl_window == 20 || t->cl_window == 24) && t->cl_chunk != 8) return TPC_ERR_ARG;
  if (t->cl_chunk != 4 && t->cl_chunk != 8 && t->cl_chunk != 16) return TPC_ERR_ARG;
  // shared windows (mode 2) of 24 or 32 bins
  if (t->cl_mode < 0 || t->cl_mode > 2) return TPC_ERR_ARG;
  if (t->cl_mode == 2 && t->cl_window < 24) return TPC_ERR_ARG;
  if (t->follow_block != 64 && t->follow_block != 128 && t->follow_block != 256) return TPC_ERR_ARG;
  if (t->follow_mode < 0 || t->follow_mode > 2) return TPC_ERR_ARG;
  if (t->refit_waves != 0 && t->refit_waves != 4 && t->refit_waves != 5 && t->refit_waves != 6 &&
      t->refit_waves != 8)
    return TPC_ERR_ARG;
  c->tune = *t;
  return TPC_OK;
}

int tpc_get_tuning(tpc_ctx* c, tpc_tuning* t) {
  if (!c || !t) return TPC_ERR_ARG;
  *t = c->tune;
  return TPC_OK;
}

const char* tpc_status_string(int s) {
  switch (s) {
    case TPC_OK: return "ok";
    case TPC_ERR_ARG: return "invalid argument";
    case TPC_ERR_CAPACITY: return "capacity exceeded";
    case TPC_ERR_INPUT: return "malformed input";
    case TPC_ERR_HIP: return "HIP runtime error";
    case TPC_ERR_NUMERIC: return "numeric failure";
    case TPC_ERR_STATE: return "invalid state";
    default: return "unknown status";
  }
}

}  // extern "C"
