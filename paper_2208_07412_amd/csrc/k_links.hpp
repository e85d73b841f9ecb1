// Cellular-automaton neighbour finding and tracklet building.
//
// Clusters of each (unit,row) are sorted by peak time, and the block index
// (first cluster per 4 time bins) is the per-row hit grid: a drift-window
// lookup is two table reads, and the pad direction is filtered per candidate
// (a row holds a handful of clusters per window).  All decisions are exact
// integer arithmetic on the fixed-point positions.
#pragma once

#include "common.hpp"
#include "k_cluster.hpp"

struct ClusterView {
  const int32_t* y_fx;
  const int32_t* z_fx;
  const int2* pos;           // (y_fx, z_fx) packed, one load per cluster
  const uint16_t* ptime;
  const uint32_t* crow;      // [n_ur+1]
  const uint32_t* n_clusters;
  uint32_t capacity;
  // row table entry clamped to the arrays, whatever the table holds
  __device__ uint32_t row_start(uint32_t ur) const {
    const uint32_t v = crow[ur];
    return v < capacity ? v : capacity;
  }
};

// Packed copy of the fixed-point positions for the search kernels.
__global__ void k_pack_pos(const int32_t* __restrict__ y, const int32_t* __restrict__ z,
                           const uint32_t* n_dev, uint32_t n_cap, int2* __restrict__ pos,
                           const DevStatus* st) {
  if (failed(st)) return;
  const uint32_t n = scan_count(n_dev, n_cap);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    pos[i] = make_int2(y[i], z[i]);
}

// The cluster grid (block index over peak times) has one entry per
// 2^CG_BSHIFT time bins.
#ifndef CG_BSHIFT
#define CG_BSHIFT 1
#endif

// Candidate cluster range of row ur for a drift position z (fixed point):
// |z_c - z| <= win_z and the centroid lies within 2 bins of the peak time.
__device__ __forceinline__ void nb_candidates(const ClusterView& cl, const uint32_t* cblk,
                                              uint32_t nblk, uint32_t ur, int64_t z, int64_t wz,
                                              uint32_t& a, uint32_t& b) {
  const int64_t lo = floor_div64(z - wz, 32768) - 3;
  const int64_t hi = floor_div64(z + wz, 32768) + 3;
  int32_t blo = lo < 0 ? 0 : (int32_t)(lo >> CG_BSHIFT);
  int32_t bhi = hi < 0 ? -1 : (int32_t)(hi >> CG_BSHIFT);
  if (blo > (int32_t)nblk - 1) blo = nblk - 1;
  if (bhi > (int32_t)nblk - 1) bhi = nblk - 1;
  row_range(cblk + (size_t)ur * (nblk + 1), nblk, blo, bhi + 1, cl.row_start(ur),
            cl.row_start(ur + 1), a, b);
}

// Best (j, k) pair for cluster i among the candidates [ja, jb) in row r-1
// and [ka, kb) in row r+1 (positions pos[]).  The k candidates inside the
// window are marked once in a 64-bit mask when the range has at most 64
// (most of a time window's candidates lie outside the y window), else listed
// in registers (up to NB_KLIST; beyond that the whole range is scanned per
// j).  Positions are below 2^30 in magnitude and
// windows are capped at 2^30 (far beyond any row), so every difference fits
// 32 bits and a score (sum of two squares) fits 64 bits unsigned; the
// decision is the exact integer one.
#define NB_KLIST 8
__device__ __forceinline__ bool nb_in(int32_t a, int32_t b, int32_t w) {
  const int32_t d = a - b;
  return d <= w && d >= -w;
}
template <class PJ, class PK>
__device__ __forceinline__ void nb_best(PJ J, PK K, int32_t yi, int32_t zi, int32_t wy,
                                        int32_t wz, uint64_t smax, uint32_t ja, uint32_t jb,
                                        uint32_t ka, uint32_t kb, int32_t& bd, int32_t& bu) {
  if (kb - ka <= 64) {
    // the in-window k candidates as a bit mask, walked in ascending order
    uint64_t km = 0;
    for (uint32_t k = ka; k < kb; ++k) {
      const int2 pk = K(k);
      if (nb_in(pk.x, yi, wy) && nb_in(pk.y, zi, wz)) km |= 1ull << (k - ka);
    }
    if (km == 0) return;
    uint64_t best = ~0ull;
    for (uint32_t j = ja; j < jb; ++j) {
      const int2 pj = J(j);
      if (!nb_in(pj.x, yi, wy) || !nb_in(pj.y, zi, wz)) continue;
      const int32_t ay = yi - pj.x, az = zi - pj.y;
      for (uint64_t m = km; m != 0; m &= m - 1) {
        const uint32_t k = ka + (uint32_t)__builtin_ctzll(m);
        const int2 pk = K(k);
        const int32_t dy = ay + (yi - pk.x), dz = az + (zi - pk.y);
        const uint64_t sc = (uint64_t)((int64_t)dy * dy) + (uint64_t)((int64_t)dz * dz);
        // j and k ascend, so a strict "<" keeps the smallest (j, k) on ties
        if (sc <= smax && sc < best) {
          best = sc;
          bd = (int32_t)j;
          bu = (int32_t)k;
        }
      }
    }
    return;
  }
  uint32_t kl[NB_KLIST];
  int nk = 0;
  bool over = false;
  for (uint32_t k = ka; k < kb; ++k) {
    const int2 pk = K(k);
    if (!nb_in(pk.x, yi, wy) || !nb_in(pk.y, zi, wz)) continue;
    if (nk < NB_KLIST) {
#pragma unroll
      for (int m = 0; m < NB_KLIST; ++m)
        if (m == nk) kl[m] = k;
      ++nk;
    } else {
      over = true;
    }
  }
  if (nk == 0) return;
  uint64_t best = ~0ull;
  for (uint32_t j = ja; j < jb; ++j) {
    const int2 pj = J(j);
    if (!nb_in(pj.x, yi, wy) || !nb_in(pj.y, zi, wz)) continue;
    // 2 y_i - y_j - y_k = (y_i - y_j) + (y_i - y_k), each term inside its window
    const int32_t ay = yi - pj.x, az = zi - pj.y;
    auto consider = [&](uint32_t k, int2 pk) {
      const int32_t dy = ay + (yi - pk.x), dz = az + (zi - pk.y);
      const uint64_t sc = (uint64_t)((int64_t)dy * dy) + (uint64_t)((int64_t)dz * dz);
      // j and k ascend, so a strict "<" keeps the smallest (j, k) on ties
      if (sc <= smax && sc < best) {
        best = sc;
        bd = (int32_t)j;
        bu = (int32_t)k;
      }
    };
    if (!over) {
#pragma unroll
      for (int m = 0; m < NB_KLIST; ++m) {
        if (m >= nk) break;
        consider(kl[m], K(kl[m]));
      }
    } else {
      for (uint32_t k = ka; k < kb; ++k) {
        const int2 pk = K(k);
        if (!nb_in(pk.x, yi, wy) || !nb_in(pk.y, zi, wz)) continue;
        consider(k, pk);
      }
    }
  }
}

// One lane per cluster, NB_PARTS workgroups per (unit,row), each part's
// clusters in batches of 64 per wave.  Each wave copies the union of its lanes'
// candidate ranges in rows r-1 and r+1 (contiguous: rows are time-sorted)
// into its own LDS slice when it fits and scores from there; no workgroup
// barrier is involved (a wave reads back its own LDS writes in order), so
// waves run independently and hide each other's latency.  (Staging per
// workgroup batch of 256 behind barriers serialised each workgroup's batches:
// 1.40 ms for the slice; reading every candidate through the caches: 1.13 ms.)
#define NB_WSTAGE 256
// parts of a row, each a workgroup taking a contiguous run of its 64-cluster
// batches (fewer idle compute units in the last round of rows; a 2 ms Pb-Pb
// slice: 0.645, 0.615, 0.625 and 0.631 ms with 1, 2, 4 and 8 parts)
#define NB_PARTS 2
__global__ __launch_bounds__(256) void k_neighbours(ClusterView cl, const uint32_t* __restrict__ cblk,
                                                    uint32_t nblk, uint32_t n_ur,
                                                    int32_t* __restrict__ down,
                                                    int32_t* __restrict__ up,
                                                    const DevParams* __restrict__ P,
                                                    const DevStatus* st) {
  __shared__ int2 sp[4][2][NB_WSTAGE];
  if (failed(st)) return;
  const int64_t wz64 = P->win_z;
  const int32_t wy = (int32_t)min(P->win_y, (int64_t)1 << 30);
  const int32_t wz = (int32_t)min(wz64, (int64_t)1 << 30);
  const uint64_t smax = (uint64_t)P->s_max;
  const uint32_t w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int2* sj = sp[w][0];
  int2* sk = sp[w][1];
  const uint32_t n_items = n_ur * NB_PARTS;
  for (uint32_t b = blockIdx.x; b < n_items; b += gridDim.x) {
    // consecutive rows of a sector share an XCD (and its L2) when the grid
    // covers every row
    const uint32_t item = gridDim.x == n_items ? xcd_remap(b, n_items) : b;
    const uint32_t ur = item / NB_PARTS, part = item % NB_PARTS;
    const int r = ur % NROW;
    const uint32_t r0 = cl.row_start(ur), r1 = cl.row_start(ur + 1);
    const uint32_t nbat = (r1 - r0 + 63) / 64;
    const uint32_t c0 = r0 + 64 * (nbat * part / NB_PARTS);
    const uint32_t c1 = min(r1, r0 + 64 * (nbat * (part + 1) / NB_PARTS));
    if (r < 1 || r > NROW - 2) {
      for (uint32_t i = c0 + threadIdx.x; i < c1; i += blockDim.x) {
        down[i] = -1;
        up[i] = -1;
      }
      continue;
    }
    for (uint32_t base = c0 + w * 64; base < c1; base += blockDim.x) {  // uniform per wave
      const uint32_t i = base + lane;
      const bool valid = i < c1;
      int32_t yi = 0, zi = 0;
      uint32_t ja = 0, jb = 0, ka = 0, kb = 0;
      if (valid) {
        const int2 pi = cl.pos[i];
        yi = pi.x;
        zi = pi.y;
        nb_candidates(cl, cblk, nblk, ur - 1, zi, wz64, ja, jb);
        nb_candidates(cl, cblk, nblk, ur + 1, zi, wz64, ka, kb);
      }
      const bool act = valid && jb > ja && kb > ka;
      // the wave's union ranges (inactive lanes contribute nothing)
      const uint32_t JA = (uint32_t)wave_min_i32(act ? (int32_t)ja : INT32_MAX);
      const uint32_t JB = (uint32_t)wave_max_i32(act ? (int32_t)jb : 0);
      const uint32_t KA = (uint32_t)wave_min_i32(act ? (int32_t)ka : INT32_MAX);
      const uint32_t KB = (uint32_t)wave_max_i32(act ? (int32_t)kb : 0);
      const bool stage = JB > JA && KB > KA && JB - JA <= NB_WSTAGE && KB - KA <= NB_WSTAGE;
      if (stage) {
        for (uint32_t t = lane; t < JB - JA; t += 64) sj[t] = cl.pos[JA + t];
        for (uint32_t t = lane; t < KB - KA; t += 64) sk[t] = cl.pos[KA + t];
      }
      // the wave's LDS writes before its reads (in order within a wave)
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      int32_t bd = -1, bu = -1;
      if (act) {
        if (stage) {
          auto J = [&](uint32_t c) { return sj[c - JA]; };
          auto K = [&](uint32_t c) { return sk[c - KA]; };
          nb_best(J, K, yi, zi, wy, wz, smax, ja, jb, ka, kb, bd, bu);
        } else {
          auto G = [&](uint32_t c) { return cl.pos[c]; };
          nb_best(G, G, yi, zi, wy, wz, smax, ja, jb, ka, kb, bd, bu);
        }
      }
      if (valid) {
        down[i] = bd;
        up[i] = bu;
      }
    }
  }
}

// Reciprocal links.  Also flags the start clusters of chains (no cleaned
// down-link, a cleaned up-link) in a byte per cluster, which the scan that
// lists them reads.
__global__ void k_ca_clean(const int32_t* __restrict__ down, const int32_t* __restrict__ up,
                           int32_t* __restrict__ downc, int32_t* __restrict__ upc,
                           uint8_t* __restrict__ start, const uint32_t* n_dev, uint32_t n_cap,
                           const DevStatus* st) {
  if (failed(st)) return;
  const uint32_t n = scan_count(n_dev, n_cap);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int32_t u = up[i], d = down[i];
    const int32_t uc = (u >= 0 && (uint32_t)u < n && down[u] == (int32_t)i) ? u : -1;
    const int32_t dc = (d >= 0 && (uint32_t)d < n && up[d] == (int32_t)i) ? d : -1;
    upc[i] = uc;
    downc[i] = dc;
    start[i] = (uint8_t)(dc == -1 && uc != -1);
  }
}

// Start clusters of chains, listed in ascending order by a scan so that the
// chain walks below run one lane per start on dense waves.
struct GetStart {
  const uint8_t* start;
  __device__ uint32_t operator()(uint32_t i) const { return start[i]; }
};
struct EmitStart {
  uint32_t* cand;
  uint32_t capacity;
  __device__ void operator()(uint32_t i, uint32_t pos, uint32_t v) const {
    if (v && pos < capacity) cand[pos] = i;
  }
};

// Length of the chain of every listed start (0 below min_tracklet).  Chains
// cross one row per link, so a walk longer than 152 means corrupt links and
// is cut.
__global__ void k_chain_len(const uint32_t* __restrict__ cand, const uint32_t* n_cand_dev,
                            uint32_t cand_cap, const int32_t* __restrict__ upc,
                            const uint32_t* n_cl_dev, uint32_t n_cl_cap,
                            uint16_t* __restrict__ len, const DevParams* __restrict__ P,
                            const DevStatus* st) {
  if (failed(st)) return;
  const uint32_t n = scan_count(n_cand_dev, cand_cap);
  const uint32_t n_cl = scan_count(n_cl_dev, n_cl_cap);
  uint32_t dp;
  for (uint32_t p = xcd_thread_item(n, dp); p < n; p += dp) {
    uint32_t L = 1;
    int32_t c = upc[cand[p]];
    while (c >= 0 && (uint32_t)c < n_cl && L < NROW) {
      ++L;
      c = upc[c];
    }
    if ((int)L < P->min_tracklet) L = 0;
    len[p] = (uint16_t)L;
  }
}

struct GetKeepLen {
  const uint16_t* len;
  __device__ uint32_t operator()(uint32_t p) const { return len[p] != 0 ? 1u : 0u; }
};

struct EmitTracklet {
  const uint32_t* cand;
  const uint16_t* len;
  uint32_t* start;
  uint16_t* out_len;
  uint32_t capacity;
  __device__ void operator()(uint32_t p, uint32_t pos, uint32_t v) const {
    if (v && pos < capacity) {
      start[pos] = cand[p];
      out_len[pos] = len[p];
    }
  }
};

__global__ void k_tracklet_count(const uint32_t* n_tl, uint32_t capacity, uint32_t* out_n,
                                 DevStatus* st) {
  // after a latched error the scan that wrote *n_tl did not run
  if (failed(st)) return;
  const uint32_t n = *n_tl;
  st->n_tracklets = n;
  if (out_n) *out_n = n;
  if (n > capacity) latch_capacity(st, OVF_TRACKLETS, n);
}
