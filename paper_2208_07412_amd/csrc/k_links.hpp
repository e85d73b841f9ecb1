// Cellular-automaton neighbour finding and tracklet building.
//
// Clusters of each (unit,row) are sorted by peak time, and the block index
// (first cluster per 8 time bins) is the per-row hit grid: a drift-window
// lookup is two table reads, and the pad direction is filtered per candidate
// (a row holds a handful of clusters per window).  All decisions are exact
// integer arithmetic on the fixed-point positions.
#pragma once

#include "common.hpp"
#include "k_cluster.hpp"

struct ClusterView {
  const int32_t* y_fx;
  const int32_t* z_fx;
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

// Candidate cluster range of row ur for a drift position z (fixed point):
// |z_c - z| <= win_z and the centroid lies within 2 bins of the peak time.
__device__ __forceinline__ void nb_candidates(const ClusterView& cl, const uint32_t* cblk,
                                              uint32_t nblk, uint32_t ur, int64_t z, int64_t wz,
                                              uint32_t& a, uint32_t& b) {
  const int64_t lo = floor_div64(z - wz, 32768) - 3;
  const int64_t hi = floor_div64(z + wz, 32768) + 3;
  int32_t blo = lo < 0 ? 0 : (int32_t)(lo >> 3);
  int32_t bhi = hi < 0 ? -1 : (int32_t)(hi >> 3);
  if (blo > (int32_t)nblk - 1) blo = nblk - 1;
  if (bhi > (int32_t)nblk - 1) bhi = nblk - 1;
  row_range(cblk + (size_t)ur * (nblk + 1), nblk, blo, bhi + 1, cl.row_start(ur),
            cl.row_start(ur + 1), a, b);
}

__global__ __launch_bounds__(256) void k_neighbours(ClusterView cl, const uint32_t* __restrict__ cblk,
                                                    uint32_t nblk, uint32_t n_ur,
                                                    int32_t* __restrict__ down,
                                                    int32_t* __restrict__ up,
                                                    const DevParams* __restrict__ P,
                                                    const DevStatus* st) {
  if (failed(st)) return;
  const int64_t wy = P->win_y, wz = P->win_z, smax = P->s_max;
  const uint32_t nb = gridDim.x;
  for (uint32_t bid = blockIdx.x; bid < n_ur; bid += nb) {
    const uint32_t ur = bid;
    const int r = ur % NROW;
    const uint32_t c0 = cl.row_start(ur), c1 = cl.row_start(ur + 1);
    for (uint32_t i = c0 + threadIdx.x; i < c1; i += blockDim.x) {
      int32_t bd = -1, bu = -1;
      if (r >= 1 && r <= NROW - 2) {
        const int64_t yi = cl.y_fx[i], zi = cl.z_fx[i];
        uint32_t ja, jb, ka, kb;
        nb_candidates(cl, cblk, nblk, ur - 1, zi, wz, ja, jb);
        nb_candidates(cl, cblk, nblk, ur + 1, zi, wz, ka, kb);
        int64_t best = -1;
        for (uint32_t j = ja; j < jb; ++j) {
          const int64_t yj = cl.y_fx[j], zj = cl.z_fx[j];
          if (yj - yi > wy || yi - yj > wy || zj - zi > wz || zi - zj > wz) continue;
          const int64_t ay = 2 * yi - yj, az = 2 * zi - zj;
          for (uint32_t k = ka; k < kb; ++k) {
            const int64_t yk = cl.y_fx[k], zk = cl.z_fx[k];
            if (yk - yi > wy || yi - yk > wy || zk - zi > wz || zi - zk > wz) continue;
            const int64_t dy = ay - yk, dz = az - zk;
            const int64_t s = dy * dy + dz * dz;
            // j and k ascend, so a strict "<" keeps the smallest (j, k) on ties
            if (s <= smax && (best < 0 || s < best)) {
              best = s;
              bd = (int32_t)j;
              bu = (int32_t)k;
            }
          }
        }
      }
      down[i] = bd;
      up[i] = bu;
    }
  }
}

// Reciprocal links.
__global__ void k_ca_clean(const int32_t* __restrict__ down, const int32_t* __restrict__ up,
                           int32_t* __restrict__ downc, int32_t* __restrict__ upc,
                           const uint32_t* n_dev, uint32_t n_cap, const DevStatus* st) {
  if (failed(st)) return;
  const uint32_t n = scan_count(n_dev, n_cap);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int32_t u = up[i], d = down[i];
    upc[i] = (u >= 0 && (uint32_t)u < n && down[u] == (int32_t)i) ? u : -1;
    downc[i] = (d >= 0 && (uint32_t)d < n && up[d] == (int32_t)i) ? d : -1;
  }
}

// Length of the chain starting at every start cluster (0 for non-starts and
// chains shorter than min_tracklet).  Chains cross one row per link, so a
// walk longer than 152 means corrupt links and is cut.
__global__ void k_chain_len(const int32_t* __restrict__ downc, const int32_t* __restrict__ upc,
                            uint16_t* __restrict__ len, const uint32_t* n_dev, uint32_t n_cap,
                            const DevParams* __restrict__ P, const DevStatus* st) {
  if (failed(st)) return;
  const uint32_t n = scan_count(n_dev, n_cap);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    uint32_t L = 0;
    if (downc[i] == -1 && upc[i] != -1) {
      L = 1;
      int32_t c = upc[i];
      while (c >= 0 && (uint32_t)c < n && L < NROW) {
        ++L;
        c = upc[c];
      }
      if ((int)L < P->min_tracklet) L = 0;
    }
    len[i] = (uint16_t)L;
  }
}

struct GetKeepLen {
  const uint16_t* len;
  __device__ uint32_t operator()(uint32_t i) const { return len[i] != 0 ? 1u : 0u; }
};

struct EmitTracklet {
  const uint16_t* len;
  uint32_t* start;
  uint16_t* out_len;
  uint32_t capacity;
  __device__ void operator()(uint32_t i, uint32_t pos, uint32_t v) const {
    if (v && pos < capacity) {
      start[pos] = i;
      out_len[pos] = len[i];
    }
  }
};

__global__ void k_tracklet_count(const uint32_t* n_tl, uint32_t capacity, uint32_t* out_n,
                                 DevStatus* st) {
  const uint32_t n = *n_tl;
  st->n_tracklets = n;
  if (out_n) *out_n = n;
  if (n > capacity) latch(st, TPC_ERR_CAPACITY, n);
}
