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
#define CG_BSHIFT 1

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

// Best (j, k) pair for cluster i among the candidates [ja, jb) x [ka, kb),
// positions read through the accessors J (row r-1) and K (row r+1), which
// return (y, z) from LDS-staged rows or global memory.  The k candidates
// inside the window are listed once in registers (up to NB_KLIST; beyond
// that the whole range is scanned per j).  Positions are below 2^30 in
// magnitude and windows are capped at 2^30 (far beyond any row), so every
// difference fits 32 bits and a score (sum of two squares) fits 64 bits
// unsigned; the decision is the exact integer one.
#define NB_KLIST 8
__device__ __forceinline__ bool nb_in(int32_t a, int32_t b, int32_t w) {
  const int32_t d = a - b;
  return d <= w && d >= -w;
}
template <class PJ, class PK>
__device__ __forceinline__ void nb_best(PJ J, PK K, int32_t yi, int32_t zi, int32_t wy,
                                        int32_t wz, uint64_t smax, uint32_t ja, uint32_t jb,
                                        uint32_t ka, uint32_t kb, int32_t& bd, int32_t& bu) {
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

// One workgroup per (unit,row) walks the row's clusters in batches of 256
// (time order).  The candidate clusters of the two neighbouring rows for the
// whole batch -- a contiguous range in each, since rows are time-sorted --
// are staged in LDS when they fit, so every candidate is read from HBM once.
#define NB_STAGE 1024
__global__ __launch_bounds__(256) void k_neighbours(ClusterView cl, const uint32_t* __restrict__ cblk,
                                                    uint32_t nblk, uint32_t n_ur,
                                                    int32_t* __restrict__ down,
                                                    int32_t* __restrict__ up,
                                                    const DevParams* __restrict__ P,
                                                    const DevStatus* st) {
  __shared__ int2 sp[2][NB_STAGE];
  __shared__ uint32_t rng[4];
  if (failed(st)) return;
  const int64_t wz64 = P->win_z;
  const int32_t wy = (int32_t)min(P->win_y, (int64_t)1 << 30);
  const int32_t wz = (int32_t)min(wz64, (int64_t)1 << 30);
  const uint64_t smax = (uint64_t)P->s_max;
  for (uint32_t b = blockIdx.x; b < n_ur; b += gridDim.x) {
    // consecutive rows of a sector share an XCD (and its L2) when the grid
    // covers every row
    const uint32_t ur = gridDim.x == n_ur ? xcd_remap(b, n_ur) : b;
    const int r = ur % NROW;
    const uint32_t c0 = cl.row_start(ur), c1 = cl.row_start(ur + 1);
    if (r < 1 || r > NROW - 2) {
      for (uint32_t i = c0 + threadIdx.x; i < c1; i += blockDim.x) {
        down[i] = -1;
        up[i] = -1;
      }
      continue;
    }
    for (uint32_t base = c0; base < c1; base += blockDim.x) {
      const uint32_t i = base + threadIdx.x;
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
      if (threadIdx.x == 0) {
        rng[0] = 0xFFFFFFFFu;
        rng[1] = 0;
        rng[2] = 0xFFFFFFFFu;
        rng[3] = 0;
      }
      __syncthreads();
      if (valid && jb > ja) {
        atomicMin(&rng[0], ja);
        atomicMax(&rng[1], jb);
      }
      if (valid && kb > ka) {
        atomicMin(&rng[2], ka);
        atomicMax(&rng[3], kb);
      }
      __syncthreads();
      const uint32_t JA = rng[0], JB = rng[1], KA = rng[2], KB = rng[3];
      const bool stage_j = JB > JA && JB - JA <= NB_STAGE;
      const bool stage_k = KB > KA && KB - KA <= NB_STAGE;
      if (stage_j)
        for (uint32_t t = threadIdx.x; t < JB - JA; t += blockDim.x) {
          sp[0][t] = cl.pos[JA + t];
        }
      if (stage_k)
        for (uint32_t t = threadIdx.x; t < KB - KA; t += blockDim.x) {
          sp[1][t] = cl.pos[KA + t];
        }
      __syncthreads();
      int32_t bd = -1, bu = -1;
      if (valid && jb > ja && kb > ka) {
        auto Jl = [&](uint32_t c) { return sp[0][c - JA]; };
        auto Kl = [&](uint32_t c) { return sp[1][c - KA]; };
        auto G = [&](uint32_t c) { return cl.pos[c]; };
        if (stage_j && stage_k) nb_best(Jl, Kl, yi, zi, wy, wz, smax, ja, jb, ka, kb, bd, bu);
        else if (stage_j) nb_best(Jl, G, yi, zi, wy, wz, smax, ja, jb, ka, kb, bd, bu);
        else if (stage_k) nb_best(G, Kl, yi, zi, wy, wz, smax, ja, jb, ka, kb, bd, bu);
        else nb_best(G, G, yi, zi, wy, wz, smax, ja, jb, ka, kb, bd, bu);
      }
      if (valid) {
        down[i] = bd;
        up[i] = bu;
      }
      __syncthreads();
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
