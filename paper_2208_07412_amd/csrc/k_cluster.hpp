// Clusterizer kernels.
//
// Work unit: one (unit,row) x one window of W time bins.  The samples of the
// window plus an 8-bin halo on each side are scattered into an LDS tile
// (ADC per (time, pad)); every sample then finds its uphill neighbour
// ("up code", the argmax of the (adc, time, pad) key over the 3x3
// neighbourhood) and every peak gathers the samples of its 5x5 window that
// reach it in at most two uphill steps.  Clusters are written in the order
// of their peaks (time, then pad), so a count pass, a device-wide scan over
// the windows and an emit pass give the canonical order without atomics.
#pragma once

#include "common.hpp"

#define CL_HALO 8
#define CL_TP 142  // tile row stride: pad p is stored in column p + 2

struct ZsArgs {
  const uint16_t* pad;
  const uint16_t* time;
  const uint16_t* adc;
  const uint32_t* row_start;
  uint32_t n_samples, n_units, n_time_bins;
};

struct ClusterOut {
  uint32_t capacity;
  int32_t *y_fx, *z_fx;
  float *dpad, *dtime, *s2pad, *s2time;
  uint16_t *qtot, *qmax, *ppad, *ptime;
  uint8_t* flags;
  int32_t *sp, *st, *spp, *stt;
  uint16_t* nsamp;
  int32_t* sample_label;
};

// Offsets of the samples (or clusters) of each (unit,row) per block of 8 time
// bins: blk[ur*(nblk+1) + b] = first index with key time >= 8b; the entry at
// nblk is the row end.  One workgroup per (unit,row); rows are time-sorted.
__global__ __launch_bounds__(256) void k_block_index(const uint16_t* __restrict__ tkey,
                                                     const uint16_t* __restrict__ pkey,
                                                     const uint32_t* __restrict__ rstart,
                                                     uint32_t n_ur, uint32_t nblk, uint32_t T,
                                                     uint32_t n_total, uint32_t* __restrict__ blk,
                                                     const DevParams* __restrict__ P,
                                                     DevStatus* st, int check_input) {
  if (failed(st)) return;
  for (uint32_t ur = blockIdx.x; ur < n_ur; ur += gridDim.x) {
    uint32_t s0 = rstart[ur], s1 = rstart[ur + 1];
    if (s1 > n_total) s1 = n_total;
    if (s0 > s1) s0 = s1;
    uint32_t* b = blk + (size_t)ur * (nblk + 1);
    if (s0 == s1) {
      for (uint32_t k = threadIdx.x; k <= nblk; k += blockDim.x) b[k] = s0;
      continue;
    }
    const int np = P->np[ur % NROW];
    for (uint32_t s = s0 + threadIdx.x; s < s1; s += blockDim.x) {
      uint32_t t = tkey[s];
      if (t >= T) {
        latch(st, TPC_ERR_INPUT);
        t = T - 1;
      }
      const uint32_t cur = t >> 3;
      int32_t prev = -1;
      if (s > s0) {
        uint32_t tp = tkey[s - 1];
        if (tp >= T) tp = T - 1;
        prev = (int32_t)(tp >> 3);
      }
      for (int32_t k = prev + 1; k <= (int32_t)cur; ++k) b[k] = s;
      if (s == s1 - 1)
        for (uint32_t k = cur + 1; k <= nblk; ++k) b[k] = s1;
      if (check_input) {
        const uint32_t p = pkey[s];
        if ((int)p >= np) latch(st, TPC_ERR_INPUT);
        if (P->validate && s > s0) {
          const uint32_t k0 = ((uint32_t)tkey[s - 1] << 8) | pkey[s - 1];
          const uint32_t k1 = (t << 8) | p;
          if (k1 <= k0) latch(st, TPC_ERR_INPUT);
        }
      }
      // a time-unsorted row leaves some entries stale; readers clamp every
      // range to the row, so this is reported but never read out of bounds
      if ((int32_t)cur < prev) latch(st, TPC_ERR_INPUT);
    }
  }
}

// After an input error the block table may be inconsistent; clamp it so that
// later stages read only inside each row.
__device__ __forceinline__ void row_range(const uint32_t* blk_row, uint32_t nblk, int32_t b_lo,
                                          int32_t b_hi, uint32_t s0, uint32_t s1, uint32_t& a,
                                          uint32_t& b) {
  if (b_lo < 0) b_lo = 0;
  if (b_hi > (int32_t)nblk) b_hi = nblk;
  if (b_hi < b_lo) b_hi = b_lo;
  a = blk_row[b_lo];
  b = blk_row[b_hi];
  if (a < s0) a = s0;
  if (a > s1) a = s1;
  if (b < a) b = a;
  if (b > s1) b = s1;
}

// Up code of the sample in tile cell (lt, col): index (dt+1)*3 + (dp+1) of the
// neighbour with the largest key (adc, then time, then pad); 4 = itself.
__device__ __forceinline__ int up_code(const uint16_t* __restrict__ tile, int lt, int col) {
  const int c = lt * CL_TP + col;
  int best = (int)tile[c] * 16 + 4;
  int code = 4;
#pragma unroll
  for (int dt = -1; dt <= 1; ++dt)
#pragma unroll
    for (int dp = -1; dp <= 1; ++dp) {
      if (dt == 0 && dp == 0) continue;
      const int a = tile[c + dt * CL_TP + dp];
      const int idx = (dt + 1) * 3 + (dp + 1);
      const int k = a * 16 + idx;
      if (a != 0 && k > best) {
        best = k;
        code = idx;
      }
    }
  return code;
}

__device__ __forceinline__ int code_offset(int code) {
  return (code / 3 - 1) * CL_TP + (code % 3 - 1);
}

template <int W, bool EMIT>
__global__ __launch_bounds__(256) void k_cluster(ZsArgs in, const uint32_t* __restrict__ zblk,
                                                 uint32_t nblk, uint32_t nwin, uint32_t n_ur,
                                                 uint32_t* __restrict__ win_cnt,
                                                 const uint32_t* __restrict__ win_off,
                                                 ClusterOut out, const DevParams* __restrict__ P,
                                                 DevStatus* st) {
  constexpr int ROWS = W + 2 * CL_HALO;
  constexpr int TILE = ROWS * CL_TP;
  __shared__ __attribute__((aligned(16))) uint16_t tile[TILE];
  __shared__ uint8_t codes[EMIT ? TILE : 1];
  __shared__ uint32_t lds_scan[256 / 64 + 1];
  if (failed(st)) return;
  const uint32_t logical = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t ur = logical / nwin, w = logical % nwin;
  if (ur >= n_ur) return;
  const int r = ur % NROW;
  const int np = P->np[r];
  const int t0 = (int)w * W;
  const int b0 = t0 >> 3;
  const uint32_t* zb = zblk + (size_t)ur * (nblk + 1);
  uint32_t rs0 = in.row_start[ur], rs1 = in.row_start[ur + 1];
  if (rs1 > in.n_samples) rs1 = in.n_samples;
  if (rs0 > rs1) rs0 = rs1;
  uint32_t s_lo, s_hi, c_lo, c_hi;
  row_range(zb, nblk, b0 - 1, b0 + W / 8 + 1, rs0, rs1, s_lo, s_hi);
  row_range(zb, nblk, b0, b0 + W / 8, rs0, rs1, c_lo, c_hi);
  const int tile_t0 = t0 - CL_HALO;

  // zero the ADC tile with 16-byte stores
  {
    uint4* t4 = reinterpret_cast<uint4*>(tile);
    constexpr int N4 = TILE * 2 / 16;
    for (int i = threadIdx.x; i < N4; i += 256) t4[i] = make_uint4(0, 0, 0, 0);
    for (int i = N4 * 8 + threadIdx.x; i < TILE; i += 256) tile[i] = 0;
  }
  __syncthreads();
  for (uint32_t s = s_lo + threadIdx.x; s < s_hi; s += 256) {
    const int lt = (int)in.time[s] - tile_t0;
    const int p = in.pad[s];
    if (lt >= 0 && lt < ROWS && p < np) tile[lt * CL_TP + p + 2] = in.adc[s];
  }
  __syncthreads();

  if constexpr (!EMIT) {
    uint32_t cnt = 0;
    for (uint32_t s = c_lo + threadIdx.x; s < c_hi; s += 256) {
      const int lt = (int)in.time[s] - tile_t0;
      const int p = in.pad[s];
      if (lt < CL_HALO || lt >= CL_HALO + W || p >= np) continue;
      const int a = tile[lt * CL_TP + p + 2];
      cnt += (a >= P->qmax_min && up_code(tile, lt, p + 2) == 4) ? 1u : 0u;
    }
    uint32_t total;
    block_excl_scan<uint32_t, 256>(cnt, lds_scan, total);
    if (threadIdx.x == 0) win_cnt[(size_t)ur * nwin + w] = total;
    return;
  } else {
    // up codes (bit 4: peak) of every sample within 4 bins of the core
    for (uint32_t s = s_lo + threadIdx.x; s < s_hi; s += 256) {
      const int lt = (int)in.time[s] - tile_t0;
      const int p = in.pad[s];
      if (lt < CL_HALO - 4 || lt >= CL_HALO + W + 4 || p >= np) continue;
      const int col = p + 2;
      const int code = up_code(tile, lt, col);
      const bool peak = code == 4 && tile[lt * CL_TP + col] >= P->qmax_min;
      codes[lt * CL_TP + col] = (uint8_t)(code | (peak ? 16 : 0));
    }
    __syncthreads();
    const uint32_t base = win_off[(size_t)ur * nwin + w];
    uint32_t running = 0;
    const int64_t pfx = P->pfx[r];
    for (uint32_t s0 = c_lo; s0 < c_hi; s0 += 256) {
      const uint32_t s = s0 + threadIdx.x;
      int lt = 0, col = 0;
      bool pk = false;
      if (s < c_hi) {
        lt = (int)in.time[s] - tile_t0;
        const int p = in.pad[s];
        col = p + 2;
        if (lt >= CL_HALO && lt < CL_HALO + W && p < np) pk = (codes[lt * CL_TP + col] & 16) != 0;
      }
      uint32_t chunk_total;
      const uint32_t rank = block_excl_scan<uint32_t, 256>(pk ? 1u : 0u, lds_scan, chunk_total);
      if (pk) {
        const int c = lt * CL_TP + col;
        // Branch-free gather over the 5x5 window: every cell is read, and a
        // cell counts with weight adc when it is the peak or reaches the
        // peak in one or two uphill steps.  Empty cells (adc 0) point to
        // themselves, so their code bytes, which are never written, are
        // only compared, never followed.
        int q = 0, sp = 0, st_ = 0, spp = 0, stt = 0, ns = 0, sat = 0;
#pragma unroll
        for (int dt = -2; dt <= 2; ++dt)
#pragma unroll
          for (int dp = -2; dp <= 2; ++dp) {
            const int x = c + dt * CL_TP + dp;
            const int a = tile[x];
            const int kx = a != 0 ? (codes[x] & 15) : 4;
            const int y = x + code_offset(kx);
            const int cy = codes[y];
            const int z = y + code_offset(cy & 15);
            const int mine = (a != 0) & ((y == c) | (((cy & 16) == 0) & (z == c)) | (x == c));
            const int wgt = mine ? a : 0;
            q += wgt;
            sp += wgt * dp;
            st_ += wgt * dt;
            spp += wgt * dp * dp;
            stt += wgt * dt * dt;
            ns += mine;
            sat |= mine & (a >= 1023 ? 1 : 0);
          }
        const uint32_t k = base + running + rank;
        if (k < out.capacity) {
          const int ppad = col - 2;
          const int ptime = lt + tile_t0;
          const int64_t Q = q;
          const int64_t u = 2 * ((int64_t)ppad * Q + sp) - (int64_t)(np - 1) * Q;
          out.y_fx[k] = (int32_t)floor_div64(u * pfx + Q, 2 * Q);
          out.z_fx[k] = (int32_t)floor_div64(65536 * ((int64_t)ptime * Q + st_) + Q, 2 * Q);
          const float fq = (float)q;
          const float mp = (float)sp / fq, mt = (float)st_ / fq;
          out.dpad[k] = mp;
          out.dtime[k] = mt;
          out.s2pad[k] = (float)spp / fq - mp * mp;
          out.s2time[k] = (float)stt / fq - mt * mt;
          out.qtot[k] = (uint16_t)q;
          out.qmax[k] = tile[c];
          out.ppad[k] = (uint16_t)ppad;
          out.ptime[k] = (uint16_t)ptime;
          out.flags[k] = (uint8_t)(((ppad <= 1 || ppad >= np - 2) ? 1 : 0) | (sat ? 2 : 0));
          if (out.sp) {
            out.sp[k] = sp;
            out.st[k] = st_;
            out.spp[k] = spp;
            out.stt[k] = stt;
            out.nsamp[k] = (uint16_t)ns;
          }
        }
      }
      running += chunk_total;
    }
    // sample -> peak position (resolved to a cluster id by k_sample_label)
    if (out.sample_label) {
      for (uint32_t s = c_lo + threadIdx.x; s < c_hi; s += 256) {
        const int lt = (int)in.time[s] - tile_t0;
        const int p = in.pad[s];
        int32_t lab = -1;
        if (lt >= CL_HALO && lt < CL_HALO + W && p < np) {
          // owner peak in at most two uphill steps (all cells here hold samples)
          const int x = lt * CL_TP + p + 2;
          const int cx = codes[x];
          const int y = x + code_offset(cx & 15);
          const int cy = codes[y];
          const int z = y + code_offset(cy & 15);
          const int cz = codes[z];
          const int pk = (cx & 16) ? x : ((cy & 16) ? y : ((cz & 16) ? z : -1));
          if (pk >= 0) lab = ((pk / CL_TP + tile_t0) << 8) | (pk % CL_TP - 2);
        }
        out.sample_label[s] = lab;
      }
    }
  }
}

// crow_start[ur] = first cluster of (unit,row), from the scanned window counts.
__global__ void k_crow_start(const uint32_t* __restrict__ win_off, uint32_t nwin, uint32_t n_ur,
                             const uint32_t* __restrict__ n_clusters, uint32_t capacity,
                             uint32_t* __restrict__ crow, DevStatus* st) {
  const uint32_t n = *n_clusters;
  for (uint32_t ur = blockIdx.x * blockDim.x + threadIdx.x; ur <= n_ur;
       ur += gridDim.x * blockDim.x)
    crow[ur] = ur < n_ur ? win_off[(size_t)ur * nwin] : n;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->n_clusters = n;
    if (n > capacity) latch(st, TPC_ERR_CAPACITY, n);
  }
}

// Replace the packed peak position of every sample by its cluster id
// (binary search among the row's clusters, which are sorted by peak).
__global__ __launch_bounds__(256) void k_sample_label(ZsArgs in, const uint32_t* __restrict__ crow,
                                                      const uint16_t* __restrict__ ppad,
                                                      const uint16_t* __restrict__ ptime,
                                                      uint32_t n_ur, int32_t* __restrict__ label,
                                                      const DevStatus* st) {
  if (failed(st)) return;
  for (uint32_t ur = blockIdx.x; ur < n_ur; ur += gridDim.x) {
    uint32_t s0 = in.row_start[ur], s1 = in.row_start[ur + 1];
    if (s1 > in.n_samples) s1 = in.n_samples;
    for (uint32_t s = s0 + threadIdx.x; s < s1; s += blockDim.x) {
      const int32_t v = label[s];
      if (v < 0) continue;
      const uint32_t key = (uint32_t)v;
      uint32_t a = crow[ur], b = crow[ur + 1];
      while (a < b) {
        const uint32_t m = (a + b) >> 1;
        const uint32_t km = ((uint32_t)ptime[m] << 8) | ppad[m];
        if (km < key) a = m + 1;
        else b = m;
      }
      label[s] = (a < crow[ur + 1] && (((uint32_t)ptime[a] << 8) | ppad[a]) == key) ? (int32_t)a : -1;
    }
  }
}
