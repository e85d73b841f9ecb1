// Clusterizer kernels.
//
// Work unit: one (unit,row) x one window of W time bins.  The samples of the
// window plus an 8-bin halo on each side are scattered into an LDS tile
// (ADC per (time, pad)); every sample then finds its uphill neighbour
// ("up code", the argmax of the (adc, time, pad) key over the 3x3
// neighbourhood, index (dt+1)*3 + (dp+1), 4 = itself) and every peak gathers
// the samples of its 5x5 window that reach it in at most two uphill steps.
// Clusters are written in the order of their peaks (time, then pad); windows
// find their output offsets by a decoupled look-back in ticket order, so the
// canonical order needs no second pass and no atomics on the outputs.
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

__device__ __forceinline__ int code_offset(int code) {
  return (code / 3 - 1) * CL_TP + (code % 3 - 1);
}

// ------------------------------------------------------------ window loop
// A workgroup is one wave (64 lanes); it walks K consecutive windows of one
// (unit,row).  The samples of the next window (core plus an 8-bin halo on
// each side) are loaded into registers while the current window is worked on
// from LDS, and the tile is cleared by writing zero back into exactly the
// cells that were filled.  Tile cells hold the ADC in bits 0-9; the emit pass
// adds the up code (bits 10-13) and the peak flag (bit 14) in place -- a
// cell's ADC bits never change, so neighbours reading them concurrently are
// unaffected.  Compaction is a ballot plus a population count per 64 samples.

#define CL_PRE 4     // samples per lane held in registers for the next window
#define CL_SLOTS 64  // peaks whose moments are accumulated per batch

struct WinRange {
  uint32_t s_lo, s_hi;  // window plus halo
  uint32_t c_lo, c_hi;  // core
};

__device__ __forceinline__ WinRange window_range(const uint32_t* zb, uint32_t nblk, int w, int W,
                                                 uint32_t rs0, uint32_t rs1) {
  WinRange R;
  const int b0 = (w * W) >> 3;
  row_range(zb, nblk, b0 - 1, b0 + W / 8 + 1, rs0, rs1, R.s_lo, R.s_hi);
  row_range(zb, nblk, b0, b0 + W / 8, rs0, rs1, R.c_lo, R.c_hi);
  return R;
}

// sample packed as time << 16 | pad (0xFFFFFFFF: none), plus its ADC
struct SampleRegs {
  uint32_t tp[CL_PRE];
  uint16_t a[CL_PRE];
};

__device__ __forceinline__ void prefetch(const ZsArgs& in, const WinRange& R, SampleRegs& S) {
#pragma unroll
  for (int j = 0; j < CL_PRE; ++j) {
    const uint32_t s = R.s_lo + threadIdx.x + j * 64;
    if (s < R.s_hi) {
      S.tp[j] = ((uint32_t)in.time[s] << 16) | in.pad[s];
      S.a[j] = in.adc[s];
    } else {
      S.tp[j] = 0xFFFFFFFFu;
      S.a[j] = 0;
    }
  }
}

// packed sample j of this lane's share of [s_lo, s_hi): registers first
__device__ __forceinline__ uint32_t sample_tp(const ZsArgs& in, const SampleRegs& S, uint32_t j,
                                              uint32_t s) {
  uint32_t tp = 0xFFFFFFFFu;
#pragma unroll
  for (int jj = 0; jj < CL_PRE; ++jj)
    if (j == (uint32_t)jj) tp = S.tp[jj];
  if (j >= CL_PRE) tp = ((uint32_t)in.time[s] << 16) | in.pad[s];
  return tp;
}

// tile cell of a sample, or -1 if it falls outside the tile or the row
template <int ROWS>
__device__ __forceinline__ int cell_of(uint32_t tp, int tile_t0, int np) {
  if (tp == 0xFFFFFFFFu) return -1;
  const int lt = (int)(tp >> 16) - tile_t0;
  const int p = (int)(tp & 0xFFFF);
  return (lt >= 0 && lt < ROWS && p < np) ? lt * CL_TP + p + 2 : -1;
}

// place (place = true) or clear the window's samples in the tile
template <int ROWS>
__device__ __forceinline__ void scatter(uint16_t* tile, const ZsArgs& in, const WinRange& R,
                                        const SampleRegs& S, int tile_t0, int np, bool place) {
#pragma unroll
  for (int j = 0; j < CL_PRE; ++j) {
    const int c = cell_of<ROWS>(S.tp[j], tile_t0, np);
    if (c >= 0) tile[c] = place ? (uint16_t)(S.a[j] & 0x3FF) : 0;
  }
  for (uint32_t s = R.s_lo + CL_PRE * 64 + threadIdx.x; s < R.s_hi; s += 64) {
    const uint32_t tp = ((uint32_t)in.time[s] << 16) | in.pad[s];
    const int c = cell_of<ROWS>(tp, tile_t0, np);
    if (c >= 0) tile[c] = place ? (uint16_t)(in.adc[s] & 0x3FF) : 0;
  }
}

// up code (bits 0-3) and peak flag (bit 4) of the sample in cell c
__device__ __forceinline__ int up_code_of(const uint16_t* tile, int c, int qmin) {
  const int a = tile[c] & 0x3FF;
  int best = a * 16 + 4, code = 4;
#pragma unroll
  for (int dt = -1; dt <= 1; ++dt)
#pragma unroll
    for (int dp = -1; dp <= 1; ++dp) {
      if (dt == 0 && dp == 0) continue;
      const int an = tile[c + dt * CL_TP + dp] & 0x3FF;
      const int idx = (dt + 1) * 3 + (dp + 1);
      const int k = an * 16 + idx;
      if (an != 0 && k > best) {
        best = k;
        code = idx;
      }
    }
  return code | ((code == 4 && a >= qmin) ? 16 : 0);
}

__device__ __forceinline__ uint32_t lanes_below() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

template <int W, int K>
__global__ __launch_bounds__(64) void k_cluster_count(ZsArgs in, const uint32_t* __restrict__ zblk,
                                                      uint32_t nblk, uint32_t nwin,
                                                      uint32_t nchunk, uint32_t n_ur,
                                                      uint32_t* __restrict__ win_cnt,
                                                      const DevParams* __restrict__ P,
                                                      const DevStatus* st) {
  constexpr int ROWS = W + 2 * CL_HALO;
  constexpr int TILE = ROWS * CL_TP;
  __shared__ __attribute__((aligned(16))) uint16_t tile[TILE];
  if (failed(st)) return;
  const uint32_t logical = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t ur = logical / nchunk, chunk = logical % nchunk;
  if (ur >= n_ur) return;
  const int np = P->np[ur % NROW], qmin = P->qmax_min;
  const uint32_t* zb = zblk + (size_t)ur * (nblk + 1);
  uint32_t rs0 = zb[0], rs1 = zb[nblk];
  if (rs1 > in.n_samples) rs1 = in.n_samples;
  if (rs0 > rs1) rs0 = rs1;
  const int w0 = chunk * K;
  const int w1 = min((int)nwin, w0 + K);
  {
    uint4* t4 = reinterpret_cast<uint4*>(tile);
    constexpr int N4 = TILE * 2 / 16;
    for (int i = threadIdx.x; i < N4; i += 64) t4[i] = make_uint4(0, 0, 0, 0);
    for (int i = N4 * 8 + threadIdx.x; i < TILE; i += 64) tile[i] = 0;
  }
  WinRange R = window_range(zb, nblk, w0, W, rs0, rs1);
  SampleRegs cur, nxt;
  prefetch(in, R, cur);
  __syncthreads();
  for (int w = w0; w < w1; ++w) {
    const int tile_t0 = w * W - CL_HALO;
    scatter<ROWS>(tile, in, R, cur, tile_t0, np, true);
    WinRange Rn = R;
    if (w + 1 < w1) {
      Rn = window_range(zb, nblk, w + 1, W, rs0, rs1);
      prefetch(in, Rn, nxt);
    }
    __syncthreads();
    uint32_t cnt = 0;
    for (uint32_t s0 = R.s_lo; s0 < R.c_hi; s0 += 64) {
      const uint32_t s = s0 + threadIdx.x;
      bool pk = false;
      if (s >= R.c_lo && s < R.c_hi) {
        const int c = cell_of<ROWS>(sample_tp(in, cur, (s0 - R.s_lo) >> 6, s), tile_t0, np);
        pk = c >= 0 && (up_code_of(tile, c, qmin) & 16);
      }
      cnt += __popcll(__ballot(pk));
    }
    if (threadIdx.x == 0) win_cnt[(size_t)ur * nwin + w] = cnt;
    __syncthreads();
    scatter<ROWS>(tile, in, R, cur, tile_t0, np, false);
    __syncthreads();
    R = Rn;
    cur = nxt;
  }
}

template <int W, int K>
__global__ __launch_bounds__(64) void k_cluster_emit(ZsArgs in, const uint32_t* __restrict__ zblk,
                                                     uint32_t nblk, uint32_t nwin, uint32_t nchunk,
                                                     uint32_t n_ur,
                                                     const uint32_t* __restrict__ win_off,
                                                     ClusterOut out,
                                                     const DevParams* __restrict__ P,
                                                     const DevStatus* st) {
  constexpr int ROWS = W + 2 * CL_HALO;
  constexpr int TILE = ROWS * CL_TP;
  __shared__ __attribute__((aligned(16))) uint16_t tile[TILE];
  __shared__ uint16_t pk_cell[CL_SLOTS];
  // per peak of the batch: q, sp, st, spp, stt, n, sat
  __shared__ int32_t acc[7][CL_SLOTS];
  if (failed(st)) return;
  const uint32_t logical = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t ur = logical / nchunk, chunk = logical % nchunk;
  if (ur >= n_ur) return;
  const int r = ur % NROW;
  const int np = P->np[r], qmin = P->qmax_min;
  const int64_t pfx = P->pfx[r];
  const uint32_t* zb = zblk + (size_t)ur * (nblk + 1);
  uint32_t rs0 = zb[0], rs1 = zb[nblk];
  if (rs1 > in.n_samples) rs1 = in.n_samples;
  if (rs0 > rs1) rs0 = rs1;
  const int w0 = chunk * K;
  const int w1 = min((int)nwin, w0 + K);
  {
    uint4* t4 = reinterpret_cast<uint4*>(tile);
    constexpr int N4 = TILE * 2 / 16;
    for (int i = threadIdx.x; i < N4; i += 64) t4[i] = make_uint4(0, 0, 0, 0);
    for (int i = N4 * 8 + threadIdx.x; i < TILE; i += 64) tile[i] = 0;
  }
  WinRange R = window_range(zb, nblk, w0, W, rs0, rs1);
  SampleRegs cur, nxt;
  prefetch(in, R, cur);
  __syncthreads();
  for (int w = w0; w < w1; ++w) {
    const int tile_t0 = w * W - CL_HALO;
    scatter<ROWS>(tile, in, R, cur, tile_t0, np, true);
    WinRange Rn = R;
    if (w + 1 < w1) {
      Rn = window_range(zb, nblk, w + 1, W, rs0, rs1);
      prefetch(in, Rn, nxt);
    }
    const uint32_t base = win_off[(size_t)ur * nwin + w];
    __syncthreads();
    // up codes of the samples within 4 bins of the core, written in place
    for (uint32_t s0 = R.s_lo; s0 < R.s_hi; s0 += 64) {
      const uint32_t s = s0 + threadIdx.x;
      if (s >= R.s_hi) continue;
      const uint32_t tp = sample_tp(in, cur, (s0 - R.s_lo) >> 6, s);
      const int c = cell_of<ROWS>(tp, tile_t0, np);
      const int lt = (int)(tp >> 16) - tile_t0;
      if (c < 0 || lt < CL_HALO - 4 || lt >= CL_HALO + W + 4) continue;
      const int code = up_code_of(tile, c, qmin);
      tile[c] = (uint16_t)((tile[c] & 0x3FF) | (code << 10));
    }
    __syncthreads();
    // peaks of the core in sample order, in batches of CL_SLOTS
    uint32_t done = 0;  // peaks handled in earlier batches
    for (;;) {
      uint32_t rank = 0, nb = 0;
      for (uint32_t s0 = R.s_lo; s0 < R.c_hi; s0 += 64) {
        const uint32_t s = s0 + threadIdx.x;
        int c = -1;
        if (s >= R.c_lo && s < R.c_hi)
          c = cell_of<ROWS>(sample_tp(in, cur, (s0 - R.s_lo) >> 6, s), tile_t0, np);
        const bool pk = c >= 0 && (tile[c] & 0x4000) != 0;
        const uint64_t m = __ballot(pk);
        const uint32_t k = rank + (uint32_t)__popcll(m & ((1ull << threadIdx.x) - 1ull));
        if (pk && k >= done && k < done + CL_SLOTS) pk_cell[k - done] = (uint16_t)c;
        rank += (uint32_t)__popcll(m);
      }
      nb = min(rank - done, (uint32_t)CL_SLOTS);
      if (nb == 0) break;
#pragma unroll
      for (int m = 0; m < 7; ++m) acc[m][threadIdx.x] = 0;
      __syncthreads();
      const int c_first = pk_cell[0], c_last = pk_cell[nb - 1];
      // every sample within two bins of the core adds itself to its peak
      for (uint32_t s0 = R.s_lo; s0 < R.s_hi; s0 += 64) {
        const uint32_t s = s0 + threadIdx.x;
        if (s >= R.s_hi) continue;
        const uint32_t tp = sample_tp(in, cur, (s0 - R.s_lo) >> 6, s);
        const int x = cell_of<ROWS>(tp, tile_t0, np);
        const int lt = (int)(tp >> 16) - tile_t0;
        if (x < 0 || lt < CL_HALO - 2 || lt >= CL_HALO + W + 2) continue;
        const int tx = tile[x];
        int own = -1;
        if (tx & 0x4000) {
          own = x;
        } else {
          const int y = x + code_offset((tx >> 10) & 15);
          const int ty = tile[y];
          if (ty & 0x4000) {
            own = y;
          } else {
            const int z = y + code_offset((ty >> 10) & 15);
            if (tile[z] & 0x4000) own = z;
          }
        }
        if (own < c_first || own > c_last) continue;
        // slot of the owner peak: binary search of the batch (ascending cells)
        int lo = 0, hi = (int)nb - 1;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if ((int)pk_cell[mid] < own) lo = mid + 1;
          else hi = mid;
        }
        if ((int)pk_cell[lo] != own) continue;
        const int a = tx & 0x3FF;
        const int d = x - own;
        const int dt = (d + 2 * CL_TP + 2) / CL_TP - 2;
        const int dp = d - dt * CL_TP;
        atomicAdd(&acc[0][lo], a);
        atomicAdd(&acc[1][lo], a * dp);
        atomicAdd(&acc[2][lo], a * dt);
        atomicAdd(&acc[3][lo], a * dp * dp);
        atomicAdd(&acc[4][lo], a * dt * dt);
        atomicAdd(&acc[5][lo], 1);
        if (a >= 1023) atomicOr(&acc[6][lo], 1);
      }
      __syncthreads();
      const uint32_t i = threadIdx.x;
      if (i < nb) {
        const int c = pk_cell[i];
        const int q = acc[0][i], sp = acc[1][i], st_ = acc[2][i], spp = acc[3][i],
                  stt = acc[4][i], ns = acc[5][i], sat = acc[6][i];
        const uint32_t k = base + done + i;
        if (k < out.capacity) {
          const int lt = c / CL_TP;
          const int ppad = c - lt * CL_TP - 2;
          const int ptime = lt + tile_t0;
          // exact: numerators below 2^53, quotients far from the rounding gap
          const double Q = q;
          const double u = 2.0 * ((double)ppad * Q + sp) - (double)(np - 1) * Q;
          out.y_fx[k] = (int32_t)floor((u * (double)pfx + Q) / (2.0 * Q));
          out.z_fx[k] = (int32_t)floor((65536.0 * ((double)ptime * Q + st_) + Q) / (2.0 * Q));
          const float fq = (float)q;
          const float mp = (float)sp / fq, mt = (float)st_ / fq;
          out.dpad[k] = mp;
          out.dtime[k] = mt;
          out.s2pad[k] = (float)spp / fq - mp * mp;
          out.s2time[k] = (float)stt / fq - mt * mt;
          out.qtot[k] = (uint16_t)q;
          out.qmax[k] = (uint16_t)(tile[c] & 0x3FF);
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
      done += nb;
      __syncthreads();
      if (done >= rank) break;
    }
    if (out.sample_label) {
      for (uint32_t s = R.c_lo + threadIdx.x; s < R.c_hi; s += 64) {
        const uint32_t tp = ((uint32_t)in.time[s] << 16) | in.pad[s];
        const int lt = (int)(tp >> 16) - tile_t0;
        const int c = cell_of<ROWS>(tp, tile_t0, np);
        int32_t lab = -1;
        if (c >= 0 && lt >= CL_HALO && lt < CL_HALO + W) {
          const int cx = tile[c];
          const int y = c + code_offset((cx >> 10) & 15);
          const int cy = tile[y];
          const int z = y + code_offset((cy >> 10) & 15);
          const int cz = tile[z];
          const int pk = (cx & 0x4000) ? c : ((cy & 0x4000) ? y : ((cz & 0x4000) ? z : -1));
          if (pk >= 0) lab = ((pk / CL_TP + tile_t0) << 8) | (pk % CL_TP - 2);
        }
        out.sample_label[s] = lab;
      }
    }
    __syncthreads();
    scatter<ROWS>(tile, in, R, cur, tile_t0, np, false);
    __syncthreads();
    R = Rn;
    cur = nxt;
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
