// Clusterizer kernels.
//
// Work unit: one (unit,row) x one window of W time bins.  The samples of the
// window plus a 4-bin halo on each side are scattered into an LDS tile
// (ADC per (time, pad)); every sample then finds its uphill neighbour
// ("up code", the argmax of the (adc, time, pad) key over the 3x3
// neighbourhood, encoded (dt+1)*4 + (dp+1), 5 = itself) and every peak
// accumulates the samples of its 5x5 window that reach it in at most two
// uphill steps.  Clusters come out in the order of their peaks (time, then
// pad): the peak pass writes one raw record per peak beside the window's
// samples and each window's peak count, a device-wide scan turns the counts
// into output offsets, and the output pass writes each cluster at its final
// index, with no atomics on the outputs.
#pragma once

#include "common.hpp"

#define CL_HALO 4    // time bins loaded on each side of a window
// time bins kept in the shared-window tile on each side of a window: a
// sample reaches a core peak in two uphill steps only from within 2 bins of
// the core, so up codes are needed there and ADCs one bin further out
#define CL_TH 3
#define CL_BSHIFT 2  // the sample index has one entry per 4 time bins
#define CL_TP 142    // tile row stride: pad p is stored in column p + 2

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

// Offsets of the samples (or clusters) of each (unit,row) per block of
// 2^bshift time bins: blk[ur*(nblk+1) + b] = first index with key time >=
// b << bshift; the entry at nblk is the row end.  Rows are time-sorted.  A
// key needs only the key before it (read from memory), so without LDS
// staging a row is split into BI_PARTS workgroups, each taking a contiguous
// part of its keys (the last part writes the row end); with staging, one
// workgroup per (unit,row).  Each thread takes 8 consecutive keys
// per step (one 16-byte load when the key array is 16-byte aligned; the
// aligned block never crosses a page, and keys outside the row are masked).
// A key writes the entries of the blocks between its predecessor's and its
// own; with USE_LDS, when the row's table fits (BI_LDS entries), these writes
// go to LDS and the table is copied out in one coalesced pass (worth it where
// keys are sparse in time, as clusters are: ~9 entries per key, against
// one per 16 keys for the samples).
__device__ __forceinline__ void bi_sample(uint32_t s, uint32_t t, int32_t prev, uint32_t s1,
                                          uint32_t nblk, uint32_t bshift, uint32_t* b,
                                          DevStatus* st) {
  const int32_t cur = (int32_t)(t >> bshift);
  for (int32_t k = prev + 1; k <= cur; ++k) b[k] = s;
  if (s == s1 - 1)
    for (uint32_t k = cur + 1; k <= nblk; ++k) b[k] = s1;
  // a time-unsorted row leaves some entries stale; readers clamp every
  // range to the row, so this is reported but never read out of bounds
  if (cur < prev) latch(st, TPC_ERR_INPUT);
}

#define BI_LDS 6144
// parts per row of the unstaged index (a 2 ms Pb-Pb slice: 0.256, 0.233, 0.244
// and 0.275 ms with 1, 4, 8 and 16 parts)
#define BI_PARTS 4
template <bool USE_LDS>
__global__ __launch_bounds__(256) void k_block_index(const uint16_t* __restrict__ tkey,
                                                     const uint16_t* __restrict__ pkey,
                                                     const uint16_t* __restrict__ akey,
                                                     const uint32_t* __restrict__ rstart,
                                                     uint32_t n_ur, uint32_t nblk, uint32_t bshift,
                                                     uint32_t T, uint32_t n_total,
                                                     uint32_t* __restrict__ blk,
                                                     const DevParams* __restrict__ P,
                                                     DevStatus* st, int check_input) {
  __shared__ uint32_t lt[USE_LDS ? BI_LDS : 1];
  if (failed(st)) return;
  const bool vec = ((uintptr_t)tkey & 15) == 0 && (!check_input || ((uintptr_t)pkey & 15) == 0);
  const bool staged = USE_LDS && nblk + 1 <= BI_LDS;
  constexpr uint32_t parts = USE_LDS ? 1 : BI_PARTS;
  for (uint32_t item = blockIdx.x; item < n_ur * parts; item += gridDim.x) {
    const uint32_t ur = item / parts, part = item % parts;
    uint32_t s0 = rstart[ur], s1 = rstart[ur + 1];
    if (s1 > n_total) s1 = n_total;
    if (s0 > s1) s0 = s1;
    uint32_t* const bg = blk + (size_t)ur * (nblk + 1);
    if (s0 == s1) {
      if (part == 0)
        for (uint32_t k = threadIdx.x; k <= nblk; k += blockDim.x) bg[k] = s0;
      continue;
    }
    // this part's 8-key groups
    const uint32_t glo = s0 >> 3, ng = ((s1 + 7) >> 3) - glo;
    const uint32_t g0 = glo + (uint32_t)((uint64_t)ng * part / parts);
    const uint32_t g1 = glo + (uint32_t)((uint64_t)ng * (part + 1) / parts);
    // the row's table: in LDS (every entry preset to the row start, so an
    // unsorted row, which is reported, leaves no stale entry) or in place
    uint32_t* b = bg;
    if (staged) {
      __syncthreads();  // the previous row's copy-out has read lt
      for (uint32_t k = threadIdx.x; k <= nblk; k += blockDim.x) lt[k] = s0;
      __syncthreads();
      b = lt;
    }
    const int np = P->np[ur % NROW];
    const bool validate = check_input && P->validate;
    for (uint32_t g = g0 + threadIdx.x; g < g1; g += blockDim.x) {
      const uint32_t base = g << 3;
      uint16_t tv[8], pv[8];
      if (vec) {
        const uint4 tq = *reinterpret_cast<const uint4*>(tkey + base);
        const uint32_t tw[4] = {tq.x, tq.y, tq.z, tq.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) tv[e] = (uint16_t)(tw[e >> 1] >> ((e & 1) * 16));
        if (check_input) {
          const uint4 pq = *reinterpret_cast<const uint4*>(pkey + base);
          const uint32_t pw[4] = {pq.x, pq.y, pq.z, pq.w};
#pragma unroll
          for (int e = 0; e < 8; ++e) pv[e] = (uint16_t)(pw[e >> 1] >> ((e & 1) * 16));
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const uint32_t s = base + e;
          tv[e] = (s >= s0 && s < s1) ? tkey[s] : 0;
          pv[e] = (check_input && s >= s0 && s < s1) ? pkey[s] : 0;
        }
      }
      if (vec && check_input && !validate && base >= s0 && base + 8 < s1) {
        // a group inside the row, not holding its last key: the checks of
        // the general path below, without its per-key range tests, and one
        // report per group
        uint32_t tq0 = (base > s0) ? (uint32_t)tkey[base - 1] : 0;
        int32_t prev = base > s0 ? (int32_t)((tq0 < T ? tq0 : T - 1) >> bshift) : -1;
        bool bad = false;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          uint32_t t = tv[e];
          bad |= t >= T || (int)pv[e] >= np;
          if (t >= T) t = T - 1;
          const int32_t cur = (int32_t)(t >> bshift);
          for (int32_t k = prev + 1; k <= cur; ++k) b[k] = base + e;
          bad |= cur < prev;
          prev = cur;
        }
        if (bad) latch(st, TPC_ERR_INPUT);
        continue;
      }
      // key before this group (inside the row)
      uint32_t tp = (base > s0) ? (uint32_t)tkey[base - 1] : 0;
      uint32_t pp = (validate && base > s0) ? (uint32_t)pkey[base - 1] : 0;
      if (tp >= T) tp = T - 1;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const uint32_t s = base + e;
        uint32_t t = tv[e];
        const uint32_t p = pv[e];
        if (s >= s0 && s < s1) {
          const uint32_t traw = t;
          if (t >= T) {
            latch(st, TPC_ERR_INPUT);
            t = T - 1;
          }
          bi_sample(s, t, s > s0 ? (int32_t)(tp >> bshift) : -1, s1, nblk, bshift, b, st);
          if (check_input) {
            if ((int)p >= np) latch(st, TPC_ERR_INPUT);
            if (validate && s > s0 && ((traw << 8) | p) <= ((tp << 8) | pp))
              latch(st, TPC_ERR_INPUT);
            // a zero-suppressed sample carries a 10-bit ADC above zero
            if (validate && akey) {
              const uint32_t a = akey[s];
              if (a == 0 || a > 1023) latch(st, TPC_ERR_INPUT);
            }
          }
          tp = t;
          pp = p;
        }
      }
    }
    if (staged) {
      __syncthreads();
      for (uint32_t k = threadIdx.x; k <= nblk; k += blockDim.x) bg[k] = lt[k];
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

// tile offset of the neighbour an up code points at
__device__ __forceinline__ int code_offset(int code) {
  // (code >> 2) < 4: a 24-bit multiply
  return (int)__umul24((uint32_t)(code >> 2) & 3u, CL_TP) - CL_TP + ((code & 3) - 1);
}

// ------------------------------------------------------------ tile cells
// A 16-bit tile cell holds the ADC in bits 0-9.  The emit pass adds, in place:
//   non-peak: the up code in bits 10-13;
//   peak:     bit 14, and the peak's slot in the current moment batch in
//             bits 10-13 (low four bits) and 15 (fifth bit); slot 31 = none.
// A cell's ADC bits never change, so neighbours reading them concurrently are
// unaffected.
#define CL_PEAK 0x4000
#define CL_SLOTS 31  // peaks whose moments are accumulated per batch
#define CL_NOSLOT 0xBC00

__device__ __forceinline__ int slot_bits(int k) { return ((k & 15) << 10) | ((k & 16) << 11); }
__device__ __forceinline__ int slot_of(int cell) {
  return ((cell >> 10) & 15) | ((cell >> 11) & 16);
}
// up code of a cell for the owner chase; a peak points at itself
__device__ __forceinline__ int chase_code(int cell) {
  return (cell & CL_PEAK) ? 5 : ((cell >> 10) & 15);
}

// ------------------------------------------------------------ window loop
// A workgroup is one wave (64 lanes); it walks K consecutive windows of one
// (unit,row).  The samples of the next window (core plus halo) are loaded
// into registers while the current window is worked on from LDS, and the tile
// is cleared by writing zero back into exactly the cells that were filled.
// Compaction is a ballot plus a population count per 64 samples.

struct WinRange {
  uint32_t s_lo, s_hi;  // window plus halo
  uint32_t c_lo, c_hi;  // core
};

template <int W>
__device__ __forceinline__ WinRange window_range(const uint32_t* zb, uint32_t nblk, int w,
                                                 uint32_t rs0, uint32_t rs1) {
  constexpr int BW = W >> CL_BSHIFT, BH = CL_HALO >> CL_BSHIFT;
  WinRange R;
  const int b0 = w * BW;
  row_range(zb, nblk, b0 - BH, b0 + BW + BH, rs0, rs1, R.s_lo, R.s_hi);
  row_range(zb, nblk, b0, b0 + BW, rs0, rs1, R.c_lo, R.c_hi);
  R.s_lo = uni(R.s_lo);
  R.s_hi = uni(R.s_hi);
  R.c_lo = uni(R.c_lo);
  R.c_hi = uni(R.c_hi);
  return R;
}

// sample packed as time << 16 | pad (0xFFFFFFFF: none), plus its ADC
template <int PRE>
struct SampleRegs {
  uint32_t tp[PRE];
  uint16_t a[PRE];
};

template <int PRE>
__device__ __forceinline__ void prefetch(const ZsArgs& in, const WinRange& R, SampleRegs<PRE>& S) {
#pragma unroll
  for (int j = 0; j < PRE; ++j) {
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
template <int PRE>
__device__ __forceinline__ uint32_t sample_tp(const ZsArgs& in, const SampleRegs<PRE>& S,
                                              uint32_t j, uint32_t s) {
  uint32_t tp = 0xFFFFFFFFu;
#pragma unroll
  for (int jj = 0; jj < PRE; ++jj)
    if (j == (uint32_t)jj) tp = S.tp[jj];
  if (j >= PRE) tp = ((uint32_t)in.time[s] << 16) | in.pad[s];
  return tp;
}

// tile cell of a sample, or -1 if it falls outside the tile or the row
template <int ROWS>
__device__ __forceinline__ int cell_of(uint32_t tp, int tile_t0, int np) {
  if (tp == 0xFFFFFFFFu) return -1;
  const int lt = (int)(tp >> 16) - tile_t0;
  const int p = (int)(tp & 0xFFFF);
  // lt < ROWS < 256 where used: a 24-bit multiply
  return (lt >= 0 && lt < ROWS && p < np)
             ? (int)__umul24(__builtin_amdgcn_ubfe((uint32_t)lt, 0, 8), CL_TP) + p + 2
             : -1;
}

// place (place = true) or clear the window's samples in the tile
template <int ROWS, int PRE>
__device__ __forceinline__ void scatter(uint16_t* tile, const ZsArgs& in, const WinRange& R,
                                        const SampleRegs<PRE>& S, int tile_t0, int np, bool place) {
#pragma unroll
  for (int j = 0; j < PRE; ++j) {
    const int c = cell_of<ROWS>(S.tp[j], tile_t0, np);
    if (c >= 0) tile[c] = place ? (uint16_t)(S.a[j] & 0x3FF) : 0;
  }
  for (uint32_t s = R.s_lo + PRE * 64 + threadIdx.x; s < R.s_hi; s += 64) {
    const uint32_t tp = ((uint32_t)in.time[s] << 16) | in.pad[s];
    const int c = cell_of<ROWS>(tp, tile_t0, np);
    if (c >= 0) tile[c] = place ? (uint16_t)(in.adc[s] & 0x3FF) : 0;
  }
}

// ADC of the cells c-1, c, c+1 of one tile row (bits 0-9 of three 16-bit
// fields): two aligned 32-bit LDS reads cover them whatever the parity of c.
struct Row3 {
  int l, m, r;
};
__device__ __forceinline__ Row3 row3(const uint16_t* tile, int c) {
  const uint32_t* t32 = reinterpret_cast<const uint32_t*>(tile);
  const int w = (c - 1) >> 1;
  const uint64_t v = ((uint64_t)t32[w + 1] << 32 | t32[w]) >> (((c - 1) & 1) * 16);
  return Row3{(int)(v & 0x3FF), (int)((v >> 16) & 0x3FF), (int)((v >> 32) & 0x3FF)};
}

// up code (bits 0-3) and peak flag (bit 4) of the sample in cell c: the
// argmax of the key (adc, time, pad) over the cell and its present neighbours;
// a = the cell's ADC
//
// key = adc * 16 + code: the codes order the nine cells by (time, pad), so
// the largest key is the argmax of (adc, time, pad) and its low bits are the
// up code.  An empty cell (adc 0) has a key below 16 and never beats a
// present cell; if nothing present is left (an ADC-0 sample alone), the
// sample keeps its own code.  Keys fit 14 bits, so the two cells of a 32-bit
// word are keyed and compared as a pair (packed 16-bit max).
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pk_max_u16(uint32_t x, uint32_t y) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u16x2, x),
                                                                __builtin_bit_cast(u16x2, y)));
}
// keys of the cells c-1 and c (lo) and c+1 (hi, upper half 0) of one tile
// row, with the codes of those cells in lo_code (c-1 low, c high) and hi_code
__device__ __forceinline__ void row_keys(const uint16_t* tile, int c, uint32_t lo_code,
                                         uint32_t hi_code, uint32_t& lo, uint32_t& hi) {
  const uint32_t* t32 = reinterpret_cast<const uint32_t*>(tile);
  const int w = (c - 1) >> 1;
  const uint32_t w0 = t32[w], w1 = t32[w + 1];
  const uint32_t sh = ((c - 1) & 1) * 16;
  lo = __builtin_amdgcn_alignbit(w1, w0, sh);  // cells c-1, c
  hi = w1 >> sh;                               // cell c+1 (and c+2 or nothing)
  lo = ((lo & 0x03FF03FFu) << 4) | lo_code;
  hi = ((hi & 0x3FFu) << 4) | hi_code;
}
__device__ __forceinline__ int up_code_of(const uint16_t* tile, int c, int qmin, int& a) {
  uint32_t ul, uh, ml, mh, dl, dh;
  row_keys(tile, c - CL_TP, 0x00010000u, 2u, ul, uh);
  row_keys(tile, c, 0x00050004u, 6u, ml, mh);
  row_keys(tile, c + CL_TP, 0x00090008u, 10u, dl, dh);
  a = (int)(ml >> 20);  // the cell's own key is its ADC * 16 + 5
  const uint32_t m2 = pk_max_u16(pk_max_u16(pk_max_u16(ul, ml), pk_max_u16(dl, uh)),
                                 pk_max_u16(mh, dh));
  const int best = (int)max(m2 & 0xFFFFu, m2 >> 16);
  const int code = best >= 16 ? (best & 15) : 5;
  return code | ((code == 5 && a >= qmin) ? 16 : 0);
}

// The peak test alone: the sample's key beats its 8 neighbours (earlier
// neighbours may tie on ADC, later ones may not) and its ADC reaches qmin.
__device__ __forceinline__ bool is_peak(const uint16_t* tile, int c, int qmin) {
  const Row3 u = row3(tile, c - CL_TP), m = row3(tile, c), d = row3(tile, c + CL_TP);
  const int a = m.m;
  const int e = max(max(u.l, u.m), max(u.r, m.l));
  const int l = max(max(m.r, d.l), max(d.m, d.r));
  return a >= qmin && e <= a && l < a;
}

__device__ __forceinline__ uint32_t lanes_below() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

template <int ROWS>
__device__ __forceinline__ void clear_tile(uint16_t* tile) {
  constexpr int TILE = ROWS * CL_TP;
  uint4* t4 = reinterpret_cast<uint4*>(tile);
  constexpr int N4 = TILE * 2 / 16;
  for (int i = threadIdx.x; i < N4; i += 64) t4[i] = make_uint4(0, 0, 0, 0);
  for (int i = N4 * 8 + threadIdx.x; i < TILE; i += 64) tile[i] = 0;
}

// Raw record of one cluster, written by the peak pass at the sample index of
// the window's first core sample plus the peak's rank in the window (a
// window has no more peaks than core samples, so windows never overlap):
//   m0: q (15 bits) | n (5 bits) << 15 | n_sat (5 bits) << 20 |
//       sum a(dp+2) (17 bits) << 25 | sum a dp^2 (17 bits) << 42
//   m1: sum a(dt+2) (17 bits) | sum a dt^2 (17 bits) << 32
//   m2: ppad | ptime << 8 | qmax << 32
// Every field stays below its width: at most 25 samples of ADC <= 1023 per
// peak.
struct ClusterRec {
  unsigned long long m0, m1, m2;
};

// Peak pass: one wave walks K windows of one (unit,row); per window it
// finds the up codes and peaks, accumulates each peak's moments in LDS
// (batches of CL_SLOTS peaks), writes one raw record per peak and the
// window's peak count.
// The peak passes run one wave per workgroup: the LDS operations of a wave
// complete in order, so ordering them needs only a compiler fence, not a
// workgroup barrier (which would also wait for every outstanding LDS access).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <int W>
struct PeaksLds {
  __attribute__((aligned(16))) uint16_t tile[(W + 2 * CL_HALO) * CL_TP];
  uint16_t pk_cell[CL_SLOTS + 1];
  unsigned long long acc0[CL_SLOTS + 1], acc1[CL_SLOTS + 1];
};

template <int W, int K, int PRE>
__device__ __forceinline__ void peaks_chunk(const ZsArgs& in, const uint32_t* __restrict__ zblk,
                                            uint32_t nblk, uint32_t nwin, uint32_t nchunk,
                                            uint32_t n_ur, uint32_t* __restrict__ win_cnt,
                                            ClusterRec* __restrict__ rec,
                                            int32_t* __restrict__ sample_label,
                                            const DevParams* __restrict__ P, uint32_t logical,
                                            PeaksLds<W>& L) {
  constexpr int ROWS = W + 2 * CL_HALO;
  uint16_t* tile = L.tile;
  uint16_t* pk_cell = L.pk_cell;
  unsigned long long* acc0 = L.acc0;
  unsigned long long* acc1 = L.acc1;
  const uint32_t ur = logical / nchunk, chunk = logical % nchunk;
  if (ur >= n_ur) return;
  const int np = uni(P->np[ur % NROW]), qmin = uni(P->qmax_min);
  const uint32_t* zb = zblk + (size_t)ur * (nblk + 1);
  uint32_t rs0 = uni(zb[0]), rs1 = uni(zb[nblk]);
  if (rs1 > in.n_samples) rs1 = in.n_samples;
  if (rs0 > rs1) rs0 = rs1;
  const int w0 = chunk * K;
  const int w1 = min((int)nwin, w0 + K);
  clear_tile<ROWS>(tile);
  WinRange R = window_range<W>(zb, nblk, w0, rs0, rs1);
  SampleRegs<PRE> cur, nxt;
  prefetch(in, R, cur);
  wave_sync();
  for (int w = w0; w < w1; ++w) {
    const int tile_t0 = w * W - CL_HALO;
    scatter<ROWS>(tile, in, R, cur, tile_t0, np, true);
    WinRange Rn = R;
    if (w + 1 < w1) {
      Rn = window_range<W>(zb, nblk, w + 1, rs0, rs1);
      prefetch(in, Rn, nxt);
    }
    wave_sync();
    // Up codes of the samples within 3 bins of the core, written in place;
    // core peaks are ranked in sample order and the first CL_SLOTS get slots.
    uint32_t total = 0;
    for (uint32_t s0 = R.s_lo; s0 < R.s_hi; s0 += 64) {
      const uint32_t s = s0 + threadIdx.x;
      int c = -1, lt = -1;
      if (s < R.s_hi) {
        const uint32_t tp = sample_tp(in, cur, (s0 - R.s_lo) >> 6, s);
        c = cell_of<ROWS>(tp, tile_t0, np);
        lt = (int)(tp >> 16) - tile_t0;
      }
      const bool live = c >= 0 && lt >= CL_HALO - 3 && lt < CL_HALO + W + 3;
      int a = 0;
      const int code = live ? up_code_of(tile, c, qmin, a) : 0;
      const bool pk = live && (code & 16) && lt >= CL_HALO && lt < CL_HALO + W;
      const uint64_t m = __ballot(pk);
      const uint32_t k = total + (uint32_t)__popcll(m & ((1ull << threadIdx.x) - 1ull));
      const bool pslot = pk && k < CL_SLOTS;
      // non-peak: its up code; peak: the flag and its slot (or none); the
      // cell's own lane is its only writer, so its ADC bits are a
      const int v = (code & 16) ? (a | CL_PEAK | (pslot ? slot_bits((int)k) : CL_NOSLOT))
                                : (a | (code << 10));
      if (live) tile[c] = (uint16_t)v;
      if (pslot) pk_cell[k] = (uint16_t)c;
      total += (uint32_t)__popcll(m);
    }
    ClusterRec* wrec = rec + R.c_lo;  // this window's records
    uint32_t done = 0;                // peaks handled in earlier batches
    uint32_t nb = min(total, (uint32_t)CL_SLOTS);
    while (nb > 0) {
      if (threadIdx.x < CL_SLOTS) {
        acc0[threadIdx.x] = 0;
        acc1[threadIdx.x] = 0;
      }
      wave_sync();
      // every sample within two bins of the core adds itself to its peak;
      // the offset to the peak is the sum of the two chase steps
      for (uint32_t s0 = R.s_lo; s0 < R.s_hi; s0 += 64) {
        const uint32_t s = s0 + threadIdx.x;
        if (s >= R.s_hi) continue;
        const uint32_t tp = sample_tp(in, cur, (s0 - R.s_lo) >> 6, s);
        const int x = cell_of<ROWS>(tp, tile_t0, np);
        const int lt = (int)(tp >> 16) - tile_t0;
        if (x < 0 || lt < CL_HALO - 2 || lt >= CL_HALO + W + 2) continue;
        const int tx = tile[x];
        const int cx = chase_code(tx);
        const int y = x + code_offset(cx);
        const int ty = tile[y];
        const int cy = chase_code(ty);
        const int tz = tile[y + code_offset(cy)];
        const int slot = slot_of(tz);
        if (!(tz & CL_PEAK) || slot == CL_SLOTS) continue;
        const uint32_t a = tx & 0x3FF;
        const uint32_t dt2 = 4 - (cx >> 2) - (cy >> 2);  // dt + 2, dt = sample - peak
        const uint32_t dp2 = 4 - (cx & 3) - (cy & 3);
        const int dt = (int)dt2 - 2, dp = (int)dp2 - 2;
        const uint32_t dtt = (uint32_t)__mul24(dt, dt), dpp = (uint32_t)__mul24(dp, dp);
        const uint32_t ap = __umul24(a, dp2), at = __umul24(a, dt2);
        // the packed fields assembled as two 32-bit halves
        const uint32_t lo0 = a | (1u << 15) | ((uint32_t)(a >= 1023) << 20) | (ap << 25);
        // a * dp^2 as one 24-bit multiply (left to itself the compiler
        // reassociates it with the shift into a quarter-rate 32-bit multiply)
        uint32_t adpp;
        asm("v_mul_u32_u24 %0, %1, %2" : "=v"(adpp) : "v"(a), "v"(dpp));
        const uint32_t hi0 = (ap >> 7) | (adpp << 10);
        const uint64_t v0 = ((uint64_t)hi0 << 32) | lo0;
        const uint64_t v1 = ((uint64_t)__umul24(a, dtt) << 32) | at;
        atomicAdd(&acc0[slot], (unsigned long long)v0);
        atomicAdd(&acc1[slot], (unsigned long long)v1);
      }
      wave_sync();
      if (threadIdx.x < nb) {
        // the batch's records; the peak leaves the batch
        const int c = pk_cell[threadIdx.x];
        const int cell = tile[c];
        const int lt = c / CL_TP;
        const uint64_t meta = (uint64_t)(uint32_t)(c - lt * CL_TP - 2) |
                              ((uint64_t)(uint32_t)(lt + tile_t0) << 8) |
                              ((uint64_t)(cell & 0x3FF) << 32);
        ClusterRec rr;
        rr.m0 = acc0[threadIdx.x];
        rr.m1 = acc1[threadIdx.x];
        rr.m2 = meta;
        wrec[done + threadIdx.x] = rr;
        tile[c] = (uint16_t)((cell & 0x43FF) | CL_NOSLOT);
      }
      done += nb;
      nb = min(total - done, (uint32_t)CL_SLOTS);
      if (nb == 0) break;
      wave_sync();
      // slots for the next batch of core peaks, in sample order
      uint32_t rank = 0;
      for (uint32_t s0 = R.s_lo; s0 < R.c_hi; s0 += 64) {
        const uint32_t s = s0 + threadIdx.x;
        int c = -1;
        if (s >= R.c_lo && s < R.c_hi)
          c = cell_of<ROWS>(sample_tp(in, cur, (s0 - R.s_lo) >> 6, s), tile_t0, np);
        const bool pk = c >= 0 && (tile[c] & CL_PEAK) != 0;
        const uint64_t m = __ballot(pk);
        const uint32_t k = rank + (uint32_t)__popcll(m & ((1ull << threadIdx.x) - 1ull));
        if (pk && k >= done && k < done + nb) {
          tile[c] = (uint16_t)((tile[c] & 0x43FF) | slot_bits(k - done));
          pk_cell[k - done] = (uint16_t)c;
        }
        rank += (uint32_t)__popcll(m);
      }
    }
    if (threadIdx.x == 0) win_cnt[(size_t)ur * nwin + w] = total;
    if (sample_label) {
      wave_sync();
      for (uint32_t s = R.c_lo + threadIdx.x; s < R.c_hi; s += 64) {
        const uint32_t tp = ((uint32_t)in.time[s] << 16) | in.pad[s];
        const int lt = (int)(tp >> 16) - tile_t0;
        const int x = cell_of<ROWS>(tp, tile_t0, np);
        int32_t lab = -1;
        if (x >= 0 && lt >= CL_HALO && lt < CL_HALO + W) {
          const int y = x + code_offset(chase_code(tile[x]));
          const int z = y + code_offset(chase_code(tile[y]));
          if (tile[z] & CL_PEAK) lab = ((z / CL_TP + tile_t0) << 8) | (z % CL_TP - 2);
        }
        sample_label[s] = lab;
      }
    }
    wave_sync();
    scatter<ROWS>(tile, in, R, cur, tile_t0, np, false);
    wave_sync();
    R = Rn;
    cur = nxt;
  }
}

template <int W, int K, int PRE>
__global__ __launch_bounds__(64) void k_cluster_peaks(ZsArgs in, const uint32_t* __restrict__ zblk,
                                                      uint32_t nblk, uint32_t nwin,
                                                      uint32_t nchunk, uint32_t n_ur,
                                                      uint32_t* __restrict__ win_cnt,
                                                      ClusterRec* __restrict__ rec,
                                                      int32_t* __restrict__ sample_label,
                                                      const DevParams* __restrict__ P,
                                                      const DevStatus* st) {
  __shared__ PeaksLds<W> L;
  if (failed(st)) return;
  peaks_chunk<W, K, PRE>(in, zblk, nblk, nwin, nchunk, n_ur, win_cnt, rec, sample_label, P,
                         xcd_remap(blockIdx.x, gridDim.x), L);
}

// The windowed pass over the chunks that the streaming pass handed back:
// list[0] is their count, list[1 + i] the chunks (any order).
template <int W, int K, int PRE>
__global__ __launch_bounds__(64) void k_cluster_peaks_list(ZsArgs in,
                                                           const uint32_t* __restrict__ zblk,
                                                           uint32_t nblk, uint32_t nwin,
                                                           uint32_t nchunk, uint32_t n_ur,
                                                           uint32_t* __restrict__ win_cnt,
                                                           ClusterRec* __restrict__ rec,
                                                           int32_t* __restrict__ sample_label,
                                                           const uint32_t* __restrict__ list,
                                                           const DevParams* __restrict__ P,
                                                           const DevStatus* st) {
  __shared__ PeaksLds<W> L;
  if (failed(st)) return;
  const uint32_t n = uni(list[0]);
  for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
    peaks_chunk<W, K, PRE>(in, zblk, nblk, nwin, nchunk, n_ur, win_cnt, rec, sample_label, P,
                           uni(list[1 + i]), L);
    wave_sync();
  }
}

// ------------------------------------------------------------ shared-tile pass
// The per-window pass is bound by the latency of its dependent LDS and memory
// steps rather than by issue: its time follows the number of windows in
// flight per compute unit, which the tile's LDS limits (one tile per wave).
// Here NW waves (the library launches two) share the tile of one window of W
// bins: each wave takes every NW-th 64-sample step of the window, so a
// compute unit holds NW times as many waves for the same tile, and longer
// windows recompute less halo per core sample.  The phases of a window are
// ordered by workgroup barriers (four per window when one moment batch
// suffices), whose waits take back most of what the extra waves gain.  The
// results are those of the per-window pass.
//
// Tile cell: ADC in bits 0-9; v = bits 10-15 is a non-peak's up code
// (v <= 10) or, for a peak, MW_V0 + its moment slot (v <= 61); v = MW_PEND
// marks a core peak still waiting for a slot, v = MW_NONE a peak with no
// record to write here (outside the core, or already written).  Each wave
// owns MW_SW(NW) slots and hands them out in its own sample order, so no slot
// counter is shared.
#define MW_V0 11
#define MW_PEND 62
#define MW_NONE 63
#define MW_SW(NW) (51 / (NW))  // slots per wave (NW * MW_SW <= 51)
// 64-sample steps of a window (core and halo) that a valid input can fill:
// at most one sample per cell, at most 138 pads
#define MW_GROUPS(W) ((((W) + 2 * CL_HALO) * (CL_TP - 4) + 63) / 64)

__device__ __forceinline__ int mw_code(int cell) {
  const int v = cell >> 10;
  return v <= 10 ? v : 5;
}
__device__ __forceinline__ int mw_cell(int a, int v) { return a | (v << 10); }

template <int W, int NW>
struct PeaksLdsMw {
  __attribute__((aligned(16))) uint16_t tile[(W + 2 * CL_TH) * CL_TP];
  unsigned long long acc0[NW * MW_SW(NW)], acc1[NW * MW_SW(NW)];
  uint32_t grp[MW_GROUPS(W) + 1];  // core peaks per 64-sample step (ranks sum them)
  uint16_t pk_cell[NW * MW_SW(NW)];
  uint16_t pk_gi[NW * MW_SW(NW)];  // step << 6 | rank within the step
  uint16_t pk_a[NW * MW_SW(NW)];   // the peak's ADC
  uint32_t wcnt[NW];               // slots used by each wave in the batch
};

template <int PRE, int NT>
__device__ __forceinline__ void prefetch_mw(const ZsArgs& in, const WinRange& R,
                                            SampleRegs<PRE>& S) {
#pragma unroll
  for (int j = 0; j < PRE; ++j) {
    const uint32_t s = R.s_lo + threadIdx.x + j * NT;
    if (s < R.s_hi) {
      S.tp[j] = ((uint32_t)in.time[s] << 16) | in.pad[s];
      S.a[j] = in.adc[s];
    } else {
      S.tp[j] = 0xFFFFFFFFu;
      S.a[j] = 0;
    }
  }
}

template <int ROWS, int PRE, int NT>
__device__ __forceinline__ void scatter_mw(uint16_t* tile, const ZsArgs& in, const WinRange& R,
                                           const SampleRegs<PRE>& S, int tile_t0, int np,
                                           bool place) {
#pragma unroll
  for (int j = 0; j < PRE; ++j) {
    const int c = cell_of<ROWS>(S.tp[j], tile_t0, np);
    if (c >= 0) tile[c] = place ? (uint16_t)(S.a[j] & 0x3FF) : 0;
  }
  for (uint32_t s = R.s_lo + PRE * NT + threadIdx.x; s < R.s_hi; s += NT) {
    const uint32_t tp = ((uint32_t)in.time[s] << 16) | in.pad[s];
    const int c = cell_of<ROWS>(tp, tile_t0, np);
    if (c >= 0) tile[c] = place ? (uint16_t)(in.adc[s] & 0x3FF) : 0;
  }
}

template <int W, int K, int NW, int PRE>
__device__ __forceinline__ void peaks_chunk_mw(const ZsArgs& in, const uint32_t* __restrict__ zblk,
                                               uint32_t nblk, uint32_t nwin, uint32_t nchunk,
                                               uint32_t n_ur, uint32_t* __restrict__ win_cnt,
                                               ClusterRec* __restrict__ rec,
                                               int32_t* __restrict__ sample_label,
                                               const DevParams* __restrict__ P, DevStatus* st,
                                               uint32_t logical, PeaksLdsMw<W, NW>& L) {
  constexpr int ROWS = W + 2 * CL_TH, NT = 64 * NW, SW = MW_SW(NW);
  uint16_t* tile = L.tile;
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t below = (1ull << lane) - 1ull;
  const uint32_t ur = logical / nchunk, chunk = logical % nchunk;
  if (ur >= n_ur) return;
  const int np = uni(P->np[ur % NROW]), qmin = uni(P->qmax_min);
  const uint32_t* zb = zblk + (size_t)ur * (nblk + 1);
  uint32_t rs0 = uni(zb[0]), rs1 = uni(zb[nblk]);
  if (rs1 > in.n_samples) rs1 = in.n_samples;
  if (rs0 > rs1) rs0 = rs1;
  const int w0 = chunk * K;
  const int w1 = min((int)nwin, w0 + K);
  for (int i = threadIdx.x; i < ROWS * CL_TP / 8; i += NT)
    reinterpret_cast<uint4*>(tile)[i] = make_uint4(0, 0, 0, 0);
  for (int i = ROWS * CL_TP / 8 * 8 + threadIdx.x; i < ROWS * CL_TP; i += NT) tile[i] = 0;
  if (threadIdx.x < NW * SW) {
    L.acc0[threadIdx.x] = 0;
    L.acc1[threadIdx.x] = 0;
  }
  WinRange R = window_range<W>(zb, nblk, w0, rs0, rs1);
  SampleRegs<PRE> cur, nxt;
  prefetch_mw<PRE, NT>(in, R, cur);
  __syncthreads();
  for (int w = w0; w < w1; ++w) {
    const int tile_t0 = w * W - CL_TH;
    scatter_mw<ROWS, PRE, NT>(tile, in, R, cur, tile_t0, np, true);
    WinRange Rn = R;
    if (w + 1 < w1) {
      Rn = window_range<W>(zb, nblk, w + 1, rs0, rs1);
      prefetch_mw<PRE, NT>(in, Rn, nxt);
    }
    __syncthreads();
    // more samples than cells: not a valid input (uniform over the workgroup)
    const bool fits = R.s_hi - R.s_lo <= (uint32_t)MW_GROUPS(W) * 64u;
    if (!fits && threadIdx.x == 0) latch(st, TPC_ERR_INPUT);
    uint32_t total = 0;
    if (fits) {
      // up codes of the samples within 2 bins of the core, in place; each
      // wave gives its core peaks its own slots in sample order
      uint32_t used = 0;
      uint32_t j = 0;
      for (uint32_t s0 = R.s_lo + wave * 64; s0 < R.s_hi; s0 += NT, ++j) {
        const uint32_t s = s0 + lane;
        int c = -1, lt = -1;
        if (s < R.s_hi) {
          const uint32_t tp = sample_tp(in, cur, j, s);
          c = cell_of<ROWS>(tp, tile_t0, np);
          lt = (int)(tp >> 16) - tile_t0;
        }
        const bool live = c >= 0 && lt >= CL_TH - 2 && lt < CL_TH + W + 2;
        int a = 0;
        const int code = live ? up_code_of(tile, c, qmin, a) : 0;
        const bool pk = live && (code & 16) && lt >= CL_TH && lt < CL_TH + W;
        const uint64_t m = __ballot(pk);
        const uint32_t idx = (uint32_t)__popcll(m & below);
        const uint32_t k = used + idx;
        const bool pslot = pk && k < (uint32_t)SW;
        const uint32_t slot = wave * SW + k;
        const int v = (code & 16) ? (pk ? (pslot ? MW_V0 + (int)slot : MW_PEND) : MW_NONE)
                                  : (code & 15);
        if (live) tile[c] = (uint16_t)mw_cell(a, v);
        const uint32_t g = (s0 - R.s_lo) >> 6;
        if (pslot) {
          L.pk_cell[slot] = (uint16_t)c;
          L.pk_a[slot] = (uint16_t)a;
          L.pk_gi[slot] = (uint16_t)((g << 6) | idx);
        }
        if (lane == 0) L.grp[g] = (uint32_t)__popcll(m);
        used += (uint32_t)__popcll(m);
      }
      if (lane == 0) L.wcnt[wave] = min(used, (uint32_t)SW);
      __syncthreads();
      const uint32_t ng = (R.s_hi - R.s_lo + 63) >> 6;
      for (uint32_t g = 0; g < ng; ++g) total += L.grp[g];
      ClusterRec* wrec = rec + R.c_lo;
      uint32_t nb = 0;
#pragma unroll
      for (int q = 0; q < NW; ++q) nb += L.wcnt[q];
      uint32_t done = 0;
      // the moment sums start at zero: cleared at the start and by each record
      while (nb > 0) {
        // every sample within two bins of the core adds itself to the core
        // peak that two uphill steps reach
        j = 0;
        for (uint32_t s0 = R.s_lo + wave * 64; s0 < R.s_hi; s0 += NT, ++j) {
          const uint32_t s = s0 + lane;
          if (s >= R.s_hi) continue;
          const uint32_t tp = sample_tp(in, cur, j, s);
          const int x = cell_of<ROWS>(tp, tile_t0, np);
          const int lt = (int)(tp >> 16) - tile_t0;
          if (x < 0 || lt < CL_TH - 2 || lt >= CL_TH + W + 2) continue;
          const int tx = tile[x];
          const int cx = mw_code(tx);
          const int ly = lt + (cx >> 2) - 1;
          if (ly < CL_TH - 1 || ly >= CL_TH + W + 1) continue;
          const int y = x + code_offset(cx);
          const int cy = mw_code(tile[y]);
          const int vz = tile[y + code_offset(cy)] >> 10;
          if (vz < MW_V0 || vz >= MW_V0 + NW * SW) continue;
          const int slot = vz - MW_V0;
          const uint32_t a = tx & 0x3FF;
          const uint32_t dt2 = 4 - (cx >> 2) - (cy >> 2);  // dt + 2, dt = sample - peak
          const uint32_t dp2 = 4 - (cx & 3) - (cy & 3);
          const int dt = (int)dt2 - 2, dp = (int)dp2 - 2;
          const uint32_t dtt = (uint32_t)__mul24(dt, dt), dpp = (uint32_t)__mul24(dp, dp);
          const uint32_t ap = __umul24(a, dp2), at = __umul24(a, dt2);
          const uint32_t lo0 = a | (1u << 15) | ((uint32_t)(a >= 1023) << 20) | (ap << 25);
          uint32_t adpp;
          asm("v_mul_u32_u24 %0, %1, %2" : "=v"(adpp) : "v"(a), "v"(dpp));
          const uint32_t hi0 = (ap >> 7) | (adpp << 10);
          const uint64_t v0 = ((uint64_t)hi0 << 32) | lo0;
          const uint64_t v1 = ((uint64_t)__umul24(a, dtt) << 32) | at;
          atomicAdd(&L.acc0[slot], (unsigned long long)v0);
          atomicAdd(&L.acc1[slot], (unsigned long long)v1);
        }
        __syncthreads();
        // the batch's records, at the peak's rank in the window; the tile
        // is read again only if another batch follows
        const bool more = done + nb < total;
        if (threadIdx.x < NW * SW && threadIdx.x % SW < L.wcnt[threadIdx.x / SW]) {
          const int c = L.pk_cell[threadIdx.x];
          const uint32_t gi = L.pk_gi[threadIdx.x];
          uint32_t rank = gi & 63;
          for (uint32_t g = 0; g < (gi >> 6); ++g) rank += L.grp[g];
          const int lt = c / CL_TP;
          const uint64_t meta = (uint64_t)(uint32_t)(c - lt * CL_TP - 2) |
                                ((uint64_t)(uint32_t)(lt + tile_t0) << 8) |
                                ((uint64_t)L.pk_a[threadIdx.x] << 32);
          ClusterRec rr;
          rr.m0 = L.acc0[threadIdx.x];
          rr.m1 = L.acc1[threadIdx.x];
          rr.m2 = meta;
          wrec[rank] = rr;
          L.acc0[threadIdx.x] = 0;
          L.acc1[threadIdx.x] = 0;
          if (more) tile[c] = (uint16_t)mw_cell(L.pk_a[threadIdx.x], MW_NONE);
        }
        done += nb;
        if (!more) break;
        __syncthreads();
        // slots for the core peaks still waiting, each wave in its sample order
        used = 0;
        j = 0;
        for (uint32_t s0 = R.s_lo + wave * 64; s0 < R.c_hi; s0 += NT, ++j) {
          const uint32_t s = s0 + lane;
          int c = -1;
          if (s >= R.c_lo && s < R.c_hi) c = cell_of<ROWS>(sample_tp(in, cur, j, s), tile_t0, np);
          const int cell = c >= 0 ? tile[c] : 0;
          const int v = cell >> 10;
          const bool pk = v >= MW_V0;  // a peak in the core
          const bool pend = v == MW_PEND;
          const uint64_t m = __ballot(pk), mp = __ballot(pend);
          const uint32_t k = used + (uint32_t)__popcll(mp & below);
          if (pend && k < (uint32_t)SW) {
            const uint32_t slot = wave * SW + k;
            tile[c] = (uint16_t)mw_cell(cell & 0x3FF, MW_V0 + (int)slot);
            L.pk_cell[slot] = (uint16_t)c;
            L.pk_a[slot] = (uint16_t)(cell & 0x3FF);
            L.pk_gi[slot] = (uint16_t)((((s0 - R.s_lo) >> 6) << 6) | (uint32_t)__popcll(m & below));
          }
          used += (uint32_t)__popcll(mp);
        }
        if (lane == 0) L.wcnt[wave] = min(used, (uint32_t)SW);
        __syncthreads();
        nb = 0;
#pragma unroll
        for (int q = 0; q < NW; ++q) nb += L.wcnt[q];
      }
    }
    if (threadIdx.x == 0) win_cnt[(size_t)ur * nwin + w] = total;
    if (sample_label && fits) {
      // the tile is final: the last batch wrote none of it
      for (uint32_t s = R.c_lo + threadIdx.x; s < R.c_hi; s += NT) {
        const uint32_t tp = ((uint32_t)in.time[s] << 16) | in.pad[s];
        const int lt = (int)(tp >> 16) - tile_t0;
        const int x = cell_of<ROWS>(tp, tile_t0, np);
        int32_t lab = -1;
        if (x >= 0 && lt >= CL_TH && lt < CL_TH + W) {
          const int y = x + code_offset(mw_code(tile[x]));
          const int z = y + code_offset(mw_code(tile[y]));
          if ((tile[z] >> 10) >= MW_V0) lab = ((z / CL_TP + tile_t0) << 8) | (z % CL_TP - 2);
        }
        sample_label[s] = lab;
      }
      __syncthreads();
    }
    // the clear writes only cells that no wave reads any more
    scatter_mw<ROWS, PRE, NT>(tile, in, R, cur, tile_t0, np, false);
    __syncthreads();
    R = Rn;
    cur = nxt;
  }
}

template <int W, int K, int NW, int PRE>
__global__ __launch_bounds__(64 * NW) void k_cluster_peaks_mw(ZsArgs in,
                                                             const uint32_t* __restrict__ zblk,
                                                             uint32_t nblk, uint32_t nwin,
                                                             uint32_t nchunk, uint32_t n_ur,
                                                             uint32_t* __restrict__ win_cnt,
                                                             ClusterRec* __restrict__ rec,
                                                             int32_t* __restrict__ sample_label,
                                                             const DevParams* __restrict__ P,
                                                             DevStatus* st) {
  __shared__ PeaksLdsMw<W, NW> L;
  if (failed(st)) return;
  peaks_chunk_mw<W, K, NW, PRE>(in, zblk, nblk, nwin, nchunk, n_ur, win_cnt, rec, sample_label, P,
                                st, xcd_remap(blockIdx.x, gridDim.x), L);
}

// ------------------------------------------------------------ streaming pass
// Same records, window counts and labels as the windowed pass, without its
// per-window halo work and partly filled 64-sample steps.  One wave walks the
// chunk's samples (time, pad order) through a ring tile of CS_RB time bins
// (time t in ring row t mod CS_RB) with four cursors, each taking up to 64
// samples per round:
//   place:  the ADC of samples in [T0-3, T1+3) into the ring;
//   code:   up code and peak flag of samples in [T0-2, T1+2), once every
//           sample up to t+1 is placed; core peaks get a moment slot and a
//           record index (window start + rank in the window);
//   gather: each sample in [T0-2, T1+2) adds itself to the core peak it
//           reaches in two uphill steps (and labels itself, for core
//           samples), once every code up to t+2 is written;
//   clear:  zeroes the cells of samples below the rows the gather still
//           reads, so the ring rows can take later times.
// The ring holds the times [R, R + CS_RB), R the lowest row still read: a
// time is placed, and a row read, only inside that range, so a row with no
// sample reads as empty rather than as the cells of a time CS_RB apart.
// A peak's record is written once the gather has passed its time + 2.  Slots
// are reused in rank order (CL_SLOTS live at most); a chunk that would need
// more, or that stops making progress (input not sorted), is appended to a
// list for the windowed pass.
#define CS_RB 32

struct SCur {
  uint32_t x;         // first sample not taken (uniform)
  uint32_t tp0, tp1;  // samples x + lane and x + 64 + lane: time << 16 | pad, or ~0u
};

__device__ __forceinline__ uint32_t cs_tp(const ZsArgs& in, uint32_t s, uint32_t s_hi) {
  return s < s_hi ? (((uint32_t)in.time[s] << 16) | in.pad[s]) : 0xFFFFFFFFu;
}

__device__ __forceinline__ void cs_init(SCur& c, const ZsArgs& in, uint32_t x, uint32_t s_hi) {
  c.x = x;
  c.tp0 = cs_tp(in, x + threadIdx.x, s_hi);
  c.tp1 = cs_tp(in, x + 64 + threadIdx.x, s_hi);
}

// the lane's value of lane (lane + n) of the pair (v0, v1), n in [1, 64]
__device__ __forceinline__ uint32_t cs_shift(uint32_t v0, uint32_t v1, uint32_t n) {
  const uint32_t src = threadIdx.x + n;
  const int addr = (int)((src & 63u) << 2);
  const uint32_t a = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)v0);
  const uint32_t b = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)v1);
  return src < 64 ? a : b;
}

// take n (uniform, 0..64) samples; the next 64 are loaded for the round after
__device__ __forceinline__ void cs_take(SCur& c, uint32_t n, const ZsArgs& in, uint32_t s_hi) {
  if (n == 0) return;
  c.tp0 = cs_shift(c.tp0, c.tp1, n);
  c.x += n;
  c.tp1 = cs_tp(in, c.x + 64 + threadIdx.x, s_hi);
}

// time of the first sample not taken, CS_END when none is left
#define CS_END (1 << 20)
__device__ __forceinline__ int cs_front(const SCur& c) {
  const uint32_t v = __builtin_amdgcn_readfirstlane(c.tp0);
  return v == 0xFFFFFFFFu ? CS_END : (int)(v >> 16);
}

// number of leading lanes (a prefix, as times are sorted) with ok set
__device__ __forceinline__ uint32_t cs_count(bool ok) {
  const uint64_t m = __ballot(ok);
  return m == ~0ull ? 64u : (uint32_t)__builtin_ctzll(~m);
}

__device__ __forceinline__ int cs_cell(int t, int p) {
  return (int)__umul24((uint32_t)t & (CS_RB - 1), CL_TP) + p + 2;
}

template <int W, int K>
__global__ __launch_bounds__(64) void k_cluster_stream(ZsArgs in, const uint32_t* __restrict__ zblk,
                                                       uint32_t nblk, uint32_t nwin,
                                                       uint32_t nchunk, uint32_t n_ur,
                                                       uint32_t* __restrict__ win_cnt,
                                                       ClusterRec* __restrict__ rec,
                                                       int32_t* __restrict__ sample_label,
                                                       uint32_t* __restrict__ list,
                                                       const DevParams* __restrict__ P,
                                                       const DevStatus* st) {
  static_assert(K <= 64, "one lane per window");
  __shared__ __attribute__((aligned(16))) uint16_t tile[CS_RB * CL_TP];
  __shared__ unsigned long long acc0[CL_SLOTS], acc1[CL_SLOTS], meta[CL_SLOTS];
  __shared__ uint32_t ridx[CL_SLOTS];
  __shared__ uint32_t clo[K], wfirst[K], wcnt[K];
  if (failed(st)) return;
  const uint32_t logical = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t ur = logical / nchunk, chunk = logical % nchunk;
  if (ur >= n_ur) return;
  const uint32_t lane = threadIdx.x;
  const int np = uni(P->np[ur % NROW]), qmin = uni(P->qmax_min);
  const uint32_t* zb = zblk + (size_t)ur * (nblk + 1);
  uint32_t rs0 = uni(zb[0]), rs1 = uni(zb[nblk]);
  if (rs1 > in.n_samples) rs1 = in.n_samples;
  if (rs0 > rs1) rs0 = rs1;
  constexpr int BW = W >> CL_BSHIFT;
  const int w0 = (int)(chunk * K);
  const int nw = min((int)nwin - w0, K);
  const int T0 = w0 * W, T1 = (w0 + nw) * W;
  uint32_t s_lo, s_hi;
  row_range(zb, nblk, w0 * BW - 1, (w0 + nw) * BW + 1, rs0, rs1, s_lo, s_hi);
  s_lo = uni(s_lo);
  s_hi = uni(s_hi);
  if ((int)lane < nw) {
    uint32_t a, b;
    row_range(zb, nblk, (w0 + (int)lane) * BW, (w0 + (int)lane + 1) * BW, rs0, rs1, a, b);
    clo[lane] = a;
    wfirst[lane] = 0xFFFFFFFFu;
    wcnt[lane] = 0;
  }
  {
    uint4* t4 = reinterpret_cast<uint4*>(tile);
    constexpr int N4 = CS_RB * CL_TP * 2 / 16;
    for (int i = lane; i < N4; i += 64) t4[i] = make_uint4(0, 0, 0, 0);
  }
  SCur cp, cq, cg, cc;  // place, code, gather, clear
  cs_init(cp, in, s_lo, s_hi);
  uint32_t a0 = cp.tp0 != 0xFFFFFFFFu ? in.adc[s_lo + lane] : 0u;
  uint32_t a1 = cp.tp1 != 0xFFFFFFFFu ? in.adc[s_lo + 64 + lane] : 0u;
  cq = cp;
  cg = cp;
  cc = cp;
  uint32_t nrank = 0, drank = 0;  // core peaks ranked / whose records are written
  bool handed_back = false;
  wave_sync();
  for (;;) {
    // the ring holds the times [R, R + CS_RB): R is the lowest row still read
    // (the gather reads two bins below its front, rows below an uncleared
    // sample keep their data), even where no sample falls in it
    const int R = min(cs_front(cc), cs_front(cg) - 2);
    // ---- place
    uint32_t n_p;
    {
      const int t = (int)(cp.tp0 >> 16), p = (int)(cp.tp0 & 0xFFFF);
      const bool ok = cp.tp0 != 0xFFFFFFFFu && t < R + CS_RB;
      n_p = cs_count(ok);
      if (lane < n_p && t >= T0 - 3 && t < T1 + 3 && p < np)
        tile[cs_cell(t, p)] = (uint16_t)(a0 & 0x3FF);
      if (n_p) {
        a0 = cs_shift(a0, a1, n_p);
        cs_take(cp, n_p, in, s_hi);
        a1 = cp.tp1 != 0xFFFFFFFFu ? in.adc[cp.x + 64 + lane] : 0u;
      }
    }
    // rows at or above R + CS_RB are not in the ring yet: a read there would
    // see an older time's cells
    const int Fp = min(cs_front(cp), R + CS_RB);
    wave_sync();
    // ---- code
    uint32_t n_q;
    {
      const int t = (int)(cq.tp0 >> 16), p = (int)(cq.tp0 & 0xFFFF);
      const bool ok = cq.tp0 != 0xFFFFFFFFu && t + 2 <= Fp;
      const bool live = ok && t >= T0 - 2 && t < T1 + 2 && p < np;
      int code = 0, a = 0, c = 0;
      if (live) {
        c = cs_cell(t, p);
        const int bu = (int)__umul24((uint32_t)(t - 1) & (CS_RB - 1), CL_TP);
        const int bm = (int)__umul24((uint32_t)t & (CS_RB - 1), CL_TP);
        const int bd = (int)__umul24((uint32_t)(t + 1) & (CS_RB - 1), CL_TP);
        const Row3 u = row3(tile, bu + p + 2), m = row3(tile, bm + p + 2),
                   d = row3(tile, bd + p + 2);
        a = m.m;
        int best = (a << 4) | 5;
        best = max(best, max(u.l << 4, (u.m << 4) | 1));
        best = max(best, max((u.r << 4) | 2, (m.l << 4) | 4));
        best = max(best, max((m.r << 4) | 6, (d.l << 4) | 8));
        best = max(best, max((d.m << 4) | 9, (d.r << 4) | 10));
        code = best >= 16 ? (best & 15) : 5;
        code |= (code == 5 && a >= qmin) ? 16 : 0;
      }
      const bool pk = live && (code & 16) && t >= T0 && t < T1;
      // a core peak needs a free slot: take the samples before the first
      // peak that would overflow the slots
      const uint64_t pm = __ballot(pk);
      const uint32_t below = (uint32_t)__popcll(pm & ((1ull << lane) - 1ull));
      const uint32_t room = CL_SLOTS - (nrank - drank);
      const uint64_t over = __ballot(pk && below >= room);
      n_q = cs_count(ok);
      if (over) n_q = min(n_q, (uint32_t)__builtin_ctzll(over));
      const bool take = lane < n_q;
      const uint32_t rank = nrank + below;
      const uint32_t slot = rank % CL_SLOTS;
      int wi = 0;
      if (take && pk) {
        wi = (t - T0) / W;
        atomicMin(&wfirst[wi], rank);
        acc0[slot] = 0;
        acc1[slot] = 0;
        meta[slot] = (uint64_t)(uint32_t)p | ((uint64_t)(uint32_t)t << 8) | ((uint64_t)(uint32_t)a << 32);
      }
      if (take && live)
        tile[c] = (uint16_t)((code & 16) ? (a | CL_PEAK | (pk ? slot_bits((int)slot) : CL_NOSLOT))
                                         : (a | ((code & 15) << 10)));
      wave_sync();
      if (take && pk) {
        const uint32_t r = rank - wfirst[wi];
        ridx[slot] = clo[wi] + r;
        atomicMax(&wcnt[wi], r + 1);
      }
      nrank += (uint32_t)__popcll(pm & (n_q >= 64 ? ~0ull : ((1ull << n_q) - 1ull)));
      cs_take(cq, n_q, in, s_hi);
    }
    const int Fq = min(cs_front(cq), R + CS_RB);
    wave_sync();
    // ---- gather
    uint32_t n_g;
    {
      const int t = (int)(cg.tp0 >> 16), p = (int)(cg.tp0 & 0xFFFF);
      const bool ok = cg.tp0 != 0xFFFFFFFFu && t + 3 <= Fq;
      n_g = cs_count(ok);
      int32_t lab = -1;
      if (lane < n_g && t >= T0 - 2 && t < T1 + 2 && p < np) {
        const int tx = tile[cs_cell(t, p)];
        const int cx = chase_code(tx);
        const int yt = t + (cx >> 2) - 1, yp = p + (cx & 3) - 1;
        if (yt >= T0 - 2 && yt < T1 + 2) {
          const int ty = tile[cs_cell(yt, yp)];
          const int cy = chase_code(ty);
          const int zt = yt + (cy >> 2) - 1, zp = yp + (cy & 3) - 1;
          const int tz = tile[cs_cell(zt, zp)];
          if (tz & CL_PEAK) lab = (zt << 8) | zp;
          const int slot = slot_of(tz);
          if ((tz & CL_PEAK) && slot != CL_SLOTS && zt >= T0 && zt < T1) {
            const uint32_t av = tx & 0x3FF;
            const uint32_t dt2 = 4 - (cx >> 2) - (cy >> 2);  // dt + 2, dt = sample - peak
            const uint32_t dp2 = 4 - (cx & 3) - (cy & 3);
            const int dt = (int)dt2 - 2, dp = (int)dp2 - 2;
            const uint32_t dtt = (uint32_t)__mul24(dt, dt), dpp = (uint32_t)__mul24(dp, dp);
            const uint32_t ap = __umul24(av, dp2), at = __umul24(av, dt2);
            const uint32_t lo0 = av | (1u << 15) | ((uint32_t)(av >= 1023) << 20) | (ap << 25);
            uint32_t adpp;
            asm("v_mul_u32_u24 %0, %1, %2" : "=v"(adpp) : "v"(av), "v"(dpp));
            const uint32_t hi0 = (ap >> 7) | (adpp << 10);
            const uint64_t v0 = ((uint64_t)hi0 << 32) | lo0;
            const uint64_t v1 = ((uint64_t)__umul24(av, dtt) << 32) | at;
            atomicAdd(&acc0[slot], (unsigned long long)v0);
            atomicAdd(&acc1[slot], (unsigned long long)v1);
          }
        }
      }
      if (sample_label && lane < n_g && t >= T0 && t < T1) sample_label[cg.x + lane] = lab;
      cs_take(cg, n_g, in, s_hi);
    }
    const int Fg = cs_front(cg);
    wave_sync();
    // ---- records of the peaks the gather has passed (ranks are in time order)
    uint32_t n_r;
    {
      const uint32_t r = drank + lane;
      bool ok = false;
      uint32_t slot = 0;
      if (r < nrank) {
        slot = r % CL_SLOTS;
        ok = (int)((meta[slot] >> 8) & 0xFFFF) + 3 <= Fg;
      }
      n_r = cs_count(ok);
      if (lane < n_r) {
        ClusterRec rr;
        rr.m0 = acc0[slot];
        rr.m1 = acc1[slot];
        rr.m2 = meta[slot];
        rec[ridx[slot]] = rr;
      }
      drank += n_r;
    }
    // ---- clear the cells of samples below the rows still read
    uint32_t n_c;
    {
      const int t = (int)(cc.tp0 >> 16), p = (int)(cc.tp0 & 0xFFFF);
      const bool ok = cc.tp0 != 0xFFFFFFFFu && t + 3 <= Fg;
      n_c = cs_count(ok);
      if (lane < n_c && t >= T0 - 3 && t < T1 + 3 && p < np) tile[cs_cell(t, p)] = 0;
      cs_take(cc, n_c, in, s_hi);
    }
    wave_sync();
    if (cg.x >= s_hi && drank == nrank) break;
    if (n_p + n_q + n_g + n_r + n_c == 0) {  // no progress: not sorted
      handed_back = true;
      break;
    }
  }
  if (handed_back) {
    if (lane == 0) list[1 + atomicAdd(&list[0], 1u)] = logical;
    return;
  }
  if ((int)lane < nw) win_cnt[(size_t)ur * nwin + w0 + lane] = wcnt[lane];
}

// Output pass: clusters from the raw records, one thread per cluster.  A
// workgroup takes 256 consecutive windows (of all units and rows, in
// canonical order): their scanned counts give each cluster its window and
// rank, the window's first core sample gives the record.
template <int W>
__global__ __launch_bounds__(256) void k_cluster_output(const uint32_t* __restrict__ win_off,
                                                     const uint32_t* __restrict__ n_clusters,
                                                     uint32_t nwin, uint32_t n_ur,
                                                     const uint32_t* __restrict__ zblk,
                                                     uint32_t nblk, uint32_t n_samples,
                                                     const ClusterRec* __restrict__ rec,
                                                     ClusterOut out, const DevParams* __restrict__ P,
                                                     const DevStatus* st) {
  __shared__ uint32_t off[257], clo[256];
  if (failed(st)) return;
  const uint32_t nw_all = n_ur * nwin;
  const uint32_t total = *n_clusters;
  for (uint32_t wb = blockIdx.x * 256u; wb < nw_all; wb += gridDim.x * 256u) {
    const uint32_t g = wb + threadIdx.x;
    if (g < nw_all) {
      off[threadIdx.x] = win_off[g];
      const uint32_t ur = g / nwin, w = g % nwin;
      const uint32_t* zb = zblk + (size_t)ur * (nblk + 1);
      uint32_t rs0 = zb[0], rs1 = zb[nblk];
      if (rs1 > n_samples) rs1 = n_samples;
      if (rs0 > rs1) rs0 = rs1;
      uint32_t a, b;
      row_range(zb, nblk, (int32_t)(w * (W >> CL_BSHIFT)), (int32_t)((w + 1) * (W >> CL_BSHIFT)),
                rs0, rs1, a, b);
      clo[threadIdx.x] = a;
    }
    if (threadIdx.x == 0) off[min(256u, nw_all - wb)] = wb + 256 < nw_all ? win_off[wb + 256] : total;
    __syncthreads();
    const uint32_t nt = min(256u, nw_all - wb);
    const uint32_t c0 = off[0], c1 = off[nt];
    for (uint32_t k = c0 + threadIdx.x; k < c1; k += 256) {
      // window of cluster k: last j with off[j] <= k
      uint32_t lo = 0, hi = nt;
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (off[mid] <= k) lo = mid;
        else hi = mid;
      }
      if (k >= out.capacity) continue;
      const uint32_t g = wb + lo;
      const ClusterRec rr = rec[clo[lo] + (k - off[lo])];
      const int np = P->np[(g / nwin) % NROW];
      const int64_t pfx = P->pfx[(g / nwin) % NROW];
      const uint64_t v0 = rr.m0, v1 = rr.m1, v2 = rr.m2;
      const int q = (int)(v0 & 0x7FFF);
      const int ns = (int)((v0 >> 15) & 31);
      const int sat = (int)((v0 >> 20) & 31);
      const int sp = (int)((v0 >> 25) & 0x1FFFF) - 2 * q;
      const int spp = (int)((v0 >> 42) & 0x1FFFF);
      const int st_ = (int)(v1 & 0x1FFFF) - 2 * q;
      const int stt = (int)((v1 >> 32) & 0x1FFFF);
      const int ppad = (int)(v2 & 0xFF);
      const int ptime = (int)((v2 >> 8) & 0xFFFF);
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
      out.qmax[k] = (uint16_t)(v2 >> 32);
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
    __syncthreads();
  }
}

// crow_start[ur] = first cluster of (unit,row), from the scanned window
// counts (nwin windows per unit-row).
__global__ void k_crow_start(const uint32_t* __restrict__ win_off, uint32_t nwin,
                             uint32_t n_ur, const uint32_t* __restrict__ n_clusters,
                             uint32_t capacity, uint32_t* __restrict__ crow, DevStatus* st) {
  // after a latched error the scan that wrote *n_clusters did not run
  if (failed(st)) return;
  const uint32_t n = *n_clusters;
  for (uint32_t ur = blockIdx.x * blockDim.x + threadIdx.x; ur <= n_ur;
       ur += gridDim.x * blockDim.x)
    crow[ur] = ur < n_ur ? win_off[(size_t)ur * nwin] : n;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->n_clusters = n;
    if (n > capacity) latch_capacity(st, OVF_CLUSTERS, n);
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
