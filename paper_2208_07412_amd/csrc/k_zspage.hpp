// Decoder of raw zero-suppressed pages into the sample arrays the clusterizer
// reads (pad, time, adc, per-(unit,row) offsets).
//
// Page format (8 KiB, TPC_ZS_PAGE_WORDS little-endian 32-bit words; every
// field is defined in include/tpc.h): a 4-word header (magic and version;
// unit and row; run count and sample count; zero), a table of runs (one
// word each: time bin, first pad, length - 1), then the runs' ADC values as
// one stream of 10-bit fields, sample k at bits [10k, 10k + 10).  A run is a
// set of consecutive pads of one time bin.
//
// Work: a device scan of the pages' sample counts gives each page its output
// offset; a workgroup per page in turn then loads the page into LDS, scans the
// run lengths, expands them into a per-sample run index and writes every
// sample at its final index (stores of consecutive samples are consecutive).
// Bound: HBM (each page is read once, 6 bytes written per sample).
#pragma once

#include "common.hpp"

#define ZSP_WORDS TPC_ZS_PAGE_WORDS
#define ZSP_HDR 4
#define ZSP_MAGIC 0x5A53u
#define ZSP_VERSION 1u
// most samples a page can hold: 4 header words + 1 run + 10-bit fields
#define ZSP_MAX_SAMPLES (((ZSP_WORDS - ZSP_HDR - 1) * 32) / 10)

struct ZsPageHdr {
  uint32_t ur;     // unit * 152 + row
  uint32_t nruns;
  uint32_t nsamp;
  bool ok;         // header well formed and the page's fields fit it
};

// Header of a page from its first four words.  A page whose header is
// malformed counts no samples.
__device__ __forceinline__ ZsPageHdr zsp_header_of(uint32_t w0, uint32_t w1, uint32_t w2,
                                                   uint32_t w3, uint32_t n_units) {
  ZsPageHdr h;
  const uint32_t unit = w1 & 0xFFFFu, row = (w1 >> 16) & 0xFFu;
  h.nruns = w2 & 0xFFFFu;
  h.nsamp = w2 >> 16;
  h.ur = unit * NROW + row;
  const uint32_t stream_words = (h.nsamp * 10u + 31u) >> 5;
  h.ok = (w0 == (ZSP_MAGIC | (ZSP_VERSION << 16))) && (w1 >> 24) == 0 && w3 == 0 &&
         unit < n_units && row < NROW && ZSP_HDR + h.nruns + stream_words <= ZSP_WORDS &&
         (h.nruns > 0) == (h.nsamp > 0);
  if (!h.ok) h.nsamp = 0;
  return h;
}
// Header of page p.
__device__ __forceinline__ ZsPageHdr zsp_header(const uint32_t* __restrict__ pages, uint32_t p,
                                                uint32_t n_units) {
  const uint32_t* pg = pages + (size_t)p * ZSP_WORDS;
  return zsp_header_of(pg[0], pg[1], pg[2], pg[3], n_units);
}

struct GetPageSamples {
  const uint32_t* pages;
  uint32_t n_units;
  __device__ uint32_t operator()(uint32_t p) const { return zsp_header(pages, p, n_units).nsamp; }
};
struct EmitPageOffset {
  uint32_t* off;
  __device__ void operator()(uint32_t p, uint32_t pre, uint32_t) const { off[p] = pre; }
};

// Samples of one page at their final indices; also checks every field that
// the writes depend on (always) and the order and ADC range (validate mode).
// The page (8 KiB: 8 words per thread) is loaded whole into LDS with one
// coalesced load per thread, and the next page's load is issued before the
// current one is decoded, so the run table and the bit stream are read from
// LDS and only one memory round trip per page is exposed.
#define ZSP_BLOCK 256
static_assert(ZSP_WORDS == ZSP_BLOCK * 8, "a page is 8 words per thread");
__global__ __launch_bounds__(ZSP_BLOCK) void k_zs_decode(const uint32_t* __restrict__ pages,
                                                         uint32_t n_pages, uint32_t n_units,
                                                         uint32_t n_time_bins,
                                                         const uint32_t* __restrict__ off,
                                                         uint32_t capacity,
                                                         uint16_t* __restrict__ pad,
                                                         uint16_t* __restrict__ time,
                                                         uint16_t* __restrict__ adc,
                                                         const DevParams* __restrict__ P,
                                                         DevStatus* st) {
  __shared__ __attribute__((aligned(16))) uint32_t pg[ZSP_WORDS];
  __shared__ uint16_t first[ZSP_WORDS];
  __shared__ uint16_t run_of[ZSP_MAX_SAMPLES];
  __shared__ uint32_t lds_scan[ZSP_BLOCK / 64 + 1];
  __shared__ int bad;
  if (failed(st)) return;
  const bool validate = P->validate != 0;
  const uint4* src = reinterpret_cast<const uint4*>(pages);
  uint32_t p = blockIdx.x;
  uint4 q0 = make_uint4(0, 0, 0, 0), q1 = q0;
  if (p < n_pages) {
    q0 = src[(size_t)p * (ZSP_WORDS / 4) + threadIdx.x * 2];
    q1 = src[(size_t)p * (ZSP_WORDS / 4) + threadIdx.x * 2 + 1];
  }
  for (; p < n_pages; p += gridDim.x) {
    __syncthreads();  // the previous page's LDS reads are done
    reinterpret_cast<uint4*>(pg)[threadIdx.x * 2] = q0;
    reinterpret_cast<uint4*>(pg)[threadIdx.x * 2 + 1] = q1;
    const uint32_t pn = p + gridDim.x;
    if (pn < n_pages) {  // the next page's words, in flight while this one is decoded
      q0 = src[(size_t)pn * (ZSP_WORDS / 4) + threadIdx.x * 2];
      q1 = src[(size_t)pn * (ZSP_WORDS / 4) + threadIdx.x * 2 + 1];
    }
    const uint32_t o = off[p];
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    const ZsPageHdr h = zsp_header_of(pg[0], pg[1], pg[2], pg[3], n_units);
    if (!h.ok) {  // uniform: every thread read the same header
      if (threadIdx.x == 0) latch(st, TPC_ERR_INPUT);
      continue;
    }
    if (h.nsamp == 0) continue;
    if ((uint64_t)o + h.nsamp > capacity) continue;  // overflow, latched by the row kernel
    const uint32_t* runs = pg + ZSP_HDR;
    const uint32_t* stream = runs + h.nruns;
    const int np = P->np[h.ur % NROW];
    // each thread's 8 consecutive run lengths
    const uint32_t r0 = threadIdx.x * 8;
    uint32_t len[8];
    uint32_t acc = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const uint32_t r = r0 + e;
      len[e] = r < h.nruns ? (runs[r] >> 24) + 1 : 0;
      acc += len[e];
    }
    uint32_t sum;
    uint32_t pre = block_excl_scan<uint32_t, ZSP_BLOCK>(acc, lds_scan, sum);  // has barriers
    if (sum != h.nsamp) {  // uniform
      if (threadIdx.x == 0) latch(st, TPC_ERR_INPUT);
      continue;
    }
    int my_bad = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const uint32_t r = r0 + e;
      if (r < h.nruns) {
        const uint32_t w = runs[r];
        const uint32_t t = w & 0xFFFFu, p0 = (w >> 16) & 0xFFu;
        if (t >= n_time_bins || p0 + len[e] > (uint32_t)np) my_bad = 1;
        if (validate && r > 0) {
          // (time, pad) strictly increasing, runs not overlapping
          const uint32_t v = runs[r - 1];
          const uint32_t tv = v & 0xFFFFu, pv = ((v >> 16) & 0xFFu) + (v >> 24) + 1;
          if (t < tv || (t == tv && p0 < pv)) my_bad = 1;
        }
        first[r] = (uint16_t)pre;
        for (uint32_t j = 0; j < len[e]; ++j) run_of[pre + j] = (uint16_t)r;
        pre += len[e];
      }
    }
    if (my_bad) bad = 1;
    __syncthreads();
    if (bad) {  // uniform after the barrier
      if (threadIdx.x == 0) latch(st, TPC_ERR_INPUT);
      continue;
    }
    for (uint32_t k = threadIdx.x; k < h.nsamp; k += ZSP_BLOCK) {
      const uint32_t r = run_of[k];
      const uint32_t w = runs[r];
      const uint32_t bit = k * 10u, wi = bit >> 5, sh = bit & 31u;
      uint32_t a = stream[wi] >> sh;
      if (sh > 22) a |= stream[wi + 1] << (32u - sh);
      a &= 0x3FFu;
      if (validate && a == 0) latch(st, TPC_ERR_INPUT);
      pad[o + k] = (uint16_t)(((w >> 16) & 0xFFu) + (k - first[r]));
      time[o + k] = (uint16_t)(w & 0xFFFFu);
      adc[o + k] = (uint16_t)a;
    }
    if (validate && threadIdx.x == 0 && p > 0) {
      // across pages of one (unit,row): the first run follows the last one
      const ZsPageHdr q = zsp_header(pages, p - 1, n_units);
      if (q.ok && q.ur == h.ur && q.nruns > 0) {
        const uint32_t v = pages[(size_t)(p - 1) * ZSP_WORDS + ZSP_HDR + q.nruns - 1];
        const uint32_t w = runs[0];
        const uint32_t tv = v & 0xFFFFu, pv = ((v >> 16) & 0xFFu) + (v >> 24) + 1;
        const uint32_t t = w & 0xFFFFu, p0 = (w >> 16) & 0xFFu;
        if (t < tv || (t == tv && p0 < pv)) latch(st, TPC_ERR_INPUT);
      }
    }
  }
}

// Row offsets and the sample count: page p sets row_start for the units-rows
// after its predecessor's up to its own; the last page closes the table.
// Pages must come in (unit,row) order; a step back is reported.
__global__ void k_zs_rows(const uint32_t* __restrict__ pages, uint32_t n_pages, uint32_t n_units,
                          const uint32_t* __restrict__ off, const uint32_t* total_dev,
                          uint32_t capacity, uint32_t* __restrict__ row_start,
                          uint32_t* __restrict__ n_samples, DevStatus* st) {
  if (failed(st)) return;
  const uint32_t n_ur = n_units * NROW;
  const uint32_t total = *total_dev;
  const uint32_t tc = total < capacity ? total : capacity;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p <= n_pages; p += stride) {
    // page p covers the units-rows (prev, cur]; p == n_pages closes the table
    int64_t prev = -1, cur = (int64_t)n_ur;
    uint32_t v = tc;
    if (p > 0) {
      const ZsPageHdr q = zsp_header(pages, p - 1, n_units);
      prev = q.ok ? (int64_t)q.ur : -1;
    }
    if (p < n_pages) {
      const ZsPageHdr h = zsp_header(pages, p, n_units);
      if (!h.ok) continue;  // reported by the decoder
      cur = h.ur;
      v = off[p] < tc ? off[p] : tc;
      if (cur < prev) latch(st, TPC_ERR_INPUT);
    }
    for (int64_t u = prev + 1; u <= cur; ++u) row_start[u] = v;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *n_samples = total;
    if (total > capacity) latch(st, TPC_ERR_CAPACITY, total);
  }
}
