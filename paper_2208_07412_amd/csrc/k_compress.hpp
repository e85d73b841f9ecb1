// Track-model cluster compression (encoder and decoder) and the track-cluster
// residual histograms.
//
// Format (stated field by field in include/tpc.h): a header, a directory of
// bit offsets (one per track record, one per (unit,row) block of clusters on
// no track) and an LSB-first bit stream of Exp-Golomb codes.  Positions are
// quantised to 2^-7 cm; a cluster on a track is coded as its residual to an
// integer helix evaluated row by row from the track's fitted parameters, so
// every value in the stream is integer arithmetic and decoding gives the
// quantised clusters whatever the model predicts.
//
// Encoder: one wave per track computes its record's length (and the residual
// histograms), its hits 64 at a time on a table of the helix at every row;
// one wave per (unit,row) the lengths of its clusters on no track; two device
// scans turn the lengths into the directory; a finishing kernel writes the
// header and checks the capacity; the payload is cleared and written by the
// same waves, each lane accumulating its codes' bits and storing whole words
// (atomic OR because a code's first and last word may be shared with a
// neighbour).  Decoder: the record sizes come
// from the directory and the fixed-width hit counts, a scan gives the output
// offsets, and one lane per record decodes it.
#pragma once

#include "common.hpp"

#define CM_MAGIC 0x54434D31u
#define CM_HDR 8
#define CM_VERSION 2u
#define CM_CHUNK 64  // clusters on no track per independently decodable chunk of a row
#define CM_STAGE_WORDS 3072  // LDS words per wave for staging a record
#define CM_QSHIFT 9  // positions quantised to 2^(9-16) cm

// ---------------------------------------------------------------- arithmetic
__device__ __forceinline__ int64_t cm_q(int64_t v) { return (v + 256) >> CM_QSHIFT; }

// a / 2^k rounded to the nearest integer, halves up (arithmetic shift = floor)
__device__ __forceinline__ int64_t cm_rshift(int64_t a, int k) {
  return (a + ((int64_t)1 << (k - 1))) >> k;
}
// a / d rounded to the nearest integer, halves up: floor((2a + d) / 2d).  In
// the helix step 2^25 < d <= 2^31 and |a| < 2^56, so the quotient is below
// 2^31 and the double quotient (two roundings, relative error <= 2^-52) is
// within 2^-21 of it: its floor is off by at most one, which the exact
// remainder repairs.  (A 64-bit integer division is a long software sequence
// on the GPU.)
__device__ __forceinline__ int64_t cm_rdiv(int64_t a, int64_t d) {
  const int64_t n = 2 * a + d, m = 2 * d;
  int64_t q = (int64_t)floor((double)n / (double)m);
  const int64_t r = n - q * m;
  if (r < 0) --q;
  else if (r >= m) ++q;
  return q;
}
// floor(sqrt(n)), n >= 0: the double square root, then exact corrections
// (0 for n <= 0, which only a malformed record reaches)
__device__ __forceinline__ int64_t cm_isqrt(int64_t n) {
  if (n <= 0) return 0;
  int64_t r = (int64_t)sqrt((double)n);
  while (r > 0 && r * r > n) --r;
  while ((r + 1) * (r + 1) <= n) ++r;
  return r;
}
__device__ __forceinline__ uint64_t cm_zig(int64_t v) {
  return v >= 0 ? (uint64_t)v << 1 : ((uint64_t)(-v) << 1) - 1;
}
__device__ __forceinline__ int64_t cm_unzig(uint64_t u) {
  return (u & 1) ? -(int64_t)((u + 1) >> 1) : (int64_t)(u >> 1);
}
// length of the order-k Exp-Golomb code of v
__device__ __forceinline__ uint32_t cm_eg_len(uint64_t v, int k) {
  const uint64_t q = (v >> k) + 1;
  const uint32_t n = 63 - __builtin_clzll(q);
  return 2 * n + 1 + k;
}

// Integer helix of one track (y, z in 2^-16 cm; sin phi, tan lambda in 2^-30;
// C in 2^-46 per cm), stepped outward one row at a time.  Sc is
// floor(sqrt(2^60 - S^2)) of the current S, kept so that a step computes one
// such root for its new S instead of two.
struct CmModel {
  int64_t Y, Z, S, T, C, Sc;
  int row;
  bool frozen;
};

struct CmParams {  // the track's integers as stored in its record
  int64_t Y, Z, S, T, K;
};

// From the float32 parameters: each scaled by a power of two (exact) and
// rounded to the nearest integer, ties to even.
__device__ __forceinline__ CmParams cm_params(const float* p, int32_t z_anchor) {
  CmParams m;
  const int64_t lim = ((int64_t)1 << 30) - 1;
  int64_t S = (int64_t)rintf(p[2] * 1073741824.0f);
  int64_t T = (int64_t)rintf(p[3] * 1073741824.0f);
  int64_t K = (int64_t)rintf(p[4] * 65536.0f);
  S = S > lim ? lim : (S < -lim ? -lim : S);
  T = T > 4 * lim ? 4 * lim : (T < -4 * lim ? -4 * lim : T);
  K = K > 20 * 65536 ? 20 * 65536 : (K < -20 * 65536 ? -20 * 65536 : K);
  m.Y = (int64_t)rintf(p[0] * 65536.0f);
  m.Z = (int64_t)rintf(p[1] * 65536.0f) + z_anchor;
  m.S = S;
  m.T = T;
  m.K = K;
  return m;
}

__device__ __forceinline__ CmModel cm_model(const CmParams& q, int64_t b30, int row) {
  return CmModel{q.Y, q.Z, q.S, q.T, -b30 * q.K, cm_isqrt(((int64_t)1 << 60) - q.S * q.S), row,
                 false};
}

__device__ __forceinline__ void cm_step(CmModel& m, const int32_t* xfx) {
  const int a = m.row;
  m.row = a + 1;
  if (m.frozen || a + 1 >= NROW) return;
  const int64_t D = (int64_t)xfx[a + 1] - xfx[a];
  const int64_t S1 = m.S + cm_rshift(m.C * D, 32);
  const int64_t smax = ((int64_t)1 << 30) - ((int64_t)1 << 20);
  if (S1 >= smax || S1 <= -smax) {
    m.frozen = true;
    return;
  }
  const int64_t one = (int64_t)1 << 60;
  const int64_t c1 = cm_isqrt(one - S1 * S1);
  const int64_t F = cm_rdiv((m.S + S1) * ((int64_t)1 << 24), m.Sc + c1);
  m.Y += cm_rshift(D * F, 24);
  const int64_t L = cm_rshift(D * cm_isqrt(((int64_t)1 << 48) + F * F), 24);
  m.Z += cm_rshift(m.T * L, 30);
  m.S = S1;
  m.Sc = c1;
}

// (unit,row) of cluster c: the last entry of crow[0..n_ur) not above c
__device__ __forceinline__ uint32_t cm_find_ur(const uint32_t* crow, uint32_t n_ur, uint32_t c) {
  uint32_t lo = 0, hi = n_ur;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (crow[mid] <= c) lo = mid;
    else hi = mid;
  }
  return lo;
}

// ------------------------------------------------------------- bit writing
// One lane's sequential writer over a contiguous bit range: completed words
// are OR-ed into the (cleared) stream, the last partial word at the end.
struct CmWriter {
  uint32_t* w;
  uint64_t limit;  // payload words (no store beyond them, whatever the lengths)
  uint64_t pos;
  uint64_t acc;   // pending bits, the lowest at stream position (pos & ~31)
  uint32_t nacc;  // pending bit count = pos & 31 plus what was added
  __device__ void init(uint32_t* words, uint64_t n_words, uint64_t bitpos) {
    w = words;
    limit = n_words;
    pos = bitpos;
    acc = 0;
    nacc = (uint32_t)(bitpos & 31);
  }
  __device__ void store(uint64_t word, uint32_t v) {
    if (word < limit && v) atomicOr(&w[word], v);
  }
  __device__ void put(uint64_t v, uint32_t n) {  // n <= 32
    if (n == 0) return;
    v &= (n == 64) ? ~0ull : ((1ull << n) - 1);
    acc |= v << nacc;
    nacc += n;
    pos += n;
    if (nacc >= 32) {
      store((pos - nacc) >> 5, (uint32_t)acc);
      acc >>= 32;
      nacc -= 32;
    }
  }
  __device__ void eg(uint64_t v, int k) {
    const uint64_t q = (v >> k) + 1;
    const uint32_t n = 63 - __builtin_clzll(q);
    // n zeros, a one, the n low bits of q, the k low bits of v
    for (uint32_t z = n; z > 0;) {
      const uint32_t m = z > 32 ? 32 : z;
      put(0, m);
      z -= m;
    }
    put(1, 1);
    put(q, n);
    put(v, k);
  }
  __device__ void flush() {
    if (nacc) store((pos - nacc) >> 5, (uint32_t)acc);
    nacc = 0;
    acc = 0;
  }
};

// ------------------------------------------------------------- bit reading
// Sequential reader of a bit range; w points at payload word woff (a staged
// copy in LDS, or the payload itself with woff = 0).
// LSB-first reader over payload words w (w[0] is payload word woff) with a
// 64-bit bit buffer: one word read per 32 bits consumed.  Bits at or past
// `end` read as zero; a read that would pass `end` (or a zero prefix longer
// than 31) marks the reader bad and moves it to `end`.  P is the word
// pointer: global, or LDS for a staged record (an LDS pointer keeps the
// reads off the counter that the decoder's global stores also raise, so a
// read does not wait for the stores before it).
typedef const __attribute__((address_space(3))) uint32_t lds_u32;
template <typename P>
struct CmReaderT {
  P w;
  uint64_t pos, end;  // next bit, end of the readable bits (payload bits)
  bool bad;
  uint64_t woff;
  uint64_t buf;    // bits from pos on; nbuf of them loaded, zeros above
  uint32_t nbuf;
  uint64_t wnext;  // payload index of the next word to load
  __device__ CmReaderT(P w_, uint64_t pos_, uint64_t end_, bool bad_, uint64_t woff_)
      : w(w_), pos(0), end(end_), bad(bad_), woff(woff_), buf(0), nbuf(0), wnext(0) {
    seek(pos_);
  }
  __device__ void seek(uint64_t p) {
    pos = p;
    buf = 0;
    nbuf = 0;
    wnext = p >> 5;
    if (p < end) {
      buf = (uint64_t)(w[wnext - woff] >> (uint32_t)(p & 31));
      nbuf = 32 - (uint32_t)(p & 31);
      ++wnext;
    }
  }
  // at least 32 loaded bits, or every word up to the one holding end - 1
  __device__ void fill() {
    if (nbuf < 32 && (wnext << 5) < end) {
      buf |= (uint64_t)w[wnext - woff] << nbuf;
      nbuf += 32;
      ++wnext;
    }
  }
  __device__ void skip(uint32_t n) {
    buf >>= n;
    nbuf -= n;
    pos += n;
  }
  __device__ void fail() {
    bad = true;
    pos = end;
    buf = 0;
    nbuf = 0;
  }
  __device__ uint64_t get(uint32_t n) {  // n <= 32
    if (n == 0) return 0;
    if (pos + n > end) {
      fail();
      return 0;
    }
    fill();
    const uint64_t v = buf & ((1ull << n) - 1);
    skip(n);
    return v;
  }
  // up to 32 bits from pos on without advancing (bits past the end read 0)
  __device__ uint32_t peek32() {
    if (pos >= end) return 0;
    fill();
    uint32_t v = (uint32_t)buf;
    const uint64_t avail = end - pos;
    if (avail < 32) v &= (1u << (uint32_t)avail) - 1u;
    return v;
  }
  __device__ uint64_t eg(int k) {
    // the zero prefix: the trailing zeros of the next 32 bits (LSB first)
    const uint32_t v = peek32();
    if (v == 0) {  // no one bit among the next 32: malformed
      fail();
      return 0;
    }
    const uint32_t n = (uint32_t)__builtin_ctz(v);
    skip(n + 1);
    const uint64_t q = (1ull << n) | get(n);
    return ((q - 1) << k) | get(k);
  }
};
typedef CmReaderT<const uint32_t*> CmReader;

// -------------------------------------------------------------- cluster view
struct CmClusters {
  const uint32_t* crow;
  const int32_t *y, *z;
  const uint16_t *qtot, *qmax;
  const uint8_t* flags;
  const uint32_t* n_dev;
  uint32_t cap;
  uint32_t n_ur;
};

struct CmTracks {
  const float* par;
  const uint8_t* row;
  const int32_t* z_anchor;
  const uint32_t* hit_start;
  const uint32_t* hits;
  const int32_t* cluster_track;
  const uint32_t* n_dev;
  uint32_t cap, hit_cap;
};

__device__ __forceinline__ uint32_t cm_cluster_len(uint16_t qt, uint16_t qm) {
  return cm_eg_len(qt, 6) + cm_eg_len(qm, 5) + 2;
}
__device__ __forceinline__ void cm_cluster_put(CmWriter& b, uint16_t qt, uint16_t qm, uint8_t f) {
  b.eg(qt, 6);
  b.eg(qm, 5);
  b.put(f & 3u, 2);
}

// (unit,row) of cluster c found by a whole wave (every lane gets it): the
// last entry of crow[0..n_ur) not above c, as cm_find_ur; each round probes
// 64 evenly spaced entries, so 5,472 rows take three dependent loads.
__device__ __forceinline__ uint32_t cm_find_ur_wave(const uint32_t* crow, uint32_t n_ur,
                                                    uint32_t c) {
  const uint32_t lane = threadIdx.x & 63;
  uint32_t lo = 0, hi = n_ur;
  while (hi - lo > 1) {  // uniform
    const uint32_t step = (hi - lo + 63) / 64;
    const uint32_t p = lo + lane * step;
    // the probes not above c are a prefix of the lanes (crow does not decrease)
    const uint64_t b = __ballot(p < hi && crow[p] <= c);
    lo += (b ? 63u - (uint32_t)__builtin_clzll(b) : 0u) * step;
    hi = min(hi, lo + step);
  }
  return lo;
}

__device__ __forceinline__ uint32_t cm_wave_incl_max(uint32_t v) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t o = __shfl_up(v, d, 64);
    if ((int)(threadIdx.x & 63) >= d) v = max(v, o);
  }
  return v;
}

// The helix m at every row from m.row (< NROW) to the last, one wave: q(y)
// and q(z) at row r in ty[r] and tz[r].  Along a track C is constant, so the
// S after each step is S0 plus a prefix sum of per-step increments, and a
// step's changes of y and z depend only on the S before and after it: wave
// prefix sums give the same integers as cm_step row after row.  The first
// step whose S leaves the range freezes that step and all after it.  Ends
// with the table visible to the whole wave.
__device__ void cm_helix_rows(const CmModel& m, const int32_t* xs, int64_t* ty, int64_t* tz) {
  const uint32_t lane = threadIdx.x & 63;
  const int64_t one = (int64_t)1 << 60;
  const int64_t smax = ((int64_t)1 << 30) - ((int64_t)1 << 20);
  int64_t S = m.S, Sc = m.Sc, Y = m.Y, Z = m.Z;
  bool frozen = false;
  if (lane == 0) {
    ty[m.row] = cm_q(Y);
    tz[m.row] = cm_q(Z);
  }
  for (int base = m.row; base + 1 < NROW; base += 64) {  // uniform
    const int a = base + (int)lane;  // this lane's step: row a to row a + 1
    const bool valid = a + 1 < NROW;
    const int64_t D = valid ? (int64_t)xs[a + 1] - xs[a] : 0;
    const int64_t inc = valid ? cm_rshift(m.C * D, 32) : 0;
    const int64_t S1 = S + (int64_t)wave_incl_scan((uint64_t)inc);
    const int64_t S0 = S1 - inc;
    const uint64_t out = __ballot(valid && (S1 >= smax || S1 <= -smax));
    const uint32_t first_out = out ? (uint32_t)__builtin_ctzll(out) : 64u;
    const bool live = valid && !frozen && lane < first_out;  // a prefix of the lanes
    const int64_t c1 = live ? cm_isqrt(one - S1 * S1) : 0;
    const int64_t c_up = __shfl_up(c1, 1, 64);
    const int64_t c0 = lane == 0 ? Sc : c_up;
    int64_t dY = 0, dZ = 0;
    if (live) {
      const int64_t F = cm_rdiv((S0 + S1) * ((int64_t)1 << 24), c0 + c1);
      dY = cm_rshift(D * F, 24);
      const int64_t L = cm_rshift(D * cm_isqrt(((int64_t)1 << 48) + F * F), 24);
      dZ = cm_rshift(m.T * L, 30);
    }
    const int64_t Y1 = Y + (int64_t)wave_incl_scan((uint64_t)dY);
    const int64_t Z1 = Z + (int64_t)wave_incl_scan((uint64_t)dZ);
    if (valid) {
      ty[a + 1] = cm_q(Y1);
      tz[a + 1] = cm_q(Z1);
    }
    // the state after the last of these 64 steps (S and its root matter only
    // while nothing is frozen)
    Y = __shfl(Y1, 63, 64);
    Z = __shfl(Z1, 63, 64);
    S = __shfl(S1, 63, 64);
    Sc = __shfl(c1, 63, 64);
    if (out) frozen = true;
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Per-track record lengths, the hits' residual codes (kept for the writing
// pass) and the residual histograms (per workgroup in LDS, then added to the
// caller's): one wave per track, its hits 64 at a time.  The same lengths
// and codes as stepping the helix hit by hit with cm_step: a hit's (unit,row)
// is the largest reached so far (rows are searched forward only), the helix
// is taken at the highest row reached so far (it is never stepped back), from
// a table of all rows (cm_helix_rows); the rows are found in the first hit's
// unit's row starts staged in LDS, or in all of them for a hit outside it.
// Seven waves per SIMD (71 VGPRs, no spill) where the compiler would allow
// six: a track's wave mostly waits on memory, and more waves hide more of it
// (1.00 -> 0.96 ms on the 2 ms slice).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7))) void k_cm_track_bits(CmClusters cl, CmTracks tr, int64_t b30,
                                                       const DevParams* __restrict__ P,
                                                       uint32_t* __restrict__ tbits,
                                                       uint32_t* __restrict__ hist_out,
                                                       uint64_t* __restrict__ res, uint32_t res_cap,
                                                       DevStatus* st) {
  __shared__ uint32_t h[256];
  __shared__ int32_t xs[NROW];
  __shared__ int64_t tab[4][2][NROW];  // per wave: q(y), q(z) of the helix per row
  __shared__ uint32_t rs[4][NROW + 1];  // per wave: row starts of the track's unit
  if (failed(st)) return;
  for (uint32_t i = threadIdx.x; i < 256; i += blockDim.x) h[i] = 0;
  for (uint32_t i = threadIdx.x; i < NROW; i += blockDim.x) xs[i] = P->xfx[i];
  __syncthreads();
  const uint32_t n = scan_count(tr.n_dev, tr.cap);
  const uint32_t n_cl = scan_count(cl.n_dev, cl.cap);
  const uint32_t w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int64_t* ty = tab[w][0];
  int64_t* tz = tab[w][1];
  uint32_t* rw = rs[w];
  const bool staged = cl.n_ur >= NROW;
  for (uint32_t j = blockIdx.x * 4 + w; j < n; j += gridDim.x * 4) {  // uniform per wave
    uint32_t h0 = tr.hit_start[j], h1 = tr.hit_start[j + 1];
    if (h1 > tr.hit_cap) h1 = tr.hit_cap;
    if (h0 > h1) h0 = h1;
    uint32_t ur0 = 0;
    if (h1 > h0) {
      const uint32_t c = tr.hits[h0];
      ur0 = cm_find_ur_wave(cl.crow, cl.n_ur, c < n_cl ? c : 0);
    }
    const uint32_t ub = ur0 / NROW * NROW;  // ub + NROW <= n_ur: n_ur is a multiple of NROW
    const int r0 = tr.row[j];
    const int rt = r0 < NROW ? r0 : NROW - 1;  // a helix at a row past the last is never stepped
    const CmParams q = cm_params(tr.par + (size_t)j * 5, tr.z_anchor[j]);
    if (staged)
      for (uint32_t k = lane; k <= NROW; k += 64) rw[k] = cl.crow[ub + k];
    cm_helix_rows(cm_model(q, b30, rt), xs, ty, tz);  // also makes rw visible
    const bool cached = res != nullptr && h1 <= res_cap;
    uint64_t len = 0;
    bool bad = false;
    uint32_t ur_c = ur0;  // the (unit,row) reached so far
    int prev_c = r0;      // the previous hit's row (the track's row before the first)
    int mrow_c = rt;      // the helix's row so far
    for (uint32_t base = h0; base < h1; base += 64) {  // uniform
      const uint32_t hh = base + lane;
      const bool act = hh < h1;
      uint32_t c = act ? tr.hits[hh] : 0u;
      if (c >= n_cl) {
        bad = bad || act;
        c = 0;
      }
      uint32_t f;
      if (staged && c >= rw[0] && c < rw[NROW]) {
        uint32_t lo = 0, hi = NROW;
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) >> 1;
          if (rw[mid] <= c) lo = mid;
          else hi = mid;
        }
        f = ub + lo;
      } else {
        f = cm_find_ur(cl.crow, cl.n_ur, c);
      }
      const uint32_t u = cm_wave_incl_max(act ? max(f, ur_c) : ur_c);
      const int r = (int)(u % NROW);
      const int r_up = __shfl_up(r, 1, 64);
      const int prev = lane == 0 ? prev_c : r_up;
      const int step = r - prev - (hh > h0 ? 1 : 0);
      if (act && step < 0) bad = true;
      const uint64_t stp = step < 0 ? 0 : (uint64_t)step;
      const int mr = (int)cm_wave_incl_max((uint32_t)(act ? max(r, mrow_c) : mrow_c));
      if (act) {
        const int64_t dy = cm_q(cl.y[c]) - ty[mr];
        const int64_t dz = cm_q(cl.z[c]) - tz[mr];
        const uint64_t zy = cm_zig(dy), zz = cm_zig(dz);
        if (cached) {
          res[2 * (size_t)hh] = zy;
          res[2 * (size_t)hh + 1] = zz;
        }
        len += cm_eg_len(stp, 0) + cm_eg_len(zy, 2) + cm_eg_len(zz, 2) +
               cm_cluster_len(cl.qtot[c], cl.qmax[c]);
        if (hist_out) {
          atomicAdd(&h[(dy < -64 ? -64 : dy > 63 ? 63 : dy) + 64], 1u);
          atomicAdd(&h[128 + (dz < -64 ? -64 : dz > 63 ? 63 : dz) + 64], 1u);
        }
      }
      // the carries: the last hit of these 64
      const int last = (int)min(63u, h1 - 1 - base);
      ur_c = __shfl(u, last, 64);
      prev_c = __shfl(r, last, 64);
      mrow_c = __shfl(mr, last, 64);
    }
    const uint64_t tot = 8 + 16 + 8 + 5 * 32 + __shfl(wave_incl_scan(len), 63, 64);
    const bool any_bad = __ballot(bad) != 0;
    if (lane == 0) {
      if (any_bad) latch(st, TPC_ERR_INPUT);
      tbits[j] = (uint32_t)(tot < 0xFFFFFFFFull ? tot : 0xFFFFFFFFull);
    }
    // the wave's LDS reads are done before the next track overwrites them
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  if (hist_out)
    for (uint32_t i = threadIdx.x; i < 256; i += blockDim.x)
      if (h[i]) atomicAdd(&hist_out[i], h[i]);
}

// Clusters on no track of one (unit,row), one wave: each lane's cluster code
// length, with the drift position relative to the previous such cluster.
// Calls fn(lane's cluster, its bit offset in the row block, yq zig, z code,
// z order) for every such cluster; returns the block's length.
template <class Fn>
__device__ uint64_t cm_row(const CmClusters& cl, const int32_t* __restrict__ ct, uint32_t ur,
                           uint64_t base, Fn fn) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t n_cl = scan_count(cl.n_dev, cl.cap);
  uint32_t c0 = cl.crow[ur], c1 = cl.crow[ur + 1];
  if (c1 > n_cl) c1 = n_cl;
  if (c0 > c1) c0 = c1;
  // the count first
  uint32_t cnt = 0;
  for (uint32_t b = c0; b < c1; b += 64) {
    const uint32_t c = b + lane;
    const bool un = c < c1 && ct[c] < 0;
    cnt += (uint32_t)__popcll(__ballot(un));
  }
  uint64_t off = base;
  const uint64_t cnt_len = cm_eg_len(cnt, 0);
  fn.count(cnt, off);
  // chunks of CM_CHUNK clusters: a 32-bit field per chunk after the first
  // (its bit offset from the end of the fields), each chunk's first z whole
  const uint32_t n_chunks = (cnt + CM_CHUNK - 1) / CM_CHUNK;
  const uint64_t fields = off + cnt_len;
  off = fields + 32ull * (n_chunks > 1 ? n_chunks - 1 : 0);
  const uint64_t chunk0 = off;
  int64_t zprev = 0;
  uint32_t rank0 = 0;  // clusters on no track in earlier batches
  for (uint32_t b = c0; b < c1; b += 64) {
    const uint32_t c = b + lane;
    const bool un = c < c1 && ct[c] < 0;
    const uint64_t mask = __ballot(un);
    int64_t zq = 0, yq = 0;
    uint32_t len = 0;
    if (un) {
      zq = cm_q(cl.z[c]);
      yq = cm_q(cl.y[c]);
    }
    // the previous cluster on no track: the highest set lane below, else the
    // carry from earlier batches
    const uint64_t below = mask & ((1ull << lane) - 1);
    const uint32_t rank = rank0 + (uint32_t)__popcll(below);
    const int src = below ? 63 - __builtin_clzll(below) : (int)lane;
    const int64_t zp_lane = __shfl(zq, src, 64);
    const bool first = rank % CM_CHUNK == 0;
    const int64_t zp = below ? zp_lane : zprev;
    uint64_t zcode = 0;
    int zk = 12;
    if (un) {
      if (first) {
        zcode = cm_zig(zq);
        zk = 12;
      } else {
        zcode = cm_zig(zq - zp);
        zk = 6;
      }
      len = cm_eg_len(cm_zig(yq), 10) + cm_eg_len(zcode, zk) + cm_cluster_len(cl.qtot[c], cl.qmax[c]);
    }
    // exclusive prefix of the lengths in lane order
    uint64_t incl = wave_incl_scan((uint64_t)len);
    const uint64_t tot = __shfl(incl, 63, 64);
    if (un) {
      const uint64_t at = off + incl - len;
      if (first && rank > 0) fn.field(at - chunk0, fields + 32ull * (rank / CM_CHUNK - 1));
      fn.cluster(c, at, cm_zig(yq), zcode, zk);
    }
    off += tot;
    if (mask) {  // uniform
      const int last = 63 - __builtin_clzll(mask);
      zprev = __shfl(zq, last, 64);
      rank0 += (uint32_t)__popcll(mask);
    }
  }
  return off - base;
}

struct CmRowLen {
  __device__ void count(uint32_t, uint64_t) const {}
  __device__ void field(uint64_t, uint64_t) const {}
  __device__ void cluster(uint32_t, uint64_t, uint64_t, uint64_t, int) const {}
};

__global__ __launch_bounds__(256) void k_cm_row_bits(CmClusters cl, const int32_t* __restrict__ ct,
                                                     uint32_t* __restrict__ rbits,
                                                     const DevStatus* st) {
  if (failed(st)) return;
  const uint32_t wpb = blockDim.x >> 6;
  for (uint32_t ur = blockIdx.x * wpb + (threadIdx.x >> 6); ur < cl.n_ur;
       ur += gridDim.x * wpb) {
    const uint64_t len = cm_row(cl, ct, ur, 0, CmRowLen{});
    if ((threadIdx.x & 63) == 0) rbits[ur] = (uint32_t)(len < 0xFFFFFFFFull ? len : 0xFFFFFFFFull);
  }
}

// Directory entries from the scans: track j at stream[CM_HDR + j], row block
// ur at stream[CM_HDR + n_tracks + 1 + ur] (after the tracks' total).
struct CmEmitTrack {
  uint32_t* s;
  uint32_t cap;
  __device__ void operator()(uint32_t j, unsigned long long pre, unsigned long long) const {
    if (CM_HDR + (uint64_t)j < cap) s[CM_HDR + j] = (uint32_t)pre;
  }
};
struct CmEmitRow {
  uint32_t* s;
  uint32_t cap;
  const uint32_t* n_tracks_dev;
  uint32_t tr_cap;
  const unsigned long long* track_total;
  __device__ void operator()(uint32_t ur, unsigned long long pre, unsigned long long) const {
    const uint64_t i = CM_HDR + (uint64_t)scan_count(n_tracks_dev, tr_cap) + 1 + ur;
    if (i < cap) s[i] = (uint32_t)(pre + *track_total);
  }
};
struct CmEmitOff {
  uint32_t* out;
  __device__ void operator()(uint32_t i, unsigned long long pre, unsigned long long) const {
    out[i] = (uint32_t)pre;
  }
};
struct CmGetU32 {
  const uint32_t* a;
  __device__ unsigned long long operator()(uint32_t i) const { return a[i]; }
};

// Header, the closing directory entries, the size check.  tot[0] = tracks'
// bits, tot[1] = rows' bits; info[0] = words needed (0 after an error).
__global__ void k_cm_finish(uint32_t* __restrict__ s, uint32_t cap, uint32_t n_units,
                            const uint32_t* n_tracks_dev, uint32_t tr_cap,
                            const uint32_t* hit_start, const uint32_t* n_cl_dev, uint32_t cl_cap,
                            const unsigned long long* tot, uint32_t* n_words_out,
                            uint32_t* info, DevStatus* st) {
  info[0] = 0;
  if (failed(st)) return;
  const uint32_t n_tr = scan_count(n_tracks_dev, tr_cap);
  const uint32_t n_ur = n_units * NROW;
  const unsigned long long bits = tot[0] + tot[1];
  const uint64_t dir = CM_HDR + (uint64_t)n_tr + 1 + n_ur + 1;
  const uint64_t need = dir + (bits + 31) / 32;
  *n_words_out = (uint32_t)(need < 0xFFFFFFFFull ? need : 0xFFFFFFFFull);
  if (bits > 0xFFFFFFFFull || need > cap) {
    latch(st, TPC_ERR_CAPACITY, (uint32_t)(need < 0xFFFFFFFFull ? need : 0xFFFFFFFFull));
    return;
  }
  s[0] = CM_MAGIC;
  s[1] = CM_VERSION;
  s[2] = n_units;
  s[3] = n_tr;
  s[4] = scan_count(n_cl_dev, cl_cap);
  s[5] = n_tr ? hit_start[n_tr] : 0;
  s[6] = (uint32_t)bits;
  s[7] = 0;
  s[CM_HDR + n_tr] = (uint32_t)tot[0];
  s[dir - 1] = (uint32_t)bits;
  info[0] = (uint32_t)need;
  info[1] = (uint32_t)dir;
}

// clear the payload words [dir, need)
__global__ void k_cm_clear(uint32_t* __restrict__ s, const uint32_t* info, const DevStatus* st) {
  if (failed(st)) return;
  const uint32_t need = info[0], dir = info[1];
  for (uint32_t i = dir + blockIdx.x * blockDim.x + threadIdx.x; i < need;
       i += gridDim.x * blockDim.x)
    s[i] = 0;
}

// The track records' bits at their directory offsets, one wave per track:
// lane 0 writes the record's fixed fields, and each hit's lane its codes at
// the record's start + 192 bits + the lengths of the hits before it (a wave
// prefix sum), each lane with its own writer (atomic OR: a word may be shared
// with a neighbouring hit or record).  The residuals come from the sizing
// pass's cache, else from the helix table, as in k_cm_track_bits.
// Six waves per SIMD (80 VGPRs, no spill; seven would spill) where the
// compiler would allow five (1.17 -> 1.06 ms on the 2 ms slice).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_cm_track_write(CmClusters cl, CmTracks tr, int64_t b30,
                                                        const DevParams* __restrict__ P,
                                                        uint32_t* __restrict__ s,
                                                        const uint32_t* info,
                                                        const uint64_t* __restrict__ res,
                                                        uint32_t res_cap, DevStatus* st) {
  __shared__ int32_t xs[NROW];
  __shared__ int64_t tab[4][2][NROW];
  __shared__ uint32_t rs[4][NROW + 1];
  if (failed(st) || info[0] == 0) return;
  for (uint32_t i = threadIdx.x; i < NROW; i += blockDim.x) xs[i] = P->xfx[i];
  __syncthreads();
  const uint32_t n = scan_count(tr.n_dev, tr.cap);
  const uint32_t n_cl = scan_count(cl.n_dev, cl.cap);
  uint32_t* payload = s + info[1];
  const uint64_t pw = info[0] - info[1];
  const uint32_t w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int64_t* ty = tab[w][0];
  int64_t* tz = tab[w][1];
  uint32_t* rw = rs[w];
  const bool staged = cl.n_ur >= NROW;
  for (uint32_t j = blockIdx.x * 4 + w; j < n; j += gridDim.x * 4) {  // uniform per wave
    uint32_t h0 = tr.hit_start[j], h1 = tr.hit_start[j + 1];
    if (h1 > tr.hit_cap) h1 = tr.hit_cap;
    if (h0 > h1) h0 = h1;
    uint32_t ur0 = 0;
    if (h1 > h0) {
      const uint32_t c = tr.hits[h0];
      ur0 = cm_find_ur_wave(cl.crow, cl.n_ur, c < n_cl ? c : 0);
    }
    const uint32_t ub = ur0 / NROW * NROW;
    const int r0 = tr.row[j];
    const int rt = r0 < NROW ? r0 : NROW - 1;
    const CmParams q = cm_params(tr.par + (size_t)j * 5, tr.z_anchor[j]);
    const uint64_t start = s[CM_HDR + j];
    const bool cached = res != nullptr && h1 <= res_cap;  // uniform
    if (staged)
      for (uint32_t k = lane; k <= NROW; k += 64) rw[k] = cl.crow[ub + k];
    if (!cached) {
      cm_helix_rows(cm_model(q, b30, rt), xs, ty, tz);  // also makes rw visible
    } else {
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
    if (lane == 0) {
      CmWriter wr;
      wr.init(payload, pw, start);
      wr.put(h1 - h0, 8);
      wr.put(ur0 / NROW, 16);
      wr.put((uint32_t)r0, 8);
      wr.put((uint32_t)(int32_t)q.Y, 32);
      wr.put((uint32_t)(int32_t)q.Z, 32);
      wr.put((uint32_t)(int32_t)q.S, 32);
      wr.put((uint32_t)(int32_t)q.T, 32);
      wr.put((uint32_t)(int32_t)q.K, 32);
      wr.flush();
    }
    uint64_t off = start + 8 + 16 + 8 + 5 * 32;
    uint32_t ur_c = ur0;
    int prev_c = r0;
    int mrow_c = rt;
    for (uint32_t base = h0; base < h1; base += 64) {  // uniform
      const uint32_t hh = base + lane;
      const bool act = hh < h1;
      uint32_t c = act ? tr.hits[hh] : 0u;
      if (c >= n_cl) c = 0;
      uint32_t f;
      if (staged && c >= rw[0] && c < rw[NROW]) {
        uint32_t lo = 0, hi = NROW;
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) >> 1;
          if (rw[mid] <= c) lo = mid;
          else hi = mid;
        }
        f = ub + lo;
      } else {
        f = cm_find_ur(cl.crow, cl.n_ur, c);
      }
      const uint32_t u = cm_wave_incl_max(act ? max(f, ur_c) : ur_c);
      const int r = (int)(u % NROW);
      const int r_up = __shfl_up(r, 1, 64);
      const int prev = lane == 0 ? prev_c : r_up;
      const int step = r - prev - (hh > h0 ? 1 : 0);
      const uint64_t stp = step < 0 ? 0 : (uint64_t)step;
      const int mr = (int)cm_wave_incl_max((uint32_t)(act ? max(r, mrow_c) : mrow_c));
      uint64_t zy = 0, zz = 0;
      uint16_t qt = 0, qm = 0;
      uint8_t fl = 0;
      uint64_t hl = 0;
      if (act) {
        if (cached) {
          zy = res[2 * (size_t)hh];
          zz = res[2 * (size_t)hh + 1];
        } else {
          zy = cm_zig(cm_q(cl.y[c]) - ty[mr]);
          zz = cm_zig(cm_q(cl.z[c]) - tz[mr]);
        }
        qt = cl.qtot[c];
        qm = cl.qmax[c];
        fl = cl.flags[c];
        hl = cm_eg_len(stp, 0) + cm_eg_len(zy, 2) + cm_eg_len(zz, 2) + cm_cluster_len(qt, qm);
      }
      const uint64_t incl = wave_incl_scan(hl);
      if (act) {
        CmWriter wr;
        wr.init(payload, pw, off + incl - hl);
        wr.eg(stp, 0);
        wr.eg(zy, 2);
        wr.eg(zz, 2);
        cm_cluster_put(wr, qt, qm, fl);
        wr.flush();
      }
      off += __shfl(incl, 63, 64);
      const int last = (int)min(63u, h1 - 1 - base);
      ur_c = __shfl(u, last, 64);
      prev_c = __shfl(r, last, 64);
      mrow_c = __shfl(mr, last, 64);
    }
    // the wave's LDS reads are done before the next track overwrites them
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

struct CmRowPut {
  const CmClusters* cl;
  uint32_t* payload;
  uint64_t pw;  // payload words
  __device__ void count(uint32_t cnt, uint64_t off) const {
    if ((threadIdx.x & 63) == 0) {
      CmWriter w;
      w.init(payload, pw, off);
      w.eg(cnt, 0);
      w.flush();
    }
  }
  // a chunk's 32-bit offset field (its value < 2^32: payload offsets are)
  __device__ void field(uint64_t v, uint64_t off) const {
    CmWriter w;
    w.init(payload, pw, off);
    w.put((uint32_t)v, 32);
    w.flush();
  }
  __device__ void cluster(uint32_t c, uint64_t off, uint64_t yz, uint64_t zcode, int zk) const {
    CmWriter w;
    w.init(payload, pw, off);
    w.eg(yz, 10);
    w.eg(zcode, zk);
    cm_cluster_put(w, cl->qtot[c], cl->qmax[c], cl->flags[c]);
    w.flush();
  }
};

__global__ __launch_bounds__(256) void k_cm_row_write(CmClusters cl, const int32_t* __restrict__ ct,
                                                      uint32_t* __restrict__ s,
                                                      const uint32_t* n_tracks_dev, uint32_t tr_cap,
                                                      const uint32_t* info, const DevStatus* st) {
  if (failed(st) || info[0] == 0) return;
  const uint32_t n_tr = scan_count(n_tracks_dev, tr_cap);
  uint32_t* payload = s + info[1];
  const uint32_t wpb = blockDim.x >> 6;
  for (uint32_t ur = blockIdx.x * wpb + (threadIdx.x >> 6); ur < cl.n_ur;
       ur += gridDim.x * wpb) {
    const uint64_t base = s[CM_HDR + n_tr + 1 + ur];
    cm_row(cl, ct, ur, base, CmRowPut{&cl, payload, (uint64_t)(info[0] - info[1])});
  }
}

// ------------------------------------------------------------------ decoder
struct CmDecOut {
  uint32_t capacity;
  uint16_t* unit;
  uint8_t* row;
  int32_t *y, *z;
  uint16_t *qtot, *qmax;
  uint8_t* flags;
  int32_t* track;
};

// Header checks; info = {n_units, n_tracks, n_clusters, payload bits, dir
// words, records (tracks + rows), ok}.
__global__ void k_cm_dec_header(const uint32_t* __restrict__ s, uint32_t n_words, uint32_t max_units,
                                uint32_t max_tracks, uint32_t out_cap, uint32_t* n_out,
                                uint32_t* info, DevStatus* st) {
  info[6] = 0;
  if (failed(st)) return;
  if (n_words < CM_HDR || s[0] != CM_MAGIC || s[1] != CM_VERSION || s[7] != 0) {
    latch(st, TPC_ERR_INPUT);
    return;
  }
  const uint32_t nu = s[2], nt = s[3], nc = s[4], bits = s[6];
  const uint64_t dir = CM_HDR + (uint64_t)nt + 1 + (uint64_t)nu * NROW + 1;
  if (nu > max_units || nt > max_tracks || dir > n_words || bits > (n_words - dir) * 32ull ||
      s[CM_HDR + nt + 1 + (uint64_t)nu * NROW] != bits || s[CM_HDR] != 0 ||
      s[CM_HDR + nt] != s[CM_HDR + nt + 1]) {  // the rows begin where the tracks end
    latch(st, TPC_ERR_INPUT);
    return;
  }
  *n_out = nc;
  if (nc > out_cap) {
    latch(st, TPC_ERR_CAPACITY, nc);
    return;
  }
  info[0] = nu;
  info[1] = nt;
  info[2] = nc;
  info[3] = bits;
  info[4] = (uint32_t)dir;
  info[5] = nt + nu * NROW;
  info[6] = 1;
}

// Clusters per record: a track's fixed-width hit count, a row's count code.
__global__ void k_cm_dec_counts(const uint32_t* __restrict__ s, const uint32_t* info,
                                uint32_t* __restrict__ cnt, DevStatus* st) {
  if (failed(st) || !info[6]) return;
  const uint32_t nt = info[1], nrec = info[5];
  CmReader r{s + info[4], 0, info[3], false, 0};
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nrec; i += gridDim.x * blockDim.x) {
    r.bad = false;
    r.seek(s[CM_HDR + (i < nt ? i : i + 1)]);
    cnt[i] = (uint32_t)(i < nt ? r.get(8) : r.eg(0));
    if (r.bad || cnt[i] > 0xFFFFFFu) {
      cnt[i] = 0;
      latch(st, TPC_ERR_INPUT);
    }
  }
}

// Track record i decoded from r at output offset k; false if it is malformed
// or does not end at `end`.
template <typename Reader>
__device__ bool cm_decode_record(Reader& r, uint32_t i, uint32_t nu, uint32_t nt, uint32_t nc,
                                 uint32_t k, uint64_t end, int64_t b30, const int32_t* xfx,
                                 const CmDecOut& o) {
  bool bad = false;
  if (i < nt) {
    const uint32_t nh = (uint32_t)r.get(8);
    const uint32_t unit = (uint32_t)r.get(16);
    const int r0 = (int)r.get(8);
    CmParams q;
    q.Y = (int32_t)r.get(32);
    q.Z = (int32_t)r.get(32);
    q.S = (int32_t)r.get(32);
    q.T = (int32_t)r.get(32);
    q.K = (int32_t)r.get(32);
    if (unit >= nu || r0 >= NROW) bad = true;
    CmModel m = cm_model(q, b30, r0);
    int prev = r0;
    for (uint32_t h = 0; h < nh && !bad && !r.bad; ++h, ++k) {
      const uint64_t stp = r.eg(0);
      const int rr = prev + (int)(stp > NROW ? NROW : stp) + (h > 0 ? 1 : 0);
      if (rr >= NROW || k >= nc || k >= o.capacity) {
        bad = true;
        break;
      }
      prev = rr;
      while (m.row < rr) cm_step(m, xfx);
      const int64_t yq = cm_q(m.Y) + cm_unzig(r.eg(2));
      const int64_t zq = cm_q(m.Z) + cm_unzig(r.eg(2));
      o.unit[k] = (uint16_t)unit;
      o.row[k] = (uint8_t)rr;
      o.y[k] = (int32_t)(yq << CM_QSHIFT);
      o.z[k] = (int32_t)(zq << CM_QSHIFT);
      o.qtot[k] = (uint16_t)r.eg(6);
      o.qmax[k] = (uint16_t)r.eg(5);
      o.flags[k] = (uint8_t)r.get(2);
      o.track[k] = (int32_t)i;
    }
  }
  return !(bad || r.bad || r.pos != end);
}

// One chunk of row record ur (k-th, `count` clusters) from r, written at
// output index k0 on; false if malformed or not ending at `end`.
template <typename Reader>
__device__ bool cm_decode_chunk(Reader& r, uint32_t ur, uint32_t count, uint32_t k0, uint32_t nc,
                                uint64_t end, const CmDecOut& o) {
  int64_t zprev = 0;
  uint32_t k = k0;
  for (uint32_t c = 0; c < count && !r.bad; ++c, ++k) {
    if (k >= nc || k >= o.capacity) return false;
    const int64_t yq = cm_unzig(r.eg(10));
    const int64_t zq = c == 0 ? cm_unzig(r.eg(12)) : zprev + cm_unzig(r.eg(6));
    zprev = zq;
    o.unit[k] = (uint16_t)(ur / NROW);
    o.row[k] = (uint8_t)(ur % NROW);
    o.y[k] = (int32_t)(yq << CM_QSHIFT);
    o.z[k] = (int32_t)(zq << CM_QSHIFT);
    o.qtot[k] = (uint16_t)r.eg(6);
    o.qmax[k] = (uint16_t)r.eg(5);
    o.flags[k] = (uint8_t)r.get(2);
    o.track[k] = -1;
  }
  return !(r.bad || r.pos != end);
}

// Row record ur at bits [b0, b1): the count and the chunk fields, then lane
// l decodes chunks l, l + 64, ...; every chunk must end where the next one
// (or the record) ends.  Reader: the row's bits (staged in LDS, or global).
template <typename Reader>
__device__ void cm_decode_row(Reader r, uint32_t ur, uint32_t k_row, uint32_t nc, uint64_t b0,
                              uint64_t b1, const CmDecOut& o, DevStatus* st) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t n = r.eg(0);
  if (r.bad || n > 0xFFFFFFu) {
    if (lane == 0) latch(st, TPC_ERR_INPUT);
    return;
  }
  const uint32_t m = ((uint32_t)n + CM_CHUNK - 1) / CM_CHUNK;
  const uint64_t fields = r.pos;
  const uint64_t chunk0 = fields + 32ull * (m > 1 ? m - 1 : 0);
  if (m == 0) {
    if (lane == 0 && r.pos != b1) latch(st, TPC_ERR_INPUT);
    return;
  }
  if (chunk0 > b1) {
    if (lane == 0) latch(st, TPC_ERR_INPUT);
    return;
  }
  for (uint32_t k = lane; k < m; k += 64) {
    uint64_t cs = chunk0, ce = b1;
    if (k > 0) {
      r.seek(fields + 32ull * (k - 1));
      cs = chunk0 + r.get(32);
    }
    if (k + 1 < m) {
      r.seek(fields + 32ull * k);
      ce = chunk0 + r.get(32);
    }
    bool ok = !r.bad && cs <= ce && ce <= b1;
    if (ok) {
      const uint64_t end_save = r.end;
      r.end = ce;  // reads stop at the chunk's end
      r.seek(cs);
      const uint32_t count = min((uint32_t)n - CM_CHUNK * k, (uint32_t)CM_CHUNK);
      ok = cm_decode_chunk(r, ur, count, k_row + CM_CHUNK * k, nc, ce, o);
      r.end = end_save;
      r.bad = false;
    }
    if (!ok) latch(st, TPC_ERR_INPUT);
  }
}

// Row records: one wave per record, its bits first copied into the wave's
// part of LDS when they fit, one lane per chunk.
__global__ __launch_bounds__(256) void k_cm_dec_rows(const uint32_t* __restrict__ s,
                                                     const uint32_t* info,
                                                     const uint32_t* __restrict__ off,
                                                     const unsigned long long* total,
                                                     CmDecOut o, DevStatus* st) {
  __shared__ uint32_t stage[4][CM_STAGE_WORDS];
  if (failed(st) || !info[6]) return;
  const uint32_t nt = info[1], nc = info[2], nrec = info[5];
  const uint64_t bits = info[3];
  const uint32_t* pay = s + info[4];
  if (blockIdx.x == 0 && threadIdx.x == 0 && *total != nc) latch(st, TPC_ERR_INPUT);
  const uint32_t w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (uint32_t i = nt + blockIdx.x * 4 + w; i < nrec; i += gridDim.x * 4) {
    uint64_t b0 = s[CM_HDR + i + 1], b1 = s[CM_HDR + i + 2];
    if (b0 > bits) b0 = bits;
    if (b1 > bits) b1 = bits;
    if (b1 < b0) b1 = b0;
    const uint64_t w0 = b0 >> 5, w1 = (b1 + 31) >> 5;
    const bool staged = w1 - w0 <= CM_STAGE_WORDS;
    if (staged) {
      for (uint64_t k = lane; k < w1 - w0; k += 64) stage[w][k] = pay[w0 + k];
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (staged) {
      cm_decode_row(CmReaderT<lds_u32*>((lds_u32*)stage[w], b0, b1, false, w0), i - nt, off[i], nc,
                    b0, b1, o, st);
    } else {
      cm_decode_row(CmReader(pay, b0, b1, false, 0), i - nt, off[i], nc, b0, b1, o, st);
    }
    // the wave's LDS reads are done before the next record overwrites it
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// Track records: 64 per wave, one per lane; the wave's records' bits are
// first copied into its part of LDS when they fit (a dependent chain of
// global reads is what bounds a sequential decoder), else read from the
// payload.
__global__ __launch_bounds__(256) void k_cm_dec_tracks(const uint32_t* __restrict__ s,
                                                       const uint32_t* info,
                                                       const uint32_t* __restrict__ off,
                                                       int64_t b30, const DevParams* __restrict__ P,
                                                       CmDecOut o, DevStatus* st) {
  __shared__ uint32_t stage[4][CM_STAGE_WORDS];
  __shared__ int32_t xs[NROW];  // row radii: the helix steps read them per lane
  if (failed(st) || !info[6]) return;
  for (uint32_t i = threadIdx.x; i < NROW; i += blockDim.x) xs[i] = P->xfx[i];
  __syncthreads();
  const uint32_t nu = info[0], nt = info[1], nc = info[2];
  const uint64_t bits = info[3];
  const uint32_t* pay = s + info[4];
  const uint32_t w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t n_groups = (nt + 63) / 64;
  for (uint32_t g = blockIdx.x * 4 + w; g < n_groups; g += gridDim.x * 4) {
    const uint32_t i0 = g * 64;
    const uint32_t i1 = min(i0 + 64, nt);
    // the wave's bit range: from the first record's start to the last one's end
    uint64_t b0 = s[CM_HDR + i0];
    uint64_t b1 = s[CM_HDR + i1];
    if (b0 > bits) b0 = bits;
    if (b1 > bits) b1 = bits;
    if (b1 < b0) b1 = b0;
    const uint64_t w0 = b0 >> 5, w1 = (b1 + 31) >> 5;
    const bool staged = w1 - w0 <= CM_STAGE_WORDS;
    if (staged) {
      for (uint64_t k = lane; k < w1 - w0; k += 64) stage[w][k] = pay[w0 + k];
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const uint32_t i = i0 + lane;
    if (i < i1) {
      const uint64_t start = s[CM_HDR + i];
      const uint64_t end = s[CM_HDR + i + 1];
      // from LDS when the record lies in the staged range (reads stop at its
      // end), else (a malformed directory) from the payload
      const bool in_lds = staged && start >= b0 && end <= b1;
      bool ok;
      if (in_lds) {
        CmReaderT<lds_u32*> r((lds_u32*)stage[w], start, b1, false, w0);
        ok = cm_decode_record(r, i, nu, nt, nc, off[i], end, b30, xs, o);
      } else {
        CmReader r(pay, start, bits, false, 0);
        ok = cm_decode_record(r, i, nu, nt, nc, off[i], end, b30, xs, o);
      }
      if (!ok) latch(st, TPC_ERR_INPUT);
    }
    // the wave's LDS reads are done before the next group overwrites it
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}
