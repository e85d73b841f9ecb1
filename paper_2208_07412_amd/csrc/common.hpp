// Device-side building blocks shared by the kernels of libtpcreco:
// parameter block, status word, wave64 / workgroup scans and the
// three-phase device-wide scan used for every order-preserving compaction.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tpc.h"

#define NROW TPC_NROW
#define SCAN_BLOCK 256
#define SCAN_ITEMS 8
#define SCAN_TILE (SCAN_BLOCK * SCAN_ITEMS)

// Parameters and row tables, resident in device memory for one context.
// DevParams32 holds everything but the FP64 copies, which only the refit's
// FP64 path reads: kernels that compute in FP32 copy just this part into LDS.
struct DevParams32 {
  int32_t np[NROW];   // pads per row
  int32_t xfx[NROW];  // row radius, 2^-16 cm
  int32_t pfx[NROW];  // pad pitch, 2^-16 cm
  float x[NROW], hw[NROW], vy[NROW], vz[NROW];
  int32_t qmax_min, min_tracklet, max_miss, min_track_hits;
  int64_t win_y, win_z, s_max;
  float chi2_max, snp_max, bz_b, c0_snp2, c0_tgl2, c0_qpt2, qpt_clamp, edge_margin, lowpt_qpt;
  float c0r2[5], refit_snp_max;  // refit prior variances (y, z, snp, tgl, q/pT)
  int32_t validate, force_fallback;
};
struct DevParams : DevParams32 {
  double xd[NROW], hwd[NROW], vyd[NROW], vzd[NROW];
  double chi2_max_d, snp_max_d, bz_b_d, c0_snp2_d, c0_tgl2_d, c0_qpt2_d, qpt_clamp_d,
      edge_margin_d;
  double c0r2_d[5], refit_snp_max_d;
};

// The parameters and row tables (all of them, or the FP32 part: PD is
// DevParams or DevParams32, the first part of a DevParams) copied into LDS by
// the whole workgroup (a barrier follows): per-lane row lookups in long
// serial loops then cost an LDS read instead of a round trip to the caches.
template <typename PD>
__device__ __forceinline__ const PD* params_to_lds(const DevParams* P, PD* lds) {
  static_assert(sizeof(PD) % 8 == 0, "copied in 8-byte words");
  const uint2* src = reinterpret_cast<const uint2*>(static_cast<const PD*>(P));
  uint2* dst = reinterpret_cast<uint2*>(lds);
  for (uint32_t i = threadIdx.x; i < sizeof(PD) / 8; i += blockDim.x) dst[i] = src[i];
  __syncthreads();
  return lds;
}

// Status word and device-side counts of one context.
struct DevStatus {
  int32_t status;
  uint32_t required;
  uint32_t n_clusters, n_tracklets, n_tracks, n_hits;
  uint32_t n_fallback, n_fallback_fail, n_not_pd, n_refit_fail;
  uint32_t n_fp64_redo;
  uint32_t overflow;  // bit k set: capacity k (OVF_*) was too small
  uint32_t req[4];    // count that capacity k needed
  unsigned long long f_steps, f_cands, f_upds, f_slots;  // following work (measurement)
};

__device__ __forceinline__ void latch(DevStatus* st, int code, uint32_t required = 0) {
  atomicCAS(&st->status, 0, code);
  if (required) atomicMax(&st->required, required);
}

// Capacities whose overflow is reported, each with the count it needed.
enum { OVF_CLUSTERS = 0, OVF_TRACKLETS = 1, OVF_TRACKS = 2, OVF_HITS = 3 };
__device__ __forceinline__ void latch_capacity(DevStatus* st, int kind, uint32_t required) {
  atomicOr(&st->overflow, 1u << kind);
  atomicMax(&st->req[kind], required);
  latch(st, TPC_ERR_CAPACITY, required);
}

__device__ __forceinline__ bool failed(const DevStatus* st) {
  return __atomic_load_n(&st->status, __ATOMIC_RELAXED) != 0;
}

__device__ __forceinline__ int64_t floor_div64(int64_t a, int64_t b) {  // b > 0
  int64_t q = a / b;
  if ((a % b != 0) && (a < 0)) --q;
  return q;
}

// Bijective remap of a 1-D grid so that consecutive logical blocks land on
// the same XCD (blocks are dispatched round-robin over 8 XCDs), which keeps
// neighbouring tiles in one L2.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t bid, uint32_t nb) {
  const uint32_t full = nb & ~7u;
  if (bid >= full) return bid;
  const uint32_t per = full >> 3;
  return (bid & 7u) * per + (bid >> 3);
}

// One item per wave over n items, in rounds of the grid's waves (stride):
// this wave's first item, with the workgroups that the dispatcher places on
// one XCD (every eighth) taking consecutive items of each round (of all
// items, when one round covers them).
__device__ __forceinline__ uint32_t xcd_wave_item(uint32_t n, uint32_t& stride) {
  const uint32_t wpb = blockDim.x >> 6;
  const uint32_t nb = (n + wpb - 1) / wpb;
  stride = gridDim.x * wpb;
  uint32_t b = blockIdx.x;
  if (nb > gridDim.x) b = xcd_remap(b, gridDim.x);
  else if (b < nb) b = xcd_remap(b, nb);
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)(b * wpb + (threadIdx.x >> 6)));
}

// One item per thread over n items, in rounds of the grid's threads
// (stride): this thread's first item, with the workgroups that the
// dispatcher places on one XCD taking consecutive blocks of items.
__device__ __forceinline__ uint32_t xcd_thread_item(uint32_t n, uint32_t& stride) {
  const uint32_t nb = (n + blockDim.x - 1) / blockDim.x;
  stride = gridDim.x * blockDim.x;
  uint32_t b = blockIdx.x;
  if (nb > gridDim.x) b = xcd_remap(b, gridDim.x);
  else if (b < nb) b = xcd_remap(b, nb);
  return b * blockDim.x + threadIdx.x;
}

// A value the whole wave holds alike, moved to a scalar register so that
// the loop control and address arithmetic built on it stay scalar.
__device__ __forceinline__ uint32_t uni(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// ------------------------------------------------------------ wave64 scans
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T o = __shfl_up(v, d, 64);
    if ((int)lane_id() >= d) v += o;
  }
  return v;
}

__device__ __forceinline__ int32_t wave_min_i32(int32_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = min(v, __shfl_xor(v, d, 64));
  return v;
}
__device__ __forceinline__ int32_t wave_max_i32(int32_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = max(v, __shfl_xor(v, d, 64));
  return v;
}
__device__ __forceinline__ unsigned long long wave_sum_u64(uint32_t v) {
  unsigned long long x = v;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

// Exclusive scan over a workgroup of BLOCK threads; returns the prefix and
// the block total.  lds needs BLOCK/64 + 1 entries.
template <typename T, int BLOCK>
__device__ __forceinline__ T block_excl_scan(T v, T* lds, T& total) {
  const int w = threadIdx.x >> 6;
  const T inc = wave_incl_scan(v);
  if (lane_id() == 63) lds[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    T acc = 0;
    for (int i = 0; i < BLOCK / 64; ++i) {
      const T t = lds[i];
      lds[i] = acc;
      acc += t;
    }
    lds[BLOCK / 64] = acc;
  }
  __syncthreads();
  const T res = lds[w] + inc - v;
  total = lds[BLOCK / 64];
  __syncthreads();
  return res;
}

// ------------------------------------------------- device-wide scan (3 phases)
// Get:  T operator()(uint32_t i) const -- value of element i (i < n)
// Emit: void operator()(uint32_t i, T prefix, T value) const
// The element count is min(*n_dev, n_cap) when n_dev is given, else n_cap.
__device__ __forceinline__ uint32_t scan_count(const uint32_t* n_dev, uint32_t n_cap) {
  if (!n_dev) return n_cap;
  const uint32_t n = *n_dev;
  return n < n_cap ? n : n_cap;
}

template <typename T, class Get>
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_reduce(Get get, const uint32_t* n_dev,
                                                            uint32_t n_cap, T* bsum,
                                                            const DevStatus* st) {
  __shared__ T lds[SCAN_BLOCK / 64 + 1];
  if (failed(st)) return;
  const uint32_t n = scan_count(n_dev, n_cap);
  const uint32_t base = blockIdx.x * SCAN_TILE;
  T acc = 0;
  if (base < n) {
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
      const uint32_t i = base + k * SCAN_BLOCK + threadIdx.x;
      if (i < n) acc += get(i);
    }
  }
  T total;
  block_excl_scan<T, SCAN_BLOCK>(acc, lds, total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// Exclusive scan of the block sums in place, by one workgroup of 1024.
template <typename T>
__global__ __launch_bounds__(1024) void k_scan_blocks(T* bsum, uint32_t nb, T* total_out,
                                                      uint32_t* total32_out, const DevStatus* st) {
  __shared__ T lds[1024 / 64 + 1];
  if (failed(st)) return;
  T carry = 0;
  for (uint32_t off = 0; off < nb; off += 1024) {
    const uint32_t i = off + threadIdx.x;
    const T v = i < nb ? bsum[i] : T(0);
    T tot;
    const T ex = block_excl_scan<T, 1024>(v, lds, tot);
    if (i < nb) bsum[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    if (total_out) *total_out = carry;
    if (total32_out) *total32_out = (uint32_t)carry;
  }
}

template <typename T, class Get, class Emit>
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_down(Get get, Emit emit, const uint32_t* n_dev,
                                                          uint32_t n_cap, const T* bsum,
                                                          const DevStatus* st) {
  __shared__ T lds[SCAN_BLOCK / 64 + 1];
  if (failed(st)) return;
  const uint32_t n = scan_count(n_dev, n_cap);
  const uint32_t base = blockIdx.x * SCAN_TILE;
  if (base >= n) return;  // uniform per block
  // each thread owns SCAN_ITEMS consecutive elements for an ordered scan
  const uint32_t first = base + threadIdx.x * SCAN_ITEMS;
  T vals[SCAN_ITEMS];
  T acc = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const uint32_t i = first + k;
    vals[k] = i < n ? get(i) : T(0);
    acc += vals[k];
  }
  T total;
  T pre = block_excl_scan<T, SCAN_BLOCK>(acc, lds, total) + bsum[blockIdx.x];
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const uint32_t i = first + k;
    if (i < n) emit(i, pre, vals[k]);
    pre += vals[k];
  }
}

template <typename T>
__global__ void k_fill(T* p, T v, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    p[i] = v;
}

// fill the first min(*n_dev, n_cap) entries
template <typename T>
__global__ void k_fill_dev(T* p, T v, const uint32_t* n_dev, uint32_t n_cap) {
  const uint32_t n = scan_count(n_dev, n_cap);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    p[i] = v;
}
