// Quality-control histograms of one reconstruction: cluster total and peak
// charge, hits per track, and clusters on / off a track.  Each workgroup
// fills its own histograms in LDS (LDS atomics only), writes them out whole,
// and a second kernel sums the workgroups' histograms bin by bin, so no
// device-scope atomic is involved.
#pragma once

#include "common.hpp"

#define QC_QTOT 0      // 256 bins: min(qtot >> 3, 255)
#define QC_QMAX 256    // 256 bins: min(qmax >> 2, 255)
#define QC_NHITS 512   // 153 bins: hits per track, 0..152
#define QC_ATTACH 665  // 2 bins: cluster not on a track / on a track
#define QC_BINS 667
#define QC_WG 1024     // workgroups of the fill kernel (4 per CU)

__global__ __launch_bounds__(256) void k_qc_fill(const uint16_t* __restrict__ qtot,
                                                 const uint16_t* __restrict__ qmax,
                                                 const int32_t* __restrict__ cluster_track,
                                                 const uint32_t* n_cl_dev, uint32_t cl_cap,
                                                 const uint32_t* __restrict__ hit_start,
                                                 const uint32_t* n_trk_dev, uint32_t trk_cap,
                                                 uint32_t* __restrict__ part, const DevStatus* st) {
  // one histogram per wave (fewer lanes contend for a hot bin); the two
  // on/off-track bins are counted in registers and added once per wave
  __shared__ uint32_t h[4][QC_BINS];
  const uint32_t w = threadIdx.x >> 6;
  for (uint32_t i = threadIdx.x; i < 4 * QC_BINS; i += blockDim.x) (&h[0][0])[i] = 0;
  __syncthreads();
  // after a latched error the outputs are not valid: empty histograms (no
  // status word, st == nullptr: the caller vouches for the outputs)
  const bool ok = st == nullptr || !failed(st);
  const uint32_t n_cl = ok ? scan_count(n_cl_dev, cl_cap) : 0u;
  const uint32_t n_trk = ok ? scan_count(n_trk_dev, trk_cap) : 0u;
  const uint32_t stride = gridDim.x * blockDim.x;
  uint32_t on = 0, off = 0;
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n_cl; c += stride) {
    atomicAdd(&h[w][QC_QTOT + min((uint32_t)qtot[c] >> 3, 255u)], 1u);
    atomicAdd(&h[w][QC_QMAX + min((uint32_t)qmax[c] >> 2, 255u)], 1u);
    if (cluster_track[c] >= 0) ++on;
    else ++off;
  }
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n_trk; j += stride) {
    const uint32_t n = hit_start[j + 1] - hit_start[j];
    atomicAdd(&h[w][QC_NHITS + min(n, (uint32_t)NROW)], 1u);
  }
  const unsigned long long son = wave_sum_u64(on), soff = wave_sum_u64(off);
  if ((threadIdx.x & 63) == 0) {
    h[w][QC_ATTACH] += (uint32_t)soff;
    h[w][QC_ATTACH + 1] += (uint32_t)son;
  }
  __syncthreads();
  uint32_t* mine = part + (size_t)blockIdx.x * QC_BINS;
  for (uint32_t i = threadIdx.x; i < QC_BINS; i += blockDim.x)
    mine[i] = h[0][i] + h[1][i] + h[2][i] + h[3][i];
}

// hist[i] = sum over the nwg workgroup histograms of bin i: one workgroup
// per bin, its threads taking every 256th workgroup histogram
__global__ __launch_bounds__(256) void k_qc_sum(const uint32_t* __restrict__ part, uint32_t nwg,
                                                uint32_t* __restrict__ hist) {
  __shared__ unsigned long long ws[4];
  const uint32_t i = blockIdx.x;
  uint32_t s = 0;
  for (uint32_t w = threadIdx.x; w < nwg; w += blockDim.x) s += part[(size_t)w * QC_BINS + i];
  const unsigned long long t = wave_sum_u64(s);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) hist[i] = (uint32_t)(ws[0] + ws[1] + ws[2] + ws[3]);
}
