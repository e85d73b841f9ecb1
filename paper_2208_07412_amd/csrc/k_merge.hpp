// Segment merging (sector boundaries, looper legs) and the continuous-readout
// T0 / z fit of the merged tracks.
//
// A segment's two ends (innermost and outermost hit) carry their global
// position, drift z and the tangent of the segment's outward fit there.  Ends
// are binned by (frame, side, 30.5 cm squares of the bending plane, 36 cm of
// drift); one lane per end tests the ends of later segments in the 3 x 3 x 3
// cells around it with the joining rule (every joinable pair has ends within
// 35 cm in drift and 30 cm in the bending plane, so the cells hold all
// candidates), and joins
// segments by a lock-free union-find that always hangs the larger root under
// the smaller, so the final root of a component is its smallest segment
// whatever the order of the unions.  The members of each component are then
// sorted by (root, index), and one lane per component fits all its hits in
// FP64 in ascending segment order: the algebraic circle fit about the
// centroid, the line of drift z against the unwrapped azimuth, the beam-axis
// crossing and T0.  The arithmetic follows the joining rule and the fit as
// stated in include/tpc.h.
#pragma once

#include "common.hpp"

#define MG_GAP 30.0
#define MG_DZMAX 35.0
#define MG_PERP 0.5
#define MG_DZ 1.0
#define MG_DZ_ARC 0.02
#define MG_SIN 0.1
#define MG_DC_REL 0.2
#define MG_DC_ABS 1e-3
#define MG_C_LINE 1e-4
#define MG_TIE 1e-9
#define MG_ZBIN 36.0  // drift cell (cm), above MG_DZMAX
#define MG_XYBIN 30.5  // bending-plane cell (cm), above MG_GAP with its tie band
#define MG_XY0 260.0   // the cells cover [-MG_XY0, MG_XY0) in x and y (outer radius ~247 cm)
#define MG_NXY 18      // cells per axis: ceil(2 MG_XY0 / MG_XYBIN)
#define MG_FIT 12     // doubles per merged-track fit record

struct MgSegs {  // per segment (track), device SoA
  uint32_t* fs;  // frame * 2 + side, 0xFFFFFFFF = no hits
  uint8_t* sector;
  double *C, *tgl;
  double* e;     // [n * 10]: per end X, Y, z, tx, ty
};

__device__ __forceinline__ uint32_t mg_ur_of(const uint32_t* crow, uint32_t n_ur, uint32_t c) {
  uint32_t lo = 0, hi = n_ur;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (crow[mid] <= c) lo = mid;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ double mg_wrap(double a) {
  while (a > M_PI) a -= 2 * M_PI;
  while (a <= -M_PI) a += 2 * M_PI;
  return a;
}

__device__ __forceinline__ bool mg_cut(double v, double cut, bool& tie) {
  if (fabs(v - cut) <= MG_TIE * cut) tie = true;
  return v <= cut;
}

// Bending-plane cell index of a coordinate (clamped: a pair within MG_GAP
// still falls in neighbouring cells).
__device__ __forceinline__ uint32_t mg_xy_bin(double v) {
  double b = floor((v + MG_XY0) / MG_XYBIN);
  if (!(b >= 0.0)) b = 0.0;
  if (b > MG_NXY - 1) b = MG_NXY - 1;
  return (uint32_t)b;
}

// Per segment: frame-side, curvature, dip and the two ends; per end its cell.
__global__ void k_mg_segments(const uint32_t* __restrict__ crow, uint32_t n_ur,
                              const int32_t* __restrict__ y_fx, const int32_t* __restrict__ z_fx,
                              const uint32_t* n_cl_dev, uint32_t cl_cap,
                              const float* __restrict__ par, const uint8_t* __restrict__ trow,
                              const uint32_t* __restrict__ hit_start,
                              const uint32_t* __restrict__ hits, uint32_t hit_cap,
                              const uint32_t* n_trk_dev, uint32_t trk_cap,
                              const double* __restrict__ cs18, double bz_b, uint32_t nzb,
                              MgSegs S, uint32_t* __restrict__ cell_of_end,
                              uint32_t* __restrict__ cell_cnt, const DevParams* __restrict__ P,
                              const DevStatus* st) {
  if (failed(st)) return;
  const uint32_t n = scan_count(n_trk_dev, trk_cap);
  const uint32_t n_cl = scan_count(n_cl_dev, cl_cap);
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    uint32_t h0 = hit_start[j], h1 = hit_start[j + 1];
    if (h1 > hit_cap) h1 = hit_cap;
    bool ok = h1 > h0;
    uint32_t c0 = 0, c1 = 0;
    if (ok) {
      c0 = hits[h0];
      c1 = hits[h1 - 1];
      ok = c0 < n_cl && c1 < n_cl;
    }
    if (!ok) {
      S.fs[j] = 0xFFFFFFFFu;
      cell_of_end[2 * j] = cell_of_end[2 * j + 1] = 0xFFFFFFFFu;
      continue;
    }
    const uint32_t ur0 = mg_ur_of(crow, n_ur, c0), ur1 = mg_ur_of(crow, n_ur, c1);
    const uint32_t unit = ur0 / NROW, sector = unit % 36;
    const uint32_t fs = (unit / 36) * 2 + sector / 18;
    S.fs[j] = fs;
    S.sector[j] = (uint8_t)sector;
    const double C = -bz_b * (double)par[(size_t)j * 5 + 4];
    S.C[j] = C;
    S.tgl[j] = (double)par[(size_t)j * 5 + 3];
    const double ca = cs18[2 * (sector % 18)], sa = cs18[2 * (sector % 18) + 1];
    const double xp = P->xd[trow[j] < NROW ? trow[j] : 0];
    const double sp = (double)par[(size_t)j * 5 + 2];
    const int rows[2] = {(int)(ur0 % NROW), (int)(ur1 % NROW)};
    const uint32_t cs[2] = {c0, c1};
    for (int e = 0; e < 2; ++e) {
      const double x = P->xd[rows[e]], y = y_fx[cs[e]] / 65536.0;
      double snp = sp + C * (x - xp);
      if (snp > 0.999999) snp = 0.999999;
      if (snp < -0.999999) snp = -0.999999;
      const double cp = sqrt(1.0 - snp * snp);
      double* E = S.e + (size_t)j * 10 + 5 * e;
      E[0] = x * ca - y * sa;
      E[1] = x * sa + y * ca;
      E[2] = z_fx[cs[e]] / 65536.0;
      E[3] = cp * ca - snp * sa;
      E[4] = cp * sa + snp * ca;
      int64_t zb = (int64_t)floor((E[2] + 1.0) / MG_ZBIN);
      if (zb < 0) zb = 0;
      if (zb >= (int64_t)nzb) zb = nzb - 1;
      const uint32_t cell = ((fs * MG_NXY + mg_xy_bin(E[1])) * MG_NXY + mg_xy_bin(E[0])) * nzb +
                            (uint32_t)zb;
      cell_of_end[2 * j + e] = cell;
      atomicAdd(&cell_cnt[cell], 1u);
    }
  }
}

// ends into their cells (any order within a cell: the unions do not depend on it)
__global__ void k_mg_fill_cells(const uint32_t* __restrict__ cell_of_end, const uint32_t* n_trk_dev,
                                uint32_t trk_cap, uint32_t* __restrict__ cursor,
                                uint32_t* __restrict__ cell_ends, const DevStatus* st) {
  if (failed(st)) return;
  const uint32_t n_ends = 2 * scan_count(n_trk_dev, trk_cap);  // only this call's ends
  for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < n_ends; e += gridDim.x * blockDim.x) {
    const uint32_t c = cell_of_end[e];
    if (c == 0xFFFFFFFFu) continue;
    cell_ends[atomicAdd(&cursor[c], 1u)] = e;
  }
}

__device__ __forceinline__ uint32_t mg_find(const uint32_t* parent, uint32_t x) {
  uint32_t p = __atomic_load_n(&parent[x], __ATOMIC_RELAXED);
  while (p != x) {
    x = p;
    p = __atomic_load_n(&parent[x], __ATOMIC_RELAXED);
  }
  return x;
}

__device__ __forceinline__ void mg_union(uint32_t* parent, uint32_t a, uint32_t b) {
  while (true) {
    uint32_t ra = mg_find(parent, a), rb = mg_find(parent, b);
    if (ra == rb) return;
    if (ra < rb) {
      const uint32_t t = ra;
      ra = rb;
      rb = t;
    }
    // hang the larger root under the smaller; retry if it stopped being a root
    if (atomicCAS(&parent[ra], ra, rb) == ra) return;
    a = ra;
    b = rb;
  }
}

// End b seen from end a of a segment with curvature C and dip tgl.
__device__ __forceinline__ bool mg_follows(double C, double tgl, const double* a, const double* b,
                                           bool& tie) {
  const double dx = b[0] - a[0], dy = b[1] - a[1];
  double perp, arc, tx, ty;
  if (fabs(C) >= MG_C_LINE) {
    const double r = 1.0 / C;
    const double cx = a[0] - r * a[4], cy = a[1] + r * a[3];
    const double ux = a[0] - cx, uy = a[1] - cy, vx = b[0] - cx, vy = b[1] - cy;
    const double vr = sqrt(vx * vx + vy * vy);
    perp = fabs(vr - fabs(r));
    const double dpsi = atan2(ux * vy - uy * vx, ux * vx + uy * vy);
    arc = dpsi / C;
    // the tangent where b projects onto the circle (radius vector turned a
    // quarter turn in the sense of the motion)
    tx = C > 0 ? -vy / vr : vy / vr;
    ty = C > 0 ? vx / vr : -vx / vr;
  } else {
    perp = fabs(a[3] * dy - a[4] * dx);
    arc = a[3] * dx + a[4] * dy;
    tx = a[3];
    ty = a[4];
  }
  bool ok = mg_cut(perp, MG_PERP, tie);
  ok &= mg_cut(fabs(arc), MG_GAP, tie);
  ok &= mg_cut(fabs(b[2] - a[2] - tgl * arc), MG_DZ + MG_DZ_ARC * fabs(arc), tie);
  ok &= mg_cut(fabs(tx * b[4] - ty * b[3]), MG_SIN, tie);
  return ok;
}

// The drift z and bending-plane position of every end, in cell order, so
// that the candidate scans below read consecutive memory.
__global__ void k_mg_pack(const uint32_t* __restrict__ cell_ends, const uint32_t* total_dev,
                          const double* __restrict__ e_all, double* __restrict__ pk,
                          const DevStatus* st) {
  if (failed(st)) return;
  const uint32_t total = *total_dev;
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < total; k += gridDim.x * blockDim.x) {
    const uint32_t e = cell_ends[k];
    const double* E = e_all + (size_t)(e >> 1) * 10 + 5 * (e & 1);
    pk[3 * (size_t)k] = E[2];
    pk[3 * (size_t)k + 1] = E[0];
    pk[3 * (size_t)k + 2] = E[1];
  }
}

// The joining test of end t (cell order) against candidate end k: the
// remaining gates and cuts, then the union; near ties flag both segments.
__device__ __forceinline__ void mg_pair_check(const MgSegs& S, const uint32_t* cell_ends,
                                              const double* pk, uint32_t t, uint32_t k,
                                              uint32_t* parent, uint8_t* near_tie) {
  const uint32_t e = cell_ends[t], f = cell_ends[k];
  const uint32_t A = e >> 1, B = f >> 1;
  const double* a = S.e + (size_t)A * 10 + 5 * (e & 1);
  const double* b = S.e + (size_t)B * 10 + 5 * (f & 1);
  const double ax = pk[3 * (size_t)t + 1], ay = pk[3 * (size_t)t + 2];
  const double bx = pk[3 * (size_t)k + 1], by = pk[3 * (size_t)k + 2];
  const double dxy = sqrt((ax - bx) * (ax - bx) + (ay - by) * (ay - by));
  const double CA = S.C[A], CB = S.C[B], ca = fabs(CA), cb = fabs(CB), cm = ca > cb ? ca : cb;
  bool tie = false;
  bool ok = mg_cut(dxy, MG_GAP, tie);
  if (ok) {
    ok = mg_cut(fabs(ca - cb), MG_DC_REL * cm + MG_DC_ABS, tie);
    ok &= mg_follows(CA, S.tgl[A], a, b, tie);
    ok &= mg_follows(CB, S.tgl[B], b, a, tie);
  }
  if (tie) {
    near_tie[A] = 1;
    near_tie[B] = 1;
  }
  if (ok) mg_union(parent, A, B);
}

// One lane per end, ends taken in cell order (the lanes of a wave mostly
// share their cells and so scan the same neighbour cells in step): the ends of
// later segments in the 3 x 3 x 3 cells around it (nine runs of three
// consecutive drift cells) are gated on the packed drift z and position; the
// pairs that pass go to the wave's queue in LDS, and every
// 64 of them are tested by the 64 lanes together (the full test is long and
// few lanes pass a gate at a time).
#define MG_QCAP 128
__global__ __launch_bounds__(256) void k_mg_pairs(MgSegs S, uint32_t nzb,
                                                  const uint32_t* total_dev,
                                                  const uint32_t* __restrict__ cell_off,
                                                  const uint32_t* __restrict__ cell_ends,
                                                  const uint32_t* __restrict__ cell_of_end,
                                                  const double* __restrict__ pk,
                                                  uint32_t* __restrict__ parent,
                                                  uint8_t* __restrict__ near_tie,
                                                  const DevStatus* st) {
  __shared__ uint32_t qa[4][MG_QCAP], qb[4][MG_QCAP];
  if (failed(st)) return;
  const uint32_t total = *total_dev;
  const uint32_t w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint64_t below = (1ull << lane) - 1ull;
  for (uint32_t t0 = blockIdx.x * blockDim.x + w * 64; t0 < total;
       t0 += gridDim.x * blockDim.x) {  // uniform per wave
    const uint32_t t = t0 + lane;
    const bool have = t < total;
    uint32_t A = 0, zb = 0, ix = 0, iy = 0, fs = 0;
    double az = 0, ax = 0, ay = 0;
    if (have) {
      const uint32_t e = cell_ends[t];
      A = e >> 1;
      const uint32_t cell = cell_of_end[e];
      zb = cell % nzb;
      ix = (cell / nzb) % MG_NXY;
      iy = (cell / nzb / MG_NXY) % MG_NXY;
      fs = cell / nzb / MG_NXY / MG_NXY;
      az = pk[3 * (size_t)t];
      ax = pk[3 * (size_t)t + 1];
      ay = pk[3 * (size_t)t + 2];
    }
    uint32_t qn = 0;  // queued pairs (the same in every lane)
    for (int ci = 0; ci < 9; ++ci) {
      const int dy = ci / 3 - 1, dx = ci % 3 - 1;
      uint32_t k0 = 0, k1 = 0;
      const int x2 = (int)ix + dx, y2 = (int)iy + dy;
      if (have && x2 >= 0 && x2 < MG_NXY && y2 >= 0 && y2 < MG_NXY) {
        // the drift cells zb - 1, zb, zb + 1 (those that exist) of a
        // neighbouring (x, y) cell are consecutive cells: their ends form one
        // run, taken in the same order as cell by cell
        const uint32_t cb = ((fs * MG_NXY + (uint32_t)y2) * MG_NXY + (uint32_t)x2) * nzb;
        const uint32_t zlo = zb > 0 ? zb - 1 : 0, zhi = zb + 1 < nzb ? zb + 1 : nzb - 1;
        k0 = cell_off[cb + zlo];
        k1 = cell_off[cb + zhi + 1];
      }
      const uint32_t len = k1 - k0;
      const uint32_t maxlen = (uint32_t)wave_max_i32((int32_t)len);
      // each candidate's gate data is loaded one candidate ahead of its test
      double bz_next = 0.0, bx_next = 0.0, by_next = 0.0;
      if (len > 0) {
        bz_next = pk[3 * (size_t)k0];
        bx_next = pk[3 * (size_t)k0 + 1];
        by_next = pk[3 * (size_t)k0 + 2];
      }
      for (uint32_t it = 0; it < maxlen; ++it) {
        bool pass = false;
        const uint32_t k = k0 + it;
        const double bz = bz_next, bx = bx_next, by = by_next;
        if (it + 1 < len) {
          bz_next = pk[3 * (size_t)(k + 1)];
          bx_next = pk[3 * (size_t)(k + 1) + 1];
          by_next = pk[3 * (size_t)(k + 1) + 2];
        }
        if (it < len) {
          if (fabs(az - bz) <= MG_DZMAX) {
            const double d2 = (ax - bx) * (ax - bx) + (ay - by) * (ay - by);
            // beyond the near-tie band of the gap cut nothing can pass or tie
            // (squared distances: the band's margin of 2e-9 dwarfs the rounding)
            constexpr double g = MG_GAP * (1 + 2 * MG_TIE);
            pass = d2 <= g * g && (cell_ends[k] >> 1) > A;
          }
        }
        const uint64_t m = __ballot(pass);
        if (m) {  // uniform
          const uint32_t pos = qn + (uint32_t)__popcll(m & below);
          if (pass) {
            qa[w][pos] = t;
            qb[w][pos] = k;
          }
          qn += (uint32_t)__popcll(m);
          if (qn >= 64) {  // uniform: the 64 newest pairs, one per lane
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            const uint32_t q = qn - 64 + lane;
            mg_pair_check(S, cell_ends, pk, qa[w][q], qb[w][q], parent, near_tie);
            qn -= 64;
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
          }
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (lane < qn) mg_pair_check(S, cell_ends, pk, qa[w][lane], qb[w][lane], parent, near_tie);
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// Global position of every hit of every track (the fit reads it three times):
// one thread per hit, its cluster's (unit,row) found by a binary search of the
// row starts (one lane per track walking its hits took 0.68 ms on a 2 ms
// Pb-Pb slice, the longest tracks setting the pace; per hit: 0.21 ms).
__global__ void k_mg_hits(const uint32_t* __restrict__ crow, uint32_t n_ur,
                          const int32_t* __restrict__ y_fx, const uint32_t* n_cl_dev,
                          uint32_t cl_cap, const uint32_t* __restrict__ hit_start,
                          const uint32_t* __restrict__ hits, uint32_t hit_cap,
                          const uint32_t* n_trk_dev, uint32_t trk_cap,
                          const double* __restrict__ cs18, double* __restrict__ hxy,
                          const DevParams* __restrict__ P, const DevStatus* st) {
  if (failed(st)) return;
  const uint32_t n = scan_count(n_trk_dev, trk_cap);
  const uint32_t n_cl = scan_count(n_cl_dev, cl_cap);
  uint32_t nh = n ? hit_start[n] : 0;  // the tracks' hits are [0, hit_start[n])
  if (nh > hit_cap) nh = hit_cap;
  for (uint32_t h = blockIdx.x * blockDim.x + threadIdx.x; h < nh; h += gridDim.x * blockDim.x) {
    const uint32_t c = hits[h] < n_cl ? hits[h] : 0;
    const uint32_t ur = mg_ur_of(crow, n_ur, c);
    const uint32_t s18 = (ur / NROW) % 36 % 18;
    const double ca = cs18[2 * s18], sa = cs18[2 * s18 + 1];
    const double x = P->xd[ur % NROW], y = y_fx[c] / 65536.0;
    hxy[2 * (size_t)h] = x * ca - y * sa;
    hxy[2 * (size_t)h + 1] = x * sa + y * ca;
  }
}

__global__ void k_mg_init(uint32_t* __restrict__ parent, uint8_t* __restrict__ near_tie,
                          uint32_t* __restrict__ idx, uint32_t cap, const DevStatus* st) {
  if (failed(st)) return;
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < cap; j += gridDim.x * blockDim.x) {
    parent[j] = j;
    near_tie[j] = 0;
    idx[j] = j;
  }
}

// label = the root; also counts the components (roots) by a reduction's input
__global__ void k_mg_labels(const uint32_t* __restrict__ parent, const uint32_t* n_trk_dev,
                            uint32_t trk_cap, int32_t* __restrict__ label,
                            uint32_t* __restrict__ key, const DevStatus* st) {
  if (failed(st)) return;
  const uint32_t n = scan_count(n_trk_dev, trk_cap);
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < trk_cap; j += gridDim.x * blockDim.x) {
    if (j < n) {
      const uint32_t r = mg_find(parent, j);
      label[j] = (int32_t)r;
      key[j] = r;
    } else {
      key[j] = 0xFFFFFFFFu;  // beyond the tracks: sorted to the end
    }
  }
}

// One lane per component (the first of its run in the sorted members): the
// FP64 helix fit of all its hits, members in ascending index.
__global__ __launch_bounds__(64) void k_mg_fit(const uint32_t* __restrict__ skey,
                                               const uint32_t* __restrict__ sidx,
                                               const uint32_t* n_trk_dev, uint32_t trk_cap,
                                               const int32_t* __restrict__ z_fx,
                                               const uint32_t* __restrict__ hit_start,
                                               const uint32_t* __restrict__ hits,
                                               uint32_t hit_cap, const double* __restrict__ hxy,
                                               double* __restrict__ fit, const DevStatus* st) {
  if (failed(st)) return;
  const uint32_t n = scan_count(n_trk_dev, trk_cap);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t root = skey[i];
    if (i > 0 && skey[i - 1] == root) continue;
    uint32_t end = i + 1;
    while (end < n && skey[end] == root) ++end;
    double* f = fit + (size_t)root * MG_FIT;
    for (int k = 0; k < MG_FIT; ++k) f[k] = 0;
    // global position of hit h (computed by k_mg_hits)
    auto hit_xy = [&](uint32_t h, double& X, double& Y) {
      X = hxy[2 * (size_t)h];
      Y = hxy[2 * (size_t)h + 1];
    };
    auto hit_range = [&](uint32_t j, uint32_t& h0, uint32_t& h1) {
      h0 = hit_start[j];
      h1 = hit_start[j + 1];
      if (h1 > hit_cap) h1 = hit_cap;
      if (h0 > h1) h0 = h1;
    };
    // every pass loads the next hit's data one hit ahead of its use (same
    // order of the sums)
    double sx = 0, sy = 0;
    int64_t nh = 0;
    for (uint32_t m = i; m < end; ++m) {
      uint32_t h0, h1;
      hit_range(sidx[m], h0, h1);
      double Xn = 0, Yn = 0;
      if (h0 < h1) hit_xy(h0, Xn, Yn);
      for (uint32_t h = h0; h < h1; ++h) {
        const double X = Xn, Y = Yn;
        if (h + 1 < h1) hit_xy(h + 1, Xn, Yn);
        sx += X;
        sy += Y;
        ++nh;
      }
    }
    f[0] = (double)(end - i);
    f[1] = (double)nh;
    const double mx = nh ? sx / nh : 0, my = nh ? sy / nh : 0;
    double suu = 0, svv = 0, suv = 0, suuu = 0, svvv = 0, suvv = 0, svuu = 0;
    for (uint32_t m = i; m < end; ++m) {
      uint32_t h0, h1;
      hit_range(sidx[m], h0, h1);
      double Xn = 0, Yn = 0;
      if (h0 < h1) hit_xy(h0, Xn, Yn);
      for (uint32_t h = h0; h < h1; ++h) {
        const double X = Xn, Y = Yn;
        if (h + 1 < h1) hit_xy(h + 1, Xn, Yn);
        const double u = X - mx, v = Y - my;
        suu += u * u;
        svv += v * v;
        suv += u * v;
        suuu += u * u * u;
        svvv += v * v * v;
        suvv += u * v * v;
        svuu += v * u * u;
      }
    }
    const double det = suu * svv - suv * suv;
    if (nh < 3 || !(fabs(det) > 0)) continue;
    const double b1 = 0.5 * (suuu + suvv), b2 = 0.5 * (svvv + svuu);
    const double uc = (b1 * svv - b2 * suv) / det, vc = (suu * b2 - suv * b1) / det;
    const double xc = mx + uc, yc = my + vc;
    f[2] = xc;
    f[3] = yc;
    f[4] = sqrt(uc * uc + vc * vc + (suu + svv) / nh);
    f[9] = 1;
    double psi_prev = 0, acc = 0, sp = 0, sp2 = 0, sz = 0, szp = 0, pmin = 0, pmax = 0;
    int64_t k = 0;
    for (uint32_t m = i; m < end; ++m) {
      uint32_t h0, h1;
      hit_range(sidx[m], h0, h1);
      double Xn = 0, Yn = 0;
      int32_t zn = 0;
      if (h0 < h1) {
        hit_xy(h0, Xn, Yn);
        zn = z_fx[hits[h0]];
      }
      for (uint32_t h = h0; h < h1; ++h) {
        const double X = Xn, Y = Yn;
        const int32_t zq = zn;
        if (h + 1 < h1) {
          hit_xy(h + 1, Xn, Yn);
          zn = z_fx[hits[h + 1]];
        }
        const double psi = atan2(Y - yc, X - xc);
        acc = k == 0 ? 0.0 : acc + mg_wrap(psi - psi_prev);
        psi_prev = psi;
        const double z = zq / 65536.0;
        sp += acc;
        sp2 += acc * acc;
        sz += z;
        szp += z * acc;
        if (k == 0 || acc < pmin) pmin = acc;
        if (k == 0 || acc > pmax) pmax = acc;
        ++k;
      }
    }
    const double dd = k * sp2 - sp * sp;
    if (!(dd > 0)) continue;
    const double slope = (k * szp - sp * sz) / dd, icpt = (sz - slope * sp) / k;
    f[5] = slope;
    f[8] = fabs(slope) / f[4];
    f[10] = pmax - pmin;
    if (pmax - pmin < 2 * M_PI) {
      const double psi0 = atan2(-yc, -xc);
      double a = acc + mg_wrap(psi0 - psi_prev);
      if (slope >= 0) {
        while (a < pmax) a += 2 * M_PI;
        while (a - 2 * M_PI >= pmax) a -= 2 * M_PI;
      } else {
        while (a > pmin) a -= 2 * M_PI;
        while (a + 2 * M_PI <= pmin) a += 2 * M_PI;
      }
      const double zd0 = icpt + slope * a;
      f[6] = zd0;
      f[7] = 2.0 * (zd0 - 250.0);
      f[9] = 3;
    }
  }
}

// The cell table's closing entry (the scan's total).
__global__ void k_mg_total(uint32_t* __restrict__ off, const uint32_t* total, uint32_t n_cells,
                           const DevStatus* st) {
  if (failed(st)) return;
  off[n_cells] = *total;
}

// One pass of a stable least-significant-digit radix sort of (key, value)
// pairs on the 8-bit digit at `shift`: the count step writes, per block of
// MG_SORT_BLOCK elements, the count of each digit to bins[digit * nb + block];
// after an exclusive scan of bins, the scatter step places each element at
// its digit's position, ranking equal digits in index order (a wave's lanes
// by ballot, the waves of a block one after the other).  Three passes order
// keys below 2^24 with equal keys in index order.
#define MG_SORT_BLOCK 1024
template <bool SCATTER>
__global__ __launch_bounds__(256) void k_mg_rsort(const uint32_t* __restrict__ kin,
                                                  const uint32_t* __restrict__ vin,
                                                  const uint32_t* n_dev, uint32_t cap, int shift,
                                                  uint32_t* __restrict__ bins,
                                                  uint32_t* __restrict__ kout,
                                                  uint32_t* __restrict__ vout,
                                                  const DevStatus* st) {
  if (failed(st)) return;
  __shared__ uint32_t h[4][256];
  const uint32_t n = scan_count(n_dev, cap);
  const uint32_t nb = (n + MG_SORT_BLOCK - 1) / MG_SORT_BLOCK;
  if (blockIdx.x >= nb) return;  // uniform per workgroup
  const uint32_t b0 = blockIdx.x * MG_SORT_BLOCK;
  const uint32_t m = min((uint32_t)MG_SORT_BLOCK, n - b0);
  const uint32_t w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < 4; ++j) h[j][threadIdx.x] = 0;
  __syncthreads();
  uint32_t dig[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t i = 256u * w + 64u * j + lane;
    dig[j] = i < m ? (kin[b0 + i] >> shift) & 255u : 0u;
    if (i < m) atomicAdd(&h[w][dig[j]], 1u);
  }
  __syncthreads();
  const uint32_t d = threadIdx.x;
  const uint32_t c0 = h[0][d], c1 = h[1][d], c2 = h[2][d], c3 = h[3][d];
  const size_t bi = (size_t)d * nb + blockIdx.x;
  if (!SCATTER) {
    bins[bi] = c0 + c1 + c2 + c3;
    return;
  }
  const uint32_t base = bins[bi];
  __syncthreads();
  h[0][d] = base;
  h[1][d] = base + c0;
  h[2][d] = base + c0 + c1;
  h[3][d] = base + c0 + c1 + c2;
  __syncthreads();
  const uint64_t below = (1ull << lane) - 1ull;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t i = 256u * w + 64u * j + lane;
    const bool v = i < m;
    uint64_t eq = __ballot(v);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool on = (dig[j] >> bit) & 1u;
      const uint64_t bb = __ballot(on);
      eq &= on ? bb : ~bb;
    }
    if (v) {
      const uint32_t pos = h[w][dig[j]] + (uint32_t)__popcll(eq & below);
      kout[pos] = kin[b0 + i];
      vout[pos] = vin[b0 + i];
    }
    // the highest lane of each digit advances the digit's position
    if (v && (eq >> lane) == 1ull) h[w][dig[j]] += (uint32_t)__popcll(eq);
  }
}

struct MgIsRoot {
  const int32_t* label;
  __device__ uint32_t operator()(uint32_t j) const { return label[j] == (int32_t)j ? 1u : 0u; }
};
