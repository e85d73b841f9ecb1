// Kalman track following, conflict resolution, refit and output.
//
// One tracklet per lane.  The state is (y, z - z_anchor, sin phi, tan lambda,
// q/pT) at the local x of a pad row; z is kept relative to the tracklet's
// first cluster so that FP32 keeps full precision in long time frames.  The
// covariance is a packed 5x5 upper triangle in registers.  Propagation is
// the exact helix in a uniform Bz field (no material, no process noise).
#pragma once

#include <type_traits>

#include "common.hpp"
#include "k_cluster.hpp"
#include "k_links.hpp"

#define FX_SCALE 1.52587890625e-05  // 2^-16

enum { TF_NOT_PD = 1, TF_REFIT_FAIL = 2, TF_FP64 = 4, TF_FP64_FAIL = 8, TF_TO_FP64 = 16 };

template <typename T>
struct Trk {
  T p[5];
  T c[15];
};

__device__ __forceinline__ constexpr int PI(int i, int j) {  // i <= j
  return i * 5 - i * (i - 1) / 2 + (j - i);
}

template <typename T>
__device__ __forceinline__ T cov(const T* c, int i, int j) {
  return i <= j ? c[PI(i, j)] : c[PI(j, i)];
}

// per-precision views of the parameter block
template <typename T>
struct PV;
template <>
struct PV<float> {
  const DevParams32* P;
  __device__ float x(int r) const { return P->x[r]; }
  __device__ float hw(int r) const { return P->hw[r]; }
  __device__ float vy(int r) const { return P->vy[r]; }
  __device__ float vz(int r) const { return P->vz[r]; }
  __device__ float chi2_max() const { return P->chi2_max; }
  __device__ float snp_max() const { return P->snp_max; }
  __device__ float b() const { return P->bz_b; }
  __device__ float c0_snp2() const { return P->c0_snp2; }
  __device__ float c0_tgl2() const { return P->c0_tgl2; }
  __device__ float c0_qpt2() const { return P->c0_qpt2; }
  __device__ float qpt_clamp() const { return P->qpt_clamp; }
  __device__ float edge_margin() const { return P->edge_margin; }
  __device__ float refit_snp_max() const { return P->refit_snp_max; }
  __device__ float c0r(int i) const { return P->c0r2[i]; }
};
template <>
struct PV<double> {
  const DevParams* P;
  __device__ double x(int r) const { return P->xd[r]; }
  __device__ double hw(int r) const { return P->hwd[r]; }
  __device__ double vy(int r) const { return P->vyd[r]; }
  __device__ double vz(int r) const { return P->vzd[r]; }
  __device__ double chi2_max() const { return P->chi2_max_d; }
  __device__ double snp_max() const { return P->snp_max_d; }
  __device__ double b() const { return P->bz_b_d; }
  __device__ double c0_snp2() const { return P->c0_snp2_d; }
  __device__ double c0_tgl2() const { return P->c0_tgl2_d; }
  __device__ double c0_qpt2() const { return P->c0_qpt2_d; }
  __device__ double qpt_clamp() const { return P->qpt_clamp_d; }
  __device__ double edge_margin() const { return P->edge_margin_d; }
  __device__ double refit_snp_max() const { return P->refit_snp_max_d; }
  __device__ double c0r(int i) const { return P->c0r2_d[i]; }
};

// Low-order parts of y and sin phi carried beside an FP32 state.  Over many
// rows a stiff track adds almost the same increment C dx to sin phi at every
// step, so FP32 rounding errs the same way each time and the sum drifts like
// a curvature offset of about ulp(sin phi) / dx; adding each increment with
// an error-free two-sum and keeping the rounding error removes the drift.
template <typename T>
struct LoParts {
  T y, s;
};

// a + b = hi + lo exactly (two-sum); lo accumulates into *acc
template <typename T>
__device__ __forceinline__ T two_sum_acc(T a, T b, T* acc) {
  const T b2 = b + *acc;
  const T hi = a + b2;
  const T bb = hi - a;
  *acc = (a - (hi - bb)) + (b2 - bb);
  return hi;
}

// exact row-to-row distance from the integer radii
template <typename T>
__device__ __forceinline__ T row_dx(const DevParams32* P, int r1, int r2) {
  return (T)(P->xfx[r2] - P->xfx[r1]) * (T)FX_SCALE;
}

// d(signed arc)/dC at fixed dx: integral over u in [0, dx] of
// u * s / (1 - s^2)^(3/2), s = s1 + C u, by 8-point Gauss-Legendre.
template <typename T>
__device__ __forceinline__ T darc_dc(T s1, T C, T dx) {
  const T X[8] = {(T)0.01985507175123188, (T)0.10166676129318664, (T)0.2372337950418355,
                  (T)0.4082826787521751,  (T)0.5917173212478249,  (T)0.7627662049581645,
                  (T)0.8983332387068134,  (T)0.9801449282487681};
  const T Wt[8] = {(T)0.05061426814518813, (T)0.11119051722668724, (T)0.15685332293894363,
                   (T)0.18134189168918100, (T)0.18134189168918100, (T)0.15685332293894363,
                   (T)0.11119051722668724, (T)0.05061426814518813};
  T acc = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const T s = s1 + C * dx * X[i];
    const T w = (T)1 - s * s;
    acc += Wt[i] * X[i] * s / (w * sqrt(w));
  }
  return acc * dx * dx;
}

// FP32: the same quadrature with w^(-3/2) from the hardware reciprocal square
// root (a Jacobian element: a few ulp are far below what the fit resolves).
template <>
__device__ __forceinline__ float darc_dc<float>(float s1, float C, float dx) {
  const float Cdx = C * dx;
  const float X[8] = {0.01985507175123188f, 0.10166676129318664f, 0.2372337950418355f,
                      0.4082826787521751f,  0.5917173212478249f,  0.7627662049581645f,
                      0.8983332387068134f,  0.9801449282487681f};
  const float Wt[8] = {0.05061426814518813f, 0.11119051722668724f, 0.15685332293894363f,
                       0.18134189168918100f, 0.18134189168918100f, 0.15685332293894363f,
                       0.11119051722668724f, 0.05061426814518813f};
  float acc = 0.0f;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const float s = s1 + Cdx * X[i];
    const float r = __builtin_amdgcn_rsqf(1.0f - s * s);
    acc += (Wt[i] * X[i]) * s * (r * r * r);
  }
  return acc * dx * dx;
}

// Off-diagonal elements of the helix Jacobian d(state after)/d(state before)
// over one step.  Every other element is that of the identity: the Jacobian
// is unit upper triangular in (y, z, sin phi, tan lambda, q/pT).
template <typename T>
struct HJac {
  T j02, j04, j12, j13, j14, j24;
};

// Helix step of the state over dx; with J also the Jacobian.  Returns false
// (state untouched) if |sin phi| would reach snp_lim.
template <typename T>
__device__ __forceinline__ bool helix_step(T p[5], T dx, const PV<T>& pv, T snp_lim,
                                           LoParts<T>* lo, HJac<T>* J) {
  const T b = pv.b();
  const T C = -b * p[4];
  const T s1 = p[2];
  T slo = lo ? lo->s : (T)0;
  const T s2 = lo ? two_sum_acc(s1, C * dx, &slo) : s1 + C * dx;
  if (!(fabs(s2) < snp_lim)) return false;
  T c1, c2, ic1, ic2, iD, f, chord, L;
  const T N = s1 + s2;
  if constexpr (std::is_same<T, float>::value) {
    // FP32: hardware reciprocal and reciprocal square root (about 1 ulp)
    // instead of correctly rounded division and square root, and the series
    // of asin(h)/h for the small turning angles of one row step
    ic1 = __builtin_amdgcn_rsqf(1.0f - s1 * s1);
    ic2 = __builtin_amdgcn_rsqf(1.0f - s2 * s2);
    c1 = (1.0f - s1 * s1) * ic1;
    c2 = (1.0f - s2 * s2) * ic2;
    iD = __builtin_amdgcn_rcpf(c1 + c2);
    f = N * iD;
    const float q = 1.0f + f * f;
    chord = fabsf(dx) * (q * __builtin_amdgcn_rsqf(q));
    float h = chord * fabsf(C) * 0.5f;
    if (h > 1.0f) h = 1.0f;
    if (h < 0.1f) {
      const float h2 = h * h;
      L = chord * (1.0f + h2 * (1.0f / 6.0f + h2 * (3.0f / 40.0f + h2 * (5.0f / 112.0f +
                                                                         h2 * (35.0f / 1152.0f)))));
    } else {
      L = chord * asinf(h) / h;
    }
  } else {
    c1 = sqrt((T)1 - s1 * s1);
    c2 = sqrt((T)1 - s2 * s2);
    ic1 = (T)1 / c1;
    ic2 = (T)1 / c2;
    iD = (T)1 / (c1 + c2);
    f = N * iD;
    chord = fabs(dx) * sqrt((T)1 + f * f);
    T h = chord * fabs(C) * (T)0.5;
    if (h > (T)1) h = (T)1;
    L = h > (T)0 ? chord * asin(h) / h : chord;
  }
  const T D = c1 + c2;
  const T A = dx >= (T)0 ? L : -L;
  if (J) {
    const T iD2 = iD * iD;
    J->j02 = dx * ((T)2 * D + N * (s1 * ic1 + s2 * ic2)) * iD2;
    J->j04 = -b * dx * dx * (D + N * s2 * ic2) * iD2;
    J->j12 = p[3] * dx * N * (ic1 * ic2 * iD);
    J->j13 = A;
    J->j14 = -b * p[3] * darc_dc(s1, C, dx);
    J->j24 = -b * dx;
  }
  if (lo) {
    p[0] = two_sum_acc(p[0], dx * f, &lo->y);
    lo->s = slo;
  } else {
    p[0] += dx * f;
  }
  p[1] += p[3] * A;
  p[2] = s2;
  return true;
}

// Helix propagation over dx; with_cov also transports the covariance,
// C <- J C J^T.  Returns false (state untouched) if |sin phi| would reach
// snp_lim.
template <typename T>
__device__ __forceinline__ bool propagate(Trk<T>& k, T dx, const PV<T>& pv, bool with_cov,
                                          T snp_lim, LoParts<T>* lo = nullptr) {
  HJac<T> J;
  if (!helix_step(k.p, dx, pv, snp_lim, lo, with_cov ? &J : nullptr)) return false;
  if (with_cov) {
    const T j02 = J.j02, j04 = J.j04, j12 = J.j12, j13 = J.j13, j14 = J.j14, j24 = J.j24;
    T m[5][5];
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
      for (int j = 0; j < 5; ++j) m[i][j] = cov(k.c, i, j);
    T t[5][5];  // J * M
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      t[0][j] = m[0][j] + j02 * m[2][j] + j04 * m[4][j];
      t[1][j] = m[1][j] + j12 * m[2][j] + j13 * m[3][j] + j14 * m[4][j];
      t[2][j] = m[2][j] + j24 * m[4][j];
      t[3][j] = m[3][j];
      t[4][j] = m[4][j];
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) {  // (J M) J^T, upper triangle
      const T col[5] = {t[i][0] + j02 * t[i][2] + j04 * t[i][4],
                        t[i][1] + j12 * t[i][2] + j13 * t[i][3] + j14 * t[i][4],
                        t[i][2] + j24 * t[i][4], t[i][3], t[i][4]};
#pragma unroll
      for (int j = i; j < 5; ++j) k.c[PI(i, j)] = col[j];
    }
  }
  return true;
}

// inverse of the residual covariance S = C_yz + V, once per row
template <typename T>
struct SInv {
  T i00, i01, i11;
};
template <typename T>
__device__ __forceinline__ SInv<T> s_inverse(const Trk<T>& k, T vy, T vz) {
  const T S00 = k.c[0] + vy, S01 = k.c[1], S11 = k.c[5] + vz;
  const T rd = (T)1 / (S00 * S11 - S01 * S01);
  return SInv<T>{S11 * rd, -S01 * rd, S00 * rd};
}

template <typename T>
__device__ __forceinline__ T chi2_of(const Trk<T>& k, T my, T mz, const SInv<T>& si) {
  const T r0 = my - k.p[0], r1 = mz - k.p[1];
  return r0 * r0 * si.i00 + (T)2 * r0 * r1 * si.i01 + r1 * r1 * si.i11;
}

// Kalman update with a (y, z) measurement.  Returns false (state untouched)
// if |sin phi| >= 1 afterwards.
template <typename T>
__device__ __forceinline__ bool update(Trk<T>& k, T my, T mz, T vy, T vz, T* chi2) {
  const T r0 = my - k.p[0], r1 = mz - k.p[1];
  const SInv<T> si = s_inverse(k, vy, vz);
  const T I00 = si.i00, I01 = si.i01, I11 = si.i11;
  if (chi2) *chi2 = r0 * r0 * I00 + (T)2 * r0 * r1 * I01 + r1 * r1 * I11;
  T K0[5], K1[5], c0[5], c1v[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    c0[i] = cov(k.c, 0, i);
    c1v[i] = cov(k.c, 1, i);
    K0[i] = c0[i] * I00 + c1v[i] * I01;
    K1[i] = c0[i] * I01 + c1v[i] * I11;
  }
  const T np2 = k.p[2] + K0[2] * r0 + K1[2] * r1;
  if (!(fabs(np2) < (T)1)) return false;
#pragma unroll
  for (int i = 0; i < 5; ++i) k.p[i] += K0[i] * r0 + K1[i] * r1;
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = i; j < 5; ++j) k.c[PI(i, j)] -= K0[i] * c0[j] + K1[i] * c1v[j];
  return true;
}

template <typename T>
__device__ __forceinline__ void c0_reset(Trk<T>& k, const PV<T>& pv, int r) {
#pragma unroll
  for (int i = 0; i < 15; ++i) k.c[i] = 0;
  k.c[PI(0, 0)] = pv.vy(r);
  k.c[PI(1, 1)] = pv.vz(r);
  k.c[PI(2, 2)] = pv.c0_snp2();
  k.c[PI(3, 3)] = pv.c0_tgl2();
  k.c[PI(4, 4)] = pv.c0_qpt2();
}

// unit-row of a cluster: the last ur with crow[ur] <= c
__device__ __forceinline__ uint32_t cluster_ur(const uint32_t* crow, uint32_t n_ur, uint32_t c) {
  uint32_t a = 0, b = n_ur;
  while (b - a > 1) {
    const uint32_t m = (a + b) >> 1;
    if (crow[m] <= c) a = m;
    else b = m;
  }
  return a;
}

struct FollowOut {
  int32_t* hits;      // [cap*152], rows [lo, hi] written
  float* state;       // [cap*6]: pass-B state + its row
  uint16_t* nhits;    // [cap]
  uint16_t* range;    // [cap]: lo | hi << 8
  uint8_t* ok;        // [cap]
  uint8_t* krow;      // [cap*152]: rows of the kept hits, ascending (after resolution)
};

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Raw buffer resource over a device array (uniform base, no range limit:
// callers read inside the array; word 3 = 32-bit data format).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)0xFFFFFFFF,
                                           0x00020000);
}

// Best candidate of row ur for the track state k: the cluster with the least
// chi2 within the cut, the lower index on ties (-1 if none).  Only the grid
// blocks within the z residual bound that chi2 alone sets (plus a margin) are
// scanned; bq receives the chosen cluster's position.
__device__ __forceinline__ int32_t search_row(const ClusterView& cl, const uint32_t* cblk,
                                              uint32_t nblk, uint32_t ur, const Trk<float>& k,
                                              int32_t anchor, float vy, float vz, float chi2max,
                                              uint32_t& n_cand, int2& bq) {
  const float w = sqrtf(chi2max * (k.c[5] + vz));
  const float zabs = k.p[1] + (float)anchor * (float)FX_SCALE;
  const float flo = floorf(2.0f * (zabs - w)) - 3.0f, fhi = ceilf(2.0f * (zabs + w)) + 3.0f;
  // NaN or out-of-range windows collapse to an empty or clamped block range
  int32_t blo = flo > 0.0f ? (flo < 1.0e6f ? ((int32_t)flo >> CG_BSHIFT) : (int32_t)nblk) : 0;
  int32_t bhi = fhi >= 0.0f ? (fhi < 1.0e6f ? ((int32_t)fhi >> CG_BSHIFT) : (int32_t)nblk - 1) : -1;
  if (!(fhi >= 0.0f) || !(flo == flo)) bhi = -1;
  if (blo > (int32_t)nblk - 1) blo = nblk - 1;
  if (bhi > (int32_t)nblk - 1) bhi = nblk - 1;
  // Every load below is a cache line of its own per lane, and the following
  // is bound by their number: the row bounds come in one 8-byte load, the two
  // grid entries in one 16-byte load when the range spans at most 3 blocks,
  // the candidates two per 16-byte load.  Same clamps as row_range.
  // (buffer loads: the compiler keeps them whole; every read lies inside the
  // arrays, the row's own table included)
  const u32x2 rb = __builtin_amdgcn_raw_buffer_load_b64(buffer_of(cl.crow), (int)(ur * 4u), 0, 0);
  const uint32_t cap = cl.capacity;
  const uint32_t s0 = rb.x < cap ? rb.x : cap, s1 = rb.y < cap ? rb.y : cap;
  int32_t ilo = blo < 0 ? 0 : blo, ihi = bhi + 1 > (int32_t)nblk ? (int32_t)nblk : bhi + 1;
  if (ihi < ilo) ihi = ilo;
  const size_t rowe = (size_t)ur * (nblk + 1);
  uint32_t a, b;
  if (ihi - ilo <= 3 && ilo + 3 <= (int32_t)nblk) {
    const u32x4 e = __builtin_amdgcn_raw_buffer_load_b128(buffer_of(cblk), (int)((rowe + ilo) * 4u),
                                                          0, 0);
    const int d = ihi - ilo;
    a = e.x;
    b = d == 0 ? e.x : d == 1 ? e.y : d == 2 ? e.z : e.w;
  } else {
    a = cblk[rowe + ilo];
    b = cblk[rowe + ihi];
  }
  if (a < s0) a = s0;
  if (a > s1) a = s1;
  if (b < a) b = a;
  if (b > s1) b = s1;
  int32_t best = -1;
  float bchi = 0.0f;
  const SInv<float> si = s_inverse(k, vy, vz);
  n_cand += b - a;
  // candidates in index order, two at a time (both loads of a pair in flight)
  for (uint32_t c0 = a; c0 < b; c0 += 2) {
    int2 q[2];
    if (c0 + 1 < b) {
      const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(buffer_of(cl.pos), (int)(c0 * 8u), 0, 0);
      q[0] = make_int2((int)v.x, (int)v.y);
      q[1] = make_int2((int)v.z, (int)v.w);
    } else {
      q[0] = cl.pos[c0];
      q[1] = make_int2(0, 0);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (c0 + j >= b) break;
      const float my = (float)q[j].x * (float)FX_SCALE;
      const float mz = (float)(q[j].y - anchor) * (float)FX_SCALE;
      const float x2 = chi2_of(k, my, mz, si);
      if (x2 <= chi2max && (best < 0 || x2 < bchi)) {
        best = (int32_t)(c0 + j);
        bchi = x2;
        bq = q[j];
      }
    }
  }
  return best;
}

// Per tracklet (a walk of its cleaned up-links): its middle and end clusters
// (0xFFFFFFFF for a tracklet that cannot be followed: broken chain or rows
// beyond the last), its start unit-row, and the sort key of the outward
// following pass: the rows above its start row (the most rows that pass can
// take), 0 if it cannot be followed.
__global__ __launch_bounds__(256) void k_tracklet_points(ClusterView cl, uint32_t n_ur,
                                                         const int32_t* __restrict__ upc,
                                                         const uint32_t* __restrict__ tl_start,
                                                         const uint16_t* __restrict__ tl_len,
                                                         const uint32_t* n_tl_dev, uint32_t tl_cap,
                                                         uint32_t* __restrict__ pts,
                                                         uint8_t* __restrict__ key,
                                                         const DevStatus* st) {
  if (failed(st)) return;
  const uint32_t n_tl = scan_count(n_tl_dev, tl_cap);
  const uint32_t n_cl = scan_count(cl.n_clusters, cl.capacity);
  uint32_t dt;
  for (uint32_t t = xcd_thread_item(n_tl, dt); t < n_tl; t += dt) {
    const uint32_t A = tl_start[t];
    const int L = tl_len[t];
    uint32_t M = 0xFFFFFFFFu, E = 0xFFFFFFFFu, urA = 0;
    uint8_t rows = 0;
    if (A < n_cl && L >= 3) {
      urA = cluster_ur(cl.crow, n_ur, A);
      const int r1 = (int)(urA % NROW);
      if (r1 + L <= NROW) {
        const int im = (L + 1) / 2 - 1;
        uint32_t c = A, m = A;
        bool bad = false;
        for (int i = 1; i < L; ++i) {
          const int32_t nx = upc[c];
          if (nx < 0 || (uint32_t)nx >= n_cl) {
            bad = true;
            break;
          }
          c = (uint32_t)nx;
          if (i == im) m = c;
        }
        if (!bad) {
          M = m;
          E = c;
          rows = (uint8_t)(NROW - 1 - r1);
        }
      }
    }
    pts[(size_t)t * 3 + 0] = M;
    pts[(size_t)t * 3 + 1] = E;
    pts[(size_t)t * 3 + 2] = urA;
    key[t] = rows;
  }
}

// Stable counting sort of the tracklets by an 8-bit key, largest first.  The
// key is the most rows a following pass can take (rows above the start row
// outward; the row of the outermost pass-A hit inward): the passes that can
// run longest start first, and the lanes of a wave start on one row and step
// through the same rows, reading the same parts of the hit grid.  The sort
// can first split the tracklets into ngrp groups of consecutive blocks (so of
// consecutive units) and sort each group on its own: the following gives group
// g to the workgroups that the dispatcher places on XCD g, so each XCD's L2
// holds the hit data of its own units only.  Three steps: k_sort_work<false>
// counts each block of SORT_BLOCK tracklets per key into
// bins[(g * 256 + key') * npg + block in group] (key' = 255 - key, npg blocks per
// group); an exclusive scan of bins in place gives every (group, key', block)
// its first position, and bins[g * 256 * npg] is where group g starts;
// k_sort_work<true> writes perm, ranking the elements of one key in index
// order.  Tracklets of equal estimate keep their order (unit, row, time), so
// neighbouring tracks share a wave.  Wave w of a workgroup takes the elements
// [256 w, 256 w + 256) of its block.  Launch at least
// ceil(capacity / SORT_BLOCK) + ngrp - 1 workgroups, over as many times 256
// bins.
#define SORT_BLOCK 1024
#define XCD_GROUPS 8  // sort groups of the following: one per XCD
__device__ __forceinline__ uint32_t sort_blocks_per_group(uint32_t n, uint32_t ngrp) {
  return ((n + SORT_BLOCK - 1) / SORT_BLOCK + ngrp - 1) / ngrp;
}

// One item per thread over the sorted order of n items in ngrp groups:
// workgroup b takes group b % ngrp (gridDim.x is a multiple of ngrp), in the
// group's order; [i0, i1) with stride di are this thread's positions.
__device__ __forceinline__ void sorted_items(const uint32_t* __restrict__ bins, uint32_t ngrp,
                                             uint32_t n, uint32_t& i0, uint32_t& i1,
                                             uint32_t& di) {
  const uint32_t g = blockIdx.x % ngrp, j = blockIdx.x / ngrp, per = gridDim.x / ngrp;
  const uint32_t npg = sort_blocks_per_group(n, ngrp);
  const size_t gsz = (size_t)256 * npg;
  const uint32_t gs = npg ? bins[g * gsz] : 0u;
  i1 = npg == 0 ? 0u : g + 1 < ngrp ? bins[(g + 1) * gsz] : n;
  i0 = j < per ? gs + j * blockDim.x + threadIdx.x : i1;
  di = per * blockDim.x;
}

template <bool SCATTER>
__global__ __launch_bounds__(256) void k_sort_work(const uint8_t* __restrict__ key,
                                                   const uint32_t* n_tl_dev, uint32_t tl_cap,
                                                   uint32_t ngrp, uint32_t* __restrict__ bins,
                                                   uint32_t* __restrict__ perm,
                                                   const DevStatus* st) {
  if (failed(st)) return;
  __shared__ uint32_t h[4][256];  // per wave: count per key, then next position per key
  const uint32_t n = scan_count(n_tl_dev, tl_cap);
  const uint32_t npg = sort_blocks_per_group(n, ngrp);
  if (blockIdx.x >= ngrp * npg) return;  // uniform per workgroup
  const uint32_t grp = blockIdx.x / npg, lb = blockIdx.x - grp * npg;
  const uint32_t b0 = blockIdx.x * SORT_BLOCK;
  const uint32_t m = b0 < n ? min((uint32_t)SORT_BLOCK, n - b0) : 0u;
  if (SCATTER && m == 0) return;  // uniform per workgroup
  const uint32_t w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < 4; ++j) h[j][threadIdx.x] = 0;
  __syncthreads();
  uint32_t bin[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t i = 256u * w + 64u * j + lane;
    bin[j] = i < m ? 255u - key[b0 + i] : 0u;
    if (i < m) atomicAdd(&h[w][bin[j]], 1u);
  }
  __syncthreads();
  const uint32_t k = threadIdx.x;
  const uint32_t c0 = h[0][k], c1 = h[1][k], c2 = h[2][k], c3 = h[3][k];
  const size_t bi = (size_t)(grp * 256u + k) * npg + lb;
  if (!SCATTER) {
    bins[bi] = c0 + c1 + c2 + c3;
    return;
  }
  const uint32_t base = bins[bi];
  __syncthreads();
  h[0][k] = base;
  h[1][k] = base + c0;
  h[2][k] = base + c0 + c1;
  h[3][k] = base + c0 + c1 + c2;
  __syncthreads();
  const uint64_t below = (1ull << lane) - 1ull;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t i = 256u * w + 64u * j + lane;
    const bool v = i < m;
    uint64_t eq = __ballot(v);  // valid lanes with the same key
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool on = (bin[j] >> bit) & 1u;
      const uint64_t bb = __ballot(on);
      eq &= on ? bb : ~bb;
    }
    if (v) perm[h[w][bin[j]] + (uint32_t)__popcll(eq & below)] = b0 + i;
    // the highest lane of each key advances the key's position; the reads
    // above belong to an earlier instruction of this wave
    if (v && (eq >> lane) == 1ull) h[w][bin[j]] += (uint32_t)__popcll(eq);
  }
}

// Following of one tracklet per lane: seed and first update, pass A outward
// row by row, pass B inward from the outermost pass-A hit, result.

struct FollowLane {
  Trk<float> k;   // state at row r
  float sp[5];    // state after the last update (pass A, then pass B)
  uint32_t t;
  int32_t anchor;
  int32_t pre;    // candidate of the next row known before its helix step, or -1
  uint32_t ubase;
  int r, r1, L, nmiss, nh, hi, lo, rs;  // rs: row of sp
  uint32_t n_steps, n_cands, n_upds;      // work done (measurement)
};

// Seed and first update of tracklet t; false if it cannot be followed.
__device__ __forceinline__ bool follow_init(FollowLane& f, uint32_t t, const ClusterView& cl,
                                            const uint32_t* tl_start, const uint16_t* tl_len,
                                            const int32_t* upc, const uint32_t* pts, FollowOut& fo,
                                            const DevParams32* P, const PV<float>& pv) {
  fo.ok[t] = 0;
  fo.nhits[t] = 0;
  fo.range[t] = 0;
  const uint32_t M = pts[(size_t)t * 3 + 0], E = pts[(size_t)t * 3 + 1];
  if (M == 0xFFFFFFFFu) return false;
  const uint32_t urA = pts[(size_t)t * 3 + 2];
  const uint32_t A = tl_start[t];
  const int L = tl_len[t];
  const int r1 = urA % NROW;
  f.t = t;
  f.L = L;
  f.r1 = r1;
  f.ubase = urA - r1;
  const int im = (L + 1) / 2 - 1;
  const int rM = r1 + im, rE = r1 + L - 1;
  const int2 qA = cl.pos[A], qM = cl.pos[M], qE = cl.pos[E];
  const int32_t anchor = qA.y;
  f.anchor = anchor;
  // ---- seed: circle through A, M, E; differences are exact integers
  const int64_t dxm = P->xfx[rM] - P->xfx[r1], dym = (int64_t)qM.x - qA.x;
  const int64_t dxe = P->xfx[rE] - P->xfx[r1], dye = (int64_t)qE.x - qA.x;
  const int64_t dxx = P->xfx[rE] - P->xfx[rM], dyy = (int64_t)qE.x - qM.x;
  const float cross = (float)(dxm * dye - dym * dxe) * (float)(FX_SCALE * FX_SCALE);
  const float fma_ = hypotf((float)dxm, (float)dym) * (float)FX_SCALE;
  const float fea = hypotf((float)dxe, (float)dye) * (float)FX_SCALE;
  const float fem = hypotf((float)dxx, (float)dyy) * (float)FX_SCALE;
  const float b = pv.b();
  float C = 2.0f * cross / (fma_ * fem * fea);
  float qpt = -C / b;
  qpt = fminf(fmaxf(qpt, -pv.qpt_clamp()), pv.qpt_clamp());
  C = -b * qpt;
  const float sarg = fminf(fmaxf(fea * C * 0.5f, -1.0f), 1.0f);
  const float phiA = atan2f((float)dye, (float)dxe) - asinf(sarg);
  const float h = fea * fabsf(C) * 0.5f;
  const float arc = h > 0.0f ? fea * asinf(fminf(h, 1.0f)) / h : fea;
  Trk<float>& k = f.k;
  k.p[0] = (float)qA.x * (float)FX_SCALE;
  k.p[1] = 0.0f;
  k.p[2] = sinf(phiA);
  k.p[3] = (float)(qE.y - anchor) * (float)FX_SCALE / arc;
  k.p[4] = qpt;
  if (!(fabsf(k.p[2]) < pv.snp_max())) return false;
  c0_reset(k, pv, r1);
  f.n_upds += 1;
  if (!update(k, k.p[0], 0.0f, pv.vy(r1), pv.vz(r1), (float*)nullptr)) return false;
  fo.hits[(size_t)t * NROW + r1] = (int32_t)A;
  f.nh = 1;
#pragma unroll
  for (int i = 0; i < 5; ++i) f.sp[i] = k.p[i];
  f.rs = r1;
  f.nmiss = 0;
  f.hi = r1;
  f.pre = L > 1 ? upc[A] : -1;  // the next row is on the tracklet's own chain
  f.r = r1;
  return true;
}

// Pass B start: the outermost pass-A hit (row rs) with a reset covariance;
// false if its update fails (the tracklet then ends with the pass-A state).
__device__ __forceinline__ bool follow_start_b(FollowLane& f, const ClusterView& cl,
                                               const FollowOut& fo, const PV<float>& pv) {
  Trk<float>& k = f.k;
#pragma unroll
  for (int i = 0; i < 5; ++i) k.p[i] = f.sp[i];
  c0_reset(k, pv, f.rs);
  f.lo = f.r1;
  const int32_t co = fo.hits[(size_t)f.t * NROW + f.rs];
  const int2 q = cl.pos[co];
  const float my = (float)q.x * (float)FX_SCALE;
  const float mz = (float)(q.y - f.anchor) * (float)FX_SCALE;
  ++f.n_upds;
  if (!update(k, my, mz, pv.vy(f.rs), pv.vz(f.rs), (float*)nullptr)) return false;
#pragma unroll
  for (int i = 0; i < 5; ++i) f.sp[i] = k.p[i];
  f.nmiss = 0;
  f.r = f.rs;
  f.pre = f.rs - 1 >= f.r1 ? fo.hits[(size_t)f.t * NROW + f.rs - 1] : -1;
  return true;
}

__device__ __forceinline__ void follow_finish(const FollowLane& f, FollowOut& fo) {
  // six floats per tracklet at 8-byte alignment: three 8-byte stores
  float2* S = reinterpret_cast<float2*>(fo.state + (size_t)f.t * 6);
  S[0] = make_float2(f.sp[0], f.sp[1]);
  S[1] = make_float2(f.sp[2], f.sp[3]);
  S[2] = make_float2(f.sp[4], (float)f.rs);
  fo.nhits[f.t] = (uint16_t)f.nh;
  fo.range[f.t] = (uint16_t)(f.lo | (f.hi << 8));
  fo.ok[f.t] = 1;
}

// One row of pass A (outward, PA = 1) or pass B (inward, PA = 0).  Returns
// true when the pass has ended.
template <int PA>
__device__ __forceinline__ bool follow_step(FollowLane& f, const ClusterView& cl,
                                            const uint32_t* cblk, uint32_t nblk,
                                            const int32_t* upc, FollowOut& fo, const DevParams32* P,
                                            const PV<float>& pv, float chi2max) {
  constexpr bool pa = PA == 1;
  const int rn = f.r + (pa ? 1 : -1);
  if (rn >= NROW || rn < 0) return true;
  int32_t* H = fo.hits + (size_t)f.t * NROW;
  // Rows whose candidate is known before the helix step: the tracklet's own
  // chain (pass A) and the rows pass A covered (pass B: its hit, or -1 for a
  // row it missed, which is searched).  The candidate's position and the
  // next row's known candidate are loaded before the step, so their latency
  // overlaps its arithmetic.
  const bool known = pa ? rn < f.r1 + f.L : rn >= f.r1;
  int32_t cand = known ? f.pre : -1;
  int2 q = make_int2(0, 0);
  if (cand >= 0) q = cl.pos[cand];
  const int rn2 = rn + (pa ? 1 : -1);
  int32_t pre2 = -1;
  if (pa ? (rn2 < f.r1 + f.L && cand >= 0) : (rn2 >= f.r1 && rn2 >= 0)) pre2 = pa ? upc[cand] : H[rn2];
  Trk<float>& k = f.k;
  if (!propagate(k, row_dx<float>(P, f.r, rn), pv, true, pv.snp_max())) return true;
  ++f.n_steps;
  bool fresh = false;
  if (!known || (!pa && cand < 0)) {
    if (fabsf(k.p[0]) > pv.hw(rn) + pv.edge_margin()) return true;
    cand = search_row(cl, cblk, nblk, f.ubase + rn, k, f.anchor, pv.vy(rn), pv.vz(rn), chi2max,
                      f.n_cands, q);
    fresh = true;
  }
  f.pre = pre2;
  f.r = rn;
  // a row this pass visits first gets exactly one store: its hit, or -1
  const bool first = pa || (fresh && rn < f.lo);
  if (pa) f.hi = rn;
  else if (first) f.lo = rn;
  if (cand < 0) {
    if (first) H[rn] = -1;
    if ((pa || rn < f.r1) && ++f.nmiss >= P->max_miss) return true;
    return false;
  }
  const float my = (float)q.x * (float)FX_SCALE;
  const float mz = (float)(q.y - f.anchor) * (float)FX_SCALE;
  ++f.n_upds;
  if (!update(k, my, mz, pv.vy(rn), pv.vz(rn), (float*)nullptr)) {
    if (first) H[rn] = -1;
    return true;
  }
  if (pa || fresh) {
    H[rn] = cand;
    ++f.nh;
  }
#pragma unroll
  for (int i = 0; i < 5; ++i) f.sp[i] = k.p[i];
  f.rs = rn;
  f.nmiss = 0;
  return false;
}

// Pass B start of tracklet t from what pass A left in the outputs: the
// state at the outermost pass-A hit, its row, the hit count and row range.
__device__ __forceinline__ void follow_resume(FollowLane& f, uint32_t t, const ClusterView& cl,
                                              const uint32_t* tl_start, const uint16_t* tl_len,
                                              const uint32_t* pts, const FollowOut& fo) {
  const uint32_t urA = pts[(size_t)t * 3 + 2];
  f.t = t;
  f.r1 = (int)(urA % NROW);
  f.ubase = urA - (uint32_t)f.r1;
  f.L = tl_len[t];
  f.anchor = cl.pos[tl_start[t]].y;
  const float2* S = reinterpret_cast<const float2*>(fo.state + (size_t)t * 6);
  const float2 s01 = S[0], s23 = S[1], s4r = S[2];
  f.sp[0] = s01.x;
  f.sp[1] = s01.y;
  f.sp[2] = s23.x;
  f.sp[3] = s23.y;
  f.sp[4] = s4r.x;
  f.rs = (int)s4r.y;
  f.nh = fo.nhits[t];
  f.hi = fo.range[t] >> 8;
  f.pre = -1;
}

enum { FP_A = 0, FP_B = 1, FP_AB = 2 };

// Following, one tracklet per lane.  FP_A: seed and pass A of the tracklets
// in the order perm gives, leaving the pass-A
// result in the outputs and the sort key of pass B (the row of the outermost
// pass-A hit) in key; FP_B: pass B of the tracklets that pass A
// followed, in the order perm gives; FP_AB: both passes per lane, tracklets in
// index order (perm unused).  Either way a tracklet's result is the same.
// COUNT: also count the work done (helix steps, candidates, updates) into
// per-wave counters, for measurement only.
template <int B, int PASS, bool COUNT>
__global__ __launch_bounds__(B) void k_follow(ClusterView cl, const uint32_t* __restrict__ cblk,
                                               uint32_t nblk, const int32_t* __restrict__ upc,
                                               const uint32_t* __restrict__ tl_start,
                                               const uint16_t* __restrict__ tl_len,
                                               const uint32_t* __restrict__ pts,
                                               const uint32_t* __restrict__ perm,
                                               const uint32_t* __restrict__ bins, uint32_t ngrp,
                                               uint8_t* __restrict__ key,
                                               const uint32_t* n_tl_dev, uint32_t tl_cap,
                                               FollowOut fo, ulonglong4* __restrict__ work,
                                               const DevParams* __restrict__ Pg, DevStatus* st) {
  const uint32_t wave = blockIdx.x * (B / 64) + (threadIdx.x >> 6);
  if (failed(st)) {
    if (COUNT && (threadIdx.x & 63) == 0) work[wave] = make_ulonglong4(0, 0, 0, 0);
    return;
  }
  // FP32 only: the parameter block without its FP64 copies
  __shared__ DevParams32 Ps;
  const DevParams32* P = params_to_lds(Pg, &Ps);
  const PV<float> pv{P};
  const uint32_t n_tl = scan_count(n_tl_dev, tl_cap);
  const float chi2max = pv.chi2_max();
  uint32_t w_steps = 0, w_cands = 0, w_upds = 0;
  uint32_t i0 = blockIdx.x * blockDim.x + threadIdx.x, i1 = n_tl, di = gridDim.x * blockDim.x;
  if (PASS != FP_AB) sorted_items(bins, ngrp, n_tl, i0, i1, di);
  for (uint32_t i = i0; i < i1; i += di) {
    const uint32_t t = PASS == FP_AB ? i : perm[i];
    FollowLane f;
    f.n_steps = f.n_cands = f.n_upds = 0;
    if (PASS == FP_B) {
      if (!fo.ok[t]) continue;
      follow_resume(f, t, cl, tl_start, tl_len, pts, fo);
    } else if (!follow_init(f, t, cl, tl_start, tl_len, upc, pts, fo, P, pv)) {
      if (PASS == FP_A) key[t] = 0;
      if (COUNT) w_upds += f.n_upds;
      continue;
    }
    if (PASS != FP_B) {
      while (!follow_step<1>(f, cl, cblk, nblk, upc, fo, P, pv, chi2max)) {
      }
    }
    if (PASS == FP_A) {
      f.lo = f.r1;
      follow_finish(f, fo);
      key[t] = (uint8_t)f.rs;
    } else if (follow_start_b(f, cl, fo, pv)) {
      while (!follow_step<0>(f, cl, cblk, nblk, upc, fo, P, pv, chi2max)) {
      }
      follow_finish(f, fo);
    } else if (PASS == FP_AB) {
      follow_finish(f, fo);
    }
    if (COUNT) {
      w_steps += f.n_steps;
      w_cands += f.n_cands;
      w_upds += f.n_upds;
    }
  }
  if (!COUNT) return;
  // work counters: one plain store per wave, summed by k_work_sum (atomics
  // from every wave on one address would serialise at the end of the kernel)
  const unsigned long long s0 = wave_sum_u64(w_steps), s1 = wave_sum_u64(w_cands),
                           s2 = wave_sum_u64(w_upds);
  // lane slots: the wave runs as long as its busiest lane (exact when each
  // lane takes at most one tracklet, as with a grid that covers the capacity)
  const uint32_t mx = (uint32_t)wave_max_i32((int32_t)w_steps);
  if ((threadIdx.x & 63) == 0) work[wave] = make_ulonglong4(s0, s1, s2, 64ull * mx);
}

// Following with lane refill, one pass (FP_A or FP_B) over the tracklets in
// sorted order.  A lane holds one tracklet; when at least FOLLOW_REFILL lanes
// of a wave are free (or none is busy), the wave takes that many next
// tracklets of its workgroup's sort group with one atomic on the group's
// counter (refill = FOLLOW_REFILL), so the wave no longer runs as long as its longest tracklet with
// the other lanes idle.  Every tracklet is followed by exactly one lane, with
// the same arithmetic as k_follow, so the results do not depend on which lane
// or wave takes it.  The grid is sized to the resident waves, at most
// FOLLOW_Q_WAVES_PER_CU per compute unit (more would find the queues empty);
// qnext holds ngrp zeroed counters.
#define FOLLOW_REFILL 32
// Waves of the lane-refill grid per compute unit.  Each lane gathers lines of
// its own (hit grid, positions, hit table) that the L2 holds only while few
// lanes compete for it: on a 2 ms Pb-Pb slice the two passes took 3.02, 2.53,
// 2.41, 2.53 and 2.63 ms with 8, 12, 16, 20 and 24 waves per compute unit.
#define FOLLOW_Q_WAVES_PER_CU 16
template <int B, int PASS, bool COUNT>
__global__ __launch_bounds__(B) void k_follow_q(ClusterView cl, const uint32_t* __restrict__ cblk,
                                                 uint32_t nblk, const int32_t* __restrict__ upc,
                                                 const uint32_t* __restrict__ tl_start,
                                                 const uint16_t* __restrict__ tl_len,
                                                 const uint32_t* __restrict__ pts,
                                                 const uint32_t* __restrict__ perm,
                                                 const uint32_t* __restrict__ bins, uint32_t ngrp,
                                                 uint32_t* __restrict__ qnext,
                                                 uint32_t refill,
                                                 uint8_t* __restrict__ key,
                                                 const uint32_t* n_tl_dev, uint32_t tl_cap,
                                                 FollowOut fo, ulonglong4* __restrict__ work,
                                                 const DevParams* __restrict__ Pg, DevStatus* st) {
  static_assert(PASS == FP_A || PASS == FP_B, "one pass per launch");
  const uint32_t wave = blockIdx.x * (B / 64) + (threadIdx.x >> 6);
  if (failed(st)) {
    if (COUNT && (threadIdx.x & 63) == 0) work[wave] = make_ulonglong4(0, 0, 0, 0);
    return;
  }
  // FP32 only: the parameter block without its FP64 copies
  __shared__ DevParams32 Ps;
  const DevParams32* P = params_to_lds(Pg, &Ps);
  const PV<float> pv{P};
  const uint32_t n_tl = scan_count(n_tl_dev, tl_cap);
  const float chi2max = pv.chi2_max();
  // this workgroup's sort group: positions [gs, ge) of perm
  const uint32_t g = blockIdx.x % ngrp;
  const uint32_t npg = sort_blocks_per_group(n_tl, ngrp);
  const size_t gsz = (size_t)256 * npg;
  const uint32_t gs = npg ? bins[g * gsz] : 0u;
  const uint32_t ge = npg == 0 ? 0u : g + 1 < ngrp ? bins[(g + 1) * gsz] : n_tl;
  const uint64_t below = (1ull << (threadIdx.x & 63)) - 1ull;
  uint32_t w_steps = 0, w_cands = 0, w_upds = 0, w_iter = 0;
  FollowLane f;
  bool busy = false, retired = false;
  for (;;) {
    const uint64_t want = __ballot(!busy && !retired);
    const uint32_t nwant = (uint32_t)__popcll(want);
    const bool any_busy = __ballot(busy) != 0ull;
    if (!any_busy && nwant == 0) break;
    if (nwant >= refill || (!any_busy && nwant > 0)) {
      const int lead = __ffsll((long long)want) - 1;
      uint32_t base = 0;
      if ((int)(threadIdx.x & 63) == lead) base = atomicAdd(&qnext[g], nwant);
      base = (uint32_t)__shfl((int)base, lead, 64);
      if (!busy && !retired) {
        const uint32_t i = gs + base + (uint32_t)__popcll(want & below);
        if (i >= ge) {
          retired = true;
        } else {
          const uint32_t t = perm[i];
          f.n_steps = f.n_cands = f.n_upds = 0;
          if (PASS == FP_B) {
            if (fo.ok[t]) {
              follow_resume(f, t, cl, tl_start, tl_len, pts, fo);
              busy = follow_start_b(f, cl, fo, pv);
            }
          } else {
            busy = follow_init(f, t, cl, tl_start, tl_len, upc, pts, fo, P, pv);
            if (!busy) key[t] = 0;
          }
          if (COUNT && !busy) w_upds += f.n_upds;
        }
      }
    }
    if (COUNT) ++w_iter;
    if (busy && follow_step<PASS == FP_A ? 1 : 0>(f, cl, cblk, nblk, upc, fo, P, pv, chi2max)) {
      busy = false;
      if (PASS == FP_A) {
        f.lo = f.r1;
        follow_finish(f, fo);
        key[f.t] = (uint8_t)f.rs;
      } else {
        follow_finish(f, fo);
      }
      if (COUNT) {
        w_steps += f.n_steps;
        w_cands += f.n_cands;
        w_upds += f.n_upds;
      }
    }
  }
  if (!COUNT) return;
  const unsigned long long s0 = wave_sum_u64(w_steps), s1 = wave_sum_u64(w_cands),
                           s2 = wave_sum_u64(w_upds);
  // lane slots: 64 per loop round of the wave
  if ((threadIdx.x & 63) == 0) work[wave] = make_ulonglong4(s0, s1, s2, 64ull * w_iter);
}

// Sum of the following's per-wave work counters into the status block.
__global__ __launch_bounds__(1024) void k_work_sum(const ulonglong4* __restrict__ work,
                                                   uint32_t n, DevStatus* st) {
  __shared__ unsigned long long part[4][16];
  unsigned long long a = 0, b = 0, c = 0, e = 0;
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
    const ulonglong4 v = work[i];
    a += v.x;
    b += v.y;
    c += v.z;
    e += v.w;
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    a += __shfl_xor(a, d, 64);
    b += __shfl_xor(b, d, 64);
    c += __shfl_xor(c, d, 64);
    e += __shfl_xor(e, d, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    part[0][threadIdx.x >> 6] = a;
    part[1][threadIdx.x >> 6] = b;
    part[2][threadIdx.x >> 6] = c;
    part[3][threadIdx.x >> 6] = e;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long s[4] = {0, 0, 0, 0};
    for (int k = 0; k < 4; ++k)
      for (uint32_t w = 0; w < blockDim.x / 64; ++w) s[k] += part[k][w];
    st->f_steps = s[0];
    st->f_cands = s[1];
    st->f_upds = s[2];
    st->f_slots = s[3];
  }
}

// Claim priority of a track: more hits first, then the lower tracklet id
// (tracklet ids stay below 2^24, hit counts below 2^8).
__device__ __forceinline__ uint32_t track_key(uint32_t nh, uint32_t t) {
  return (nh << 24) | (0xFFFFFFu - t);
}

// Conflict resolution runs one wave per tracklet: the lanes take the rows
// of the tracklet's hit table (contiguous), so every table read is coalesced.
// The tracklet index is made wave-uniform so its scalars load once.

#define KEEP_GROUP 4  // consecutive tracklets per wave of the claim and keep kernels

// Lane k of a wave loads what the claim and keep need of tracklet t0 + k
// (t0 + k < t1): 1 | hit count << 8 | row range << 16 for a tracklet that bids
// (followed, at least min_track_hits hits), else 0.  Read back per tracklet
// with a lane read, so the fields come in one coalesced load per array.
__device__ __forceinline__ uint32_t bid_info(const FollowOut& fo, uint32_t t0, uint32_t t1,
                                             int min_hits) {
  const uint32_t t = t0 + (threadIdx.x & 63);
  if (t >= t1 || !fo.ok[t]) return 0u;
  const uint32_t nh = fo.nhits[t];
  return (int)nh >= min_hits ? 1u | (nh << 8) | ((uint32_t)fo.range[t] << 16) : 0u;
}

// The hit-table entries of the first 64 rows of each bidding tracklet of a
// group (lane l: row lo + l, or -1), loaded together so that their latencies
// overlap instead of coming one tracklet after the other.
__device__ __forceinline__ void first_rows(const FollowOut& fo, uint32_t t0, uint32_t info,
                                           int32_t (&first)[KEEP_GROUP]) {
  const int lane = (int)(threadIdx.x & 63);
#pragma unroll
  for (int kk = 0; kk < KEEP_GROUP; ++kk) {
    const uint32_t inf = (uint32_t)__builtin_amdgcn_readlane((int)info, kk);
    const int lo = (inf >> 16) & 255, hi = inf >> 24;
    const int r = lo + lane;
    first[kk] = inf && r <= hi ? fo.hits[(size_t)(t0 + kk) * NROW + r] : -1;
  }
}

// Every followed tracklet with enough hits bids for its clusters: the owner
// of a cluster is the largest key among its bidders.  Two launches instead of
// one atomicMax per hit: FIX = false stores every bidder's key (one of them
// lands); FIX = true reads the owner back and raises it with atomicMax only
// where the bidder's key is larger.  Owners only grow in the second launch
// and hold bidders' keys, so the largest bidder either reads its own key or
// raises the owner to it: the result is the maximum.  Most clusters have one
// bidder and cost a plain store and a load instead of a device-scope atomic.
template <bool FIX>
__global__ __launch_bounds__(256) void k_claim(FollowOut fo, const uint32_t* n_tl_dev,
                                               uint32_t tl_cap,
                                               uint32_t* __restrict__ owner,
                                               uint32_t n_cl_cap, const DevParams* __restrict__ P,
                                               const DevStatus* st) {
  if (failed(st)) return;
  const uint32_t n_tl = scan_count(n_tl_dev, tl_cap);
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t n_grp = (n_tl + KEEP_GROUP - 1) / KEEP_GROUP;
  uint32_t nw;
  for (uint32_t i = xcd_wave_item(n_grp, nw); i < n_grp; i += nw) {
    // the stores go in descending tracklet order, so that of two bidders with
    // equal hit counts the one that wins (the lower index) tends to store
    // last (a store order sorted by key wins more clusters at once but loses
    // the locality of neighbouring tracklets and costs more than it saves)
    const uint32_t g = FIX ? i : n_grp - 1 - i;
    const uint32_t t0 = g * KEEP_GROUP, t1 = min(t0 + KEEP_GROUP, n_tl);
    const uint32_t info = bid_info(fo, t0, t1, P->min_track_hits);
    int32_t first[KEEP_GROUP];
    first_rows(fo, t0, info, first);
#pragma unroll
    for (int k = 0; k < KEEP_GROUP; ++k) {
      const int kk = FIX ? k : KEEP_GROUP - 1 - k;
      if (kk >= (int)(t1 - t0)) continue;
      const uint32_t inf = (uint32_t)__builtin_amdgcn_readlane((int)info, kk);
      if (!inf) continue;
      const uint32_t t = t0 + kk;
      const uint32_t key = track_key((inf >> 8) & 255, t);
      const int lo = (inf >> 16) & 255, hi = inf >> 24;
      const int32_t* H = fo.hits + (size_t)t * NROW;
      for (int r = lo + (int)lane; r <= hi; r += 64) {
        const int32_t c = r < lo + 64 ? first[kk] : H[r];
        if (c < 0 || (uint32_t)c >= n_cl_cap) continue;
        if (!FIX) owner[c] = key;
        else if (owner[c] < key) atomicMax(&owner[c], key);
      }
    }
  }
}

// Hits each track keeps after the claims; < min_track_hits drops the track.
// The kept count is also the refit's sort key: the refit takes the tracks
// sorted by it, so the lanes of a wave refit tracks of equal length.
__global__ __launch_bounds__(256) void k_keep(FollowOut fo, const uint32_t* n_tl_dev,
                                              uint32_t tl_cap,
                                              const uint32_t* __restrict__ owner,
                                              uint32_t n_cl_cap, uint16_t* __restrict__ nkept,
                                              uint8_t* __restrict__ key,
                                              const DevParams* __restrict__ P,
                                              const DevStatus* st) {
  if (failed(st)) return;
  const uint32_t n_tl = scan_count(n_tl_dev, tl_cap);
  const uint32_t lane = threadIdx.x & 63;
  uint32_t nw;
  // a wave takes KEEP_GROUP consecutive tracklets; lane k collects the count
  // of the k-th, and the counts go out as one run per array
  const uint32_t n_grp = (n_tl + KEEP_GROUP - 1) / KEEP_GROUP;
  for (uint32_t g = xcd_wave_item(n_grp, nw); g < n_grp; g += nw) {
    const uint32_t t0 = g * KEEP_GROUP, t1 = min(t0 + KEEP_GROUP, n_tl);
    uint32_t mine = 0;
    const uint32_t info = bid_info(fo, t0, t1, P->min_track_hits);
    int32_t first[KEEP_GROUP];
    first_rows(fo, t0, info, first);
#pragma unroll
    for (int kk = 0; kk < KEEP_GROUP; ++kk) {
      const uint32_t t = t0 + kk;
      if (t >= t1) continue;
      uint32_t n = 0;
      const uint32_t inf = (uint32_t)__builtin_amdgcn_readlane((int)info, kk);
      if (inf) {
        const uint32_t key = track_key((inf >> 8) & 255, t);
        const int lo = (inf >> 16) & 255, hi = inf >> 24;
        const int32_t* H = fo.hits + (size_t)t * NROW;
        uint8_t* KR = fo.krow + (size_t)t * NROW;
        for (int r0 = lo; r0 <= hi; r0 += 64) {
          const int r = r0 + (int)lane;
          bool kept = false;
          if (r <= hi) {
            const int32_t c = r0 == lo ? first[kk] : H[r];
            kept = c >= 0 && (uint32_t)c < n_cl_cap && owner[c] == key;
          }
          const uint64_t m = __ballot(kept);
          if (kept) KR[n + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))] = (uint8_t)r;
          n += (uint32_t)__popcll(m);
        }
        if ((int)n < P->min_track_hits) n = 0;
      }
      if (lane == (uint32_t)kk) mine = n;
    }
    if (t0 + lane < t1) {
      nkept[t0 + lane] = (uint16_t)mine;
      key[t0 + lane] = (uint8_t)mine;  // sort key of the refit (n <= NROW)
    }
  }
}

struct RefitOut {
  float* par;      // [cap*5]
  float* cov;      // [cap*15]
  float* chi2;     // [cap]
  uint8_t* row;    // [cap]
  uint8_t* flags;  // [cap]
};

__device__ __forceinline__ int32_t tl_anchor(const ClusterView& cl, const uint32_t* tl_start,
                                             uint32_t t) {
  return cl.z_fx[tl_start[t]];
}

// ------------------------------------------------------------------ refit
// The refit keeps its covariance as UD factors, C = U D U^T, with U unit
// upper triangular (u[i][j] for j > i; the rest is implied) and D diagonal.
// The helix Jacobian is unit upper triangular too and there is no process
// noise, so a propagation is U <- J U with D unchanged.  A (y, z)
// measurement with independent errors is two scalar updates in Bierman's
// form: each pivot d_j becomes d_j alpha_(j-1) / alpha_j with alpha a running
// sum of non-negative terms, so the covariance stays positive definite and
// keeps FP32 precision while the broad start variances collapse by orders
// of magnitude (the dense form loses it to cancellation there).
template <typename T>
struct UDCov {
  T u[5][5];  // strictly upper part only
  T d[5];
};

__device__ __forceinline__ float rcp_of(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_of(double x) { return 1.0 / x; }

// U <- J U (rows 0..2 change; row 2 is read before it is written)
template <typename T>
__device__ __forceinline__ void ud_propagate(UDCov<T>& c, const HJac<T>& J) {
  const T u23 = c.u[2][3], u24 = c.u[2][4], u34 = c.u[3][4];
  c.u[0][2] += J.j02;
  c.u[0][3] += J.j02 * u23;
  c.u[0][4] += J.j02 * u24 + J.j04;
  c.u[1][2] += J.j12;
  c.u[1][3] += J.j12 * u23 + J.j13;
  c.u[1][4] += J.j12 * u24 + J.j13 * u34 + J.j14;
  c.u[2][4] += J.j24;
}

// Scalar measurement of parameter M with variance r (Bierman): updates the
// factors, writes the gain K and returns the residual variance alpha.
template <int M, typename T>
__device__ __forceinline__ T ud_update(UDCov<T>& c, T r, T K[5]) {
  T f[5], v[5], b[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    f[j] = j < M ? (T)0 : (j == M ? (T)1 : c.u[M][j]);
    v[j] = c.d[j] * f[j];
    b[j] = 0;
  }
  T alpha = r, ia = rcp_of(r);
#pragma unroll
  for (int j = M; j < 5; ++j) {
    const T ap = alpha, iap = ia;
    alpha = ap + f[j] * v[j];
    ia = rcp_of(alpha);
    c.d[j] *= ap * ia;
    const T lam = -f[j] * iap;
#pragma unroll
    for (int i = 0; i < j; ++i) {
      const T uij = c.u[i][j];
      c.u[i][j] = uij + b[i] * lam;
      b[i] += uij * v[j];
    }
    b[j] = v[j];
  }
#pragma unroll
  for (int i = 0; i < 5; ++i) K[i] = b[i] * ia;
  return alpha;
}

// C = U D U^T, packed upper triangle
template <typename T>
__device__ __forceinline__ void ud_to_cov(const UDCov<T>& c, T* out) {
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = i; j < 5; ++j) {
      T a = 0;
#pragma unroll
      for (int k = j; k < 5; ++k) {
        const T uik = k == i ? (T)1 : c.u[i][k];
        const T ujk = k == j ? (T)1 : c.u[j][k];
        a += uik * c.d[k] * ujk;
      }
      out[PI(i, j)] = a;
    }
}

// positive definite: every pivot of the factorisation > 0 (NaN fails)
template <typename T>
__device__ __forceinline__ bool ud_pd(const UDCov<T>& c) {
  bool ok = true;
#pragma unroll
  for (int j = 0; j < 5; ++j) ok = ok && c.d[j] > (T)0;
  return ok;
}

// Kalman update of the refit with the (y, z) measurement, as a y update then
// a z update; the y residual includes the low-order part of y.  Returns false
// if |sin phi| >= 1 afterwards (the track then fails).
template <typename T>
__device__ __forceinline__ bool ud_measure(T p[5], UDCov<T>& c, LoParts<T>* lo, T my, T mz, T vy,
                                           T vz, T* chi2) {
  T K[5];
  const T ry = lo ? (my - p[0]) - lo->y : my - p[0];
  const T ay = ud_update<0>(c, vy, K);
  if (lo) {
    p[0] = two_sum_acc(p[0], K[0] * ry, &lo->y);
    p[2] = two_sum_acc(p[2], K[2] * ry, &lo->s);
  } else {
    p[0] += K[0] * ry;
    p[2] += K[2] * ry;
  }
  p[1] += K[1] * ry;
  p[3] += K[3] * ry;
  p[4] += K[4] * ry;
  const T rz = mz - p[1];
  const T az = ud_update<1>(c, vz, K);
  if (lo) {
    p[0] = two_sum_acc(p[0], K[0] * rz, &lo->y);
    p[2] = two_sum_acc(p[2], K[2] * rz, &lo->s);
  } else {
    p[0] += K[0] * rz;
    p[2] += K[2] * rz;
  }
  p[1] += K[1] * rz;
  p[3] += K[3] * rz;
  p[4] += K[4] * rz;
  *chi2 = ry * ry * rcp_of(ay) + rz * rz * rcp_of(az);
  return fabs(p[2]) < (T)1;
}

// Kalman steps of the refit over the kept hits i, i-1, ... (rows
// descending); the state sits at row r_state.  On return i is the next kept
// hit.  Returns 1 if the helix cannot reach a hit's row or an update fails;
// pd turns false if an update left a pivot that is not positive.
template <typename T>
__device__ int refit_run(uint32_t t, const ClusterView& cl, int32_t anchor, const FollowOut& fo,
                         const DevParams* P, T p[5], UDCov<T>& c, T& chi2s, int& r_state, int& i,
                         bool& pd, LoParts<T>* lp) {
  const PV<T> pv{P};
  const int32_t* H = fo.hits + (size_t)t * NROW;
  const uint8_t* KR = fo.krow + (size_t)t * NROW;
  if (i < 0) return 0;
  // the row, cluster and position of the next hit are read a step ahead,
  // each behind a part of this step's arithmetic, so that their dependent
  // loads overlap it
  int r = KR[i];
  int2 q = cl.pos[H[r]];
  for (; i >= 0; --i) {
    const bool more = i > 0;
    const int r_n = more ? (int)KR[i - 1] : r;
    if (r != r_state) {
      HJac<T> J;
      if (!helix_step(p, row_dx<T>(P, r_state, r), pv, pv.refit_snp_max(), lp, &J)) return 1;
      ud_propagate(c, J);
    }
    const int32_t c_n = more ? H[r_n] : 0;
    const T my = (T)q.x * (T)FX_SCALE;
    const T mz = (T)(q.y - anchor) * (T)FX_SCALE;
    T x2;
    if (!ud_measure(p, c, lp, my, mz, pv.vy(r), pv.vz(r), &x2)) return 1;
    const int2 q_n = more ? cl.pos[c_n] : q;
    chi2s += x2;
    if (!ud_pd(c)) pd = false;
    r_state = r;
    r = r_n;
    q = q_n;
  }
  return 0;
}

// Start of the refit: the circle through the innermost, middle and outermost
// kept clusters, evaluated at the outermost one (fixed-point differences are
// exact integers), and the broad refit prior as UD factors (U = I).  Returns
// the outermost kept row, or -1 if the track has fewer than 3 kept hits.
template <typename T>
__device__ int refit_seed(uint32_t t, const ClusterView& cl, int32_t anchor, const FollowOut& fo,
                          int n, const DevParams* P, T p[5], UDCov<T>& c) {
  const PV<T> pv{P};
  if (n < 3) return -1;
  const int32_t* H = fo.hits + (size_t)t * NROW;
  const uint8_t* KR = fo.krow + (size_t)t * NROW;
  const int im = (n + 1) / 2 - 1;  // middle, counted from the innermost
  const int rA = KR[0], rM = KR[im], rE = KR[n - 1];
  const int32_t cA = H[rA], cM = H[rM], cE = H[rE];
  const int2 qA = cl.pos[cA], qM = cl.pos[cM], qE = cl.pos[cE];
  const int64_t dxm = P->xfx[rM] - P->xfx[rA], dym = (int64_t)qM.x - qA.x;
  const int64_t dxe = P->xfx[rE] - P->xfx[rA], dye = (int64_t)qE.x - qA.x;
  const int64_t dxx = P->xfx[rE] - P->xfx[rM], dyy = (int64_t)qE.x - qM.x;
  const T S = (T)FX_SCALE;
  const T cross = (T)(dxm * dye - dym * dxe) * S * S;
  const T dma = hypot((T)dxm, (T)dym) * S, dea = hypot((T)dxe, (T)dye) * S;
  const T dem = hypot((T)dxx, (T)dyy) * S;
  const T b = pv.b();
  T C = (T)2 * cross / (dma * dem * dea);
  T qpt = -C / b;
  qpt = fmin(fmax(qpt, -pv.qpt_clamp()), pv.qpt_clamp());
  C = -b * qpt;
  const T sarg = fmin(fmax(dea * C * (T)0.5, (T)-1), (T)1);
  const T h = dea * fabs(C) * (T)0.5;
  const T arc = h > (T)0 ? dea * asin(fmin(h, (T)1)) / h : dea;
  p[0] = (T)qE.x * S;
  p[1] = (T)(qE.y - anchor) * S;
  p[2] = sin(atan2((T)dye, (T)dxe) + asin(sarg));  // tangent at the far end of the chord
  p[3] = (T)(qE.y - qA.y) * S / arc;
  p[4] = qpt;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
#pragma unroll
    for (int j = 0; j < 5; ++j) c.u[i][j] = 0;
    c.d[i] = pv.c0r(i);
  }
  return rE;
}

// The refit of each kept track, tracks taken in the order perm gives (sorted
// by kept hits): in FP32 from the circle seed, with y and sin phi carried
// with their rounding errors.  A low-pT track (|q/pT| >= lowpt_qpt at the
// seed) whose FP32 covariance loses positive definiteness is refit again in
// FP64 from its seed by the same lane (TF_TO_FP64 marks it; the mark is
// internal and counted by a reduction); force_fallback sends every track
// there (a test hook).
__global__ __launch_bounds__(64) void k_refit(ClusterView cl, const uint32_t* __restrict__ tl_start,
                                              FollowOut fo, const uint32_t* n_tl_dev,
                                              uint32_t tl_cap, const uint16_t* __restrict__ nkept,
                                              const uint32_t* __restrict__ perm,
                                              const uint32_t* __restrict__ bins, uint32_t ngrp,
                                              RefitOut ro,
                                              const DevParams* __restrict__ Pg, DevStatus* st) {
  if (failed(st)) return;
  __shared__ DevParams Ps;
  const DevParams* P = params_to_lds(Pg, &Ps);
  const uint32_t n_tl = scan_count(n_tl_dev, tl_cap);
  uint32_t j0, j1, dj;
  sorted_items(bins, ngrp, n_tl, j0, j1, dj);
  for (uint32_t j = j0; j < j1; j += dj) {
    const uint32_t t = perm[j];
    ro.flags[t] = 0;
    const int n = nkept[t];
    if (n == 0) continue;
    const int32_t anchor = tl_anchor(cl, tl_start, t);
    if (!P->force_fallback) {
      float p[5];
      UDCov<float> c;
      int rs = refit_seed<float>(t, cl, anchor, fo, n, P, p, c);
      const bool lowpt = rs >= 0 && fabsf(p[4]) >= (float)P->lowpt_qpt;
      int r = n - 1;
      bool pd = true;
      float chi2s = 0.0f;
      LoParts<float> lo{0.0f, 0.0f};
      if (rs < 0 || refit_run<float>(t, cl, anchor, fo, P, p, c, chi2s, rs, r, pd, &lo)) {
        ro.flags[t] = TF_REFIT_FAIL;
        atomicAdd(&st->n_refit_fail, 1u);
        continue;
      }
      if (pd || !lowpt) {
        p[0] += lo.y;
        p[2] += lo.s;
        float cv[15];
        ud_to_cov(c, cv);
#pragma unroll
        for (int i = 0; i < 5; ++i) ro.par[(size_t)t * 5 + i] = p[i];
#pragma unroll
        for (int i = 0; i < 15; ++i) ro.cov[(size_t)t * 15 + i] = cv[i];
        ro.chi2[t] = chi2s;
        ro.row[t] = (uint8_t)rs;
        if (!pd) {
          ro.flags[t] = TF_NOT_PD;
          atomicAdd(&st->n_not_pd, 1u);
        }
        continue;
      }
    }
    // the whole refit again in FP64 (an FP32 result is discarded)
    double p[5];
    UDCov<double> c;
    double c2 = 0;
    int rs = refit_seed<double>(t, cl, anchor, fo, n, P, p, c);
    int r = n - 1;
    bool pd = true;
    const bool fail = rs < 0 || refit_run<double>(t, cl, anchor, fo, P, p, c, c2, rs, r, pd,
                                                  (LoParts<double>*)nullptr) != 0;
    if (fail || !pd) {
      ro.flags[t] = TF_TO_FP64 | (fail ? TF_REFIT_FAIL : TF_FP64_FAIL);
      atomicAdd(fail ? &st->n_refit_fail : &st->n_fallback_fail, 1u);
      continue;
    }
    double cv[15];
    ud_to_cov(c, cv);
#pragma unroll
    for (int i = 0; i < 5; ++i) ro.par[(size_t)t * 5 + i] = (float)p[i];
#pragma unroll
    for (int i = 0; i < 15; ++i) ro.cov[(size_t)t * 15 + i] = (float)cv[i];
    ro.chi2[t] = (float)c2;
    ro.row[t] = (uint8_t)rs;
    ro.flags[t] = TF_TO_FP64 | TF_FP64;
  }
}

// The tracks refit in FP64 (counted for the status).
struct GetToFp64 {
  const uint8_t* flags;
  __device__ uint32_t operator()(uint32_t t) const { return (flags[t] & TF_TO_FP64) ? 1u : 0u; }
};

// final keep flag of a tracklet slot
__device__ __forceinline__ bool final_kept(const uint16_t* nkept, const RefitOut& ro, uint32_t t) {
  return nkept[t] != 0 && (ro.flags[t] & (TF_REFIT_FAIL | TF_FP64_FAIL)) == 0;
}

struct GetTrackPair {
  const uint16_t* nkept;
  RefitOut ro;
  __device__ unsigned long long operator()(uint32_t t) const {
    return final_kept(nkept, ro, t) ? ((1ull << 32) | nkept[t]) : 0ull;
  }
};

struct EmitTrackPair {
  uint32_t* trk_index;  // [cap] track index or 0xFFFFFFFF
  uint32_t* hit_off;    // [cap]
  uint32_t* tlist;      // [cap] tracklet of each track
  uint32_t cap;
  __device__ void operator()(uint32_t t, unsigned long long pre, unsigned long long v) const {
    const uint32_t j = (uint32_t)(pre >> 32);
    trk_index[t] = v ? j : 0xFFFFFFFFu;
    hit_off[t] = (uint32_t)pre;
    if (v && j < cap) tlist[j] = t;
  }
};

struct TrackOut {
  uint32_t capacity, hit_capacity;
  uint32_t* tracklet;
  float *par, *cov, *chi2;
  uint16_t* ndf;
  uint8_t *row, *flags;
  int32_t* z_anchor;
  uint32_t* hit_start;
  uint32_t* hits;
  int32_t* cluster_track;
};

__global__ void k_track_totals(const unsigned long long* total, TrackOut to, uint32_t* n_tracks,
                               uint32_t* n_hits, DevStatus* st) {
  // after a latched error the scan that wrote *total did not run
  if (failed(st)) return;
  const unsigned long long v = *total;
  const uint32_t nt = (uint32_t)(v >> 32), nh = (uint32_t)v;
  st->n_tracks = nt;
  st->n_hits = nh;
  st->n_fallback = st->n_fp64_redo;
  if (n_tracks) *n_tracks = nt;
  if (n_hits) *n_hits = nh;
  if (nt > to.capacity) latch_capacity(st, OVF_TRACKS, nt);
  if (nh > to.hit_capacity) latch_capacity(st, OVF_HITS, nh);
  if (nt <= to.capacity) to.hit_start[nt] = nh;
}

// One wave per 64 consecutive tracks (the tracklets that became tracks,
// listed in order), so that every output array is written in contiguous
// runs: lane i writes the fields of track j0 + i, the wave writes the
// parameters and covariances of its tracks as one run each, then the kept hits
// of all its tracks (one output run, in track order, each track's hits in
// ascending row order), lane e taking element e of the run: its track is the
// last one whose first hit is at or before e.
__global__ __launch_bounds__(256) void k_track_emit(
    ClusterView cl, const uint32_t* __restrict__ tl_start, FollowOut fo,
    const uint32_t* __restrict__ tlist, const uint16_t* __restrict__ nkept, RefitOut ro,
    const uint32_t* __restrict__ hit_off, TrackOut to, const DevStatus* st) {
  if (failed(st)) return;
  const uint32_t n_trk = min(st->n_tracks, to.capacity);
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t nw = gridDim.x * (blockDim.x >> 6);
  for (uint32_t w = uni(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)); w < (n_trk + 63) / 64;
       w += nw) {
    const uint32_t j0 = w * 64, m = min(64u, n_trk - j0);
    const uint32_t j = j0 + lane;
    uint32_t t = 0, o = 0, n = 0;
    if (lane < m) {
      t = tlist[j];
      o = hit_off[t];
      n = nkept[t];
      to.tracklet[j] = t;
      to.chi2[j] = ro.chi2[t];
      to.ndf[j] = (uint16_t)(2 * n - 5);
      to.row[j] = ro.row[t];
      to.flags[j] = ro.flags[t] & ~TF_TO_FP64;
      to.z_anchor[j] = cl.z_fx[tl_start[t]];
      to.hit_start[j] = o;
    }
    // every lane takes part in each shuffle (the loops are uniform)
    for (uint32_t e0 = 0; e0 < m * 5; e0 += 64) {
      const uint32_t e = e0 + lane, k = min(e / 5, 63u);
      const uint32_t tk = (uint32_t)__shfl((int)t, (int)k);
      if (e < m * 5) to.par[(size_t)j0 * 5 + e] = ro.par[(size_t)tk * 5 + (e - k * 5)];
    }
    for (uint32_t e0 = 0; e0 < m * 15; e0 += 64) {
      const uint32_t e = e0 + lane, k = min(e / 15, 63u);
      const uint32_t tk = (uint32_t)__shfl((int)t, (int)k);
      if (e < m * 15) to.cov[(size_t)j0 * 15 + e] = ro.cov[(size_t)tk * 15 + (e - k * 15)];
    }
    // the wave's hits: offsets relative to its first track's (lanes past the
    // last track hold the end, so no element maps to them)
    const uint32_t o0 = uni((uint32_t)__shfl((int)o, 0));
    const uint32_t last = m - 1;
    const uint32_t end = uni((uint32_t)__shfl((int)(o + n), (int)last)) - o0;
    const uint32_t rel = lane < m ? o - o0 : end;
    for (uint32_t e0 = 0; e0 < end; e0 += 64) {
      const uint32_t e = e0 + lane;
      uint32_t k = 0;
#pragma unroll
      for (uint32_t step = 32; step > 0; step >>= 1) {
        const uint32_t rk = (uint32_t)__shfl((int)rel, (int)(k + step));
        if (k + step < m && rk <= e) k += step;
      }
      const uint32_t tk = (uint32_t)__shfl((int)t, (int)k);
      const uint32_t rk = (uint32_t)__shfl((int)rel, (int)k);
      if (e < end && o0 + e < to.hit_capacity) {
        const uint32_t i = e - rk;
        to.hits[o0 + e] = (uint32_t)fo.hits[(size_t)tk * NROW + fo.krow[(size_t)tk * NROW + i]];
      }
    }
  }
}

__global__ void k_cluster_track(const uint32_t* __restrict__ owner,
                                const uint32_t* __restrict__ trk_index, const uint32_t* n_cl_dev,
                                uint32_t n_cl_cap, uint32_t tl_cap, int32_t* __restrict__ out,
                                const DevStatus* st) {
  if (failed(st)) return;
  const uint32_t n = scan_count(n_cl_dev, n_cl_cap);
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
    const uint32_t key = owner[c];
    int32_t v = -1;
    if (key) {
      const uint32_t t = 0xFFFFFFu - (key & 0xFFFFFFu);
      if (t < tl_cap) {
        const uint32_t j = trk_index[t];
        if (j != 0xFFFFFFFFu) v = (int32_t)j;
      }
    }
    out[c] = v;
  }
}

// Per-tracklet following result as full rows (debug output).
__global__ void k_follow_export(FollowOut fo, const uint32_t* n_tl_dev, uint32_t tl_cap,
                                int32_t* __restrict__ out, const DevStatus* st) {
  if (failed(st)) return;
  const uint32_t n_tl = scan_count(n_tl_dev, tl_cap);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_tl * NROW;
       i += gridDim.x * blockDim.x) {
    const uint32_t t = i / NROW;
    const int r = i % NROW;
    const int lo = fo.range[t] & 255, hi = fo.range[t] >> 8;
    out[i] = (fo.ok[t] && r >= lo && r <= hi) ? fo.hits[i] : -1;
  }
}
