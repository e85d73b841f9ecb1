/*
 * Seeded synthetic TPC event generator: native core.
 *
 * Input side only.  This file computes where charged-particle helices in a
 * uniform Bz field cross the pad-row planes of the 36 TPC sectors, and turns
 * those crossings into zero-suppressed ADC samples (Gaussian charge spread,
 * electronic noise, rounding, saturation, threshold).  It holds none of the
 * reconstruction arithmetic; both the CPU oracle and the GPU library consume
 * the arrays it produces.
 *
 * Detector model (a reading of the paper's TPC, which it does not specify):
 *   sector s (0..35) is centred at azimuth ((s mod 18) + 0.5) * 20 deg and
 *   spans +-10 deg; sectors 0..17 see z > 0, 18..35 see z < 0;
 *   row r (0..151) sits at local x_r = 85 + 160 r / 151 cm with
 *   n_r = round(66 + 72 r / 151) pads of pitch 2 x_r tan(10 deg) / n_r;
 *   time bin j is centred at tau = j, one bin = 0.5 cm of drift, and a charge
 *   at |z| from a collision at T0 arrives at tau = T0 + 500 - 2|z|.
 *
 * Random numbers: every (unit,row) of the digitizer owns a splitmix64 stream
 * seeded from (seed, unit, row), so results do not depend on threading.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NROW 152
#define PI_D 3.14159265358979323846

/* ---------------------------------------------------------------- geometry */
static double g_x[NROW], g_pitch[NROW];
static int g_np[NROW];
static int g_geo_ready = 0;

static void geo_init(void) {
  if (g_geo_ready) return;
  const double t10 = tan(10.0 * PI_D / 180.0);
  for (int r = 0; r < NROW; ++r) {
    g_x[r] = 85.0 + r * 160.0 / 151.0;
    g_np[r] = (int)floor(66.0 + 72.0 * r / 151.0 + 0.5);
    g_pitch[r] = 2.0 * g_x[r] * t10 / g_np[r];
  }
  g_geo_ready = 1;
}

void synth_geometry(double* x, double* pitch, int32_t* npads) {
  geo_init();
  for (int r = 0; r < NROW; ++r) {
    x[r] = g_x[r];
    pitch[r] = g_pitch[r];
    npads[r] = g_np[r];
  }
}

/* -------------------------------------------------------------- crossings */
/*
 * One crossing of a helix with a row plane.  The helix starts at the vertex
 * (vx,vy,vz) with transverse direction phi0, curvature C = dphi/ds
 * (= -q * 1.49896229e-3 / pT per cm at 0.5 T) and dip tgl = dz/ds; it is
 * followed for a turning angle of at most 2 pi and while |z| <= 250 cm.
 */
typedef struct {
  int32_t track, unit, row, leg;  /* leg: +1 outgoing (local cos phi > 0), -1 incoming */
  double s;                       /* 2-D arc length from the vertex */
  double y, z, snp, mu_pad, mu_time;
} crossing_t;

static int cmp_s(const void* a, const void* b) {
  double sa = ((const crossing_t*)a)->s, sb = ((const crossing_t*)b)->s;
  return (sa > sb) - (sa < sb);
}

/*
 * Crossings of n tracks.  sector_mode 0: all 36 sectors; 1: sector 0 only.
 * Count pass (offsets == NULL): writes the number of crossings of each track
 * to counts[].  Fill pass: writes track i's crossings, ordered by arc length,
 * starting at offsets[i].
 */
void synth_crossings(int64_t n, const double* vx, const double* vy, const double* vz,
                     const double* phi0, const double* curv, const double* tgl,
                     const double* t0, int32_t sector_mode, int32_t n_time_bins,
                     int64_t* counts, const int64_t* offsets, int32_t* o_track,
                     int32_t* o_unit, int32_t* o_row, int32_t* o_leg, double* o_y,
                     double* o_z, double* o_snp, double* o_mu_pad, double* o_mu_time,
                     double* o_s) {
  geo_init();
  const double t10 = tan(10.0 * PI_D / 180.0);
#pragma omp parallel
  {
    crossing_t* buf = (crossing_t*)malloc(sizeof(crossing_t) * 18 * NROW * 2);
#pragma omp for schedule(dynamic, 64)
    for (int64_t it = 0; it < n; ++it) {
      const double C = curv[it];
      const double cx = vx[it] - sin(phi0[it]) / C;
      const double cy = vy[it] + cos(phi0[it]) / C;
      const double smax = 2.0 * PI_D / fabs(C);
      int nb = 0;
      const int naz = sector_mode == 1 ? 1 : 18;
      for (int a = 0; a < naz; ++a) {
        const double alpha = (a + 0.5) * 20.0 * PI_D / 180.0;
        const double ca = cos(alpha), sa = sin(alpha);
        const double nc = ca * cx + sa * cy;  /* centre along the row normal */
        const double mc = -sa * cx + ca * cy; /* centre along the row */
        for (int r = 0; r < NROW; ++r) {
          const double k = C * (g_x[r] - nc);
          if (k < -1.0 || k > 1.0) continue;
          const double as = asin(k);
          for (int br = 0; br < 2; ++br) {
            /* local direction angle psi - alpha = asin(k) or pi - asin(k) */
            const double rel = br == 0 ? as : PI_D - as;
            const double psi = alpha + rel;
            /* arc s with |C| s = turning angle in [0, 2 pi) */
            double turn = C > 0 ? psi - phi0[it] : phi0[it] - psi;
            turn = fmod(turn, 2.0 * PI_D);
            if (turn < 0) turn += 2.0 * PI_D;
            const double s = turn / fabs(C);
            if (s > smax) continue;
            const double cosrel = cos(rel);
            const double y = mc - cosrel / C;
            if (fabs(y) > g_x[r] * t10) continue;
            const double z = vz[it] + s * tgl[it];
            if (fabs(z) > 250.0 || z == 0.0) continue;
            const int sector = a + (z < 0 ? 18 : 0);
            if (sector_mode == 1 && sector != 0) continue;
            const double mu_pad = y / g_pitch[r] + 0.5 * (g_np[r] - 1);
            const double mu_time = t0[it] + 500.0 - 2.0 * fabs(z);
            if (mu_pad < -0.5 || mu_pad > g_np[r] - 0.5) continue;
            if (mu_time < -0.5 || mu_time > n_time_bins - 0.5) continue;
            crossing_t* c = &buf[nb++];
            c->track = (int32_t)it;
            c->unit = sector_mode == 1 ? 0 : sector;
            c->row = r;
            c->leg = cosrel > 0 ? 1 : -1;
            c->s = s;
            c->y = y;
            c->z = z;
            c->snp = k;
            c->mu_pad = mu_pad;
            c->mu_time = mu_time;
          }
        }
      }
      counts[it] = nb;
      if (!offsets) continue;
      qsort(buf, nb, sizeof(crossing_t), cmp_s);
      for (int i = 0; i < nb; ++i) {
        const int64_t o = offsets[it] + i;
        const crossing_t* c = &buf[i];
        o_track[o] = c->track;
        o_unit[o] = c->unit;
        o_row[o] = c->row;
        o_leg[o] = c->leg;
        o_y[o] = c->y;
        o_z[o] = c->z;
        o_snp[o] = c->snp;
        o_mu_pad[o] = c->mu_pad;
        o_mu_time[o] = c->mu_time;
        o_s[o] = c->s;
      }
    }
    free(buf);
  }
}

/* ------------------------------------------------------------ random bits */
static inline uint64_t splitmix64(uint64_t* st) {
  uint64_t z = (*st += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
/* uniform in (0,1) */
static inline double u01(uint64_t* st) {
  return ((splitmix64(st) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}
static inline double gauss(uint64_t* st) {
  /* Box-Muller, one of the pair */
  const double u1 = u01(st), u2 = u01(st);
  return sqrt(-2.0 * log(u1)) * cos(2.0 * PI_D * u2);
}
/* standard normal conditioned on x >= a (a > 0): Marsaglia's tail method */
static inline double gauss_tail(uint64_t* st, double a) {
  for (;;) {
    const double x = -log(u01(st)) / a;
    const double y = -log(u01(st));
    if (2.0 * y > x * x) return a + x;
  }
}

/* ------------------------------------------------------------- digitizer */
typedef struct {
  int64_t n;
  uint16_t *pad, *time, *adc;
} rowout_t;

static rowout_t* g_rows = NULL;
static int64_t g_nrows = 0;

static double phi_cdf(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }

/*
 * Digitize deposits into zero-suppressed samples, one (unit,row) at a time.
 * Deposits are grouped by unit*152+row through dep_start[n_units*152+1].
 * Every sample that receives charge from a deposit's +-3 window gets
 * Gaussian noise of width sigma_noise; every other sample fires as noise with
 * probability P(noise >= 2.5), with its value drawn from the conditioned
 * normal.  ADC = clip(rint(v), 0, 1023); samples with ADC >= 3 are kept,
 * except on dead pads (dead[(unit*152+row)*138+pad] != 0), which are dropped.
 * Results are held until synth_digitize_fetch copies them out.
 */
int64_t synth_digitize(int32_t n_units, int32_t n_time_bins, const int64_t* dep_start,
                       const double* mu_pad, const double* mu_time, const double* q,
                       double sigma_shape, double sigma_noise, const uint8_t* dead,
                       uint64_t seed, int64_t* row_counts) {
  geo_init();
  if (g_rows) {
    for (int64_t i = 0; i < g_nrows; ++i) {
      free(g_rows[i].pad);
      free(g_rows[i].time);
      free(g_rows[i].adc);
    }
    free(g_rows);
  }
  g_nrows = (int64_t)n_units * NROW;
  g_rows = (rowout_t*)calloc(g_nrows, sizeof(rowout_t));
  const double p_noise = 0.5 * erfc(2.5 / sigma_noise / sqrt(2.0));
  const double log1mp = log1p(-p_noise);
  const int64_t T = n_time_bins;
  const int64_t npos_max = T * 138;
  const int64_t nwords_max = (npos_max + 63) / 64;
  int64_t total = 0;
#pragma omp parallel reduction(+ : total)
  {
    /* per-thread dense accumulator and "signal touched" bitmap, cleared
       sparsely after each row */
    float* buf = (float*)calloc((size_t)npos_max, sizeof(float));
    uint64_t* bits = (uint64_t*)calloc((size_t)nwords_max, sizeof(uint64_t));
#pragma omp for schedule(dynamic, 4)
    for (int64_t ur = 0; ur < g_nrows; ++ur) {
      const int r = (int)(ur % NROW);
      const int np = g_np[r];
      const int64_t npos = T * np;
      const int64_t nwords = (npos + 63) / 64;
      for (int64_t d = dep_start[ur]; d < dep_start[ur + 1]; ++d) {
        const int pc = (int)floor(mu_pad[d] + 0.5), tc = (int)floor(mu_time[d] + 0.5);
        double fp[7], ft[7];
        for (int k = 0; k < 7; ++k) {
          const double p = pc - 3 + k, t = tc - 3 + k;
          fp[k] = phi_cdf((p + 0.5 - mu_pad[d]) / sigma_shape) -
                  phi_cdf((p - 0.5 - mu_pad[d]) / sigma_shape);
          ft[k] = phi_cdf((t + 0.5 - mu_time[d]) / sigma_shape) -
                  phi_cdf((t - 0.5 - mu_time[d]) / sigma_shape);
        }
        for (int kt = 0; kt < 7; ++kt) {
          const int t = tc - 3 + kt;
          if (t < 0 || t >= T) continue;
          for (int kp = 0; kp < 7; ++kp) {
            const int p = pc - 3 + kp;
            if (p < 0 || p >= np) continue;
            const int64_t pos = (int64_t)t * np + p;
            buf[pos] += (float)(q[d] * fp[kp] * ft[kt]);
            bits[pos >> 6] |= 1ull << (pos & 63);
          }
        }
      }
      uint64_t st = seed ^ (0xD1B54A32D192ED03ull * (uint64_t)(ur + 1));
      splitmix64(&st);
      const uint8_t* dmask = dead ? dead + ur * 138 : NULL;
      int64_t cap = 256, n = 0;
      uint16_t* op = (uint16_t*)malloc(cap * 2);
      uint16_t* ot = (uint16_t*)malloc(cap * 2);
      uint16_t* oa = (uint16_t*)malloc(cap * 2);
      /* noise-only candidates: geometric skipping over all positions; a
         candidate that lands on a signal position is discarded, so every
         signal-free position fires independently with probability p_noise */
      int64_t next_noise = p_noise > 0 ? (int64_t)floor(log(u01(&st)) / log1mp) : npos;
      int64_t w = 0;
      uint64_t cur = nwords > 0 ? bits[0] : 0;
      for (;;) {
        /* next signal position */
        while (cur == 0 && w + 1 < nwords) cur = bits[++w];
        const int64_t next_sig = cur ? (w << 6) + __builtin_ctzll(cur) : npos;
        int64_t pos;
        double v;
        if (next_sig >= npos && next_noise >= npos) break;
        if (next_sig <= next_noise) {
          pos = next_sig;
          cur &= cur - 1;
          if (next_noise == pos)
            next_noise = pos + 1 + (int64_t)floor(log(u01(&st)) / log1mp);
          v = buf[pos] + sigma_noise * gauss(&st);
          buf[pos] = 0.0f;
        } else {
          pos = next_noise;
          v = sigma_noise * gauss_tail(&st, 2.5 / sigma_noise);
          next_noise = pos + 1 + (int64_t)floor(log(u01(&st)) / log1mp);
        }
        double a = rint(v);
        if (a < 0) a = 0;
        if (a > 1023) a = 1023;
        if (a < 3) continue;
        const int p = (int)(pos % np), t = (int)(pos / np);
        if (dmask && dmask[p]) continue;
        if (n == cap) {
          cap *= 2;
          op = (uint16_t*)realloc(op, cap * 2);
          ot = (uint16_t*)realloc(ot, cap * 2);
          oa = (uint16_t*)realloc(oa, cap * 2);
        }
        op[n] = (uint16_t)p;
        ot[n] = (uint16_t)t;
        oa[n] = (uint16_t)a;
        ++n;
      }
      for (int64_t k = 0; k < nwords; ++k) bits[k] = 0;
      g_rows[ur].n = n;
      g_rows[ur].pad = op;
      g_rows[ur].time = ot;
      g_rows[ur].adc = oa;
      row_counts[ur] = n;
      total += n;
    }
    free(buf);
    free(bits);
  }
  return total;
}

/* Copy the held samples out, in (unit,row,time,pad) order, and release them. */
void synth_digitize_fetch(uint16_t* pad, uint16_t* time, uint16_t* adc) {
  int64_t off = 0;
  for (int64_t i = 0; i < g_nrows; ++i) {
    memcpy(pad + off, g_rows[i].pad, g_rows[i].n * 2);
    memcpy(time + off, g_rows[i].time, g_rows[i].n * 2);
    memcpy(adc + off, g_rows[i].adc, g_rows[i].n * 2);
    off += g_rows[i].n;
    free(g_rows[i].pad);
    free(g_rows[i].time);
    free(g_rows[i].adc);
  }
  free(g_rows);
  g_rows = NULL;
  g_nrows = 0;
}

/* ------------------------------------------------------------ raw pages */
/* Packs sorted zero-suppressed samples into the library's raw page format
 * (8 KiB pages of 2048 little-endian words; header, run table, 10-bit ADC
 * stream; the format is stated with tpc_decode_zs_pages).  One (unit,row)
 * per page; a row continues on a new page when the next sample no longer
 * fits.  Consecutive pads of one time bin form a run of up to 256 samples.
 * out == NULL counts the pages only.  Returns the number of pages. */
#define PG_WORDS 2048
static void pg_flush(uint32_t* pg, int unit, int row, const uint32_t* runs, int nr,
                     const uint16_t* adc, int ns) {
  memset(pg, 0, PG_WORDS * sizeof(uint32_t));
  pg[0] = 0x5A53u | (1u << 16);
  pg[1] = (uint32_t)unit | ((uint32_t)row << 16);
  pg[2] = (uint32_t)nr | ((uint32_t)ns << 16);
  for (int i = 0; i < nr; ++i) pg[4 + i] = runs[i];
  uint32_t* st = pg + 4 + nr;
  for (int k = 0; k < ns; ++k) {
    const uint64_t bit = (uint64_t)k * 10;
    const uint64_t v = (uint64_t)(adc[k] & 0x3FF) << (bit & 31);
    st[bit >> 5] |= (uint32_t)v;
    if ((bit & 31) > 22) st[(bit >> 5) + 1] |= (uint32_t)(v >> 32);
  }
}

int64_t synth_pack_pages(int32_t n_units, const uint32_t* row_start, const uint16_t* pad,
                         const uint16_t* time, const uint16_t* adc, uint32_t* out) {
  static uint32_t runs[PG_WORDS];
  static uint16_t padc[PG_WORDS * 4];
  int64_t np = 0;
  for (int64_t ur = 0; ur < (int64_t)n_units * NROW; ++ur) {
    const int unit = (int)(ur / NROW), row = (int)(ur % NROW);
    int nr = 0, ns = 0;
    int last_t = -1, last_p = -2, last_len = 0;
    for (uint32_t s = row_start[ur]; s < row_start[ur + 1]; ++s) {
      const int t = time[s], p = pad[s];
      const int joins = nr > 0 && t == last_t && p == last_p + 1 && last_len < 256;
      const int nr2 = nr + (joins ? 0 : 1);
      if (4 + nr2 + (int)(((ns + 1) * 10 + 31) / 32) > PG_WORDS) {
        if (out) pg_flush(out + np * PG_WORDS, unit, row, runs, nr, padc, ns);
        ++np;
        nr = ns = 0;
      }
      if (nr > 0 && t == last_t && p == last_p + 1 && last_len < 256) {
        ++last_len;
        runs[nr - 1] += 1u << 24;
      } else {
        runs[nr++] = (uint32_t)t | ((uint32_t)p << 16);
        last_len = 1;
      }
      last_t = t;
      last_p = p;
      padc[ns++] = adc[s];
    }
    if (ns > 0) {
      if (out) pg_flush(out + np * PG_WORDS, unit, row, runs, nr, padc, ns);
      ++np;
    }
  }
  return np;
}
