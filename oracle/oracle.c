/*
 * CPU ORACLE FOR TPC TRACK RECONSTRUCTION -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, double-precision reference of the reconstruction chain that
 * the paper names as the most compute-intensive part of synchronous
 * processing (section "Hardware and data flow": full online TPC track
 * reconstruction on the EPN GPUs).  The paper gives no algorithmic detail;
 * every step below follows the stated reading of it, one function per step:
 *
 *   geometry ............ detector reading (36 sectors x 152 rows)
 *   clusterize .......... peak finding + 2-step uphill assignment + moments
 *   fixed-point position  y_fx / z_fx from the integer moments
 *   neighbours .......... cellular-automaton neighbour choice per cluster
 *   CA clean / tracklets  reciprocal links, chains of >= MIN_TRACKLET hits
 *   seed ................ 3-point circle + dip
 *   Kalman primitives ... exact helix propagation, Jacobian, update
 *   following ........... outward pass A, inward pass B with hit pick-up
 *   resolution .......... each cluster kept by its highest-priority track
 *   refit ............... inward Kalman refit over the kept hits
 *
 * Only tests/, the smoke check and the benchmark's cpu_baseline leg may load
 * this library.  It shares no code, header or table with the GPU library.
 * Integer steps are exact; floating-point steps use IEEE binary64.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NROW 152
#define NPADMAX 138
#define PI_D 3.14159265358979323846

/* ------------------------------------------------------------ parameters */
typedef struct {
  int32_t qmax_min;        /* peak threshold on the peak ADC */
  int32_t min_tracklet;    /* minimum tracklet length */
  int32_t max_miss;        /* consecutive empty rows that stop following */
  int32_t min_track_hits;  /* minimum hits of a kept track */
  int64_t win_y, win_z;    /* neighbour windows, 2^-16 cm */
  int64_t s_max;           /* neighbour score cut */
  double chi2_max;         /* hit acceptance */
  double snp_max;          /* stop when |sin phi| reaches this */
  double bz_b;             /* curvature per unit q/pT [1/cm per c/GeV] */
  double c0_snp, c0_tgl, c0_qpt; /* seed covariance sigmas */
  double qpt_clamp;        /* |q/pT| clamp of the seed */
  double edge_margin;      /* cm beyond the pad plane that stops following */
  double lowpt_qpt;        /* |q/pT| above which a track counts as low-pT */
  double c0r_y, c0r_z, c0r_snp, c0r_tgl, c0r_qpt; /* refit prior sigmas (broad) */
  double refit_snp_max;    /* |sin phi| a refit step may not reach */
  double sigma_y[NROW], sigma_z[NROW]; /* per-row measurement errors [cm] */
  int32_t brute_force;     /* 1: scan whole rows instead of time windows */
  int32_t n_threads;
} oparams;

/* -------------------------------------------------------------- geometry */
/* Row r at x = 85 + 160 r/151 cm, n_r = round(66 + 72 r/151) pads, pad pitch
   2 x tan(10 deg)/n_r; fixed-point tables in units of 2^-16 cm. */
static int32_t G_NP[NROW];
static int64_t G_XFX[NROW], G_PFX[NROW];
static double G_X[NROW], G_HW[NROW];
static int G_READY = 0;

static void geometry_init(void) {
  if (G_READY) return;
  for (int r = 0; r < NROW; ++r) {
    /* round(num/den) with half up, exact in integers */
    const int64_t np_num = 66 * 151 + 72 * r;
    G_NP[r] = (int32_t)((2 * np_num + 151) / (2 * 151));
    const int64_t x_num = (int64_t)(85 * 151 + 160 * r) * 65536;
    G_XFX[r] = (2 * x_num + 151) / (2 * 151);
    const double x = 85.0 + r * 160.0 / 151.0;
    const double pitch = 2.0 * x * tan(PI_D / 18.0) / G_NP[r];
    G_PFX[r] = (int64_t)floor(pitch * 65536.0 + 0.5);
    G_X[r] = (double)G_XFX[r] / 65536.0;
    G_HW[r] = (double)(G_NP[r] * G_PFX[r]) / 131072.0; /* half the pad plane */
  }
  G_READY = 1;
}

void oracle_geometry(int32_t* npads, int64_t* x_fx, int64_t* p_fx) {
  geometry_init();
  for (int r = 0; r < NROW; ++r) {
    npads[r] = G_NP[r];
    x_fx[r] = G_XFX[r];
    p_fx[r] = G_PFX[r];
  }
}

/* ----------------------------------------------------------- small utils */
static int64_t floor_div(int64_t a, int64_t b) { /* b > 0 */
  int64_t q = a / b;
  if ((a % b != 0) && (a < 0)) --q;
  return q;
}

typedef struct {
  int n_units, n_threads;
  void* ctx;
  void (*fn)(void* ctx, int unit);
  int next;
  pthread_mutex_t mu;
} pool_t;

static void* pool_worker(void* arg) {
  pool_t* p = (pool_t*)arg;
  for (;;) {
    pthread_mutex_lock(&p->mu);
    const int u = p->next++;
    pthread_mutex_unlock(&p->mu);
    if (u >= p->n_units) break;
    p->fn(p->ctx, u);
  }
  return NULL;
}

/* run fn(ctx, u) for every unit u on n_threads threads */
static void for_units(int n_units, int n_threads, void* ctx, void (*fn)(void*, int)) {
  pool_t p;
  p.n_units = n_units;
  p.n_threads = n_threads < 1 ? 1 : n_threads;
  p.ctx = ctx;
  p.fn = fn;
  p.next = 0;
  pthread_mutex_init(&p.mu, NULL);
  if (p.n_threads == 1) {
    pool_worker(&p);
  } else {
    pthread_t th[256];
    const int nt = p.n_threads > 256 ? 256 : p.n_threads;
    for (int i = 0; i < nt; ++i) pthread_create(&th[i], NULL, pool_worker, &p);
    for (int i = 0; i < nt; ++i) pthread_join(th[i], NULL);
  }
  pthread_mutex_destroy(&p.mu);
}

/* ============================================================ clusterizer */
/* Output arrays of the clusterizer (host, caller-owned, capacity = cap). */
typedef struct {
  uint16_t *ppad, *ptime, *qtot, *qmax, *nsamp;
  int32_t *sp, *st, *spp, *stt;
  uint8_t* flags;
  double *pad, *time, *s2pad, *s2time;
  int32_t *y_fx, *z_fx;
  int32_t* sample_label;  /* [n_samples] cluster id or -1 (may be NULL) */
  uint32_t* crow_start;   /* [n_units*152+1] */
} oclusters;

enum { FLAG_EDGE = 1, FLAG_SAT = 2 };

typedef struct {
  /* one cluster before it is placed in the output */
  int32_t ppad, ptime, qtot, qmax, nsamp, sp, st, spp, stt, flags;
  int64_t y_fx, z_fx;
  int64_t peak_sample; /* input index of the peak sample */
} ocl;

typedef struct {
  const oparams* par;
  int32_t n_units, n_time_bins;
  const uint16_t *pad, *time, *adc;
  const uint32_t* row_start;
  ocl** rows;        /* per (unit,row) cluster list */
  int64_t* nrow;     /* per (unit,row) cluster count */
  int32_t* label_peak; /* per sample: input index of its peak, or -1 */
} clus_job;

/* key order: larger ADC wins, then larger time, then larger pad */
static inline int64_t sample_key(int64_t adc, int64_t t, int64_t p) {
  return adc * (1LL << 24) + t * (1LL << 8) + p;
}

static void clusterize_row(clus_job* J, int64_t ur) {
  const int r = (int)(ur % NROW);
  const int np = G_NP[r];
  const int64_t s0 = J->row_start[ur], s1 = J->row_start[ur + 1];
  const int64_t n = s1 - s0;
  J->rows[ur] = NULL;
  J->nrow[ur] = 0;
  if (n == 0) return;
  /* dense map (time,pad) -> sample index within the row, -1 if absent,
     over the time bins the row occupies (samples are time-sorted) */
  const int64_t tmin = J->time[s0], tspan = (int64_t)J->time[s1 - 1] - tmin + 1;
  int32_t* grid = (int32_t*)malloc(sizeof(int32_t) * (size_t)(tspan * np));
  for (int64_t i = 0; i < tspan * np; ++i) grid[i] = -1;
  for (int64_t i = 0; i < n; ++i)
    grid[((int64_t)J->time[s0 + i] - tmin) * np + J->pad[s0 + i]] = (int32_t)i;
  /* up(s): argmax of the key over s and its present 8-neighbours */
  int32_t* up = (int32_t*)malloc(sizeof(int32_t) * n);
  for (int64_t i = 0; i < n; ++i) {
    const int t = J->time[s0 + i], p = J->pad[s0 + i];
    int64_t best_key = sample_key(J->adc[s0 + i], t, p);
    int32_t best = (int32_t)i;
    for (int dt = -1; dt <= 1; ++dt)
      for (int dp = -1; dp <= 1; ++dp) {
        const int tt = t + dt, pp = p + dp;
        if ((dt == 0 && dp == 0) || tt < tmin || tt >= tmin + tspan || pp < 0 || pp >= np)
          continue;
        const int32_t j = grid[((int64_t)tt - tmin) * np + pp];
        if (j < 0) continue;
        const int64_t k = sample_key(J->adc[s0 + j], tt, pp);
        if (k > best_key) {
          best_key = k;
          best = j;
        }
      }
    up[i] = best;
  }
  /* peak: a key maximum of its neighbourhood whose ADC reaches the threshold */
  uint8_t* is_peak = (uint8_t*)malloc(n);
  for (int64_t i = 0; i < n; ++i)
    is_peak[i] = (up[i] == i) && (J->adc[s0 + i] >= J->par->qmax_min);
  /* assignment: the peak reached in at most two uphill steps */
  int32_t* owner = (int32_t*)malloc(sizeof(int32_t) * n);
  for (int64_t i = 0; i < n; ++i) {
    const int32_t u1 = up[i], u2 = up[u1];
    owner[i] = is_peak[u1] ? u1 : (is_peak[u2] ? u2 : -1);
  }
  /* moments, in the order of the peaks (time, then pad) */
  int64_t npk = 0;
  for (int64_t i = 0; i < n; ++i) npk += is_peak[i];
  ocl* out = (ocl*)calloc(npk > 0 ? npk : 1, sizeof(ocl));
  int32_t* slot = (int32_t*)malloc(sizeof(int32_t) * n);
  int64_t k = 0;
  for (int64_t i = 0; i < n; ++i) {
    slot[i] = -1;
    if (!is_peak[i]) continue;
    slot[i] = (int32_t)k;
    out[k].ppad = J->pad[s0 + i];
    out[k].ptime = J->time[s0 + i];
    out[k].qmax = J->adc[s0 + i];
    out[k].peak_sample = s0 + i;
    ++k;
  }
  for (int64_t i = 0; i < n; ++i) {
    const int32_t o = owner[i];
    if (J->label_peak) J->label_peak[s0 + i] = o < 0 ? -1 : (int32_t)(s0 + o);
    if (o < 0) continue;
    ocl* c = &out[slot[o]];
    const int a = J->adc[s0 + i];
    const int dp = (int)J->pad[s0 + i] - c->ppad, dt = (int)J->time[s0 + i] - c->ptime;
    c->qtot += a;
    c->sp += a * dp;
    c->st += a * dt;
    c->spp += a * dp * dp;
    c->stt += a * dt * dt;
    c->nsamp += 1;
    if (a >= 1023) c->flags |= FLAG_SAT;
  }
  for (int64_t j = 0; j < npk; ++j) {
    ocl* c = &out[j];
    if (c->ppad <= 1 || c->ppad >= np - 2) c->flags |= FLAG_EDGE;
    /* fixed-point positions, round half up */
    const int64_t Q = c->qtot;
    const int64_t u = 2 * ((int64_t)c->ppad * Q + c->sp) - (int64_t)(np - 1) * Q;
    c->y_fx = floor_div(u * G_PFX[r] + Q, 2 * Q);
    c->z_fx = floor_div(65536 * ((int64_t)c->ptime * Q + c->st) + Q, 2 * Q);
  }
  J->rows[ur] = out;
  J->nrow[ur] = npk;
  free(grid);
  free(up);
  free(is_peak);
  free(owner);
  free(slot);
}

static void clusterize_unit(void* ctx, int unit) {
  clus_job* J = (clus_job*)ctx;
  for (int r = 0; r < NROW; ++r) clusterize_row(J, (int64_t)unit * NROW + r);
}

/* Returns the number of clusters (written only if it fits cap), or -1 if the
   input is not sorted or out of range (pad beyond the row, time beyond the
   frame, ADC 0 or above 10 bits). */
int64_t oracle_cluster(const oparams* par, int32_t n_units, int32_t n_time_bins,
                       const uint16_t* pad, const uint16_t* time, const uint16_t* adc,
                       const uint32_t* row_start, int64_t cap, oclusters* out) {
  geometry_init();
  const int64_t nur = (int64_t)n_units * NROW;
  /* input contract: sorted by (time, pad) within each (unit,row), in range */
  for (int64_t ur = 0; ur < nur; ++ur) {
    const int np = G_NP[ur % NROW];
    if (row_start[ur + 1] < row_start[ur]) return -1;
    for (int64_t s = row_start[ur]; s < row_start[ur + 1]; ++s) {
      if (pad[s] >= np || time[s] >= n_time_bins) return -1;
      if (adc[s] == 0 || adc[s] > 1023) return -1; /* 10-bit ADC, zero never stored */
      if (s > row_start[ur] &&
          (int64_t)time[s] * 256 + pad[s] <= (int64_t)time[s - 1] * 256 + pad[s - 1])
        return -1;
    }
  }
  clus_job J;
  J.par = par;
  J.n_units = n_units;
  J.n_time_bins = n_time_bins;
  J.pad = pad;
  J.time = time;
  J.adc = adc;
  J.row_start = row_start;
  J.rows = (ocl**)calloc(nur, sizeof(ocl*));
  J.nrow = (int64_t*)calloc(nur, sizeof(int64_t));
  const int64_t ns = row_start[nur];
  J.label_peak = out->sample_label ? (int32_t*)malloc(sizeof(int32_t) * (ns > 0 ? ns : 1)) : NULL;
  for_units(n_units, par->n_threads, &J, clusterize_unit);
  int64_t total = 0;
  for (int64_t ur = 0; ur < nur; ++ur) total += J.nrow[ur];
  if (total <= cap) {
    int64_t k = 0;
    int32_t* peak_to_cluster = J.label_peak ? (int32_t*)malloc(sizeof(int32_t) * (ns > 0 ? ns : 1)) : NULL;
    for (int64_t ur = 0; ur < nur; ++ur) {
      out->crow_start[ur] = (uint32_t)k;
      for (int64_t j = 0; j < J.nrow[ur]; ++j, ++k) {
        const ocl* c = &J.rows[ur][j];
        out->ppad[k] = (uint16_t)c->ppad;
        out->ptime[k] = (uint16_t)c->ptime;
        out->qtot[k] = (uint16_t)c->qtot;
        out->qmax[k] = (uint16_t)c->qmax;
        out->nsamp[k] = (uint16_t)c->nsamp;
        out->sp[k] = c->sp;
        out->st[k] = c->st;
        out->spp[k] = c->spp;
        out->stt[k] = c->stt;
        out->flags[k] = (uint8_t)c->flags;
        const double Q = c->qtot;
        out->pad[k] = c->ppad + c->sp / Q;
        out->time[k] = c->ptime + c->st / Q;
        out->s2pad[k] = c->spp / Q - (c->sp / Q) * (c->sp / Q);
        out->s2time[k] = c->stt / Q - (c->st / Q) * (c->st / Q);
        out->y_fx[k] = (int32_t)c->y_fx;
        out->z_fx[k] = (int32_t)c->z_fx;
        if (peak_to_cluster) peak_to_cluster[c->peak_sample] = (int32_t)k;
      }
    }
    out->crow_start[nur] = (uint32_t)k;
    if (J.label_peak)
      for (int64_t s = 0; s < ns; ++s)
        out->sample_label[s] = J.label_peak[s] < 0 ? -1 : peak_to_cluster[J.label_peak[s]];
    free(peak_to_cluster);
  }
  for (int64_t ur = 0; ur < nur; ++ur) free(J.rows[ur]);
  free(J.rows);
  free(J.nrow);
  free(J.label_peak);
  return total;
}

/* ============================================================ neighbours */
/* first cluster of [a,b) (sorted by peak time) with ptime >= t */
static int64_t lower_time(const uint16_t* ptime, int64_t a, int64_t b, int64_t t) {
  while (a < b) {
    const int64_t m = (a + b) / 2;
    if ((int64_t)ptime[m] < t) a = m + 1;
    else b = m;
  }
  return a;
}

typedef struct {
  const oparams* par;
  const int32_t *y, *z;
  const uint16_t* ptime;
  const uint32_t* crow_start;
  int32_t *down, *up;
} nb_job;

/* candidate range of a neighbour row for a cluster at z (fixed point):
   |z_c - z| <= win_z and the centroid lies within 2 bins of the peak time */
static void nb_range(const nb_job* J, int64_t ur, int64_t z, int64_t* a, int64_t* b) {
  *a = J->crow_start[ur];
  *b = J->crow_start[ur + 1];
  if (J->par->brute_force) return;
  const int64_t lo = floor_div(z - J->par->win_z, 32768) - 3;
  const int64_t hi = floor_div(z + J->par->win_z, 32768) + 4;
  *a = lower_time(J->ptime, *a, *b, lo);
  *b = lower_time(J->ptime, *a, *b, hi);
}

static void neighbours_unit(void* ctx, int unit) {
  nb_job* J = (nb_job*)ctx;
  const int64_t base = (int64_t)unit * NROW;
  for (int r = 0; r < NROW; ++r) {
    for (int64_t i = J->crow_start[base + r]; i < J->crow_start[base + r + 1]; ++i) {
      J->down[i] = -1;
      J->up[i] = -1;
      if (r == 0 || r == NROW - 1) continue;
      const int64_t yi = J->y[i], zi = J->z[i];
      int64_t ja, jb, ka, kb;
      nb_range(J, base + r - 1, zi, &ja, &jb);
      nb_range(J, base + r + 1, zi, &ka, &kb);
      int64_t best_s = -1, best_j = -1, best_k = -1;
      for (int64_t j = ja; j < jb; ++j) {
        if (llabs(J->y[j] - yi) > J->par->win_y || llabs(J->z[j] - zi) > J->par->win_z) continue;
        for (int64_t k = ka; k < kb; ++k) {
          if (llabs(J->y[k] - yi) > J->par->win_y || llabs(J->z[k] - zi) > J->par->win_z)
            continue;
          const int64_t dy = 2 * yi - J->y[j] - J->y[k];
          const int64_t dz = 2 * zi - J->z[j] - J->z[k];
          const int64_t s = dy * dy + dz * dz;
          if (s > J->par->s_max) continue;
          /* lexicographic minimum of (score, j, k); j and k ascend here */
          if (best_s < 0 || s < best_s) {
            best_s = s;
            best_j = j;
            best_k = k;
          }
        }
      }
      if (best_s >= 0) {
        J->down[i] = (int32_t)best_j;
        J->up[i] = (int32_t)best_k;
      }
    }
  }
}

void oracle_find_neighbours(const oparams* par, int32_t n_units, const int32_t* y_fx,
                            const int32_t* z_fx, const uint16_t* ptime,
                            const uint32_t* crow_start, int32_t* down, int32_t* up) {
  geometry_init();
  nb_job J = {par, y_fx, z_fx, ptime, crow_start, down, up};
  for_units(n_units, par->n_threads, &J, neighbours_unit);
}

/* ============================================================ CA/tracklets */
/* Cleaned links keep only reciprocal pairs; a start has no cleaned down-link
   and a cleaned up-link; a tracklet is a start plus its up-chain, kept when it
   has at least min_tracklet clusters.  Tracklets are numbered by ascending
   start cluster.  Returns the number of tracklets (written if <= cap). */
int64_t oracle_build_tracklets(const oparams* par, int64_t n_clusters, const int32_t* down,
                               const int32_t* up, int32_t* downc, int32_t* upc, int64_t cap,
                               uint32_t* tl_start, uint16_t* tl_len) {
  for (int64_t i = 0; i < n_clusters; ++i) {
    upc[i] = (up[i] >= 0 && down[up[i]] == i) ? up[i] : -1;
    downc[i] = (down[i] >= 0 && up[down[i]] == i) ? down[i] : -1;
  }
  int64_t nt = 0;
  for (int64_t i = 0; i < n_clusters; ++i) {
    if (downc[i] != -1 || upc[i] == -1) continue;
    int64_t len = 1;
    for (int64_t c = upc[i]; c != -1; c = upc[c]) ++len;
    if (len < par->min_tracklet) continue;
    if (nt < cap) {
      tl_start[nt] = (uint32_t)i;
      tl_len[nt] = (uint16_t)len;
    }
    ++nt;
  }
  return nt;
}

/* ============================================================ Kalman */
/* Track state p = (y, z, snp, tgl, q/pT) at local x; z relative to the
   tracklet anchor; covariance as a full symmetric 5x5 matrix. */
typedef struct {
  double p[5];
  double C[5][5];
  double x;
} kstate;

typedef struct {
  int near_tie; /* decisions within the stated margins */
  double snp_margin;
} ktrace;

static const double GL8_X[8] = {0.01985507175123188, 0.10166676129318664, 0.2372337950418355,
                                0.4082826787521751,  0.5917173212478249,  0.7627662049581645,
                                0.8983332387068134,  0.9801449282487681};
static const double GL8_W[8] = {0.05061426814518813, 0.11119051722668724, 0.15685332293894363,
                                0.18134189168918100, 0.18134189168918100, 0.15685332293894363,
                                0.11119051722668724, 0.05061426814518813};

/* d(signed arc)/dC at fixed dx and s1: the integral over u in [0, dx] of
   u * s (1 - s^2)^(-3/2) with s = s1 + C u, by 8-point Gauss-Legendre */
static double darc_dc(double s1, double C, double dx) {
  double acc = 0.0;
  for (int i = 0; i < 8; ++i) {
    const double s = s1 + C * dx * GL8_X[i];
    const double w = 1.0 - s * s;
    acc += GL8_W[i] * GL8_X[i] * s / (w * sqrt(w));
  }
  return acc * dx * dx;
}

/* Exact helix propagation in a uniform Bz from x1 to x2 (no material).
   Returns 0 on success, 1 if |snp| would reach snp_max.  If J is given it
   receives the 5x5 Jacobian. */
static int helix_propagate(const oparams* par, double p[5], double x1, double x2, double J[5][5],
                           ktrace* tr) {
  const double dx = x2 - x1;
  const double C = -par->bz_b * p[4];
  const double s1 = p[2], s2 = s1 + C * dx;
  if (tr && fabs(fabs(s2) - par->snp_max) < 1e-5) tr->near_tie++;
  if (fabs(s2) >= par->snp_max) return 1;
  const double c1 = sqrt(1.0 - s1 * s1), c2 = sqrt(1.0 - s2 * s2);
  const double D = c1 + c2, N = s1 + s2, f = N / D;
  const double chord = fabs(dx) * sqrt(1.0 + f * f);
  const double h = chord * fabs(C) / 2.0;
  const double L = h > 0 ? chord * asin(h) / h : chord;
  const double A = dx >= 0 ? L : -L; /* signed arc */
  if (J) {
    for (int i = 0; i < 5; ++i)
      for (int j = 0; j < 5; ++j) J[i][j] = i == j;
    J[0][2] = dx * (2.0 * D + N * (s1 / c1 + s2 / c2)) / (D * D);
    J[0][4] = -par->bz_b * dx * dx * (D + N * s2 / c2) / (D * D);
    J[1][2] = p[3] * dx * N / (c1 * c2 * D);
    J[1][3] = A;
    J[1][4] = -par->bz_b * p[3] * darc_dc(s1, C, dx);
    J[2][4] = -par->bz_b * dx;
  }
  p[0] += dx * f;
  p[1] += p[3] * A;
  p[2] = s2;
  return 0;
}

static int kstate_propagate(const oparams* par, kstate* k, double x2, ktrace* tr) {
  double J[5][5];
  double p[5];
  memcpy(p, k->p, sizeof p);
  if (helix_propagate(par, p, k->x, x2, J, tr)) return 1;
  double T[5][5], Cn[5][5];
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) {
      double a = 0;
      for (int m = 0; m < 5; ++m) a += J[i][m] * k->C[m][j];
      T[i][j] = a;
    }
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) {
      double a = 0;
      for (int m = 0; m < 5; ++m) a += T[i][m] * J[j][m];
      Cn[i][j] = a;
    }
  memcpy(k->p, p, sizeof p);
  memcpy(k->C, Cn, sizeof Cn);
  k->x = x2;
  return 0;
}

/* chi^2 of a 2-D measurement (my, mz) with variances (vy, vz) */
static double kstate_chi2(const kstate* k, double my, double mz, double vy, double vz) {
  const double r0 = my - k->p[0], r1 = mz - k->p[1];
  const double S00 = k->C[0][0] + vy, S01 = k->C[0][1], S11 = k->C[1][1] + vz;
  const double det = S00 * S11 - S01 * S01;
  return (r0 * r0 * S11 - 2.0 * r0 * r1 * S01 + r1 * r1 * S00) / det;
}

/* Kalman update; returns 1 (and leaves k unchanged) if |snp| >= 1 after it */
static int kstate_update(kstate* k, double my, double mz, double vy, double vz, double* chi2,
                         ktrace* tr) {
  const double r0 = my - k->p[0], r1 = mz - k->p[1];
  const double S00 = k->C[0][0] + vy, S01 = k->C[0][1], S11 = k->C[1][1] + vz;
  const double det = S00 * S11 - S01 * S01;
  const double I00 = S11 / det, I01 = -S01 / det, I11 = S00 / det;
  if (chi2) *chi2 = r0 * r0 * I00 + 2.0 * r0 * r1 * I01 + r1 * r1 * I11;
  double K[5][2];
  for (int i = 0; i < 5; ++i) {
    K[i][0] = k->C[i][0] * I00 + k->C[i][1] * I01;
    K[i][1] = k->C[i][0] * I01 + k->C[i][1] * I11;
  }
  double p[5];
  for (int i = 0; i < 5; ++i) p[i] = k->p[i] + K[i][0] * r0 + K[i][1] * r1;
  if (tr && fabs(fabs(p[2]) - 1.0) < 1e-5) tr->near_tie++;
  if (fabs(p[2]) >= 1.0) return 1;
  double Cn[5][5];
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) Cn[i][j] = k->C[i][j] - (K[i][0] * k->C[0][j] + K[i][1] * k->C[1][j]);
  /* keep the stored matrix exactly symmetric */
  for (int i = 0; i < 5; ++i)
    for (int j = i + 1; j < 5; ++j) Cn[j][i] = Cn[i][j] = 0.5 * (Cn[i][j] + Cn[j][i]);
  memcpy(k->p, p, sizeof p);
  memcpy(k->C, Cn, sizeof Cn);
  return 0;
}

/* positive definiteness through an LDL^T factorisation: all pivots > 0 */
static int is_pd(const double C[5][5]) {
  double L[5][5] = {{0}}, D[5];
  for (int j = 0; j < 5; ++j) {
    double d = C[j][j];
    for (int m = 0; m < j; ++m) d -= L[j][m] * L[j][m] * D[m];
    if (!(d > 0)) return 0;
    D[j] = d;
    L[j][j] = 1;
    for (int i = j + 1; i < 5; ++i) {
      double a = C[i][j];
      for (int m = 0; m < j; ++m) a -= L[i][m] * L[j][m] * D[m];
      L[i][j] = a / d;
    }
  }
  return 1;
}

static void c0_reset(const oparams* par, kstate* k, int row) {
  memset(k->C, 0, sizeof k->C);
  k->C[0][0] = par->sigma_y[row] * par->sigma_y[row];
  k->C[1][1] = par->sigma_z[row] * par->sigma_z[row];
  k->C[2][2] = par->c0_snp * par->c0_snp;
  k->C[3][3] = par->c0_tgl * par->c0_tgl;
  k->C[4][4] = par->c0_qpt * par->c0_qpt;
}

/* ============================================================ following */
typedef struct {
  const oparams* par;
  int32_t n_units;
  const int32_t *y, *z;
  const uint16_t* ptime;
  const uint32_t* crow_start;
  const uint32_t* tl_start;
  const uint16_t* tl_len;
  const int32_t* upc;
  int64_t n_tracklets;
  const int64_t* unit_tl; /* [n_units+1] tracklets of each unit */
  /* following outputs */
  int32_t* hits;          /* [Nt*152] cluster per row or -1 */
  int32_t* near_tie;      /* [Nt] */
  int32_t* follow_ok;     /* [Nt] 1 if seeded and followed */
  double* pb_state;       /* [Nt*6]: pass-B state (y z snp tgl qpt) + row */
  /* resolution / refit outputs (per tracklet slot) */
  int32_t* cluster_owner; /* [Nc] tracklet owning the cluster after resolution, or -1 */
  int32_t* kept;          /* [Nt] 1 if the track survives */
  double* out_par;        /* [Nt*5] */
  double* out_cov;        /* [Nt*15] */
  double* out_chi2;       /* [Nt] */
  int32_t* out_row;       /* [Nt] innermost kept row */
  int32_t* out_nhits;     /* [Nt] */
  int32_t* out_flags;     /* [Nt] */
  double* out_par_cond;   /* [Nt*5] refit from a perturbed start, or NULL */
  int64_t* pd_fail;       /* per unit counters */
} fit_job;

static int cluster_unit_row(const fit_job* J, int64_t c, int unit) {
  /* row of cluster c inside its unit (binary search of the row table) */
  int64_t a = (int64_t)unit * NROW, b = a + NROW;
  while (b - a > 1) {
    const int64_t m = (a + b) / 2;
    if (J->crow_start[m] <= c) a = m;
    else b = m;
  }
  return (int)(a - (int64_t)unit * NROW);
}

/* Search row r of the unit for the cluster with the smallest (chi2, id) among
   those with chi2 <= chi2_max.  Returns the cluster or -1. */
static int64_t search_row(const fit_job* J, int unit, int r, const kstate* k, int64_t anchor,
                          ktrace* tr) {
  const oparams* par = J->par;
  const double vy = par->sigma_y[r] * par->sigma_y[r], vz = par->sigma_z[r] * par->sigma_z[r];
  const int64_t ur = (int64_t)unit * NROW + r;
  int64_t a = J->crow_start[ur], b = J->crow_start[ur + 1];
  if (!par->brute_force) {
    /* chi2 <= chi2_max implies |dz| <= sqrt(chi2_max * S_zz) (Cauchy-Schwarz);
       the centroid is within 2 bins of the peak time */
    const double w = sqrt(par->chi2_max * (k->C[1][1] + vz));
    const double zabs = k->p[1] + anchor / 65536.0;
    const int64_t lo = (int64_t)floor(2.0 * (zabs - w)) - 3;
    const int64_t hi = (int64_t)ceil(2.0 * (zabs + w)) + 4;
    const int64_t a0 = lower_time(J->ptime, a, b, lo);
    b = lower_time(J->ptime, a0, b, hi);
    a = a0;
  }
  int64_t best = -1;
  double best_chi2 = 0, second = INFINITY;
  for (int64_t c = a; c < b; ++c) {
    const double my = J->y[c] / 65536.0, mz = (J->z[c] - anchor) / 65536.0;
    const double chi2 = kstate_chi2(k, my, mz, vy, vz);
    if (tr && fabs(chi2 - par->chi2_max) <= 1e-3 * par->chi2_max) tr->near_tie++;
    if (!(chi2 <= par->chi2_max)) continue;
    if (best < 0 || chi2 < best_chi2) {
      second = best < 0 ? second : best_chi2;
      best = c;
      best_chi2 = chi2;
    } else if (chi2 < second) {
      second = chi2;
    }
  }
  if (tr && best >= 0 && second - best_chi2 <= 1e-3 * fmax(1.0, best_chi2)) tr->near_tie++;
  return best;
}

static int edge_stop(const fit_job* J, const kstate* k, int r, ktrace* tr) {
  const double lim = G_HW[r] + J->par->edge_margin;
  if (tr && fabs(fabs(k->p[0]) - lim) < 1e-4) tr->near_tie++;
  return fabs(k->p[0]) > lim;
}

static void meas(const fit_job* J, int64_t c, int64_t anchor, double* my, double* mz) {
  *my = J->y[c] / 65536.0;
  *mz = (J->z[c] - anchor) / 65536.0;
}

/* seed from the first, middle and last tracklet clusters */
static int seed_tracklet(const fit_job* J, const int64_t* th, int L, int r1, kstate* k) {
  const oparams* par = J->par;
  const int64_t A = th[0], M = th[(L + 1) / 2 - 1], E = th[L - 1];
  const double xA = G_X[r1], xM = G_X[r1 + (L + 1) / 2 - 1], xE = G_X[r1 + L - 1];
  const double yA = J->y[A] / 65536.0, yM = J->y[M] / 65536.0, yE = J->y[E] / 65536.0;
  const double mx = xM - xA, my = yM - yA, ex = xE - xA, ey = yE - yA;
  const double dMA = hypot(mx, my), dEA = hypot(ex, ey), dEM = hypot(xE - xM, yE - yM);
  double C = 2.0 * (mx * ey - my * ex) / (dMA * dEM * dEA);
  double qpt = -C / par->bz_b;
  if (qpt > par->qpt_clamp) qpt = par->qpt_clamp;
  if (qpt < -par->qpt_clamp) qpt = -par->qpt_clamp;
  C = -par->bz_b * qpt;
  double sarg = dEA * C / 2.0;
  if (sarg > 1.0) sarg = 1.0;
  if (sarg < -1.0) sarg = -1.0;
  const double phiA = atan2(ey, ex) - asin(sarg);
  const double h = dEA * fabs(C) / 2.0;
  const double arc = h > 0 ? dEA * asin(h > 1.0 ? 1.0 : h) / h : dEA;
  k->x = xA;
  k->p[0] = yA;
  k->p[1] = 0.0;
  k->p[2] = sin(phiA);
  k->p[3] = (double)(J->z[E] - J->z[A]) / 65536.0 / arc;
  k->p[4] = qpt;
  c0_reset(par, k, r1);
  return fabs(k->p[2]) >= par->snp_max;
}

static void follow_tracklet(fit_job* J, int unit, int64_t t) {
  const oparams* par = J->par;
  int32_t* H = J->hits + t * NROW;
  for (int r = 0; r < NROW; ++r) H[r] = -1;
  J->follow_ok[t] = 0;
  ktrace tr = {0, 0};
  const int L = J->tl_len[t];
  int64_t th[NROW];
  th[0] = J->tl_start[t];
  for (int i = 1; i < L; ++i) th[i] = J->upc[th[i - 1]];
  const int r1 = cluster_unit_row(J, th[0], unit);
  const int64_t anchor = J->z[th[0]];
  kstate k;
  if (seed_tracklet(J, th, L, r1, &k)) {
    J->near_tie[t] = tr.near_tie;
    return;
  }
  double my, mz;
  /* ---- pass A: outward */
  meas(J, th[0], anchor, &my, &mz);
  if (kstate_update(&k, my, mz, par->sigma_y[r1] * par->sigma_y[r1],
                    par->sigma_z[r1] * par->sigma_z[r1], NULL, &tr)) {
    J->near_tie[t] = tr.near_tie;
    return;
  }
  H[r1] = (int32_t)th[0];
  kstate last = k;
  int r_out = r1, nmiss = 0;
  for (int r = r1 + 1; r < NROW; ++r) {
    if (kstate_propagate(par, &k, G_X[r], &tr)) break;
    const double vy = par->sigma_y[r] * par->sigma_y[r], vz = par->sigma_z[r] * par->sigma_z[r];
    int64_t c;
    if (r < r1 + L) {
      c = th[r - r1];
    } else {
      if (edge_stop(J, &k, r, &tr)) break;
      c = search_row(J, unit, r, &k, anchor, &tr);
      if (c < 0) {
        if (++nmiss >= par->max_miss) break;
        continue;
      }
    }
    meas(J, c, anchor, &my, &mz);
    if (kstate_update(&k, my, mz, vy, vz, NULL, &tr)) break;
    H[r] = (int32_t)c;
    last = k;
    r_out = r;
    nmiss = 0;
  }
  /* ---- pass B: inward from the outermost pass-A hit, covariance reset */
  k = last;
  c0_reset(par, &k, r_out);
  meas(J, H[r_out], anchor, &my, &mz);
  kstate innermost;
  int r_in = r_out;
  if (kstate_update(&k, my, mz, par->sigma_y[r_out] * par->sigma_y[r_out],
                    par->sigma_z[r_out] * par->sigma_z[r_out], NULL, &tr) == 0) {
    innermost = k;
    nmiss = 0;
    for (int r = r_out - 1; r >= 0; --r) {
      if (kstate_propagate(par, &k, G_X[r], &tr)) break;
      const double vy = par->sigma_y[r] * par->sigma_y[r], vz = par->sigma_z[r] * par->sigma_z[r];
      int64_t c;
      int fresh = 0;
      if (H[r] >= 0) {
        c = H[r];
      } else {
        if (edge_stop(J, &k, r, &tr)) break;
        c = search_row(J, unit, r, &k, anchor, &tr);
        if (c < 0) {
          if (r < r1 && ++nmiss >= par->max_miss) break;
          continue;
        }
        fresh = 1;
      }
      meas(J, c, anchor, &my, &mz);
      if (kstate_update(&k, my, mz, vy, vz, NULL, &tr)) break;
      if (fresh) H[r] = (int32_t)c;
      innermost = k;
      r_in = r;
      nmiss = 0;
    }
  } else {
    innermost = last;
  }
  double* pb = J->pb_state + t * 6;
  for (int i = 0; i < 5; ++i) pb[i] = innermost.p[i];
  pb[5] = r_in;
  J->follow_ok[t] = 1;
  J->near_tie[t] = tr.near_tie;
}

static void follow_unit(void* ctx, int unit) {
  fit_job* J = (fit_job*)ctx;
  for (int64_t t = J->unit_tl[unit]; t < J->unit_tl[unit + 1]; ++t) follow_tracklet(J, unit, t);
}

/* ------------------------------------------------------------ resolution */
static void resolve_unit(void* ctx, int unit) {
  fit_job* J = (fit_job*)ctx;
  const oparams* par = J->par;
  const int64_t c0 = J->crow_start[(int64_t)unit * NROW];
  const int64_t c1 = J->crow_start[(int64_t)(unit + 1) * NROW];
  const int64_t t0 = J->unit_tl[unit], t1 = J->unit_tl[unit + 1];
  /* owner key: (hits << 32) | (0xFFFFFFFF - tracklet id); larger wins */
  uint64_t* best = (uint64_t*)calloc(c1 - c0 > 0 ? c1 - c0 : 1, sizeof(uint64_t));
  for (int64_t t = t0; t < t1; ++t) {
    J->kept[t] = 0;
    if (!J->follow_ok[t]) continue;
    const int32_t* H = J->hits + t * NROW;
    int n = 0;
    for (int r = 0; r < NROW; ++r) n += H[r] >= 0;
    if (n < par->min_track_hits) continue;
    J->kept[t] = 1;
    const uint64_t key = ((uint64_t)n << 32) | (0xFFFFFFFFull - (uint64_t)t);
    for (int r = 0; r < NROW; ++r)
      if (H[r] >= 0 && key > best[H[r] - c0]) best[H[r] - c0] = key;
  }
  for (int64_t c = c0; c < c1; ++c) J->cluster_owner[c] = -1;
  for (int64_t c = c0; c < c1; ++c)
    if (best[c - c0]) J->cluster_owner[c] = (int32_t)(0xFFFFFFFFull - (best[c - c0] & 0xFFFFFFFFull));
  for (int64_t t = t0; t < t1; ++t) {
    if (!J->kept[t]) continue;
    const int32_t* H = J->hits + t * NROW;
    int n = 0;
    for (int r = 0; r < NROW; ++r) n += H[r] >= 0 && J->cluster_owner[H[r]] == t;
    if (n < par->min_track_hits) J->kept[t] = 0;
  }
  /* clusters of dropped tracks are not handed to anyone else */
  for (int64_t c = c0; c < c1; ++c)
    if (J->cluster_owner[c] >= 0 && !J->kept[J->cluster_owner[c]]) J->cluster_owner[c] = -1;
  free(best);
}

/* ------------------------------------------------------------ refit */
enum { TFLAG_NOT_PD = 1, TFLAG_REFIT_FAIL = 2 };

/* Refit of a track over its kept hits.  The start is the circle through the
   innermost, middle and outermost kept clusters, evaluated at the outermost
   one, with a broad covariance, so that the result depends on the kept hits
   alone; the Kalman filter then runs inward through every kept hit.  A step
   fails only if the helix cannot reach the next hit's row.  rows[0..n) are
   the kept rows, outermost first.  seed_scale multiplies every start
   parameter (1 for the result itself).  Returns 1 if a step fails. */
static int refit_from_seed(const fit_job* J, int64_t t, const int* rows, int n, double seed_scale,
                           kstate* k, double* chi2_out, int* pd_ok, ktrace* tr) {
  const oparams* par = J->par;
  const int32_t* H = J->hits + t * NROW;
  const int64_t anchor = J->z[J->tl_start[t]];
  /* circle through A (innermost), M (middle), E (outermost) kept clusters */
  const int rA = rows[n - 1], rM = rows[n - 1 - ((n + 1) / 2 - 1)], rE = rows[0];
  const int64_t cA = H[rA], cM = H[rM], cE = H[rE];
  const double mx = G_X[rM] - G_X[rA], my = (J->y[cM] - J->y[cA]) / 65536.0;
  const double ex = G_X[rE] - G_X[rA], ey = (J->y[cE] - J->y[cA]) / 65536.0;
  const double dMA = hypot(mx, my), dEA = hypot(ex, ey), dEM = hypot(G_X[rE] - G_X[rM], ey - my);
  double C = 2.0 * (mx * ey - my * ex) / (dMA * dEM * dEA);
  double qpt = -C / par->bz_b;
  if (qpt > par->qpt_clamp) qpt = par->qpt_clamp;
  if (qpt < -par->qpt_clamp) qpt = -par->qpt_clamp;
  C = -par->bz_b * qpt;
  double sarg = dEA * C / 2.0;
  if (sarg > 1.0) sarg = 1.0;
  if (sarg < -1.0) sarg = -1.0;
  const double h = dEA * fabs(C) / 2.0;
  const double arc = h > 0 ? dEA * asin(h > 1.0 ? 1.0 : h) / h : dEA;
  k->x = G_X[rE];
  k->p[0] = J->y[cE] / 65536.0;
  k->p[1] = (J->z[cE] - anchor) / 65536.0;
  k->p[2] = sin(atan2(ey, ex) + asin(sarg)); /* tangent at the far end of the chord */
  k->p[3] = (double)(J->z[cE] - J->z[cA]) / 65536.0 / arc;
  k->p[4] = qpt;
  if (seed_scale != 1.0)
    for (int i = 0; i < 5; ++i) k->p[i] *= seed_scale;
  memset(k->C, 0, sizeof k->C);
  k->C[0][0] = par->c0r_y * par->c0r_y;
  k->C[1][1] = par->c0r_z * par->c0r_z;
  k->C[2][2] = par->c0r_snp * par->c0r_snp;
  k->C[3][3] = par->c0r_tgl * par->c0r_tgl;
  k->C[4][4] = par->c0r_qpt * par->c0r_qpt;
  oparams rp = *par;
  rp.snp_max = par->refit_snp_max;
  double chi2sum = 0;
  *pd_ok = 1;
  for (int i = 0; i < n; ++i) {
    const int r = rows[i];
    if (i > 0 && kstate_propagate(&rp, k, G_X[r], tr)) return 1;
    double mmy, mmz, chi2;
    meas(J, H[r], anchor, &mmy, &mmz);
    if (kstate_update(k, mmy, mmz, par->sigma_y[r] * par->sigma_y[r],
                      par->sigma_z[r] * par->sigma_z[r], &chi2, tr))
      return 1;
    chi2sum += chi2;
    if (!is_pd(k->C)) *pd_ok = 0;
  }
  *chi2_out = chi2sum;
  return 0;
}

static void refit_track(fit_job* J, int64_t t) {
  const int32_t* H = J->hits + t * NROW;
  int rows[NROW], n = 0;
  for (int r = NROW - 1; r >= 0; --r)
    if (H[r] >= 0 && J->cluster_owner[H[r]] == t) rows[n++] = r;
  J->out_flags[t] = 0;
  ktrace tr = {0, 0};
  kstate k;
  double chi2sum;
  int pd_ok;
  if (refit_from_seed(J, t, rows, n, 1.0, &k, &chi2sum, &pd_ok, &tr)) {
    J->out_flags[t] |= TFLAG_REFIT_FAIL;
    J->kept[t] = 0;
    return;
  }
  if (!pd_ok) J->out_flags[t] |= TFLAG_NOT_PD;
  for (int i = 0; i < 5; ++i) J->out_par[t * 5 + i] = k.p[i];
  int m = 0;
  for (int i = 0; i < 5; ++i)
    for (int j = i; j < 5; ++j) J->out_cov[t * 15 + m++] = k.C[i][j];
  J->out_chi2[t] = chi2sum;
  J->out_row[t] = rows[n - 1];
  J->out_nhits[t] = n;
  J->near_tie[t] += tr.near_tie;
  /* conditioning of the result: the same refit from a start perturbed by one
     rounding unit of binary32 (2^-24), for comparisons made in that precision;
     NaN if that refit fails */
  if (J->out_par_cond) {
    kstate kc;
    double c2;
    int pdc;
    const int f = refit_from_seed(J, t, rows, n, 1.0 + 0x1p-24, &kc, &c2, &pdc, NULL);
    for (int i = 0; i < 5; ++i) J->out_par_cond[t * 5 + i] = f ? NAN : kc.p[i];
  }
}

static void refit_unit(void* ctx, int unit) {
  fit_job* J = (fit_job*)ctx;
  for (int64_t t = J->unit_tl[unit]; t < J->unit_tl[unit + 1]; ++t)
    if (J->kept[t]) refit_track(J, t);
}

/* Following, resolution and refit of all tracklets.
   Per-tracklet outputs are indexed by tracklet id; emitted tracks are the
   tracklets with kept[t] = 1, in ascending tracklet order.  cluster_owner[c]
   is the tracklet that keeps cluster c after resolution (or -1). */
typedef struct {
  int32_t* hits;        /* [Nt*152] following result (pass A + pass B) */
  int32_t* near_tie;    /* [Nt] */
  int32_t* follow_ok;   /* [Nt] */
  double* pb_state;     /* [Nt*6] */
  int32_t* cluster_owner; /* [Nc] */
  int32_t* kept;        /* [Nt] */
  double* par;          /* [Nt*5] */
  double* cov;          /* [Nt*15] packed upper triangle, row-major */
  double* chi2;         /* [Nt] */
  int32_t* row;         /* [Nt] innermost kept row */
  int32_t* nhits;       /* [Nt] */
  int32_t* flags;       /* [Nt] */
  double* par_cond;     /* [Nt*5] refit from the start scaled by 1 + 2^-24 (NULL: skipped) */
} ofit;

void oracle_fit_tracks(const oparams* par, int32_t n_units, const int32_t* y_fx,
                       const int32_t* z_fx, const uint16_t* ptime, const uint32_t* crow_start,
                       const int32_t* upc, int64_t n_tracklets, const uint32_t* tl_start,
                       const uint16_t* tl_len, ofit* out) {
  geometry_init();
  int64_t* unit_tl = (int64_t*)calloc(n_units + 1, sizeof(int64_t));
  /* tracklets ascend by start cluster, so units are contiguous */
  int64_t t = 0;
  for (int u = 0; u < n_units; ++u) {
    unit_tl[u] = t;
    const uint32_t cend = crow_start[(int64_t)(u + 1) * NROW];
    while (t < n_tracklets && tl_start[t] < cend) ++t;
  }
  unit_tl[n_units] = t;
  fit_job J;
  memset(&J, 0, sizeof J);
  J.par = par;
  J.n_units = n_units;
  J.y = y_fx;
  J.z = z_fx;
  J.ptime = ptime;
  J.crow_start = crow_start;
  J.tl_start = tl_start;
  J.tl_len = tl_len;
  J.upc = upc;
  J.n_tracklets = n_tracklets;
  J.unit_tl = unit_tl;
  J.hits = out->hits;
  J.near_tie = out->near_tie;
  J.follow_ok = out->follow_ok;
  J.pb_state = out->pb_state;
  J.cluster_owner = out->cluster_owner;
  J.kept = out->kept;
  J.out_par = out->par;
  J.out_cov = out->cov;
  J.out_chi2 = out->chi2;
  J.out_row = out->row;
  J.out_nhits = out->nhits;
  J.out_flags = out->flags;
  J.out_par_cond = out->par_cond;
  for (int64_t i = 0; i < n_tracklets; ++i) {
    out->nhits[i] = 0;
    out->flags[i] = 0;
    out->row[i] = -1;
    out->chi2[i] = 0;
  }
  for_units(n_units, par->n_threads, &J, follow_unit);
  for_units(n_units, par->n_threads, &J, resolve_unit);
  for_units(n_units, par->n_threads, &J, refit_unit);
  /* a track that fails the refit releases its clusters */
  const int64_t nc = crow_start[(int64_t)n_units * NROW];
  for (int64_t c = 0; c < nc; ++c)
    if (out->cluster_owner[c] >= 0 && !out->kept[out->cluster_owner[c]]) out->cluster_owner[c] = -1;
  free(unit_tl);
}

/* ------------------------------------------------------- Kalman test hooks */
/* Exposed for the tests that pin the primitives to closed forms. */
int oracle_helix_propagate(const oparams* par, double* p, double x1, double x2, double* J) {
  double JJ[5][5];
  const int rc = helix_propagate(par, p, x1, x2, J ? JJ : NULL, NULL);
  if (J && rc == 0)
    for (int i = 0; i < 5; ++i)
      for (int j = 0; j < 5; ++j) J[i * 5 + j] = JJ[i][j];
  return rc;
}

/* Kalman fit of a sequence of measurements (rows given outermost first) from
   a given start state and covariance at rows[0]; returns the state and
   covariance at the last row. */
int oracle_kalman_fit(const oparams* par, int n, const int32_t* rows, const double* my,
                      const double* mz, const double* vy, const double* vz, double* p,
                      double* C, double* chi2_out) {
  geometry_init();
  kstate k;
  for (int i = 0; i < 5; ++i) k.p[i] = p[i];
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) k.C[i][j] = C[i * 5 + j];
  k.x = G_X[rows[0]];
  double chi2sum = 0;
  for (int i = 0; i < n; ++i) {
    if (i > 0 && kstate_propagate(par, &k, G_X[rows[i]], NULL)) return 1;
    double c2;
    if (kstate_update(&k, my[i], mz[i], vy[i], vz[i], &c2, NULL)) return 2;
    chi2sum += c2;
  }
  for (int i = 0; i < 5; ++i) p[i] = k.p[i];
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) C[i * 5 + j] = k.C[i][j];
  if (chi2_out) *chi2_out = chi2sum;
  return is_pd(k.C) ? 0 : 3;
}

int oracle_seed(const oparams* par, const int32_t* y_fx, const int32_t* z_fx, int r1, int L,
                double* p_out) {
  geometry_init();
  fit_job J;
  memset(&J, 0, sizeof J);
  J.par = par;
  J.y = y_fx;
  J.z = z_fx;
  int64_t th[NROW];
  for (int i = 0; i < L; ++i) th[i] = i;
  kstate k;
  const int rc = seed_tracklet(&J, th, L, r1, &k);
  for (int i = 0; i < 5; ++i) p_out[i] = k.p[i];
  return rc;
}

int oracle_is_pd(const double* C) {
  double M[5][5];
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) M[i][j] = C[i * 5 + j];
  return is_pd(M);
}

/* ------------------------------------------------------- raw ZS pages */
/* Decoder of the library's raw zero-suppressed page format (the paper,
 * section "Hardware and data flow": zero suppression runs on the readout
 * FPGA; the format itself is this project's): each 2048-word page holds a
 * header (magic 0x5A53 | version 1 << 16; unit | row << 16; n_runs | n_samples
 * << 16; 0), n_runs run words (time | first pad << 16 | (length - 1) << 24)
 * and a stream of 10-bit ADC fields, sample k at bits [10k, 10k + 10).
 * Samples are appended page by page, run by run, pad by pad.  Returns 0, -3
 * for malformed input (header, pads beyond the row, time beyond the frame,
 * run lengths not adding up, pages out of (unit,row) order; with validate
 * also runs out of (time, pad) order and zero ADC values) or -2 when more
 * than `capacity` samples result; *n_out is the sample count. */
int oracle_decode_zs_pages(const uint32_t* pages, int64_t n_pages, int32_t n_units,
                           int32_t n_time_bins, int32_t validate, uint16_t* pad, uint16_t* time,
                           uint16_t* adc, uint32_t* row_start, int64_t capacity, int64_t* n_out) {
  geometry_init();
  int64_t n = 0, prev_ur = -1;
  int64_t last_t = -1, last_end = 0; /* end pad (exclusive) of the last run of prev_ur */
  int status = 0;
  for (int64_t u = 0; u <= (int64_t)n_units * NROW; ++u) row_start[u] = 0;
  for (int64_t p = 0; p < n_pages; ++p) {
    const uint32_t* pg = pages + p * 2048;
    const int64_t unit = pg[1] & 0xFFFF, row = (pg[1] >> 16) & 0xFF;
    const int64_t nr = pg[2] & 0xFFFF, ns = pg[2] >> 16;
    if (pg[0] != (0x5A53u | (1u << 16)) || (pg[1] >> 24) != 0 || pg[3] != 0 ||
        unit >= n_units || row >= NROW || 4 + nr + (ns * 10 + 31) / 32 > 2048 ||
        (nr > 0) != (ns > 0))
      return -3;
    const int64_t ur = unit * NROW + row;
    if (ur < prev_ur) return -3;
    if (ur != prev_ur) { /* rows between the previous page's and this one start here */
      for (int64_t u = prev_ur + 1; u <= ur; ++u) row_start[u] = (uint32_t)n;
      prev_ur = ur;
      last_t = -1;
      last_end = 0;
    }
    int64_t total = 0;
    for (int64_t i = 0; i < nr; ++i) total += (pg[4 + i] >> 24) + 1;
    if (total != ns) return -3;
    const uint32_t* stream = pg + 4 + nr;
    int64_t k = 0;
    for (int64_t i = 0; i < nr; ++i) {
      const uint32_t w = pg[4 + i];
      const int64_t t = w & 0xFFFF, p0 = (w >> 16) & 0xFF, len = (w >> 24) + 1;
      if (t >= n_time_bins || p0 + len > G_NP[row]) return -3;
      if (validate && (t < last_t || (t == last_t && p0 < last_end))) return -3;
      last_t = t;
      last_end = p0 + len;
      for (int64_t j = 0; j < len; ++j, ++k) {
        /* bits [10k, 10k + 10) of the stream, least significant first */
        uint32_t a = 0;
        for (int b = 0; b < 10; ++b) {
          const int64_t bit = 10 * k + b;
          a |= ((stream[bit / 32] >> (bit % 32)) & 1u) << b;
        }
        if (validate && a == 0) return -3;
        if (n < capacity) {
          pad[n] = (uint16_t)(p0 + j);
          time[n] = (uint16_t)t;
          adc[n] = (uint16_t)a;
        }
        ++n;
      }
    }
  }
  for (int64_t u = prev_ur + 1; u <= (int64_t)n_units * NROW; ++u) row_start[u] = (uint32_t)n;
  *n_out = n;
  if (n > capacity) status = -2;
  return status;
}

/* ------------------------------------------- track-model cluster compression */
/* The paper (section "Hardware and data flow") says data compression relies on
 * the TPC tracking; it gives no codec.  Reading (the library's own format,
 * stated with tpc_compress): cluster positions are quantised to 2^-7 cm; a
 * cluster on a track is stored as its residual to the track model, an integer
 * helix evaluated row by row from the fitted parameters; clusters on no track
 * are stored per (unit,row) with the drift position relative to the previous
 * one.  Every value is an Exp-Golomb code in an LSB-first bit stream, so the
 * whole stream is integer arithmetic and decodes to the quantised clusters
 * whatever the model predicts.  Returns -3 for input the format cannot hold
 * (a track hit below the row of its parameters). */
#define CM_MAGIC 0x54434D31u
#define CM_VERSION 2u
#define CM_CHUNK 64 /* clusters on no track per independently decodable chunk of a row */
#define CM_HDR 8

static int64_t cm_q(int64_t v) { return floor_div(v + 256, 512); } /* 2^-7 cm steps */

static int64_t cm_isqrt(int64_t n) { /* floor(sqrt(n)), n >= 0 */
  int64_t r = (int64_t)sqrt((double)n);
  while (r > 0 && r * r > n) --r;
  while ((r + 1) * (r + 1) <= n) ++r;
  return r;
}

static uint64_t cm_zig(int64_t v) { return v >= 0 ? (uint64_t)v * 2 : (uint64_t)(-v) * 2 - 1; }
static int64_t cm_unzig(uint64_t u) { return (u & 1) ? -(int64_t)((u + 1) / 2) : (int64_t)(u / 2); }

/* Integer helix of one track: fixed-point state at the current row. */
typedef struct {
  int64_t Y, Z, S, T, C; /* y, z in 2^-16 cm; sin phi, tan lambda in 2^-30; C in 2^-46 / cm */
  int row, frozen;
} cm_model;

/* The model's integers from the fitted float32 parameters: each value scaled
 * by a power of two (exact) and rounded to the nearest integer, ties to even. */
static void cm_model_init(cm_model* m, const oparams* par, const float p[5], int32_t z_anchor,
                          int row, int64_t* Yo, int64_t* Zo, int64_t* So, int64_t* To,
                          int64_t* Ko) {
  int64_t S = (int64_t)rint((double)p[2] * 1073741824.0);
  int64_t T = (int64_t)rint((double)p[3] * 1073741824.0);
  int64_t K = (int64_t)rint((double)p[4] * 65536.0);
  const int64_t lim = ((int64_t)1 << 30) - 1;
  if (S > lim) S = lim;
  if (S < -lim) S = -lim;
  if (T > 4 * lim) T = 4 * lim;
  if (T < -4 * lim) T = -4 * lim;
  if (K > 20 * 65536) K = 20 * 65536;
  if (K < -20 * 65536) K = -20 * 65536;
  *Yo = (int64_t)rint((double)p[0] * 65536.0);
  *Zo = (int64_t)rint((double)p[1] * 65536.0) + z_anchor;
  *So = S;
  *To = T;
  *Ko = K;
  m->Y = *Yo;
  m->Z = *Zo;
  m->S = S;
  m->T = T;
  m->C = -(int64_t)llrint(par->bz_b * 1073741824.0) * K;
  m->row = row;
  m->frozen = 0;
}

static void cm_model_from_ints(cm_model* m, const oparams* par, int64_t Y, int64_t Z, int64_t S,
                               int64_t T, int64_t K, int row) {
  m->Y = Y;
  m->Z = Z;
  m->S = S;
  m->T = T;
  m->C = -(int64_t)llrint(par->bz_b * 1073741824.0) * K;
  m->row = row;
  m->frozen = 0;
}

/* a / d rounded to the nearest integer, halves up (d > 0) */
static int64_t cm_rdiv(int64_t a, int64_t d) { return floor_div(2 * a + d, 2 * d); }

/* One row outward: exact helix step in fixed point (chord for the drift
 * length), every quotient rounded to the nearest unit.  The model stops
 * changing once |sin phi| would reach 1 - 2^-10. */
static void cm_model_step(cm_model* m) {
  const int a = m->row;
  m->row = a + 1;
  if (m->frozen || a + 1 >= NROW) return;
  const int64_t D = G_XFX[a + 1] - G_XFX[a];
  const int64_t S1 = m->S + cm_rdiv(m->C * D, (int64_t)1 << 32);
  const int64_t smax = ((int64_t)1 << 30) - ((int64_t)1 << 20);
  if (S1 >= smax || S1 <= -smax) {
    m->frozen = 1;
    return;
  }
  const int64_t one = (int64_t)1 << 60;
  const int64_t c0 = cm_isqrt(one - m->S * m->S), c1 = cm_isqrt(one - S1 * S1);
  const int64_t F = cm_rdiv((m->S + S1) * ((int64_t)1 << 24), c0 + c1);
  m->Y += cm_rdiv(D * F, (int64_t)1 << 24);
  const int64_t L = cm_rdiv(D * cm_isqrt(((int64_t)1 << 48) + F * F), (int64_t)1 << 24);
  m->Z += cm_rdiv(m->T * L, (int64_t)1 << 30);
  m->S = S1;
}

/* LSB-first bit stream: bit b is bit b % 32 of word b / 32. */
typedef struct {
  uint32_t* w;
  int64_t cap_bits, pos;
  int over;
} cm_writer;

static void cm_put(cm_writer* b, uint64_t v, int n) {
  for (int i = 0; i < n; ++i, ++b->pos) {
    if (b->pos >= b->cap_bits) {
      b->over = 1;
      continue;
    }
    if ((v >> i) & 1) b->w[b->pos / 32] |= 1u << (b->pos % 32);
  }
}

/* Exp-Golomb code of order k: with q = (v >> k) + 1 and n = floor(log2 q),
 * n zero bits, a one bit, the n low bits of q, then the k low bits of v. */
static void cm_eg(cm_writer* b, uint64_t v, int k) {
  const uint64_t q = (v >> k) + 1;
  int n = 0;
  while ((q >> (n + 1)) != 0) ++n;
  cm_put(b, 0, n);
  cm_put(b, 1, 1);
  cm_put(b, q, n);
  cm_put(b, v, k);
}

typedef struct {
  const uint32_t* w;
  int64_t n_bits, pos;
  int bad;
} cm_reader;

static uint64_t cm_get(cm_reader* r, int n) {
  uint64_t v = 0;
  for (int i = 0; i < n; ++i, ++r->pos) {
    if (r->pos >= r->n_bits) {
      r->bad = 1;
      continue;
    }
    v |= (uint64_t)((r->w[r->pos / 32] >> (r->pos % 32)) & 1u) << i;
  }
  return v;
}

static uint64_t cm_geteg(cm_reader* r, int k) {
  int n = 0;
  while (!r->bad && cm_get(r, 1) == 0) {
    if (++n > 31) { /* no code of the format has a prefix of 32 zeros or more */
      r->bad = 1;
      return 0;
    }
  }
  const uint64_t q = ((uint64_t)1 << n) | cm_get(r, n);
  return ((q - 1) << k) | cm_get(r, k);
}

static void cm_cluster_fields(cm_writer* b, uint16_t qtot, uint16_t qmax, uint8_t flags) {
  cm_eg(b, qtot, 6);
  cm_eg(b, qmax, 5);
  cm_put(b, flags & 3, 2);
}

/* Writes the stream into out (zeroed here, out_cap words) and, when hist is
 * given, the residual histograms (bins [0,128) y, [128,256) z; residual d in
 * 2^-7 cm at bin clamp(d, -64, 63) + 64).  Returns 0, or -2 when the stream
 * needs more than out_cap words; *n_words is the size it needs. */
int oracle_compress(const oparams* par, int32_t n_units, const uint32_t* crow_start,
                    const int32_t* y_fx, const int32_t* z_fx, const uint16_t* qtot,
                    const uint16_t* qmax, const uint8_t* flags, int64_t n_tracks,
                    const float* tpar, const int32_t* z_anchor, const uint8_t* trow,
                    const uint32_t* hit_start, const uint32_t* hits, const int32_t* cluster_track,
                    uint32_t* out, int64_t out_cap, int64_t* n_words, int64_t* hist) {
  geometry_init();
  const int64_t n_ur = (int64_t)n_units * NROW;
  const int64_t nc = crow_start[n_ur];
  const int64_t dir = CM_HDR + (n_tracks + 1) + (n_ur + 1);
  if (hist)
    for (int i = 0; i < 256; ++i) hist[i] = 0;
  /* pass 1 counts the bits, pass 2 writes them */
  int64_t total_bits = 0;
  for (int pass = 0; pass < 2; ++pass) {
    int64_t need = dir + (total_bits + 31) / 32;
    if (pass == 1) {
      *n_words = need;
      if (need > out_cap) return -2;
      for (int64_t i = 0; i < need; ++i) out[i] = 0;
      out[0] = CM_MAGIC;
      out[1] = CM_VERSION;
      out[2] = (uint32_t)n_units;
      out[3] = (uint32_t)n_tracks;
      out[4] = (uint32_t)nc;
      out[5] = n_tracks ? hit_start[n_tracks] : 0;
      out[6] = (uint32_t)total_bits;
      out[7] = 0;
    }
    uint32_t scratch = 0;
    cm_writer b = {pass ? out + dir : &scratch, pass ? (need - dir) * 32 : 0, 0, 0};
    for (int64_t j = 0; j < n_tracks; ++j) {
      if (pass) out[CM_HDR + j] = (uint32_t)b.pos;
      const uint32_t h0 = hit_start[j], h1 = hit_start[j + 1];
      int64_t u = 0;
      if (h1 > h0) { /* the unit of the first hit's (unit,row) */
        int64_t lo = 0, hi = n_ur; /* crow_start[lo] <= c < crow_start[hi] */
        const int64_t c = hits[h0];
        while (hi - lo > 1) {
          const int64_t mid = (lo + hi) / 2;
          if ((int64_t)crow_start[mid] <= c) lo = mid;
          else hi = mid;
        }
        u = lo / NROW;
      }
      cm_model m;
      int64_t Y, Z, S, T, K;
      cm_model_init(&m, par, tpar + 5 * j, z_anchor[j], trow[j], &Y, &Z, &S, &T, &K);
      cm_put(&b, h1 - h0, 8);
      cm_put(&b, (uint64_t)u, 16);
      cm_put(&b, trow[j], 8);
      cm_put(&b, (uint64_t)(uint32_t)(int32_t)Y, 32);
      cm_put(&b, (uint64_t)(uint32_t)(int32_t)Z, 32);
      cm_put(&b, (uint64_t)(uint32_t)(int32_t)S, 32);
      cm_put(&b, (uint64_t)(uint32_t)(int32_t)T, 32);
      cm_put(&b, (uint64_t)(uint32_t)(int32_t)K, 32);
      int prev = trow[j];
      for (uint32_t h = h0; h < h1; ++h) {
        const int64_t c = hits[h];
        int64_t lo = 0, hi = n_ur;
        while (hi - lo > 1) {
          const int64_t mid = (lo + hi) / 2;
          if ((int64_t)crow_start[mid] <= c) lo = mid;
          else hi = mid;
        }
        const int r = (int)(lo % NROW);
        if (r - prev - (h > h0 ? 1 : 0) < 0) return -3; /* hits ascend from the model's row */
        cm_eg(&b, (uint64_t)(r - prev - (h > h0 ? 1 : 0)), 0);
        prev = r;
        while (m.row < r) cm_model_step(&m);
        const int64_t dy = cm_q(y_fx[c]) - cm_q(m.Y), dz = cm_q(z_fx[c]) - cm_q(m.Z);
        cm_eg(&b, cm_zig(dy), 2);
        cm_eg(&b, cm_zig(dz), 2);
        cm_cluster_fields(&b, qtot[c], qmax[c], flags[c]);
        if (hist && pass == 1) {
          hist[(dy < -64 ? -64 : dy > 63 ? 63 : dy) + 64]++;
          hist[128 + (dz < -64 ? -64 : dz > 63 ? 63 : dz) + 64]++;
        }
      }
    }
    if (pass) out[CM_HDR + n_tracks] = (uint32_t)b.pos;
    for (int64_t ur = 0; ur < n_ur; ++ur) {
      if (pass) out[CM_HDR + n_tracks + 1 + ur] = (uint32_t)b.pos;
      int64_t n = 0;
      for (int64_t c = crow_start[ur]; c < (int64_t)crow_start[ur + 1]; ++c) n += cluster_track[c] < 0;
      cm_eg(&b, (uint64_t)n, 0);
      /* the row's clusters in chunks of CM_CHUNK; chunks 1.. start where the
         32-bit fields after the count say (bit offsets from the end of the
         fields), each with its z coded whole */
      const int64_t n_chunks = (n + CM_CHUNK - 1) / CM_CHUNK;
      const int64_t fields = b.pos;
      for (int64_t k = 1; k < n_chunks; ++k) cm_put(&b, 0, 32);
      const int64_t chunk0 = b.pos;
      int64_t zprev = 0, i = 0;
      for (int64_t c = crow_start[ur]; c < (int64_t)crow_start[ur + 1]; ++c) {
        if (cluster_track[c] >= 0) continue;
        if (i > 0 && i % CM_CHUNK == 0 && pass) { /* this chunk's offset field */
          cm_writer f = b;
          f.pos = fields + 32 * (i / CM_CHUNK - 1);
          cm_put(&f, (uint64_t)(b.pos - chunk0), 32);
        }
        const int64_t zq = cm_q(z_fx[c]);
        cm_eg(&b, cm_zig(cm_q(y_fx[c])), 10);
        if (i % CM_CHUNK == 0) cm_eg(&b, cm_zig(zq), 12);
        else cm_eg(&b, cm_zig(zq - zprev), 6);
        zprev = zq;
        ++i;
        cm_cluster_fields(&b, qtot[c], qmax[c], flags[c]);
      }
    }
    if (pass) out[CM_HDR + n_tracks + 1 + n_ur] = (uint32_t)b.pos;
    total_bits = b.pos;
    if (total_bits > 0xFFFFFFFFll) return -2; /* offsets are 32-bit */
  }
  return 0;
}

/* Decodes a stream into clusters in stream order: the tracks' hits (track by
 * track, ascending row), then the clusters on no track per (unit,row).
 * Positions are the quantised ones (q * 512 in 2^-16 cm); track[i] is the
 * track index or -1.  Returns the number of clusters, -3 for a malformed
 * stream, -2 when more than cap clusters result. */
int64_t oracle_decompress(const oparams* par, const uint32_t* in, int64_t n_words, int64_t cap,
                          uint16_t* unit, uint8_t* row, int32_t* y_fx, int32_t* z_fx,
                          uint16_t* qtot, uint16_t* qmax, uint8_t* flags, int32_t* track) {
  geometry_init();
  if (n_words < CM_HDR || in[0] != CM_MAGIC || in[1] != CM_VERSION || in[7] != 0) return -3;
  const int64_t n_units = in[2], n_tracks = in[3], nc = in[4];
  const int64_t n_ur = n_units * NROW;
  const int64_t dir = CM_HDR + (n_tracks + 1) + (n_ur + 1);
  if (dir > n_words || (int64_t)in[6] > (n_words - dir) * 32) return -3;
  if (nc > cap) return -2;
  cm_reader r = {in + dir, in[6], 0, 0};
  int64_t k = 0;
  for (int64_t j = 0; j < n_tracks; ++j) {
    if (r.pos != in[CM_HDR + j]) return -3;
    const int64_t nh = cm_get(&r, 8);
    const int64_t u = cm_get(&r, 16);
    const int r0 = (int)cm_get(&r, 8);
    const int64_t Y = (int32_t)cm_get(&r, 32), Z = (int32_t)cm_get(&r, 32);
    const int64_t S = (int32_t)cm_get(&r, 32), T = (int32_t)cm_get(&r, 32);
    const int64_t K = (int32_t)cm_get(&r, 32);
    if (u >= n_units || r0 >= NROW) return -3;
    cm_model m;
    cm_model_from_ints(&m, par, Y, Z, S, T, K, r0);
    int prev = r0;
    for (int64_t h = 0; h < nh; ++h) {
      const int rr = prev + (int)cm_geteg(&r, 0) + (h > 0 ? 1 : 0);
      if (rr >= NROW || k >= nc) return -3;
      prev = rr;
      while (m.row < rr) cm_model_step(&m);
      const int64_t yq = cm_q(m.Y) + cm_unzig(cm_geteg(&r, 2));
      const int64_t zq = cm_q(m.Z) + cm_unzig(cm_geteg(&r, 2));
      unit[k] = (uint16_t)u;
      row[k] = (uint8_t)rr;
      y_fx[k] = (int32_t)(yq * 512);
      z_fx[k] = (int32_t)(zq * 512);
      qtot[k] = (uint16_t)cm_geteg(&r, 6);
      qmax[k] = (uint16_t)cm_geteg(&r, 5);
      flags[k] = (uint8_t)cm_get(&r, 2);
      track[k] = (int32_t)j;
      ++k;
    }
  }
  for (int64_t ur = 0; ur < n_ur; ++ur) {
    if (r.pos != in[CM_HDR + n_tracks + 1 + ur]) return -3;
    if (ur == 0 && r.pos != in[CM_HDR + n_tracks]) return -3;
    const int64_t n = cm_geteg(&r, 0);
    const int64_t n_chunks = (n + CM_CHUNK - 1) / CM_CHUNK;
    const int64_t fields = r.pos;
    r.pos += 32 * (n_chunks > 1 ? n_chunks - 1 : 0);
    const int64_t chunk0 = r.pos;
    int64_t zprev = 0;
    for (int64_t i = 0; i < n; ++i) {
      if (k >= nc) return -3;
      if (i > 0 && i % CM_CHUNK == 0) { /* a chunk starts where its field says */
        cm_reader f = r;
        f.pos = fields + 32 * (i / CM_CHUNK - 1);
        if (chunk0 + (int64_t)cm_get(&f, 32) != r.pos || f.bad) return -3;
      }
      const int64_t yq = cm_unzig(cm_geteg(&r, 10));
      const int64_t zq = i % CM_CHUNK == 0 ? cm_unzig(cm_geteg(&r, 12)) : zprev + cm_unzig(cm_geteg(&r, 6));
      zprev = zq;
      unit[k] = (uint16_t)(ur / NROW);
      row[k] = (uint8_t)(ur % NROW);
      y_fx[k] = (int32_t)(yq * 512);
      z_fx[k] = (int32_t)(zq * 512);
      qtot[k] = (uint16_t)cm_geteg(&r, 6);
      qmax[k] = (uint16_t)cm_geteg(&r, 5);
      flags[k] = (uint8_t)cm_get(&r, 2);
      track[k] = -1;
      ++k;
    }
  }
  if (r.bad || r.pos != (int64_t)in[6] || k != nc) return -3;
  return k;
}

/* The integer track model at the rows of a list (for the pins): positions in
 * 2^-16 cm after stepping from row0 to each row (rows ascending). */
void oracle_track_model(const oparams* par, const float* p, int32_t z_anchor, int row0, int n,
                        const int32_t* rows, int64_t* y, int64_t* z, int32_t* frozen) {
  geometry_init();
  cm_model m;
  int64_t Y, Z, S, T, K;
  cm_model_init(&m, par, p, z_anchor, row0, &Y, &Z, &S, &T, &K);
  for (int i = 0; i < n; ++i) {
    while (m.row < rows[i]) cm_model_step(&m);
    y[i] = m.Y;
    z[i] = m.Z;
    frozen[i] = m.frozen;
  }
}

/* ------------------------------------ segment merging and the T0 / z fit */
/* The paper (section "Hardware and data flow") asks for full online TPC track
 * reconstruction; the per-sector following leaves a particle that crosses a
 * sector boundary, or loops back inside a sector, as several segments, and
 * the drift coordinate of continuous readout is known only up to the
 * collision's start time T0.  Reading: two segments of one frame and one
 * side are joined when an end of one and an end of the other are within
 * MG_DZMAX cm in drift and MG_GAP cm in the bending plane and each is reached
 * from the other along the other segment's helix: within MG_PERP cm of its
 * circle, an arc of at most MG_GAP cm, within MG_DZ (+ MG_DZ_ARC per cm of
 * arc) cm of its dip line, with tangents that differ by |sin| <= MG_SIN
 * there; and their curvatures differ by at most MG_DC_REL of the larger plus
 * MG_DC_ABS.  A merged track is a
 * connected component of that relation, named by its smallest segment index.
 * Each merged track gets a helix fit of all its hits in global coordinates:
 * an algebraic (Kasa) circle fit about the centroid, then a straight-line fit
 * of the drift coordinate against the unwrapped azimuth about the centre.
 * For a particle from z = 0, |z| grows along the path, so the drift
 * coordinate grows towards the vertex: the helix is followed to the beam axis
 * (the azimuth of the origin about the centre) in the direction in which the
 * drift coordinate grows, to the first such azimuth beyond the hits; the
 * drift coordinate there is 250 + T0/2 (T0 in time bins). */
#define MG_GAP 30.0     /* cm: longest arc between two joined ends */
#define MG_DZMAX 35.0   /* cm: largest drift distance between two joined ends */
#define MG_PERP 0.5     /* cm off the other segment's circle */
#define MG_DZ 1.0       /* cm off the other segment's dip line, plus MG_DZ_ARC per cm of arc */
#define MG_DZ_ARC 0.02
#define MG_SIN 0.1      /* |sin| of the angle between the tangents at the joined end */
#define MG_DC_REL 0.2
#define MG_DC_ABS 1e-3  /* 1/cm */
#define MG_C_LINE 1e-4  /* 1/cm: below it a segment is followed as a straight line */
#define MG_TIE 1e-9     /* relative margin at which a cut counts as a near tie */

typedef struct {
  double X, Y, z, tx, ty; /* global position, drift z, global tangent (outward fit sense) */
} mg_end;

typedef struct {
  int64_t frame, side;
  double C, tgl; /* signed curvature and dip (drift) of the outward fit */
  mg_end e[2];   /* innermost, outermost hit */
  int ok;
} mg_seg;

static int mg_row_of(const uint32_t* crow, int64_t n_ur, int64_t c, int64_t* ur) {
  int64_t lo = 0, hi = n_ur;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) / 2;
    if ((int64_t)crow[mid] <= c) lo = mid;
    else hi = mid;
  }
  *ur = lo;
  return (int)(lo % NROW);
}

static void mg_alpha(int64_t sector, double* ca, double* sa) {
  const double a = ((double)(sector % 18) + 0.5) * 20.0 * PI_D / 180.0;
  *ca = cos(a);
  *sa = sin(a);
}

static double mg_wrap(double a) { /* into (-pi, pi] */
  while (a > PI_D) a -= 2 * PI_D;
  while (a <= -PI_D) a += 2 * PI_D;
  return a;
}

/* one cut: passes when v <= cut; a value within the margin is a near tie */
static int mg_cut(double v, double cut, int* tie) {
  if (fabs(v - cut) <= MG_TIE * cut) *tie = 1;
  return v <= cut;
}

/* End b seen from end a of segment A, following A's helix from a: the
 * distance of b from A's circle, the signed arc to b's nearest point on it,
 * the drift z that A's dip line gives there and the tangent there. */
static int mg_follows(const mg_seg* A, const mg_end* a, const mg_end* b, int* tie) {
  const double dx = b->X - a->X, dy = b->Y - a->Y;
  double perp, arc, tx, ty;
  if (fabs(A->C) >= MG_C_LINE) {
    const double r = 1.0 / A->C; /* signed: the centre lies to the left when C > 0 */
    const double cx = a->X - r * a->ty, cy = a->Y + r * a->tx;
    const double ux = a->X - cx, uy = a->Y - cy, vx = b->X - cx, vy = b->Y - cy;
    const double vr = sqrt(vx * vx + vy * vy);
    perp = fabs(vr - fabs(r));
    const double dpsi = atan2(ux * vy - uy * vx, ux * vx + uy * vy);
    arc = dpsi / A->C;
    /* the tangent where b projects onto the circle: the radius vector turned
       by a quarter turn in the sense of the motion */
    tx = A->C > 0 ? -vy / vr : vy / vr;
    ty = A->C > 0 ? vx / vr : -vx / vr;
  } else {
    perp = fabs(a->tx * dy - a->ty * dx);
    arc = a->tx * dx + a->ty * dy;
    tx = a->tx;
    ty = a->ty;
  }
  int ok = mg_cut(perp, MG_PERP, tie);
  ok &= mg_cut(fabs(arc), MG_GAP, tie);
  ok &= mg_cut(fabs(b->z - a->z - A->tgl * arc), MG_DZ + MG_DZ_ARC * fabs(arc), tie);
  ok &= mg_cut(fabs(tx * b->ty - ty * b->tx), MG_SIN, tie);
  return ok;
}

/* 1 joined, 0 not; *tie set when a cut is met within the near-tie margin */
static int mg_compatible(const mg_seg* A, const mg_seg* B, int* tie) {
  if (!A->ok || !B->ok || A->frame != B->frame || A->side != B->side) return 0;
  const double ca = fabs(A->C), cb = fabs(B->C), cm = ca > cb ? ca : cb;
  int found = 0;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      const mg_end* a = &A->e[i];
      const mg_end* b = &B->e[j];
      /* two gates first: the ends near in drift and in the bending plane;
         the other cuts (and their near ties) count only inside both.  Drift
         positions are multiples of 2^-16 cm, so their difference is exact
         and the first gate has no near tie. */
      if (!(fabs(a->z - b->z) <= MG_DZMAX)) continue;
      const double dxy = sqrt((a->X - b->X) * (a->X - b->X) + (a->Y - b->Y) * (a->Y - b->Y));
      if (!mg_cut(dxy, MG_GAP, tie)) continue;
      int ok = mg_cut(fabs(ca - cb), MG_DC_REL * cm + MG_DC_ABS, tie);
      ok &= mg_follows(A, a, b, tie);
      ok &= mg_follows(B, b, a, tie);
      if (ok) found = 1;
    }
  return found;
}

static int64_t mg_find(int64_t* p, int64_t x) {
  while (p[x] != x) x = p[x];
  return x;
}

/* Inputs as for oracle_compress (tracks with their hits in ascending row).
 * Outputs per track: label (component = smallest member), near_tie; per
 * component, at its label: fit[12] = {n_segments, n_hits, xc, yc, radius,
 * dz_d/dpsi, z_d at the axis, T0, |tan lambda|, flags, turning angle of the
 * hits, 0} with flags 1 = circle fit, 2 = T0 estimated.  With T0 the global
 * |z| of a point of drift coordinate z_d is 250 + T0/2 - z_d. */
void oracle_merge_tracks(const oparams* par, int32_t n_units, const uint32_t* crow_start,
                         const int32_t* y_fx, const int32_t* z_fx, int64_t n_tracks,
                         const float* tpar, const uint8_t* trow, const uint32_t* hit_start,
                         const uint32_t* hits, int64_t* label, int32_t* near_tie, double* fit) {
  geometry_init();
  const int64_t n_ur = (int64_t)n_units * NROW;
  mg_seg* S = (mg_seg*)calloc(n_tracks > 0 ? n_tracks : 1, sizeof(mg_seg));
  for (int64_t j = 0; j < n_tracks; ++j) {
    const uint32_t h0 = hit_start[j], h1 = hit_start[j + 1];
    mg_seg* s = &S[j];
    s->ok = h1 > h0;
    if (!s->ok) continue;
    int64_t ur0, ur1;
    const int r0 = mg_row_of(crow_start, n_ur, hits[h0], &ur0);
    const int r1 = mg_row_of(crow_start, n_ur, hits[h1 - 1], &ur1);
    const int64_t unit = ur0 / NROW, sector = unit % 36;
    s->frame = unit / 36;
    s->side = sector / 18;
    s->C = -par->bz_b * (double)tpar[5 * j + 4];
    s->tgl = (double)tpar[5 * j + 3];
    double ca, sa;
    mg_alpha(sector, &ca, &sa);
    /* sin phi at the parameters' row, then at the two end rows (exact circle) */
    const double xp = G_X[trow[j]];
    const double sp = (double)tpar[5 * j + 2];
    const int rows[2] = {r0, r1};
    const int64_t cs[2] = {hits[h0], hits[h1 - 1]};
    for (int e = 0; e < 2; ++e) {
      const double x = G_X[rows[e]], y = y_fx[cs[e]] / 65536.0;
      double snp = sp + s->C * (x - xp);
      if (snp > 0.999999) snp = 0.999999;
      if (snp < -0.999999) snp = -0.999999;
      const double cp = sqrt(1.0 - snp * snp);
      s->e[e].X = x * ca - y * sa;
      s->e[e].Y = x * sa + y * ca;
      s->e[e].z = z_fx[cs[e]] / 65536.0;
      s->e[e].tx = cp * ca - snp * sa;
      s->e[e].ty = cp * sa + snp * ca;
    }
  }
  /* components of the pair relation (all pairs: plain, obviously complete) */
  int64_t* p = (int64_t*)malloc((n_tracks > 0 ? n_tracks : 1) * sizeof(int64_t));
  for (int64_t j = 0; j < n_tracks; ++j) {
    p[j] = j;
    near_tie[j] = 0;
  }
  for (int64_t a = 0; a < n_tracks; ++a)
    for (int64_t b = a + 1; b < n_tracks; ++b) {
      if (S[a].frame != S[b].frame || S[a].side != S[b].side) continue;
      int tie = 0;
      const int ok = mg_compatible(&S[a], &S[b], &tie);
      if (tie) near_tie[a] = near_tie[b] = 1;
      if (ok) {
        const int64_t ra = mg_find(p, a), rb = mg_find(p, b);
        if (ra < rb) p[rb] = ra;
        else if (rb < ra) p[ra] = rb;
      }
    }
  for (int64_t j = 0; j < n_tracks; ++j) label[j] = mg_find(p, j);
  /* the fit of each component, members in ascending index, hits in order */
  for (int64_t j = 0; j < 12 * n_tracks; ++j) fit[j] = 0;
  for (int64_t root = 0; root < n_tracks; ++root) {
    if (label[root] != root) continue;
    double* f = fit + 12 * root;
    double sx = 0, sy = 0;
    int64_t n = 0, nseg = 0;
    for (int pass = 0; pass < 2; ++pass) {
      double mx = n ? sx / n : 0, my = n ? sy / n : 0;
      double suu = 0, svv = 0, suv = 0, suuu = 0, svvv = 0, suvv = 0, svuu = 0;
      for (int64_t j = root; j < n_tracks; ++j) {
        if (label[j] != root) continue;
        if (pass == 0) ++nseg;
        for (uint32_t h = hit_start[j]; h < hit_start[j + 1]; ++h) {
          int64_t ur;
          const int r = mg_row_of(crow_start, n_ur, hits[h], &ur);
          double ca, sa;
          mg_alpha((ur / NROW) % 36, &ca, &sa);
          const double x = G_X[r], y = y_fx[hits[h]] / 65536.0;
          const double X = x * ca - y * sa, Y = x * sa + y * ca;
          if (pass == 0) {
            sx += X;
            sy += Y;
            ++n;
          } else {
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
      }
      if (pass == 1) {
        f[0] = (double)nseg;
        f[1] = (double)n;
        const double det = suu * svv - suv * suv;
        if (n < 3 || !(fabs(det) > 0)) break;
        const double b1 = 0.5 * (suuu + suvv), b2 = 0.5 * (svvv + svuu);
        const double uc = (b1 * svv - b2 * suv) / det, vc = (suu * b2 - suv * b1) / det;
        f[2] = mx + uc;
        f[3] = my + vc;
        f[4] = sqrt(uc * uc + vc * vc + (suu + svv) / n);
        f[9] = 1;
      }
    }
    if (f[9] == 0) continue;
    /* drift coordinate against the unwrapped azimuth about the centre */
    const double xc = f[2], yc = f[3];
    double psi_prev = 0, acc = 0, spsi = 0, spsi2 = 0, sz = 0, szp = 0;
    double pmin = 0, pmax = 0;
    int64_t k = 0;
    for (int64_t j = root; j < n_tracks; ++j) {
      if (label[j] != root) continue;
      for (uint32_t h = hit_start[j]; h < hit_start[j + 1]; ++h) {
        int64_t ur;
        const int r = mg_row_of(crow_start, n_ur, hits[h], &ur);
        double ca, sa;
        mg_alpha((ur / NROW) % 36, &ca, &sa);
        const double x = G_X[r], y = y_fx[hits[h]] / 65536.0;
        const double X = x * ca - y * sa, Y = x * sa + y * ca;
        const double psi = atan2(Y - yc, X - xc);
        acc = k == 0 ? 0.0 : acc + mg_wrap(psi - psi_prev);
        psi_prev = psi;
        const double z = z_fx[hits[h]] / 65536.0;
        spsi += acc;
        spsi2 += acc * acc;
        sz += z;
        szp += z * acc;
        if (k == 0 || acc < pmin) pmin = acc;
        if (k == 0 || acc > pmax) pmax = acc;
        ++k;
      }
    }
    const double dd = k * spsi2 - spsi * spsi;
    if (!(dd > 0)) continue;
    const double slope = (k * szp - spsi * sz) / dd, icpt = (sz - slope * spsi) / k;
    f[5] = slope;
    f[8] = fabs(slope) / f[4]; /* |tan lambda| = |dz/ds| of the merged helix */
    f[10] = pmax - pmin;
    if (pmax - pmin < 2 * PI_D) {
      /* the origin's azimuth about the centre, unwrapped next to the last
         hit, then moved to the first value beyond the hits on the side where
         the drift coordinate grows */
      const double psi0 = atan2(-yc, -xc);
      double a = acc + mg_wrap(psi0 - psi_prev);
      if (slope >= 0) {
        while (a < pmax) a += 2 * PI_D;
        while (a - 2 * PI_D >= pmax) a -= 2 * PI_D;
      } else {
        while (a > pmin) a -= 2 * PI_D;
        while (a + 2 * PI_D <= pmin) a += 2 * PI_D;
      }
      const double zd0 = icpt + slope * a;
      f[6] = zd0;
      f[7] = 2.0 * (zd0 - 250.0); /* T0 in time bins */
      f[9] = 3;
    }
  }
  free(p);
  free(S);
}
