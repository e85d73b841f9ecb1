/*
 * tpc.h -- C ABI of the MI355X TPC track-reconstruction library (libtpcreco).
 *
 * The paper (section "Hardware and data flow") names full online TPC track
 * reconstruction on the EPN GPUs as the most compute-intensive part of
 * synchronous processing, fed with zero-suppressed data of complete
 * collisions.  This library implements that path on gfx950 in five calls:
 *
 *   tpc_cluster            zero-suppressed ADC samples -> clusters
 *   tpc_find_neighbours    clusters -> cellular-automaton links
 *   tpc_build_tracklets    links -> cleaned links + tracklets
 *   tpc_fit_tracks         tracklets -> followed, resolved, refitted tracks
 *   tpc_process_timeframe  all four in one launch sequence
 * and, beside them, tpc_decode_zs_pages (raw zero-suppressed pages -> the
 * samples), tpc_compress / tpc_decompress (track-model cluster compression),
 * tpc_merge_tracks (segment merging and the T0 / z fit) and
 * tpc_qc_histograms (quality-control histograms of the outputs).
 *
 * Conventions
 *   - Every array pointer inside the structs below is a DEVICE pointer,
 *     allocated and owned by the caller.  The library never frees caller
 *     memory and keeps no reference to it after tpc_sync returns.
 *   - The library owns only its context: parameters, a status word and the
 *     scratch buffers sized by tpc_create from a tpc_sizes bound.
 *   - Every call validates its host-side arguments (TPC_ERR_ARG, returned
 *     synchronously), then only enqueues kernels on the context's stream.
 *     Errors found on the device (capacity overflow, malformed input when
 *     params.validate is set, numeric failure) latch into the status word;
 *     a later stage that sees a latched error exits without writing, and
 *     tpc_sync returns the first latched error together with the counts.
 *   - No exception crosses the ABI; every function returns a tpc_status.
 *   - One context per stream; distinct contexts are independent and may be
 *     used from different threads.
 *
 * Units: lengths in cm; fixed-point positions in 2^-16 cm; local x of row r
 * is X_fx[r] * 2^-16 with X_fx[r] = round((85 + 160 r / 151) * 2^16); the
 * drift coordinate of time bin tau is z = tau / 2 cm.  A "unit" is one sector
 * of one time frame; sector geometry is identical for every unit, so many
 * frames are batched by concatenating their units.
 */
#ifndef TPC_H
#define TPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TPC_NROW 152
#define TPC_NPAD_MAX 138

typedef enum {
  TPC_OK = 0,
  TPC_ERR_ARG = -1,      /* bad host-side argument (returned synchronously) */
  TPC_ERR_CAPACITY = -2, /* an output or scratch capacity was too small */
  TPC_ERR_INPUT = -3,    /* input not sorted or out of range (validate mode) */
  TPC_ERR_HIP = -4,      /* a HIP runtime call failed */
  TPC_ERR_NUMERIC = -5,  /* a refit stayed non-positive-definite in FP64 */
  TPC_ERR_STATE = -6     /* context misuse */
} tpc_status;

/* Reconstruction constants.  The paper specifies none of them; the values
 * of tpc_params_default are the readings stated with the method. */
typedef struct {
  int32_t qmax_min;       /* peak threshold on the peak ADC (5; 10 at noise 2) */
  int32_t min_tracklet;   /* minimum tracklet length (5) */
  int32_t max_miss;       /* consecutive empty rows that stop following (6) */
  int32_t min_track_hits; /* minimum hits of a kept track (15) */
  int64_t win_y, win_z;   /* neighbour search windows, 2^-16 cm (2.5 cm) */
  int64_t s_max;          /* neighbour score cut (2^32 = 0.5 cm midpoint) */
  double chi2_max;        /* hit acceptance in following (16) */
  double snp_max;         /* |sin phi| that stops propagation (0.95) */
  double bz_b;            /* curvature per unit q/pT: 0.3e-3 * Bz[kG] */
  double c0_snp, c0_tgl, c0_qpt; /* seed covariance sigmas (0.1, 0.1, 10) */
  double qpt_clamp;       /* |q/pT| clamp of the seed (20 c/GeV) */
  double edge_margin;     /* cm beyond the pad plane that stops following */
  double lowpt_qpt;       /* |q/pT| at or above which FP64 fallback applies (5) */
  double c0r_y, c0r_z;    /* refit prior sigmas of y, z (5 cm: broad) */
  double c0r_snp, c0r_tgl, c0r_qpt; /* refit prior sigmas (0.5, 0.5, 10) */
  double refit_snp_max;   /* |sin phi| a refit step may not reach (0.999) */
  double sigma_y[TPC_NROW], sigma_z[TPC_NROW]; /* measurement errors [cm] */
  int32_t validate;       /* 1: check on the device that samples are sorted
                             and that every ADC is in 1..1023 */
  int32_t force_fallback; /* 1: redo every refit in FP64 (test hook) */
} tpc_params;

/* Upper bounds used to size the context's scratch. */
typedef struct {
  uint32_t max_units;     /* units per call (36 per time frame) */
  uint32_t max_time_bins; /* time bins per unit, at most 65000 (z_fx stays below 2^31) */
  uint32_t max_clusters;  /* clusters per call */
  uint32_t max_tracklets; /* tracklets per call, at most 2^24 */
  uint32_t max_samples;   /* zero-suppressed samples per call (24 bytes of scratch each) */
} tpc_sizes;

/* Zero-suppressed input: samples sorted by (unit, row, time, pad). */
typedef struct {
  const uint16_t* pad;        /* [n_samples] pad index, < pads of the row */
  const uint16_t* time;       /* [n_samples] time bin, < n_time_bins */
  const uint16_t* adc;        /* [n_samples] ADC value, 1..1023 (10 bit; zero is
                                 never stored).  Outside that range the result
                                 is undefined unless params.validate is set,
                                 which reports TPC_ERR_INPUT */
  const uint32_t* row_start;  /* [n_units*152 + 1] first sample of each (unit,row) */
  uint32_t n_samples;
  uint32_t n_units;
  uint32_t n_time_bins;
} tpc_zs_input;

/* Raw zero-suppressed pages (section "Hardware and data flow": zero
 * suppression runs in the user logic of the FPGA readout cards, and the EPNs
 * receive the data of complete collisions).  The paper fixes no format; this
 * one is the library's own.  A page is TPC_ZS_PAGE_WORDS little-endian 32-bit
 * words (8 KiB) holding samples of one (unit, row):
 *   word 0   0x5A53 | 1 << 16 (magic, version 1)
 *   word 1   unit (bits 0-15) | row << 16 (bits 24-31 zero)
 *   word 2   n_runs (bits 0-15) | n_samples << 16
 *   word 3   0
 *   words 4 .. 4 + n_runs - 1: runs, one word each:
 *            time bin (bits 0-15) | first pad << 16 | (length - 1) << 24;
 *            a run is `length` consecutive pads of one time bin
 *   then the ADC values of the runs' samples in run order, as one stream of
 *   10-bit fields: sample k occupies bits [10k, 10k + 10) of the stream (bit
 *   b is bit b % 32 of the stream's word b / 32); the rest of the page is
 *   padding.
 * n_samples = sum of the run lengths, n_runs = 0 exactly when n_samples = 0,
 * and 4 + n_runs + ceil(10 n_samples / 32) <= TPC_ZS_PAGE_WORDS.  Pages come
 * in (unit, row) order, a (unit, row) may continue over several consecutive
 * pages, and runs are in (time, pad) order without overlap; samples then come
 * out sorted as tpc_zs_input requires.  ADC values are 1..1023. */
#define TPC_ZS_PAGE_WORDS 2048

/* Decoded samples: the layout of tpc_zs_input, written by the library. */
typedef struct {
  uint32_t capacity;          /* samples the three arrays hold */
  uint32_t n_units;           /* units of the frame (set by the caller) */
  uint32_t n_time_bins;       /* time bins of the frame (set by the caller) */
  uint32_t* n_samples;        /* [1] device count written by the decoder */
  uint16_t *pad, *time, *adc; /* [capacity] */
  uint32_t* row_start;        /* [n_units*152 + 1] first sample of each (unit,row) */
} tpc_zs_soa;

/* Clusters in canonical order (unit, row, peak time, peak pad). */
typedef struct {
  uint32_t capacity;          /* entries available in each per-cluster array */
  uint32_t n_units;           /* set by the caller (same as the input's) */
  uint32_t n_time_bins;       /* set by the caller (same as the input's) */
  uint32_t* n_clusters;       /* [1] device count, written by tpc_cluster */
  uint32_t* crow_start;       /* [n_units*152 + 1] first cluster of each (unit,row) */
  int32_t* y_fx;              /* local y of the centroid, 2^-16 cm */
  int32_t* z_fx;              /* drift z of the centroid, 2^-16 cm */
  float *dpad, *dtime;        /* centroid minus peak, in pads / time bins */
  float *s2pad, *s2time;      /* second central moments */
  uint16_t *qtot, *qmax;      /* total and peak charge (ADC) */
  uint16_t *ppad, *ptime;     /* peak position */
  uint8_t* flags;             /* 1 = peak on an edge pad, 2 = saturated sample */
  /* optional (NULL to skip): integer moments and the sample -> cluster map */
  int32_t *sp, *st, *spp, *stt;
  uint16_t* nsamp;
  int32_t* sample_label;      /* [n_samples] cluster id or -1 */
} tpc_clusters;

/* Cellular-automaton links, one entry per cluster (-1 = none). */
typedef struct {
  uint32_t capacity;
  int32_t *down, *up;         /* raw best pair in rows r-1 / r+1 */
  int32_t *downc, *upc;       /* reciprocal (cleaned) links */
} tpc_links;

/* Tracklets: a start cluster plus its chain of cleaned up-links. */
typedef struct {
  uint32_t capacity;
  uint32_t* n_tracklets;      /* [1] device count */
  uint32_t* start;            /* start cluster, ascending */
  uint16_t* len;              /* clusters in the chain (>= min_tracklet) */
} tpc_tracklets;

/* Fitted tracks in ascending tracklet order. */
typedef struct {
  uint32_t capacity;          /* tracks */
  uint32_t hit_capacity;      /* entries of hits[] */
  uint32_t* n_tracks;         /* [1] device count */
  uint32_t* n_hits;           /* [1] device count */
  uint32_t* tracklet;         /* source tracklet id */
  float* par;                 /* [cap*5] y, z - z_anchor, sin phi, tan lambda, q/pT */
  float* cov;                 /* [cap*15] packed upper triangle, row-major */
  float* chi2;
  uint16_t* ndf;              /* 2 n_hits - 5 */
  uint8_t* row;               /* row of the parameters (innermost kept hit) */
  uint8_t* flags;             /* 1 not PD (high pT), 4 refit redone in FP64 */
  int32_t* z_anchor;          /* drift z of the tracklet start, 2^-16 cm */
  uint32_t* hit_start;        /* [cap+1] offsets into hits[] */
  uint32_t* hits;             /* cluster ids, ascending row */
  int32_t* cluster_track;     /* [clusters] track index or -1 */
  /* optional (NULL to skip): per-tracklet following result before
     resolution, cluster per row or -1 */
  int32_t* follow_hits;       /* [tracklet capacity * 152] */
} tpc_tracks;

typedef struct {
  int32_t status;             /* first latched error (tpc_status) */
  uint32_t required;          /* capacity that an overflow needed */
  uint32_t n_samples, n_clusters, n_tracklets, n_tracks, n_hits;
  uint32_t n_fallback;        /* refits redone in FP64 (low-pT tracks whose FP32
                                 pivots failed, or every track under force_fallback) */
  uint32_t n_fallback_fail;   /* FP64 refits still not PD (dropped) */
  uint32_t n_not_pd;          /* high-pT tracks flagged not PD */
  uint32_t n_refit_fail;      /* tracks dropped by a failed refit step */
  uint32_t overflow;          /* TPC_ERR_CAPACITY: bit k set when capacity k
                                 (TPC_OVF_*) was too small */
  uint32_t required_by[4];    /* the count capacity k needed (0 if it fit) */
  /* work of the last following stage (measurement): helix steps with
     covariance transport, candidate chi2 evaluations, Kalman updates; and
     the lane slots its waves held: 64 x the most steps of any lane, summed
     over the waves (follow_steps / follow_lane_slots is the share of lanes
     that did a step while their wave ran) */
  uint64_t follow_steps, follow_candidates, follow_updates, follow_lane_slots;
} tpc_counts;

/* Capacities named by tpc_counts.overflow / required_by: clusters
 * (tpc_clusters.capacity), tracklets (tpc_tracklets.capacity), tracks
 * (tpc_tracks.capacity) and track hits (tpc_tracks.hit_capacity). */
#define TPC_OVF_CLUSTERS 0
#define TPC_OVF_TRACKLETS 1
#define TPC_OVF_TRACKS 2
#define TPC_OVF_HITS 3

typedef struct tpc_ctx tpc_ctx;

/* Fill p with the default constants for a given electronic-noise sigma
 * (the peak threshold is round(5 * noise_sigma)). */
int tpc_params_default(tpc_params* p, double noise_sigma);

/* Library-side geometry: pads per row and fixed-point row radius / pitch. */
int tpc_geometry(int32_t* npads, int32_t* x_fx, int32_t* pitch_fx);

/* Bytes of device scratch a context with these bounds allocates.  Bounds
 * beyond what a context supports give TPC_ERR_ARG here and in tpc_create:
 * max_time_bins above 65000, max_tracklets above 2^24, max_clusters * 8
 * bytes or the cluster grid (max_units * 152 * (max_time_bins / 2 + 1)
 * entries of 4 bytes) at 4 GiB or more. */
int tpc_workspace_size(const tpc_sizes* max, size_t* bytes);

/* Create a context on the current device bound to hip_stream (a
 * hipStream_t; NULL = the null stream).  Allocates the scratch. */
int tpc_create(tpc_ctx** out, const tpc_params* p, const tpc_sizes* max, void* hip_stream);
int tpc_destroy(tpc_ctx* ctx);

/* Decode n_pages raw pages (DEVICE pointer, 16-byte aligned, n_pages *
 * TPC_ZS_PAGE_WORDS words, caller-owned, read only) into out's arrays, in
 * page order (section
 * "Hardware and data flow": the readout cards zero-suppress, the EPNs
 * reconstruct).  Writes *out->n_samples and row_start; the arrays then serve
 * as a tpc_zs_input with n_samples = out->capacity (the device count bounds
 * every row).  Always checked on the device (TPC_ERR_INPUT): the header of
 * every page, runs inside the row's pads and the frame's time bins, run
 * lengths adding up to the page's sample count, pages in (unit, row) order;
 * with params.validate also the (time, pad) order of runs within and across
 * pages and ADC values above zero.  A decoded count above out->capacity
 * gives TPC_ERR_CAPACITY with the count needed in tpc_counts.required, and
 * the pages that do not fit are not written.  Host errors (TPC_ERR_ARG):
 * missing pointers, a pages pointer not 16-byte aligned, n_units or
 * n_time_bins beyond the context's bounds, n_pages above max_samples / 16 +
 * 152 * max_units. */
int tpc_decode_zs_pages(tpc_ctx* ctx, const uint32_t* pages, uint32_t n_pages, tpc_zs_soa* out);

/* Clusterizer.  Paper, section "Hardware and data flow": the EPNs run full
 * online TPC track reconstruction on the data zero-suppressed in the readout
 * FPGA; its first step turns the pad/time samples into clusters (the paper
 * gives no algorithm; the rule below is the reading stated with the method).
 * Peaks are samples whose (adc, time, pad) key exceeds that of
 * every present 8-neighbour and whose ADC reaches qmax_min; each sample joins
 * the peak it reaches in at most two uphill steps.  Writes n_clusters,
 * crow_start and every non-NULL per-cluster array.  in->n_samples must not
 * exceed the context's max_samples (TPC_ERR_ARG). */
int tpc_cluster(tpc_ctx* ctx, const tpc_zs_input* in, tpc_clusters* out);

/* Cellular-automaton neighbour finding (same passage: the tracking step of
 * the full reconstruction; the paper gives no rule, this is the library's
 * reading).
 * For each cluster in rows 1..150: the pair (j in row r-1, k in row r+1)
 * inside the windows minimising (2y_i-y_j-y_k)^2 + (2z_i-z_j-z_k)^2 <= s_max,
 * ties to the smaller (j, k).  Writes down/up. */
int tpc_find_neighbours(tpc_ctx* ctx, const tpc_clusters* cl, tpc_links* links);

/* Tracklet seeding (same passage; reading as above).
 * Keeps reciprocal links (downc/upc) and emits chains of at least
 * min_tracklet clusters that start at a cluster without a cleaned down-link. */
int tpc_build_tracklets(tpc_ctx* ctx, const tpc_clusters* cl, tpc_links* links,
                        tpc_tracklets* out);

/* Track fit (same passage: the track reconstruction that TPC calibration
 * and compression rely on; the Kalman filter of a helix in a uniform field is
 * the library's reading).
 * Kalman following (outward pass A, inward pass B), conflict resolution
 * (each cluster kept by the track with the most hits, then the lower
 * tracklet id) and the inward FP32 refit with FP64 fallback for low-pT
 * tracks whose covariance loses positive definiteness. */
int tpc_fit_tracks(tpc_ctx* ctx, const tpc_clusters* cl, const tpc_links* links,
                   const tpc_tracklets* tl, tpc_tracks* out);

/* The four stages in one launch sequence on the context's stream (section
 * "Hardware and data flow": the full TPC processing of complete collisions on
 * the GPU; section "Software": intermediate results stay on the GPU, no
 * transfer between steps).  Arguments, errors and ownership as for the four
 * calls above; the input must satisfy tpc_cluster's contract and the outputs
 * the capacities of each stage (TPC_ERR_ARG otherwise). */
int tpc_process_timeframe(tpc_ctx* ctx, const tpc_zs_input* in, tpc_clusters* cl,
                          tpc_links* links, tpc_tracklets* tl, tpc_tracks* tr);

/* Quality-control histograms of a reconstruction's outputs (section
 * "Software": the synchronous processing also validates the detector data in
 * real time; the paper names no quantities, so these are chosen here).
 * hist: DEVICE array of TPC_QC_BINS uint32 counts, caller-owned, overwritten:
 *   [TPC_QC_QTOT,   +256)  clusters by total charge, bin min(qtot >> 3, 255)
 *   [TPC_QC_QMAX,   +256)  clusters by peak charge, bin min(qmax >> 2, 255)
 *   [TPC_QC_NHITS,  +153)  tracks by hit count (hit_start[j+1] - hit_start[j])
 *   [TPC_QC_ATTACH, +2)    clusters with cluster_track -1 / >= 0
 * Reads cl->qtot, cl->qmax, tr->cluster_track over *cl->n_clusters clusters
 * and tr->hit_start over *tr->n_tracks tracks (device counts, limited to the
 * capacities).  Enqueued on the context's stream behind the reconstruction;
 * after a latched error every count is 0.  TPC_ERR_ARG for a missing
 * pointer. */
#define TPC_QC_QTOT 0
#define TPC_QC_QMAX 256
#define TPC_QC_NHITS 512
#define TPC_QC_ATTACH 665
#define TPC_QC_BINS 667
int tpc_qc_histograms(tpc_ctx* ctx, const tpc_clusters* cl, const tpc_tracks* tr, uint32_t* hist);

/* The same histograms without a context and without any allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  The per-workgroup
 * partial histograms live in a fixed device array inside the library, one
 * copy per GPU, resolved on the first call on each device and held until the
 * process ends: one partial histogram per 65,536 entries of the larger of
 * cl->capacity and tr->capacity, at most 1,024 of them (2.7 MB).  A larger
 * capacity (above TPC_QC_NOALLOC_MAX) is rejected with TPC_ERR_CAPACITY and a
 * message on stderr; missing pointers give TPC_ERR_ARG.  Enqueued on
 * hip_stream (a hipStream_t; NULL = the null stream); no call here allocates
 * or frees memory.  There is no status word: the caller passes the outputs of
 * a reconstruction that completed without error.  Every call on one GPU uses
 * that GPU's one array, so calls that overlap in time on the same GPU (on
 * different streams, or from different threads) race and must be serialised
 * by the caller.  Results equal tpc_qc_histograms on the same outputs. */
#define TPC_QC_NOALLOC_MAX (1024ull * 65536ull)
int tpc_qc_histograms_noalloc(const tpc_clusters* cl, const tpc_tracks* tr, uint32_t* hist,
                              void* hip_stream);

/* Track-model cluster compression (section "Hardware and data flow": TPC
 * data compression relies on the information from the TPC tracking).  The
 * paper fixes no codec; this one is the library's own, all integer:
 *   positions  q(v) = floor((v + 256) / 512): y_fx, z_fx in steps of 2^-7 cm
 *   model      per track, from its float32 parameters p at row r0 = tr->row
 *              and its z anchor A: Y = rne(p[0] 2^16), Z = rne(p[1] 2^16) + A,
 *              S = rne(p[2] 2^30) (|S| <= 2^30 - 1), T = rne(p[3] 2^30)
 *              (|T| <= 4 (2^30 - 1)), K = rne(p[4] 2^16) (|K| <= 20 * 2^16),
 *              rne = to the nearest integer, ties to even; C = -rne(bz_b 2^30) K.
 *              A step from row a to a + 1, with D = X_fx[a+1] - X_fx[a] and
 *              [x / d] = floor((2x + d) / (2d)) (nearest, halves up):
 *                S1 = S + [C D / 2^32]; if |S1| >= 2^30 - 2^20 the model stops
 *                (no later step changes it); else c = isqrt(2^60 - S^2),
 *                c1 = isqrt(2^60 - S1^2), F = [(S + S1) 2^24 / (c + c1)],
 *                Y += [D F / 2^24], L = [D isqrt(2^48 + F^2) / 2^24],
 *                Z += [T L / 2^30], S = S1 (isqrt = floor of the root).
 *   codes      bit b of the stream is bit b % 32 of its word b / 32; an n-bit
 *              field holds its value least significant bit first; EG(k) of v:
 *              with q = (v >> k) + 1 and n = floor(log2 q): n zero bits, a one,
 *              the n low bits of q, the k low bits of v; signed values are
 *              zigzag-mapped (v >= 0: 2v, else -2v - 1).
 *   stream     words 0-7: 0x54434D31, 2 (format), n_units, n_tracks, n_clusters,
 *              hits on tracks, payload bits, 0; then n_tracks + 1 bit offsets
 *              of the track records (the last = end of the tracks, equal
 *              to the first row block's), then n_units * 152 + 1 bit offsets
 *              of the row blocks (the last = end of the payload), then the
 *              payload words.
 *   track      n_hits (8 bits), unit (16), r0 (8), Y, Z, S, T, K (32 each, two's
 *              complement); per hit in ascending row: EG(0) of the row step
 *              (r - r0 for the first hit, r - r_prev - 1 after), with the
 *              model stepped to r: EG(2) of zig(q(y) - q(Y)), EG(2) of
 *              zig(q(z) - q(Z)), then the cluster fields.
 *   row block  per (unit, row): EG(0) of the number n of clusters on no
 *              track; they form m = ceil(n / 64) chunks of 64 (the last
 *              shorter); m - 1 fields of 32 bits give the bit offsets of
 *              chunks 1..m-1 from the end of these fields (where chunk 0
 *              starts); then the clusters in canonical order: EG(10) of
 *              zig(q(y)), EG(12) of zig(q(z)) for the first of a chunk, EG(6)
 *              of zig(q(z) - q(z_prev)) after, then the cluster fields.  Each
 *              chunk decodes on its own; a row of at most 64 has no field.
 *   cluster    EG(6) of qtot, EG(5) of qmax, flags (2 bits).
 * Decoding gives every cluster's quantised position (within 2^-8 cm of the
 * original), its charges, flags and track, whatever the model predicts. */
typedef struct {
  uint32_t capacity;          /* words of stream[] */
  uint32_t* stream;           /* [capacity] output */
  uint32_t* n_words;          /* [1] device: words the stream needs (also on overflow) */
  uint32_t* res_hist;         /* optional [256]: residuals of the clusters on
                                 tracks, q(y) - q(Y) at bin clamp(d, -64, 63) + 64,
                                 q(z) - q(Z) at 128 + the same (NULL to skip) */
} tpc_compressed;

/* Encode a reconstruction's clusters and tracks (the outputs of
 * tpc_process_timeframe or equivalent; tracks in any order, each with its
 * hits in ascending row from tr->row on).  Reads cl->y_fx, z_fx, qtot, qmax,
 * flags, crow_start, n_clusters and tr->par, row, z_anchor, hit_start, hits,
 * cluster_track, n_tracks.  Errors: TPC_ERR_ARG (missing pointers, a track
 * capacity above the context's max_tracklets), TPC_ERR_CAPACITY (the stream
 * needs more than out->capacity words, or more than 2^32 - 1 payload bits;
 * *out->n_words and tpc_counts.required give the words needed),
 * TPC_ERR_INPUT (a hit below its track's row). */
int tpc_compress(tpc_ctx* ctx, const tpc_clusters* cl, const tpc_tracks* tr, tpc_compressed* out);

/* Decoded clusters, in stream order: the tracks' hits (track by track,
 * ascending row), then the clusters on no track per (unit, row). */
typedef struct {
  uint32_t capacity;
  uint32_t* n_clusters;       /* [1] device count (the header's) */
  uint16_t* unit;
  uint8_t* row;
  int32_t *y_fx, *z_fx;       /* quantised: q(v) * 512 */
  uint16_t *qtot, *qmax;
  uint8_t* flags;
  int32_t* track;             /* track record index, -1 for none */
} tpc_decoded_clusters;

/* Decode a stream of stream_words words (DEVICE pointer).  TPC_ERR_INPUT for
 * a malformed stream (header, directory, codes, a record not ending where the
 * next begins, more units than max_units or tracks than max_tracklets),
 * TPC_ERR_CAPACITY when it holds more than out->capacity clusters. */
int tpc_decompress(tpc_ctx* ctx, const uint32_t* stream, uint32_t stream_words,
                   tpc_decoded_clusters* out);

/* Merging of track segments and the continuous-readout T0 / z fit (section
 * "Hardware and data flow": full online TPC track reconstruction).  The
 * per-sector following leaves a particle that crosses sector boundaries or
 * loops back as several segments, and continuous readout measures drift
 * times only up to the collision's start time T0; the paper gives no rule,
 * the reading is this library's:
 *   joining  two segments of one frame (36 consecutive units) and one side
 *            (units 0-17 / 18-35 of the frame) are joined when an end of one
 *            (its innermost or outermost hit: global position, drift z, and
 *            the tangent of its outward fit there) and an end of the other
 *            are within 35 cm in drift and 30 cm in the bending plane, each
 *            is reached from the other along the other's helix (off its circle
 *            by at most 0.5 cm, an arc of at most 30 cm, on its dip line
 *            within 1 cm + 0.02 x the arc, tangents within |sin| 0.1; helices
 *            with |C| < 1e-4/cm are followed as lines), and their curvatures
 *            differ by at most 0.2 x the larger + 1e-3/cm (C = -bz_b q/pT);
 *   merged   a connected component of that relation, named by its smallest
 *            track index;
 *   fit      all hits of a merged track (tracks in ascending index, hits in
 *            order) in global coordinates (sector s at azimuth
 *            ((s mod 18) + 0.5) 20 deg): an algebraic circle fit about the
 *            centroid, then a least-squares line of drift z against the
 *            azimuth about the centre, unwrapped hit to hit; when the hits
 *            turn less than a full turn, the helix is followed to the
 *            azimuth of the beam axis, first reached beyond the hits in the
 *            direction in which drift z grows (|z| grows away from a vertex at
 *            z = 0); the drift z there is 250 cm + T0 / 2 (T0 in time bins),
 *            and a point of drift z_d lies at |z| = 250 + T0 / 2 - z_d.
 * Comparisons within 1e-9 (relative) of a cut are flagged as near ties. */
#define TPC_MERGE_FIT 12
typedef struct {
  uint32_t capacity;          /* entries of label / near_tie, records of fit */
  uint32_t* n_merged;         /* [1] device: number of merged tracks */
  int32_t* label;             /* [capacity] merged track of each track: its smallest member */
  uint8_t* near_tie;          /* [capacity] 1 where a joining decision was a near tie */
  double* fit;                /* [capacity * TPC_MERGE_FIT], filled at each merged
                                 track's label (zero elsewhere): n_segments, n_hits,
                                 centre x, y, radius (cm), dz_drift / d azimuth
                                 (cm/rad), drift z at the beam axis, T0 (bins),
                                 |tan lambda|, flags (1 circle fitted, 3 and T0),
                                 azimuth range of the hits (rad), 0 */
} tpc_merged;

/* Join the segments of a reconstruction and fit the merged tracks.  Reads
 * cl->crow_start, y_fx, z_fx, n_clusters and tr->par, row, hit_start, hits,
 * n_tracks (hits in ascending row).  TPC_ERR_ARG for missing pointers, a
 * track capacity above max_tracklets or out->capacity below it. */
int tpc_merge_tracks(tpc_ctx* ctx, const tpc_clusters* cl, const tpc_tracks* tr,
                     tpc_merged* out);

/* Wait for the stream, then report the first latched error and the counts.
 * Clears the status word for the next call. */
int tpc_sync(tpc_ctx* ctx, tpc_counts* counts);

/* The stream the context launches on (a hipStream_t). */
void* tpc_stream(tpc_ctx* ctx);

/* Stage timing for measurement (not part of the reconstruction).  When on,
 * every later call records a pair of HIP events on the context's stream
 * around each of the TPC_PROF_STAGES stages below; tpc_profile_read waits
 * for the stream, writes the summed milliseconds and the number of timed
 * launches per stage, and clears them.  Leave it off while a launch sequence
 * is captured into a HIP graph.  on = 1: stage timers; on = 2: work counters
 * of the following (tpc_counts.follow_*), from a slower counting variant of
 * its kernel; 3: both.  Stages: 0 sample index, 1 cluster peaks
 * (peak finding and moments, one pass over the samples), 2 cluster scan,
 * 3 cluster output, 4 cluster grid, 5 neighbours, 6 tracklets (and their
 * seed points, timed inside the fit call), 7 following (sorts and passes),
 * 8 resolution, 9 refit (FP32, FP64 redo of failing low-pT tracks), 10 count of the FP64
 * redos, 11 track output, 12 raw ZS page decoding (tpc_decode_zs_pages),
 * 13 compression (tpc_compress), 14 decompression (tpc_decompress), 15 merging
 * and the T0 fit (tpc_merge_tracks). */
#define TPC_PROF_STAGES 16
int tpc_profile_enable(tpc_ctx* ctx, int on);
int tpc_profile_read(tpc_ctx* ctx, double* ms, uint32_t* launches);
const char* tpc_profile_stage_name(int stage);

const char* tpc_status_string(int status);

/* Launch shapes (performance only: every choice gives the same results).
 * cl_window: clusterizer window in time bins, 8, 16, 20, 24 or 32 (24 or
 * 32 in cl_mode 2);
 * cl_chunk: windows walked by one workgroup, 4, 8 or 16 (8 only for windows
 * of 20 and 24 bins); follow_block: threads per workgroup
 * of the following kernel, 64, 128 or 256; follow_mode: 0 one launch per
 * pass (outward, then inward), each over the tracklets sorted by the most
 * rows the pass can take, longest first; 1 one launch that runs both passes
 * of a tracklet per lane, in tracklet order; 2 as 0, but a lane whose
 * tracklet has ended takes the next one in the sorted order (lane refill,
 * in batches of 32 free lanes per wave, on a grid of the resident waves).
 * One tracklet per lane at a time in every mode.  refit_waves: most waves of the FP32 refit resident per compute
 * unit, 0 (no limit), 4, 5, 6 or 8; the refit lasts as long as its longest
 * tracks' serial chains, which run faster with fewer waves sharing a SIMD
 * (the limit is a reservation of LDS per workgroup).  cl_mode: 0 the
 * clusterizer's peak pass per window (each window with its own halo of time
 * bins), 1 per chunk of cl_chunk windows as one stream of samples through a
 * ring of 32 time bins, handing chunks whose live peaks exceed its 31 moment
 * slots to the per-window pass; 2 per window as 0, with two waves sharing
 * each window's tile (twice the waves per compute unit for the same LDS,
 * at the cost of a workgroup barrier per phase).  tpc_set_tuning rejects
 * other values with TPC_ERR_ARG and leaves
 * the context unchanged; it takes effect at the next call (a captured graph
 * keeps the shapes it was captured with). */
typedef struct {
  int32_t cl_window;
  int32_t cl_chunk;
  int32_t follow_block;
  int32_t follow_mode;
  int32_t refit_waves;
  int32_t cl_mode;
} tpc_tuning;
int tpc_tuning_default(tpc_tuning* t);
int tpc_set_tuning(tpc_ctx* ctx, const tpc_tuning* t);
int tpc_get_tuning(tpc_ctx* ctx, tpc_tuning* t);

#ifdef __cplusplus
}
#endif

#endif /* TPC_H */
