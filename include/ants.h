/*
 * ants.h -- C ABI of the MI355X contracting-grid reconstruction library
 * (statistical event reconstruction for Anger-camera detectors after the
 * ANTS2 package, arXiv:1602.07247).
 *
 * Conventions for every entry point:
 *   - Return value: ants_status, 0 = OK, < 0 = error.  No entry point aborts
 *     or throws; after an error, ants_last_error() returns a message
 *     (thread-local, valid until the next call on the same thread).
 *   - Pointers named d_* are device pointers on the current HIP device;
 *     all other pointers are host pointers.  Host arrays inside descriptors
 *     are copied before the call returns; the caller keeps ownership.
 *   - Event and output buffers belong to the caller; the library never
 *     frees or reallocates them.
 *   - Work is enqueued asynchronously on `hip_stream` (a hipStream_t, NULL
 *     = the default stream); the caller synchronises.  Handles own their
 *     device memory and may be used from one stream at a time.
 *   - Floating-point layouts are row-major.
 */
#ifndef ANTS_H
#define ANTS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ANTS_OK = 0,
  ANTS_E_ARG = -1,          /* invalid argument (NULL, size, range)          */
  ANTS_E_FORMAT = -2,       /* malformed descriptor or file                  */
  ANTS_E_DEVICE = -3,       /* HIP runtime error                             */
  ANTS_E_NOMEM = -4,        /* device or host allocation failed              */
  ANTS_E_UNSUPPORTED = -5,  /* valid but not supported combination           */
  ANTS_E_STATE = -6         /* handle not ready (e.g. network not trained)   */
} ants_status;

/* Per-event status bits (ants_out.status).  Per-event problems never fail
 * a call.  Events with EMPTY, BAD_INPUT or NO_ACTIVE get NaN outputs. */
#define ANTS_EV_EMPTY 1          /* sum of active signals <= 0               */
#define ANTS_EV_BAD_INPUT 2      /* an active signal is NaN, Inf or negative */
#define ANTS_EV_NO_ACTIVE 4      /* every sensor is passive                  */
#define ANTS_EV_NO_VALID_NODE 8  /* at some iteration no node had S > 0      */
#define ANTS_EV_FALLBACK 16      /* seeded path re-ran the event on the full grid */
#define ANTS_EV_TIE 32           /* an exact tie of the statistic was broken by node index */

const char* ants_last_error(void);
const char* ants_version(void);

/* ------------------------------------------------------------------ */
/* LRF sets (Sec. 6: light response functions as cubic B-splines;      */
/* Sec. 6.1.1 "Axial" and "XY"; Sec. 6.1.2 r-z as a 2-D spline in the   */
/* distance from the sensor axis and the depth; Sec. 6.2 one LRF shared */
/* by a group with relative gains; Sec. 5.3 passive sensors).           */
/*                                                                     */
/* Spline convention: on each axis nb breakpoints lo + m*(hi-lo)/(nb-1) */
/* (m = 0..nb-1) and nb+2 coefficients of the uniform cubic B-spline on */
/* the extended knot vector; coefficient j belongs to the B-spline      */
/* centred on breakpoint j-1.  LRF = max(spline, 0) inside the domain   */
/* (with a relative slack of 1e-9 of the span), 0 outside.  For AXIAL   */
/* and RZ the first axis is r (lo[0] must be 0); RZ's second axis is z; */
/* XY's axes are global x and y.                                        */
/* ------------------------------------------------------------------ */
typedef enum {
  ANTS_LRF_AXIAL = 1,
  ANTS_LRF_XY = 2,
  ANTS_LRF_RZ = 3,
  /* Sec. 6.1.1 "Composite": an Axial LRF (the first-axis fields below, one
   * table shared by all sensors: shared must be 1) plus an XY LRF of the
   * residual (the xy_* fields, per sensor or shared); each part is 0
   * outside its own domain and the LRF is max(axial + residual, 0). */
  ANTS_LRF_COMPOSITE = 4,
  /* Sec. 6.1.2 "Sliced": XY LRFs (the fields below describe x and y) on
   * n_planes z planes at z_lo + p (z_hi - z_lo) / (n_planes - 1); the LRF
   * is (1 - t) L_p + t L_p+1 of the two closest planes' (clamped) values,
   * 0 outside [z_lo, z_hi] (relative slack 1e-9).  3-D grids only. */
  ANTS_LRF_SLICED = 5
} ants_lrf_kind;

typedef struct {
  int32_t n_sensors;          /* 1 .. 256                                       */
  const double* sensor_xy;    /* [n_sensors][2] sensor centres, mm               */
  const double* gain;         /* [n_sensors] relative gains g_i > 0; NULL = 1    */
  const uint8_t* active;      /* [n_sensors] 0 = passive; NULL = all active      */
  int32_t kind;               /* ants_lrf_kind                                   */
  int32_t shared;             /* 1: one table for all sensors; 0: one per sensor
                                 (RZ requires 1)                                  */
  int32_t n_knots[2];         /* breakpoints per axis (>= 2, <= 256); axis 1
                                 ignored for AXIAL                                */
  double lo[2], hi[2];        /* spline domain per axis, mm                      */
  const double* coef;         /* [n_tables][n_knots[1]+2][n_knots[0]+2] FP64;
                                 AXIAL and COMPOSITE: [n_tables][n_knots[0]+2];
                                 SLICED: [n_tables][n_planes][n_knots[1]+2]
                                 [n_knots[0]+2]                                   */
  /* COMPOSITE only: the XY residual (global x, y)                             */
  int32_t xy_knots[2];        /* breakpoints per axis, 2..256                      */
  double xy_lo[2], xy_hi[2];  /* residual domain, mm                               */
  const double* xy_coef;      /* [n_xy][xy_knots[1]+2][xy_knots[0]+2] FP64         */
  int32_t xy_shared;          /* 1: one residual for all sensors; 0: per sensor   */
  /* SLICED only                                                                 */
  int32_t n_planes;           /* 2..64                                            */
  double z_lo, z_hi;          /* z of the first and last plane, mm                */
} ants_lrf_desc;

typedef struct ants_lrfset ants_lrfset;   /* opaque; owns its device copies */

/* Validates the descriptor, compacts the active sensors and uploads FP32
 * piecewise-polynomial tables (for the screening pass) and the FP64
 * coefficients (for decisions and reported values) to the current device.
 * Errors: ANTS_E_ARG (NULL / sizes), ANTS_E_FORMAT (non-finite values,
 * lo >= hi, gain <= 0), ANTS_E_UNSUPPORTED (lo[0] != 0 for r, RZ per
 * sensor), ANTS_E_NOMEM, ANTS_E_DEVICE.  *out is NULL on error. */
ants_status ants_lrfset_create(const ants_lrf_desc* desc, ants_lrfset** out);
ants_status ants_lrfset_destroy(ants_lrfset* set);   /* NULL is a no-op */
/* n_sensors (row length of the signal matrix), active count and kind. */
ants_status ants_lrfset_info(const ants_lrfset* set, int32_t* n_sensors, int32_t* n_active,
                             int32_t* kind);

/* LRF-set file (Sec. 6: LRFs are stored and reloaded with the detector
 * configuration; here one binary file per set, version 1, little endian):
 *   char[8]  magic "ANTSLRF1"
 *   int32    n_sensors, kind, shared, n_knots[0], n_knots[1] (0 for AXIAL),
 *            reserved (0)
 *   double   lo[2], hi[2]          (axis 1 = 0 for AXIAL)
 *   int64    n_coef = (n_knots[0]+2) * (n_knots[1]+2 or 1) * (1 or n_sensors)
 *   double   sensor_xy[n_sensors][2], gain[n_sensors]
 *   uint8    active[n_sensors], zero padding to a multiple of 8 bytes
 *   double   coef[n_coef]          (layout of ants_lrf_desc.coef)
 *   uint64   FNV-1a (64-bit) hash of every preceding byte.
 * Composite and sliced sets are not written (ANTS_E_UNSUPPORTED).
 * ants_lrf_write writes a descriptor (NULL gain/active are written as 1);
 * ants_lrfset_save writes what a set was created from (all sensors, passive
 * ones included).  Errors: ANTS_E_ARG (NULL, sizes, unwritable path).
 * ants_lrfset_load reads a file and creates the set on the current device:
 * ANTS_E_ARG when the file cannot be opened, ANTS_E_FORMAT for a foreign,
 * truncated, extended or corrupted file (magic, header ranges, size,
 * checksum) and every error of ants_lrfset_create; *out is NULL on error. */
ants_status ants_lrf_write(const ants_lrf_desc* desc, const char* path);
ants_status ants_lrfset_save(const ants_lrfset* set, const char* path);
ants_status ants_lrfset_load(const char* path, ants_lrfset** out);

/* ------------------------------------------------------------------ */
/* Contracting-grid search (Sec. 5.1.2.2).  Per event:                  */
/*  - start at the gain-weighted centroid (Sec. 5.1.1), the strongest    */
/*    active sensor (Sec. 5.1.2.1; lowest index on ties) or a seed;      */
/*  - iteration k evaluates a regular nodes[0] x nodes[1] x nodes[2]     */
/*    grid with step step0 * shrink^k centred on the current centre;     */
/*    node j = (jz*ny + jy)*nx + jx sits at centre + (j_a - (n_a-1)/2)*s_a;*/
/*  - at each node: S = sum_active g_i L_i, A = N/S with N = sum_active   */
/*    n_i (energy as the ratio of the two sums, Sec. 5.1.2.2), and the    */
/*    statistic (Sec. 5.1.2: maximum likelihood or least squares):       */
/*      ML:   -lnL, lnL = sum[n_i ln(A g_i max(L_i,l_floor)) - A g_i L_i] */
/*            (terms with n_i = 0 reduce to -A g_i L_i; -sum ln n_i!      */
/*            dropped);                                                   */
/*      CHI2: sum (n_i - A g_i L_i)^2 / max(A g_i L_i, v_floor);          */
/*    S <= 0 makes a node invalid (+inf);                                 */
/*  - the node with the smallest (statistic, index) becomes the centre.  */
/* Outputs at the final centre: x, y, z (z = z_start for 2-D grids),     */
/* E = A, lnl = lnL, chi2 (both always), ndf = n_active - (d+1) with     */
/* d = 2 or 3.  Decisions between close nodes are taken in FP64, so the  */
/* path matches an FP64 evaluation of the same definitions.             */
/* ------------------------------------------------------------------ */
typedef enum { ANTS_STAT_ML = 0, ANTS_STAT_CHI2 = 1 } ants_stat;
typedef enum { ANTS_START_COG = 0, ANTS_START_MAXSENSOR = 1, ANTS_START_SEED = 2 } ants_start;

typedef struct {
  int32_t nodes[3];        /* odd, >= 1; nodes[2] = 1 for 2-D (<= 101 for r-z);
                              product <= 512                                    */
  int32_t iterations;      /* K grids evaluated, 0 .. 64 (0 returns the start) */
  double shrink;           /* step factor per iteration, (0, 1]                */
  double step0[3];         /* initial step per axis, mm (> 0 where nodes > 1)  */
  double z_start;          /* z of the start for 3-D grids and z output of 2-D */
  int32_t stat;            /* ants_stat                                        */
  int32_t start;           /* ants_start                                       */
  double l_floor;          /* floor of L inside the logarithm (default 1e-9)   */
  double v_floor;          /* chi2 variance floor (default 1)                  */
  double screen_scale;     /* multiplier (>= 1) on the error bound of the FP32
                              screening pass; nodes within it of the best are
                              re-decided in FP64.  0 = default (1).            */
  /* Per-event steps for refining a seed (start == SEED only; seed_steps = 0
   * keeps step0 and iterations).  With seed_steps = 1 the seed row is
   * (x, y, z, s) with s a log-variance: sigma_a = seed_scale[a] * exp(s/2)
   * per axis; the final step is s_f = step0 * shrink^(iterations-1) (per
   * axis, iterated products) and the event runs K in [seed_kmin, seed_kmax]
   * iterations from s_f * shrink^-(K-1) (iterated quotients), K the
   * smallest with s_f * shrink^-(K-1) >= seed_kappa * sigma_a on every axis
   * with nodes > 1 (seed_kmax when s is not finite).  Requires
   * 1 <= seed_kmin <= seed_kmax <= min(iterations, 16). */
  int32_t seed_steps;
  double seed_kappa;
  int32_t seed_kmin, seed_kmax;
  double seed_scale[3];
  /* Sensor cuts (Sec. 5.1.2): an event ignores the active sensors with a
   * signal below cut_signal, or farther in x-y than cut_distance (mm) from
   * its start position; 0 disables a cut.  The start position uses every
   * active sensor; the ignored ones then leave the statistic, the energy
   * ratio, the outputs and ndf, as if passive for that event.  No sensor
   * left gives ANTS_EV_NO_ACTIVE, no signal left ANTS_EV_EMPTY. */
  double cut_signal;
  double cut_distance;
} ants_grid_cfg;

/* Caller-owned device arrays of length n_events (path: [n][iterations]).
 * x..status are required; path and n_fp64 may be NULL. */
typedef struct {
  float* x;
  float* y;
  float* z;
  float* E;
  float* lnl;
  float* chi2;
  int32_t* ndf;
  int32_t* status;
  int32_t* path;     /* optional: winning node index per iteration (-1 = none) */
  int32_t* n_fp64;   /* optional: node evaluations re-done in FP64 per event   */
} ants_out;

/* Reconstruct d_signals [n_events][n_sensors] (FP32, row-major; counts or
 * gain-corrected amplitudes).  d_seeds [n_events][4] = (x, y, z, unused) is
 * read only when cfg->start == ANTS_START_SEED.  n_events may be 0. */
ants_status ants_reconstruct(ants_lrfset* set, const ants_grid_cfg* cfg, int64_t n_events,
                             const float* d_signals, const float* d_seeds, ants_out out,
                             void* hip_stream);

/* Launch plan of ants_reconstruct (and of the refinement and fallback
 * grids of the seeded path) for one grid configuration of one set.  The
 * reconstructed values do not depend on it. */
typedef struct {
  int32_t waves_per_block;   /* events in flight per block: 1, 2 or 4 (default 4) */
  int32_t blocks_per_cu;     /* cap on resident blocks per compute unit; 0 = as many
                                as fit (default)                                   */
  int32_t screen;            /* 0 (default): a factored screen where one applies:
                                r-z column-factored (ML, 3, 5 or 7 z planes, <= 64
                                active sensors), or XY with each sensor's
                                coefficients collapsed along y for the grid's node
                                rows and staged in LDS (one z plane, <= 64 node
                                columns and rows, rows x nc0 <= 1536); 1: the
                                per-node screen (XY: coefficients read through the
                                cache)                                             */
} ants_grid_plan;

/* Autotuner (per set and grid configuration): times the candidate plans
 * (screen variant where both apply, waves per block 4/2/1, blocks per CU
 * as many as fit or 2) on the first n_sample events of d_signals (d_seeds
 * as for ants_reconstruct), writing into `scratch` (n_sample rows); only
 * the kernel is timed, between HIP events, after a warm-up launch.  The
 * fastest goes to *best and is stored in the set for this configuration
 * (up to 8 configurations per set, the oldest dropped first); host_ms
 * [12] (or NULL) receives each candidate's time in search order (screen
 * outermost, then waves per block, then blocks per CU).  Synchronises the
 * stream.  ants_set_plan stores a plan explicitly (NULL removes it), for
 * a deterministic choice. */
ants_status ants_autotune(ants_lrfset* set, const ants_grid_cfg* cfg, int64_t n_sample,
                          const float* d_signals, const float* d_seeds, ants_out scratch,
                          ants_grid_plan* best, double* host_ms, void* hip_stream);
ants_status ants_set_plan(ants_lrfset* set, const ants_grid_cfg* cfg,
                          const ants_grid_plan* plan);

/* ------------------------------------------------------------------ */
/* Simplex search (Sec. 5.1.2.1: the Minuit2 Simplex minimiser over the  */
/* position, x, y or x, y, z, from the centroid or the strongest        */
/* sensor; here also from a seed).  The Nelder-Mead method as defined by */
/* Lagarias, Reeds, Wright and Wright (SIAM J. Optim. 9, 1998):         */
/* coefficients 1 (reflection), 2 (expansion), 1/2 (contraction), 1/2   */
/* (shrink); initial simplex = the start and the start moved by step0[a] */
/* along each searched axis a; vertices ordered by the statistic of the */
/* grid search (same definitions, energy A = N/S at every point), values */
/* within 1e-12 N equal and a new vertex placed after the vertices equal */
/* to it; stop when every vertex is within tol of the best on every     */
/* searched axis, or after max_iter iterations.  Everything is FP64.    */
/* Outputs as for ants_reconstruct at the best vertex (z = z_start for  */
/* dims = 2); d_iters [n] (optional, device) receives the iterations    */
/* run per event and out.n_fp64 (optional) the statistic evaluations    */
/* (all FP64).  ANTS_EV_NO_VALID_NODE: the search ended on a point with */
/* S <= 0 (outputs NaN).                                                */
/* ------------------------------------------------------------------ */
typedef struct {
  int32_t dims;          /* 2: x, y;  3: x, y, z (r-z LRFs only)             */
  int32_t stat;          /* ants_stat                                        */
  int32_t start;         /* ants_start; SEED reads d_seeds [n][4] (x, y, z, -) */
  double step0[3];       /* initial simplex edge per searched axis, mm (> 0)  */
  double z_start;        /* start z (also the output z of 2-D searches)      */
  double tol;            /* convergence size, mm (> 0)                       */
  int32_t max_iter;      /* iteration cap, 0 .. 100000                       */
  double l_floor, v_floor;
} ants_simplex_cfg;

ants_status ants_reconstruct_simplex(ants_lrfset* set, const ants_simplex_cfg* cfg,
                                     int64_t n_events, const float* d_signals,
                                     const float* d_seeds, ants_out out, int32_t* d_iters,
                                     void* hip_stream);

/* ------------------------------------------------------------------ */
/* Variable-metric search (Sec. 5.1.2.1: the Minuit2 Migrad minimiser,  */
/* a variable-metric method with numerical derivatives), over x, y or   */
/* x, y, z from the centroid, the strongest sensor or a seed, on the    */
/* grid's statistic.  Steps: gradient g by central differences with     */
/* step h per searched axis; initial inverse curvature V diagonal, 1 /  */
/* the central second difference at the start, or step0[a]^2 where that  */
/* is not positive; EDM = g^T V g / 2, stop when EDM < edm_tol or after */
/* max_iter accepted steps; direction -V g (V reset to diag(step0^2)    */
/* when it is not a descent direction); step length 1 halved (at most  */
/* 20 times) until F decreases by at least 1e-4 of the linear          */
/* prediction; BFGS update of V when s^T y > 0.  Coordinates that are  */
/* spline arguments (z of r-z and sliced LRFs, x and y of XY and sliced */
/* LRFs) are limited to the spline's domain [lo, hi] as Minuit limits  */
/* parameters: the search runs in u, position lo + (hi - lo)(sin u + 1)/2,*/
/* with h and step0 divided by (hi - lo) / 2.  A non-finite gradient   */
/* ends the search at the current point; a start with a non-finite     */
/* statistic gives ANTS_EV_NO_VALID_NODE.  Everything is FP64.  Outputs */
/* and d_iters / out.n_fp64 (accepted steps / evaluations) as for the   */
/* simplex search.                                                      */
/* ------------------------------------------------------------------ */
typedef struct {
  int32_t dims;          /* 2: x, y;  3: x, y, z (r-z and sliced LRFs only)  */
  int32_t stat;          /* ants_stat                                        */
  int32_t start;         /* ants_start; SEED reads d_seeds [n][4] (x, y, z, -) */
  double step0[3];       /* per-axis scale, mm (> 0): the fallback curvature */
  double z_start;        /* start z (also the output z of 2-D searches)      */
  double h;              /* central-difference step, mm (> 0)               */
  double edm_tol;        /* EDM stop, statistic units (> 0)                  */
  int32_t max_iter;      /* cap on accepted steps, 0 .. 100000              */
  double l_floor, v_floor;
} ants_migrad_cfg;

ants_status ants_reconstruct_migrad(ants_lrfset* set, const ants_migrad_cfg* cfg,
                                    int64_t n_events, const float* d_signals,
                                    const float* d_seeds, ants_out out, int32_t* d_iters,
                                    void* hip_stream);

/* ------------------------------------------------------------------ */
/* k-NN reconstruction (Sec. 5.1.4): an event is the point of its       */
/* normalised active-sensor signals n_i / N (N = sum over the active    */
/* sensors; divided in double, rounded to single precision); its        */
/* position is the mean of the known positions of the k calibration    */
/* events closest to it.  Distance: squared Euclidean over the active   */
/* sensors in single precision, accumulated in sensor order with every  */
/* operation rounded as written (it decides an integer result, so it is */
/* exactly reproducible); neighbours ordered by (distance, calibration  */
/* index).  Exact brute force over the whole calibration set.           */
/* ------------------------------------------------------------------ */
typedef struct ants_knn ants_knn;   /* opaque; owns the normalised calibration set */

/* Calibration set of n_cal events of `set`'s detector (at most 128 active
 * sensors): d_signals [n_cal][n_sensors] and d_pos [n_cal][3] (x, y, z)
 * FP32 device arrays, copied and normalised on `hip_stream` (usable on
 * that stream right away; the caller's arrays may be freed once the
 * stream has passed this call).  Calibration events with N <= 0 or a
 * non-finite or negative active signal never become neighbours. */
ants_status ants_knn_create(ants_lrfset* set, int64_t n_cal, const float* d_signals,
                            const float* d_pos, ants_knn** out, void* hip_stream);
ants_status ants_knn_destroy(ants_knn* knn);   /* NULL is a no-op */
/* k in 1..32.  d_xyz [n][3] FP32 positions (the mean of the neighbours'
 * positions in double), d_status [n] the grid's input status bits
 * (EMPTY, BAD_INPUT, NO_ACTIVE; NO_VALID_NODE when no calibration event is
 * valid), NaN positions for those events.  Optional d_idx [n][k] int32 and
 * d_dist [n][k] FP32: the neighbours in order (-1 / +inf past the valid
 * calibration events). */
ants_status ants_knn_reconstruct(ants_knn* knn, int32_t k, int64_t n_events,
                                 const float* d_signals, float* d_xyz, int32_t* d_status,
                                 int32_t* d_idx, float* d_dist, void* hip_stream);

/* ------------------------------------------------------------------ */
/* One persistent launch over event chunks from several detectors (one  */
/* LRF set and grid configuration per detector; every set must have the */
/* same LRF kind and the same statistic).  Chunk c holds n_events rows   */
/* of its set's n_sensors signals and writes output rows out_offset ..   */
/* out_offset + n_events - 1.  Results equal ants_reconstruct of each   */
/* chunk with its set and configuration, for every plan.                */
/* ------------------------------------------------------------------ */
typedef struct {
  int32_t set;              /* index into sets / cfgs                        */
  int64_t n_events;
  const float* d_signals;   /* [n_events][n_sensors of the set]              */
  int64_t out_offset;
} ants_chunk;

/* Launch plan: events per work item, resident blocks per compute unit,
 * and whether the LRF tables are staged in LDS (1) or read through the
 * cache (0), for every set.  NULL plan = each set's part of the plan that
 * ants_autotune_multi stored in its handle for its configuration, else
 * {32, 8, 1}.  Within one launch each set also runs with the fewest sensor
 * slots per lane that hold its sensors. */
typedef struct {
  int32_t events_per_item;   /* 1 .. 4096 */
  int32_t blocks_per_cu;     /* 1 .. 32   */
  int32_t table_in_lds;      /* 0 or 1    */
} ants_plan;

/* ants_out.path is ignored (n_fp64 likewise).  Up to 64 sets and 2^24 chunks.
 * The library keeps descriptor workspace in sets[0] (device memory and a
 * pinned host staging area); the descriptors are copied on the stream and
 * the call does not wait for the device, except that it waits for the
 * previous call's descriptor copy before reusing the staging area.  Calls
 * sharing sets[0] must not overlap on different streams. */
ants_status ants_reconstruct_multi(ants_lrfset* const* sets, const ants_grid_cfg* cfgs,
                                   int32_t n_sets, const ants_chunk* chunks, int32_t n_chunks,
                                   const ants_plan* plan, ants_out out, void* hip_stream);

/* Autotuner: times candidate plans on a sample of `sample_events` events
 * made of whole chunks taken at an even stride through the stream (every
 * detector in proportion), writing into `scratch` (rows 0 ..
 * sample_events-1).  Only the kernel is timed (HIP events around the
 * launch, descriptors uploaded before).  Search: blocks per CU 4/8/16 with
 * the default per-set plan, then for each set in turn events per item
 * 8/32/128 x tables in LDS or not, keeping the best so far.  Each set's
 * part of the result is stored in its handle for its configuration (used
 * when ants_reconstruct_multi gets a NULL plan); *best receives the first
 * set's part; host_ms [3 + 6 n_sets] (or NULL) each candidate's time in
 * search order.  Synchronises the stream.  The choice depends on timing;
 * the reconstructed values do not. */
ants_status ants_autotune_multi(ants_lrfset* const* sets, const ants_grid_cfg* cfgs,
                                int32_t n_sets, const ants_chunk* chunks, int32_t n_chunks,
                                int64_t sample_events, ants_out scratch, ants_plan* best,
                                double* host_ms, void* hip_stream);

/* ------------------------------------------------------------------ */
/* Event generator: flood-field events drawn from the LRF model itself  */
/* (Sec. 4.1.1 "flood field"; Sec. 5.1.1 relative gains).  For event    */
/* index i = first_event + e: position uniform over a disc of radius    */
/* `extent` (region 0: r = extent*sqrt(u1), phi = 2*pi*u2) or a square  */
/* of half-width `extent` (region 1), depth z = z_lo + (z_hi-z_lo)*u3   */
/* (z_lo when z_hi <= z_lo), E_tot = e_lo + (e_hi-e_lo)*u4; expected    */
/* counts mu_i = A g_i L_i with sum over active sensors = E_tot; counts */
/* ~ Poisson(mu_i) (or mu_i when noiseless), passive sensors 0.          */
/* Uniforms come from Philox4x32-10 (Salmon et al., SC'11) with key =   */
/* seed and counter (i, stream, call): position/energy stream          */
/* 0xFFFFFFFF calls 0 and 1; sensor column c uses stream c.  Two 32-bit */
/* words (a, b) give u = ((a:b) >> 11 + 0.5) * 2^-53.  Poisson: below  */
/* mu = 10 sequential-search inversion of one uniform; otherwise the    */
/* transformed rejection method of Hoermann (1993), call t for trial t. */
/* ------------------------------------------------------------------ */
typedef struct {
  int32_t region;      /* 0 disc, 1 square                                 */
  double extent;       /* disc radius or square half-width, mm             */
  double z_lo, z_hi;   /* depth range, mm                                  */
  double e_lo, e_hi;   /* total expected photoelectrons                    */
  int32_t noiseless;   /* 1: write the means instead of Poisson draws      */
} ants_gen_cfg;

/* d_signals [n_events][n_sensors] FP32 (caller-owned device memory);
 * d_truth [n_events][4] = (x, y, z, E_tot) or NULL. */
ants_status ants_generate(ants_lrfset* set, const ants_gen_cfg* cfg, int64_t n_events,
                          uint64_t seed, uint64_t first_event, float* d_signals, float* d_truth,
                          void* hip_stream);

/* ------------------------------------------------------------------ */
/* Learned seed (Sec. 5.1.3: neural-network reconstruction trained on   */
/* events with known positions; here a fully connected ReLU network     */
/* n_in -> hidden x n_layers -> 4 maps the normalised signals           */
/* x_a = n_a * n_active / N of the active sensors to (p_x, p_y, p_z, s):*/
/* position p = (pos - pos_offset) / pos_scale and log-variance s).     */
/* Weights: FP32 master copy and BF16 copy; activations BF16; products  */
/* accumulate in FP32 on the matrix cores.  Training loss per event:    */
/* 0.5 exp(-s) |p - t|^2 + 1.5 s, averaged over the batch; Adam.        */
/* Flat parameter order: W1 [hidden][n_in_pad], b1, W2 [hidden][hidden], */
/* b2, ..., W_out [4][hidden], b_out; n_in_pad = n_in rounded up to 32   */
/* (padding columns are zero).                                          */
/* ------------------------------------------------------------------ */
typedef struct ants_mlp ants_mlp;   /* opaque; owns parameters, optimiser state, workspace */

typedef struct {
  int32_t n_in;            /* inputs = active sensors of the LRF set used, 1..64 */
  int32_t hidden;          /* 256                                               */
  int32_t n_layers;        /* hidden layers, 1..4                               */
  uint64_t seed;           /* initialisation: He-uniform weights, zero biases   */
  double pos_scale[3];     /* mm per output unit                                */
  double pos_offset[3];    /* mm                                                */
} ants_mlp_cfg;

typedef struct {
  double lr, beta1, beta2, eps;   /* Adam step size and decay rates            */
} ants_adam_cfg;

typedef struct {
  int64_t n_train, n_val;   /* events drawn with ants_generate                    */
  int32_t batch, epochs;
  ants_adam_cfg adam;
  double lr_decay;          /* step size multiplied by this after every epoch     */
  uint64_t seed;            /* generator seed (training events start at index 0,  */
                            /* validation events at index n_train)               */
  ants_gen_cfg events;      /* event recipe                                       */
} ants_train_cfg;

ants_status ants_mlp_create(const ants_mlp_cfg* cfg, ants_mlp** out);
ants_status ants_mlp_destroy(ants_mlp* mlp);     /* NULL is a no-op */
int64_t ants_mlp_num_params(const ants_mlp* mlp);
/* Copy the FP32 master parameters to / from host memory (n = num_params).
 * Setting parameters refreshes the BF16 copy and clears the Adam state. */
ants_status ants_mlp_get_params(const ants_mlp* mlp, float* host, int64_t n);
ants_status ants_mlp_set_params(ants_mlp* mlp, const float* host, int64_t n);
/* Network outputs d_pred [n][4] = (p_x, p_y, p_z, s) for d_signals
 * [n][n_sensors] of `set` (its active sensors are the inputs). */
ants_status ants_mlp_forward(ants_mlp* mlp, const ants_lrfset* set, int64_t n,
                             const float* d_signals, float* d_pred, void* hip_stream);
/* Gradient of the mean loss over the batch (n <= 65536) with respect to the
 * flat parameters (d_grad, FP32) and the mean loss (d_loss, one float);
 * d_target [n][3] true positions in mm.  No update. */
ants_status ants_mlp_grad(ants_mlp* mlp, const ants_lrfset* set, int64_t n,
                          const float* d_signals, const float* d_target, float* d_grad,
                          float* d_loss, void* hip_stream);
/* One Adam step on a batch (n <= 65536); d_loss may be NULL. */
ants_status ants_mlp_train_step(ants_mlp* mlp, const ants_lrfset* set, int64_t n,
                                const float* d_signals, const float* d_target,
                                const ants_adam_cfg* adam, float* d_loss, void* hip_stream);
/* Whole training run on events drawn from `set`'s own LRF model
 * (ants_generate): epochs over n_train events, validation loss on n_val
 * held-out events after each epoch; the parameters of the best validation
 * epoch are kept.  host_losses [epochs][2] = (train, validation) mean loss
 * or NULL.  Synchronises the stream. */
ants_status ants_mlp_train(ants_mlp* mlp, const ants_lrfset* set, const ants_train_cfg* cfg,
                           double* host_losses, void* hip_stream);
/* Binary file: magic "ANTSMLP1", the ants_mlp_cfg fields, then the FP32
 * parameters (little endian). */
ants_status ants_mlp_save(const ants_mlp* mlp, const char* path);
ants_status ants_mlp_load(const char* path, ants_mlp** out);

/* Seeded reconstruction: seeds from the network (or from d_seeds [n][4] =
 * (x, y, z, log-variance) in mm when d_seeds is not NULL, and then mlp may be
 * NULL), a refinement grid `refine` started at the seed (start = SEED,
 * normally seed_steps = 1), and events whose refined chi2/ndf exceeds
 * chi2ndf_max >= 0 (or is not finite, or ndf <= 0) run again with `fallback`
 * (normally the plain grid from the centroid) and get ANTS_EV_FALLBACK.
 * d_n_fallback (one int32, device) receives the number of such events.
 * The network runs as one fused kernel (no activation buffers).  The
 * library keeps, in the LRF set, a workspace of 16 bytes per event for the
 * seeds and 4 bytes per event for the fallback list; calls that share a set
 * must not overlap in time. */
ants_status ants_reconstruct_seeded(ants_lrfset* set, ants_mlp* mlp,
                                    const ants_grid_cfg* refine, const ants_grid_cfg* fallback,
                                    double chi2ndf_max, int64_t n_events, const float* d_signals,
                                    const float* d_seeds, ants_out out, int32_t* d_n_fallback,
                                    void* hip_stream);

/* Allocation-free variant of ants_reconstruct_seeded, for callers that
 * cannot allocate device memory (code under HIP graph capture, serving
 * loops that forbid hipMalloc).  Same arguments, checks, results and status
 * bits; it calls no hipMalloc/hipFree.  Its workspace (fallback counter,
 * fallback list, network seeds) is one fixed array per device, 20 MiB for
 * ANTS_NOALLOC_MAX_EVENTS events, held from the first call on a device until
 * the process ends.  n_events above ANTS_NOALLOC_MAX_EVENTS gives ANTS_E_ARG
 * (split the batch).  Every call on a device shares that device's array:
 * calls that overlap in time on one device race (use one stream, or
 * serialise them). */
#define ANTS_NOALLOC_MAX_EVENTS (1 << 20)
ants_status ants_reconstruct_seeded_noalloc(ants_lrfset* set, ants_mlp* mlp,
                                            const ants_grid_cfg* refine,
                                            const ants_grid_cfg* fallback, double chi2ndf_max,
                                            int64_t n_events, const float* d_signals,
                                            const float* d_seeds, ants_out out,
                                            int32_t* d_n_fallback, void* hip_stream);

/* ------------------------------------------------------------------ */
/* LRF fit from events (Sec. 6: LRFs computed from signals and event    */
/* positions; Sec. 6.2: one LRF for all sensors with relative gains;    */
/* Sec. 8: the iterative procedure alternates it with the               */
/* reconstruction and keeps only events that pass a filter).  Axial LRF,*/
/* one shared table of nb + 2 cubic B-spline coefficients c: least      */
/* squares on the estimates n_ie / (E_e g_i) of L(r_ie), one per (event */
/* e, active sensor i) pair with lo <= r_ie <= hi (relative slack 1e-9  */
/* of the span), all weighted 1; ridge * (mean diagonal) is added to    */
/* the diagonal of the normal matrix.  An event enters when its status  */
/* has none of the bits EMPTY, BAD_INPUT, NO_ACTIVE, NO_VALID_NODE (TIE */
/* and FALLBACK only describe how a valid position was found), 0 < E <  */
/* inf and, if chi2ndf_max > 0, ndf > 0 and chi2 / ndf <= chi2ndf_max. */
/* ------------------------------------------------------------------ */
typedef struct {
  int32_t nb;           /* breakpoints of the fitted spline, 4..62           */
  double lo, hi;        /* domain in mm (lo = 0 for tables the reconstruction reads) */
  double ridge;         /* relative ridge, >= 0 (1e-9 typical)               */
  double chi2ndf_max;   /* event filter; <= 0: no chi2 cut                   */
} ants_fit_cfg;

/* Sensors (positions, gains, active set) are `set`'s; its LRF is not read.
 * d_signals [n_events][ld] FP32 (ld >= n_sensors); rec: x, y, E, chi2, ndf
 * and status per event (an ants_reconstruct output; z and lnl are not
 * read).  Writes d_coef [nb + 2] FP64 and, when not NULL, d_counts [2]
 * int64 = (events used, pairs used); both device memory, caller-owned.
 * Everything runs on the device in FP64: per-wave normal equations in LDS,
 * summed over the waves by a fixed tree, then a Cholesky solve.  A normal
 * matrix that is not positive definite (part of the domain without data
 * and ridge 0) gives NaN coefficients.  The set keeps a workspace of
 * 8 (5 (nb + 2) + 2) bytes per wave (at most 32 waves per compute unit, plus
 * one for the sums); calls that share a set must not overlap in time. */
ants_status ants_fit_axial_lrf(ants_lrfset* set, const ants_fit_cfg* cfg, int64_t n_events,
                               const float* d_signals, int64_t ld, ants_out rec, double* d_coef,
                               int64_t* d_counts, void* hip_stream);

/* Grouped fit (Sec. 6.2: sensors in groups that share one LRF, each with
 * its relative gain; one group for all, groups by distance from the array
 * centre or by symmetry, or every sensor its own).  d_group [n_sensors]
 * int32, device memory, caller-owned: the group of each sensor (by sensor
 * index), 0..n_groups-1; other values (e.g. -1) leave the sensor out of
 * every fit; passive sensors are always out.  Each group's table is fitted
 * as ants_fit_axial_lrf fits the shared one, from its members' pairs only.
 * d_shift [n_events][2] FP32 or NULL: added to each event's (x, y) before
 * the fit (Sec. 8: a small random shift of the reconstructed positions
 * helps the first iterations; the caller draws it).  Writes d_coef
 * [n_groups][nb + 2] FP64 (NaN rows for groups without pairs and ridge 0,
 * or without any pair) and, when not NULL, d_counts [n_groups][2] int64 =
 * (events used, pairs of the group).  n_groups 1..4096.  Same determinism,
 * workspace rule and stream behaviour as ants_fit_axial_lrf (workspace:
 * 8 (5 (nb + 2) + 2) bytes per wave of each group). */
ants_status ants_fit_axial_lrf_grouped(ants_lrfset* set, const ants_fit_cfg* cfg,
                                       int32_t n_groups, const int32_t* d_group,
                                       int64_t n_events, const float* d_signals, int64_t ld,
                                       ants_out rec, const float* d_shift, double* d_coef,
                                       int64_t* d_counts, void* hip_stream);

/* Two-dimensional LRF fits (Sec. 6: LRFs from signals and positions; r-z
 * LRFs in r and depth and per-sensor XY LRFs, Sec. 6.1.1; groups, Sec.
 * 6.2): least squares on n / (E g) against the reconstruction's
 * tensor-product cubic B-spline (table [nb[1] + 2][nb[0] + 2]), one table
 * per group, from the pairs whose arguments (r, z) (kind r-z; z from
 * rec.z) or (x, y) (kind XY) lie in the domains (relative slack 1e-9);
 * ridge * mean diagonal on the diagonal; the event filter, groups
 * (d_group by sensor index, -1 left out) and shifts as for
 * ants_fit_axial_lrf_grouped.  Writes d_coef [n_groups][nb[1] + 2][nb[0] +
 * 2] FP64 (NaN tables for groups without a positive definite system) and
 * d_counts [n_groups][2] (events used, pairs) when not NULL.  The events
 * are bucketed by the interval of their second coordinate and the normal
 * equations summed per interval in LDS, then added in a fixed order:
 * results repeat bit for bit and agree with an FP64 reference to rounding.
 * nb 4..64 per axis, 1..1024 groups, at most 2^31 - 1 events; workspace,
 * kept in the set: 8 (nb[0] + 2)(nb[1] + 2)(3 nb[0] + 12) bytes per group,
 * plus 1216 n_groups (nb[0] - 1)(nb[1] - 1)(segments + 1) bytes with about
 * 4 x (compute units) / ((nb[1] - 1) x batches of groups) segments (a batch
 * holds up to about 65 / (nb[0] - 1) groups; 29 MB for one 24 x 16 table
 * on 256 compute units), plus 4 bytes per event.  Asynchronous on
 * hip_stream. */
typedef struct {
  int32_t kind;         /* ANTS_LRF_RZ or ANTS_LRF_XY                       */
  int32_t nb[2];        /* breakpoints per axis (u = r or x, w = z or y)     */
  double lo[2], hi[2];  /* domains in mm (r-z: lo[0] >= 0)                  */
  double ridge;         /* relative ridge, >= 0                              */
  double chi2ndf_max;   /* event filter; <= 0: no chi2 cut                   */
  /* Residual of a composite LRF (Sec. 6.1.1; kind XY only): an axial
   * spline, its value at the pair's distance r from the sensor (not
   * clamped, 0 outside [base_lo, base_hi]) subtracted from every estimate.
   * d_base [base_nb + 2] FP64, device memory, caller-owned; NULL: none.  */
  const double* d_base;
  int32_t base_nb;      /* 2..256                                            */
  double base_lo, base_hi;   /* 0 <= base_lo < base_hi, mm                  */
  /* Depth window (one plane of a sliced LRF, Sec. 6.1.2): only events with
   * ev_z_lo <= rec.z < ev_z_hi enter; ev_z_lo >= ev_z_hi: no window.
   * Infinite bounds are allowed, NaN is not.                              */
  double ev_z_lo, ev_z_hi;
} ants_fit2d_cfg;

ants_status ants_fit_lrf2d_grouped(ants_lrfset* set, const ants_fit2d_cfg* cfg,
                                   int32_t n_groups, const int32_t* d_group, int64_t n_events,
                                   const float* d_signals, int64_t ld, ants_out rec,
                                   const float* d_shift, double* d_coef, int64_t* d_counts,
                                   void* hip_stream);

/* Relative gains re-calculated within fixed groups (Sec. 6.3), the LRF
 * profiles unchanged: for each active sensor i with d_table_of[i] in
 * 0..n_tables-1, the least-squares scale g_i = sum (n/E) L / sum L^2 of
 * its estimates n_ie / E_e against the reconstruction's LRF of its table,
 * L(r) = max(spline, 0) (d_tables [n_tables][nb + 2] FP64 on cfg's nb, lo,
 * hi), over its pairs inside the domain and the events cfg's filter keeps
 * (cfg->ridge is not used).  Writes d_gains[i] (NaN without pairs or with
 * sum L^2 = 0) and, when not NULL, d_pairs[i] int64, for those sensors
 * only (by sensor index; other entries untouched).  d_shift as in the
 * grouped fit.  All arrays are device memory, caller-owned. */
ants_status ants_fit_axial_gains(ants_lrfset* set, const ants_fit_cfg* cfg, int32_t n_tables,
                                 const double* d_tables, const int32_t* d_table_of,
                                 int64_t n_events, const float* d_signals, int64_t ld,
                                 ants_out rec, const float* d_shift, double* d_gains,
                                 int64_t* d_pairs, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* ANTS_H */
