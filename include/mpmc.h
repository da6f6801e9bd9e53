/*
 * mpmc.h — C ABI of the MI355X massively parallel local Monte Carlo (MPMC)
 * sampler for hard disks (Engel, Anderson, Glotzer, Isobe, Bernard, Krauth,
 * "Hard-disk equation of state: first-order liquid-hexatic transition in two
 * dimensions with three simulation methods", arXiv:1211.1645).
 *
 * Model (Sec. II.A): N hard disks of radius sigma = 1 in a periodic L x L
 * square box at packing fraction eta = N pi / L^2, sampled in the NVT
 * ensemble.  Sampler (Sec. II.B): a four-colour checkerboard of cells of
 * width w >= 2 sigma, shifted at random every sweep; all cells of one colour
 * make local trial moves at once, rejecting moves that leave the cell or
 * overlap another disk.  Observables: the contact pair histogram and the
 * pressure from the contact value of g(r) (Sec. II.C.1, Eqs. (1), (2), (4)),
 * and the orientational order psi_j, Psi_6 (Eq. (8), Sec. III).
 *
 * Conventions for every entry point:
 *  - Return value: MPMC_OK (0) or a negative MPMC_E* code; the message of the
 *    last failure on the calling thread is mpmc_last_error().  No C++
 *    exception crosses this interface.  After MPMC_EDEVICE a handle may only
 *    be freed.
 *  - Ownership: a box handle owns all its device state; buffers passed in are
 *    owned by the caller and only read or written during the call.
 *  - Pointers are host pointers unless a parameter says "device".
 *  - Work is enqueued on the box's stream (mpmc_params.stream, a hipStream_t;
 *    NULL = the default stream).  Calls that return host data synchronise
 *    that stream before returning.
 *  - Units: sigma = 1.  Positions are on the lattice of spacing q = 2^-22; a
 *    "q unit" is one lattice step.  Coordinates inside a cell are fp32.
 */
#ifndef MPMC_H
#define MPMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPMC_OK 0
#define MPMC_EINVAL (-1)    /* invalid argument or parameter combination */
#define MPMC_ENOMEM (-2)    /* device or host allocation failed */
#define MPMC_EDEVICE (-3)   /* HIP runtime error; the handle may only be freed */
#define MPMC_ESTATE (-4)    /* call not valid in the current state */
#define MPMC_EOVERFLOW (-5) /* a cell exceeded its capacity (corrupt input) */
#define MPMC_EIO (-6)       /* checkpoint file error */

#define MPMC_LATTICE_SQUARE 0     /* sqrt(N) x sqrt(N) square lattice */
#define MPMC_LATTICE_TRIANGULAR 1 /* sqrt(N) rows, odd rows offset by half */
#define MPMC_LATTICE_NONE 2       /* no start; call mpmc_set_positions */

#define MPMC_SCHED_AUTO 0   /* fused tile kernel, autotuned tile */
#define MPMC_SCHED_SIMPLE 1 /* one kernel per colour sub-sweep */
#define MPMC_SCHED_FUSED 2  /* one LDS-tiled kernel per sweep, tile given */

typedef struct mpmc_box_s *mpmc_box;

typedef void *(*mpmc_alloc_fn)(size_t bytes, void *ctx);
typedef void (*mpmc_free_fn)(void *ptr, void *ctx);

typedef struct mpmc_params {
    uint32_t step_m;    /* trial step d = step_m * 2^-8 sigma, 1..255; each
                           axis of a displacement is uniform over 2^14 odd
                           multiples of step_m q inside (-d, d) */
    uint32_t n_trial;   /* trials per non-empty active cell and sweep, >= 1
                           ("fixed independent of cell occupancy", Sec. II.B) */
    int32_t lattice;    /* MPMC_LATTICE_* start */
    double cell_min;    /* minimum cell width in sigma (>= 2, Sec. II.B) */
    double hist_dr;     /* contact histogram bin width (Sec. II.C.1: 1e-3) */
    uint32_t hist_bins; /* bins from r = 2 sigma (Sec. II.C.1: 100 -> 2.1) */
    uint32_t fit_order; /* polynomial order of the contact fit (Sec. II.C.1: 4) */
    uint32_t hist_block;/* configurations per block for the pressure standard
                           error; 0 = no blocking (se = NaN) */
    uint32_t schedule;  /* MPMC_SCHED_* (the trajectory does not depend on it) */
    uint32_t tile;      /* fused-kernel tile side in cells; 0 = autotune */
    void *stream;       /* hipStream_t for all work of the box */
    mpmc_alloc_fn alloc;/* optional device allocator (both or neither) */
    mpmc_free_fn free;
    void *alloc_ctx;
} mpmc_params;

typedef struct mpmc_info {
    uint32_t N, M, cap, n_trial, step_m, tile, schedule, hist_bins;
    int64_t W;          /* cell width in q units */
    double L;           /* nominal sqrt(N pi / eta) */
    double L_eff;       /* M w, the simulated box side */
    double w, eta, eta_eff, hist_dr;
    uint64_t sweep;     /* sweeps done */
    int64_t Sx, Sy;     /* accumulated grid shift, q units, mod M W */
    uint64_t trials, accepts; /* counted since creation */
    uint64_t n_conf;    /* configurations in the contact histogram */
} mpmc_info;

/* Fills *p with defaults: step_m 26 (d = 0.1015625), n_trial 1, triangular
 * start, cell_min 2, hist_dr 1e-3, hist_bins 100, fit_order 4, hist_block 0,
 * schedule AUTO, tile 0, stream NULL, no allocator.  MPMC_EINVAL if p NULL. */
int mpmc_default_params(mpmc_params *p);

/* Creates a box of N disks at packing fraction eta with Philox key `seed`.
 * Geometry: L = sqrt(N pi / eta); M = largest even integer <= L / cell_min
 * (>= 4 required); w = nearest multiple of q to L / M; the simulated box is
 * M w (eta_eff in mpmc_info).  p == NULL means defaults.  The lattice starts
 * need N a perfect square and place row b, column a at
 * X = floor((2a + 1 + [triangular and b odd]) M W / (2 sqrt N)) mod M W,
 * Y = floor((2b + 1) M W / (2 sqrt N)), tag b sqrt(N) + a.
 * Errors: MPMC_EINVAL (N == 0, eta outside (0, pi/4], M < 4, w + d >= 4,
 * non-square N with a lattice start, bad step or trial count),
 * MPMC_ENOMEM, MPMC_EDEVICE. */
int mpmc_init_box(mpmc_box *out, uint32_t N, double eta, uint64_t seed, const mpmc_params *p);

/* Releases all device memory of the box.  b == NULL is allowed. */
int mpmc_free_box(mpmc_box b);

/* Replaces the configuration: disk t (tag t) at absolute position
 * (X[t], Y[t]) in q units, 0 <= X, Y < M W (host arrays of N).  Resets the
 * accumulated shift.  MPMC_EOVERFLOW if a cell would exceed its capacity. */
int mpmc_set_positions(mpmc_box b, const int64_t *X, const int64_t *Y);

/* Changes the trial step (1..255); for tuning during equilibration only. */
int mpmc_set_step(mpmc_box b, uint32_t step_m);

/* Runs k sweeps (Sec. II.B).  Sweep s: (1) shift the cell grid by a random
 * multiple of q in [0, w)^2 and re-bin; (2) visit the four colour subsets in
 * a random order; in each, every non-empty cell makes n_trial trials.  The
 * Philox4x32-10 counter layout (seed; sweep, cell, trial, stream) makes the
 * result independent of launch shape.  Asynchronous unless trials or accepts
 * is non-NULL: then it synchronises and returns the counts of this call. */
int mpmc_sweep(mpmc_box b, uint64_t k, uint64_t *trials, uint64_t *accepts);

/* Adds the current configuration to the device contact histogram: unordered
 * pairs with 4 <= fp32 r^2 < fp32((2 + K dr)^2), bin k holding
 * fp32((2 + k dr)^2) <= r^2 < fp32((2 + (k+1) dr)^2) (Eq. (2) counting). */
int mpmc_accumulate_contacts(mpmc_box b);
int mpmc_reset_contacts(mpmc_box b);
/* Copies the K unordered counts and the number of configurations. */
int mpmc_get_contacts(mpmc_box b, int64_t *counts, uint64_t *n_conf);

/* Pressure from the accumulated histogram (Sec. II.C.1): g_k from Eq. (2)
 * with p = N(N-1)/2 pairs per configuration and r_k the bin centre; an
 * unweighted least-squares polynomial (fit_order) in r - 2 gives g(2+);
 * Z = 1 + 2 eta (N-1)/N g(2+) (Eq. (4) at finite N); P* = 4 eta Z / pi
 * (Eq. (1)).  *se is the standard error of P* over completed blocks of
 * hist_block configurations (NaN if fewer than 2).  Any output may be NULL.
 * MPMC_ESTATE if nothing was accumulated. */
int mpmc_measure_pressure(mpmc_box b, double *p_star, double *g_contact, double *z, double *se);

/* Diagnostic: ordered pair counts (i, j != i) of the current configuration
 * for the disks i with sel[tag] != 0 (host array of N), into counts[K]. */
int mpmc_contact_hist_subset(mpmc_box b, const uint8_t *sel, int64_t *counts);

/* Orientational order, Eq. (8): psi_j = (1/6) sum over the six nearest
 * neighbours (fp32 minimum-image r^2, ties to the lower tag) of
 * exp(6 i phi_jk), phi from the +x axis, evaluated as (z^2)^3 / |z|^6.
 * re/im: psi_j by tag (N floats each); field_re/field_im: per cell of the
 * current grid (M*M floats, cell i + M j), the mean psi_j over its 3 x 3
 * block; Psi: the global mean (Sec. III).  Array outputs are device pointers
 * when on_device != 0, else host; any output may be NULL.  MPMC_EINVAL if
 * N < 7 or the neighbourhood search would span the box. */
int mpmc_psi6_field(mpmc_box b, float *re, float *im, float *field_re, float *field_im,
                    double *Psi_re, double *Psi_im, int on_device);

/* Positional order, Sec. IV.C (S(q), q0, chi_j: Eqs. (10), (11)) and Sec. IV.D
 * (C_q0(r): Eq. (12)).  Wave vectors are those the periodic box
 * allows, q = (2 pi / L_eff)(h, k) with integers |h|, |k| < 4096 and
 * L_eff = M w.  Positions are the exact absolute ones in q units; each phase
 * (h X + k Y) / (M W) is formed in fp64 (structure factor) or reduced
 * exactly in integers (chi) before its sine and cosine. */

/* Structure factor S(q) = |sum_n exp(i q.x_n)|^2 / N (the double sum over
 * n, m of Sec. IV.C) at nq wave vectors: hk holds (h, k) pairs, S receives
 * nq values (host arrays).  Each term exp(i q.x) is an fp32 root of unity
 * from a 256-entry table, chosen by the fp64 phase, rotated by the residual
 * angle in fp32, and summed in fp64: every term carries an absolute error
 * below 1e-6, so |dS| <= 2e-6 sqrt(N S) + 1e-12 N.
 * MPMC_EINVAL for an index outside (-4096, 4096). */
int mpmc_structure_factor(mpmc_box b, const int32_t *hk, uint32_t nq, double *S);

/* mpmc_structure_factor for callers that cannot allocate device memory
 * (code under stream capture, serving loops, harnesses that forbid
 * hipMalloc): hk (2 nq int32) and S (nq doubles) are DEVICE pointers, the
 * work is enqueued on the box's stream and the call returns without waiting
 * for it.  The per-workgroup partial sums live in a fixed 4 MiB device array
 * of the library (one per device, held until the process ends) instead of
 * the box's work buffer, so nothing is allocated: at most 4096 wave vectors
 * per call (MPMC_EINVAL beyond).  A wave vector with an index outside
 * (-4096, 4096) gets S = NaN.  Every call on one device shares the array:
 * calls that may overlap on one device (different streams, or threads)
 * race and must be serialised by the caller.  The call reads the box's
 * device scalars to the host first (a synchronising copy, no allocation). */
int mpmc_structure_factor_noalloc(mpmc_box b, const int32_t *hk, uint32_t nq, double *S);

/* The first diffraction peak: of the allowed wave vectors q != 0 with
 * q_lo <= |q| <= q_hi and direction atan2(k, h) in [theta0, theta0 + dtheta)
 * modulo 2 pi (radians; dtheta >= 2 pi means every direction), the one with
 * the largest S (the first in the order k, then h ascending on ties).
 * Outputs may be NULL.  MPMC_EINVAL if the window is empty, q_hi reaches
 * the index limit or the annulus holds more than 2^24 wave vectors. */
int mpmc_find_q0(mpmc_box b, double q_lo, double q_hi, double theta0, double dtheta,
                 int32_t *h, int32_t *k, double *S);

/* Positional order parameter chi_j = exp(i q0.x_j), q0 = (2 pi / L_eff)(h, k),
 * by tag into re/im (N floats each, phase reduced exactly in integers and
 * evaluated in fp64); field_re/field_im: per cell of the current grid
 * (M*M floats, cell i + M j) the mean chi_j over its 3 x 3 block, the field
 * chi(x) drawn in Sec. IV.C.  Device pointers when on_device != 0, else
 * host; any output may be NULL. */
int mpmc_chi_field(mpmc_box b, int32_t h, int32_t k, float *re, float *im, float *field_re,
                   float *field_im, int on_device);

/* Positional correlation C_q(r) (Sec. IV.D) for any wave vector (qx, qy) in
 * 1/sigma, so that each configuration can use its own rotated q0: over the
 * unordered pairs whose minimum-image separation d (exact in q units)
 * satisfies r_b - 1 <= |d| <= r_b + 1 with r_b = b dr, b = 0..nbins-1 (the
 * lower edge clamped at 0), ADDS the sum of cos(q.d) (fp64) to num[b] and the
 * number of pairs to cnt[b] (host arrays), so that calls over several
 * configurations accumulate the configuration average; C_q(r_b) =
 * num[b] / cnt[b].  The window test is exact in 64-bit integers.
 * MPMC_EINVAL unless dr is a positive multiple of 2^-22, 1 <= nbins <= 4096
 * and (nbins - 1) dr + 1 < min(L_eff / 2, 512). */
int mpmc_cq(mpmc_box b, double qx, double qy, double dr, uint32_t nbins, double *num,
            int64_t *cnt);

/* mpmc_cq with the configuration turned to a reference orientation
 * (Sec. IV.D): the wave vector (qx, qy) is rotated by
 * angle = remainder(arg Psi_6 - psi_arg_ref, 2 pi) / 6, Psi_6 the current
 * global mean of Eq. (8), before the windows are accumulated; *angle (may be
 * NULL) receives it.  Calling it on successive configurations with the same
 * reference gives the coherent configuration average.  MPMC_EINVAL if
 * Psi_6 = 0 or for the arguments mpmc_cq rejects. */
int mpmc_cq_aligned(mpmc_box b, double qx, double qy, double psi_arg_ref, double dr,
                    uint32_t nbins, double *num, int64_t *cnt, double *angle);

/* Incoherent averaging (appendix on configuration averaging): out[g] = the
 * maximum of C[i] over the windows g*width <= i < min((g+1)*width, n), for
 * g < ceil(n / width); the caller averages these maxima over
 * configurations.  Host arrays; MPMC_EINVAL if n or width is 0. */
int mpmc_cq_bin_max(const double *C, uint32_t n, uint32_t width, double *out);

/* Equation-of-state loop (Sec. IV.A).  In a finite box P*(eta) near the
 * transition shows a Mayer-Wood loop; integrating it gives the interface free
 * energy per disk.  With v = pi / eta the area per disk (sigma the radius) and
 * beta P sigma^2 = P* / 4:
 *   - P*(v) is the least-squares polynomial of the given order (3..9) in
 *     v - mean(v), weighted by 1/se^2 when se != NULL (host arrays of n >=
 *     order + 2 points);
 *   - eta_max/p_max: its local maximum (the lower-density extremum), and
 *     eta_min/p_min: its local minimum, both inside the data range;
 *   - p_coex: the Maxwell pressure, equal areas of P* - p_coex between the
 *     outer roots of P* = p_coex, eta_liquid < eta_solid being those roots;
 *   - delta_f: beta Delta f, a quarter of the area between P* and p_coex from
 *     the solid root to the middle root (the free energy per disk above the
 *     common tangent at its largest).
 * MPMC_EINVAL for bad input; MPMC_ESTATE if the fit has no loop (not exactly
 * one maximum below the density of exactly one minimum) or the construction
 * would need data outside the range. */
typedef struct {
    double eta_max, p_max, eta_min, p_min;
    double p_coex, eta_liquid, eta_solid;
    double delta_f;
} mpmc_eos_loop_result;
int mpmc_eos_loop(const double *eta, const double *p_star, const double *se, uint32_t n,
                  uint32_t order, mpmc_eos_loop_result *out);

/* Finite-size scaling (Sec. IV.A): y = prefactor * x^exponent by least
 * squares on (ln x, ln y), e.g. Delta f against N, where -1/2 marks a
 * first-order transition in two dimensions and -1 a continuous one.  Either
 * output may be NULL; MPMC_EINVAL unless n >= 2, all values positive and the
 * x not all equal. */
int mpmc_power_law(const double *x, const double *y, uint32_t n, double *exponent,
                   double *prefactor);

/* Asynchronous measurement of the current configuration: adds it to the
 * contact histogram (as mpmc_accumulate_contacts) and evaluates psi_6 (as
 * mpmc_psi6_field: a 2-cell stencil, then the widest staged stencil, 3
 * cells, where the first fell short, decided on the device) on a
 * stream of the box's own, so that the kernels overlap the sweeps that
 * follow; nothing is copied to the host.  Psi (may be NULL): device pointer
 * to two doubles that receive the global Psi_6 (re, im) once the kernels
 * have run; field != 0 also refreshes the psi field (mpmc_psi6_field's
 * buffers).  The next sweeps wait for the measurement only before their last
 * sweep overwrites the state it reads; every other call on the box waits for
 * it on the box's stream.  A neighbour search too short even with the
 * widest stencil sets a flag that mpmc_measure_wait reports.  MPMC_EINVAL
 * with hist_block > 0 or where the staged kernels do not apply (cells of
 * more than 4 disks, M < 6); MPMC_ESTATE for a box of a batch. */
int mpmc_measure_async(mpmc_box b, double *Psi, int field);

/* Waits on the host for the asynchronous measurements of the box; *failed
 * (may be NULL) receives 1 if any of them since the last wait had a
 * neighbour search too short (its psi values are then not exact), else 0. */
int mpmc_measure_wait(mpmc_box b, uint32_t *failed);

/* Absolute positions by tag: (i w + u + S) mod L_eff in sigma (double) or
 * in q units (int64); either pair may be NULL. */
int mpmc_get_positions(mpmc_box b, double *x, double *y, int64_t *X, int64_t *Y);

/* Cell lists of the current grid in their canonical slot order: cnt[M*M],
 * tag/x/y[M*M*cap] (slot s of cell c at c*cap + s, unused slots 0).  The
 * order after each re-bin: disks of old cell (I, J) that stay, then those
 * of (I+1, J) wrapping in x, of (I, J+1) wrapping in y, of (I+1, J+1)
 * wrapping in both, each in old slot order. */
int mpmc_get_cells(mpmc_box b, uint8_t *cnt, uint32_t *tag, float *x, float *y);

int mpmc_get_info(mpmc_box b, mpmc_info *info);

/* Checks the state on the device: *n_overlaps = unordered pairs with
 * fp32 r^2 < 4 (3 x 3 cell stencil, exhaustive since w >= 2 sigma);
 * *n_bad = offsets outside [0, w) plus count, tag and capacity violations. */
int mpmc_validate(mpmc_box b, uint64_t *n_overlaps, uint64_t *n_bad);

/* Checkpoint: writes the cell lists, shift, sweep counter, counters, step,
 * seed and the contact histogram to `path`; mpmc_load creates a box from
 * it (p supplies stream, allocator and schedule; NULL = defaults).
 * Continuing a loaded box reproduces the uninterrupted run bit for bit. */
int mpmc_save(mpmc_box b, const char *path);
int mpmc_load(mpmc_box *out, const char *path, const mpmc_params *p);

/* Time-series analysis of Sec. III on host arrays.  mpmc_acf: C(dt) of
 * Eq. (9) for dt = 0..maxlag from a complex series of length n, the real
 * part of the mean over all time origins of Psi(t) Psi*(t+dt) over the mean
 * of |Psi|^2.  mpmc_tau: tau of the exponential tail, from least squares of
 * ln C over the first run of lags with lo <= C <= hi (MPMC_ESTATE if fewer
 * than 3 such lags), and the integrated time 1/2 + sum C up to the first
 * lag >= 6 tau_int (either output may be NULL). */
int mpmc_acf(const double *re, const double *im, uint32_t n, uint32_t maxlag, double *C);
int mpmc_tau(const double *C, uint32_t maxlag, double lo, double hi, double *tau,
             double *tau_int);

/* Sweep schedule of an existing box: MPMC_SCHED_SIMPLE, MPMC_SCHED_FUSED
 * with the given tile side and threads per workgroup (0 = default: 64 for
 * tile 8, 256 up to tile 34, 512 for 48, 1024 above), or MPMC_SCHED_AUTO
 * (autotune: time every fused shape that fits on this machine's state, keep the
 * fastest; cached per device, M and n_trial for the
 * process, and across processes in the text file named by the environment
 * variable MPMC_TUNE_CACHE if it is set: one line "<arch> <CUs> <M>
 * <n_trial> <tile> <threads>" per choice, read before tuning and appended
 * after; lines whose shape does not fit are ignored, and a file that cannot
 * be read or written only costs the tuning).  The state and the trajectory
 * are unaffected.  Shapes (tile, threads): (8, 64), (8, 128), (16, 128),
 * (16, 256), (24, 256), (32, 256), (32, 512), (34, 256), (48, 512),
 * (48, 1024), (56, 1024); the 34- and 48-cell ones keep two slots per cell
 * in LDS and slots 2 and 3 of fuller cells in a side table of 32 entries (a
 * region with more such cells runs as four-slot sub-tiles).  MPMC_EINVAL if
 * the shape is not one of these or does not fit (fused tiles need cells of
 * at most 4 slots and tile + 10 <= M). */
int mpmc_set_schedule(mpmc_box b, uint32_t schedule, uint32_t tile, uint32_t threads);

/* Phase profile of the fused sweep kernel: runs `sweeps` sweeps (the chain
 * advances exactly as with mpmc_sweep), each workgroup recording the device
 * realtime clock at its entry and at its phase boundaries, and returns in
 * phase_us[12]: [0..7] the mean duration per tile in microseconds of the
 * region load, colour passes 1-4 (in sweep order), the re-bin's class
 * counts, its scatter and the whole tile; [8] the mean time per tile from
 * the workgroup's entry to the start of its work (reading the sweep counter
 * and drawing the sweep's shift and colour order); per launch, averaged over
 * the sweeps: [9] the span from the first workgroup's entry to the last
 * one's end (us), [10] the mean number of tiles in flight over that span
 * (summed entry-to-end time / span), [11] the time from the first entry to
 * the last (us).  A two-slot tile that runs as four-slot sub-tiles books
 * their whole time under colour pass 1.  Allocates a stamp buffer for the
 * call.  MPMC_EINVAL unless the box runs the fused schedule. */
int mpmc_profile_phases(mpmc_box b, uint32_t sweeps, double *phase_us);

/* Long runs replay a captured HIP graph of this many sweeps (even, default
 * 128 fused / 32 simple); 0 launches every sweep directly.  Learned sweeps
 * (mpmc_sweep_learned) replay graphs of 8 sweeps while graphs are on (any
 * nonzero value) and launch every sweep directly when they are off; either
 * way the trajectory is the same. */
int mpmc_set_graphs(mpmc_box b, uint32_t sweeps_per_graph);

/* ---- batches of independent boxes ----------------------------------------
 * Many boxes of different N and eta swept together: every sweep of the
 * batch is one persistent kernel launch whose workgroups stride over a
 * (box, tile) work list, and runs of sweeps replay a captured HIP graph.
 * Box b evolves exactly as a single box created with N[b], eta[b], seed[b]
 * and the same params would (independent Philox keys and geometry).
 * Error bars from independent runs are how the paper quotes its pressures
 * (Table I); a batch of seeds provides them in one launch per sweep. */
typedef struct mpmc_batch_s *mpmc_batch;

/* Creates nbox boxes (1 <= nbox < 4096) from host arrays N, eta, seed and
 * common params (lattice start, step, trials, histogram; no allocator hook).
 * The fused tile shape is autotuned over the shapes that fit every box,
 * unless p->tile is set or p->schedule is MPMC_SCHED_SIMPLE. */
int mpmc_batch_create(mpmc_batch *out, uint32_t nbox, const uint32_t *N, const double *eta,
                      const uint64_t *seed, const mpmc_params *p);
int mpmc_batch_free(mpmc_batch b);
/* k sweeps of every box; counts (if non-NULL) are summed over boxes. */
int mpmc_batch_sweep(mpmc_batch b, uint64_t k, uint64_t *trials, uint64_t *accepts);
/* Borrowed handle of box i for the single-box read and measurement calls
 * (mpmc_get_*, mpmc_psi6_field, mpmc_accumulate_contacts, ...).  It must not
 * be swept or freed on its own (MPMC_ESTATE). */
int mpmc_batch_box(mpmc_batch b, uint32_t i, mpmc_box *out);
/* Contact histogram of every box; per-box P* and standard error (arrays of
 * nbox, either may be NULL), as mpmc_measure_pressure. */
int mpmc_batch_accumulate_contacts(mpmc_batch b);
int mpmc_batch_measure_pressure(mpmc_batch b, double *p_star, double *se);
/* Tile shape: (tile, threads) as for mpmc_set_schedule; (0, 0) autotunes;
 * (0, 1) runs each box with the simple per-colour kernels. */
int mpmc_batch_set_schedule(mpmc_batch b, uint32_t tile, uint32_t threads);
int mpmc_batch_info(mpmc_batch b, uint32_t *nbox, uint32_t *tile, uint32_t *threads,
                    uint32_t *n_items);
/* Sweeps per captured graph (even, > 0; default 64). */
int mpmc_batch_set_graphs(mpmc_batch b, uint32_t sweeps_per_graph);

/* ---- learned proposal ------------------------------------------------------
 * An extension of the uniform trial move of Sec. II.B: a small network maps
 * the moving disk's neighbourhood to a displacement density, and a
 * Metropolis-Hastings correction keeps every trial exact.
 *  features: the up to 12 nearest other disks within 3 sigma of the disk's
 *    position, as (dx, dy) pairs sorted by fp32 r^2 (ties: enumeration order
 *    over the 3 x 3 cell block, rows dj = -1..1 outer, columns inner, slots
 *    ascending), zero padded to 24 floats.
 *  network: 24 -> 64 -> 64 -> 20 with SiLU; parameters (7060 floats) in the
 *    order W1[64][24], b1[64], W2[64][64], b2[64], W3[20][64], b3[20];
 *    output k (0..3) = (logit, mu_x, mu_y, a_x, a_y) at 5k..5k+4, component
 *    width exp(clamp(a, -10, 1)); BF16 weights, FP32 accumulation.
 *  proposal: a mixture of the plain step (weight eps) and the network's
 *    Gaussian mixture, as a law on the q lattice (written out below at
 *    mpmc_learned_propose).
 *  acceptance: min(1, P(-D | f(x')) / P(D | f(x))) if x' stays in its cell
 *    and overlaps no disk.
 * Boxes swept with the learned proposal need cells of width >= 3 sigma
 * (mpmc_params.cell_min = 3): the 3 sigma neighbourhoods of x and x' then
 * lie in cells that no other thread moves during the colour sub-sweep. */
#define MPMC_MLP_PARAMS 7060
typedef struct mpmc_learner_s *mpmc_learner;

/* Creates a network with default weights (uniform +-1/sqrt(fan_in) from
 * Philox words of `seed`) and room for `capacity` recorded moves; stream is
 * a hipStream_t (NULL = default). */
int mpmc_learner_create(mpmc_learner *out, uint64_t seed, uint64_t capacity, void *stream);
int mpmc_learner_free(mpmc_learner l);
/* Host arrays of MPMC_MLP_PARAMS floats; setting resets the Adam state. */
int mpmc_learner_set_params(mpmc_learner l, const float *params);
int mpmc_learner_get_params(mpmc_learner l, float *params);
/* Runs `sweeps` plain sweeps of box b (cell_min >= 3; same trajectory as
 * mpmc_sweep) and records every accepted move as (features at the old
 * position, delta).  *n_total: moves recorded so far
 * (at most capacity). */
int mpmc_learner_collect(mpmc_learner l, mpmc_box b, uint64_t sweeps, uint64_t *n_total);
/* `steps` Adam steps (lr; beta 0.9/0.999, eps 1e-8) on minibatches of
 * `batch` moves drawn with replacement by Philox; loss = mean
 * -log q_GMM(delta | f), the continuous mixture density.
 * *mean_loss: the loss of the last minibatch. */
int mpmc_learner_train(mpmc_learner l, uint32_t steps, uint32_t batch, float lr, double *mean_loss);
/* Diagnostics on host arrays: network outputs out[B][20] for F[B][24];
 * the gradient (MPMC_MLP_PARAMS floats) and value of the mean loss over the
 * moves (F[B][24], D[B][2]). */
int mpmc_learner_forward(mpmc_learner l, const float *F, uint32_t B, float *out);
int mpmc_learner_nll_grad(mpmc_learner l, const float *F, const float *D, uint32_t B, float *grad,
                          double *loss);
/* Moves recorded, neighbourhoods seen with more than 12 disks within 3
 * sigma (impossible for valid configurations), training steps done. */
int mpmc_learner_info(mpmc_learner l, uint64_t *n_data, uint64_t *n_feature_overflow,
                      uint32_t *steps);
/* Features of the disks with the given tags at their current positions,
 * F[n][24] (host). */
int mpmc_learned_features(mpmc_box b, const uint32_t *tags, uint32_t n, float *F);
/* Active cells per wave of the learned colour pass: 16, 32 or 64, or 0
 * (the default) to choose from the box size: the smallest of 16 and 32 that
 * needs no more waves than the device has SIMDs, else 64 (a wave's network
 * work shrinks with its cells, and small boxes then use more SIMDs).  The
 * trajectory is the same for every value.  MPMC_EINVAL for other values. */
int mpmc_set_learned_cells_per_wave(mpmc_box b, uint32_t cells);
/* k sweeps with the learned proposal (eps in [0, 1] is the weight of the
 * uniform fallback); counts as mpmc_sweep. */
int mpmc_sweep_learned(mpmc_box b, mpmc_learner l, uint64_t k, float eps, uint64_t *trials,
                       uint64_t *accepts);

/* Phase profile of the learned colour pass: runs `sweeps` learned sweeps
 * (the chain advances as with mpmc_sweep_learned), lane 0 of every wave
 * recording the device realtime clock, and returns in phase_us[9] the mean
 * microseconds per wave and pass of: start-up (weights, neighbourhood,
 * random words), features at x, network at x, the draw and P(D), the
 * overlap test, features at x', network at x', the acceptance, and the
 * count.  Allocates a stamp buffer for the call. */
int mpmc_profile_learned(mpmc_box b, mpmc_learner l, uint32_t sweeps, float eps, double *phase_us);

/* The proposal as a law on the q lattice.  A trial proposes an integer
 * displacement D = (Dx, Dy) (delta = D q) with probability
 *   P(D) = e U(D) + (1 - e) G(D),  e = E / 2^32, E = nearest integer to
 *          eps 2^32 (the branch compares a 32-bit word with E);
 *   U(D): the plain trial's step, per axis D = step_m j with j odd,
 *         |j| <= 2^14 - 1, probability 2^-14 each;
 *   G(D): component k with probability pi_k, a point of N(mu_k,
 *         diag(s_k^2)) drawn in double precision from 53-bit uniforms and
 *         rounded to the nearest lattice point; a draw with |D| > 2^22 - 1
 *         on an axis fails (the trial is rejected).  A lattice point's
 *         probability is the Gaussian mass of its cell [D - 1/2, D + 1/2] q,
 *         per axis (q/s) phi(u)(1 + h^2 He2(u)/6 + h^4 He4(u)/120),
 *         u = (D q - mu)/s, h = q/(2 s).
 * Acceptance: min(1, P(-D | out(x')) / P(D | out(x))) against a 53-bit
 * uniform.  Random words of trial t in cell c, sweep k: stream 0 (disk,
 * uniform step as in the plain trial, branch), stream 2 (component and
 * acceptance uniforms), stream 4 (the Gaussian pair).  With eps = 1 the
 * learned sweep is the plain sweep, word for word.
 *
 * Diagnostics of that law on host arrays (they allocate device memory for
 * the call): mpmc_learned_propose draws n proposals from one fixed network
 * output out[20], draw i with the words of counter (sweep 0, cell i,
 * trial 0) under key seed, into D[2n] (0 where the draw failed), drawn[n]
 * and logp[n] = ln P(D) (NaN where the draw failed); mpmc_learned_logp gives
 * logp[i] = ln P(D_i | out_i) for out[n][20], D[n][2] (-inf below 1e-300).
 * MPMC_EINVAL for n = 0, step_m outside 1..255 or eps outside [0, 1]. */
int mpmc_learned_propose(const float *out, uint32_t step_m, float eps, uint64_t seed, uint32_t n,
                         int32_t *D, uint8_t *drawn, double *logp);
int mpmc_learned_logp(const float *out, const int32_t *D, uint32_t n, uint32_t step_m, float eps,
                      double *logp);
/* Diagnostics of the learner: recorded moves first..first+n-1 into host
 * arrays F[n][24], D[n][2] (recording order follows the device's atomic
 * counter; MPMC_EINVAL beyond the moves recorded); one Adam step with the
 * given gradient (MPMC_MLP_PARAMS floats) and learning rate. */
int mpmc_learner_moves(mpmc_learner l, uint64_t first, uint64_t n, float *F, float *D);
int mpmc_learner_adam_step(mpmc_learner l, const float *grad, float lr);

/* Message of the last failing call on this thread ("" if none). */
const char *mpmc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
