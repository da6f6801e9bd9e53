/*
 * orc.h — plain single-threaded CPU oracle for the massively parallel local
 * Monte Carlo (MPMC) hard-disk sampler of Engel et al., "Hard-disk equation
 * of state" (Phys. Rev. E 87, 042134; arXiv:1211.1645).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source with the HIP path: the two
 * sides agree because both implement the same written definitions (counter
 * layout, dyadic coordinate lattice, rebin order, overlap predicate), not
 * because they share code.
 *
 * Precision: the sampler itself is carried out in fp32 on the dyadic lattice
 * of spacing q = 2^-22 sigma, where every coordinate addition is exact (the
 * paper's MPMC runs in single precision with cell-local coordinates,
 * Sec. II.B); observables (g(r) normalisation, fit, psi_6 values, ACF) are
 * evaluated in fp64.
 */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_box orc_box;

/* Geometry of Sec. II.A with the cell grid of Sec. II.B.
 * L = sqrt(N*pi/eta) (sigma = 1); M = largest even integer <= L/cell_min;
 * W = nearest integer to L/(M q); w = W q.  Returns 0, or -1 when M < 4,
 * N == 0 or eta outside (0, pi/4].  cap = most disks a w x w cell can hold. */
int orc_geometry(uint32_t N, double eta, double cell_min, double *L, uint32_t *M,
                 int64_t *W, uint32_t *cap);

/* Creates a box with a lattice start (lattice 0 = square, 1 = row-offset
 * triangular stacking, 2 = empty until orc_set_positions_q), step d = step_m * 2^-8 sigma, n_trial trials per
 * non-empty active cell.  Returns NULL on invalid parameters. */
orc_box *orc_create(uint32_t N, double eta, uint64_t seed, double cell_min,
                    int lattice, uint32_t step_m, uint32_t n_trial);
void orc_free(orc_box *b);
orc_box *orc_clone(const orc_box *b);

/* Replaces the configuration with the given absolute positions in q units
 * (0 <= X, Y < M W), tags 0..N-1 in argument order.  Returns 0, or -1 if a
 * cell would exceed its capacity. */
int orc_set_positions_q(orc_box *b, const int64_t *X, const int64_t *Y);

void orc_set_step(orc_box *b, uint32_t step_m);

/* Runs k sweeps (shift + rebin, then the four colour sub-sweeps in random
 * order).  cell_order: 0 = row-major, 1 = reversed, 2 = column-major; the
 * result does not depend on it (same-colour cells are independent). */
void orc_sweep(orc_box *b, uint64_t k, int cell_order);

/* Info: L_eff = M w, eta_eff, w, M, W, cap, sweep counter, shift S (q). */
void orc_info(const orc_box *b, double *L_eff, double *eta_eff, double *w, uint32_t *M,
              int64_t *W, uint32_t *cap, uint64_t *sweep, int64_t *Sx, int64_t *Sy,
              uint64_t *trials, uint64_t *accepts);

/* Cell lists in the canonical slot order: cnt[M*M], tag/x/y[M*M*cap]
 * (slot s of cell c at c*cap + s; unused slots are written as 0). */
void orc_get_cells(const orc_box *b, uint8_t *cnt, uint32_t *tag, float *x, float *y);
/* Absolute positions (q units, in [0, M W)) indexed by tag. */
void orc_get_positions_q(const orc_box *b, int64_t *X, int64_t *Y);

/* Number of unordered pairs violating the fp32 overlap predicate (all pairs). */
uint64_t orc_count_overlaps(const orc_box *b);

/* Squared bin edges E_k = fp32(e_k^2), e_k = 2 + k dr, k = 0..K. */
void orc_hist_edges(uint32_t K, double dr, float *E);
/* Unordered contact-pair histogram of the current configuration, all pairs,
 * minimum image (Eq. (2) counting).  counts[K] is ADDED to. */
void orc_pair_hist(const orc_box *b, uint32_t K, double dr, int64_t *counts);
/* Ordered pair counts (i, j != i) for the disks whose tag has sel[tag] != 0. */
void orc_pair_hist_subset(const orc_box *b, const uint8_t *sel, uint32_t K, double dr,
                          int64_t *counts);

/* Contact value by an unweighted least-squares polynomial fit of g(r) over
 * the bins (Sec. II.C.1), then Z from Eq. (4) in its finite-N form and
 * P* = 4 eta Z / pi (Eq. (1)).  Returns 0 or -1 (no counts / singular). */
int orc_pressure(const int64_t *counts, uint32_t K, double dr, uint32_t order,
                 uint64_t n_conf, uint32_t N, double L_eff, double *g_contact, double *Z,
                 double *P_star, double *coef);

/* psi_j of Eq. (8) for the disks with sel[tag] != 0 (sel == NULL: all), by
 * brute-force six nearest neighbours (fp32 squared distance, ties to the
 * lower tag).  Results by tag; unselected entries untouched. */
void orc_psi6(const orc_box *b, const uint8_t *sel, double *re, double *im);
/* Coarse field: mean psi_j over the 3 x 3 cell block around every cell. */
void orc_psi6_field(const orc_box *b, const double *re, const double *im, double *fre,
                    double *fim);

/* C(dt) of Eq. (9), dt = 0..maxlag, from a complex series of length n. */
/* Positional order (Sec. IV.C).  Structure factor
 * S(q) = |sum_n exp(i q.x_n)|^2 / N at the wave vectors the periodic box
 * allows, q = (2 pi / L_eff)(h, k); the phase (h X + k Y) mod Lq is reduced
 * exactly in integers (X, Y absolute positions in q units).  hk holds nq
 * (h, k) pairs. */
void orc_structure_factor(const orc_box *b, const int32_t *hk, uint32_t nq, double *S);

/* chi_j = exp(i q0.x_j) with q0 = (2 pi / L_eff)(h, k), by tag. */
void orc_chi(const orc_box *b, int32_t h, int32_t k, double *re, double *im);

/* Positional correlation (Sec. IV.D, Eq. (12))
 * C_q(r) = <exp(i q.(x_n - x_m))> over the unordered
 * pairs with minimum-image separation |x_n - x_m| in [r - 1, r + 1] (sigma = 1),
 * at r_b = b dr, b = 0..B-1.  Adds sum cos(q.d) to num[b] and the pair count
 * to cnt[b] (the sine parts cancel between (n, m) and (m, n)).  dr must be a
 * multiple of 2^-22 and (B - 1) dr + 1 < min(L_eff / 2, 512); the window
 * test is exact in integers.  Returns 0, or -1 if the bins are out of range. */
int orc_cq(const orc_box *b, double qx, double qy, double dr, uint32_t B, double *num,
           int64_t *cnt);

void orc_acf(const double *re, const double *im, uint32_t n, uint32_t maxlag, double *C);
/* Exponential-tail fit: tau from least squares of ln C over the first run of
 * lags with lo <= C <= hi.  Returns tau, or -1 when fewer than 3 points. */
double orc_tau_fit(const double *C, uint32_t maxlag, double lo, double hi);
/* Integrated time 1/2 + sum_{dt=1}^{W} Re C(dt), W the first lag >= c*tau_int. */
double orc_tau_int(const double *C, uint32_t maxlag, double c);

/* Philox4x32-10 (Salmon et al., SC'11): out = bijection(key, ctr). */
void orc_philox(uint32_t k0, uint32_t k1, const uint32_t ctr[4], uint32_t out[4]);

/* ---- learned proposal (MLP + Gaussian mixture), fp64 reference ---- */
/* Parameter vector layout (7060 doubles): W1[64][24], b1[64], W2[64][64],
 * b2[64], W3[20][64], b3[20]. */
enum { ORC_NF = 24, ORC_NH = 64, ORC_NO = 20, ORC_NK = 4, ORC_NPARAM = 7060 };
/* Features of a disk placed at cell-local (x, y) in cell c, all other disks
 * frozen, the disk with tag `self` excluded: the up to 12 nearest neighbours
 * within 3 sigma, (dx, dy) each, sorted by (fp32 r^2, enumeration order),
 * zero-padded.  Returns the number found (<= 12). */
int orc_features(const orc_box *b, uint32_t cell, uint32_t self, float x, float y, float *f);
/* MLP forward: out[20] from features f[24]. */
void orc_mlp_forward(const double *p, const double *f, double *out);
/* log q_GMM(delta | out) of the 4-component diagonal mixture. */
double orc_gmm_logpdf(const double *out, double dx, double dy);
/* Mean negative log-likelihood over a batch and its gradient wrt params. */
double orc_nll_grad(const double *p, const double *F, const double *D, uint32_t B,
                    double *grad);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8), t >= 1. */
void orc_adam(double *p, double *m, double *v, const double *g, uint32_t n, double lr,
              uint32_t t);

/* The learned proposal as a law on the q lattice (the definition is written
 * out above orc_learned_logp in orc.c): ln P(D | out) for the network output
 * out[20], uniform-branch weight eps and plain step step_m. */
double orc_learned_logp(const double *out, int64_t Dx, int64_t Dy, uint32_t step_m, float eps);
/* n proposals from the fixed output out[20], draw i using the words of
 * counter (sweep 0, cell i, trial 0) under key seed: D[2n] (0 where the
 * Gaussian draw failed), drawn[n] (may be NULL) and ln P(D) (NaN where the
 * draw failed; may be NULL). */
void orc_learned_proposals(const double *out, uint32_t step_m, float eps, uint64_t seed,
                           uint32_t n, int64_t *D, uint8_t *drawn, double *logp);
/* k sweeps whose trials use the learned proposal with the fp64 network
 * params[7060] and the Metropolis-Hastings acceptance. */
void orc_sweep_learned(orc_box *b, const double *params, float eps, uint64_t k);
/* k plain sweeps (cell order 0) that record every accepted move as the
 * features at the old position, F[24], and the displacement, D[2]; the
 * first cap moves are stored.  Returns the number of accepted moves. */
uint64_t orc_sweep_collect(orc_box *b, uint64_t k, float *F, float *D, uint64_t cap);

#ifdef __cplusplus
}
#endif
#endif
