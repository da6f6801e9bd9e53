/*
 * orc.c — plain single-threaded CPU oracle for the MPMC hard-disk sampler.
 *
 * TEST INFRASTRUCTURE ONLY (see orc.h).  Written for readability against the
 * paper (Engel et al., arXiv:1211.1645), not for speed: every step follows
 * the order of the method's description, with no blocking or fusion.
 *
 * Conventions written down once and followed literally here (the GPU library
 * implements the same conventions in its own code):
 *   sigma = 1; q = 2^-22; cell-local fp32 offsets are multiples of q in
 *   [0, w); w = W q with W an integer.
 *   Philox4x32-10 key = (seed_lo, seed_hi); counter =
 *     (sweep_lo, cell, trial, (sweep_hi << 8) | stream).
 *   stream 0: trial words (select, dx, dy, spare); stream 1: in-cell shuffle;
 *   stream 2: learned-proposal words; stream 3 with cell = 0xFFFFFFFF:
 *   per-sweep global words (shift x, shift y, colour permutation).
 *   Rebin order of a new cell (I, J): disks of old (I, J) that do not wrap,
 *   then old (I+1, J) wrapping in x only, old (I, J+1) wrapping in y only,
 *   old (I+1, J+1) wrapping in both, each in old slot order.
 *   Overlap: fp32 fl(fl(dx*dx) + fl(dy*dy)) < 4 with exact dx, dy.
 */
#include "orc.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define Q_SHIFT 22
#define QF ((float)(1.0 / 4194304.0))  /* q = 2^-22 */
#define QD (1.0 / 4194304.0)
#define GLOBAL_CELL 0xFFFFFFFFu

struct orc_box {
    uint32_t N;
    double eta;
    uint64_t seed;
    double cell_min;
    uint32_t step_m, n_trial;
    double L;       /* nominal L from (N, eta) */
    uint32_t M;     /* cells per side (even, >= 4) */
    int64_t W;      /* w in q units */
    float w;        /* w as fp32 (exact) */
    int64_t Lq;     /* M W */
    uint32_t cap;   /* slots per cell */
    uint8_t *cnt;
    uint32_t *tag;
    float *x, *y;
    int64_t Sx, Sy; /* accumulated grid shift, q units, mod Lq */
    uint64_t sweep;
    uint64_t trials, accepts;
};

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from the definition in Salmon, Moraes, Dror, Shaw, "Parallel
 * random numbers: as easy as 1, 2, 3" (SC'11): ten rounds of
 * (L0,R0,L1,R1) -> (hi(M1 R1) ^ L0' ^ k0, lo(M1 R1), hi(M0 R0) ^ L1' ^ k1,
 * lo(M0 R0)) on the word order (R0, L0, R1, L1) = (x0, x1, x2, x3), with the
 * Weyl key schedule k += (0x9E3779B9, 0xBB67AE85) between rounds. */
void orc_philox(uint32_t k0, uint32_t k1, const uint32_t ctr[4], uint32_t out[4]) {
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        x0 = n0; x1 = n1; x2 = n2; x3 = n3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void draw(const orc_box *b, uint64_t sweep, uint32_t cell, uint32_t t, uint32_t stream,
                 uint32_t w[4]) {
    uint32_t ctr[4] = {(uint32_t)sweep, cell, t, (uint32_t)((sweep >> 32) << 8) | stream};
    orc_philox((uint32_t)b->seed, (uint32_t)(b->seed >> 32), ctr, w);
}

/* floor(a * n / 2^32): an integer in [0, n) from a uniform 32-bit word. */
static uint32_t mulhi(uint32_t a, uint32_t n) { return (uint32_t)(((uint64_t)a * n) >> 32); }

/* ------------------------------------------------------------------------ */
/* Geometry, Sec. II.A (eta = N pi sigma^2 / L^2) and Sec. II.B (cells of
 * width w >~ 2 sigma, four colours, hence an even number of cells per side). */
static uint32_t capacity_for(double w) {
    /* Most points with pairwise distance >= 2 in a half-open w x w square:
     * k points fit only when w reaches 2 / d_k, d_k the largest minimum
     * distance of k points in the unit square (d_5 = sqrt(2)/2,
     * d_6 = 0.6009, d_7 = 0.5359, d_8 = 0.5176, d_9 = 0.5). */
    if (w < 2.0 * sqrt(2.0)) return 4;
    if (w < 2.0 / 0.6009) return 5;
    if (w < 2.0 / 0.5359) return 6;
    if (w < 2.0 / 0.5176) return 7;
    return 8;
}

int orc_geometry(uint32_t N, double eta, double cell_min, double *L, uint32_t *M,
                 int64_t *W, uint32_t *cap) {
    if (N == 0 || !(eta > 0.0) || eta > M_PI / 4.0 || !(cell_min >= 2.0)) return -1;
    double l = sqrt((double)N * M_PI / eta);
    uint32_t m = 2u * (uint32_t)floor(l / (2.0 * cell_min));
    if (m < 4) return -1;
    int64_t w = llround(l / ((double)m * QD));
    if (L) *L = l;
    if (M) *M = m;
    if (W) *W = w;
    if (cap) *cap = capacity_for((double)w * QD);
    return 0;
}

static orc_box *alloc_box(uint32_t N, double eta, uint64_t seed, double cell_min,
                          uint32_t step_m, uint32_t n_trial) {
    double L;
    uint32_t M, cap;
    int64_t W;
    if (orc_geometry(N, eta, cell_min, &L, &M, &W, &cap) != 0) return NULL;
    if (step_m == 0 || step_m > 255 || n_trial == 0) return NULL;
    /* every sum of an offset and a displacement must stay below 4 so that it
     * is exact on the q lattice in fp32 */
    if ((double)W * QD + step_m / 256.0 >= 4.0) return NULL;
    orc_box *b = (orc_box *)calloc(1, sizeof(orc_box));
    b->N = N; b->eta = eta; b->seed = seed; b->cell_min = cell_min;
    b->step_m = step_m; b->n_trial = n_trial;
    b->L = L; b->M = M; b->W = W; b->w = (float)((double)W * QD);
    b->Lq = (int64_t)M * W; b->cap = cap;
    size_t nc = (size_t)M * M;
    b->cnt = (uint8_t *)calloc(nc, 1);
    b->tag = (uint32_t *)calloc(nc * cap, sizeof(uint32_t));
    b->x = (float *)calloc(nc * cap, sizeof(float));
    b->y = (float *)calloc(nc * cap, sizeof(float));
    return b;
}

void orc_free(orc_box *b) {
    if (!b) return;
    free(b->cnt); free(b->tag); free(b->x); free(b->y); free(b);
}

orc_box *orc_clone(const orc_box *b) {
    orc_box *c = (orc_box *)malloc(sizeof(orc_box));
    *c = *b;
    size_t nc = (size_t)b->M * b->M;
    c->cnt = (uint8_t *)malloc(nc);
    c->tag = (uint32_t *)malloc(nc * b->cap * sizeof(uint32_t));
    c->x = (float *)malloc(nc * b->cap * sizeof(float));
    c->y = (float *)malloc(nc * b->cap * sizeof(float));
    memcpy(c->cnt, b->cnt, nc);
    memcpy(c->tag, b->tag, nc * b->cap * sizeof(uint32_t));
    memcpy(c->x, b->x, nc * b->cap * sizeof(float));
    memcpy(c->y, b->y, nc * b->cap * sizeof(float));
    return c;
}

/* Places disk `tag` at absolute q position (X, Y) (frame of the current
 * grid, i.e. S = 0), appending to its cell. */
static int place(orc_box *b, uint32_t tag, int64_t X, int64_t Y) {
    int64_t i = X / b->W, j = Y / b->W;
    uint32_t c = (uint32_t)(i + (int64_t)b->M * j);
    if (b->cnt[c] >= b->cap) return -1;
    uint32_t s = c * b->cap + b->cnt[c]++;
    b->tag[s] = tag;
    b->x[s] = (float)((double)(X - i * b->W) * QD);
    b->y[s] = (float)((double)(Y - j * b->W) * QD);
    return 0;
}

int orc_set_positions_q(orc_box *b, const int64_t *X, const int64_t *Y) {
    memset(b->cnt, 0, (size_t)b->M * b->M);
    b->Sx = b->Sy = 0;
    for (uint32_t t = 0; t < b->N; ++t) {
        int64_t xx = ((X[t] % b->Lq) + b->Lq) % b->Lq;
        int64_t yy = ((Y[t] % b->Lq) + b->Lq) % b->Lq;
        if (place(b, t, xx, yy) != 0) return -1;
    }
    return 0;
}

/* Lattice start.  With n = sqrt(N) and the box side Lq = M W in q units:
 * row b, column a sits at X = floor((2a + 1 + (b mod 2)) Lq / (2n)) mod Lq
 * (row offset only for the triangular stacking), Y = floor((2b + 1) Lq / (2n));
 * tag = b n + a.  Disks are appended to their cells in tag order. */
orc_box *orc_create(uint32_t N, double eta, uint64_t seed, double cell_min, int lattice,
                    uint32_t step_m, uint32_t n_trial) {
    uint32_t n = (uint32_t)llround(sqrt((double)N));
    if (lattice == 2) /* no lattice: positions come from orc_set_positions_q */
        return alloc_box(N, eta, seed, cell_min, step_m, n_trial);
    if ((uint64_t)n * n != N || (lattice != 0 && lattice != 1)) return NULL;
    orc_box *b = alloc_box(N, eta, seed, cell_min, step_m, n_trial);
    if (!b) return NULL;
    for (uint32_t r = 0; r < n; ++r)
        for (uint32_t a = 0; a < n; ++a) {
            int64_t off = (lattice == 1) ? (int64_t)(r & 1u) : 0;
            int64_t X = ((2 * (int64_t)a + 1 + off) * b->Lq) / (2 * (int64_t)n);
            int64_t Y = ((2 * (int64_t)r + 1) * b->Lq) / (2 * (int64_t)n);
            X %= b->Lq;
            if (place(b, r * n + a, X, Y) != 0) { orc_free(b); return NULL; }
        }
    return b;
}

void orc_set_step(orc_box *b, uint32_t step_m) { b->step_m = step_m; }

void orc_info(const orc_box *b, double *L_eff, double *eta_eff, double *w, uint32_t *M,
              int64_t *W, uint32_t *cap, uint64_t *sweep, int64_t *Sx, int64_t *Sy,
              uint64_t *trials, uint64_t *accepts) {
    double le = (double)b->Lq * QD;
    if (L_eff) *L_eff = le;
    if (eta_eff) *eta_eff = (double)b->N * M_PI / (le * le);
    if (w) *w = (double)b->w;
    if (M) *M = b->M;
    if (W) *W = b->W;
    if (cap) *cap = b->cap;
    if (sweep) *sweep = b->sweep;
    if (Sx) *Sx = b->Sx;
    if (Sy) *Sy = b->Sy;
    if (trials) *trials = b->trials;
    if (accepts) *accepts = b->accepts;
}

void orc_get_cells(const orc_box *b, uint8_t *cnt, uint32_t *tag, float *x, float *y) {
    size_t nc = (size_t)b->M * b->M;
    for (size_t c = 0; c < nc; ++c) {
        if (cnt) cnt[c] = b->cnt[c];
        for (uint32_t s = 0; s < b->cap; ++s) {
            size_t k = c * b->cap + s;
            int used = s < b->cnt[c];
            if (tag) tag[k] = used ? b->tag[k] : 0;
            if (x) x[k] = used ? b->x[k] : 0.0f;
            if (y) y[k] = used ? b->y[k] : 0.0f;
        }
    }
}

/* Absolute position (q units) of the disk in slot k of cell c:
 * (i W + U + S) mod (M W), with U = x / q exactly. */
static void abs_q(const orc_box *b, uint32_t c, uint32_t k, int64_t *X, int64_t *Y) {
    int64_t i = c % b->M, j = c / b->M;
    int64_t U = (int64_t)ldexp((double)b->x[k], Q_SHIFT);
    int64_t V = (int64_t)ldexp((double)b->y[k], Q_SHIFT);
    *X = (i * b->W + U + b->Sx) % b->Lq;
    *Y = (j * b->W + V + b->Sy) % b->Lq;
}

void orc_get_positions_q(const orc_box *b, int64_t *X, int64_t *Y) {
    for (uint32_t c = 0; c < b->M * b->M; ++c)
        for (uint32_t s = 0; s < b->cnt[c]; ++s) {
            uint32_t k = c * b->cap + s;
            abs_q(b, c, k, &X[b->tag[k]], &Y[b->tag[k]]);
        }
}

/* ------------------------------------------------------------------------ */
/* One sweep, Sec. II.B: the cell grid is shifted at random (here as a
 * translation of all disks by -s, the shift being recorded in S), then the
 * four checkerboard subsets are visited in a random order; within each
 * active cell a fixed number of trials is made on disks chosen in shuffled
 * order, rejecting moves that leave the cell or overlap another disk. */

static void rebin(orc_box *b, uint32_t sx, uint32_t sy) {
    uint32_t M = b->M, cap = b->cap;
    size_t nc = (size_t)M * M;
    uint8_t *ncnt = (uint8_t *)calloc(nc, 1);
    uint32_t *ntag = (uint32_t *)calloc(nc * cap, sizeof(uint32_t));
    float *nx = (float *)calloc(nc * cap, sizeof(float));
    float *ny = (float *)calloc(nc * cap, sizeof(float));
    float fsx = (float)((double)sx * QD), fsy = (float)((double)sy * QD);
    for (uint32_t J = 0; J < M; ++J)
        for (uint32_t I = 0; I < M; ++I) {
            uint32_t dst = I + M * J;
            /* sources in the fixed rebin order: (di, dj) = wrap flags */
            static const int src_d[4][2] = {{0, 0}, {1, 0}, {0, 1}, {1, 1}};
            for (int sidx = 0; sidx < 4; ++sidx) {
                int di = src_d[sidx][0], dj = src_d[sidx][1];
                uint32_t src = ((I + di) % M) + M * ((J + dj) % M);
                for (uint32_t s = 0; s < b->cnt[src]; ++s) {
                    uint32_t k = src * cap + s;
                    float u = b->x[k] - fsx, v = b->y[k] - fsy;  /* exact */
                    int wx = u < 0.0f, wy = v < 0.0f;
                    if (wx != di || wy != dj) continue;
                    if (wx) u = u + b->w;  /* exact */
                    if (wy) v = v + b->w;
                    uint32_t o = dst * cap + ncnt[dst]++;
                    ntag[o] = b->tag[k];
                    nx[o] = u;
                    ny[o] = v;
                }
            }
        }
    free(b->cnt); free(b->tag); free(b->x); free(b->y);
    b->cnt = ncnt; b->tag = ntag; b->x = nx; b->y = ny;
    b->Sx = (b->Sx + sx) % b->Lq;
    b->Sy = (b->Sy + sy) % b->Lq;
}

/* Overlap predicate for a pair with exact separation (dx, dy): hard disks of
 * radius 1 overlap when the centre distance is below 2 (Sec. II.A). */
static int overlaps(float dx, float dy) {
    volatile float a = dx * dx;  /* volatile: keep the three roundings */
    volatile float c = dy * dy;
    float r2 = a + c;
    return r2 < 4.0f;
}

/* The shuffled order of a cell's slots for several trials (Sec. II.B):
 * Fisher-Yates, for i = n-1 down to 1 swap slot i with slot
 * floor(word * (i+1) / 2^32); word e = n-1-i of stream 1, call index e / 4
 * in the trial field. */
static void shuffle_slots(const orc_box *b, uint32_t cell, uint32_t n, uint32_t perm[8]) {
    for (uint32_t s = 0; s < n; ++s) perm[s] = s;
    uint32_t wds[4];
    uint32_t have = 0xFFFFFFFFu;
    for (uint32_t i = n - 1; i >= 1; --i) {
        uint32_t e = n - 1 - i;
        if (e / 4 != have) { draw(b, b->sweep, cell, e / 4, 1, wds); have = e / 4; }
        uint32_t j = mulhi(wds[e % 4], i + 1);
        uint32_t tmp = perm[i]; perm[i] = perm[j]; perm[j] = tmp;
    }
}

/* Accepted moves recorded by the collecting sweep: features at the old
 * position and the displacement. */
typedef struct {
    float *F, *D;
    uint64_t cap, n;
} recorder;

/* Any other disk of the 3 x 3 block overlapping the disk of slot `slot` of
 * cell (ci, cj) placed at cell-local (xn, yn) (Sec. II.A, Sec. II.B: the
 * neighbour cells hold every disk within reach since w >= 2). */
static int overlaps_block(const orc_box *b, uint32_t ci, uint32_t cj, uint32_t slot, float xn,
                          float yn) {
    uint32_t M = b->M, cell = ci + M * cj;
    for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di) {
            uint32_t nb = ((ci + M + di) % M) + M * ((cj + M + dj) % M);
            float cwx = (float)di * b->w, cwy = (float)dj * b->w;
            for (uint32_t s = 0; s < b->cnt[nb]; ++s) {
                if (nb == cell && s == slot) continue;
                uint32_t kk = nb * b->cap + s;
                float ddx = (b->x[kk] - xn) + cwx;
                float ddy = (b->y[kk] - yn) + cwy;
                if (overlaps(ddx, ddy)) return 1;
            }
        }
    return 0;
}

static void trial_cell(orc_box *b, uint32_t ci, uint32_t cj, void *ctx) {
    recorder *rec = (recorder *)ctx;
    uint32_t M = b->M, cap = b->cap;
    uint32_t cell = ci + M * cj;
    uint32_t n = b->cnt[cell];
    if (n == 0) return;
    uint32_t perm[8];
    if (b->n_trial > 1) shuffle_slots(b, cell, n, perm);
    for (uint32_t t = 0; t < b->n_trial; ++t) {
        uint32_t w4[4];
        draw(b, b->sweep, cell, t, 0, w4);
        uint32_t slot = (b->n_trial == 1) ? mulhi(w4[0], n) : perm[t % n];
        int32_t jx = 2 * (int32_t)(w4[1] >> 18) + 1 - 16384;
        int32_t jy = 2 * (int32_t)(w4[2] >> 18) + 1 - 16384;
        float dx = (float)((int32_t)b->step_m * jx) * QF;
        float dy = (float)((int32_t)b->step_m * jy) * QF;
        uint32_t k = cell * cap + slot;
        float xn = b->x[k] + dx, yn = b->y[k] + dy;  /* exact */
        b->trials++;
        if (!(xn >= 0.0f && xn < b->w && yn >= 0.0f && yn < b->w)) continue;
        if (overlaps_block(b, ci, cj, slot, xn, yn)) continue;
        if (rec) {
            if (rec->n < rec->cap) {
                orc_features(b, cell, b->tag[k], b->x[k], b->y[k], rec->F + rec->n * 24);
                rec->D[2 * rec->n] = dx;
                rec->D[2 * rec->n + 1] = dy;
            }
            rec->n++;
        }
        b->x[k] = xn;
        b->y[k] = yn;
        b->accepts++;
    }
}

/* colour of cell (i, j): bit 0 = i mod 2, bit 1 = j mod 2 */
static void colour_order(uint32_t p, int order[4]) {
    int avail[4] = {0, 1, 2, 3};
    int navail = 4;
    uint32_t digits[3] = {p / 6, (p % 6) / 2, p % 2};
    for (int d = 0; d < 3; ++d) {
        order[d] = avail[digits[d]];
        for (int e = (int)digits[d]; e < navail - 1; ++e) avail[e] = avail[e + 1];
        --navail;
    }
    order[3] = avail[0];
}

typedef void (*cell_fn)(orc_box *b, uint32_t ci, uint32_t cj, void *ctx);

/* k sweeps, each cell of a colour running `trials` (the plain trial, the
 * learned trial or the recording plain trial). */
static void sweeps_with(orc_box *b, uint64_t k, int cell_order, cell_fn trials, void *ctx) {
    uint32_t M = b->M;
    for (uint64_t it = 0; it < k; ++it) {
        uint32_t g[4];
        draw(b, b->sweep, GLOBAL_CELL, 0, 3, g);
        uint32_t sx = mulhi(g[0], (uint32_t)b->W);
        uint32_t sy = mulhi(g[1], (uint32_t)b->W);
        int order[4];
        colour_order(mulhi(g[2], 24), order);
        rebin(b, sx, sy);
        for (int p = 0; p < 4; ++p) {
            uint32_t cx = (uint32_t)order[p] & 1u, cy = ((uint32_t)order[p] >> 1) & 1u;
            uint32_t h = M / 2;
            for (uint32_t a = 0; a < h; ++a)
                for (uint32_t bb = 0; bb < h; ++bb) {
                    uint32_t ai = a, bi = bb;
                    if (cell_order == 1) { ai = h - 1 - a; bi = h - 1 - bb; }
                    uint32_t ci, cj;
                    if (cell_order == 2) { ci = 2 * ai + cx; cj = 2 * bi + cy; }
                    else { ci = 2 * bi + cx; cj = 2 * ai + cy; }
                    trials(b, ci, cj, ctx);
                }
        }
        b->sweep++;
    }
}

void orc_sweep(orc_box *b, uint64_t k, int cell_order) {
    sweeps_with(b, k, cell_order, trial_cell, NULL);
}

uint64_t orc_sweep_collect(orc_box *b, uint64_t k, float *F, float *D, uint64_t cap) {
    recorder rec = {F, D, cap, 0};
    sweeps_with(b, k, 0, trial_cell, &rec);
    return rec.n;
}

/* ------------------------------------------------------------------------ */
/* Brute-force checks and observables over absolute q positions. */

static int64_t min_image(int64_t d, int64_t Lq) {
    d %= Lq;
    if (d < 0) d += Lq;
    if (2 * d > Lq) d -= Lq;
    return d;
}

/* fp32 squared distance of the minimum-image separation: the separation is
 * exact in q units and rounded once to fp32. */
static float r2_f32(int64_t dxq, int64_t dyq, float *fx, float *fy) {
    float dx = (float)((double)dxq * QD), dy = (float)((double)dyq * QD);
    if (fx) *fx = dx;
    if (fy) *fy = dy;
    volatile float a = dx * dx;
    volatile float c = dy * dy;
    return a + c;
}

static void all_positions(const orc_box *b, int64_t **X, int64_t **Y) {
    *X = (int64_t *)malloc(sizeof(int64_t) * b->N);
    *Y = (int64_t *)malloc(sizeof(int64_t) * b->N);
    orc_get_positions_q(b, *X, *Y);
}

uint64_t orc_count_overlaps(const orc_box *b) {
    int64_t *X, *Y;
    all_positions(b, &X, &Y);
    uint64_t n = 0;
    for (uint32_t i = 0; i < b->N; ++i)
        for (uint32_t j = i + 1; j < b->N; ++j) {
            int64_t dx = min_image(X[j] - X[i], b->Lq), dy = min_image(Y[j] - Y[i], b->Lq);
            if (llabs(dx) >= 4 * 4194304LL || llabs(dy) >= 4 * 4194304LL) continue;
            if (r2_f32(dx, dy, NULL, NULL) < 4.0f) ++n;
        }
    free(X); free(Y);
    return n;
}

/* ------------------------------------------------------------------------ */
/* Positional order: the structure factor and chi_j (Sec. IV.C, Eqs. (10),
 * (11)), and the positional correlation function C_q(r) averaged over pairs
 * in a window of half-width sigma around r (Sec. IV.D, Eq. (12)). */

void orc_structure_factor(const orc_box *b, const int32_t *hk, uint32_t nq, double *S) {
    int64_t *X, *Y;
    all_positions(b, &X, &Y);
    for (uint32_t iq = 0; iq < nq; ++iq) {
        int64_t h = hk[2 * iq], k = hk[2 * iq + 1];
        double re = 0.0, im = 0.0;
        for (uint32_t n = 0; n < b->N; ++n) {
            /* phase 2 pi (h X + k Y) / Lq, reduced exactly */
            int64_t t = (int64_t)(((__int128)h * X[n] + (__int128)k * Y[n]) % b->Lq);
            if (t < 0) t += b->Lq;
            double ph = 2.0 * M_PI * ((double)t / (double)b->Lq);
            re += cos(ph);
            im += sin(ph);
        }
        S[iq] = (re * re + im * im) / (double)b->N;
    }
    free(X); free(Y);
}

void orc_chi(const orc_box *b, int32_t h, int32_t k, double *re, double *im) {
    int64_t *X, *Y;
    all_positions(b, &X, &Y);
    for (uint32_t n = 0; n < b->N; ++n) {
        int64_t t = (int64_t)(((__int128)h * X[n] + (__int128)k * Y[n]) % b->Lq);
        if (t < 0) t += b->Lq;
        double ph = 2.0 * M_PI * ((double)t / (double)b->Lq);
        re[n] = cos(ph);
        im[n] = sin(ph);
    }
    free(X); free(Y);
}

int orc_cq(const orc_box *b, double qx, double qy, double dr, uint32_t B, double *num,
           int64_t *cnt) {
    const double L_eff = (double)b->Lq * QD;
    const double Dr = ldexp(dr, Q_SHIFT);
    if (B == 0 || Dr != floor(Dr) || Dr <= 0.0) return -1;
    const double top = (double)(B - 1) * dr + 1.0;
    if (!(top < 0.5 * L_eff) || !(top < 512.0)) return -1;
    const int64_t Rq = (int64_t)Dr, one = (int64_t)1 << Q_SHIFT;
    int64_t *X, *Y;
    all_positions(b, &X, &Y);
    for (uint32_t n = 0; n < b->N; ++n)
        for (uint32_t m = n + 1; m < b->N; ++m) {
            int64_t dx = min_image(X[m] - X[n], b->Lq), dy = min_image(Y[m] - Y[n], b->Lq);
            const int64_t reach = (int64_t)ldexp(top, Q_SHIFT);
            if (llabs(dx) > reach || llabs(dy) > reach) continue;
            const uint64_t d2 = (uint64_t)(dx * dx) + (uint64_t)(dy * dy);
            const double phase = qx * ((double)dx * QD) + qy * ((double)dy * QD);
            const double c = cos(phase);
            /* candidate windows from the distance, each confirmed exactly */
            const double d = sqrt((double)d2) * QD;
            int64_t b0 = (int64_t)floor((d - 1.0) / dr) - 1, b1 = (int64_t)ceil((d + 1.0) / dr) + 1;
            if (b0 < 0) b0 = 0;
            if (b1 > (int64_t)B - 1) b1 = (int64_t)B - 1;
            for (int64_t bb = b0; bb <= b1; ++bb) {
                /* window [r_b - 1, r_b + 1] in q units, squared exactly */
                const int64_t R = (int64_t)bb * Rq;
                const int64_t lo = R > one ? R - one : 0, hi = R + one;
                if (d2 >= (uint64_t)(lo * lo) && d2 <= (uint64_t)(hi * hi)) {
                    num[bb] += c;
                    cnt[bb] += 1;
                }
            }
        }
    free(X); free(Y);
    return 0;
}

void orc_hist_edges(uint32_t K, double dr, float *E) {
    for (uint32_t k = 0; k <= K; ++k) {
        double e = 2.0 + (double)k * dr;
        E[k] = (float)(e * e);
    }
}

static int bin_of(const float *E, uint32_t K, float r2) {
    if (!(r2 >= E[0]) || !(r2 < E[K])) return -1;
    uint32_t k = 0;
    while (!(r2 < E[k + 1])) ++k;
    return (int)k;
}

/* Eq. (2) counts: number n_k of pair distances in bin k. */
void orc_pair_hist(const orc_box *b, uint32_t K, double dr, int64_t *counts) {
    float *E = (float *)malloc(sizeof(float) * (K + 1));
    orc_hist_edges(K, dr, E);
    int64_t *X, *Y;
    all_positions(b, &X, &Y);
    for (uint32_t i = 0; i < b->N; ++i)
        for (uint32_t j = i + 1; j < b->N; ++j) {
            int64_t dx = min_image(X[j] - X[i], b->Lq), dy = min_image(Y[j] - Y[i], b->Lq);
            int k = bin_of(E, K, r2_f32(dx, dy, NULL, NULL));
            if (k >= 0) counts[k]++;
        }
    free(X); free(Y); free(E);
}

void orc_pair_hist_subset(const orc_box *b, const uint8_t *sel, uint32_t K, double dr,
                          int64_t *counts) {
    float *E = (float *)malloc(sizeof(float) * (K + 1));
    orc_hist_edges(K, dr, E);
    int64_t *X, *Y;
    all_positions(b, &X, &Y);
    for (uint32_t i = 0; i < b->N; ++i) {
        if (!sel[i]) continue;
        for (uint32_t j = 0; j < b->N; ++j) {
            if (j == i) continue;
            int64_t dx = min_image(X[j] - X[i], b->Lq), dy = min_image(Y[j] - Y[i], b->Lq);
            int k = bin_of(E, K, r2_f32(dx, dy, NULL, NULL));
            if (k >= 0) counts[k]++;
        }
    }
    free(X); free(Y); free(E);
}

/* ------------------------------------------------------------------------ */
/* Pressure from the contact value of g(r), Sec. II.C.1.
 * g_k = (n_k / p) / (2 pi r_k dr / V), Eq. (2), with p = N(N-1)/2 pairs per
 * configuration and r_k the bin centre; a polynomial of the given order in
 * (r - 2) is fitted to g_k by unweighted least squares and its constant term
 * is g(2 sigma+).  Eq. (4) at finite N reads Z = beta P V / N =
 * 1 + 2 eta (N-1)/N g(2 sigma+), and P* = beta P (2 sigma)^2 = 4 eta Z / pi. */
int orc_pressure(const int64_t *counts, uint32_t K, double dr, uint32_t order,
                 uint64_t n_conf, uint32_t N, double L_eff, double *g_contact, double *Z,
                 double *P_star, double *coef) {
    if (n_conf == 0 || N < 2 || K < order + 1 || order > 8) return -1;
    double V = L_eff * L_eff;
    double p = 0.5 * (double)N * (double)(N - 1) * (double)n_conf;
    uint32_t nc = order + 1;
    /* Householder QR of the K x nc design matrix A, columns t^e with
     * t = (r_k - 2) / (K dr) scaled into (0, 1). */
    double *A = (double *)malloc(sizeof(double) * K * nc);
    double *y = (double *)malloc(sizeof(double) * K);
    for (uint32_t k = 0; k < K; ++k) {
        double r = 2.0 + ((double)k + 0.5) * dr;
        y[k] = ((double)counts[k] / p) / (2.0 * M_PI * r * dr / V);
        double t = (r - 2.0) / ((double)K * dr), v = 1.0;
        for (uint32_t e = 0; e < nc; ++e) { A[k * nc + e] = v; v *= t; }
    }
    for (uint32_t e = 0; e < nc; ++e) {
        double nrm = 0.0;
        for (uint32_t k = e; k < K; ++k) nrm += A[k * nc + e] * A[k * nc + e];
        nrm = sqrt(nrm);
        if (nrm == 0.0) { free(A); free(y); return -1; }
        double alpha = A[e * nc + e] > 0 ? -nrm : nrm;
        /* v = a - alpha e1 */
        double *v = (double *)malloc(sizeof(double) * K);
        for (uint32_t k = 0; k < K; ++k) v[k] = (k < e) ? 0.0 : A[k * nc + e];
        v[e] -= alpha;
        double vv = 0.0;
        for (uint32_t k = e; k < K; ++k) vv += v[k] * v[k];
        if (vv > 0.0) {
            for (uint32_t c = e; c < nc; ++c) {
                double s = 0.0;
                for (uint32_t k = e; k < K; ++k) s += v[k] * A[k * nc + c];
                s = 2.0 * s / vv;
                for (uint32_t k = e; k < K; ++k) A[k * nc + c] -= s * v[k];
            }
            double s = 0.0;
            for (uint32_t k = e; k < K; ++k) s += v[k] * y[k];
            s = 2.0 * s / vv;
            for (uint32_t k = e; k < K; ++k) y[k] -= s * v[k];
        }
        free(v);
    }
    double c[9];
    for (int e = (int)nc - 1; e >= 0; --e) {
        double s = y[e];
        for (uint32_t f = (uint32_t)e + 1; f < nc; ++f) s -= A[e * nc + f] * c[f];
        if (A[e * nc + e] == 0.0) { free(A); free(y); return -1; }
        c[e] = s / A[e * nc + e];
    }
    free(A); free(y);
    double eta = (double)N * M_PI / V;
    double g0 = c[0];
    double z = 1.0 + 2.0 * eta * ((double)(N - 1) / (double)N) * g0;
    if (g_contact) *g_contact = g0;
    if (Z) *Z = z;
    if (P_star) *P_star = 4.0 * eta * z / M_PI;
    if (coef) {
        /* back to powers of (r - 2) */
        double sc = 1.0;
        for (uint32_t e = 0; e < nc; ++e) { coef[e] = c[e] / sc; sc *= (double)K * dr; }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Local orientational order, Eq. (8): psi_j = (1/6) sum over the six closest
 * neighbours of exp(6 i phi_jk), phi measured from the +x axis on the shortest
 * periodic separation.  exp(6 i phi) = (z^2)^3 / |z|^6 with z = dx + i dy. */
void orc_psi6(const orc_box *b, const uint8_t *sel, double *re, double *im) {
    int64_t *X, *Y;
    all_positions(b, &X, &Y);
    for (uint32_t j = 0; j < b->N; ++j) {
        if (sel && !sel[j]) continue;
        float best_r2[6];
        uint32_t best_t[6];
        int64_t best_dx[6], best_dy[6];
        int nb = 0;
        for (uint32_t k = 0; k < b->N; ++k) {
            if (k == j) continue;
            int64_t dx = min_image(X[k] - X[j], b->Lq), dy = min_image(Y[k] - Y[j], b->Lq);
            float r2 = r2_f32(dx, dy, NULL, NULL);
            /* insertion into the sorted list of the six best (r2, tag) */
            int pos = nb;
            while (pos > 0 && (r2 < best_r2[pos - 1] ||
                               (r2 == best_r2[pos - 1] && k < best_t[pos - 1])))
                --pos;
            if (pos >= 6) continue;
            int last = nb < 6 ? nb : 5;
            for (int e = last; e > pos; --e) {
                best_r2[e] = best_r2[e - 1]; best_t[e] = best_t[e - 1];
                best_dx[e] = best_dx[e - 1]; best_dy[e] = best_dy[e - 1];
            }
            best_r2[pos] = r2; best_t[pos] = k; best_dx[pos] = dx; best_dy[pos] = dy;
            if (nb < 6) ++nb;
        }
        double sr = 0.0, si = 0.0;
        for (int e = 0; e < nb; ++e) {
            double dx = (double)best_dx[e] * QD, dy = (double)best_dy[e] * QD;
            double r2 = dx * dx + dy * dy;
            double ar = dx * dx - dy * dy, ai = 2.0 * dx * dy;        /* z^2 */
            double br = ar * ar - ai * ai, bi = 2.0 * ar * ai;        /* z^4 */
            double cr = br * ar - bi * ai, ci = br * ai + bi * ar;    /* z^6 */
            double r6 = r2 * r2 * r2;
            sr += cr / r6;
            si += ci / r6;
        }
        re[j] = sr / 6.0;
        im[j] = si / 6.0;
    }
    free(X); free(Y);
}

/* psi field: for each cell, the mean psi_j over disks in its 3 x 3 block
 * (a sampling area of about 8 disks, Sec. IV.B uses 5 to 20). */
void orc_psi6_field(const orc_box *b, const double *re, const double *im, double *fre,
                    double *fim) {
    uint32_t M = b->M;
    for (uint32_t cj = 0; cj < M; ++cj)
        for (uint32_t ci = 0; ci < M; ++ci) {
            double sr = 0.0, si = 0.0;
            uint32_t n = 0;
            for (int dj = -1; dj <= 1; ++dj)
                for (int di = -1; di <= 1; ++di) {
                    uint32_t nb = ((ci + M + di) % M) + M * ((cj + M + dj) % M);
                    for (uint32_t s = 0; s < b->cnt[nb]; ++s) {
                        uint32_t t = b->tag[nb * b->cap + s];
                        sr += re[t]; si += im[t]; ++n;
                    }
                }
            fre[ci + M * cj] = n ? sr / n : 0.0;
            fim[ci + M * cj] = n ? si / n : 0.0;
        }
}

/* ------------------------------------------------------------------------ */
/* Eq. (9): C(dt) = < Psi(t) Psi*(t+dt) >_t / < |Psi|^2 >_t, real part, with
 * all time origins t = 0 .. n-1-dt. */
void orc_acf(const double *re, const double *im, uint32_t n, uint32_t maxlag, double *C) {
    double den = 0.0;
    for (uint32_t t = 0; t < n; ++t) den += re[t] * re[t] + im[t] * im[t];
    den /= (double)n;
    for (uint32_t d = 0; d <= maxlag; ++d) {
        double s = 0.0;
        uint32_t cnt = 0;
        for (uint32_t t = 0; t + d < n; ++t) {
            s += re[t] * re[t + d] + im[t] * im[t + d];
            ++cnt;
        }
        C[d] = cnt ? (s / cnt) / den : 0.0;
    }
}

/* C ~ exp(-dt / tau) in the asymptotic regime (Sec. III): least squares of
 * ln C against dt over the lags where lo <= C <= hi, stopping at the first
 * lag below lo. */
double orc_tau_fit(const double *C, uint32_t maxlag, double lo, double hi) {
    double sx = 0, sy = 0, sxx = 0, sxy = 0;
    uint32_t n = 0;
    for (uint32_t d = 1; d <= maxlag; ++d) {
        if (C[d] < lo) break;
        if (C[d] > hi) continue;
        double y = log(C[d]);
        sx += d; sy += y; sxx += (double)d * d; sxy += d * y; ++n;
    }
    if (n < 3) return -1.0;
    double slope = (n * sxy - sx * sy) / (n * sxx - sx * sx);
    if (!(slope < 0)) return -1.0;
    return -1.0 / slope;
}

double orc_tau_int(const double *C, uint32_t maxlag, double c) {
    double tau = 0.5;
    for (uint32_t d = 1; d <= maxlag; ++d) {
        tau += C[d];
        if ((double)d >= c * tau) break;
    }
    return tau;
}

/* ------------------------------------------------------------------------ */
/* Learned proposal, fp64 reference.  Features: neighbours within 3 sigma of
 * the trial position, enumerated over the 3 x 3 cell block (rows dj = -1..1
 * outer, columns di = -1..1 inner, slots ascending), sorted by (fp32 r^2,
 * enumeration index), first 12 kept. */
int orc_features(const orc_box *b, uint32_t cell, uint32_t self, float x, float y, float *f) {
    uint32_t M = b->M, ci = cell % M, cj = cell / M;
    float cr2[72], cdx[72], cdy[72];
    int n = 0;
    for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di) {
            uint32_t nb = ((ci + M + di) % M) + M * ((cj + M + dj) % M);
            float cwx = (float)di * b->w, cwy = (float)dj * b->w;
            for (uint32_t s = 0; s < b->cnt[nb]; ++s) {
                uint32_t k = nb * b->cap + s;
                if (b->tag[k] == self) continue;
                float dx = (b->x[k] - x) + cwx, dy = (b->y[k] - y) + cwy;
                volatile float a = dx * dx;
                volatile float c = dy * dy;
                float r2 = a + c;
                if (!(r2 < 9.0f)) continue;
                /* stable insertion by r2 keeps enumeration order on ties */
                int pos = n;
                while (pos > 0 && r2 < cr2[pos - 1]) --pos;
                for (int e = n; e > pos; --e) {
                    cr2[e] = cr2[e - 1]; cdx[e] = cdx[e - 1]; cdy[e] = cdy[e - 1];
                }
                cr2[pos] = r2; cdx[pos] = dx; cdy[pos] = dy;
                ++n;
            }
        }
    int m = n < 12 ? n : 12;
    for (int e = 0; e < 12; ++e) {
        f[2 * e] = e < m ? cdx[e] : 0.0f;
        f[2 * e + 1] = e < m ? cdy[e] : 0.0f;
    }
    return m;
}

static double silu(double v) { return v / (1.0 + exp(-v)); }
static double dsilu(double v) {
    double s = 1.0 / (1.0 + exp(-v));
    return s * (1.0 + v * (1.0 - s));
}

#define P_W1 0
#define P_B1 (P_W1 + 64 * 24)
#define P_W2 (P_B1 + 64)
#define P_B2 (P_W2 + 64 * 64)
#define P_W3 (P_B2 + 64)
#define P_B3 (P_W3 + 20 * 64)

static void forward_full(const double *p, const double *f, double *a1, double *h1, double *a2,
                         double *h2, double *out) {
    for (int o = 0; o < 64; ++o) {
        double s = p[P_B1 + o];
        for (int i = 0; i < 24; ++i) s += p[P_W1 + o * 24 + i] * f[i];
        a1[o] = s; h1[o] = silu(s);
    }
    for (int o = 0; o < 64; ++o) {
        double s = p[P_B2 + o];
        for (int i = 0; i < 64; ++i) s += p[P_W2 + o * 64 + i] * h1[i];
        a2[o] = s; h2[o] = silu(s);
    }
    for (int o = 0; o < 20; ++o) {
        double s = p[P_B3 + o];
        for (int i = 0; i < 64; ++i) s += p[P_W3 + o * 64 + i] * h2[i];
        out[o] = s;
    }
}

void orc_mlp_forward(const double *p, const double *f, double *out) {
    double a1[64], h1[64], a2[64], h2[64];
    forward_full(p, f, a1, h1, a2, h2, out);
}

/* Component k of the network output: (logit, mu_x, mu_y, a_x, a_y) at
 * out[5k..5k+4]; sigma = exp(a) with a clamped to [A_MIN, A_MAX]: widths
 * from about 190 q to e sigma. */
#define A_MIN (-10.0)
#define A_MAX 1.0
static double clampa(double a) { return a < A_MIN ? A_MIN : (a > A_MAX ? A_MAX : a); }

double orc_gmm_logpdf(const double *out, double dx, double dy) {
    double lmax = -INFINITY, l[4], lw[4];
    for (int k = 0; k < 4; ++k) lmax = out[5 * k] > lmax ? out[5 * k] : lmax;
    double z = 0.0;
    for (int k = 0; k < 4; ++k) z += exp(out[5 * k] - lmax);
    for (int k = 0; k < 4; ++k) lw[k] = out[5 * k] - lmax - log(z);
    double best = -INFINITY;
    for (int k = 0; k < 4; ++k) {
        double ax = clampa(out[5 * k + 3]), ay = clampa(out[5 * k + 4]);
        double ux = (dx - out[5 * k + 1]) * exp(-ax), uy = (dy - out[5 * k + 2]) * exp(-ay);
        l[k] = lw[k] - log(2.0 * M_PI) - ax - ay - 0.5 * (ux * ux + uy * uy);
        best = l[k] > best ? l[k] : best;
    }
    double s = 0.0;
    for (int k = 0; k < 4; ++k) s += exp(l[k] - best);
    return best + log(s);
}

/* Mean over the batch of -log q_GMM(D_b | MLP(F_b)); grad += d/dparams. */
double orc_nll_grad(const double *p, const double *F, const double *D, uint32_t B,
                    double *grad) {
    memset(grad, 0, sizeof(double) * ORC_NPARAM);
    double total = 0.0;
    for (uint32_t bi = 0; bi < B; ++bi) {
        const double *f = F + (size_t)bi * 24;
        double dx = D[2 * bi], dy = D[2 * bi + 1];
        double a1[64], h1[64], a2[64], h2[64], out[20];
        forward_full(p, f, a1, h1, a2, h2, out);
        /* loss = -log sum_k exp(l_k); l_k = log softmax_k - log 2pi - ax - ay
         *        - (ux^2 + uy^2)/2 */
        double lmax = -INFINITY, lw[4], l[4], r[4], pi_[4];
        for (int k = 0; k < 4; ++k) lmax = out[5 * k] > lmax ? out[5 * k] : lmax;
        double z = 0.0;
        for (int k = 0; k < 4; ++k) z += exp(out[5 * k] - lmax);
        for (int k = 0; k < 4; ++k) { lw[k] = out[5 * k] - lmax - log(z); pi_[k] = exp(lw[k]); }
        double best = -INFINITY;
        double ux[4], uy[4], ax[4], ay[4];
        for (int k = 0; k < 4; ++k) {
            ax[k] = clampa(out[5 * k + 3]); ay[k] = clampa(out[5 * k + 4]);
            ux[k] = (dx - out[5 * k + 1]) * exp(-ax[k]);
            uy[k] = (dy - out[5 * k + 2]) * exp(-ay[k]);
            l[k] = lw[k] - log(2.0 * M_PI) - ax[k] - ay[k] - 0.5 * (ux[k] * ux[k] + uy[k] * uy[k]);
            best = l[k] > best ? l[k] : best;
        }
        double s = 0.0;
        for (int k = 0; k < 4; ++k) s += exp(l[k] - best);
        double lse = best + log(s);
        total += -lse;
        for (int k = 0; k < 4; ++k) r[k] = exp(l[k] - lse);  /* responsibilities */
        /* d(-lse)/d out */
        double dout[20];
        for (int k = 0; k < 4; ++k) {
            dout[5 * k] = pi_[k] - r[k];
            dout[5 * k + 1] = -r[k] * ux[k] * exp(-ax[k]);
            dout[5 * k + 2] = -r[k] * uy[k] * exp(-ay[k]);
            double inx = out[5 * k + 3] > A_MIN && out[5 * k + 3] < A_MAX;
            double iny = out[5 * k + 4] > A_MIN && out[5 * k + 4] < A_MAX;
            dout[5 * k + 3] = -r[k] * (ux[k] * ux[k] - 1.0) * inx;
            dout[5 * k + 4] = -r[k] * (uy[k] * uy[k] - 1.0) * iny;
        }
        double dh2[64] = {0}, dh1[64] = {0};
        for (int o = 0; o < 20; ++o) {
            grad[P_B3 + o] += dout[o];
            for (int i = 0; i < 64; ++i) {
                grad[P_W3 + o * 64 + i] += dout[o] * h2[i];
                dh2[i] += dout[o] * p[P_W3 + o * 64 + i];
            }
        }
        for (int o = 0; o < 64; ++o) {
            double da = dh2[o] * dsilu(a2[o]);
            grad[P_B2 + o] += da;
            for (int i = 0; i < 64; ++i) {
                grad[P_W2 + o * 64 + i] += da * h1[i];
                dh1[i] += da * p[P_W2 + o * 64 + i];
            }
        }
        for (int o = 0; o < 64; ++o) {
            double da = dh1[o] * dsilu(a1[o]);
            grad[P_B1 + o] += da;
            for (int i = 0; i < 24; ++i) grad[P_W1 + o * 24 + i] += da * f[i];
        }
    }
    for (int e = 0; e < ORC_NPARAM; ++e) grad[e] /= (double)B;
    return total / (double)B;
}

/* Adam (Kingma & Ba, 2015) with bias correction. */
void orc_adam(double *p, double *m, double *v, const double *g, uint32_t n, double lr,
              uint32_t t) {
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (uint32_t e = 0; e < n; ++e) {
        m[e] = b1 * m[e] + (1.0 - b1) * g[e];
        v[e] = b2 * v[e] + (1.0 - b2) * g[e] * g[e];
        p[e] -= lr * (m[e] / c1) / (sqrt(v[e] / c2) + eps);
    }
}

/* ------------------------------------------------------------------------ */
/* Learned proposal: an extension of the uniform trial move of Sec. II.B (the
 * paper has no learned proposal).  A network maps the moving disk's
 * neighbourhood f(x) to 20 numbers, read as a four-component Gaussian
 * mixture, and the trial displacement D (delta = D q, D integer per axis)
 * is drawn from the law on the q lattice
 *
 *   P(D | out) = e U(D) + (1 - e) G(D | out),
 *
 *   e     = E / 2^32, E the nearest integer to eps * 2^32 (the branch test
 *           compares a 32-bit word with E, so e is exactly the branch
 *           probability);
 *   U(D)  = the plain trial's step: per axis D = m j, j odd, |j| <= 2^14 - 1,
 *           each of the 2^14 values with probability 2^-14;
 *   G(D)  = sum_k pi_k g_k(Dx; mu_xk, s_xk) g_k(Dy; mu_yk, s_yk): a component
 *           k is chosen with probability pi_k (softmax of the logits), a
 *           point is drawn from N(mu_k, diag(s_k^2)) (s = exp(clamp(a))) in
 *           double precision and rounded to the nearest lattice point; draws
 *           with |D| > 2^22 - 1 on either axis fail (the trial is rejected).
 *           g(D; mu, s) is the Gaussian mass of the lattice cell
 *           [D - 1/2, D + 1/2] q, written through the even Taylor terms of
 *           the cell integral: (q/s) phi(u) (1 + h^2 He2(u) / 6 +
 *           h^4 He4(u) / 120) with u = (D q - mu) / s, h = q / (2 s),
 *           He2 = u^2 - 1, He4 = u^4 - 6 u^2 + 3; the next term, h^6 He6 / 5040,
 *           is below 2e-14 relative for s >= e^-10 and |u| <= 9.
 *
 * Random words of trial t in cell c of sweep k (counter layout as above):
 *   A = stream 0: A0 selects the disk and A1, A2 give the uniform step,
 *       exactly as in the plain trial; A3 < E chooses U;
 *   B = stream 2: (B0, B1) the component uniform, (B2, B3) the acceptance
 *       uniform;
 *   C = stream 4: (C0, C1) u1 in (0, 1], (C2, C3) u2 in [0, 1); the normal
 *       pair is sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2) (Box-Muller).
 *   A 53-bit uniform from (hi, lo) is ((hi << 21) | (lo >> 11)) 2^-53.
 *
 * The trial is the Metropolis-Hastings step (extending Sec. II.B's local
 * move): propose x' = x + D q; reject if the draw failed, x' leaves the cell
 * or overlaps a disk; else accept when
 * ln u_a < ln P(-D | out(x')) - ln P(D | out(x)).  With e = 1 it is the
 * plain trial, word for word. */

#define NBRANCH_SHIFT 32
typedef struct {
    double lp[4], mx[4], my[4], ax[4], ay[4];
} mixture;

static void mixture_of(const double *out, mixture *g) {
    double lmax = -INFINITY;
    for (int k = 0; k < 4; ++k) lmax = out[5 * k] > lmax ? out[5 * k] : lmax;
    double z = 0.0;
    for (int k = 0; k < 4; ++k) z += exp(out[5 * k] - lmax);
    double lz = lmax + log(z);
    for (int k = 0; k < 4; ++k) {
        g->lp[k] = out[5 * k] - lz;
        g->mx[k] = out[5 * k + 1];
        g->my[k] = out[5 * k + 2];
        g->ax[k] = clampa(out[5 * k + 3]);
        g->ay[k] = clampa(out[5 * k + 4]);
    }
}

static uint64_t branch_threshold(float eps) {
    return (uint64_t)llrint((double)eps * 4294967296.0);
}

static double u53(uint32_t hi, uint32_t lo) {
    return ldexp((double)(((uint64_t)hi << 21) | (lo >> 11)), -53);
}

static int on_step_lattice(int64_t D, uint32_t m) {
    if (D % (int64_t)m != 0) return 0;
    int64_t j = D / (int64_t)m;
    return (j & 1) != 0 && llabs(j) <= 16383;
}

/* ln of the Gaussian mass of lattice cell D on one axis. */
static double log_cell_mass(int64_t D, double mu, double a) {
    double is = exp(-a);
    double u = ((double)D * QD - mu) * is;
    double h = 0.5 * QD * is;
    double u2 = u * u, h2 = h * h;
    double he2 = u2 - 1.0, he4 = (u2 - 6.0) * u2 + 3.0;
    double corr = h2 * he2 / 6.0 + (h2 * h2) * he4 / 120.0;
    return log(QD) - a - 0.5 * log(2.0 * M_PI) - 0.5 * u2 + log1p(corr);
}

static double log_add(double a, double b) {
    double m = a > b ? a : b;
    if (m == -INFINITY) return m;
    return m + log1p(exp(-fabs(a - b)));
}

static double log_p(const mixture *g, int64_t Dx, int64_t Dy, uint32_t m, uint64_t E) {
    double e = ldexp((double)E, -NBRANCH_SHIFT);
    double lu = (on_step_lattice(Dx, m) && on_step_lattice(Dy, m)) ? -28.0 * M_LN2 : -INFINITY;
    double lg = -INFINITY;
    if (llabs(Dx) <= 4194303 && llabs(Dy) <= 4194303) {
        double l[4], best = -INFINITY;
        for (int k = 0; k < 4; ++k) {
            l[k] = g->lp[k] + log_cell_mass(Dx, g->mx[k], g->ax[k]) +
                   log_cell_mass(Dy, g->my[k], g->ay[k]);
            best = l[k] > best ? l[k] : best;
        }
        if (best > -INFINITY) {
            double s = 0.0;
            for (int k = 0; k < 4; ++k) s += exp(l[k] - best);
            lg = best + log(s);
        }
    }
    return log_add(log(e) + lu, log1p(-e) + lg);
}

/* Draws D from P(. | g) with the words A, B, C; returns 0 for a failed draw. */
static int learned_draw(const mixture *g, const uint32_t A[4], const uint32_t B[4],
                        const uint32_t C[4], uint32_t m, uint64_t E, int64_t *Dx, int64_t *Dy) {
    if ((uint64_t)A[3] < E) {
        *Dx = (int64_t)m * (2 * (int64_t)(A[1] >> 18) + 1 - 16384);
        *Dy = (int64_t)m * (2 * (int64_t)(A[2] >> 18) + 1 - 16384);
        return 1;
    }
    double uc = u53(B[0], B[1]);
    int k = 3;
    double cum = 0.0;
    for (int c = 0; c < 3; ++c) {
        cum += exp(g->lp[c]);
        if (uc < cum) { k = c; break; }
    }
    double u1 = ldexp((double)((((uint64_t)C[0] << 21) | (C[1] >> 11)) + 1), -53);
    double u2 = u53(C[2], C[3]);
    double r = sqrt(-2.0 * log(u1));
    double th = 2.0 * M_PI * u2;
    double tx = (g->mx[k] + (exp(g->ax[k]) * r) * cos(th)) * 4194304.0;
    double ty = (g->my[k] + (exp(g->ay[k]) * r) * sin(th)) * 4194304.0;
    if (!(fabs(tx) < 4194303.5 && fabs(ty) < 4194303.5)) return 0;
    *Dx = (int64_t)rint(tx);
    *Dy = (int64_t)rint(ty);
    return 1;
}

double orc_learned_logp(const double *out, int64_t Dx, int64_t Dy, uint32_t step_m, float eps) {
    mixture g;
    mixture_of(out, &g);
    return log_p(&g, Dx, Dy, step_m, branch_threshold(eps));
}

void orc_learned_proposals(const double *out, uint32_t step_m, float eps, uint64_t seed,
                           uint32_t n, int64_t *D, uint8_t *drawn, double *logp) {
    mixture g;
    mixture_of(out, &g);
    uint64_t E = branch_threshold(eps);
    for (uint32_t i = 0; i < n; ++i) {
        uint32_t A[4], B[4], Cw[4];
        uint32_t ca[4] = {0, i, 0, 0}, cb[4] = {0, i, 0, 2}, cc[4] = {0, i, 0, 4};
        orc_philox((uint32_t)seed, (uint32_t)(seed >> 32), ca, A);
        orc_philox((uint32_t)seed, (uint32_t)(seed >> 32), cb, B);
        orc_philox((uint32_t)seed, (uint32_t)(seed >> 32), cc, Cw);
        int64_t Dx = 0, Dy = 0;
        int ok = learned_draw(&g, A, B, Cw, step_m, E, &Dx, &Dy);
        D[2 * i] = Dx;
        D[2 * i + 1] = Dy;
        if (drawn) drawn[i] = (uint8_t)ok;
        if (logp) logp[i] = ok ? log_p(&g, Dx, Dy, step_m, E) : NAN;
    }
}

typedef struct {
    const double *params;
    uint64_t E;
} learned_ctx;

/* The network's mixture for the disk of tag `self` at cell-local (x, y) of
 * `cell`, all other disks where they are. */
static void mixture_at(const orc_box *b, const double *params, uint32_t cell, uint32_t self,
                       float x, float y, mixture *g) {
    float f32[24];
    double f[24], out[20];
    orc_features(b, cell, self, x, y, f32);
    for (int e = 0; e < 24; ++e) f[e] = (double)f32[e];
    orc_mlp_forward(params, f, out);
    mixture_of(out, g);
}

static void trial_cell_learned(orc_box *b, uint32_t ci, uint32_t cj, void *ctx) {
    const learned_ctx *L = (const learned_ctx *)ctx;
    uint32_t M = b->M, cap = b->cap;
    uint32_t cell = ci + M * cj;
    uint32_t n = b->cnt[cell];
    if (n == 0) return;
    uint32_t perm[8];
    if (b->n_trial > 1) shuffle_slots(b, cell, n, perm);
    for (uint32_t t = 0; t < b->n_trial; ++t) {
        uint32_t A[4], B[4], Cw[4];
        draw(b, b->sweep, cell, t, 0, A);
        draw(b, b->sweep, cell, t, 2, B);
        draw(b, b->sweep, cell, t, 4, Cw);
        uint32_t slot = (b->n_trial == 1) ? mulhi(A[0], n) : perm[t % n];
        uint32_t k = cell * cap + slot, self = b->tag[k];
        b->trials++;
        mixture g, gr;
        mixture_at(b, L->params, cell, self, b->x[k], b->y[k], &g);
        int64_t Dx, Dy;
        if (!learned_draw(&g, A, B, Cw, b->step_m, L->E, &Dx, &Dy)) continue;
        int64_t U = (int64_t)ldexp((double)b->x[k], Q_SHIFT) + Dx;
        int64_t V = (int64_t)ldexp((double)b->y[k], Q_SHIFT) + Dy;
        if (U < 0 || U >= b->W || V < 0 || V >= b->W) continue;
        float xn = (float)((double)U * QD), yn = (float)((double)V * QD);  /* exact */
        if (overlaps_block(b, ci, cj, slot, xn, yn)) continue;
        mixture_at(b, L->params, cell, self, xn, yn, &gr);
        double d = log_p(&gr, -Dx, -Dy, b->step_m, L->E) - log_p(&g, Dx, Dy, b->step_m, L->E);
        if (!(d >= 0.0) && !(log(u53(B[2], B[3])) < d)) continue;
        b->x[k] = xn;
        b->y[k] = yn;
        b->accepts++;
    }
}

void orc_sweep_learned(orc_box *b, const double *params, float eps, uint64_t k) {
    learned_ctx L = {params, branch_threshold(eps)};
    sweeps_with(b, k, 0, trial_cell_learned, &L);
}
