// learned.hip — a learned local proposal for the MPMC sweep, kept exact by a
// Metropolis-Hastings correction (an extension of the paper's uniform trial
// move of Sec. II.B; the uniform move stays in the mixture as fallback).
//
//  features  f(x): the up to 12 nearest other disks within 3 sigma of the
//            trial position, (dx, dy) each, sorted by (fp32 r^2, enumeration
//            order over the 3 x 3 cell block), zero padded to 24.
//  network   24 -> 64 -> 64 -> 20, SiLU, BF16 weights with FP32 accumulate
//            on the matrix cores (v_mfma_f32_16x16x16bf16), the 64 lanes of
//            a wave forming the GEMM row dimension.
//  proposal  q(delta | f) = eps U_d(delta) + (1 - eps) sum_k pi_k
//            N(delta; mu_k, diag(s_k^2)), 4 components, s = exp(clamp(a)).
//  MH        accept with min(1, q(-delta | f(x')) / q(delta | f(x))) if x'
//            stays in the cell and overlaps nothing.  Cells of width >= 3
//            sigma keep the 3 sigma neighbourhoods of x and x' frozen while a
//            colour sub-sweep runs, so each trial is an exact MH step.
//  training  accepted plain moves (f(x), delta) are recorded; the network
//            is trained to maximise log q_GMM(delta | f) with the same MFMA
//            GEMMs run forward and backward, and Adam on FP32 master weights.
#include <math.h>
#include <string.h>

#include <vector>

#include "mpmc_host.hpp"

namespace mpmc {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kNF = 24, kNH = 64, kNO = 20, kNPARAM = 7060;
constexpr int kPW1 = 0, kPB1 = kPW1 + kNH * kNF, kPW2 = kPB1 + kNH, kPB2 = kPW2 + kNH * kNH,
              kPW3 = kPB2 + kNH, kPB3 = kPW3 + kNO * kNH;
static_assert(kPB3 + kNO == kNPARAM, "flat parameter vector: W1, b1, W2, b2, W3, b3");
constexpr int kStreamTrain = 5;

// BF16 weights in the layouts the GEMMs read (k contiguous), zero padded:
// w1[64 out][32 in], w2[64][64], w3[32 out][64 in] and, for the backward
// pass, w2t[64 in][64 out], w3t[64 in][32 out].
struct PackedW {
    uint16_t w1[64 * 32];
    uint16_t w2[64 * 64];
    uint16_t w3[32 * 64];
    uint16_t w2t[64 * 64];
    uint16_t w3t[64 * 32];
    float b1[64], b2[64], b3[32];
};
// The inference weights in LDS, as the MFMA A-operand fragments of the
// transposed products: fragment f = nt * KS + ks holds, for lane l, the four
// bf16 W[16 nt + l%16][16 ks + 4 (l/16) ..+3], so that a wave reads a
// fragment as 512 consecutive bytes (no bank conflicts).
struct InferW {
    v4s w1[8][64];   // 4 row tiles x 2 k-steps
    v4s w2[16][64];  // 4 x 4
    v4s w3[8][64];   // 2 x 4 (outputs 0..31)
    float b1[64], b2[64], b3[32];
};
// Row strides in LDS of the network input (bf16) and output (fp32), padded
// so that the 16 rows a wave touches at once fall in different banks.
constexpr int kXS = 40, kOS = 33;

__host__ __device__ inline uint16_t f2bf(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
    return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline float silu(float v) { return v / (1.0f + __expf(-v)); }
__device__ inline float dsilu(float v) {
    const float s = 1.0f / (1.0f + __expf(-v));
    return s * (1.0f + v * (1.0f - s));
}

// All 64 lanes of the wave see each other's LDS writes after this.
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// acc[mi][ni] += A[16 mi.., :] Bt[16 ni.., :]^T over K = 16 KT, with A and
// Bt bf16 row-major in LDS (k contiguous).  Lane l holds, for the 16 x 16 x
// 16 MFMA, A[row l%16][k = 4(l/16)..+3], B[k = 4(l/16)..+3][col l%16] and
// C[rows 4(l/16)..+3][col l%16].
template <int MT, int NT, int KT>
__device__ inline void wave_gemm(const uint16_t *A, int lda, const uint16_t *Bt, int ldb,
                                 v4f (&acc)[MT][NT]) {
    const int l = threadIdx.x & 63, r = l & 15, kg = (l >> 4) * 4;
#pragma unroll
    for (int ks = 0; ks < KT; ++ks) {
        v4s a[MT], b[NT];
#pragma unroll
        for (int mi = 0; mi < MT; ++mi)
            a[mi] = *reinterpret_cast<const v4s *>(A + (16 * mi + r) * lda + 16 * ks + kg);
#pragma unroll
        for (int ni = 0; ni < NT; ++ni)
            b[ni] = *reinterpret_cast<const v4s *>(Bt + (16 * ni + r) * ldb + 16 * ks + kg);
#pragma unroll
        for (int mi = 0; mi < MT; ++mi)
#pragma unroll
            for (int ni = 0; ni < NT; ++ni)
                acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[mi], b[ni], acc[mi][ni], 0, 0, 0);
    }
}

template <int MT, int NT>
__device__ inline void zero_acc(v4f (&acc)[MT][NT]) {
#pragma unroll
    for (int mi = 0; mi < MT; ++mi)
#pragma unroll
        for (int ni = 0; ni < NT; ++ni) acc[mi][ni] = v4f{0.f, 0.f, 0.f, 0.f};
}

// Forward pass of one wave: X[64][32] -> H1, H2 -> OUT[64][32] (fp32; the
// 20 outputs in columns 0..19).  If A1/A2 are given the pre-activations are
// kept (fp32 [64][64]) and transposed bf16 copies of X, H1, H2 are written
// for the backward pass.
struct FwdBufs {
    uint16_t *X, *H1, *H2;       // row-major bf16
    uint16_t *XT, *H1T, *H2T;    // transposed bf16 (training only)
    float *A1, *A2;              // pre-activations (training only)
    float *OUT;                  // [64][32]
};

template <class WT>
__device__ inline void mlp_forward_wave(const WT &W, const FwdBufs &B) {
    const int l = threadIdx.x & 63, col = l & 15, rg = (l >> 4) * 4;
    {
        v4f acc[4][4];
        zero_acc(acc);
        wave_gemm<4, 4, 2>(B.X, 32, W.w1, 32, acc);
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int ni = 0; ni < 4; ++ni)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int m = 16 * mi + rg + e, n = 16 * ni + col;
                    const float a = acc[mi][ni][e] + W.b1[n];
                    const uint16_t h = f2bf(silu(a));
                    B.H1[m * 64 + n] = h;
                    if (B.A1) {
                        B.A1[m * 64 + n] = a;
                        B.H1T[n * 64 + m] = h;
                    }
                }
    }
    wave_sync();
    {
        v4f acc[4][4];
        zero_acc(acc);
        wave_gemm<4, 4, 4>(B.H1, 64, W.w2, 64, acc);
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int ni = 0; ni < 4; ++ni)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int m = 16 * mi + rg + e, n = 16 * ni + col;
                    const float a = acc[mi][ni][e] + W.b2[n];
                    const uint16_t h = f2bf(silu(a));
                    B.H2[m * 64 + n] = h;
                    if (B.A2) {
                        B.A2[m * 64 + n] = a;
                        B.H2T[n * 64 + m] = h;
                    }
                }
    }
    wave_sync();
    {
        v4f acc[4][2];
        zero_acc(acc);
        wave_gemm<4, 2, 4>(B.H2, 64, W.w3, 64, acc);
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int ni = 0; ni < 2; ++ni)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int m = 16 * mi + rg + e, n = 16 * ni + col;
                    B.OUT[m * 32 + n] = acc[mi][ni][e] + W.b3[n];
                }
    }
    wave_sync();
}

// Inference for one wave's 64 samples with the activations in registers.
// Each layer forms the transposed product H^T = W X^T (weights as the A
// operand, samples as the 16 columns of an MFMA tile): the lanes then hold
// accumulator rows 4(l/16)..+3 of column l%16, which is exactly how the next
// layer's B operand is laid out, so between layers the activations only pass
// through the bias, SiLU and the rounding to bf16 in place.  Only the input
// rows X (bf16 [64][kXS], 32 used) and the outputs OUT (fp32 [64][kOS], the
// 20 used in columns 0..19) go through LDS; OUT must not overlap X.
__device__ inline float silu_fast(float v) {
    return v * __builtin_amdgcn_rcpf(1.0f + __expf(-v));
}

typedef __bf16 v4bf __attribute__((ext_vector_type(4)));

// Bias, SiLU and rounding to bf16 (to nearest even, the hardware's packed
// conversion) of four accumulator rows.
__device__ inline v4s act_bf16(v4f c, const float *bias, int n0) {
    v4bf h;
#pragma unroll
    for (int e = 0; e < 4; ++e) h[e] = (__bf16)silu_fast(c[e] + bias[n0 + e]);
    return __builtin_bit_cast(v4s, h);
}

__device__ inline void mlp_infer_wave(const InferW &W, const uint16_t *X, float *OUT, int nblk = 4) {
    const int l = threadIdx.x & 63, r = l & 15, kg = (l >> 4) * 4;
#pragma unroll 1
    for (int mt = 0; mt < nblk; ++mt) {
        v4f c1[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) c1[nt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const v4s b = *reinterpret_cast<const v4s *>(X + (16 * mt + r) * kXS + 16 * ks + kg);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const v4s a = W.w1[nt * 2 + ks][l];
                c1[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c1[nt], 0, 0, 0);
            }
        }
        v4s h1[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) h1[nt] = act_bf16(c1[nt], W.b1, 16 * nt + kg);
        v4f c2[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) c2[nt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const v4s a = W.w2[nt * 4 + ks][l];
                c2[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, h1[ks], c2[nt], 0, 0, 0);
            }
        v4s h2[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) h2[nt] = act_bf16(c2[nt], W.b2, 16 * nt + kg);
        v4f c3[2];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) c3[nt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                const v4s a = W.w3[nt * 4 + ks][l];
                c3[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, h2[ks], c3[nt], 0, 0, 0);
            }
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int n = 16 * nt + kg + e;
                OUT[(16 * mt + r) * kOS + n] = c3[nt][e] + W.b3[n];
            }
    }
    wave_sync();
}

// ---------------------------------------------------------------------------
// The mixture for training (fp32): component k of the network output is
// (logit, mu_x, mu_y, a_x, a_y) at 5k..5k+4, width s = exp(clamp(a)).
constexpr float kAMin = -10.0f, kAMax = 1.0f;

struct Gmm {
    float lw[4], mx[4], my[4], ax[4], ay[4];
};

__device__ inline float clampa(float a) { return a < kAMin ? kAMin : (a > kAMax ? kAMax : a); }

__device__ inline Gmm gmm_from(const float *o) {
    Gmm g;
    float mx = o[0];
#pragma unroll
    for (int k = 1; k < 4; ++k) mx = fmaxf(mx, o[5 * k]);
    float z = 0.0f;
#pragma unroll
    for (int k = 0; k < 4; ++k) z += expf(o[5 * k] - mx);
    const float lz = logf(z) + mx;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        g.lw[k] = o[5 * k] - lz;
        g.mx[k] = o[5 * k + 1];
        g.my[k] = o[5 * k + 2];
        g.ax[k] = clampa(o[5 * k + 3]);
        g.ay[k] = clampa(o[5 * k + 4]);
    }
    return g;
}

// ---------------------------------------------------------------------------
// The proposal as a law on the q lattice of displacements D (delta = D q):
//
//   P(D) = e U(D) + (1 - e) G(D),   e = E / 2^32 exactly,
//
// U: the plain trial's step (per axis D = m j, j odd, |j| <= 2^14 - 1, each
// with probability 2^-14); G: component k with probability pi_k, a point of
// N(mu_k, diag(s_k^2)) drawn in double precision from 53-bit uniforms
// (Box-Muller) and rounded to the nearest lattice point, draws with
// |D| > 2^22 - 1 on an axis failing.  The probability of a lattice point
// under one component is the Gaussian mass of its cell, per axis
// (q/s) phi(u) (1 + c), u = (D q - mu)/s, c = h^2 He2(u)/6 + h^4 He4(u)/120,
// h = q/(2s) (even Taylor terms of the cell integral; the next is below
// 2e-14 relative for s >= e^-10 and |u| <= 9).  Everything after the
// network's fp32 outputs is double precision, and the Metropolis-Hastings
// ratio is the ratio of these lattice probabilities.
//
// Words of trial t in cell c, sweep k: A (stream 0): A.w0 selects the disk,
// A.w1 and A.w2 give the uniform step (as in the plain trial), A.w3 < E
// takes U; B (stream 2): (w0, w1) the component uniform, (w2, w3) the
// acceptance uniform; C (stream 4): (w0, w1) u1 in (0, 1], (w2, w3) u2 in
// [0, 1).  A 53-bit uniform from (hi, lo) is ((hi << 21) | (lo >> 11)) 2^-53.
struct Mix {
    double pi[4];        // component weights
    double mx[4], my[4]; // means
    double isx[4], isy[4];  // 1 / s
    float ax[4], ay[4];  // clamped log widths
};

__device__ inline Mix mix_from(const float *o) {
    Mix g;
    double lmax = -INFINITY;
#pragma unroll
    for (int k = 0; k < 4; ++k) lmax = (double)o[5 * k] > lmax ? (double)o[5 * k] : lmax;
    double z = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        g.pi[k] = exp((double)o[5 * k] - lmax);
        z += g.pi[k];
    }
    const double iz = 1.0 / z;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        g.pi[k] *= iz;
        g.mx[k] = (double)o[5 * k + 1];
        g.my[k] = (double)o[5 * k + 2];
        g.ax[k] = clampa(o[5 * k + 3]);
        g.ay[k] = clampa(o[5 * k + 4]);
        g.isx[k] = exp(-(double)g.ax[k]);
        g.isy[k] = exp(-(double)g.ay[k]);
    }
    return g;
}

__device__ inline double u53(uint32_t hi, uint32_t lo) {
    return (double)(((uint64_t)hi << 21) | (lo >> 11)) * 0x1p-53;
}

__device__ inline bool on_step_lattice(int D, uint32_t m) {
    const int j = D / (int)m;
    return j * (int)m == D && (j & 1) != 0 && (j < 0 ? -j : j) <= 16383;
}

// (1 + c) of one axis, with u the normalised offset and is = 1 / s.
__device__ inline double cell_factor(double u2, double is) {
    const double h = (0.5 * kQd) * is;
    const double h2 = h * h;
    const double he2 = u2 - 1.0, he4 = (u2 - 6.0) * u2 + 3.0;
    const double c = h2 * he2 * (1.0 / 6.0) + (h2 * h2) * he4 * (1.0 / 120.0);
    return 1.0 + c;
}

// P(D) of the lattice law (probabilities below 1e-300 round to 0).
__device__ inline double lattice_p(const Mix &g, int Dx, int Dy, uint32_t m, double e) {
    double pu = (on_step_lattice(Dx, m) && on_step_lattice(Dy, m)) ? 0x1p-28 : 0.0;
    double pg = 0.0;
    if ((Dx < 0 ? -Dx : Dx) <= 4194303 && (Dy < 0 ? -Dy : Dy) <= 4194303) {
        const double dx = (double)Dx * kQd, dy = (double)Dy * kQd;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double ux = (dx - g.mx[k]) * g.isx[k], uy = (dy - g.my[k]) * g.isy[k];
            const double ux2 = ux * ux, uy2 = uy * uy;
            pg += g.pi[k] * (g.isx[k] * g.isy[k]) * exp(-0.5 * (ux2 + uy2)) *
                  (cell_factor(ux2, g.isx[k]) * cell_factor(uy2, g.isy[k]));
        }
        pg *= kQd * kQd * (1.0 / 6.283185307179586);
    }
    return e * pu + (1.0 - e) * pg;
}

// Draws D with the words A, B, C; false for a failed Gaussian draw.
__device__ inline bool lattice_draw(const Mix &g, const Words &A, const Words &B, const Words &C,
                                    uint32_t m, uint64_t E, int &Dx, int &Dy) {
    if ((uint64_t)A.w3 < E) {
        Dx = (int)m * (2 * (int)(A.w1 >> 18) + 1 - 16384);
        Dy = (int)m * (2 * (int)(A.w2 >> 18) + 1 - 16384);
        return true;
    }
    // component: the first c with uc below the cumulative weight (3 if none);
    // its parameters are carried along by selects
    const double uc = u53(B.w0, B.w1);
    bool chosen = false;
    double cum = 0.0, mx = g.mx[3], my = g.my[3];
    float ax = g.ax[3], ay = g.ay[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cum += g.pi[c];
        const bool take = !chosen && uc < cum;
        mx = take ? g.mx[c] : mx;
        my = take ? g.my[c] : my;
        ax = take ? g.ax[c] : ax;
        ay = take ? g.ay[c] : ay;
        chosen = chosen || take;
    }
    const double u1 = (double)((((uint64_t)C.w0 << 21) | (C.w1 >> 11)) + 1) * 0x1p-53;
    const double u2 = u53(C.w2, C.w3);
    const double r = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincos(6.283185307179586 * u2, &sn, &cs);
    const double tx = (mx + (exp((double)ax) * r) * cs) * 4194304.0;
    const double ty = (my + (exp((double)ay) * r) * sn) * 4194304.0;
    if (!(fabs(tx) < 4194303.5 && fabs(ty) < 4194303.5)) return false;
    Dx = (int)rint(tx);
    Dy = (int)rint(ty);
    return true;
}

// ---------------------------------------------------------------------------
// The disks of the 3 x 3 cell block around cell (ci, cj) (M >= 4, so the nine
// cells are distinct and the own cell is k = 4, k = 3 (dj + 1) + di + 1):
// the nine counts (3 bits each) and slots 0 and 1 are loaded together, one
// round trip; slots 2 and 3 are read from the lists where a count asks.
constexpr int kExtra = 8;  // slots >= 2 of a 3 x 3 block staged in LDS per lane
struct Nbhd {
    uint32_t m;           // count of cell k in bits 3k..3k+2
    float x[9][2], y[9][2];
    uint32_t ci, cj, M;
    const float2 *ex;     // slots >= 2 in cell order, the first kExtra of them
                          // (NULL: read from the lists)
};

__device__ inline uint32_t nbhd_cell(const Nbhd &N, int k) {
    const uint32_t i = (uint32_t)((int)N.ci + k % 3 - 1 + (int)N.M) % N.M;
    const uint32_t j = (uint32_t)((int)N.cj + k / 3 - 1 + (int)N.M) % N.M;
    return i + N.M * j;
}

__device__ inline void load_nbhd(const uint8_t *cnt, const float *px, const float *py,
                                 uint32_t M, uint32_t ci, uint32_t cj, Nbhd &N) {
    N.ci = ci;
    N.cj = cj;
    N.M = M;
    N.m = 0;
    N.ex = nullptr;
    const uint32_t NC = M * M;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const uint32_t nb = nbhd_cell(N, k);
        N.m |= (uint32_t)cnt[nb] << (3 * k);
        N.x[k][0] = px[nb];
        N.x[k][1] = px[NC + nb];
        N.y[k][0] = py[nb];
        N.y[k][1] = py[NC + nb];
    }
}

// Copies slots 2.. of the nine cells (in cell order, at most kExtra) into
// this lane's LDS area `ex` and points N at it: the neighbourhood is then
// read from registers and LDS only.
__device__ inline void stage_extras(Nbhd &N, const float *px, const float *py, float2 *ex) {
    const uint32_t NC = N.M * N.M;
    // entries before each cell
    uint32_t before[9];
    uint32_t e = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        before[k] = e;
        const uint32_t m = (N.m >> (3 * k)) & 7u;
        e += m > 2 ? m - 2 : 0;
    }
    // entry q is slot 2 + q - before[k] of the last cell k with before[k] <= q;
    // all loads are issued before any is stored, one round trip
    float xs[kExtra], ys[kExtra];
#pragma unroll
    for (int q = 0; q < kExtra; ++q) {
        int k = 0;
        uint32_t bk = 0;
#pragma unroll
        for (int c = 1; c < 9; ++c) {
            const bool later = before[c] <= (uint32_t)q;
            k = later ? c : k;
            bk = later ? before[c] : bk;
        }
        const uint32_t at = slot_at(nbhd_cell(N, k), 2u + (uint32_t)q - bk, NC);
        xs[q] = (uint32_t)q < e ? px[at] : 0.0f;
        ys[q] = (uint32_t)q < e ? py[at] : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < kExtra; ++q)
        if ((uint32_t)q < e) ex[q] = make_float2(xs[q], ys[q]);
    N.ex = ex;
}

// Calls f(dx, dy) for every disk of the block but slot `self` of the own
// cell, in the order of cells k, then slots, with (dx, dy) its separation
// from the point (x, y) of the own cell (each cell's offset c w added last).
template <class F>
__device__ inline void for_each_other(const Nbhd &N, const float *px, const float *py, float w,
                                      uint32_t self, float x, float y, F &&f) {
    const uint32_t NC = N.M * N.M;
    int eb = 0;  // staged entries of the cells before k
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const float cwx = (float)(k % 3 - 1) * w, cwy = (float)(k / 3 - 1) * w;
        const uint32_t m = (N.m >> (3 * k)) & 7u;
#pragma unroll
        for (uint32_t s = 0; s < 2; ++s)
            if (s < m && !(k == 4 && s == self)) f((N.x[k][s] - x) + cwx, (N.y[k][s] - y) + cwy);
        // slots 2.. from the staged copy, beyond it (or without one) from
        // the lists
        for (uint32_t s = 2; s < m; ++s, ++eb) {
            if (k == 4 && s == self) continue;
            float xs, ys;
            if (N.ex && eb < kExtra) {
                const float2 e = N.ex[eb];
                xs = e.x;
                ys = e.y;
            } else {
                const uint32_t nb = nbhd_cell(N, k);
                xs = px[slot_at(nb, s, NC)];
                ys = py[slot_at(nb, s, NC)];
            }
            f((xs - x) + cwx, (ys - y) + cwy);
        }
    }
}

// A 32-entry bf16 input row (64 bytes, 16-byte aligned) set to zero.
__device__ inline void zero_row(uint16_t *row) {
    uint4 *r = reinterpret_cast<uint4 *>(row);
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] = make_uint4(0u, 0u, 0u, 0u);
}

// Features of the disk in slot `self` of the block's own cell at cell-local
// (x, y).  scr: this lane's 36-float scratch.  Writes bf16 into Xrow[0..31]
// and/or fp32 into Frow[0..23] (either may be NULL).  Returns the neighbour
// count.
__device__ inline int lane_features(const Nbhd &N, const float *px, const float *py, float w,
                                    uint32_t self, float x, float y, float *scr, uint16_t *Xrow,
                                    float *Frow) {
    int n = 0;
    for_each_other(N, px, py, w, self, x, y, [&](float dx, float dy) {
        const float r2 = r2_f32(dx, dy);
        if (!(r2 < 9.0f)) return;
        if (n < 12) {
            scr[3 * n] = dx;
            scr[3 * n + 1] = dy;
            scr[3 * n + 2] = r2;
        }
        ++n;
    });
    const int nn = n < 12 ? n : 12;
    // ranks by (r^2, order found), all twelve squared distances read at once
    // and compared in registers; entries from nn on hold +inf and never count
    float r2v[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) r2v[c] = c < nn ? scr[3 * c + 2] : INFINITY;
    if (Xrow) zero_row(Xrow);
    if (Frow)
        for (int k = 0; k < 24; ++k) Frow[k] = 0.0f;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        if (c < nn) {
            // earlier entries count on equal r^2 (order found breaks ties)
            int rank = 0;
#pragma unroll
            for (int e = 0; e < 12; ++e)
                if (e != c) rank += (e < c ? r2v[e] <= r2v[c] : r2v[e] < r2v[c]) ? 1 : 0;
            const float dx = scr[3 * c], dy = scr[3 * c + 1];
            if (Xrow) {
                Xrow[2 * rank] = f2bf(dx);
                Xrow[2 * rank + 1] = f2bf(dy);
            }
            if (Frow) {
                Frow[2 * rank] = dx;
                Frow[2 * rank + 1] = dy;
            }
        }
    }
    return n;
}

// The same from the cell lists directly, for a disk of cell (ci, cj).
__device__ inline int lane_features(const uint8_t *cnt, const float *px, const float *py,
                                    uint32_t M, float w, uint32_t ci, uint32_t cj,
                                    uint32_t self, float x, float y, float *scr, uint16_t *Xrow,
                                    float *Frow) {
    Nbhd N;
    load_nbhd(cnt, px, py, M, ci, cj, N);
    return lane_features(N, px, py, w, self, x, y, scr, Xrow, Frow);
}

// ---------------------------------------------------------------------------
// Learned colour sub-sweep: one wave per 64 active cells, every lane running
// its cell's trials; the two network evaluations of a trial are wave-wide.
struct LearnView {
    const PackedW *W;
    uint64_t E;                      // uniform branch: a 32-bit word below E
    double e;                        // its probability, E / 2^32
    unsigned long long *nfeat_over;  // neighbourhoods with more than 12 disks
    unsigned long long *stamps;      // phase profile (NULL normally): kLearnStamps per wave
    uint32_t cpw;                    // active cells per wave: 16, 32 or 64
};

// Phase profile of the learned pass: lane 0 of each wave records the device
// realtime clock at the start, before the features, after them, after the
// network, after the draw, after the overlap test, after the reverse
// features, after the reverse network, after the acceptance and at the end
// (first trial of the cell only).
constexpr int kLearnStamps = 10;
__device__ __forceinline__ void learn_stamp(const LearnView &lv, int lane, uint32_t tr, int k) {
    if (lv.stamps && lane == 0 && tr == 0)
        lv.stamps[((size_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * kLearnStamps + k] =
            wall_clock64();
}

constexpr int kLearnWaves = 4;  // waves per workgroup of the learned pass

constexpr int kSS = 37;  // per-lane feature scratch stride (floats), odd: no bank conflicts

struct LdsLearn {
    InferW w;  // shared by the workgroup's waves
    struct Wave {
        uint16_t X[64 * kXS];  // network input rows
        float so[64 * kSS];    // feature scratch, then the network output [64][kOS]
        float2 ex[64 * kExtra];  // staged slots >= 2 of each lane's block
    } pw[kLearnWaves];
};

// Copies the inference weights into LDS in fragment order, with all threads
// of the workgroup.
__device__ inline void load_infer_weights(InferW &dstw, const PackedW *W, int tid, int nthreads) {
    for (int i = tid; i < 32 * 64; i += nthreads) {
        const int f = i >> 6, l = i & 63;
        const uint16_t *src;
        v4s *dst;
        int K, nt, ks;
        if (f < 8) {
            nt = f >> 1, ks = f & 1, K = 32, src = W->w1, dst = &dstw.w1[f][l];
        } else if (f < 24) {
            nt = (f - 8) >> 2, ks = (f - 8) & 3, K = 64, src = W->w2, dst = &dstw.w2[f - 8][l];
        } else {
            nt = (f - 24) >> 2, ks = (f - 24) & 3, K = 64, src = W->w3, dst = &dstw.w3[f - 24][l];
        }
        *dst = *reinterpret_cast<const v4s *>(src + (16 * nt + (l & 15)) * K + 16 * ks + 4 * (l >> 4));
    }
    for (int k = tid; k < 64; k += nthreads) {
        dstw.b1[k] = W->b1[k];
        dstw.b2[k] = W->b2[k];
        if (k < 32) dstw.b3[k] = W->b3[k];
    }
}

__global__ void __launch_bounds__(64 * kLearnWaves) k_pass_learned(BoxView v, uint32_t pass,
                                                                   LearnView lv) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    LdsLearn &L = *reinterpret_cast<LdsLearn *>(lds_raw);
    const int lane = threadIdx.x & 63;
    LdsLearn::Wave &P = L.pw[threadIdx.x >> 6];
    learn_stamp(lv, lane, 0, 0);
    // the weights' copy overlaps the first trial's loads and random numbers:
    // the barrier that completes it comes just before the first network
    load_infer_weights(L.w, lv.W, threadIdx.x, 64 * kLearnWaves);
    const uint32_t M = v.M, h = M / 2;
    // wave w of the grid takes active cells w cpw .. w cpw + cpw - 1, one per
    // lane; lanes from cpw on have no cell, and the network runs on cpw / 16
    // blocks of 16 rows
    const uint32_t t = (blockIdx.x * kLearnWaves + (threadIdx.x >> 6)) * lv.cpw + (uint32_t)lane;
    const int nblk = (int)(lv.cpw >> 4);
    const uint64_t sweep = v.dev->sweep + v.offset;
    const SweepDraws sd = sweep_draws(v.seed_lo, v.seed_hi, sweep, v.W);
    const uint32_t colour = colour_of_pass(sd.perm, pass);
    const bool valid = (uint32_t)lane < lv.cpw && t < h * h;
    const uint32_t ci = valid ? 2 * (t % h) + (colour & 1u) : 0;
    const uint32_t cj = valid ? 2 * (t / h) + (colour >> 1) : 0;
    const uint32_t cell = ci + M * cj;
    // the neighbourhood (own cell k = 4 included) in one round trip; it is
    // frozen during a trial and serves the forward features, the overlap
    // test and the reverse features, and it is read again for every further
    // trial of the cell
    Nbhd nbh;
    float2 *ex = P.ex + kExtra * lane;
    if (valid) {
        load_nbhd(v.cnt_out, v.x_out, v.y_out, M, ci, cj, nbh);
        stage_extras(nbh, v.x_out, v.y_out, ex);
    }
    const uint32_t n = valid ? (nbh.m >> 12) & 7u : 0u;
    float *scr = P.so + kSS * lane;  // scratch before the MLP
    uint32_t trials = 0, accepts = 0;
    uint32_t perm = 0x76543210u;
    if (n > 1 && v.n_trial > 1) {
        const Words wd = draw(v.seed_lo, v.seed_hi, sweep, cell, 0, kStreamShuffle);
        const uint32_t wv[4] = {wd.w0, wd.w1, wd.w2, wd.w3};
        for (uint32_t i = n - 1; i >= 1; --i) {
            const uint32_t e = n - 1 - i;
            Words we = wd;
            if (e >= 4) we = draw(v.seed_lo, v.seed_hi, sweep, cell, e / 4, kStreamShuffle);
            const uint32_t q4 = e & 3u;
            const uint32_t word = e < 4 ? wv[e] : (q4 == 0 ? we.w0 : q4 == 1 ? we.w1 : q4 == 2 ? we.w2 : we.w3);
            const uint32_t jj = mulhi32(word, i + 1);
            const uint32_t pi = (perm >> (4 * i)) & 0xFu, pj = (perm >> (4 * jj)) & 0xFu;
            perm &= ~((0xFu << (4 * i)) | (0xFu << (4 * jj)));
            perm |= (pj << (4 * i)) | (pi << (4 * jj));
        }
    }
    for (uint32_t tr = 0; tr < v.n_trial; ++tr) {
        const bool act = n > 0;
        Words wa{0, 0, 0, 0}, wb{0, 0, 0, 0};
        uint32_t slot = 0;
        float x = 0.0f, y = 0.0f;
        if (act && tr > 0) {
            load_nbhd(v.cnt_out, v.x_out, v.y_out, M, ci, cj, nbh);
            stage_extras(nbh, v.x_out, v.y_out, ex);
        }
        if (act) {
            wa = draw(v.seed_lo, v.seed_hi, sweep, cell, tr, kStreamTrial);
            wb = draw(v.seed_lo, v.seed_hi, sweep, cell, tr, kStreamLearned);
            slot = (v.n_trial == 1) ? mulhi32(wa.w0, n) : (perm >> (4 * (tr % n))) & 0xFu;
            x = slot == 0 ? nbh.x[4][0] : slot == 1 ? nbh.x[4][1] : v.x_out[slot_at(cell, slot, M * M)];
            y = slot == 0 ? nbh.y[4][0] : slot == 1 ? nbh.y[4][1] : v.y_out[slot_at(cell, slot, M * M)];
        }
        wave_sync();
        learn_stamp(lv, lane, tr, 1);
        // sorted features into this lane's row of X
        if (act) {
            const int nf = lane_features(nbh, v.x_out, v.y_out, v.w, slot, x, y, scr,
                                         P.X + kXS * lane, nullptr);
            if (nf > 12) atomicAdd(lv.nfeat_over, 1ull);
        } else {
            zero_row(P.X + kXS * lane);
        }
        wave_sync();
        learn_stamp(lv, lane, tr, 2);
        if (tr == 0) __syncthreads();  // the weights are in LDS
        float *OUT = P.so;
        mlp_infer_wave(L.w, P.X, OUT, nblk);
        learn_stamp(lv, lane, tr, 3);
        // propose D from the lattice law and keep P(D)
        int Dx = 0, Dy = 0;
        bool drawn = false;
        double pf = 1.0;
        if (act) {
            const Mix g = mix_from(OUT + kOS * lane);
            const Words wc = (uint64_t)wa.w3 < lv.E
                                 ? Words{0, 0, 0, 0}
                                 : draw(v.seed_lo, v.seed_hi, sweep, cell, tr, kStreamGauss);
            drawn = lattice_draw(g, wa, wb, wc, v.step_m, lv.E, Dx, Dy);
            if (drawn) pf = lattice_p(g, Dx, Dy, v.step_m, lv.e);
        }
        learn_stamp(lv, lane, tr, 4);
        // geometry in q units: exact
        const int U = (int)(x * 4194304.0f) + Dx, V = (int)(y * 4194304.0f) + Dy;
        bool ok = act && drawn && U >= 0 && U < (int)v.W && V >= 0 && V < (int)v.W;
        const float xn = (float)U * kQ, yn = (float)V * kQ;
        if (ok)
            for_each_other(nbh, v.x_out, v.y_out, v.w, slot, xn, yn,
                           [&](float ddx, float ddy) { ok = ok && !overlap_f32(ddx, ddy); });
        // reverse law at x' (every lane takes part in the wave GEMMs)
        wave_sync();
        learn_stamp(lv, lane, tr, 5);
        if (ok) {
            lane_features(nbh, v.x_out, v.y_out, v.w, slot, xn, yn, scr, P.X + kXS * lane, nullptr);
        } else {
            zero_row(P.X + kXS * lane);
        }
        wave_sync();
        learn_stamp(lv, lane, tr, 6);
        mlp_infer_wave(L.w, P.X, OUT, nblk);
        learn_stamp(lv, lane, tr, 7);
        if (act) ++trials;
        if (ok) {
            const Mix gr = mix_from(OUT + kOS * lane);
            const double pr = lattice_p(gr, -Dx, -Dy, v.step_m, lv.e);
            // min(1, pr / pf) against the 53-bit acceptance uniform
            if (pr >= pf || u53(wb.w2, wb.w3) * pf < pr) {
                v.x_out[slot_at(cell, slot, M * M)] = xn;
                v.y_out[slot_at(cell, slot, M * M)] = yn;
                ++accepts;
            }
        }
        wave_sync();
        learn_stamp(lv, lane, tr, 8);
    }
    count_trials(v.dev, trials, accepts);
    learn_stamp(lv, lane, 0, 9);
}

// ---------------------------------------------------------------------------
// Plain colour sub-sweep that also records accepted moves: (f(x) at the old
// position, delta) into the data set.  The trajectory is the plain one.
struct CollectView {
    float *F;       // [cap][24]
    float *D;       // [cap][2]
    unsigned long long *count;
    uint64_t cap;
};

__global__ void __launch_bounds__(128) k_pass_collect(BoxView v, uint32_t pass, CollectView cv) {
    __shared__ float scr_all[128 * 36];
    float *scr = scr_all + 36 * threadIdx.x;
    const uint32_t M = v.M, h = M / 2;
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t sweep = v.dev->sweep + v.offset;
    const SweepDraws sd = sweep_draws(v.seed_lo, v.seed_hi, sweep, v.W);
    const uint32_t colour = colour_of_pass(sd.perm, pass);
    uint32_t trials = 0, accepts = 0;
    if (t < h * h) {
        const uint32_t ci = 2 * (t % h) + (colour & 1u), cj = 2 * (t / h) + (colour >> 1);
        const uint32_t cell = ci + M * cj;
        const uint32_t n = v.cnt_out[cell];
        uint32_t perm = 0x76543210u;
        if (n > 1 && v.n_trial > 1) {
            const Words wd = draw(v.seed_lo, v.seed_hi, sweep, cell, 0, kStreamShuffle);
            const uint32_t wv[4] = {wd.w0, wd.w1, wd.w2, wd.w3};
            for (uint32_t i = n - 1; i >= 1; --i) {
                const uint32_t e = n - 1 - i;
                Words we = wd;
                if (e >= 4) we = draw(v.seed_lo, v.seed_hi, sweep, cell, e / 4, kStreamShuffle);
                const uint32_t q4 = e & 3u;
                const uint32_t word = e < 4 ? wv[e] : (q4 == 0 ? we.w0 : q4 == 1 ? we.w1 : q4 == 2 ? we.w2 : we.w3);
                const uint32_t jj = mulhi32(word, i + 1);
                const uint32_t pi = (perm >> (4 * i)) & 0xFu, pj = (perm >> (4 * jj)) & 0xFu;
                perm &= ~((0xFu << (4 * i)) | (0xFu << (4 * jj)));
                perm |= (pj << (4 * i)) | (pi << (4 * jj));
            }
        }
        for (uint32_t tr = 0; tr < v.n_trial && n > 0; ++tr) {
            const Words w4 = draw(v.seed_lo, v.seed_hi, sweep, cell, tr, kStreamTrial);
            const uint32_t slot = (v.n_trial == 1) ? mulhi32(w4.w0, n) : (perm >> (4 * (tr % n))) & 0xFu;
            const uint32_t k = slot_at(cell, slot, M * M);
            const float dx = step_from_word(w4.w1, v.step_m), dy = step_from_word(w4.w2, v.step_m);
            const float x = v.x_out[k], y = v.y_out[k];
            const float xn = x + dx, yn = y + dy;
            ++trials;
            if (!(xn >= 0.0f && xn < v.w && yn >= 0.0f && yn < v.w)) continue;
            bool bad = false;
            for (int dj = -1; dj <= 1 && !bad; ++dj)
                for (int di = -1; di <= 1 && !bad; ++di) {
                    const uint32_t i = (uint32_t)((int)ci + di + (int)M) % M;
                    const uint32_t j = (uint32_t)((int)cj + dj + (int)M) % M;
                    const uint32_t nb = i + M * j;
                    const float cwx = (float)di * v.w, cwy = (float)dj * v.w;
                    const uint32_t m = v.cnt_out[nb];
                    for (uint32_t s = 0; s < m; ++s) {
                        if (nb == cell && s == slot) continue;
                        const float ddx = (v.x_out[slot_at(nb, s, M * M)] - xn) + cwx;
                        const float ddy = (v.y_out[slot_at(nb, s, M * M)] - yn) + cwy;
                        if (overlap_f32(ddx, ddy)) { bad = true; break; }
                    }
                }
            if (bad) continue;
            const unsigned long long idx = atomicAdd(cv.count, 1ull);
            if (idx < cv.cap) {
                lane_features(v.cnt_out, v.x_out, v.y_out, M, v.w, ci, cj, slot, x, y, scr,
                              nullptr, cv.F + idx * 24);
                cv.D[2 * idx] = dx;
                cv.D[2 * idx + 1] = dy;
            }
            v.x_out[k] = xn;
            v.y_out[k] = yn;
            ++accepts;
        }
    }
    count_trials(v.dev, trials, accepts);
}

// Features of selected disks at their current positions (diagnostic): the
// disk of tag t goes to row row_of[t] (or nowhere if -1).
__global__ void k_features(const uint8_t *cnt, const float *px, const float *py, const uint32_t *tag,
                           uint32_t M, uint32_t CS, float w, const int32_t *row_of, float *F) {
    __shared__ float scr_all[256 * 36];
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t s = gid / (M * M), cell = gid - s * (M * M);
    if (s >= CS || s >= cnt[cell]) return;
    const int32_t r = row_of[tag[gid]];
    if (r < 0) return;
    lane_features(cnt, px, py, M, w, cell % M, cell / M, s, px[gid], py[gid],
                  scr_all + 36 * threadIdx.x, nullptr, F + (size_t)r * 24);
}

// ---------------------------------------------------------------------------
// Training: one wave per 64 samples, forward with saved activations, the
// gradient of the mean negative log-likelihood, backward GEMMs on the matrix
// cores, gradients accumulated into an fp32 buffer.
struct LdsTrain {
    PackedW w;
    uint16_t X[64 * 32], XT[32 * 64];
    uint16_t H1[64 * 64], H1T[64 * 64];
    uint16_t H2[64 * 64], H2T[64 * 64];
    float A1[64 * 64], A2[64 * 64];
    float OUT[64 * 32];
    uint16_t DO[64 * 32], DOT[32 * 64];
};

struct TrainView {
    const PackedW *W;
    const float *F, *D;           // data set
    uint64_t n_data;              // samples in the data set
    const uint32_t *index;        // explicit sample list (or NULL: Philox draws)
    uint32_t batch;               // samples in this step (mean over these)
    uint32_t seed_lo, seed_hi;
    uint32_t step;
    float *grad;                  // [7060] accumulated
    double *loss;                 // accumulated sum of NLL
};

__global__ void __launch_bounds__(64) k_train(TrainView tv) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    LdsTrain &L = *reinterpret_cast<LdsTrain *>(lds_raw);
    const int lane = threadIdx.x, col = lane & 15, rg = (lane >> 4) * 4;
    {
        const uint32_t *src = reinterpret_cast<const uint32_t *>(tv.W);
        uint32_t *dst = reinterpret_cast<uint32_t *>(&L.w);
        for (uint32_t k = lane; k < sizeof(PackedW) / 4; k += 64) dst[k] = src[k];
    }
    // this lane's sample
    const uint32_t sidx = blockIdx.x * 64 + lane;
    const bool live = sidx < tv.batch;
    uint64_t di = 0;
    if (live) {
        if (tv.index) {
            di = tv.index[sidx];
        } else {
            const Words wd = philox(tv.seed_lo, tv.seed_hi, tv.step, sidx, 0, kStreamTrain);
            di = (((uint64_t)wd.w0 << 32) | wd.w1) % tv.n_data;
        }
    }
    float f[24];
    for (int k = 0; k < 24; ++k) f[k] = live ? tv.F[di * 24 + k] : 0.0f;
    const float ddx = live ? tv.D[2 * di] : 0.0f, ddy = live ? tv.D[2 * di + 1] : 0.0f;
    for (int k = 0; k < 32; ++k) {
        const uint16_t b = k < 24 ? f2bf(f[k]) : 0;
        L.X[32 * lane + k] = b;
        L.XT[k * 64 + lane] = b;
    }
    __syncthreads();
    FwdBufs fb{L.X, L.H1, L.H2, L.XT, L.H1T, L.H2T, L.A1, L.A2, L.OUT};
    mlp_forward_wave(L.w, fb);
    // d(-log q_GMM)/d out for this sample, scaled by 1/batch
    const float inv = 1.0f / (float)tv.batch;
    float dout[20];
    {
        const float *o = L.OUT + 32 * lane;
        const Gmm g = gmm_from(o);
        float l[4], best = -INFINITY, ux[4], uy[4];
        for (int k = 0; k < 4; ++k) {
            ux[k] = (ddx - g.mx[k]) * expf(-g.ax[k]);
            uy[k] = (ddy - g.my[k]) * expf(-g.ay[k]);
            l[k] = g.lw[k] - 1.8378770664093453f - g.ax[k] - g.ay[k] - 0.5f * (ux[k] * ux[k] + uy[k] * uy[k]);
            best = fmaxf(best, l[k]);
        }
        float s = 0.0f;
        for (int k = 0; k < 4; ++k) s += expf(l[k] - best);
        const float lse = best + logf(s);
        for (int k = 0; k < 4; ++k) {
            const float r = expf(l[k] - lse), pk = expf(g.lw[k]);
            const float inx = (o[5 * k + 3] > kAMin && o[5 * k + 3] < kAMax) ? 1.0f : 0.0f;
            const float iny = (o[5 * k + 4] > kAMin && o[5 * k + 4] < kAMax) ? 1.0f : 0.0f;
            dout[5 * k] = (pk - r) * inv;
            dout[5 * k + 1] = -r * ux[k] * expf(-g.ax[k]) * inv;
            dout[5 * k + 2] = -r * uy[k] * expf(-g.ay[k]) * inv;
            dout[5 * k + 3] = -r * (ux[k] * ux[k] - 1.0f) * inx * inv;
            dout[5 * k + 4] = -r * (uy[k] * uy[k] - 1.0f) * iny * inv;
        }
        double nll = live ? -(double)lse : 0.0;
        for (int off = 32; off > 0; off >>= 1) nll += __shfl_xor(nll, off, 64);
        if (lane == 0) atomicAdd(tv.loss, nll);
    }
    for (int k = 0; k < 32; ++k) {
        const float gk = (live && k < 20) ? dout[k < 20 ? k : 0] : 0.0f;
        const uint16_t b = f2bf(gk);
        L.DO[32 * lane + k] = b;
        L.DOT[k * 64 + lane] = b;
    }
    // db3: sum over the samples
    for (int k = 0; k < 20; ++k) {
        float gk = live ? dout[k] : 0.0f;
        for (int off = 32; off > 0; off >>= 1) gk += __shfl_xor(gk, off, 64);
        if (lane == 0) atomicAdd(&tv.grad[kPB3 + k], gk);
    }
    __syncthreads();
    // dW3[o][i] = sum_s dOut[s][o] H2[s][i]
    {
        v4f acc[2][4];
        zero_acc(acc);
        wave_gemm<2, 4, 4>(L.DOT, 64, L.H2T, 64, acc);
        for (int mi = 0; mi < 2; ++mi)
            for (int ni = 0; ni < 4; ++ni)
                for (int e = 0; e < 4; ++e) {
                    const int o = 16 * mi + rg + e, i = 16 * ni + col;
                    if (o < 20) atomicAdd(&tv.grad[kPW3 + o * 64 + i], acc[mi][ni][e]);
                }
    }
    // dH2[s][i] = sum_o dOut[s][o] W3[o][i]; dA2 = dH2 * silu'(A2), stored
    // over H2 (row-major) and H2T (transposed)
    {
        v4f acc[4][4];
        zero_acc(acc);
        wave_gemm<4, 4, 2>(L.DO, 32, L.w.w3t, 32, acc);
        __syncthreads();
        for (int ni = 0; ni < 4; ++ni) {
            float cs = 0.0f;
            for (int mi = 0; mi < 4; ++mi)
                for (int e = 0; e < 4; ++e) {
                    const int s = 16 * mi + rg + e, i = 16 * ni + col;
                    const float dA = acc[mi][ni][e] * dsilu(L.A2[s * 64 + i]);
                    cs += dA;
                    const uint16_t b = f2bf(dA);
                    L.H2[s * 64 + i] = b;
                    L.H2T[i * 64 + s] = b;
                }
            cs += __shfl_xor(cs, 16, 64);
            cs += __shfl_xor(cs, 32, 64);
            if (lane < 16) atomicAdd(&tv.grad[kPB2 + 16 * ni + col], cs);
        }
    }
    __syncthreads();
    // dW2[o][i] = sum_s dA2[s][o] H1[s][i]
    {
        v4f acc[4][4];
        zero_acc(acc);
        wave_gemm<4, 4, 4>(L.H2T, 64, L.H1T, 64, acc);
        for (int mi = 0; mi < 4; ++mi)
            for (int ni = 0; ni < 4; ++ni)
                for (int e = 0; e < 4; ++e) {
                    const int o = 16 * mi + rg + e, i = 16 * ni + col;
                    atomicAdd(&tv.grad[kPW2 + o * 64 + i], acc[mi][ni][e]);
                }
    }
    // dH1[s][i] = sum_o dA2[s][o] W2[o][i]; dA1 = dH1 * silu'(A1), stored
    // transposed over H1T
    {
        v4f acc[4][4];
        zero_acc(acc);
        wave_gemm<4, 4, 4>(L.H2, 64, L.w.w2t, 64, acc);
        __syncthreads();
        for (int ni = 0; ni < 4; ++ni) {
            float cs = 0.0f;
            for (int mi = 0; mi < 4; ++mi)
                for (int e = 0; e < 4; ++e) {
                    const int s = 16 * mi + rg + e, i = 16 * ni + col;
                    const float dA = acc[mi][ni][e] * dsilu(L.A1[s * 64 + i]);
                    cs += dA;
                    L.H1T[i * 64 + s] = f2bf(dA);
                }
            cs += __shfl_xor(cs, 16, 64);
            cs += __shfl_xor(cs, 32, 64);
            if (lane < 16) atomicAdd(&tv.grad[kPB1 + 16 * ni + col], cs);
        }
    }
    __syncthreads();
    // dW1[o][i] = sum_s dA1[s][o] X[s][i]
    {
        v4f acc[4][2];
        zero_acc(acc);
        wave_gemm<4, 2, 4>(L.H1T, 64, L.XT, 64, acc);
        for (int mi = 0; mi < 4; ++mi)
            for (int ni = 0; ni < 2; ++ni)
                for (int e = 0; e < 4; ++e) {
                    const int o = 16 * mi + rg + e, i = 16 * ni + col;
                    if (i < 24) atomicAdd(&tv.grad[kPW1 + o * 24 + i], acc[mi][ni][e]);
                }
    }
}

// Forward only, for given features (diagnostic): out[B][20].
// It runs the sampler's inference path (mlp_infer_wave).
struct LdsForward {
    InferW w;
    uint16_t X[64 * kXS];
    float OUT[64 * kOS];
};

__global__ void __launch_bounds__(64) k_forward(const PackedW *W, const float *F, uint32_t B,
                                                float *out) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    LdsForward &L = *reinterpret_cast<LdsForward *>(lds_raw);
    const int lane = threadIdx.x;
    load_infer_weights(L.w, W, lane, 64);
    const uint32_t s = blockIdx.x * 64 + lane;
    for (int k = 0; k < 32; ++k) L.X[kXS * lane + k] = (s < B && k < 24) ? f2bf(F[(size_t)s * 24 + k]) : 0;
    __syncthreads();
    mlp_infer_wave(L.w, L.X, L.OUT);
    if (s < B)
        for (int k = 0; k < 20; ++k) out[(size_t)s * 20 + k] = L.OUT[kOS * lane + k];
}

// Adam on the fp32 master vector; rewrites the packed bf16 weights and
// clears the gradient.
__global__ void k_adam(float *p, float *m, float *vv, float *grad, PackedW *W, uint32_t step,
                       float lr, int update) {
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (uint32_t)kNPARAM) return;
    float x = p[e];
    if (update) {
        const float g = grad[e];
        const float b1 = 0.9f, b2 = 0.999f;
        const float mm = b1 * m[e] + (1.0f - b1) * g;
        const float v2 = b2 * vv[e] + (1.0f - b2) * g * g;
        m[e] = mm;
        vv[e] = v2;
        const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
        x -= lr * (mm / c1) / (sqrtf(v2 / c2) + 1e-8f);
        p[e] = x;
    }
    grad[e] = 0.0f;
    const uint16_t b = f2bf(x);
    if (e < (uint32_t)kPB1) {
        const uint32_t o = e / 24, i = e % 24;
        W->w1[o * 32 + i] = b;
    } else if (e < (uint32_t)kPW2) {
        W->b1[e - kPB1] = x;
    } else if (e < (uint32_t)kPB2) {
        const uint32_t o = (e - kPW2) / 64, i = (e - kPW2) % 64;
        W->w2[o * 64 + i] = b;
        W->w2t[i * 64 + o] = b;
    } else if (e < (uint32_t)kPW3) {
        W->b2[e - kPB2] = x;
    } else if (e < (uint32_t)kPB3) {
        const uint32_t o = (e - kPW3) / 64, i = (e - kPW3) % 64;
        W->w3[o * 64 + i] = b;
        W->w3t[i * 32 + o] = b;
    } else {
        W->b3[e - kPB3] = x;
    }
}

// Diagnostics of the lattice law: n draws from one fixed network output with
// the words of counter (sweep 0, cell i, trial 0), and P(D) at given points.
__global__ void k_lattice_propose(const float *out, uint32_t m, uint64_t E, double e, uint32_t k0,
                                  uint32_t k1, uint32_t n, int32_t *D, uint8_t *drawn, double *lp) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Mix g = mix_from(out);
    const Words A = draw(k0, k1, 0, i, 0, kStreamTrial);
    const Words B = draw(k0, k1, 0, i, 0, kStreamLearned);
    const Words Cw = draw(k0, k1, 0, i, 0, kStreamGauss);
    int Dx = 0, Dy = 0;
    const bool ok = lattice_draw(g, A, B, Cw, m, E, Dx, Dy);
    D[2 * i] = ok ? Dx : 0;
    D[2 * i + 1] = ok ? Dy : 0;
    drawn[i] = ok ? 1 : 0;
    lp[i] = ok ? log(lattice_p(g, Dx, Dy, m, e)) : __builtin_nan("");
}

__global__ void k_lattice_p(const float *out, const int32_t *D, uint32_t n, uint32_t m, double e,
                            double *lp) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Mix g = mix_from(out + (size_t)20 * i);
    lp[i] = log(lattice_p(g, D[2 * i], D[2 * i + 1], m, e));
}

}  // namespace mpmc

// ===========================================================================
// host side
using namespace mpmc;

#define HIPCHK(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(MPMC_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));           \
    } while (0)

// E: the uniform branch is taken when a 32-bit word is below E, the
// nearest integer to eps 2^32 (0 <= E <= 2^32).
static uint64_t branch_threshold(float eps) {
    return (uint64_t)llrint((double)eps * 4294967296.0);
}

namespace {
struct Learner {
    hipStream_t stream = nullptr;
    uint64_t seed = 0;
    float *p = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    PackedW *W = nullptr;
    double *loss = nullptr;
    float *F = nullptr, *D = nullptr;
    unsigned long long *count = nullptr, *over = nullptr;
    uint64_t cap = 0;
    uint32_t step = 0;
    std::vector<void *> allocs;

    int alloc(void **q, size_t n) {
        hipError_t e = hipMalloc(q, n ? n : 4);
        if (e != hipSuccess) return fail(MPMC_ENOMEM, "hipMalloc(%zu): %s", n, hipGetErrorString(e));
        allocs.push_back(*q);
        return MPMC_OK;
    }
    void release() {
        for (void *q : allocs) (void)hipFree(q);
        allocs.clear();
    }
    // re-pack bf16 weights from the master vector without an update
    int pack() {
        k_adam<<<(kNPARAM + 255) / 256, 256, 0, stream>>>(p, m, v, grad, W, 1, 0.0f, 0);
        HIPCHK(hipGetLastError());
        return MPMC_OK;
    }
};
Learner *LR(mpmc_learner l) { return reinterpret_cast<Learner *>(l); }
Box *BX(mpmc_box b) { return reinterpret_cast<Box *>(b); }

// Default initialisation: weights uniform in +-1/sqrt(fan_in) from Philox
// words, biases zero except the log widths of the mixture, log(0.05).
void default_params(uint64_t seed, std::vector<float> &P) {
    P.assign(kNPARAM, 0.0f);
    auto uni = [&](uint32_t i) {
        const Words w = philox((uint32_t)seed, (uint32_t)(seed >> 32), i, 0, 0, 6);
        return ((float)(w.w0 >> 8) + 0.5f) * (1.0f / 16777216.0f) * 2.0f - 1.0f;
    };
    for (int e = kPW1; e < kPB1; ++e) P[e] = uni(e) / sqrtf(24.0f);
    for (int e = kPW2; e < kPB2; ++e) P[e] = uni(e) / sqrtf(64.0f);
    for (int e = kPW3; e < kPB3; ++e) P[e] = 0.1f * uni(e) / sqrtf(64.0f);
    for (int k = 0; k < 4; ++k) {
        P[kPB3 + 5 * k + 3] = logf(0.05f);
        P[kPB3 + 5 * k + 4] = logf(0.05f);
    }
}
}  // namespace

extern "C" int mpmc_learner_create(mpmc_learner *out, uint64_t seed, uint64_t capacity,
                                   void *stream) {
    if (!out) return fail(MPMC_EINVAL, "out is NULL");
    *out = nullptr;
    Learner *l = new Learner();
    l->stream = (hipStream_t)stream;
    l->seed = seed;
    l->cap = capacity;
    int rc = MPMC_OK;
    for (float **q : {&l->p, &l->m, &l->v, &l->grad})
        if (!rc) rc = l->alloc((void **)q, kNPARAM * 4);
    if (!rc) rc = l->alloc((void **)&l->W, sizeof(PackedW));
    if (!rc) rc = l->alloc((void **)&l->loss, 8);
    if (!rc) rc = l->alloc((void **)&l->count, 16);
    if (!rc) rc = l->alloc((void **)&l->F, capacity * 24 * 4);
    if (!rc) rc = l->alloc((void **)&l->D, capacity * 2 * 4);
    if (rc) {
        l->release();
        delete l;
        return rc;
    }
    l->over = l->count + 1;
    std::vector<float> P;
    default_params(seed, P);
    hipError_t e = hipMemsetAsync(l->W, 0, sizeof(PackedW), l->stream);
    for (float *q : {l->m, l->v, l->grad})
        if (e == hipSuccess) e = hipMemsetAsync(q, 0, kNPARAM * 4, l->stream);
    if (e == hipSuccess) e = hipMemsetAsync(l->count, 0, 16, l->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(l->p, P.data(), kNPARAM * 4, hipMemcpyHostToDevice, l->stream);
    if (e != hipSuccess) {
        l->release();
        delete l;
        return fail(MPMC_EDEVICE, "learner set-up: %s", hipGetErrorString(e));
    }
    rc = l->pack();
    if (rc == MPMC_OK && hipStreamSynchronize(l->stream) != hipSuccess) rc = fail(MPMC_EDEVICE, "sync");
    if (rc) {
        l->release();
        delete l;
        return rc;
    }
    *out = reinterpret_cast<mpmc_learner>(l);
    return MPMC_OK;
}

extern "C" int mpmc_learner_free(mpmc_learner lh) {
    if (!lh) return MPMC_OK;
    (void)hipStreamSynchronize(LR(lh)->stream);
    LR(lh)->release();
    delete LR(lh);
    return MPMC_OK;
}

extern "C" int mpmc_learner_set_params(mpmc_learner lh, const float *params) {
    if (!lh || !params) return fail(MPMC_EINVAL, "NULL argument");
    Learner *l = LR(lh);
    HIPCHK(hipMemcpyAsync(l->p, params, kNPARAM * 4, hipMemcpyHostToDevice, l->stream));
    HIPCHK(hipMemsetAsync(l->m, 0, kNPARAM * 4, l->stream));
    HIPCHK(hipMemsetAsync(l->v, 0, kNPARAM * 4, l->stream));
    l->step = 0;
    int rc = l->pack();
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(l->stream));
    return MPMC_OK;
}

extern "C" int mpmc_learner_get_params(mpmc_learner lh, float *params) {
    if (!lh || !params) return fail(MPMC_EINVAL, "NULL argument");
    Learner *l = LR(lh);
    HIPCHK(hipMemcpyAsync(params, l->p, kNPARAM * 4, hipMemcpyDeviceToHost, l->stream));
    HIPCHK(hipStreamSynchronize(l->stream));
    return MPMC_OK;
}

static int check_learned_box(Box *b) {
    if ((double)b->g.w < 3.0)
        return fail(MPMC_EINVAL, "the learned proposal needs cells of width >= 3 sigma "
                                 "(create the box with cell_min = 3)");
    if (!b->placed) return fail(MPMC_ESTATE, "no configuration");
    if (b->in_batch) return fail(MPMC_ESTATE, "batch members are swept by the batch");
    return MPMC_OK;
}

extern "C" int mpmc_learner_collect(mpmc_learner lh, mpmc_box bh, uint64_t sweeps, uint64_t *n_total) {
    if (!lh || !bh) return fail(MPMC_EINVAL, "NULL argument");
    Learner *l = LR(lh);
    Box *b = BX(bh);
    int rc = check_learned_box(b);
    if (rc) return rc;
    CollectView cv{l->F, l->D, l->count, l->cap};
    const uint32_t na = (b->g.M / 2) * (b->g.M / 2);
    for (uint64_t s = 0; s < sweeps; ++s) {
        BoxView v = b->view(b->cur);
        const BoxView pv = in_place(v);
        for (uint32_t p = 0; p < 4; ++p) k_pass_collect<<<(na + 127) / 128, 128, 0, b->stream>>>(pv, p, cv);
        v.offset = 1;  // binned for the next sweep
        launch_rebin(v, b->stream);
        launch_advance(b->dev, (uint32_t)b->seed, (uint32_t)(b->seed >> 32), (uint32_t)b->g.W, b->g.Lq,
                       1, b->stream);
        HIPCHK(hipGetLastError());
        b->cur ^= 1;
        b->canon_in_c = false;
    }
    if (n_total) {
        unsigned long long c = 0;
        HIPCHK(hipMemcpyAsync(&c, l->count, 8, hipMemcpyDeviceToHost, b->stream));
        HIPCHK(hipStreamSynchronize(b->stream));
        *n_total = c < l->cap ? c : l->cap;
    }
    return MPMC_OK;
}

extern "C" int mpmc_learner_train(mpmc_learner lh, uint32_t steps, uint32_t batch, float lr,
                                  double *mean_loss) {
    if (!lh || batch == 0) return fail(MPMC_EINVAL, "bad arguments");
    Learner *l = LR(lh);
    unsigned long long n = 0;
    HIPCHK(hipMemcpyAsync(&n, l->count, 8, hipMemcpyDeviceToHost, l->stream));
    HIPCHK(hipStreamSynchronize(l->stream));
    if (n > l->cap) n = l->cap;
    if (n == 0) return fail(MPMC_ESTATE, "the data set is empty: collect moves first");
    const size_t lds = sizeof(LdsTrain);
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)k_train, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        attr = true;
    }
    double last = 0.0;
    for (uint32_t s = 0; s < steps; ++s) {
        ++l->step;
        TrainView tv{l->W, l->F, l->D, n, nullptr, batch, (uint32_t)l->seed, (uint32_t)(l->seed >> 32),
                     l->step, l->grad, l->loss};
        HIPCHK(hipMemsetAsync(l->loss, 0, 8, l->stream));
        k_train<<<(batch + 63) / 64, 64, lds, l->stream>>>(tv);
        k_adam<<<(kNPARAM + 255) / 256, 256, 0, l->stream>>>(l->p, l->m, l->v, l->grad, l->W, l->step, lr, 1);
        HIPCHK(hipGetLastError());
        if (s + 1 == steps) {
            HIPCHK(hipMemcpyAsync(&last, l->loss, 8, hipMemcpyDeviceToHost, l->stream));
            HIPCHK(hipStreamSynchronize(l->stream));
        }
    }
    if (mean_loss) *mean_loss = last / batch;
    return MPMC_OK;
}

extern "C" int mpmc_learner_forward(mpmc_learner lh, const float *F, uint32_t B, float *out) {
    if (!lh || !F || !out || B == 0) return fail(MPMC_EINVAL, "bad arguments");
    Learner *l = LR(lh);
    float *dF = nullptr, *dO = nullptr;
    HIPCHK(hipMalloc((void **)&dF, (size_t)B * 24 * 4));
    hipError_t e = hipMalloc((void **)&dO, (size_t)B * 20 * 4);
    if (e == hipSuccess) e = hipMemcpyAsync(dF, F, (size_t)B * 24 * 4, hipMemcpyHostToDevice, l->stream);
    const size_t lds = sizeof(LdsForward);
    if (e == hipSuccess) {
        e = hipFuncSetAttribute((const void *)k_forward, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        k_forward<<<(B + 63) / 64, 64, lds, l->stream>>>(l->W, dF, B, dO);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(out, dO, (size_t)B * 20 * 4, hipMemcpyDeviceToHost, l->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(l->stream);
    (void)hipFree(dF);
    if (dO) (void)hipFree(dO);
    if (e != hipSuccess) return fail(MPMC_EDEVICE, "forward: %s", hipGetErrorString(e));
    return MPMC_OK;
}

extern "C" int mpmc_learner_nll_grad(mpmc_learner lh, const float *F, const float *D, uint32_t B,
                                     float *grad, double *loss) {
    if (!lh || !F || !D || !grad || B == 0) return fail(MPMC_EINVAL, "bad arguments");
    Learner *l = LR(lh);
    float *dF = nullptr, *dD = nullptr;
    uint32_t *idx = nullptr;
    HIPCHK(hipMalloc((void **)&dF, (size_t)B * 24 * 4));
    hipError_t e = hipMalloc((void **)&dD, (size_t)B * 2 * 4);
    if (e == hipSuccess) e = hipMalloc((void **)&idx, (size_t)B * 4);
    std::vector<uint32_t> hi(B);
    for (uint32_t i = 0; i < B; ++i) hi[i] = i;
    if (e == hipSuccess) e = hipMemcpyAsync(dF, F, (size_t)B * 24 * 4, hipMemcpyHostToDevice, l->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dD, D, (size_t)B * 2 * 4, hipMemcpyHostToDevice, l->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(idx, hi.data(), (size_t)B * 4, hipMemcpyHostToDevice, l->stream);
    if (e == hipSuccess) e = hipMemsetAsync(l->grad, 0, kNPARAM * 4, l->stream);
    if (e == hipSuccess) e = hipMemsetAsync(l->loss, 0, 8, l->stream);
    const size_t lds = sizeof(LdsTrain);
    if (e == hipSuccess) {
        e = hipFuncSetAttribute((const void *)k_train, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        TrainView tv{l->W, dF, dD, B, idx, B, 0, 0, 0, l->grad, l->loss};
        k_train<<<(B + 63) / 64, 64, lds, l->stream>>>(tv);
        e = hipGetLastError();
    }
    double sum = 0.0;
    if (e == hipSuccess) e = hipMemcpyAsync(grad, l->grad, kNPARAM * 4, hipMemcpyDeviceToHost, l->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&sum, l->loss, 8, hipMemcpyDeviceToHost, l->stream);
    if (e == hipSuccess) e = hipMemsetAsync(l->grad, 0, kNPARAM * 4, l->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(l->stream);
    (void)hipFree(dF);
    if (dD) (void)hipFree(dD);
    if (idx) (void)hipFree(idx);
    if (e != hipSuccess) return fail(MPMC_EDEVICE, "nll_grad: %s", hipGetErrorString(e));
    if (loss) *loss = sum / B;
    return MPMC_OK;
}

extern "C" int mpmc_learned_features(mpmc_box bh, const uint32_t *tags, uint32_t n, float *F) {
    if (!bh || !tags || !F || n == 0) return fail(MPMC_EINVAL, "bad arguments");
    Box *b = BX(bh);
    if ((double)b->g.w < 3.0) return fail(MPMC_EINVAL, "features need cells of width >= 3 sigma");
    std::vector<int32_t> row(b->N, -1);
    for (uint32_t i = 0; i < n; ++i) {
        if (tags[i] >= b->N) return fail(MPMC_EINVAL, "tag %u out of range", tags[i]);
        row[tags[i]] = (int32_t)i;
    }
    int32_t *drow = nullptr;
    float *dF = nullptr;
    HIPCHK(hipMalloc((void **)&drow, (size_t)b->N * 4));
    hipError_t e = hipMalloc((void **)&dF, (size_t)n * 24 * 4);
    if (e == hipSuccess) e = hipMemcpyAsync(drow, row.data(), (size_t)b->N * 4, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(dF, 0, (size_t)n * 24 * 4, b->stream);
    if (e == hipSuccess) {
        const uint32_t tot = b->g.M * b->g.M * b->g.CS;
        const CellBuf cb = b->canon();
        k_features<<<(tot + 255) / 256, 256, 0, b->stream>>>(cb.cnt, cb.x, cb.y, cb.tag, b->g.M, b->g.CS,
                                                             b->g.w, drow, dF);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(F, dF, (size_t)n * 24 * 4, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    (void)hipFree(drow);
    if (dF) (void)hipFree(dF);
    if (e != hipSuccess) return fail(MPMC_EDEVICE, "features: %s", hipGetErrorString(e));
    return MPMC_OK;
}

// k learned sweeps of box b: four colour passes, the re-bin and the counter
// update per sweep.  With `stamps` (room for the waves of one pass) each
// sweep is synchronised and the phase durations of every wave of every pass
// are added to phase_ticks[kLearnStamps - 1].
// Active cells per wave of the learned pass.  A wave's time is mostly the
// latency of its per-lane work (one wave runs per SIMD), and its network
// part shrinks with the rows it holds, so a pass that would not give every
// SIMD a wave of 64 cells spreads its cells over more waves of 16 or 32:
// the smallest of 16, 32 that needs no more waves than the GPU has SIMDs,
// else 64.  A box's own setting (mpmc_set_learned_cells_per_wave) wins.
// The trajectory does not depend on it: random numbers are keyed by cell,
// and each network row is computed on its own.
static uint32_t learned_cells_per_wave(const Box *b, uint32_t na) {
    if (b->learned_cpw) return b->learned_cpw;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    const uint32_t simds = 4u * (uint32_t)cus;
    for (uint32_t c = 16; c < 64; c *= 2)
        if ((na + c - 1) / c <= simds) return c;
    return 64;
}

// Workgroups of kLearnWaves waves for na active cells at cpw cells per wave.
static uint32_t learned_grid(uint32_t na, uint32_t cpw) {
    const uint32_t waves = (na + cpw - 1) / cpw;
    return (waves + kLearnWaves - 1) / kLearnWaves;
}

// A run of learned sweeps replays a captured graph of this many sweeps (even:
// the double-buffered lists return to the buffer they started in) while the
// box uses graphs; shorter remainders are launched one sweep at a time.
constexpr uint32_t kLearnGraphSweeps = 8;

// Learned sweep j of a run that starts at the device's sweep counter with the
// lists in P[from]: the four colour passes update those lists in place, then
// the re-bin writes them into the other buffer in the grid of sweep j + 1.
// The counter is advanced by the caller.
static void launch_learned_sweep(Box *b, int from, uint32_t j, const LearnView &lv, uint32_t grid,
                                 size_t lds, hipStream_t st) {
    BoxView v = b->view(from);
    v.offset = j;
    const BoxView pv = in_place(v);
    for (uint32_t p = 0; p < 4; ++p) k_pass_learned<<<grid, 64 * kLearnWaves, lds, st>>>(pv, p, lv);
    v.offset = j + 1;
    launch_rebin(v, st);
}

// The box's graph of kLearnGraphSweeps learned sweeps from P[0] and the
// counter update after them, captured again when the learner or the branch
// threshold differs from the last capture.
static int learned_graph(Box *b, const LearnView &lv, uint32_t grid, size_t lds) {
    if (b->lgraph_exec && b->lgraph_W == (const void *)lv.W && b->lgraph_over == (const void *)lv.nfeat_over &&
        b->lgraph_E == lv.E && b->lgraph_cpw == lv.cpw)
        return MPMC_OK;
    if (b->lgraph_exec) (void)hipGraphExecDestroy(b->lgraph_exec);
    b->lgraph_exec = nullptr;
    hipGraph_t graph;
    HIPCHK(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    for (uint32_t j = 0; j < kLearnGraphSweeps; ++j)
        launch_learned_sweep(b, (int)(j & 1u), j, lv, grid, lds, b->cap_stream);
    launch_advance(b->dev, (uint32_t)b->seed, (uint32_t)(b->seed >> 32), (uint32_t)b->g.W, b->g.Lq,
                   kLearnGraphSweeps, b->cap_stream);
    HIPCHK(hipStreamEndCapture(b->cap_stream, &graph));
    hipError_t e = hipGraphInstantiate(&b->lgraph_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        b->lgraph_exec = nullptr;
        return fail(MPMC_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    b->lgraph_W = lv.W;
    b->lgraph_over = lv.nfeat_over;
    b->lgraph_E = lv.E;
    b->lgraph_cpw = lv.cpw;
    return MPMC_OK;
}

static int learned_sweeps(Box *b, Learner *l, uint64_t k, float eps, unsigned long long *stamps,
                          double *phase_ticks) {
    const size_t lds = sizeof(LdsLearn);
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)k_pass_learned, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
        attr = true;
    }
    const uint64_t E = branch_threshold(eps);
    const uint32_t na = (b->g.M / 2) * (b->g.M / 2);
    constexpr uint32_t nt = 64 * kLearnWaves;
    const uint32_t cpw = learned_cells_per_wave(b, na);
    const uint32_t grid = learned_grid(na, cpw), waves = grid * kLearnWaves;
    const LearnView lv{l->W, E, ldexp((double)E, -32), l->over, stamps, cpw};
    std::vector<unsigned long long> h(stamps ? (size_t)waves * kLearnStamps : 0);
    for (uint64_t s = 0; s < k;) {
        if (!stamps && b->use_graphs && b->cur == 0 && k - s >= kLearnGraphSweeps) {
            int rc = learned_graph(b, lv, grid, lds);
            if (rc) return rc;
            HIPCHK(hipGraphLaunch(b->lgraph_exec, b->stream));
            s += kLearnGraphSweeps;
            b->canon_in_c = false;
            continue;
        }
        if (!stamps) {
            launch_learned_sweep(b, b->cur, 0, lv, grid, lds, b->stream);
        } else {
            // one pass at a time, each followed by the read-back of its stamps
            BoxView v = b->view(b->cur);
            const BoxView pv = in_place(v);
            for (uint32_t p = 0; p < 4; ++p) {
                k_pass_learned<<<grid, nt, lds, b->stream>>>(pv, p, lv);
                HIPCHK(hipMemcpyAsync(h.data(), stamps, h.size() * 8, hipMemcpyDeviceToHost, b->stream));
                HIPCHK(hipStreamSynchronize(b->stream));
                for (uint32_t w = 0; w < waves; ++w)
                    for (int ph = 0; ph + 1 < kLearnStamps; ++ph)
                        phase_ticks[ph] += (double)(long long)(h[(size_t)w * kLearnStamps + ph + 1] -
                                                               h[(size_t)w * kLearnStamps + ph]);
            }
            v.offset = 1;  // binned for the next sweep
            launch_rebin(v, b->stream);
        }
        launch_advance(b->dev, (uint32_t)b->seed, (uint32_t)(b->seed >> 32), (uint32_t)b->g.W, b->g.Lq,
                       1, b->stream);
        HIPCHK(hipGetLastError());
        b->cur ^= 1;
        b->canon_in_c = false;
        ++s;
    }
    return MPMC_OK;
}

extern "C" int mpmc_sweep_learned(mpmc_box bh, mpmc_learner lh, uint64_t k, float eps,
                                  uint64_t *trials, uint64_t *accepts) {
    if (!bh || !lh) return fail(MPMC_EINVAL, "NULL argument");
    if (!(eps >= 0.0f) || eps > 1.0f) return fail(MPMC_EINVAL, "eps must be in [0, 1]");
    Box *b = BX(bh);
    Learner *l = LR(lh);
    int rc = check_learned_box(b);
    if (rc) return rc;
    DevScalars before{};
    if (trials || accepts) {
        rc = b->read_scalars();
        if (rc) return rc;
        before = b->host;
    }
    rc = learned_sweeps(b, l, k, eps, nullptr, nullptr);
    if (rc) return rc;
    if (trials || accepts) {
        rc = b->read_scalars();
        if (rc) return rc;
        if (trials) *trials = b->host.trials - before.trials;
        if (accepts) *accepts = b->host.accepts - before.accepts;
    }
    return MPMC_OK;
}

extern "C" int mpmc_profile_learned(mpmc_box bh, mpmc_learner lh, uint32_t sweeps, float eps,
                                    double *phase_us) {
    if (!bh || !lh || !phase_us || sweeps == 0) return fail(MPMC_EINVAL, "bad arguments");
    if (!(eps >= 0.0f) || eps > 1.0f) return fail(MPMC_EINVAL, "eps must be in [0, 1]");
    Box *b = BX(bh);
    Learner *l = LR(lh);
    int rc = check_learned_box(b);
    if (rc) return rc;
    const uint32_t na = (b->g.M / 2) * (b->g.M / 2);
    const uint32_t waves = learned_grid(na, learned_cells_per_wave(b, na)) * kLearnWaves;
    unsigned long long *d = nullptr;
    rc = b->alloc_dev((void **)&d, (size_t)waves * kLearnStamps * 8);
    if (rc) return rc;
    double ticks[kLearnStamps - 1] = {};
    rc = learned_sweeps(b, l, sweeps, eps, d, ticks);
    b->free_dev(d);
    if (rc) return rc;
    int dev = 0, khz = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    const double us_per_tick = 1e3 / (double)(khz > 0 ? khz : 100000);
    for (int ph = 0; ph + 1 < kLearnStamps; ++ph)
        phase_us[ph] = ticks[ph] / ((double)waves * 4 * sweeps) * us_per_tick;
    return MPMC_OK;
}

extern "C" int mpmc_set_learned_cells_per_wave(mpmc_box bh, uint32_t cells) {
    if (!bh) return fail(MPMC_EINVAL, "NULL box");
    if (cells != 0 && cells != 16 && cells != 32 && cells != 64)
        return fail(MPMC_EINVAL, "cells per wave must be 0 (automatic), 16, 32 or 64");
    BX(bh)->learned_cpw = cells;
    return MPMC_OK;
}

extern "C" int mpmc_learner_info(mpmc_learner lh, uint64_t *n_data, uint64_t *n_feature_overflow,
                                 uint32_t *steps) {
    if (!lh) return fail(MPMC_EINVAL, "NULL learner");
    Learner *l = LR(lh);
    unsigned long long c[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(c, l->count, 16, hipMemcpyDeviceToHost, l->stream));
    HIPCHK(hipStreamSynchronize(l->stream));
    if (n_data) *n_data = c[0] < l->cap ? c[0] : l->cap;
    if (n_feature_overflow) *n_feature_overflow = c[1];
    if (steps) *steps = l->step;
    return MPMC_OK;
}

extern "C" int mpmc_learner_moves(mpmc_learner lh, uint64_t first, uint64_t n, float *F, float *D) {
    if (!lh || (n && (!F || !D))) return fail(MPMC_EINVAL, "bad arguments");
    Learner *l = LR(lh);
    unsigned long long c = 0;
    HIPCHK(hipMemcpyAsync(&c, l->count, 8, hipMemcpyDeviceToHost, l->stream));
    HIPCHK(hipStreamSynchronize(l->stream));
    const uint64_t have = c < l->cap ? c : l->cap;
    if (first > have || n > have - first) return fail(MPMC_EINVAL, "moves %llu..%llu of %llu",
                                                      (unsigned long long)first,
                                                      (unsigned long long)(first + n),
                                                      (unsigned long long)have);
    if (n == 0) return MPMC_OK;
    HIPCHK(hipMemcpyAsync(F, l->F + first * 24, n * 24 * 4, hipMemcpyDeviceToHost, l->stream));
    HIPCHK(hipMemcpyAsync(D, l->D + first * 2, n * 2 * 4, hipMemcpyDeviceToHost, l->stream));
    HIPCHK(hipStreamSynchronize(l->stream));
    return MPMC_OK;
}

extern "C" int mpmc_learner_adam_step(mpmc_learner lh, const float *grad, float lr) {
    if (!lh || !grad) return fail(MPMC_EINVAL, "NULL argument");
    Learner *l = LR(lh);
    HIPCHK(hipMemcpyAsync(l->grad, grad, kNPARAM * 4, hipMemcpyHostToDevice, l->stream));
    ++l->step;
    k_adam<<<(kNPARAM + 255) / 256, 256, 0, l->stream>>>(l->p, l->m, l->v, l->grad, l->W, l->step, lr, 1);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(l->stream));
    return MPMC_OK;
}

// Device buffers of a diagnostic call, released on every path.
namespace {
struct DiagBufs {
    std::vector<void *> p;
    ~DiagBufs() {
        for (void *q : p) (void)hipFree(q);
    }
    hipError_t get(void **q, size_t bytes) {
        hipError_t e = hipMalloc(q, bytes ? bytes : 4);
        if (e == hipSuccess) p.push_back(*q);
        return e;
    }
};
}  // namespace

extern "C" int mpmc_learned_propose(const float *out, uint32_t step_m, float eps, uint64_t seed,
                                    uint32_t n, int32_t *D, uint8_t *drawn, double *logp) {
    if (!out || !D || !drawn || !logp || n == 0) return fail(MPMC_EINVAL, "bad arguments");
    if (step_m == 0 || step_m > 255) return fail(MPMC_EINVAL, "step_m must be in 1..255");
    if (!(eps >= 0.0f) || eps > 1.0f) return fail(MPMC_EINVAL, "eps must be in [0, 1]");
    DiagBufs B;
    float *dout = nullptr;
    int32_t *dD = nullptr;
    uint8_t *dd = nullptr;
    double *dl = nullptr;
    HIPCHK(B.get((void **)&dout, 20 * 4));
    HIPCHK(B.get((void **)&dD, (size_t)n * 8));
    HIPCHK(B.get((void **)&dd, n));
    HIPCHK(B.get((void **)&dl, (size_t)n * 8));
    HIPCHK(hipMemcpy(dout, out, 20 * 4, hipMemcpyHostToDevice));
    const uint64_t E = branch_threshold(eps);
    k_lattice_propose<<<(n + 255) / 256, 256>>>(dout, step_m, E, ldexp((double)E, -32), (uint32_t)seed,
                                                (uint32_t)(seed >> 32), n, dD, dd, dl);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpy(D, dD, (size_t)n * 8, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(drawn, dd, n, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(logp, dl, (size_t)n * 8, hipMemcpyDeviceToHost));
    return MPMC_OK;
}

extern "C" int mpmc_learned_logp(const float *out, const int32_t *D, uint32_t n, uint32_t step_m,
                                 float eps, double *logp) {
    if (!out || !D || !logp || n == 0) return fail(MPMC_EINVAL, "bad arguments");
    if (step_m == 0 || step_m > 255) return fail(MPMC_EINVAL, "step_m must be in 1..255");
    if (!(eps >= 0.0f) || eps > 1.0f) return fail(MPMC_EINVAL, "eps must be in [0, 1]");
    DiagBufs B;
    float *dout = nullptr;
    int32_t *dD = nullptr;
    double *dl = nullptr;
    HIPCHK(B.get((void **)&dout, (size_t)n * 20 * 4));
    HIPCHK(B.get((void **)&dD, (size_t)n * 8));
    HIPCHK(B.get((void **)&dl, (size_t)n * 8));
    HIPCHK(hipMemcpy(dout, out, (size_t)n * 20 * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dD, D, (size_t)n * 8, hipMemcpyHostToDevice));
    const uint64_t E = branch_threshold(eps);
    k_lattice_p<<<(n + 255) / 256, 256>>>(dout, dD, n, step_m, ldexp((double)E, -32), dl);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpy(logp, dl, (size_t)n * 8, hipMemcpyDeviceToHost));
    return MPMC_OK;
}
