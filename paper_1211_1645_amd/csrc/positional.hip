// positional.hip — positional order: the structure factor at the
// wave vectors the periodic box allows and chi_j = exp(i q0.x_j) (Sec. IV.C,
// Eqs. (10), (11)), and the positional correlation C_q(r) averaged over pairs
// in a window of half-width sigma around r (Sec. IV.D, Eq. (12)).  One thread per cell serves the (mostly one)
// disks of that cell; absolute positions come from the cell lists and the
// accumulated shift as exact integers in q units.
#include "mpmc_kernels.hpp"

namespace mpmc {

namespace {
constexpr int kQC = 16;          // wave vectors per workgroup of the structure factor
constexpr uint32_t kRhoSplit = 64;  // workgroups sharing the cells of one wave-vector group

__device__ __forceinline__ uint32_t wrapm(int v, uint32_t M) {
    int r = v % (int)M;
    return (uint32_t)(r < 0 ? r + (int)M : r);
}

// Absolute position of slot s of cell c in q units, in [0, Lq).
__device__ __forceinline__ void abs_q(const MeasureView &m, uint32_t c, uint32_t s, long long *X,
                                      long long *Y) {
    const uint32_t NC = m.M * m.M;
    const long long U = (long long)(m.x[slot_at(c, s, NC)] * 4194304.0f);
    const long long V = (long long)(m.y[slot_at(c, s, NC)] * 4194304.0f);
    *X = ((long long)(c % m.M) * m.W + U + m.Sx) % m.Lq;
    *Y = ((long long)(c / m.M) * m.W + V + m.Sy) % m.Lq;
}
}  // namespace

// ---------------------------------------------------------------------------
// rho(q) = sum_n exp(2 pi i (h X_n + k Y_n) / Lq) for kQC wave vectors per
// workgroup column (blockIdx.y); the gridDim.x workgroups of a column split
// the cells, each thread serving cells c, c + stride, ...
//
// Each term: the phase in turns, scaled by 256, t = 256 (h X + k Y) / Lq, is
// formed in fp64 (|t| < 2^22, error below 2^-30) and split into its integer
// part i and fraction r; exp(2 pi i t / 256) = T[i mod 256] exp(2 pi i r / 256)
// with T a table of fp32 roots of unity and the second factor from its
// Taylor series to fifth order (|angle| < 2 pi / 256: truncation below
// 1e-12).  The product is formed in fp32 with fused multiply-adds and summed
// in fp64: every term carries an absolute error below 5e-7.  Each workgroup
// leaves its kQC partial sums in part[(by * gridDim.x + bx) * kQC + j].
__global__ void __launch_bounds__(256) k_rho(MeasureView m, const int32_t *hk, uint32_t nq,
                                             double2 *part) {
    __shared__ double2 wsum[4][kQC];
    __shared__ float2 roots[256];
    {
        double sn, cs;
        sincospi((double)threadIdx.x / 128.0, &sn, &cs);
        roots[threadIdx.x] = make_float2((float)cs, (float)sn);
    }
    __syncthreads();
    const uint32_t NC = m.M * m.M;
    const uint32_t q0 = blockIdx.y * kQC;
    double fh[kQC], fk[kQC];
    double re[kQC], im[kQC];
#pragma unroll
    for (int j = 0; j < kQC; ++j) {
        const uint32_t iq = q0 + j < nq ? q0 + j : nq - 1;
        fh[j] = 256.0 * (double)hk[2 * iq];
        fk[j] = 256.0 * (double)hk[2 * iq + 1];
        re[j] = im[j] = 0.0;
    }
    const double inv = 1.0 / (double)m.Lq;
    const float turn = 6.283185307179586f / 256.0f;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < NC; c += stride) {
        const uint32_t n = m.cnt[c];
        for (uint32_t s = 0; s < n; ++s) {
            // the position in q units without its reduction modulo Lq (a
            // whole period more leaves every phase unchanged): below 2 Lq
            const long long X = (long long)(c % m.M) * m.W +
                                (long long)(m.x[slot_at(c, s, NC)] * 4194304.0f) + m.Sx;
            const long long Y = (long long)(c / m.M) * m.W +
                                (long long)(m.y[slot_at(c, s, NC)] * 4194304.0f) + m.Sy;
            const double xh = (double)X * inv, yh = (double)Y * inv;
#pragma unroll
            for (int j = 0; j < kQC; ++j) {
                const double t = fma(fh[j], xh, fk[j] * yh);
                const double i = floor(t);
                const float a = (float)(t - i) * turn;  // residual angle in [0, 2 pi / 256]
                const float2 T = roots[(int)i & 255];
                const float a2 = a * a;
                const float cr = fmaf(a2, fmaf(a2, 1.0f / 24.0f, -0.5f), 1.0f);
                const float sr = a * fmaf(a2, fmaf(a2, 1.0f / 120.0f, -1.0f / 6.0f), 1.0f);
                re[j] += (double)fmaf(T.x, cr, -T.y * sr);
                im[j] += (double)fmaf(T.y, cr, T.x * sr);
            }
        }
    }
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < kQC; ++j) {
        double a = re[j], b = im[j];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            a += __shfl_xor(a, off, 64);
            b += __shfl_xor(b, off, 64);
        }
        if (lane == 0) wsum[wave][j] = make_double2(a, b);
    }
    __syncthreads();
    if (threadIdx.x < kQC) {
        const int j = threadIdx.x;
        double a = 0.0, b = 0.0;
        for (int w = 0; w < 4; ++w) {
            a += wsum[w][j].x;
            b += wsum[w][j].y;
        }
        part[((size_t)blockIdx.y * gridDim.x + blockIdx.x) * kQC + j] = make_double2(a, b);
    }
}

// S(q) = |sum of the partials|^2 / N; one thread per wave vector.  A wave
// vector with an index outside (-4096, 4096), beyond the accuracy the phase
// arithmetic is stated for, gets NaN (the host entry points reject such
// indices before the launch; device arrays are checked here).
__global__ void k_rho_reduce(const double2 *part, const int32_t *hk, uint32_t nbx, uint32_t nq,
                             uint32_t N, double *S) {
    const uint32_t iq = blockIdx.x * blockDim.x + threadIdx.x;
    if (iq >= nq) return;
    const int32_t h = hk[2 * iq], k = hk[2 * iq + 1];
    if (h <= -4096 || h >= 4096 || k <= -4096 || k >= 4096) {
        S[iq] = __builtin_nan("");
        return;
    }
    const uint32_t by = iq / kQC, j = iq % kQC;
    double a = 0.0, b = 0.0;
    for (uint32_t bx = 0; bx < nbx; ++bx) {
        const double2 p = part[((size_t)by * nbx + bx) * kQC + j];
        a += p.x;
        b += p.y;
    }
    S[iq] = (a * a + b * b) / (double)N;
}

uint32_t rho_split(const MeasureView &m) {
    const uint32_t nb = (m.M * m.M + 255) / 256;
    return nb < kRhoSplit ? nb : kRhoSplit;
}

size_t rho_work_bytes(const MeasureView &m, uint32_t nq) {
    return (size_t)rho_split(m) * ((nq + kQC - 1) / kQC) * kQC * sizeof(double2);
}

void launch_structure_factor(const MeasureView &m, const int32_t *hk, uint32_t nq, double *S,
                             void *work, hipStream_t st) {
    const uint32_t nbx = rho_split(m), nby = (nq + kQC - 1) / kQC;
    double2 *part = static_cast<double2 *>(work);
    k_rho<<<dim3(nbx, nby), 256, 0, st>>>(m, hk, nq, part);
    k_rho_reduce<<<(nq + 255) / 256, 256, 0, st>>>(part, hk, nbx, nq, m.N, S);
}

// ---------------------------------------------------------------------------
// chi_j = exp(i q0.x_j), q0 = (2 pi / L)(h, k), by tag; the phase is reduced
// exactly in integers: (h X + k Y) mod Lq.
__global__ void __launch_bounds__(256) k_chi(MeasureView m, int32_t h, int32_t k, float *re,
                                             float *im) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= m.M * m.M) return;
    const uint32_t n = m.cnt[c], NC = m.M * m.M;
    for (uint32_t s = 0; s < n; ++s) {
        long long X, Y;
        abs_q(m, c, s, &X, &Y);
        const long long hm = (long long)h % m.Lq, km = (long long)k % m.Lq;
        // products below 2^63: |h|, |k| < 2^12 is checked by the host and Lq < 2^40
        long long t = ((hm * X) % m.Lq + (km * Y) % m.Lq) % m.Lq;
        if (t < 0) t += m.Lq;
        const double ph = 2.0 * ((double)t / (double)m.Lq);
        double sn, cs;
        sincospi(ph, &sn, &cs);
        const uint32_t tg = m.tag[slot_at(c, s, NC)];
        re[tg] = (float)cs;
        im[tg] = (float)sn;
    }
}

void launch_chi(const MeasureView &m, int32_t h, int32_t k, float *re, float *im, hipStream_t st) {
    k_chi<<<(m.M * m.M + 255) / 256, 256, 0, st>>>(m, h, k, re, im);
}

// ---------------------------------------------------------------------------
// C_q(r): every disk visits the disks of the (2R+1)^2 cells around its own
// (R cells reach the top window edge), so each unordered pair is seen twice
// and the host halves the sums.  Separations are exact integers in q units;
// a pair lies in window b when (b Dr - 2^22)^2 <= d^2 <= (b Dr + 2^22)^2,
// Dr = dr / q, tested exactly in 64-bit integers.  Per workgroup, per bin:
// sum of cos(q.d) (fp64) and the pair count, left in rows[bx * B + b].
__global__ void __launch_bounds__(256) k_cq(MeasureView m, double qx, double qy, long long Dr,
                                            uint32_t B, int R, long long reach, double dr,
                                            double *rnum, unsigned long long *rcnt) {
    extern __shared__ unsigned char cq_lds[];
    double *snum = reinterpret_cast<double *>(cq_lds);
    unsigned int *scnt = reinterpret_cast<unsigned int *>(snum + B);
    for (uint32_t b = threadIdx.x; b < B; b += blockDim.x) {
        snum[b] = 0.0;
        scnt[b] = 0u;
    }
    __syncthreads();
    const uint32_t M = m.M, NC = M * M;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    const long long one = 1ll << 22;
    const uint32_t n = c < NC ? m.cnt[c] : 0u;
    const int ci = (int)(c % M), cj = (int)(c / M);
    const double inv_dr = 1.0 / dr;  // candidate windows only: each is confirmed exactly
    // a neighbour cell whose nearest corner lies beyond the reach holds no
    // partner: (|di| - 1)^2 + (|dj| - 1)^2 > (reach / W)^2 in cells
    const double rc = (double)reach / (double)m.W, rc2 = rc * rc;
    for (uint32_t s = 0; s < n; ++s) {
        const long long Ui = (long long)(m.x[slot_at(c, s, NC)] * 4194304.0f);
        const long long Vi = (long long)(m.y[slot_at(c, s, NC)] * 4194304.0f);
        for (int dj = -R; dj <= R; ++dj) {
            const double ey = (double)(abs(dj) > 0 ? abs(dj) - 1 : 0);
            for (int di = -R; di <= R; ++di) {
                const double ex = (double)(abs(di) > 0 ? abs(di) - 1 : 0);
                if (ex * ex + ey * ey > rc2) continue;
                const uint32_t nb = wrapm(ci + di, M) + M * wrapm(cj + dj, M);
                const uint32_t mm = m.cnt[nb];
                for (uint32_t t = 0; t < mm; ++t) {
                    if (di == 0 && dj == 0 && t == s) continue;
                    const long long dX = (long long)di * m.W +
                                         (long long)(m.x[slot_at(nb, t, NC)] * 4194304.0f) - Ui;
                    const long long dY = (long long)dj * m.W +
                                         (long long)(m.y[slot_at(nb, t, NC)] * 4194304.0f) - Vi;
                    if (dX > reach || dX < -reach || dY > reach || dY < -reach) continue;
                    const unsigned long long d2 = (unsigned long long)(dX * dX) +
                                                  (unsigned long long)(dY * dY);
                    const double d = sqrt((double)d2) * (1.0 / 4194304.0);
                    long long b0 = (long long)floor((d - 1.0) * inv_dr) - 1;
                    long long b1 = (long long)ceil((d + 1.0) * inv_dr) + 1;
                    if (b0 < 0) b0 = 0;
                    if (b1 > (long long)B - 1) b1 = (long long)B - 1;
                    if (b0 > b1) continue;
                    const double cs = cos(qx * ((double)dX * (1.0 / 4194304.0)) +
                                          qy * ((double)dY * (1.0 / 4194304.0)));
                    for (long long b = b0; b <= b1; ++b) {
                        const long long Rb = b * Dr;
                        const long long lo = Rb > one ? Rb - one : 0, hi = Rb + one;
                        if (d2 >= (unsigned long long)(lo * lo) && d2 <= (unsigned long long)(hi * hi)) {
                            atomicAdd(&snum[b], cs);
                            atomicAdd(&scnt[b], 1u);
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < B; b += blockDim.x) {
        rnum[(size_t)blockIdx.x * B + b] = snum[b];
        rcnt[(size_t)blockIdx.x * B + b] = scnt[b];
    }
}

// One workgroup per bin: sums the rows (halving the ordered pairs).
__global__ void __launch_bounds__(256) k_cq_reduce(const double *rnum, const unsigned long long *rcnt,
                                                   uint32_t G, uint32_t B, double *num,
                                                   unsigned long long *cnt) {
    __shared__ double pn[4];
    __shared__ unsigned long long pc[4];
    const uint32_t b = blockIdx.x;
    double sn = 0.0;
    unsigned long long sc = 0;
    for (uint32_t g = threadIdx.x; g < G; g += blockDim.x) {
        sn += rnum[(size_t)g * B + b];
        sc += rcnt[(size_t)g * B + b];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        sn += __shfl_xor(sn, off, 64);
        sc += __shfl_xor(sc, off, 64);
    }
    if ((threadIdx.x & 63u) == 0) {
        pn[threadIdx.x >> 6] = sn;
        pc[threadIdx.x >> 6] = sc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        num[b] = 0.5 * (pn[0] + pn[1] + pn[2] + pn[3]);
        cnt[b] = (pc[0] + pc[1] + pc[2] + pc[3]) / 2;
    }
}

size_t cq_work_bytes(const MeasureView &m, uint32_t B) {
    const uint32_t G = (m.M * m.M + 255) / 256;
    return (size_t)G * B * (sizeof(double) + sizeof(unsigned long long)) + B * 16;
}

void launch_cq(const MeasureView &m, double qx, double qy, double dr, uint32_t B, int R,
               double top, void *work, double *num, unsigned long long *cnt, hipStream_t st) {
    const uint32_t G = (m.M * m.M + 255) / 256;
    double *rnum = static_cast<double *>(work);
    unsigned long long *rcnt = reinterpret_cast<unsigned long long *>(rnum + (size_t)G * B);
    const long long Dr = (long long)llround(dr * 4194304.0);
    const long long reach = (long long)ceil(top * 4194304.0);
    const size_t lds = B * (sizeof(double) + sizeof(unsigned int));
    k_cq<<<G, 256, lds, st>>>(m, qx, qy, Dr, B, R, reach, dr, rnum, rcnt);
    k_cq_reduce<<<B, 256, 0, st>>>(rnum, rcnt, G, B, num, cnt);
}

}  // namespace mpmc
