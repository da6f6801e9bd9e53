// measure.hip — observables on the device: the contact pair histogram behind
// the pressure (Sec. II.C.1, Eq. (2)), the local orientational order psi_j
// and its coarse field (Eq. (8), Secs. III and IV.B), the state validator
// and the absolute positions.  One thread per cell or per cell slot; the
// cell grid bounds every neighbour search (w >= 2 sigma).
#include "mpmc_kernels.hpp"

namespace mpmc {

__device__ __forceinline__ uint32_t wrapc(int v, uint32_t M) {
    int r = v % (int)M;
    return (uint32_t)(r < 0 ? r + (int)M : r);
}

// ---------------------------------------------------------------------------
// Contact histogram: for every disk i (optionally restricted by sel[tag]) and
// every disk j != i in the (2h+1)^2 cell stencil, bin fp32 r^2 against the
// squared edges.  Pairs are counted ordered; an unordered count is half.
// With h = 2 and M = 4 a cell is visited at offsets -2 and +2, i.e. as two
// different periodic images, of which at most one lies below r_max < L/2.
__global__ void __launch_bounds__(256) k_contact_hist(MeasureView m, const float *__restrict__ E,
                                                      uint32_t K, int h,
                                                      unsigned long long *hist,
                                                      const uint8_t *sel, const uint32_t *loc) {
    extern __shared__ uint32_t bins[];
    for (uint32_t k = threadIdx.x; k < K; k += blockDim.x) bins[k] = 0;
    __syncthreads();
    const uint32_t M = m.M;
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < m.N && (!sel || sel[t])) {
        const uint32_t NC = M * M, s = loc[t] / NC, cell = loc[t] - s * NC;
        const uint32_t ci = cell % M, cj = cell / M;
        const float e0 = E[0], eK = E[K];
        const float rmax = sqrtf(eK) * 1.0001f + 1e-4f;  // conservative reach
        const float xi = m.x[loc[t]], yi = m.y[loc[t]];
        for (int dj = -h; dj <= h; ++dj) {
            // smallest |dy| to any disk of row dj: skip rows out of reach
            const float gy = dj > 1 ? (float)(dj - 1) * m.w + (m.w - yi)
                           : dj < -1 ? (float)(-dj - 1) * m.w + yi : 0.0f;
            if (gy > rmax) continue;
            for (int di = -h; di <= h; ++di) {
                const float gx = di > 1 ? (float)(di - 1) * m.w + (m.w - xi)
                               : di < -1 ? (float)(-di - 1) * m.w + xi : 0.0f;
                if (gx > rmax) continue;
                const uint32_t nb = wrapc((int)ci + di, M) + M * wrapc((int)cj + dj, M);
                const float cwx = (float)di * m.w, cwy = (float)dj * m.w;
                const uint32_t mm = m.cnt[nb];
                for (uint32_t q = 0; q < mm; ++q) {
                    if (di == 0 && dj == 0 && q == s) continue;
                    const float dx = (m.x[slot_at(nb, q, NC)] - xi) + cwx;
                    const float dy = (m.y[slot_at(nb, q, NC)] - yi) + cwy;
                    const float r2 = r2_f32(dx, dy);
                    if (!(r2 >= e0) || !(r2 < eK)) continue;
                    // start from the square-root estimate, then settle on the
                    // exact fp32 edges
                    int k = (int)((sqrtf(r2) - 2.0f) * (float)K / (sqrtf(eK) - 2.0f));
                    k = k < 0 ? 0 : (k >= (int)K ? (int)K - 1 : k);
                    while (k > 0 && r2 < E[k]) --k;
                    while (k + 1 < (int)K && !(r2 < E[k + 1])) ++k;
                    atomicAdd(&bins[k], 1u);
                }
            }
        }
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < K; k += blockDim.x)
        if (bins[k]) atomicAdd(&hist[k], (unsigned long long)bins[k]);
}

// ---------------------------------------------------------------------------
// Tiled forms for boxes of at most 4 slots per cell.  A workgroup of 256
// threads stages a 16 x 16 block of cells plus a halo of H cells in LDS
// (offsets with a far sentinel in empty slots, tags, counts), lists the
// block's disks and gives each lane one disk.  The stencil is unrolled over
// its (2H+1)^2 cells and SL slots per cell (SL = 2, or 4 when some staged
// cell holds more than two disks), so no lane runs a trip count of its own.
// A persistent grid of at most kMeasGrid workgroups strides over the blocks
// and leaves one partial result per workgroup, which a second kernel sums:
// no two workgroups add to one address.
constexpr int kPT = 16, kStageHalo = 3, kSR = kPT + 2 * kStageHalo;
constexpr float kFarM = 1.0e6f;  // sentinel offset of an empty slot
constexpr uint32_t kMeasGrid = 1536;  // six workgroups per CU, as LDS allows

struct Stage {
    float4 x[kSR * kSR], y[kSR * kSR];
    uint4 tag[kSR * kSR];
    uint8_t cnt[kSR * kSR];
    uint16_t disk[4 * kPT * kPT];  // the block's disks: own cell << 2 | slot
    uint32_t wsum[4], wbig[4];
};

size_t measure_work_bytes(uint32_t K) { return (size_t)kMeasGrid * (K * 4 + sizeof(double2)) + 16; }

bool measure_tiled(const MeasureView &m, uint32_t h) {
    return m.cap <= 4 && h >= 1 && h <= (uint32_t)kStageHalo;
}

__device__ __forceinline__ float comp4f(const float4 &v, int s) {
    return s == 0 ? v.x : s == 1 ? v.y : s == 2 ? v.z : v.w;
}
__device__ __forceinline__ uint32_t comp4u(const uint4 &v, int s) {
    return s == 0 ? v.x : s == 1 ? v.y : s == 2 ? v.z : v.w;
}

// Stages block (I0, J0) with halo H (region cell (rx, ry) at rx + SR ry,
// SR = 16 + 2H) and lists the block's disks.  Returns the number of listed
// disks; *big tells whether some staged cell holds more than two.
template <int H>
__device__ int stage_block(Stage &S, const MeasureView &m, uint32_t I0, uint32_t J0, bool *big) {
    constexpr int SR = kPT + 2 * H, NS = SR * SR, NIT = (NS + 255) / 256;
    const uint32_t M = m.M, NC = M * M;
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    // this thread's own cell (for the list of the block's disks), then the
    // counts and slots 0, 1 of every staged cell: all in one round trip, the
    // loads issued at raised priority so that they leave before the other
    // waves' arithmetic (unused slots hold stale values and are replaced by
    // the sentinel); slots 2, 3 afterwards where the count asks for them
    const int tx = threadIdx.x % kPT, ty = threadIdx.x / kPT;
    const bool inb = I0 + tx < M && J0 + ty < M;
    uint32_t nown = 0;
    __builtin_amdgcn_s_setprio(3);
    if (inb) nown = m.cnt[wrapc((int)I0 + tx, M) + M * wrapc((int)J0 + ty, M)];
    uint32_t c_r[NIT], n_r[NIT], ta[NIT], tb[NIT];
    float xa[NIT], xb[NIT], ya[NIT], yb[NIT];
#pragma unroll
    for (int i = 0; i < NIT; ++i) {
        const int e = (int)threadIdx.x + 256 * i, ee = e < NS ? e : 0;
        const int rx = ee % SR, ry = ee / SR;
        const uint32_t c = wrapc((int)I0 - H + rx, M) + M * wrapc((int)J0 - H + ry, M);
        c_r[i] = c;
        n_r[i] = m.cnt[c];
        xa[i] = m.x[c];
        xb[i] = m.x[NC + c];
        ya[i] = m.y[c];
        yb[i] = m.y[NC + c];
        ta[i] = m.tag[c];
        tb[i] = m.tag[NC + c];
    }
    __builtin_amdgcn_s_setprio(0);
    bool crowded = false;
#pragma unroll
    for (int i = 0; i < NIT; ++i) {
        const int e = (int)threadIdx.x + 256 * i;
        if (e >= NS) break;
        const uint32_t c = c_r[i], n = n_r[i] > 4 ? 4 : n_r[i];
        float4 x4 = make_float4(kFarM, kFarM, kFarM, kFarM), y4 = x4;
        uint4 t4 = make_uint4(0u, 0u, 0u, 0u);
        if (n > 0) { x4.x = xa[i]; y4.x = ya[i]; t4.x = ta[i]; }
        if (n > 1) { x4.y = xb[i]; y4.y = yb[i]; t4.y = tb[i]; }
        if (n > 2) { x4.z = m.x[2 * NC + c]; y4.z = m.y[2 * NC + c]; t4.z = m.tag[2 * NC + c]; }
        if (n > 3) { x4.w = m.x[3 * NC + c]; y4.w = m.y[3 * NC + c]; t4.w = m.tag[3 * NC + c]; }
        S.x[e] = x4;
        S.y[e] = y4;
        S.tag[e] = t4;
        S.cnt[e] = (uint8_t)n;
        crowded |= n > 2;
    }
    // prefix sums of the own counts over the block from bit-plane ballots (a
    // count is below 8)
    nown = nown > 4 ? 4 : nown;
    const unsigned long long lt = (1ull << lane) - 1ull;
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const unsigned long long bb = __ballot((nown >> b) & 1u);
        pre += (uint32_t)__popcll(bb & lt) << b;
        tot += (uint32_t)__popcll(bb) << b;
    }
    const unsigned long long bg = __ballot(crowded);
    if (lane == 0) {
        S.wsum[wave] = tot;
        S.wbig[wave] = bg != 0ull;
    }
    __syncthreads();
    uint32_t off = 0, all = 0, anybig = 0;
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
        off += q < wave ? S.wsum[q] : 0u;
        all += S.wsum[q];
        anybig |= S.wbig[q];
    }
    for (uint32_t k = 0; k < nown; ++k) S.disk[off + pre + k] = (uint16_t)((threadIdx.x << 2) | k);
    __syncthreads();
    *big = anybig != 0;
    return (int)all;
}

// Bin of a pair with E[0] <= r2 < E[K]: start from the square-root estimate,
// then settle on the exact fp32 edges.
__device__ __forceinline__ int contact_bin(float r2, const float *E, uint32_t K, float eK) {
    int k = (int)((sqrtf(r2) - 2.0f) * (float)K / (sqrtf(eK) - 2.0f));
    k = k < 0 ? 0 : (k >= (int)K ? (int)K - 1 : k);
    while (k > 0 && r2 < E[k]) --k;
    while (k + 1 < (int)K && !(r2 < E[k + 1])) ++k;
    return k;
}

// Ordered contact pairs of the listed disks into the LDS bins.
template <int H, int SL>
__device__ void contact_disks(const Stage &S, const MeasureView &m, const float *E,
                              uint32_t K, const uint8_t *sel, int ndisk, uint32_t *bins) {
    constexpr int SR = kPT + 2 * H;
    const float e0 = E[0], eK = E[K];
    for (int j = threadIdx.x; j < ndisk; j += blockDim.x) {
        const uint32_t d = S.disk[j];
        const int cl = (int)(d >> 2), s = (int)(d & 3u);
        const int me = (cl % kPT + H) + SR * (cl / kPT + H);
        if (sel && !sel[comp4u(S.tag[me], s)]) continue;
        const float xi = comp4f(S.x[me], s), yi = comp4f(S.y[me], s);
#pragma unroll
        for (int dj = -H; dj <= H; ++dj)
#pragma unroll
            for (int di = -H; di <= H; ++di) {
                const int ne = me + di + SR * dj;
                const float cwx = (float)di * m.w, cwy = (float)dj * m.w;
                const float4 qx = S.x[ne], qy = S.y[ne];
#pragma unroll
                for (int q = 0; q < SL; ++q) {
                    const float dx = (comp4f(qx, q) - xi) + cwx;
                    const float dy = (comp4f(qy, q) - yi) + cwy;
                    const float r2 = r2_f32(dx, dy);
                    const bool self = di == 0 && dj == 0 && q == s;
                    if (self || !(r2 >= e0) || !(r2 < eK)) continue;
                    atomicAdd(&bins[contact_bin(r2, E, K, eK)], 1u);
                }
            }
    }
}

// Dynamic LDS: K bins, then the K + 1 squared edges, so that settling a
// pair on its bin reads no global memory.
template <int H>
__global__ void __launch_bounds__(256) k_contact_hist_tile(MeasureView m, const float *__restrict__ E,
                                                           uint32_t K, const uint8_t *sel,
                                                           uint32_t *rows) {
    __shared__ Stage S;
    extern __shared__ uint32_t bins[];
    float *El = reinterpret_cast<float *>(bins + K);
    for (uint32_t k = threadIdx.x; k < K; k += blockDim.x) bins[k] = 0;
    for (uint32_t k = threadIdx.x; k <= K; k += blockDim.x) El[k] = E[k];
    const uint32_t M = m.M, nbx = (M + kPT - 1) / kPT;
    for (uint32_t blk = blockIdx.x; blk < nbx * nbx; blk += gridDim.x) {
        bool big;
        const int nd = stage_block<H>(S, m, (blk % nbx) * kPT, (blk / nbx) * kPT, &big);
        if (big) contact_disks<H, 4>(S, m, El, K, sel, nd, bins);
        else contact_disks<H, 2>(S, m, El, K, sel, nd, bins);
        __syncthreads();  // S is restaged for the next block
    }
    for (uint32_t k = threadIdx.x; k < K; k += blockDim.x) rows[blockIdx.x * K + k] = bins[k];
}

// hist[k] += sum over the G rows; one workgroup per bin.
__global__ void __launch_bounds__(256) k_hist_rows_reduce(const uint32_t *rows, uint32_t G, uint32_t K,
                                                          unsigned long long *hist) {
    __shared__ unsigned long long part[4];
    const uint32_t k = blockIdx.x;
    unsigned long long s = 0;
    for (uint32_t g = threadIdx.x; g < G; g += blockDim.x) s += rows[g * K + k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63u) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) hist[k] += part[0] + part[1] + part[2] + part[3];
}

void launch_contact_tiled(const MeasureView &m, const float *edges, uint32_t K, uint32_t h,
                          unsigned long long *hist, const uint8_t *sel, void *work, hipStream_t st) {
    const uint32_t nb = (m.M + kPT - 1) / kPT;
    const uint32_t G = nb * nb < kMeasGrid ? nb * nb : kMeasGrid;
    uint32_t *rows = static_cast<uint32_t *>(work);
    const size_t lds = (2 * (size_t)K + 1) * sizeof(uint32_t);
    if (h == 1) k_contact_hist_tile<1><<<G, 256, lds, st>>>(m, edges, K, sel, rows);
    else if (h == 2) k_contact_hist_tile<2><<<G, 256, lds, st>>>(m, edges, K, sel, rows);
    else k_contact_hist_tile<3><<<G, 256, lds, st>>>(m, edges, K, sel, rows);
    k_hist_rows_reduce<<<K, 256, 0, st>>>(rows, G, K, hist);
}

// Slot of every disk by tag: loc[tag] = slot_at(cell, slot, M * M).
__global__ void __launch_bounds__(256) k_locate(MeasureView m, uint32_t *loc) {
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t NC = m.M * m.M, s = gid / NC, cell = gid - s * NC;
    if (s >= m.CS || s >= m.cnt[cell]) return;
    const uint32_t tg = m.tag[gid];
    if (tg < m.N) loc[tg] = gid;
}

void launch_locate(const MeasureView &m, uint32_t *loc, hipStream_t st) {
    const uint32_t n = m.M * m.M * m.CS;
    k_locate<<<(n + 255) / 256, 256, 0, st>>>(m, loc);
}

void launch_contact_hist(const MeasureView &m, const float *edges, uint32_t K, uint32_t h,
                         unsigned long long *hist, const uint8_t *sel, const uint32_t *loc,
                         void *work, hipStream_t st) {
    if (measure_tiled(m, h)) {
        launch_contact_tiled(m, edges, K, h, hist, sel, work, st);
        return;
    }
    k_contact_hist<<<(m.N + 255) / 256, 256, K * sizeof(uint32_t), st>>>(m, edges, K, (int)h, hist,
                                                                          sel, loc);
}

// ---------------------------------------------------------------------------
// psi_j: the six nearest other disks by (fp32 r^2, tag) within the
// (2h+1)^2 stencil.  The search is exact when the sixth distance is below
// h w (every disk closer than h w lies in the stencil); otherwise the disk
// sets *fail and the host repeats with a larger h.
struct Nb6 {
    float r2[6];
    uint32_t tag[6];
    float dx[6], dy[6];
};

__device__ __forceinline__ bool nb_less(float ra, uint32_t ta, float rb, uint32_t tb) {
    return ra < rb || (ra == rb && ta < tb);
}

// psi_j of Eq. (8) from the six neighbours: mean of z^6 / |z|^6, z = dx + i dy.
__device__ __forceinline__ void psi6_sum(const Nb6 &b, float &sr, float &si) {
    sr = 0.0f;
    si = 0.0f;
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        const float dx = b.dx[e], dy = b.dy[e];
        const float ar = dx * dx - dy * dy, ai = 2.0f * dx * dy;     // z^2
        const float br = ar * ar - ai * ai, bi = 2.0f * ar * ai;     // z^4
        const float cr = br * ar - bi * ai, cim = br * ai + bi * ar; // z^6
        const float r6 = b.r2[e] * b.r2[e] * b.r2[e];
        sr += cr / r6;
        si += cim / r6;
    }
    sr *= (1.0f / 6.0f);
    si *= (1.0f / 6.0f);
}

__global__ void __launch_bounds__(256) k_psi6(MeasureView m, int h, float *re, float *im,
                                              uint32_t *fail, const uint32_t *loc) {
    const uint32_t M = m.M;
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t NC = M * M, at = gid < m.N ? loc[gid] : 0;
    const uint32_t s = at / NC, cell = at - s * NC;
    double pr = 0.0, pi = 0.0;
    if (gid < m.N) {
        const uint32_t ci = cell % M, cj = cell / M;
        const float xi = m.x[at], yi = m.y[at];
        const uint32_t ti = m.tag[at];
        Nb6 b;
#pragma unroll
        for (int e = 0; e < 6; ++e) { b.r2[e] = INFINITY; b.tag[e] = 0xFFFFFFFFu; b.dx[e] = 0; b.dy[e] = 0; }
        for (int dj = -h; dj <= h; ++dj)
            for (int di = -h; di <= h; ++di) {
                const uint32_t nb = wrapc((int)ci + di, M) + M * wrapc((int)cj + dj, M);
                const float cwx = (float)di * m.w, cwy = (float)dj * m.w;
                const uint32_t mm = m.cnt[nb];
                for (uint32_t t = 0; t < mm; ++t) {
                    if (di == 0 && dj == 0 && t == s) continue;
                    const float dx = (m.x[slot_at(nb, t, NC)] - xi) + cwx;
                    const float dy = (m.y[slot_at(nb, t, NC)] - yi) + cwy;
                    const float r2 = r2_f32(dx, dy);
                    const uint32_t tg = m.tag[slot_at(nb, t, NC)];
                    if (!nb_less(r2, tg, b.r2[5], b.tag[5])) continue;
                    b.r2[5] = r2; b.tag[5] = tg; b.dx[5] = dx; b.dy[5] = dy;
#pragma unroll
                    for (int e = 5; e > 0; --e) {
                        if (nb_less(b.r2[e], b.tag[e], b.r2[e - 1], b.tag[e - 1])) {
                            float fr = b.r2[e]; b.r2[e] = b.r2[e - 1]; b.r2[e - 1] = fr;
                            uint32_t ft = b.tag[e]; b.tag[e] = b.tag[e - 1]; b.tag[e - 1] = ft;
                            float fx = b.dx[e]; b.dx[e] = b.dx[e - 1]; b.dx[e - 1] = fx;
                            float fy = b.dy[e]; b.dy[e] = b.dy[e - 1]; b.dy[e - 1] = fy;
                        }
                    }
                }
            }
        const double reach = (double)h * (double)m.w;
        if (!((double)b.r2[5] < reach * reach * (1.0 - 1e-6))) atomicOr(fail, 1u);
        float sr = 0.0f, si = 0.0f;
        psi6_sum(b, sr, si);
        re[ti] = sr;
        im[ti] = si;
        pr = sr;
        pi = si;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        pr += __shfl_xor(pr, off, 64);
        pi += __shfl_xor(pi, off, 64);
    }
    if ((threadIdx.x & 63u) == 0) {
        atomicAdd(&m.dev->psi_re, pr);
        atomicAdd(&m.dev->psi_im, pi);
    }
}

// psi_j of the listed disks; returns this lane's contribution to the sums.
// The six nearest by (fp32 r^2, tag) are kept sorted as 64-bit keys
// r^2 bits << 32 | tag (r^2 >= 0, so its bits order as the value), each with
// its place in the stage; a candidate is one compare against the sixth key,
// an insertion a chain of compare-exchanges of key and place.  The
// neighbours' offsets are recomputed from their places at the end, in the
// same arithmetic.  Empty slots hold a far sentinel: they enter only a list
// that then fails the reach test.  sre, sim (may be NULL) receive psi_j by
// cell slot as well.  With CT the same scan also bins the ordered contact
// pairs (squared edges E[0..K] and bins in LDS), as contact_disks does.
template <int H, int SL, bool CT>
__device__ void psi6_disks(const Stage &S, const MeasureView &m, uint32_t I0, uint32_t J0, int ndisk,
                           float *re, float *im, float *sre, float *sim, uint32_t *fail, double &pr,
                           double &pi, const float *E, uint32_t K, uint32_t *bins) {
    constexpr int SR = kPT + 2 * H;
    const float e0 = CT ? E[0] : 0.0f, eK = CT ? E[K] : 0.0f;
    for (int j = threadIdx.x; j < ndisk; j += blockDim.x) {
        const uint32_t d = S.disk[j];
        const int cl = (int)(d >> 2), s = (int)(d & 3u);
        const int me = (cl % kPT + H) + SR * (cl / kPT + H);
        const float xi = comp4f(S.x[me], s), yi = comp4f(S.y[me], s);
        const uint32_t ti = comp4u(S.tag[me], s);
        unsigned long long key[6];
        uint32_t at[6];
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            key[e] = ~0ull;
            at[e] = (uint32_t)me << 2;
        }
#pragma unroll 1
        for (int dj = -H; dj <= H; ++dj)
#pragma unroll
            for (int di = -H; di <= H; ++di) {
                const int ne = me + di + SR * dj;
                const float cwx = (float)di * m.w, cwy = (float)dj * m.w;
                const float4 qx = S.x[ne], qy = S.y[ne];
                const uint4 qt = S.tag[ne];
#pragma unroll
                for (int q = 0; q < SL; ++q) {
                    const float dx = (comp4f(qx, q) - xi) + cwx;
                    const float dy = (comp4f(qy, q) - yi) + cwy;
                    const float r2 = r2_f32(dx, dy);
                    const unsigned long long k =
                        ((unsigned long long)__float_as_uint(r2) << 32) | comp4u(qt, q);
                    const bool self = di == 0 && dj == 0 && q == s;
                    if (CT && !self && r2 >= e0 && r2 < eK) atomicAdd(&bins[contact_bin(r2, E, K, eK)], 1u);
                    if (self || !(k < key[5])) continue;
                    key[5] = k;
                    at[5] = ((uint32_t)ne << 2) | (uint32_t)q;
#pragma unroll
                    for (int e = 5; e > 0; --e) {
                        const bool sw = key[e] < key[e - 1];
                        const unsigned long long ka = key[e], kb = key[e - 1];
                        const uint32_t pa = at[e], pb = at[e - 1];
                        key[e] = sw ? kb : ka;
                        key[e - 1] = sw ? ka : kb;
                        at[e] = sw ? pb : pa;
                        at[e - 1] = sw ? pa : pb;
                    }
                }
            }
        Nb6 b;
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            const int ne = (int)(at[e] >> 2), q = (int)(at[e] & 3u);
            const int di = ne % SR - me % SR, dj = ne / SR - me / SR;
            const float cwx = (float)di * m.w, cwy = (float)dj * m.w;
            b.dx[e] = (comp4f(S.x[ne], q) - xi) + cwx;
            b.dy[e] = (comp4f(S.y[ne], q) - yi) + cwy;
            b.r2[e] = __uint_as_float((uint32_t)(key[e] >> 32));
            b.tag[e] = (uint32_t)key[e];
        }
        // exact only if every disk closer than the sixth lies in the stencil
        const double reach = (double)H * (double)m.w;
        if (!((double)b.r2[5] < reach * reach * (1.0 - 1e-6))) atomicOr(fail, 1u);
        float sr6 = 0.0f, si6 = 0.0f;
        psi6_sum(b, sr6, si6);
        re[ti] = sr6;
        im[ti] = si6;
        if (sre) {
            const uint32_t c = (I0 + (uint32_t)(cl % kPT)) + m.M * (J0 + (uint32_t)(cl / kPT));
            const uint32_t a = (uint32_t)s * m.M * m.M + c;
            sre[a] = sr6;
            sim[a] = si6;
        }
        pr += sr6;
        pi += si6;
    }
}

// gate: NULL, or a flag that a narrower pass set when its search fell short;
// with the flag clear the launch does nothing and leaves that pass's psi_j
// and partials in place.
// With CT the workgroup also counts the ordered contact pairs (squared edges
// E[0..K] from global memory; dynamic LDS of K bins and K + 1 edges) and
// leaves its row of counts in rows, as k_contact_hist_tile does: one staging
// of each block serves both measurements.
template <int H, bool CT>
__global__ void __launch_bounds__(256) k_psi6_tile(MeasureView m, float *re, float *im, float *sre,
                                                   float *sim, uint32_t *fail, double2 *part,
                                                   const uint32_t *gate, const float *__restrict__ E,
                                                   uint32_t K, uint32_t *rows) {
    if (gate != nullptr && *gate == 0u) return;  // uniform over the grid
    __shared__ Stage S;
    __shared__ double2 wpart[4];
    extern __shared__ uint32_t bins[];
    float *El = reinterpret_cast<float *>(bins + K);
    if (CT) {
        for (uint32_t k = threadIdx.x; k < K; k += blockDim.x) bins[k] = 0;
        for (uint32_t k = threadIdx.x; k <= K; k += blockDim.x) El[k] = E[k];
    }
    const uint32_t M = m.M, nbx = (M + kPT - 1) / kPT;
    double pr = 0.0, pi = 0.0;
    for (uint32_t blk = blockIdx.x; blk < nbx * nbx; blk += gridDim.x) {
        bool big;
        const uint32_t I0 = (blk % nbx) * kPT, J0 = (blk / nbx) * kPT;
        const int nd = stage_block<H>(S, m, I0, J0, &big);
        if (big) psi6_disks<H, 4, CT>(S, m, I0, J0, nd, re, im, sre, sim, fail, pr, pi, El, K, bins);
        else psi6_disks<H, 2, CT>(S, m, I0, J0, nd, re, im, sre, sim, fail, pr, pi, El, K, bins);
        __syncthreads();  // S is restaged for the next block
    }
    if (CT)
        for (uint32_t k = threadIdx.x; k < K; k += blockDim.x) rows[blockIdx.x * K + k] = bins[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        pr += __shfl_xor(pr, off, 64);
        pi += __shfl_xor(pi, off, 64);
    }
    if ((threadIdx.x & 63u) == 0) wpart[threadIdx.x >> 6] = make_double2(pr, pi);
    __syncthreads();
    if (threadIdx.x == 0)
        part[blockIdx.x] = make_double2(wpart[0].x + wpart[1].x + wpart[2].x + wpart[3].x,
                                        wpart[0].y + wpart[1].y + wpart[2].y + wpart[3].y);
}

// Global psi sum from the G workgroup partials (overwrites dev->psi_re/im).
__global__ void __launch_bounds__(256) k_psi_reduce(const double2 *part, uint32_t G, DevScalars *dev) {
    __shared__ double2 wpart[4];
    double pr = 0.0, pi = 0.0;
    for (uint32_t g = threadIdx.x; g < G; g += blockDim.x) {
        pr += part[g].x;
        pi += part[g].y;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        pr += __shfl_xor(pr, off, 64);
        pi += __shfl_xor(pi, off, 64);
    }
    if ((threadIdx.x & 63u) == 0) wpart[threadIdx.x >> 6] = make_double2(pr, pi);
    __syncthreads();
    if (threadIdx.x == 0) {
        dev->psi_re = wpart[0].x + wpart[1].x + wpart[2].x + wpart[3].x;
        dev->psi_im = wpart[0].y + wpart[1].y + wpart[2].y + wpart[3].y;
    }
}

namespace {
void launch_psi6_tile(const MeasureView &m, uint32_t h, float *re, float *im, float *sre, float *sim,
                      uint32_t *fail, double2 *part, const uint32_t *gate, uint32_t G, hipStream_t st) {
    if (h == 1) k_psi6_tile<1, false><<<G, 256, 0, st>>>(m, re, im, sre, sim, fail, part, gate, nullptr, 0, nullptr);
    else if (h == 2) k_psi6_tile<2, false><<<G, 256, 0, st>>>(m, re, im, sre, sim, fail, part, gate, nullptr, 0, nullptr);
    else k_psi6_tile<3, false><<<G, 256, 0, st>>>(m, re, im, sre, sim, fail, part, gate, nullptr, 0, nullptr);
}
// The same pass also counting contacts into rows (G rows of K).
void launch_psi6_contact_tile(const MeasureView &m, uint32_t h, float *re, float *im, float *sre,
                              float *sim, uint32_t *fail, double2 *part, const float *E, uint32_t K,
                              uint32_t *rows, uint32_t G, hipStream_t st) {
    const size_t lds = (2 * (size_t)K + 1) * sizeof(uint32_t);
    if (h == 1) k_psi6_tile<1, true><<<G, 256, lds, st>>>(m, re, im, sre, sim, fail, part, nullptr, E, K, rows);
    else if (h == 2) k_psi6_tile<2, true><<<G, 256, lds, st>>>(m, re, im, sre, sim, fail, part, nullptr, E, K, rows);
    else k_psi6_tile<3, true><<<G, 256, lds, st>>>(m, re, im, sre, sim, fail, part, nullptr, E, K, rows);
}
uint32_t psi6_grid(const MeasureView &m) {
    const uint32_t nb = (m.M + kPT - 1) / kPT;
    return nb * nb < kMeasGrid ? nb * nb : kMeasGrid;
}
}  // namespace

void launch_psi6_tiled(const MeasureView &m, uint32_t h, float *re, float *im, float *sre, float *sim,
                       uint32_t *fail, void *work, hipStream_t st) {
    const uint32_t G = psi6_grid(m);
    double2 *part = static_cast<double2 *>(work);
    launch_psi6_tile(m, h, re, im, sre, sim, fail, part, nullptr, G, st);
    k_psi_reduce<<<1, 256, 0, st>>>(part, G, m.dev);
}

// Stencil h1 first; a second pass with h2 > h1 runs only if the first one's
// search fell short for some disk (flag short1, which the caller has
// cleared), decided on the device.  fail receives the second pass's verdict.
void launch_psi6_retry(const MeasureView &m, uint32_t h1, uint32_t h2, float *re, float *im,
                       float *sre, float *sim, uint32_t *short1, uint32_t *fail, void *work,
                       hipStream_t st) {
    const uint32_t G = psi6_grid(m);
    double2 *part = static_cast<double2 *>(work);
    launch_psi6_tile(m, h1, re, im, sre, sim, short1, part, nullptr, G, st);
    launch_psi6_tile(m, h2, re, im, sre, sim, fail, part, short1, G, st);
    k_psi_reduce<<<1, 256, 0, st>>>(part, G, m.dev);
}

void launch_measure_tiled(const MeasureView &m, uint32_t h1, uint32_t h2, const float *edges,
                          uint32_t K, unsigned long long *hist, float *re, float *im, float *sre,
                          float *sim, uint32_t *short1, uint32_t *fail, void *work, hipStream_t st) {
    const uint32_t G = psi6_grid(m);
    uint32_t *rows = static_cast<uint32_t *>(work);
    const size_t off = ((size_t)G * K * sizeof(uint32_t) + 15) & ~(size_t)15;
    double2 *part = reinterpret_cast<double2 *>(static_cast<char *>(work) + off);
    launch_psi6_contact_tile(m, h1, re, im, sre, sim, h2 > h1 ? short1 : fail, part, edges, K, rows, G, st);
    k_hist_rows_reduce<<<K, 256, 0, st>>>(rows, G, K, hist);
    if (h2 > h1) launch_psi6_tile(m, h2, re, im, sre, sim, fail, part, short1, G, st);
    k_psi_reduce<<<1, 256, 0, st>>>(part, G, m.dev);
}

void launch_psi6(const MeasureView &m, uint32_t h, float *re, float *im, float *sre, float *sim,
                 uint32_t *fail, const uint32_t *loc, void *work, hipStream_t st) {
    if (measure_tiled(m, h)) {
        launch_psi6_tiled(m, h, re, im, sre, sim, fail, work, st);
        return;
    }
    k_psi6<<<(m.N + 255) / 256, 256, 0, st>>>(m, (int)h, re, im, fail, loc);
}

// Coarse field: per cell, the mean psi_j over the disks of its 3 x 3 block.
__global__ void __launch_bounds__(256) k_psi6_field(MeasureView m, const float *re,
                                                    const float *im, float *fre, float *fim) {
    const uint32_t M = m.M;
    const uint32_t cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= M * M) return;
    const uint32_t ci = cell % M, cj = cell / M;
    float sr = 0.0f, si = 0.0f;
    uint32_t n = 0;
    for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di) {
            const uint32_t nb = wrapc((int)ci + di, M) + M * wrapc((int)cj + dj, M);
            for (uint32_t t = 0; t < m.cnt[nb]; ++t) {
                const uint32_t tg = m.tag[slot_at(nb, t, M * M)];
                sr += re[tg];
                si += im[tg];
                ++n;
            }
        }
    fre[cell] = n ? sr / (float)n : 0.0f;
    fim[cell] = n ? si / (float)n : 0.0f;
}

void launch_psi6_field(const MeasureView &m, const float *re, const float *im, float *fre,
                       float *fim, hipStream_t st) {
    const uint32_t nc = m.M * m.M;
    k_psi6_field<<<(nc + 255) / 256, 256, 0, st>>>(m, re, im, fre, fim);
}

// The same field from psi_j stored by cell slot (as the cell lists): the
// reads follow the cells instead of the tags, and the sums run in the same
// order, so the result is the same.
// The loads go out in two rounds (the nine counts, then the values of the
// slots they cover, at most 4 per cell here) and the sums run afterwards in
// the cell-then-slot order of k_psi6_field.
__global__ void __launch_bounds__(256) k_psi6_field_slots(MeasureView m, const float *sre,
                                                          const float *sim, float *fre, float *fim) {
    const uint32_t M = m.M, NC = M * M;
    const uint32_t cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= NC) return;
    const uint32_t ci = cell % M, cj = cell / M;
    uint32_t nb[9], cnt[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        nb[k] = wrapc((int)ci + k % 3 - 1, M) + M * wrapc((int)cj + k / 3 - 1, M);
        cnt[k] = m.cnt[nb[k]];
    }
    float vr[9][4], vi[9][4];
#pragma unroll
    for (int k = 0; k < 9; ++k)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            vr[k][t] = (uint32_t)t < cnt[k] ? sre[slot_at(nb[k], (uint32_t)t, NC)] : 0.0f;
            vi[k][t] = (uint32_t)t < cnt[k] ? sim[slot_at(nb[k], (uint32_t)t, NC)] : 0.0f;
        }
    float sr = 0.0f, si = 0.0f;
    uint32_t n = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k)
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if ((uint32_t)t < cnt[k]) {
                sr += vr[k][t];
                si += vi[k][t];
                ++n;
            }
    fre[cell] = n ? sr / (float)n : 0.0f;
    fim[cell] = n ? si / (float)n : 0.0f;
}

void launch_psi6_field_slots(const MeasureView &m, const float *sre, const float *sim, float *fre,
                             float *fim, hipStream_t st) {
    const uint32_t nc = m.M * m.M;
    k_psi6_field_slots<<<(nc + 255) / 256, 256, 0, st>>>(m, sre, sim, fre, fim);
}

// ---------------------------------------------------------------------------
// Validator: offsets in [0, w), counts within capacity, every tag exactly
// once, and no pair closer than 2 sigma in the 3 x 3 stencil (exhaustive for
// w >= 2 sigma).  Overlaps are counted ordered.
__global__ void __launch_bounds__(256) k_validate(MeasureView m, uint32_t *tag_seen) {
    const uint32_t M = m.M;
    const uint32_t cell = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long bad = 0, ov = 0;
    if (cell < M * M) {
        const uint32_t ci = cell % M, cj = cell / M;
        uint32_t n = m.cnt[cell];
        if (n > m.cap) { ++bad; n = m.cap; }
        for (uint32_t s = 0; s < n; ++s) {
            const float xi = m.x[slot_at(cell, s, M * M)], yi = m.y[slot_at(cell, s, M * M)];
            const uint32_t tg = m.tag[slot_at(cell, s, M * M)];
            if (!(xi >= 0.0f && xi < m.w && yi >= 0.0f && yi < m.w)) ++bad;
            if (tg < m.N) atomicAdd(&tag_seen[tg], 1u); else ++bad;
            for (int dj = -1; dj <= 1; ++dj)
                for (int di = -1; di <= 1; ++di) {
                    const uint32_t nb = wrapc((int)ci + di, M) + M * wrapc((int)cj + dj, M);
                    const float cwx = (float)di * m.w, cwy = (float)dj * m.w;
                    uint32_t mm = m.cnt[nb];
                    mm = mm > m.cap ? m.cap : mm;
                    for (uint32_t t = 0; t < mm; ++t) {
                        if (di == 0 && dj == 0 && t == s) continue;
                        const float dx = (m.x[slot_at(nb, t, M * M)] - xi) + cwx;
                        const float dy = (m.y[slot_at(nb, t, M * M)] - yi) + cwy;
                        if (overlap_f32(dx, dy)) ++ov;
                    }
                }
        }
    }
    if (bad) atomicAdd(&m.dev->bad, bad);
    if (ov) atomicAdd(&m.dev->overlaps, ov);
}

__global__ void k_tags_once(const uint32_t *tag_seen, uint32_t N, DevScalars *dev) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < N && tag_seen[t] != 1u) atomicAdd(&dev->bad, 1ull);
}

void launch_validate(const MeasureView &m, uint32_t *tag_seen, hipStream_t st) {
    const uint32_t nc = m.M * m.M;
    k_validate<<<(nc + 255) / 256, 256, 0, st>>>(m, tag_seen);
    k_tags_once<<<(m.N + 255) / 256, 256, 0, st>>>(tag_seen, m.N, m.dev);
}

// ---------------------------------------------------------------------------
// Absolute q position of every disk, by tag: (i W + U + S) mod (M W).
__global__ void __launch_bounds__(256) k_positions(MeasureView m, long long *X, long long *Y) {
    const uint32_t M = m.M;
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t s = gid / (M * M), cell = gid - s * (M * M);
    if (s >= m.CS || s >= m.cnt[cell]) return;
    const long long U = (long long)(m.x[gid] * 4194304.0f);
    const long long V = (long long)(m.y[gid] * 4194304.0f);
    const uint32_t tg = m.tag[gid];
    if (tg >= m.N) return;
    X[tg] = ((long long)(cell % M) * m.W + U + m.Sx) % m.Lq;
    Y[tg] = ((long long)(cell / M) * m.W + V + m.Sy) % m.Lq;
}

// Psi_6 = (sum of psi_j) / N into out[0..1] (device).
__global__ void k_psi_mean(const DevScalars *dev, double inv_n, double *out) {
    if (threadIdx.x == 0) {
        out[0] = dev->psi_re * inv_n;
        out[1] = dev->psi_im * inv_n;
    }
}

void launch_psi_mean(const DevScalars *dev, uint32_t N, double *out, hipStream_t st) {
    k_psi_mean<<<1, 64, 0, st>>>(dev, 1.0 / (double)N, out);
}

void launch_positions(const MeasureView &m, long long *X, long long *Y, hipStream_t st) {
    const uint32_t n = m.M * m.M * m.CS;
    k_positions<<<(n + 255) / 256, 256, 0, st>>>(m, X, Y);
}

}  // namespace mpmc
