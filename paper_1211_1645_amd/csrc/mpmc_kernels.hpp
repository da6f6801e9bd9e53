// mpmc_kernels.hpp — device helpers and launch wrappers of the MPMC library.
#pragma once
#include "mpmc_common.hpp"

namespace mpmc {

// Workgroup sum of the per-lane trial and acceptance counts: a wave
// reduction, one LDS atomic per wave, then one 64-bit global atomic per
// workgroup into slot (blockIdx mod 64).  Every thread of the workgroup must
// call it (it contains barriers).
// Sum over the wave of a small per-lane count, one bit plane per ballot.
__device__ __forceinline__ uint32_t wave_sum_bits(uint32_t v) {
    uint32_t s = 0;
    for (int b = 0; b < 32 && __ballot((v >> b) != 0u) != 0ull; ++b)
        s += (uint32_t)__popcll(__ballot((v >> b) & 1u)) << b;
    return s;
}

// Adds the wave's trial and acceptance counts (per lane t, a) to the box
// totals: lane 0 adds the wave sums to one count slot, chosen by workgroup
// and wave.  Every lane of the wave must call it; no barrier is involved.
__device__ __forceinline__ void count_trials(DevScalars *dev, uint32_t t, uint32_t a) {
    const uint32_t st = wave_sum_bits(t), sa = wave_sum_bits(a);
    if ((threadIdx.x & 63u) == 0 && st != 0) {
        const uint32_t s = (blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) % kCountSlots;
        atomicAdd(&dev->slots[s].trials, (unsigned long long)st);
        atomicAdd(&dev->slots[s].accepts, (unsigned long long)sa);
    }
}

// sweep_simple.hip
// passes in place on v's input lists, then the re-bin of them into v's
// output lists for sweep dev->sweep + offset + 1
void launch_simple_sweep(const BoxView &v, hipStream_t st);
// the re-bin alone: v's input lists into v's output lists, binned in the
// grid of sweep dev->sweep + offset
void launch_rebin(const BoxView &v, hipStream_t st);
// v with its output lists set to its input lists
BoxView in_place(const BoxView &v);
void launch_advance(DevScalars *dev, uint32_t seed_lo, uint32_t seed_hi, uint32_t W,
                    long long Lq, uint32_t count, hipStream_t st);

// sweep_fused.hip
struct FusedShape { uint32_t tile, threads; };
bool fused_supported(const BoxView &v, const FusedShape &s);
const FusedShape *fused_shapes(uint32_t *count);
// stamps (NULL normally): kStampWords realtime-clock words per tile, for
// the phase profile
constexpr uint32_t kStampWords = 9;
void launch_fused_sweep(const BoxView &v, const FusedShape &s, hipStream_t st,
                        unsigned long long *stamps = nullptr);
// views[2 b + parity]: box b read from buffer `parity`; items: box << 20 | tile
void launch_fused_batch(const BoxView *views, const uint32_t *items, uint32_t n_items,
                        uint32_t parity, uint32_t offset, const FusedShape &s, hipStream_t st);
struct AdvanceDesc {
    DevScalars *dev;
    uint32_t seed_lo, seed_hi, W;
    long long Lq;
};
void launch_advance_batch(const AdvanceDesc *desc, uint32_t nbox, uint32_t count, hipStream_t st);

// measure.hip
struct MeasureView {
    const uint8_t *cnt;
    const float *x, *y;
    const uint32_t *tag;
    DevScalars *dev;
    uint32_t M, W, cap, CS, N;
    float w;
    long long Sx, Sy, Lq;
};
// h: stencil half-width in cells (1 when w covers the histogram range)
// Kernels over disks take loc[tag] = slot_at(cell, slot, M * M) (launch_locate).
void launch_locate(const MeasureView &m, uint32_t *loc, hipStream_t st);
// the contact and psi_6 kernels stage 16 x 16 cell blocks in LDS (and need
// no loc) when cells hold at most 4 disks and the stencil half-width h <= 3
bool measure_tiled(const MeasureView &m, uint32_t h);
// work: device scratch of measure_work_bytes(K) bytes for the tiled kernels
size_t measure_work_bytes(uint32_t K);
void launch_contact_hist(const MeasureView &m, const float *edges, uint32_t K, uint32_t h,
                         unsigned long long *hist, const uint8_t *sel, const uint32_t *loc,
                         void *work, hipStream_t st);
// psi_j by tag into re, im; the staged kernels (measure_tiled) also write it
// by cell slot into sre, sim (CS * M * M each; may be NULL)
void launch_psi6(const MeasureView &m, uint32_t h, float *re, float *im, float *sre, float *sim,
                 uint32_t *fail, const uint32_t *loc, void *work, hipStream_t st);
// psi6 with stencil h1, then h2 on the device only where h1 fell short (tiled
// kernels only; h1 < h2).
void launch_psi6_retry(const MeasureView &m, uint32_t h1, uint32_t h2, float *re, float *im,
                       float *sre, float *sim, uint32_t *short1, uint32_t *fail, void *work,
                       hipStream_t st);
// The asynchronous measurement's staged pass: the contact histogram (into
// hist, exact for any stencil h1 >= the one the histogram range needs) and
// psi_j with stencil h1 in one scan; then psi_j with h2 > h1 on the device
// only where h1 fell short (flag short1, cleared by the caller; h2 == h1:
// no second pass, and fail takes the first pass's verdict).
void launch_measure_tiled(const MeasureView &m, uint32_t h1, uint32_t h2, const float *edges,
                          uint32_t K, unsigned long long *hist, float *re, float *im, float *sre,
                          float *sim, uint32_t *short1, uint32_t *fail, void *work, hipStream_t st);
// the 3 x 3 cell field from psi_j by tag, or (same result) by cell slot
void launch_psi6_field(const MeasureView &m, const float *re, const float *im, float *fre,
                       float *fim, hipStream_t st);
void launch_psi6_field_slots(const MeasureView &m, const float *sre, const float *sim, float *fre,
                             float *fim, hipStream_t st);
void launch_validate(const MeasureView &m, uint32_t *tag_seen, hipStream_t st);
void launch_positions(const MeasureView &m, long long *X, long long *Y, hipStream_t st);
// out[0..1] = (psi_re, psi_im) / N from the device sums
void launch_psi_mean(const DevScalars *dev, uint32_t N, double *out, hipStream_t st);

// Positional order.  Structure factor at nq wave vectors (2 pi / L)(h, k)
// (device hk[2 nq], S[nq]); work: rho_work_bytes(m, nq) bytes.
size_t rho_work_bytes(const MeasureView &m, uint32_t nq);
void launch_structure_factor(const MeasureView &m, const int32_t *hk, uint32_t nq, double *S,
                             void *work, hipStream_t st);
// chi_j = exp(i (2 pi / L)(h X_j + k Y_j)) by tag
void launch_chi(const MeasureView &m, int32_t h, int32_t k, float *re, float *im, hipStream_t st);
// C_q(r) windows b < B of half-width 1 around b dr (dr a multiple of 2^-22,
// top = (B - 1) dr + 1 < min(L / 2, 512)), stencil half-width R >= top / w + 1
// cells; sums over unordered pairs into num[B], cnt[B] (overwritten);
// work: cq_work_bytes(m, B) bytes.
size_t cq_work_bytes(const MeasureView &m, uint32_t B);
void launch_cq(const MeasureView &m, double qx, double qy, double dr, uint32_t B, int R,
               double top, void *work, double *num, unsigned long long *cnt, hipStream_t st);

}  // namespace mpmc
