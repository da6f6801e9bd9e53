// mpmc_common.hpp — definitions shared by the kernels and the host runtime of
// the MI355X MPMC hard-disk library (the library's own code; the CPU oracle is
// a separate program).
//
// Coordinates.  sigma = 1.  Every position is a multiple of q = 2^-22 and is
// stored as an fp32 offset in [0, w) inside its cell, w = W q < 4, so every
// sum or difference of offsets and displacements that the sampler forms is
// exact in fp32 (the paper keeps cell-local single-precision coordinates to
// limit cancellation, Sec. II.B); only squared distances round.
//
// Random numbers.  Philox4x32-10 (Salmon et al., SC'11) with key = seed and
// counter (sweep_lo, cell, trial, (sweep_hi << 8) | stream):
//   stream 0  trial words: w0 selects the disk, w1/w2 give the x/y step
//   stream 1  in-cell shuffle words (n_trial > 1), trial field = word / 4
//   stream 2  learned-proposal words: component and acceptance uniforms
//   stream 3  cell = 0xFFFFFFFF: per-sweep shift x, shift y, colour order
//   stream 4  learned-proposal words: the Gaussian pair
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpmc {

constexpr float kQ = 1.0f / 4194304.0f;  // 2^-22
constexpr double kQd = 1.0 / 4194304.0;
constexpr uint32_t kGlobalCell = 0xFFFFFFFFu;
constexpr int kStreamTrial = 0, kStreamShuffle = 1, kStreamLearned = 2, kStreamGlobal = 3,
              kStreamGauss = 4;

struct Words { uint32_t w0, w1, w2, w3; };

__host__ __device__ __forceinline__ uint32_t mulhi32(uint32_t a, uint32_t n) {
    return (uint32_t)(((uint64_t)a * n) >> 32);
}

// Ten Philox rounds; the Weyl key increments are applied between rounds.
__host__ __device__ __forceinline__ Words philox(uint32_t k0, uint32_t k1, uint32_t c0,
                                                 uint32_t c1, uint32_t c2, uint32_t c3) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Words{c0, c1, c2, c3};
}

__host__ __device__ __forceinline__ Words draw(uint32_t k0, uint32_t k1, uint64_t sweep,
                                               uint32_t cell, uint32_t trial, uint32_t stream) {
    return philox(k0, k1, (uint32_t)sweep, cell, trial,
                  ((uint32_t)(sweep >> 32) << 8) | stream);
}

// Per-sweep global draws: the grid shift (kx, ky) in q units, uniform in
// [0, W), and the colour order, a uniform permutation of {0,1,2,3} decoded
// from an index in [0, 24) (Sec. II.B: random shift, random sub-sweep order).
struct SweepDraws { uint32_t kx, ky, perm; };

__host__ __device__ __forceinline__ SweepDraws sweep_draws(uint32_t k0, uint32_t k1,
                                                           uint64_t sweep, uint32_t W) {
    const Words g = draw(k0, k1, sweep, kGlobalCell, 0, kStreamGlobal);
    return SweepDraws{mulhi32(g.w0, W), mulhi32(g.w1, W), mulhi32(g.w2, 24)};
}

// Colour of pass p (0..3): Lehmer decode of perm over the list (0, 1, 2, 3).
__host__ __device__ __forceinline__ uint32_t colour_of_pass(uint32_t perm, uint32_t p) {
    uint32_t avail = 0x3210u;  // 4-bit fields, remaining colours in order
    uint32_t d[3] = {perm / 6, (perm % 6) / 2, perm % 2};
    uint32_t c = 0;
    for (uint32_t e = 0; e <= p; ++e) {
        const uint32_t pick = (e < 3) ? d[e] : 0;
        c = (avail >> (4 * pick)) & 0xFu;
        // remove field `pick`
        const uint32_t lo = avail & ((1u << (4 * pick)) - 1u);
        const uint32_t hi = (pick < 7) ? (avail >> (4 * (pick + 1))) : 0u;
        avail = lo | (hi << (4 * pick));
    }
    return c;
}

// Displacement of one axis from a trial word: an odd multiple j of step_m q,
// |j| <= 2^14 - 1, symmetric about 0.
__host__ __device__ __forceinline__ float step_from_word(uint32_t word, uint32_t step_m) {
    const int32_t j = 2 * (int32_t)(word >> 18) + 1 - 16384;
    return (float)((int32_t)step_m * j) * kQ;
}

// Overlap predicate (hard disks of radius 1 overlap below centre distance 2)
// for an exact separation (dx, dy): the three fp32 roundings of
// dx*dx + dy*dy, no contraction.
__device__ __forceinline__ bool overlap_f32(float dx, float dy) {
    const float a = __fmul_rn(dx, dx);
    const float b = __fmul_rn(dy, dy);
    return __fadd_rn(a, b) < 4.0f;
}

__device__ __forceinline__ float r2_f32(float dx, float dy) {
    return __fadd_rn(__fmul_rn(dx, dx), __fmul_rn(dy, dy));
}

// Device-resident scalars of one box.
constexpr int kCountSlots = 1024;
struct CountSlot {
    unsigned long long trials, accepts;
};

struct DevScalars {
    unsigned long long sweep;     // sweeps completed
    unsigned long long trials;    // counted trials (host view: sum of the slots)
    unsigned long long accepts;   // accepted trials (host view: sum of the slots)
    long long Sx, Sy;             // accumulated shift, q units, mod M W
    unsigned int overflow;        // a cell exceeded its capacity
    unsigned int error;           // a kernel-side check failed
    double psi_re, psi_im;        // global psi sum (measurement scratch)
    unsigned long long bad, overlaps;  // validate results
    // Trial and acceptance counts, spread over slots (one per workgroup and
    // wave, modulo kCountSlots) so that atomics rarely meet on one address.
    CountSlot slots[kCountSlots];
};

// Cell lists are stored slot-major: slot s of cell c is element s * NC + c
// of the x, y and tag arrays (NC = M * M cells, CS slots allocated per cell).
// Only slots below the cell's count hold disks; the rest keep stale values
// and are never read, so a wave that walks consecutive cells reads and
// writes consecutive words of the slots in use and nothing else.
__host__ __device__ __forceinline__ uint32_t slot_at(uint32_t c, uint32_t s, uint32_t NC) {
    return s * NC + c;
}

// Everything a sweep kernel needs (cnt[c], x/y/tag slot-major as above):
// the cell lists the sweep reads, binned in its own grid (in); the lists
// binned for the next sweep that it writes (out); and where it writes the
// box's canonical state after the sweep, in this sweep's grid (can; NULL
// for launches that only time the kernel).
struct BoxView {
    const uint8_t *cnt_in;
    const float *x_in, *y_in;
    const uint32_t *tag_in;
    uint8_t *cnt_out;
    float *x_out, *y_out;
    uint32_t *tag_out;
    uint8_t *cnt_can;
    float *x_can, *y_can;
    uint32_t *tag_can;
    DevScalars *dev;
    uint32_t M, W, cap, CS;
    uint32_t step_m, n_trial;
    float w;
    uint32_t seed_lo, seed_hi;
    uint32_t offset;  // this launch works on sweep dev->sweep + offset
};

}  // namespace mpmc
