// sweep_simple.hip — the straightforward schedule of one MPMC sweep (Sec.
// II.B): one kernel per colour sub-sweep with one thread per active cell
// reading its 3 x 3 neighbourhood from global memory, on cell lists already
// binned in the sweep's shifted grid, then a re-bin kernel into the next
// sweep's grid.  It is the baseline the fused tile kernel is checked
// against and the fallback for boxes too small to tile.
#include "mpmc_kernels.hpp"

namespace mpmc {

// New cell (I, J) of the grid shifted by s: the disks of old (I, J) that do
// not wrap, then those of (I+1, J) wrapping in x only, (I, J+1) wrapping in y
// only and (I+1, J+1) wrapping in both, each in old slot order.  Offsets move
// by -s (+w when they wrap), exactly.
__global__ void __launch_bounds__(256) k_rebin(BoxView v) {
    const uint32_t M = v.M;
    const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= M * M) return;
    const uint32_t I = idx % M, J = idx / M;
    const uint64_t sweep = v.dev->sweep + v.offset;
    const SweepDraws d = sweep_draws(v.seed_lo, v.seed_hi, sweep, v.W);
    const float sx = (float)d.kx * kQ, sy = (float)d.ky * kQ;
    const uint32_t NC = M * M;
    uint32_t n = 0;
    for (uint32_t src = 0; src < 4; ++src) {
        const uint32_t di = src & 1u, dj = src >> 1;
        const uint32_t i = (I + di == M) ? 0 : I + di;
        const uint32_t j = (J + dj == M) ? 0 : J + dj;
        const uint32_t c = i + M * j;
        const uint32_t m = v.cnt_in[c];
        for (uint32_t s = 0; s < m; ++s) {
            float u = v.x_in[slot_at(c, s, NC)] - sx;
            float w = v.y_in[slot_at(c, s, NC)] - sy;
            const uint32_t wx = u < 0.0f, wy = w < 0.0f;
            if (wx != di || wy != dj) continue;
            if (wx) u += v.w;
            if (wy) w += v.w;
            if (n < v.cap) {
                const uint32_t o = slot_at(idx, n, NC);
                v.x_out[o] = u;
                v.y_out[o] = w;
                v.tag_out[o] = v.tag_in[slot_at(c, s, NC)];
                ++n;
            } else {
                atomicOr(&v.dev->overflow, 1u);
            }
        }
    }
    v.cnt_out[idx] = (uint8_t)n;
}

// One colour sub-sweep on the state in (cnt_out, x_out, y_out).
__global__ void __launch_bounds__(256) k_pass(BoxView v, uint32_t pass) {
    const uint32_t M = v.M, h = M / 2;
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t sweep = v.dev->sweep + v.offset;
    const SweepDraws d = sweep_draws(v.seed_lo, v.seed_hi, sweep, v.W);
    const uint32_t colour = colour_of_pass(d.perm, pass);
    uint32_t trials = 0, accepts = 0;
    if (t < h * h) {
        const uint32_t ci = 2 * (t % h) + (colour & 1u);
        const uint32_t cj = 2 * (t / h) + (colour >> 1);
        const uint32_t cell = ci + M * cj;
        const uint32_t n = v.cnt_out[cell];
        if (n > 0) {
            uint32_t perm[8];
            if (v.n_trial > 1) {
                for (uint32_t s = 0; s < n; ++s) perm[s] = s;
                Words wd{0, 0, 0, 0};
                for (uint32_t i = n - 1; i >= 1; --i) {
                    const uint32_t e = n - 1 - i;
                    if ((e & 3u) == 0)
                        wd = draw(v.seed_lo, v.seed_hi, sweep, cell, e >> 2, kStreamShuffle);
                    const uint32_t word = (e & 3u) == 0 ? wd.w0 : (e & 3u) == 1 ? wd.w1
                                        : (e & 3u) == 2 ? wd.w2 : wd.w3;
                    const uint32_t j = mulhi32(word, i + 1);
                    const uint32_t tmp = perm[i];
                    perm[i] = perm[j];
                    perm[j] = tmp;
                }
            }
            const uint32_t im = (ci == 0) ? M - 1 : ci - 1, ip = (ci == M - 1) ? 0 : ci + 1;
            const uint32_t jm = (cj == 0) ? M - 1 : cj - 1, jp = (cj == M - 1) ? 0 : cj + 1;
            const uint32_t cols[3] = {im, ci, ip}, rows[3] = {jm, cj, jp};
            for (uint32_t tr = 0; tr < v.n_trial; ++tr) {
                const Words w4 = draw(v.seed_lo, v.seed_hi, sweep, cell, tr, kStreamTrial);
                const uint32_t slot = (v.n_trial == 1) ? mulhi32(w4.w0, n) : perm[tr % n];
                const uint32_t k = slot_at(cell, slot, M * M);
                const float xn = v.x_out[k] + step_from_word(w4.w1, v.step_m);
                const float yn = v.y_out[k] + step_from_word(w4.w2, v.step_m);
                ++trials;
                if (!(xn >= 0.0f && xn < v.w && yn >= 0.0f && yn < v.w)) continue;
                bool bad = false;
                for (int dj = 0; dj < 3 && !bad; ++dj)
                    for (int di = 0; di < 3 && !bad; ++di) {
                        const uint32_t nb = cols[di] + M * rows[dj];
                        const float cwx = (float)(di - 1) * v.w, cwy = (float)(dj - 1) * v.w;
                        const uint32_t m = v.cnt_out[nb];
                        for (uint32_t s = 0; s < m; ++s) {
                            if (nb == cell && s == slot) continue;
                            const float dx = (v.x_out[slot_at(nb, s, M * M)] - xn) + cwx;
                            const float dy = (v.y_out[slot_at(nb, s, M * M)] - yn) + cwy;
                            if (overlap_f32(dx, dy)) { bad = true; break; }
                        }
                    }
                if (bad) continue;
                v.x_out[k] = xn;
                v.y_out[k] = yn;
                ++accepts;
            }
        }
    }
    count_trials(v.dev, trials, accepts);
}

// Advances the device sweep counter by `count` and the accumulated shift by
// the shifts of those sweeps.
// One wave: lane l adds the shifts of sweeps l, l + 64, ...; the sums are
// reduced across the wave and applied once (modulo the box side).
__global__ void k_advance(DevScalars *dev, uint32_t seed_lo, uint32_t seed_hi, uint32_t W,
                          long long Lq, uint32_t count) {
    if (blockIdx.x != 0) return;
    const unsigned long long s = dev->sweep;
    unsigned long long sx = 0, sy = 0;
    for (uint32_t g = threadIdx.x; g < count; g += 64) {
        const SweepDraws d = sweep_draws(seed_lo, seed_hi, s + g, W);
        sx += d.kx;
        sy += d.ky;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        sx += __shfl_xor(sx, off, 64);
        sy += __shfl_xor(sy, off, 64);
    }
    if (threadIdx.x == 0) {
        dev->Sx = (long long)(((unsigned long long)dev->Sx + sx) % (unsigned long long)Lq);
        dev->Sy = (long long)(((unsigned long long)dev->Sy + sy) % (unsigned long long)Lq);
        dev->sweep = s + count;
    }
}

// The same for every box of a batch, one thread per box.
__global__ void k_advance_batch(const AdvanceDesc *desc, uint32_t nbox, uint32_t count) {
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbox) return;
    const AdvanceDesc a = desc[b];
    unsigned long long s = a.dev->sweep;
    long long Sx = a.dev->Sx, Sy = a.dev->Sy;
    for (uint32_t g = 0; g < count; ++g) {
        const SweepDraws d = sweep_draws(a.seed_lo, a.seed_hi, s + g, a.W);
        Sx = (Sx + d.kx) % a.Lq;
        Sy = (Sy + d.ky) % a.Lq;
    }
    a.dev->Sx = Sx;
    a.dev->Sy = Sy;
    a.dev->sweep = s + count;
}

void launch_advance_batch(const AdvanceDesc *desc, uint32_t nbox, uint32_t count, hipStream_t st) {
    k_advance_batch<<<(nbox + 63) / 64, 64, 0, st>>>(desc, nbox, count);
}

BoxView in_place(const BoxView &v) {
    BoxView p = v;
    p.cnt_out = const_cast<uint8_t *>(v.cnt_in);
    p.x_out = const_cast<float *>(v.x_in);
    p.y_out = const_cast<float *>(v.y_in);
    p.tag_out = const_cast<uint32_t *>(v.tag_in);
    return p;
}

void launch_rebin(const BoxView &v, hipStream_t st) {
    const uint32_t nc = v.M * v.M;
    k_rebin<<<(nc + 255) / 256, 256, 0, st>>>(v);
}

// The four passes on the input lists in place (they become the canonical
// state), then the re-bin into the next sweep's grid.
void launch_simple_sweep(const BoxView &v, hipStream_t st) {
    const BoxView pv = in_place(v);
    const uint32_t na = (v.M / 2) * (v.M / 2);
    for (uint32_t p = 0; p < 4; ++p) k_pass<<<(na + 255) / 256, 256, 0, st>>>(pv, p);
    BoxView rv = v;
    rv.offset = v.offset + 1;
    launch_rebin(rv, st);
}

void launch_advance(DevScalars *dev, uint32_t seed_lo, uint32_t seed_hi, uint32_t W,
                    long long Lq, uint32_t count, hipStream_t st) {
    k_advance<<<1, 64, 0, st>>>(dev, seed_lo, seed_hi, W, Lq, count);
}

}  // namespace mpmc
