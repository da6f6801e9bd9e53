// sweep_fused.hip — one kernel launch per MPMC sweep (Sec. II.B).
//
// A workgroup owns a TILE x TILE block of cells of the shifted grid.  It
// re-bins the block plus a halo of 4 cells into LDS straight from the
// previous sweep's cell lists, runs all four colour sub-sweeps on LDS with a
// barrier between them, and writes back only its own block.  Pass p (0..3)
// updates the cells of its colour within 3 - p cells of the block: exactly
// the cells whose state the block's final state depends on, so the halo
// work reproduces what the neighbouring workgroups compute.  Because every
// random number is keyed by (seed, sweep, cell, trial), the recomputed halo
// is identical to theirs and the trajectory does not depend on TILE.
//
// In LDS a cell keeps its (at most 4) disks as centred offsets s = u - c,
// c = floor(W/2) q, so |s| <= w/2 and, for a trial position s' and a
// neighbour cell at column offset di, q_di = s' - di w is exact (|q_di| < 4)
// and dx = s_k - q_di is the exact separation whenever |dx| < 4: one
// subtraction per axis and pair, with the same overlap decision as the
// cell-local formula.  Empty slots hold a far sentinel so every pair test
// runs without branches.  Cells are stored by colour plane so that the
// lanes of a wave, which work on cells of one colour, read consecutive
// 16-byte records.
#include "mpmc_kernels.hpp"

namespace mpmc {

namespace {
constexpr int kHalo = 4;
constexpr float kFar = 1.0e6f;  // sentinel offset of an empty slot

template <int TILE>
struct Lds {
    static constexpr int R = TILE + 2 * kHalo;  // region side (new grid), even
    static constexpr int NC = R * R;
    static constexpr int NO = (R + 1) * (R + 1);  // old-grid region
    static constexpr int NA = (R / 2 - 1) * (R / 2 - 1);  // most active cells in a pass
    float4 x[NC];
    float4 y[NC];
    uint8_t cnt[NC];
    uint16_t gcnt[NO];   // per old cell: disks per wrap class, 3 bits each
    uint16_t list[NA];   // non-empty active cells of the current pass
    uint32_t wsum[17];   // per-wave counts for the compaction scan
};

// LDS index of region cell (rx, ry): colour plane, then row-major in plane.
template <int R>
__device__ __forceinline__ int pidx(int rx, int ry) {
    return ((rx & 1) | ((ry & 1) << 1)) * (R / 2) * (R / 2) + (rx >> 1) + (R / 2) * (ry >> 1);
}

__device__ __forceinline__ uint32_t wrap_add(uint32_t a, int d, uint32_t M) {
    int v = (int)a + d;
    if (v < 0) v += (int)M;
    if (v >= (int)M) v -= (int)M;
    return (uint32_t)v;
}

__device__ __forceinline__ float pick4(const float4 &v, uint32_t s) {
    const float a = (s & 1u) ? v.y : v.x;
    const float b = (s & 1u) ? v.w : v.z;
    return (s & 2u) ? b : a;
}
__device__ __forceinline__ float4 put4(float4 v, uint32_t s, float f) {
    v.x = (s == 0) ? f : v.x;
    v.y = (s == 1) ? f : v.y;
    v.z = (s == 2) ? f : v.z;
    v.w = (s == 3) ? f : v.w;
    return v;
}
__device__ __forceinline__ float comp4(const float4 &v, int s) {
    return s == 0 ? v.x : s == 1 ? v.y : s == 2 ? v.z : v.w;
}
__device__ __forceinline__ uint32_t compu4(const uint4 &v, int s) {
    return s == 0 ? v.x : s == 1 ? v.y : s == 2 ? v.z : v.w;
}
}  // namespace

struct PassCtx {
    uint64_t sweep;
    uint32_t gx0, gy0;
    int own_x, own_y;
    float cen;
};

// One colour sub-sweep over the LDS region: pass p updates the cells of
// colour (CX, CY) with region coordinates in [p+1, R-p-1).  The non-empty
// ones are compacted into a list first; each is then visited by one lane.
template <int TILE, int THREADS, int CX, int CY>
__device__ __forceinline__ void run_pass(Lds<TILE> &L, const BoxView &v, const PassCtx &ctx,
                                         int p, uint32_t &trials, uint32_t &accepts) {
    constexpr int R = Lds<TILE>::R, H = R / 2, PB = (CX | (CY << 1)) * H * H;
    const int lo = p + 1, hi = R - p - 1;
    const uint32_t M = v.M;
    int total = 0;
    for (int base = 0; base < H * H; base += THREADS) {
        const int a = base + (int)threadIdx.x;
        const bool cand = a < H * H;
        const int ax = a % H, ay = a / H;
        const int rx = 2 * ax + CX, ry = 2 * ay + CY;
        const bool live = cand && rx >= lo && rx < hi && ry >= lo && ry < hi &&
                          L.cnt[PB + (cand ? a : 0)] != 0;
        const unsigned long long bal = __ballot(live);
        const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
        if (lane == 0) L.wsum[wave] = (uint32_t)__popcll(bal);
        __syncthreads();
        uint32_t before = 0, all = 0;
#pragma unroll
        for (uint32_t q = 0; q < THREADS / 64; ++q) {
            const uint32_t cq = L.wsum[q];
            before += q < wave ? cq : 0u;
            all += cq;
        }
        const uint32_t rank = (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
        if (live) L.list[total + before + rank] = (uint16_t)a;
        total += (int)all;
        __syncthreads();
    }
    const float w = v.w, cen = ctx.cen;
    const float lo_b = -cen, hi_b = w - cen;  // in-cell range of centred offsets
    for (int j = threadIdx.x; j < total; j += THREADS) {
        const int a = L.list[j];
        const int ax = a % H, ay = a / H;
        const int rx = 2 * ax + CX, ry = 2 * ay + CY;
        const int e = PB + a;
        const uint32_t n = L.cnt[e];
        const uint32_t cell = wrap_add(ctx.gx0, rx, M) + M * wrap_add(ctx.gy0, ry, M);
        const bool own = (rx - kHalo) >= 0 && (rx - kHalo) < ctx.own_x && (ry - kHalo) >= 0 &&
                         (ry - kHalo) < ctx.own_y;
        uint32_t perm = 0x3210u;  // 4-bit slot fields
        if (v.n_trial > 1) {
            const Words wd = draw(v.seed_lo, v.seed_hi, ctx.sweep, cell, 0, kStreamShuffle);
            for (uint32_t i = n - 1; i >= 1; --i) {
                const uint32_t e2 = n - 1 - i;
                const uint32_t word = e2 == 0 ? wd.w0 : e2 == 1 ? wd.w1 : wd.w2;
                const uint32_t jj = mulhi32(word, i + 1);
                const uint32_t pi = (perm >> (4 * i)) & 0xFu, pj = (perm >> (4 * jj)) & 0xFu;
                perm &= ~((0xFu << (4 * i)) | (0xFu << (4 * jj)));
                perm |= (pj << (4 * i)) | (pi << (4 * jj));
            }
        }
        const int base_ax = a;  // ax + H * ay inside a plane
        float4 mx = L.x[e], my = L.y[e];
        for (uint32_t t = 0; t < v.n_trial; ++t) {
            const Words w4 = draw(v.seed_lo, v.seed_hi, ctx.sweep, cell, t, kStreamTrial);
            const uint32_t slot = (v.n_trial == 1) ? mulhi32(w4.w0, n)
                                                   : (perm >> (4 * (t % n))) & 0xFu;
            const float xn = pick4(mx, slot) + step_from_word(w4.w1, v.step_m);
            const float yn = pick4(my, slot) + step_from_word(w4.w2, v.step_m);
            if (own) ++trials;
            const bool inside = xn >= lo_b && xn < hi_b && yn >= lo_b && yn < hi_b;
            const float ax3[3] = {xn + w, xn, xn - w};  // q_di = s' - di w
            const float ay3[3] = {yn + w, yn, yn - w};
            bool bad = false;
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const int di = k % 3 - 1, dj = k / 3 - 1;
                const float gx = ax3[k % 3], gy = ay3[k / 3];
                if (k == 4) {
                    // own cell: every slot but the moving one
                    bad |= slot != 0 && overlap_f32(mx.x - gx, my.x - gy);
                    bad |= slot != 1 && overlap_f32(mx.y - gx, my.y - gy);
                    bad |= slot != 2 && overlap_f32(mx.z - gx, my.z - gy);
                    bad |= slot != 3 && overlap_f32(mx.w - gx, my.w - gy);
                    continue;
                }
                // neighbour (rx + di, ry + dj): its colour plane and in-plane
                // offset are compile-time constants for this colour
                            const int cxn = (CX + di) & 1, cyn = (CY + dj) & 1;
                const int offx = (CX + di + 2) / 2 - 1, offy = (CY + dj + 2) / 2 - 1;
                const int ne = (cxn | (cyn << 1)) * H * H + base_ax + offx + H * offy;
                const float4 qx = L.x[ne], qy = L.y[ne];
                bad |= overlap_f32(qx.x - gx, qy.x - gy);
                bad |= overlap_f32(qx.y - gx, qy.y - gy);
                bad |= overlap_f32(qx.z - gx, qy.z - gy);
                bad |= overlap_f32(qx.w - gx, qy.w - gy);
                // one row of neighbour records in flight at a time keeps the
                // register budget of four waves per SIMD
                if (k == 2 || k == 5) __asm__ volatile("" ::: "memory");
            }
            const bool acc = inside && !bad;
            mx = acc ? put4(mx, slot, xn) : mx;
            my = acc ? put4(my, slot, yn) : my;
            if (own && acc) ++accepts;
        }
        L.x[e] = mx;
        L.y[e] = my;
    }
}

// The work of one tile: re-bin, four colour passes, write-back, counts.
template <int TILE, int THREADS>
__device__ __forceinline__ void fused_tile(Lds<TILE> &L, const BoxView &v, uint32_t I0,
                                           uint32_t J0) {
    constexpr int R = Lds<TILE>::R;
    const uint32_t M = v.M;
    const int own_x = (M - I0 < (uint32_t)TILE) ? (int)(M - I0) : TILE;
    const int own_y = (M - J0 < (uint32_t)TILE) ? (int)(M - J0) : TILE;

    const uint64_t sweep = v.dev->sweep + v.offset;
    const SweepDraws d = sweep_draws(v.seed_lo, v.seed_hi, sweep, v.W);
    const float sx = (float)d.kx * kQ, sy = (float)d.ky * kQ;
    const float w = v.w;
    const float cen = (float)(v.W >> 1) * kQ;  // centring offset c
    const uint32_t gx0 = wrap_add(I0, -kHalo, M), gy0 = wrap_add(J0, -kHalo, M);

    // ---- re-bin the region from the previous sweep's cell lists ----------
    // New cell (I, J) takes the disks of old (I, J) that do not wrap, then
    // those of (I+1, J) wrapping in x only, (I, J+1) in y only, (I+1, J+1)
    // in both, each in old slot order.  Old region cell (ox, oy) is global
    // old cell (gx0 + ox, gy0 + oy) and feeds new region cells (ox - wx,
    // oy - wy).  Step 1 classifies every old disk once and counts the four
    // wrap classes per old cell; step 2 scatters each disk to its slot,
    // whose index follows from the class counts of the cells before it in
    // the new cell's order.  Own-block counts and tags are final here.
    constexpr int RO = R + 1;
    const float4 far4 = make_float4(kFar, kFar, kFar, kFar);
    for (int e = threadIdx.x; e < RO * RO; e += THREADS) {
        const int ox = e % RO, oy = e / RO;
        const uint32_t c = wrap_add(gx0, ox, M) + M * wrap_add(gy0, oy, M);
        const uint32_t m = v.cnt_in[c];
        const float4 px = *reinterpret_cast<const float4 *>(v.x_in + (size_t)c * 4);
        const float4 py = *reinterpret_cast<const float4 *>(v.y_in + (size_t)c * 4);
        uint32_t g = 0;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const uint32_t cls = (uint32_t)(comp4(px, s) < sx) | ((uint32_t)(comp4(py, s) < sy) << 1);
            g += ((uint32_t)s < m) ? (1u << (3 * cls)) : 0u;
        }
        L.gcnt[e] = (uint16_t)g;
        if (e < R * R) {
            L.x[e] = far4;
            L.y[e] = far4;
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < RO * RO; e += THREADS) {
        const int ox = e % RO, oy = e / RO;
        const uint32_t c = wrap_add(gx0, ox, M) + M * wrap_add(gy0, oy, M);
        const uint32_t m = v.cnt_in[c];
        const float4 px = *reinterpret_cast<const float4 *>(v.x_in + (size_t)c * 4);
        const float4 py = *reinterpret_cast<const float4 *>(v.y_in + (size_t)c * 4);
        const bool own_src = ox >= kHalo - 1 && ox <= kHalo + own_x && oy >= kHalo - 1 &&
                             oy <= kHalo + own_y;
        const uint4 tg = own_src ? *reinterpret_cast<const uint4 *>(v.tag_in + (size_t)c * 4)
                                 : make_uint4(0, 0, 0, 0);
        // class counts of the old cells before this one in each destination
        const int oxm = ox > 0 ? ox - 1 : 0, oym = oy > 0 ? oy - 1 : 0;
        const int oxp = ox < R ? ox + 1 : R;
        const uint32_t g_l = L.gcnt[oxm + RO * oy];    // (ox-1, oy)
        const uint32_t g_d = L.gcnt[ox + RO * oym];    // (ox, oy-1)
        const uint32_t g_dr = L.gcnt[oxp + RO * oym];  // (ox+1, oy-1)
        const uint32_t g_dl = L.gcnt[oxm + RO * oym];  // (ox-1, oy-1)
        const uint32_t g_me = L.gcnt[e];
        // base slot of each class in its destination, 8 bits per class
        const uint32_t b1 = g_l & 7u;
        const uint32_t b2 = (g_d & 7u) + ((g_dr >> 3) & 7u);
        const uint32_t b3 = (g_dl & 7u) + ((g_d >> 3) & 7u) + ((g_l >> 6) & 7u);
        const uint32_t bases = (b1 << 8) | (b2 << 16) | (b3 << 24);
        // destination of each class: (ox - wx, oy - wy), inside the region?
        const bool in0 = ox < R && oy < R, in1 = ox >= 1 && oy < R;
        const bool in2 = ox < R && oy >= 1, in3 = ox >= 1 && oy >= 1;
        const uint32_t ok = (uint32_t)in0 | ((uint32_t)in1 << 1) | ((uint32_t)in2 << 2) |
                            ((uint32_t)in3 << 3);
        const int d0 = pidx<R>(ox, oy), d1 = pidx<R>(ox - 1, oy);
        const int d2 = pidx<R>(ox, oy - 1), d3 = pidx<R>(ox - 1, oy - 1);
        // own-block destinations get their tags written here
        const int ex = ox - kHalo, ey = oy - kHalo;
        uint32_t seen = 0;  // 3-bit counters per class within this old cell
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const float xs = comp4(px, s), ys = comp4(py, s);
            const uint32_t wx = xs < sx, wy = ys < sy, cls = wx | (wy << 1);
            const uint32_t slot = ((bases >> (8 * cls)) & 0xFFu) + ((seen >> (3 * cls)) & 7u);
            seen += 1u << (3 * cls);
            const bool go = (uint32_t)s < m && ((ok >> cls) & 1u) && slot < 4;
            if (!go) continue;
            const int dst = cls == 0 ? d0 : cls == 1 ? d1 : cls == 2 ? d2 : d3;
            const float u = ((xs - sx) + (wx ? w : 0.0f)) - cen;
            const float t = ((ys - sy) + (wy ? w : 0.0f)) - cen;
            reinterpret_cast<float *>(&L.x[dst])[slot] = u;
            reinterpret_cast<float *>(&L.y[dst])[slot] = t;
            const int dxo = ex - (int)wx, dyo = ey - (int)wy;
            if (dxo >= 0 && dxo < own_x && dyo >= 0 && dyo < own_y) {
                const size_t oc = (size_t)(I0 + dxo) + (size_t)M * (J0 + dyo);
                v.tag_out[oc * 4 + slot] = compu4(tg, s);
            }
        }
        if (in0) {  // the count of new cell (ox, oy)
            const uint32_t g_r = L.gcnt[oxp + RO * oy];        // (ox+1, oy)
            const uint32_t g_u = L.gcnt[ox + RO * (oy + 1)];   // (ox, oy+1)
            const uint32_t g_ur = L.gcnt[oxp + RO * (oy + 1)]; // (ox+1, oy+1)
            const uint32_t n = (g_me & 7u) + ((g_r >> 3) & 7u) + ((g_u >> 6) & 7u) +
                               ((g_ur >> 9) & 7u);
            if (n > 4) atomicOr(&v.dev->overflow, 1u);
            const uint32_t nc = n > 4 ? 4 : n;
            L.cnt[d0] = (uint8_t)nc;
            if (ex >= 0 && ex < own_x && ey >= 0 && ey < own_y)
                v.cnt_out[(size_t)(I0 + ex) + (size_t)M * (J0 + ey)] = (uint8_t)nc;
        }
    }
    __syncthreads();

    // ---- four colour sub-sweeps --------------------------------------------
    PassCtx ctx;
    ctx.sweep = sweep;
    ctx.gx0 = gx0;
    ctx.gy0 = gy0;
    ctx.own_x = own_x;
    ctx.own_y = own_y;
    ctx.cen = cen;
    uint32_t trials = 0, accepts = 0;
    for (int p = 0; p < 4; ++p) {
        // I0 and J0 are even, so the colour parity in region coordinates
        // equals the global one; each colour has its own instantiation with
        // compile-time neighbour offsets
        switch (colour_of_pass(d.perm, p)) {
        case 0: run_pass<TILE, THREADS, 0, 0>(L, v, ctx, p, trials, accepts); break;
        case 1: run_pass<TILE, THREADS, 1, 0>(L, v, ctx, p, trials, accepts); break;
        case 2: run_pass<TILE, THREADS, 0, 1>(L, v, ctx, p, trials, accepts); break;
        default: run_pass<TILE, THREADS, 1, 1>(L, v, ctx, p, trials, accepts); break;
        }
        __syncthreads();
    }

    // ---- write the own block's offsets back (cell-local, slots >= n as 0) ---
    for (int e = threadIdx.x; e < TILE * TILE; e += THREADS) {
        const int ox = e % TILE, oy = e / TILE;
        if (ox >= own_x || oy >= own_y) continue;
        const int li = pidx<R>(ox + kHalo, oy + kHalo);
        const uint32_t n = L.cnt[li];
        const float4 sx4 = L.x[li], sy4 = L.y[li];
        float4 ux, uy;
        ux.x = n > 0 ? sx4.x + cen : 0.0f;
        ux.y = n > 1 ? sx4.y + cen : 0.0f;
        ux.z = n > 2 ? sx4.z + cen : 0.0f;
        ux.w = n > 3 ? sx4.w + cen : 0.0f;
        uy.x = n > 0 ? sy4.x + cen : 0.0f;
        uy.y = n > 1 ? sy4.y + cen : 0.0f;
        uy.z = n > 2 ? sy4.z + cen : 0.0f;
        uy.w = n > 3 ? sy4.w + cen : 0.0f;
        const size_t c = (size_t)(I0 + ox) + (size_t)M * (J0 + oy);
        *reinterpret_cast<float4 *>(v.x_out + c * 4) = ux;
        *reinterpret_cast<float4 *>(v.y_out + c * 4) = uy;
    }
    count_trials(v.dev, trials, accepts);
}

template <int TILE, int THREADS>
__global__ void __launch_bounds__(THREADS) k_fused(BoxView v, uint32_t ntx, uint32_t nty,
                                                   uint32_t per_xcd) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    Lds<TILE> &L = *reinterpret_cast<Lds<TILE> *>(lds_raw);
    // Consecutive workgroups go to different XCDs; give each XCD a
    // contiguous run of tiles so that shared halo cells meet in its L2.
    const uint32_t tile = (blockIdx.x % 8u) * per_xcd + blockIdx.x / 8u;
    if (tile >= ntx * nty) return;
    fused_tile<TILE, THREADS>(L, v, (tile % ntx) * TILE, (tile / ntx) * TILE);
}

// Persistent form for a batch of independent boxes: workgroups stride over
// a work list of (box, tile) items, item = box << 20 | tile.  All boxes of a
// batch advance in step, so one buffer parity serves them all.
template <int TILE, int THREADS>
__global__ void __launch_bounds__(THREADS) k_fused_batch(const BoxView *views,
                                                         const uint32_t *items, uint32_t n_items,
                                                         uint32_t parity, uint32_t offset) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    Lds<TILE> &L = *reinterpret_cast<Lds<TILE> *>(lds_raw);
    for (uint32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const uint32_t item = items[it], box = item >> 20, tile = item & 0xFFFFFu;
        BoxView v = views[2 * box + parity];
        v.offset = offset;
        const uint32_t ntx = (v.M + TILE - 1) / TILE;
        fused_tile<TILE, THREADS>(L, v, (tile % ntx) * TILE, (tile / ntx) * TILE);
        __syncthreads();
    }
}

namespace {
template <int TILE, int THREADS>
void launch_t(const BoxView &v, hipStream_t st) {
    const uint32_t ntx = (v.M + TILE - 1) / TILE, nty = ntx;
    const uint32_t nt = ntx * nty, per_xcd = (nt + 7) / 8;
    const size_t lds = sizeof(Lds<TILE>);
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)k_fused<TILE, THREADS>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        attr = true;
    }
    k_fused<TILE, THREADS><<<8 * per_xcd, THREADS, lds, st>>>(v, ntx, nty, per_xcd);
}

template <int TILE, int THREADS>
void launch_batch_t(const BoxView *views, const uint32_t *items, uint32_t n_items, uint32_t grid,
                    uint32_t parity, uint32_t offset, hipStream_t st) {
    const size_t lds = sizeof(Lds<TILE>);
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)k_fused_batch<TILE, THREADS>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        attr = true;
    }
    k_fused_batch<TILE, THREADS><<<grid, THREADS, lds, st>>>(views, items, n_items, parity, offset);
}

template <int TILE, int THREADS>
int occupancy_t() {
    int blocks = 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_fused_batch<TILE, THREADS>, THREADS,
                                                       sizeof(Lds<TILE>));
    return blocks;
}

struct Entry {
    uint32_t tile, threads;
    void (*fn)(const BoxView &, hipStream_t);
    void (*batch)(const BoxView *, const uint32_t *, uint32_t, uint32_t, uint32_t, uint32_t,
                  hipStream_t);
    int (*occ)();
};
const Entry kShapes[] = {
    {8, 64, launch_t<8, 64>, launch_batch_t<8, 64>, occupancy_t<8, 64>},       {8, 128, launch_t<8, 128>, launch_batch_t<8, 128>, occupancy_t<8, 128>},
    {16, 128, launch_t<16, 128>, launch_batch_t<16, 128>, occupancy_t<16, 128>},   {16, 256, launch_t<16, 256>, launch_batch_t<16, 256>, occupancy_t<16, 256>},
    {24, 256, launch_t<24, 256>, launch_batch_t<24, 256>, occupancy_t<24, 256>},   {32, 256, launch_t<32, 256>, launch_batch_t<32, 256>, occupancy_t<32, 256>},
    {32, 512, launch_t<32, 512>, launch_batch_t<32, 512>, occupancy_t<32, 512>},   {48, 512, launch_t<48, 512>, launch_batch_t<48, 512>, occupancy_t<48, 512>},
    {48, 1024, launch_t<48, 1024>, launch_batch_t<48, 1024>, occupancy_t<48, 1024>}, {56, 1024, launch_t<56, 1024>, launch_batch_t<56, 1024>, occupancy_t<56, 1024>},
};
}  // namespace

const FusedShape *fused_shapes(uint32_t *count) {
    static FusedShape s[sizeof(kShapes) / sizeof(kShapes[0])];
    for (size_t i = 0; i < sizeof(kShapes) / sizeof(kShapes[0]); ++i)
        s[i] = FusedShape{kShapes[i].tile, kShapes[i].threads};
    *count = (uint32_t)(sizeof(kShapes) / sizeof(kShapes[0]));
    return s;
}

bool fused_supported(const BoxView &v, const FusedShape &s) {
    if (v.CS != 4 || v.cap > 4) return false;
    // the halo region must not wrap onto itself: every index below is
    // reduced modulo M with a single conditional subtraction
    if (s.tile + 2 * kHalo > v.M || (s.tile & 1u)) return false;
    for (const Entry &e : kShapes)
        if (e.tile == s.tile && e.threads == s.threads) return true;
    return false;
}

void launch_fused_batch(const BoxView *views, const uint32_t *items, uint32_t n_items,
                        uint32_t parity, uint32_t offset, const FusedShape &s, hipStream_t st) {
    for (const Entry &e : kShapes)
        if (e.tile == s.tile && e.threads == s.threads) {
            int dev = 0, cus = 0;
            (void)hipGetDevice(&dev);
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            const int per_cu = e.occ() > 0 ? e.occ() : 1;
            uint32_t grid = (uint32_t)(cus > 0 ? cus : 256) * (uint32_t)per_cu;
            if (grid > n_items) grid = n_items;
            if (grid == 0) return;
            e.batch(views, items, n_items, grid, parity, offset, st);
            return;
        }
}

void launch_fused_sweep(const BoxView &v, const FusedShape &s, hipStream_t st) {
    for (const Entry &e : kShapes)
        if (e.tile == s.tile && e.threads == s.threads) {
            e.fn(v, st);
            return;
        }
}

}  // namespace mpmc
