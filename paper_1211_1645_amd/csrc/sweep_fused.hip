// sweep_fused.hip — one kernel launch per MPMC sweep (Sec. II.B).
//
// The cell lists a sweep reads are already binned in that sweep's shifted
// grid (the previous launch re-binned them).  A workgroup owns a TILE x TILE
// block of cells.  It loads the block, extended by one row and column on
// the +x and +y sides, plus a halo of 4 cells into LDS, runs all four
// colour sub-sweeps there with a barrier between them, and then
//   - writes its own block's final state (the canonical state of the box
//     after this sweep), and
//   - re-bins the extended block into the next sweep's grid and writes the
//     block's cells of that grid: new cell (I, J) draws only on old cells
//     (I..I+1, J..J+1), all inside the extended block.
// Pass p (0..3) updates the cells of its colour within 3 - p cells of the
// extended block: exactly the cells its final state depends on, so the
// halo work reproduces what the neighbouring workgroups compute.  Every
// random number is keyed by (seed, sweep, cell, trial), so the recomputed
// halo is identical to theirs and the trajectory does not depend on TILE.
//
// In LDS a cell keeps its (at most 4) disks as centred offsets s = u - c
// (four slots per record, or two with a side table for the rare fuller
// cells),
// c = floor(W/2) q, so |s| <= w/2 and, for a trial position s' and a
// neighbour cell at column offset di, q_di = s' - di w is exact (|q_di| < 4)
// and dx = s_k - q_di is the exact separation whenever |dx| < 4: one
// subtraction per axis and pair, with the same overlap decision as the
// cell-local formula.  Empty slots hold a far sentinel so every pair test
// runs without branches.  Cells are stored by colour plane so that the
// lanes of a wave, which work on cells of one colour, read consecutive
// records.
#include <type_traits>

#include "mpmc_kernels.hpp"

namespace mpmc {

#define MPMC_GLOBAL __attribute__((address_space(1)))

// BoxView with its buffers typed as global memory.  A view read from memory
// (the batch work list) would otherwise leave generic pointers behind, and
// every access through them would compile to a flat instruction.
struct GlobalView {
    const MPMC_GLOBAL uint8_t *cnt_in;
    const MPMC_GLOBAL float *x_in, *y_in;
    const MPMC_GLOBAL uint32_t *tag_in;
    MPMC_GLOBAL uint8_t *cnt_out;
    MPMC_GLOBAL float *x_out, *y_out;
    MPMC_GLOBAL uint32_t *tag_out;
    MPMC_GLOBAL uint8_t *cnt_can;
    MPMC_GLOBAL float *x_can, *y_can;
    MPMC_GLOBAL uint32_t *tag_can;
    MPMC_GLOBAL DevScalars *dev;
    uint32_t M, W, cap, CS;
    uint32_t step_m, n_trial;
    float w;
    uint32_t seed_lo, seed_hi;
    uint32_t offset;
};

namespace {
constexpr int kHalo = 4;
constexpr float kFar = 1.0e6f;  // sentinel offset of an empty slot

// Four-slot records: every cell of the region keeps up to four disks.
template <int TILE_>
struct Lds {
    static constexpr int TILE = TILE_;
    static constexpr bool kTwo = false;
    static constexpr int RL = TILE + 2 * kHalo + 1;  // loaded region side
    static constexpr int R = RL + 1;                 // allocated side (even)
    static constexpr int NC = R * R;
    static constexpr int TE = TILE + 1;              // extended block side
    float4 x[NC];
    float4 y[NC];
    uint8_t cnt[NC];
    uint16_t gcnt[TE * TE];  // re-bin: per old cell, disks per wrap class, 3 bits each
    uint32_t big[16];        // per wave: a cell it loaded holds more than two disks
};

// Two-slot records (x0, x1, y0, y1), half the LDS of the four-slot form, so
// that a larger tile still fits four workgroups per CU.  Slots 2 and 3 of
// the few cells of more than two disks go to a side table of kSide
// entries; a region with more such cells runs as four-slot sub-tiles.
constexpr int kSide = 32;         // side-table entries of a two-slot region
constexpr uint8_t kNoSide = 0xFF;  // a cell without a side entry
template <int TILE_>
struct Lds2 {
    static constexpr int TILE = TILE_;
    static constexpr bool kTwo = true;
    static constexpr int RL = TILE + 2 * kHalo + 1;
    static constexpr int R = RL + 1;
    static constexpr int NC = R * R;
    static constexpr int TE = TILE + 1;
    float4 xy[NC];
    float4 side[kSide];         // crowded cells' slots 2 and 3: x2, x3, y2, y3
    uint8_t cnt[NC];
    uint8_t sidx[NC];           // crowded regions only: the cell's side entry or kNoSide
    uint16_t gcnt[TE * TE];
    uint16_t side_at[kSide];    // region coordinates of a side entry's cell, x | y << 8
    uint32_t big[16];
    uint32_t nside;
};

// Side of the four-slot sub-tiles that stand in for a two-slot tile of side
// TILE (two by two of them; even, so that colours keep their parity).
template <int TILE>
constexpr int sub_tile() { return ((TILE / 2) + 1) & ~1; }

// LDS index of region cell (rx, ry): colour plane, then row-major in plane.
template <int R>
__device__ __forceinline__ int pidx(int rx, int ry) {
    return ((rx & 1) | ((ry & 1) << 1)) * (R / 2) * (R / 2) + (rx >> 1) + (R / 2) * (ry >> 1);
}

// threadIdx.x through an opaque move: in the batch kernel's work loop the
// values derived from it are then recomputed for each item instead of being
// hoisted out of the loop and kept live in registers throughout.
__device__ __forceinline__ int opaque_tid() {
    int t;
    __asm__ volatile("v_mov_b32 %0, %1" : "=v"(t) : "v"((int)threadIdx.x));
    return t;
}

__device__ __forceinline__ uint32_t wrap_add(uint32_t a, int d, uint32_t M) {
    int v = (int)a + d;
    if (v < 0) v += (int)M;
    if (v >= (int)M) v -= (int)M;
    return (uint32_t)v;
}

// Element i of a buffer through a 32-bit byte offset, so that the access
// compiles to a scalar base plus one 32-bit vector offset (every buffer of a
// box is below 4 GiB, which the geometry check guarantees).
template <typename T>
__device__ __forceinline__ T &el(T *p, uint32_t i) {
    return *(T *)((char *)p + i * (uint32_t)sizeof(T));
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

// The records of region cell e as four-wide x and y vectors (in the two-slot
// layout slots 2 and 3 read as the far sentinel), and their write-back.
template <int T>
__device__ __forceinline__ void rec_get(const Lds<T> &L, int e, float4 &mx, float4 &my) {
    mx = L.x[e];
    my = L.y[e];
}
template <int T>
__device__ __forceinline__ void rec_get(const Lds2<T> &L, int e, float4 &mx, float4 &my) {
    const float4 r = L.xy[e];
    mx = make_float4(r.x, r.y, kFar, kFar);
    my = make_float4(r.z, r.w, kFar, kFar);
}
template <int T>
__device__ __forceinline__ void rec_put(Lds<T> &L, int e, const float4 &mx, const float4 &my) {
    L.x[e] = mx;
    L.y[e] = my;
}
template <int T>
__device__ __forceinline__ void rec_put(Lds2<T> &L, int e, const float4 &mx, const float4 &my) {
    L.xy[e] = make_float4(mx.x, mx.y, my.x, my.y);
}
// The records of a two-slot region cell with its slots 2 and 3 from the
// side table (crowded regions only), and their write-back.
template <int T>
__device__ __forceinline__ void rec_get_side(const Lds2<T> &L, int e, float4 &mx, float4 &my) {
    rec_get(L, e, mx, my);
    const uint32_t k = L.sidx[e];
    if (k != kNoSide) {
        const float4 r = L.side[k];
        mx.z = r.x;
        mx.w = r.y;
        my.z = r.z;
        my.w = r.w;
    }
}
template <int T>
__device__ __forceinline__ void rec_put_side(Lds2<T> &L, int e, const float4 &mx,
                                             const float4 &my) {
    rec_put(L, e, mx, my);
    const uint32_t k = L.sidx[e];
    if (k != kNoSide) L.side[k] = make_float4(mx.z, mx.w, my.z, my.w);
}
// The records of a cell with SL slots: in the two-slot layout slots 2 and 3
// come from the side table.
template <int SL, int T>
__device__ __forceinline__ void rec_get_slots(const Lds<T> &L, int e, float4 &mx, float4 &my) {
    rec_get(L, e, mx, my);
}
template <int SL, int T>
__device__ __forceinline__ void rec_get_slots(const Lds2<T> &L, int e, float4 &mx, float4 &my) {
    if constexpr (SL > 2) rec_get_side(L, e, mx, my);
    else rec_get(L, e, mx, my);
}
// Slots 0 and 1 of a neighbour cell.
template <int T>
__device__ __forceinline__ void rec_get2(const Lds<T> &L, int e, float2 &qx, float2 &qy) {
    qx = *reinterpret_cast<const float2 *>(&L.x[e]);
    qy = *reinterpret_cast<const float2 *>(&L.y[e]);
}
template <int T>
__device__ __forceinline__ void rec_get2(const Lds2<T> &L, int e, float2 &qx, float2 &qy) {
    const float4 r = L.xy[e];
    qx = make_float2(r.x, r.y);
    qy = make_float2(r.z, r.w);
}
}  // namespace

struct PassCtx {
    uint64_t sweep;
    uint32_t gx0, gy0;
    int own_x, own_y;
    float cen;
    bool big;
    int nside;  // side-table entries in use (two-slot layout, crowded region)
};

// Does a disk at centred offsets (xn, yn) of region cell (CX + 2 ax, CY + 2 ay)
// overlap any disk of its 3 x 3 neighbourhood other than slot `slot` of its
// own cell (whose records are mx, my)?  Only slots below SL are tested: the
// caller knows that no cell of the region holds more than SL disks, and the
// empty slots hold the far sentinel.  In the two-slot form the squared
// separations of a row of three cells (each rounded as in overlap_f32) are
// reduced by a running minimum and compared once per row: the minimum is
// below 4 exactly when one of them is.  The rare four-slot form compares the
// neighbours' pairs one by one, which holds fewer registers live.  NB is the
// number of neighbour slots read from the records (the two-slot layout's
// crowded form tests all four own slots but reads two per neighbour and
// takes the neighbours' slots 2 and 3 from the side table).
template <int SL, int H, int CX, int CY, int NB = SL, typename LdsT>
__device__ __forceinline__ bool overlaps_any(const LdsT &L, int base_ax, uint32_t slot,
                                             const float4 &mx, const float4 &my, float xn,
                                             float yn, float w) {
    const float ax3[3] = {xn + w, xn, xn - w};  // q_di = s' - di w
    const float ay3[3] = {yn + w, yn, yn - w};
    constexpr float kNone = 16.0f;  // stands for a pair that is not tested
    float dmin = kNone;
    bool bad = false;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int di = k % 3 - 1, dj = k / 3 - 1;
        const float gx = ax3[k % 3], gy = ay3[k / 3];
        if (k == 4) {
            // own cell: every slot but the moving one
            dmin = fminf(dmin, slot != 0 ? r2_f32(mx.x - gx, my.x - gy) : kNone);
            dmin = fminf(dmin, slot != 1 ? r2_f32(mx.y - gx, my.y - gy) : kNone);
            if (SL > 2) {
                dmin = fminf(dmin, slot != 2 ? r2_f32(mx.z - gx, my.z - gy) : kNone);
                dmin = fminf(dmin, slot != 3 ? r2_f32(mx.w - gx, my.w - gy) : kNone);
            }
        } else {
            // neighbour (rx + di, ry + dj): its colour plane and in-plane
            // offset are compile-time constants for this colour
            const int cxn = (CX + di) & 1, cyn = (CY + dj) & 1;
            const int offx = (CX + di + 2) / 2 - 1, offy = (CY + dj + 2) / 2 - 1;
            const int ne = (cxn | (cyn << 1)) * H * H + base_ax + offx + H * offy;
            if constexpr (NB > 2) {
                const float4 qx = L.x[ne], qy = L.y[ne];
                bad |= overlap_f32(qx.x - gx, qy.x - gy);
                bad |= overlap_f32(qx.y - gx, qy.y - gy);
                bad |= overlap_f32(qx.z - gx, qy.z - gy);
                bad |= overlap_f32(qx.w - gx, qy.w - gy);
            } else {
                float2 qx, qy;
                rec_get2(L, ne, qx, qy);
                dmin = fminf(dmin, r2_f32(qx.x - gx, qy.x - gy));
                dmin = fminf(dmin, r2_f32(qx.y - gx, qy.y - gy));
            }
        }
        if (k % 3 == 2) {
            bad |= dmin < 4.0f;
            dmin = kNone;
            // one row of neighbour records in flight at a time keeps the
            // register budget of four waves per SIMD
            __asm__ volatile("" ::: "memory");
        }
    }
    return bad;
}

// One trial of slot `slot` of the cell whose records are (mx, my), with the
// step (dxs, dys): the in-cell test, the overlap test and, if both pass, the
// move.  SL = 2 when no cell of the region holds more than two disks, so the
// slot is 0 or 1 and only the first two components are read and written.
template <int SL, int H, int CX, int CY, typename LdsT>
__device__ __forceinline__ bool try_move(const LdsT &L, int base_ax, uint32_t slot, float4 &mx,
                                         float4 &my, float dxs, float dys, float lo_b, float hi_b,
                                         float w) {
    const float ox = SL > 2 ? pick4(mx, slot) : ((slot & 1u) ? mx.y : mx.x);
    const float oy = SL > 2 ? pick4(my, slot) : ((slot & 1u) ? my.y : my.x);
    const float xn = ox + dxs, yn = oy + dys;
    const bool inside = xn >= lo_b && xn < hi_b && yn >= lo_b && yn < hi_b;
    const bool acc = inside && !overlaps_any<SL, H, CX, CY>(L, base_ax, slot, mx, my, xn, yn, w);
    if (SL > 2) {
        mx = acc ? put4(mx, slot, xn) : mx;
        my = acc ? put4(my, slot, yn) : my;
    } else {
        const bool a0 = acc && slot == 0u, a1 = acc && slot == 1u;
        mx.x = a0 ? xn : mx.x;
        mx.y = a1 ? xn : mx.y;
        my.x = a0 ? yn : my.x;
        my.y = a1 ? yn : my.y;
    }
    return acc;
}

// Does a disk at centred offsets (xn, yn) of region cell (rx, ry) overlap
// slot 2 or 3 of a neighbouring crowded cell?  Those are the side table's
// entries whose cell is one of the eight neighbours (the own cell's entry is
// tested with its records); the separations are formed as in overlaps_any.
template <typename LdsT>
__device__ __forceinline__ bool side_overlaps(const LdsT &L, int nside, int rx, int ry, float xn,
                                              float yn, float w) {
    bool bad = false;
    for (int k = 0; k < nside; ++k) {
        const uint32_t at = L.side_at[k];
        const int di = (int)(at & 0xFFu) - rx, dj = (int)(at >> 8) - ry;
        if (di < -1 || di > 1 || dj < -1 || dj > 1 || (di == 0 && dj == 0)) continue;
        const float gx = di == 0 ? xn : (di > 0 ? xn - w : xn + w);
        const float gy = dj == 0 ? yn : (dj > 0 ? yn - w : yn + w);
        const float4 r = L.side[k];
        bad |= overlap_f32(r.x - gx, r.z - gy);
        bad |= overlap_f32(r.y - gx, r.w - gy);
    }
    return bad;
}

// try_move for a crowded two-slot region: any of the own cell's four slots
// (slots 2 and 3 loaded from the side table into mx, my), the neighbours'
// slots 0 and 1 from their records and slots 2 and 3 from the side table.
template <int H, int CX, int CY, typename LdsT>
__device__ __forceinline__ bool try_move_side(const LdsT &L, int base_ax, int rx, int ry,
                                              int nside, uint32_t slot, float4 &mx, float4 &my,
                                              float dxs, float dys, float lo_b, float hi_b,
                                              float w) {
    const float xn = pick4(mx, slot) + dxs, yn = pick4(my, slot) + dys;
    const bool inside = xn >= lo_b && xn < hi_b && yn >= lo_b && yn < hi_b;
    const bool acc = inside &&
                     !overlaps_any<4, H, CX, CY, 2>(L, base_ax, slot, mx, my, xn, yn, w) &&
                     !side_overlaps(L, nside, rx, ry, xn, yn, w);
    mx = acc ? put4(mx, slot, xn) : mx;
    my = acc ? put4(my, slot, yn) : my;
    return acc;
}

// One colour sub-sweep over the LDS region: pass p updates the cells of
// colour (CX, CY) with region coordinates in [p + 1, RL - p - 1), one lane per
// cell of that rectangle of the colour plane; lanes of empty cells idle.
// (Listing the non-empty cells first saves those lanes but costs a ballot,
// a scan and two barriers per pass, more than it saves.)
template <typename LdsT, int THREADS, int CX, int CY, typename View>
__device__ __forceinline__ void run_pass(LdsT &L, const View &v, const PassCtx &ctx, int tid,
                                         int p, uint32_t &trials, uint32_t &accepts) {
    constexpr int H = LdsT::R / 2, PB = (CX | (CY << 1)) * H * H;
    constexpr int RL = LdsT::RL;
    const uint32_t M = v.M;
    const float w = v.w, cen = ctx.cen;
    const float lo_b = -cen, hi_b = w - cen;  // in-cell range of centred offsets
    // plane cells (ax, ay) with 2 ax + CX and 2 ay + CY in [p + 1, RL - p - 1)
    const int lo = p + 1, hi = RL - p - 1;
    const int ax0 = (lo - CX + 1) >> 1, ax1 = (hi - CX + 1) >> 1;
    const int ay0 = (lo - CY + 1) >> 1, ay1 = (hi - CY + 1) >> 1;
    const int wdt = ax1 - ax0, ncell = wdt * (ay1 - ay0);
    for (int j = tid; j < ncell; j += THREADS) {
        const int ax = ax0 + j % wdt, ay = ay0 + j / wdt;
        const int a = ax + H * ay;
        if (L.cnt[PB + a] == 0) continue;
        const int rx = 2 * ax + CX, ry = 2 * ay + CY;
        const int e = PB + a;
        const uint32_t n = L.cnt[e];
        const uint32_t cell = wrap_add(ctx.gx0, rx, M) + __umul24(M, wrap_add(ctx.gy0, ry, M));
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
        float4 mx, my;
        if constexpr (LdsT::kTwo) {
            if (ctx.big) rec_get_side(L, e, mx, my);
            else rec_get(L, e, mx, my);
        } else {
            rec_get(L, e, mx, my);
        }
        for (uint32_t t = 0; t < v.n_trial; ++t) {
            const Words w4 = draw(v.seed_lo, v.seed_hi, ctx.sweep, cell, t, kStreamTrial);
            const uint32_t slot = (v.n_trial == 1) ? mulhi32(w4.w0, n)
                                                   : (perm >> (4 * (t % n))) & 0xFu;
            const float dxs = step_from_word(w4.w1, v.step_m);
            const float dys = step_from_word(w4.w2, v.step_m);
            if (own) ++trials;
            bool acc;
            if constexpr (LdsT::kTwo)
                acc = ctx.big ? try_move_side<H, CX, CY>(L, base_ax, rx, ry, ctx.nside, slot, mx, my,
                                                         dxs, dys, lo_b, hi_b, w)
                              : try_move<2, H, CX, CY>(L, base_ax, slot, mx, my, dxs, dys, lo_b,
                                                       hi_b, w);
            else
                acc = ctx.big
                          ? try_move<4, H, CX, CY>(L, base_ax, slot, mx, my, dxs, dys, lo_b, hi_b, w)
                          : try_move<2, H, CX, CY>(L, base_ax, slot, mx, my, dxs, dys, lo_b, hi_b, w);
            if (own && acc) ++accepts;
        }
        if constexpr (LdsT::kTwo) {
            if (ctx.big) rec_put_side(L, e, mx, my);
            else rec_put(L, e, mx, my);
        } else {
            rec_put(L, e, mx, my);
        }
    }
}

// Phase profiling: with a non-NULL `stamp` (kStampWords words per tile),
// thread 0 records the realtime clock when the tile's work starts, after the
// region load, after each colour pass, after the re-bin's class counts and at
// the end (words 0-7); word 8 is written by the kernel when its workgroup
// enters, before it reads the sweep counter.
__device__ __forceinline__ void stamp_at(unsigned long long *stamp, int tid, int k) {
    if (stamp && tid == 0) stamp[k] = wall_clock64();
}

// The work of one tile: load, four colour passes, canonical write-back,
// re-bin into the next sweep's grid, counts.  The tile owns the cells
// [I0, I0 + lim_x) x [J0, J0 + lim_y) (lim <= TILE) that lie in the box.
// In the two-slot layout a region holding more than kSide cells of more than
// two disks makes it return false before it writes anything outside LDS;
// otherwise it returns true.  `pace` (uniform) selects the wave priorities
// described at the region load.
template <typename LdsT, int THREADS, typename View>
__device__ __forceinline__ bool fused_tile(LdsT &L, const View &v, int tid, uint32_t I0,
                                           uint32_t J0, int lim_x, int lim_y, bool pace,
                                           unsigned long long *stamp) {
    constexpr bool kTwo = LdsT::kTwo;
    static_assert(THREADS % 64 == 0 && THREADS <= 64 * 16, "whole waves, at most 16");
    constexpr int RL = LdsT::RL, R = LdsT::R, TE = LdsT::TE;
    constexpr int NL = RL * RL, NIT = (NL + THREADS - 1) / THREADS;  // loaded cells per thread
    constexpr int NE = TE * TE, NEIT = (NE + THREADS - 1) / THREADS;  // extended-block cells
    const uint32_t M = v.M, NC = M * M;
    const int own_x = (M - I0 < (uint32_t)lim_x) ? (int)(M - I0) : lim_x;
    const int own_y = (M - J0 < (uint32_t)lim_y) ? (int)(M - J0) : lim_y;

    const uint64_t sweep = v.dev->sweep + v.offset;
    const SweepDraws d = sweep_draws(v.seed_lo, v.seed_hi, sweep, v.W);
    const float w = v.w;
    const float cen = (float)(v.W >> 1) * kQ;  // centring offset c
    const uint32_t gx0 = wrap_add(I0, -kHalo, M), gy0 = wrap_add(J0, -kHalo, M);
    stamp_at(stamp, tid, 0);

    // ---- load the region ----------------------------------------------------
    // Counts and slots 0 and 1 are loaded together (slot 1 is read whether
    // used or not: one dependent round trip fewer), slots 2 and 3 where the
    // count asks for them (in the four-slot layout; the two-slot one only
    // notes that they exist).
    // Wave priorities.  The global loads of the region and the tags are
    // issued at raised priority, so that they leave before the arithmetic
    // of the other workgroups on the CU.  In a launch of at most two rounds
    // of workgroups (`pace`) the priority also falls as the tile progresses:
    // 3 from here through the first colour pass, 2 in the second, 1 in the
    // third and fourth, 0 in the re-bin.  The least advanced of the
    // workgroups sharing a CU then issues first, so they keep pace and the
    // last tiles of the launch do not run alone at one wave per SIMD.  At
    // N = 1024^2, eta = 0.716 the one-round 34-cell tile sweeps in 31.2 us
    // with it against 33.5 us without; at N = 4096^2 (16 rounds) it costs
    // 6 %, and the other waves stay at 0 there.
    __builtin_amdgcn_s_setprio(3);
    uint32_t m_r[NIT], c_r[NIT];
    float4 px_r[NIT], py_r[NIT];
#pragma unroll
    for (int i = 0; i < NIT; ++i) {
        const int e = tid + i * THREADS;
        const int ee = e < NL ? e : 0;
        const uint32_t c = wrap_add(gx0, ee % RL, M) + __umul24(M, wrap_add(gy0, ee / RL, M));
        c_r[i] = c;
        const uint32_t m = el(v.cnt_in, c);
        m_r[i] = e < NL ? m : 0u;
        px_r[i] = make_float4(el(v.x_in, c), el(v.x_in, NC + c), kFar, kFar);
        py_r[i] = make_float4(el(v.y_in, c), el(v.y_in, NC + c), kFar, kFar);
    }
    if (!pace) __builtin_amdgcn_s_setprio(0);
#pragma unroll
    for (int i = 0; i < NIT; ++i) {
        const uint32_t c = c_r[i], m = m_r[i];
        if (!kTwo && m > 2) {
            px_r[i].z = el(v.x_in, 2 * NC + c);
            py_r[i].z = el(v.y_in, 2 * NC + c);
            if (m > 3) {
                px_r[i].w = el(v.x_in, 3 * NC + c);
                py_r[i].w = el(v.y_in, 3 * NC + c);
            }
        }
    }
    bool crowded = false;
#pragma unroll
    for (int i = 0; i < NIT; ++i) {
        const int e = tid + i * THREADS;
        if (e >= NL) break;
        const uint32_t m = m_r[i];
        const int li = pidx<R>(e % RL, e / RL);
        float4 sx4 = px_r[i], sy4 = py_r[i];
        sx4.x = m > 0 ? sx4.x - cen : kFar;
        sy4.x = m > 0 ? sy4.x - cen : kFar;
        sx4.y = m > 1 ? sx4.y - cen : kFar;
        sy4.y = m > 1 ? sy4.y - cen : kFar;
        sx4.z = m > 2 ? sx4.z - cen : kFar;
        sy4.z = m > 2 ? sy4.z - cen : kFar;
        sx4.w = m > 3 ? sx4.w - cen : kFar;
        sy4.w = m > 3 ? sy4.w - cen : kFar;
        rec_put(L, li, sx4, sy4);
        L.cnt[li] = (uint8_t)m;
        crowded |= m > 2;
    }
    // Every wave writes its own word, so no word needs clearing first: a
    // shared flag cleared by one thread and set by others is not ordered
    // without a barrier between the two.
    const bool wave_crowded = __any((int)crowded);
    if ((tid & 63) == 0) L.big[tid >> 6] = wave_crowded ? 1u : 0u;
    __syncthreads();
    stamp_at(stamp, tid, 1);
    uint32_t any_big = 0;
#pragma unroll
    for (int w = 0; w < THREADS / 64; ++w) any_big |= L.big[w];
    const bool big = __builtin_amdgcn_readfirstlane(any_big) != 0u;
    int nside = 0;
    if constexpr (kTwo) {
        if (big) {
            // The first wave lists the crowded cells in region order and
            // loads their slots 2 and 3 into the side table.
            if (tid < 64) {
                uint32_t base = 0;
                for (int e0 = 0; e0 < NL; e0 += 64) {
                    const int e = e0 + tid;
                    const int li = e < NL ? pidx<R>(e % RL, e / RL) : 0;
                    const uint32_t m = e < NL ? (uint32_t)L.cnt[li] : 0u;
                    const unsigned long long bal = __ballot(m > 2);
                    const uint32_t idx =
                        base + (uint32_t)__popcll(bal & ((1ull << (uint32_t)tid) - 1ull));
                    const bool listed = m > 2 && idx < (uint32_t)kSide;
                    if (e < NL) L.sidx[li] = listed ? (uint8_t)idx : kNoSide;
                    if (listed) {
                        const uint32_t c =
                            wrap_add(gx0, e % RL, M) + __umul24(M, wrap_add(gy0, e / RL, M));
                        const float x2 = el(v.x_in, 2 * NC + c) - cen;
                        const float y2 = el(v.y_in, 2 * NC + c) - cen;
                        const float x3 = m > 3 ? el(v.x_in, 3 * NC + c) - cen : kFar;
                        const float y3 = m > 3 ? el(v.y_in, 3 * NC + c) - cen : kFar;
                        L.side[idx] = make_float4(x2, x3, y2, y3);
                        L.side_at[idx] = (uint16_t)((e % RL) | ((e / RL) << 8));
                    }
                    base += (uint32_t)__popcll(bal);
                }
                if (tid == 0) L.nside = base;
            }
            __syncthreads();
            nside = (int)__builtin_amdgcn_readfirstlane(L.nside);
            if (nside > kSide) return false;  // too many: four-slot sub-tiles
        }
    }

    // Tags of the extended block, loaded now and held in registers through
    // the passes: a disk keeps its slot while the passes move it.
    uint4 tg_r[NEIT];
    if (!pace) __builtin_amdgcn_s_setprio(3);
#pragma unroll
    for (int i = 0; i < NEIT; ++i) {
        const int f = tid + i * THREADS;
        const int ex = f % TE, ey = f / TE;
        tg_r[i] = make_uint4(0u, 0u, 0u, 0u);
        if (f < NE && ex <= own_x && ey <= own_y) {
            const uint32_t m = L.cnt[pidx<R>(ex + kHalo, ey + kHalo)];
            const uint32_t c = wrap_add(I0, ex, M) + __umul24(M, wrap_add(J0, ey, M));
            if (m > 0) tg_r[i].x = el(v.tag_in, c);
            if (m > 1) tg_r[i].y = el(v.tag_in, NC + c);
            if ((!kTwo || big) && m > 2) tg_r[i].z = el(v.tag_in, 2 * NC + c);
            if ((!kTwo || big) && m > 3) tg_r[i].w = el(v.tag_in, 3 * NC + c);
        }
    }
    if (!pace) __builtin_amdgcn_s_setprio(0);

    // ---- four colour sub-sweeps --------------------------------------------
    PassCtx ctx;
    ctx.sweep = sweep;
    ctx.gx0 = gx0;
    ctx.gy0 = gy0;
    ctx.own_x = own_x;
    ctx.own_y = own_y;
    ctx.cen = cen;
    ctx.big = big;
    ctx.nside = nside;
    // I0 and J0 are even, so the colour parity in region coordinates equals
    // the global one
    uint32_t col[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) col[p] = colour_of_pass(d.perm, p);
    uint32_t trials = 0, accepts = 0;
    for (int p = 0; p < 4; ++p) {
        if (pace) {
            switch (p) {  // s_setprio takes an immediate
            case 0: break;
            case 1: __builtin_amdgcn_s_setprio(2); break;
            default: __builtin_amdgcn_s_setprio(1); break;
            }
        }
        // each colour has its own instantiation with compile-time neighbour
        // offsets
        switch (col[p]) {
        case 0: run_pass<LdsT, THREADS, 0, 0>(L, v, ctx, tid, p, trials, accepts); break;
        case 1: run_pass<LdsT, THREADS, 1, 0>(L, v, ctx, tid, p, trials, accepts); break;
        case 2: run_pass<LdsT, THREADS, 0, 1>(L, v, ctx, tid, p, trials, accepts); break;
        default: run_pass<LdsT, THREADS, 1, 1>(L, v, ctx, tid, p, trials, accepts); break;
        }
        __syncthreads();
        stamp_at(stamp, tid, 2 + p);
    }

    // ---- canonical state of the own block; wrap classes for the next grid ---
    // Old cell (ex, ey) of the extended block sends its disks to new cell
    // (ex - wx, ey - wy) of the next sweep's grid, shifted by s'.
    __builtin_amdgcn_s_setprio(0);
    const SweepDraws dn = sweep_draws(v.seed_lo, v.seed_hi, sweep + 1, v.W);
    const float sxn = (float)dn.kx * kQ, syn = (float)dn.ky * kQ;
    // Only the slots in use are read: two when no region cell holds more
    // (the counts do not change during the passes), else four.
    auto rebin = [&](auto slots) {
        constexpr int SL = decltype(slots)::value;
        float4 ux_r[NEIT], uy_r[NEIT];
        uint32_t me_r[NEIT];
#pragma unroll
        for (int i = 0; i < NEIT; ++i) {
            const int f = tid + i * THREADS;
            const int ex = f % TE, ey = f / TE;
            const bool in_ext = f < NE && ex <= own_x && ey <= own_y;
            const int li = pidx<R>(ex + kHalo, ey + kHalo);
            const uint32_t m = in_ext ? L.cnt[li] : 0u;
            float4 sx4, sy4;
            rec_get_slots<SL>(L, in_ext ? li : 0, sx4, sy4);
            float4 ux, uy;
            ux.x = sx4.x + cen;
            ux.y = sx4.y + cen;
            uy.x = sy4.x + cen;
            uy.y = sy4.y + cen;
            ux.z = SL > 2 ? sx4.z + cen : 0.0f;
            ux.w = SL > 2 ? sx4.w + cen : 0.0f;
            uy.z = SL > 2 ? sy4.z + cen : 0.0f;
            uy.w = SL > 2 ? sy4.w + cen : 0.0f;
            me_r[i] = m;
            ux_r[i] = ux;
            uy_r[i] = uy;
            if (in_ext && ex < own_x && ey < own_y && v.cnt_can) {
                const uint32_t c = (I0 + ex) + __umul24(M, J0 + ey);
                el(v.cnt_can, c) = (uint8_t)m;
#pragma unroll
                for (int s = 0; s < SL; ++s) {
                    if ((uint32_t)s < m) {
                        el(v.x_can, s * NC + c) = comp4(ux, s);
                        el(v.y_can, s * NC + c) = comp4(uy, s);
                        el(v.tag_can, s * NC + c) = s == 0 ? tg_r[i].x : s == 1 ? tg_r[i].y
                                              : s == 2 ? tg_r[i].z : tg_r[i].w;
                    }
                }
            }
            uint32_t g = 0;
#pragma unroll
            for (int s = 0; s < SL; ++s) {
                const uint32_t cls = (uint32_t)(comp4(ux, s) < sxn) | ((uint32_t)(comp4(uy, s) < syn) << 1);
                g += ((uint32_t)s < m) ? (1u << (3 * cls)) : 0u;
            }
            if (f < NE) L.gcnt[f] = (uint16_t)g;
        }
        __syncthreads();
        stamp_at(stamp, tid, 6);

        // ---- scatter into the next sweep's cell lists ---------------------------
        // New cell (I, J) takes the disks of old (I, J) that do not wrap, then
        // those of (I+1, J) wrapping in x only, (I, J+1) in y only, (I+1, J+1) in
        // both, each in old slot order.  A disk's slot follows from the class
        // counts of the old cells before its own in that order.
#pragma unroll
        for (int i = 0; i < NEIT; ++i) {
            const int f = tid + i * THREADS;
            const int ex = f % TE, ey = f / TE;
            if (f >= NE || ex > own_x || ey > own_y) continue;
            const uint32_t m = me_r[i];
            const float4 ux = ux_r[i], uy = uy_r[i];
            const uint4 tg = tg_r[i];
            const int exm = ex > 0 ? ex - 1 : 0, eym = ey > 0 ? ey - 1 : 0;
            const int exp1 = ex < TE - 1 ? ex + 1 : TE - 1;
            const uint32_t g_l = L.gcnt[exm + TE * ey];     // (ex-1, ey)
            const uint32_t g_d = L.gcnt[ex + TE * eym];     // (ex, ey-1)
            const uint32_t g_dr = L.gcnt[exp1 + TE * eym];  // (ex+1, ey-1)
            const uint32_t g_dl = L.gcnt[exm + TE * eym];   // (ex-1, ey-1)
            // base slot of each class in its destination, 8 bits per class
            const uint32_t b1 = g_l & 7u;
            const uint32_t b2 = (g_d & 7u) + ((g_dr >> 3) & 7u);
            const uint32_t b3 = (g_dl & 7u) + ((g_d >> 3) & 7u) + ((g_l >> 6) & 7u);
            const uint32_t bases = (b1 << 8) | (b2 << 16) | (b3 << 24);
            uint32_t seen = 0;  // 3-bit counters per class within this old cell
            const uint32_t nc0 = (I0 + ex) + __umul24(M, J0 + ey);  // new cell (ex, ey)
#pragma unroll
            for (int s = 0; s < SL; ++s) {
                if ((uint32_t)s >= m) break;
                const float us = comp4(ux, s), vs = comp4(uy, s);
                const uint32_t wx = us < sxn, wy = vs < syn, cls = wx | (wy << 1);
                const uint32_t slot = ((bases >> (8 * cls)) & 0xFFu) + ((seen >> (3 * cls)) & 7u);
                seen += 1u << (3 * cls);
                const int nx = ex - (int)wx, ny = ey - (int)wy;
                if (nx < 0 || nx >= own_x || ny < 0 || ny >= own_y || slot >= 4) continue;
                const uint32_t at = nc0 - wx - (wy ? M : 0u) + slot * NC;
                el(v.x_out, at) = (us - sxn) + (wx ? w : 0.0f);
                el(v.y_out, at) = (vs - syn) + (wy ? w : 0.0f);
                el(v.tag_out, at) = s == 0 ? tg.x : s == 1 ? tg.y : s == 2 ? tg.z : tg.w;
            }
            if (ex < own_x && ey < own_y) {  // the count of new cell (ex, ey)
                const uint32_t g_me = L.gcnt[f];
                const uint32_t g_r = L.gcnt[ex + 1 + TE * ey];         // (ex+1, ey)
                const uint32_t g_u = L.gcnt[ex + TE * (ey + 1)];       // (ex, ey+1)
                const uint32_t g_ur = L.gcnt[ex + 1 + TE * (ey + 1)];  // (ex+1, ey+1)
                const uint32_t n = (g_me & 7u) + ((g_r >> 3) & 7u) + ((g_u >> 6) & 7u) +
                                   ((g_ur >> 9) & 7u);
                if (n > 4) atomicOr((uint32_t *)&v.dev->overflow, 1u);
                el(v.cnt_out, nc0) = (uint8_t)(n > 4 ? 4 : n);
            }
        }
    };
    if (ctx.big) rebin(std::integral_constant<int, 4>{});
    else rebin(std::integral_constant<int, 2>{});
    count_trials((DevScalars *)v.dev, trials, accepts);
    if (stamp) {
        __syncthreads();
        stamp_at(stamp, tid, 7);
    }
    return true;
}

// Bytes of dynamic LDS a tile shape needs: its own records, and in the
// two-slot form also those of the four-slot sub-tiles it may fall back on.
template <int TILE, bool TWO>
constexpr size_t tile_lds_bytes() {
    if constexpr (TWO)
        return sizeof(Lds2<TILE>) > sizeof(Lds<sub_tile<TILE>()>) ? sizeof(Lds2<TILE>)
                                                                  : sizeof(Lds<sub_tile<TILE>()>);
    else
        return sizeof(Lds<TILE>);
}

// One tile of side TILE at (I0, J0).  The two-slot form holds the region in
// two-slot records and the slots 2 and 3 of its crowded cells in a side
// table; where the region holds more crowded cells than the table has
// entries (a dilute box of wide cells), the same block runs as two by two
// four-slot sub-tiles, each with its own halo, which gives the same
// trajectory.
template <int TILE, int THREADS, bool TWO, typename View>
__device__ __forceinline__ void tile_work(unsigned char *lds, const View &v, int tid, uint32_t I0,
                                          uint32_t J0, bool pace, unsigned long long *stamp) {
    if constexpr (!TWO) {
        fused_tile<Lds<TILE>, THREADS>(*reinterpret_cast<Lds<TILE> *>(lds), v, tid, I0, J0, TILE,
                                       TILE, pace, stamp);
    } else {
        if (fused_tile<Lds2<TILE>, THREADS>(*reinterpret_cast<Lds2<TILE> *>(lds), v, tid, I0, J0,
                                            TILE, TILE, pace, stamp))
            return;
        constexpr int SUB = sub_tile<TILE>();
        Lds<SUB> &L4 = *reinterpret_cast<Lds<SUB> *>(lds);
        for (int sj = 0; sj < TILE; sj += SUB)
            for (int si = 0; si < TILE; si += SUB) {
                __syncthreads();  // every read of the previous layout is done
                if (I0 + (uint32_t)si < v.M && J0 + (uint32_t)sj < v.M)
                    fused_tile<Lds<SUB>, THREADS>(L4, v, opaque_tid(), I0 + si, J0 + sj,
                                                  TILE - si < SUB ? TILE - si : SUB,
                                                  TILE - sj < SUB ? TILE - sj : SUB, pace,
                                                  nullptr);
            }
        if (stamp) {  // the sub-tiles' whole time is booked as the first colour pass
            __syncthreads();
            for (int k = 2; k < 8; ++k) stamp_at(stamp, tid, k);
        }
    }
}

template <int TILE, int THREADS, bool TWO>
__global__ void __launch_bounds__(THREADS) k_fused(BoxView v, uint32_t ntx, uint32_t nty,
                                                   uint32_t per_xcd, uint32_t pace,
                                                   unsigned long long *stamps) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    // Consecutive workgroups go to different XCDs; give each XCD a
    // contiguous run of tiles so that shared halo cells meet in its L2.
    const uint32_t tile = (blockIdx.x % 8u) * per_xcd + blockIdx.x / 8u;
    if (tile >= ntx * nty) return;
    unsigned long long *stamp = stamps ? stamps + kStampWords * (size_t)tile : nullptr;
    stamp_at(stamp, (int)threadIdx.x, 8);
    tile_work<TILE, THREADS, TWO>(lds_raw, v, (int)threadIdx.x, (tile % ntx) * TILE,
                                  (tile / ntx) * TILE, pace != 0u, stamp);
}

// Persistent form for a batch of independent boxes: workgroups stride over
// a work list of (box, tile) items, item = box << 20 | tile.  All boxes of a
// batch advance in step, so one buffer parity serves them all.
template <int TILE, int THREADS, bool TWO>
__global__ void __launch_bounds__(THREADS) k_fused_batch(const BoxView *__restrict__ views,
                                                         const uint32_t *__restrict__ items,
                                                         uint32_t n_items, uint32_t parity,
                                                         uint32_t offset, uint32_t pace) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    for (uint32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const uint32_t item = items[it], box = item >> 20, tile = item & 0xFFFFFu;
        const BoxView &src = views[2 * box + parity];
        GlobalView v;
        v.cnt_in = (const MPMC_GLOBAL uint8_t *)src.cnt_in;
        v.x_in = (const MPMC_GLOBAL float *)src.x_in;
        v.y_in = (const MPMC_GLOBAL float *)src.y_in;
        v.tag_in = (const MPMC_GLOBAL uint32_t *)src.tag_in;
        v.cnt_out = (MPMC_GLOBAL uint8_t *)src.cnt_out;
        v.x_out = (MPMC_GLOBAL float *)src.x_out;
        v.y_out = (MPMC_GLOBAL float *)src.y_out;
        v.tag_out = (MPMC_GLOBAL uint32_t *)src.tag_out;
        v.cnt_can = (MPMC_GLOBAL uint8_t *)src.cnt_can;
        v.x_can = (MPMC_GLOBAL float *)src.x_can;
        v.y_can = (MPMC_GLOBAL float *)src.y_can;
        v.tag_can = (MPMC_GLOBAL uint32_t *)src.tag_can;
        v.dev = (MPMC_GLOBAL DevScalars *)src.dev;
        v.M = src.M;
        v.W = src.W;
        v.cap = src.cap;
        v.CS = src.CS;
        v.step_m = src.step_m;
        v.n_trial = src.n_trial;
        v.w = src.w;
        v.seed_lo = src.seed_lo;
        v.seed_hi = src.seed_hi;
        v.offset = offset;
        const uint32_t ntx = (v.M + TILE - 1) / TILE;
        tile_work<TILE, THREADS, TWO>(lds_raw, v, opaque_tid(), (tile % ntx) * TILE,
                                      (tile / ntx) * TILE, pace != 0u, nullptr);
        __syncthreads();
    }
}

namespace {
// Workgroups of a shape resident on the whole device at once (occupancy
// per CU times CUs), taken once per shape.
template <int TILE, int THREADS, bool TWO>
uint32_t resident_t() {
    static uint32_t slots = 0;
    if (!slots) {
        int blocks = 0, dev = 0, cus = 0;
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_fused<TILE, THREADS, TWO>,
                                                           THREADS, tile_lds_bytes<TILE, TWO>());
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        slots = (uint32_t)(blocks > 0 ? blocks : 1) * (uint32_t)(cus > 0 ? cus : 256);
    }
    return slots;
}

template <int TILE, int THREADS, bool TWO>
void launch_t(const BoxView &v, hipStream_t st, unsigned long long *stamps) {
    const uint32_t ntx = (v.M + TILE - 1) / TILE, nty = ntx;
    const uint32_t nt = ntx * nty, per_xcd = (nt + 7) / 8;
    const size_t lds = tile_lds_bytes<TILE, TWO>();
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)k_fused<TILE, THREADS, TWO>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        attr = true;
    }
    const uint32_t pace = nt <= 2u * resident_t<TILE, THREADS, TWO>() ? 1u : 0u;
    k_fused<TILE, THREADS, TWO><<<8 * per_xcd, THREADS, lds, st>>>(v, ntx, nty, per_xcd, pace,
                                                                    stamps);
}

template <int TILE, int THREADS, bool TWO>
void launch_batch_t(const BoxView *views, const uint32_t *items, uint32_t n_items, uint32_t grid,
                    uint32_t parity, uint32_t offset, hipStream_t st) {
    const size_t lds = tile_lds_bytes<TILE, TWO>();
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)k_fused_batch<TILE, THREADS, TWO>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        attr = true;
    }
    const uint32_t pace = n_items <= 2u * grid ? 1u : 0u;  // grid: every resident slot
    k_fused_batch<TILE, THREADS, TWO><<<grid, THREADS, lds, st>>>(views, items, n_items, parity,
                                                                   offset, pace);
}

template <int TILE, int THREADS, bool TWO>
int occupancy_t() {
    int blocks = 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_fused_batch<TILE, THREADS, TWO>,
                                                       THREADS, tile_lds_bytes<TILE, TWO>());
    return blocks;
}

struct Entry {
    uint32_t tile, threads;
    void (*fn)(const BoxView &, hipStream_t, unsigned long long *);
    void (*batch)(const BoxView *, const uint32_t *, uint32_t, uint32_t, uint32_t, uint32_t,
                  hipStream_t);
    int (*occ)();
};
#define MPMC_SHAPE(T, N, TWO) \
    {T, N, launch_t<T, N, TWO>, launch_batch_t<T, N, TWO>, occupancy_t<T, N, TWO>}
// The 34- and 48-cell tiles hold two-slot records: 37 KB of LDS and four
// workgroups of 256 threads per CU, 64 KB and two of 512.  At N = 1024^2,
// eta = 0.716 (M = 1072) the 34-cell tile gives 1024 tiles, one round.
const Entry kShapes[] = {
    MPMC_SHAPE(8, 64, false),    MPMC_SHAPE(8, 128, false),  MPMC_SHAPE(16, 128, false),
    MPMC_SHAPE(16, 256, false),  MPMC_SHAPE(24, 256, false), MPMC_SHAPE(32, 256, false),
    MPMC_SHAPE(32, 512, false),  MPMC_SHAPE(34, 256, true),  MPMC_SHAPE(48, 512, true),
    MPMC_SHAPE(48, 1024, false), MPMC_SHAPE(56, 1024, false),
};
#undef MPMC_SHAPE
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
    // the loaded region (tile + 9 cells a side) must not wrap onto itself:
    // every index is reduced modulo M with a single conditional subtraction
    if (s.tile + 2 * kHalo + 2 > v.M || (s.tile & 1u)) return false;
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

void launch_fused_sweep(const BoxView &v, const FusedShape &s, hipStream_t st,
                        unsigned long long *stamps) {
    for (const Entry &e : kShapes)
        if (e.tile == s.tile && e.threads == s.threads) {
            e.fn(v, st, stamps);
            return;
        }
}

}  // namespace mpmc
