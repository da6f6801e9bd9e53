// capi.hip — host runtime and C ABI of the MPMC library (declared in
// include/mpmc.h).  Owns the device state of each box, launches the sweep
// and measurement kernels on the box's stream, replays captured HIP graphs
// for long runs, and does the small host-side analysis (contact fit, C(dt)).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "../../include/mpmc.h"
#include "mpmc_kernels.hpp"
#include "mpmc_host.hpp"

using namespace mpmc;

// ---------------------------------------------------------------------------
// error reporting
static thread_local std::string g_err;

int mpmc::fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

extern "C" const char *mpmc_last_error(void) { return g_err.c_str(); }

#define HIPCHK(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(MPMC_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));           \
    } while (0)

// ---------------------------------------------------------------------------
// geometry (Sec. II.A: eta = N pi / L^2; Sec. II.B: cells of width >= 2 sigma
// in a four-colour checkerboard, hence an even count per side)
static uint32_t cell_capacity(double w) {
    // k points with mutual distance >= 2 fit in a w x w square only once w
    // reaches 2 / d_k, d_k the best minimum distance of k points in the unit
    // square: d_5 = 0.70711, d_6 = 0.60093, d_7 = 0.53590, d_8 = 0.51764.
    if (w < 2.0 / 0.70710678) return 4;
    if (w < 2.0 / 0.6009) return 5;
    if (w < 2.0 / 0.5359) return 6;
    if (w < 2.0 / 0.5176) return 7;
    return 8;
}

int mpmc::compute_geometry(Geometry *g, uint32_t N, double eta, double cell_min,
                           uint32_t step_m) {
    if (N == 0) return fail(MPMC_EINVAL, "N must be positive");
    if (!(eta > 0.0) || eta > M_PI / 4.0) return fail(MPMC_EINVAL, "eta must be in (0, pi/4]");
    if (!(cell_min >= 2.0)) return fail(MPMC_EINVAL, "cell_min must be >= 2 sigma");
    if (step_m < 1 || step_m > 255) return fail(MPMC_EINVAL, "step_m must be in 1..255");
    g->L = sqrt((double)N * M_PI / eta);
    g->M = 2u * (uint32_t)floor(g->L / (2.0 * cell_min));
    if (g->M < 4) return fail(MPMC_EINVAL, "box too small: %u cells per side (need >= 4)", g->M);
    g->W = (int64_t)llround(g->L / ((double)g->M * kQd));
    const double w = (double)g->W * kQd;
    if (w + step_m / 256.0 >= 4.0)
        return fail(MPMC_EINVAL, "cell width %.4f plus step %.4f must stay below 4", w,
                    step_m / 256.0);
    g->w = (float)w;
    g->Lq = (int64_t)g->M * g->W;
    g->cap = cell_capacity(w);
    g->CS = g->cap <= 4 ? 4 : 8;
    // slot indices s * M^2 + c and their byte offsets are 32-bit on the device
    if ((uint64_t)g->M * g->M * g->CS * 4 > 0xFFFFFFFFull)
        return fail(MPMC_EINVAL, "box too large: %u^2 cells x %u slots exceed 32-bit byte offsets",
                    g->M, g->CS);
    return MPMC_OK;
}

// ---------------------------------------------------------------------------
// device memory through the optional allocator hook
int Box::alloc_dev(void **ptr, size_t bytes) {
    *ptr = nullptr;
    if (bytes == 0) bytes = 4;
    if (p.alloc) {
        *ptr = p.alloc(bytes, p.alloc_ctx);
        if (!*ptr) return fail(MPMC_ENOMEM, "allocator hook returned NULL for %zu bytes", bytes);
    } else {
        hipError_t e = hipMalloc(ptr, bytes);
        if (e != hipSuccess) {
            *ptr = nullptr;
            return fail(e == hipErrorOutOfMemory ? MPMC_ENOMEM : MPMC_EDEVICE,
                        "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
        }
    }
    allocations.push_back(*ptr);
    return MPMC_OK;
}

void Box::free_dev(void *ptr) {
    if (!ptr) return;
    for (size_t i = 0; i < allocations.size(); ++i)
        if (allocations[i] == ptr) {
            allocations.erase(allocations.begin() + i);
            if (p.alloc) p.free(ptr, p.alloc_ctx);
            else (void)hipFree(ptr);
            return;
        }
}

void Box::release() {
    if (meas_stream) {
        (void)hipStreamSynchronize(meas_stream);
        (void)hipStreamDestroy(meas_stream);
        meas_stream = nullptr;
    }
    if (ev_swept) (void)hipEventDestroy(ev_swept);
    if (ev_meas) (void)hipEventDestroy(ev_meas);
    ev_swept = ev_meas = nullptr;
    meas_pending = false;
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    graph_exec = nullptr;
    if (lgraph_exec) (void)hipGraphExecDestroy(lgraph_exec);
    lgraph_exec = nullptr;
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    cap_stream = nullptr;
    for (void *a : allocations) {
        if (p.alloc) p.free(a, p.alloc_ctx);
        else (void)hipFree(a);
    }
    allocations.clear();
}

BoxView Box::view(int from) const {
    BoxView v;
    v.cnt_in = P[from].cnt;
    v.x_in = P[from].x;
    v.y_in = P[from].y;
    v.tag_in = P[from].tag;
    v.cnt_out = P[from ^ 1].cnt;
    v.x_out = P[from ^ 1].x;
    v.y_out = P[from ^ 1].y;
    v.tag_out = P[from ^ 1].tag;
    v.cnt_can = C.cnt;
    v.x_can = C.x;
    v.y_can = C.y;
    v.tag_can = C.tag;
    v.dev = dev;
    v.M = g.M;
    v.W = (uint32_t)g.W;
    v.cap = g.cap;
    v.CS = g.CS;
    v.step_m = p.step_m;
    v.n_trial = p.n_trial;
    v.w = g.w;
    v.seed_lo = (uint32_t)seed;
    v.seed_hi = (uint32_t)(seed >> 32);
    v.offset = 0;
    return v;
}

MeasureView Box::mview() const {
    MeasureView m;
    const CellBuf c = canon();
    m.cnt = c.cnt;
    m.x = c.x;
    m.y = c.y;
    m.tag = c.tag;
    m.dev = dev;
    m.M = g.M;
    m.W = (uint32_t)g.W;
    m.cap = g.cap;
    m.CS = g.CS;
    m.N = N;
    m.w = g.w;
    m.Sx = host.Sx;
    m.Sy = host.Sy;
    m.Lq = g.Lq;
    return m;
}

int Box::sync() {
    HIPCHK(hipStreamSynchronize(stream));
    return MPMC_OK;
}

int Box::read_scalars() {
    HIPCHK(hipMemcpyAsync(&host, dev, sizeof(DevScalars), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    host.trials = host.accepts = 0;
    for (int s = 0; s < kCountSlots; ++s) {
        host.trials += host.slots[s].trials;
        host.accepts += host.slots[s].accepts;
    }
    if (host.overflow) return fail(MPMC_EOVERFLOW, "a cell exceeded its capacity");
    return MPMC_OK;
}

// Uploads cell lists built on the host (cnt, slot-major tag, x, y) as the
// canonical state, resets the device scalars, and bins the lists in the
// grid of the next sweep.
int Box::join_meas() {
    if (meas_pending) HIPCHK(hipStreamWaitEvent(stream, ev_meas, 0));
    return MPMC_OK;
}

int Box::upload(const std::vector<uint8_t> &hc, const std::vector<uint32_t> &ht,
                const std::vector<float> &hx, const std::vector<float> &hy,
                const DevScalars &s) {
    const size_t nc = (size_t)g.M * g.M, ns = nc * g.CS;
    int jrc = join_meas();
    if (jrc) return jrc;
    HIPCHK(hipMemcpyAsync(C.cnt, hc.data(), nc, hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(C.tag, ht.data(), ns * 4, hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(C.x, hx.data(), ns * 4, hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(C.y, hy.data(), ns * 4, hipMemcpyHostToDevice, stream));
    host = s;
    HIPCHK(hipMemcpyAsync(dev, &host, sizeof(DevScalars), hipMemcpyHostToDevice, stream));
    BoxView v = view(1);  // output: P[0]
    v.cnt_in = C.cnt;
    v.x_in = C.x;
    v.y_in = C.y;
    v.tag_in = C.tag;
    launch_rebin(v, stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(stream));
    cur = 0;
    canon_in_c = true;
    return MPMC_OK;
}

int Box::materialize() {
    if (canon_in_c) return MPMC_OK;
    int jrc = join_meas();
    if (jrc) return jrc;
    const size_t nc = (size_t)g.M * g.M, ns = nc * g.CS;
    const CellBuf s = P[cur ^ 1];
    HIPCHK(hipMemcpyAsync(C.cnt, s.cnt, nc, hipMemcpyDeviceToDevice, stream));
    HIPCHK(hipMemcpyAsync(C.tag, s.tag, ns * 4, hipMemcpyDeviceToDevice, stream));
    HIPCHK(hipMemcpyAsync(C.x, s.x, ns * 4, hipMemcpyDeviceToDevice, stream));
    HIPCHK(hipMemcpyAsync(C.y, s.y, ns * 4, hipMemcpyDeviceToDevice, stream));
    canon_in_c = true;
    return MPMC_OK;
}

// Host-side cell lists from absolute q positions (tag order of appending).
int mpmc::build_cells(const Geometry &g, uint32_t N, const int64_t *X, const int64_t *Y,
                      std::vector<uint8_t> &hc, std::vector<uint32_t> &ht,
                      std::vector<float> &hx, std::vector<float> &hy) {
    const size_t nc = (size_t)g.M * g.M;
    hc.assign(nc, 0);
    ht.assign(nc * g.CS, 0);
    hx.assign(nc * g.CS, 0.0f);
    hy.assign(nc * g.CS, 0.0f);
    for (uint32_t t = 0; t < N; ++t) {
        if (X[t] < 0 || X[t] >= g.Lq || Y[t] < 0 || Y[t] >= g.Lq)
            return fail(MPMC_EINVAL, "position of disk %u outside [0, M W)", t);
        const int64_t i = X[t] / g.W, j = Y[t] / g.W;
        const size_t c = (size_t)i + (size_t)g.M * (size_t)j;
        if (hc[c] >= g.cap) return fail(MPMC_EOVERFLOW, "cell %zu exceeds capacity %u", c, g.cap);
        const size_t o = (size_t)hc[c]++ * nc + c;  // slot-major
        ht[o] = t;
        hx[o] = (float)((double)(X[t] - i * g.W) * kQd);
        hy[o] = (float)((double)(Y[t] - j * g.W) * kQd);
    }
    return MPMC_OK;
}

static void lattice_positions(const Geometry &g, uint32_t N, int lattice, std::vector<int64_t> &X,
                              std::vector<int64_t> &Y) {
    const int64_t n = (int64_t)llround(sqrt((double)N));
    X.resize(N);
    Y.resize(N);
    for (int64_t b = 0; b < n; ++b)
        for (int64_t a = 0; a < n; ++a) {
            const int64_t off = (lattice == MPMC_LATTICE_TRIANGULAR) ? (b & 1) : 0;
            X[b * n + a] = ((2 * a + 1 + off) * g.Lq) / (2 * n) % g.Lq;
            Y[b * n + a] = ((2 * b + 1) * g.Lq) / (2 * n);
        }
}

int mpmc::create_box(Box **out, uint32_t N, double eta, uint64_t seed, const mpmc_params *pp) {
    *out = nullptr;
    mpmc_params p;
    mpmc_default_params(&p);
    if (pp) p = *pp;
    if ((p.alloc == nullptr) != (p.free == nullptr))
        return fail(MPMC_EINVAL, "alloc and free hooks must be given together");
    if (p.n_trial < 1 || p.n_trial > 64) return fail(MPMC_EINVAL, "n_trial must be in 1..64");
    if (p.hist_bins < 1 || p.hist_bins > 4096) return fail(MPMC_EINVAL, "hist_bins must be in 1..4096");
    if (!(p.hist_dr > 0.0) || 2.0 + p.hist_bins * p.hist_dr >= 4.0)
        return fail(MPMC_EINVAL, "the contact histogram must end below r = 4 sigma");
    if (p.fit_order < 1 || p.fit_order > 8 || p.fit_order + 1 > p.hist_bins)
        return fail(MPMC_EINVAL, "fit_order must be in 1..8 and below hist_bins");
    if (p.schedule > MPMC_SCHED_FUSED) return fail(MPMC_EINVAL, "unknown schedule");
    if (p.lattice < 0 || p.lattice > 2) return fail(MPMC_EINVAL, "unknown lattice");
    Geometry g;
    int rc = compute_geometry(&g, N, eta, p.cell_min, p.step_m);
    if (rc) return rc;
    if (p.lattice != MPMC_LATTICE_NONE) {
        const uint64_t n = (uint64_t)llround(sqrt((double)N));
        if (n * n != N) return fail(MPMC_EINVAL, "a lattice start needs N a perfect square");
    }
    Box *b = new Box();
    b->N = N;
    b->eta = eta;
    b->seed = seed;
    b->p = p;
    b->g = g;
    b->stream = (hipStream_t)p.stream;
    const size_t nc = (size_t)g.M * g.M, ns = nc * g.CS;
    const uint32_t K = p.hist_bins;
#define ALLOC(ptr, bytes)                                             \
    do {                                                              \
        rc = b->alloc_dev((void **)&(ptr), (bytes));                  \
        if (rc) { b->release(); delete b; return rc; }                \
    } while (0)
    for (int k = 0; k < 3; ++k) {
        CellBuf &c = k < 2 ? b->P[k] : b->C;
        ALLOC(c.cnt, nc);
        ALLOC(c.x, ns * 4);
        ALLOC(c.y, ns * 4);
        ALLOC(c.tag, ns * 4);
    }
    ALLOC(b->dev, sizeof(DevScalars));
    ALLOC(b->hist, K * sizeof(unsigned long long));
    ALLOC(b->edges, (K + 1) * sizeof(float));
    ALLOC(b->scratch_u32, (size_t)(N > nc ? N : nc) * 4 + 64);
#undef ALLOC
    hipError_t e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        b->release();
        delete b;
        return fail(MPMC_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
    }
    // squared histogram edges fp32((2 + k dr)^2), from doubles
    std::vector<float> E(K + 1);
    for (uint32_t k = 0; k <= K; ++k) {
        const double r = 2.0 + (double)k * p.hist_dr;
        E[k] = (float)(r * r);
    }
    e = hipMemcpyAsync(b->edges, E.data(), (K + 1) * 4, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b->hist, 0, K * 8, b->stream);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipMemsetAsync(b->P[k].cnt, 0, nc, b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b->C.cnt, 0, nc, b->stream);
    if (e != hipSuccess) {
        b->release();
        delete b;
        return fail(MPMC_EDEVICE, "initialising device buffers: %s", hipGetErrorString(e));
    }
    std::vector<uint8_t> hc;
    std::vector<uint32_t> ht;
    std::vector<float> hx, hy;
    DevScalars s;
    memset(&s, 0, sizeof s);
    if (p.lattice != MPMC_LATTICE_NONE) {
        std::vector<int64_t> X, Y;
        lattice_positions(g, N, p.lattice, X, Y);
        rc = build_cells(g, N, X.data(), Y.data(), hc, ht, hx, hy);
    } else {
        // no disks placed yet: all cells empty until mpmc_set_positions
        hc.assign(nc, 0);
        ht.assign(ns, 0);
        hx.assign(ns, 0.0f);
        hy.assign(ns, 0.0f);
        b->placed = false;
    }
    if (rc == MPMC_OK) rc = b->upload(hc, ht, hx, hy, s);
    if (rc) {
        b->release();
        delete b;
        return rc;
    }
    *out = b;
    return MPMC_OK;
}

// ---------------------------------------------------------------------------
// sweeps
int Box::launch_one(int from, uint32_t offset, hipStream_t st, bool canon) {
    BoxView v = view(from);
    v.offset = offset;
    if (!canon) {  // only the last sweep of a run leaves the canonical state
        v.cnt_can = nullptr;
        v.x_can = v.y_can = nullptr;
        v.tag_can = nullptr;
    }
    if (sched == MPMC_SCHED_SIMPLE) launch_simple_sweep(v, st);
    else launch_fused_sweep(v, shape, st);
    return MPMC_OK;
}

int Box::build_graph() {
    if (graph_exec) {
        (void)hipGraphExecDestroy(graph_exec);
        graph_exec = nullptr;
    }
    // the graph holds the first G - 1 sweeps of a run; the last one, which
    // writes the canonical state, and the counter update are launched
    // directly after it, so that the run can wait for a pending measurement
    // of the previous canonical state just before overwriting it
    hipGraph_t graph;
    HIPCHK(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
    for (uint32_t k = 0; k + 1 < graph_sweeps; ++k)
        launch_one((int)(k & 1u), k, cap_stream, false);
    HIPCHK(hipStreamEndCapture(cap_stream, &graph));
    hipError_t e = hipGraphInstantiate(&graph_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        graph_exec = nullptr;
        return fail(MPMC_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    graph_key = key();
    return MPMC_OK;
}

uint64_t Box::key() const {
    return ((uint64_t)sched << 56) ^ ((uint64_t)shape.tile << 40) ^ ((uint64_t)shape.threads << 24) ^
           ((uint64_t)p.step_m << 8) ^ p.n_trial;
}

int Box::run_sweeps(uint64_t k) {
    if (!placed) return fail(MPMC_ESTATE, "no configuration: call mpmc_set_positions first");
    while (k > 0) {
        if (cur == 0 && k >= graph_sweeps && use_graphs) {
            if (!graph_exec || graph_key != key()) {
                int rc = build_graph();
                if (rc) return rc;
            }
            HIPCHK(hipGraphLaunch(graph_exec, stream));
            int jrc = join_meas();
            if (jrc) return jrc;
            launch_one((int)((graph_sweeps - 1) & 1u), graph_sweeps - 1, stream, true);
            launch_advance(dev, (uint32_t)seed, (uint32_t)(seed >> 32), (uint32_t)g.W, g.Lq,
                           graph_sweeps, stream);
            HIPCHK(hipGetLastError());
            k -= graph_sweeps;
            host_sweeps += graph_sweeps;
            canon_in_c = sched != MPMC_SCHED_SIMPLE;
            continue;
        }
        if (k == 1 || sched == MPMC_SCHED_SIMPLE) {  // writes the canonical state
            int jrc = join_meas();
            if (jrc) return jrc;
        }
        launch_one(cur, 0, stream, k == 1);
        launch_advance(dev, (uint32_t)seed, (uint32_t)(seed >> 32), (uint32_t)g.W, g.Lq, 1, stream);
        HIPCHK(hipGetLastError());
        cur ^= 1;
        --k;
        ++host_sweeps;
        canon_in_c = sched != MPMC_SCHED_SIMPLE;
    }
    return MPMC_OK;
}

// ---------------------------------------------------------------------------
// C ABI
extern "C" int mpmc_default_params(mpmc_params *p) {
    if (!p) return fail(MPMC_EINVAL, "params is NULL");
    memset(p, 0, sizeof *p);
    p->step_m = 26;
    p->n_trial = 1;
    p->lattice = MPMC_LATTICE_TRIANGULAR;
    p->cell_min = 2.0;
    p->hist_dr = 1e-3;
    p->hist_bins = 100;
    p->fit_order = 4;
    p->hist_block = 0;
    p->schedule = MPMC_SCHED_AUTO;
    p->tile = 0;
    return MPMC_OK;
}

extern "C" int mpmc_init_box(mpmc_box *out, uint32_t N, double eta, uint64_t seed,
                             const mpmc_params *p) {
    if (!out) return fail(MPMC_EINVAL, "out is NULL");
    *out = nullptr;
    Box *b = nullptr;
    int rc = create_box(&b, N, eta, seed, p);
    if (rc) return rc;
    rc = b->choose_schedule();
    if (rc) {
        b->release();
        delete b;
        return rc;
    }
    *out = reinterpret_cast<mpmc_box>(b);
    return MPMC_OK;
}

extern "C" int mpmc_free_box(mpmc_box bh) {
    if (!bh) return MPMC_OK;
    Box *b = reinterpret_cast<Box *>(bh);
    if (b->in_batch) return fail(MPMC_ESTATE, "this box belongs to a batch; free the batch");
    (void)hipStreamSynchronize(b->stream);
    b->release();
    delete b;
    return MPMC_OK;
}

static Box *B(mpmc_box b) { return reinterpret_cast<Box *>(b); }

extern "C" int mpmc_set_positions(mpmc_box bh, const int64_t *X, const int64_t *Y) {
    if (!bh || !X || !Y) return fail(MPMC_EINVAL, "NULL argument");
    Box *b = B(bh);
    std::vector<uint8_t> hc;
    std::vector<uint32_t> ht;
    std::vector<float> hx, hy;
    int rc = build_cells(b->g, b->N, X, Y, hc, ht, hx, hy);
    if (rc) return rc;
    rc = b->read_scalars();
    if (rc && rc != MPMC_EOVERFLOW) return rc;
    DevScalars s = b->host;
    s.Sx = s.Sy = 0;
    s.overflow = 0;
    rc = b->upload(hc, ht, hx, hy, s);
    if (rc) return rc;
    b->placed = true;
    return MPMC_OK;
}

extern "C" int mpmc_set_step(mpmc_box bh, uint32_t step_m) {
    if (!bh) return fail(MPMC_EINVAL, "NULL box");
    Box *b = B(bh);
    if (step_m < 1 || step_m > 255) return fail(MPMC_EINVAL, "step_m must be in 1..255");
    if ((double)b->g.w + step_m / 256.0 >= 4.0) return fail(MPMC_EINVAL, "step too large for w");
    b->p.step_m = step_m;
    return MPMC_OK;
}

extern "C" int mpmc_sweep(mpmc_box bh, uint64_t k, uint64_t *trials, uint64_t *accepts) {
    if (!bh) return fail(MPMC_EINVAL, "NULL box");
    Box *b = B(bh);
    if (b->in_batch) return fail(MPMC_ESTATE, "boxes of a batch are swept with mpmc_batch_sweep");
    DevScalars before;
    if (trials || accepts) {
        int rc = b->read_scalars();
        if (rc) return rc;
        before = b->host;
    }
    int rc = b->run_sweeps(k);
    if (rc) return rc;
    if (trials || accepts) {
        rc = b->read_scalars();
        if (rc) return rc;
        if (trials) *trials = b->host.trials - before.trials;
        if (accepts) *accepts = b->host.accepts - before.accepts;
    }
    return MPMC_OK;
}

extern "C" int mpmc_profile_phases(mpmc_box bh, uint32_t sweeps, double *phase_us) {
    if (!bh || !phase_us || sweeps == 0) return fail(MPMC_EINVAL, "bad arguments");
    Box *b = B(bh);
    if (b->in_batch) return fail(MPMC_ESTATE, "boxes of a batch are swept with mpmc_batch_sweep");
    if (!b->placed) return fail(MPMC_ESTATE, "no configuration: call mpmc_set_positions first");
    if (b->sched != MPMC_SCHED_FUSED)
        return fail(MPMC_EINVAL, "phase profiles need the fused schedule");
    const uint32_t nt = (b->g.M + b->shape.tile - 1) / b->shape.tile;
    const size_t tiles = (size_t)nt * nt, words = tiles * kStampWords;
    unsigned long long *d = nullptr;
    int rc = b->alloc_dev((void **)&d, words * 8);
    if (rc) return rc;
    int dev = 0, khz = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    std::vector<unsigned long long> h(words);
    // per tile: the seven phases, the whole tile, entry to start of work;
    // per launch: first entry to last end, busy tile-time over that span,
    // first entry to last entry
    double sum[12] = {};
    rc = b->join_meas();
    for (uint32_t k = 0; k < sweeps && rc == MPMC_OK && e == hipSuccess; ++k) {
        // one sweep as mpmc_sweep launches it outside a graph, with stamps
        BoxView v = b->view(b->cur);
        if (k + 1 < sweeps) {
            v.cnt_can = nullptr;
            v.x_can = v.y_can = nullptr;
            v.tag_can = nullptr;
        }
        launch_fused_sweep(v, b->shape, b->stream, d);
        launch_advance(b->dev, (uint32_t)b->seed, (uint32_t)(b->seed >> 32), (uint32_t)b->g.W,
                       b->g.Lq, 1, b->stream);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(h.data(), d, words * 8, hipMemcpyDeviceToHost, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        b->cur ^= 1;
        ++b->host_sweeps;
        b->canon_in_c = true;
        unsigned long long first = ~0ull, last_entry = 0, last_end = 0;
        double busy = 0;
        for (size_t t = 0; t < tiles; ++t) {
            const unsigned long long *w = &h[kStampWords * t];
            for (int ph = 0; ph < 7; ++ph) sum[ph] += (double)(long long)(w[ph + 1] - w[ph]);
            sum[7] += (double)(long long)(w[7] - w[0]);
            sum[8] += (double)(long long)(w[0] - w[8]);
            busy += (double)(long long)(w[7] - w[8]);
            first = w[8] < first ? w[8] : first;
            last_entry = w[8] > last_entry ? w[8] : last_entry;
            last_end = w[7] > last_end ? w[7] : last_end;
        }
        const double span = (double)(long long)(last_end - first);
        sum[9] += span;
        sum[10] += span > 0 ? busy / span : 0.0;
        sum[11] += (double)(long long)(last_entry - first);
    }
    b->free_dev(d);
    if (rc) return rc;
    if (e != hipSuccess) return fail(MPMC_EDEVICE, "phase profile: %s", hipGetErrorString(e));
    const double us_per_tick = 1e3 / (double)(khz > 0 ? khz : 100000);
    for (int ph = 0; ph < 9; ++ph) phase_us[ph] = sum[ph] / ((double)tiles * sweeps) * us_per_tick;
    phase_us[9] = sum[9] / sweeps * us_per_tick;
    phase_us[10] = sum[10] / sweeps;
    phase_us[11] = sum[11] / sweeps * us_per_tick;
    return MPMC_OK;
}

extern "C" int mpmc_get_info(mpmc_box bh, mpmc_info *info) {
    if (!bh || !info) return fail(MPMC_EINVAL, "NULL argument");
    Box *b = B(bh);
    int rc = b->read_scalars();
    if (rc) return rc;
    memset(info, 0, sizeof *info);
    info->N = b->N;
    info->M = b->g.M;
    info->cap = b->g.cap;
    info->n_trial = b->p.n_trial;
    info->step_m = b->p.step_m;
    info->tile = b->shape.tile;
    info->schedule = b->sched;
    info->hist_bins = b->p.hist_bins;
    info->W = b->g.W;
    info->L = b->g.L;
    info->L_eff = (double)b->g.Lq * kQd;
    info->w = (double)b->g.w;
    info->eta = b->eta;
    info->eta_eff = (double)b->N * M_PI / (info->L_eff * info->L_eff);
    info->hist_dr = b->p.hist_dr;
    info->sweep = b->host.sweep;
    info->Sx = b->host.Sx;
    info->Sy = b->host.Sy;
    info->trials = b->host.trials;
    info->accepts = b->host.accepts;
    info->n_conf = b->n_conf;
    return MPMC_OK;
}

extern "C" int mpmc_get_cells(mpmc_box bh, uint8_t *cntp, uint32_t *tagp, float *xp, float *yp) {
    if (!bh) return fail(MPMC_EINVAL, "NULL box");
    Box *b = B(bh);
    const size_t nc = (size_t)b->g.M * b->g.M, ns = nc * b->g.CS;
    std::vector<uint8_t> hc(nc);
    std::vector<uint32_t> ht(ns);
    std::vector<float> hx(ns), hy(ns);
    const CellBuf cb = b->canon();
    HIPCHK(hipMemcpyAsync(hc.data(), cb.cnt, nc, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipMemcpyAsync(ht.data(), cb.tag, ns * 4, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipMemcpyAsync(hx.data(), cb.x, ns * 4, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipMemcpyAsync(hy.data(), cb.y, ns * 4, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    const uint32_t cap = b->g.cap;
    for (size_t c = 0; c < nc; ++c) {
        if (cntp) cntp[c] = hc[c];
        for (uint32_t s = 0; s < cap; ++s) {
            const bool used = s < hc[c];
            const size_t src = (size_t)s * nc + c, dst = c * cap + s;
            if (tagp) tagp[dst] = used ? ht[src] : 0;
            if (xp) xp[dst] = used ? hx[src] : 0.0f;
            if (yp) yp[dst] = used ? hy[src] : 0.0f;
        }
    }
    return MPMC_OK;
}

extern "C" int mpmc_get_positions(mpmc_box bh, double *xo, double *yo, int64_t *Xo, int64_t *Yo) {
    if (!bh) return fail(MPMC_EINVAL, "NULL box");
    Box *b = B(bh);
    int rc = b->read_scalars();
    if (rc) return rc;
    long long *dX = reinterpret_cast<long long *>(b->scratch_pos(0));
    long long *dY = reinterpret_cast<long long *>(b->scratch_pos(1));
    if (!dX || !dY) return fail(MPMC_ENOMEM, "position scratch");
    launch_positions(b->mview(), dX, dY, b->stream);
    HIPCHK(hipGetLastError());
    std::vector<int64_t> X(b->N), Y(b->N);
    HIPCHK(hipMemcpyAsync(X.data(), dX, (size_t)b->N * 8, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipMemcpyAsync(Y.data(), dY, (size_t)b->N * 8, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    for (uint32_t t = 0; t < b->N; ++t) {
        if (Xo) Xo[t] = X[t];
        if (Yo) Yo[t] = Y[t];
        if (xo) xo[t] = (double)X[t] * kQd;
        if (yo) yo[t] = (double)Y[t] * kQd;
    }
    return MPMC_OK;
}

void *Box::scratch_pos(int which) {
    if (!pos_scratch[which]) {
        if (alloc_dev(&pos_scratch[which], (size_t)N * 8)) return nullptr;
    }
    return pos_scratch[which];
}

extern "C" int mpmc_validate(mpmc_box bh, uint64_t *n_overlaps, uint64_t *n_bad) {
    if (!bh) return fail(MPMC_EINVAL, "NULL box");
    Box *b = B(bh);
    int rc = b->read_scalars();
    if (rc && rc != MPMC_EOVERFLOW) return rc;
    HIPCHK(hipMemsetAsync(b->scratch_u32, 0, (size_t)b->N * 4, b->stream));
    HIPCHK(hipMemsetAsync(&b->dev->bad, 0, 16, b->stream));
    launch_validate(b->mview(), b->scratch_u32, b->stream);
    HIPCHK(hipGetLastError());
    rc = b->read_scalars();
    if (rc && rc != MPMC_EOVERFLOW) return rc;
    if (n_overlaps) *n_overlaps = b->host.overlaps / 2;
    if (n_bad) *n_bad = b->host.bad + (b->host.overflow ? 1 : 0);
    return MPMC_OK;
}
