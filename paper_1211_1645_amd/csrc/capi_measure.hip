// capi_measure.hip — C ABI of the observables: contact histogram and
// pressure (Sec. II.C.1), psi_6 (Eq. (8)), C(dt) and tau (Eq. (9), Sec. III),
// checkpoints.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "mpmc_host.hpp"

using namespace mpmc;

#define HIPCHK(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(MPMC_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));           \
    } while (0)

static Box *B(mpmc_box b) { return reinterpret_cast<Box *>(b); }

// ---------------------------------------------------------------------------
// Least squares by modified Gram-Schmidt on the columns t^e, then back
// substitution.
int mpmc::lsq_poly(const std::vector<double> &t, const std::vector<double> &yv, uint32_t order,
                   double *coef) {
    const size_t K = t.size(), nc = order + 1;
    if (K < nc) return -1;
    std::vector<double> Q(K * nc), R(nc * nc, 0.0);
    for (size_t k = 0; k < K; ++k) {
        double v = 1.0;
        for (size_t e = 0; e < nc; ++e) { Q[e * K + k] = v; v *= t[k]; }
    }
    for (size_t e = 0; e < nc; ++e) {
        double *qe = &Q[e * K];
        for (size_t f = 0; f < e; ++f) {
            const double *qf = &Q[f * K];
            double d = 0.0;
            for (size_t k = 0; k < K; ++k) d += qf[k] * qe[k];
            R[f * nc + e] = d;
            for (size_t k = 0; k < K; ++k) qe[k] -= d * qf[k];
        }
        double nrm = 0.0;
        for (size_t k = 0; k < K; ++k) nrm += qe[k] * qe[k];
        nrm = sqrt(nrm);
        if (!(nrm > 0.0)) return -1;
        R[e * nc + e] = nrm;
        for (size_t k = 0; k < K; ++k) qe[k] /= nrm;
    }
    std::vector<double> qty(nc);
    for (size_t e = 0; e < nc; ++e) {
        double d = 0.0;
        for (size_t k = 0; k < K; ++k) d += Q[e * K + k] * yv[k];
        qty[e] = d;
    }
    for (int e = (int)nc - 1; e >= 0; --e) {
        double s = qty[e];
        for (size_t f = e + 1; f < nc; ++f) s -= R[e * nc + f] * coef[f];
        coef[e] = s / R[e * nc + e];
    }
    return 0;
}

int Box::measure_work() {
    if (meas_work) return MPMC_OK;
    return alloc_dev(&meas_work, measure_work_bytes(p.hist_bins));
}

int Box::locate() {
    if (!loc) {
        int rc = alloc_dev((void **)&loc, (size_t)N * 4);
        if (rc) return rc;
    }
    launch_locate(mview(), loc, stream);
    HIPCHK(hipGetLastError());
    return MPMC_OK;
}

// P* from ordered pair counts of n_conf configurations.
static int pressure_from_counts(const Box *b, const unsigned long long *ordered, uint64_t n_conf,
                                double *P, double *g0, double *Z) {
    const uint32_t K = b->p.hist_bins;
    const double dr = b->p.hist_dr;
    const double Le = (double)b->g.Lq * kQd, V = Le * Le;
    const double eta = (double)b->N * M_PI / V;
    const double pairs = 0.5 * (double)b->N * (double)(b->N - 1) * (double)n_conf;
    std::vector<double> t(K), gk(K);
    for (uint32_t k = 0; k < K; ++k) {
        const double r = 2.0 + ((double)k + 0.5) * dr;  // bin centre
        const double n = 0.5 * (double)ordered[k];      // unordered pairs
        gk[k] = (n / pairs) / (2.0 * M_PI * r * dr / V);  // Eq. (2)
        t[k] = (r - 2.0) / ((double)K * dr);
    }
    double c[9];
    if (lsq_poly(t, gk, b->p.fit_order, c) != 0) return fail(MPMC_ESTATE, "contact fit is singular");
    const double z = 1.0 + 2.0 * eta * ((double)(b->N - 1) / (double)b->N) * c[0];
    if (g0) *g0 = c[0];
    if (Z) *Z = z;
    if (P) *P = 4.0 * eta * z / M_PI;
    return MPMC_OK;
}

extern "C" int mpmc_accumulate_contacts(mpmc_box bh) {
    if (!bh) return fail(MPMC_EINVAL, "NULL box");
    Box *b = B(bh);
    if (int jrc = b->join_meas()) return jrc;
    if (b->N < 2) return fail(MPMC_EINVAL, "need at least two disks");
    const uint32_t K = b->p.hist_bins;
    const double rmax = 2.0 + K * b->p.hist_dr;
    const uint32_t h = ((double)b->g.w >= rmax) ? 1u : 2u;
    if (!measure_tiled(b->mview(), h)) {
        int lrc = b->locate();
        if (lrc) return lrc;
    }
    int wrc = b->measure_work();
    if (wrc) return wrc;
    launch_contact_hist(b->mview(), b->edges, K, h, b->hist, nullptr, b->loc, b->meas_work, b->stream);
    HIPCHK(hipGetLastError());
    ++b->n_conf;
    if (b->p.hist_block > 0 && b->n_conf - b->block_conf0 == b->p.hist_block) {
        std::vector<unsigned long long> now(K), diff(K);
        HIPCHK(hipMemcpyAsync(now.data(), b->hist, K * 8, hipMemcpyDeviceToHost, b->stream));
        HIPCHK(hipStreamSynchronize(b->stream));
        if (b->block_snapshot.size() != K) b->block_snapshot.assign(K, 0);
        for (uint32_t k = 0; k < K; ++k) diff[k] = now[k] - b->block_snapshot[k];
        double P;
        int rc = pressure_from_counts(b, diff.data(), b->p.hist_block, &P, nullptr, nullptr);
        if (rc == MPMC_OK) b->block_P.push_back(P);
        b->block_snapshot = now;
        b->block_conf0 = b->n_conf;
    }
    return MPMC_OK;
}

extern "C" int mpmc_reset_contacts(mpmc_box bh) {
    if (!bh) return fail(MPMC_EINVAL, "NULL box");
    Box *b = B(bh);
    if (int jrc = b->join_meas()) return jrc;
    HIPCHK(hipMemsetAsync(b->hist, 0, b->p.hist_bins * 8, b->stream));
    b->n_conf = 0;
    b->block_conf0 = 0;
    b->block_snapshot.clear();
    b->block_P.clear();
    return MPMC_OK;
}

extern "C" int mpmc_get_contacts(mpmc_box bh, int64_t *counts, uint64_t *n_conf) {
    if (!bh) return fail(MPMC_EINVAL, "NULL box");
    Box *b = B(bh);
    if (int jrc = b->join_meas()) return jrc;
    const uint32_t K = b->p.hist_bins;
    std::vector<unsigned long long> h(K);
    HIPCHK(hipMemcpyAsync(h.data(), b->hist, K * 8, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    if (counts)
        for (uint32_t k = 0; k < K; ++k) counts[k] = (int64_t)(h[k] / 2);
    if (n_conf) *n_conf = b->n_conf;
    return MPMC_OK;
}

extern "C" int mpmc_measure_pressure(mpmc_box bh, double *p_star, double *g_contact, double *z,
                                     double *se) {
    if (!bh) return fail(MPMC_EINVAL, "NULL box");
    Box *b = B(bh);
    if (int jrc = b->join_meas()) return jrc;
    if (b->n_conf == 0) return fail(MPMC_ESTATE, "no configuration accumulated");
    const uint32_t K = b->p.hist_bins;
    std::vector<unsigned long long> h(K);
    HIPCHK(hipMemcpyAsync(h.data(), b->hist, K * 8, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    int rc = pressure_from_counts(b, h.data(), b->n_conf, p_star, g_contact, z);
    if (rc) return rc;
    if (se) {
        const size_t nb = b->block_P.size();
        if (nb < 2) {
            *se = NAN;
        } else {
            double m = 0.0, v = 0.0;
            for (double x : b->block_P) m += x;
            m /= (double)nb;
            for (double x : b->block_P) v += (x - m) * (x - m);
            *se = sqrt(v / (double)(nb - 1) / (double)nb);
        }
    }
    return MPMC_OK;
}

extern "C" int mpmc_contact_hist_subset(mpmc_box bh, const uint8_t *sel, int64_t *counts) {
    if (!bh || !sel || !counts) return fail(MPMC_EINVAL, "NULL argument");
    Box *b = B(bh);
    if (int jrc = b->join_meas()) return jrc;
    const uint32_t K = b->p.hist_bins;
    uint8_t *dsel = nullptr;
    unsigned long long *dh = nullptr;
    int rc = b->alloc_dev((void **)&dsel, b->N);
    if (rc) return rc;
    rc = b->alloc_dev((void **)&dh, K * 8);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(dsel, sel, b->N, hipMemcpyHostToDevice, b->stream));
    HIPCHK(hipMemsetAsync(dh, 0, K * 8, b->stream));
    const double rmax = 2.0 + K * b->p.hist_dr;
    const uint32_t hs = ((double)b->g.w >= rmax) ? 1u : 2u;
    if (!measure_tiled(b->mview(), hs)) {
        rc = b->locate();
        if (rc) return rc;
    }
    rc = b->measure_work();
    if (rc) return rc;
    launch_contact_hist(b->mview(), b->edges, K, hs, dh, dsel, b->loc, b->meas_work, b->stream);
    HIPCHK(hipGetLastError());
    std::vector<unsigned long long> h(K);
    HIPCHK(hipMemcpyAsync(h.data(), dh, K * 8, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    for (uint32_t k = 0; k < K; ++k) counts[k] = (int64_t)h[k];
    // release the temporaries now rather than with the box
    for (void *ptr : {(void *)dsel, (void *)dh}) {
        for (size_t i = 0; i < b->allocations.size(); ++i)
            if (b->allocations[i] == ptr) {
                if (b->p.alloc) b->p.free(ptr, b->p.alloc_ctx);
                else (void)hipFree(ptr);
                b->allocations.erase(b->allocations.begin() + i);
                break;
            }
    }
    return MPMC_OK;
}

// ---------------------------------------------------------------------------
// psi_j by tag (re[N], im[N]), the cell field (re, im[M * M]) and psi_j by
// cell slot (re, im[CS * M * M]), allocated on first use.
int Box::psi_work() {
    if (psi_buf) return MPMC_OK;
    const size_t nc = (size_t)g.M * g.M;
    return alloc_dev((void **)&psi_buf, (2 * (size_t)N + 2 * nc + 2 * nc * g.CS) * 4);
}

extern "C" int mpmc_psi6_field(mpmc_box bh, float *re, float *im, float *fre, float *fim,
                               double *Psi_re, double *Psi_im, int on_device) {
    if (!bh) return fail(MPMC_EINVAL, "NULL box");
    Box *b = B(bh);
    if (int jrc = b->join_meas()) return jrc;
    if (b->N < 7) return fail(MPMC_EINVAL, "psi_6 needs at least 7 disks");
    const uint32_t M = b->g.M;
    const size_t nc = (size_t)M * M;
    if (int rc = b->psi_work()) return rc;
    float *dre = b->psi_buf, *dim = dre + b->N, *dfr = dim + b->N, *dfi = dfr + nc;
    float *dsr = dfi + nc, *dsi = dsr + nc * b->g.CS;
    const uint32_t hmax = (M - 2) / 2;  // 2h + 1 <= M - 1: no cell seen twice
    uint32_t h = hmax < 2 ? hmax : 2;
    if (h < 1) return fail(MPMC_EINVAL, "box too small for the neighbour search");
    int rc = b->measure_work();
    if (rc) return rc;
    bool located = false;
    // One host synchronisation per attempt: the field and the copies are
    // queued behind the psi kernel and discarded if its search was too short.
    for (;;) {
        if (!measure_tiled(b->mview(), h) && !located) {
            rc = b->locate();
            if (rc) return rc;
            located = true;
        }
        HIPCHK(hipMemsetAsync(&b->dev->psi_re, 0, 16, b->stream));
        HIPCHK(hipMemsetAsync(b->scratch_u32, 0, 4, b->stream));
        launch_psi6(b->mview(), h, dre, dim, dsr, dsi, b->scratch_u32, b->loc, b->meas_work, b->stream);
        HIPCHK(hipGetLastError());
        if (measure_tiled(b->mview(), h)) launch_psi6_field_slots(b->mview(), dsr, dsi, dfr, dfi, b->stream);
        else launch_psi6_field(b->mview(), dre, dim, dfr, dfi, b->stream);
        HIPCHK(hipGetLastError());
        const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        if (re) HIPCHK(hipMemcpyAsync(re, dre, (size_t)b->N * 4, kind, b->stream));
        if (im) HIPCHK(hipMemcpyAsync(im, dim, (size_t)b->N * 4, kind, b->stream));
        if (fre) HIPCHK(hipMemcpyAsync(fre, dfr, nc * 4, kind, b->stream));
        if (fim) HIPCHK(hipMemcpyAsync(fim, dfi, nc * 4, kind, b->stream));
        uint32_t failed = 0;
        HIPCHK(hipMemcpyAsync(&failed, b->scratch_u32, 4, hipMemcpyDeviceToHost, b->stream));
        rc = b->read_scalars();  // synchronises the stream
        if (rc) return rc;
        if (!failed) break;
        if (h >= hmax) return fail(MPMC_EINVAL, "six nearest neighbours lie beyond %u cells", h);
        ++h;
    }
    if (Psi_re) *Psi_re = b->host.psi_re / (double)b->N;
    if (Psi_im) *Psi_im = b->host.psi_im / (double)b->N;
    return MPMC_OK;
}

// ---------------------------------------------------------------------------
// The contact histogram and psi_6 of the current configuration on a stream of
// the box's own, so that they overlap the sweeps that follow: the kernels
// read the canonical state C, which the next run of sweeps overwrites only in
// its last sweep, after waiting for them.
constexpr int kAsyncPsiHalo = 3;

int Box::measure_async(double *Psi_dev, bool field) {
    if (in_batch) return fail(MPMC_ESTATE, "a batch box is measured through its batch");
    if (N < 7) return fail(MPMC_EINVAL, "psi_6 needs at least 7 disks");
    if (p.hist_block > 0) return fail(MPMC_EINVAL, "asynchronous measurement keeps no pressure blocks (hist_block must be 0)");
    const uint32_t K = p.hist_bins;
    const double rmax = 2.0 + K * p.hist_dr;
    const uint32_t hc = ((double)g.w >= rmax) ? 1u : 2u;
    // as mpmc_psi6_field: stencil 2 first, then the widest staged stencil,
    // but the second pass is launched always and decides on the device
    // whether it has anything to do (a wider stencil finds the same six
    // nearest, summed in its own stencil order; both paths keep the first
    // stencil that suffices, so they agree bit for bit)
    const uint32_t hmax = (g.M - 2) / 2;
    const uint32_t hp = hmax < (uint32_t)kAsyncPsiHalo ? hmax : (uint32_t)kAsyncPsiHalo;
    const uint32_t h1 = hp < 2u ? hp : 2u;
    if (hp < 1 || !measure_tiled(mview(), hc) || !measure_tiled(mview(), hp))
        return fail(MPMC_EINVAL, "asynchronous measurement needs the staged kernels (cells of at most 4 disks, a box of at least 6 cells)");
    int rc = materialize();  // the kernels read C
    if (rc) return rc;
    rc = measure_work();
    if (rc) return rc;
    const size_t nc = (size_t)g.M * g.M;
    rc = psi_work();
    if (rc) return rc;
    if (!async_fail) {  // [0]: verdict reported by mpmc_measure_wait, [1]: first pass
        rc = alloc_dev((void **)&async_fail, 8);
        if (rc) return rc;
        HIPCHK(hipMemsetAsync(async_fail, 0, 8, stream));
    }
    if (!meas_stream) {
        HIPCHK(hipStreamCreateWithFlags(&meas_stream, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&ev_swept, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&ev_meas, hipEventDisableTiming));
    }
    HIPCHK(hipEventRecord(ev_swept, stream));
    HIPCHK(hipStreamWaitEvent(meas_stream, ev_swept, 0));
    const MeasureView m = mview();
    float *dre = psi_buf, *dim = dre + N, *dfr = dim + N, *dfi = dfr + nc;
    float *dsr = dfi + nc, *dsi = dsr + nc * g.CS;
    if (h1 < hp) HIPCHK(hipMemsetAsync(async_fail + 1, 0, 4, meas_stream));
    if (hc <= h1) {
        // one staged scan for the contacts and the first psi_6 pass
        launch_measure_tiled(m, h1, hp, edges, K, hist, dre, dim, dsr, dsi, async_fail + 1,
                             async_fail, meas_work, meas_stream);
    } else {
        launch_contact_hist(m, edges, K, hc, hist, nullptr, loc, meas_work, meas_stream);
        HIPCHK(hipGetLastError());
        if (h1 < hp)
            launch_psi6_retry(m, h1, hp, dre, dim, dsr, dsi, async_fail + 1, async_fail, meas_work,
                              meas_stream);
        else
            launch_psi6(m, hp, dre, dim, dsr, dsi, async_fail, loc, meas_work, meas_stream);
    }
    HIPCHK(hipGetLastError());
    ++n_conf;
    if (field) {  // the staged kernels ran (checked above): psi_j by cell slot is there
        launch_psi6_field_slots(m, dsr, dsi, dfr, dfi, meas_stream);
        HIPCHK(hipGetLastError());
    }
    if (Psi_dev) {
        launch_psi_mean(dev, N, Psi_dev, meas_stream);
        HIPCHK(hipGetLastError());
    }
    HIPCHK(hipEventRecord(ev_meas, meas_stream));
    meas_pending = true;
    return MPMC_OK;
}

extern "C" int mpmc_measure_async(mpmc_box bh, double *Psi, int field) {
    if (!bh) return fail(MPMC_EINVAL, "NULL box");
    return B(bh)->measure_async(Psi, field != 0);
}

extern "C" int mpmc_measure_wait(mpmc_box bh, uint32_t *failed) {
    if (!bh) return fail(MPMC_EINVAL, "NULL box");
    Box *b = B(bh);
    uint32_t f = 0;
    if (b->meas_stream) {
        if (b->async_fail) {
            HIPCHK(hipMemcpyAsync(&f, b->async_fail, 4, hipMemcpyDeviceToHost, b->meas_stream));
            HIPCHK(hipMemsetAsync(b->async_fail, 0, 4, b->meas_stream));
        }
        HIPCHK(hipStreamSynchronize(b->meas_stream));
    }
    b->meas_pending = false;
    if (failed) *failed = f;
    return MPMC_OK;
}

// ---------------------------------------------------------------------------
// Eq. (9) with all time origins; tau from the exponential tail (Sec. III).
extern "C" int mpmc_acf(const double *re, const double *im, uint32_t n, uint32_t maxlag,
                        double *C) {
    if (!re || !im || !C || n == 0) return fail(MPMC_EINVAL, "bad series");
    double den = 0.0;
    for (uint32_t t = 0; t < n; ++t) den += re[t] * re[t] + im[t] * im[t];
    den /= n;
    if (!(den > 0.0)) return fail(MPMC_EINVAL, "series is zero");
    for (uint32_t d = 0; d <= maxlag; ++d) {
        if (d >= n) { C[d] = 0.0; continue; }
        double s = 0.0;
        for (uint32_t t = 0; t + d < n; ++t) s += re[t] * re[t + d] + im[t] * im[t + d];
        C[d] = s / (double)(n - d) / den;
    }
    return MPMC_OK;
}

extern "C" int mpmc_tau(const double *C, uint32_t maxlag, double lo, double hi, double *tau,
                        double *tau_int) {
    if (!C) return fail(MPMC_EINVAL, "NULL C");
    if (tau) {
        std::vector<double> t, y;
        for (uint32_t d = 1; d <= maxlag; ++d) {
            if (C[d] < lo) break;
            if (C[d] <= hi) { t.push_back(d); y.push_back(log(C[d])); }
        }
        double c[2];
        if (t.size() < 3 || lsq_poly(t, y, 1, c) != 0 || !(c[1] < 0.0))
            return fail(MPMC_ESTATE, "too few lags in the exponential window");
        *tau = -1.0 / c[1];
    }
    if (tau_int) {
        double ti = 0.5;
        for (uint32_t d = 1; d <= maxlag; ++d) {
            ti += C[d];
            if ((double)d >= 6.0 * ti) break;
        }
        *tau_int = ti;
    }
    return MPMC_OK;
}

// ---------------------------------------------------------------------------
// Checkpoints: a fixed header, then the current cell lists and the histogram.
namespace {
struct CkptHeader {
    char magic[8];
    uint32_t version, N;
    double eta;
    uint64_t seed;
    uint32_t step_m, n_trial, hist_bins, fit_order, hist_block, M;
    double cell_min, hist_dr;
    int64_t W;
    uint32_t cap, CS;
    DevScalars s;
    uint64_t n_conf, block_conf0, n_blocks;
};
const char kMagic[8] = {'M', 'P', 'M', 'C', 'C', 'K', 'P', '1'};
}  // namespace

extern "C" int mpmc_save(mpmc_box bh, const char *path) {
    if (!bh || !path) return fail(MPMC_EINVAL, "NULL argument");
    Box *b = B(bh);
    if (int jrc = b->join_meas()) return jrc;
    int rc = b->read_scalars();
    if (rc) return rc;
    const size_t nc = (size_t)b->g.M * b->g.M, ns = nc * b->g.CS;
    const uint32_t K = b->p.hist_bins;
    std::vector<uint8_t> hc(nc);
    std::vector<uint32_t> ht(ns);
    std::vector<float> hx(ns), hy(ns);
    std::vector<unsigned long long> hh(K);
    const CellBuf cb = b->canon();
    HIPCHK(hipMemcpyAsync(hc.data(), cb.cnt, nc, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipMemcpyAsync(ht.data(), cb.tag, ns * 4, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipMemcpyAsync(hx.data(), cb.x, ns * 4, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipMemcpyAsync(hy.data(), cb.y, ns * 4, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipMemcpyAsync(hh.data(), b->hist, K * 8, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    CkptHeader H;
    memset(&H, 0, sizeof H);
    memcpy(H.magic, kMagic, 8);
    H.version = 2;  // slot-major cell lists
    H.N = b->N;
    H.eta = b->eta;
    H.seed = b->seed;
    H.step_m = b->p.step_m;
    H.n_trial = b->p.n_trial;
    H.hist_bins = K;
    H.fit_order = b->p.fit_order;
    H.hist_block = b->p.hist_block;
    H.M = b->g.M;
    H.cell_min = b->p.cell_min;
    H.hist_dr = b->p.hist_dr;
    H.W = b->g.W;
    H.cap = b->g.cap;
    H.CS = b->g.CS;
    H.s = b->host;
    H.n_conf = b->n_conf;
    H.block_conf0 = b->block_conf0;
    H.n_blocks = b->block_P.size();
    std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "wb");
    if (!f) return fail(MPMC_EIO, "cannot open %s", tmp.c_str());
    bool ok = fwrite(&H, sizeof H, 1, f) == 1;
    ok = ok && fwrite(hc.data(), 1, nc, f) == nc;
    ok = ok && fwrite(ht.data(), 4, ns, f) == ns;
    ok = ok && fwrite(hx.data(), 4, ns, f) == ns;
    ok = ok && fwrite(hy.data(), 4, ns, f) == ns;
    ok = ok && fwrite(hh.data(), 8, K, f) == K;
    if (H.n_blocks) ok = ok && fwrite(b->block_P.data(), 8, H.n_blocks, f) == H.n_blocks;
    std::vector<unsigned long long> snap = b->block_snapshot;
    snap.resize(K, 0);
    ok = ok && fwrite(snap.data(), 8, K, f) == K;
    ok = (fclose(f) == 0) && ok;
    if (!ok || rename(tmp.c_str(), path) != 0) return fail(MPMC_EIO, "writing %s failed", path);
    return MPMC_OK;
}

extern "C" int mpmc_load(mpmc_box *out, const char *path, const mpmc_params *pp) {
    if (!out || !path) return fail(MPMC_EINVAL, "NULL argument");
    *out = nullptr;
    FILE *f = fopen(path, "rb");
    if (!f) return fail(MPMC_EIO, "cannot open %s", path);
    CkptHeader H;
    if (fread(&H, sizeof H, 1, f) != 1 || memcmp(H.magic, kMagic, 8) != 0 || H.version != 2) {
        fclose(f);
        return fail(MPMC_EIO, "%s is not an MPMC checkpoint", path);
    }
    mpmc_params p;
    mpmc_default_params(&p);
    if (pp) p = *pp;
    p.step_m = H.step_m;
    p.n_trial = H.n_trial;
    p.hist_bins = H.hist_bins;
    p.fit_order = H.fit_order;
    p.hist_block = H.hist_block;
    p.cell_min = H.cell_min;
    p.hist_dr = H.hist_dr;
    p.lattice = MPMC_LATTICE_NONE;
    Box *b = nullptr;
    int rc = create_box(&b, H.N, H.eta, H.seed, &p);
    if (rc) { fclose(f); return rc; }
    if (b->g.M != H.M || b->g.W != H.W || b->g.cap != H.cap || b->g.CS != H.CS) {
        fclose(f);
        b->release();
        delete b;
        return fail(MPMC_EIO, "checkpoint geometry does not match the box these parameters give");
    }
    const size_t nc = (size_t)H.M * H.M, ns = nc * H.CS;
    const uint32_t K = H.hist_bins;
    std::vector<uint8_t> hc(nc);
    std::vector<uint32_t> ht(ns);
    std::vector<float> hx(ns), hy(ns);
    std::vector<unsigned long long> hh(K), snap(K);
    std::vector<double> blocks(H.n_blocks);
    bool ok = fread(hc.data(), 1, nc, f) == nc && fread(ht.data(), 4, ns, f) == ns &&
              fread(hx.data(), 4, ns, f) == ns && fread(hy.data(), 4, ns, f) == ns &&
              fread(hh.data(), 8, K, f) == K;
    if (ok && H.n_blocks) ok = fread(blocks.data(), 8, H.n_blocks, f) == H.n_blocks;
    ok = ok && fread(snap.data(), 8, K, f) == K;
    fclose(f);
    if (!ok) {
        b->release();
        delete b;
        return fail(MPMC_EIO, "%s is truncated", path);
    }
    rc = b->upload(hc, ht, hx, hy, H.s);
    if (rc == MPMC_OK) {
        hipError_t e = hipMemcpyAsync(b->hist, hh.data(), K * 8, hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) rc = fail(MPMC_EDEVICE, "upload: %s", hipGetErrorString(e));
    }
    if (rc == MPMC_OK) rc = b->choose_schedule();
    if (rc) {
        b->release();
        delete b;
        return rc;
    }
    b->placed = true;
    b->n_conf = H.n_conf;
    b->block_conf0 = H.block_conf0;
    b->block_P = blocks;
    b->block_snapshot = snap;
    *out = reinterpret_cast<mpmc_box>(b);
    return MPMC_OK;
}
