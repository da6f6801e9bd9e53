// capi_positional.hip — C ABI of the positional order: the
// structure factor at the wave vectors of the periodic box, the search for
// the first diffraction peak q0, chi_j and its field (Sec. IV.C), and C_q(r)
// (Sec. IV.D).
#include <math.h>

#include <mutex>
#include <vector>

#include "mpmc_host.hpp"

using namespace mpmc;

#define HIPCHK(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(MPMC_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));           \
    } while (0)

namespace {
Box *B(mpmc_box b) { return reinterpret_cast<Box *>(b); }

constexpr int32_t kMaxIndex = 4096;   // |h|, |k| below this
constexpr uint32_t kChunk = 65536;    // wave vectors per launch
constexpr uint32_t kMaxBins = 4096;   // C_q windows (LDS: 12 bytes each)
constexpr uint32_t kMaxScan = 1u << 24;  // wave vectors one q0 search may visit
constexpr double kQunit = 1.0 / 4194304.0;  // 2^-22

// S at nq wave vectors (host hk, host S), in launches of at most kChunk.
int structure_factor(Box *b, const int32_t *hk, uint32_t nq, double *S) {
    int rc = b->read_scalars();  // the accumulated shift places the disks
    if (rc) return rc;
    const MeasureView m = b->mview();
    const uint32_t chunk = nq < kChunk ? nq : kChunk;
    const size_t part = (rho_work_bytes(m, chunk) + 255) & ~(size_t)255;
    const size_t stage = (size_t)chunk * 8;
    rc = b->pos_work_at_least(part + 2 * stage);
    if (rc) return rc;
    char *base = static_cast<char *>(b->pos_work);
    int32_t *dhk = reinterpret_cast<int32_t *>(base + part);
    double *dS = reinterpret_cast<double *>(base + part + stage);
    for (uint32_t q0 = 0; q0 < nq; q0 += chunk) {
        const uint32_t n = nq - q0 < chunk ? nq - q0 : chunk;
        HIPCHK(hipMemcpyAsync(dhk, hk + 2 * (size_t)q0, (size_t)n * 8, hipMemcpyHostToDevice,
                              b->stream));
        launch_structure_factor(m, dhk, n, dS, base, b->stream);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(S + q0, dS, (size_t)n * 8, hipMemcpyDeviceToHost, b->stream));
        HIPCHK(hipStreamSynchronize(b->stream));
    }
    return MPMC_OK;
}
}  // namespace

int Box::pos_work_at_least(size_t bytes) {
    if (pos_work && pos_work_bytes >= bytes) return MPMC_OK;
    if (pos_work) {
        HIPCHK(hipStreamSynchronize(stream));
        free_dev(pos_work);
        pos_work = nullptr;
        pos_work_bytes = 0;
    }
    int rc = alloc_dev(&pos_work, bytes);
    if (rc) return rc;
    pos_work_bytes = bytes;
    return MPMC_OK;
}

extern "C" int mpmc_structure_factor(mpmc_box bh, const int32_t *hk, uint32_t nq, double *S) {
    if (!bh) return fail(MPMC_EINVAL, "NULL box");
    if (nq == 0) return MPMC_OK;
    if (!hk || !S) return fail(MPMC_EINVAL, "NULL wave-vector or output array");
    for (uint32_t i = 0; i < 2 * nq; ++i)
        if (hk[i] <= -kMaxIndex || hk[i] >= kMaxIndex)
            return fail(MPMC_EINVAL, "wave-vector index %d outside (-%d, %d)", hk[i], kMaxIndex,
                        kMaxIndex);
    return structure_factor(B(bh), hk, nq, S);
}

// ---------------------------------------------------------------------------
// Structure factor without allocation.  The per-workgroup partial sums of
// k_rho go to a fixed device array instead of the box's growable work
// buffer: at most kNoAllocQ wave vectors per call, 64 workgroup rows each of
// 16 bytes, 4 MiB held by every device the library runs on until the process
// ends.  Host code never passes `scratch` itself to a kernel or copy (its
// host-side name is not a device address): it uses the address that
// hipGetSymbolAddress returns for the device, looked up once per device.
namespace {
constexpr uint32_t kNoAllocQ = 4096;
constexpr size_t kScratchBytes = (size_t)64 * kNoAllocQ * 16;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// The scratch address on the device of stream st (NULL: the current device).
static int scratch_on(hipStream_t st, void **out) {
    int cur = 0, dev = 0;
    HIPCHK(hipGetDevice(&cur));
    dev = cur;
    if (st) HIPCHK(hipStreamGetDevice(st, &dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(MPMC_EDEVICE, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        if (dev != cur) HIPCHK(hipSetDevice(dev));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (dev != cur) HIPCHK(hipSetDevice(cur));
        if (e != hipSuccess)
            return fail(MPMC_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return MPMC_OK;
}

extern "C" int mpmc_structure_factor_noalloc(mpmc_box bh, const int32_t *hk, uint32_t nq,
                                             double *S) {
    if (!bh) return fail(MPMC_EINVAL, "NULL box");
    if (nq == 0) return MPMC_OK;
    if (!hk || !S) return fail(MPMC_EINVAL, "NULL wave-vector or output array");
    if (nq > kNoAllocQ)
        return fail(MPMC_EINVAL, "%u wave vectors: at most %u per call without allocation", nq,
                    kNoAllocQ);
    Box *b = B(bh);
    void *work = nullptr;
    int rc = scratch_on(b->stream, &work);
    if (rc) return rc;
    rc = b->read_scalars();  // the accumulated shift places the disks
    if (rc) return rc;
    const MeasureView m = b->mview();
    if (rho_work_bytes(m, nq) > kScratchBytes)
        return fail(MPMC_EINVAL, "partials of %zu bytes exceed the %zu-byte scratch",
                    rho_work_bytes(m, nq), kScratchBytes);
    launch_structure_factor(m, hk, nq, S, work, b->stream);
    HIPCHK(hipGetLastError());
    return MPMC_OK;
}

extern "C" int mpmc_find_q0(mpmc_box bh, double q_lo, double q_hi, double theta0, double dtheta,
                            int32_t *h_out, int32_t *k_out, double *S_out) {
    if (!bh) return fail(MPMC_EINVAL, "NULL box");
    Box *b = B(bh);
    if (!(q_lo >= 0.0) || !(q_hi > q_lo) || !(dtheta > 0.0) || !isfinite(theta0))
        return fail(MPMC_EINVAL, "bad search window");
    const double L = (double)b->g.Lq * kQunit, unit = 2.0 * M_PI / L;
    const double n_hi = q_hi / unit;
    if (!(n_hi < (double)kMaxIndex)) return fail(MPMC_EINVAL, "q_hi beyond the index range");
    const double n2lo = (q_lo / unit) * (q_lo / unit), n2hi = n_hi * n_hi;
    const double full = 2.0 * M_PI;
    std::vector<int32_t> hk;
    const int32_t r = (int32_t)ceil(n_hi);
    // every index pair of the annulus owns a unit square inside the annulus
    // widened by sqrt 2 on both sides, so this area bounds their number
    const double wlo = fmax(0.0, sqrt(n2lo) - M_SQRT2), whi = n_hi + M_SQRT2;
    if (M_PI * (whi * whi - wlo * wlo) > (double)kMaxScan)
        return fail(MPMC_EINVAL, "search window holds more than %u wave vectors", kMaxScan);
    for (int32_t k = -r; k <= r; ++k)
        for (int32_t h = -r; h <= r; ++h) {
            const double n2 = (double)h * h + (double)k * k;
            if (n2 < n2lo || n2 > n2hi || n2 == 0.0) continue;
            if (dtheta < full) {
                double a = fmod(atan2((double)k, (double)h) - theta0, full);
                if (a < 0.0) a += full;
                if (!(a < dtheta)) continue;
            }
            hk.push_back(h);
            hk.push_back(k);
        }
    const uint32_t nq = (uint32_t)(hk.size() / 2);
    if (nq == 0) return fail(MPMC_EINVAL, "no allowed wave vector in the search window");
    std::vector<double> S(nq);
    int rc = structure_factor(b, hk.data(), nq, S.data());
    if (rc) return rc;
    uint32_t best = 0;
    for (uint32_t i = 1; i < nq; ++i)
        if (S[i] > S[best]) best = i;
    if (h_out) *h_out = hk[2 * best];
    if (k_out) *k_out = hk[2 * best + 1];
    if (S_out) *S_out = S[best];
    return MPMC_OK;
}

extern "C" int mpmc_chi_field(mpmc_box bh, int32_t h, int32_t k, float *re, float *im,
                              float *fre, float *fim, int on_device) {
    if (!bh) return fail(MPMC_EINVAL, "NULL box");
    Box *b = B(bh);
    if (h <= -kMaxIndex || h >= kMaxIndex || k <= -kMaxIndex || k >= kMaxIndex)
        return fail(MPMC_EINVAL, "wave-vector index outside (-%d, %d)", kMaxIndex, kMaxIndex);
    const size_t nc = (size_t)b->g.M * b->g.M;
    if (!b->chi_buf) {
        int rc = b->alloc_dev((void **)&b->chi_buf, (2 * (size_t)b->N + 2 * nc) * 4);
        if (rc) return rc;
    }
    float *dre = b->chi_buf, *dim = dre + b->N, *dfr = dim + b->N, *dfi = dfr + nc;
    int rc = b->read_scalars();  // the accumulated shift places the disks
    if (rc) return rc;
    const MeasureView m = b->mview();
    launch_chi(m, h, k, dre, dim, b->stream);
    HIPCHK(hipGetLastError());
    if (fre || fim) {
        launch_psi6_field(m, dre, dim, dfr, dfi, b->stream);
        HIPCHK(hipGetLastError());
    }
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (re) HIPCHK(hipMemcpyAsync(re, dre, (size_t)b->N * 4, kind, b->stream));
    if (im) HIPCHK(hipMemcpyAsync(im, dim, (size_t)b->N * 4, kind, b->stream));
    if (fre) HIPCHK(hipMemcpyAsync(fre, dfr, nc * 4, kind, b->stream));
    if (fim) HIPCHK(hipMemcpyAsync(fim, dfi, nc * 4, kind, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    return MPMC_OK;
}

extern "C" int mpmc_cq(mpmc_box bh, double qx, double qy, double dr, uint32_t nbins, double *num,
                       int64_t *cnt) {
    if (!bh) return fail(MPMC_EINVAL, "NULL box");
    Box *b = B(bh);
    if (!num || !cnt) return fail(MPMC_EINVAL, "NULL output");
    if (nbins == 0 || nbins > kMaxBins) return fail(MPMC_EINVAL, "bins must be 1..%u", kMaxBins);
    if (!isfinite(qx) || !isfinite(qy)) return fail(MPMC_EINVAL, "non-finite wave vector");
    const double Dr = ldexp(dr, 22);
    if (!(Dr > 0.0) || Dr != floor(Dr)) return fail(MPMC_EINVAL, "dr must be a positive multiple of 2^-22");
    const double L = (double)b->g.Lq * kQunit;
    const double top = (double)(nbins - 1) * dr + 1.0;
    if (!(top < 0.5 * L) || !(top < 512.0))
        return fail(MPMC_EINVAL, "outer window edge %.6g beyond min(L/2, 512)", top);
    const double wq = (double)b->g.W;
    const int R = (int)floor(ldexp(top, 22) / wq) + 1;
    const MeasureView m = b->mview();
    const size_t rows = (cq_work_bytes(m, nbins) + 255) & ~(size_t)255;
    const size_t outb = (size_t)nbins * 16;
    int rc = b->pos_work_at_least(rows + outb);
    if (rc) return rc;
    char *base = static_cast<char *>(b->pos_work);
    double *dnum = reinterpret_cast<double *>(base + rows);
    unsigned long long *dcnt = reinterpret_cast<unsigned long long *>(dnum + nbins);
    launch_cq(m, qx, qy, dr, nbins, R, top, base, dnum, dcnt, b->stream);
    HIPCHK(hipGetLastError());
    std::vector<double> hn(nbins);
    std::vector<unsigned long long> hc(nbins);
    HIPCHK(hipMemcpyAsync(hn.data(), dnum, (size_t)nbins * 8, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipMemcpyAsync(hc.data(), dcnt, (size_t)nbins * 8, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    for (uint32_t i = 0; i < nbins; ++i) {
        num[i] += hn[i];
        cnt[i] += (int64_t)hc[i];
    }
    return MPMC_OK;
}

// Sec. IV.D: before averaging over configurations, each one is turned so that
// its Psi_6 points the same way; equivalently q0 turns with the
// configuration, by one sixth of the change in arg Psi_6 (principal value).
extern "C" int mpmc_cq_aligned(mpmc_box bh, double qx, double qy, double psi_arg_ref, double dr,
                               uint32_t nbins, double *num, int64_t *cnt, double *angle) {
    if (!bh) return fail(MPMC_EINVAL, "NULL box");
    if (!isfinite(psi_arg_ref)) return fail(MPMC_EINVAL, "non-finite reference phase");
    double pr = 0.0, pi = 0.0;
    int rc = mpmc_psi6_field(bh, nullptr, nullptr, nullptr, nullptr, &pr, &pi, 0);
    if (rc) return rc;
    if (!(pr * pr + pi * pi > 0.0)) return fail(MPMC_EINVAL, "Psi_6 vanishes: no orientation");
    double d = atan2(pi, pr) - psi_arg_ref;
    d = remainder(d, 2.0 * M_PI);  // (-pi, pi]
    const double a = d / 6.0;
    const double c = cos(a), s = sin(a);
    rc = mpmc_cq(bh, c * qx - s * qy, s * qx + c * qy, dr, nbins, num, cnt);
    if (rc) return rc;
    if (angle) *angle = a;
    return MPMC_OK;
}

// Incoherent averaging (appendix on configuration averaging): the maximum of
// C within each group of `width` consecutive windows.
extern "C" int mpmc_cq_bin_max(const double *C, uint32_t n, uint32_t width, double *out) {
    if (!C || !out || n == 0 || width == 0) return fail(MPMC_EINVAL, "bad series");
    for (uint32_t g = 0; g * width < n; ++g) {
        double m = C[(size_t)g * width];
        for (uint32_t i = g * width + 1; i < n && i < (g + 1) * width; ++i)
            if (C[i] > m) m = C[i];
        out[g] = m;
    }
    return MPMC_OK;
}
