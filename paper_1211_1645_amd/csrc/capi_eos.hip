// capi_eos.hip — host analysis of the equation of state (Sec. IV.A): the
// Mayer-Wood loop of P*(eta) in a finite box, its Maxwell pressure, the
// interface free energy per disk, and its scaling with N.  No device code.
#include <math.h>

#include <vector>

#include "mpmc_host.hpp"

using namespace mpmc;

namespace {

constexpr int kGrid = 8192;  // samples of [lo, hi] when bracketing stationary points

// Weighted least squares: minimise sum ((y_k - sum_e c_e t_k^e) / s_k)^2 by
// modified Gram-Schmidt on the scaled columns, then back substitution.
int wlsq(const std::vector<double> &t, const std::vector<double> &y, const std::vector<double> &s,
         int order, std::vector<double> &c) {
    const size_t K = t.size(), nc = (size_t)order + 1;
    std::vector<double> Q(K * nc), R(nc * nc, 0.0), b(K);
    for (size_t k = 0; k < K; ++k) {
        double p = 1.0 / s[k];
        b[k] = y[k] / s[k];
        for (size_t e = 0; e < nc; ++e) { Q[e * K + k] = p; p *= t[k]; }
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
    c.assign(nc, 0.0);
    for (int e = (int)nc - 1; e >= 0; --e) {
        double d = 0.0;
        for (size_t k = 0; k < K; ++k) d += Q[e * K + k] * b[k];
        for (size_t f = e + 1; f < nc; ++f) d -= R[e * nc + f] * c[f];
        c[e] = d / R[e * nc + e];
    }
    return 0;
}

double horner(const std::vector<double> &c, double u) {
    double r = 0.0;
    for (int e = (int)c.size() - 1; e >= 0; --e) r = r * u + c[e];
    return r;
}

std::vector<double> deriv(const std::vector<double> &c) {
    std::vector<double> d(c.size() > 1 ? c.size() - 1 : 1, 0.0);
    for (size_t e = 1; e < c.size(); ++e) d[e - 1] = (double)e * c[e];
    return d;
}

std::vector<double> integ(const std::vector<double> &c) {
    std::vector<double> I(c.size() + 1, 0.0);
    for (size_t e = 0; e < c.size(); ++e) I[e + 1] = c[e] / (double)(e + 1);
    return I;
}

// Root of f(u) - level on [a, b] where f(a) - level and f(b) - level differ
// in sign (bisection to the last bit).
double bisect(const std::vector<double> &f, double level, double a, double b) {
    double fa = horner(f, a) - level;
    for (int it = 0; it < 200; ++it) {
        const double m = 0.5 * (a + b);
        if (m <= a || m >= b) break;
        const double fm = horner(f, m) - level;
        if (fm == 0.0) return m;
        if ((fm < 0.0) == (fa < 0.0)) { a = m; fa = fm; } else b = m;
    }
    return 0.5 * (a + b);
}

}  // namespace

extern "C" int mpmc_eos_loop(const double *eta, const double *p_star, const double *se,
                             uint32_t n, uint32_t order, mpmc_eos_loop_result *out) {
    if (!eta || !p_star || !out) return fail(MPMC_EINVAL, "NULL argument");
    if (order < 3 || order > 9) return fail(MPMC_EINVAL, "order must be 3..9");
    if (n < order + 2) return fail(MPMC_EINVAL, "need at least order + 2 points");
    std::vector<double> v(n), y(n), s(n, 1.0);
    double mean = 0.0;
    for (uint32_t i = 0; i < n; ++i) {
        if (!(eta[i] > 0.0 && eta[i] <= M_PI / 4) || !isfinite(p_star[i]))
            return fail(MPMC_EINVAL, "point %u out of range", i);
        if (se && !(se[i] > 0.0 && isfinite(se[i])))
            return fail(MPMC_EINVAL, "standard error %u not positive", i);
        v[i] = M_PI / eta[i];  // area per disk, sigma the radius
        y[i] = p_star[i];
        if (se) s[i] = se[i];
        mean += v[i];
    }
    mean /= n;
    double lo = INFINITY, hi = -INFINITY;
    for (uint32_t i = 0; i < n; ++i) {
        v[i] -= mean;
        lo = fmin(lo, v[i]);
        hi = fmax(hi, v[i]);
    }
    if (!(hi > lo)) return fail(MPMC_EINVAL, "all densities equal");
    std::vector<double> c;
    if (wlsq(v, y, s, (int)order, c)) return fail(MPMC_EINVAL, "polynomial fit is singular");
    const std::vector<double> d1 = deriv(c), d2 = deriv(d1);
    // stationary points of P*(v) in [lo, hi]
    std::vector<double> st;
    double prev = horner(d1, lo), uprev = lo;
    for (int g = 1; g <= kGrid; ++g) {
        const double u = g == kGrid ? hi : lo + (hi - lo) * g / kGrid;
        const double f = horner(d1, u);
        if (prev == 0.0) st.push_back(uprev);
        else if ((f < 0.0) != (prev < 0.0) && f != 0.0) st.push_back(bisect(d1, 0.0, uprev, u));
        prev = f;
        uprev = u;
    }
    if (prev == 0.0) st.push_back(hi);
    int nmax = 0, nmin = 0;
    double umax = 0.0, umin = 0.0;
    for (double u : st) {
        const double cur = horner(d2, u);
        if (cur < 0.0) { ++nmax; umax = u; }
        if (cur > 0.0) { ++nmin; umin = u; }
    }
    if (nmax != 1 || nmin != 1 || !(umin < umax))
        return fail(MPMC_ESTATE, "no Mayer-Wood loop (one maximum at lower density, one "
                                 "minimum at higher density) in the fitted range");
    const double Pmax = horner(c, umax), Pmin = horner(c, umin);
    // admissible coexistence pressures: the outer roots stay inside the data
    const double plo = fmax(Pmin, horner(c, hi)), phi = fmin(Pmax, horner(c, lo));
    const std::vector<double> I = integ(c);
    auto roots = [&](double Pc, double r[3]) {
        r[0] = bisect(c, Pc, lo, umin);
        r[1] = bisect(c, Pc, umin, umax);
        r[2] = bisect(c, Pc, umax, hi);
    };
    auto area = [&](double Pc, double a, double b) {
        return (horner(I, b) - horner(I, a)) - Pc * (b - a);
    };
    if (!(phi > plo)) return fail(MPMC_ESTATE, "the Maxwell construction leaves the data range");
    double a = plo, b = phi, r[3];
    roots(a, r);
    const double ga = area(a, r[0], r[2]);
    roots(b, r);
    const double gb = area(b, r[0], r[2]);
    if (!((ga > 0.0) && (gb < 0.0)))
        return fail(MPMC_ESTATE, "the Maxwell construction leaves the data range");
    for (int it = 0; it < 200; ++it) {
        const double m = 0.5 * (a + b);
        if (m <= a || m >= b) break;
        roots(m, r);
        if (area(m, r[0], r[2]) > 0.0) a = m; else b = m;
    }
    const double Pc = 0.5 * (a + b);
    roots(Pc, r);
    out->eta_max = M_PI / (umax + mean);
    out->p_max = Pmax;
    out->eta_min = M_PI / (umin + mean);
    out->p_min = Pmin;
    out->p_coex = Pc;
    out->eta_liquid = M_PI / (r[2] + mean);
    out->eta_solid = M_PI / (r[0] + mean);
    out->delta_f = 0.25 * fabs(area(Pc, r[0], r[1]));
    return MPMC_OK;
}

extern "C" int mpmc_power_law(const double *x, const double *y, uint32_t n, double *exponent,
                              double *prefactor) {
    if (!x || !y || n < 2) return fail(MPMC_EINVAL, "need at least two points");
    double mx = 0.0, my = 0.0;
    for (uint32_t i = 0; i < n; ++i) {
        if (!(x[i] > 0.0) || !(y[i] > 0.0) || !isfinite(x[i]) || !isfinite(y[i]))
            return fail(MPMC_EINVAL, "point %u not positive", i);
        mx += log(x[i]);
        my += log(y[i]);
    }
    mx /= n;
    my /= n;
    double sxx = 0.0, sxy = 0.0;
    for (uint32_t i = 0; i < n; ++i) {
        const double dx = log(x[i]) - mx;
        sxx += dx * dx;
        sxy += dx * (log(y[i]) - my);
    }
    if (!(sxx > 0.0)) return fail(MPMC_EINVAL, "all x equal");
    const double b = sxy / sxx;
    if (exponent) *exponent = b;
    if (prefactor) *prefactor = exp(my - b * mx);
    return MPMC_OK;
}
