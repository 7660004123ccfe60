// Host-side plan construction (see plan_host.hpp).
#include "plan_host.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <numeric>

namespace phi {

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;
// Size of the neglected tails that fixes the default sigma and c (Sec. 2.1
// leaves the constants to the cost trade-off sigma = O(1/P)): the periodic
// images of the I1 kernel on the 2x padded box and the disk tail e^{-c^2/sigma^2}
// are both exp(-lambda) with lambda = ln(1e16).
constexpr double kLogInvEpsSplit = 36.841361487904734;  // ln(1e16)

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

std::string fmt(const char* f, double a = 0, double b = 0) {
    char buf[256];
    std::snprintf(buf, sizeof(buf), f, a, b);
    return buf;
}

// Modulo for possibly negative numerators.
int posmod(int a, int b) { int r = a % b; return r < 0 ? r + b : r; }

}  // namespace

phi_status fill_defaults(phi_params* p, int32_t n, double h, phi_dtype dtype) {
    if (!p) return PHI_ERR_INVALID_ARG;
    p->nx = p->ny = n;
    p->hx = p->hy = h;
    p->n_r = 64;
    p->n_theta = 128;
    p->tol = (dtype == PHI_F32) ? 1e-7 : 1e-12;
    p->pad = 2;
    p->sigma = 0.0;
    p->cutoff = 0.0;
    p->dtype = dtype;
    p->flags = 0;
    p->bin = 0;
    p->sub_nodes = 0;
    return PHI_OK;
}

// Gauss-Legendre rule on [-1, 1], nodes ascending.  Newton's method is run on
// the angle theta (x = cos theta) with P_n from the three-term recurrence
// n P_n = (2n-1) x P_{n-1} - (n-1) P_{n-2} and the identity
// (1 - x^2) P_n'(x) = n (P_{n-1} - x P_n); the weight
// 2 / ((1 - x^2) P_n'^2) = 2 sin^2(theta) / (n (P_{n-1} - x P_n))^2 then never
// forms 1 - x^2 by cancellation near the interval ends.
void gauss_legendre(int n, double* x, double* w) {
    auto legendre = [n](double z, double* pn, double* pn1) {
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        *pn = p1;
        *pn1 = p0;
    };
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double th = kPi * (i + 0.75) / (n + 0.5);
        for (int it = 0; it < 100; ++it) {
            double pn, pn1;
            const double z = std::cos(th);
            legendre(z, &pn, &pn1);
            const double s = std::sin(th);
            // d/dtheta P_n(cos theta) = -sin(theta) P_n'(x) = -n (P_{n-1} - x P_n) / sin(theta)
            const double deriv = -n * (pn1 - z * pn) / s;
            const double dth = pn / deriv;
            th -= dth;
            if (std::fabs(dth) < 1e-16) break;
        }
        double pn, pn1;
        const double z = std::cos(th);
        legendre(z, &pn, &pn1);
        const double s = std::sin(th);
        const double d = n * (pn1 - z * pn);
        const double wi = 2.0 * s * s / (d * d);
        x[i] = -z;            // theta increases from 0: the largest nodes come first
        x[n - 1 - i] = z;
        w[i] = wi;
        w[n - 1 - i] = wi;
    }
    if (n % 2 == 1) x[n / 2] = 0.0;
}

// Gauss-Jacobi rule for the weight (1 + x) on [-1, 1] (alpha = 0, beta = 1),
// nodes ascending.  P_n = P_n^{(0,1)} from the three-term recurrence
//   (k+1)(2k-1) P_k = ((2k+1)(2k-1) x - 1) P_{k-1} - (k-1)(2k+1) P_{k-2},
// P_0 = 1, P_1 = (3x - 1)/2, its derivative from
//   (2n+1)(1 - x^2) P_n' = -n (1 + (2n+1) x) P_n + 2 n (n+1) P_{n-1},
// Newton from the asymptotic zeros cos((k - 1/4) pi / (n + 1)), and the
// weights 4 / ((1 - x^2) P_n'(x)^2).
void gauss_jacobi01(int n, double* x, double* w) {
    auto jacobi = [n](double z, double* pn, double* pn1) {
        double p0 = 1.0, p1 = 0.5 * (3.0 * z - 1.0);
        if (n == 1) {
            *pn = p1;
            *pn1 = p0;
            return;
        }
        for (int k = 2; k <= n; ++k) {
            const double p2 = (((2.0 * k + 1.0) * (2.0 * k - 1.0) * z - 1.0) * p1 - (k - 1.0) * (2.0 * k + 1.0) * p0) /
                              ((k + 1.0) * (2.0 * k - 1.0));
            p0 = p1;
            p1 = p2;
        }
        *pn = p1;
        *pn1 = p0;
    };
    auto deriv = [n](double z, double pn, double pn1) {
        return (-n * (1.0 + (2.0 * n + 1.0) * z) * pn + 2.0 * n * (n + 1.0) * pn1) / ((2.0 * n + 1.0) * (1.0 - z * z));
    };
    for (int k = 1; k <= n; ++k) {
        double z = std::cos((k - 0.25) * kPi / (n + 1.0));
        for (int it = 0; it < 100; ++it) {
            double pn, pn1;
            jacobi(z, &pn, &pn1);
            const double dz = pn / deriv(z, pn, pn1);
            z -= dz;
            if (std::fabs(dz) < 1e-16 * std::max(1.0, std::fabs(z))) break;
        }
        double pn, pn1;
        jacobi(z, &pn, &pn1);
        const double d = deriv(z, pn, pn1);
        x[n - k] = z;                       // k = 1 is the largest zero
        w[n - k] = 4.0 / ((1.0 - z * z) * d * d);
    }
}

double es_kernel(double z, double beta) {
    if (!(std::fabs(z) < 1.0)) return 0.0;
    return std::exp(beta * (std::sqrt(1.0 - z * z) - 1.0));
}

double es_transform(double omega, double beta) {
    // phi is even: 2 int_0^1 phi(z) cos(omega z) dz by a 512-point Gauss rule on
    // [0, 1].  The integrand is analytic inside the interval; the square-root
    // branch points sit at z = +-1 where phi is e^{-beta}, far below rounding.
    static thread_local std::vector<double> gx, gw;
    const int nq = 512;
    if (gx.empty()) {
        gx.resize(nq);
        gw.resize(nq);
        gauss_legendre(nq, gx.data(), gw.data());
    }
    double s = 0.0;
    for (int i = 0; i < nq; ++i) {
        double z = 0.5 * (gx[i] + 1.0);
        s += 0.5 * gw[i] * es_kernel(z, beta) * std::cos(omega * z);
    }
    return 2.0 * s;
}

void unit_root(long long m, long long n, double* re, double* im) {
    // angle 2 pi r / n with r = m mod n, written as octant * (pi/4) + frac * (pi/4)
    // so that sin and cos only see arguments in [0, pi/4]
    const long long r = ((m % n) + n) % n;
    const long long e8 = 8 * r;
    const long long oct = e8 / n;
    const double frac = static_cast<double>(e8 - oct * n) / static_cast<double>(n);
    const double th = frac * (kPi / 4.0);
    const double c = std::cos(th), s = std::sin(th);
    const double cq = std::cos(kPi / 4.0 - th), sq = std::sin(kPi / 4.0 - th);
    double cr, sr;
    switch (oct) {
        case 0: cr = c; sr = s; break;
        case 1: cr = sq; sr = cq; break;
        case 2: cr = -s; sr = c; break;
        case 3: cr = -cq; sr = sq; break;
        case 4: cr = -c; sr = -s; break;
        case 5: cr = -sq; sr = -cq; break;
        case 6: cr = s; sr = -c; break;
        default: cr = cq; sr = -sq; break;
    }
    *re = cr;
    *im = -sr;
}

void round_unit_pairs(const std::vector<double>& in, std::vector<float>* out) {
    out->resize(in.size());
    for (size_t i = 0; i + 1 < in.size(); i += 2) {
        const double re = in[i], im = in[i + 1];
        const float r0 = static_cast<float>(re), i0 = static_cast<float>(im);
        const float rc[3] = {std::nextafter(r0, -2.0f), r0, std::nextafter(r0, 2.0f)};
        const float ic[3] = {std::nextafter(i0, -2.0f), i0, std::nextafter(i0, 2.0f)};
        float br = r0, bi = i0;
        double bm = std::fabs(static_cast<double>(r0) * r0 + static_cast<double>(i0) * i0 - 1.0);
        double bd = 0.0;
        for (float a : rc) {
            for (float b : ic) {
                const double m = std::fabs(static_cast<double>(a) * a + static_cast<double>(b) * b - 1.0);
                const double d = std::fabs(a - re) + std::fabs(b - im);
                if (m < bm || (m == bm && d < bd)) {
                    bm = m;
                    bd = d;
                    br = a;
                    bi = b;
                }
            }
        }
        (*out)[i] = br;
        (*out)[i + 1] = bi;
    }
}

void fft_stage_twiddles(int log, std::vector<double>* out) {
    const int s16 = log / 4, rem = log % 4, nst = s16 + (rem ? 1 : 0);
    const long long f = 1LL << log;
    out->clear();
    long long p = 16;                       // span of stage 1
    for (int s = 1; s < nst; ++s) {
        const int r = (s < s16) ? 16 : (1 << rem);
        const long long step = f / (p * r);  // W_{pR}^{tk} = W_F^{t k step}
        for (int t = 1; t < r; ++t) {
            for (long long k = 0; k < p; ++k) {
                double re, im;
                unit_root(t * k * step, f, &re, &im);
                out->push_back(re);
                out->push_back(im);
            }
        }
        p *= r;
    }
}

phi_status derive(const phi_params* p, HostPlan* hp, std::string* err) {
    if (!p || !hp) { *err = "NULL argument"; return PHI_ERR_INVALID_ARG; }
    if (p->nx != p->ny) { *err = "nx != ny: only square grids are implemented"; return PHI_ERR_UNSUPPORTED; }
    if (!(p->hx > 0.0) || !(p->hy > 0.0) || !std::isfinite(p->hx) || !std::isfinite(p->hy)) {
        *err = "spacing must be positive and finite"; return PHI_ERR_INVALID_ARG;
    }
    if (p->hx != p->hy) { *err = "hx != hy: only equal spacings are implemented"; return PHI_ERR_UNSUPPORTED; }
    const int n = p->nx;
    if (n < 2 || n % 2 != 0) { *err = fmt("grid side must be even and >= 2 (got %g)", n); return PHI_ERR_INVALID_ARG; }
    if (n < kMinGrid) { *err = fmt("grid side %g: grids from 8 points per side are implemented", n); return PHI_ERR_UNSUPPORTED; }
    if (p->n_r < 1 || p->n_r > 1024) { *err = "n_r must be in [1, 1024]"; return PHI_ERR_INVALID_ARG; }
    if (p->n_theta < 2 || p->n_theta > 4096 || p->n_theta % 2 != 0) {
        *err = "n_theta must be even and in [2, 4096]"; return PHI_ERR_INVALID_ARG;
    }
    const int kappa = (p->pad == 0) ? 2 : p->pad;
    if (kappa < 2) { *err = "padding factor kappa must be >= 2"; return PHI_ERR_INVALID_ARG; }
    if (kappa > kMaxPad) { *err = fmt("padding factor kappa %g: at most %g is implemented", kappa, kMaxPad); return PHI_ERR_UNSUPPORTED; }
    // the padded box (Sec. 2.1) is the smallest power-of-two side >= kappa N:
    // a box of factor F / N >= kappa, on which both FFT directions are radix-16 /
    // radix-2^r register transforms
    long long fine = 1LL << kMinLogFine;
    while (fine < static_cast<long long>(kappa) * n) fine *= 2;
    if (fine > (1LL << kMaxLogFine)) {
        *err = fmt("grid side %g with kappa %g needs a padded side above 8192", n, kappa);
        return PHI_ERR_UNSUPPORTED;
    }
    if (p->dtype != PHI_F64 && p->dtype != PHI_F32) { *err = "unknown dtype"; return PHI_ERR_INVALID_ARG; }
    if (!(p->tol > 0.0) || !std::isfinite(p->tol)) { *err = "tol must be positive"; return PHI_ERR_INVALID_ARG; }
    const double tol_min = (p->dtype == PHI_F32) ? 1e-7 : 1e-15;
    if (p->tol < tol_min * (1.0 - 1e-9) || p->tol > 0.1) {
        *err = fmt("tol %g outside [%g, 0.1] for this dtype", p->tol, tol_min);
        return PHI_ERR_TOL_UNREACHABLE;
    }
    if ((p->flags & ~(PHI_COMPONENT_Y | PHI_COMPONENT_XY | PHI_COMPONENT_COULOMB | PHI_PARTITION_GAUSS |
                      PHI_AUTOTUNE | PHI_RADIAL_JACOBI | PHI_KERNEL_GAUSSIAN | PHI_TWO_STREAMS)) != 0) {
        *err = "unknown flag bits"; return PHI_ERR_INVALID_ARG;
    }
    {
        const int comps = ((p->flags & PHI_COMPONENT_Y) ? 1 : 0) + ((p->flags & PHI_COMPONENT_XY) ? 1 : 0) +
                          ((p->flags & PHI_COMPONENT_COULOMB) ? 1 : 0);
        if (comps > 1) {
            *err = "PHI_COMPONENT_Y, PHI_COMPONENT_XY and PHI_COMPONENT_COULOMB exclude each other";
            return PHI_ERR_INVALID_ARG;
        }
    }
    if ((p->flags & PHI_PARTITION_GAUSS) && !(p->flags & PHI_COMPONENT_COULOMB)) {
        *err = "PHI_PARTITION_GAUSS applies to PHI_COMPONENT_COULOMB only (the Gaussian partition is the "
               "default of the other multipliers)";
        return PHI_ERR_INVALID_ARG;
    }
    if ((p->flags & PHI_COMPONENT_COULOMB) && (p->flags & PHI_RADIAL_JACOBI)) {
        *err = "the Coulomb multiplier cancels the polar Jacobian: its radial rule is Gauss-Legendre";
        return PHI_ERR_INVALID_ARG;
    }
    if (p->bin != 0 && p->bin != 4 && p->bin != 8 && p->bin != kMaxBinSize) {
        *err = "bin must be 0, 4, 8 or 16"; return PHI_ERR_INVALID_ARG;
    }
    if (p->sub_nodes != 0 && (p->sub_nodes < 8 || p->sub_nodes > kMaxNodesPerSub)) {
        *err = "sub_nodes must be 0 or in [8, 64]"; return PHI_ERR_INVALID_ARG;
    }

    hp->n = n;
    hp->n_fine = static_cast<int>(fine);
    hp->log_fine = ilog2(hp->n_fine);
    hp->log_n = is_pow2(n) ? ilog2(n) : -1;
    hp->kappa = kappa;
    hp->n_r = p->n_r;
    hp->n_theta = p->n_theta;
    hp->n_nodes = p->n_r * p->n_theta;
    hp->component = (p->flags & PHI_COMPONENT_COULOMB) ? 3 : (p->flags & PHI_COMPONENT_XY) ? 2
                    : (p->flags & PHI_COMPONENT_Y) ? 1 : 0;
    hp->partition_erfc = ((p->flags & PHI_COMPONENT_COULOMB) && !(p->flags & PHI_PARTITION_GAUSS)) ? 1 : 0;
    hp->radial_jacobi = (p->flags & PHI_RADIAL_JACOBI) ? 1 : 0;
    hp->gaussian_kernel = (p->flags & PHI_KERNEL_GAUSSIAN) ? 1 : 0;
    hp->two_streams = (p->flags & PHI_TWO_STREAMS) ? 1 : 0;
    hp->dtype = p->dtype;
    hp->h = p->hx;
    hp->half_width = 0.5 * n * p->hx;
    // the padding factor of the box actually used, F / N, sets the default sigma:
    // (kappa - 1) L = (F - N) h / 2
    const double kappa_eff = static_cast<double>(hp->n_fine) / n;
    hp->sigma = (p->sigma > 0.0) ? p->sigma
                                 : std::sqrt(kLogInvEpsSplit) / (2.0 * kPi * (kappa_eff - 1.0) * hp->half_width);
    hp->cutoff = (p->cutoff > 0.0) ? p->cutoff : std::sqrt(kLogInvEpsSplit) * hp->sigma;
    if (!std::isfinite(hp->sigma) || !std::isfinite(hp->cutoff)) { *err = "sigma / cutoff not finite"; return PHI_ERR_INVALID_ARG; }

    // Kernel width from the requested accuracy (published rule for the
    // exponential-of-semicircle kernel at oversampling 2: w = ceil(log10 1/tol) + 1,
    // beta = 2.30 w).
    int w = static_cast<int>(std::ceil(std::log10(1.0 / p->tol) - 1e-9)) + 1;
    w = std::max(2, std::min(kMaxEsWidth, w));
    hp->beta = 2.30 * w;
    if (hp->gaussian_kernel) {
        // Greengard-Lee gridding at oversampling R = 2: spreading half-width M
        // cells with aliasing error about e^{-pi M (R-1)/(R-1/2)} = e^{-2 pi M/3},
        // so M = ceil(1.5 ln(1/tol) / pi); in cell units the Gaussian is
        // exp(-pi (R - 1/2)/(R M) t^2) = exp(-(3 pi/(4 M)) t^2).
        const int m = std::max(2, static_cast<int>(std::ceil(1.5 * std::log(1.0 / p->tol) / kPi - 1e-9)));
        w = 2 * m;
        hp->beta = 0.75 * kPi / m;
    }
    hp->width = w;

    // Window of fine-grid cells touched by the kernel taps of the nodes.  The
    // nodes lie in |k| <= c, i.e. within n_fine h c cells of the origin.
    const double umax = hp->n_fine * hp->h * hp->cutoff;
    int lmax = static_cast<int>(std::ceil(umax + 0.5 * w)) + 1;
    int q = 16;
    while (q / 2 < lmax + 1 && q < hp->n_fine) q *= 2;
    if (q > hp->n_fine) q = hp->n_fine;
    hp->patch = q;
    hp->patch_lo = -q / 2;
    // bins never exceed the window (which is a power of two >= 16)
    hp->bin = std::min(p->bin > 0 ? p->bin : kBinSize, q);
    if (w > kMaxKernelWidth || hp->bin + w - 1 > kMaxTile) {
        *err = fmt("kernel width %g with bin side %g exceeds the spread tile (bin + w - 1 <= 31)", w, hp->bin);
        return PHI_ERR_UNSUPPORTED;
    }
    hp->sub_nodes = p->sub_nodes > 0 ? p->sub_nodes : kMaxNodesPerSub;
    return PHI_OK;
}

void polar_nodes(const HostPlan& hp, std::vector<double>* kx, std::vector<double>* ky,
                 std::vector<double>* q) {
    // Sec. 2.1, eq. 12: radial Gauss rule on [0, c] (r_i = c (1 + x_i)/2, weight
    // (c/2) w_i r_i with the polar Jacobian folded in), azimuthal trapezoid
    // theta_j = 2 pi j / N_theta with weight 2 pi / N_theta;
    // q_ij = -w_r w_theta cos^2(theta_j) exp(-r_i^2 / sigma^2)   (sin^2 for the y component,
    // cos sin for the mixed one: the multiplier's value on the unit circle).
    // Coulomb (1/|k|): the multiplier cancels the Jacobian, q_ij = (c/2) w_i w_theta p(r_i)
    // with p = erfc(r/sigma) or the Gaussian (Gauss-Legendre only).
    std::vector<double> gx(hp.n_r), gw(hp.n_r);
    if (hp.radial_jacobi) gauss_jacobi01(hp.n_r, gx.data(), gw.data());
    else gauss_legendre(hp.n_r, gx.data(), gw.data());
    const int m = hp.n_r * hp.n_theta;
    kx->resize(m);
    ky->resize(m);
    q->resize(m);
    const double wt = 2.0 * kPi / hp.n_theta;
    for (int i = 0; i < hp.n_r; ++i) {
        const double r = 0.5 * hp.cutoff * (1.0 + gx[i]);
        // Gauss-Jacobi(0, 1) carries the Jacobian r as its weight (1 + x);
        // Gauss-Legendre gets it folded into the weight
        const double wr = hp.radial_jacobi ? 0.25 * hp.cutoff * hp.cutoff * gw[i] : 0.5 * hp.cutoff * gw[i] * r;
        const double damp = std::exp(-(r * r) / (hp.sigma * hp.sigma));
        if (hp.component == 3) {
            const double part = hp.partition_erfc ? std::erfc(r / hp.sigma) : damp;
            const double w0 = 0.5 * hp.cutoff * gw[i];
            for (int j = 0; j < hp.n_theta; ++j) {
                const double th = kPi * (2.0 * j / hp.n_theta);
                const int idx = i * hp.n_theta + j;
                (*kx)[idx] = r * std::cos(th);
                (*ky)[idx] = r * std::sin(th);
                (*q)[idx] = w0 * wt * part;
            }
            continue;
        }
        for (int j = 0; j < hp.n_theta; ++j) {
            // angle 2 pi j / N_theta evaluated as pi * (2j / N_theta) in [0, 2 pi)
            const double th = kPi * (2.0 * j / hp.n_theta);
            const double cs = std::cos(th), sn = std::sin(th);
            const double ang = hp.component == 2 ? cs * sn : hp.component == 1 ? sn * sn : cs * cs;
            const int idx = i * hp.n_theta + j;
            (*kx)[idx] = r * cs;
            (*ky)[idx] = r * sn;
            (*q)[idx] = -wr * wt * ang * damp;
        }
    }
}

phi_status build_host_plan(const phi_params* p, HostPlan* hp, std::string* err) {
    phi_status st = derive(p, hp, err);
    if (st != PHI_OK) return st;
    const int n = hp->n, nf = hp->n_fine, w = hp->width;
    const double half_w = 0.5 * w;

    // ---- polar nodes, first kernel tap, sort by first-tap cell, taps ------------
    std::vector<double> kx, ky, q;
    polar_nodes(*hp, &kx, &ky, &q);
    const int m = hp->n_nodes;
    const int q_side = hp->patch, lo = hp->patch_lo;
    std::vector<double> ux(m), uy(m);
    std::vector<int> cx(m), cy(m);
    for (int j = 0; j < m; ++j) {
        // t_j / Delta with t_j = 2 pi h k_j, Delta = 2 pi / n_fine: node position in cells
        ux[j] = nf * hp->h * kx[j];
        uy[j] = nf * hp->h * ky[j];
        // first tap l0 = ceil(u - w/2), as a window cell (wrapped when the window is
        // the whole periodic fine grid)
        const int ax = posmod(static_cast<int>(std::ceil(ux[j] - half_w)) - lo, nf);
        const int ay = posmod(static_cast<int>(std::ceil(uy[j] - half_w)) - lo, nf);
        if (q_side < nf && (ax + w > q_side || ay + w > q_side)) {
            *err = "internal: node taps outside the fine-grid window";
            return PHI_ERR_INTERNAL;
        }
        cx[j] = ax;
        cy[j] = ay;
    }
    // bins of bin x bin window cells; nodes sorted by the bin of their first tap
    const int bin = hp->bin;
    const int nb = q_side / bin;        // the window side is a power of two >= 16
    const bool whole = (q_side == nf);
    std::vector<int> key(m);
    for (int j = 0; j < m; ++j) key[j] = (cy[j] / bin) * nb + cx[j] / bin;
    std::vector<int> order(m);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key[a] < key[b]; });
    hp->kx.resize(m); hp->ky.resize(m); hp->q.resize(m);
    hp->cell.resize(2 * static_cast<size_t>(m));
    hp->taps.resize(static_cast<size_t>(m) * 2 * w);
    for (int i = 0; i < m; ++i) {
        const int j = order[i];
        hp->kx[i] = kx[j]; hp->ky[i] = ky[j]; hp->q[i] = q[j];
        hp->cell[2 * i] = cx[j];
        hp->cell[2 * i + 1] = cy[j];
        // psi(u - l) for the w taps l = l0 .. l0 + w - 1
        const double l0x = std::ceil(ux[j] - half_w), l0y = std::ceil(uy[j] - half_w);
        for (int t = 0; t < w; ++t) {
            const double dx = ux[j] - (l0x + t), dy = uy[j] - (l0y + t);
            hp->taps[(static_cast<size_t>(i) * 2 + 0) * w + t] =
                hp->gaussian_kernel ? std::exp(-hp->beta * dx * dx) : es_kernel(dx / half_w, hp->beta);
            hp->taps[(static_cast<size_t>(i) * 2 + 1) * w + t] =
                hp->gaussian_kernel ? std::exp(-hp->beta * dy * dy) : es_kernel(dy / half_w, hp->beta);
        }
    }
    // subproblems: runs of at most sub_nodes nodes of one bin
    hp->sub.clear();
    int max_bin = 0;
    for (int i = 0; i < m;) {
        const int k = key[order[i]];
        int e = i;
        while (e < m && key[order[e]] == k) ++e;
        max_bin = std::max(max_bin, e - i);
        for (int s0 = i; s0 < e; s0 += hp->sub_nodes) {
            hp->sub.push_back(k % nb);
            hp->sub.push_back(k / nb);
            hp->sub.push_back(s0);
            hp->sub.push_back(std::min(hp->sub_nodes, e - s0));
        }
        i = e;
    }
    hp->nb = nb;
    hp->tile = bin + w - 1;
    hp->n_sub = static_cast<int>(hp->sub.size() / 4);
    hp->max_cell_nodes = max_bin;
    // window cell <- tile entries: every tile cell inside the box its nodes' taps
    // can reach, mapped to its window cell (wrapped when the window is periodic)
    const int E = hp->tile;
    std::vector<std::pair<int, int>> pairs;   // (window cell, flat tile index)
    for (int sidx = 0; sidx < hp->n_sub; ++sidx) {
        const int bx = hp->sub[4 * sidx], by = hp->sub[4 * sidx + 1];
        const int first = hp->sub[4 * sidx + 2], count = hp->sub[4 * sidx + 3];
        int ox0 = bin, ox1 = -1, oy0 = bin, oy1 = -1;
        for (int i = first; i < first + count; ++i) {
            ox0 = std::min(ox0, hp->cell[2 * i] - bx * bin);
            ox1 = std::max(ox1, hp->cell[2 * i] - bx * bin);
            oy0 = std::min(oy0, hp->cell[2 * i + 1] - by * bin);
            oy1 = std::max(oy1, hp->cell[2 * i + 1] - by * bin);
        }
        for (int cb = oy0; cb <= oy1 + w - 1; ++cb) {
            for (int ca = ox0; ca <= ox1 + w - 1; ++ca) {
                int wx = bx * bin + ca, wy = by * bin + cb;
                if (whole) {
                    wx %= q_side;
                    wy %= q_side;
                } else if (wx >= q_side || wy >= q_side) {
                    continue;
                }
                pairs.emplace_back(wx * q_side + wy, sidx * E * E + cb * E + ca);
            }
        }
    }
    std::stable_sort(pairs.begin(), pairs.end(),
                     [](const std::pair<int, int>& a, const std::pair<int, int>& b) { return a.first < b.first; });
    hp->contrib_start.assign(static_cast<size_t>(q_side) * q_side + 1, 0);
    hp->contrib.resize(pairs.size());
    for (size_t k = 0; k < pairs.size(); ++k) {
        hp->contrib_start[pairs[k].first + 1] += 1;
        hp->contrib[k] = pairs[k].second;
    }
    int max_gather = 0;
    for (size_t c = 1; c < hp->contrib_start.size(); ++c) {
        max_gather = std::max(max_gather, hp->contrib_start[c]);
        hp->contrib_start[c] += hp->contrib_start[c - 1];
    }
    hp->max_gather = max_gather;

    // ---- deconvolution factors 2 pi / (n_fine psi_hat(n')) ---------------------
    // psi(x) = phi(x / a) with a = (w/2) Delta the kernel half-width in radians:
    // psi_hat(k) = a int_{-1}^{1} phi(z) cos(k a z) dz.
    hp->deconv.resize(n);
    const double a_rad = half_w * 2.0 * kPi / nf;
    for (int i = 0; i < n; ++i) {
        const int np = i - n / 2;
        double ph;
        if (hp->gaussian_kernel) {
            // psi(x) = exp(-x^2 / (4 tau)) in radians, tau = Delta^2 / (4 beta), has
            // psi_hat(k) = sqrt(4 pi tau) e^{-k^2 tau} (the truncation at |t| = w/2
            // is part of the kernel's error)
            const double delta = 2.0 * kPi / nf;
            const double tau = delta * delta / (4.0 * hp->beta);
            ph = std::sqrt(4.0 * kPi * tau) * std::exp(-static_cast<double>(np) * np * tau);
        } else {
            ph = a_rad * es_transform(np * a_rad, hp->beta);
        }
        hp->deconv[i] = 2.0 * kPi / (nf * ph);
    }

    // ---- I1 multiplier tables --------------------------------------------------
    const double s2 = hp->sigma * hp->sigma;
    hp->gx.resize(2 * (nf / 2 + 1));
    for (int m1 = 0; m1 <= nf / 2; ++m1) {
        const double k = m1 / (nf * hp->h);
        const double a = k * k / s2;
        hp->gx[2 * m1] = a;
        hp->gx[2 * m1 + 1] = -std::expm1(-a);
    }
    hp->gy.resize(2 * nf);
    for (int m2 = 0; m2 < nf; ++m2) {
        const int ms = (m2 < nf / 2) ? m2 : m2 - nf;
        const double k = ms / (nf * hp->h);
        const double b = k * k / s2;
        hp->gy[2 * m2] = b;
        hp->gy[2 * m2 + 1] = -std::expm1(-b);
    }

    // ---- register-FFT stage twiddles --------------------------------------------
    const int lg = hp->log_fine;
    fft_stage_twiddles(lg, &hp->twr);
    hp->twn.clear();
    if (hp->log_n >= kMinLogFine) fft_stage_twiddles(hp->log_n, &hp->twn);
    return PHI_OK;
}

}  // namespace phi
