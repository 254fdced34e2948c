#include "host_math.hpp"

#include <cmath>
#include <stdexcept>

namespace celes {

static long double fact(int n) {
    static long double tab[64];
    static bool init = false;
    if (!init) {
        tab[0] = 1.0L;
        for (int i = 1; i < 64; ++i) tab[i] = tab[i - 1] * (long double)i;
        init = true;
    }
    if (n < 0 || n >= 64) throw std::runtime_error("factorial argument out of range");
    return tab[n];
}

double wigner3j(int j1, int j2, int j3, int m1, int m2, int m3) {
    if (m1 + m2 + m3 != 0) return 0.0;
    if (j3 < std::abs(j1 - j2) || j3 > j1 + j2) return 0.0;
    if (std::abs(m1) > j1 || std::abs(m2) > j2 || std::abs(m3) > j3) return 0.0;
    // Racah: sqrt(Delta) sqrt(prod (j+-m)!) sum_k (-1)^k / (...)
    long double delta = fact(j1 + j2 - j3) * fact(j1 - j2 + j3) * fact(-j1 + j2 + j3) /
                        fact(j1 + j2 + j3 + 1);
    long double pre = std::sqrt(delta * fact(j1 + m1) * fact(j1 - m1) * fact(j2 + m2) *
                                fact(j2 - m2) * fact(j3 + m3) * fact(j3 - m3));
    int kmin = std::max(0, std::max(j2 - j3 - m1, j1 - j3 + m2));
    int kmax = std::min(j1 + j2 - j3, std::min(j1 - m1, j2 + m2));
    long double s = 0.0L;
    for (int k = kmin; k <= kmax; ++k) {
        long double den = fact(k) * fact(j3 - j2 + k + m1) * fact(j3 - j1 + k - m2) *
                          fact(j1 + j2 - j3 - k) * fact(j1 - k - m1) * fact(j2 - k + m2);
        s += ((k & 1) ? -1.0L : 1.0L) / den;
    }
    int e = j1 - j2 - m3;
    long double sign = (((e % 2) + 2) % 2) ? -1.0L : 1.0L;
    return (double)(sign * pre * s);
}

// i^e for integer e, returned as (re, im) with mathematical modulo
static cplx ipow(int e) {
    switch (((e % 4) + 4) % 4) {
        case 0: return {1, 0};
        case 1: return {0, 1};
        case 2: return {-1, 0};
        default: return {0, -1};
    }
}

double a5_coef(int l, int m, int lp, int mp, int p) {
    if (p < std::abs(l - lp) || p > l + lp || ((l + lp + p) & 1)) return 0.0;
    double w1 = wigner3j(l, lp, p, m, -mp, mp - m);
    double w2 = wigner3j(l, lp, p, 0, 0, 0);
    if (w1 == 0.0 || w2 == 0.0) return 0.0;
    double c = (double)(l * (l + 1) + lp * (lp + 1) - p * (p + 1));
    double v = c * std::sqrt(2.0 * p + 1.0) *
               std::sqrt((2.0 * l + 1.0) * (2.0 * lp + 1.0) / (2.0 * l * (l + 1) * lp * (lp + 1))) *
               w1 * w2;
    if ((m - mp) & 1) v = -v;
    cplx ph = ipow(std::abs(m - mp) - std::abs(m) - std::abs(mp) + lp - l + p);
    return ph.real() * v;  // exponent is even here: ph is +-1
}

double b5im_coef(int l, int m, int lp, int mp, int p) {
    if (p < std::abs(l - lp) + 1 || p > l + lp || !((l + lp + p) & 1)) return 0.0;
    double w1 = wigner3j(l, lp, p, m, -mp, mp - m);
    double w2 = wigner3j(l, lp, p - 1, 0, 0, 0);
    if (w1 == 0.0 || w2 == 0.0) return 0.0;
    double rad = (double)(l + lp + 1 + p) * (double)(l + lp + 1 - p) * (double)(p + l - lp) *
                 (double)(p - l + lp) * (2.0 * p + 1.0);
    if (rad <= 0.0) return 0.0;
    double v = std::sqrt(rad) *
               std::sqrt((2.0 * lp + 1.0) * (2.0 * l + 1.0) / (2.0 * l * (l + 1) * lp * (lp + 1))) *
               w1 * w2;
    if ((m - mp) & 1) v = -v;
    cplx ph = ipow(std::abs(m - mp) - std::abs(m) - std::abs(mp) + lp - l + p);
    return ph.imag() * v;  // exponent is odd here: ph is +-i
}

void legendre_table(int lmax, double ct, double st, double* out) {
    const int W = lmax + 1;
    for (int i = 0; i < W * W; ++i) out[i] = 0.0;
    double pmm = 1.0 / std::sqrt(2.0);
    for (int m = 0; m <= lmax; ++m) {
        if (m > 0) pmm *= std::sqrt((2.0 * m + 1.0) / (2.0 * m)) * st;
        out[m * W + m] = pmm;
        if (m + 1 <= lmax) out[(m + 1) * W + m] = std::sqrt(2.0 * m + 3.0) * ct * pmm;
        for (int l = m + 2; l <= lmax; ++l) {
            double a = std::sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
            double b = std::sqrt((2.0 * l + 1.0) * ((l - 1.0) * (l - 1.0) - (double)m * m) /
                                 ((2.0 * l - 3.0) * ((double)l * l - (double)m * m)));
            out[l * W + m] = a * ct * out[(l - 1) * W + m] - b * out[(l - 2) * W + m];
        }
    }
}

void pi_tau(int l, int m, double theta, double* pi, double* tau) {
    // P_l^m(cos t) = sin^m(t) R_l^m(cos t) with R a polynomial; evaluate R and
    // its derivative by the same three-term recursion applied to R itself.
    m = std::abs(m);
    double ct = std::cos(theta), st = std::fabs(std::sin(theta));
    // R_m^m = N_mm (2m-1)!!, recursion in l identical to P's (the sin^m factor is common)
    std::vector<double> R(l + 2, 0.0), dR(l + 2, 0.0);
    double rmm = 1.0 / std::sqrt(2.0);
    for (int k = 1; k <= m; ++k) rmm *= std::sqrt((2.0 * k + 1.0) / (2.0 * k));
    R[m] = rmm;
    dR[m] = 0.0;
    if (m + 1 <= l + 1) {
        R[m + 1] = std::sqrt(2.0 * m + 3.0) * ct * rmm;
        dR[m + 1] = std::sqrt(2.0 * m + 3.0) * rmm;
    }
    for (int q = m + 2; q <= l + 1; ++q) {
        double a = std::sqrt((4.0 * q * q - 1.0) / ((double)q * q - (double)m * m));
        double b = std::sqrt((2.0 * q + 1.0) * ((q - 1.0) * (q - 1.0) - (double)m * m) /
                             ((2.0 * q - 3.0) * ((double)q * q - (double)m * m)));
        R[q] = a * ct * R[q - 1] - b * R[q - 2];
        dR[q] = a * (R[q - 1] + ct * dR[q - 1]) - b * dR[q - 2];
    }
    double r = R[l], dr = dR[l];
    if (m == 0) {
        *pi = 0.0;  // only ever multiplied by m = 0
        *tau = -st * dr;
    } else {
        double sm1 = std::pow(st, m - 1);
        *pi = sm1 * r;
        *tau = m * sm1 * ct * r - sm1 * st * st * dr;
    }
}

void sph_hankel(int pmax, double x, cplx* h, cplx* dh) {
    for (int p = 0; p <= pmax; ++p)
        h[p] = cplx(std::sph_bessel((unsigned)p, x), std::sph_neumann((unsigned)p, x));
    dh[0] = -h[1 <= pmax ? 1 : 0];
    if (pmax == 0) dh[0] = cplx(std::sph_bessel(0u, x), std::sph_neumann(0u, x));
    if (pmax >= 1) dh[0] = -h[1];
    else {
        cplx h1(std::sph_bessel(1u, x), std::sph_neumann(1u, x));
        dh[0] = -h1;
    }
    for (int p = 1; p <= pmax; ++p) dh[p] = h[p - 1] - (double)(p + 1) / x * h[p];
}

void mie_Q(int L, double x, cplx m, cplx* Q1, cplx* Q2) {
    // Riccati-Bessel form: psi_l(z) = z j_l(z), xi_l(x) = x h_l(x).  The
    // logarithmic derivative D_l(mx) = psi_l'(mx)/psi_l(mx) comes from the
    // downward recurrence D_{l-1} = l/z - 1/(D_l + l/z).  With
    // Q_{1l} = -b_l, Q_{2l} = -a_l (Appendix B in Riccati form):
    //   b_l = [(m D_l + l/x) psi_l(x) - psi_{l-1}(x)] / [(m D_l + l/x) xi_l - xi_{l-1}]
    //   a_l = [(D_l/m + l/x) psi_l(x) - psi_{l-1}(x)] / [(D_l/m + l/x) xi_l - xi_{l-1}]
    cplx mx = m * x;
    int nst = std::max(L, (int)std::abs(mx)) + 20;
    std::vector<cplx> D(nst + 1, cplx(0, 0));
    for (int n = nst; n >= 1; --n) D[n - 1] = (double)n / mx - 1.0 / (D[n] + (double)n / mx);
    double psi_m1 = std::cos(x), psi0 = std::sin(x);   // psi_{-1}, psi_0
    double y_m1 = std::sin(x), y0 = -std::cos(x);      // x y_{-1}, x y_0
    double psi_prev = psi0, psi_pp = psi_m1;
    double yy_prev = y0, yy_pp = y_m1;
    for (int l = 1; l <= L; ++l) {
        double psi = (2.0 * l - 1.0) / x * psi_prev - psi_pp;
        double yy = (2.0 * l - 1.0) / x * yy_prev - yy_pp;
        cplx xi(psi, yy), xi_prev(psi_prev, yy_prev);
        cplx tb = m * D[l] + (double)l / x;
        cplx ta = D[l] / m + (double)l / x;
        cplx b = (tb * psi - psi_prev) / (tb * xi - xi_prev);
        cplx a = (ta * psi - psi_prev) / (ta * xi - xi_prev);
        Q1[l - 1] = -b;
        Q2[l - 1] = -a;
        psi_pp = psi_prev;
        psi_prev = psi;
        yy_pp = yy_prev;
        yy_prev = yy;
    }
}

void gauss_legendre(int n, double* x, double* w) {
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            double pn = (n == 1) ? z : p1, pnm1 = (n == 1) ? 1.0 : p0;
            double dp = n * (z * pn - pnm1) / (z * z - 1.0);
            double dz = pn / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) {
                p0 = 1.0; p1 = z;
                for (int k = 2; k <= n; ++k) {
                    double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                    p0 = p1; p1 = p2;
                }
                pn = (n == 1) ? z : p1; pnm1 = (n == 1) ? 1.0 : p0;
                dp = n * (z * pn - pnm1) / (z * z - 1.0);
                break;
            }
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1; p1 = p2;
        }
        double pn = (n == 1) ? z : p1, pnm1 = (n == 1) ? 1.0 : p0;
        double dp = n * (z * pn - pnm1) / (z * z - 1.0);
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

cplx b_dagger(int tau, int l, int m, int j, double beta) {
    double pi, ta;
    pi_tau(l, std::abs(m), beta, &pi, &ta);
    // -1/(-i)^{l+1} = -i^{l+1}
    cplx pref = -ipow(l + 1) / std::sqrt(2.0 * l * (l + 1));
    cplx pol = (j == 1) ? cplx(0, -1) : cplx(1, 0);
    double ang = (tau == j) ? ta : m * pi;
    return pref * pol * ang;
}

}  // namespace celes
