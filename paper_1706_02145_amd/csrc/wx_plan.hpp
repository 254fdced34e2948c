// Compile-time enumeration of the translation-block terms evaluated by the
// coupling kernels.  The host builds its coefficient table by walking exactly
// the same loops, so the kernel can address the table with constants.
//
// Notation (Section 2.2 and Appendix A.2 of the paper): the receiving
// multipole is (tau, l, m), the source multipole (tau', l', m'); the block
// entry is W^{ii'}_{nn'} = A_{n'n}(r_i - r_i') with
//   A_{m'l', ml}(d) = e^{i(m'-m)phi} sum_p a5(l',m'|l,m|p) h_p(kd) P_p^{|m'-m|}(cos theta)
// and B likewise with b5 (= i * b5im).  Outputs are grouped in passes by
// |m| = M0; a pass handles m = +M0 and its mirror m = -M0, which reuse the
// same reduced coefficients (a5 is even and b5 odd under m, m' -> -m, -m').
// Within a pass the loop order is
//   mu = |m' - M0| (0..min(2L, L+M0)), sign of (m' - M0), l', l,
//   then the p terms of A and of B.
#pragma once

namespace celes {
namespace plan {

constexpr int iabs(int a) { return a < 0 ? -a : a; }
constexpr int imax(int a, int b) { return a > b ? a : b; }
constexpr int imin(int a, int b) { return a < b ? a : b; }

constexpr int mu_max(int L, int M0) { return imin(2 * L, L + M0); }

// p range of the A sum: |l-l'| <= p <= l+l', l+l'+p even, p >= mu
constexpr int pa_lo(int l, int lp, int mu) {
    int p = imax(iabs(l - lp), mu);
    return ((l + lp + p) & 1) ? p + 1 : p;
}
constexpr int pa_hi(int l, int lp) { return l + lp; }
constexpr int na(int l, int lp, int mu) {
    return pa_lo(l, lp, mu) <= pa_hi(l, lp) ? (pa_hi(l, lp) - pa_lo(l, lp, mu)) / 2 + 1 : 0;
}
// p range of the B sum: |l-l'|+1 <= p <= l+l'-1, l+l'+p odd, p >= mu
constexpr int pb_lo(int l, int lp, int mu) {
    int p = imax(iabs(l - lp) + 1, mu);
    return ((l + lp + p) & 1) ? p : p + 1;
}
constexpr int pb_hi(int l, int lp) { return l + lp - 1; }
constexpr int nb(int l, int lp, int mu) {
    return pb_lo(l, lp, mu) <= pb_hi(l, lp) ? (pb_hi(l, lp) - pb_lo(l, lp, mu)) / 2 + 1 : 0;
}

// is the (mu, sign) branch present in pass M0?  sign = +1 or -1; m' = M0 + sign*mu
constexpr bool branch(int L, int M0, int mu, int sgn) {
    if (sgn < 0 && mu == 0) return false;          // mu = 0 appears once
    if (M0 == 0 && sgn < 0) return false;          // for M0 = 0 the -mu source is the mirror
    int mp = M0 + sgn * mu;
    return iabs(mp) <= L;
}
constexpr int l_lo(int M0) { return M0 > 1 ? M0 : 1; }
constexpr int lp_lo(int mp) { return iabs(mp) > 1 ? iabs(mp) : 1; }

constexpr int pass_ncoef(int L, int M0) {
    int n = 0;
    for (int mu = 0; mu <= mu_max(L, M0); ++mu)
        for (int s = 0; s < 2; ++s) {
            int sgn = s == 0 ? 1 : -1;
            if (!branch(L, M0, mu, sgn)) continue;
            int mp = M0 + sgn * mu;
            for (int lp = lp_lo(mp); lp <= L; ++lp)
                for (int l = l_lo(M0); l <= L; ++l) n += na(l, lp, mu) + nb(l, lp, mu);
        }
    return n;
}
constexpr int pass_offset(int L, int M0) {
    int o = 0;
    for (int m = 0; m < M0; ++m) o += pass_ncoef(L, m);
    return o;
}
constexpr int total_ncoef(int L) { return pass_offset(L, L + 1); }

// entries (l, m | l', m') handled per pair in pass M0, counting mirror reuse
// once; used for flop accounting
constexpr int pass_entries(int L, int M0) {
    int n = 0;
    for (int mu = 0; mu <= mu_max(L, M0); ++mu)
        for (int s = 0; s < 2; ++s) {
            int sgn = s == 0 ? 1 : -1;
            if (!branch(L, M0, mu, sgn)) continue;
            int mp = M0 + sgn * mu;
            n += (L - lp_lo(mp) + 1) * (L - l_lo(M0) + 1);
        }
    return n;
}

// compile-time square root (Newton), for recursion constants
constexpr double csqrt(double x) {
    if (x <= 0.0) return 0.0;
    double r = x > 1.0 ? x : 1.0;
    for (int i = 0; i < 200; ++i) {
        double n = 0.5 * (r + x / r);
        if (n == r) break;
        r = n;
    }
    return r;
}
// normalized Legendre recursion constants (no Condon-Shortley phase)
//   P_m^m = sqrt((2m+1)/(2m)) sin(t) P_{m-1}^{m-1},  P_0^0 = 1/sqrt(2)
//   P_{m+1}^m = sqrt(2m+3) cos(t) P_m^m
//   P_p^m = a(p,m) cos(t) P_{p-1}^m - b(p,m) P_{p-2}^m
constexpr double leg_diag(int m) { return csqrt((2.0 * m + 1.0) / (2.0 * m)); }
constexpr double leg_sub(int m) { return csqrt(2.0 * m + 3.0); }
constexpr double leg_a(int p, int m) { return csqrt((4.0 * p * p - 1.0) / ((double)p * p - (double)m * m)); }
constexpr double leg_b(int p, int m) {
    return csqrt((2.0 * p + 1.0) * ((p - 1.0) * (p - 1.0) - (double)m * m) /
                 ((2.0 * p - 3.0) * ((double)p * p - (double)m * m)));
}

// compile-time Wigner-3j (Racah formula in double precision) and the a5 /
// b5 translation coefficients of Appendix A.2.  b5 is purely imaginary; cb5im
// returns its imaginary part.
constexpr double cfact(int n) {
    double r = 1.0;
    for (int i = 2; i <= n; ++i) r *= (double)i;
    return r;
}
constexpr double cw3j(int j1, int j2, int j3, int m1, int m2, int m3) {
    if (m1 + m2 + m3 != 0) return 0.0;
    if (j3 < iabs(j1 - j2) || j3 > j1 + j2) return 0.0;
    if (iabs(m1) > j1 || iabs(m2) > j2 || iabs(m3) > j3) return 0.0;
    double delta = cfact(j1 + j2 - j3) * cfact(j1 - j2 + j3) * cfact(-j1 + j2 + j3) / cfact(j1 + j2 + j3 + 1);
    double pre = csqrt(delta * cfact(j1 + m1) * cfact(j1 - m1) * cfact(j2 + m2) * cfact(j2 - m2) *
                       cfact(j3 + m3) * cfact(j3 - m3));
    int kmin = imax(0, imax(j2 - j3 - m1, j1 - j3 + m2));
    int kmax = imin(j1 + j2 - j3, imin(j1 - m1, j2 + m2));
    double s = 0.0;
    for (int k = kmin; k <= kmax; ++k) {
        double den = cfact(k) * cfact(j3 - j2 + k + m1) * cfact(j3 - j1 + k - m2) * cfact(j1 + j2 - j3 - k) *
                     cfact(j1 - k - m1) * cfact(j2 - k + m2);
        s += ((k & 1) ? -1.0 : 1.0) / den;
    }
    int e = j1 - j2 - m3;
    return (((e % 2) + 2) % 2 ? -1.0 : 1.0) * pre * s;
}
// real part of i^e (e even) or imaginary part (e odd)
constexpr double ipow_sign(int e) {
    int r = ((e % 4) + 4) % 4;
    return (r == 0 || r == 1) ? 1.0 : -1.0;
}
constexpr double ca5(int l, int m, int lp, int mp, int p) {
    if (p < iabs(l - lp) || p > l + lp || ((l + lp + p) & 1)) return 0.0;
    double c = (double)(l * (l + 1) + lp * (lp + 1) - p * (p + 1));
    double v = c * csqrt(2.0 * p + 1.0) *
               csqrt((2.0 * l + 1.0) * (2.0 * lp + 1.0) / (2.0 * l * (l + 1) * lp * (lp + 1))) *
               cw3j(l, lp, p, m, -mp, mp - m) * cw3j(l, lp, p, 0, 0, 0);
    if ((m - mp) & 1) v = -v;
    return ipow_sign(iabs(m - mp) - iabs(m) - iabs(mp) + lp - l + p) * v;
}
constexpr double cb5im(int l, int m, int lp, int mp, int p) {
    if (p < iabs(l - lp) + 1 || p > l + lp || !((l + lp + p) & 1)) return 0.0;
    double rad = (double)(l + lp + 1 + p) * (double)(l + lp + 1 - p) * (double)(p + l - lp) *
                 (double)(p - l + lp) * (2.0 * p + 1.0);
    double v = csqrt(rad) *
               csqrt((2.0 * lp + 1.0) * (2.0 * l + 1.0) / (2.0 * l * (l + 1) * lp * (lp + 1))) *
               cw3j(l, lp, p, m, -mp, mp - m) * cw3j(l, lp, p - 1, 0, 0, 0);
    if ((m - mp) & 1) v = -v;
    return ipow_sign(iabs(m - mp) - iabs(m) - iabs(mp) + lp - l + p) * v;
}

// offset (within pass M0) of the first coefficient of entry (mu, sgn, lp, l)
constexpr int coef_index(int L, int M0, int mu_t, int sgn_t, int lp_t, int l_t) {
    int n = 0;
    for (int mu = 0; mu <= mu_max(L, M0); ++mu)
        for (int s = 0; s < 2; ++s) {
            int sgn = s == 0 ? 1 : -1;
            if (!branch(L, M0, mu, sgn)) continue;
            int mp = M0 + sgn * mu;
            for (int lp = lp_lo(mp); lp <= L; ++lp)
                for (int l = l_lo(M0); l <= L; ++l) {
                    if (mu == mu_t && sgn == sgn_t && lp == lp_t && l == l_t) return n;
                    n += na(l, lp, mu) + nb(l, lp, mu);
                }
        }
    return -1;
}
}  // namespace plan
}  // namespace celes
