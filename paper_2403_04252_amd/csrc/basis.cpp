// Host construction of one centre's basis (setup, run once per basis).
//
// The paper (Sec. II) expands the scattering wave function in bound
// eigenstates and wave-packet pseudostates and evaluates every radial
// quantity on one r-grid from 0 to ~100 a.u. that is denser near the origin.
// This file builds that grid and basis:
//   * grid r_i = r_max (i/n_r)^2 with composite-Simpson weights in x = i/n_r
//     (Jacobian 2 r_max x);
//   * bound states: closed-form hydrogen-like R_nl (Laguerre recurrence);
//   * bins: Delta_k^{-1/2} int_bin sqrt(2/pi) F_l(-Z/k, k r)/r dk with the
//     regular Coulomb function obtained from its power series at the origin
//     and Taylor continuation of the radial equation between grid nodes,
//     normalised by the closed-form Coulomb constant C_l(eta);
//   * per-l modified Gram-Schmidt (bound states first, then bins by k).
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "wpccc_impl.h"

namespace wpccc {

namespace {

constexpr int kGaussK = 16;       // Gauss-Legendre nodes per k-bin
constexpr double kPi = 3.14159265358979323846;

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& wt) {
    x.assign(n, 0.0);
    wt.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        long double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
        long double dp = 0;
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1, p1 = z;
            for (int k = 2; k <= n; ++k) {
                long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1);
            long double dz = p1 / dp;
            z -= dz;
            if (std::fabs((double)dz) < 1e-19) break;
        }
        // recompute derivative at the converged node
        long double p0 = 1, p1 = z;
        for (int k = 2; k <= n; ++k) {
            long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1);
        double ww = (double)(2.0L / ((1 - z * z) * dp * dp));
        x[i] = -(double)z;
        x[n - 1 - i] = (double)z;
        wt[i] = ww;
        wt[n - 1 - i] = ww;
    }
}

// Hydrogen-like R_nl(r) = N e^{-rho/2} rho^l L^{2l+1}_{n-l-1}(rho), rho = 2Zr/n.
double hydrogen(int n, int l, double Z, double r) {
    const double rho = 2.0 * Z * r / n;
    const int k = n - l - 1;
    const double alpha = 2 * l + 1;
    double L0 = 1.0, L1 = 1.0 + alpha - rho, Lk = (k == 0) ? 1.0 : L1;
    for (int j = 1; j < k; ++j) {
        double L2 = ((2 * j + 1 + alpha - rho) * L1 - (j + alpha) * L0) / (j + 1);
        L0 = L1;
        L1 = L2;
        Lk = L2;
    }
    // normalisation sqrt((2Z/n)^3 (n-l-1)! / (2n (n+l)!))
    long double ratio = 1.0L;  // (n-l-1)!/(n+l)!
    for (int j = n - l; j <= n + l; ++j) ratio /= j;
    const double norm = std::sqrt(std::pow(2.0 * Z / n, 3) * (double)ratio / (2.0 * n));
    return norm * std::exp(-0.5 * rho) * std::pow(rho, l) * Lk;
}

// C_l(eta) with C_0^2 = 2 pi eta / (e^{2 pi eta} - 1).
double coulomb_constant(int l, double eta) {
    const double x = 2.0 * kPi * eta;
    double c = std::sqrt(x / std::expm1(x));
    for (int j = 1; j <= l; ++j) c *= std::sqrt(j * (double)j + eta * eta) / (j * (2.0 * j + 1));
    return c;
}

// Regular solution u (u ~ r^{l+1}) of u'' = (l(l+1)/r^2 - 2Z/r - k^2) u on the
// grid nodes r[0..n].  Series about 0 for r <= r_sw, then Taylor steps.
void coulomb_regular(int l, double k, double Z, const std::vector<double>& r,
                     std::vector<double>& u) {
    const int n = (int)r.size();
    u.assign(n, 0.0);
    const double k2 = k * k;
    const double r_sw = 0.3;
    // power series coefficients a_j: j (j + 2l + 1) a_j = -2Z a_{j-1} - k^2 a_{j-2}
    const int n_ser = 120;
    std::vector<double> a(n_ser + 1, 0.0);
    a[0] = 1.0;
    for (int j = 1; j <= n_ser; ++j)
        a[j] = (-2.0 * Z * a[j - 1] - (j >= 2 ? k2 * a[j - 2] : 0.0)) / (double)(j * (j + 2 * l + 1));
    int last = 0;
    double uval = 0.0, uder = 0.0;
    for (int i = 0; i < n && r[i] <= r_sw; ++i) {
        const double ri = r[i];
        double s = 0.0, ds = 0.0, p = 1.0;
        int small = 0;
        for (int j = 0; j <= n_ser; ++j) {
            const double t = a[j] * p;
            s += t;
            ds += (j + l + 1) * t;
            p *= ri;
            if (std::fabs(t) < 1e-20 * std::fabs(s)) {
                if (++small >= 3) break;
            } else {
                small = 0;
            }
        }
        u[i] = std::pow(ri, l + 1) * s;
        uval = u[i];
        uder = (ri > 0) ? std::pow(ri, l) * ds : (l == 0 ? 1.0 : 0.0);
        last = i;
    }
    const double L = l * (l + 1.0);
    double c[80];
    for (int i = last + 1; i < n; ++i) {
        const double r0 = r[i - 1];
        const double t = r[i] - r0;
        const double A = L - 2.0 * Z * r0 - k2 * r0 * r0;
        const double B = -(2.0 * Z + 2.0 * k2 * r0);
        const double inv = 1.0 / (r0 * r0);
        c[0] = uval;
        c[1] = uder;
        double val = c[0] + c[1] * t, der = c[1];
        double tp = t;  // t^(m-1) for the term m being added
        int small = 0;
        for (int m = 2; m < 80; ++m) {
            const int nn = m - 2;
            double num = A * c[nn] - 2.0 * r0 * nn * (nn + 1) * c[nn + 1] - nn * (nn - 1.0) * c[nn];
            if (nn >= 1) num += B * c[nn - 1];
            if (nn >= 2) num -= k2 * c[nn - 2];
            c[m] = num * inv / ((nn + 1.0) * (nn + 2.0));
            der += m * c[m] * tp;
            tp *= t;
            const double term = c[m] * tp;
            val += term;
            if (std::fabs(term) <= 1e-19 * (std::fabs(val) + std::fabs(der) * t)) {
                if (++small >= 2) break;
            } else {
                small = 0;
            }
        }
        uval = val;
        uder = der;
        u[i] = val;
    }
}

void modified_gram_schmidt(std::vector<std::vector<double>>& f, const std::vector<double>& meas) {
    const size_t n = meas.size();
    for (size_t j = 0; j < f.size(); ++j) {
        for (size_t i = 0; i < j; ++i) {
            double d = 0.0;
            for (size_t q = 0; q < n; ++q) d += meas[q] * f[i][q] * f[j][q];
            for (size_t q = 0; q < n; ++q) f[j][q] -= d * f[i][q];
        }
        double nn = 0.0;
        for (size_t q = 0; q < n; ++q) nn += meas[q] * f[j][q] * f[j][q];
        const double s = 1.0 / std::sqrt(nn);
        for (size_t q = 0; q < n; ++q) f[j][q] *= s;
    }
}

}  // namespace

int build_host_basis(const wpccc_basis_spec& spec, HostBasis& hb) {
    if (spec.l_max < 0 || spec.l_max > 10 || spec.n_max < 1 || spec.n_bins < 0 ||
        spec.n_r < 2 || spec.n_r > 20000 || (spec.n_r % 2) != 0 || !(spec.r_max > 0) ||
        !(spec.Z > 0) || (spec.n_bins > 0 && !(spec.k_max > 0))) {
        set_error("wpccc_basis: invalid spec (l_max 0..10, n_max >= 1, n_bins >= 0, "
                  "even n_r in 2..20000, r_max > 0, Z > 0, k_max > 0 with bins)");
        return WPCCC_EINVAL;
    }
    hb.spec = spec;
    const int nr = spec.n_r;
    hb.n_r = nr;
    hb.r.resize(nr + 1);
    hb.w.resize(nr + 1);
    for (int i = 0; i <= nr; ++i) {
        const double x = (double)i / nr;
        hb.r[i] = spec.r_max * x * x;
        const double s = (i == 0 || i == nr) ? 1.0 : ((i % 2) ? 4.0 : 2.0);
        hb.w[i] = s / (3.0 * nr) * 2.0 * spec.r_max * x;
    }
    std::vector<double> meas(nr + 1);
    for (int i = 0; i <= nr; ++i) meas[i] = hb.w[i] * hb.r[i] * hb.r[i];

    std::vector<double> gx, gw;
    gauss_legendre(kGaussK, gx, gw);

    hb.n_l.clear();
    hb.rad_off.clear();
    hb.rad_l.clear();
    hb.rad_eps.clear();
    hb.phi.clear();
    std::vector<double> u;
    for (int l = 0; l <= spec.l_max; ++l) {
        std::vector<std::vector<double>> rows;
        std::vector<double> e;
        for (int n = l + 1; n <= spec.n_max; ++n) {
            std::vector<double> f(nr + 1);
            for (int i = 0; i <= nr; ++i) f[i] = hydrogen(n, l, spec.Z, hb.r[i]);
            rows.push_back(std::move(f));
            e.push_back(-spec.Z * spec.Z / (2.0 * n * n));
        }
        const double dk = spec.n_bins > 0 ? spec.k_max / spec.n_bins : 0.0;
        for (int b = 0; b < spec.n_bins; ++b) {
            const double lo = b * dk, hi = (b + 1) * dk;
            std::vector<double> f(nr + 1, 0.0);
            for (int g = 0; g < kGaussK; ++g) {
                const double k = 0.5 * (lo + hi) + 0.5 * (hi - lo) * gx[g];
                const double wk = 0.5 * (hi - lo) * gw[g];
                coulomb_regular(l, k, spec.Z, hb.r, u);
                const double pref = wk * std::sqrt(2.0 / kPi) *
                                    coulomb_constant(l, -spec.Z / k) * std::pow(k, l + 1);
                for (int i = 0; i <= nr; ++i) {
                    double ur;
                    if (hb.r[i] > 0) ur = u[i] / hb.r[i];
                    else ur = (l == 0) ? 1.0 : 0.0;
                    f[i] += pref * ur;
                }
            }
            const double s = 1.0 / std::sqrt(hi - lo);
            for (double& x : f) x *= s;
            rows.push_back(std::move(f));
            e.push_back((lo * lo + lo * hi + hi * hi) / 6.0);
        }
        if (rows.empty()) {
            set_error("wpccc_basis: l = %d has no radial functions (n_max too small, no bins)", l);
            return WPCCC_EINVAL;
        }
        modified_gram_schmidt(rows, meas);
        hb.rad_off.push_back((int)hb.rad_l.size());
        hb.n_l.push_back((int)rows.size());
        for (size_t q = 0; q < rows.size(); ++q) {
            hb.phi.insert(hb.phi.end(), rows[q].begin(), rows[q].end());
            hb.rad_l.push_back(l);
            hb.rad_eps.push_back(e[q]);
        }
    }
    hb.n_f = (int)hb.rad_l.size();
    hb.st_l.clear();
    hb.st_m.clear();
    hb.st_i.clear();
    hb.eps.clear();
    hb.state_off.clear();
    for (int l = 0; l <= spec.l_max; ++l) {
        hb.state_off.push_back((int)hb.st_l.size());
        for (int m = -l; m <= l; ++m)
            for (int i = 0; i < hb.n_l[l]; ++i) {
                hb.st_l.push_back(l);
                hb.st_m.push_back(m);
                hb.st_i.push_back(hb.rad_off[l] + i);
                hb.eps.push_back(hb.rad_eps[hb.rad_off[l] + i]);
            }
    }
    hb.n_states = (int)hb.st_l.size();
    return WPCCC_OK;
}

double clebsch_gordan(int j1, int m1, int j2, int m2, int J, int M) {
    if (m1 + m2 != M || std::abs(m1) > j1 || std::abs(m2) > j2 || std::abs(M) > J) return 0.0;
    if (J < std::abs(j1 - j2) || J > j1 + j2) return 0.0;
    auto fact = [](int n) {
        long double f = 1.0L;
        for (int i = 2; i <= n; ++i) f *= i;
        return f;
    };
    long double pre = (2 * J + 1) * fact(J + j1 - j2) * fact(J - j1 + j2) * fact(j1 + j2 - J) /
                      fact(j1 + j2 + J + 1);
    pre *= fact(J + M) * fact(J - M) * fact(j1 - m1) * fact(j1 + m1) * fact(j2 - m2) * fact(j2 + m2);
    long double s = 0.0L;
    for (int k = 0; k <= j1 + j2 - J; ++k) {
        const int a[6] = {k, j1 + j2 - J - k, j1 - m1 - k, j2 + m2 - k, J - j2 + m1 + k, J - j1 - m2 + k};
        bool ok = true;
        for (int q = 0; q < 6; ++q) ok = ok && a[q] >= 0;
        if (!ok) continue;
        long double den = 1.0L;
        for (int q = 0; q < 6; ++q) den *= fact(a[q]);
        s += ((k % 2) ? -1.0L : 1.0L) / den;
    }
    return (double)(std::sqrt(pre) * s);
}

}  // namespace wpccc
