// Rational approximation of x^(-1/2) for the EOFA heatbath (Section 3.2).
//
// The heatbath needs x^(-1/2) ~ alpha0 + sum_l alpha_l / (beta_l + x) on an
// interval [lo, hi] that holds the spectrum of M_EOFA.  The best such
// approximation in relative error (type (n, n)) has Zolotarev's closed form.
// On y = x / lo in [1, kappa], kappa = hi / lo, with elliptic parameter
// m = 1 - 1/kappa, u_j = j K(m) / (2n + 1) and c_j = sn^2(u_j) / cn^2(u_j):
//   y^(-1/2) ~ d prod_{l=1..n} (y + c_{2l}) / (y + c_{2l-1}).
// sqrt(y) times the product is smallest at y = 1 and largest at y = kappa;
// d = 2 / (min + max) centres the relative error, which then alternates
// 2n + 2 times with magnitude delta = (max - min) / (max + min).
//
// K, sn and cn come from the arithmetic-geometric mean (the AGM scale of
// Abramowitz and Stegun, 16.4 and 17.6).  Host code only.
#include <cmath>
#include <vector>

namespace eofa {
namespace {

constexpr double kPi = 3.14159265358979323846;

// AGM scale for parameter m: a_0 = 1, b_0 = sqrt(1 - m), c_0 = sqrt(m);
// a_{j+1} = (a_j + b_j)/2, b_{j+1} = sqrt(a_j b_j), c_{j+1} = (a_j - b_j)/2.
struct Agm {
    std::vector<double> a, c;
};

Agm agm_scale(double m) {
    Agm s;
    double a = 1.0, b = std::sqrt(1.0 - m), c = std::sqrt(m);
    s.a.push_back(a);
    s.c.push_back(c);
    for (int it = 0; it < 64 && std::fabs(c) > 1e-17 * a; ++it) {
        const double an = 0.5 * (a + b), bn = std::sqrt(a * b);
        c = 0.5 * (a - b);
        a = an;
        b = bn;
        s.a.push_back(a);
        s.c.push_back(c);
    }
    return s;
}

// Complete elliptic integral of the first kind: K(m) = pi / (2 AGM(1, sqrt(1 - m))).
double ellip_k(const Agm& s) { return kPi / (2.0 * s.a.back()); }

// Jacobi sn and cn at argument u: phi_N = 2^N a_N u, then
// phi_{j-1} = (phi_j + asin(c_j sin(phi_j) / a_j)) / 2; sn = sin phi_0, cn = cos phi_0.
void ellip_sncn(const Agm& s, double u, double* sn, double* cn) {
    const int N = (int)s.a.size() - 1;
    double phi = std::ldexp(s.a[N] * u, N);
    for (int j = N; j >= 1; --j) phi = 0.5 * (phi + std::asin(s.c[j] * std::sin(phi) / s.a[j]));
    *sn = std::sin(phi);
    *cn = std::cos(phi);
}

}  // namespace

// Arguments are validated by the caller (0 < lo <= hi finite, n >= 1).
void zolotarev_inv_sqrt(double lo, double hi, int n, double* alpha0, double* alpha, double* beta,
                        double* delta_out) {
    const double kappa = hi / lo;
    const double m = 1.0 - 1.0 / kappa;
    const Agm s = agm_scale(m);
    const double K = ellip_k(s);
    std::vector<double> pole(n), zero(n);
    for (int j = 1; j <= 2 * n; ++j) {
        double sn, cn;
        ellip_sncn(s, j * K / (2 * n + 1), &sn, &cn);
        const double cj = (sn * sn) / (cn * cn);
        if (j & 1) pole[(j - 1) / 2] = cj;
        else zero[j / 2 - 1] = cj;
    }
    auto prod_at = [&](double y) {
        double p = 1.0;
        for (int l = 0; l < n; ++l) p *= (y + zero[l]) / (y + pole[l]);
        return p;
    };
    const double fmin = prod_at(1.0), fmax = std::sqrt(kappa) * prod_at(kappa);
    const double d = 2.0 / (fmin + fmax);
    if (delta_out) *delta_out = std::fabs(fmax - fmin) / (fmax + fmin);
    // x^(-1/2) ~ lo^(-1/2) d prod (x + lo c_2l) / (x + lo c_2l-1); partial fractions
    // prod (x + A_j) / (x + B_j) = 1 + sum_l r_l / (x + B_l),
    // r_l = prod_j (A_j - B_l) / prod_{j != l} (B_j - B_l).
    const double a0 = d / std::sqrt(lo);
    for (int l = 0; l < n; ++l) {
        const double Bl = lo * pole[l];
        double num = 1.0, den = 1.0;
        for (int j = 0; j < n; ++j) {
            num *= lo * zero[j] - Bl;
            if (j != l) den *= lo * pole[j] - Bl;
        }
        alpha[l] = a0 * num / den;
        beta[l] = Bl;
    }
    *alpha0 = a0;
}

}  // namespace eofa
