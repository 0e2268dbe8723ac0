// Host-side tables of the spherical-harmonic machinery, built once per degree
// and uploaded to the device.
//
//  * Gauss-Legendre grid (Sec. 2.1): Newton's method on the orthonormal
//    Legendre polynomial from asymptotic initial guesses.
//  * Normalized associated Legendre functions (Sec. 1.1, Appendix A): the
//    fully normalized three-term recursion in n, and theta-derivatives from
//    the ladder identity of Appendix A,
//        dP_n^m/dtheta = alpha_n^m P_n^{m+1} + m cot(theta) P_n^m,
//    alpha_n^m = sqrt((n-m)(n+m+1)), differentiated once more for the second
//    derivative.
//  * Wigner small-d matrices of Appendix B. The explicit factorial sum there
//    cancels catastrophically in FP64 beyond degree ~24, so the same matrix
//    is evaluated through its Jacobi-polynomial form
//        d^n_{m'm}(b) = sqrt((n+m)!(n-m)!/((n+m')!(n-m')!))
//                       sin(b/2)^{m-m'} cos(b/2)^{m+m'} P^{(m-m', m+m')}_{n-m}(cos b)
//    (valid for m >= |m'|, the other index pairs by the symmetries
//    d_{m'm} = (-1)^{m-m'} d_{mm'} = d_{-m,-m'}), with the Jacobi polynomial
//    from its stable three-term recursion in degree.
#include "internal.hpp"

#include <cmath>
#include <vector>

namespace bim {

static const double kPi = 3.14159265358979323846;

void gauss_legendre(int q, std::vector<double> &t, std::vector<double> &w)
{
    const int N = q + 1;
    t.assign(N, 0.0);
    w.assign(N, 0.0);
    for (int i = 0; i < N; ++i) {
        // Tricomi-type asymptotic guess for the (i+1)-th largest root.
        double th = kPi * (4.0 * i + 3.0) / (4.0 * N + 2.0);
        double x = (1.0 - (N - 1.0) / (8.0 * N * N * N)) * std::cos(th);
        double der = 1.0;
        for (int it = 0; it < 60; ++it) {
            // orthonormal Legendre q_k = sqrt(k + 1/2) P_k, recursion in k
            double qm = 0.0, qk = std::sqrt(0.5);
            for (int k = 1; k <= N; ++k) {
                double a = std::sqrt((4.0 * k * k - 1.0)) / k;
                double b = (k > 1) ? std::sqrt((2.0 * k + 1.0) / (2.0 * k - 3.0)) * (k - 1.0) / k : 0.0;
                double qn = a * x * qk - b * qm;
                qm = qk;
                qk = qn;
            }
            // qk = q_N(x), qm = q_{N-1}(x); derivative of P_N via
            // (1 - x^2) P_N' = N (P_{N-1} - x P_N)
            double PN = qk / std::sqrt(N + 0.5), PNm = qm / std::sqrt(N - 0.5);
            der = N * (PNm - x * PN) / (1.0 - x * x);
            double dx = PN / der;
            x -= dx;
            if (std::fabs(dx) <= 1e-17) break;
        }
        {
            double qm = 0.0, qk = std::sqrt(0.5);
            for (int k = 1; k <= N; ++k) {
                double a = std::sqrt((4.0 * k * k - 1.0)) / k;
                double b = (k > 1) ? std::sqrt((2.0 * k + 1.0) / (2.0 * k - 3.0)) * (k - 1.0) / k : 0.0;
                double qn = a * x * qk - b * qm;
                qm = qk;
                qk = qn;
            }
            double PN = qk / std::sqrt(N + 0.5), PNm = qm / std::sqrt(N - 0.5);
            der = N * (PNm - x * PN) / (1.0 - x * x);
        }
        t[i] = x;
        w[i] = 2.0 / ((1.0 - x * x) * der * der);
    }
}

// P[tri(n,m)], D1, D2 at t = cos(theta), 0 < theta < pi.
void legendre_table(int nmax, double t, double *P, double *D1, double *D2)
{
    const double s = std::sqrt(std::max(0.0, 1.0 - t * t));
    // sectoral values: P_m^m = (-1)^m sqrt((2m+1)!!/(4 pi (2m)!!)) s^m, by a product
    double pmm = 1.0 / std::sqrt(4.0 * kPi);
    for (int m = 0; m <= nmax; ++m) {
        if (m > 0) pmm *= -std::sqrt((2.0 * m + 1.0) / (2.0 * m)) * s;
        P[tri(m, m)] = pmm;
        if (m + 1 <= nmax) P[tri(m + 1, m)] = std::sqrt(2.0 * m + 3.0) * t * pmm;
        for (int n = m + 2; n <= nmax; ++n) {
            double an = std::sqrt((2.0 * n + 1.0) * (2.0 * n - 1.0) / ((double)(n - m) * (n + m)));
            double bn = std::sqrt((2.0 * n + 1.0) * (double)(n + m - 1) * (n - m - 1) /
                                  ((2.0 * n - 3.0) * (double)(n - m) * (n + m)));
            P[tri(n, m)] = an * t * P[tri(n - 1, m)] - bn * P[tri(n - 2, m)];
        }
    }
    if (!D1) return;
    const double cot = t / s;
    for (int n = 0; n <= nmax; ++n)
        for (int m = 0; m <= n; ++m) {
            double up = (m + 1 <= n) ? std::sqrt((double)(n - m) * (n + m + 1)) * P[tri(n, m + 1)] : 0.0;
            D1[tri(n, m)] = up + m * cot * P[tri(n, m)];
        }
    if (!D2) return;
    // d/dtheta of the ladder identity:
    //   P'' = alpha_n^m (P_n^{m+1})' - m / sin^2 P_n^m + m cot (P_n^m)'
    for (int n = 0; n <= nmax; ++n)
        for (int m = 0; m <= n; ++m) {
            double up = (m + 1 <= n) ? std::sqrt((double)(n - m) * (n + m + 1)) * D1[tri(n, m + 1)] : 0.0;
            D2[tri(n, m)] = up - m / (s * s) * P[tri(n, m)] + m * cot * D1[tri(n, m)];
        }
}

// Jacobi polynomials P_k^{(a,b)}(x), k = 0..K, by the three-term recursion.
static void jacobi(int K, int a, int b, double x, double *out)
{
    out[0] = 1.0;
    if (K == 0) return;
    out[1] = (a + 1.0) + (a + b + 2.0) * (x - 1.0) / 2.0;
    for (int k = 2; k <= K; ++k) {
        double c = 2.0 * k + a + b;
        double A = 2.0 * k * (k + a + b) * (c - 2.0);
        double B = (c - 1.0) * (c * (c - 2.0) * x + (double)a * a - (double)b * b);
        double C = 2.0 * (k + a - 1.0) * (k + b - 1.0) * c;
        out[k] = (B * out[k - 1] - C * out[k - 2]) / A;
    }
}

// d^n_{m'm}(beta) for every n <= nmax, m' in [-n, n], m in [-n, n]:
// d[off(n) + (m'+n)(2n+1) + (m+n)], off(n) = sum_{k<n} (2k+1)^2.
void wigner_table(int nmax, double beta, std::vector<double> &d)
{
    auto off = [](int n) { return (size_t)n * (4 * (size_t)n * n - 1) / 3; };
    d.assign(off(nmax + 1), 0.0);
    const double x = std::cos(beta), sh = std::sin(beta / 2.0), ch = std::cos(beta / 2.0);
    std::vector<double> jac(nmax + 2);
    // canonical region m >= |m'|: loop m, m'; Jacobi degree k = n - m, n = m..nmax
    for (int m = 0; m <= nmax; ++m)
        for (int mp = -m; mp <= m; ++mp) {
            const int a = m - mp, b = m + mp;
            jacobi(nmax - m, a, b, x, jac.data());
            const double pw = std::pow(sh, a) * std::pow(ch, b);
            for (int n = m; n <= nmax; ++n) {
                // sqrt((n+m)!(n-m)!/((n+m')!(n-m')!)) as a product of a ratios
                double ratio = 1.0;
                for (int s = 1; s <= a; ++s) ratio *= (double)(n + mp + s) / (double)(n - m + s);
                const double v = std::sqrt(ratio) * pw * jac[n - m];
                const size_t N2 = 2 * n + 1;
                auto at = [&](int r, int c) -> double & { return d[off(n) + (size_t)(r + n) * N2 + (c + n)]; };
                const double sg = ((m - mp) & 1) ? -1.0 : 1.0;
                at(mp, m) = v;              // canonical
                at(m, mp) = sg * v;         // swap
                at(-m, -mp) = v;            // d_{m'm} = d_{-m,-m'}
                at(-mp, -m) = sg * v;       // both
            }
        }
}

// Rotation tables of one degree-p target grid: for every latitude j and
// degree n, the real (n+1)x(n+1) matrices (rows nu = 0..n, columns mu = 0..n)
//   A+_{nu mu} = d_{nu mu} + (-1)^nu d_{-nu,mu}   (nu >= 1),  A+_{0 mu} = d_{0 mu}
//   A-_{nu mu} = d_{nu mu} - (-1)^nu d_{-nu,mu}   (nu >= 1),  A-_{0 mu} = d_{0 mu}
// so that, for a real field with g^nu = e^{i nu phi} f^nu (nu >= 0), the
// rotated coefficients are Re f'^mu = sum_nu A+ Re g^nu, Im f'^mu = sum_nu A- Im g^nu.
void rotation_tables(int p, const std::vector<double> &theta, std::vector<double> &Ap, std::vector<double> &Am)
{
    const size_t per = rot_lat_size(p);
    Ap.assign(per * (p + 1), 0.0);
    Am.assign(per * (p + 1), 0.0);
    std::vector<double> d;
    auto off = [](int n) { return (size_t)n * (4 * (size_t)n * n - 1) / 3; };
    for (int j = 0; j <= p; ++j) {
        wigner_table(p, theta[j], d);
        for (int n = 0; n <= p; ++n) {
            const size_t N2 = 2 * n + 1;
            for (int nu = 0; nu <= n; ++nu)
                for (int mu = 0; mu <= n; ++mu) {
                    double dp = d[off(n) + (size_t)(nu + n) * N2 + (mu + n)];
                    double dm = d[off(n) + (size_t)(-nu + n) * N2 + (mu + n)];
                    double sg = (nu & 1) ? -1.0 : 1.0;
                    size_t o = per * j + rot_off(n) + (size_t)nu * (n + 1) + mu;
                    if (nu == 0) {
                        Ap[o] = dp;
                        Am[o] = dp;
                    } else {
                        Ap[o] = dp + sg * dm;
                        Am[o] = dp - sg * dm;
                    }
                }
        }
    }
}

// Legendre polynomial sum  sum_{n=0}^{q} P_n(t)  (weights of Theorem 1), from
// the orthonormal recursion q_k = sqrt(k + 1/2) P_k used for the grid above.
double legendre_sum(int q, double t)
{
    double qm = 0.0, qk = std::sqrt(0.5);
    double sum = qk / std::sqrt(0.5);
    for (int k = 1; k <= q; ++k) {
        double a = std::sqrt((4.0 * k * k - 1.0)) / k;
        double b = (k > 1) ? std::sqrt((2.0 * k + 1.0) / (2.0 * k - 3.0)) * (k - 1.0) / k : 0.0;
        double qn = a * t * qk - b * qm;
        qm = qk;
        qk = qn;
        sum += qk / std::sqrt(k + 0.5);
    }
    return sum;
}

}  // namespace bim
