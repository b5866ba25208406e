// Stochastic Lanczos quadrature on the host in FP64 (LightGP Sec. 3
// "Inference": CG with a stochastic Lanczos log-determinant).
//
// The Lanczos tridiagonal T of a CG run started at x0 = 0 follows from its
// coefficients (Saad, Iterative Methods for Sparse Linear Systems, Sec. 6.7.3):
//   T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},  T_j,j+1 = sqrt(beta_j)/alpha_j.
// Gauss quadrature then gives z^T log(A) z ~= ||z||^2 sum_k w_k log(theta_k),
// theta_k the eigenvalues of T and w_k the squared first components of its
// unit eigenvectors (Golub & Welsch 1969).  The eigen-system comes from the
// implicit symmetric tridiagonal QR iteration with the Wilkinson shift (Golub
// & Van Loan, Matrix Computations, Sec. 8.3), carrying only the first row of
// the eigenvector matrix, which keeps the cost O(m^2) and the memory O(m).
// T is first scaled by a power of two so that no entry exceeds 1 in
// magnitude (exact, and log theta = log theta' - log scale): the rotations
// then take sqrt(x^2 + z^2) without overflow, about twice as fast as
// std::hypot on this serial chain of rotations.
#include <cmath>
#include <vector>

#include "../../include/mfgp.h"

namespace mfgp {

// Eigenvalues of the symmetric tridiagonal (d, e) into d, and in w the
// squared first components of the unit eigenvectors.  Returns false if the
// iteration did not converge.
bool tridiag_eig_first_row(std::vector<double>& d, std::vector<double>& e, std::vector<double>& w) {
    const int m = static_cast<int>(d.size());
    std::vector<double> v(m, 0.0);  // v = P e_0 with T = P^T diag(theta) P
    v[0] = 1.0;
    const double eps = 2.220446049250313e-16;
    int hi = m - 1;
    long budget = 64L * m + 64;
    while (hi > 0) {
        if (std::fabs(e[hi - 1]) <= eps * (std::fabs(d[hi - 1]) + std::fabs(d[hi]))) {
            e[hi - 1] = 0.0;
            --hi;
            continue;
        }
        int lo = hi - 1;
        while (lo > 0 && std::fabs(e[lo - 1]) > eps * (std::fabs(d[lo - 1]) + std::fabs(d[lo]))) --lo;
        if (--budget < 0) return false;
        // Wilkinson shift: eigenvalue of the trailing 2x2 block nearer d[hi].
        const double delta = 0.5 * (d[hi - 1] - d[hi]);
        const double b2 = e[hi - 1] * e[hi - 1];
        const double sgn = delta >= 0.0 ? 1.0 : -1.0;
        const double mu = d[hi] - b2 / (delta + sgn * std::sqrt(delta * delta + b2));
        // Implicit QR step: a chain of rotations R_k on (k, k+1) chasing the bulge.
        double x = d[lo] - mu;
        double z = e[lo];
        for (int k = lo; k < hi; ++k) {
            const double r = std::sqrt(x * x + z * z);
            const double c = r > 0.0 ? x / r : 1.0;
            const double s = r > 0.0 ? z / r : 0.0;
            if (k > lo) e[k - 1] = r;
            const double dk = d[k], dk1 = d[k + 1], ek = e[k];
            d[k] = c * c * dk + 2.0 * c * s * ek + s * s * dk1;
            d[k + 1] = s * s * dk - 2.0 * c * s * ek + c * c * dk1;
            e[k] = c * s * (dk1 - dk) + (c * c - s * s) * ek;
            if (k + 1 < hi) {
                x = e[k];
                z = s * e[k + 1];
                e[k + 1] = c * e[k + 1];
            }
            const double vk = v[k], vk1 = v[k + 1];
            v[k] = c * vk + s * vk1;
            v[k + 1] = -s * vk + c * vk1;
        }
    }
    w.resize(m);
    for (int k = 0; k < m; ++k) w[k] = v[k] * v[k];
    return true;
}

int slq_quadrature(const double* coeffs, int m, double znorm2, double* q) {
    std::vector<double> d(m), e(m > 1 ? m - 1 : 1, 0.0), w;
    for (int j = 0; j < m; ++j) {
        const double a = coeffs[2 * j];
        if (!(a > 0.0) || !std::isfinite(a)) return MFGP_BREAKDOWN;
        d[j] = 1.0 / a;
        if (j > 0) d[j] += coeffs[2 * (j - 1) + 1] / coeffs[2 * (j - 1)];
        if (j + 1 < m) {
            const double b = coeffs[2 * j + 1];
            if (!(b >= 0.0) || !std::isfinite(b)) return MFGP_BREAKDOWN;
            e[j] = std::sqrt(b) / a;
        }
    }
    if (m == 1) {
        *q = znorm2 * std::log(d[0]);
        return MFGP_OK;
    }
    double amax = 0.0;
    for (int j = 0; j < m; ++j) amax = std::fmax(amax, std::fabs(d[j]));
    for (int j = 0; j + 1 < m; ++j) amax = std::fmax(amax, std::fabs(e[j]));
    if (!std::isfinite(amax) || !(amax > 0.0)) return MFGP_BREAKDOWN;
    int ex = 0;
    (void)std::frexp(amax, &ex);   // amax = f 2^ex, f in [0.5, 1)
    for (int j = 0; j < m; ++j) d[j] = std::ldexp(d[j], -ex);
    for (int j = 0; j + 1 < m; ++j) e[j] = std::ldexp(e[j], -ex);
    if (!tridiag_eig_first_row(d, e, w)) return MFGP_NOT_CONVERGED;
    double acc = 0.0, wsum = 0.0;
    for (int k = 0; k < m; ++k) {
        if (!(d[k] > 0.0)) return MFGP_BREAKDOWN;
        acc += w[k] * std::log(d[k]);
        wsum += w[k];
    }
    // log theta = log theta' + ex ln 2, weighted by the (unit-sum) weights
    *q = znorm2 * (acc + wsum * ex * 0.69314718055994530942);
    return MFGP_OK;
}

}  // namespace mfgp
