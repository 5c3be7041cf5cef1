// host_linalg.cpp -- eigenvalues of the effective Hamiltonian (host code).
//
// The last step of a sector's solution is the diagonalisation of H_eff =
// (H Omega)_Cl, a small dense complex non-Hermitian matrix (one row and
// column per model state: 6 active spinors, 15 active pairs at the
// production size); its eigenvalues are the state energies.  Method (the
// standard dense non-symmetric eigenvalue algorithm, e.g. Golub and Van Loan,
// Matrix Computations, ch. 7):
//   1. reduce to upper Hessenberg form by Householder reflections
//      H = Q^H A Q (unitary similarity, eigenvalues unchanged);
//   2. single-shift complex QR iterations on the active window [lo, hi] of
//      the Hessenberg matrix with the Wilkinson shift (the eigenvalue of the
//      trailing 2 x 2 block closer to its last diagonal element), each step
//      H - mu I = Q R by Givens rotations, H <- R Q + mu I; a subdiagonal
//      element below eps (|h_kk| + |h_k-1,k-1|) is set to zero, which splits
//      the problem (deflation); an exceptional shift after 10 steps without
//      deflation breaks cycles;
//   3. the diagonal of the resulting triangular matrix, sorted by real part
//      (ties by imaginary part).
// Only the eigenvalues are wanted, so each rotation is applied to the rows
// and columns of the active window alone.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "../../include/fscc.h"

namespace {

using cd = std::complex<double>;

// Householder reduction of the n x n row-major matrix a to Hessenberg form.
void hessenberg(std::vector<cd>& a, int n) {
    std::vector<cd> v(n);
    for (int k = 0; k + 2 < n; ++k) {
        double norm = 0.0;
        for (int i = k + 1; i < n; ++i) norm += std::norm(a[(size_t)i * n + k]);
        norm = std::sqrt(norm);
        if (norm == 0.0) continue;
        const cd x0 = a[(size_t)(k + 1) * n + k];
        const cd phase = std::abs(x0) > 0.0 ? x0 / std::abs(x0) : cd(1.0, 0.0);
        const cd alpha = -phase * norm;     // reflected vector = alpha e_1 (sign avoids cancellation)
        double vn = 0.0;
        for (int i = k + 1; i < n; ++i) {
            v[i] = a[(size_t)i * n + k] - (i == k + 1 ? alpha : cd(0.0));
            vn += std::norm(v[i]);
        }
        vn = std::sqrt(vn);
        if (vn == 0.0) continue;
        for (int i = k + 1; i < n; ++i) v[i] /= vn;
        // a <- (I - 2 v v^H) a  on rows k+1..n-1
        for (int j = 0; j < n; ++j) {
            cd s = 0.0;
            for (int i = k + 1; i < n; ++i) s += std::conj(v[i]) * a[(size_t)i * n + j];
            for (int i = k + 1; i < n; ++i) a[(size_t)i * n + j] -= 2.0 * v[i] * s;
        }
        // a <- a (I - 2 v v^H)  on columns k+1..n-1
        for (int i = 0; i < n; ++i) {
            cd s = 0.0;
            for (int j = k + 1; j < n; ++j) s += a[(size_t)i * n + j] * v[j];
            for (int j = k + 1; j < n; ++j) a[(size_t)i * n + j] -= 2.0 * s * std::conj(v[j]);
        }
        for (int i = k + 2; i < n; ++i) a[(size_t)i * n + k] = 0.0;
    }
}

// Eigenvalues of the upper Hessenberg matrix h; false if the iteration does
// not converge in 60 n steps.
bool hessenberg_qr(std::vector<cd>& h, int n, std::vector<cd>& w) {
    const double eps = 2.220446049250313e-16;
    auto H = [&](int i, int j) -> cd& { return h[(size_t)i * n + j]; };
    w.assign(n, 0.0);
    int hi = n - 1, since = 0, total = 0;
    std::vector<double> cs(n);
    std::vector<cd> sn(n);
    while (hi >= 0) {
        if (hi == 0) {
            w[0] = H(0, 0);
            break;
        }
        int lo = hi;
        while (lo > 0) {
            const double scale = std::abs(H(lo, lo)) + std::abs(H(lo - 1, lo - 1));
            if (std::abs(H(lo, lo - 1)) <= eps * (scale > 0.0 ? scale : 1.0)) {
                H(lo, lo - 1) = 0.0;
                break;
            }
            --lo;
        }
        if (lo == hi) {
            w[hi] = H(hi, hi);
            --hi;
            since = 0;
            continue;
        }
        if (++total > 60 * n) return false;
        cd mu;
        if (++since % 11 == 0) {
            // exceptional shift: breaks a cycle of the Wilkinson shift
            mu = H(hi, hi) + 0.75 * std::abs(H(hi, hi - 1));
        } else {
            const cd a = H(hi - 1, hi - 1), b = H(hi - 1, hi), c = H(hi, hi - 1), d = H(hi, hi);
            const cd half = 0.5 * (a - d);
            const cd disc = std::sqrt(half * half + b * c);
            const cd m1 = 0.5 * (a + d) + disc, m2 = 0.5 * (a + d) - disc;
            mu = std::abs(m1 - d) < std::abs(m2 - d) ? m1 : m2;
        }
        for (int k = lo; k <= hi; ++k) H(k, k) -= mu;
        // Q^H (H - mu I) = R: rotation k acts on rows k, k+1 and zeroes H(k+1, k)
        for (int k = lo; k < hi; ++k) {
            const cd x = H(k, k), y = H(k + 1, k);
            const double r = std::hypot(std::abs(x), std::abs(y));
            double c;
            cd s;
            if (r == 0.0) {
                c = 1.0;
                s = 0.0;
            } else {
                c = std::abs(x) / r;
                const cd ph = std::abs(x) > 0.0 ? x / std::abs(x) : cd(1.0, 0.0);
                s = ph * std::conj(y) / r;
            }
            cs[k] = c;
            sn[k] = s;
            for (int j = k; j <= hi; ++j) {
                const cd p = H(k, j), q = H(k + 1, j);
                H(k, j) = c * p + s * q;
                H(k + 1, j) = -std::conj(s) * p + c * q;
            }
        }
        // R Q: the conjugate-transposed rotations on columns k, k+1
        for (int k = lo; k < hi; ++k) {
            const double c = cs[k];
            const cd s = sn[k];
            const int last = std::min(k + 2, hi);
            for (int i = lo; i <= last; ++i) {
                const cd p = H(i, k), q = H(i, k + 1);
                H(i, k) = c * p + std::conj(s) * q;
                H(i, k + 1) = -s * p + c * q;
            }
        }
        for (int k = lo; k <= hi; ++k) H(k, k) += mu;
    }
    return true;
}

}  // namespace

extern "C" fscc_status fscc_heff_eig(int n, const fscc_c128* heff_host, fscc_c128* eig_host) {
    if (n < 0 || n > 4096 || (n > 0 && (!heff_host || !eig_host))) return FSCC_EINVAL;
    if (n == 0) return FSCC_OK;
    std::vector<cd> a((size_t)n * n);
    for (size_t k = 0; k < a.size(); ++k) {
        if (!std::isfinite(heff_host[k].re) || !std::isfinite(heff_host[k].im)) return FSCC_EINVAL;
        a[k] = cd(heff_host[k].re, heff_host[k].im);
    }
    hessenberg(a, n);
    std::vector<cd> w;
    if (!hessenberg_qr(a, n, w)) return FSCC_ENOCONV;
    std::sort(w.begin(), w.end(), [](const cd& x, const cd& y) {
        return x.real() < y.real() || (x.real() == y.real() && x.imag() < y.imag());
    });
    for (int k = 0; k < n; ++k) {
        eig_host[k].re = w[k].real();
        eig_host[k].im = w[k].imag();
    }
    return FSCC_OK;
}
