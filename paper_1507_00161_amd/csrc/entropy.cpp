// entropy.cpp - orbital entropies from measured correlations and the
// entropy-based chain ordering (host side; the entropy paragraph).
//
// With the proton and neutron numbers and 2M conserved, rho_i =
// diag(1 - <n_i>, <n_i>), and rho_ij in the basis |00>, |01>, |10>, |11> of
// (n_i, n_j) is diagonal except for the |01>/|10> pair, which <c+_i c_j>
// couples.  Its eigenvalues are therefore the two diagonal corners and the
// two eigenvalues of [[<n_j> - <n_i n_j>, h], [h, <n_i> - <n_i n_j>]].
//
// The ordering minimises the relaxed eta = 2 entanglement distance: sort the
// sites by the Fiedler vector of the Laplacian of the mutual information,
// found with the cyclic Jacobi method (Golub and Van Loan, symmetric Schur
// rotations swept over all pairs until the off-diagonal norm vanishes).
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "engine.h"

namespace dm {

static double xlogx(double w) { return w > 0.0 ? w * std::log(w) : 0.0; }

double entropy_one(double n) { return -(xlogx(1.0 - n) + xlogx(n)); }

double entropy_two(double ni, double nj, double nn, double h) {
    const double a = nj - nn, b = ni - nn;
    const double m = 0.5 * (a + b), d = std::sqrt(0.25 * (a - b) * (a - b) + h * h);
    return -(xlogx(1.0 - ni - nj + nn) + xlogx(nn) + xlogx(m + d) + xlogx(m - d));
}

// Eigen-decomposition of the symmetric n x n row-major A (destroyed): w[k]
// and column k of V (row-major) are the k-th eigenpair, unsorted.
static void jacobi_eigh(std::vector<double>& A, int n, std::vector<double>& w, std::vector<double>& V) {
    V.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    double fro = 0.0;
    for (double x : A) fro += x * x;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += A[(size_t)p * n + q] * A[(size_t)p * n + q];
        if (!(off > 1e-32 * fro)) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[(size_t)p * n + q];
                if (apq == 0.0) continue;
                const double tau = (A[(size_t)q * n + q] - A[(size_t)p * n + p]) / (2.0 * apq);
                const double t = tau >= 0.0 ? 1.0 / (tau + std::sqrt(1.0 + tau * tau))
                                            : -1.0 / (-tau + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                for (int k = 0; k < n; ++k) {   // A <- A J (columns p, q)
                    const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = c * akp - s * akq;
                    A[(size_t)k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {   // A <- J^T A (rows p, q)
                    const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                    A[(size_t)p * n + k] = c * apk - s * aqk;
                    A[(size_t)q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {   // V <- V J
                    const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = c * vkp - s * vkq;
                    V[(size_t)k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    w.resize(n);
    for (int i = 0; i < n; ++i) w[i] = A[(size_t)i * n + i];
}

bool fiedler_ordering(const double* I, int n, int32_t* ordering, double* fiedler_value) {
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) {
            const double a = I[(size_t)i * n + k], b = I[(size_t)k * n + i];
            if (!std::isfinite(a) || a != b) return false;
        }
    if (n == 1) {
        ordering[0] = 0;
        if (fiedler_value) *fiedler_value = 0.0;
        return true;
    }
    // L = diag(row sums) - I (the diagonal of I does not enter)
    std::vector<double> L((size_t)n * n);
    for (int i = 0; i < n; ++i) {
        double d = 0.0;
        for (int k = 0; k < n; ++k)
            if (k != i) {
                d += I[(size_t)i * n + k];
                L[(size_t)i * n + k] = -I[(size_t)i * n + k];
            }
        L[(size_t)i * n + i] = d;
    }
    std::vector<double> w, V;
    jacobi_eigh(L, n, w, V);
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return w[a] < w[b]; });
    const int k = idx[1];
    std::vector<double> f(n);
    double big = 0.0;
    for (int i = 0; i < n; ++i) {
        f[i] = V[(size_t)i * n + k];
        big = std::max(big, std::fabs(f[i]));
    }
    for (int i = 0; i < n; ++i)
        if (std::fabs(f[i]) > 1e-9 * big) {
            if (f[i] > 0.0)
                for (double& x : f) x = -x;
            break;
        }
    // components within 1e-10 of the largest magnitude are ties, in site order
    std::vector<double> key(n);
    for (int i = 0; i < n; ++i) key[i] = big > 0.0 ? std::nearbyint(f[i] / (1e-10 * big)) : 0.0;
    std::vector<int> ord(n);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return key[a] < key[b]; });
    for (int i = 0; i < n; ++i) ordering[i] = ord[i];
    if (fiedler_value) *fiedler_value = w[k];
    return true;
}

}  // namespace dm
