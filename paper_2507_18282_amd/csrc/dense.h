// Small dense FP64 linear algebra on the host (matrices of order <= a few
// hundred): cyclic Jacobi for symmetric eigenproblems and Cholesky.
#pragma once

#include <algorithm>
#include <cmath>
#include <vector>

namespace ew {

// Row-major n x n matrix helper.
struct Mat {
    int n = 0, m = 0;
    std::vector<double> a;
    Mat() = default;
    Mat(int rows, int cols) : n(rows), m(cols), a((size_t)rows * cols, 0.0) {}
    double& operator()(int i, int j) { return a[(size_t)i * m + j]; }
    double operator()(int i, int j) const { return a[(size_t)i * m + j]; }
};

// Symmetric eigendecomposition A = Q diag(w) Q^T by cyclic Jacobi rotations
// (Golub & Van Loan, Alg. 8.5.3 with the threshold strategy).  A is
// overwritten; columns of Q are the eigenvectors.
inline void jacobi_eigh(Mat& A, std::vector<double>& w, Mat& Q) {
    const int n = A.n;
    Q = Mat(n, n);
    for (int i = 0; i < n; ++i) Q(i, i) = 1.0;
    double fro = 0.0;
    for (double v : A.a) fro += v * v;
    fro = std::sqrt(fro);
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) off += A(i, j) * A(i, j);
        if (std::sqrt(off) <= 1e-17 * fro || off == 0.0) break;
        for (int p = 0; p < n; ++p) {
            for (int q = p + 1; q < n; ++q) {
                const double apq = A(p, q);
                if (apq == 0.0) continue;
                const double app = A(p, p), aqq = A(q, q);
                const double tau = (aqq - app) / (2.0 * apq);
                const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                for (int k = 0; k < n; ++k) {
                    const double akp = A(k, p), akq = A(k, q);
                    A(k, p) = c * akp - s * akq;
                    A(k, q) = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    const double apk = A(p, k), aqk = A(q, k);
                    A(p, k) = c * apk - s * aqk;
                    A(q, k) = s * apk + c * aqk;
                }
                A(p, q) = A(q, p) = 0.0;
                for (int k = 0; k < n; ++k) {
                    const double qkp = Q(k, p), qkq = Q(k, q);
                    Q(k, p) = c * qkp - s * qkq;
                    Q(k, q) = s * qkp + c * qkq;
                }
            }
        }
    }
    w.resize(n);
    for (int i = 0; i < n; ++i) w[i] = A(i, i);
}

// Lower Cholesky factor of a symmetric positive definite matrix; false if not SPD.
inline bool cholesky(const Mat& A, Mat& Lc) {
    const int n = A.n;
    Lc = Mat(n, n);
    for (int j = 0; j < n; ++j) {
        double d = A(j, j);
        for (int k = 0; k < j; ++k) d -= Lc(j, k) * Lc(j, k);
        if (!(d > 0.0)) return false;
        Lc(j, j) = std::sqrt(d);
        for (int i = j + 1; i < n; ++i) {
            double s = A(i, j);
            for (int k = 0; k < j; ++k) s -= Lc(i, k) * Lc(j, k);
            Lc(i, j) = s / Lc(j, j);
        }
    }
    return true;
}

// Inverse of a lower-triangular matrix.
inline Mat lower_inverse(const Mat& Lc) {
    const int n = Lc.n;
    Mat X(n, n);
    for (int j = 0; j < n; ++j) {
        X(j, j) = 1.0 / Lc(j, j);
        for (int i = j + 1; i < n; ++i) {
            double s = 0.0;
            for (int k = j; k < i; ++k) s += Lc(i, k) * X(k, j);
            X(i, j) = -s / Lc(i, i);
        }
    }
    return X;
}

// Indices ordering |v| descending, ties kept in input order.
inline std::vector<int> order_by_abs_desc(const std::vector<double>& v) {
    std::vector<int> idx(v.size());
    for (size_t i = 0; i < v.size(); ++i) idx[i] = (int)i;
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return std::fabs(v[x]) > std::fabs(v[y]); });
    return idx;
}

}  // namespace ew
