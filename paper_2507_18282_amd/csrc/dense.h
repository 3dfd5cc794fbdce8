// Dense FP64 linear algebra on the host for the projected problems of the
// eigensolver: symmetric eigenproblems (cyclic Jacobi for small orders,
// Householder tridiagonalisation + implicit QR for large ones), Cholesky and
// triangular inverses.
#pragma once

#include <algorithm>
#include <atomic>
#include <cmath>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace ew {

// A small pool of host threads for the O(n^3) loops of the large projected
// problems: run(f) calls f(t) once on every thread t of the pool (t = 0 is the
// calling thread) and returns when all have finished.  Thread t always gets
// index t, so a caller that partitions data by t keeps each part in the same
// core's cache from call to call.
class HostPool {
public:
    explicit HostPool(int nthreads) {
        for (int t = 1; t < nthreads; ++t) workers_.emplace_back([this, t] { loop(t); });
    }
    ~HostPool() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_.store(true);
        }
        cv_.notify_all();
        for (auto& w : workers_) w.join();
    }
    int size() const { return (int)workers_.size() + 1; }
    void run(const std::function<void(int)>& f) {
        if (workers_.empty()) {
            f(0);
            return;
        }
        job_ = &f;
        remaining_.store((int)workers_.size(), std::memory_order_relaxed);
        {
            std::lock_guard<std::mutex> lk(mu_);
            gen_.fetch_add(1, std::memory_order_release);
        }
        cv_.notify_all();
        f(0);
        while (remaining_.load(std::memory_order_acquire) != 0) std::this_thread::yield();
    }
    // threads for the projected problems: the host's cores, at most 16
    static int default_threads() {
        const unsigned hc = std::thread::hardware_concurrency();
        return (int)std::max(1u, std::min(hc, 16u));
    }

private:
    // Workers poll for the next job for a while (runs come in quick
    // succession during a decomposition), then sleep on the condition variable.
    void loop(int t) {
        uint64_t seen = 0;
        for (;;) {
            uint64_t g;
            int polls = 0;
            while ((g = gen_.load(std::memory_order_acquire)) == seen && !stop_.load()) {
                if (++polls < 4096) {
                    std::this_thread::yield();
                    continue;
                }
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return stop_.load() || gen_.load() != seen; });
            }
            if (stop_.load()) return;
            seen = g;
            (*job_)(t);
            remaining_.fetch_sub(1, std::memory_order_release);
        }
    }
    std::vector<std::thread> workers_;
    std::mutex mu_;
    std::condition_variable cv_;
    const std::function<void(int)>* job_ = nullptr;
    std::atomic<int> remaining_{0};
    std::atomic<uint64_t> gen_{0};
    std::atomic<bool> stop_{false};
};

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

// Symmetric eigendecomposition A = Q diag(w) Q^T for larger orders:
// Householder reduction to tridiagonal form (Golub & Van Loan, Alg. 8.3.1),
// then implicit symmetric QR steps with the Wilkinson shift and deflation
// (Alg. 8.3.2/8.3.3).  The transform is kept transposed (row j = column j of
// Q), so every Givens rotation updates two contiguous rows.  A is overwritten.
// Returns false if the QR iteration has not converged after 30 n steps.
inline bool tridiag_eigh(Mat& A, std::vector<double>& w, Mat& Q) {
    const int n = A.n;
    HostPool pool(n >= 200 ? HostPool::default_threads() : 1);
    // [lo, hi) split into one contiguous range per pool thread (range t to thread t)
    auto split = [&](int lo, int hi, const std::function<void(int, int)>& f) {
        const int len = hi - lo;
        if (len <= 0) return;
        const int parts = pool.size();
        pool.run([&](int t) {
            const int a = lo + (int)((int64_t)len * t / parts), b = lo + (int)((int64_t)len * (t + 1) / parts);
            if (a < b) f(a, b);
        });
    };
    std::vector<double> d(n), e(n > 1 ? n - 1 : 0);
    // Householder vectors, v[k] of length n - k - 1 with leading 1, and betas
    std::vector<std::vector<double>> hv(n > 2 ? n - 2 : 0);
    std::vector<double> hb(n > 2 ? n - 2 : 0, 0.0);
    std::vector<double> p(n), wv(n);
    for (int k = 0; k + 2 < n; ++k) {
        const int len = n - k - 1;
        std::vector<double>& v = hv[k];
        v.assign(len, 0.0);
        double sig = 0.0;
        for (int i = 1; i < len; ++i) sig += A(k + 1 + i, k) * A(k + 1 + i, k);
        const double x0 = A(k + 1, k);
        v[0] = 1.0;
        for (int i = 1; i < len; ++i) v[i] = A(k + 1 + i, k);
        double beta = 0.0, alpha = x0;
        if (sig != 0.0) {
            const double mu = std::sqrt(x0 * x0 + sig);
            const double v0 = x0 <= 0.0 ? x0 - mu : -sig / (x0 + mu);
            beta = 2.0 * v0 * v0 / (sig + v0 * v0);
            for (int i = 1; i < len; ++i) v[i] /= v0;
            alpha = mu;  // (I - beta v v^T) x = mu e_1
        }
        hb[k] = beta;
        if (beta != 0.0) {
            // p = beta A22 v, w = p - (beta p^T v / 2) v, A22 -= v w^T + w v^T
            split(0, len, [&](int i0, int i1) {
                for (int i = i0; i < i1; ++i) {
                    const double* row = &A.a[(size_t)(k + 1 + i) * n + (k + 1)];
                    double s = 0.0;
                    for (int j = 0; j < len; ++j) s += row[j] * v[j];
                    p[i] = beta * s;
                }
            });
            double pv = 0.0;
            for (int i = 0; i < len; ++i) pv += p[i] * v[i];
            const double half = 0.5 * beta * pv;
            for (int i = 0; i < len; ++i) wv[i] = p[i] - half * v[i];
            split(0, len, [&](int i0, int i1) {
                for (int i = i0; i < i1; ++i) {
                    double* row = &A.a[(size_t)(k + 1 + i) * n + (k + 1)];
                    const double vi = v[i], wi = wv[i];
                    for (int j = 0; j < len; ++j) row[j] -= vi * wv[j] + wi * v[j];
                }
            });
        }
        A(k + 1, k) = A(k, k + 1) = alpha;
        for (int i = 2; i <= len; ++i) A(k + i, k) = A(k, k + i) = 0.0;
    }
    for (int i = 0; i < n; ++i) d[i] = A(i, i);
    for (int i = 0; i + 1 < n; ++i) e[i] = A(i + 1, i);
    // Q = H_0 H_1 ... H_{n-3} by backward accumulation, stored transposed:
    // Zt = Q^T, so H_k applied on the left of Q's trailing block is applied on
    // the right of Zt's trailing block.  Row r changes only through the H_k
    // with k < r, so each thread takes a range of rows through all k.
    Mat Zt(n, n);
    for (int i = 0; i < n; ++i) Zt(i, i) = 1.0;
    split(0, n, [&](int r0, int r1) {
        for (int k = n - 3; k >= 0; --k) {
            if (hb[k] == 0.0) continue;
            const int len = n - k - 1;
            const std::vector<double>& v = hv[k];
            // Zt[r, k+1:] -= beta (Zt[r, k+1:] . v) v for rows r >= k+1
            for (int r = std::max(r0, k + 1); r < r1; ++r) {
                double* row = &Zt.a[(size_t)r * n + (k + 1)];
                double s = 0.0;
                for (int j = 0; j < len; ++j) s += row[j] * v[j];
                s *= hb[k];
                if (s != 0.0)
                    for (int j = 0; j < len; ++j) row[j] -= s * v[j];
            }
        }
    });
    // implicit QR on (d, e); the rotations are logged, then applied to the
    // rows of Zt in one pass at the end, each thread taking a range of
    // columns through the whole log (the same operations in the same order
    // for every element, whatever the thread count)
    const double eps = 2.220446049250313e-16;
    const double tiny = 1e-300;
    struct Rot {
        int k;
        double c, s;
    };
    std::vector<Rot> log;
    log.reserve((size_t)n * 8);
    int hi = n - 1;
    int64_t steps = 0;
    while (hi > 0) {
        // deflate converged couplings at the bottom
        if (std::fabs(e[hi - 1]) <= eps * (std::fabs(d[hi - 1]) + std::fabs(d[hi])) + tiny) {
            e[hi - 1] = 0.0;
            --hi;
            continue;
        }
        int lo = hi - 1;
        while (lo > 0 && std::fabs(e[lo - 1]) > eps * (std::fabs(d[lo - 1]) + std::fabs(d[lo])) + tiny) --lo;
        if (lo > 0) e[lo - 1] = 0.0;
        if (++steps > 30 * (int64_t)n) return false;
        // Wilkinson shift from the trailing 2 x 2 block
        const double del = 0.5 * (d[hi - 1] - d[hi]);
        const double f = e[hi - 1];
        const double den = del + (del >= 0.0 ? 1.0 : -1.0) * std::hypot(del, f);
        const double mu = d[hi] - f * f / den;
        double x = d[lo] - mu, z = e[lo];
        for (int k = lo; k < hi; ++k) {
            const double r = std::hypot(x, z);
            const double c = r == 0.0 ? 1.0 : x / r, s = r == 0.0 ? 0.0 : z / r;
            if (k > lo) e[k - 1] = r;
            const double a = d[k], b = d[k + 1], g = e[k];
            d[k] = c * c * a + 2.0 * c * s * g + s * s * b;
            d[k + 1] = s * s * a - 2.0 * c * s * g + c * c * b;
            e[k] = c * s * (b - a) + (c * c - s * s) * g;
            if (k + 1 < hi) {
                z = s * e[k + 1];
                e[k + 1] *= c;
                x = e[k];
            }
            log.push_back({k, c, s});
        }
    }
    // Each thread copies its columns of Zt into a contiguous panel (rows of
    // the panel stay within a few pages, so the long rotation log runs
    // without TLB misses), applies the log, and writes its rows of Q = Zt^T.
    w = d;
    Q = Mat(n, n);
    const int nb8 = (n + 7) / 8;
    pool.run([&](int t) {
        const int parts = pool.size();
        const int j0 = std::min(n, 8 * (int)((int64_t)nb8 * t / parts));
        const int j1 = std::min(n, 8 * (int)((int64_t)nb8 * (t + 1) / parts));
        const int pw = j1 - j0;
        if (pw <= 0) return;
        std::vector<double> panel((size_t)n * pw);
        for (int r = 0; r < n; ++r)
            std::copy(&Zt.a[(size_t)r * n + j0], &Zt.a[(size_t)r * n + j1], &panel[(size_t)r * pw]);
        for (const Rot& q : log) {
            double* rk = &panel[(size_t)q.k * pw];
            double* rk1 = rk + pw;
            const double c = q.c, s = q.s;
            for (int j = 0; j < pw; ++j) {
                const double u = rk[j], v = rk1[j];
                rk[j] = c * u + s * v;
                rk1[j] = c * v - s * u;
            }
        }
        for (int i = j0; i < j1; ++i) {
            double* qrow = &Q.a[(size_t)i * n];
            for (int r = 0; r < n; ++r) qrow[r] = panel[(size_t)r * pw + (i - j0)];
        }
    });
    return true;
}

// Symmetric eigendecomposition for any order: Jacobi up to order 64 (the
// orders of the default Krylov dimensions), tridiagonal QR above; Jacobi if
// QR fails to converge.  A is overwritten.
inline void sym_eigh(Mat& A, std::vector<double>& w, Mat& Q) {
    if (A.n > 64) {
        Mat B = A;
        if (tridiag_eigh(B, w, Q)) return;
    }
    jacobi_eigh(A, w, Q);
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
    // row by row: X(i, :) = (e_i - sum_{k<i} Lc(i, k) X(k, :)) / Lc(i, i)
    const int n = Lc.n;
    Mat X(n, n);
    for (int i = 0; i < n; ++i) {
        double* xi = &X.a[(size_t)i * n];
        for (int k = 0; k < i; ++k) {
            const double l = Lc(i, k);
            const double* xk = &X.a[(size_t)k * n];
            for (int j = 0; j <= k; ++j) xi[j] -= l * xk[j];
        }
        const double inv = 1.0 / Lc(i, i);
        for (int j = 0; j < i; ++j) xi[j] *= inv;
        xi[i] = inv;
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
