// Host-side FP64 linear algebra for the coarse-space set-up: the inverse of a
// Hermitian positive definite matrix whose nonzeros lie in an envelope (each
// row i has nonzeros only in columns first[i] .. i of its lower triangle).
// The coarse matrices G = W^H W couple a subdomain's basis columns only with
// those of its neighbours, so with tiles in row-major order the envelope is
// about one row of tiles wide and the profile Cholesky factorisation and the
// column solves cost O(n^2 w) instead of O(n^3).  Plain C++ (no HIP), so the
// routine can be built and checked on its own.
#pragma once

#include <algorithm>
#include <cmath>
#include <complex>
#include <thread>
#include <vector>

namespace nosdd {

// Ginv = G^-1 for Hermitian positive definite G (n x n, row-major; only the
// lower triangle is read).  Returns false when a pivot is not positive.
// threads <= 0: one per hardware thread, at most 16.
inline bool hpd_inverse_profile(int n, const std::vector<std::complex<double>> &G,
                                std::vector<std::complex<double>> &Ginv, int threads = 0) {
    using cd = std::complex<double>;
    Ginv.assign((size_t)n * n, cd(0, 0));
    if (n == 0) return true;
    // envelope of the lower triangle
    std::vector<int> first(n);
    for (int i = 0; i < n; ++i) {
        int f = i;
        for (int j = 0; j < i; ++j)
            if (G[(size_t)i * n + j] != cd(0, 0)) {
                f = j;
                break;
            }
        first[i] = f;
    }
    // profile Cholesky G = L L^H (L keeps the envelope of G's lower triangle)
    std::vector<cd> L((size_t)n * n, cd(0, 0));
    for (int i = 0; i < n; ++i) {
        cd *Li = &L[(size_t)i * n];
        for (int j = first[i]; j < i; ++j) {
            const cd *Lj = &L[(size_t)j * n];
            cd s = G[(size_t)i * n + j];
            for (int k = std::max(first[i], first[j]); k < j; ++k) s -= Li[k] * std::conj(Lj[k]);
            Li[j] = s / Lj[j].real();
        }
        double d = G[(size_t)i * n + i].real();
        for (int k = first[i]; k < i; ++k) d -= std::norm(Li[k]);
        if (!(d > 0.0)) return false;
        Li[i] = std::sqrt(d);
    }
    // column c of G^-1: y = L^-1 e_c (zero above c), then x = L^-H y
    auto solve_columns = [&](int c0, int c1) {
        std::vector<cd> x(n);
        for (int c = c0; c < c1; ++c) {
            std::fill(x.begin(), x.end(), cd(0, 0));
            x[c] = 1.0 / L[(size_t)c * n + c].real();
            for (int i = c + 1; i < n; ++i) {
                const cd *Li = &L[(size_t)i * n];
                cd s = 0;
                for (int k = std::max(first[i], c); k < i; ++k) s += Li[k] * x[k];
                x[i] = -s / Li[i].real();
            }
            for (int k = n - 1; k >= 0; --k) {
                const cd *Lk = &L[(size_t)k * n];
                x[k] /= Lk[k].real();
                const cd xk = x[k];
                for (int i = first[k]; i < k; ++i) x[i] -= std::conj(Lk[i]) * xk;
            }
            for (int i = 0; i < n; ++i) Ginv[(size_t)i * n + c] = x[i];
        }
    };
    int nt = threads > 0 ? threads : (int)std::thread::hardware_concurrency();
    nt = std::max(1, std::min({nt, 16, n}));
    auto range = [&](int t, int &c0, int &c1) {
        c0 = (int)((long long)n * t / nt);
        c1 = (int)((long long)n * (t + 1) / nt);
    };
    std::vector<std::thread> pool;
    int started = 0;
    if (nt > 1) {
        try {
            for (int t = 0; t < nt; ++t) {
                int c0, c1;
                range(t, c0, c1);
                pool.emplace_back(solve_columns, c0, c1);
                started = t + 1;
            }
        } catch (...) {
            // no more threads: the calling thread takes the remaining columns
        }
    }
    for (int t = started; t < nt; ++t) {
        int c0, c1;
        range(t, c0, c1);
        solve_columns(c0, c1);
    }
    for (auto &th : pool) th.join();
    return true;
}

}  // namespace nosdd
