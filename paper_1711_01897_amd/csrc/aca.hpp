// Adaptive cross approximation as a resumable state machine (host, FP64).
//
// Algorithm "ACA" of Section 2.1: pick a row i_k, form the residual row
// v~ = a_{i_k,:} - sum_l (u_l)_{i_k} v_l, pick the column j_k of its largest
// modulus, scale v_k = v~ / v~_{j_k}, form the residual column
// u_k = a_{:,j_k} - sum_l (v_l)_{j_k} u_l, and repeat; the block is U V^T.
// Choices the paper leaves open:
//   * row pivots: first local row, then the unused row where |u_k| is
//     largest (ties: lowest index);
//   * a residual row with max |v~| <= zero_abs vanishes: before the first
//     pivot (k = 0) it is marked used and the lowest unused row is tried
//     next (blocks whose leading rows are zero); once k >= 1 the row was
//     chosen where the newest column u_k is largest, so a vanishing residual
//     there means the remaining rows are resolved to the entries' own noise
//     level and the approximation stops (walking the rows one request at a
//     time would spend a request per row on FP32 rounding noise);
//   * stop when ||u_k|| ||v_k|| <= tol ||S_k||_F, with ||S_k||_F updated by
//     ||S_k||^2 = ||S_{k-1}||^2 + 2 Re sum_{l<k} (u_l^H u_k)(v_l^H v_k)
//                + ||u_k||^2 ||v_k||^2,
//     or when every row is used, or k reaches min(m, n, max_rank).
// The state machine asks for one block row or column at a time, so one host
// thread can keep many blocks in flight on the device.
#pragma once

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

namespace bem {

// Vector kernels of the residual updates (defined in aca_kernels.cpp with an
// AVX2 clone selected at run time):  y -= a x,  sum conj(x) y,  sum |x|^2.
void aca_axpy(double *y, const double *x, double a, int64_t n);
void aca_axpy(std::complex<double> *y, const std::complex<double> *x, std::complex<double> a, int64_t n);
double aca_dot(const double *x, const double *y, int64_t n);
std::complex<double> aca_dot(const std::complex<double> *x, const std::complex<double> *y, int64_t n);
double aca_norm2(const double *x, int64_t n);
double aca_norm2(const std::complex<double> *x, int64_t n);

// Growable column store for U or V: the residual row or column of each step
// is formed in place as the next column, without a copy (a std::vector would
// zero or copy it), and growth does not initialise.  Elements are trivially
// copyable (double, std::complex<double>).
template <typename T>
class AcaBuf {
public:
    AcaBuf() = default;
    AcaBuf(const AcaBuf &) = delete;
    AcaBuf &operator=(const AcaBuf &) = delete;
    ~AcaBuf() { std::free(p_); }
    void clear() { n_ = 0; }
    void reserve(size_t c)
    {
        if (c <= cap_) return;
        // a new block and a copy of the elements held (realloc would copy the
        // whole old block)
        T *q = static_cast<T *>(std::malloc(c * sizeof(T)));
        if (!q) throw std::bad_alloc();
        if (n_) std::memcpy(q, p_, n_ * sizeof(T));
        std::free(p_);
        p_ = q;
        cap_ = c;
    }
    // size n, new elements uninitialised
    void resize_uninit(size_t n)
    {
        if (n > cap_) reserve(std::max(n, 2 * cap_));
        n_ = n;
    }
    size_t size() const { return n_; }
    T *data() { return p_; }
    const T *data() const { return p_; }
    T &operator[](size_t i) { return p_[i]; }
    const T &operator[](size_t i) const { return p_[i]; }

private:
    T *p_ = nullptr;
    size_t n_ = 0, cap_ = 0;
};

inline double abs2(double x) { return x * x; }
inline double abs2(const std::complex<double> &x) { return x.real() * x.real() + x.imag() * x.imag(); }
inline double re_of(double x) { return x; }
inline double re_of(const std::complex<double> &x) { return x.real(); }
inline double conj_of(double x) { return x; }
inline std::complex<double> conj_of(const std::complex<double> &x) { return std::conj(x); }

template <typename T>
struct AcaCore {
    enum Phase { NEED_ROW = 0, NEED_COL = 1, DONE = 2 };
    int64_t m = 0, n = 0;
    double tol = 1e-5, zero_abs = 0.0;
    int max_rank = 0, limit = 0;
    AcaBuf<T> U, V;        // column l of U at U[l*m], of V at V[l*n]; the current residual
                           // row is formed as column k of V, the residual column as column k of U
    std::vector<char> used;
    int64_t nused = 0;
    int k = 0;
    double norm2 = 0.0;
    int64_t i = 0, j = 0;
    Phase phase = NEED_ROW;

    void init(int64_t m_, int64_t n_, double tol_, int max_rank_, double zero_abs_)
    {
        m = m_;
        n = n_;
        tol = tol_;
        max_rank = max_rank_;
        zero_abs = zero_abs_;
        limit = (int)std::min<int64_t>(std::min<int64_t>(m, n), max_rank);
        U.clear();
        V.clear();
        U.reserve((size_t)m * 16);
        V.reserve((size_t)n * 16);
        used.assign(m, 0);
        nused = 0;
        k = 0;
        norm2 = 0.0;
        i = 0;
        j = 0;
        phase = (m > 0 && n > 0 && limit > 0) ? NEED_ROW : DONE;
    }

    // Raw block row i (length n), FP32 or FP64 entries (widened on the copy).
    template <typename In>
    void consume_row(const In *row)
    {
        const size_t base = (size_t)k * (size_t)n;
        V.resize_uninit(base + (size_t)n);
        T *v = V.data() + base;
        for (int64_t c = 0; c < n; ++c) v[c] = T(row[c]);
        for (int l = 0; l < k; ++l) aca_axpy(v, V.data() + (size_t)l * n, U[(size_t)l * m + i], n);
        if (!used[i]) {
            used[i] = 1;
            ++nused;
        }
        double amax2 = -1.0;
        int64_t jm = 0;
        for (int64_t c = 0; c < n; ++c) {
            const double a = abs2(v[c]);
            if (a > amax2) {
                amax2 = a;
                jm = c;
            }
        }
        if (!(std::sqrt(amax2) > zero_abs)) {
            V.resize_uninit(base);   // the row is not kept
            if (nused == m || k > 0) {
                phase = DONE;
                return;
            }
            for (int64_t r = 0; r < m; ++r)
                if (!used[r]) {
                    i = r;
                    break;
                }
            phase = NEED_ROW;
            return;
        }
        j = jm;
        const T f = T(1.0) / v[j];
        for (int64_t c = 0; c < n; ++c) v[c] = v[c] * f;
        phase = NEED_COL;
    }

    // Raw block column j (length m), FP32 or FP64 entries.
    template <typename In>
    void consume_col(const In *col)
    {
        const size_t base = (size_t)k * (size_t)m;
        U.resize_uninit(base + (size_t)m);
        T *u = U.data() + base;
        const T *v = V.data() + (size_t)k * n;   // the scaled residual row of this step
        for (int64_t r = 0; r < m; ++r) u[r] = T(col[r]);
        for (int l = 0; l < k; ++l) aca_axpy(u, U.data() + (size_t)l * m, V[(size_t)l * n + j], m);
        double cross = 0.0;
        for (int l = 0; l < k; ++l) {
            const T du = aca_dot(U.data() + (size_t)l * m, u, m);
            const T dv = aca_dot(V.data() + (size_t)l * n, v, n);
            cross += re_of(du * dv);
        }
        const double su = aca_norm2(u, m), sv = aca_norm2(v, n);
        const double nu = std::sqrt(su), nv = std::sqrt(sv);
        norm2 = norm2 + 2.0 * cross + (nu * nv) * (nu * nv);
        ++k;   // u and v are column k - 1 of U and V
        if (nu * nv <= tol * std::sqrt(std::max(norm2, 0.0))) {
            phase = DONE;
            return;
        }
        if (nused == m || k >= limit) {
            phase = DONE;
            return;
        }
        double best = -1.0;
        int64_t ib = 0;
        for (int64_t r = 0; r < m; ++r) {
            if (used[r]) continue;
            const double a = abs2(u[r]);
            if (a > best) {
                best = a;
                ib = r;
            }
        }
        i = ib;
        phase = NEED_ROW;
    }
};

}  // namespace bem
