// Vector kernels of the host ACA updates.  Each has an AVX2 clone chosen at
// run time on CPUs that support it and a baseline x86-64 clone otherwise.
#include <complex>
#include <cstdint>

#include "aca.hpp"

#define BEM_CLONES __attribute__((target_clones("avx2", "default")))

namespace bem {

BEM_CLONES void aca_axpy(double *__restrict__ y, const double *__restrict__ x, double a, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) y[i] = y[i] - a * x[i];
}

BEM_CLONES void aca_axpy(std::complex<double> *y, const std::complex<double> *x, std::complex<double> a, int64_t n)
{
    double *__restrict__ yy = reinterpret_cast<double *>(y);
    const double *__restrict__ xx = reinterpret_cast<const double *>(x);
    const double ar = a.real(), ai = a.imag();
    for (int64_t i = 0; i < n; ++i) {
        const double xr = xx[2 * i], xi = xx[2 * i + 1];
        yy[2 * i] = yy[2 * i] - (ar * xr - ai * xi);
        yy[2 * i + 1] = yy[2 * i + 1] - (ar * xi + ai * xr);
    }
}

BEM_CLONES double aca_dot(const double *__restrict__ x, const double *__restrict__ y, int64_t n)
{
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int64_t i = 0;
    for (; i + 4 <= n; i += 4) {
        s0 += x[i] * y[i];
        s1 += x[i + 1] * y[i + 1];
        s2 += x[i + 2] * y[i + 2];
        s3 += x[i + 3] * y[i + 3];
    }
    for (; i < n; ++i) s0 += x[i] * y[i];
    return (s0 + s1) + (s2 + s3);
}

BEM_CLONES std::complex<double> aca_dot(const std::complex<double> *x, const std::complex<double> *y, int64_t n)
{
    const double *__restrict__ xx = reinterpret_cast<const double *>(x);
    const double *__restrict__ yy = reinterpret_cast<const double *>(y);
    double re0 = 0.0, im0 = 0.0, re1 = 0.0, im1 = 0.0;
    int64_t i = 0;
    for (; i + 2 <= n; i += 2) {
        re0 += xx[2 * i] * yy[2 * i] + xx[2 * i + 1] * yy[2 * i + 1];
        im0 += xx[2 * i] * yy[2 * i + 1] - xx[2 * i + 1] * yy[2 * i];
        re1 += xx[2 * i + 2] * yy[2 * i + 2] + xx[2 * i + 3] * yy[2 * i + 3];
        im1 += xx[2 * i + 2] * yy[2 * i + 3] - xx[2 * i + 3] * yy[2 * i + 2];
    }
    for (; i < n; ++i) {
        re0 += xx[2 * i] * yy[2 * i] + xx[2 * i + 1] * yy[2 * i + 1];
        im0 += xx[2 * i] * yy[2 * i + 1] - xx[2 * i + 1] * yy[2 * i];
    }
    return {re0 + re1, im0 + im1};
}

BEM_CLONES double aca_norm2(const double *__restrict__ x, int64_t n)
{
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int64_t i = 0;
    for (; i + 4 <= n; i += 4) {
        s0 += x[i] * x[i];
        s1 += x[i + 1] * x[i + 1];
        s2 += x[i + 2] * x[i + 2];
        s3 += x[i + 3] * x[i + 3];
    }
    for (; i < n; ++i) s0 += x[i] * x[i];
    return (s0 + s1) + (s2 + s3);
}

BEM_CLONES double aca_norm2(const std::complex<double> *x, int64_t n)
{
    return aca_norm2(reinterpret_cast<const double *>(x), 2 * n);
}

}  // namespace bem
