// dual.h -- forward-mode dual numbers (value + derivative along one
// parameter), usable on host and device.  Comparisons look at the value
// only, so every branch of the potential takes the same path as in plain
// arithmetic.
#pragma once
#include <hip/hip_runtime.h>
#include <cmath>

namespace ctbop {

struct Dual {
    double v, d;
    __host__ __device__ Dual() : v(0.0), d(0.0) {}
    __host__ __device__ Dual(double x) : v(x), d(0.0) {}
    __host__ __device__ Dual(double x, double dx) : v(x), d(dx) {}
};

__host__ __device__ inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
__host__ __device__ inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
__host__ __device__ inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
__host__ __device__ inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
__host__ __device__ inline Dual operator/(Dual a, Dual b)
{
    const double iv = 1.0 / b.v;
    return Dual(a.v * iv, (a.d - a.v * iv * b.d) * iv);
}
__host__ __device__ inline Dual operator+(Dual a, double b) { return Dual(a.v + b, a.d); }
__host__ __device__ inline Dual operator+(double a, Dual b) { return Dual(a + b.v, b.d); }
__host__ __device__ inline Dual operator-(Dual a, double b) { return Dual(a.v - b, a.d); }
__host__ __device__ inline Dual operator-(double a, Dual b) { return Dual(a - b.v, -b.d); }
__host__ __device__ inline Dual operator*(Dual a, double b) { return Dual(a.v * b, a.d * b); }
__host__ __device__ inline Dual operator*(double a, Dual b) { return Dual(a * b.v, a * b.d); }
__host__ __device__ inline Dual operator/(Dual a, double b) { return Dual(a.v / b, a.d / b); }
__host__ __device__ inline Dual operator/(double a, Dual b)
{
    const double iv = 1.0 / b.v;
    return Dual(a * iv, -a * iv * iv * b.d);
}
__host__ __device__ inline Dual &operator+=(Dual &a, Dual b) { a = a + b; return a; }
__host__ __device__ inline Dual &operator-=(Dual &a, Dual b) { a = a - b; return a; }
__host__ __device__ inline Dual &operator*=(Dual &a, Dual b) { a = a * b; return a; }
__host__ __device__ inline Dual &operator/=(Dual &a, Dual b) { a = a / b; return a; }
__host__ __device__ inline bool operator<(Dual a, Dual b) { return a.v < b.v; }
__host__ __device__ inline bool operator>(Dual a, Dual b) { return a.v > b.v; }
__host__ __device__ inline bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
__host__ __device__ inline bool operator>=(Dual a, Dual b) { return a.v >= b.v; }
__host__ __device__ inline bool operator!=(Dual a, Dual b) { return a.v != b.v || a.d != b.d; }

__host__ __device__ inline Dual exp(Dual a)
{
    const double e = ::exp(a.v);
    return Dual(e, e * a.d);
}
__host__ __device__ inline Dual log(Dual a) { return Dual(::log(a.v), a.d / a.v); }
__host__ __device__ inline Dual sqrt(Dual a)
{
    const double s = ::sqrt(a.v);
    return Dual(s, 0.5 * a.d / s);
}
__host__ __device__ inline Dual sin(Dual a) { return Dual(::sin(a.v), ::cos(a.v) * a.d); }
__host__ __device__ inline Dual cos(Dual a) { return Dual(::cos(a.v), -::sin(a.v) * a.d); }
// a^b for a > 0 (both may carry derivatives)
__host__ __device__ inline Dual pow(Dual a, Dual b)
{
    const double p = ::pow(a.v, b.v);
    return Dual(p, p * (b.d * ::log(a.v) + b.v * a.d / a.v));
}
__host__ __device__ inline Dual pow(Dual a, double b)
{
    const double p = ::pow(a.v, b);
    return Dual(p, b * ::pow(a.v, b - 1.0) * a.d);
}

} // namespace ctbop

namespace ctbop {
__host__ __device__ inline void dev_sincos(Dual a, Dual *s, Dual *c)
{
    const double sv = ::sin(a.v), cv = ::cos(a.v);
    *s = Dual(sv, cv * a.d);
    *c = Dual(cv, -sv * a.d);
}
} // namespace ctbop
