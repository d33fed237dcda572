// Device helpers: quintic spline kernel, minimum image, neighbour traversal.
#pragma once

#include "sph_internal.h"

// 7 / (478 pi), the 2D normalisation of the quintic spline (eq. kernel).
#define SPH_SIGMA2 0.00466144184787978
// Inflection point of the quintic spline (section 2.1).
#define SPH_XI 0.759298480738450
#define SPH_SIN60 0.8660254037844386

// ---- quintic spline: f(q) and df/dq, q = r/h, support q < 3 ---------------

template <typename T>
__device__ __forceinline__ T p5(T a) { T a2 = a * a; return a2 * a2 * a; }
template <typename T>
__device__ __forceinline__ T p4(T a) { T a2 = a * a; return a2 * a2; }

template <typename T>
__device__ __forceinline__ T kern_f(T q)
{
    if (q >= T(3)) return T(0);
    T v = p5<T>(T(3) - q);
    if (q < T(2)) v = v - T(6) * p5<T>(T(2) - q);
    if (q < T(1)) v = v + T(15) * p5<T>(T(1) - q);
    return v;
}

template <typename T>
__device__ __forceinline__ T kern_fp(T q)
{
    if (q >= T(3)) return T(0);
    T v = T(-5) * p4<T>(T(3) - q);
    if (q < T(2)) v = v + T(30) * p4<T>(T(2) - q);
    if (q < T(1)) v = v - T(75) * p4<T>(T(1) - q);
    return v;
}

// W(r, h) and dW/dr in double, operation order fixed (bit-exact paths).
__device__ __forceinline__ double kern_w64(double r, double h)
{
    double q = r / h;
    return (SPH_SIGMA2 / (h * h)) * kern_f<double>(q);
}
__device__ __forceinline__ double kern_dw64(double r, double h)
{
    double q = r / h;
    return (SPH_SIGMA2 / (h * h)) * kern_fp<double>(q) / h;
}

// Fast reciprocal / square root per precision (FP32: hardware 1-ulp ops).
template <typename T> __device__ __forceinline__ T rcp(T x);
template <> __device__ __forceinline__ float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double rcp<double>(double x) { return 1.0 / x; }
template <typename T> __device__ __forceinline__ T fsqrt(T x);
template <> __device__ __forceinline__ float fsqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
template <> __device__ __forceinline__ double fsqrt<double>(double x) { return sqrt(x); }

// Neumaier-compensated sum (FP32 path); plain sum in double.
template <typename T>
struct CSum {
    T s, c;
    __device__ __forceinline__ CSum() : s(T(0)), c(T(0)) {}
    __device__ __forceinline__ void add(T x)
    {
        T t = s + x;
        if (fabs(s) >= fabs(x)) c += (s - t) + x;
        else c += (x - t) + s;
        s = t;
    }
    __device__ __forceinline__ T get() const { return s + c; }
};
template <>
struct CSum<double> {
    double s;
    __device__ __forceinline__ CSum() : s(0.0) {}
    __device__ __forceinline__ void add(double x) { s += x; }
    __device__ __forceinline__ double get() const { return s; }
};

// ---- geometry -------------------------------------------------------------

__device__ __forceinline__ double mi_axis(const Grid& g, int a, double d)
{
    if (g.periodic[a]) {
        if (d > g.half[a]) d = d - g.L[a];
        else if (d < -g.half[a]) d = d + g.L[a];
    }
    return d;
}

__device__ __forceinline__ double wrap_axis(const Grid& g, int a, double x)
{
    if (g.periodic[a]) {
        if (x < g.lo[a]) x = x + g.L[a];
        else if (x >= g.hi[a]) x = x - g.L[a];
        if (x >= g.hi[a] || x < g.lo[a]) x = g.lo[a];
    }
    return x;
}

__device__ __forceinline__ int level_of(const Grid& g, double h)
{
    double t = 3.0 * h;
    double c = g.cmin0;
    int l = 0;
    while (t > c && l < g.nlev - 1) {
        c *= 2.0;
        ++l;
    }
    return l;
}

__device__ __forceinline__ int cell0(const Grid& g, int a, double x)
{
    double k = floor((x - g.org[a]) / g.cw0[a]);
    if (!(k >= 0.0)) k = 0.0;
    double mx = (double)(g.nx0[a] - 1);
    if (k > mx) k = mx;
    return (int)k;
}

__device__ __forceinline__ uint64_t spread2(uint32_t v)
{
    uint64_t x = v;
    x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
    x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
    x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}
__device__ __forceinline__ uint32_t compact2(uint64_t x)
{
    x &= 0x5555555555555555ull;
    x = (x | (x >> 1)) & 0x3333333333333333ull;
    x = (x | (x >> 2)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x >> 4)) & 0x00FF00FF00FF00FFull;
    x = (x | (x >> 8)) & 0x0000FFFF0000FFFFull;
    x = (x | (x >> 16)) & 0x00000000FFFFFFFFull;
    return (uint32_t)x;
}

// Cell intervals (resolution Q) covering [x - R, x + R] on axis a.  Returns
// the number of disjoint intervals (1 or 2) written to iv[0..3].  Every
// interval lies in [0, nq - 1] for any input, NaN and far-out positions
// included (those only cost time).
__device__ __forceinline__ int axis_ranges(const Grid& g, int a, double x, double R, int Q, int* iv)
{
    const int nx0 = g.nx0[a];
    const int nq = g.nxq[Q][a];
    double slack = 1e-9 * R + 1e-12 * (fabs(x) + fabs(g.org[a]) + g.cw0[a] * nx0);
    double fa = floor((x - R - slack - g.org[a]) / g.cw0[a]);
    double fb = floor((x + R + slack - g.org[a]) / g.cw0[a]);
    if (!(fa > -1e15 && fa < 1e15 && fb > -1e15 && fb < 1e15 && fb >= fa)) {
        iv[0] = 0; iv[1] = nq - 1;
        return 1;
    }
    if (g.periodic[a]) {
        if (fb - fa + 1.0 >= (double)nx0) {
            iv[0] = 0; iv[1] = nq - 1;
            return 1;
        }
        // shift by whole periods so that fa lies in [0, nx0)
        double sh = floor(fa / (double)nx0) * (double)nx0;
        int ka = (int)(fa - sh), kb = (int)(fb - sh);
        if (ka < 0) { kb += nx0; ka += nx0; }
        if (ka > nx0 - 1) { ka -= nx0; kb -= nx0; }
        if (kb >= nx0) {
            int A = ka >> Q, B = (kb - nx0) >> Q;
            if (A <= B + 1) { iv[0] = 0; iv[1] = nq - 1; return 1; }
            iv[0] = 0; iv[1] = B; iv[2] = A; iv[3] = nq - 1;
            return 2;
        }
        iv[0] = ka >> Q; iv[1] = kb >> Q;
        return 1;
    }
    if (fa < 0.0) fa = 0.0;
    if (fb > (double)(nx0 - 1)) fb = (double)(nx0 - 1);
    if (fa > (double)(nx0 - 1)) fa = (double)(nx0 - 1);
    if (fb < 0.0) fb = 0.0;
    iv[0] = ((int)fa) >> Q; iv[1] = ((int)fb) >> Q;
    return 1;
}

__device__ __forceinline__ int key_level(const Grid& g, uint64_t key) { return (int)(key >> (2 * g.bits)); }

// Visits every j with |r_i - r_j|^2 < (3 max(h_i, h_j))^2, calling
// f(js, dx, dy, r2, hj) with js the sorted position of j and (dx, dy) the
// minimum-image displacement r_i - r_j.  The predicate is evaluated in
// double with the operation order of the definition.
template <class F>
__device__ __forceinline__ void for_each_neighbor(const Grid& g, const NbrView& nv, double xi,
                                                  double yi, double hi, int li, F&& f)
{
    for (int l = 0; l < g.nlev; ++l) {
        if (nv.lcount[l] == 0) continue;
        double hl = __longlong_as_double((long long)nv.hmax_bits[l]);
        double R = 3.0 * (hi > hl ? hi : hl);
        int Q = l > li ? l : li;
        int xv[4], yv[4];
        int nxv = axis_ranges(g, 0, xi, R, Q, xv);
        int nyv = axis_ranges(g, 1, yi, R, Q, yv);
        const int2* tab = nv.tab + g.lbase[l] + g.cumq[Q];
        const int nq = g.nxq[Q][0];
        for (int a = 0; a < nyv; ++a) {
            for (int cy = yv[2 * a]; cy <= yv[2 * a + 1]; ++cy) {
                for (int b = 0; b < nxv; ++b) {
                    for (int cx = xv[2 * b]; cx <= xv[2 * b + 1]; ++cx) {
                        int2 se = tab[(int64_t)cy * nq + cx];
                        for (int js = se.x; js < se.y; ++js) {
                            double xj = nv.xs[js], yj = nv.ys[js], hj = nv.hs[js];
                            double dx = mi_axis(g, 0, xi - xj);
                            double dy = mi_axis(g, 1, yi - yj);
                            double r2 = dx * dx + dy * dy;
                            double hm = hi > hj ? hi : hj;
                            double RR = 3.0 * hm;
                            if (r2 < RR * RR) f(js, dx, dy, r2, hj);
                        }
                    }
                }
            }
        }
    }
}
