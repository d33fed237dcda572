// Device helpers: quintic spline kernel, minimum image, neighbour traversal.
#pragma once

#include <type_traits>

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

// Kahan-compensated sum (FP32 path): the running correction c (the
// low-order part lost so far, negated) is fed back into the next term; the
// error stays within about 2 eps of the sum of the terms' magnitudes.  Plain
// sum in double.
template <typename T>
struct KSum {
    T s, c;
    __device__ __forceinline__ KSum() : s(T(0)), c(T(0)) {}
    __device__ __forceinline__ void add(T x)
    {
        const T y = x - c;
        const T t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ __forceinline__ T get() const { return s - c; }
    // adds the sum held by lane (this lane ^ o) of the wave
    __device__ __forceinline__ void merge_xor(int o)
    {
        const T so = __shfl_xor(s, o, 64), co = __shfl_xor(c, o, 64);
        add(so);
        c += co;
    }
};
template <>
struct KSum<double> {
    double s;
    __device__ __forceinline__ KSum() : s(0.0) {}
    __device__ __forceinline__ void add(double x) { s += x; }
    __device__ __forceinline__ double get() const { return s; }
    __device__ __forceinline__ void merge_xor(int o) { s += __shfl_xor(s, o, 64); }
};

// ---- geometry -------------------------------------------------------------

// Minimum image r_i - r_j on axis a: beyond +L/2 subtract L, below -L/2 add
// L (a displacement of exactly L/2 is kept).  Written as two selects so the
// pair loops do not branch; open axes have L = 0 and L/2 = +inf, leaving d
// unchanged.
__device__ __forceinline__ double mi_axis(const Grid& g, int a, double d)
{
    const double lo = d - g.mi_l[a], hi = d + g.mi_l[a];
    d = d > g.mi_h[a] ? lo : d;
    d = d < -g.mi_h[a] ? hi : d;
    return d;
}

// mi_axis on an axis whose periodicity P is known at compile time (an open
// axis leaves d as mi_axis does), and f(integral_constant<bool, px>,
// integral_constant<bool, py>) called for the grid's periodicity: one
// uniform branch outside a pair loop instead of selects in every pair.
template <bool P>
__device__ __forceinline__ double mi_axis_c(const Grid& g, int a, double d)
{
    if constexpr (P) return mi_axis(g, a, d);
    else return d;
}
template <class F>
__device__ __forceinline__ void with_periodicity(const Grid& g, F&& f)
{
    using Y = std::integral_constant<bool, true>;
    using N = std::integral_constant<bool, false>;
    if (g.periodic[0]) {
        if (g.periodic[1]) f(Y{}, Y{});
        else f(Y{}, N{});
    } else {
        if (g.periodic[1]) f(N{}, Y{});
        else f(N{}, N{});
    }
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

// Hilbert index of cell (x, y) on the 2^bits x 2^bits square.  Every aligned
// 2^Q x 2^Q block is one contiguous index range, identified by d >> 2Q, and
// consecutive indices are adjacent cells (no jumps, unlike Morton order).
__device__ __forceinline__ uint64_t hilbert_d(uint32_t x, uint32_t y, int bits)
{
    uint64_t d = 0;
    const uint32_t n1 = (bits >= 32) ? 0xffffffffu : ((1u << bits) - 1u);
    for (int b = bits - 1; b >= 0; --b) {
        const uint32_t s = 1u << b;
        const uint32_t rx = (x & s) ? 1u : 0u, ry = (y & s) ? 1u : 0u;
        d += (uint64_t)s * s * ((3u * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) {
                x = n1 - x;
                y = n1 - y;
            }
            const uint32_t t = x;
            x = y;
            y = t;
        }
    }
    return d;
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

// Cell intervals (resolution Q) covering [x - R, x + R] on axis a: n (1 or
// 2) disjoint intervals [a0, b0], [a1, b1].  Every interval lies in
// [0, nq - 1] for any input, NaN and far-out positions included (those only
// cost time).
struct Span {
    int n, a0, b0, a1, b1;
};

__device__ __forceinline__ Span axis_span(const Grid& g, int a, double x, double R, int Q)
{
    const int nx0 = g.nx0[a];
    const int nq = g.nxq[Q][a];
    Span sp{1, 0, nq - 1, 0, -1};
    const double slack = 1e-9 * R + 1e-12 * (fabs(x) + fabs(g.org[a]) + g.cw0[a] * nx0);
    double fa = floor((x - R - slack - g.org[a]) * g.icw0[a]);
    double fb = floor((x + R + slack - g.org[a]) * g.icw0[a]);
    if (!(fa > -1e15 && fa < 1e15 && fb > -1e15 && fb < 1e15 && fb >= fa)) return sp;
    if (g.periodic[a]) {
        if (fb - fa + 1.0 >= (double)nx0) return sp;
        // shift by whole periods so that fa lies in [0, nx0)
        double sh = floor(fa / (double)nx0) * (double)nx0;
        int ka = (int)(fa - sh), kb = (int)(fb - sh);
        if (ka < 0) { kb += nx0; ka += nx0; }
        if (ka > nx0 - 1) { ka -= nx0; kb -= nx0; }
        if (kb >= nx0) {
            int A = ka >> Q, B = (kb - nx0) >> Q;
            if (A <= B + 1) return sp;
            sp.n = 2; sp.a0 = 0; sp.b0 = B; sp.a1 = A; sp.b1 = nq - 1;
            return sp;
        }
        sp.a0 = ka >> Q; sp.b0 = kb >> Q;
        return sp;
    }
    if (fa < 0.0) fa = 0.0;
    if (fb > (double)(nx0 - 1)) fb = (double)(nx0 - 1);
    if (fa > (double)(nx0 - 1)) fa = (double)(nx0 - 1);
    if (fb < 0.0) fb = 0.0;
    sp.a0 = ((int)fa) >> Q; sp.b0 = ((int)fb) >> Q;
    return sp;
}

// Distance along axis a from x to cell k of resolution Q (0 inside).  On
// open axes the first and last cells extend to infinity, because positions
// outside the box are clamped into them.
__device__ __forceinline__ double cell_gap(const Grid& g, int a, double x, int k, int Q)
{
    const int nx0 = g.nx0[a];
    const int k0 = k << Q;
    int k1 = (k + 1) << Q;
    if (k1 > nx0) k1 = nx0;
    const double lo = g.org[a] + (double)k0 * g.cw0[a];
    const double hi = g.org[a] + (double)k1 * g.cw0[a];
    if (g.periodic[a]) {
        const double d = fabs(mi_axis(g, a, x - 0.5 * (lo + hi))) - 0.5 * (hi - lo);
        return d > 0.0 ? d : 0.0;
    }
    if (x < lo && k0 > 0) return lo - x;
    if (x > hi && k1 < nx0) return x - hi;
    return 0.0;
}

__device__ __forceinline__ int key_level(const Grid& g, uint64_t key) { return (int)(key >> (2 * g.bits)); }

// Visits every j of level l with |r_i - r_j|^2 < (3 max(h_i, h_j))^2,
// calling f(js, dx, dy, r2, hj) with js the sorted position of j and
// (dx, dy) the minimum-image displacement r_i - r_j.  Level l is searched
// with radius 3 max(h_i, hmax_l) at resolution max(l, l_i); cells whose box
// misses that disk are skipped.  The predicate is evaluated in double with
// the operation order of the definition.
// With sf > 1 the radius 3 max(h_i, h_j) is scaled by sf (a superset of
// N(i), used for reusable lists); sf = 1 is the exact predicate.
template <class F>
__device__ __forceinline__ void for_each_neighbor_level(const Grid& g, const NbrView& nv,
                                                        double xi, double yi, double hi, int li,
                                                        int l, F&& f, double sf = 1.0)
{
    const double hl = __longlong_as_double((long long)nv.hmax_bits[l]);
    const double R = 3.0 * (hi > hl ? hi : hl) * sf;
    const double Rs = R * (1.0 + 1e-9) + 1e-12 * (fabs(xi) + fabs(yi) + R);
    const double Rs2 = Rs * Rs;
    const int Q = l > li ? l : li;
    const Span xr = axis_span(g, 0, xi, R, Q);
    const Span yr = axis_span(g, 1, yi, R, Q);
    const int2* tab = nv.tab + g.lbase[l] + g.cumq[Q];
    const int nq = g.nxq[Q][0];
    const int x0n = xr.b0 - xr.a0 + 1, y0n = yr.b0 - yr.a0 + 1;
    const int nxc = x0n + (xr.n == 2 ? xr.b1 - xr.a1 + 1 : 0);
    const int nyc = y0n + (yr.n == 2 ? yr.b1 - yr.a1 + 1 : 0);
    if (nxc <= 3 && nyc <= 3) {
        // at most 3 x 3 cells (the usual case): issue every table load of the
        // level before walking any run, in the same cell order as below
        int cxs[3], cys[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            cxs[k] = k < x0n ? xr.a0 + k : xr.a1 + (k - x0n);
            cys[k] = k < y0n ? yr.a0 + k : yr.a1 + (k - y0n);
        }
        int2 se[9];
#pragma unroll
        for (int ty = 0; ty < 3; ++ty) {
            const double gy = ty < nyc ? cell_gap(g, 1, yi, cys[ty], Q) : HUGE_VAL;
#pragma unroll
            for (int tx = 0; tx < 3; ++tx) {
                se[ty * 3 + tx] = make_int2(0, 0);
                if (ty < nyc && tx < nxc && gy <= Rs) {
                    const double gx = cell_gap(g, 0, xi, cxs[tx], Q);
                    if (gx * gx + gy * gy <= Rs2) se[ty * 3 + tx] = tab[(int64_t)cys[ty] * nq + cxs[tx]];
                }
            }
        }
        auto test = [&](int js, const double4& aj) __attribute__((always_inline)) {
            const double dx = mi_axis(g, 0, xi - aj.x);
            const double dy = mi_axis(g, 1, yi - aj.y);
            const double r2 = dx * dx + dy * dy;
            const double hm = hi > aj.z ? hi : aj.z;
            const double RR = (3.0 * hm) * sf;
            if (r2 < RR * RR) f(js, dx, dy, r2, aj.z);
        };
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            // runs are contiguous: four records are loaded before they are tested
            int js = se[k].x;
            for (; js + 4 <= se[k].y; js += 4) {
                double4 a[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) a[u] = nv.xyh[js + u];
#pragma unroll
                for (int u = 0; u < 4; ++u) test(js + u, a[u]);
            }
            for (; js < se[k].y; ++js) test(js, nv.xyh[js]);
        }
        return;
    }
    for (int ty = 0; ty < yr.n; ++ty) {
        const int cy0 = ty ? yr.a1 : yr.a0, cy1 = ty ? yr.b1 : yr.b0;
        for (int cy = cy0; cy <= cy1; ++cy) {
            const double gy = cell_gap(g, 1, yi, cy, Q);
            if (gy > Rs) continue;
            for (int tx = 0; tx < xr.n; ++tx) {
                const int cx0 = tx ? xr.a1 : xr.a0, cx1 = tx ? xr.b1 : xr.b0;
                for (int cx = cx0; cx <= cx1; ++cx) {
                    const double gx = cell_gap(g, 0, xi, cx, Q);
                    if (gx * gx + gy * gy > Rs2) continue;
                    const int2 se = tab[(int64_t)cy * nq + cx];
                    for (int js = se.x; js < se.y; ++js) {
                        const double4 aj = nv.xyh[js];
                const double xj = aj.x, yj = aj.y, hj = aj.z;
                        const double dx = mi_axis(g, 0, xi - xj);
                        const double dy = mi_axis(g, 1, yi - yj);
                        const double r2 = dx * dx + dy * dy;
                        const double hm = hi > hj ? hi : hj;
                        const double RR = (3.0 * hm) * sf;
                        if (r2 < RR * RR) f(js, dx, dy, r2, hj);
                    }
                }
            }
        }
    }
}

// All levels: every j with |r_i - r_j| < sf 3 max(h_i, h_j).
template <class F>
__device__ __forceinline__ void for_each_neighbor(const Grid& g, const NbrView& nv, double xi,
                                                  double yi, double hi, int li, F&& f,
                                                  double sf = 1.0)
{
    for (int l = 0; l < g.nlev; ++l) {
        if (nv.lcount[l] == 0) continue;
        for_each_neighbor_level(g, nv, xi, yi, hi, li, l, f, sf);
    }
}

// ---- the same walk shared by a group of G adjacent lanes ------------------
// The G lanes of a group (lane gl of the group, 0 <= gl < G) hold the same
// particle i and visit the same cells; within every cell run the records are
// dealt round-robin to the lanes, so a group reads consecutive records
// together and each lane tests about 1/G of the candidates.  f(js, pass, dx,
// dy, r2, hj) is called by all G lanes together (the loop bounds depend only
// on i), once per record slot: `pass` is false for a slot past the run's end
// (whose js is not a record to use) and for a record outside the support.
// pad (when given): per level, a distance added to the search radius for
// particles that moved since the build (they stay filed in their old cells).
// With an array E ext (sorted order) the walk reads ext[js] beside each
// record, before any test, and passes it to f as a seventh argument, so a
// caller that needs it for passing neighbours waits for one load, not a
// second one after its test.  NoExt: no array, f takes six arguments.
struct NoExt {};
template <int G, class E, class F>
__device__ __forceinline__ void group_walk_level_x(const Grid& g, const NbrView& nv,
                                                   const E* __restrict__ ext, double xi,
                                                   double yi, double hi, int li, int l, int gl,
                                                   F&& f, double sf,
                                                   const unsigned long long* pad = nullptr)
{
    constexpr bool HX = !std::is_same<E, NoExt>::value;
    const double hl = __longlong_as_double((long long)nv.hmax_bits[l]);
    double R = 3.0 * (hi > hl ? hi : hl) * sf;
    if (pad) R += __longlong_as_double((long long)pad[l]);
    const double Rs = R * (1.0 + 1e-9) + 1e-12 * (fabs(xi) + fabs(yi) + R);
    const double Rs2 = Rs * Rs;
    const int Q = l > li ? l : li;
    const Span xr = axis_span(g, 0, xi, R, Q);
    const Span yr = axis_span(g, 1, yi, R, Q);
    const int2* tab = nv.tab + g.lbase[l] + g.cumq[Q];
    const int nq = g.nxq[Q][0];
    auto run = [&](int2 se) __attribute__((always_inline)) {
        for (int base = se.x; base < se.y; base += 4 * G) {
            int js[4];
            double4 a[4];
            E ev[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                js[u] = base + gl + G * u;
                // a slot past the end reads the run's first record (in bounds)
                a[u] = nv.xyh[js[u] < se.y ? js[u] : se.x];
            }
            if constexpr (HX) {
#pragma unroll
                for (int u = 0; u < 4; ++u) ev[u] = ext[js[u] < se.y ? js[u] : se.x];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const double dx = mi_axis(g, 0, xi - a[u].x);
                const double dy = mi_axis(g, 1, yi - a[u].y);
                const double r2 = dx * dx + dy * dy;
                const double hm = hi > a[u].z ? hi : a[u].z;
                const double RR = (3.0 * hm) * sf;
                if constexpr (HX) f(js[u], js[u] < se.y && r2 < RR * RR, dx, dy, r2, a[u].z, ev[u]);
                else f(js[u], js[u] < se.y && r2 < RR * RR, dx, dy, r2, a[u].z);
            }
        }
    };
    const int x0n = xr.b0 - xr.a0 + 1, y0n = yr.b0 - yr.a0 + 1;
    const int nxc = x0n + (xr.n == 2 ? xr.b1 - xr.a1 + 1 : 0);
    const int nyc = y0n + (yr.n == 2 ? yr.b1 - yr.a1 + 1 : 0);
    constexpr int CPL = (16 + G - 1) / G;  // cells per lane in the batched case
    if (nxc * nyc <= 16) {
        // up to 4 x 4 cells (the usual case): the lanes of the group share
        // the cells' gap tests and table loads (cell k on lane k % G), all
        // issued before any run is walked; runs are then taken in cell order
        int2 own[CPL];
#pragma unroll
        for (int t = 0; t < CPL; ++t) {
            const int k = gl + G * t;
            own[t] = make_int2(0, 0);
            if (k < nxc * nyc) {
                const int kx = k % nxc, ky = k / nxc;
                const int cx = kx < x0n ? xr.a0 + kx : xr.a1 + (kx - x0n);
                const int cy = ky < y0n ? yr.a0 + ky : yr.a1 + (ky - y0n);
                const double gx = cell_gap(g, 0, xi, cx, Q), gy = cell_gap(g, 1, yi, cy, Q);
                if (gx * gx + gy * gy <= Rs2) own[t] = tab[(int64_t)cy * nq + cx];
            }
        }
        // The runs are walked as one sequence in cell order: candidate kk of
        // the group lies in the cell whose prefix (the lengths of the cells
        // before it) is the largest not above kk, and each lane follows its
        // candidates with a cursor over the group's cells.  A group's lanes
        // take consecutive candidates as they did run by run, so f sees the
        // same candidates in the same order, but a wave no longer steps
        // through every cell slot as long as its longest run in that slot.
        // The group's cell table sits in LDS (written and read by the
        // group's own lanes; kernels calling this run 256 threads a block).
        __shared__ int s_pre[(256 / G) * 17];
        __shared__ int s_js0[(256 / G) * 16];
        const int grp = (int)(threadIdx.x / G);
        int* const gpre = s_pre + grp * 17;
        int* const gjs0 = s_js0 + grp * 16;
        const int gb = __lane_id() & ~(G - 1);
        int carry = 0;
#pragma unroll
        for (int t = 0; t < CPL; ++t) {
            const int len = own[t].y - own[t].x;
            int incl = len;
#pragma unroll
            for (int o = 1; o < G; o <<= 1) {
                const int v = __shfl(incl, gb + (gl >= o ? gl - o : gl), 64);
                if (gl >= o) incl += v;
            }
            const int k = gl + G * t;
            if (k < 16) {
                gpre[k] = carry + incl - len;
                gjs0[k] = own[t].x - (carry + incl - len);
            }
            carry += __shfl(incl, gb + G - 1, 64);
        }
        const int tot = carry;
        if (gl == 0) gpre[16] = tot;
        __builtin_amdgcn_wave_barrier();
        int c = 0, cend = gpre[1], js0 = gjs0[0];
        // the loop specialised on the grid's periodicity (no minimum image
        // on open axes)
        with_periodicity(g, [&](auto pxc, auto pyc) __attribute__((always_inline)) {
        constexpr bool PX = decltype(pxc)::value, PY = decltype(pyc)::value;
        for (int base = 0; base < tot; base += 4 * G) {
            int js[4];
            bool ok[4];
            double4 a[4];
            E ev[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int kk = base + gl + G * u;
                ok[u] = kk < tot;
                const int kq = ok[u] ? kk : tot - 1;
                while (kq >= cend) {
                    ++c;
                    cend = gpre[c + 1];
                    js0 = gjs0[c];
                }
                js[u] = kq + js0;
                a[u] = nv.xyh[js[u]];
            }
            if constexpr (HX) {
#pragma unroll
                for (int u = 0; u < 4; ++u) ev[u] = ext[js[u]];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const double dx = mi_axis_c<PX>(g, 0, xi - a[u].x);
                const double dy = mi_axis_c<PY>(g, 1, yi - a[u].y);
                const double r2 = dx * dx + dy * dy;
                const double hm = hi > a[u].z ? hi : a[u].z;
                const double RR = (3.0 * hm) * sf;
                if constexpr (HX) f(js[u], ok[u] && r2 < RR * RR, dx, dy, r2, a[u].z, ev[u]);
                else f(js[u], ok[u] && r2 < RR * RR, dx, dy, r2, a[u].z);
            }
        }
        });
        __builtin_amdgcn_wave_barrier();
        return;
    }
    for (int ty = 0; ty < yr.n; ++ty) {
        const int cy0 = ty ? yr.a1 : yr.a0, cy1 = ty ? yr.b1 : yr.b0;
        for (int cy = cy0; cy <= cy1; ++cy) {
            const double gy = cell_gap(g, 1, yi, cy, Q);
            if (gy > Rs) continue;
            for (int tx = 0; tx < xr.n; ++tx) {
                const int cx0 = tx ? xr.a1 : xr.a0, cx1 = tx ? xr.b1 : xr.b0;
                for (int cx = cx0; cx <= cx1; ++cx) {
                    const double gx = cell_gap(g, 0, xi, cx, Q);
                    if (gx * gx + gy * gy > Rs2) continue;
                    run(tab[(int64_t)cy * nq + cx]);
                }
            }
        }
    }
}

template <int G, class F>
__device__ __forceinline__ void group_walk_level(const Grid& g, const NbrView& nv, double xi,
                                                 double yi, double hi, int li, int l, int gl,
                                                 F&& f, double sf,
                                                 const unsigned long long* pad = nullptr)
{
    group_walk_level_x<G, NoExt>(g, nv, nullptr, xi, yi, hi, li, l, gl, f, sf, pad);
}

template <int G, class F>
__device__ __forceinline__ void group_walk(const Grid& g, const NbrView& nv, double xi, double yi,
                                           double hi, int li, int gl, F&& f, double sf = 1.0,
                                           const unsigned long long* pad = nullptr)
{
    for (int l = 0; l < g.nlev; ++l) {
        if (nv.lcount[l] == 0) continue;
        group_walk_level<G>(g, nv, xi, yi, hi, li, l, gl, f, sf, pad);
    }
}

// group_walk with ext[js] read beside every record (group_walk_level_x)
template <int G, class E, class F>
__device__ __forceinline__ void group_walk_x(const Grid& g, const NbrView& nv,
                                             const E* __restrict__ ext, double xi, double yi,
                                             double hi, int li, int gl, F&& f, double sf = 1.0,
                                             const unsigned long long* pad = nullptr)
{
    for (int l = 0; l < g.nlev; ++l) {
        if (nv.lcount[l] == 0) continue;
        group_walk_level_x<G, E>(g, nv, ext, xi, yi, hi, li, l, gl, f, sf, pad);
    }
}

// Rank of this lane's `pass` among the passing lanes of its group of G
// (lanes G k .. G k + G - 1 of the wave), and the group's pass count.
template <int G>
__device__ __forceinline__ int group_rank(bool pass, int gl, int* total)
{
    const unsigned long long bal = __ballot(pass);
    const unsigned gm = (unsigned)(bal >> (__lane_id() & ~(G - 1))) & ((1u << G) - 1u);
    *total = __popc(gm);
    return __popc(gm & ((1u << gl) - 1u));
}

// Lane Q of this lane's group of G (G = 2 or 4 adjacent lanes, inside one
// quad), through a DPP quad permutation: one VALU move per dword, no LDS.
// Every lane of the quad must be active or inactive together.
template <int G, int Q>
__device__ __forceinline__ int grp_bcast_i(int v)
{
    static_assert((G == 2 || G == 4) && Q >= 0 && Q < G, "groups of 2 or 4 lanes");
    constexpr int ctrl = G == 4 ? (Q | (Q << 2) | (Q << 4) | (Q << 6))
                                : (Q | (Q << 2) | ((2 + Q) << 4) | ((2 + Q) << 6));
    return __builtin_amdgcn_mov_dpp(v, ctrl, 0xF, 0xF, true);
}
template <int G, int Q>
__device__ __forceinline__ double grp_bcast(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = grp_bcast_i<G, Q>((int)b);
    const int hi = grp_bcast_i<G, Q>((int)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// A guarded kernel stops when a kernel enqueued before it has tripped.
__device__ __forceinline__ bool guard_stop(const Guard& gd) { return gd.trip && *gd.trip < gd.seq; }
__device__ __forceinline__ void guard_trip(const Guard& gd)
{
    if (gd.trip) atomicMin(gd.trip, gd.seq);
}

// ---- XCD-aware block order -----------------------------------------------------
// Workgroups are dispatched to the 8 XCDs round-robin (XCD = blockIdx % 8),
// and each XCD has its own L2.  Renumbering so that XCD x runs a contiguous
// 1/8 of the blocks keeps each XCD on one spatial region of the sorted
// particles.  A bijection on [0, nb).
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7;
    const int x = b & 7, loc = b >> 3;
    return x < r ? x * (q + 1) + loc : r * (q + 1) + (x - r) * q + loc;
}

// ---- batched launches ------------------------------------------------------
// Simulation of block b in block map `map` (binary search over the block
// starts; b is uniform over the block, so is the result), and the block's
// index within that simulation.
__device__ __forceinline__ int batch_find(const Batch& B, int map, int b, int* local)
{
    const int32_t* st = B.bstart + map * (B.nsim + 1);
    int lo = 0, hi = B.nsim - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (st[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    *local = b - st[lo];
    return lo;
}

// Descriptor s of a batch read through the constant address space: its
// address is uniform over the block and nothing in a kernel writes it, so
// its fields are scalar loads kept in scalar registers (as a kernel
// argument's are); a copy in LDS would hold them in vector registers.
typedef __attribute__((address_space(4))) const SimDesc SimDescK;
__device__ __forceinline__ const SimDesc& batch_desc(const Batch& B, int s)
{
    return *(const SimDesc*)(SimDescK*)(B.sims + s);
}

// The neighbour view of simulation s of a batch: its own tables and
// per-level maxima and counts; the sorted arrays are the batch's.
// A simulation's level maxima and counts sit at its counter slot, which it
// keeps while resident (its place in the batch changes with the resident
// set; a simulation that keeps its structure keeps them).
__device__ __forceinline__ NbrView batch_view(NbrView nv, const SimDesc& sd, int)
{
    nv.tab += sd.toff;
    nv.hmax_bits += (int64_t)sd.slot * SPH_MAXL;
    nv.lcount += (int64_t)sd.slot * SPH_MAXL;
    return nv;
}

// ---- wave64 helpers ----------------------------------------------------------

__device__ __forceinline__ double wave_min_d(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_max_d(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_min_i(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
// Value of lane k (k wave-uniform) for every lane.
__device__ __forceinline__ double lane_bcast(double v, int k)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, k);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };

// Column-major neighbour list written by pass A and read by pass B:
// entry k of sorted particle s is idx[k * stride + s] (coalesced across a
// wave); rows longer than K fall back to the traversal.
struct NbrList {
    int32_t* idx;
    int32_t* cnt;
    int K;
    int stride;
    int32_t* flag;  // set to 1 when a row overflows K
};

// Row s of the list, four neighbours per iteration: the index and position
// loads of four neighbours are issued before any of their pair terms, so a
// wave keeps several gathers in flight.
// Rows may hold a superset of N(i) (a list built with a skin and reused
// after the particles moved); every entry is re-tested with the exact
// predicate r2 < (3 max(h_i, h_j))^2, written as r2 < max((3 h_i)^2,
// (3 h_j)^2), which is the same test because scaling and squaring round
// monotonically.
template <class F>
__device__ __forceinline__ void for_each_listed(const Grid& g, const NbrView& nv,
                                                const NbrList& nl, int s, int cnt, double xi,
                                                double yi, double hi, F&& body)
{
    const double ri3 = 3.0 * hi, ri2 = ri3 * ri3;
    auto test = [&](int js, double dx, double dy, double hj) __attribute__((always_inline)) {
        const double r2 = dx * dx + dy * dy;
        const double rj3 = 3.0 * hj;
        if (r2 < fmax(ri2, rj3 * rj3)) body(js, dx, dy, r2, hj);
    };
    int k = 0;
    for (; k + 4 <= cnt; k += 4) {
        int j[4];
        double dx[4], dy[4], hj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) j[u] = nl.idx[(int64_t)(k + u) * nl.stride + s];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            dx[u] = mi_axis(g, 0, xi - nv.xs[j[u]]);
            dy[u] = mi_axis(g, 1, yi - nv.ys[j[u]]);
            hj[u] = nv.hs[j[u]];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) test(j[u], dx[u], dy[u], hj[u]);
    }
    for (; k < cnt; ++k) {
        const int js = nl.idx[(int64_t)k * nl.stride + s];
        test(js, mi_axis(g, 0, xi - nv.xs[js]), mi_axis(g, 1, yi - nv.ys[js]), nv.hs[js]);
    }
}

// Row s of the list against the packed {x, y, h, p} records, four
// neighbours per iteration; body(js, dx, dy, r2, hj, pj).  Same exact
// predicate as for_each_listed.
template <class F>
__device__ __forceinline__ void for_each_listed_packed(const Grid& g, const double4* __restrict__ pa,
                                                       const NbrList& nl, int s, int cnt,
                                                       double xi, double yi, double hi, F&& body)
{
    const double ri3 = 3.0 * hi, ri2 = ri3 * ri3;
    auto test = [&](int js, const double4& a) __attribute__((always_inline)) {
        const double dx = mi_axis(g, 0, xi - a.x);
        const double dy = mi_axis(g, 1, yi - a.y);
        const double r2 = dx * dx + dy * dy;
        const double rj3 = 3.0 * a.z;
        if (r2 < fmax(ri2, rj3 * rj3)) body(js, dx, dy, r2, a.z, a.w);
    };
    int k = 0;
    for (; k + 4 <= cnt; k += 4) {
        int j[4];
        double4 a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) j[u] = nl.idx[(int64_t)(k + u) * nl.stride + s];
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] = pa[j[u]];
#pragma unroll
        for (int u = 0; u < 4; ++u) test(j[u], a[u]);
    }
    for (; k < cnt; ++k) {
        const int js = nl.idx[(int64_t)k * nl.stride + s];
        test(js, pa[js]);
    }
}

