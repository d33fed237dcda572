// Rate evaluation and time stepping on gfx950.
//
// Pass A (per particle, gather over its neighbours): summation density
// (eq. sd-gather), the variable-h correction beta (eq. beta, d = 2), the
// neighbour count and average pressure (eq. pavg) and the limited Lind
// shifting displacement (eqs. shift-deltar, shift-limit).
// Pass B: EDAC pressure rate (eq. edac:sph) and momentum (eq. mom-sph) with
// the averaged kernel gradient (eq. dw-avg), the harmonic EDAC viscosity
// (eqs. edac-alpha, nu-cleary), the pressure reduction of eq. (mom:pre) and
// the transport-velocity term u~ - u = dr/dt (eq. shift-tvf).
// Readings: the EDAC diffusion term is divided by (r^2 + eta_i) like the
// viscous term; A_i, A_j and the third line of eq. (mom-sph) are not used
// (the remark after eq. mom-corr); both P_i and P_j subtract p_avg,i.
//
// Pair arithmetic is templated on T (float or double).  Position, velocity
// and pressure differences are always formed in double and then converted.
// In float every pair sum is Kahan-compensated: density, beta, average
// pressure and shift in pass A; divergence, EDAC diffusion, pressure
// gradient and viscous term in pass B.  The neighbour predicate is always
// the double-precision one.
#include <math.h>

#include "sph_device.h"

// columns of the exact neighbour rows pass A hands to pass B
#define EX_K 160
// lanes per particle in pass A and in pass B
#define RGA 4
#define RGB 2
// pass B, FP32 kernels: exact-row entries loaded ahead per lane, and the
// minimum number of waves per SIMD their register allocation must allow
// (0: the compiler's choice)
#ifndef PB_UNROLL
#define PB_UNROLL 2
#endif
#ifndef PB_WAVES
#define PB_WAVES 4
#endif
#if PB_WAVES > 0
#define PB_ATTR __attribute__((amdgpu_waves_per_eu(PB_WAVES)))
#else
#define PB_ATTR
#endif
// pass A, FP32 kernel: the same register budget knob
#ifndef PA_WAVES
#define PA_WAVES 5
#endif
#if PA_WAVES > 0
#define PA_ATTR __attribute__((amdgpu_waves_per_eu(PA_WAVES)))
#else
#define PA_ATTR
#endif
// the same knobs for the FP64 kernels
#ifndef PB64_WAVES
#define PB64_WAVES 0
#endif
#if PB64_WAVES > 0
#define PB64_ATTR __attribute__((amdgpu_waves_per_eu(PB64_WAVES)))
#else
#define PB64_ATTR
#endif
#ifndef PA64_WAVES
#define PA64_WAVES 4
#endif
#if PA64_WAVES > 0
#define PA64_ATTR __attribute__((amdgpu_waves_per_eu(PA64_WAVES)))
#else
#define PA64_ATTR
#endif
// Pair arithmetic of the rate passes: FMA contraction is allowed inside it
// (the neighbour predicate, outside it, stays uncontracted).
#define RATES_FP_CONTRACT _Pragma("clang fp contract(fast)")

// The spline and its derivative for the rate passes, in the branch-free
// form (every bracket clamped at zero).
template <typename T>
__device__ __forceinline__ void rate_kern(T q, T& f, T& fp)
{
    if constexpr (sizeof(T) == 8) {
        RATES_FP_CONTRACT
        const T a = fmax(T(3) - q, T(0)), b = fmax(T(2) - q, T(0)), c = fmax(T(1) - q, T(0));
        const T a2 = a * a, b2 = b * b, c2 = c * c;
        const T a4 = a2 * a2, b4 = b2 * b2, c4 = c2 * c2;
        f = a4 * a - T(6) * (b4 * b) + T(15) * (c4 * c);
        fp = T(-5) * a4 + T(30) * b4 - T(75) * c4;
    } else {
        // every bracket clamped at zero and the powers shared between W
        // and W', contracted into FMAs
        RATES_FP_CONTRACT
        const T a = fmaxf(T(3) - q, T(0)), b = fmaxf(T(2) - q, T(0)), c = fmaxf(T(1) - q, T(0));
        const T a2 = a * a, b2 = b * b, c2 = c * c;
        const T a4 = a2 * a2, b4 = b2 * b2, c4 = c2 * c2;
        f = a4 * a - T(6) * (b4 * b) + T(15) * (c4 * c);
        fp = T(-5) * a4 + T(30) * b4 - T(75) * c4;
    }
}
// q = r * (1/h), rounded before the spline's brackets use it (so the
// brackets are plain subtractions, not contracted with the product)
template <typename T>
__device__ __forceinline__ T rate_q(T r, T ih)
{
    return r * ih;
}
template <typename T>
__device__ __forceinline__ T rate_kern_fp(T q)
{
    if constexpr (sizeof(T) == 8) {
        RATES_FP_CONTRACT
        const T a = fmax(T(3) - q, T(0)), b = fmax(T(2) - q, T(0)), c = fmax(T(1) - q, T(0));
        const T a2 = a * a, b2 = b * b, c2 = c * c;
        return T(-5) * (a2 * a2) + T(30) * (b2 * b2) - T(75) * (c2 * c2);
    } else {
        RATES_FP_CONTRACT
        const T a = fmaxf(T(3) - q, T(0)), b = fmaxf(T(2) - q, T(0)), c = fmaxf(T(1) - q, T(0));
        const T a2 = a * a, b2 = b * b, c2 = c * c;
        return T(-5) * (a2 * a2) + T(30) * (b2 * b2) - T(75) * (c2 * c2);
    }
}

template <typename T>
struct RatesBufs {
    T *m, *rho, *beta, *dpav, *dxs, *dys, *V, *B, *ih, *nnb;
    double *ps;     // sorted pressure (double)
};

template <typename T>
static RatesBufs<T> rbufs(sph_ctx* c)
{
    Work& w = c->w;
    RatesBufs<T> b;
    b.m = (T*)w.sc0;
    b.rho = (T*)w.sc2;
    b.beta = (T*)w.sc3;
    b.dpav = (T*)w.sc4;
    b.dxs = (T*)w.sc5;
    b.dys = (T*)w.sc6;
    b.V = (T*)w.sc7;
    b.B = (T*)w.sc8;
    b.ih = (T*)w.sc10;
    b.nnb = (T*)w.sc11;
    b.ps = w.sc1;
    return b;
}

template <typename T>
__global__ __launch_bounds__(256) void k_gather_state(int n, const int32_t* __restrict__ perm,
                                                      const double* __restrict__ u,
                                                      const double* __restrict__ v,
                                                      const double* __restrict__ p,
                                                      const int64_t* __restrict__ mq, double mass_q,
                                                      const double* __restrict__ x,
                                                      const double* __restrict__ y,
                                                      const double* __restrict__ h, double* xs,
                                                      double* ys, double* hs, double4* xyh,
                                                      double4* pa,
                                                      double2* puv, T* ms,
                                                      const double* __restrict__ ug,
                                                      const double* __restrict__ vg, double* ugs,
                                                      double* vgs, const int32_t* __restrict__ kind, Guard gd)
{
    if (guard_stop(gd)) return;
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    int i = perm[s];
    // the sorted positions too: a reused list skips the neighbour build
    const double xi = x[i], yi = y[i], hi = h[i];
    xs[s] = xi;
    ys[s] = yi;
    hs[s] = hi;
    xyh[s] = make_double4(xi, yi, hi, 0.0);
    pa[s] = make_double4(xi, yi, hi, p[i]);
    puv[s] = make_double2(u[i], v[i]);
    ms[s] = (T)((double)mq[i] * mass_q);
    if (ug) {
        // the ghost velocity of a solid (fluid, inlet and outlet: their u)
        const bool sol = kind[i] == SPH_SOLID;
        ugs[s] = sol ? ug[i] : u[i];
        vgs[s] = sol ? vg[i] : v[i];
    }
}

// Batched gather (fluid only): the packed records and masses of every
// simulation of a batch, in sorted order.
template <typename T>
__global__ __launch_bounds__(256) void k_gather_state_b(Batch B, const int32_t* __restrict__ perm,
                                                        const double* __restrict__ x,
                                                        const double* __restrict__ y,
                                                        const double* __restrict__ h,
                                                        const double* __restrict__ u,
                                                        const double* __restrict__ v,
                                                        const double* __restrict__ p,
                                                        const int64_t* __restrict__ mq,
                                                        double4* pa, double2* puv, T* ms,
                                                        double4* xyh)
{
    int lb;
    const int sid = batch_find(B, BM_P256, blockIdx.x, &lb);
    const SimDesc* d = B.sims + sid;
    const int il = lb * 256 + threadIdx.x;
    if (il >= d->n) return;
    const int s = (int)(d->off + il);
    const int i = perm[s];
    const double xi = x[i], yi = y[i], hi = h[i];
    pa[s] = make_double4(xi, yi, hi, p[i]);
    puv[s] = make_double2(u[i], v[i]);
    ms[s] = (T)((double)mq[i] * d->mass_q);
    // the sorted records of the cell walks, current also for a simulation
    // that kept its structure
    xyh[s] = make_double4(xi, yi, hi, 0.0);
}

// Rebuild flags of an evaluation.  A simulation without a list skin
// rebuilds every time; one with a skin when some particle moved by 1.5 skin
// h or more since its list was built, or changed h (the test a context
// applies to its own list; the flags of the first evaluation after
// admission are set by h = -1 at build).
__global__ void k_rebuild_init_b(Batch B, int32_t* rebuild)
{
    const int sid = blockIdx.x * blockDim.x + threadIdx.x;
    if (sid < B.nsim) rebuild[sid] = B.sims[sid].skin > 0.0 ? 0 : 1;
}

__global__ __launch_bounds__(256) void k_list_check_b(Batch B, const double* __restrict__ x,
                                                      const double* __restrict__ y,
                                                      const double* __restrict__ h,
                                                      const double* __restrict__ xref,
                                                      const double* __restrict__ yref,
                                                      const double* __restrict__ href,
                                                      int32_t* rebuild)
{
    int lb;
    const int sid = batch_find(B, BM_P256, blockIdx.x, &lb);
    const SimDesc& sd = batch_desc(B, sid);
    const int il = lb * 256 + threadIdx.x;
    if (!(sd.skin > 0.0) || il >= sd.n) return;
    const int64_t i = sd.off + il;
    const double dx = mi_axis(sd.g, 0, x[i] - xref[i]);
    const double dy = mi_axis(sd.g, 1, y[i] - yref[i]);
    const double r = (1.5 * sd.skin) * href[i];
    if (!(dx * dx + dy * dy < r * r) || h[i] != href[i]) rebuild[sid] = 1;
}

// Positions and h a rebuilt simulation's list was built at.
__global__ __launch_bounds__(256) void k_list_ref_b(Batch B, const double* __restrict__ x,
                                                    const double* __restrict__ y,
                                                    const double* __restrict__ h, double* xref,
                                                    double* yref, double* href,
                                                    const int32_t* __restrict__ rebuild)
{
    int lb;
    const int sid = batch_find(B, BM_P256, blockIdx.x, &lb);
    if (!rebuild[sid]) return;
    const SimDesc& sd = batch_desc(B, sid);
    const int il = lb * 256 + threadIdx.x;
    if (il >= sd.n) return;
    const int64_t i = sd.off + il;
    xref[i] = x[i];
    yref[i] = y[i];
    href[i] = h[i];
}

// Inlet/outlet rule of the boundary pass: mode, reference state, rho0 c.
struct IoRule {
    int mode;
    double ur, vr, pr, z;
};

struct PassAOut {
    double *rho, *beta, *pavg, *nnb, *dxs, *dys; // slot order, optional
};

// Boundary pass (section 2.2).  The boundary particles (non-fluid kinds)
// are first listed by their sorted positions (order of listing is
// immaterial: each is then reduced by one wave on its own).  A boundary
// particle b sums over its fluid neighbours f, with the weights
// W(r_bf, (h_b + h_f)/2) of eq. (shepard): the Shepard averages of u, v, p
// and of rho_f (r_b - r_f), which gives the wall pressure of eq. (bc-pre)
// (g the body force, a_w the wall acceleration).  Solids keep their own
// (prescribed) velocity and get the no-slip ghost velocity 2 u_b - u^ of
// eq. (bc-wall) for the viscous term.  Inlet and outlet, rule 0: inlet
// particles get p, outlet particles get u, v and p (zero gradient).  Rule 1,
// the non-reflecting condition of Lastiwka et al.: the acoustic
// characteristic variables about the reference state (u_r, v_r, p_r),
// J2 = z (u - u_r) + (p - p_r) and J3 = -z (u - u_r) + (p - p_r) with
// z = rho0 c, are taken from the averaged fluid where they leave (J3 at the
// upstream inlet, J2 at the downstream outlet) and are 0 where they enter;
// p = p_r + (J2 + J3)/2, u = u_r + (J2 - J3)/(2z), v = v_r at the inlet and
// the average at the outlet.  Only boundary slots are written and only
// fluid slots are read, so waves do not race.
__global__ __launch_bounds__(256) void k_bmark(int n, const int32_t* __restrict__ perm,
                                               const int32_t* __restrict__ kind, int32_t* list,
                                               int32_t* count, Guard gd)
{
    if (guard_stop(gd)) return;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const bool bnd = s < n && kind[perm[s]] != SPH_FLUID;
    const uint64_t m = __ballot(bnd);
    if (m == 0ull) return;
    const int lane = __lane_id();
    int base = 0;
    if (lane == 0) base = atomicAdd(count, (int)__popcll(m));
    base = __shfl(base, 0, 64);
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    if (bnd) list[base + __popcll(m & lt)] = s;
}

__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// One wave per listed boundary particle; a fixed grid strides over the list
// (every wave leaves once the list is exhausted).
// Positions are read from the slot arrays (the sorted copies are refreshed
// later in the evaluation).  `count` was filled by k_bmark; `next_count`,
// the counter of the following evaluation, is cleared here.
__global__ __launch_bounds__(256) void k_boundary(Grid g, NbrView nv, NbrList nl, int n,
                                                  const int32_t* __restrict__ list,
                                                  const int32_t* __restrict__ count,
                                                  int32_t* next_count,
                                                  const int32_t* __restrict__ kind,
                                                  const double* __restrict__ x,
                                                  const double* __restrict__ y,
                                                  const double* __restrict__ h,
                                                  const double* __restrict__ rho, double* u,
                                                  double* v, double* p, double* ug, double* vg,
                                                  double gx, double gy, IoRule io, Guard gd)
{
    if (guard_stop(gd)) return;
    const int lane = __lane_id();
    const int nw = (gridDim.x * blockDim.x) >> 6;
    if (blockIdx.x == 0 && threadIdx.x == 0) next_count[0] = 0;
    const int total = *count;
    for (int e = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; e < total; e += nw) {
        const int s = list[e];
        const int b = nv.perm[s];
        const int kb = kind[b];
        const double xb = x[b], yb = y[b], hb = h[b];
        double S = 0.0, su = 0.0, sv = 0.0, sp = 0.0, srx = 0.0, sry = 0.0;
        auto body = [&](int js, double dx, double dy, double r2, double hj) {
            const int f = nv.perm[js];
            if (kind[f] != SPH_FLUID) return;
            const double w = kern_w64(sqrt(r2), 0.5 * (hb + hj));
            S += w;
            su += u[f] * w;
            sv += v[f] * w;
            sp += p[f] * w;
            srx += rho[f] * dx * w;
            sry += rho[f] * dy * w;
        };
        const int cnt = nl.idx ? nl.cnt[s] : nl.K + 1;
        if (cnt <= nl.K) {
            const double rb3 = 3.0 * hb, rb2 = rb3 * rb3;
            for (int k = lane; k < cnt; k += 64) {
                const int js = nl.idx[(int64_t)k * nl.stride + s];
                const int j = nv.perm[js];
                const double dx = mi_axis(g, 0, xb - x[j]);
                const double dy = mi_axis(g, 1, yb - y[j]);
                const double hj = h[j];
                const double r2 = dx * dx + dy * dy;
                const double rj3 = 3.0 * hj;
                if (r2 < fmax(rb2, rj3 * rj3)) body(js, dx, dy, r2, hj);
            }
        } else if (lane == 0) {
            // a row longer than the list: walk the cells (the sorted
            // positions are those of the last build, refreshed here)
            for_each_neighbor(g, nv, xb, yb, hb, key_level(g, nv.keys[s]),
                              [&](int js, double, double, double, double) {
                                  const int j = nv.perm[js];
                                  const double dx = mi_axis(g, 0, xb - x[j]);
                                  const double dy = mi_axis(g, 1, yb - y[j]);
                                  const double hj = h[j];
                                  const double r2 = dx * dx + dy * dy;
                                  const double rr = 3.0 * (hb > hj ? hb : hj);
                                  if (r2 < rr * rr) body(js, dx, dy, r2, hj);
                              });
        }
        S = wave_sum_d(S);
        su = wave_sum_d(su);
        sv = wave_sum_d(sv);
        sp = wave_sum_d(sp);
        srx = wave_sum_d(srx);
        sry = wave_sum_d(sry);
        if (lane != 0) continue;
        double ub = u[b], vb = v[b];
        if (S > 0.0) {
            if (kb == SPH_SOLID) {
                p[b] = (sp + (gx * srx + gy * sry)) / S;
                ug[b] = 2.0 * ub - su / S;
                vg[b] = 2.0 * vb - sv / S;
                continue;
            }
            if (io.mode == 1) {
                const double du = su / S - io.ur;
                const double dp = sp / S - io.pr;
                double pb;
                if (kb == SPH_INLET) {
                    const double j3 = dp - io.z * du;
                    ub = io.ur - j3 / (2.0 * io.z);
                    vb = io.vr;
                    pb = io.pr + 0.5 * j3;
                } else {
                    const double j2 = dp + io.z * du;
                    ub = io.ur + j2 / (2.0 * io.z);
                    vb = sv / S;
                    pb = io.pr + 0.5 * j2;
                }
                u[b] = ub;
                v[b] = vb;
                p[b] = pb;
            } else if (kb == SPH_INLET) {
                p[b] = sp / S;
            } else {
                ub = su / S;
                vb = sv / S;
                u[b] = ub;
                v[b] = vb;
                p[b] = sp / S;
            }
        }
        ug[b] = ub;
        vg[b] = vb;
    }
}

// When ex.idx is set, pass A also writes the exact neighbours of each row
// (self excluded), column-major with K columns, for pass B; a row with more
// gets count K + 1 and pass B uses the skin list (or the cell walk) for it.
// Without a list (nl.idx NULL) pass A walks the cells.
// GT: Grid for a kernel's parameter list, const Grid& for the body (a
// by-value Grid in a device function with indexed tables goes to scratch)
#define PASS_A_PARAMS_(GT, T)                                                                \
    GT g, NbrView nv, int n, RatesBufs<T> b, NbrList nl, const double4 *__restrict__ pa,     \
        typename Vec4<T>::type *pf, double rho0, PassAOut out, double *r_dxs, double *r_dys,  \
        const int32_t *__restrict__ kind, NbrList ex, Guard gd
#define PASS_A_PARAMS(T) PASS_A_PARAMS_(Grid, T)
#define PASS_A_ARGS g, nv, n, b, nl, pa, pf, rho0, out, r_dxs, r_dys, kind, ex, gd

// Sorted particle s, lane gl of its group of G lanes (all lanes of the
// group call it together).
// SP: the pair loop specialised on the grid's periodicity (one copy per
// case); the batched kernels keep one loop with the minimum image on both
// axes (a minimum image leaves an open axis unchanged).
template <typename T, int G, bool SP = true>
__device__ __forceinline__ void pass_a_body(PASS_A_PARAMS_(const Grid&, T), int s, int gl)
{
    const double4 ai = pa[s];
    const double xi = ai.x, yi = ai.y, hi = ai.z, pi = ai.w;
    const int li = key_level(g, nv.keys[s]);
    const T ih = (T)(1.0 / hi);
    const T sig = T(SPH_SIGMA2) * ih * ih;
    const T irho0 = T(1.0 / rho0);
    const T ifxi = T(1.0) / kern_f<T>(T(SPH_XI));
    // Kahan-compensated sums (error within about 2 eps of the sum of the
    // terms' magnitudes, for terms of either sign)
    KSum<T> sr, sb, sp, sx, sy;
    int nn = 0;  // |N(i)|
    // one pair's terms; r = 0 (the self pair, or coincident particles)
    // adds nothing to the shift sums
    auto terms = [&](double dx, double dy, double r2, double hj, double pj, T mj)
        __attribute__((always_inline)) {
        RATES_FP_CONTRACT
        const T r = fsqrt<T>((T)r2);
        T f, fp;
        rate_kern<T>(r * ih, f, fp);
        sr.add(mj * (sig * f));
        sb.add(mj * r * (sig * ih * fp));
        sp.add((T)(pj - pi));
        const T ihij = rcp<T>((T)(0.5 * (hi + hj)));
        T fij, fpij;
        rate_kern<T>(rate_q<T>(r, ihij), fij, fpij);
        const T wr = fij * ifxi;
        const T wr2 = wr * wr;
        const T coef = (mj * irho0) * (T(1) + T(0.24) * (wr2 * wr2));
        const T dwij = T(SPH_SIGMA2) * ihij * ihij * ihij * fpij;
        const T t = r > T(0) ? coef * dwij * rcp<T>(r) : T(0);
        sx.add(t * (T)dx);
        sy.add(t * (T)dy);
    };
    const int cnt = nl.idx ? nl.cnt[s] : nl.K + 1;
    int32_t* const exo = ex.idx;
    int ne = 0;  // exact entries of the row (the same in every lane of the group)
    // called by all lanes of the group together; `pass` marks a neighbour
    auto body = [&](int js, bool pass, double dx, double dy, double r2, double hj, double pj, T mj)
        __attribute__((always_inline)) {
        const bool ext = pass && js != s;
        int tot;
        const int k = ne + group_rank<G>(ext, gl, &tot);
        if (exo && ext && k < ex.K) exo[(int64_t)k * ex.stride + s] = js;
        ne += tot;
        if (pass) {
            ++nn;
            terms(dx, dy, r2, hj, pj, mj);
        }
    };
    if (cnt <= nl.K) {
        // the lanes of the group take every G-th entry of the row; four
        // entries' loads are issued before their tests
        const double ri3 = 3.0 * hi, ri2 = ri3 * ri3;
        auto list_loop = [&](auto pxc, auto pyc) __attribute__((always_inline)) {
            constexpr bool PX = decltype(pxc)::value, PY = decltype(pyc)::value;
            for (int base = 0; base < cnt; base += 4 * G) {
                unsigned j[4];
                double4 a[4];
                T mj[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int k = base + gl + G * u;
                    j[u] = (unsigned)(k < cnt ? nl.idx[(int64_t)k * nl.stride + s] : s);
                }
                // records and masses requested together, before any test
#pragma unroll
                for (int u = 0; u < 4; ++u) a[u] = pa[j[u]];
#pragma unroll
                for (int u = 0; u < 4; ++u) mj[u] = b.m[j[u]];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const double dx = mi_axis_c<PX>(g, 0, xi - a[u].x);
                    const double dy = mi_axis_c<PY>(g, 1, yi - a[u].y);
                    const double r2 = dx * dx + dy * dy;
                    const double rj3 = 3.0 * a[u].z;
                    const bool pass = base + gl + G * u < cnt && r2 < fmax(ri2, rj3 * rj3);
                    body((int)j[u], pass, dx, dy, r2, a[u].z, a[u].w, mj[u]);
                }
            }
        };
        if constexpr (SP) with_periodicity(g, list_loop);
        else list_loop(std::true_type{}, std::true_type{});
    } else {
        group_walk<G>(g, nv, xi, yi, hi, li, gl,
                       [&](int js, bool pass, double dx, double dy, double r2, double hj) {
                           body(js, pass, dx, dy, r2, hj, pass ? pa[js].w : 0.0,
                                pass ? b.m[js] : T(0));
                       });
    }
    if (exo && gl == 0) ex.cnt[s] = ne <= ex.K ? ne : ex.K + 1;
    // the group's partial sums, combined in every lane
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
        sr.merge_xor(o);
        sb.merge_xor(o);
        sp.merge_xor(o);
        sx.merge_xor(o);
        sy.merge_xor(o);
        nn += __shfl_xor(nn, o, 64);
    }
    if (gl) return;
    const T rho = sr.get();
    const T beta = -sb.get() / (T(2) * rho);
    const T N = (T)nn;
    const T dpav = sp.get() / N;
    const T pref = T(-0.5) * (T)(hi * hi);
    T ddx = pref * sx.get(), ddy = pref * sy.get();
    const T mag = fsqrt<T>(ddx * ddx + ddy * ddy);
    const T lim = T(0.25) * (T)hi;
    if (mag > lim) {
        const T th = lim / mag;
        ddx *= th;
        ddy *= th;
    }
    b.rho[s] = rho;
    b.beta[s] = beta;
    b.dpav[s] = dpav;
    b.dxs[s] = ddx;
    b.dys[s] = ddy;
    b.nnb[s] = N;
    // per-particle factors for pass B, packed with rho and m; the volume of
    // a solid (wall) particle is stored negated, which tells pass B to use
    // its ghost velocity in the viscous term
    const int slot = nv.perm[s];
    const T ms = b.m[s];
    const T Vs = ms / rho;
    // beta <= 0 only when no neighbour lies inside the particle's own
    // support: its pressure term is taken as zero (and so are its 1/beta sums)
    const T Bs = beta > T(0) ? T(1) / (rho * rho * beta) : T(0);
    typename Vec4<T>::type f;
    f.x = (kind && kind[slot] == SPH_SOLID) ? -Vs : Vs;
    f.y = Bs;
    f.z = rho;
    f.w = ms;
    pf[s] = f;
    r_dxs[slot] = (double)ddx;
    r_dys[slot] = (double)ddy;
    if (out.rho) out.rho[slot] = (double)rho;
    if (out.beta) out.beta[slot] = (double)beta;
    if (out.pavg) out.pavg[slot] = pi + (double)dpav;
    if (out.nnb) out.nnb[slot] = (double)nn;
    if (out.dxs) out.dxs[slot] = (double)ddx;
    if (out.dys) out.dys[slot] = (double)ddy;
}

#define PASS_A_SINGLE(T, G)                                                                  \
    if (guard_stop(gd)) return;                                                              \
    const int t = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;               \
    const int s = t / (G), gl = t % (G);                                                     \
    if (s >= n) return;                                                                      \
    pass_a_body<T, G>(PASS_A_ARGS, s, gl);

template <typename T>
__global__ __launch_bounds__(256) void k_pass_a(PASS_A_PARAMS(T))
{
    PASS_A_SINGLE(T, RGA)
}
template <>
__global__ __launch_bounds__(256) PA64_ATTR void k_pass_a<double>(PASS_A_PARAMS(double))
{
    PASS_A_SINGLE(double, RGA)
}
// FP32 schedule variants: G lanes per particle, and the minimum waves per
// SIMD W that the register allocation must allow (1: the compiler's choice;
// more waves hide more of the gathers' latency)
template <int G, int W>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W))) void k_pass_a_f(
    PASS_A_PARAMS(float))
{
    PASS_A_SINGLE(float, G)
}

// Batched pass A: every simulation of a batch (fluid only, no exact rows),
// its grid, tables and rho0 from its descriptor.
#define PASS_A_BATCH(T)                                                                      \
    int lb;                                                                                  \
    const int sid = batch_find(B, BM_P64, xcd_block(blockIdx.x, gridDim.x), &lb);            \
    const SimDesc& sd = batch_desc(B, sid);                                                  \
    const int t = lb * 256 + threadIdx.x;                                                    \
    const int sl = t / RGA, gl = t % RGA;                                                    \
    if (sl >= sd.n) return;                                                                  \
    const NbrList ex{nullptr, nullptr, EX_K, 0, nullptr};                                    \
    const Guard gd{nullptr, 0};                                                              \
    pass_a_body<T, RGA, false>(sd.g, batch_view(nv, sd, sid), 0, b, nl, pa, pf, sd.rho0, out,\
                        r_dxs, r_dys, nullptr, ex, gd, (int)(sd.off + sl), gl);

#define PASS_A_BATCH_PARAMS(T)                                                               \
    Batch B, NbrView nv, RatesBufs<T> b, NbrList nl, const double4 *__restrict__ pa,          \
        typename Vec4<T>::type *pf, PassAOut out, double *r_dxs, double *r_dys
template <typename T>
__global__ __launch_bounds__(256) void k_pass_a_b(PASS_A_BATCH_PARAMS(T));
template <>
// four waves per SIMD: at five the register budget spills the list
// addresses of the batched loop, and each list load then waits on a scratch load
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_pass_a_b<float>(
    PASS_A_BATCH_PARAMS(float))
{
    PASS_A_BATCH(float)
}
template <>
__global__ __launch_bounds__(256) PA64_ATTR void k_pass_a_b<double>(PASS_A_BATCH_PARAMS(double))
{
    PASS_A_BATCH(double)
}

struct PassBParams {
    double rho0, cs, nu, alpha_e, fx, fy, dt;
};

// GH: boundary particles present; the viscous term then takes the velocity
// difference of (ugs, vgs), which holds the ghost velocity of solids and u
// of everything else.
#define PASS_B_PARAMS_(GT, T)                                                                \
    GT g, NbrView nv, int n, RatesBufs<T> b, NbrList nl, NbrList ex,                          \
        const double4 *__restrict__ pa, const double2 *__restrict__ puv,                      \
        const typename Vec4<T>::type *__restrict__ pf, const double *__restrict__ ugs,        \
        const double *__restrict__ vgs, PassBParams P, double *dpdt, double *dudt,            \
        double *dvdt, Guard gd
#define PASS_B_PARAMS(T) PASS_B_PARAMS_(Grid, T)
#define PASS_B_ARGS g, nv, n, b, nl, ex, pa, puv, pf, ugs, vgs, P, dpdt, dudt, dvdt, gd

// Sorted particle s, lane gl of its group of G lanes; UN exact-row entries
// loaded ahead per lane.
template <typename T, bool GH, int G, int UN, bool SP = true>
__device__ __forceinline__ void pass_b_body(PASS_B_PARAMS_(const Grid&, T), int s, int gl)
{
    const double4 ai = pa[s];
    const double xi = ai.x, yi = ai.y, hi = ai.z, pi = ai.w;
    const double2 uvi = puv[s];
    const double ui = uvi.x, vi = uvi.y;
    const typename Vec4<T>::type fi4 = pf[s];
    // a negative volume marks a solid particle (ghost velocity in ugs, vgs)
    double ugi = ui, vgi = vi;
    bool solid_i = false;
    if constexpr (GH) {
        solid_i = fi4.x < T(0);
        if (solid_i) {
            ugi = ugs[s];
            vgi = vgs[s];
        }
    }
    const T ih = (T)(1.0 / hi);
    const T sigi = T(SPH_SIGMA2) * ih * ih * ih;
    const T rhoi = fi4.z;
    const T dpav = b.dpav[s];
    const T Bi = fi4.y;
    const T Pi = -dpav * Bi;
    const T aecs8 = (T)(P.alpha_e * P.cs / 8.0);
    const T nui = aecs8 * (T)hi;
    const T eta = (T)(0.001 * hi * hi);
    const T nu4 = (T)(4.0 * P.nu);
    // every pair sum is Kahan-compensated in float (the divergence, the
    // diffusion, the pressure gradient G and the viscous term all cancel
    // between neighbours; the error stays within about 2 eps of the sum of
    // the terms' magnitudes)
    KSum<T> sdiv, sdif, gx, gy, vx, vy;
    auto body = [&](int js, double dx, double dy, double r2, double hj, double pj, double2 uvj,
                    typename Vec4<T>::type fj4) __attribute__((always_inline)) {
        RATES_FP_CONTRACT
        // r and 1/r; r = 0 (the self pair, or coincident particles): every
        // term below carries a factor 1/r * r-free gradient or r itself, and
        // is zero.  In float both come from one reciprocal square root.
        T r, ir;
        if constexpr (sizeof(T) == 4) {
            const T r2f = (T)r2;
            ir = r2f > T(0) ? __builtin_amdgcn_rsqf(r2f) : T(0);
            r = r2f * ir;
        } else {
            r = fsqrt<T>((T)r2);
            ir = r > T(0) ? rcp<T>(r) : T(0);
        }
        const T ihj = rcp<T>((T)hj);
        const T dwi = sigi * rate_kern_fp<T>(r * ih);
        const T dwj = T(SPH_SIGMA2) * ihj * ihj * ihj * rate_kern_fp<T>(r * ihj);
        const T fi = dwi * ir, fj = dwj * ir;
        const T dxT = (T)dx, dyT = (T)dy;
        const T uij = (T)(ui - uvj.x), vij = (T)(vi - uvj.y);
        const T dpij = (T)(pi - pj);
        const T Vraw = fj4.x, mj = fj4.w;
        const T Vj = GH ? fabs(Vraw) : Vraw;
        const T Pj = (-dpij - dpav) * fj4.y;
        const T nuj = aecs8 * (T)hj;
        const T rdotg = T(0.5) * (dwi + dwj) * r;
        // the denominators nu_i + nu_j (harmonic EDAC viscosity), r^2 + eta
        // and rho_i + rho_j; in float from one reciprocal of their product
        T nuij_iden, cv_den;  // nu_ij / (r^2 + eta), 1 / ((rho_i + rho_j)(r^2 + eta))
        if constexpr (sizeof(T) == 4) {
            const T da = nui + nuj, db = (T)r2 + eta, dc = rhoi + fj4.z;
            const T inv = rcp<T>(da * db * dc);
            nuij_iden = T(4) * nui * nuj * (inv * dc);
            cv_den = inv * da;
        } else {
            const T iden = rcp<T>((T)r2 + eta);
            nuij_iden = T(4) * nui * nuj * rcp<T>(nui + nuj) * iden;
            cv_den = rcp<T>(rhoi + fj4.z) * iden;
        }
        sdiv.add(Vj * (fi * (uij * dxT + vij * dyT)));
        sdif.add(Vj * nuij_iden * dpij * rdotg);
        const T gf = mj * (Pi * fi + Pj * fj);
        gx.add(gf * dxT);
        gy.add(gf * dyT);
        const T cv = mj * nu4 * cv_den * rdotg;
        if constexpr (GH) {
            if (solid_i || Vraw < T(0)) {
                const double ugj = Vraw < T(0) ? ugs[js] : uvj.x;
                const double vgj = Vraw < T(0) ? vgs[js] : uvj.y;
                vx.add(cv * (T)(ugi - ugj));
                vy.add(cv * (T)(vgi - vgj));
            } else {
                vx.add(cv * uij);
                vy.add(cv * vij);
            }
        } else {
            vx.add(cv * uij);
            vy.add(cv * vij);
        }
    };
    // the body with the neighbour's velocity and factors read here
    auto body_ld = [&](int js, double dx, double dy, double r2, double hj, double pj)
        __attribute__((always_inline)) { body(js, dx, dy, r2, hj, pj, puv[js], pf[js]); };
    const int ecnt = ex.idx ? ex.cnt[s] : ex.K + 1;
    const int cnt = nl.idx ? nl.cnt[s] : nl.K + 1;
    // the lanes of the group take every G-th entry of the row
    if (ecnt <= ex.K) {
        // the exact neighbours pass A found (self excluded), UN per lane
        // loaded at a time; the next UN indices are read before this
        // chunk's terms, so their latency overlaps the gathers and the math
        int k = gl;
        auto ex_loop = [&](auto pxc, auto pyc) __attribute__((always_inline)) {
            constexpr bool PX = decltype(pxc)::value, PY = decltype(pyc)::value;
            unsigned jn[UN];
            if (k + (UN - 1) * G < ecnt) {
#pragma unroll
                for (int u = 0; u < UN; ++u)
                    jn[u] = (unsigned)ex.idx[(int64_t)(k + G * u) * ex.stride + s];
            }
            for (; k + (UN - 1) * G < ecnt; k += UN * G) {
                unsigned j[UN];
                double4 a[UN];
                double2 uv[UN];
                typename Vec4<T>::type f4[UN];
#pragma unroll
                for (int u = 0; u < UN; ++u) j[u] = jn[u];
                // every record of the chunk is requested before any is used
#pragma unroll
                for (int u = 0; u < UN; ++u) a[u] = pa[j[u]];
#pragma unroll
                for (int u = 0; u < UN; ++u) uv[u] = puv[j[u]];
#pragma unroll
                for (int u = 0; u < UN; ++u) f4[u] = pf[j[u]];
                if (k + UN * G + (UN - 1) * G < ecnt) {
#pragma unroll
                    for (int u = 0; u < UN; ++u)
                        jn[u] = (unsigned)ex.idx[(int64_t)(k + UN * G + G * u) * ex.stride + s];
                }
#pragma unroll
                for (int u = 0; u < UN; ++u) {
                    const double dx = mi_axis_c<PX>(g, 0, xi - a[u].x);
                    const double dy = mi_axis_c<PY>(g, 1, yi - a[u].y);
                    body((int)j[u], dx, dy, dx * dx + dy * dy, a[u].z, a[u].w, uv[u], f4[u]);
                }
            }
        };
        if constexpr (SP) with_periodicity(g, ex_loop);
        else ex_loop(std::true_type{}, std::true_type{});
        for (; k < ecnt; k += G) {
            const int js = ex.idx[(int64_t)k * ex.stride + s];
            const double4 a = pa[js];
            const double dx = mi_axis(g, 0, xi - a.x);
            const double dy = mi_axis(g, 1, yi - a.y);
            body_ld(js, dx, dy, dx * dx + dy * dy, a.z, a.w);
        }
    } else if (cnt <= nl.K) {
        // a list with a skin, one entry per lane at a time (a context's pass B
        // and the pool's add the same terms in the same order with this loop)
        const double ri3 = 3.0 * hi, ri2 = ri3 * ri3;
        int k = gl;
        for (; k < cnt; k += G) {
            const int js = nl.idx[(int64_t)k * nl.stride + s];
            const double4 a = pa[js];
            const double dx = mi_axis(g, 0, xi - a.x);
            const double dy = mi_axis(g, 1, yi - a.y);
            const double r2 = dx * dx + dy * dy;
            const double rj3 = 3.0 * a.z;
            if (r2 < fmax(ri2, rj3 * rj3)) body_ld(js, dx, dy, r2, a.z, a.w);
        }
    } else {
        group_walk<G>(g, nv, xi, yi, hi, key_level(g, nv.keys[s]), gl,
                       [&](int js, bool pass, double dx, double dy, double r2, double hj) {
                           if (pass) body_ld(js, dx, dy, r2, hj, pa[js].w);
                       });
    }
    // the group's partial sums, combined in every lane
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
        sdiv.merge_xor(o);
        sdif.merge_xor(o);
        gx.merge_xor(o);
        gy.merge_xor(o);
        vx.merge_xor(o);
        vy.merge_xor(o);
    }
    if (gl) return;
    const T beta = b.beta[s];
    const T ib = beta > T(0) ? T(1) / beta : T(0);
    const double dxs = (double)b.dxs[s], dys = (double)b.dys[s];
    const int slot = nv.perm[s];
    const T Gx = gx.get(), Gy = gy.get();
    dpdt[slot] = (double)((T)(P.rho0 * P.cs * P.cs) * ib * sdiv.get() + sdif.get() * ib) +
                 (dxs / P.dt) * (double)Gx + (dys / P.dt) * (double)Gy;
    dudt[slot] = (double)(-Gx + vx.get() * ib) + P.fx;
    dvdt[slot] = (double)(-Gy + vy.get() * ib) + P.fy;
}

#define PASS_B_SINGLE(T, GH, G, UN)                                                          \
    if (guard_stop(gd)) return;                                                              \
    const int t = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;               \
    const int s = t / (G), gl = t % (G);                                                     \
    if (s >= n) return;                                                                      \
    pass_b_body<T, GH, G, UN>(PASS_B_ARGS, s, gl);

template <typename T, bool GH>
__global__ __launch_bounds__(256) void k_pass_b(PASS_B_PARAMS(T))
{
    PASS_B_SINGLE(T, GH, RGB, 4)
}
template <>
__global__ __launch_bounds__(256) PB64_ATTR void k_pass_b<double, true>(PASS_B_PARAMS(double))
{
    PASS_B_SINGLE(double, true, RGB, 4)
}
template <>
__global__ __launch_bounds__(256) PB64_ATTR void k_pass_b<double, false>(PASS_B_PARAMS(double))
{
    PASS_B_SINGLE(double, false, RGB, 4)
}
// FP32 schedule variants: G lanes per particle, UN row entries loaded ahead
// per lane, at least W waves per SIMD (1: the compiler's choice)
template <bool GH, int G, int UN, int W>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W))) void k_pass_b_f(
    PASS_B_PARAMS(float))
{
    PASS_B_SINGLE(float, GH, G, UN)
}

// Batched pass B (fluid only, the list re-tested): every simulation of a
// batch, its grid, tables and constants from its descriptor.
#define PASS_B_BATCH(T)                                                                      \
    int lb;                                                                                  \
    const int sid = batch_find(B, BM_P128, xcd_block(blockIdx.x, gridDim.x), &lb);           \
    const SimDesc& sd = batch_desc(B, sid);                                                  \
    const int t = lb * 256 + threadIdx.x;                                                    \
    const int sl = t / RGB, gl = t % RGB;                                                    \
    if (sl >= sd.n) return;                                                                  \
    /* a list built with no skin is the simulation's exact rows (self        */            \
    /* included, whose terms are zero), taken in chunks without the predicate */            \
    const NbrList ex = sd.skin == 0.0 ? nl : NbrList{nullptr, nullptr, EX_K, 0, nullptr};   \
    const Guard gd{nullptr, 0};                                                              \
    const PassBParams P{sd.rho0, sd.cs, sd.nu, sd.alpha_e, sd.fx, sd.fy, sd.dt};             \
    pass_b_body<T, false, RGB, (sizeof(T) == 4 ? PB_UNROLL : 4), false>(                     \
        sd.g, batch_view(nv, sd, sid), 0, b, nl, ex, pa, puv, pf, nullptr, nullptr, P, dpdt,  \
        dudt, dvdt, gd, (int)(sd.off + sl), gl);

#define PASS_B_BATCH_PARAMS(T)                                                               \
    Batch B, NbrView nv, RatesBufs<T> b, NbrList nl, const double4 *__restrict__ pa,          \
        const double2 *__restrict__ puv, const typename Vec4<T>::type *__restrict__ pf,       \
        double *dpdt, double *dudt, double *dvdt
template <typename T>
__global__ __launch_bounds__(256) void k_pass_b_b(PASS_B_BATCH_PARAMS(T));
template <>
__global__ __launch_bounds__(256) PB_ATTR void k_pass_b_b<float>(PASS_B_BATCH_PARAMS(float))
{
    PASS_B_BATCH(float)
}
template <>
__global__ __launch_bounds__(256) PB64_ATTR void k_pass_b_b<double>(PASS_B_BATCH_PARAMS(double))
{
    PASS_B_BATCH(double)
}

// Adds the evaluation's interacting ordered pairs, sum over i of
// (|N(i)| - 1), to *acc (one atomic per block).
template <typename T>
__global__ __launch_bounds__(256) void k_count_pairs(int n, const T* __restrict__ nnb,
                                                     unsigned long long* acc, Guard gd)
{
    if (guard_stop(gd)) return;
    __shared__ int part[4];
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    int v = s < n ? (int)nnb[s] - 1 : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (__lane_id() == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0)
        atomicAdd(acc, (unsigned long long)((long long)part[0] + part[1] + part[2] + part[3]));
}

// Does the list built on (xref, yref, href) still hold N(i) for (x, y, h)?
// Not if some particle moved by 1.5 skin h_i or more (then a pair may have
// closed by 3 skin max(h_i, h_j)) or changed h; flag[0] is set then.
__global__ __launch_bounds__(256) void k_list_check(Grid g, int n, const double* __restrict__ x,
                                                    const double* __restrict__ y,
                                                    const double* __restrict__ h,
                                                    const double* __restrict__ xref,
                                                    const double* __restrict__ yref,
                                                    const double* __restrict__ href, double lim,
                                                    int32_t* flag)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double dx = mi_axis(g, 0, x[i] - xref[i]);
    const double dy = mi_axis(g, 1, y[i] - yref[i]);
    const double r = lim * href[i];
    if (!(dx * dx + dy * dy < r * r) || h[i] != href[i]) flag[0] = 1;
}

// Launches the list check of the next evaluation on (x, y, h) when a list
// is held (flag left in the list flag); returns whether it was launched.
bool launch_list_check(sph_ctx* c, int n, const double* x, const double* y, const double* h)
{
    if (!(c->list_valid && c->list_n == n && c->skin > 0 && n > 0)) return false;
    if (c->fused_x == x) {
        // the corrector that wrote x already ran the check
        c->fused_x = nullptr;
        return true;
    }
    Work& w = c->w;
    hipLaunchKernelGGL(k_list_check, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, c->stream, c->grid, n,
                       x, y, h, w.xref, w.yref, w.href, 1.5 * c->skin, w.list_flag);
    return hipGetLastError() == hipSuccess;
}

__global__ void k_clear_flag(int32_t* flag)
{
    if (threadIdx.x == 0) flag[0] = 0;
}

__global__ __launch_bounds__(256) void k_copy3(int n, const double* __restrict__ a,
                                               const double* __restrict__ b,
                                               const double* __restrict__ c, double* a2,
                                               double* b2, double* c2)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    a2[i] = a[i];
    b2[i] = b[i];
    c2[i] = c[i];
}

// Neighbour structure and list for (x, y, h): reuses the last list (only
// the sorted positions are refreshed) when it still covers every pair, else
// sorts and builds a list with a skin.
static int ensure_list(sph_ctx* c, int n, const double* x, const double* y, const double* h)
{
    Work& w = c->w;
    bool reuse = c->list_valid && c->list_n == n && c->skin > 0 && n > 0;
    unsigned nb = (unsigned)cdiv(n > 0 ? n : 1, 256);
    if (reuse && c->precheck_valid) {
        // checked on these very positions already (combined step call)
        reuse = c->precheck_ok != 0;
    } else if (reuse) {
        if (c->fused_x != x) {
            hipLaunchKernelGGL(k_list_check, dim3(nb), dim3(256), 0, c->stream, c->grid, n, x, y, h,
                               w.xref, w.yref, w.href, 1.5 * c->skin, w.list_flag);
            LAUNCHCHK(c, "list_check");
        }
        int32_t f = 1;
        const Readback rb{&f, w.list_flag, 4};
        int rc = readback(c, &rb, 1);
        if (rc) return rc;
        reuse = (f == 0);
    }
    c->precheck_valid = 0;
    c->fused_x = nullptr;
    if (reuse) {
        // the sorted positions are refreshed by the evaluation's gather
        c->list_reuses++;
        return SPH_OK;
    }
    int rc = nbr_build(c, n, x, y, h);
    if (rc || n == 0) return rc;
    hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, c->stream, w.list_flag);
    rc = nbr_build_list(c, n, c->skin);
    if (rc) return rc;
    hipLaunchKernelGGL(k_copy3, dim3(nb), dim3(256), 0, c->stream, n, x, y, h, w.xref, w.yref, w.href);
    LAUNCHCHK(c, "list_ref");
    c->list_valid = 1;
    c->list_n = n;
    c->list_builds++;
    return SPH_OK;
}

// One evaluation on (x, y, u, v, p, h, mq): neighbours, the boundary pass
// when kinds are given (it writes p, and u, v of outlet particles, of the
// boundary slots; rho_in is the stored density it reads), pass A, pass B.
// The FP32 schedule variants compiled in, by (lanes, waves) for pass A and
// (solid ghosts, lanes, unroll, waves) for pass B.
using PassAF = void (*)(PASS_A_PARAMS(float));
using PassBF = void (*)(PASS_B_PARAMS(float));

static PassAF pass_a_variant(int G, int W)
{
#define PA_V(g, w) \
    if (G == g && W == w) return k_pass_a_f<g, w>;
    PA_V(2, 1) PA_V(2, 4) PA_V(2, 5) PA_V(4, 1) PA_V(4, 4) PA_V(4, 5)
    PA_V(8, 1) PA_V(8, 4) PA_V(8, 5)
#undef PA_V
    return nullptr;
}

template <bool GH>
static PassBF pass_b_variant(int G, int U, int W)
{
#define PB_V(g, u, w) \
    if (G == g && U == u && W == w) return k_pass_b_f<GH, g, u, w>;
    PB_V(1, 2, 1) PB_V(1, 2, 4) PB_V(1, 4, 1) PB_V(1, 4, 4)
    PB_V(2, 2, 1) PB_V(2, 2, 4) PB_V(2, 4, 1) PB_V(2, 4, 4)
    PB_V(4, 2, 1) PB_V(4, 2, 4) PB_V(4, 4, 1) PB_V(4, 4, 4)
#undef PB_V
    return nullptr;
}

bool rate_schedule_valid(const sph_schedule& s)
{
    return pass_a_variant(s.a_lanes, s.a_waves) && pass_b_variant<false>(s.b_lanes, s.b_unroll, s.b_waves);
}

template <typename T>
static int eval_T(sph_ctx* c, int n, const double* x, const double* y, double* u, double* v,
                  double* p, const double* h, const int64_t* mq, const int32_t* kind,
                  const double* rho_in, double dt, PassAOut aout, double* dpdt, double* dudt,
                  double* dvdt, Guard gd)
{
    Work& w = c->w;
    // in a run of steps the caller holds a valid list; its checks run on
    // the device and trip the run when the list expires.  (A cell walk inside
    // pass A, with no list, was measured slower than the list build plus a
    // list-driven pass A: in the walk most lanes carry a rejected candidate
    // through the pair terms.)
    int rc = gd.trip ? SPH_OK : ensure_list(c, n, x, y, h);
    if (rc) return rc;
    if (n == 0) return SPH_OK;
    NbrView nv = nbr_view(c);
    RatesBufs<T> b = rbufs<T>(c);
    const sph_config& cf = c->cfg;
    unsigned nb = (unsigned)cdiv(n, 256);
    const bool gh = kind != nullptr;
    NbrList nl{w.nl_idx, w.nl_cnt, w.nl_k, n, w.list_flag};
    if (gh) {
        int32_t* blist = (int32_t*)w.ugs;  // free until the gather below fills it
        // two counters used alternately: each evaluation's boundary kernel
        // clears the other one, so no separate clearing launch is needed
        int32_t* bcount = w.status + 16 + c->bparity;
        int32_t* bnext = w.status + 16 + (c->bparity ^ 1);
        c->bparity ^= 1;
        hipLaunchKernelGGL(k_bmark, dim3(nb), dim3(256), 0, c->stream, n, (const int32_t*)nv.perm, kind,
                           blist, bcount, gd);
        const unsigned nbw = (unsigned)(nb < 512 ? nb : 512);
        hipLaunchKernelGGL(k_boundary, dim3(nbw), dim3(256), 0, c->stream, c->grid, nv, nl, n,
                           (const int32_t*)blist, (const int32_t*)bcount, bnext, kind, x, y, h,
                           rho_in, u, v, p, w.ug, w.vg, cf.body_force[0] - cf.wall_accel[0],
                           cf.body_force[1] - cf.wall_accel[1],
                           IoRule{cf.io_mode, cf.io_ref[0], cf.io_ref[1], cf.io_ref[2],
                                  cf.rho0 * cf.cs},
                           gd);
        LAUNCHCHK(c, "boundary");
    }
    using T4 = typename Vec4<T>::type;
    T4* pf = (T4*)w.pf;
    hipLaunchKernelGGL(k_gather_state<T>, dim3(nb), dim3(256), 0, c->stream, n, nv.perm, u, v, p, mq,
                       cf.mass_q, x, y, h, w.xs, w.ys, w.hs, w.xyh, w.pa, w.puv, b.m,
                       gh ? (const double*)w.ug : nullptr, gh ? (const double*)w.vg : nullptr,
                       w.ugs, w.vgs, kind, gd);
    LAUNCHCHK(c, "gather_state");
    prof_begin(c, SPH_PROF_PASS_A, &gd);
    // exact rows for pass B in the adaptation CSR buffer (free during the
    // rate passes; absent from a lean workspace)
    NbrList ex{w.col_tmp, w.cnt_ex, EX_K, n, nullptr};
    if (!w.col_tmp || !w.cnt_ex || w.col_cap < (int64_t)EX_K * n) ex.idx = nullptr;
    const sph_schedule& sc = c->sched;
    // FP32: the context's schedule; FP64: the fixed plain schedule
    const int ga = sizeof(T) == 4 ? sc.a_lanes : RGA;
    if constexpr (sizeof(T) == 4)
        hipLaunchKernelGGL(pass_a_variant(sc.a_lanes, sc.a_waves), dim3((unsigned)cdiv((int64_t)n * ga, 256)),
                           dim3(256), 0, c->stream, c->grid, nv, n, b, nl, (const double4*)w.pa, pf,
                           cf.rho0, aout, w.r_dxs, w.r_dys, kind, ex, gd);
    else
        hipLaunchKernelGGL(k_pass_a<T>, dim3((unsigned)cdiv((int64_t)n * ga, 256)), dim3(256), 0, c->stream,
                           c->grid, nv, n, b, nl, (const double4*)w.pa, pf, cf.rho0, aout, w.r_dxs,
                           w.r_dys, kind, ex, gd);
    prof_end(c, SPH_PROF_PASS_A);
    LAUNCHCHK(c, "pass_a");
    const int gb = sizeof(T) == 4 ? sc.b_lanes : RGB;
    const unsigned nbb = (unsigned)cdiv((int64_t)n * gb, 256);
    // without exact rows from pass A (a lean workspace) a list built with no
    // skin is itself the exact rows (self included, whose terms are zero):
    // pass B takes it in chunks without the predicate, as the batched pass B
    // does, so a lone simulation and a pool member add the same terms in
    // the same order
    if (!ex.idx && c->skin == 0.0 && nl.idx) ex = nl;
    PassBParams P{cf.rho0, cf.cs, cf.nu, cf.alpha_e, cf.body_force[0], cf.body_force[1], dt};
    prof_begin(c, SPH_PROF_PASS_B, &gd);
    if constexpr (sizeof(T) == 4) {
        if (gh)
            hipLaunchKernelGGL(pass_b_variant<true>(sc.b_lanes, sc.b_unroll, sc.b_waves), dim3(nbb), dim3(256),
                               0, c->stream, c->grid, nv, n, b, nl, ex, (const double4*)w.pa,
                               (const double2*)w.puv, (const T4*)pf, (const double*)w.ugs,
                               (const double*)w.vgs, P, dpdt, dudt, dvdt, gd);
        else
            hipLaunchKernelGGL(pass_b_variant<false>(sc.b_lanes, sc.b_unroll, sc.b_waves), dim3(nbb), dim3(256),
                               0, c->stream, c->grid, nv, n, b, nl, ex, (const double4*)w.pa,
                               (const double2*)w.puv, (const T4*)pf, (const double*)nullptr,
                               (const double*)nullptr, P, dpdt, dudt, dvdt, gd);
    } else {
        if (gh)
            hipLaunchKernelGGL((k_pass_b<T, true>), dim3(nbb), dim3(256), 0, c->stream, c->grid, nv, n, b, nl,
                               ex, (const double4*)w.pa, (const double2*)w.puv, (const T4*)pf,
                               (const double*)w.ugs, (const double*)w.vgs, P, dpdt, dudt, dvdt, gd);
        else
            hipLaunchKernelGGL((k_pass_b<T, false>), dim3(nbb), dim3(256), 0, c->stream, c->grid, nv, n, b, nl,
                               ex, (const double4*)w.pa, (const double2*)w.puv, (const T4*)pf,
                               (const double*)nullptr, (const double*)nullptr, P, dpdt, dudt, dvdt, gd);
    }
    prof_end(c, SPH_PROF_PASS_B);
    LAUNCHCHK(c, "pass_b");
    if (c->pair_acc) {
        hipLaunchKernelGGL(k_count_pairs<T>, dim3(nb), dim3(256), 0, c->stream, n, (const T*)b.nnb,
                           c->pair_acc, gd);
        LAUNCHCHK(c, "count_pairs");
    }
    return SPH_OK;
}

static int eval(sph_ctx* c, int n, const double* x, const double* y, double* u, double* v, double* p,
                const double* h, const int64_t* mq, const int32_t* kind, const double* rho_in,
                double dt, PassAOut aout, double* dpdt, double* dudt, double* dvdt,
                Guard gd = Guard{nullptr, 0})
{
    if (c->cfg.precision == SPH_FP32)
        return eval_T<float>(c, n, x, y, u, v, p, h, mq, kind, rho_in, dt, aout, dpdt, dudt, dvdt, gd);
    return eval_T<double>(c, n, x, y, u, v, p, h, mq, kind, rho_in, dt, aout, dpdt, dudt, dvdt, gd);
}

int rates_eval(sph_ctx* c, int n, const sph_particles* ps, double dt, const sph_rates_out* out)
{
    Work& w = c->w;
    PassAOut a{out->rho, out->beta, out->pavg, out->nnb, out->dxs, out->dys};
    int rc = eval(c, n, ps->x, ps->y, ps->u, ps->v, ps->p, ps->h, ps->mq, ps->kind, ps->rho, dt, a,
                  w.r_dpdt, w.r_dudt, w.r_dvdt);
    if (rc) return rc;
    if (n > 0) {
        if (out->dpdt)
            HIPCHK(c, hipMemcpyAsync(out->dpdt, w.r_dpdt, 8 * (size_t)n, hipMemcpyDeviceToDevice, c->stream));
        if (out->dudt)
            HIPCHK(c, hipMemcpyAsync(out->dudt, w.r_dudt, 8 * (size_t)n, hipMemcpyDeviceToDevice, c->stream));
        if (out->dvdt)
            HIPCHK(c, hipMemcpyAsync(out->dvdt, w.r_dvdt, 8 * (size_t)n, hipMemcpyDeviceToDevice, c->stream));
    }
    return SPH_OK;
}

// ---------------------------------------------------------------------------
// Predict-evaluate-correct, eqs. (int-pre) and (int-cor), in double.
// ---------------------------------------------------------------------------

// The list check of the next evaluation, fused into the kernel that writes
// its positions: flag[0] is set when particle i moved by lim h_i or more
// since the list was built, or h_i changed (flag == nullptr: no list held).
struct ListCheck {
    const double *xref, *yref, *href;
    double lim;
    int32_t* flag;
};

__device__ __forceinline__ void list_check_at(const Grid& g, const ListCheck& lc, const Guard& gd,
                                              int i, double x, double y, double h)
{
    if (!lc.flag) return;
    const double dx = mi_axis(g, 0, x - lc.xref[i]);
    const double dy = mi_axis(g, 1, y - lc.yref[i]);
    const double r = lc.lim * lc.href[i];
    if (!(dx * dx + dy * dy < r * r) || h != lc.href[i]) {
        lc.flag[0] = 1;
        guard_trip(gd);  // in a run of steps the next evaluation waits for the host
    }
}

__global__ __launch_bounds__(256) void k_predict(Grid g, int n, const int32_t* __restrict__ kind,
                                                 const double* __restrict__ x,
                                                 const double* __restrict__ y,
                                                 const double* __restrict__ u,
                                                 const double* __restrict__ v,
                                                 const double* __restrict__ p,
                                                 const double* __restrict__ ap,
                                                 const double* __restrict__ au,
                                                 const double* __restrict__ av,
                                                 const double* __restrict__ dxs,
                                                 const double* __restrict__ dys, double dt,
                                                 double* xh, double* yh, double* uh, double* vh,
                                                 double* ph, const double* __restrict__ h,
                                                 ListCheck lc, Guard gd)
{
    if (guard_stop(gd)) return;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double xn, yn;
    if (kind && kind[i] != SPH_FLUID) {
        // inlet and outlet particles move with their own velocity; solids stay
        const bool adv = kind[i] == SPH_INLET || kind[i] == SPH_OUTLET;
        xn = adv ? wrap_axis(g, 0, x[i] + 0.5 * dt * u[i]) : x[i];
        yn = adv ? wrap_axis(g, 1, y[i] + 0.5 * dt * v[i]) : y[i];
        uh[i] = u[i]; vh[i] = v[i]; ph[i] = p[i];
    } else {
        double un = u[i] + 0.5 * dt * au[i];
        double vn = v[i] + 0.5 * dt * av[i];
        double tu = un + dxs[i] / dt;
        double tv = vn + dys[i] / dt;
        xn = wrap_axis(g, 0, x[i] + 0.5 * dt * tu);
        yn = wrap_axis(g, 1, y[i] + 0.5 * dt * tv);
        uh[i] = un;
        vh[i] = vn;
        ph[i] = p[i] + 0.5 * dt * ap[i];
    }
    xh[i] = xn;
    yh[i] = yn;
    list_check_at(g, lc, gd, i, xn, yn, h[i]);
}

__global__ __launch_bounds__(256) void k_correct(Grid g, int n, const int32_t* __restrict__ kind,
                                                 double* x, double* y, double* u, double* v,
                                                 double* p, const double* __restrict__ ap,
                                                 const double* __restrict__ au,
                                                 const double* __restrict__ av,
                                                 const double* __restrict__ dxs,
                                                 const double* __restrict__ dys, double dt,
                                                 const double* __restrict__ uh,
                                                 const double* __restrict__ vh,
                                                 const double* __restrict__ ph,
                                                 const double* __restrict__ h, ListCheck lc, Guard gd)
{
    if (guard_stop(gd)) return;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double xn = x[i], yn = y[i];
    if (kind && kind[i] != SPH_FLUID) {
        // boundary particles keep the half-step boundary values; inlet and
        // outlet particles advance with the half-step velocity
        if (kind[i] == SPH_INLET || kind[i] == SPH_OUTLET) {
            xn = wrap_axis(g, 0, xn + dt * uh[i]);
            yn = wrap_axis(g, 1, yn + dt * vh[i]);
            x[i] = xn;
            y[i] = yn;
        }
        u[i] = uh[i];
        v[i] = vh[i];
        p[i] = ph[i];
    } else {
        double un = u[i] + dt * au[i];
        double vn = v[i] + dt * av[i];
        double tu = un + dxs[i] / dt;
        double tv = vn + dys[i] / dt;
        xn = wrap_axis(g, 0, xn + dt * tu);
        yn = wrap_axis(g, 1, yn + dt * tv);
        x[i] = xn;
        y[i] = yn;
        u[i] = un;
        v[i] = vn;
        p[i] = p[i] + dt * ap[i];
    }
    list_check_at(g, lc, gd, i, xn, yn, h[i]);
}

// The list check of an evaluation runs inside the kernel that writes its
// positions while a reusable list is held.
static ListCheck list_check_for(sph_ctx* c, int n)
{
    Work& w = c->w;
    const bool held = c->list_valid && c->list_n == n && c->skin > 0;
    return held ? ListCheck{w.xref, w.yref, w.href, 1.5 * c->skin, w.list_flag}
                : ListCheck{nullptr, nullptr, nullptr, 0.0, nullptr};
}

// First half of a PEC step: the evaluation at the current state, then the
// predictor (eq. int-pre).  gd1 guards the evaluation, gd2 the predictor
// (which trips the run when the list expires at the predicted positions).
int step_half1(sph_ctx* c, sph_particles* ps, double dt, Guard gd1, Guard gd2)
{
    Work& w = c->w;
    const int n = (int)ps->n;
    const unsigned nb = (unsigned)cdiv(n, 256);
    // every evaluation stores its summation density: the next boundary pass
    // reads it, and the caller gets the last one
    PassAOut withrho{ps->rho, nullptr, nullptr, nullptr, nullptr, nullptr};
    int rc = eval(c, n, ps->x, ps->y, ps->u, ps->v, ps->p, ps->h, ps->mq, ps->kind, ps->rho, dt,
                  withrho, w.r_dpdt, w.r_dudt, w.r_dvdt, gd1);
    if (rc) return rc;
    ListCheck lc = list_check_for(c, n);
    hipLaunchKernelGGL(k_predict, dim3(nb), dim3(256), 0, c->stream, c->grid, n, ps->kind, ps->x,
                       ps->y, ps->u, ps->v, ps->p, w.r_dpdt, w.r_dudt, w.r_dvdt, w.r_dxs,
                       w.r_dys, dt, w.xh, w.yh, w.uh, w.vh, w.ph, (const double*)ps->h, lc, gd2);
    LAUNCHCHK(c, "predict");
    c->fused_x = (lc.flag && !gd2.trip) ? w.xh : nullptr;
    return SPH_OK;
}

// Second half: the evaluation at the predicted state, then the corrector
// (eq. int-cor), whose list check is for the next step's first evaluation.
int step_half2(sph_ctx* c, sph_particles* ps, double dt, Guard gd3, Guard gd4)
{
    Work& w = c->w;
    const int n = (int)ps->n;
    const unsigned nb = (unsigned)cdiv(n, 256);
    PassAOut withrho{ps->rho, nullptr, nullptr, nullptr, nullptr, nullptr};
    int rc = eval(c, n, w.xh, w.yh, w.uh, w.vh, w.ph, ps->h, ps->mq, ps->kind, ps->rho, dt, withrho,
                  w.r_dpdt, w.r_dudt, w.r_dvdt, gd3);
    if (rc) return rc;
    ListCheck lc = list_check_for(c, n);
    hipLaunchKernelGGL(k_correct, dim3(nb), dim3(256), 0, c->stream, c->grid, n, ps->kind, ps->x,
                       ps->y, ps->u, ps->v, ps->p, w.r_dpdt, w.r_dudt, w.r_dvdt, w.r_dxs,
                       w.r_dys, dt, (const double*)w.uh, (const double*)w.vh,
                       (const double*)w.ph, (const double*)ps->h, lc, gd4);
    LAUNCHCHK(c, "correct");
    c->fused_x = (lc.flag && !gd4.trip) ? ps->x : nullptr;
    return SPH_OK;
}

int step_run(sph_ctx* c, sph_particles* ps, double dt, int nsteps)
{
    const int n = (int)ps->n;
    if (n == 0) return SPH_OK;
    const Guard none{nullptr, 0};
    c->fused_x = nullptr;
    for (int s = 0; s < nsteps; ++s) {
        int rc = step_half1(c, ps, dt, none, none);
        if (rc) return rc;
        rc = step_half2(c, ps, dt, none, none);
        if (rc) return rc;
    }
    return SPH_OK;
}

// ---------------------------------------------------------------------------
// Batched step: one predict-evaluate-correct step of every simulation of a
// batch (fluid only, periodic or open boxes, each with its own grid, dt and
// constants), with one launch per kernel for the whole batch.  Each
// simulation sees exactly what a lone context with a lean workspace and the
// list rebuilt at every evaluation computes: its particles are sorted within
// its own range, its tables and per-level data are its own, and every pair
// sum runs in the same order.
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(RS_THREADS) void k_count_pairs_b(Batch B, const T* __restrict__ nnb,
                                                              unsigned long long* acc)
{
    // one block per sort tile (RS_TILE particles of one simulation), so that
    // a simulation's counter takes one atomic per tile: the counters sit in
    // device memory and atomics from every XCD on one address serialise
    __shared__ int part[RS_THREADS / 64];
    int t;
    const int sid = batch_find(B, BM_TILE, blockIdx.x, &t);
    const SimDesc* d = B.sims + sid;
    const int64_t beg = (int64_t)t * RS_TILE;
    int v = 0;
#pragma unroll
    for (int k = 0; k < RS_ITEMS; ++k) {
        const int64_t il = beg + (int64_t)k * RS_THREADS + threadIdx.x;
        if (il < d->n) v += (int)nnb[d->off + il] - 1;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (__lane_id() == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long tot = 0;
#pragma unroll
        for (int w = 0; w < RS_THREADS / 64; ++w) tot += part[w];
        atomicAdd(acc + d->slot, (unsigned long long)tot);
    }
}

// Predictor (eq. int-pre) and corrector (eq. int-cor) of the batch, each
// particle with its simulation's dt and box.
__global__ __launch_bounds__(256) void k_predict_b(Batch B, const double* __restrict__ x,
                                                   const double* __restrict__ y,
                                                   const double* __restrict__ u,
                                                   const double* __restrict__ v,
                                                   const double* __restrict__ p,
                                                   const double* __restrict__ ap,
                                                   const double* __restrict__ au,
                                                   const double* __restrict__ av,
                                                   const double* __restrict__ dxs,
                                                   const double* __restrict__ dys, double* xh,
                                                   double* yh, double* uh, double* vh, double* ph)
{
    int lb;
    const int sid = batch_find(B, BM_P256, blockIdx.x, &lb);
    const SimDesc& sd = batch_desc(B, sid);
    const int il = lb * 256 + threadIdx.x;
    if (il >= sd.n) return;
    const int64_t i = sd.off + il;
    const double dt = sd.dt;
    const double un = u[i] + 0.5 * dt * au[i];
    const double vn = v[i] + 0.5 * dt * av[i];
    const double tu = un + dxs[i] / dt;
    const double tv = vn + dys[i] / dt;
    xh[i] = wrap_axis(sd.g, 0, x[i] + 0.5 * dt * tu);
    yh[i] = wrap_axis(sd.g, 1, y[i] + 0.5 * dt * tv);
    uh[i] = un;
    vh[i] = vn;
    ph[i] = p[i] + 0.5 * dt * ap[i];
}

__global__ __launch_bounds__(256) void k_correct_b(Batch B, double* x, double* y, double* u,
                                                   double* v, double* p,
                                                   const double* __restrict__ ap,
                                                   const double* __restrict__ au,
                                                   const double* __restrict__ av,
                                                   const double* __restrict__ dxs,
                                                   const double* __restrict__ dys)
{
    int lb;
    const int sid = batch_find(B, BM_P256, blockIdx.x, &lb);
    const SimDesc& sd = batch_desc(B, sid);
    const int il = lb * 256 + threadIdx.x;
    if (il >= sd.n) return;
    const int64_t i = sd.off + il;
    const double dt = sd.dt;
    const double un = u[i] + dt * au[i];
    const double vn = v[i] + dt * av[i];
    const double tu = un + dxs[i] / dt;
    const double tv = vn + dys[i] / dt;
    x[i] = wrap_axis(sd.g, 0, x[i] + dt * tu);
    y[i] = wrap_axis(sd.g, 1, y[i] + dt * tv);
    u[i] = un;
    v[i] = vn;
    p[i] = p[i] + dt * ap[i];
}

// One evaluation of the batch at (x, y, u, v, p); the summation density
// goes to b.rho (the state's), the rates to b.r_*.
template <typename T>
static int batch_eval_T(hipStream_t st, const BatchBufs& b, const BatchLaunch& L, const double* x,
                        const double* y, const double* u, const double* v, const double* p)
{
    const uint64_t* keys = nullptr;
    const int32_t* perm = nullptr;
    const unsigned nb = (unsigned)L.nblk[BM_P256];
    hipLaunchKernelGGL(k_rebuild_init_b, dim3((unsigned)cdiv(L.B.nsim, 256)), dim3(256), 0, st, L.B,
                       L.rebuild);
    hipLaunchKernelGGL(k_list_check_b, dim3(nb), dim3(256), 0, st, L.B, x, y, (const double*)b.h,
                       (const double*)b.xref, (const double*)b.yref, (const double*)b.href, L.rebuild);
    int rc = batch_build(st, b, L, x, y, b.h, &keys, &perm);
    if (rc) return rc;
    hipLaunchKernelGGL(k_list_ref_b, dim3(nb), dim3(256), 0, st, L.B, x, y, (const double*)b.h, b.xref,
                       b.yref, b.href, (const int32_t*)L.rebuild);
    RatesBufs<T> rb;
    rb.m = (T*)b.m;
    rb.rho = (T*)b.brho;
    rb.beta = (T*)b.beta;
    rb.dpav = (T*)b.dpav;
    rb.dxs = (T*)b.dxs;
    rb.dys = (T*)b.dys;
    rb.nnb = (T*)b.nnb;
    rb.V = rb.B = rb.ih = nullptr;
    rb.ps = nullptr;
    using T4 = typename Vec4<T>::type;
    hipLaunchKernelGGL(k_gather_state_b<T>, dim3((unsigned)L.nblk[BM_P256]), dim3(256), 0, st, L.B,
                       perm, x, y, b.h, u, v, p, (const int64_t*)b.mq, b.pa, b.puv, rb.m, b.xyh);
    const NbrView nv{nullptr, nullptr, nullptr, b.xyh, perm, keys, b.tab, b.hmax, b.lcount};
    const NbrList nl{b.nl_idx, b.nl_cnt, b.nl_k, (int)b.stride, b.list_flag};
    const PassAOut aout{b.rho, nullptr, nullptr, nullptr, nullptr, nullptr};
    hipLaunchKernelGGL(k_pass_a_b<T>, dim3((unsigned)L.nblk[BM_P64]), dim3(256), 0, st, L.B, nv, rb, nl,
                       (const double4*)b.pa, (T4*)b.pf, aout, b.r_dxs, b.r_dys);
    hipLaunchKernelGGL(k_pass_b_b<T>, dim3((unsigned)L.nblk[BM_P128]), dim3(256), 0, st, L.B, nv, rb,
                       nl, (const double4*)b.pa, (const double2*)b.puv, (const T4*)b.pf, b.r_dpdt,
                       b.r_dudt, b.r_dvdt);
    hipLaunchKernelGGL(k_count_pairs_b<T>, dim3((unsigned)L.nblk[BM_TILE]), dim3(RS_THREADS), 0, st, L.B,
                       (const T*)rb.nnb, b.pairs);
    return hipGetLastError() == hipSuccess ? SPH_OK : SPH_E_DEVICE;
}

int batch_step(hipStream_t st, const BatchBufs& b, const BatchLaunch& L)
{
    if (L.B.nsim == 0) return SPH_OK;
    auto eval = [&](const double* x, const double* y, const double* u, const double* v,
                    const double* p) {
        return L.precision == SPH_FP32 ? batch_eval_T<float>(st, b, L, x, y, u, v, p)
                                       : batch_eval_T<double>(st, b, L, x, y, u, v, p);
    };
    int rc = eval(b.x, b.y, b.u, b.v, b.p);
    if (rc) return rc;
    const unsigned nb = (unsigned)L.nblk[BM_P256];
    hipLaunchKernelGGL(k_predict_b, dim3(nb), dim3(256), 0, st, L.B, (const double*)b.x,
                       (const double*)b.y, (const double*)b.u, (const double*)b.v,
                       (const double*)b.p, (const double*)b.r_dpdt, (const double*)b.r_dudt,
                       (const double*)b.r_dvdt, (const double*)b.r_dxs, (const double*)b.r_dys, b.xh,
                       b.yh, b.uh, b.vh, b.ph);
    rc = eval(b.xh, b.yh, b.uh, b.vh, b.ph);
    if (rc) return rc;
    hipLaunchKernelGGL(k_correct_b, dim3(nb), dim3(256), 0, st, L.B, b.x, b.y, b.u, b.v, b.p,
                       (const double*)b.r_dpdt, (const double*)b.r_dudt, (const double*)b.r_dvdt,
                       (const double*)b.r_dxs, (const double*)b.r_dys);
    return hipGetLastError() == hipSuccess ? SPH_OK : SPH_E_DEVICE;
}

// Clears the boundary-list counters (after skipped evaluations of a run of
// steps the alternation of the two counters no longer holds).
__global__ void k_reset_bcounters(int32_t* st)
{
    if (threadIdx.x < 2) st[threadIdx.x] = 0;
}

void reset_bcounters(sph_ctx* c)
{
    hipLaunchKernelGGL(k_reset_bcounters, dim3(1), dim3(64), 0, c->stream, c->w.status + 16);
    c->bparity = 0;
}

// Makes the list valid for the current positions (building or checking it).
int list_ready(sph_ctx* c, const sph_particles* ps)
{
    return ensure_list(c, (int)ps->n, ps->x, ps->y, ps->h);
}

// ---------------------------------------------------------------------------
// Diagnostics: deterministic two-stage reductions.
// ---------------------------------------------------------------------------

#define DIAG_BLOCKS 256

// ---------------------------------------------------------------------------
// Force on the solid particles, eq. (force-sph) of section 2.3, from the state
// the last evaluation left in the workspace (sorted records, pass A's
// density, beta and mass, the solids' ghost velocities).  For every solid
// particle i and fluid neighbour j (in FP64):
//   f_p    += -m_i m_j (P_i gradW(r_ij, h_i) + P_j gradW(r_ij, h_j)),
//             P = p / (rho^2 beta), the unreduced pressure;
//   f_visc += m_i (1/beta_i) m_j 4 nu/(rho_i + rho_j) (r_ij . gradW_ij)
//             / (r_ij^2 + eta_i) (u~_i - u_j), gradW_ij the average of the
//             gradients at h_i and h_j, u~_i the ghost velocity.
// Each thread takes a fixed set of sorted particles and each block reduces
// in a fixed tree, so the totals do not depend on scheduling.
// ---------------------------------------------------------------------------

#define FORCE_BLOCKS 256

template <typename T>
__global__ __launch_bounds__(256) void k_body_force(Grid g, NbrView nv, NbrList nl, int n,
                                                    const int32_t* __restrict__ kind,
                                                    const double4* __restrict__ pa,
                                                    const double2* __restrict__ puv,
                                                    const typename Vec4<T>::type* __restrict__ pf,
                                                    const T* __restrict__ beta,
                                                    const double* __restrict__ ugs,
                                                    const double* __restrict__ vgs, double nu,
                                                    double* part)
{
    __shared__ double sh[8][256];
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x) {
        if (kind[nv.perm[s]] != SPH_SOLID) continue;
        const double4 ai = pa[s];
        const typename Vec4<T>::type fi = pf[s];
        const double hi = ai.z, rhoi = (double)fi.z, mi = (double)fi.w, bi = (double)beta[s];
        const double Pi = bi > 0.0 ? ai.w / (rhoi * rhoi * bi) : 0.0;
        const double eta = 0.001 * hi * hi;
        const double ugi = ugs[s], vgi = vgs[s];
        auto term = [&](int js, double dx, double dy, double r2, double hj) {
            if (kind[nv.perm[js]] != SPH_FLUID) return;
            const double r = sqrt(r2);
            double gix = 0.0, giy = 0.0, gjx = 0.0, gjy = 0.0;
            if (r > 0.0) {
                const double fa = kern_dw64(r, hi) / r, fb = kern_dw64(r, hj) / r;
                gix = fa * dx; giy = fa * dy;
                gjx = fb * dx; gjy = fb * dy;
            }
            const double pj = pa[js].w;
            const typename Vec4<T>::type fj = pf[js];
            const double rhoj = (double)fj.z, mj = (double)fj.w, bj = (double)beta[js];
            const double Pj = bj > 0.0 ? pj / (rhoj * rhoj * bj) : 0.0;
            const double tpx = -mi * mj * (Pi * gix + Pj * gjx);
            const double tpy = -mi * mj * (Pi * giy + Pj * gjy);
            acc[0] += tpx; acc[1] += tpy;
            acc[4] += fabs(tpx); acc[5] += fabs(tpy);
            if (bi > 0.0) {
                const double2 uvj = puv[js];
                const double rdotg = dx * 0.5 * (gix + gjx) + dy * 0.5 * (giy + gjy);
                const double cv = mj * (4.0 * nu / (rhoi + rhoj)) * rdotg / (r2 + eta);
                const double tvx = mi * cv * (ugi - uvj.x) / bi;
                const double tvy = mi * cv * (vgi - uvj.y) / bi;
                acc[2] += tvx; acc[3] += tvy;
                acc[6] += fabs(tvx); acc[7] += fabs(tvy);
            }
        };
        const int cnt = nl.idx ? nl.cnt[s] : nl.K + 1;
        if (cnt <= nl.K) {
            const double ri3 = 3.0 * hi, ri2 = ri3 * ri3;
            for (int k = 0; k < cnt; ++k) {
                const int js = nl.idx[(int64_t)k * nl.stride + s];
                const double4 a = pa[js];
                const double dx = mi_axis(g, 0, ai.x - a.x);
                const double dy = mi_axis(g, 1, ai.y - a.y);
                const double r2 = dx * dx + dy * dy;
                const double rj3 = 3.0 * a.z;
                if (r2 < fmax(ri2, rj3 * rj3)) term(js, dx, dy, r2, a.z);
            }
        } else {
            for_each_neighbor(g, nv, ai.x, ai.y, hi, key_level(g, nv.keys[s]),
                              [&](int js, double dx, double dy, double r2, double hj) {
                                  term(js, dx, dy, r2, hj);
                              });
        }
    }
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < 8; ++k) sh[k][t] = acc[k];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o)
            for (int k = 0; k < 8; ++k) sh[k][t] += sh[k][t + o];
        __syncthreads();
    }
    if (t < 8) part[t * FORCE_BLOCKS + blockIdx.x] = sh[t][0];
}

// The FORCE_BLOCKS partial sums of each component, in a fixed tree.
__global__ __launch_bounds__(256) void k_force_total(const double* __restrict__ part, double* tot)
{
    __shared__ double sh[256];
    const int t = threadIdx.x;
    for (int k = 0; k < 8; ++k) {
        sh[t] = part[k * FORCE_BLOCKS + t];
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (t < o) sh[t] += sh[t + o];
            __syncthreads();
        }
        if (t == 0) tot[k] = sh[0];
        __syncthreads();
    }
}

// Rigid motion of the solid particles between steps: translation (wrapped
// on periodic axes) and the body's velocity.
__global__ __launch_bounds__(256) void k_move_solids(Grid g, int n,
                                                     const int32_t* __restrict__ kind, double dx,
                                                     double dy, double vx, double vy, double* x,
                                                     double* y, double* u, double* v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || kind[i] != SPH_SOLID) return;
    x[i] = wrap_axis(g, 0, x[i] + dx);
    y[i] = wrap_axis(g, 1, y[i] + dy);
    u[i] = vx;
    v[i] = vy;
}

int move_solids_run(sph_ctx* c, sph_particles* ps, const double* disp, const double* vel)
{
    const int n = (int)ps->n;
    if (n == 0) return SPH_OK;
    hipLaunchKernelGGL(k_move_solids, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, c->stream, c->grid,
                       n, (const int32_t*)ps->kind, disp[0], disp[1], vel[0], vel[1], ps->x, ps->y,
                       ps->u, ps->v);
    LAUNCHCHK(c, "move_solids");
    return SPH_OK;
}

int body_force_run(sph_ctx* c, sph_particles* ps, double* force)
{
    Work& w = c->w;
    const int n = (int)ps->n;
    for (int k = 0; k < 8; ++k) force[k] = 0.0;
    if (n == 0) return SPH_OK;
    // one evaluation (its pass B output is not needed; dt only scales it)
    PassAOut none{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    int rc = eval(c, n, ps->x, ps->y, ps->u, ps->v, ps->p, ps->h, ps->mq, ps->kind, ps->rho, 1.0,
                  none, w.r_dpdt, w.r_dudt, w.r_dvdt);
    if (rc) return rc;
    NbrView nv = nbr_view(c);
    NbrList nl{w.nl_idx, w.nl_cnt, w.nl_k, n, w.list_flag};
    if (!(c->list_valid && c->list_n == n)) nl.idx = nullptr;
    double* part = (double*)w.red;   // 8 FORCE_BLOCKS doubles
    double* tot = w.sc9;
    if (c->cfg.precision == SPH_FP32) {
        RatesBufs<float> b = rbufs<float>(c);
        hipLaunchKernelGGL(k_body_force<float>, dim3(FORCE_BLOCKS), dim3(256), 0, c->stream, c->grid, nv,
                           nl, n, (const int32_t*)ps->kind, (const double4*)w.pa,
                           (const double2*)w.puv, (const float4*)w.pf, (const float*)b.beta,
                           (const double*)w.ugs, (const double*)w.vgs, c->cfg.nu, part);
    } else {
        RatesBufs<double> b = rbufs<double>(c);
        hipLaunchKernelGGL(k_body_force<double>, dim3(FORCE_BLOCKS), dim3(256), 0, c->stream, c->grid, nv,
                           nl, n, (const int32_t*)ps->kind, (const double4*)w.pa,
                           (const double2*)w.puv, (const double4*)w.pf, (const double*)b.beta,
                           (const double*)w.ugs, (const double*)w.vgs, c->cfg.nu, part);
    }
    hipLaunchKernelGGL(k_force_total, dim3(1), dim3(256), 0, c->stream, (const double*)part, tot);
    LAUNCHCHK(c, "body_force");
    const Readback rb{force, tot, 64};
    return readback(c, &rb, 1);
}

// Also counts the particles holding a NaN or infinite value in x, y, u, v,
// p, rho or h (the host reports them as SPH_E_NONFINITE).
__global__ __launch_bounds__(256) void k_diag_partial(int n, const double* __restrict__ x,
                                                      const double* __restrict__ y,
                                                      const double* __restrict__ u,
                                                      const double* __restrict__ v,
                                                      const double* __restrict__ p,
                                                      const double* __restrict__ rho,
                                                      const double* __restrict__ h,
                                                      const int64_t* __restrict__ mq,
                                                      double mass_q, double* part,
                                                      int64_t* partq)
{
    __shared__ double sh[5][256];
    __shared__ int64_t sq[256], snf[256], sbad[256];
    double ke = 0, vol = 0, mx = 0, my = 0, um = 0;
    // the ledger total is summed in int64 with overflow checks: an overflow
    // (or a negative mass) is counted in bad
    int64_t q = 0, nf = 0, bad = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double m = (double)mq[i] * mass_q;
        double s2 = u[i] * u[i] + v[i] * v[i];
        ke += 0.5 * m * s2;
        vol += m / rho[i];
        mx += m * u[i];
        my += m * v[i];
        um = fmax(um, sqrt(s2));
        const int64_t mi = mq[i];
        if (mi < 0 || __builtin_add_overflow(q, mi, &q)) bad = 1;
        const bool fin = isfinite(x[i]) && isfinite(y[i]) && isfinite(u[i]) && isfinite(v[i]) &&
                         isfinite(p[i]) && isfinite(rho[i]) && isfinite(h[i]);
        nf += fin ? 0 : 1;
    }
    int t = threadIdx.x;
    sh[0][t] = ke; sh[1][t] = vol; sh[2][t] = mx; sh[3][t] = my; sh[4][t] = um; sq[t] = q;
    snf[t] = nf;
    sbad[t] = bad;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) {
            for (int k = 0; k < 4; ++k) sh[k][t] += sh[k][t + o];
            sh[4][t] = fmax(sh[4][t], sh[4][t + o]);
            if (__builtin_add_overflow(sq[t], sq[t + o], &sq[t])) sbad[t] = 1;
            sbad[t] |= sbad[t + o];
            snf[t] += snf[t + o];
        }
        __syncthreads();
    }
    if (t == 0) {
        for (int k = 0; k < 5; ++k) part[k * DIAG_BLOCKS + blockIdx.x] = sh[k][0];
        partq[blockIdx.x] = sq[0];
        partq[DIAG_BLOCKS + blockIdx.x] = snf[0];
        partq[2 * DIAG_BLOCKS + blockIdx.x] = sbad[0];
    }
}

int diag_run(sph_ctx* c, const sph_particles* ps, sph_diag* out)
{
    Work& w = c->w;
    const int n = (int)ps->n;
    double* part = w.sc9;  // 5 * DIAG_BLOCKS doubles
    int64_t* partq = w.red;
    hipLaunchKernelGGL(k_diag_partial, dim3(DIAG_BLOCKS), dim3(256), 0, c->stream, n, ps->x, ps->y,
                       ps->u, ps->v, ps->p, ps->rho, ps->h, ps->mq, c->cfg.mass_q, part, partq);
    LAUNCHCHK(c, "diag");
    double hp[5 * DIAG_BLOCKS];
    int64_t hq[3 * DIAG_BLOCKS];
    HIPCHK(c, hipMemcpyAsync(hp, part, sizeof(hp), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(hq, partq, sizeof(hq), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double r[5] = {0, 0, 0, 0, 0};
    int64_t q = 0, nf = 0;
    bool bad = false;
    for (int b = 0; b < DIAG_BLOCKS; ++b) {
        for (int k = 0; k < 4; ++k) r[k] += hp[k * DIAG_BLOCKS + b];
        r[4] = r[4] > hp[4 * DIAG_BLOCKS + b] ? r[4] : hp[4 * DIAG_BLOCKS + b];
        if (__builtin_add_overflow(q, hq[b], &q)) bad = true;
        nf += hq[DIAG_BLOCKS + b];
        bad = bad || hq[2 * DIAG_BLOCKS + b] != 0;
    }
    out->ke = r[0];
    out->vol = r[1];
    out->mom_x = r[2];
    out->mom_y = r[3];
    out->umax = r[4];
    out->mq_total = q;
    out->n = n;
    if (nf > 0) {
        set_err(c, "%lld particles hold NaN or infinite values", (long long)nf);
        return SPH_E_NONFINITE;
    }
    if (bad) {
        set_err(c, "the mass ledger total does not fit int64 (or a mass is negative): "
                   "choose a coarser mass quantum");
        return SPH_E_INVAL;
    }
    return SPH_OK;
}
