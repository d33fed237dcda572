// Adaptive refinement on gfx950 (section 3 of the paper).
//
//  - fluid m_ref from the background (section 3.3; algorithm of section 3.4,
//    item 4): minimum background m_ref within 3 max(h_i, h_b), else the
//    nearest background particle;
//  - split (section 3.1): m > mmax_f m_ref -> 7 children, the centre child in
//    the parent slot, six on a hexagon of radius eps h appended in
//    (parent slot, k) order; integer mass ledger (six get floor(mq/7));
//  - mutual-closest merge (section 3.2, eqs. merged-pos, merged-prop,
//    merged-h) with stable compaction of the deleted slots;
//  - shifting with Taylor correction (eqs. shift-deltar, shift-limit,
//    shift-correct) and h = C sqrt(mbar/rho) (section 3.1);
//  - background update (section 3.3 steps 1-4, eq. h-smoothing).
//
// Everything is double precision.  Sums run over CSR rows in ascending slot
// order with the operation order of the definition, so results are
// bit-exact with a sequential evaluation; argmin / min / any are
// order-free.  Compaction uses wave ballots: a lane's rank among the set
// flags of its wave is popcount(ballot & lanes-below), plus the wave and
// block offsets.
#include <math.h>
#include <string.h>

#include <type_traits>

#include "sph_device.h"

int scan_exclusive_i32(sph_ctx* c, const int32_t* in, int32_t* out, int64_t n);

// ---------------------------------------------------------------------------
// Ballot compaction: rank[i] = number of set flags before i; returns total.
// ---------------------------------------------------------------------------

// lanes per particle in the cell walks of the m_ref lookup and the merge search
#ifndef WG
#define WG 4
#endif
#ifndef MG
#define MG 4
#endif

__global__ __launch_bounds__(256) void k_flag_count(int n, const int32_t* __restrict__ flag,
                                                    int32_t* bcount)
{
    __shared__ int32_t wc[4];
    int i = blockIdx.x * 256 + threadIdx.x;
    bool f = i < n && flag[i] != 0;
    uint64_t b = __ballot(f);
    if (__lane_id() == 0) wc[threadIdx.x >> 6] = __popcll(b);
    __syncthreads();
    if (threadIdx.x == 0) bcount[blockIdx.x] = wc[0] + wc[1] + wc[2] + wc[3];
}

__global__ __launch_bounds__(256) void k_flag_rank(int n, const int32_t* __restrict__ flag,
                                                   const int32_t* __restrict__ boff, int32_t* rank)
{
    __shared__ int32_t wc[4];
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    int i = blockIdx.x * 256 + threadIdx.x;
    bool f = i < n && flag[i] != 0;
    uint64_t b = __ballot(f);
    if (lane == 0) wc[w] = __popcll(b);
    __syncthreads();
    int off = boff[blockIdx.x];
    for (int q = 0; q < w; ++q) off += wc[q];
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    if (i < n) rank[i] = off + __popcll(b & lt);
}

// `before_wait` enqueues work that needs the ranks but not the total, so
// that the device has it queued while the host waits for the total.
struct NoWork {
    void operator()() const {}
};
template <class F = NoWork>
static int compact_ranks(sph_ctx* c, int n, const int32_t* flag, int32_t* rank, int32_t* total,
                         F&& before_wait = F{})
{
    Work& w = c->w;
    *total = 0;
    if (n <= 0) return SPH_OK;
    int nb = (int)cdiv(n, 256);
    hipLaunchKernelGGL(k_flag_count, dim3(nb), dim3(256), 0, c->stream, n, flag, w.idx_b);
    LAUNCHCHK(c, "flag_count");
    int rc = scan_exclusive_i32(c, w.idx_b, w.idx_b, nb);
    if (rc) return rc;
    hipLaunchKernelGGL(k_flag_rank, dim3(nb), dim3(256), 0, c->stream, n, flag, w.idx_b, rank);
    LAUNCHCHK(c, "flag_rank");
    before_wait();
    LAUNCHCHK(c, "before_wait");
    const Readback rb{total, w.idx_b + nb, 4};
    return readback(c, &rb, 1);
}

// ---------------------------------------------------------------------------
// m_ref lookup
// ---------------------------------------------------------------------------

// Queries run in `order` (a spatial order of the fluid slots) when given.
__global__ __launch_bounds__(256) void k_gather_f64(int n, const int32_t* __restrict__ perm,
                                                    const double* __restrict__ src, double* dst)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) dst[s] = src[perm[s]];
}

__global__ __launch_bounds__(256) void k_mref_lookup(Grid g, NbrView nv, int n,
                                                     const double* __restrict__ x,
                                                     const double* __restrict__ y,
                                                     const double* __restrict__ h,
                                                     const double* __restrict__ bms,
                                                     double* mref_out, int32_t* none,
                                                     const int32_t* __restrict__ order)
{
    // bms: the background's m_ref in its sorted order
    const int tt = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const int t = tt / WG, gl = tt % WG;
    if (t >= n) return;
    const int i = order ? order[t] : t;
    const double xi = x[i], yi = y[i], hi = h[i];
    const int li = level_of(g, hi);
    double mn = 0.0;
    int found = 0;
    group_walk_x<WG>(g, nv, bms, xi, yi, hi, li, gl,
                     [&](int, bool pass, double, double, double, double, double v) {
                         if (!pass) return;
                         if (!found || v < mn) mn = v;
                         found = 1;
                     });
    // the minimum over the group's lanes (exact, independent of order)
#pragma unroll
    for (int o = 1; o < WG; o <<= 1) {
        const double mo = __shfl_xor(mn, o, 64);
        const int fo = __shfl_xor(found, o, 64);
        if (fo && (!found || mo < mn)) mn = mo;
        found |= fo;
    }
    if (gl) return;
    none[i] = !found;
    if (found) mref_out[i] = mn;
}

// Nearest background particle for the (rare) fluid particles with none in
// range: brute force, ties to the lower background slot.
__global__ __launch_bounds__(256) void k_mref_nearest(Grid g, int n, const double* __restrict__ x,
                                                      const double* __restrict__ y,
                                                      const int32_t* __restrict__ none, int nb,
                                                      const double* __restrict__ bx,
                                                      const double* __restrict__ by,
                                                      const double* __restrict__ bmref,
                                                      double* mref_out)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !none[i]) return;
    int best = -1;
    double br = 0.0;
    for (int b = 0; b < nb; ++b) {
        double dx = mi_axis(g, 0, x[i] - bx[b]);
        double dy = mi_axis(g, 1, y[i] - by[b]);
        double r2 = dx * dx + dy * dy;
        if (best < 0 || r2 < br) { best = b; br = r2; }
    }
    if (best >= 0) mref_out[i] = bmref[best];
}

static int mref_lookup_into(sph_ctx* c, const sph_particles* ps, const sph_background* bg,
                            double* mref_out)
{
    Work& w = c->w;
    int n = (int)ps->n, nb = (int)bg->n;
    if (n == 0 || nb == 0) return SPH_OK;
    // the fluid's last sorted order (if it still covers these slots) keeps
    // neighbouring queries together; the background build overwrites it
    const int32_t* order = nullptr;
    if (c->built_n == n) {
        HIPCHK(c, hipMemcpyAsync(w.idx_b, w.vals_a, sizeof(int32_t) * (size_t)n,
                                 hipMemcpyDeviceToDevice, c->stream));
        order = w.idx_b;
    }
    int rc = nbr_build(c, nb, bg->x, bg->y, bg->h);
    if (rc) return rc;
    NbrView nv = nbr_view(c);
    // m_ref of the background in its sorted order (the rate passes' record
    // buffer is free here), so that the walk reads it next to the positions
    double* bms = (double*)w.pa;
    hipLaunchKernelGGL(k_gather_f64, dim3((unsigned)cdiv(nb, 256)), dim3(256), 0, c->stream, nb,
                       (const int32_t*)nv.perm, bg->mref, bms);
    hipLaunchKernelGGL(k_mref_lookup, dim3((unsigned)cdiv((int64_t)n * WG, 256)), dim3(256), 0, c->stream, c->grid,
                       nv, n, ps->x, ps->y, ps->h, (const double*)bms, mref_out, w.flag, order);
    hipLaunchKernelGGL(k_mref_nearest, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, c->stream, c->grid,
                       n, ps->x, ps->y, w.flag, nb, bg->x, bg->y, bg->mref, mref_out);
    LAUNCHCHK(c, "mref_lookup");
    return SPH_OK;
}

int mref_lookup_run(sph_ctx* c, const sph_particles* ps, const sph_background* bg)
{
    return mref_lookup_into(c, ps, bg, ps->mref);
}

// ---------------------------------------------------------------------------
// Split
// ---------------------------------------------------------------------------

struct FluidState {
    double *x, *y, *u, *v, *p, *rho, *h, *mref;
    int64_t *mq, *origin;
    int32_t *kind, *sat;
};

__global__ __launch_bounds__(256) void k_split_flags(int n, const int64_t* __restrict__ mq,
                                                     const double* __restrict__ mref,
                                                     const int32_t* __restrict__ kind, double q,
                                                     double mmax_f, int32_t* flag)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double m = (double)mq[i] * q;
    int k = kind ? kind[i] : SPH_FLUID;
    flag[i] = (k == SPH_FLUID && m > mmax_f * mref[i]) ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_init_map(int n, int64_t* origin, int32_t* sat)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    origin[i] = i;
    sat[i] = 0;
}

__global__ __launch_bounds__(256) void k_split_apply(Grid g, int n, FluidState s,
                                                     const int32_t* __restrict__ flag,
                                                     const int32_t* __restrict__ rank,
                                                     double alpha, double eps)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flag[i]) return;
    const double ck[6] = {1.0, 0.5, -0.5, -1.0, -0.5, 0.5};
    const double sk[6] = {0.0, SPH_SIN60, SPH_SIN60, 0.0, -SPH_SIN60, -SPH_SIN60};
    const int64_t c = s.mq[i] / 7;
    const double r = eps * s.h[i];
    const double hc = alpha * s.h[i];
    const double xi = s.x[i], yi = s.y[i];
    const int64_t base = (int64_t)n + 6 * (int64_t)rank[i];
    for (int k = 0; k < 6; ++k) {
        int64_t t = base + k;
        s.x[t] = wrap_axis(g, 0, xi + r * ck[k]);
        s.y[t] = wrap_axis(g, 1, yi + r * sk[k]);
        s.u[t] = s.u[i];
        s.v[t] = s.v[i];
        s.p[t] = s.p[i];
        s.rho[t] = s.rho[i];
        s.h[t] = hc;
        s.mref[t] = s.mref[i];
        s.mq[t] = c;
        if (s.kind) s.kind[t] = s.kind[i];
        s.origin[t] = s.origin[i];
        s.sat[t] = 1;
    }
    s.mq[i] = s.mq[i] - 6 * c;
    s.h[i] = hc;
}

// ---------------------------------------------------------------------------
// Merge
// ---------------------------------------------------------------------------

// Per sorted particle: m_max (the split threshold mmax_f m_ref), or -1 for
// a particle that is not fluid, and its mass quanta.
struct __align__(16) MergeRec {
    double mm;
    int64_t mq;
};

__global__ __launch_bounds__(256) void k_merge_pack(int n, const int32_t* __restrict__ perm,
                                                   FluidState s, double mmax_f, MergeRec* rec)
{
    int js = blockIdx.x * blockDim.x + threadIdx.x;
    if (js >= n) return;
    const int j = perm[js];
    if (j < 0) {  // merged away since the build
        rec[js] = MergeRec{-1.0, 0};
        return;
    }
    const bool fl = !s.kind || s.kind[j] == SPH_FLUID;
    MergeRec r;
    r.mm = fl ? mmax_f * s.mref[j] : -1.0;
    r.mq = s.mq[j];
    rec[js] = r;
}

// Closest allowed partner of every sorted particle (or, when `affected` is
// given, of the affected ones only); the walk pads each level's radius by
// `pad` (particles moved since the build).
__global__ __launch_bounds__(256) void k_merge_closest(Grid g, NbrView nv, int n, FluidState s,
                                                       double q, double mmax_f,
                                                       const MergeRec* __restrict__ rec,
                                                       int32_t* closest,
                                                       const int32_t* __restrict__ affected,
                                                       const unsigned long long* __restrict__ pad)
{
    const int tt = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const int sp = tt / MG, gl = tt % MG;
    if (sp >= n) return;
    const int i = nv.perm[sp];
    if (i < 0 || (affected && !affected[i])) return;
    const double4 ai = nv.xyh[sp];  // the current position and h
    const double xi = ai.x, yi = ai.y, hi = ai.z;
    const int li = key_level(g, nv.keys[sp]);
    const int64_t mqi = s.mq[i];
    const double mi = (double)mqi * q;
    const double mmi = mmax_f * s.mref[i];
    const int ki = s.kind ? s.kind[i] : SPH_FLUID;
    int best = -1;
    double br = 0.0;
    if (ki == SPH_FLUID && !(mi > mmi)) {
        // a merge partner lies within (h_i + h_j)/2 <= max(h_i, h_j): a third
        // of the support radius (0.34 leaves margin for rounding) bounds it
        group_walk_x<MG>(g, nv, rec, xi, yi, hi, li, gl,
                         [&](int js, bool pass, double dx, double dy, double r2, double hj, MergeRec rj) {
            if (!pass || js == sp) return;
            if (best >= 0 && r2 > br) return;  // cannot beat the current best
            if (!(rj.mm >= 0.0)) return;       // not fluid
            const int64_t mqj = rj.mq;
            const double mj = (double)mqj * q;
            const double mmj = rj.mm;
            if (mj > mmj) return;
            const double hh = 0.5 * (hi + hj);
            if (!(r2 < hh * hh)) return;
            const double msum = (double)(mqi + mqj) * q;
            const double mm = mmi > mmj ? mmi : mmj;
            if (!(msum < mm)) return;
            const int j = nv.perm[js];
            if (best < 0 || r2 < br || j < best) {
                best = j;
                br = r2;
            }
        }, 0.34, pad);
    }
    // the group's closest (ties to the lower slot), independent of order
#pragma unroll
    for (int o = 1; o < MG; o <<= 1) {
        const int bo = __shfl_xor(best, o, 64);
        const double ro = __shfl_xor(br, o, 64);
        if (bo >= 0 && (best < 0 || ro < br || (ro == br && bo < best))) {
            best = bo;
            br = ro;
        }
    }
    if (gl == 0) closest[i] = best;
}

__global__ __launch_bounds__(256) void k_merge_keep(int n, const int32_t* __restrict__ closest,
                                                    int32_t* keep)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int j = closest[i];
    bool mutual = j >= 0 && closest[j] == i;
    keep[i] = (mutual && j < i) ? 0 : 1;
}

__global__ __launch_bounds__(256) void k_merge_apply(Grid g, int n, FluidState s, FluidState d,
                                                     const int32_t* __restrict__ closest,
                                                     const int32_t* __restrict__ keep,
                                                     const int32_t* __restrict__ rank, double q)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !keep[i]) return;
    const int t = rank[i];
    const int j = closest[i];
    const bool mutual = j >= 0 && closest[j] == i;
    d.x[t] = s.x[i]; d.y[t] = s.y[i]; d.u[t] = s.u[i]; d.v[t] = s.v[i];
    d.p[t] = s.p[i]; d.rho[t] = s.rho[i]; d.h[t] = s.h[i]; d.mref[t] = s.mref[i];
    d.mq[t] = s.mq[i]; d.origin[t] = s.origin[i]; d.sat[t] = s.sat[i];
    if (s.kind) d.kind[t] = s.kind[i];
    if (!mutual) return;
    // i < j: i is kept and absorbs j
    const double ma = (double)s.mq[i] * q;
    const double mb = (double)s.mq[j] * q;
    const int64_t mqm = s.mq[i] + s.mq[j];
    const double mm = (double)mqm * q;
    const double xa = s.x[i], ya = s.y[i];
    const double xb = xa - mi_axis(g, 0, xa - s.x[j]);
    const double yb = ya - mi_axis(g, 1, ya - s.y[j]);
    const double xm = (ma * xa + mb * xb) / mm;
    const double ym = (ma * ya + mb * yb) / mm;
    const double dax = xm - xa, day = ym - ya;
    const double dbx = xm - xb, dby = ym - yb;
    const double ra = sqrt(dax * dax + day * day);
    const double rb = sqrt(dbx * dbx + dby * dby);
    const double den = ma * kern_w64(ra, s.h[i]) + mb * kern_w64(rb, s.h[j]);
    const double w01 = kern_w64(0.0, 1.0);
    d.h[t] = sqrt(mm * w01 / den);
    d.x[t] = wrap_axis(g, 0, xm);
    d.y[t] = wrap_axis(g, 1, ym);
    d.u[t] = (ma * s.u[i] + mb * s.u[j]) / mm;
    d.v[t] = (ma * s.v[i] + mb * s.v[j]) / mm;
    d.p[t] = (ma * s.p[i] + mb * s.p[j]) / mm;
    d.rho[t] = (ma * s.rho[i] + mb * s.rho[j]) / mm;
    d.mref[t] = s.mref[i] < s.mref[j] ? s.mref[i] : s.mref[j];
    d.mq[t] = mqm;
}

// Merge iterations after the first reuse the first iteration's neighbour
// structure.  Only merged pairs change: the slot that absorbed its partner
// moves to the merged position and takes the merged h, the other slot goes.
// The sorted records are updated in place (slots renumbered by the
// compaction, removed ones marked -1, a merged particle's record moved), and
// each level's search radius grows by the largest distance a particle filed
// in it has moved since the build.  A particle keeps its last closest
// partner unless it merged, its partner merged or went, or a merged particle
// now lies within its merge reach; only those search again.  The argmin and
// its tie order (the lower slot; the compaction keeps slot order) are those
// of a search from scratch.

// Sorted position js: the slot after the compaction, and for a particle that
// absorbed its partner the moved record, the level's pad and h maximum, and
// an entry in the list of merged particles.
__global__ __launch_bounds__(256) void k_merge_remap_sorted(Grid g, int nsorted, int32_t* perm,
                                                            const uint64_t* __restrict__ keys,
                                                            const double* __restrict__ xs,
                                                            const double* __restrict__ ys,
                                                            double4* xyh, unsigned long long* hmax,
                                                            unsigned long long* pad, FluidState s,
                                                            const int32_t* __restrict__ keep,
                                                            const int32_t* __restrict__ rank,
                                                            const int32_t* __restrict__ closest,
                                                            int32_t* mlist, int32_t* mcount)
{
    const int js = blockIdx.x * blockDim.x + threadIdx.x;
    bool merged = false;
    double d = 0.0, h = 0.0;
    int l = 0;
    if (js < nsorted) {
        const int i = perm[js];
        if (i >= 0 && !keep[i]) {
            perm[js] = -1;
        } else if (i >= 0) {
            const int t = rank[i];
            perm[js] = t;
            const int j = closest[i];
            if (j >= 0 && closest[j] == i) {
                merged = true;
                const double x = s.x[t], y = s.y[t];
                h = s.h[t];
                xyh[js] = make_double4(x, y, h, 0.0);
                // distance from the position the particle was filed at (the build's)
                const double dx = mi_axis(g, 0, x - xs[js]), dy = mi_axis(g, 1, y - ys[js]);
                d = sqrt(dx * dx + dy * dy);
                l = key_level(g, keys[js]);
            }
        }
    }
    // the wave's merged particles take one run of the list (one atomic), and
    // each level present among them one maximum of d and of h (the same
    // maxima as one atomic per particle, without thousands of atomics on a
    // few words); every lane of the wave reaches this point
    const unsigned long long mb = __ballot(merged);
    if (!mb) return;
    const int lane = __lane_id();
    const int lead = __builtin_ctzll(mb);
    int base = 0;
    if (lane == lead) base = atomicAdd(mcount, (int)__popcll(mb));
    base = __shfl(base, lead, 64);
    if (merged) mlist[base + __popcll(mb & ((1ull << lane) - 1ull))] = js;
    unsigned long long todo = mb;
    while (todo) {
        const int ld = __builtin_ctzll(todo);
        const int lv = __shfl(l, ld, 64);
        const bool mine = merged && l == lv;
        double dm = mine ? d : 0.0, hm = mine ? h : 0.0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            dm = fmax(dm, __shfl_xor(dm, o, 64));
            hm = fmax(hm, __shfl_xor(hm, o, 64));
        }
        if (lane == ld) {
            atomicMax(&pad[lv], (unsigned long long)__double_as_longlong(dm));
            atomicMax(&hmax[lv], (unsigned long long)__double_as_longlong(hm));
        }
        todo &= ~__ballot(mine);
    }
}

// Old slot i (kept): its new slot's last closest partner, renumbered, or the
// mark that it searches again (it merged, or its partner merged or went).
__global__ __launch_bounds__(256) void k_merge_remap_slots(int nprev, const int32_t* __restrict__ keep,
                                                           const int32_t* __restrict__ rank,
                                                           const int32_t* __restrict__ closest,
                                                           int32_t* closest_new, int32_t* affected)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nprev || !keep[i]) return;
    const int t = rank[i];
    const int j = closest[i];
    int aff = 0, cn = -1;
    if (j >= 0) {
        if (closest[j] == i) {
            aff = 1;  // i absorbed j
        } else {
            const int jj = closest[j];
            const bool jmerged = keep[j] && jj >= 0 && closest[jj] == j;
            if (!keep[j] || jmerged) aff = 1;
            else cn = rank[j];
        }
    }
    affected[t] = aff;
    closest_new[t] = cn;
}

// Every particle within merge reach of a merged one searches again.
__global__ __launch_bounds__(256) void k_merge_mark(Grid g, NbrView nv, int count,
                                                    const int32_t* __restrict__ mlist,
                                                    int32_t* affected,
                                                    const unsigned long long* __restrict__ pad)
{
    const int tt = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const int k = tt / MG, gl = tt % MG;
    if (k >= count) return;
    const int jm = mlist[k];
    const double4 a = nv.xyh[jm];
    const int lm = key_level(g, nv.keys[jm]);
    // a partner lies within (h_i + h_j) / 2 <= max(h_i, h_j): a third of the
    // support radius, as in the search
    group_walk_x<MG>(g, nv, nv.perm, a.x, a.y, a.z, lm, gl,
                     [&](int, bool pass, double, double, double, double, int32_t j) {
                         if (pass && j >= 0) affected[j] = 1;
                     }, 0.34, pad);
}

// ---------------------------------------------------------------------------
// Shift + Taylor correction, h update (CSR rows in ascending slot order)
// ---------------------------------------------------------------------------

// Per-slot records for the shift and h-update sweeps, so that a neighbour
// costs two 32-byte loads: A = {x, y, h, m}, B = {u, v, p, rho} (m = mq q,
// the same double the oracle uses).
// With rho0 > 0 (the shift sweeps) the last members are the quotients the
// shift terms use, m / rho0 and V = m / rho: the same correctly rounded
// divisions of the same operands, taken once per particle instead of once
// per pair.
__global__ __launch_bounds__(256) void k_pack_shift(int n, FluidState s, double q, double rho0,
                                                    double4* A, double4* B)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double m = (double)s.mq[i] * q;
    const double rho = s.rho[i];
    A[i] = make_double4(s.x[i], s.y[i], s.h[i], rho0 > 0.0 ? m / rho0 : m);
    B[i] = make_double4(s.u[i], s.v[i], s.p[i], rho0 > 0.0 ? m / rho : rho);
}

// The neighbours of each fluid row in the current positions, kept in
// ascending column order: the entries of the (superset) row that pass the
// pair predicate, self excluded, written from rp[i] on with their count in
// rcnt[i].  Four lanes share a row; entry base + gl goes to lane gl, and
// passing entries are ranked by lane, so the order is the row's.
#define FG 4
// Radius of the first superset CSR of an adaptation beyond the support
// (fraction of it); the shifts' measured displacements decide whether it
// still covers their rows.
#ifndef SHIFT_SKIN
#define SHIFT_SKIN 0.15
#endif

__global__ void k_clear_u64(unsigned long long* p, int k)
{
    if ((int)threadIdx.x < k) p[threadIdx.x] = 0ull;
}
__global__ void k_clear_i32_1(int32_t* p)
{
    if (threadIdx.x == 0) p[0] = 0;
}
__global__ __launch_bounds__(256) void k_shift_filter(Grid g, int n, const int32_t* __restrict__ kind,
                                                      const double4* __restrict__ A,
                                                      const int64_t* __restrict__ rp,
                                                      const int32_t* __restrict__ col,
                                                      int32_t* __restrict__ colf,
                                                      int32_t* __restrict__ rcnt,
                                                      const int32_t* __restrict__ order)
{
    const int tt = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const int t = tt / FG, gl = tt % FG;
    if (t >= n) return;
    const int i = order ? order[t] : t;
    if (kind && kind[i] != SPH_FLUID) {
        if (gl == 0) rcnt[i] = 0;
        return;
    }
    const double4 ai = A[i];
    const double xi = ai.x, yi = ai.y, hi = ai.z;
    const int64_t b0 = rp[i], e = rp[i + 1];
    int cnt = 0;
    // the next chunk's column entries are read before this chunk's records
    // are tested, so the two loads of a chunk overlap the previous chunk
    int jn[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t k = b0 + FG * u + gl;
        jn[u] = k < e ? col[k] : i;
    }
    for (int64_t base = b0; base < e; base += 4 * FG) {
        int j[4];
        double4 aj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) j[u] = jn[u];
#pragma unroll
        for (int u = 0; u < 4; ++u) aj[u] = A[j[u]];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t k = base + 4 * FG + FG * u + gl;
            jn[u] = k < e ? col[k] : i;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double dx = mi_axis(g, 0, xi - aj[u].x);
            const double dy = mi_axis(g, 1, yi - aj[u].y);
            const double r2 = dx * dx + dy * dy;
            const double RR = 3.0 * (hi > aj[u].z ? hi : aj[u].z);
            // r = sqrt(r2) > 0 exactly when r2 > 0
            const bool pass = base + FG * u + gl < e && r2 < RR * RR && r2 > 0.0;
            int tot;
            const int k = cnt + group_rank<FG>(pass, gl, &tot);
            if (pass) colf[b0 + k] = j[u];
            cnt += tot;
        }
    }
    if (gl == 0) rcnt[i] = cnt;
}

// Lanes per row of the shift and h-update sweeps (1, 2 or 4) and entries
// each lane loads ahead.  The lanes of a row compute the terms of every G-th
// entry and the group adds them in column order (a DPP broadcast per term),
// so each sum is the one sequential evaluation gives; the wider group keeps
// more rows' gathers in flight.
#ifndef SHIFT_G
#define SHIFT_G 2
#endif
#ifndef SHIFT_U
#define SHIFT_U 2
#endif

// Value of lane Q of the group (the lane itself when G = 1).
template <int G, int Q>
__device__ __forceinline__ double grp_val(double v)
{
    if constexpr (G == 1) return v;
    else return grp_bcast<G, Q>(v);
}
template <int G, int Q>
__device__ __forceinline__ int grp_val_i(int v)
{
    if constexpr (G == 1) return v;
    else return grp_bcast_i<G, Q>(v);
}
// f(integral_constant<int, Q>) for Q = 0 .. G-1, in that order.
template <int G, int Q = 0, class F>
__device__ __forceinline__ void grp_each(F&& f)
{
    if constexpr (Q < G) {
        f(std::integral_constant<int, Q>{});
        grp_each<G, Q + 1>(f);
    }
}

// One entry's shift and Taylor-correction terms, each formed as the
// sequential loop forms it before adding.
struct ShiftTerms {
    double sx, sy, gux, guy, gvx, gvy, gpx, gpy;
    int ok;
};

// EXACT: rows hold exactly the neighbours (from k_shift_filter), counts in
// rcnt; otherwise rows may be a superset, re-tested entry by entry.
// One fluid row of the shift and Taylor correction, lane gl of its group of
// G (every lane of the group calls it and gets the same sums); returns
// |dr_i| / h_i.  Lane 0 of the group writes the row's results.
template <bool EXACT, int G, int U>
__device__ __forceinline__ double shift_row(const Grid& g, const double4* __restrict__ A,
                                            const double4* __restrict__ B,
                                            const int64_t* __restrict__ rp,
                                            const int32_t* __restrict__ col,
                                            const int32_t* __restrict__ rcnt, double rho0, int i,
                                            int gl, double4 ai, double4 bi, double* ddx_o,
                                            double* ddy_o, double* nu_o, double* nv_o,
                                            double* np_o)
{
    const double ui = bi.x, vi = bi.y, pi = bi.z;
    // shift sums and the Taylor gradients share one sweep over the row; every
    // accumulator still adds its terms in ascending column order
    const double fxi = kern_f<double>(SPH_XI);
    double sx = 0.0, sy = 0.0;
    double gux = 0, guy = 0, gvx = 0, gvy = 0, gpx = 0, gpy = 0;
    const double xi = ai.x, yi = ai.y, hi = ai.z;
    auto term = [&](const double4& aj, const double4& bj, bool valid) __attribute__((always_inline)) {
        ShiftTerms o{0, 0, 0, 0, 0, 0, 0, 0, 0};
        if (!valid) return o;
        const double dx = mi_axis(g, 0, xi - aj.x);
        const double dy = mi_axis(g, 1, yi - aj.y);
        const double r2 = dx * dx + dy * dy;
        const double hj = aj.z;
        if constexpr (!EXACT) {
            const double RR = 3.0 * (hi > hj ? hi : hj);
            if (!(r2 < RR * RR)) return o;  // the row may be a superset of N(i)
        }
        const double r = sqrt(r2);
        if constexpr (!EXACT) {
            if (r <= 0.0) return o;
        }
        // aj.w = m_j / rho0 and bj.w = V_j = m_j / rho_j (k_pack_shift)
        // shifting term at h_ij
        const double hij = 0.5 * (hi + hj);
        const double wr = kern_f<double>(r / hij) / fxi;
        const double coef = aj.w * (1.0 + 0.24 * ((wr * wr) * (wr * wr)));
        const double tt = coef * (kern_dw64(r, hij) / r);
        o.sx = tt * dx;
        o.sy = tt * dy;
        // gradients at h_i
        const double f = kern_dw64(r, hi) / r;
        const double wx = f * dx, wy = f * dy;
        const double Vj = bj.w;
        const double du = bj.x - ui, dv = bj.y - vi, dp = bj.z - pi;
        o.gux = Vj * du * wx; o.guy = Vj * du * wy;
        o.gvx = Vj * dv * wx; o.gvy = Vj * dv * wy;
        o.gpx = Vj * dp * wx; o.gpy = Vj * dp * wy;
        o.ok = 1;
        return o;
    };
    auto add = [&](const ShiftTerms& o) __attribute__((always_inline)) {
        sx = sx + o.sx; sy = sy + o.sy;
        gux = gux + o.gux; guy = guy + o.guy;
        gvx = gvx + o.gvx; gvy = gvy + o.gvy;
        gpx = gpx + o.gpx; gpy = gpy + o.gpy;
    };
    // lane gl takes entries base + u G + gl; U entries' loads are issued
    // before their terms, which are then added one by one in column order
    const int64_t b0 = rp[i];
    const int64_t e = EXACT ? b0 + rcnt[i] : rp[i + 1];
    for (int64_t base = b0; base < e; base += G * U) {
        int j[U];
        double4 aj[U], bj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t k = base + u * G + gl;
            j[u] = k < e ? col[k] : i;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            aj[u] = A[j[u]];
            bj[u] = B[j[u]];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const ShiftTerms o = term(aj[u], bj[u], base + u * G + gl < e);
            grp_each<G>([&](auto q) __attribute__((always_inline)) {
                constexpr int Q = decltype(q)::value;
                ShiftTerms b;
                b.ok = grp_val_i<G, Q>(o.ok);
                b.sx = grp_val<G, Q>(o.sx); b.sy = grp_val<G, Q>(o.sy);
                b.gux = grp_val<G, Q>(o.gux); b.guy = grp_val<G, Q>(o.guy);
                b.gvx = grp_val<G, Q>(o.gvx); b.gvy = grp_val<G, Q>(o.gvy);
                b.gpx = grp_val<G, Q>(o.gpx); b.gpy = grp_val<G, Q>(o.gpy);
                if (b.ok) add(b);
            });
        }
    }
    const double pref = -0.5 * (hi * hi);
    double ddx = pref * sx, ddy = pref * sy;
    const double mag = sqrt(ddx * ddx + ddy * ddy);
    const double lim = 0.25 * hi;
    if (mag > lim) {
        const double th = lim / mag;
        ddx = ddx * th;
        ddy = ddy * th;
    }
    if (gl == 0) {
        ddx_o[i] = ddx;
        ddy_o[i] = ddy;
        nu_o[i] = ui + (gux * ddx + guy * ddy);
        nv_o[i] = vi + (gvx * ddx + gvy * ddy);
        np_o[i] = pi + (gpx * ddx + gpy * ddy);
    }
    return sqrt(ddx * ddx + ddy * ddy) / hi;
}

template <bool EXACT>
__global__ __launch_bounds__(256) void k_shift_taylor(Grid g, int n, const int32_t* __restrict__ kind,
                                                      const double4* __restrict__ A,
                                                      const double4* __restrict__ B,
                                                      const int64_t* __restrict__ rp,
                                                      const int32_t* __restrict__ col,
                                                      const int32_t* __restrict__ rcnt,
                                                      double rho0, double* ddx_o, double* ddy_o,
                                                      double* nu_o, double* nv_o, double* np_o,
                                                      const int32_t* __restrict__ order,
                                                      unsigned long long* dmax)
{
    // rows are taken in `order` (a spatial order of the slots) when given,
    // so that a wave's neighbours share cache lines
    const int tt = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const int t = tt / SHIFT_G, gl = tt % SHIFT_G;
    double rel = 0.0;  // |dr_i| / h_i
    if (t < n) {
        const int i = order ? order[t] : t;
        const double4 ai = A[i], bi = B[i];
        const double ui = bi.x, vi = bi.y, pi = bi.z;
        if (kind && kind[i] != SPH_FLUID) {
            if (gl == 0) {
                ddx_o[i] = 0.0; ddy_o[i] = 0.0;
                nu_o[i] = ui; nv_o[i] = vi; np_o[i] = pi;
            }
        } else {
            rel = shift_row<EXACT, SHIFT_G, SHIFT_U>(g, A, B, rp, col, rcnt, rho0, i, gl, ai, bi,
                                                     ddx_o, ddy_o, nu_o, nv_o, np_o);
        }
    }
    // dmax (when given) receives the largest |dr_i| / h_i of the launch:
    // every lane of the wave is here (no early exit above)
    if (dmax) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) rel = fmax(rel, __shfl_xor(rel, o, 64));
        if (__lane_id() == 0 && rel > 0.0) atomicMax(dmax, (unsigned long long)__double_as_longlong(rel));
    }
}

__global__ __launch_bounds__(256) void k_shift_apply(Grid g, int n, FluidState s,
                                                     const double* __restrict__ ddx,
                                                     const double* __restrict__ ddy,
                                                     const double* __restrict__ nu,
                                                     const double* __restrict__ nv,
                                                     const double* __restrict__ np)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    s.x[i] = wrap_axis(g, 0, s.x[i] + ddx[i]);
    s.y[i] = wrap_axis(g, 1, s.y[i] + ddy[i]);
    s.u[i] = nu[i];
    s.v[i] = nv[i];
    s.p[i] = np[i];
}

// h = C sqrt(m_bar / rho) with m_bar the mean mass over N(i), self
// included; the row may be a superset of N(i), filtered by the predicate.
// SHIFT_G lanes per row, the masses added in column order as in the shift.
__global__ __launch_bounds__(256) void k_hupdate(Grid g, int n, const int64_t* __restrict__ rp,
                                                 const int32_t* __restrict__ col,
                                                 const double4* __restrict__ A,
                                                 const double* __restrict__ rho,
                                                 const int32_t* __restrict__ kind, double hdx,
                                                 double* nh, const int32_t* __restrict__ order)
{
    constexpr int G = SHIFT_G, U = SHIFT_U;
    const int tt = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const int t = tt / G, gl = tt % G;
    if (t >= n) return;
    const int i = order ? order[t] : t;
    const double4 ai = A[i];
    if (kind && kind[i] != SPH_FLUID) {
        if (gl == 0) nh[i] = ai.z;
        return;
    }
    const double xi = ai.x, yi = ai.y, hi = ai.z;
    double sm = 0.0;
    int64_t cnt = 0;
    const int64_t b0 = rp[i], e = rp[i + 1];
    // the next chunk's column entries are read before this chunk's records
    int jn[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t k = b0 + u * G + gl;
        jn[u] = k < e ? col[k] : i;
    }
    for (int64_t base = b0; base < e; base += G * U) {
        double4 aj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) aj[u] = A[jn[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t k = base + G * U + u * G + gl;
            jn[u] = k < e ? col[k] : i;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double dx = mi_axis(g, 0, xi - aj[u].x);
            const double dy = mi_axis(g, 1, yi - aj[u].y);
            const double RR = 3.0 * (hi > aj[u].z ? hi : aj[u].z);
            const int ok = base + u * G + gl < e && dx * dx + dy * dy < RR * RR;
            grp_each<G>([&](auto q) __attribute__((always_inline)) {
                constexpr int Q = decltype(q)::value;
                const double m = grp_val<G, Q>(aj[u].w);
                if (grp_val_i<G, Q>(ok)) {
                    sm += m;
                    ++cnt;
                }
            });
        }
    }
    if (gl) return;
    const double mbar = sm / (double)cnt;
    nh[i] = hdx * sqrt(mbar / rho[i]);
}

__global__ void k_copy_f64(int n, const double* __restrict__ a, double* b)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// Builds the neighbour structure of (x, y, h) and exports CSR to the
// internal buffers (rows ascending).
static int internal_csr(sph_ctx* c, int n, const double* x, const double* y, const double* h,
                        double sf = 1.0)
{
    Work& w = c->w;
    int rc = nbr_build(c, n, x, y, h);
    if (rc) return rc;
    int64_t nnz = 0;
    rc = nbr_export_csr(c, n, w.rp_tmp, w.col_tmp, w.col_cap, &nnz, sf);
    if (rc == SPH_E_CAPACITY) {
        // the count pass gave the size: the workspace is short of that
        const int64_t k = cdiv(nnz, w.capacity > 0 ? w.capacity : 1);
        set_err(c,
                "internal neighbour list needs %lld entries (%lld bytes), the workspace holds "
                "%lld: create the context with csr_k >= %lld",
                (long long)nnz, (long long)(4 * nnz), (long long)w.col_cap, (long long)k);
        rc = SPH_E_NOMEM;
    }
    return rc;
}

static FluidState fluid_of(sph_particles* ps, sph_adapt_map* map)
{
    FluidState s{ps->x, ps->y, ps->u, ps->v, ps->p, ps->rho, ps->h, ps->mref,
                 ps->mq, map->origin, ps->kind, map->sat};
    return s;
}

static FluidState tmp_state(sph_ctx* c, bool with_kind)
{
    Work& w = c->w;
    FluidState d{w.tmp_d[0], w.tmp_d[1], w.tmp_d[2], w.tmp_d[3], w.tmp_d[4], w.tmp_d[5],
                 w.tmp_d[6], w.tmp_d[7], w.tmp_i64[0], w.tmp_i64[1],
                 with_kind ? w.tmp_i32[0] : nullptr, w.tmp_i32[1]};
    return d;
}

__global__ __launch_bounds__(256) void k_copy_state(FluidState a, FluidState b, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    b.x[i] = a.x[i];
    b.y[i] = a.y[i];
    b.u[i] = a.u[i];
    b.v[i] = a.v[i];
    b.p[i] = a.p[i];
    b.rho[i] = a.rho[i];
    b.h[i] = a.h[i];
    b.mref[i] = a.mref[i];
    b.mq[i] = a.mq[i];
    b.origin[i] = a.origin[i];
    b.sat[i] = a.sat[i];
    if (a.kind && b.kind) b.kind[i] = a.kind[i];
}

static int copy_state(sph_ctx* c, const FluidState& a, FluidState& b, int n)
{
    if (n <= 0) return SPH_OK;
    hipLaunchKernelGGL(k_copy_state, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, c->stream, a, b, n);
    LAUNCHCHK(c, "copy_state");
    return SPH_OK;
}

int adapt_run(sph_ctx* c, sph_particles* ps, const sph_background* bg, sph_adapt_map* map)
{
    Work& w = c->w;
    const sph_config& cf = c->cfg;
    int n = (int)ps->n;
    map->n_split = 0;
    map->n_required = n;
    for (int k = 0; k < 8; ++k) map->n_merged[k] = 0;
    if (!map->origin || !map->sat) {
        set_err(c, "adapt map arrays not set");
        return SPH_E_INVAL;
    }
    // m_ref from the background goes to scratch first: nothing visible
    // changes before the capacity check
    double* mref_new = w.tmp_d[9];
    if (n > 0) {
        HIPCHK(c, hipMemcpyAsync(mref_new, ps->mref, 8 * (size_t)n, hipMemcpyDeviceToDevice, c->stream));
        if (bg) {
            int rc = mref_lookup_into(c, ps, bg, mref_new);
            if (rc) return rc;
        }
    }
    const unsigned nbk = (unsigned)cdiv(n > 0 ? n : 1, 256);
    hipLaunchKernelGGL(k_split_flags, dim3(nbk), dim3(256), 0, c->stream, n, ps->mq, mref_new,
                       ps->kind, cf.mass_q, cf.mmax_f, w.flag);
    LAUNCHCHK(c, "split_flags");
    int32_t ns = 0;
    int rc = compact_ranks(c, n, w.flag, w.idx_a, &ns);
    if (rc) return rc;
    map->n_split = ns;
    map->n_required = (int64_t)n + 6 * (int64_t)ns;
    if (map->n_required > ps->capacity) {
        set_err(c, "split needs %lld slots, capacity %lld", (long long)map->n_required,
                (long long)ps->capacity);
        return SPH_E_CAPACITY;
    }
    if (n > 0)
        HIPCHK(c, hipMemcpyAsync(ps->mref, mref_new, 8 * (size_t)n, hipMemcpyDeviceToDevice, c->stream));
    FluidState s = fluid_of(ps, map);
    hipLaunchKernelGGL(k_init_map, dim3(nbk), dim3(256), 0, c->stream, n, map->origin, map->sat);
    hipLaunchKernelGGL(k_split_apply, dim3(nbk), dim3(256), 0, c->stream, c->grid, n, s, w.flag,
                       w.idx_a, cf.split_alpha, cf.split_eps);
    LAUNCHCHK(c, "split_apply");
    n = n + 6 * ns;

    FluidState d = tmp_state(c, ps->kind != nullptr);
    // the first iteration builds the neighbour structure, the later ones
    // reuse it (see k_merge_remap_sorted); buffers free during adaptation:
    // closest partners alternate between w.closest and i64_a, the affected
    // marks in i64_b, the merged particles' sorted positions in tmp_i64[2],
    // the per-level pads in red, their count in status[32]
    int32_t* cur = w.closest;
    int32_t* nxt = (int32_t*)w.i64_a;
    int32_t* affected = (int32_t*)w.i64_b;
    int32_t* mlist = (int32_t*)w.tmp_i64[2];
    int32_t* mcount = w.status + 32;
    unsigned long long* pad = (unsigned long long*)w.red;
    int nsorted = 0, nprev = 0, nmerged = 0;
    for (int it = 0; it < cf.merge_iters; ++it) {
        if (n == 0) break;
        if (it > 0 && nmerged == 0) break;  // the state did not change: nothing more merges
        NbrView nv;
        const bool reuse = it > 0;
        if (!reuse) {
            rc = nbr_build(c, n, ps->x, ps->y, ps->h);
            if (rc) return rc;
            nsorted = n;
            hipLaunchKernelGGL(k_clear_u64, dim3(1), dim3(64), 0, c->stream, pad, (int)SPH_MAXL);
            nv = nbr_view(c);
        } else {
            const unsigned nbs = (unsigned)cdiv(nsorted, 256);
            hipLaunchKernelGGL(k_clear_i32_1, dim3(1), dim3(64), 0, c->stream, mcount);
            hipLaunchKernelGGL(k_merge_remap_sorted, dim3(nbs), dim3(256), 0, c->stream, c->grid, nsorted,
                               w.vals_a, (const uint64_t*)w.keys_a, (const double*)w.xs, (const double*)w.ys,
                               w.xyh, w.hmax_bits, pad, s, (const int32_t*)w.flag, (const int32_t*)w.idx_a,
                               (const int32_t*)cur, mlist, mcount);
            hipLaunchKernelGGL(k_merge_remap_slots, dim3((unsigned)cdiv(nprev, 256)), dim3(256), 0,
                               c->stream, nprev, (const int32_t*)w.flag, (const int32_t*)w.idx_a,
                               (const int32_t*)cur, nxt, affected);
            nv = nbr_view(c);
            hipLaunchKernelGGL(k_merge_mark, dim3((unsigned)cdiv((int64_t)nmerged * MG, 256)), dim3(256), 0,
                               c->stream, c->grid, nv, nmerged, (const int32_t*)mlist, affected,
                               (const unsigned long long*)pad);
            LAUNCHCHK(c, "merge_remap");
            int32_t* tsw = cur; cur = nxt; nxt = tsw;
        }
        const unsigned nbs = (unsigned)cdiv(nsorted, 256);
        const unsigned nb = (unsigned)cdiv(n, 256);
        // sorted-order records of the mergeability data (the rate passes'
        // record buffer is free during adaptation)
        MergeRec* mrec = (MergeRec*)w.pa;
        hipLaunchKernelGGL(k_merge_pack, dim3(nbs), dim3(256), 0, c->stream, nsorted,
                           (const int32_t*)nv.perm, s, cf.mmax_f, mrec);
        hipLaunchKernelGGL(k_merge_closest, dim3((unsigned)cdiv((int64_t)nsorted * MG, 256)), dim3(256), 0,
                           c->stream, c->grid, nv, nsorted, s, cf.mass_q, cf.mmax_f, (const MergeRec*)mrec,
                           cur, reuse ? (const int32_t*)affected : (const int32_t*)nullptr,
                           reuse ? (const unsigned long long*)pad : (const unsigned long long*)nullptr);
        hipLaunchKernelGGL(k_merge_keep, dim3(nb), dim3(256), 0, c->stream, n, cur, w.flag);
        LAUNCHCHK(c, "merge_closest");
        // number of pairs = number of deleted slots
        int32_t nkeep = 0;
        // the merged state is written while the host waits for the count
        rc = compact_ranks(c, n, w.flag, w.idx_a, &nkeep, [&] {
            hipLaunchKernelGGL(k_merge_apply, dim3(nb), dim3(256), 0, c->stream, c->grid, n, s, d,
                               cur, w.flag, w.idx_a, cf.mass_q);
        });
        if (rc) return rc;
        map->n_merged[it] = n - nkeep;
        rc = copy_state(c, d, s, nkeep);
        if (rc) return rc;
        nprev = n;
        nmerged = n - nkeep;
        n = nkeep;
    }

    // One CSR serves every shift and the h update: each shift moves a
    // particle by at most 0.25 h (the limiter), so after k shifts a pair's
    // distance changed by at most 0.5 k max(h_i, h_j) and every later
    // neighbour pair lies within (1 + k/6) of the support radius now.  The
    // kernels re-apply the exact predicate to the ascending rows, so the
    // sums are those of a fresh neighbour list.  If that superset does not
    // fit the internal buffer, each pass builds its own exact list.
    //
    // The superset is first built tighter than that worst case: with radius
    // factor sf it covers every later pair while the shifts so far moved
    // the particles by sum_k D_k <= 1.5 (sf - 1), D_k the largest |dr|/h of
    // shift k (a pair's distance changes by at most 2 D_k max(h_i, h_j) per
    // shift).  Each shift publishes its D_k; once the sum would leave the
    // allowance the superset is rebuilt with the worst-case factor for the
    // shifts that remain.
    bool super = false;
    double allow = 0.0, spent = 0.0;  // allow < 0: worst-case rows, no check
    auto build_super = [&](int remaining, bool tight) -> int {
        const double sf = tight ? 1.0 + SHIFT_SKIN : 1.0 + remaining / 6.0;
        int r = internal_csr(c, n, ps->x, ps->y, ps->h, sf + 1e-9);
        allow = tight ? 1.5 * SHIFT_SKIN : -1.0;
        spent = 0.0;
        return r;
    };
    if (n > 0) {
        rc = build_super(cf.shift_iters, cf.shift_iters > 0);
        if (rc == SPH_OK) super = true;
        else if (rc != SPH_E_NOMEM) return rc;  // a superset that does not fit: exact lists
    }
    unsigned long long* dmax = (unsigned long long*)(w.ctr + 4);
    // each shift first filters its rows into the rate-list buffer (free
    // here; it is rebuilt after adaptation) when that holds every row
    const bool filt = w.cnt_ex && (int64_t)w.nl_k * w.capacity >= w.col_cap;
    for (int it = 0; it < cf.shift_iters; ++it) {
        if (n == 0) break;
        if (!super) {
            rc = internal_csr(c, n, ps->x, ps->y, ps->h);
            if (rc) return rc;
        } else if (allow >= 0.0 && spent > allow) {
            rc = build_super(cf.shift_iters - it, false);
            if (rc) return rc;
        }
        const bool measure = super && allow >= 0.0;
        if (measure) hipLaunchKernelGGL(k_clear_u64, dim3(1), dim3(64), 0, c->stream, dmax, 1);
        const unsigned nb = (unsigned)cdiv(n, 256);
        const unsigned nbg = (unsigned)cdiv((int64_t)n * SHIFT_G, 256);
        // packed records in the rate passes' buffers (free during adaptation);
        // rows in the sorted order of the last build (slots unchanged since)
        double4 *pA = w.pa, *pB = (double4*)w.pf;
        hipLaunchKernelGGL(k_pack_shift, dim3(nb), dim3(256), 0, c->stream, n, s, cf.mass_q, cf.rho0, pA,
                           pB);
        if (filt) {
            hipLaunchKernelGGL(k_shift_filter, dim3((unsigned)cdiv((int64_t)n * FG, 256)), dim3(256), 0,
                               c->stream, c->grid, n, (const int32_t*)s.kind, (const double4*)pA,
                               w.rp_tmp, w.col_tmp, w.nl_idx, w.cnt_ex, (const int32_t*)w.vals_a);
            hipLaunchKernelGGL(k_shift_taylor<true>, dim3(nbg), dim3(256), 0, c->stream, c->grid, n,
                               (const int32_t*)s.kind, (const double4*)pA, (const double4*)pB, w.rp_tmp,
                               w.nl_idx, (const int32_t*)w.cnt_ex, cf.rho0, w.tmp_d[0], w.tmp_d[1],
                               w.tmp_d[2], w.tmp_d[3], w.tmp_d[4], (const int32_t*)w.vals_a,
                               measure ? dmax : nullptr);
        } else {
            hipLaunchKernelGGL(k_shift_taylor<false>, dim3(nbg), dim3(256), 0, c->stream, c->grid, n,
                               (const int32_t*)s.kind, (const double4*)pA, (const double4*)pB, w.rp_tmp,
                               w.col_tmp, (const int32_t*)nullptr, cf.rho0, w.tmp_d[0], w.tmp_d[1],
                               w.tmp_d[2], w.tmp_d[3], w.tmp_d[4], (const int32_t*)w.vals_a,
                               measure ? dmax : nullptr);
        }
        hipLaunchKernelGGL(k_shift_apply, dim3(nb), dim3(256), 0, c->stream, c->grid, n, s, w.tmp_d[0],
                           w.tmp_d[1], w.tmp_d[2], w.tmp_d[3], w.tmp_d[4]);
        LAUNCHCHK(c, "shift");
        if (measure) {
            unsigned long long bits = 0;
            const Readback rb{&bits, dmax, 8};
            rc = readback(c, &rb, 1);
            if (rc) return rc;
            double d = 0.0;
            memcpy(&d, &bits, sizeof(d));
            // bound taken with a margin for the rounding of |dr| / h
            spent += d * (1.0 + 1e-12) + 1e-15;
        }
    }
    if (n > 0) {
        if (!super) {
            rc = internal_csr(c, n, ps->x, ps->y, ps->h);
            if (rc) return rc;
        } else if (allow >= 0.0 && spent > allow) {
            // the h update needs the neighbours of the final positions
            rc = internal_csr(c, n, ps->x, ps->y, ps->h);
            if (rc) return rc;
        }
        unsigned nb = (unsigned)cdiv(n, 256);
        hipLaunchKernelGGL(k_pack_shift, dim3(nb), dim3(256), 0, c->stream, n, s, cf.mass_q, 0.0, w.pa,
                           (double4*)w.pf);
        hipLaunchKernelGGL(k_hupdate, dim3((unsigned)cdiv((int64_t)n * SHIFT_G, 256)), dim3(256), 0,
                           c->stream, c->grid, n, w.rp_tmp, w.col_tmp,
                           (const double4*)w.pa, (const double*)ps->rho, (const int32_t*)ps->kind,
                           cf.hdx, w.tmp_d[0], (const int32_t*)w.vals_a);
        hipLaunchKernelGGL(k_copy_f64, dim3(nb), dim3(256), 0, c->stream, n, w.tmp_d[0], ps->h);
        LAUNCHCHK(c, "hupdate");
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    ps->n = n;
    return SPH_OK;
}

// ---------------------------------------------------------------------------
// Background update (section 3.3)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_bg_mask(Grid g, NbrView nv, int nb,
                                                 const double* __restrict__ bx,
                                                 const double* __restrict__ by,
                                                 const double* __restrict__ bh,
                                                 const double* __restrict__ phi, double phi_thresh,
                                                 double ds_min, int32_t* mask, double* ds,
                                                 int have_solids, int first)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    int m = 0;
    if (have_solids) {
        const double xi = bx[b], yi = by[b], hi = bh[b];
        for_each_neighbor(g, nv, xi, yi, hi, level_of(g, hi),
                          [&](int, double, double, double, double) { m = 1; });
    }
    // solution mark (bit 2): set from phi in the first pass of an update
    // (cleared when phi is not given), kept by later passes and by split
    // children; a marked particle is refined like one near a body
    const int sol = first ? ((phi && phi[b] > phi_thresh) ? 2 : 0) : (mask[b] & 2);
    if (sol) m |= 3;
    mask[b] = m;
    if (m) ds[b] = ds_min;
}

// Long accumulator: the exact sum of doubles, rounded once.  A finite
// double is an integer multiple of 2^-1074, so the sum is V 2^-1074 with V
// an integer, kept here as signed base-2^32 digits in int64 cells (each
// addition puts at most 2^33 into a cell, so 2^30 additions never overflow
// one).  Only the cells lo..hi that the terms reached are kept (the others
// are zero), so a row whose terms span a few binades costs a few cells.
// get() returns V rounded to 53 significant bits, ties to even, times
// 2^-1074: the correctly rounded sum, the same in any order of the terms.
// The cells live in private memory; it is used only for the rows the fast
// path below cannot prove.
struct XSum {
    static constexpr int NC = 72;  // a double reaches cells 0..65; three above for carries
    long long d[NC];
    int lo = NC, hi = -1;
    // cells a..b valid, the new ones zero
    __device__ __forceinline__ void touch(int a, int b)
    {
        if (hi < lo) {
            for (int i = a; i <= b; ++i) d[i] = 0;
            lo = a;
            hi = b;
            return;
        }
        for (int i = a; i < lo; ++i) d[i] = 0;
        for (int i = hi + 1; i <= b; ++i) d[i] = 0;
        if (a < lo) lo = a;
        if (b > hi) hi = b;
    }
    __device__ __forceinline__ void add(double x)
    {
        if (x == 0.0) return;
        const unsigned long long bits = (unsigned long long)__double_as_longlong(x);
        const int ex = (int)((bits >> 52) & 0x7ff);
        unsigned long long m = bits & 0xfffffffffffffull;
        int p = 0;  // x = m 2^(p - 1074)
        if (ex != 0) {
            m |= 1ull << 52;
            p = ex - 1;
        }
        const int k = p >> 5, sh = p & 31;
        const unsigned long long a = (m & 0xffffffffull) << sh, b = (m >> 32) << sh;
        long long c0 = (long long)(a & 0xffffffffull);
        long long c1 = (long long)((a >> 32) + (b & 0xffffffffull));
        long long c2 = (long long)(b >> 32);
        if (bits >> 63) {
            c0 = -c0;
            c1 = -c1;
            c2 = -c2;
        }
        touch(k, k + 2);
        d[k] += c0;
        d[k + 1] += c1;
        d[k + 2] += c2;
    }
    // cells lo..top-1 to digits in [0, 2^32), cell top keeping the sign
    __device__ __forceinline__ void normalise(int top)
    {
        for (int i = lo; i < top; ++i) {
            const long long c = d[i] >> 32;
            d[i] &= 0xffffffffll;
            d[i + 1] += c;
        }
    }
    __device__ bool get(double& out)
    {
        if (hi < lo) {
            out = 0.0;
            return true;
        }
        const int top = hi + 3;  // <= 68: room for the carries out of hi
        touch(lo, top);
        normalise(top);
        const bool neg = d[top] < 0;
        if (neg) {
            for (int i = lo; i <= top; ++i) d[i] = -d[i];
            normalise(top);
        }
        int t = top;
        while (t >= lo && d[t] == 0) --t;
        if (t < lo) {
            out = 0.0;
            return true;
        }
        auto cell = [&](int i) -> unsigned long long {
            return (i >= lo && i <= top) ? (unsigned long long)d[i] : 0ull;
        };
        const unsigned long long w_hi = cell(t);
        const int bl = 64 - __clzll(w_hi);  // bits of the top digit
        const int nb = 32 * t + bl;          // bits of |V|
        double r;
        if (nb <= 53) {
            r = ldexp((double)((cell(1) << 32) | cell(0)), -1074);
        } else {
            // 96-bit window of the top three digits; what lies below it only
            // decides a tie
            const unsigned long long w_lo = (cell(t - 1) << 32) | cell(t - 2);
            const int cut = bl + 11;  // window bits below the 53 kept
            unsigned long long kept = (w_hi << (64 - cut)) | (w_lo >> cut);
            const unsigned long long rem = w_lo & ((1ull << cut) - 1);
            const unsigned long long half = 1ull << (cut - 1);
            bool below = false;
            for (int i = lo; i < t - 2 && !below; ++i) below = d[i] != 0;
            if (rem > half || (rem == half && (below || (kept & 1ull)))) ++kept;
            r = ldexp((double)kept, nb - 53 - 1074);
        }
        out = neg ? -r : r;
        return true;
    }
};

// Smallest spacing of the doubles next to v (below |v| when |v| is a power
// of two): 2^-1074 at zero and among the subnormals.
__device__ __forceinline__ double spacing_min(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v) & 0x7fffffffffffffffull;
    const int be = (int)(b >> 52);
    if (be == 0) return ldexp(1.0, -1074);
    const bool pow2 = (b & 0xfffffffffffffull) == 0;
    return ldexp(1.0, (pow2 && be > 1) ? be - 1076 : be - 1075);
}

__device__ __forceinline__ void two_sum(double x, double y, double& t, double& e)
{
    t = x + y;
    const double z = t - x;
    e = (x - (t - z)) + (y - z);
}

// The fast path to the same result: a two-level cascade of Knuth's TwoSum.
// The running sum s takes each term, the first-level sum c1 takes each exact
// error of s (again by TwoSum), and c2 adds up the exact errors e_k of c1
// with their magnitudes in a; so the exact sum is S = s + c1 + sum e_k, and
// |c2 - sum e_k| <= gamma_{n-1} sum |e_k| (recursive summation, any order
// or grouping).  get() forms res = s + c1 + c2 by exact steps up to one
// rounding, whose exact error is kept: when the known errors plus that bound
// (with margins for its own rounding) are below half the spacing of the
// doubles at res, S lies strictly inside res's rounding interval and res is
// the correctly rounded sum.  The bound is about n^2 u^3 sum|x|, so sums that
// cancel down to about 1e-30 of their terms are proven; get() returns false
// for the rest, and the row is summed again with XSum.  Partial sums of a
// lane group merge by the same steps.
struct FSum {
    double s = 0.0, c1 = 0.0, c2 = 0.0, a = 0.0;
    int n = 0;
    __device__ __forceinline__ void add(double x)
    {
        double e1, e2;
        two_sum(s, x, s, e1);
        two_sum(c1, e1, c1, e2);
        c2 += e2;
        a += fabs(e2);
        ++n;
    }
    // adds the partial sum held by lane (this lane ^ o) of the wave; both
    // lanes of the pair end with the same value
    __device__ __forceinline__ void merge_xor(int o)
    {
        const double s2 = __shfl_xor(s, o, 64), c12 = __shfl_xor(c1, o, 64);
        const double c22 = __shfl_xor(c2, o, 64), a2 = __shfl_xor(a, o, 64);
        const int n2 = __shfl_xor(n, o, 64);
        add(s2);
        add(c12);
        c2 += c22;
        a += a2;
        n += n2;
    }
    __device__ __forceinline__ bool get(double& out) const
    {
        double u1, v1, u2, v2, res, v3;
        two_sum(s, c1, u1, v1);
        two_sum(v1, c2, u2, v2);
        two_sum(u1, u2, res, v3);
        // S = res + v3 + v2 + (sum e_k - c2)
        if (v2 == 0.0 && a == 0.0) {
            // every e_k is zero and u2 = v1 + c2 exactly: S = u1 + u2, and
            // res is its round-to-nearest-even, ties included
            out = res;
            return true;
        }
        const double g = 2.0 * (double)(n + 2) * 0x1p-53;  // >= gamma_{n-1} / (1 - gamma_{n-1})
        const double bound = (fabs(v3) + fabs(v2) + g * a) * (1.0 + 0x1p-40);
        if (2.0 * bound < spacing_min(res)) {
            out = res;
            return true;
        }
        return false;
    }
};

// lanes per particle of the background sweeps
#define BG_G 4

// Sorted copies for the background sweeps, so that a cell run's records are
// consecutive: ds_s[sp] = ds[perm[sp]], m_s[sp] = (mq[perm[sp]] q) / rho0 (the
// volume the shifting term takes, divided once per particle: the same
// correctly rounded quotient as per pair).
__global__ __launch_bounds__(256) void k_bg_pack(int nb, const int32_t* __restrict__ perm,
                                                 const double* __restrict__ ds,
                                                 const int64_t* __restrict__ mq, double q,
                                                 double rho0, double* ds_s, double* m_s)
{
    const int sp = blockIdx.x * blockDim.x + threadIdx.x;
    if (sp >= nb) return;
    const int b = perm[sp];
    if (ds_s) ds_s[sp] = ds[b];
    if (m_s) m_s[sp] = ((double)mq[b] * q) / rho0;
}

// Size grading of background particle b (sorted position sp, lane gl of its
// group of G) over its neighbours, step 2 of section 3.3.  Acc sums the
// logarithms of the sizes (the walk is not in slot order; the sum is
// rounded once); returns false when Acc cannot prove its sum, and then
// writes nothing.  Every lane of the group returns the same.
template <int G, class Acc>
__device__ __forceinline__ bool bg_grade_row(const Grid& g, const NbrView& nv, int sp, int gl,
                                             const int32_t* __restrict__ mask,
                                             const double* __restrict__ ds,
                                             const double* __restrict__ ds_s, double cr,
                                             double ds_min, double ds_max, double* nds)
{
    const int b = nv.perm[sp];
    if (mask[b]) {
        if (gl == 0) nds[b] = ds[b];
        return true;
    }
    double mn = HUGE_VAL, mx = -HUGE_VAL;
    Acc sl;
    int cnt = 0;
    group_walk_x<G>(g, nv, ds_s, nv.xs[sp], nv.ys[sp], nv.hs[sp], key_level(g, nv.keys[sp]), gl,
                    [&](int, bool pass, double, double, double, double, double v) {
                      if (!pass) return;
                      mn = fmin(mn, v);
                      mx = fmax(mx, v);
                      sl.add(log(v));
                      ++cnt;
                  });
    if constexpr (G > 1) {
#pragma unroll
        for (int o = 1; o < G; o <<= 1) {
            mn = fmin(mn, __shfl_xor(mn, o, 64));
            mx = fmax(mx, __shfl_xor(mx, o, 64));
            cnt += __shfl_xor(cnt, o, 64);
            sl.merge_xor(o);
        }
    }
    const double cr3 = cr * cr * cr;
    double v;
    if (mx / mn < cr3) {
        v = cr * mn;
    } else {
        double sum;
        if (!sl.get(sum)) return false;
        v = exp(sum / (double)cnt);
    }
    if (v < ds_min) v = ds_min;
    if (v > ds_max) v = ds_max;
    if (gl == 0) nds[b] = v;
    return true;
}

// fast path, BG_G lanes per particle; redo[sp] = 1 where the exact sum is needed
__global__ __launch_bounds__(256) void k_bg_grade(Grid g, NbrView nv, int nb,
                                                  const int32_t* __restrict__ mask,
                                                  const double* __restrict__ ds,
                                                  const double* __restrict__ ds_s, double cr,
                                                  double ds_min, double ds_max, double* nds,
                                                  int32_t* redo)
{
    const int t = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const int sp = t / BG_G, gl = t % BG_G;
    if (sp >= nb) return;
    const bool ok = bg_grade_row<BG_G, FSum>(g, nv, sp, gl, mask, ds, ds_s, cr, ds_min, ds_max, nds);
    if (gl == 0) redo[sp] = ok ? 0 : 1;
}

__global__ __launch_bounds__(256) void k_bg_grade_exact(Grid g, NbrView nv, int nb,
                                                        const int32_t* __restrict__ mask,
                                                        const double* __restrict__ ds,
                                                        const double* __restrict__ ds_s, double cr,
                                                        double ds_min, double ds_max, double* nds,
                                                        const int32_t* __restrict__ redo)
{
    const int sp = blockIdx.x * blockDim.x + threadIdx.x;
    if (sp >= nb || !redo[sp]) return;
    bg_grade_row<1, XSum>(g, nv, sp, 0, mask, ds, ds_s, cr, ds_min, ds_max, nds);
}

__global__ __launch_bounds__(256) void k_bg_setds(int nb, const double* __restrict__ nds,
                                                  double rho0, double* ds, double* mref)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    ds[b] = nds[b];
    mref[b] = rho0 * (nds[b] * nds[b]);
}

__global__ __launch_bounds__(256) void k_bg_split_flags(int nb, const int64_t* __restrict__ mq,
                                                        const double* __restrict__ mref, double q,
                                                        double mmax_f, int32_t* flag)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    flag[b] = ((double)mq[b] * q > mmax_f * mref[b]) ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_bg_split_apply(Grid g, int nb, sph_background B,
                                                        const int32_t* __restrict__ flag,
                                                        const int32_t* __restrict__ rank,
                                                        double alpha, double eps)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb || !flag[b]) return;
    const double ck[6] = {1.0, 0.5, -0.5, -1.0, -0.5, 0.5};
    const double sk[6] = {0.0, SPH_SIN60, SPH_SIN60, 0.0, -SPH_SIN60, -SPH_SIN60};
    const int64_t c = B.mq[b] / 7;
    const double r = eps * B.h[b];
    const double hc = alpha * B.h[b];
    const int64_t base = (int64_t)nb + 6 * (int64_t)rank[b];
    for (int k = 0; k < 6; ++k) {
        int64_t t = base + k;
        B.x[t] = wrap_axis(g, 0, B.x[b] + r * ck[k]);
        B.y[t] = wrap_axis(g, 1, B.y[b] + r * sk[k]);
        B.h[t] = hc;
        B.ds[t] = B.ds[b];
        B.mask[t] = B.mask[b];
        B.mref[t] = B.mref[b];
        B.mq[t] = c;
    }
    B.mq[b] = B.mq[b] - 6 * c;
    B.h[b] = hc;
}

// Background h smoothing and shifting, section 3.3: the new h is the mean of
// the target from the neighbour count and the neighbours' mean h; the shift
// is the limited Lind shift of eqs. (shift-deltar) and (shift-limit) with
// volume m_j / rho0 and the gradient at h_ij.  Particle sp (slot b) of the
// background's own build, lane gl of its group of G, walking its cells: no
// neighbour list, so a particle may have any number of neighbours (a coarse
// particle among fine ones early in the initial passes has thousands).  The
// walk order is not the slot order, so the sums over neighbours (of h_j and
// of the shift terms) are exact sums rounded once: their results follow from
// the neighbour set alone.  Every lane of the group returns the same.
template <int G, class Acc>
__device__ __forceinline__ bool bg_smooth_row(const Grid& g, const NbrView& nv, int sp, int gl,
                                              const double* __restrict__ m_s, double rho0,
                                              double n_r, double* nh, double* ddx, double* ddy)
{
    const int b = nv.perm[sp];
    const double xb = nv.xs[sp], yb = nv.ys[sp], hb = nv.hs[sp];
    const double fxi = kern_f<double>(SPH_XI);
    Acc sh, sx, sy;
    int cnt = 0;
    group_walk_x<G>(g, nv, m_s, xb, yb, hb, key_level(g, nv.keys[sp]), gl,
                    [&](int, bool pass, double dx, double dy, double r2, double hj, double vj) {
                      // vj = m_j / rho0
                      if (!pass) return;
                      ++cnt;
                      sh.add(hj);
                      const double r = sqrt(r2);
                      if (r <= 0.0) return;
                      const double hij = 0.5 * (hb + hj);
                      const double wr = kern_f<double>(r / hij) / fxi;
                      const double coef = vj * (1.0 + 0.24 * ((wr * wr) * (wr * wr)));
                      const double t = coef * (kern_dw64(r, hij) / r);
                      sx.add(t * dx);
                      sy.add(t * dy);
                  });
    if constexpr (G > 1) {
#pragma unroll
        for (int o = 1; o < G; o <<= 1) {
            cnt += __shfl_xor(cnt, o, 64);
            sh.merge_xor(o);
            sx.merge_xor(o);
            sy.merge_xor(o);
        }
    }
    double vsh, vsx, vsy;
    const bool ok = sh.get(vsh) & sx.get(vsx) & sy.get(vsy);
    if (!ok) return false;
    if (gl) return true;
    const double N = (double)cnt;
    nh[b] = 0.5 * ((hb / 2.0) * (1.0 + sqrt(n_r / N)) + vsh / N);
    const double pref = -0.5 * (hb * hb);
    double dxs = pref * vsx, dys = pref * vsy;
    const double mag = sqrt(dxs * dxs + dys * dys);
    const double lim = 0.25 * hb;
    if (mag > lim) {
        const double th = lim / mag;
        dxs = dxs * th;
        dys = dys * th;
    }
    ddx[b] = dxs;
    ddy[b] = dys;
    return true;
}

// fast path, BG_G lanes per particle; redo[sp] = 1 where an exact sum is needed
__global__ __launch_bounds__(256) void k_bg_smooth_walk(Grid g, NbrView nv, int nb,
                                                        const double* __restrict__ m_s, double rho0,
                                                        double n_r, double* nh, double* ddx,
                                                        double* ddy, int32_t* redo)
{
    const int t = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const int sp = t / BG_G, gl = t % BG_G;
    if (sp >= nb) return;
    const bool ok = bg_smooth_row<BG_G, FSum>(g, nv, sp, gl, m_s, rho0, n_r, nh, ddx, ddy);
    if (gl == 0) redo[sp] = ok ? 0 : 1;
}

// The rows the fast path could not prove: each of the three sums in a walk
// of its own with one long accumulator (one accumulator keeps the private
// memory per lane, and with it the launch, small).
__global__ __launch_bounds__(256) void k_bg_smooth_exact(Grid g, NbrView nv, int nb,
                                                         const double* __restrict__ m_s, double rho0,
                                                         double n_r, double* nh, double* ddx,
                                                         double* ddy, const int32_t* __restrict__ redo)
{
    const int sp = blockIdx.x * blockDim.x + threadIdx.x;
    if (sp >= nb || !redo[sp]) return;
    const int b = nv.perm[sp];
    const double xb = nv.xs[sp], yb = nv.ys[sp], hb = nv.hs[sp];
    const int lb = key_level(g, nv.keys[sp]);
    const double fxi = kern_f<double>(SPH_XI);
    double v[3];
    int cnt = 0;
    for (int which = 0; which < 3; ++which) {
        XSum acc;
        for_each_neighbor(g, nv, xb, yb, hb, lb, [&](int js, double dx, double dy, double r2, double hj) {
            if (which == 0) {
                ++cnt;
                acc.add(hj);
                return;
            }
            const double r = sqrt(r2);
            if (r <= 0.0) return;
            const double hij = 0.5 * (hb + hj);
            const double wr = kern_f<double>(r / hij) / fxi;
            const double vj = m_s[js];  // m_j / rho0
            const double coef = vj * (1.0 + 0.24 * ((wr * wr) * (wr * wr)));
            const double t = coef * (kern_dw64(r, hij) / r);
            acc.add(t * (which == 1 ? dx : dy));
        });
        acc.get(v[which]);
    }
    const double N = (double)cnt;
    nh[b] = 0.5 * ((hb / 2.0) * (1.0 + sqrt(n_r / N)) + v[0] / N);
    const double pref = -0.5 * (hb * hb);
    double dxs = pref * v[1], dys = pref * v[2];
    const double mag = sqrt(dxs * dxs + dys * dys);
    const double lim = 0.25 * hb;
    if (mag > lim) {
        const double th = lim / mag;
        dxs = dxs * th;
        dys = dys * th;
    }
    ddx[b] = dxs;
    ddy[b] = dys;
}

__global__ __launch_bounds__(256) void k_bg_smooth_apply(Grid g, int nb, sph_background B,
                                                         const double* __restrict__ nh,
                                                         const double* __restrict__ ddx,
                                                         const double* __restrict__ ddy)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    B.h[b] = nh[b];
    B.x[b] = wrap_axis(g, 0, B.x[b] + ddx[b]);
    B.y[b] = wrap_axis(g, 1, B.y[b] + ddy[b]);
}

int bg_update_run(sph_ctx* c, sph_background* bg, const sph_particles* solids, const double* phi,
                  double phi_thresh, int passes, int64_t* nsplit)
{
    Work& w = c->w;
    const sph_config& cf = c->cfg;
    *nsplit = 0;
    int nb = (int)bg->n;
    const int ns = (int)solids->n;
    for (int pass = 0; pass < passes; ++pass) {
        if (nb == 0) break;
        unsigned nbk = (unsigned)cdiv(nb, 256);
        // step 1: boundary mask
        if (ns > 0) {
            int rc = nbr_build(c, ns, solids->x, solids->y, solids->h);
            if (rc) return rc;
        }
        NbrView sv = nbr_view(c);
        hipLaunchKernelGGL(k_bg_mask, dim3(nbk), dim3(256), 0, c->stream, c->grid, sv, nb, bg->x,
                           bg->y, bg->h, pass == 0 ? phi : nullptr, phi_thresh, cf.ds_min, bg->mask,
                           bg->ds, ns > 0 ? 1 : 0, pass == 0 ? 1 : 0);
        LAUNCHCHK(c, "bg_mask");
        // step 2: size grading (Jacobi)
        int rc = nbr_build(c, nb, bg->x, bg->y, bg->h);
        if (rc) return rc;
        NbrView nv = nbr_view(c);
        hipLaunchKernelGGL(k_bg_pack, dim3(nbk), dim3(256), 0, c->stream, nb, nv.perm, (const double*)bg->ds,
                           (const int64_t*)nullptr, 0.0, cf.rho0, w.tmp_d[3], (double*)nullptr);
        hipLaunchKernelGGL(k_bg_grade, dim3((unsigned)cdiv((int64_t)nb * BG_G, 256)), dim3(256), 0, c->stream,
                           c->grid, nv, nb, bg->mask, bg->ds, (const double*)w.tmp_d[3], cf.cr, cf.ds_min,
                           cf.ds_max, w.tmp_d[0], w.tmp_i32[0]);
        hipLaunchKernelGGL(k_bg_grade_exact, dim3(nbk), dim3(256), 0, c->stream, c->grid, nv, nb,
                           bg->mask, bg->ds, (const double*)w.tmp_d[3], cf.cr, cf.ds_min, cf.ds_max,
                           w.tmp_d[0], w.tmp_i32[0]);
        hipLaunchKernelGGL(k_bg_setds, dim3(nbk), dim3(256), 0, c->stream, nb, w.tmp_d[0], cf.rho0,
                           bg->ds, bg->mref);
        LAUNCHCHK(c, "bg_grade");
        // step 3: split
        hipLaunchKernelGGL(k_bg_split_flags, dim3(nbk), dim3(256), 0, c->stream, nb, bg->mq, bg->mref,
                           cf.bg_mass_q, cf.mmax_f, w.flag);
        int32_t cnt = 0;
        rc = compact_ranks(c, nb, w.flag, w.idx_a, &cnt);
        if (rc) return rc;
        if ((int64_t)nb + 6 * (int64_t)cnt > bg->capacity) {
            set_err(c, "background split needs %lld slots, capacity %lld",
                    (long long)nb + 6 * (long long)cnt, (long long)bg->capacity);
            bg->n = nb;
            return SPH_E_CAPACITY;
        }
        hipLaunchKernelGGL(k_bg_split_apply, dim3(nbk), dim3(256), 0, c->stream, c->grid, nb, *bg,
                           w.flag, w.idx_a, cf.split_alpha, cf.split_eps);
        LAUNCHCHK(c, "bg_split");
        *nsplit += cnt;
        nb += 6 * cnt;
        // step 4: h smoothing + shifting (a cell walk: rows of any length)
        for (int it = 0; it < cf.bg_smooth_iters; ++it) {
            rc = nbr_build(c, nb, bg->x, bg->y, bg->h);
            if (rc) return rc;
            unsigned nbk2 = (unsigned)cdiv(nb, 256);
            const NbrView nv2 = nbr_view(c);
            hipLaunchKernelGGL(k_bg_pack, dim3(nbk2), dim3(256), 0, c->stream, nb, nv2.perm,
                               (const double*)nullptr, (const int64_t*)bg->mq, cf.bg_mass_q, cf.rho0,
                               (double*)nullptr, w.tmp_d[3]);
            hipLaunchKernelGGL(k_bg_smooth_walk, dim3((unsigned)cdiv((int64_t)nb * BG_G, 256)), dim3(256), 0,
                               c->stream, c->grid, nv2, nb, (const double*)w.tmp_d[3], cf.rho0, cf.n_r,
                               w.tmp_d[0], w.tmp_d[1], w.tmp_d[2], w.tmp_i32[0]);
            hipLaunchKernelGGL(k_bg_smooth_exact, dim3(nbk2), dim3(256), 0, c->stream, c->grid, nv2, nb,
                               (const double*)w.tmp_d[3], cf.rho0, cf.n_r, w.tmp_d[0], w.tmp_d[1],
                               w.tmp_d[2], w.tmp_i32[0]);
            hipLaunchKernelGGL(k_bg_smooth_apply, dim3(nbk2), dim3(256), 0, c->stream, c->grid, nb, *bg,
                               w.tmp_d[0], w.tmp_d[1], w.tmp_d[2]);
            LAUNCHCHK(c, "bg_smooth");
        }
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    bg->n = nb;
    return SPH_OK;
}

// ---------------------------------------------------------------------------
// Inlet / outlet update (section 2.2)
// ---------------------------------------------------------------------------

// Flags of the update and their counts, added to cumulative counters (the
// host takes differences): cnt[0] fluid -> outlet, cnt[1] inlet copies,
// cnt[2] deletions (one atomic per wave and counter).
// In a run of steps (gd.trip set) a slot change trips the run: the host
// applies it, the rest of the run is skipped.
__global__ __launch_bounds__(256) void k_io_flags(int n, const double* __restrict__ x,
                                                  const int32_t* __restrict__ kind,
                                                  sph_inout_params io, int32_t* keep, int32_t* app,
                                                  unsigned long long* cnt, Guard gd)
{
    if (guard_stop(gd)) return;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = i < n ? kind[i] : -1;
    const double xi = i < n ? x[i] : 0.0;
    const bool to_out = k == SPH_FLUID && xi >= io.x_out;
    const bool ap = k == SPH_INLET && xi >= io.x_in;
    const bool del = k == SPH_OUTLET && xi >= io.x_out + io.len_out;
    const uint64_t b0 = __ballot(to_out), b1 = __ballot(ap), b2 = __ballot(del);
    if (__lane_id() == 0) {
        if (b0) atomicAdd(cnt + 0, (unsigned long long)__popcll(b0));
        if (b1) atomicAdd(cnt + 1, (unsigned long long)__popcll(b1));
        if (b2) atomicAdd(cnt + 2, (unsigned long long)__popcll(b2));
        if (b1 | b2) guard_trip(gd);
    }
    if (i >= n) return;
    keep[i] = !del;
    app[i] = ap;
}

// Kind changes only (no copy, no deletion): fluid past x_out becomes outlet.
__global__ __launch_bounds__(256) void k_io_kinds(int n, const double* __restrict__ x, int32_t* kind,
                                                  sph_inout_params io, Guard gd)
{
    if (guard_stop(gd)) return;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && kind[i] == SPH_FLUID && x[i] >= io.x_out) kind[i] = SPH_OUTLET;
}

// Kept slot i goes to rank_keep[i] with its new kind; an inlet particle
// that entered the fluid also leaves a copy at nkeep + rank_app[i], moved
// back by the inlet length.
__global__ __launch_bounds__(256) void k_io_apply(int n, FluidState s, FluidState d,
                                                  const int32_t* __restrict__ keep,
                                                  const int32_t* __restrict__ rk,
                                                  const int32_t* __restrict__ app,
                                                  const int32_t* __restrict__ ra, int nkeep,
                                                  sph_inout_params io)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int k = s.kind[i];
    const double xi = s.x[i];
    auto put = [&](int t) {
        d.x[t] = xi; d.y[t] = s.y[i]; d.u[t] = s.u[i]; d.v[t] = s.v[i]; d.p[t] = s.p[i];
        d.rho[t] = s.rho[i]; d.h[t] = s.h[i]; d.mref[t] = s.mref[i]; d.mq[t] = s.mq[i];
        d.origin[t] = i;
    };
    if (keep[i]) {
        const int t = rk[i];
        put(t);
        int nk = k;
        if (k == SPH_INLET && xi >= io.x_in) nk = SPH_FLUID;
        else if (k == SPH_FLUID && xi >= io.x_out) nk = SPH_OUTLET;
        d.kind[t] = nk;
    }
    if (app[i]) {
        const int t = nkeep + ra[i];
        put(t);
        d.x[t] = xi - io.len_in;
        d.kind[t] = SPH_INLET;
    }
}

__global__ __launch_bounds__(256) void k_io_copy(int n, FluidState d, FluidState s, int64_t* origin)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    s.x[t] = d.x[t]; s.y[t] = d.y[t]; s.u[t] = d.u[t]; s.v[t] = d.v[t]; s.p[t] = d.p[t];
    s.rho[t] = d.rho[t]; s.h[t] = d.h[t]; s.mref[t] = d.mref[t]; s.mq[t] = d.mq[t];
    s.kind[t] = d.kind[t];
    origin[t] = d.origin[t];
}

int inout_run(sph_ctx* c, sph_particles* ps, const sph_inout_params* io, sph_inout_map* map,
              bool precheck)
{
    Work& w = c->w;
    const int n = (int)ps->n;
    map->n_appended = map->n_deleted = map->n_to_outlet = 0;
    map->n_required = n;
    if (n == 0) return SPH_OK;
    const unsigned nb = (unsigned)cdiv(n, 256);
    // scratch that the neighbour structure does not use, so that an update
    // which keeps every slot leaves the rate passes' list valid
    int32_t *keep = w.flag, *rk = w.idx_a, *app = w.tmp_i32[1], *ra = w.closest;
    unsigned long long* cnt = w.ctr;
    hipLaunchKernelGGL(k_io_flags, dim3(nb), dim3(256), 0, c->stream, n, (const double*)ps->x,
                       (const int32_t*)ps->kind, *io, keep, app, cnt, Guard{nullptr, 0});
    LAUNCHCHK(c, "io_flags");
    // the list check of the next evaluation rides on the same round trip
    const bool checked = precheck && launch_list_check(c, n, ps->x, ps->y, ps->h);
    unsigned long long h3[3] = {0, 0, 0};
    int32_t lflag = 1;
    const Readback rb[2] = {{h3, cnt, (int)sizeof(h3)}, {&lflag, w.list_flag, 4}};
    int rc = readback(c, rb, checked ? 2 : 1);
    if (rc) return rc;
    const int32_t nto = (int32_t)(h3[0] - c->io_last[0]);
    const int32_t nap = (int32_t)(h3[1] - c->io_last[1]);
    const int32_t ndel = (int32_t)(h3[2] - c->io_last[2]);
    for (int k = 0; k < 3; ++k) c->io_last[k] = h3[k];
    if (nap == 0 && ndel == 0) {
        // no slot changes (origin is left as it is): at most kinds change,
        // and the neighbour list stays valid
        map->n_to_outlet = nto;
        if (nto > 0) {
            hipLaunchKernelGGL(k_io_kinds, dim3(nb), dim3(256), 0, c->stream, n, (const double*)ps->x,
                               ps->kind, *io, Guard{nullptr, 0});
            LAUNCHCHK(c, "io_kinds");
        }
        if (checked) {
            c->precheck_valid = 1;
            c->precheck_ok = lflag == 0;
        }
        return SPH_OK;
    }
    return inout_apply(c, ps, io, map, nto);
}

// The slot changes of an inlet/outlet update whose flags (keep, append)
// k_io_flags has left in the workspace: stable compaction of the kept
// slots, the appended copies after them.
int inout_apply(sph_ctx* c, sph_particles* ps, const sph_inout_params* io, sph_inout_map* map,
                int32_t nto)
{
    Work& w = c->w;
    const int n = (int)ps->n;
    const unsigned nb = (unsigned)cdiv(n, 256);
    int32_t *keep = w.flag, *rk = w.idx_a, *app = w.tmp_i32[1], *ra = w.closest;
    int32_t nkeep = 0, na = 0;
    int rc = compact_ranks(c, n, keep, rk, &nkeep);
    if (rc) return rc;
    rc = compact_ranks(c, n, app, ra, &na);
    if (rc) return rc;
    map->n_required = (int64_t)nkeep + na;
    if (map->n_required > ps->capacity) {
        set_err(c, "inlet/outlet update needs %lld slots, capacity %lld", (long long)map->n_required,
                (long long)ps->capacity);
        return SPH_E_CAPACITY;
    }
    map->n_to_outlet = nto;
    map->n_appended = na;
    map->n_deleted = n - nkeep;
    FluidState s{ps->x, ps->y, ps->u, ps->v, ps->p, ps->rho, ps->h, ps->mref,
                 ps->mq, map->origin, ps->kind, nullptr};
    FluidState d = tmp_state(c, true);
    d.sat = nullptr;
    hipLaunchKernelGGL(k_io_apply, dim3(nb), dim3(256), 0, c->stream, n, s, d, (const int32_t*)keep,
                       (const int32_t*)rk, (const int32_t*)app, (const int32_t*)ra, nkeep, *io);
    LAUNCHCHK(c, "io_apply");
    const int nn = nkeep + na;
    if (nn > 0) {
        hipLaunchKernelGGL(k_io_copy, dim3((unsigned)cdiv(nn, 256)), dim3(256), 0, c->stream, nn, d, s,
                           map->origin);
        LAUNCHCHK(c, "io_copy");
    }
    if (na > 0 || nkeep != n) {
        // slots moved: the neighbour structure no longer matches them
        c->list_valid = 0;
        c->built_n = -1;
    }
    ps->n = nn;
    return SPH_OK;
}

// ---------------------------------------------------------------------------
// Solution adaptivity (section 3.3): vorticity of the fluid, its magnitude
// carried to the background by the Shepard average of eq. (shepard), and
// background particles with phi > k max|omega| refined like those near a
// body.
// ---------------------------------------------------------------------------

// omega_i = sum_j V_j [(v_j - v_i) dW/dx - (u_j - u_i) dW/dy] at h_i, the
// first-order difference SPH curl; V_j = m_j / rho_j with the stored density.
__global__ __launch_bounds__(256) void k_vorticity(Grid g, NbrView nv, int n,
                                                   const double* __restrict__ u,
                                                   const double* __restrict__ v,
                                                   const double* __restrict__ rho,
                                                   const int64_t* __restrict__ mq, double q,
                                                   double* omega)
{
    int s = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int i = nv.perm[s];
    const double xi = nv.xs[s], yi = nv.ys[s], hi = nv.hs[s];
    const double ui = u[i], vi = v[i];
    double acc = 0.0;
    for_each_neighbor(g, nv, xi, yi, hi, key_level(g, nv.keys[s]),
                      [&](int js, double dx, double dy, double r2, double) {
                          const double r = sqrt(r2);
                          if (r <= 0.0) return;
                          const int j = nv.perm[js];
                          const double f = kern_dw64(r, hi) / r;
                          const double Vj = ((double)mq[j] * q) / rho[j];
                          acc += Vj * ((v[j] - vi) * (f * dx) - (u[j] - ui) * (f * dy));
                      });
    omega[i] = acc;
}

int vorticity_run(sph_ctx* c, const sph_particles* ps, double* omega)
{
    const int n = (int)ps->n;
    int rc = nbr_build(c, n, ps->x, ps->y, ps->h);
    if (rc || n == 0) return rc;
    hipLaunchKernelGGL(k_vorticity, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, c->stream, c->grid,
                       nbr_view(c), n, (const double*)ps->u, (const double*)ps->v,
                       (const double*)ps->rho, (const int64_t*)ps->mq, c->cfg.mass_q, omega);
    LAUNCHCHK(c, "vorticity");
    return SPH_OK;
}

// phi_b = sum_i |f_i| W(r_bi, (h_b + h_i)/2) / sum_i W over the fluid
// particles i with r_bi < 3 max(h_b, h_i) (0 when none), against the fluid
// neighbour structure.
__global__ __launch_bounds__(256) void k_bg_phi(Grid g, NbrView nv, int nb,
                                                const double* __restrict__ bx,
                                                const double* __restrict__ by,
                                                const double* __restrict__ bh,
                                                const int32_t* __restrict__ kind,
                                                const double* __restrict__ f, double* phi)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const double xb = bx[b], yb = by[b], hb = bh[b];
    double S = 0.0, sf = 0.0;
    for_each_neighbor(g, nv, xb, yb, hb, level_of(g, hb),
                      [&](int js, double, double, double r2, double hj) {
                          const int i = nv.perm[js];
                          if (kind && kind[i] != SPH_FLUID) return;
                          const double w = kern_w64(sqrt(r2), 0.5 * (hb + hj));
                          S += w;
                          sf += fabs(f[i]) * w;
                      });
    phi[b] = S > 0.0 ? sf / S : 0.0;
}

// max over fluid slots of |f| as the bit pattern of a non-negative double
// (monotone in the value), one atomic per block
__global__ __launch_bounds__(256) void k_absmax(int n, const double* __restrict__ f,
                                                const int32_t* __restrict__ kind,
                                                unsigned long long* out)
{
    __shared__ double part[4];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double v = (i < n && (!kind || kind[i] == SPH_FLUID)) ? fabs(f[i]) : 0.0;
    if (!(v == v)) v = 0.0;
    v = wave_max_d(v);
    if (__lane_id() == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = fmax(fmax(part[0], part[1]), fmax(part[2], part[3]));
        atomicMax(out, (unsigned long long)__double_as_longlong(m));
    }
}

__global__ void k_zero_u64_1(unsigned long long* p) { p[0] = 0ull; }

int bg_solution_run(sph_ctx* c, sph_background* bg, const sph_particles* solids,
                    const sph_particles* fluid, double k_frac, int passes, int64_t* nsplit,
                    double* omega_max)
{
    Work& w = c->w;
    const int n = (int)fluid->n, nb = (int)bg->n;
    double* om = w.sc9;
    double* phi = w.sc10;
    double mx = 0.0;
    if (n > 0) {
        int rc = vorticity_run(c, fluid, om);
        if (rc) return rc;
        unsigned long long* red = (unsigned long long*)w.red;
        hipLaunchKernelGGL(k_zero_u64_1, dim3(1), dim3(1), 0, c->stream, red);
        hipLaunchKernelGGL(k_absmax, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, c->stream, n,
                           (const double*)om, (const int32_t*)fluid->kind, red);
        if (nb > 0)
            hipLaunchKernelGGL(k_bg_phi, dim3((unsigned)cdiv(nb, 256)), dim3(256), 0, c->stream,
                               c->grid, nbr_view(c), nb, (const double*)bg->x, (const double*)bg->y,
                               (const double*)bg->h, (const int32_t*)fluid->kind,
                               (const double*)om, phi);
        LAUNCHCHK(c, "bg_phi");
        unsigned long long bits = 0;
        HIPCHK(c, hipMemcpyAsync(&bits, red, sizeof(bits), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        memcpy(&mx, &bits, sizeof(mx));
    }
    if (omega_max) *omega_max = mx;
    // with no vorticity anywhere nothing is refined by the solution
    const double thresh = k_frac * mx;
    return bg_update_run(c, bg, solids, (n > 0 && nb > 0 && mx > 0.0) ? phi : nullptr, thresh,
                         passes, nsplit);
}

// Origin maps of successive updates compose: total[t] = before[step[t]].
__global__ __launch_bounds__(256) void k_compose(int n, const int64_t* __restrict__ before,
                                                 const int64_t* __restrict__ step, int64_t* total)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) total[t] = before[step[t]];
}

__global__ __launch_bounds__(256) void k_copy_i64(int n, const int64_t* __restrict__ a, int64_t* b)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// nsteps of (PEC step, inlet/outlet update).  Counters add up over the
// steps; map->origin is the composition of the steps' maps (left unwritten
// when no step moved a slot).
__global__ void k_set_trip(int32_t* trip)
{
    if (threadIdx.x == 0) trip[0] = SPH_NOTRIP;
}

// nsteps of { step, inlet/outlet update }.  With a list skin the remaining
// steps are enqueued as one guarded run with a single host readback at its
// end: the list checks (in the predictor and corrector) and slot changes of
// the update trip the run, the kernels after the tripping one return at
// once, and the host finishes that step on the ordinary path and starts a
// new run.  The results are those of the steps taken one by one.
int step_inout_run(sph_ctx* c, sph_particles* ps, double dt, int nsteps, const sph_inout_params* io,
                   sph_inout_map* map)
{
    Work& w = c->w;
    int64_t tot_app = 0, tot_del = 0, tot_out = 0;
    bool moved = false;
    int64_t* comp = w.tmp_i64[2];  // composed map so far
    int rc = SPH_OK;
    const Guard none{nullptr, 0};
    // adds one update's counters and slot map to the totals
    auto account = [&](const sph_inout_map& m) {
        tot_app += m.n_appended;
        tot_del += m.n_deleted;
        tot_out += m.n_to_outlet;
        if (!(m.n_appended || m.n_deleted)) return;
        const int nn = (int)ps->n;
        const unsigned nb = (unsigned)cdiv(nn > 0 ? nn : 1, 256);
        if (!moved) {
            hipLaunchKernelGGL(k_copy_i64, dim3(nb), dim3(256), 0, c->stream, nn,
                               (const int64_t*)w.i64_b, comp);
        } else {
            hipLaunchKernelGGL(k_compose, dim3(nb), dim3(256), 0, c->stream, nn,
                               (const int64_t*)comp, (const int64_t*)w.i64_b, w.i64_a);
            hipLaunchKernelGGL(k_copy_i64, dim3(nb), dim3(256), 0, c->stream, nn,
                               (const int64_t*)w.i64_a, comp);
        }
        moved = true;
    };
    int s = 0;
    while (s < nsteps && rc == SPH_OK) {
        const int n = (int)ps->n;
        if (!(n > 0 && c->skin > 0 && nsteps - s > 1)) {
            // one step exactly as the separate calls take it
            rc = step_run(c, ps, dt, 1);
            if (rc) break;
            sph_inout_map m{w.i64_b, 0, 0, 0, 0};
            rc = inout_run(c, ps, io, &m, s + 1 < nsteps);
            if (rc) break;
            account(m);
            ++s;
            continue;
        }
        rc = list_ready(c, ps);
        if (rc) break;
        int32_t* trip = w.status + 24;
        hipLaunchKernelGGL(k_set_trip, dim3(1), dim3(64), 0, c->stream, trip);
        prof_run_begin(c);
        const unsigned nb = (unsigned)cdiv(n, 256);
        for (int k = s; k < nsteps && rc == SPH_OK; ++k) {
            const int32_t b = 8 * (k - s);
            rc = step_half1(c, ps, dt, Guard{trip, b + 1}, Guard{trip, b + 2});
            if (rc) break;
            rc = step_half2(c, ps, dt, Guard{trip, b + 3}, Guard{trip, b + 4});
            if (rc) break;
            hipLaunchKernelGGL(k_io_flags, dim3(nb), dim3(256), 0, c->stream, n, (const double*)ps->x,
                               (const int32_t*)ps->kind, *io, w.flag, w.tmp_i32[1], w.ctr,
                               Guard{trip, b + 5});
            hipLaunchKernelGGL(k_io_kinds, dim3(nb), dim3(256), 0, c->stream, n, (const double*)ps->x,
                               ps->kind, *io, Guard{trip, b + 6});
            LAUNCHCHK(c, "run_io");
        }
        if (rc) break;
        int32_t tr = SPH_NOTRIP;
        unsigned long long h3[3] = {0, 0, 0};
        const Readback rb[2] = {{&tr, trip, 4}, {h3, w.ctr, (int)sizeof(h3)}};
        rc = readback(c, rb, 2);
        if (rc) break;
        prof_run_end(c, tr);  // brackets of the kernels skipped after the trip are dropped
        // fluid turned outlet in the steps that ran (their kinds are set)
        tot_out += (int64_t)(h3[0] - c->io_last[0]);
        for (int k = 0; k < 3; ++k) c->io_last[k] = h3[k];
        c->fused_x = nullptr;
        c->precheck_valid = 0;
        if (tr == SPH_NOTRIP) {
            s = nsteps;
            break;
        }
        // a kernel of the run tripped; the state is as that kernel left it
        reset_bcounters(c);
        const int kk = s + tr / 8, ph = tr % 8;
        sph_inout_map m{w.i64_b, 0, 0, 0, 0};
        if (ph == 2) {
            // the list expired at step kk's predicted positions
            c->list_valid = 0;
            rc = step_half2(c, ps, dt, none, none);
            if (rc == SPH_OK) rc = inout_run(c, ps, io, &m, kk + 1 < nsteps);
        } else if (ph == 4) {
            // the corrector of step kk found the list expired
            c->list_valid = 0;
            rc = inout_run(c, ps, io, &m, false);
        } else if (ph == 5) {
            // step kk's update moves slots; its flags and counters are taken
            rc = inout_apply(c, ps, io, &m, 0);
        } else {
            set_err(c, "run of steps: unexpected trip %d", tr);
            rc = SPH_E_DEVICE;
        }
        if (rc) break;
        account(m);
        s = kk + 1;
    }
    c->precheck_valid = 0;
    map->n_appended = tot_app;
    map->n_deleted = tot_del;
    map->n_to_outlet = tot_out;
    map->n_required = ps->n;
    if (rc == SPH_OK && moved && ps->n > 0) {
        hipLaunchKernelGGL(k_copy_i64, dim3((unsigned)cdiv(ps->n, 256)), dim3(256), 0, c->stream,
                           (int)ps->n, (const int64_t*)comp, map->origin);
        LAUNCHCHK(c, "origin");
    }
    return rc;
}

// ---------------------------------------------------------------------------
// The per-iteration schedule of section 3.4.  Before iteration it > 0: the
// background update every n_bg iterations, then the adaptation every n_adapt
// iterations (its m_ref lookup sees the updated background); then one step,
// with the inlet/outlet update when zones are given.  The iterations between
// two updates go to the step runs in one call (enqueued at once, one host
// round trip per run), so the results are those of the separate calls.
// ---------------------------------------------------------------------------
int schedule_run(sph_ctx* c, sph_particles* ps, sph_background* bg, const sph_particles* solids,
                 const sph_inout_params* io, int nsteps, sph_diag* diag)
{
    const sph_config& cf = c->cfg;
    Work& w = c->w;
    const double dt = cf.dt > 0 ? cf.dt : timestep_of(cf, 0.0);
    int done = 0;
    while (done < nsteps) {
        const int64_t it = c->iter;
        if (it > 0 && bg) {
            if (cf.n_bg > 0 && it % cf.n_bg == 0) {
                int64_t nsplit = 0;
                const int rc = cf.sol_k > 0
                                   ? bg_solution_run(c, bg, solids, ps, cf.sol_k, cf.bg_passes, &nsplit,
                                                     nullptr)
                                   : bg_update_run(c, bg, solids, nullptr, 0.0, cf.bg_passes, &nsplit);
                if (rc) return rc;
            }
            if (cf.n_adapt > 0 && it % cf.n_adapt == 0) {
                sph_adapt_map m{w.sched_origin, w.sched_sat, 0, 0, {0, 0, 0, 0, 0, 0, 0, 0}};
                const int rc = adapt_run(c, ps, bg, &m);
                if (rc) return rc;
            }
        }
        // iterations up to the next update
        int64_t k = nsteps - done;
        auto upto = [&](int32_t per) {
            if (per <= 0) return;
            const int64_t nx = (it / per + 1) * per;
            if (nx - it < k) k = nx - it;
        };
        if (bg) {
            upto(cf.n_adapt);
            upto(cf.n_bg);
        }
        int rc;
        if (io) {
            sph_inout_map m{w.sched_origin, 0, 0, 0, 0};
            rc = step_inout_run(c, ps, dt, (int)k, io, &m);
        } else {
            rc = step_run(c, ps, dt, (int)k);
        }
        if (rc) return rc;
        c->iter += k;
        done += (int)k;
    }
    if (diag) return diag_run(c, ps, diag);
    return SPH_OK;
}
