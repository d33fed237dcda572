// Neighbour search for variable smoothing length on gfx950: level/Morton
// keys, stable LSD radix sort, per-(level, resolution) cell-run tables and
// CSR export.  The neighbour relation is |r_i - r_j| < 3 max(h_i, h_j) with
// the quintic support of eq. (kernel); it is symmetric because the rates of
// eqs. (edac:sph) and (mom-sph) use both W(h_i) and W(h_j).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "sph_device.h"

// ---------------------------------------------------------------------------
// Grid geometry (host)
// ---------------------------------------------------------------------------

void grid_setup(const sph_config* cfg, Grid* g)
{
    memset(g, 0, sizeof(*g));
    double hlo = cfg->h_lo > 0 ? cfg->h_lo : 1e-3;
    double hhi = cfg->h_hi > hlo ? cfg->h_hi : hlo;
    double cmin = 3.0 * hlo * (1.0 + 1e-9);
    for (int a = 0; a < 2; ++a) {
        double L = cfg->hi[a] - cfg->lo[a];
        g->lo[a] = cfg->lo[a];
        g->hi[a] = cfg->hi[a];
        g->periodic[a] = cfg->periodic[a] ? 1 : 0;
        g->L[a] = L;
        g->half[a] = 0.5 * L;
        g->org[a] = cfg->lo[a];
    }
    // keep the finest table modest: at most 2^25 level-0 cells
    for (;;) {
        double n0 = 1, n1 = 1;
        for (int a = 0; a < 2; ++a) {
            double L = g->L[a];
            double nx = g->periodic[a] ? floor(L / cmin) : floor(L / cmin) + 1;
            if (nx < 1) nx = 1;
            (a ? n1 : n0) = nx;
        }
        if (n0 * n1 <= (double)(1 << 25)) break;
        cmin *= 2.0;
    }
    for (int a = 0; a < 2; ++a) {
        double L = g->L[a];
        if (g->periodic[a]) {
            int nx = (int)floor(L / cmin);
            if (nx < 1) nx = 1;
            g->nx0[a] = nx;
            g->cw0[a] = L / nx;
        } else {
            g->nx0[a] = (int)floor(L / cmin) + 1;
            g->cw0[a] = cmin;
        }
    }
    g->cmin0 = g->cw0[0] < g->cw0[1] ? g->cw0[0] : g->cw0[1];
    g->icw0[0] = 1.0 / g->cw0[0];
    g->icw0[1] = 1.0 / g->cw0[1];
    for (int a = 0; a < 2; ++a) {
        g->mi_l[a] = g->periodic[a] ? g->L[a] : 0.0;
        g->mi_h[a] = g->periodic[a] ? g->half[a] : HUGE_VAL;
    }
    int nlev = 1;
    double c = g->cmin0;
    while (c < 3.0 * hhi * (1.0 + 1e-9) && nlev < SPH_MAXL) {
        c *= 2.0;
        ++nlev;
    }
    g->nlev = nlev;
    int mx = g->nx0[0] > g->nx0[1] ? g->nx0[0] : g->nx0[1];
    int bits = 1;
    while ((1 << bits) < mx) ++bits;
    g->bits = bits;
    g->cumq[0] = 0;
    for (int q = 0; q < SPH_MAXL; ++q) {
        for (int a = 0; a < 2; ++a) g->nxq[q][a] = ((g->nx0[a] - 1) >> q) + 1;
        g->cumq[q + 1] = g->cumq[q] + (int64_t)g->nxq[q][0] * g->nxq[q][1];
    }
    int64_t acc = 0;
    for (int l = 0; l < nlev; ++l) {
        g->lbase[l] = acc - g->cumq[l];
        acc += g->cumq[nlev] - g->cumq[l];
    }
    g->tab_total = acc;
}

static int key_bits(const Grid* g)
{
    int lb = 0;
    while ((1 << lb) < g->nlev) ++lb;
    return 2 * g->bits + lb;
}

int batch_key_bits(const Grid* g) { return key_bits(g); }


// ---------------------------------------------------------------------------
// Scans (exclusive; output has n + 1 entries, out[n] = total)
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v)
{
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

template <typename T>
__global__ __launch_bounds__(SCAN_T) void k_scan_block(const T* in, T* out, int64_t n_in,
                                                       int64_t n_out, T* bsum)
{
    __shared__ T wsum[SCAN_T / 64];
    const int t = threadIdx.x, lane = __lane_id(), wid = t >> 6;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)t * SCAN_E;
    T v[SCAN_E];
    T tot = 0;
#pragma unroll
    for (int k = 0; k < SCAN_E; ++k) {
        int64_t i = base + k;
        v[k] = (i < n_in) ? in[i] : T(0);
        tot += v[k];
    }
    T incl = wave_incl_scan<T>(tot);
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    if (wid == 0) {
        T w = lane < SCAN_T / 64 ? wsum[lane] : T(0);
        w = wave_incl_scan<T>(w);
        if (lane < SCAN_T / 64) wsum[lane] = w;
    }
    __syncthreads();
    T run = incl - tot + (wid > 0 ? wsum[wid - 1] : T(0));
#pragma unroll
    for (int k = 0; k < SCAN_E; ++k) {
        int64_t i = base + k;
        if (i < n_out) out[i] = run;
        run += v[k];
    }
    if (t == SCAN_T - 1) bsum[blockIdx.x] = wsum[SCAN_T / 64 - 1];
}

template <typename T>
__global__ void k_scan_add(T* out, int64_t n_out, const T* boff)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_out) out[i] += boff[i / SCAN_TILE];
}

// Exclusive scan of in[0, n_in) into out[0, n_out) (n_out >= n_in; entries
// past n_in scan zeros).  tmp needs about 2 * n_out / SCAN_TILE + 64 entries.
template <typename T>
static hipError_t scan_rec_s(hipStream_t st, const T* in, T* out, int64_t n_in, int64_t n_out,
                             T* tmp)
{
    int64_t nb = cdiv(n_out, SCAN_TILE);
    hipLaunchKernelGGL(k_scan_block<T>, dim3((unsigned)nb), dim3(SCAN_T), 0, st, in, out, n_in,
                       n_out, tmp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nb <= 1) return e;
    e = scan_rec_s<T>(st, tmp, tmp, nb, nb, tmp + nb);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_add<T>, dim3((unsigned)cdiv(n_out, 256)), dim3(256), 0, st, out,
                       n_out, tmp);
    return hipGetLastError();
}

template <typename T>
static int scan_rec(sph_ctx* c, const T* in, T* out, int64_t n_in, int64_t n_out, T* tmp)
{
    const hipError_t e = scan_rec_s<T>(c->stream, in, out, n_in, n_out, tmp);
    if (e != hipSuccess) return check_hip(c, e, "scan");
    return SPH_OK;
}

int scan_exclusive_i64(sph_ctx* c, const int64_t* in, int64_t* out, int64_t n)
{
    return scan_rec<int64_t>(c, in, out, n, n + 1, c->w.scan_tmp);
}

int scan_exclusive_i32(sph_ctx* c, const int32_t* in, int32_t* out, int64_t n)
{
    return scan_rec<int32_t>(c, in, out, n, n + 1, (int32_t*)c->w.scan_tmp);
}

// ---------------------------------------------------------------------------
// Keys
// ---------------------------------------------------------------------------

// Sort key of a particle: its level above the Hilbert index of its
// level-0 cell.
__device__ __forceinline__ uint64_t key_of(const Grid& g, double xi, double yi, double hi, int* lev)
{
    const int l = level_of(g, hi);
    const uint32_t kx = (uint32_t)cell0(g, 0, xi);
    const uint32_t ky = (uint32_t)cell0(g, 1, yi);
    *lev = l;
    return ((uint64_t)l << (2 * g.bits)) | hilbert_d(kx, ky, g.bits);
}

// Key and slot of particle i (when valid), and the block's per-level maxima
// of h and counts; every thread of the block calls it.
__device__ __forceinline__ void keys_body(const Grid& g, bool valid, int i,
                                          const double* __restrict__ x,
                                          const double* __restrict__ y,
                                          const double* __restrict__ h, uint64_t* keys,
                                          int32_t* vals, unsigned long long* hmax_bits,
                                          int32_t* lcount)
{
    __shared__ unsigned long long s_h[SPH_MAXL];
    __shared__ int32_t s_c[SPH_MAXL];
    if (threadIdx.x < SPH_MAXL) {
        s_h[threadIdx.x] = 0ull;
        s_c[threadIdx.x] = 0;
    }
    __syncthreads();
    if (valid) {
        double hi = h[i];
        int l;
        keys[i] = key_of(g, x[i], y[i], hi, &l);
        vals[i] = i;
        atomicMax(&s_h[l], (unsigned long long)__double_as_longlong(hi));
        atomicAdd(&s_c[l], 1);
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)g.nlev && s_c[threadIdx.x] > 0) {
        atomicMax(&hmax_bits[threadIdx.x], s_h[threadIdx.x]);
        atomicAdd(&lcount[threadIdx.x], s_c[threadIdx.x]);
    }
}

__global__ void k_zero_i32(int32_t* p, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// Clears what a build accumulates into: the cell-run table, the per-level
// h maxima and counts, and the sort's counters z[0, nz) (one launch).
__global__ void k_zero_build(int2* tab, int64_t ntab, unsigned long long* hmax, int32_t* lcount,
                             int nl, uint32_t* z, int64_t nz)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ntab) tab[i] = make_int2(0, 0);
    if (i < nl) {
        hmax[i] = 0ull;
        lcount[i] = 0;
    }
    if (i < nz) z[i] = 0u;
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort, RS_BITS-bit digits.  Each block owns RS_TILE consecutive
// keys; each wave owns a contiguous quarter of the tile and ranks its keys
// with one ballot per digit bit per 64-key chunk (lanes with equal digits), so the order of
// equal digits is the input order.
// ---------------------------------------------------------------------------

// Digit counts of one tile: keys [base, base + tn) of the tile; hist gets
// the count of digit d at hist[d * hstride].
__device__ __forceinline__ void rs_hist_tile(const uint64_t* __restrict__ keys, int64_t base, int tn,
                                             int shift, uint32_t* hist, int64_t hstride)
{
    __shared__ uint32_t h[RS_BINS];
    for (int d = threadIdx.x; d < RS_BINS; d += RS_THREADS) h[d] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < RS_ITEMS; ++k) {
        const int i = k * RS_THREADS + threadIdx.x;
        if (i < tn) atomicAdd(&h[(keys[base + i] >> shift) & (RS_BINS - 1u)], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < RS_BINS; d += RS_THREADS) hist[(int64_t)d * hstride] = h[d];
}

// Stable ranking of one tile's keys [base, base + tn) by their BITS-bit
// digit at `shift`: wave w owns the contiguous keys [w 64 ITEMS, (w + 1) 64
// ITEMS) of the tile and ranks each 64-key chunk with one ballot per digit
// bit (the lanes with equal digits), so equal digits keep the input order.
// On return wcnt[w][d] holds the offset of wave w's first digit-d key among
// the tile's digit-d keys, cnt[d] (when given) the tile's count of digit d,
// and each lane's items their key, value, digit (BINS past the end) and
// rank within the wave's digit-d keys.
template <int BITS, int ITEMS>
__device__ __forceinline__ void tile_rank(const uint64_t* __restrict__ kin,
                                          const int32_t* __restrict__ vin, int64_t base, int tn,
                                          int shift, uint32_t (*wcnt)[1 << BITS], uint32_t* cnt,
                                          uint64_t* kk, int32_t* vv, uint32_t* dd, uint32_t* rk)
{
    constexpr int NW = RS_THREADS / 64, BINS = 1 << BITS;
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    for (int d = threadIdx.x; d < NW * BINS; d += RS_THREADS) (&wcnt[0][0])[d] = 0;
    __syncthreads();
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int wbase = w * (64 * ITEMS);
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const int il = wbase + it * 64 + lane;
        const bool valid = il < tn;
        const int64_t i = base + il;
        uint64_t k = valid ? kin[i] : 0ull;
        uint32_t d = (uint32_t)(k >> shift) & (BINS - 1u);
        uint64_t mask = __ballot(valid);
#pragma unroll
        for (int b = 0; b < BITS; ++b) {
            bool bit = (d >> b) & 1u;
            uint64_t bal = __ballot(bit);
            mask &= bit ? bal : ~bal;
        }
        uint32_t before = (uint32_t)__popcll(mask & lt_mask);
        uint32_t c = (uint32_t)__popcll(mask);
        uint32_t old = valid ? wcnt[w][d] : 0u;
        // all lanes have read the running count before the group leader
        // (lowest lane of its digit group) advances it
        __builtin_amdgcn_wave_barrier();
        if (valid && before == 0) wcnt[w][d] = old + c;
        __builtin_amdgcn_wave_barrier();
        kk[it] = k;
        vv[it] = valid ? vin[i] : 0;
        dd[it] = valid ? d : (uint32_t)BINS;
        rk[it] = old + before;
    }
    __syncthreads();
    for (int d = threadIdx.x; d < BINS; d += RS_THREADS) {
        uint32_t s = 0;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            uint32_t t = wcnt[q][d];
            wcnt[q][d] = s;
            s += t;
        }
        if (cnt) cnt[d] = s;
    }
    __syncthreads();
}

// Scatter of one tile: keys [base, base + tn); digit d of the tile starts
// at offs[d * ostride] + padj of the output.
__device__ __forceinline__ void rs_scatter_tile(const uint64_t* __restrict__ kin,
                                                const int32_t* __restrict__ vin,
                                                uint64_t* __restrict__ kout,
                                                int32_t* __restrict__ vout, int64_t base, int tn,
                                                int shift, const uint32_t* __restrict__ offs,
                                                int64_t ostride, int64_t padj)
{
    constexpr int NW = RS_THREADS / 64;
    __shared__ uint32_t wcnt[NW][RS_BINS];
    const int w = threadIdx.x >> 6;
    uint64_t kk[RS_ITEMS];
    int32_t vv[RS_ITEMS];
    uint32_t dd[RS_ITEMS], rk[RS_ITEMS];
    tile_rank<RS_BITS, RS_ITEMS>(kin, vin, base, tn, shift, wcnt, nullptr, kk, vv, dd, rk);
#pragma unroll
    for (int it = 0; it < RS_ITEMS; ++it) {
        uint32_t d = dd[it];
        if (d < (uint32_t)RS_BINS) {
            const int64_t pos = (int64_t)offs[(int64_t)d * ostride] + padj + wcnt[w][d] + rk[it];
            kout[pos] = kk[it];
            vout[pos] = vv[it];
        }
    }
}

// ---------------------------------------------------------------------------
// One-sweep LSD radix sort of a context's keys: 8-bit digits, one kernel per
// digit.  The key kernel also counts every pass's digits over all keys, so a
// pass knows each digit's start; within a digit, a tile's keys follow those
// of the tiles before it.  Workgroups take tiles in order from a ticket
// counter, rank their keys (stable), publish each digit's count and find
// the count of that digit in the tiles before theirs by looking back: a
// tile's word holds either its own count (OS_AGG) or the inclusive prefix
// through it (OS_INC); the walk adds counts back to the nearest prefix,
// OS_WIN tiles per load round.  A workgroup waits only on tiles taken before
// its own, whose workgroups are running, so every wait ends; the wait is
// still bounded, and a wait that runs out sets a failure flag.
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t os_load(const uint32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void os_store(uint32_t* p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Keys, slots and level statistics as keys_body, OS_KEYS_ITEMS particles per
// thread, and the counts of every pass's digits into ghist[p][d].
#ifndef OS_KEYS_ITEMS
#define OS_KEYS_ITEMS 8
#endif
__global__ __launch_bounds__(256) void k_keys_os(Grid g, int n, const double* __restrict__ x,
                                                 const double* __restrict__ y,
                                                 const double* __restrict__ h, uint64_t* keys,
                                                 int32_t* vals, unsigned long long* hmax_bits,
                                                 int32_t* lcount, int npass, uint32_t* ghist)
{
    __shared__ unsigned long long s_h[SPH_MAXL];
    __shared__ int32_t s_c[SPH_MAXL];
    __shared__ uint32_t s_g[OS_MAXPASS * OS_BINS];
    const int t = threadIdx.x;
    if (t < SPH_MAXL) {
        s_h[t] = 0ull;
        s_c[t] = 0;
    }
    for (int e = t; e < npass * OS_BINS; e += 256) s_g[e] = 0u;
    __syncthreads();
    const int64_t b0 = (int64_t)blockIdx.x * (256 * OS_KEYS_ITEMS);
#pragma unroll
    for (int k = 0; k < OS_KEYS_ITEMS; ++k) {
        const int64_t i = b0 + k * 256 + t;
        if (i < n) {
            const double hi = h[i];
            int l;
            const uint64_t key = key_of(g, x[i], y[i], hi, &l);
            keys[i] = key;
            vals[i] = (int32_t)i;
            atomicMax(&s_h[l], (unsigned long long)__double_as_longlong(hi));
            atomicAdd(&s_c[l], 1);
            for (int p = 0; p < npass; ++p)
                atomicAdd(&s_g[p * OS_BINS + ((key >> (OS_BITS * p)) & (OS_BINS - 1u))], 1u);
        }
    }
    __syncthreads();
    if (t < g.nlev && s_c[t] > 0) {
        atomicMax(&hmax_bits[t], s_h[t]);
        atomicAdd(&lcount[t], s_c[t]);
    }
    for (int e = t; e < npass * OS_BINS; e += 256)
        if (s_g[e]) atomicAdd(&ghist[e], s_g[e]);
}

// One pass: keys and values from (kin, vin) to their places in (kout, vout)
// by the digit at bit OS_BITS * pass; ghist, look and ticket are the pass's
// digit counts, look-back words (ntile x OS_BINS) and ticket counter.
__global__ __launch_bounds__(RS_THREADS) void k_os_pass(const uint64_t* __restrict__ kin,
                                                        const int32_t* __restrict__ vin,
                                                        uint64_t* __restrict__ kout,
                                                        int32_t* __restrict__ vout, int n, int pass,
                                                        const uint32_t* __restrict__ ghist,
                                                        uint32_t* look, uint32_t* ticket,
                                                        int32_t* fail)
{
    static_assert(RS_THREADS == OS_BINS, "one thread per digit");
    constexpr int NW = RS_THREADS / 64;
    __shared__ uint32_t wcnt[NW][OS_BINS];
    __shared__ uint32_t cnt[OS_BINS];
    __shared__ uint32_t goff[OS_BINS];
    __shared__ uint32_t wsum[NW];
    __shared__ int s_tile;
    const int t = threadIdx.x, lane = __lane_id(), w = t >> 6;
    if (t == 0) s_tile = (int)atomicAdd(ticket, 1u);
    // start of digit t in the output: exclusive scan of the digit counts
    const uint32_t gc = ghist[t];
    const uint32_t gi = wave_incl_scan<uint32_t>(gc);
    if (lane == 63) wsum[w] = gi;
    __syncthreads();
    uint32_t gb = gi - gc;
    for (int q = 0; q < w; ++q) gb += wsum[q];
    const int tile = s_tile;
    const int64_t base = (int64_t)tile * OS_TILE;
    const int tn = (int)(n - base < OS_TILE ? n - base : OS_TILE);
    uint64_t kk[OS_ITEMS];
    int32_t vv[OS_ITEMS];
    uint32_t dd[OS_ITEMS], rk[OS_ITEMS];
    tile_rank<OS_BITS, OS_ITEMS>(kin, vin, base, tn, OS_BITS * pass, wcnt, cnt, kk, vv, dd, rk);
    {
        // thread t: digit t of this tile
        const uint32_t own = cnt[t];
        uint32_t* colw = look + t;  // word of tile q: colw[q * OS_BINS]
        uint32_t excl = 0;
        if (tile == 0) {
            os_store(colw, OS_INC | own);
        } else {
            os_store(colw + (int64_t)tile * OS_BINS, OS_AGG | own);
            int p = tile - 1, spin = 0;
            for (;;) {
                uint32_t v[OS_WIN];
#pragma unroll
                for (int q = 0; q < OS_WIN; ++q)
                    v[q] = p - q >= 0 ? os_load(colw + (int64_t)(p - q) * OS_BINS) : OS_INC;
                int q = 0;
                bool done = false;
                for (; q < OS_WIN; ++q) {
                    if (!(v[q] & (OS_AGG | OS_INC))) break;  // not published yet
                    excl += v[q] & OS_VAL;
                    if (v[q] & OS_INC) {
                        done = true;
                        break;
                    }
                }
                if (done) break;
                p -= q;
                if (q < OS_WIN) {
                    if (++spin > OS_SPIN) {
                        atomicOr(fail, 1);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            os_store(colw + (int64_t)tile * OS_BINS, OS_INC | (excl + own));
        }
        goff[t] = gb + excl;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < OS_ITEMS; ++it) {
        const uint32_t d = dd[it];
        if (d < (uint32_t)OS_BINS) {
            const int64_t pos = (int64_t)goff[d] + wcnt[w][d] + rk[it];
            kout[pos] = kk[it];
            vout[pos] = vv[it];
        }
    }
}

// Words the one-sweep sort of n keys of keybits bits clears before it runs
// (look-back words, digit counts, tickets), from w.os_look on.
static int64_t os_words(int n, int keybits, int* npass, int* ntile)
{
    *npass = (keybits + OS_BITS - 1) / OS_BITS;
    if (*npass < 1) *npass = 1;
    *ntile = (int)cdiv(n > 0 ? n : 1, OS_TILE);
    return (int64_t)*npass * (*ntile) * OS_BINS;
}

// ---------------------------------------------------------------------------
// Cell-run tables and sorted shadows
// ---------------------------------------------------------------------------

// Run boundaries per (level, resolution Q): consecutive sorted particles of
// one level share a Q-cell iff their curve indices agree above bit 2Q.  The
// cell's coordinates come from the particle's position, which is copied to
// the sorted shadows (xs, ys, hs and the packed xyh) on the way.
// Sorted particle s of the segment [lo, hi) (its simulation's particles):
// run boundaries into tab (the simulation's tables), shadows (xs, ys, hs may
// be NULL).
__device__ __forceinline__ void tables_body(const Grid& g, int s, int lo, int hi,
                                            const uint64_t* __restrict__ keys,
                                            const int32_t* __restrict__ perm,
                                            const double* __restrict__ x,
                                            const double* __restrict__ y,
                                            const double* __restrict__ h, double* xs, double* ys,
                                            double* hs, double4* xyh, int2* tab)
{
    const int i = perm[s];
    const double xi = x[i], yi = y[i], hi_ = h[i];
    if (xs) {
        xs[s] = xi;
        ys[s] = yi;
        hs[s] = hi_;
    }
    xyh[s] = make_double4(xi, yi, hi_, 0.0);
    const int sh = 2 * g.bits;
    const uint64_t mmask = (sh >= 64) ? ~0ull : ((1ull << sh) - 1ull);
    uint64_t key = keys[s];
    int l = (int)(key >> sh);
    uint64_t m = key & mmask;
    uint64_t kp = s > lo ? keys[s - 1] : ~0ull;
    uint64_t kn = s < hi - 1 ? keys[s + 1] : ~0ull;
    bool lp = s > lo && (int)(kp >> sh) == l;
    bool ln = s < hi - 1 && (int)(kn >> sh) == l;
    const int kx0 = cell0(g, 0, xi), ky0 = cell0(g, 1, yi);
    for (int Q = l; Q < g.nlev; ++Q) {
        uint64_t cell = m >> (2 * Q);
        bool sp = lp && ((kp & mmask) >> (2 * Q)) == cell;
        bool sn = ln && ((kn & mmask) >> (2 * Q)) == cell;
        if (sp && sn) continue;
        int cx = kx0 >> Q, cy = ky0 >> Q;
        int64_t idx = g.lbase[l] + g.cumq[Q] + (int64_t)cy * g.nxq[Q][0] + cx;
        if (!sp) tab[idx].x = s;
        if (!sn) tab[idx].y = s + 1;
    }
}

__global__ __launch_bounds__(256) void k_tables(Grid g, int n, const uint64_t* __restrict__ keys,
                                                const int32_t* __restrict__ perm,
                                                const double* __restrict__ x,
                                                const double* __restrict__ y,
                                                const double* __restrict__ h, double* xs,
                                                double* ys, double* hs, double4* xyh, int2* tab)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    tables_body(g, s, 0, n, keys, perm, x, y, h, xs, ys, hs, xyh, tab);
}

int nbr_build(sph_ctx* c, int n, const double* x, const double* y, const double* h)
{
    Work& w = c->w;
    const Grid& g = c->grid;
    c->list_valid = 0;  // a new sorted order invalidates any reusable list
    if (n >= (1 << 30)) {
        set_err(c, "%d particles: the neighbour sort takes fewer than 2^30", n);
        return SPH_E_INVAL;
    }
    prof_begin(c, SPH_PROF_BUILD);
    int npass = 1, ntile = 1;
    const int64_t nlook = n > 0 ? os_words(n, key_bits(&g), &npass, &ntile) : 0;
    if (npass > OS_MAXPASS) {
        set_err(c, "sort keys of %d bits exceed %d", key_bits(&g), OS_MAXPASS * OS_BITS);
        return SPH_E_INVAL;
    }
    // look-back words, then the digit counts and tickets of every pass
    uint32_t* ghist = w.os_look + nlook;
    uint32_t* ticket = ghist + OS_MAXPASS * OS_BINS;
    const int64_t nclr = n > 0 ? nlook + OS_MAXPASS * OS_BINS + OS_MAXPASS : 0;
    {
        int64_t nz = g.tab_total > SPH_MAXL ? g.tab_total : (int64_t)SPH_MAXL;
        if (nclr > nz) nz = nclr;
        hipLaunchKernelGGL(k_zero_build, dim3((unsigned)cdiv(nz, 256)), dim3(256), 0, c->stream, w.tab,
                           g.tab_total, w.hmax_bits, w.lcount, (int)SPH_MAXL, w.os_look, nclr);
        LAUNCHCHK(c, "zero");
    }
    if (n > 0) {
        // the passes alternate between the two buffers and end in keys_a
        uint64_t *ka = (npass & 1) ? w.keys_b : w.keys_a, *kb = (npass & 1) ? w.keys_a : w.keys_b;
        int32_t *va = (npass & 1) ? w.vals_b : w.vals_a, *vb = (npass & 1) ? w.vals_a : w.vals_b;
        hipLaunchKernelGGL(k_keys_os, dim3((unsigned)cdiv(n, 256 * OS_KEYS_ITEMS)), dim3(256), 0, c->stream,
                           g, n, x, y, h, ka, va, w.hmax_bits, w.lcount, npass, ghist);
        LAUNCHCHK(c, "keys");
        for (int p = 0; p < npass; ++p) {
            hipLaunchKernelGGL(k_os_pass, dim3((unsigned)ntile), dim3(RS_THREADS), 0, c->stream,
                               (const uint64_t*)ka, (const int32_t*)va, kb, vb, n, p,
                               (const uint32_t*)(ghist + p * OS_BINS), w.os_look + (int64_t)p * ntile * OS_BINS,
                               ticket + p, w.status + SPH_STATUS_SORT);
            LAUNCHCHK(c, "sort");
            uint64_t* tk = ka; ka = kb; kb = tk;
            int32_t* tv = va; va = vb; vb = tv;
        }
        hipLaunchKernelGGL(k_tables, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, c->stream, g, n,
                           w.keys_a, (const int32_t*)w.vals_a, x, y, h, w.xs, w.ys, w.hs, w.xyh,
                           w.tab);
        LAUNCHCHK(c, "tables");
    }
    prof_end(c, SPH_PROF_BUILD);
    c->built_n = n;
    return SPH_OK;
}

NbrView nbr_view(sph_ctx* c)
{
    NbrView v;
    v.xs = c->w.xs;
    v.ys = c->w.ys;
    v.hs = c->w.hs;
    v.xyh = c->w.xyh;
    v.perm = c->w.vals_a;
    v.keys = c->w.keys_a;
    v.tab = c->w.tab;
    v.hmax_bits = c->w.hmax_bits;
    v.lcount = c->w.lcount;
    return v;
}

// ---------------------------------------------------------------------------
// Neighbour list for the rate passes: every pair closer than (1 + skin)
// times the support radius, from a per-lane cell walk.  Entry k of sorted
// particle s goes to idx[k * stride + s], so a wave's rows are read one
// coalesced line per k; counts above K are recorded (the rate passes then
// walk the cells again for that row).
// ---------------------------------------------------------------------------

// Every j with |r_i - r_j| < sf 3 max(h_i, h_j) (FP64 predicate); G lanes
// per row walk the cells together (LG for the export and the batched build;
// the single-context list build takes the context's schedule).
#define LG 4
template <int G>
__device__ __forceinline__ void build_list_body(const Grid& g, const NbrView& nv, const NbrList& nl,
                                                int s, int gl, double sf)
{
    const double4 a = nv.xyh[s];
    const int li = key_level(g, nv.keys[s]);
    int cnt = 0;
    int32_t* const row = nl.idx + s;
    group_walk<G>(g, nv, a.x, a.y, a.z, li, gl,
                   [&](int js, bool pass, double, double, double, double) {
                       int tot;
                       const int k = cnt + group_rank<G>(pass, gl, &tot);
                       if (pass && k < nl.K) row[(int64_t)k * nl.stride] = js;
                       cnt += tot;
                   },
                   sf);
    if (gl == 0) {
        nl.cnt[s] = cnt;
        if (cnt > nl.K) nl.flag[0] = 1;
    }
}

template <int G>
__global__ __launch_bounds__(256) void k_build_list_lane(Grid g, NbrView nv, int n, NbrList nl,
                                                         double sf)
{
    const int t = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const int s = t / G, gl = t % G;
    if (s >= n) return;
    build_list_body<G>(g, nv, nl, s, gl, sf);
}

using BuildListFn = void (*)(Grid, NbrView, int, NbrList, double);
static BuildListFn build_list_variant(int G)
{
    switch (G) {
    case 2: return k_build_list_lane<2>;
    case 4: return k_build_list_lane<4>;
    case 8: return k_build_list_lane<8>;
    default: return nullptr;
    }
}

bool list_lanes_valid(int G) { return build_list_variant(G) != nullptr; }

int nbr_build_list(sph_ctx* c, int n, double skin)
{
    Work& w = c->w;
    if (n == 0) return SPH_OK;
    NbrList nl{w.nl_idx, w.nl_cnt, w.nl_k, n, w.list_flag};
    prof_begin(c, SPH_PROF_LIST);
    const Grid& g = c->grid;
    const double sf = 1.0 + skin;
    const int G = c->sched.list_lanes;
    hipLaunchKernelGGL(build_list_variant(G), dim3((unsigned)cdiv((int64_t)n * G, 256)), dim3(256), 0,
                       c->stream, g, nbr_view(c), n, nl, sf);
    prof_end(c, SPH_PROF_LIST);
    LAUNCHCHK(c, "build_list");
    return SPH_OK;
}

// ---------------------------------------------------------------------------
// CSR export: count, scan, fill, sort rows ascending
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_csr_fill(Grid g, NbrView nv, int n,
                                                  const int64_t* __restrict__ rp, int32_t* col,
                                                  double sf)
{
    int s = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (s >= n) return;
    double xi = nv.xs[s], yi = nv.ys[s], hi = nv.hs[s];
    int li = key_level(g, nv.keys[s]);
    int64_t k = rp[nv.perm[s]];
    for_each_neighbor(g, nv, xi, yi, hi, li,
                      [&](int js, double, double, double, double) { col[k++] = nv.perm[js]; }, sf);
}

// One wave per row: bitonic sort across the 64 lanes for rows of <= 64
// entries; longer rows are listed for the per-thread path.
__global__ __launch_bounds__(256) void k_sort_rows(int n, const int64_t* __restrict__ rp,
                                                   int32_t* col, int32_t* long_rows,
                                                   int32_t* n_long)
{
    const int lane = __lane_id();
    int row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= n) return;
    int64_t beg = rp[row];
    int len = (int)(rp[row + 1] - beg);
    if (len > 64) {
        if (lane == 0) long_rows[atomicAdd(n_long, 1)] = row;
        return;
    }
    int v = lane < len ? col[beg + lane] : 0x7fffffff;
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            int o = __shfl_xor(v, j, 64);
            bool up = (lane & k) == 0;
            bool low = (lane & j) == 0;
            v = (low == up) ? min(v, o) : max(v, o);
        }
    }
    if (lane < len) col[beg + lane] = v;
}

__global__ void k_sort_long_rows(const int64_t* __restrict__ rp, int32_t* col,
                                 const int32_t* long_rows, const int32_t* n_long)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= *n_long) return;
    int row = long_rows[t];
    int64_t b = rp[row], e = rp[row + 1];
    for (int64_t i = b + 1; i < e; ++i) {
        int v = col[i];
        int64_t j = i - 1;
        while (j >= b && col[j] > v) {
            col[j + 1] = col[j];
            --j;
        }
        col[j + 1] = v;
    }
}

// One traversal: each row's columns (slots, traversal order) go to a
// row-major staging area of K entries per row; cnt gets the full count and
// flag[0] is set when a row has more than K entries.
__global__ __launch_bounds__(256) void k_csr_stage(Grid g, NbrView nv, int n, int K,
                                                   int32_t* __restrict__ stage,
                                                   int64_t* __restrict__ cnt, int32_t* flag,
                                                   double sf)
{
    const int t = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const int s = t / LG, gl = t % LG;
    if (s >= n) return;
    double xi = nv.xs[s], yi = nv.ys[s], hi = nv.hs[s];
    int li = key_level(g, nv.keys[s]);
    const int slot = nv.perm[s];
    int32_t* row = stage + (int64_t)slot * K;
    int k = 0;
    group_walk_x<LG>(g, nv, nv.perm, xi, yi, hi, li, gl,
                     [&](int, bool pass, double, double, double, double, int32_t j) {
                         int tot;
                         const int e = k + group_rank<LG>(pass, gl, &tot);
                         if (pass && e < K) row[e] = j;
                         k += tot;
                     },
                     sf);
    if (gl == 0) {
        cnt[slot] = k;
        if (k > K) flag[0] = 1;
    }
}

// One wave per row: bitonic sort of up to 64 R entries held R per lane
// (element e = r 64 + lane), written ascending to the row's CSR range.
template <int R>
__device__ __forceinline__ void wave_sort_row(const int32_t* __restrict__ src, int len,
                                              int32_t* __restrict__ dst, int lane)
{
    int v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = r * 64 + lane;
        v[r] = e < len ? src[e] : 0x7fffffff;
    }
#pragma unroll
    for (int k = 2; k <= 64 * R; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= 64) {
                const int rj = j >> 6;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (r & rj) continue;
                    const int r2 = r | rj;
                    const bool up = ((r * 64 + lane) & k) == 0;
                    const int a = v[r], b = v[r2];
                    const int lo = a < b ? a : b, hi = a < b ? b : a;
                    v[r] = up ? lo : hi;
                    v[r2] = up ? hi : lo;
                }
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int o = __shfl_xor(v[r], j, 64);
                    const bool up = ((r * 64 + lane) & k) == 0;
                    const bool low = (lane & j) == 0;
                    v[r] = (low == up) ? min(v[r], o) : max(v[r], o);
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = r * 64 + lane;
        if (e < len) dst[e] = v[r];
    }
}

__global__ __launch_bounds__(256) void k_csr_sort_staged(int n, int K, const int32_t* __restrict__ stage,
                                                         const int64_t* __restrict__ rp,
                                                         int32_t* __restrict__ col)
{
    const int lane = __lane_id();
    const int row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= n) return;
    const int64_t beg = rp[row];
    const int len = (int)(rp[row + 1] - beg);
    const int32_t* src = stage + (int64_t)row * K;
    if (len <= 64)
        wave_sort_row<1>(src, len, col + beg, lane);
    else if (len <= 128)
        wave_sort_row<2>(src, len, col + beg, lane);
    else
        wave_sort_row<4>(src, len, col + beg, lane);
}

int nbr_export_csr(sph_ctx* c, int n, int64_t* row_ptr, int32_t* col, int64_t cap, int64_t* nnz,
                   double sf)
{
    Work& w = c->w;
    const Grid& g = c->grid;
    NbrView nv = nbr_view(c);
    // the staging area is the rate passes' neighbour-list buffer
    const int K = w.nl_k < 256 ? w.nl_k : 256;
    c->list_valid = 0;
    if (n > 0) {
        hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, c->stream, w.status, (int64_t)4);
        hipLaunchKernelGGL(k_csr_stage, dim3((unsigned)cdiv((int64_t)n * LG, 256)), dim3(256), 0, c->stream, g, nv,
                           n, K, w.nl_idx, w.cnt64, w.status + 2, sf);
        LAUNCHCHK(c, "csr_stage");
    }
    int rc = scan_exclusive_i64(c, w.cnt64, row_ptr, n);
    if (rc) return rc;
    int64_t tot = 0;
    int32_t st[SPH_STATUS_SORT + 1] = {0};
    const Readback rb[2] = {{&tot, row_ptr + n, 8}, {st, w.status, (int)sizeof(st)}};
    rc = readback(c, rb, n > 0 ? 2 : 1);
    if (rc) return rc;
    if (st[SPH_STATUS_SORT]) {
        set_err(c, "neighbour sort: a look-back wait ran out");
        return SPH_E_DEVICE;
    }
    *nnz = tot;
    if (tot > cap) {
        set_err(c, "neighbour list needs %lld entries, capacity %lld", (long long)tot, (long long)cap);
        return SPH_E_CAPACITY;
    }
    if (n == 0) return SPH_OK;
    if (st[2] == 0) {
        hipLaunchKernelGGL(k_csr_sort_staged, dim3((unsigned)cdiv(n, 4)), dim3(256), 0, c->stream, n, K,
                           w.nl_idx, row_ptr, col);
        LAUNCHCHK(c, "csr_sort");
        return SPH_OK;
    }
    // some row is longer than the staging width: traverse again into the CSR
    hipLaunchKernelGGL(k_csr_fill, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, c->stream, g, nv, n,
                       row_ptr, col, sf);
    hipLaunchKernelGGL(k_sort_rows, dim3((unsigned)cdiv(n, 4)), dim3(256), 0, c->stream, n, row_ptr,
                       col, w.long_rows, w.status);
    hipLaunchKernelGGL(k_sort_long_rows, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, c->stream,
                       row_ptr, col, w.long_rows, w.status);
    LAUNCHCHK(c, "csr_fill");
    return SPH_OK;
}

// ---------------------------------------------------------------------------
// Batched neighbour build: keys, segmented radix sort, cell tables and the
// rate-pass list of every simulation of a batch, one launch per kernel.  The
// digit histogram is laid out simulation by simulation ([simulation][digit]
// [tile]), so one exclusive scan over it gives, for every simulation, the
// packed prefix of the simulations before it plus its own digit offsets:
// the same result as sorting the batch by (simulation, key) with the
// simulation as the most significant digit, without sorting that digit.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_keys_b(Batch B, const double* __restrict__ x,
                                                const double* __restrict__ y,
                                                const double* __restrict__ h, uint64_t* keys,
                                                int32_t* vals, unsigned long long* hmax,
                                                int32_t* lcount, const int32_t* __restrict__ rebuild)
{
    int lb;
    const int sid = batch_find(B, BM_P256, blockIdx.x, &lb);
    if (!rebuild[sid]) return;  // the simulation keeps its structure
    const SimDesc& sd = batch_desc(B, sid);
    const int il = lb * 256 + threadIdx.x;
    keys_body(sd.g, il < sd.n, (int)(sd.off + il), x, y, h, keys, vals,
              hmax + (int64_t)sd.slot * SPH_MAXL, lcount + (int64_t)sd.slot * SPH_MAXL);
}

__global__ __launch_bounds__(RS_THREADS) void k_rs_hist_b(Batch B, const uint64_t* __restrict__ keys,
                                                          int shift, uint32_t* hist,
                                                          const int32_t* __restrict__ rebuild)
{
    int t;
    const int sid = batch_find(B, BM_TILE, blockIdx.x, &t);
    const SimDesc* d = B.sims + sid;
    const int64_t rem = d->n - (int64_t)t * RS_TILE;
    const int tn = (int)(rem < RS_TILE ? rem : RS_TILE);
    if (!rebuild[sid]) {
        // a kept simulation is not sorted, but its tiles still count their
        // particles (all in digit 0): the scan over the whole batch then
        // places the other simulations as when every one is sorted
        uint32_t* hs = hist + d->hoff + t;
        for (int dg = threadIdx.x; dg < RS_BINS; dg += RS_THREADS)
            hs[(int64_t)dg * d->ntile] = dg == 0 ? (uint32_t)tn : 0u;
        return;
    }
    rs_hist_tile(keys, d->off + (int64_t)t * RS_TILE, tn, shift, hist + d->hoff + t, d->ntile);
}

__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter_b(Batch B, const uint64_t* __restrict__ kin,
                                                             const int32_t* __restrict__ vin,
                                                             uint64_t* __restrict__ kout,
                                                             int32_t* __restrict__ vout, int shift,
                                                             const uint32_t* __restrict__ offs,
                                                             const int32_t* __restrict__ rebuild)
{
    int t;
    const int sid = batch_find(B, BM_TILE, blockIdx.x, &t);
    if (!rebuild[sid]) return;
    const SimDesc* d = B.sims + sid;
    const int64_t rem = d->n - (int64_t)t * RS_TILE;
    const int tn = (int)(rem < RS_TILE ? rem : RS_TILE);
    rs_scatter_tile(kin, vin, kout, vout, d->off + (int64_t)t * RS_TILE, tn, shift,
                    offs + d->hoff + t, d->ntile, d->off - d->packed);
}

__global__ __launch_bounds__(256) void k_tables_b(Batch B, const uint64_t* __restrict__ keys,
                                                  const int32_t* __restrict__ perm,
                                                  const double* __restrict__ x,
                                                  const double* __restrict__ y,
                                                  const double* __restrict__ h, double4* xyh,
                                                  int2* tab, const int32_t* __restrict__ rebuild)
{
    int lb;
    const int sid = batch_find(B, BM_P256, blockIdx.x, &lb);
    if (!rebuild[sid]) return;
    const SimDesc& sd = batch_desc(B, sid);
    const int il = lb * 256 + threadIdx.x;
    if (il >= sd.n) return;
    tables_body(sd.g, (int)(sd.off + il), (int)sd.off, (int)(sd.off + sd.n), keys, perm, x, y, h,
                nullptr, nullptr, nullptr, xyh, tab + sd.toff);
}

__global__ __launch_bounds__(256) void k_build_list_b(Batch B, NbrView nv0, NbrList nl,
                                                      const int32_t* __restrict__ rebuild)
{
    int lb;
    const int sid = batch_find(B, BM_P64, xcd_block(blockIdx.x, gridDim.x), &lb);
    if (!rebuild[sid]) return;
    const SimDesc& sd = batch_desc(B, sid);
    const int t = lb * 256 + threadIdx.x;
    const int sl = t / LG, gl = t % LG;
    if (sl >= sd.n) return;
    // every pair within (1 + skin) times the support, as a context's list
    build_list_body<LG>(sd.g, batch_view(nv0, sd, sid), nl, (int)(sd.off + sl), gl, 1.0 + sd.skin);
}

// The cell tables, level maxima and counts of the simulations rebuilt in
// this evaluation are cleared (blockIdx.y: the simulation).
__global__ __launch_bounds__(256) void k_zero_build_b(Batch B, int2* tab, unsigned long long* hmax,
                                                      int32_t* lcount, const int32_t* __restrict__ rebuild)
{
    const int sid = (int)blockIdx.y;
    if (sid >= B.nsim || !rebuild[sid]) return;
    const SimDesc& sd = batch_desc(B, sid);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < sd.ntab;
         i += (int64_t)gridDim.x * blockDim.x)
        tab[sd.toff + i] = make_int2(0, 0);
    if (blockIdx.x == 0 && threadIdx.x < SPH_MAXL) {
        hmax[(int64_t)sd.slot * SPH_MAXL + threadIdx.x] = 0ull;
        lcount[(int64_t)sd.slot * SPH_MAXL + threadIdx.x] = 0;
    }
}

// A rebuilt simulation's sorted keys and order, moved to the first buffer
// when the passes ended in the second.
__global__ __launch_bounds__(256) void k_keep_sorted_b(Batch B, const uint64_t* __restrict__ kin,
                                                       const int32_t* __restrict__ vin, uint64_t* kout,
                                                       int32_t* vout, const int32_t* __restrict__ rebuild)
{
    int lb;
    const int sid = batch_find(B, BM_P256, blockIdx.x, &lb);
    if (!rebuild[sid]) return;
    const SimDesc& sd = batch_desc(B, sid);
    const int il = lb * 256 + threadIdx.x;
    if (il >= sd.n) return;
    const int64_t i = sd.off + il;
    kout[i] = kin[i];
    vout[i] = vin[i];
}

int batch_build(hipStream_t st, const BatchBufs& b, const BatchLaunch& L, const double* x,
                const double* y, const double* h, const uint64_t** keys, const int32_t** perm)
{
    // only the simulations whose rebuild flag is set (L.rebuild) are sorted,
    // tabled and listed; the others keep their order, tables and list
    const int nsim = L.B.nsim;
    hipLaunchKernelGGL(k_zero_build_b, dim3(64, (unsigned)nsim), dim3(256), 0, st, L.B, b.tab, b.hmax,
                       b.lcount, (const int32_t*)L.rebuild);
    hipLaunchKernelGGL(k_keys_b, dim3((unsigned)L.nblk[BM_P256]), dim3(256), 0, st, L.B, x, y, h,
                       b.keys_a, b.vals_a, b.hmax, b.lcount, (const int32_t*)L.rebuild);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return SPH_E_DEVICE;
    uint64_t *ka = b.keys_a, *kb = b.keys_b;
    int32_t *va = b.vals_a, *vb = b.vals_b;
    for (int p = 0; p < L.npass; ++p) {
        const int shift = RS_BITS * p;
        hipLaunchKernelGGL(k_rs_hist_b, dim3((unsigned)L.nblk[BM_TILE]), dim3(RS_THREADS), 0, st, L.B,
                           (const uint64_t*)ka, shift, b.hist, (const int32_t*)L.rebuild);
        e = scan_rec_s<uint32_t>(st, b.hist, b.hist, L.hist_n, L.hist_n, b.scan_tmp);
        if (e != hipSuccess) return SPH_E_DEVICE;
        hipLaunchKernelGGL(k_rs_scatter_b, dim3((unsigned)L.nblk[BM_TILE]), dim3(RS_THREADS), 0, st,
                           L.B, (const uint64_t*)ka, (const int32_t*)va, kb, vb, shift,
                           (const uint32_t*)b.hist, (const int32_t*)L.rebuild);
        uint64_t* tk = ka; ka = kb; kb = tk;
        int32_t* tv = va; va = vb; vb = tv;
    }
    if (ka != b.keys_a) {
        // an odd number of passes: the sorted keys go back to the first
        // buffer, where a kept simulation's keys stay between builds
        hipLaunchKernelGGL(k_keep_sorted_b, dim3((unsigned)L.nblk[BM_P256]), dim3(256), 0, st, L.B,
                           (const uint64_t*)ka, (const int32_t*)va, b.keys_a, b.vals_a,
                           (const int32_t*)L.rebuild);
        ka = b.keys_a;
        va = b.vals_a;
    }
    hipLaunchKernelGGL(k_tables_b, dim3((unsigned)L.nblk[BM_P256]), dim3(256), 0, st, L.B,
                       (const uint64_t*)ka, (const int32_t*)va, x, y, h, b.xyh, b.tab,
                       (const int32_t*)L.rebuild);
    const NbrView nv{nullptr, nullptr, nullptr, b.xyh, va, ka, b.tab, b.hmax, b.lcount};
    const NbrList nlst{b.nl_idx, b.nl_cnt, b.nl_k, (int)b.stride, b.list_flag};
    hipLaunchKernelGGL(k_build_list_b, dim3((unsigned)L.nblk[BM_P64]), dim3(256), 0, st, L.B, nv,
                       nlst, (const int32_t*)L.rebuild);
    e = hipGetLastError();
    if (e != hipSuccess) return SPH_E_DEVICE;
    *keys = ka;
    *perm = va;
    return SPH_OK;
}
