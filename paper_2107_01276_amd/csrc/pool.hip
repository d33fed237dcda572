// Serving pool: continuous batching of independent simulations on one GPU.
//
// The resident simulations share one set of structure-of-arrays buffers
// carved from the caller's arena: each holds a contiguous range of particle
// slots (first fit, freed ranges coalesce) and a range of the cell-table
// region.  A pool step advances every resident simulation by one
// predict-evaluate-correct step of its own dt with one launch per kernel for
// all of them (batch_step): the blocks of each launch are dealt to the
// simulations by a per-launch-shape prefix table, and each block reads its
// simulation's descriptor (grid, dt, constants, ranges).  The launches of
// one step are captured into a HIP graph when the resident set changes and
// replayed.  FP64 and FP32 simulations form two groups, one after the other
// in the same graph.  Admission and retirement happen between steps; a
// simulation's result does not depend on the others in the batch.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "sph_internal.h"

#define POOL_LIST_K 64          // columns of the rate passes' list (a longer row is walked again)
#define POOL_MAX_SIMS_CAP 1024  // simulations resident at once, at most

namespace {

struct Range {
    int64_t off, len;
};

// First-fit allocator over [0, total) with coalescing of freed ranges.
struct FreeList {
    std::vector<Range> v;  // sorted by offset
    int64_t total = 0;
    void init(int64_t t)
    {
        total = t;
        v.clear();
        if (t > 0) v.push_back({0, t});
    }
    int64_t take(int64_t len)
    {
        for (size_t i = 0; i < v.size(); ++i)
            if (v[i].len >= len) {
                const int64_t off = v[i].off;
                v[i].off += len;
                v[i].len -= len;
                if (v[i].len == 0) v.erase(v.begin() + (long)i);
                return off;
            }
        return -1;
    }
    bool fits(int64_t len) const
    {
        for (const Range& r : v)
            if (r.len >= len) return true;
        return false;
    }
    void give(int64_t off, int64_t len)
    {
        if (len <= 0) return;
        size_t i = 0;
        while (i < v.size() && v[i].off < off) ++i;
        v.insert(v.begin() + (long)i, {off, len});
        if (i + 1 < v.size() && v[i].off + v[i].len == v[i + 1].off) {
            v[i].len += v[i + 1].len;
            v.erase(v.begin() + (long)i + 1);
        }
        if (i > 0 && v[i - 1].off + v[i - 1].len == v[i].off) {
            v[i - 1].len += v[i].len;
            v.erase(v.begin() + (long)i);
        }
    }
    int64_t largest() const
    {
        int64_t m = 0;
        for (const Range& r : v) m = std::max(m, r.len);
        return m;
    }
    int64_t free_total() const
    {
        int64_t s = 0;
        for (const Range& r : v) s += r.len;
        return s;
    }
};

struct PSim {
    bool live = false;
    int precision = SPH_FP32;
    Grid g;
    sph_config cfg;
    double dt = 0.0;
    int64_t off = 0, n = 0, toff = 0, ntab = 0;
    int32_t slot = 0;
    int64_t steps = 0;
    int64_t pairs_done = 0;  // pairs counted before the counter slot was freed
};

// Bytes per particle slot of the batch buffers.
size_t slot_bytes()
{
    return 7 * 8 + 8            // x y u v p rho h, mq
           + 2 * 8 + 2 * 4      // keys, vals (two each)
           + 32 + 32 + 16 + 32  // xyh, pa, puv, pf
           + 7 * 8              // m, rho, beta, dpav, dxs, dys, nnb (pair precision, 8-byte slots)
           + 4 * POOL_LIST_K + 4  // list and its counts
           + 5 * 8 + 5 * 8      // rates, half-step state
           + 2 * 4              // digit histogram (RS_BINS / RS_TILE entries per particle)
           + 3 * 8;             // positions and h the list was built at
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

struct sph_pool {
    char* arena;
    size_t bytes;
    hipStream_t stream;
    int32_t max_sims;
    int64_t ncap, tcap;
    BatchBufs buf;
    SimDesc* d_desc[2];
    int32_t* d_bstart[2];
    int32_t* d_rebuild[2];
    // pinned staging of the descriptors (two alternating buffers, each
    // reused once its last upload has run)
    SimDesc* h_desc[2];
    int32_t* h_bstart[2];
    hipEvent_t staged[2];
    int stage_k;
    FreeList pfree, tfree;
    std::vector<int32_t> free_slots;
    std::vector<PSim> sims;  // by id
    BatchLaunch L[2];        // per precision group (index = precision)
    bool dirty;
    bool have_graph;
    hipGraphExec_t exec;
    hipEvent_t ev0, ev1, ev_in;
    float last_ms;
    char err[512];
};

static int pool_err(sph_pool* p, int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(p->err, sizeof(p->err), fmt, ap);
    va_end(ap);
    return code;
}

static int pool_check_cfg(const sph_config* cfg)
{
    // the same limits as a context (sph_workspace_bytes is 0 for a bad one)
    sph_config c = *cfg;
    c.lean = 1;
    return sph_workspace_bytes(&c, 1) != 0;
}

extern "C" size_t sph_pool_footprint(const sph_config* cfg, int64_t n)
{
    if (!cfg || n < 0 || !pool_check_cfg(cfg)) return 0;
    Grid g;
    grid_setup(cfg, &g);
    return (size_t)n * slot_bytes() + (size_t)g.tab_total * sizeof(int2) + 4 * RS_BINS;
}

// Carves the arena: per-simulation tables and block maps, then the cell
// tables (1/16 of the arena), then the particle slots.
static bool pool_carve(sph_pool* p)
{
    char* base = p->arena;
    size_t off = 0;
    auto take = [&](size_t b) -> char* {
        off = align256(off);
        char* q = base + off;
        off += b;
        return q;
    };
    const int S = p->max_sims;
    for (int k = 0; k < 2; ++k) {
        p->d_desc[k] = (SimDesc*)take(sizeof(SimDesc) * (size_t)S);
        p->d_bstart[k] = (int32_t*)take(4 * (size_t)BM_COUNT * (S + 1));
        p->d_rebuild[k] = (int32_t*)take(4 * (size_t)S);
    }
    BatchBufs& b = p->buf;
    b.pairs = (unsigned long long*)take(8 * (size_t)S);
    b.list_flag = (int32_t*)take(256);
    b.hmax = (unsigned long long*)take(8 * (size_t)S * SPH_MAXL);
    b.lcount = (int32_t*)take(4 * (size_t)S * SPH_MAXL);
    if (off >= p->bytes) return false;
    size_t rest = p->bytes - align256(off);
    const size_t tab_bytes = rest / 16;
    p->tcap = (int64_t)(tab_bytes / sizeof(int2));
    b.tab = (int2*)take(tab_bytes);
    if (off >= p->bytes) return false;
    rest = p->bytes - align256(off);
    // particle slots; set aside the digit histogram's tile of slack per
    // simulation, and margin for the per-array alignment and the scan
    const size_t fixed = 4 * (size_t)RS_BINS * S + 64 * 256 + 65536;
    const size_t per = slot_bytes() + 1;
    const int64_t n = (int64_t)((rest > fixed ? rest - fixed : 0) / per);
    if (n < 1) return false;
    p->ncap = n;
    const size_t N = (size_t)n;
    double** f[7] = {&b.x, &b.y, &b.u, &b.v, &b.p, &b.rho, &b.h};
    for (int k = 0; k < 7; ++k) *f[k] = (double*)take(8 * N);
    b.mq = (int64_t*)take(8 * N);
    b.keys_a = (uint64_t*)take(8 * N);
    b.keys_b = (uint64_t*)take(8 * N);
    b.vals_a = (int32_t*)take(4 * N);
    b.vals_b = (int32_t*)take(4 * N);
    b.xyh = (double4*)take(32 * N);
    b.pa = (double4*)take(32 * N);
    b.puv = (double2*)take(16 * N);
    b.pf = take(32 * N);
    void** t[7] = {&b.m, &b.brho, &b.beta, &b.dpav, &b.dxs, &b.dys, &b.nnb};
    for (int k = 0; k < 7; ++k) *t[k] = take(8 * N);
    b.nl_k = POOL_LIST_K;
    b.nl_idx = (int32_t*)take(4 * (size_t)POOL_LIST_K * N);
    b.nl_cnt = (int32_t*)take(4 * N);
    b.stride = n;
    double** r[10] = {&b.r_dpdt, &b.r_dudt, &b.r_dvdt, &b.r_dxs, &b.r_dys,
                      &b.xh,     &b.yh,     &b.uh,     &b.vh,    &b.ph};
    for (int k = 0; k < 10; ++k) *r[k] = (double*)take(8 * N);
    b.xref = (double*)take(8 * N);
    b.yref = (double*)take(8 * N);
    b.href = (double*)take(8 * N);
    // digit histogram: one tile per RS_TILE particles plus one per simulation
    const int64_t hist_n = (int64_t)RS_BINS * (cdiv(n, RS_TILE) + S);
    b.hist = (uint32_t*)take(4 * (size_t)hist_n);
    b.scan_tmp = (uint32_t*)take(4 * (size_t)(2 * cdiv(hist_n, SCAN_TILE) + 256));
    return off <= p->bytes;
}

static void pool_free(sph_pool* p)
{
    if (p->have_graph) hipGraphExecDestroy(p->exec);
    for (int k = 0; k < 2; ++k) {
        if (p->h_desc[k]) hipHostFree(p->h_desc[k]);
        if (p->h_bstart[k]) hipHostFree(p->h_bstart[k]);
        if (p->staged[k]) hipEventDestroy(p->staged[k]);
    }
    if (p->ev0) hipEventDestroy(p->ev0);
    if (p->ev1) hipEventDestroy(p->ev1);
    if (p->ev_in) hipEventDestroy(p->ev_in);
    if (p->stream) hipStreamDestroy(p->stream);
    delete p;
}

__global__ void k_pool_zero_u64(unsigned long long* a, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0ull;
}

// h the list was built at, set to -1 for an admitted simulation: its first
// evaluation builds its structure and list
__global__ void k_pool_fill_f64(double* a, int64_t n, double v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

extern "C" int sph_pool_create(void* arena, size_t arena_bytes, int32_t max_sims, sph_pool** out)
{
    if (!out) return SPH_E_INVAL;
    *out = nullptr;
    if (!arena || ((uintptr_t)arena & 255) || arena_bytes < (1u << 20) || max_sims < 1 ||
        max_sims > POOL_MAX_SIMS_CAP)
        return SPH_E_INVAL;
    sph_pool* p = new sph_pool();
    memset(p->err, 0, sizeof(p->err));
    p->arena = (char*)arena;
    p->bytes = arena_bytes & ~(size_t)255;
    p->max_sims = max_sims;
    p->stream = nullptr;
    for (int k = 0; k < 2; ++k) {
        p->h_desc[k] = nullptr;
        p->h_bstart[k] = nullptr;
        p->staged[k] = nullptr;
    }
    p->ev0 = p->ev1 = p->ev_in = nullptr;
    p->have_graph = false;
    p->dirty = true;
    p->stage_k = 0;
    p->last_ms = 0.f;
    if (!pool_carve(p)) {
        delete p;
        return SPH_E_NOMEM;
    }
    bool ok = hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreate(&p->ev0) == hipSuccess && hipEventCreate(&p->ev1) == hipSuccess &&
              hipEventCreateWithFlags(&p->ev_in, hipEventDisableTiming) == hipSuccess;
    for (int k = 0; k < 2 && ok; ++k)
        ok = hipHostMalloc((void**)&p->h_desc[k], 2 * sizeof(SimDesc) * (size_t)max_sims) == hipSuccess &&
             hipHostMalloc((void**)&p->h_bstart[k],
                           4 * (size_t)2 * BM_COUNT * (max_sims + 1)) == hipSuccess &&
             hipEventCreateWithFlags(&p->staged[k], hipEventDisableTiming) == hipSuccess &&
             hipEventRecord(p->staged[k], p->stream) == hipSuccess;
    if (!ok) {
        pool_free(p);
        return SPH_E_DEVICE;
    }
    p->pfree.init(p->ncap);
    p->tfree.init(p->tcap);
    for (int s = max_sims - 1; s >= 0; --s) p->free_slots.push_back(s);
    hipLaunchKernelGGL(k_pool_zero_u64, dim3((unsigned)cdiv(max_sims, 256)), dim3(256), 0, p->stream,
                       p->buf.pairs, max_sims);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(p->stream) != hipSuccess) {
        pool_free(p);
        return SPH_E_DEVICE;
    }
    *out = p;
    return SPH_OK;
}

extern "C" void sph_pool_destroy(sph_pool* p)
{
    if (!p) return;
    hipStreamSynchronize(p->stream);
    pool_free(p);
}

extern "C" const char* sph_pool_last_error(const sph_pool* p) { return p ? p->err : "no pool"; }

static PSim* find(sph_pool* p, int32_t id)
{
    if (id < 0 || (size_t)id >= p->sims.size() || !p->sims[(size_t)id].live) return nullptr;
    return &p->sims[(size_t)id];
}

extern "C" int sph_pool_admit(sph_pool* p, const sph_config* cfg, const sph_particles* init, double dt,
                              void* stream, int32_t* sim_id)
{
    if (!p || !cfg || !init || !sim_id) return SPH_E_INVAL;
    if (!(dt > 0)) return pool_err(p, SPH_E_INVAL, "dt must be > 0");
    if (!pool_check_cfg(cfg)) return pool_err(p, SPH_E_INVAL, "invalid configuration");
    const int64_t n = init->n;
    if (n < 1 || n > init->capacity || !init->x || !init->y || !init->u || !init->v || !init->p ||
        !init->h || !init->mq || !init->rho)
        return pool_err(p, SPH_E_INVAL, "initial state incomplete (n=%lld)", (long long)n);
    if (init->kind)
        return pool_err(p, SPH_E_INVAL, "the pool steps fluid-only simulations (kind must be NULL)");
    PSim s;
    s.live = true;
    s.cfg = *cfg;
    s.precision = cfg->precision;
    grid_setup(cfg, &s.g);
    s.dt = dt;
    s.n = n;
    s.ntab = s.g.tab_total > 0 ? s.g.tab_total : 1;
    if (p->free_slots.empty() || !p->pfree.fits(n) || !p->tfree.fits(s.ntab))
        return pool_err(p, SPH_E_AGAIN, "no room for %lld particles and %lld table entries",
                        (long long)n, (long long)s.ntab);
    // the initial state is read on the pool's stream after the work the
    // caller enqueued on `stream` before this call
    hipError_t e = hipEventRecord(p->ev_in, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(p->stream, p->ev_in, 0);
    if (e != hipSuccess) return pool_err(p, SPH_E_DEVICE, "stream order: %s", hipGetErrorString(e));
    s.off = p->pfree.take(n);
    s.toff = p->tfree.take(s.ntab);
    s.slot = p->free_slots.back();
    p->free_slots.pop_back();
    const BatchBufs& b = p->buf;
    const size_t N = (size_t)n;
    const double* src[7] = {init->x, init->y, init->u, init->v, init->p, init->rho, init->h};
    double* dst[7] = {b.x, b.y, b.u, b.v, b.p, b.rho, b.h};
    for (int k = 0; k < 7 && e == hipSuccess; ++k)
        e = hipMemcpyAsync(dst[k] + s.off, src[k], 8 * N, hipMemcpyDeviceToDevice, p->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b.mq + s.off, init->mq, 8 * N, hipMemcpyDeviceToDevice, p->stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_pool_zero_u64, dim3(1), dim3(64), 0, p->stream, b.pairs + s.slot, 1);
        hipLaunchKernelGGL(k_pool_fill_f64, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, p->stream,
                           b.href + s.off, n, -1.0);
        e = hipGetLastError();
    }
    if (e != hipSuccess) {
        p->pfree.give(s.off, n);
        p->tfree.give(s.toff, s.ntab);
        p->free_slots.push_back(s.slot);
        return pool_err(p, SPH_E_DEVICE, "initial copy failed: %s", hipGetErrorString(e));
    }
    p->sims.push_back(s);
    *sim_id = (int32_t)(p->sims.size() - 1);
    p->dirty = true;
    return SPH_OK;
}

// Descriptors and block maps of each precision group, staged and uploaded
// on the pool's stream (ordered after the steps already enqueued).
static int pool_upload(sph_pool* p)
{
    const int k = p->stage_k;
    p->stage_k ^= 1;
    if (hipEventSynchronize(p->staged[k]) != hipSuccess)
        return pool_err(p, SPH_E_DEVICE, "staging wait failed");
    static const int PPB[BM_COUNT] = {256, 64, 128, RS_TILE};
    int64_t tab_n = 0;
    for (const PSim& s : p->sims)
        if (s.live) tab_n = std::max(tab_n, s.toff + s.ntab);
    for (int grp = 0; grp < 2; ++grp) {
        std::vector<const PSim*> mem;
        for (const PSim& s : p->sims)
            if (s.live && s.precision == grp) mem.push_back(&s);
        std::sort(mem.begin(), mem.end(), [](const PSim* a, const PSim* c) { return a->off < c->off; });
        const int ns = (int)mem.size();
        // each group stages into its own rows of the buffer
        SimDesc* hd = p->h_desc[k] + (size_t)grp * p->max_sims;
        int32_t* hb = p->h_bstart[k] + (size_t)grp * BM_COUNT * (p->max_sims + 1);
        BatchLaunch& L = p->L[grp];
        memset(&L, 0, sizeof(L));
        L.precision = grp;
        L.B.nsim = ns;
        if (ns == 0) continue;
        int64_t hoff = 0, packed = 0;
        int64_t nb[BM_COUNT] = {0, 0, 0, 0};
        int maxbits = 1;
        for (int i = 0; i < ns; ++i) {
            const PSim& s = *mem[(size_t)i];
            SimDesc& d = hd[i];
            memset(&d, 0, sizeof(d));
            d.g = s.g;
            d.off = s.off;
            d.n = s.n;
            d.toff = s.toff;
            d.hoff = hoff;
            d.packed = packed;
            d.ntile = (int32_t)cdiv(s.n, RS_TILE);
            d.slot = s.slot;
            d.dt = s.dt;
            d.rho0 = s.cfg.rho0;
            d.cs = s.cfg.cs;
            d.nu = s.cfg.nu;
            d.alpha_e = s.cfg.alpha_e;
            d.fx = s.cfg.body_force[0];
            d.fy = s.cfg.body_force[1];
            d.mass_q = s.cfg.mass_q;
            d.skin = s.cfg.list_skin;
            d.ntab = s.ntab;
            hoff += (int64_t)RS_BINS * d.ntile;
            packed += s.n;
            for (int m = 0; m < BM_COUNT; ++m) {
                hb[m * (ns + 1) + i] = (int32_t)nb[m];
                nb[m] += cdiv(s.n, PPB[m]);
            }
            maxbits = std::max(maxbits, batch_key_bits(&s.g));
        }
        for (int m = 0; m < BM_COUNT; ++m) {
            hb[m * (ns + 1) + ns] = (int32_t)nb[m];
            L.nblk[m] = (int32_t)nb[m];
        }
        L.hist_n = hoff;
        L.tab_n = tab_n;
        L.npass = (maxbits + RS_BITS - 1) / RS_BITS;
        L.B.sims = p->d_desc[grp];
        L.B.bstart = p->d_bstart[grp];
        L.rebuild = p->d_rebuild[grp];
        hipError_t e = hipMemcpyAsync(p->d_desc[grp], hd, sizeof(SimDesc) * (size_t)ns,
                                      hipMemcpyHostToDevice, p->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(p->d_bstart[grp], hb, 4 * (size_t)BM_COUNT * (ns + 1),
                               hipMemcpyHostToDevice, p->stream);
        if (e != hipSuccess) return pool_err(p, SPH_E_DEVICE, "upload: %s", hipGetErrorString(e));
    }
    if (hipEventRecord(p->staged[k], p->stream) != hipSuccess)
        return pool_err(p, SPH_E_DEVICE, "staging record failed");
    return SPH_OK;
}

static int pool_capture(sph_pool* p)
{
    if (p->have_graph) {
        hipGraphExecDestroy(p->exec);
        p->have_graph = false;
    }
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(p->stream, hipStreamCaptureModeRelaxed) != hipSuccess)
        return pool_err(p, SPH_E_DEVICE, "begin capture failed");
    int rc = SPH_OK;
    for (int grp = 0; grp < 2 && rc == SPH_OK; ++grp)
        if (p->L[grp].B.nsim > 0) rc = batch_step(p->stream, p->buf, p->L[grp]);
    const hipError_t e = hipStreamEndCapture(p->stream, &g);
    if (rc) {
        if (g) hipGraphDestroy(g);
        return pool_err(p, rc, "step capture failed");
    }
    if (e != hipSuccess) return pool_err(p, SPH_E_DEVICE, "end capture failed: %s", hipGetErrorString(e));
    const hipError_t ei = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (ei != hipSuccess)
        return pool_err(p, SPH_E_DEVICE, "graph instantiate failed: %s", hipGetErrorString(ei));
    p->have_graph = true;
    return SPH_OK;
}

extern "C" int sph_pool_step(sph_pool* p, int32_t nsteps)
{
    if (!p || nsteps < 0) return SPH_E_INVAL;
    bool any = false;
    for (const PSim& s : p->sims) any = any || s.live;
    if (!any || nsteps == 0) return SPH_OK;
    if (p->dirty) {
        int rc = pool_upload(p);
        if (rc == SPH_OK) rc = pool_capture(p);
        if (rc) return rc;
        p->dirty = false;
    }
    if (hipEventRecord(p->ev0, p->stream) != hipSuccess)
        return pool_err(p, SPH_E_DEVICE, "event record failed");
    for (int k = 0; k < nsteps; ++k)
        if (hipGraphLaunch(p->exec, p->stream) != hipSuccess)
            return pool_err(p, SPH_E_DEVICE, "graph launch failed");
    if (hipEventRecord(p->ev1, p->stream) != hipSuccess ||
        hipEventSynchronize(p->ev1) != hipSuccess)
        return pool_err(p, SPH_E_DEVICE, "step failed: %s", hipGetErrorString(hipGetLastError()));
    float ms = 0.f;
    hipEventElapsedTime(&ms, p->ev0, p->ev1);
    p->last_ms = ms / (float)nsteps;
    for (PSim& s : p->sims)
        if (s.live) s.steps += nsteps;
    return SPH_OK;
}

static int read_pairs(sph_pool* p, int32_t slot, int64_t* out)
{
    unsigned long long v = 0;
    if (hipMemcpyAsync(&v, p->buf.pairs + slot, 8, hipMemcpyDeviceToHost, p->stream) != hipSuccess ||
        hipStreamSynchronize(p->stream) != hipSuccess)
        return pool_err(p, SPH_E_DEVICE, "counter read failed");
    *out = (int64_t)v;
    return SPH_OK;
}

extern "C" int sph_pool_sim_stats(sph_pool* p, int32_t sim_id, double* last_ms, int64_t* steps,
                                  int64_t* pair_evals)
{
    if (!p) return SPH_E_INVAL;
    if (sim_id < 0 || (size_t)sim_id >= p->sims.size())
        return pool_err(p, SPH_E_INVAL, "no simulation %d", sim_id);
    PSim& s = p->sims[(size_t)sim_id];
    if (last_ms) *last_ms = p->last_ms;
    if (steps) *steps = s.steps;
    if (pair_evals) {
        if (!s.live) {
            *pair_evals = s.pairs_done;
        } else {
            int rc = read_pairs(p, s.slot, pair_evals);
            if (rc) return rc;
        }
    }
    return SPH_OK;
}

extern "C" int sph_pool_read(sph_pool* p, int32_t sim_id, sph_particles* dst, void* stream)
{
    if (!p || !dst) return SPH_E_INVAL;
    PSim* s = find(p, sim_id);
    if (!s) return pool_err(p, SPH_E_INVAL, "no simulation %d", sim_id);
    if (dst->capacity < s->n) return pool_err(p, SPH_E_CAPACITY, "destination too small");
    const size_t N = (size_t)s->n;
    const BatchBufs& b = p->buf;
    const double* src[7] = {b.x, b.y, b.u, b.v, b.p, b.rho, b.h};
    double* d[7] = {dst->x, dst->y, dst->u, dst->v, dst->p, dst->rho, dst->h};
    // dst may still be used by the caller's work on `stream`
    hipError_t e = hipEventRecord(p->ev_in, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(p->stream, p->ev_in, 0);
    for (int k = 0; k < 7 && e == hipSuccess; ++k)
        if (d[k]) e = hipMemcpyAsync(d[k], src[k] + s->off, 8 * N, hipMemcpyDeviceToDevice, p->stream);
    if (e == hipSuccess && dst->mq)
        e = hipMemcpyAsync(dst->mq, b.mq + s->off, 8 * N, hipMemcpyDeviceToDevice, p->stream);
    // the caller's later work on `stream` sees the copies
    if (e == hipSuccess) e = hipEventRecord(p->ev_in, p->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent((hipStream_t)stream, p->ev_in, 0);
    if (e != hipSuccess) return pool_err(p, SPH_E_DEVICE, "read failed: %s", hipGetErrorString(e));
    dst->n = s->n;
    return SPH_OK;
}

extern "C" int sph_pool_retire(sph_pool* p, int32_t sim_id)
{
    if (!p) return SPH_E_INVAL;
    PSim* s = find(p, sim_id);
    if (!s) return pool_err(p, SPH_E_INVAL, "no simulation %d", sim_id);
    int rc = read_pairs(p, s->slot, &s->pairs_done);
    if (rc) return rc;
    s->live = false;
    // later admissions reuse the ranges; their copies are ordered after the
    // steps already enqueued on the pool's stream
    p->pfree.give(s->off, s->n);
    p->tfree.give(s->toff, s->ntab);
    p->free_slots.push_back(s->slot);
    p->dirty = true;
    return SPH_OK;
}

extern "C" int sph_pool_info(sph_pool* p, sph_pool_stats* out)
{
    if (!p || !out) return SPH_E_INVAL;
    memset(out, 0, sizeof(*out));
    out->slots_total = p->ncap;
    out->slots_used = p->ncap - p->pfree.free_total();
    out->largest_free = p->pfree.largest();
    out->tables_total = p->tcap;
    out->tables_used = p->tcap - p->tfree.free_total();
    for (const PSim& s : p->sims)
        if (s.live) {
            out->resident++;
            out->particles += s.n;
        }
    out->max_resident = p->max_sims;
    out->last_step_ms = p->last_ms;
    return SPH_OK;
}
