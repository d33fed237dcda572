// Serving pool: continuous batching of independent simulations on one GPU.
//
// Each admitted simulation gets one block of the caller's arena (first fit,
// 256-byte aligned): its state arrays, a pair counter and a lean context
// workspace.  Its predict-evaluate-correct step (sph_step with nsteps = 1,
// the neighbour list rebuilt every evaluation so that no host round trip is
// needed) is captured once into a HIP graph and replayed.  Simulations are
// spread over a few streams by resident particle count, so that the graphs
// of small simulations overlap on the device.  A simulation can be admitted
// or retired between any two pool steps; admission fails with SPH_E_AGAIN
// while no free block of the arena is large enough.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "sph_internal.h"

#define POOL_MAX_STREAMS 8

namespace {

struct Sim {
    int32_t id;
    size_t off, bytes;
    sph_ctx* ctx;
    sph_particles ps;
    double dt;
    int stream;
    hipGraphExec_t exec;
    bool captured;
    hipEvent_t ev_end;
    float last_ms;
    int64_t steps;
    unsigned long long* pairs;
};

}  // namespace

struct sph_pool {
    char* arena;
    size_t bytes;
    std::vector<std::pair<size_t, size_t>> free_blocks;  // (offset, size), sorted by offset
    std::vector<Sim*> sims;                               // by id; nullptr once retired
    int nstreams;
    hipStream_t streams[POOL_MAX_STREAMS];
    hipEvent_t ev_start[POOL_MAX_STREAMS];
    int64_t stream_load[POOL_MAX_STREAMS];
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

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static size_t state_bytes(int64_t n, bool with_kind)
{
    const size_t N = (size_t)(n > 0 ? n : 1);
    return 9 * align256(8 * N) + (with_kind ? align256(4 * N) : 0) + 256;  // + pair counter
}

static sph_config lean_cfg(const sph_config* cfg)
{
    sph_config c = *cfg;
    c.lean = 1;
    return c;
}

extern "C" size_t sph_pool_footprint(const sph_config* cfg, int64_t n)
{
    if (!cfg || n < 0) return 0;
    sph_config c = lean_cfg(cfg);
    size_t ws = sph_workspace_bytes(&c, n);
    if (!ws) return 0;
    return state_bytes(n, true) + align256(ws);
}

extern "C" int sph_pool_create(void* arena, size_t arena_bytes, int32_t nstreams, sph_pool** out)
{
    if (!out) return SPH_E_INVAL;
    *out = nullptr;
    if (!arena || ((uintptr_t)arena & 255) || arena_bytes < 256 || nstreams < 1 ||
        nstreams > POOL_MAX_STREAMS)
        return SPH_E_INVAL;
    sph_pool* p = new sph_pool();
    p->arena = (char*)arena;
    p->bytes = arena_bytes & ~(size_t)255;
    p->free_blocks.push_back({0, p->bytes});
    p->nstreams = nstreams;
    p->err[0] = 0;
    for (int k = 0; k < nstreams; ++k) {
        p->stream_load[k] = 0;
        if (hipStreamCreateWithFlags(&p->streams[k], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreate(&p->ev_start[k]) != hipSuccess) {
            for (int j = 0; j < k; ++j) {
                hipStreamDestroy(p->streams[j]);
                hipEventDestroy(p->ev_start[j]);
            }
            delete p;
            return SPH_E_DEVICE;
        }
    }
    *out = p;
    return SPH_OK;
}

static void sim_free(sph_pool* p, Sim* s)
{
    if (s->captured) hipGraphExecDestroy(s->exec);
    hipEventDestroy(s->ev_end);
    sph_destroy(s->ctx);
    p->stream_load[s->stream] -= s->ps.n;
    // return the block, coalescing with its neighbours
    auto& fb = p->free_blocks;
    size_t i = 0;
    while (i < fb.size() && fb[i].first < s->off) ++i;
    fb.insert(fb.begin() + (long)i, {s->off, s->bytes});
    if (i + 1 < fb.size() && fb[i].first + fb[i].second == fb[i + 1].first) {
        fb[i].second += fb[i + 1].second;
        fb.erase(fb.begin() + (long)i + 1);
    }
    if (i > 0 && fb[i - 1].first + fb[i - 1].second == fb[i].first) {
        fb[i - 1].second += fb[i].second;
        fb.erase(fb.begin() + (long)i);
    }
    delete s;
}

extern "C" void sph_pool_destroy(sph_pool* p)
{
    if (!p) return;
    for (int k = 0; k < p->nstreams; ++k) hipStreamSynchronize(p->streams[k]);
    for (Sim* s : p->sims)
        if (s) sim_free(p, s);
    for (int k = 0; k < p->nstreams; ++k) {
        hipStreamDestroy(p->streams[k]);
        hipEventDestroy(p->ev_start[k]);
    }
    delete p;
}

extern "C" const char* sph_pool_last_error(const sph_pool* p) { return p ? p->err : "no pool"; }

__global__ void k_pool_zero(unsigned long long* a) { a[0] = 0ull; }

extern "C" int sph_pool_admit(sph_pool* p, const sph_config* cfg, const sph_particles* init, double dt,
                              int32_t* sim_id)
{
    if (!p || !cfg || !init || !sim_id) return SPH_E_INVAL;
    if (!(dt > 0)) return pool_err(p, SPH_E_INVAL, "dt must be > 0");
    const int64_t n = init->n;
    if (n < 1 || n > init->capacity || !init->x || !init->y || !init->u || !init->v || !init->p ||
        !init->h || !init->mq || !init->rho)
        return pool_err(p, SPH_E_INVAL, "initial state incomplete (n=%lld)", (long long)n);
    const sph_config lc = lean_cfg(cfg);
    const size_t ws = sph_workspace_bytes(&lc, n);
    if (!ws) return pool_err(p, SPH_E_INVAL, "invalid configuration");
    const bool with_kind = init->kind != nullptr;
    const size_t need = state_bytes(n, with_kind) + align256(ws);
    // first fit
    size_t bi = p->free_blocks.size();
    for (size_t i = 0; i < p->free_blocks.size(); ++i)
        if (p->free_blocks[i].second >= need) {
            bi = i;
            break;
        }
    if (bi == p->free_blocks.size())
        return pool_err(p, SPH_E_AGAIN, "no free block of %zu bytes", need);
    Sim* s = new Sim();
    s->off = p->free_blocks[bi].first;
    s->bytes = need;
    s->dt = dt;
    s->captured = false;
    s->last_ms = 0.f;
    s->steps = 0;
    // least-loaded stream
    int st = 0;
    for (int k = 1; k < p->nstreams; ++k)
        if (p->stream_load[k] < p->stream_load[st]) st = k;
    s->stream = st;
    char* base = p->arena + s->off;
    size_t o = 0;
    auto take = [&](size_t b) {
        char* q = base + o;
        o += align256(b);
        return q;
    };
    const size_t N = (size_t)n;
    sph_particles& ps = s->ps;
    ps.n = n;
    ps.capacity = n;
    double** f[8] = {&ps.x, &ps.y, &ps.u, &ps.v, &ps.p, &ps.rho, &ps.h, &ps.mref};
    for (int k = 0; k < 8; ++k) *f[k] = (double*)take(8 * N);
    ps.mq = (int64_t*)take(8 * N);
    ps.kind = with_kind ? (int32_t*)take(4 * N) : nullptr;
    s->pairs = (unsigned long long*)take(256);
    void* wsp = base + o;
    hipStream_t stream = p->streams[st];
    int rc = sph_create(&lc, n, wsp, ws, (void*)stream, &s->ctx);
    if (rc) {
        delete s;
        return pool_err(p, rc, "context creation failed (%d)", rc);
    }
    s->ctx->skin = 0.0;  // rebuild the list every evaluation: no host round trip
    s->ctx->pair_acc = s->pairs;
    if (hipEventCreate(&s->ev_end) != hipSuccess) {
        sph_destroy(s->ctx);
        delete s;
        return pool_err(p, SPH_E_DEVICE, "event creation failed");
    }
    const double* src[8] = {init->x, init->y, init->u, init->v, init->p, init->rho, init->h, init->mref};
    // the initial state may still be written by work on other streams (the
    // pool's streams do not wait for the null stream): wait for the device
    hipError_t e = hipDeviceSynchronize();
    // m_ref is optional (the pool does not adapt): it is copied when given
    for (int k = 0; k < 8 && e == hipSuccess; ++k)
        if (src[k]) e = hipMemcpyAsync(*f[k], src[k], 8 * N, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(ps.mq, init->mq, 8 * N, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess && with_kind)
        e = hipMemcpyAsync(ps.kind, init->kind, 4 * N, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_pool_zero, dim3(1), dim3(1), 0, stream, s->pairs);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        hipEventDestroy(s->ev_end);
        sph_destroy(s->ctx);
        delete s;
        return pool_err(p, SPH_E_DEVICE, "initial copy failed: %s", hipGetErrorString(e));
    }
    // commit the block
    auto& blk = p->free_blocks[bi];
    blk.first += need;
    blk.second -= need;
    if (blk.second == 0) p->free_blocks.erase(p->free_blocks.begin() + (long)bi);
    p->stream_load[st] += n;
    s->id = (int32_t)p->sims.size();
    p->sims.push_back(s);
    *sim_id = s->id;
    return SPH_OK;
}

static Sim* find(sph_pool* p, int32_t id)
{
    if (id < 0 || (size_t)id >= p->sims.size()) return nullptr;
    return p->sims[(size_t)id];
}

static int capture(sph_pool* p, Sim* s)
{
    hipStream_t st = p->streams[s->stream];
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed) != hipSuccess)
        return pool_err(p, SPH_E_DEVICE, "begin capture failed");
    int rc = step_run(s->ctx, &s->ps, s->dt, 1);
    hipError_t e = hipStreamEndCapture(st, &g);
    if (rc) {
        if (g) hipGraphDestroy(g);
        return pool_err(p, rc, "step capture failed: %s", s->ctx->err);
    }
    if (e != hipSuccess) return pool_err(p, SPH_E_DEVICE, "end capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&s->exec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) return pool_err(p, SPH_E_DEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
    s->captured = true;
    return SPH_OK;
}

extern "C" int sph_pool_step(sph_pool* p, int32_t nsteps)
{
    if (!p || nsteps < 0) return SPH_E_INVAL;
    for (int k = 0; k < p->nstreams; ++k)
        if (hipEventRecord(p->ev_start[k], p->streams[k]) != hipSuccess)
            return pool_err(p, SPH_E_DEVICE, "event record failed");
    for (Sim* s : p->sims) {
        if (!s) continue;
        if (!s->captured) {
            int rc = capture(p, s);
            if (rc) return rc;
        }
        hipStream_t st = p->streams[s->stream];
        for (int k = 0; k < nsteps; ++k)
            if (hipGraphLaunch(s->exec, st) != hipSuccess)
                return pool_err(p, SPH_E_DEVICE, "graph launch failed");
        if (hipEventRecord(s->ev_end, st) != hipSuccess)
            return pool_err(p, SPH_E_DEVICE, "event record failed");
    }
    for (int k = 0; k < p->nstreams; ++k)
        if (hipStreamSynchronize(p->streams[k]) != hipSuccess)
            return pool_err(p, SPH_E_DEVICE, "stream synchronize failed");
    for (Sim* s : p->sims) {
        if (!s) continue;
        float ms = 0.f;
        hipEventElapsedTime(&ms, p->ev_start[s->stream], s->ev_end);
        s->last_ms = ms;
        s->steps += nsteps;
    }
    return SPH_OK;
}

extern "C" int sph_pool_sim_stats(sph_pool* p, int32_t sim_id, double* last_ms, int64_t* steps,
                                  int64_t* pair_evals)
{
    if (!p) return SPH_E_INVAL;
    Sim* s = find(p, sim_id);
    if (!s) return pool_err(p, SPH_E_INVAL, "no simulation %d", sim_id);
    if (last_ms) *last_ms = s->last_ms;
    if (steps) *steps = s->steps;
    if (pair_evals) {
        unsigned long long v = 0;
        hipStream_t st = p->streams[s->stream];
        if (hipMemcpyAsync(&v, s->pairs, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return pool_err(p, SPH_E_DEVICE, "counter read failed");
        *pair_evals = (int64_t)v;
    }
    return SPH_OK;
}

extern "C" int sph_pool_read(sph_pool* p, int32_t sim_id, sph_particles* dst)
{
    if (!p || !dst) return SPH_E_INVAL;
    Sim* s = find(p, sim_id);
    if (!s) return pool_err(p, SPH_E_INVAL, "no simulation %d", sim_id);
    const size_t N = (size_t)s->ps.n;
    if (dst->capacity < s->ps.n) return pool_err(p, SPH_E_CAPACITY, "destination too small");
    hipStream_t st = p->streams[s->stream];
    const double* src[8] = {s->ps.x, s->ps.y, s->ps.u, s->ps.v, s->ps.p, s->ps.rho, s->ps.h, s->ps.mref};
    double* d[8] = {dst->x, dst->y, dst->u, dst->v, dst->p, dst->rho, dst->h, dst->mref};
    // dst may still be written by work on other streams: wait for the device
    hipError_t e = hipDeviceSynchronize();
    for (int k = 0; k < 8 && e == hipSuccess; ++k)
        if (d[k]) e = hipMemcpyAsync(d[k], src[k], 8 * N, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && dst->mq) e = hipMemcpyAsync(dst->mq, s->ps.mq, 8 * N, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && dst->kind && s->ps.kind)
        e = hipMemcpyAsync(dst->kind, s->ps.kind, 4 * N, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return pool_err(p, SPH_E_DEVICE, "read failed: %s", hipGetErrorString(e));
    dst->n = s->ps.n;
    return SPH_OK;
}

extern "C" int sph_pool_retire(sph_pool* p, int32_t sim_id)
{
    if (!p) return SPH_E_INVAL;
    Sim* s = find(p, sim_id);
    if (!s) return pool_err(p, SPH_E_INVAL, "no simulation %d", sim_id);
    hipStreamSynchronize(p->streams[s->stream]);
    p->sims[(size_t)sim_id] = nullptr;
    sim_free(p, s);
    return SPH_OK;
}

extern "C" int sph_pool_info(sph_pool* p, sph_pool_stats* out)
{
    if (!p || !out) return SPH_E_INVAL;
    memset(out, 0, sizeof(*out));
    size_t used = p->bytes;
    for (auto& b : p->free_blocks) {
        used -= b.second;
        if ((int64_t)b.second > out->largest_free) out->largest_free = (int64_t)b.second;
    }
    out->bytes_total = (int64_t)p->bytes;
    out->bytes_used = (int64_t)used;
    for (Sim* s : p->sims)
        if (s) {
            out->resident++;
            out->particles += s->ps.n;
        }
    return SPH_OK;
}
