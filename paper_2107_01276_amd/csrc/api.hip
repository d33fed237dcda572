// C ABI entry points (declared in include/sph.h): context creation,
// workspace carving, argument checks, error reporting and profiling.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>

#include "sph_internal.h"

#define SPH_VERSION 10000
#define COL_PER_PARTICLE 160
#define NL_K 256

void set_err(sph_ctx* c, const char* fmt, ...)
{
    if (!c) return;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(c->err, sizeof(c->err), fmt, ap);
    va_end(ap);
}

int check_hip(sph_ctx* c, hipError_t e, const char* what)
{
    set_err(c, "HIP error in %s: %s", what, hipGetErrorString(e));
    return SPH_E_DEVICE;
}

// Carves the workspace.  With base == NULL only the size is computed.
static size_t carve(Work* w, char* base, const Grid& g, int64_t cap, int lean, int list_k,
                    int csr_k = COL_PER_PARTICLE)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        off = (off + 255) & ~(size_t)255;
        void* p = base ? (void*)(base + off) : nullptr;
        off += bytes;
        return p;
    };
    int64_t C = cap > 0 ? cap : 1;
    const int64_t scan_n = C + 1;
    w->capacity = C;
    w->keys_a = (uint64_t*)take(8 * C);
    w->keys_b = (uint64_t*)take(8 * C);
    w->vals_a = (int32_t*)take(4 * C);
    w->vals_b = (int32_t*)take(4 * C);
    w->os_look = (uint32_t*)take(4 * (OS_MAXPASS * OS_BINS * cdiv(C, OS_TILE) + OS_MAXPASS * OS_BINS +
                                      OS_MAXPASS));
    w->scan_tmp = (int64_t*)take(8 * (2 * cdiv(scan_n, SCAN_TILE) + 256));
    w->tab = (int2*)take(sizeof(int2) * (g.tab_total > 0 ? g.tab_total : 1));
    w->hmax_bits = (unsigned long long*)take(8 * SPH_MAXL);
    w->lcount = (int32_t*)take(4 * SPH_MAXL);
    w->status = (int32_t*)take(4 * 64);
    w->ctr = (unsigned long long*)take(8 * 8);
    w->long_rows = (int32_t*)take(4 * C);
    w->xs = (double*)take(8 * C);
    w->ys = (double*)take(8 * C);
    w->hs = (double*)take(8 * C);
    w->xyh = (double4*)take(32 * C);
    w->us = (double*)take(8 * C);
    w->vs = (double*)take(8 * C);
    double** sc[12] = {&w->sc0, &w->sc1, &w->sc2, &w->sc3, &w->sc4, &w->sc5,
                       &w->sc6, &w->sc7, &w->sc8, &w->sc9, &w->sc10, &w->sc11};
    for (int k = 0; k < 12; ++k) *sc[k] = (double*)take(8 * (C > 1280 ? C : 1280));
    w->r_dpdt = (double*)take(8 * C);
    w->r_dudt = (double*)take(8 * C);
    w->r_dvdt = (double*)take(8 * C);
    w->r_dxs = (double*)take(8 * C);
    w->r_dys = (double*)take(8 * C);
    w->xh = (double*)take(8 * C);
    w->yh = (double*)take(8 * C);
    w->uh = (double*)take(8 * C);
    w->vh = (double*)take(8 * C);
    w->ph = (double*)take(8 * C);
    w->cnt64 = (int64_t*)take(8 * (C + 1));
    w->lean = lean;
    // adaptation, background and inlet/outlet buffers (not in a lean workspace)
    const int64_t CA = lean ? 0 : C;
    w->rp_tmp = lean ? nullptr : (int64_t*)take(8 * (C + 1));
    w->col_cap = (int64_t)csr_k * CA;
    w->col_tmp = lean ? nullptr : (int32_t*)take(4 * w->col_cap);
    w->flag = lean ? nullptr : (int32_t*)take(4 * (C + 1));
    w->closest = lean ? nullptr : (int32_t*)take(4 * C);
    w->idx_a = lean ? nullptr : (int32_t*)take(4 * (C + 1));
    w->idx_b = lean ? nullptr : (int32_t*)take(4 * (C + 1));
    w->i64_a = lean ? nullptr : (int64_t*)take(8 * (C + 1));
    w->i64_b = lean ? nullptr : (int64_t*)take(8 * (C + 1));
    for (int k = 0; k < 10; ++k) w->tmp_d[k] = lean ? nullptr : (double*)take(8 * C);
    for (int k = 0; k < 2; ++k) w->tmp_i32[k] = lean ? nullptr : (int32_t*)take(4 * C);
    for (int k = 0; k < 3; ++k) w->tmp_i64[k] = lean ? nullptr : (int64_t*)take(8 * C);
    w->red = (int64_t*)take(8 * 8192);
    w->nl_k = list_k;
    w->nl_idx = (int32_t*)take(4 * (size_t)list_k * C);
    w->nl_cnt = (int32_t*)take(4 * C);
    w->cnt_ex = lean ? nullptr : (int32_t*)take(4 * C);
    w->xref = (double*)take(8 * C);
    w->yref = (double*)take(8 * C);
    w->href = (double*)take(8 * C);
    w->list_flag = (int32_t*)take(4 * 64);
    w->ug = (double*)take(8 * C);
    w->vg = (double*)take(8 * C);
    w->ugs = (double*)take(8 * C);
    w->vgs = (double*)take(8 * C);
    w->pa = (double4*)take(32 * C);
    w->puv = (double2*)take(16 * C);
    w->pf = take(32 * C);
    w->sched_origin = lean ? nullptr : (int64_t*)take(8 * C);
    w->sched_sat = lean ? nullptr : (int32_t*)take(4 * C);
    return off + 256;
}

static int check_cfg(const sph_config* cfg)
{
    if (!cfg) return 0;
    for (int a = 0; a < 2; ++a)
        if (!(cfg->hi[a] > cfg->lo[a]) || !isfinite(cfg->hi[a]) || !isfinite(cfg->lo[a])) return 0;
    if (!(cfg->h_lo > 0) || !(cfg->h_hi >= cfg->h_lo)) return 0;
    if (cfg->precision != SPH_FP64 && cfg->precision != SPH_FP32) return 0;
    if (!(cfg->rho0 > 0) || !(cfg->mass_q > 0)) return 0;
    if (cfg->merge_iters < 0 || cfg->merge_iters > 8 || cfg->shift_iters < 0) return 0;
    if (!isfinite(cfg->wall_accel[0]) || !isfinite(cfg->wall_accel[1])) return 0;
    if (cfg->list_k < 0 || cfg->list_k > 1024 || (cfg->lean != 0 && cfg->lean != 1)) return 0;
    if (!(cfg->list_skin >= 0.0 && cfg->list_skin <= 1.0)) return 0;
    if (cfg->io_mode != 0 && cfg->io_mode != 1) return 0;
    for (int a = 0; a < 3; ++a)
        if (!isfinite(cfg->io_ref[a])) return 0;
    if (cfg->io_mode == 1 && !(cfg->cs > 0)) return 0;
    if (!(cfg->dt >= 0.0) || !isfinite(cfg->dt) || !(cfg->sol_k >= 0.0) || !isfinite(cfg->sol_k))
        return 0;
    if (cfg->n_adapt < 0 || cfg->n_bg < 0 || cfg->bg_passes < 0) return 0;
    if (cfg->csr_k < 0 || cfg->csr_k > 65536) return 0;
    return 1;
}

// eq. (timestep)
double timestep_of(const sph_config& cfg, double h_min)
{
    const double h = h_min > 0 ? h_min : cfg.h_lo;
    double dt = 0.25 * h / (cfg.u_ref + cfg.cs);
    if (cfg.nu > 0) {
        const double dv = 0.125 * h * h / cfg.nu;
        if (dv < dt) dt = dv;
    }
    return dt;
}

extern "C" int sph_set_schedule(sph_ctx* c, const sph_schedule* s)
{
    if (!c || !s) return SPH_E_INVAL;
    if (!rate_schedule_valid(*s) || !list_lanes_valid(s->list_lanes)) {
        set_err(c,
                "schedule {%d, %d, %d, %d, %d, %d} is not compiled in (a_lanes 2/4/8, a_waves 1/4/5, "
                "b_lanes 1/2/4, b_unroll 2/4, b_waves 1/4, list_lanes 2/4/8)",
                s->a_lanes, s->a_waves, s->b_lanes, s->b_unroll, s->b_waves, s->list_lanes);
        return SPH_E_INVAL;
    }
    if (s->list_lanes != c->sched.list_lanes) c->list_valid = 0;  // rebuilt with the new lanes
    c->sched = *s;
    return SPH_OK;
}

extern "C" int sph_get_schedule(const sph_ctx* c, sph_schedule* s)
{
    if (!c || !s) return SPH_E_INVAL;
    *s = c->sched;
    return SPH_OK;
}

extern "C" int32_t sph_bg_init_passes(const sph_config* cfg)
{
    if (!cfg || !(cfg->ds_min > 0.0) || !(cfg->ds_max >= cfg->ds_min) || !(cfg->cr > 1.0)) return 0;
    const double levels = log(cfg->ds_max / cfg->ds_min) / log(cfg->cr);
    return 3 * (int32_t)ceil(levels - 1e-12);
}

extern "C" double sph_timestep(const sph_config* cfg, double h_min)
{
    if (!check_cfg(cfg) || !(cfg->u_ref + cfg->cs > 0)) return 0.0;
    return timestep_of(*cfg, h_min);
}

static int csr_k_of(const sph_config* cfg) { return cfg->csr_k > 0 ? cfg->csr_k : COL_PER_PARTICLE; }

extern "C" int sph_version(void) { return SPH_VERSION; }

extern "C" size_t sph_workspace_bytes(const sph_config* cfg, int64_t capacity)
{
    if (!check_cfg(cfg) || capacity < 0) return 0;
    Grid g;
    grid_setup(cfg, &g);
    Work w;
    return carve(&w, nullptr, g, capacity, cfg->lean, cfg->list_k > 0 ? cfg->list_k : NL_K,
                 csr_k_of(cfg));
}

__global__ void k_init_counters(int32_t* status, unsigned long long* ctr)
{
    const int t = threadIdx.x;
    if (t < 64) status[t] = 0;
    if (t < 8) ctr[t] = 0ull;
}

// ---- host readbacks through the pinned mailbox ------------------------------

#define MBOX_WORDS 64

struct RbArgs {
    const uint32_t* src[4];
    int words[4];
    int n;
};

// One lane copies the words, then publishes the sequence number with a
// system-scope release, so the host sees the payload once it sees `seq`.
__global__ void k_readback(RbArgs a, uint32_t* mbox, uint32_t seq)
{
    if (threadIdx.x != 0) return;
    int o = 1;
    for (int k = 0; k < a.n; ++k)
        for (int w = 0; w < a.words[k]; ++w) mbox[o++] = a.src[k][w];
    __threadfence_system();
    __hip_atomic_store(mbox, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

int readback(sph_ctx* c, const Readback* items, int n)
{
    if (!c->mbox) {
        set_err(c, "this evaluation has no host mailbox (no readback is possible)");
        return SPH_E_INVAL;
    }
    if (n < 0 || n > 4) {
        set_err(c, "readback of %d items", n);
        return SPH_E_INVAL;
    }
    RbArgs a{};
    int tot = 0;
    for (int k = 0; k < n; ++k) {
        if (items[k].bytes % 4 || items[k].bytes < 0) {
            set_err(c, "readback of %d bytes", items[k].bytes);
            return SPH_E_INVAL;
        }
        a.src[k] = (const uint32_t*)items[k].src;
        a.words[k] = items[k].bytes / 4;
        tot += a.words[k];
    }
    a.n = n;
    if (tot > MBOX_WORDS - 4) {
        set_err(c, "readback of %d words", tot);
        return SPH_E_INVAL;
    }
    uint32_t seq = ++c->mbox_seq;
    if (seq == 0) seq = ++c->mbox_seq;
    hipLaunchKernelGGL(k_readback, dim3(1), dim3(64), 0, c->stream, a, c->mbox_dev, seq);
    LAUNCHCHK(c, "readback");
    // poll the mailbox; every few hundred polls ask the stream whether it
    // failed (or finished without publishing, which would be a fault)
    for (unsigned spin = 1;; ++spin) {
        if (__atomic_load_n(&c->mbox[0], __ATOMIC_ACQUIRE) == seq) break;
        if ((spin & 255) == 0) {
            const hipError_t e = hipStreamQuery(c->stream);
            if (e == hipErrorNotReady) continue;
            if (e == hipSuccess && __atomic_load_n(&c->mbox[0], __ATOMIC_ACQUIRE) == seq) break;
            set_err(c, "readback: %s", e == hipSuccess ? "mailbox not written" : hipGetErrorString(e));
            return SPH_E_DEVICE;
        }
    }
    int o = 1;
    for (int k = 0; k < n; ++k) {
        memcpy(items[k].dst, (const void*)(c->mbox + o), (size_t)items[k].bytes);
        o += a.words[k];
    }
    return SPH_OK;
}

extern "C" int sph_create(const sph_config* cfg, int64_t capacity, void* workspace,
                          size_t workspace_bytes, void* stream, sph_ctx** out)
{
    if (!out) return SPH_E_INVAL;
    *out = nullptr;
    if (!check_cfg(cfg) || capacity < 0 || capacity > (int64_t)INT32_MAX - 1) return SPH_E_INVAL;
    sph_ctx* c = (sph_ctx*)calloc(1, sizeof(sph_ctx));
    if (!c) return SPH_E_NOMEM;
    c->cfg = *cfg;
    grid_setup(cfg, &c->grid);
    c->capacity = capacity;
    c->stream = (hipStream_t)stream;
    const int lk = cfg->list_k > 0 ? cfg->list_k : NL_K;
    size_t need = carve(&c->w, nullptr, c->grid, capacity, cfg->lean, lk, csr_k_of(cfg));
    if (!workspace || workspace_bytes < need || ((uintptr_t)workspace & 255)) {
        free(c);
        return SPH_E_NOMEM;
    }
    carve(&c->w, (char*)workspace, c->grid, capacity, cfg->lean, lk, csr_k_of(cfg));
    void* mb = nullptr;
    if (hipHostMalloc(&mb, MBOX_WORDS * sizeof(uint32_t), hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostGetDevicePointer((void**)&c->mbox_dev, mb, 0) != hipSuccess) {
        if (mb) hipHostFree(mb);
        free(c);
        return SPH_E_DEVICE;
    }
    c->mbox = (uint32_t*)mb;
    memset(mb, 0, MBOX_WORDS * sizeof(uint32_t));
    c->prof[SPH_PROF_PASS_A].name = "pass_a";
    c->prof[SPH_PROF_PASS_B].name = "pass_b";
    c->prof[SPH_PROF_BUILD].name = "build";
    c->prof[SPH_PROF_LIST].name = "list";
    c->skin = cfg->list_skin;
    c->list_valid = 0;
    c->sched = default_schedule();
    hipLaunchKernelGGL(k_init_counters, dim3(1), dim3(64), 0, c->stream, c->w.status, c->w.ctr);
    if (hipGetLastError() != hipSuccess) {
        hipHostFree(c->mbox);
        free(c);
        return SPH_E_DEVICE;
    }
    *out = c;
    return SPH_OK;
}

static void prof_free(sph_ctx* c)
{
    if (!c->prof_on) return;
    for (int s = 0; s < 4; ++s)
        for (int k = 0; k < 512; ++k) {
            hipEventDestroy(c->prof[s].ev[0][k]);
            hipEventDestroy(c->prof[s].ev[1][k]);
        }
    c->prof_on = 0;
}

extern "C" void sph_destroy(sph_ctx* c)
{
    if (!c) return;
    prof_free(c);
    hipHostFree(c->mbox);
    free(c);
}

// message of the last failed sph_rates_noalloc call of this thread
static thread_local char t_noalloc_err[512] = "no context";

extern "C" const char* sph_last_error(const sph_ctx* c) { return c ? c->err : t_noalloc_err; }

extern "C" int sph_set_stream(sph_ctx* c, void* stream)
{
    if (!c) return SPH_E_INVAL;
    c->stream = (hipStream_t)stream;
    return SPH_OK;
}

static bool check_bg(sph_ctx* c, const sph_background* bg);
static bool check_solids(sph_ctx* c, const sph_particles* s);

static int check_ps(sph_ctx* c, const sph_particles* ps, int need_state)
{
    if (!ps) { set_err(c, "particles is NULL"); return 0; }
    if (ps->n < 0 || ps->n > ps->capacity || ps->capacity > c->capacity) {
        set_err(c, "n=%lld capacity=%lld context capacity=%lld", (long long)ps->n,
                (long long)ps->capacity, (long long)c->capacity);
        return 0;
    }
    if (!ps->x || !ps->y || !ps->h) { set_err(c, "x, y, h must be set"); return 0; }
    if (need_state && (!ps->u || !ps->v || !ps->p || !ps->mq)) {
        set_err(c, "u, v, p, mq must be set");
        return 0;
    }
    return 1;
}

extern "C" int sph_build_neighbors(sph_ctx* c, const sph_particles* ps, sph_csr* out)
{
    if (!c) return SPH_E_INVAL;
    if (!check_ps(c, ps, 0)) return SPH_E_INVAL;
    c->fused_x = nullptr;
    int rc = nbr_build(c, (int)ps->n, ps->x, ps->y, ps->h);
    if (rc || !out) return rc;
    if (!out->row_ptr || (!out->col && out->nnz_cap > 0)) {
        set_err(c, "csr arrays not set");
        return SPH_E_INVAL;
    }
    return nbr_export_csr(c, (int)ps->n, out->row_ptr, out->col, out->nnz_cap, &out->nnz);
}

extern "C" int sph_rates(sph_ctx* c, const sph_particles* ps, double dt, sph_rates_out* out)
{
    if (!c || !out) return SPH_E_INVAL;
    if (!check_ps(c, ps, 1)) return SPH_E_INVAL;
    if (!(dt > 0)) { set_err(c, "dt must be > 0"); return SPH_E_INVAL; }
    if (ps->kind && !ps->rho) { set_err(c, "boundary particles need rho"); return SPH_E_INVAL; }
    c->fused_x = nullptr;  // positions may have changed since the last call
    return rates_eval(c, (int)ps->n, ps, dt, out);
}

extern "C" int sph_set_iteration(sph_ctx* c, int64_t it)
{
    if (!c || it < 0) return SPH_E_INVAL;
    c->iter = it;
    return SPH_OK;
}

extern "C" int64_t sph_iteration(const sph_ctx* c) { return c ? c->iter : -1; }

extern "C" int sph_step(sph_ctx* c, sph_particles* ps, sph_background* bg, const sph_particles* solids,
                        const sph_inout_params* io, int32_t nsteps, sph_diag* diag)
{
    if (!c) return SPH_E_INVAL;
    if (!check_ps(c, ps, 1) || !ps->rho) return SPH_E_INVAL;
    if (nsteps < 0) { set_err(c, "nsteps >= 0"); return SPH_E_INVAL; }
    if ((bg || io) && c->cfg.lean) {
        set_err(c, "the schedule with a background or inlet/outlet zones needs the adaptation buffers");
        return SPH_E_INVAL;
    }
    if (bg && (!check_bg(c, bg) || !ps->mref)) {
        set_err(c, "adaptation needs mref and a background within the context capacity");
        return SPH_E_INVAL;
    }
    if (bg && c->cfg.n_bg > 0 && !solids) {
        set_err(c, "a background update every n_bg iterations needs the solids");
        return SPH_E_INVAL;
    }
    if (bg && c->cfg.n_bg > 0 && !check_solids(c, solids)) return SPH_E_INVAL;
    if (io) {
        if (!ps->kind || !ps->mref) { set_err(c, "inlet/outlet zones need kind and mref"); return SPH_E_INVAL; }
        if (!isfinite(io->x_in) || !isfinite(io->x_out) || !(io->len_in >= 0) || !(io->len_out >= 0) ||
            !isfinite(io->len_in) || !isfinite(io->len_out)) {
            set_err(c, "inout zones must be finite with non-negative lengths");
            return SPH_E_INVAL;
        }
    }
    if (!(c->cfg.dt > 0) && !(timestep_of(c->cfg, 0.0) > 0)) {
        set_err(c, "no time step: set dt, or h_lo, u_ref + c_s > 0");
        return SPH_E_INVAL;
    }
    c->fused_x = nullptr;  // positions may have changed since the last call
    return schedule_run(c, ps, bg, solids, io, nsteps, diag);
}

extern "C" int sph_pec(sph_ctx* c, sph_particles* ps, double dt, int32_t nsteps)
{
    if (!c) return SPH_E_INVAL;
    if (!check_ps(c, ps, 1) || !ps->rho) return SPH_E_INVAL;
    if (!(dt > 0) || nsteps < 0) { set_err(c, "dt must be > 0, nsteps >= 0"); return SPH_E_INVAL; }
    c->fused_x = nullptr;  // positions may have changed since the last call
    return step_run(c, ps, dt, nsteps);
}

extern "C" int sph_body_force(sph_ctx* c, sph_particles* ps, double* force)
{
    if (!c || !force) return SPH_E_INVAL;
    if (!check_ps(c, ps, 1) || !ps->rho || !ps->kind) {
        set_err(c, "body force needs kind and rho (the stored density)");
        return SPH_E_INVAL;
    }
    c->fused_x = nullptr;  // positions may have changed since the last call
    return body_force_run(c, ps, force);
}

extern "C" int sph_move_solids(sph_ctx* c, sph_particles* ps, const double disp[2],
                               const double vel[2], const double acc[2])
{
    if (!c || !disp || !vel || !acc) return SPH_E_INVAL;
    if (!check_ps(c, ps, 1) || !ps->kind) {
        set_err(c, "moving the solids needs kind");
        return SPH_E_INVAL;
    }
    for (int a = 0; a < 2; ++a)
        if (!isfinite(disp[a]) || !isfinite(vel[a]) || !isfinite(acc[a])) {
            set_err(c, "non-finite body motion");
            return SPH_E_INVAL;
        }
    c->cfg.wall_accel[0] = acc[0];
    c->cfg.wall_accel[1] = acc[1];
    c->fused_x = nullptr;
    return move_solids_run(c, ps, disp, vel);
}

// ---------------------------------------------------------------------------
// Checkpoint / resume (host buffer; layout in the header)
// ---------------------------------------------------------------------------

static const char CKPT_MAGIC[8] = {'S', 'P', 'H', 'C', 'K', 'P', 'T', '1'};
static const size_t CKPT_HEAD = 64;
static const int CKPT_NF64 = 8;  // x y u v p rho h mref

extern "C" size_t sph_export_bytes(int64_t n)
{
    if (n < 0) return 0;
    return CKPT_HEAD + (size_t)n * (8 * CKPT_NF64 + 8 + 4);
}

extern "C" int sph_export(sph_ctx* c, const sph_particles* ps, int64_t step, double time,
                          void* host_buf, size_t bytes)
{
    if (!c || !host_buf) return SPH_E_INVAL;
    if (!check_ps(c, ps, 1) || !ps->rho) {
        set_err(c, "export needs x, y, u, v, p, rho, h and mq");
        return SPH_E_INVAL;
    }
    const int64_t n = ps->n;
    if (bytes < sph_export_bytes(n)) {
        set_err(c, "checkpoint buffer of %zu bytes, %zu needed", bytes, sph_export_bytes(n));
        return SPH_E_INVAL;
    }
    unsigned char* b = (unsigned char*)host_buf;
    memset(b, 0, CKPT_HEAD);
    memcpy(b, CKPT_MAGIC, 8);
    const int32_t ver = 1;
    memcpy(b + 8, &ver, 4);
    memcpy(b + 16, &n, 8);
    memcpy(b + 24, &c->cfg.mass_q, 8);
    memcpy(b + 32, &step, 8);
    memcpy(b + 40, &time, 8);
    const double* f[CKPT_NF64] = {ps->x, ps->y, ps->u, ps->v, ps->p, ps->rho, ps->h, ps->mref};
    unsigned char* o = b + CKPT_HEAD;
    const size_t s8 = 8 * (size_t)n, s4 = 4 * (size_t)n;
    for (int k = 0; k < CKPT_NF64; ++k, o += s8) {
        if (n == 0) continue;
        if (f[k]) HIPCHK(c, hipMemcpyAsync(o, f[k], s8, hipMemcpyDeviceToHost, c->stream));
        else memset(o, 0, s8);
    }
    if (n > 0) HIPCHK(c, hipMemcpyAsync(o, ps->mq, s8, hipMemcpyDeviceToHost, c->stream));
    o += s8;
    if (n > 0) {
        if (ps->kind) HIPCHK(c, hipMemcpyAsync(o, ps->kind, s4, hipMemcpyDeviceToHost, c->stream));
        else memset(o, 0, s4);
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SPH_OK;
}

extern "C" int sph_import(sph_ctx* c, sph_particles* ps, const void* host_buf, size_t bytes,
                          int64_t* step, double* time)
{
    if (!c || !host_buf || !ps) return SPH_E_INVAL;
    const unsigned char* b = (const unsigned char*)host_buf;
    int32_t ver = 0;
    int64_t n = -1;
    double q = 0.0;
    if (bytes >= CKPT_HEAD) {
        memcpy(&ver, b + 8, 4);
        memcpy(&n, b + 16, 8);
        memcpy(&q, b + 24, 8);
    }
    if (bytes < CKPT_HEAD || memcmp(b, CKPT_MAGIC, 8) != 0 || ver != 1 || n < 0 ||
        bytes < sph_export_bytes(n)) {
        set_err(c, "not a checkpoint of this format, or truncated");
        return SPH_E_INVAL;
    }
    if (memcmp(&q, &c->cfg.mass_q, 8) != 0) {
        set_err(c, "checkpoint mass quantum %.17g differs from the context's %.17g", q,
                c->cfg.mass_q);
        return SPH_E_INVAL;
    }
    if (!ps->x || !ps->y || !ps->u || !ps->v || !ps->p || !ps->rho || !ps->h || !ps->mq ||
        ps->capacity > c->capacity || ps->capacity < 0) {
        set_err(c, "import needs x, y, u, v, p, rho, h and mq within the context capacity");
        return SPH_E_INVAL;
    }
    if (n > ps->capacity) {
        set_err(c, "checkpoint of %lld particles, capacity %lld", (long long)n,
                (long long)ps->capacity);
        return SPH_E_CAPACITY;
    }
    const unsigned char* in = b + CKPT_HEAD;
    const size_t s8 = 8 * (size_t)n, s4 = 4 * (size_t)n;
    for (int k = 0; k < CKPT_NF64; ++k)
        for (int64_t i = 0; i < n; ++i) {
            double v;
            memcpy(&v, in + k * s8 + 8 * (size_t)i, 8);
            if (!isfinite(v)) {
                set_err(c, "checkpoint holds a non-finite value (array %d, particle %lld)", k,
                        (long long)i);
                return SPH_E_NONFINITE;
            }
        }
    const unsigned char* kin = in + CKPT_NF64 * s8 + s8;
    if (!ps->kind)
        for (int64_t i = 0; i < n; ++i) {
            int32_t kd;
            memcpy(&kd, kin + 4 * (size_t)i, 4);
            if (kd != SPH_FLUID) {
                set_err(c, "checkpoint has non-fluid kinds and the particles have no kind array");
                return SPH_E_INVAL;
            }
        }
    double* f[CKPT_NF64] = {ps->x, ps->y, ps->u, ps->v, ps->p, ps->rho, ps->h, ps->mref};
    if (n > 0) {
        for (int k = 0; k < CKPT_NF64; ++k)
            if (f[k]) HIPCHK(c, hipMemcpyAsync(f[k], in + k * s8, s8, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(ps->mq, in + CKPT_NF64 * s8, s8, hipMemcpyHostToDevice, c->stream));
        if (ps->kind) HIPCHK(c, hipMemcpyAsync(ps->kind, kin, s4, hipMemcpyHostToDevice, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    ps->n = n;
    if (step) memcpy(step, b + 32, 8);
    if (time) memcpy(time, b + 40, 8);
    memcpy(&c->iter, b + 32, 8);
    if (c->iter < 0) c->iter = 0;
    c->list_valid = 0;  // a new state: no reusable list
    c->fused_x = nullptr;
    return SPH_OK;
}

extern "C" int sph_diagnostics(sph_ctx* c, const sph_particles* ps, sph_diag* out)
{
    if (!c || !out) return SPH_E_INVAL;
    if (!check_ps(c, ps, 1) || !ps->rho) return SPH_E_INVAL;
    c->fused_x = nullptr;  // positions may have changed since the last call
    return diag_run(c, ps, out);
}

// The background shares the context's search workspace: it must fit it.
// solid particles handed to a background update: only x, y, h are read, and
// the update builds their cells in this context
static bool check_solids(sph_ctx* c, const sph_particles* s)
{
    if (s->n < 0 || s->n > c->capacity) {
        set_err(c, "solids n=%lld beyond the context capacity %lld", (long long)s->n,
                (long long)c->capacity);
        return false;
    }
    if (s->n > 0 && (!s->x || !s->y || !s->h)) {
        set_err(c, "solids x, y, h must be set");
        return false;
    }
    return true;
}

static bool check_bg(sph_ctx* c, const sph_background* bg)
{
    if (bg->n < 0 || bg->n > bg->capacity || bg->capacity > c->capacity) {
        set_err(c, "background n=%lld capacity=%lld context capacity=%lld", (long long)bg->n,
                (long long)bg->capacity, (long long)c->capacity);
        return false;
    }
    if (bg->n > 0 && (!bg->x || !bg->y || !bg->h || !bg->mref)) {
        set_err(c, "background arrays not set");
        return false;
    }
    return true;
}

extern "C" int sph_mref_lookup(sph_ctx* c, const sph_particles* ps, const sph_background* bg)
{
    if (c && c->cfg.lean) {
        set_err(c, "this context was created lean (no adaptation buffers)");
        return SPH_E_INVAL;
    }
    if (!c || !bg) return SPH_E_INVAL;
    if (!check_ps(c, ps, 0) || !ps->mref || !check_bg(c, bg)) return SPH_E_INVAL;
    c->fused_x = nullptr;  // positions may have changed since the last call
    return mref_lookup_run(c, ps, bg);
}

extern "C" int sph_adapt(sph_ctx* c, sph_particles* ps, const sph_background* bg, sph_adapt_map* map)
{
    if (c && c->cfg.lean) {
        set_err(c, "this context was created lean (no adaptation buffers)");
        return SPH_E_INVAL;
    }
    if (!c || !map) return SPH_E_INVAL;
    if (!check_ps(c, ps, 1) || !ps->rho || !ps->mref) return SPH_E_INVAL;
    if (bg && !check_bg(c, bg)) return SPH_E_INVAL;
    c->fused_x = nullptr;  // positions may have changed since the last call
    return adapt_run(c, ps, bg, map);
}

extern "C" int sph_step_inout(sph_ctx* c, sph_particles* ps, double dt, int32_t nsteps,
                              const sph_inout_params* io, sph_inout_map* map)
{
    if (c && c->cfg.lean) {
        set_err(c, "this context was created lean (no adaptation buffers)");
        return SPH_E_INVAL;
    }
    if (!c || !io || !map) return SPH_E_INVAL;
    if (!check_ps(c, ps, 1) || !ps->rho || !ps->mref || !ps->kind) {
        set_err(c, "step_inout needs the full state including rho, mref and kind");
        return SPH_E_INVAL;
    }
    if (!(dt > 0) || nsteps < 0) { set_err(c, "dt must be > 0, nsteps >= 0"); return SPH_E_INVAL; }
    if (!map->origin) { set_err(c, "inout map origin not set"); return SPH_E_INVAL; }
    if (!isfinite(io->x_in) || !isfinite(io->x_out) || !(io->len_in >= 0) || !(io->len_out >= 0) ||
        !isfinite(io->len_in) || !isfinite(io->len_out)) {
        set_err(c, "inout zones must be finite with non-negative lengths");
        return SPH_E_INVAL;
    }
    c->fused_x = nullptr;  // positions may have changed since the last call
    return step_inout_run(c, ps, dt, nsteps, io, map);
}

extern "C" int sph_vorticity(sph_ctx* c, const sph_particles* ps, double* omega)
{
    if (!c || !omega) return SPH_E_INVAL;
    if (!check_ps(c, ps, 1) || !ps->rho) return SPH_E_INVAL;
    c->fused_x = nullptr;  // positions may have changed since the last call
    return vorticity_run(c, ps, omega);
}

extern "C" int sph_bg_update_solution(sph_ctx* c, sph_background* bg, const sph_particles* solids,
                                      const sph_particles* fluid, double k_frac, int32_t passes,
                                      int64_t* nsplit, double* omega_max)
{
    if (c && c->cfg.lean) {
        set_err(c, "this context was created lean (no adaptation buffers)");
        return SPH_E_INVAL;
    }
    if (!c || !bg || !solids || !fluid || !nsplit || passes < 0) return SPH_E_INVAL;
    if (!(k_frac >= 0.0) || !isfinite(k_frac)) { set_err(c, "k_frac must be finite and >= 0"); return SPH_E_INVAL; }
    if (!check_bg(c, bg) || !check_solids(c, solids) || !check_ps(c, fluid, 1) || !fluid->rho)
        return SPH_E_INVAL;
    c->fused_x = nullptr;  // positions may have changed since the last call
    return bg_solution_run(c, bg, solids, fluid, k_frac, passes, nsplit, omega_max);
}

extern "C" int sph_inout(sph_ctx* c, sph_particles* ps, const sph_inout_params* io, sph_inout_map* map)
{
    if (c && c->cfg.lean) {
        set_err(c, "this context was created lean (no adaptation buffers)");
        return SPH_E_INVAL;
    }
    if (!c || !io || !map) return SPH_E_INVAL;
    if (!check_ps(c, ps, 1) || !ps->rho || !ps->mref || !ps->kind) {
        set_err(c, "inout needs the full state including rho, mref and kind");
        return SPH_E_INVAL;
    }
    if (!map->origin) { set_err(c, "inout map origin not set"); return SPH_E_INVAL; }
    if (!isfinite(io->x_in) || !isfinite(io->x_out) || !(io->len_in >= 0) || !(io->len_out >= 0) ||
        !isfinite(io->len_in) || !isfinite(io->len_out)) {
        set_err(c, "inout zones must be finite with non-negative lengths");
        return SPH_E_INVAL;
    }
    c->fused_x = nullptr;  // positions may have changed since the last call
    return inout_run(c, ps, io, map);
}

extern "C" int sph_bg_update(sph_ctx* c, sph_background* bg, const sph_particles* solids,
                             const double* phi, double phi_thresh, int32_t passes, int64_t* nsplit)
{
    if (c && c->cfg.lean) {
        set_err(c, "this context was created lean (no adaptation buffers)");
        return SPH_E_INVAL;
    }
    if (!c || !bg || !solids || !nsplit || passes < 0) return SPH_E_INVAL;
    if (!check_bg(c, bg) || !check_solids(c, solids)) return SPH_E_INVAL;
    c->fused_x = nullptr;  // positions may have changed since the last call
    return bg_update_run(c, bg, solids, phi, phi_thresh, passes, nsplit);
}

// ---- profiling -------------------------------------------------------------

// Adds the brackets [0, upto) to the totals (void ones excepted) and moves
// the rest to the front.
static void prof_flush_to(sph_ctx* c, int slot, int upto)
{
    ProfSlot& s = c->prof[slot];
    if (upto <= 0) return;
    hipEventSynchronize(s.ev[1][upto - 1]);
    for (int k = 0; k < upto; ++k) {
        if (s.seq[k] == -2) continue;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, s.ev[0][k], s.ev[1][k]) == hipSuccess) s.ms += ms;
        s.launches++;
    }
    for (int k = upto; k < s.count; ++k) {
        const int d = k - upto;
        for (int e = 0; e < 2; ++e) {
            hipEvent_t t = s.ev[e][d];
            s.ev[e][d] = s.ev[e][k];
            s.ev[e][k] = t;
        }
        s.seq[d] = s.seq[k];
    }
    s.count -= upto;
    if (s.run_lo >= 0) s.run_lo = s.run_lo > upto ? s.run_lo - upto : 0;
}

static void prof_flush(sph_ctx* c, int slot) { prof_flush_to(c, slot, c->prof[slot].count); }

// Every prof_every-th launch of a selected kernel is bracketed (the event
// markers keep consecutive kernels from overlapping, so sparse sampling
// disturbs the timed work less).  A launch in a guarded run records its
// sequence number: if the run trips before it, the kernel returns at once
// and the bracket is dropped when the run ends.
void prof_begin(sph_ctx* c, int slot, const Guard* gd)
{
    if (!c->prof_on || !(c->prof_mask & (1 << slot))) return;
    ProfSlot& s = c->prof[slot];
    s.skip = (s.tick++ % (uint32_t)c->prof_every) != 0;
    if (s.skip) return;
    if (s.count == 512) {
        // keep the brackets of the run in flight unless they fill the buffer
        prof_flush_to(c, slot, s.run_lo > 0 ? s.run_lo : s.count);
        if (s.count == 512) prof_flush(c, slot);
    }
    s.seq[s.count] = (gd && gd->trip) ? gd->seq : -1;
    hipEventRecord(s.ev[0][s.count], c->stream);
}

void prof_run_begin(sph_ctx* c)
{
    if (!c->prof_on) return;
    for (int k = 0; k < 4; ++k) c->prof[k].run_lo = c->prof[k].count;
}

void prof_run_end(sph_ctx* c, int32_t tr)
{
    if (!c->prof_on) return;
    for (int k = 0; k < 4; ++k) {
        ProfSlot& s = c->prof[k];
        if (s.run_lo < 0) continue;
        for (int i = s.run_lo; i < s.count; ++i)
            if (s.seq[i] >= 0 && s.seq[i] > tr) s.seq[i] = -2;
        s.run_lo = -1;
    }
}

void prof_end(sph_ctx* c, int slot)
{
    if (!c->prof_on || !(c->prof_mask & (1 << slot))) return;
    ProfSlot& s = c->prof[slot];
    if (s.skip) return;
    hipEventRecord(s.ev[1][s.count], c->stream);
    s.count++;
}

extern "C" int sph_profile_enable(sph_ctx* c, int32_t on)
{
    if (!c) return SPH_E_INVAL;
    c->prof_mask = on & 15;
    c->prof_every = (on >> 8) & 255;
    if (c->prof_every < 1) c->prof_every = 1;
    for (int s = 0; s < 4; ++s) c->prof[s].tick = 0;
    if (on && !c->prof_on) {
        for (int s = 0; s < 4; ++s) {
            for (int k = 0; k < 512; ++k) {
                HIPCHK(c, hipEventCreate(&c->prof[s].ev[0][k]));
                HIPCHK(c, hipEventCreate(&c->prof[s].ev[1][k]));
            }
            c->prof[s].count = 0;
            c->prof[s].ms = 0;
            c->prof[s].launches = 0;
            c->prof[s].run_lo = -1;
        }
        c->prof_on = 1;
    } else if (!on) {
        for (int s = 0; s < 4; ++s) prof_flush(c, s);
        prof_free(c);
    }
    return SPH_OK;
}

extern "C" int sph_profile_reset(sph_ctx* c)
{
    if (!c) return SPH_E_INVAL;
    if (!c->prof_on) return SPH_OK;
    for (int s = 0; s < 4; ++s) {
        prof_flush(c, s);
        c->prof[s].ms = 0;
        c->prof[s].launches = 0;
    }
    return SPH_OK;
}

extern "C" int sph_profile_read(sph_ctx* c, const char* kernel, double* ms, int64_t* launches)
{
    if (!c || !kernel || !ms || !launches) return SPH_E_INVAL;
    for (int s = 0; s < 4; ++s) {
        if (strcmp(c->prof[s].name, kernel) == 0) {
            if (c->prof_on) prof_flush(c, s);
            *ms = c->prof[s].ms;
            *launches = c->prof[s].launches;
            return SPH_OK;
        }
    }
    set_err(c, "unknown kernel name %s", kernel);
    return SPH_E_INVAL;
}

// ---------------------------------------------------------------------------
// Rate evaluation without allocation.  The scratch memory is a file-scope
// device array: every GPU the library runs on holds its own copy (at its own
// address) from the moment the library's code is loaded on it until the
// process ends.  On host, `scratch` names only a host-side stand-in, so host
// code never passes it to a kernel: the device address is looked up once
// per device with hipGetSymbolAddress and kept in g_scratch.
// ---------------------------------------------------------------------------

#define SPH_NOALLOC_MAX_DEV 64

static __device__ __align__(256) unsigned char scratch[SPH_NOALLOC_SCRATCH_BYTES];
static void* g_scratch[SPH_NOALLOC_MAX_DEV];
static std::mutex g_scratch_mu;

static int noalloc_err(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(t_noalloc_err, sizeof(t_noalloc_err), fmt, ap);
    va_end(ap);
    return code;
}

// Device address of this device's scratch array (looked up on first use).
static int scratch_address(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return noalloc_err(SPH_E_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= SPH_NOALLOC_MAX_DEV)
        return noalloc_err(SPH_E_DEVICE, "device %d beyond the supported %d", dev, SPH_NOALLOC_MAX_DEV);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return noalloc_err(SPH_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                               hipGetErrorString(e));
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return SPH_OK;
}

extern "C" size_t sph_rates_noalloc_bytes(const sph_config* cfg, int64_t n)
{
    if (!check_cfg(cfg) || n < 0) return 0;
    sph_config lc = *cfg;
    lc.lean = 1;
    lc.list_skin = 0.0;
    Grid g;
    grid_setup(&lc, &g);
    Work w;
    return carve(&w, nullptr, g, n, 1, lc.list_k > 0 ? lc.list_k : NL_K);
}

extern "C" int sph_rates_noalloc(const sph_config* cfg, const sph_particles* ps, double dt,
                                 sph_rates_out* out, void* stream)
{
    if (!cfg || !ps || !out) return noalloc_err(SPH_E_INVAL, "NULL argument");
    sph_config lc = *cfg;
    lc.lean = 1;        // no adaptation buffers
    lc.list_skin = 0.0; // the list is built afresh: no host round trip
    if (!check_cfg(&lc)) return noalloc_err(SPH_E_INVAL, "invalid configuration");
    if (!(dt > 0)) return noalloc_err(SPH_E_INVAL, "dt must be > 0");
    const int64_t n = ps->n;
    if (n < 0 || n > ps->capacity || n > (int64_t)INT32_MAX - 1)
        return noalloc_err(SPH_E_INVAL, "n=%lld capacity=%lld", (long long)n, (long long)ps->capacity);
    if (!ps->x || !ps->y || !ps->h || !ps->u || !ps->v || !ps->p || !ps->mq)
        return noalloc_err(SPH_E_INVAL, "x, y, u, v, p, h, mq must be set");
    if (ps->kind && !ps->rho) return noalloc_err(SPH_E_INVAL, "boundary particles need rho");
    const int lk = lc.list_k > 0 ? lc.list_k : NL_K;
    // static: the context is host bookkeeping only, and large (profiling
    // slots); one per thread, reused
    static thread_local sph_ctx c;
    memset(&c, 0, sizeof(c));
    c.cfg = lc;
    grid_setup(&lc, &c.grid);
    const size_t need = carve(&c.w, nullptr, c.grid, n, 1, lk);
    if (need > SPH_NOALLOC_SCRATCH_BYTES)
        return noalloc_err(SPH_E_NOMEM,
                           "%lld particles need %zu bytes of scratch; the static scratch holds %zu",
                           (long long)n, need, (size_t)SPH_NOALLOC_SCRATCH_BYTES);
    void* base = nullptr;
    int rc = scratch_address(&base);
    if (rc) return rc;
    carve(&c.w, (char*)base, c.grid, n, 1, lk);
    c.capacity = n > 0 ? n : 1;
    c.stream = (hipStream_t)stream;
    c.skin = 0.0;
    c.sched = default_schedule();
    c.mbox = nullptr;  // no readback happens on this path
    // the array keeps the last call's contents: clear the counters
    hipLaunchKernelGGL(k_init_counters, dim3(1), dim3(64), 0, c.stream, c.w.status, c.w.ctr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return noalloc_err(SPH_E_DEVICE, "init: %s", hipGetErrorString(e));
    rc = rates_eval(&c, (int)n, ps, dt, out);
    if (rc) return noalloc_err(rc, "%s", c.err);
    return SPH_OK;
}
