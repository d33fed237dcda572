// Internal declarations of the gfx950 SPH library (not part of the C ABI).
//
// Neighbour search layout.  Particles are binned by smoothing-length level:
// level l holds particles with 3 h <= c0 * 2^l (c0 = finest cell width), so
// a pair of particles at levels <= l is closer than one level-l cell when it
// interacts.  All levels share one nested grid: a level-Q cell is a 2^Q x 2^Q
// block of level-0 cells.  Particles are radix-sorted by the key
// (level, Hilbert index of the level-0 cell), so the particles of any
// level inside any cell of any resolution Q form one contiguous run of the
// sorted order (a Hilbert index, like a Morton code, keeps every aligned
// 2^Q x 2^Q block contiguous).  For every level l and every resolution Q >= l a dense table gives
// that run (start, end) per cell.  Particle i visits level l with search
// radius 3 max(h_i, hmax_l) at resolution max(l, l_i): a 3x3 (or smaller)
// block of cells per level, from whichever side of the pair is coarser.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sph.h"

#define SPH_MAXL 16

// Speculatively enqueued runs of steps: every guarded kernel carries the
// sequence number of its place in the run; a kernel that finds a condition
// the host must handle (an expired neighbour list, an inlet/outlet slot
// change) lowers *trip to its own number, and every kernel with a larger
// number returns at once, leaving the state as it was after the tripping
// kernel.  trip == nullptr: not in such a run (always executes).
#define SPH_NOTRIP 0x7fffffff
struct Guard {
    int32_t* trip;
    int32_t seq;
};

struct Grid {
    double org[2];      // origin of the level-0 grid per axis
    double cw0[2];      // level-0 cell width per axis
    double L[2];        // period per axis (periodic axes)
    double half[2];     // L/2
    double lo[2], hi[2];
    double cmin0;       // min(cw0[0], cw0[1])
    double icw0[2];     // 1 / cw0 (cell ranges are conservative, so a
                        // product instead of a quotient is safe)
    double mi_l[2];     // minimum image: period (0 on open axes)
    double mi_h[2];     // minimum image: half period (+inf on open axes)
    int32_t nx0[2];     // level-0 cells per axis
    int32_t periodic[2];
    int32_t nlev;       // number of levels
    int32_t bits;       // key bits per axis
    int32_t nxq[SPH_MAXL][2];   // cells per axis at resolution Q
    int64_t cumq[SPH_MAXL + 1]; // prefix of cells(Q)
    int64_t lbase[SPH_MAXL];    // table offset(l, Q) = lbase[l] + cumq[Q]
    int64_t tab_total;          // int2 entries over all (l, Q >= l)
};

// Device view of a built neighbour structure (all in sorted order).
struct NbrView {
    const double* xs;     // positions and smoothing lengths, sorted order
    const double* ys;
    const double* hs;
    const double4* xyh;   // {x, y, h, -} packed, sorted order (one record per candidate)
    const int32_t* perm;  // sorted position -> slot
    const uint64_t* keys; // sorted keys (level in the high bits)
    const int2* tab;      // cell run tables
    const unsigned long long* hmax_bits; // per-level max h (bit pattern)
    const int32_t* lcount;               // per-level particle count
};

// ---- batched launches over many independent simulations ------------------
// The simulations of a batch hold disjoint particle ranges of one set of
// global arrays (and disjoint ranges of one cell-table array).  Every hot
// kernel is launched once for the whole batch: block b belongs to the
// simulation s with start[s] <= b < start[s + 1] in the block map of its
// launch shape, and reads that simulation's descriptor.
struct SimDesc {
    Grid g;
    int64_t off, n;     // particles [off, off + n) of the batch arrays
    int64_t toff;       // first entry of its cell tables
    int64_t hoff;       // first entry of its radix digit histogram
    int64_t packed;     // sum of n over the simulations before it
    int32_t ntile;      // radix-sort tiles (RS_TILE particles each)
    int32_t slot;       // its pair counter
    double dt, rho0, cs, nu, alpha_e, fx, fy, mass_q;
    double skin;        // list skin (0: a list per evaluation)
    int64_t ntab;       // entries of its cell tables
};
// Block maps: particles per block of each launch shape.
enum { BM_P256 = 0, BM_P64 = 1, BM_P128 = 2, BM_TILE = 3, BM_COUNT = 4 };
struct Batch {
    const SimDesc* sims;    // nsim descriptors
    const int32_t* bstart;  // bstart[map * (nsim + 1) + s]: first block of s
    int32_t nsim;
};

// Workspace carve-out (device pointers).
struct Work {
    uint64_t *keys_a, *keys_b;
    int32_t *vals_a, *vals_b;
    uint32_t* os_look;     // sort look-back words, digit counts, tickets
    int64_t* scan_tmp;     // block sums for scans
    int2* tab;
    unsigned long long* hmax_bits;
    int32_t* lcount;
    int32_t* status;       // [0] overflow rows count, [1] nonfinite flag, ...
    unsigned long long* ctr; // cumulative event counters (never cleared)
    int32_t* long_rows;    // rows needing the long-row sort path
    double *xs, *ys, *hs;  // sorted shadows
    double4* xyh;          // the same, packed
    double *us, *vs;       // sorted velocity (double: differences taken in FP64)
    double *sc0, *sc1, *sc2, *sc3, *sc4, *sc5, *sc6, *sc7, *sc8, *sc9, *sc10, *sc11; // typed scratch
    double *r_dpdt, *r_dudt, *r_dvdt, *r_dxs, *r_dys; // rates in slot order
    double *xh, *yh, *uh, *vh, *ph;                   // half-step state
    int64_t* cnt64;        // per-slot counters (scan input)
    int64_t* rp_tmp;       // internal CSR row pointers
    int32_t* col_tmp;      // internal CSR columns
    int64_t col_cap;
    // adaptation scratch
    int32_t *flag, *closest, *idx_a, *idx_b;
    int64_t *i64_a, *i64_b;
    double *tmp_d[10];
    int32_t *tmp_i32[2];
    int64_t *tmp_i64[3];
    int64_t* red;          // reduction scratch
    int32_t *nl_idx, *nl_cnt; // rate passes' neighbour list (with skin)
    int32_t* cnt_ex;          // row counts of the exact rows pass A writes for pass B
    int32_t nl_k;
    double *xref, *yref, *href; // state the list was built on (slot order)
    double *ug, *vg;            // viscous-term velocity (ghost velocity of walls), slot order
    double *ugs, *vgs;          // the same, sorted order
    // what the rate passes gather per neighbour, packed into 16-byte loads
    // (sorted order): {x, y, h, p}, {u, v}, and {V, B, rho, m} in the pair
    // precision (float4 or double4) written by pass A for pass B
    double4* pa;
    double2* puv;
    void* pf;
    int32_t* list_flag;         // [0]: rebuild needed (moved / h changed / overflow)
    int64_t* sched_origin;      // map storage of the schedule's adaptations and
    int32_t* sched_sat;         // inlet/outlet updates (not in a lean workspace)
    int32_t lean;               // 1: the adaptation buffers below are not carved
    int64_t capacity;
};

struct ProfSlot {
    const char* name;
    hipEvent_t ev[2][512];
    // guard sequence number of each bracketed launch (-1: unguarded; -2:
    // void, a launch of a guarded run after its trip, which returned at once)
    int32_t seq[512];
    int32_t run_lo;     // first bracket of the guarded run in flight, or -1
    int32_t count;
    double ms;
    int64_t launches;   // bracketed launches
    uint32_t tick;      // launches seen (bracketed or not)
    int32_t skip;       // the current launch is not bracketed
};

// schedule variants compiled in (rates.hip, nbr.hip); every context starts
// with the default
bool rate_schedule_valid(const sph_schedule& s);
bool list_lanes_valid(int lanes);
inline sph_schedule default_schedule() { return sph_schedule{4, 5, 2, 2, 4, 4}; }

struct sph_ctx {
    sph_config cfg;
    Grid grid;
    Work w;
    hipStream_t stream;
    int64_t capacity;
    int32_t nsort_blocks_max;
    char err[512];
    int32_t prof_on;
    int32_t prof_mask;  // which slots are bracketed (bit = slot)
    int32_t prof_every; // bracket every prof_every-th launch of a slot
    ProfSlot prof[4];
    int built_n;       // particle count of the last build
    // Neighbour-list reuse: the list holds every pair closer than
    // (1 + skin) 3 max(h_i, h_j) at build time, so it stays a superset of
    // N(i) while every particle has moved less than 1.5 skin h_i; the rate
    // passes re-apply the exact predicate.
    double skin;
    int list_valid;
    int list_n;
    int64_t list_builds, list_reuses;
    // when set, every rate evaluation adds its interacting ordered pairs here
    unsigned long long* pair_acc;
    int bparity;                    // which boundary-list counter the next evaluation uses
    // a list check already done (with the inlet/outlet update of a combined
    // step call) for the next evaluation: valid flag and outcome
    int precheck_valid, precheck_ok;
    // positions on which a fused list check (in the predictor or corrector)
    // has already been launched in this library call, or nullptr
    const double* fused_x;
    unsigned long long io_last[3];  // inlet/outlet event counters at the last update
    // small host readbacks: pinned, device-coherent words written by a
    // one-lane kernel; word 0 carries the sequence number of the last one
    int64_t iter;         // iteration counter of the schedule (sph_step)
    sph_schedule sched;   // launch schedule of the FP32 rate passes and the list build
    uint32_t* mbox;       // host address
    uint32_t* mbox_dev;   // the same memory as the device sees it
    uint32_t mbox_seq;
};

// One value to bring to the host: `bytes` (a multiple of 4) from device
// address src to host address dst.
struct Readback {
    void* dst;
    const void* src;
    int bytes;
};
// Copies up to 4 items (at most 240 bytes in all) once the stream's earlier
// work is complete, and returns then (the stream is idle at that point).
// Not for use while the stream is being captured.
int readback(sph_ctx* c, const Readback* items, int n);

// ---- host-side launch wrappers (implemented in the .hip files) ----------

// nbr.hip
int nbr_build(sph_ctx* c, int n, const double* x, const double* y, const double* h);
NbrView nbr_view(sph_ctx* c);
int nbr_build_list(sph_ctx* c, int n, double skin);
// Rows hold every j with |r_i - r_j| < sf 3 max(h_i, h_j) (sf = 1: the
// neighbour set), ascending.
int nbr_export_csr(sph_ctx* c, int n, int64_t* row_ptr, int32_t* col, int64_t cap, int64_t* nnz,
                   double sf = 1.0);
int scan_exclusive_i64(sph_ctx* c, const int64_t* in, int64_t* out, int64_t n);
void grid_setup(const sph_config* cfg, Grid* g);

// batched step (nbr.hip, rates.hip): global arrays of a batch
struct BatchBufs {
    double *x, *y, *u, *v, *p, *rho, *h;  // state, slot order
    int64_t* mq;
    uint64_t *keys_a, *keys_b;
    int32_t *vals_a, *vals_b;
    uint32_t *hist, *scan_tmp;
    int2* tab;
    unsigned long long* hmax;             // SPH_MAXL per simulation of a batch
    int32_t* lcount;
    double4 *xyh, *pa;
    double2* puv;
    void* pf;                             // float4 / double4 records
    void *m, *brho, *beta, *dpav, *dxs, *dys, *nnb;  // per particle, 8 bytes each
    int32_t *nl_idx, *nl_cnt, *list_flag;
    int32_t nl_k;
    int64_t stride;                       // particles of the arrays (list stride)
    double *r_dpdt, *r_dudt, *r_dvdt, *r_dxs, *r_dys;
    double *xh, *yh, *uh, *vh, *ph;
    unsigned long long* pairs;            // per counter slot
    double *xref, *yref, *href;           // positions and h each list was built at
};
struct BatchLaunch {
    Batch B;
    int32_t nblk[BM_COUNT];   // blocks of each launch shape
    int64_t hist_n;           // digit-histogram entries of the batch
    int64_t tab_n;            // cell-table entries to clear (the used extent)
    int32_t npass;            // radix passes (the widest key of the batch)
    int32_t precision;
    int32_t* rebuild;         // per simulation of the batch: its structure and
                              // list are rebuilt in this evaluation
};
// One predict-evaluate-correct step of every simulation of the batch.
int batch_step(hipStream_t st, const BatchBufs& b, const BatchLaunch& L);
// the neighbour structure of a batch at positions (x, y, h) and its list
int batch_build(hipStream_t st, const BatchBufs& b, const BatchLaunch& L, const double* x,
                const double* y, const double* h, const uint64_t** keys, const int32_t** perm);
int batch_key_bits(const Grid* g);

// rates.hip
int rates_eval(sph_ctx* c, int n, const sph_particles* ps, double dt, const sph_rates_out* out);
int step_run(sph_ctx* c, sph_particles* ps, double dt, int nsteps);
// the two halves of a PEC step, each an evaluation then the predictor or
// corrector, guarded in a speculatively enqueued run of steps
int step_half1(sph_ctx* c, sph_particles* ps, double dt, Guard gd1, Guard gd2);
int step_half2(sph_ctx* c, sph_particles* ps, double dt, Guard gd3, Guard gd4);
void reset_bcounters(sph_ctx* c);
int list_ready(sph_ctx* c, const sph_particles* ps);
// force on the solid particles (8 doubles to the host, see sph_body_force)
int move_solids_run(sph_ctx* c, sph_particles* ps, const double* disp, const double* vel);
int body_force_run(sph_ctx* c, sph_particles* ps, double* force);
bool launch_list_check(sph_ctx* c, int n, const double* x, const double* y, const double* h);
int diag_run(sph_ctx* c, const sph_particles* ps, sph_diag* out);

// adapt.hip
int adapt_run(sph_ctx* c, sph_particles* ps, const sph_background* bg, sph_adapt_map* map);
int inout_apply(sph_ctx* c, sph_particles* ps, const sph_inout_params* io, sph_inout_map* map,
                int32_t nto);
int inout_run(sph_ctx* c, sph_particles* ps, const sph_inout_params* io, sph_inout_map* map,
              bool precheck = false);
int step_inout_run(sph_ctx* c, sph_particles* ps, double dt, int nsteps, const sph_inout_params* io,
                   sph_inout_map* map);
int vorticity_run(sph_ctx* c, const sph_particles* ps, double* omega);
int bg_solution_run(sph_ctx* c, sph_background* bg, const sph_particles* solids,
                    const sph_particles* fluid, double k_frac, int passes, int64_t* nsplit,
                    double* omega_max);
int mref_lookup_run(sph_ctx* c, const sph_particles* ps, const sph_background* bg);
int bg_update_run(sph_ctx* c, sph_background* bg, const sph_particles* solids, const double* phi,
                  double phi_thresh, int passes, int64_t* nsplit);

// the per-iteration schedule of section 3.4 (sph_step)
int schedule_run(sph_ctx* c, sph_particles* ps, sph_background* bg, const sph_particles* solids,
                 const sph_inout_params* io, int nsteps, sph_diag* diag);

// api.hip
double timestep_of(const sph_config& cfg, double h_min);
void set_err(sph_ctx* c, const char* fmt, ...);
int check_hip(sph_ctx* c, hipError_t e, const char* what);
void prof_begin(sph_ctx* c, int slot, const Guard* gd = nullptr);
// a guarded run starts / ended with trip sequence tr (SPH_NOTRIP: none)
void prof_run_begin(sph_ctx* c);
void prof_run_end(sph_ctx* c, int32_t tr);
void prof_end(sph_ctx* c, int slot);

#define SPH_PROF_PASS_A 0
#define SPH_PROF_PASS_B 1
#define SPH_PROF_BUILD 2
#define SPH_PROF_LIST 3

#define HIPCHK(c, expr)                                         \
    do {                                                        \
        hipError_t e_ = (expr);                                 \
        if (e_ != hipSuccess) return check_hip((c), e_, #expr); \
    } while (0)

#define LAUNCHCHK(c, what)                                             \
    do {                                                               \
        hipError_t e_ = hipGetLastError();                             \
        if (e_ != hipSuccess) return check_hip((c), e_, (what));       \
    } while (0)

// Radix-sort tiles (keys per workgroup) and scan tiles; the workspace carve
// sizes the digit histograms and the scan block sums from them.
#define RS_THREADS 256
#ifndef RS_ITEMS
#define RS_ITEMS 8
#endif
#define RS_TILE (RS_THREADS * RS_ITEMS)
#ifndef RS_BITS
#define RS_BITS 12           // digit width of the LSD radix sort
#endif
#define RS_BINS (1 << RS_BITS)
// One-sweep sort of a context's keys: digit width, keys per tile, look-back
// window, spin bound, look-back word flags and value mask; status word that
// records a look-back wait that ran out.
#define OS_BITS 8
#define OS_BINS (1 << OS_BITS)
#ifndef OS_ITEMS
#define OS_ITEMS 8
#endif
#define OS_TILE (RS_THREADS * OS_ITEMS)
#define OS_MAXPASS 8
#define OS_WIN 16
#define OS_SPIN (1 << 16)
#define OS_AGG (1u << 30)
#define OS_INC (2u << 30)
#define OS_VAL ((1u << 30) - 1u)
#define SPH_STATUS_SORT 8
#define SCAN_T 256
#define SCAN_E 8
#define SCAN_TILE (SCAN_T * SCAN_E)

static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
