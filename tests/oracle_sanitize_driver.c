/* Host memory and undefined-behaviour checks of the oracle.  The test that
 * runs this program builds it, together with the oracle source, with
 * AddressSanitizer and UndefinedBehaviorSanitizer (host code only; no GPU
 * code is involved) and runs every oracle entry point on small seeded
 * inputs: neighbours (cell list against brute force), rates, PEC steps,
 * adaptation, the background update, m_ref lookup, vorticity and the
 * Shepard average, the boundary pass with walls and characteristic
 * inlet/outlet, the body force, body motion and the inlet/outlet update.
 * Exit status 0 when every call succeeds and every check holds. */
#include "../oracle/sph_oracle.c"

static uint64_t rs = 88172645463325252ull;
static double urand(void)
{
    rs ^= rs << 13;
    rs ^= rs >> 7;
    rs ^= rs << 17;
    return (double)(rs >> 11) * (1.0 / 9007199254740992.0);
}

#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__);   \
            return 1;                                                         \
        }                                                                     \
    } while (0)

static double* dalloc(int64_t n) { return (double*)calloc((size_t)n, sizeof(double)); }

int main(void)
{
    const double q = ldexp(1.0, -40);
    or_params P = {.rho0 = 1.0, .cs = 10.0, .nu = 0.01, .alpha_e = 1.5, .hdx = 1.0,
                   .fx = 0.0, .fy = 0.0, .split_alpha = 0.9, .split_eps = 0.4,
                   .mmax_f = 1.05, .mmin_f = 0.5, .mass_q = q, .merge_iters = 3,
                   .shift_iters = 3, .pref_mode = 1};
    or_domain d = {{0.0, 0.0}, {1.0, 1.0}, {1, 1}};

    /* a jittered periodic lattice */
    const int side = 20;
    const int64_t n = side * side, cap = 8 * n;
    double *x = dalloc(cap), *y = dalloc(cap), *u = dalloc(cap), *v = dalloc(cap);
    double *p = dalloc(cap), *h = dalloc(cap), *m = dalloc(cap), *rho = dalloc(cap);
    double *mref = dalloc(cap);
    int64_t* mq = (int64_t*)calloc((size_t)cap, sizeof(int64_t));
    int32_t* kind = (int32_t*)calloc((size_t)cap, sizeof(int32_t));
    const double dx = 1.0 / side;
    for (int i = 0; i < side; ++i)
        for (int j = 0; j < side; ++j) {
            const int64_t k = (int64_t)i * side + j;
            x[k] = (i + 0.5 + 0.1 * (urand() - 0.5)) * dx;
            y[k] = (j + 0.5 + 0.1 * (urand() - 0.5)) * dx;
            u[k] = sin(2 * M_PI * y[k]);
            v[k] = cos(2 * M_PI * x[k]);
            p[k] = 0.1 * (urand() - 0.5);
            h[k] = dx * (1.0 + 0.5 * urand());
            mq[k] = (int64_t)llround(dx * dx / q);
            m[k] = (double)mq[k] * q;
            rho[k] = 1.0;
        }

    /* neighbours: cell list against brute force */
    int64_t* rp = NULL;
    int32_t* col = NULL;
    const int64_t nnz = or_nbr_cells_alloc(&d, n, x, y, h, &rp, &col);
    CHECK(nnz > n);
    int64_t* rp2 = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t* col2 = (int32_t*)calloc((size_t)nnz, sizeof(int32_t));
    CHECK(or_nbr_brute(&d, n, x, y, h, rp2, col2, nnz) == nnz);
    CHECK(memcmp(rp, rp2, sizeof(int64_t) * (size_t)(n + 1)) == 0);
    CHECK(memcmp(col, col2, sizeof(int32_t) * (size_t)nnz) == 0);

    /* rates, vorticity, PEC steps */
    double* o[9];
    for (int k = 0; k < 9; ++k) o[k] = dalloc(n);
    CHECK(or_rates(&d, &P, n, x, y, u, v, p, h, m, 1e-4, o[0], o[1], o[2], o[3], o[4], o[5],
                   o[6], o[7], o[8]) == 0);
    double* om = dalloc(n);
    or_vorticity(&d, n, x, y, u, v, h, m, rho, rp, col, om);
    or_free(rp);
    or_free(col);
    CHECK(or_step(&d, &P, n, x, y, u, v, p, h, m, 1e-4, 3, rho) == 0);

    /* background: a coarse lattice refined around a few solid points */
    or_bgparams B = {.rho0 = 1.0, .cr = 1.2, .ds_min = 0.05, .ds_max = 0.2, .n_r = 48.0,
                     .split_alpha = 0.9, .split_eps = 0.4, .mmax_f = 1.05, .mass_q = q,
                     .smooth_iters = 3};
    const int bs = 5;
    const int64_t nb = bs * bs, bcap = 4096;
    double *bx = dalloc(bcap), *by = dalloc(bcap), *bh = dalloc(bcap), *bds = dalloc(bcap);
    double* bmref = dalloc(bcap);
    int32_t* bmask = (int32_t*)calloc((size_t)bcap, sizeof(int32_t));
    int64_t* bmq = (int64_t*)calloc((size_t)bcap, sizeof(int64_t));
    for (int i = 0; i < bs; ++i)
        for (int j = 0; j < bs; ++j) {
            const int64_t k = (int64_t)i * bs + j;
            bx[k] = (i + 0.5) * 0.2;
            by[k] = (j + 0.5) * 0.2;
            bh[k] = 1.2 * 0.2;
            bds[k] = 0.2;
            bmref[k] = 0.04;
            bmq[k] = (int64_t)llround(0.04 / q);
        }
    double sx[4] = {0.5, 0.52, 0.5, 0.52}, sy[4] = {0.5, 0.5, 0.52, 0.52};
    double sh[4] = {0.05, 0.05, 0.05, 0.05};
    int64_t nsplit = 0;
    const int64_t nb2 = or_bg_update(&d, &B, nb, bcap, bx, by, bh, bds, bmask, bmq, bmref, 4, sx,
                                     sy, sh, NULL, 0.0, 6, &nsplit);
    CHECK(nb2 > nb && nsplit > 0);
    double* phi = dalloc(nb2);
    CHECK(or_shepard_to_bg(&d, nb2, bx, by, bh, n, x, y, h, kind, om, phi) == 0);

    /* m_ref from the background, then the adaptation (split, merge, shift, h) */
    CHECK(or_mref_lookup(&d, n, x, y, h, nb2, bx, by, bh, bmref, mref) == 0);
    for (int64_t i = 0; i < n; ++i) mref[i] *= (x[i] < 0.5 ? 0.25 : 1.0);
    int64_t* origin = (int64_t*)calloc((size_t)cap, sizeof(int64_t));
    int32_t* sat = (int32_t*)calloc((size_t)cap, sizeof(int32_t));
    int64_t counts[5] = {0};
    int64_t mtot = 0;
    for (int64_t i = 0; i < n; ++i) mtot += mq[i];
    const int64_t na = or_adapt(&d, &P, n, cap, x, y, u, v, p, rho, h, mref, mq, kind, origin,
                                sat, counts);
    CHECK(na > n && counts[0] > 0);
    int64_t mtot2 = 0;
    for (int64_t i = 0; i < na; ++i) mtot2 += mq[i];
    CHECK(mtot2 == mtot);

    /* an open strip: inlet, fluid with a wall row, outlet */
    or_domain ds = {{-0.3, 0.0}, {1.3, 1.0}, {0, 1}};
    const int cols = 14, rows = 10;
    const int64_t ns = (int64_t)cols * rows, scap = 4 * ns;
    double *X = dalloc(scap), *Y = dalloc(scap), *U = dalloc(scap), *V = dalloc(scap);
    double *Pp = dalloc(scap), *H = dalloc(scap), *M = dalloc(scap), *R = dalloc(scap);
    double* MR = dalloc(scap);
    int64_t* MQ = (int64_t*)calloc((size_t)scap, sizeof(int64_t));
    int32_t* K = (int32_t*)calloc((size_t)scap, sizeof(int32_t));
    const double sdx = 0.1;
    for (int i = 0; i < cols; ++i)
        for (int j = 0; j < rows; ++j) {
            const int64_t k = (int64_t)i * rows + j;
            X[k] = -0.2 + (i + 0.5) * sdx;
            Y[k] = (j + 0.5) * sdx;
            U[k] = 1.0;
            Pp[k] = 0.01 * (urand() - 0.5);
            H[k] = 1.2 * sdx;
            MQ[k] = (int64_t)llround(sdx * sdx / q);
            M[k] = (double)MQ[k] * q;
            MR[k] = M[k];
            R[k] = 1.0;
            K[k] = X[k] < 0.0 ? OR_INLET : (X[k] >= 1.0 ? OR_OUTLET : (j == 0 ? OR_SOLID : OR_FLUID));
        }
    or_bc bc = {.awx = 0.0, .awy = 0.0, .io_mode = 1, .ur = 1.0, .vr = 0.0, .pr = 0.0};
    CHECK(or_rates_k(&ds, &P, &bc, ns, X, Y, U, V, Pp, H, M, K, R, 1e-4, o[0], o[1], o[2], o[3],
                     o[4], o[5], o[6], o[7], o[8]) == 0);
    double f[8];
    CHECK(or_body_force(&ds, &P, &bc, ns, X, Y, U, V, Pp, H, M, K, R, f) == 0);
    or_move_solids(&ds, ns, K, 0.0, 0.01, 0.0, 0.1, X, Y, U, V);
    CHECK(or_step_k(&ds, &P, &bc, ns, X, Y, U, V, Pp, H, M, K, R, 2e-3, 5) == 0);
    or_io io = {.x_in = 0.0, .len_in = 0.2, .x_out = 1.0, .len_out = 0.2};
    int64_t* org = (int64_t*)calloc((size_t)scap, sizeof(int64_t));
    int64_t ic[4] = {0};
    CHECK(or_inout(&io, ns, scap, X, Y, U, V, Pp, R, H, MR, MQ, K, org, ic) >= 0);
    printf("oracle sanitize run ok: n=%lld adapted=%lld background=%lld\n", (long long)n,
           (long long)na, (long long)nb2);
    return 0;
}
