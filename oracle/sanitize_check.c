/*
 * Driver that runs every public function of the FP64 oracle on small inputs,
 * for a build with AddressSanitizer and UndefinedBehaviorSanitizer (the CPU
 * test suite compiles and runs it; any out-of-bounds access, use after free,
 * leak or undefined arithmetic aborts with a report). It also checks that the
 * brute-force and binned neighbour searches agree and that every output is
 * finite. TEST INFRASTRUCTURE ONLY, like the oracle it includes.
 */
#include "dtsph_oracle.c"

#include <stdio.h>

static unsigned long long lcg_state = 1904ull;

static double uniform(void) /* in [-1, 1) */
{
    lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg_state >> 11) / 4503599627370496.0 - 1.0;
}

static int fails = 0;

#define CHECK(cond, what)                                                      \
    do {                                                                       \
        if (!(cond)) {                                                         \
            fprintf(stderr, "check failed: %s (%s:%d)\n", what, __FILE__, __LINE__); \
            ++fails;                                                           \
        }                                                                      \
    } while (0)

static void base_params(or_params *P, int dim, int n_side)
{
    memset(P, 0, sizeof(*P));
    P->dim = dim;
    P->h = 1.0 / n_side;
    P->kappa = 3.0;
    P->rho0 = 1.0;
    P->mass = pow(P->h, dim);
    P->vref = 1.0;
    P->beta = 10.0;
    P->nu = 0.01;
    P->eps_av = 0.01;
    P->eta = 0.01;
    P->dt = 0.25 * P->h;
    P->tol = 1e-3;
    P->max_iter = 200;
    P->stall_window = 4;
    P->stall_rel = 0.05;
    P->shift_n = 1;
    P->shift_r = 1.0;
    for (int a = 0; a < 3; ++a) {
        P->lo[a] = 0.0;
        P->hi[a] = 1.0;
        P->periodic[a] = a < dim;
    }
}

/* Periodic lattice of n_side^dim particles with jitter, TGV-like fields. */
static int lattice(const or_params *P, int n_side, double *x, double *v, double *p)
{
    int n = 0;
    const int nz = P->dim == 3 ? n_side : 1;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < n_side; ++j)
            for (int i = 0; i < n_side; ++i, ++n) {
                double c[3] = {(i + 0.5) * P->h, (j + 0.5) * P->h, P->dim == 3 ? (k + 0.5) * P->h : 0.0};
                for (int a = 0; a < 3; ++a) x[3 * n + a] = a < P->dim ? c[a] + 0.05 * P->h * uniform() : 0.0;
                v[3 * n + 0] = -cos(2 * M_PI * c[0]) * sin(2 * M_PI * c[1]);
                v[3 * n + 1] = sin(2 * M_PI * c[0]) * cos(2 * M_PI * c[1]);
                v[3 * n + 2] = 0.0;
                p[n] = -0.25 * (cos(4 * M_PI * c[0]) + cos(4 * M_PI * c[1]));
            }
    return n;
}

static int all_finite(const double *a, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

static void check_lists(const or_params *P, int nf, int nw, const double *x)
{
    const int n = nf + nw;
    int64_t *ob = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *oc = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t tb = or_neighbors(P, nf, nw, x, 0, ob, NULL, 0);
    int64_t tc = or_neighbors(P, nf, nw, x, 1, oc, NULL, 0);
    CHECK(tb == tc, "brute and binned pair totals");
    int32_t *ib = (int32_t *)malloc(sizeof(int32_t) * (size_t)(tb > 0 ? tb : 1));
    int32_t *ic = (int32_t *)malloc(sizeof(int32_t) * (size_t)(tc > 0 ? tc : 1));
    or_neighbors(P, nf, nw, x, 0, ob, ib, tb);
    or_neighbors(P, nf, nw, x, 1, oc, ic, tc);
    CHECK(memcmp(ob, oc, sizeof(int64_t) * ((size_t)n + 1)) == 0, "brute and binned offsets");
    CHECK(tb == tc && memcmp(ib, ic, sizeof(int32_t) * (size_t)tb) == 0, "brute and binned lists");
    free(ob); free(oc); free(ib); free(ic);
}

static void run_case(or_params *P, int nf, int nw, double *x, double *v, double *p)
{
    const int n = nf + nw;
    const size_t b3 = sizeof(double) * 3 * (size_t)n, b1 = sizeof(double) * (size_t)n;
    double *vp = (double *)malloc(b3), *D = (double *)calloc(n, sizeof(double));
    double *R = (double *)calloc(3 * (size_t)n, sizeof(double)), *pw = (double *)calloc(n, sizeof(double));
    double *vg = (double *)calloc(3 * (size_t)n, sizeof(double));
    memcpy(vp, v, b3);
    check_lists(P, nf, nw, x);
    or_rates(P, nf, nw, x, v, p, 1, D, R, pw, vg);
    CHECK(all_finite(D, nf) && all_finite(R, 3 * (size_t)nf), "rates finite");
    or_rates_vt(P, nf, nw, x, v, p, v, 0, D, R, pw, vg);
    CHECK(all_finite(D, nf), "advective rates finite");
    double *x0 = (double *)malloc(b3), *v0 = (double *)malloc(b3), *p0 = (double *)malloc(b1);
    double *d0 = (double *)malloc(b1), *acc = (double *)malloc(b3);
    or_predict(P, nf, nw, x, v, p, x0, v0, p0, d0, acc);
    or_report rep;
    or_pseudo_loop(P, nf, nw, x0, v, vp, v0, p0, d0, 3, 1, &rep);
    CHECK(rep.iters == 3 && all_finite(v0, 3 * (size_t)n), "fixed loop");
    P->conv_norm = 1;
    or_pseudo_loop(P, nf, nw, x0, v, vp, v0, p0, d0, 0, 0, &rep);
    P->conv_norm = 0;
    CHECK(rep.iters >= 1 && rep.iters <= P->max_iter, "free loop");
    or_correct(P, nf, nw, x, v, vp, p, v0, p0);
    CHECK(all_finite(x, 3 * (size_t)n) && all_finite(p, n), "corrector");
    int32_t rows[3] = {0, nf / 2, nf - 1};
    double vo[9], po[3], dd[3];
    or_rows(P, nf, nw, 0, x, v, p, d0, v, vp, 3, rows, vo, po, dd);
    or_rows(P, nf, nw, 1, x, v, p, d0, v, vp, 3, rows, vo, po, dd);
    CHECK(all_finite(vo, 9) && all_finite(po, 3) && all_finite(dd, 3), "sampled rows");
    double *dr = (double *)calloc(3 * (size_t)nf, sizeof(double));
    int32_t *fs = (int32_t *)calloc((size_t)nf, sizeof(int32_t));
    or_shift(P, nf, nw, x, v, p, dr, fs);
    CHECK(all_finite(dr, 3 * (size_t)nf), "shift");
    or_report reps[2];
    P->shift = 1;
    or_step(P, nf, nw, x, v, vp, p, 2, 0, reps);
    P->shift = 0;
    for (int mv = 1; mv <= 2; ++mv) {
        P->move = mv;
        or_step(P, nf, nw, x, v, vp, p, 1, 2, reps);
    }
    P->move = 0;
    P->steady = 1;
    or_step(P, nf, nw, x, v, vp, p, 1, 2, reps);
    P->steady = 0;
    CHECK(all_finite(x, 3 * (size_t)n) && all_finite(v, 3 * (size_t)n) && all_finite(p, n), "steps");
    double hp[5] = {1.0, 0.99, 0.98, 0.97, 0.96}, hv[5] = {1e-4, 1e-4, 1e-4, 1e-4, 1e-4};
    CHECK(or_stop_test(P, hp, hv, 5) == OR_STALLED, "stop test");
    free(vp); free(D); free(R); free(pw); free(vg); free(x0); free(v0); free(p0); free(d0); free(acc);
    free(dr); free(fs);
}

int main(void)
{
    or_set_num_threads(2);
    for (int dim = 2; dim <= 3; ++dim) {
        const int side = dim == 2 ? 12 : 8;
        or_params P;
        base_params(&P, dim, side);
        const int cap = dim == 2 ? side * side : side * side * side;
        double *x = (double *)malloc(sizeof(double) * 3 * cap), *v = (double *)malloc(sizeof(double) * 3 * cap);
        double *p = (double *)malloc(sizeof(double) * cap);
        const int n = lattice(&P, side, x, v, p);
        run_case(&P, n, 0, x, v, p);
        free(x); free(v); free(p);
    }
    {   /* walled 2D box: fluid block and three wall layers below it, gravity,
           artificial viscosity; one fluid particle outside the grid box */
        or_params P;
        base_params(&P, 2, 16);
        P.periodic[0] = P.periodic[1] = 0;
        P.lo[0] = P.lo[1] = -0.25;
        P.hi[0] = P.hi[1] = 1.25;
        P.g[1] = -9.81;
        P.alpha = 0.1;
        P.vref = 4.0;
        P.dt = 0.25 * P.h / P.vref;
        const int nfx = 10, nfy = 8, nwx = 16, layers = 3;
        const int nf = nfx * nfy, nw = nwx * layers, n = nf + nw;
        double *x = (double *)calloc(3 * (size_t)n, sizeof(double)), *v = (double *)calloc(3 * (size_t)n, sizeof(double));
        double *p = (double *)calloc((size_t)n, sizeof(double));
        int k = 0;
        for (int j = 0; j < nfy; ++j)
            for (int i = 0; i < nfx; ++i, ++k) {
                x[3 * k] = (i + 0.5) * P.h;
                x[3 * k + 1] = (j + 0.5) * P.h;
                p[k] = 9.81 * (nfy - j - 0.5) * P.h;
            }
        x[0] = -0.6; /* outside the grid box: clamped into an edge cell */
        for (int j = 0; j < layers; ++j)
            for (int i = 0; i < nwx; ++i, ++k) {
                x[3 * k] = (i - 3 + 0.5) * P.h;
                x[3 * k + 1] = -(j + 0.5) * P.h;
            }
        run_case(&P, nf, nw, x, v, p);
        /* a coordinate far beyond the box (a diverged run): the binned search
           caps its bins and still agrees with brute force */
        x[3] = 1e14;
        x[4] = -3e13;
        check_lists(&P, nf, nw, x);
        free(x); free(v); free(p);
    }
    if (fails) {
        fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    printf("oracle sanitizer run: all checks passed\n");
    return 0;
}
