/*
 * FP64 CPU oracle for one real time step of dual-time EDAC SPH with particles
 * frozen in pseudo-time (paper: sections 2.2 "Fixed particles in pseudo-time",
 * 3.2 "Fixed particles in pseudo-time", 3.4 "Stability and convergence" and
 * Algorithm 2 "Fixed particles in pseudo-time").
 *
 * TEST INFRASTRUCTURE ONLY. This is the slow, plain reference that the GPU
 * library is checked against. Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product path never does.
 * It shares no code, header, table or constant generator with the GPU library.
 *
 * Everything is FP64, compiled without fast-math and without FMA contraction.
 * Particles are in caller order: the first nf are fluid, the next nw are walls.
 * Vectors are stored with three components per particle (unused ones zero).
 *
 * Readings of points the paper leaves open (each one is named where it is used):
 *  R-kernel  the quintic spline is named but not printed: textbook M6 form.
 *  R-edac    EDAC diffusion uses (r^2 + eta h^2) and 4 m_j/(rho_i+rho_j), i.e.
 *            the Morris operator of the viscous term; flags restore the
 *            printed forms (r^2 + h^2) and the extra 1/rho_j.
 *  R-av      the regulariser of phi_ij is eps_av = 0.01; h_ij = h, c_ij = c,
 *            rho_ij = rho0 (uniform smoothing length, sound speed, density).
 *  R-pass    one pair pass per pseudo-iteration: stage 1 half-step of p with
 *            the stored rate, rates at (V^k, p^{k+1/2}), then stage 2.
 *  R-pre     the rate before the loop is the momentum right side with the
 *            pseudo-time derivative set to zero, at (r^n, V^n, p^n).
 *  R-frozen  the loop uses the predicted positions r^(0), frozen; neighbours
 *            are recomputed there.
 *  R-conv    residuals are means over fluid of |dp/dtau| dt/(rho c^2) and of
 *            |Vtilde|/V_ref with Vtilde = dt dV/dtau; the stall test takes the
 *            last W values of each series; max norms are computed alongside.
 *  R-wall    walls follow Adami et al. (2012): pressure from the fluid by
 *            kernel-weighted average plus the hydrostatic correction, clipped
 *            at zero; ghost velocity 2 v_w - <v_f>. In the fluid rates a wall
 *            gives p_w to the pressure terms, its ghost velocity to the viscous
 *            and artificial-viscosity terms and its prescribed velocity to
 *            the divergence term.
 *  R-shift   particle shifting (section 3.5) after the corrector, at
 *            (r^{n+1}, V^{n+1}, p^{n+1}): the printed coefficient
 *            1 + W_ij / W(dx) with dx = h (generalised to 1 + R (W_ij/W(dx))^n,
 *            R = n = 1 as printed); sums over fluid and wall neighbours with
 *            V_j = m / rho0; the free-surface test uses the SPH estimate
 *            div r_i = -sum_j V_j r_ij . gradW_ij; the Taylor correction uses
 *            (grad phi)_i = sum_j V_j (phi_j - phi_i) gradW_ij over fluid
 *            neighbours and corrects V^{n+1} and p^{n+1} (the stored V^n of the
 *            time history is left as it is); all sums see the unshifted state.
 *  R-steady  steady-state solve (sections 2.3 and 3.3): the pressure rate is
 *            eq. dp-dtau-frozen (no EDAC term), the momentum rate eq.
 *            mom-steady: no real-time term, plus minus the convective sum
 *            sum_j (V_i . gradW_ij)(V_i m_i/rho_i + V_j m_j/rho_j) (a wall
 *            gives its ghost velocity, as in the viscous term); the pseudo-time
 *            integrator is the frozen one; particles never move. A real step
 *            becomes one run of the pseudo-time loop from the current state,
 *            started with the steady pressure rate there, whose result is
 *            committed as the new state (V^{n-1} <- V^n, V^n <- V^K); eq. conv
 *            is applied with the configured dt.
 *  R-move    moving particles in pseudo-time (section 2.1, section 3.1,
 *            Algorithm 1): the rate before the loop and the predictor are those
 *            of the frozen scheme (Vtilde^0 = 0 makes the advective terms
 *            vanish there); iteration k evaluates the rates at r^{k+1/2} =
 *            r^k + dtau/2 Vtilde^k with Vtilde^k in the advective terms; the
 *            pressure's advective term is rho_i Vtilde_i . sum_j m_j (p_i/rho_i^2
 *            + p_j/rho_j^2) gradW_ij (the printed sum is grad(p)/rho; the factor
 *            rho_i makes it the Vtilde . grad(p) of eq. CE_material, the same
 *            for rho = 1), the momentum's is sum_j (Vtilde_i . gradW_ij)
 *            (V_i m_i/rho_i + V_j m_j/rho_j) with a wall's ghost velocity; then
 *            Vtilde^{k+1} = dt (dV/dtau) (eq. vtilde) and r^{k+1} = r^{k+1/2} +
 *            dtau/2 Vtilde^{k+1} (eq. rkp1), each half step wrapped. Walls stay.
 *            Neighbours: move = 1 keeps the lists of r^(0) for the whole loop
 *            (a pair leaving the support adds zero); move = 2 recomputes them at
 *            every r^{k+1/2}. After the loop eq. r-update starts from r^n.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t dim;
    int32_t pad0;
    double h, kappa;
    double rho0, mass;
    double vref, beta;
    double nu, nu_e;
    double alpha, eps_av, eta;
    double g[3];
    double dt, dtau;
    double tol;
    int32_t max_iter, stall_window;
    double stall_rel;
    int32_t conv_norm;
    int32_t pad1;
    double lo[3], hi[3];
    int32_t periodic[3];
    int32_t edac_reg_literal, edac_rho_literal;
    int32_t pad2;
    int32_t shift, shift_n; /* particle shifting on/off and the exponent n (R-shift) */
    double shift_r;         /* R of the shifting coefficient (R-shift)              */
    int32_t steady;         /* steady-state solve (R-steady)                        */
    int32_t move;           /* 0 frozen, 1 moving, 2 moving + neighbour update (R-move) */
} or_params;

typedef struct {
    int32_t iters;
    int32_t reason; /* 1 converged, 2 stalled, 3 max_iter, 4 non-finite, 5 fixed count */
    double rp_mean, rv_mean, rp_max, rv_max;
    int64_t pairs; /* fluid-row neighbour pairs per iteration */
} or_report;

enum { OR_CONVERGED = 1, OR_STALLED = 2, OR_MAXITER = 3, OR_NONFINITE = 4, OR_FIXED = 5 };

/* ---- derived constants: section 3.4 (c = beta V_ref, dtau = dt / beta) and
 *      eq. nu_edac (nu_e = h c / 16) ---------------------------------------- */
static double sound(const or_params *P) { return P->beta * P->vref; }
static double nu_edac(const or_params *P) { return P->nu_e > 0 ? P->nu_e : P->h * sound(P) / 16.0; }
static double pseudo_dt(const or_params *P) { return P->dtau > 0 ? P->dtau : P->dt / P->beta; }

/* ---- quintic spline (R-kernel) -------------------------------------------
 * w(q) = (3-q)^5 - 6(2-q)^5 + 15(1-q)^5, each term only where its base is
 * positive; W = sigma_d w(r/h) with sigma chosen so that W integrates to one:
 * sigma_1 = 1/(120 h), sigma_2 = 7/(478 pi h^2), sigma_3 = 1/(120 pi h^3).   */
double or_sigma(int dim, double h)
{
    if (dim == 1) return 1.0 / (120.0 * h);
    if (dim == 2) return 7.0 / (478.0 * M_PI * h * h);
    return 1.0 / (120.0 * M_PI * h * h * h);
}

static double pow5(double t) { return t * t * t * t * t; }
static double pow4(double t) { return t * t * t * t; }

double or_w(int dim, double h, double r)
{
    double q = r / h, w = 0.0;
    if (q < 3.0) w += pow5(3.0 - q);
    if (q < 2.0) w -= 6.0 * pow5(2.0 - q);
    if (q < 1.0) w += 15.0 * pow5(1.0 - q);
    return or_sigma(dim, h) * w;
}

/* dW/dr */
double or_dwdr(int dim, double h, double r)
{
    double q = r / h, d = 0.0;
    if (q < 3.0) d -= 5.0 * pow4(3.0 - q);
    if (q < 2.0) d += 30.0 * pow4(2.0 - q);
    if (q < 1.0) d -= 75.0 * pow4(1.0 - q);
    return or_sigma(dim, h) * d / h;
}

/* ---- geometry --------------------------------------------------------------
 * Separation r_i - r_j with the minimum-image convention on periodic axes:
 * subtract, then shift by one period if beyond half a period.               */
static void separation(const or_params *P, const double *xi, const double *xj, double d[3])
{
    for (int a = 0; a < 3; ++a) {
        if (a >= P->dim) { d[a] = 0.0; continue; }
        double s = xi[a] - xj[a];
        if (P->periodic[a]) {
            double L = P->hi[a] - P->lo[a];
            if (s > 0.5 * L) s -= L;
            else if (s < -0.5 * L) s += L;
        }
        d[a] = s;
    }
}

static double norm2(const double d[3]) { return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]; }

static double support2(const or_params *P) { double kh = P->kappa * P->h; return kh * kh; }

static int is_neighbor(const or_params *P, const double *xi, const double *xj)
{
    double d[3];
    separation(P, xi, xj, d);
    return norm2(d) < support2(P);
}

/* Position wrapped back into [lo, hi) on periodic axes. */
static double wrap(const or_params *P, int a, double x)
{
    if (a < P->dim && P->periodic[a]) {
        double L = P->hi[a] - P->lo[a];
        if (x >= P->hi[a]) x -= L;
        else if (x < P->lo[a]) x += L;
    }
    return x;
}

/* ---- neighbour lists ---------------------------------------------------------
 * N(i) = { j != i : |r_ij| < kappa h }. Fluid rows list fluid and wall j; wall
 * rows list fluid j only. Rows are in ascending j. Two finders: the definition
 * by brute force, and a binned search that must return the same sets.       */
typedef struct {
    int64_t *off; /* n + 1 */
    int32_t *idx;
} nlist;

static void nlist_free(nlist *L)
{
    free(L->off);
    free(L->idx);
    L->off = NULL;
    L->idx = NULL;
}

static int allowed(int nf, int i, int j) { return j != i && (i < nf || j < nf); }

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static void build_brute(const or_params *P, int nf, int nw, const double *x, nlist *L)
{
    int n = nf + nw;
    L->off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *cnt = (int64_t *)calloc((size_t)n, sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < n; ++i) {
        int64_t c = 0;
        for (int j = 0; j < n; ++j)
            if (allowed(nf, i, j) && is_neighbor(P, x + 3 * i, x + 3 * j)) ++c;
        cnt[i] = c;
    }
    for (int i = 0; i < n; ++i) L->off[i + 1] = L->off[i] + cnt[i];
    L->idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(L->off[n] > 0 ? L->off[n] : 1));
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < n; ++i) {
        int64_t c = L->off[i];
        for (int j = 0; j < n; ++j)
            if (allowed(nf, i, j) && is_neighbor(P, x + 3 * i, x + 3 * j)) L->idx[c++] = j;
    }
    free(cnt);
}

/* Bins along each axis no smaller than kappa h (a small relative margin keeps
 * every true neighbour within one bin after rounding); periodic axes tile the
 * period, other axes cover the particles' range. Bins hold singly linked lists
 * of particle ids. Candidates come from the bin and its adjacent bins.       */
static void build_binned(const or_params *P, int nf, int nw, const double *x, nlist *L)
{
    int n = nf + nw, dim = P->dim;
    double kh = P->kappa * P->h * (1.0 + 1e-9);
    double base[3] = {0, 0, 0}, bs[3] = {1, 1, 1};
    int nb[3] = {1, 1, 1};
    for (int a = 0; a < dim; ++a) {
        if (P->periodic[a]) {
            double Lp = P->hi[a] - P->lo[a];
            nb[a] = (int)floor(Lp / kh);
            if (nb[a] < 1) nb[a] = 1;
            base[a] = P->lo[a];
            bs[a] = Lp / nb[a];
        } else {
            double mn = INFINITY, mx = -INFINITY;
            for (int i = 0; i < n; ++i) {
                if (x[3 * i + a] < mn) mn = x[3 * i + a];
                if (x[3 * i + a] > mx) mx = x[3 * i + a];
            }
            if (!(mn <= mx)) { mn = 0; mx = 0; } /* no particle, or none finite */
            base[a] = mn;
            bs[a] = kh;
            /* at most (8n + 64)^(1/dim) + 1 bins per axis (more than twice what
               particles at any density below a lattice's fill): beyond them,
               particles share the last bin, where the exact predicate still
               decides (a search, not arithmetic) */
            const double cap = floor(pow(8.0 * n + 64.0, 1.0 / dim)) + 1.0;
            const double span = floor((mx - mn) / kh) + 1.0;
            nb[a] = span < cap ? (int)span : (int)cap;
        }
    }
    int64_t nbins = (int64_t)nb[0] * nb[1] * nb[2];
    int32_t *head = (int32_t *)malloc(sizeof(int32_t) * (size_t)nbins);
    int32_t *next = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *bin3 = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)(n > 0 ? n : 1));
    for (int64_t b = 0; b < nbins; ++b) head[b] = -1;
    for (int i = n - 1; i >= 0; --i) {
        int64_t lin = 0;
        for (int a = 2; a >= 0; --a) {
            int c = 0;
            if (a < dim) {
                double f = floor((x[3 * i + a] - base[a]) / bs[a]);
                if (!(f >= 0.0)) f = 0.0; /* below the range, or not finite */
                if (f > (double)(nb[a] - 1)) f = (double)(nb[a] - 1);
                c = (int)f;
            }
            bin3[3 * i + a] = c;
            lin = lin * nb[a] + c;
        }
        next[i] = head[lin];
        head[lin] = i;
    }
    L->off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t **rows = (int32_t **)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t *));
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < n; ++i) {
        int cand[3][3], ncand[3];
        for (int a = 0; a < 3; ++a) {
            ncand[a] = 0;
            if (a >= dim) { cand[a][ncand[a]++] = 0; continue; }
            for (int o = -1; o <= 1; ++o) {
                int c = bin3[3 * i + a] + o;
                if (P->periodic[a]) c = ((c % nb[a]) + nb[a]) % nb[a];
                else if (c < 0 || c >= nb[a]) continue;
                int dup = 0;
                for (int k = 0; k < ncand[a]; ++k) dup |= cand[a][k] == c;
                if (!dup) cand[a][ncand[a]++] = c;
            }
        }
        int cap = 64, len = 0;
        int32_t *row = (int32_t *)malloc(sizeof(int32_t) * cap);
        for (int u = 0; u < ncand[0]; ++u)
            for (int v = 0; v < ncand[1]; ++v)
                for (int w = 0; w < ncand[2]; ++w) {
                    int64_t lin = ((int64_t)cand[2][w] * nb[1] + cand[1][v]) * nb[0] + cand[0][u];
                    for (int j = head[lin]; j >= 0; j = next[j]) {
                        if (!allowed(nf, i, j) || !is_neighbor(P, x + 3 * i, x + 3 * j)) continue;
                        if (len == cap) { cap *= 2; row = (int32_t *)realloc(row, sizeof(int32_t) * cap); }
                        row[len++] = j;
                    }
                }
        qsort(row, (size_t)len, sizeof(int32_t), cmp_i32);
        rows[i] = row;
        L->off[i + 1] = len;
    }
    for (int i = 0; i < n; ++i) L->off[i + 1] += L->off[i];
    L->idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(L->off[n] > 0 ? L->off[n] : 1));
    for (int i = 0; i < n; ++i) {
        memcpy(L->idx + L->off[i], rows[i], sizeof(int32_t) * (size_t)(L->off[i + 1] - L->off[i]));
        free(rows[i]);
    }
    free(rows);
    free(head);
    free(next);
    free(bin3);
}

static void build_nlist(const or_params *P, int nf, int nw, const double *x, int method, nlist *L)
{
    if (method == 0) build_brute(P, nf, nw, x, L);
    else build_binned(P, nf, nw, x, L);
}

int64_t or_neighbors(const or_params *P, int nf, int nw, const double *x, int method,
                     int64_t *off, int32_t *idx, int64_t cap)
{
    nlist L;
    build_nlist(P, nf, nw, x, method, &L);
    int n = nf + nw;
    int64_t total = L.off[n];
    if (off) memcpy(off, L.off, sizeof(int64_t) * ((size_t)n + 1));
    if (idx && total <= cap) memcpy(idx, L.idx, sizeof(int32_t) * (size_t)total);
    nlist_free(&L);
    return total;
}

static int64_t fluid_pairs(const nlist *L, int nf) { return L->off[nf]; }

/* ---- wall pass (R-wall) ------------------------------------------------------
 * For wall w over its fluid neighbours f:
 *   p_w = max(0, (sum p_f W_wf + g . sum rho_f r_wf W_wf) / sum W_wf)
 *   vg_w = 2 v_w - sum v_f W_wf / sum W_wf
 * (walls do not accelerate); a wall with no fluid neighbour gets p_w = 0 and
 * vg_w = v_w. Inputs are indexed by particle; outputs fill wall entries.     */
static void wall_pass(const or_params *P, int nf, int nw, const double *x, const double *v,
                      const double *p, const nlist *L, double *pw, double *vg)
{
#pragma omp parallel for schedule(static)
    for (int w = nf; w < nf + nw; ++w) {
        double S0 = 0, Sp = 0, Srr[3] = {0, 0, 0}, Sv[3] = {0, 0, 0};
        for (int64_t k = L->off[w]; k < L->off[w + 1]; ++k) {
            int f = L->idx[k];
            double d[3];
            separation(P, x + 3 * w, x + 3 * f, d);
            double W = or_w(P->dim, P->h, sqrt(norm2(d)));
            S0 += W;
            Sp += p[f] * W;
            for (int a = 0; a < 3; ++a) {
                Srr[a] += P->rho0 * d[a] * W;
                Sv[a] += v[3 * f + a] * W;
            }
        }
        if (S0 > 0) {
            double gr = P->g[0] * Srr[0] + P->g[1] * Srr[1] + P->g[2] * Srr[2];
            double pv = (Sp + gr) / S0;
            pw[w] = pv > 0 ? pv : 0.0;
            for (int a = 0; a < 3; ++a) vg[3 * w + a] = 2.0 * v[3 * w + a] - Sv[a] / S0;
        } else {
            pw[w] = 0.0;
            for (int a = 0; a < 3; ++a) vg[3 * w + a] = v[3 * w + a];
        }
    }
}

/* ---- rates of one fluid particle -----------------------------------------------
 * D_i: eq. dp-dtau-frozen-edac (EDAC pressure rate, R-edac); for a steady solve
 *      eq. dp-dtau-frozen (R-steady).
 * R_i: right side of eq. mom-sph-frozen (pressure gradient with artificial
 *      viscosity eq. mom-av / eq. av-phiij, Morris viscous term, body force);
 *      for a steady solve also minus the convective sum of eq. mom-steady.
 * vdiv: velocity used in the divergence term; vvis: velocity in the viscous
 * and artificial-viscosity terms; pall: pressure of every particle.          */
static void rates_one(const or_params *P, int i, const double *x, const double *vdiv,
                      const double *vvis, const double *pall, const int32_t *nb, int64_t nnb,
                      const double *vt, double *Di, double Ri[3])
{
    const double h = P->h, c = sound(P), c2 = c * c, nue = nu_edac(P);
    const double rhoi = P->rho0, rhoj = P->rho0, mj = P->mass;
    double D = 0.0, R[3] = {0, 0, 0};
    const double *Vt = vt ? vt + 3 * i : NULL; /* Vtilde_i (R-move) */
    for (int64_t k = 0; k < nnb; ++k) {
        int j = nb[k];
        double d[3];
        separation(P, x + 3 * i, x + 3 * j, d);
        double r2 = norm2(d), r = sqrt(r2);
        double dw = or_dwdr(P->dim, h, r), gw[3];
        for (int a = 0; a < 3; ++a) gw[a] = r > 0 ? dw * d[a] / r : 0.0;
        double gw_r = gw[0] * d[0] + gw[1] * d[1] + gw[2] * d[2];

        /* divergence term: (m_j rho_i / rho_j) c^2 V_ij . grad W_ij */
        double vd[3];
        for (int a = 0; a < 3; ++a) vd[a] = vdiv[3 * i + a] - vdiv[3 * j + a];
        D += mj * rhoi / rhoj * c2 * (vd[0] * gw[0] + vd[1] * gw[1] + vd[2] * gw[2]);

        /* EDAC diffusion: 4 m_j/(rho_i+rho_j) nu_e p_ij grad W . r_ij / (r^2 + eta h^2) */
        if (!P->steady) {
            double dreg = P->edac_reg_literal ? r2 + h * h : r2 + P->eta * h * h;
            double ecoef = 4.0 * mj / (rhoi + rhoj);
            if (P->edac_rho_literal) ecoef /= rhoj;
            D += ecoef * nue * (pall[i] - pall[j]) * gw_r / dreg;
        }

        /* momentum: -m_j (p_i/rho_i^2 + p_j/rho_j^2 + Pi_ij) grad W
         *           + m_j 4 nu (grad W . r_ij) / ((rho_i+rho_j)(r^2 + eta h^2)) V_ij */
        double vv[3];
        for (int a = 0; a < 3; ++a) vv[a] = vvis[3 * i + a] - vvis[3 * j + a];
        double vr = vv[0] * d[0] + vv[1] * d[1] + vv[2] * d[2];
        double Pi = 0.0;
        if (vr < 0) {
            double phi = vr / (r2 + P->eps_av * h * h);
            Pi = -P->alpha * h * c * phi / (0.5 * (rhoi + rhoj));
        }
        double pterm = pall[i] / (rhoi * rhoi) + pall[j] / (rhoj * rhoj) + Pi;
        double vcoef = mj * 4.0 * P->nu * gw_r / ((rhoi + rhoj) * (r2 + P->eta * h * h));
        for (int a = 0; a < 3; ++a) R[a] += -mj * pterm * gw[a] + vcoef * vv[a];
        if (P->steady) {
            /* eq. mom-steady: - (V_i . grad W_ij) (V_i m_i/rho_i + V_j m_j/rho_j) */
            const double *Vi = vvis + 3 * i, *Vj = vvis + 3 * j;
            double s = Vi[0] * gw[0] + Vi[1] * gw[1] + Vi[2] * gw[2];
            for (int a = 0; a < 3; ++a) R[a] -= s * (Vi[a] * P->mass / rhoi + Vj[a] * mj / rhoj);
        }
        if (Vt) {
            /* eq. dp-dtau, first term (R-move): rho_i Vtilde_i . m_j (p_i/rho_i^2 + p_j/rho_j^2) grad W */
            double tg = Vt[0] * gw[0] + Vt[1] * gw[1] + Vt[2] * gw[2];
            D += rhoi * mj * (pall[i] / (rhoi * rhoi) + pall[j] / (rhoj * rhoj)) * tg;
            /* eq. discrete_ME, first term: (Vtilde_i . grad W)(V_i m_i/rho_i + V_j m_j/rho_j) */
            const double *Vi = vvis + 3 * i, *Vj = vvis + 3 * j;
            for (int a = 0; a < 3; ++a) R[a] += tg * (Vi[a] * P->mass / rhoi + Vj[a] * mj / rhoj);
        }
    }
    for (int a = 0; a < 3; ++a) Ri[a] = a < P->dim ? R[a] + P->g[a] : 0.0;
    *Di = D;
}

static void rates(const or_params *P, int nf, const double *x, const double *vdiv,
                  const double *vvis, const double *pall, const nlist *L, const double *vt, double *D,
                  double *R)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nf; ++i)
        rates_one(P, i, x, vdiv, vvis, pall, L->idx + L->off[i], L->off[i + 1] - L->off[i],
                  vt, D + i, R + 3 * i);
}

/* Assemble the per-particle arrays the rate sums read: fluid entries from the
 * fluid state, wall entries from the wall pass and the prescribed velocity.  */
static void assemble(int nf, int n, const double *vk, const double *pf, const double *vw,
                     const double *pw, const double *vg, double *vdiv, double *vvis, double *pall)
{
    for (int i = 0; i < n; ++i) {
        int fl = i < nf;
        for (int a = 0; a < 3; ++a) {
            vdiv[3 * i + a] = fl ? vk[3 * i + a] : vw[3 * i + a];
            vvis[3 * i + a] = fl ? vk[3 * i + a] : vg[3 * i + a];
        }
        pall[i] = fl ? pf[i] : pw[i];
    }
}

/* ---- public: rates at (x, v, p) (walls handled by the wall pass first); with
 *      vt (Vtilde per particle, may be NULL) the advective terms of eq. dp-dtau
 *      and eq. discrete_ME are included (R-move) ---------------------------- */
int64_t or_rates_vt(const or_params *P, int nf, int nw, const double *x, const double *v,
                    const double *p, const double *vt, int method, double *D, double *R, double *pw_out,
                    double *vg_out);

int64_t or_rates(const or_params *P, int nf, int nw, const double *x, const double *v,
                 const double *p, int method, double *D, double *R, double *pw_out, double *vg_out)
{
    return or_rates_vt(P, nf, nw, x, v, p, NULL, method, D, R, pw_out, vg_out);
}

int64_t or_rates_vt(const or_params *P, int nf, int nw, const double *x, const double *v,
                    const double *p, const double *vt, int method, double *D, double *R, double *pw_out,
                    double *vg_out)
{
    int n = nf + nw;
    nlist L;
    build_nlist(P, nf, nw, x, method, &L);
    double *pw = (double *)calloc((size_t)n + 1, sizeof(double));
    double *vg = (double *)calloc(3 * (size_t)n + 3, sizeof(double));
    double *vdiv = (double *)malloc(sizeof(double) * (3 * (size_t)n + 3));
    double *vvis = (double *)malloc(sizeof(double) * (3 * (size_t)n + 3));
    double *pall = (double *)malloc(sizeof(double) * ((size_t)n + 1));
    wall_pass(P, nf, nw, x, v, p, &L, pw, vg);
    assemble(nf, n, v, p, v, pw, vg, vdiv, vvis, pall);
    rates(P, nf, x, vdiv, vvis, pall, &L, vt, D, R);
    if (pw_out) memcpy(pw_out, pw, sizeof(double) * (size_t)n);
    if (vg_out) memcpy(vg_out, vg, sizeof(double) * 3 * (size_t)n);
    int64_t pairs = fluid_pairs(&L, nf);
    free(pw); free(vg); free(vdiv); free(vvis); free(pall);
    nlist_free(&L);
    return pairs;
}

/* ---- predictor (eq. v0, eq. r0; R-pre) ---------------------------------------
 * (dV/dt)^n is the momentum right side at (r^n, V^n, p^n); D^n the pressure
 * rate there. V^(0) = V^n + dt a, r^(0) = r^n + dt V^n + dt^2/2 a (wrapped),
 * p^(0) = p^n, (dp/dtau)^0 = D^n. Walls keep position and velocity.         */
int64_t or_predict(const or_params *P, int nf, int nw, const double *x, const double *v,
                   const double *p, double *x0, double *v0, double *p0, double *d0, double *acc)
{
    int n = nf + nw;
    double *R = (double *)calloc(3 * (size_t)n + 3, sizeof(double));
    double *D = (double *)calloc((size_t)n + 1, sizeof(double));
    double *pw = (double *)calloc((size_t)n + 1, sizeof(double));
    int64_t pairs = or_rates(P, nf, nw, x, v, p, 1, D, R, pw, NULL);
    const double dt = P->dt;
    for (int i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) {
            if (i < nf) {
                double av = R[3 * i + a];
                v0[3 * i + a] = v[3 * i + a] + dt * av;
                x0[3 * i + a] = wrap(P, a, (x[3 * i + a] + dt * v[3 * i + a]) + (0.5 * dt * dt) * av);
                if (acc) acc[3 * i + a] = av;
            } else {
                v0[3 * i + a] = v[3 * i + a];
                x0[3 * i + a] = x[3 * i + a];
                if (acc) acc[3 * i + a] = 0.0;
            }
        }
        p0[i] = i < nf ? p[i] : pw[i];
        d0[i] = i < nf ? D[i] : 0.0;
    }
    free(R); free(D); free(pw);
    return pairs;
}

/* ---- stop test (eq. conv and the stall rule that follows it; R-conv) ---------
 * A series is settled when its latest value is below tol, or when at least W
 * values exist and the last W vary by less than stall_rel of their maximum.
 * Returns the stop reason or 0 to continue.                                    */
static int stop_reason(const or_params *P, const double *hp, const double *hv, int count)
{
    double xp = hp[count - 1], xv = hv[count - 1];
    if (!isfinite(xp) || !isfinite(xv)) return OR_NONFINITE;
    int W = P->stall_window;
    int stalled[2] = {0, 0};
    const double *ser[2] = {hp, hv};
    if (W > 0 && count >= W) {
        for (int s = 0; s < 2; ++s) {
            double mn = INFINITY, mx = -INFINITY;
            for (int k = count - W; k < count; ++k) {
                if (ser[s][k] < mn) mn = ser[s][k];
                if (ser[s][k] > mx) mx = ser[s][k];
            }
            stalled[s] = (mx - mn) < P->stall_rel * mx;
        }
    }
    int below_p = xp < P->tol, below_v = xv < P->tol;
    if ((below_p || stalled[0]) && (below_v || stalled[1]))
        return (below_p && below_v) ? OR_CONVERGED : OR_STALLED;
    if (count >= P->max_iter) return OR_MAXITER;
    return 0;
}

/* The stop test on given residual histories (count values each), for the tests
 * that drive it with synthetic series. */
int or_stop_test(const or_params *P, const double *hp, const double *hv, int count)
{
    return count > 0 ? stop_reason(P, hp, hv, count) : 0;
}

/* ---- pseudo-time loop (eqs. pkstar_frozen, vkp1_frozen, pkp1_frozen with the
 *      frozen eq. dv_dtau_exact; Algorithm 2 inner loop; R-pass) -------------
 * In: frozen positions x0, V^n (vn), V^{n-1} (vnm1); walls' prescribed velocity
 * in vn. In/out: V^k (vk), p^k (pk), (dp/dtau)^k (dk). On return the wall
 * entries of pk hold the last wall pressure. fixed_iters > 0 runs exactly that
 * many iterations without the stop test.
 * With P->move the particles move in pseudo-time from x0 (Algorithm 1 inner
 * loop: eqs. rkstar, pkstar, vkp1, rkp1, pkp1, vtilde with eq. dp-dtau and
 * eq. discrete_ME; R-move); x0 itself is not changed.                        */
int or_pseudo_loop(const or_params *P, int nf, int nw, const double *x0, const double *vn,
                   const double *vnm1, double *vk, double *pk, double *dk, int fixed_iters,
                   int method, or_report *rep)
{
    int n = nf + nw;
    nlist L;
    build_nlist(P, nf, nw, x0, method, &L);
    const double dt = P->dt, dtau = pseudo_dt(P), c = sound(P);
    /* frozen eq. dv_dtau_exact; a steady solve has no real-time term (R-steady) */
    const double gamma = P->steady ? 1.0 : 2.0 * dt / (2.0 * dt + 3.0 * dtau);
    int cap = fixed_iters > 0 ? fixed_iters : (P->max_iter > 0 ? P->max_iter : 1);
    double *hp = (double *)malloc(sizeof(double) * (size_t)cap);
    double *hv = (double *)malloc(sizeof(double) * (size_t)cap);
    double *hpx = (double *)malloc(sizeof(double) * (size_t)cap);
    double *hvx = (double *)malloc(sizeof(double) * (size_t)cap);
    double *phalf = (double *)calloc((size_t)n + 1, sizeof(double));
    double *pw = (double *)calloc((size_t)n + 1, sizeof(double));
    double *vg = (double *)calloc(3 * (size_t)n + 3, sizeof(double));
    double *vdiv = (double *)malloc(sizeof(double) * (3 * (size_t)n + 3));
    double *vvis = (double *)malloc(sizeof(double) * (3 * (size_t)n + 3));
    double *pall = (double *)malloc(sizeof(double) * ((size_t)n + 1));
    double *D = (double *)calloc((size_t)n + 1, sizeof(double));
    double *R = (double *)calloc(3 * (size_t)n + 3, sizeof(double));
    double *vt = (double *)calloc((size_t)n + 1, sizeof(double));
    /* moving particles (R-move): r^k, r^{k+1/2} and Vtilde^k, Vtilde^0 = 0 */
    double *xk = NULL, *xh = NULL, *vtil = NULL;
    if (P->move) {
        xk = (double *)malloc(sizeof(double) * (3 * (size_t)n + 3));
        xh = (double *)malloc(sizeof(double) * (3 * (size_t)n + 3));
        vtil = (double *)calloc(3 * (size_t)n + 3, sizeof(double));
        memcpy(xk, x0, sizeof(double) * 3 * (size_t)n);
        memcpy(xh, x0, sizeof(double) * 3 * (size_t)n);
    }
    int k = 0, reason = 0;
    while (!reason) {
        /* stage 1: p^{k+1/2} = p^k + dtau/2 (dp/dtau)^k */
        for (int i = 0; i < nf; ++i) phalf[i] = pk[i] + 0.5 * dtau * dk[i];
        /* moving: r^{k+1/2} = r^k + dtau/2 Vtilde^k (eq. rkstar), lists there with move = 2 */
        const double *xe = x0;
        if (P->move) {
            for (int i = 0; i < nf; ++i)
                for (int a = 0; a < 3; ++a) xh[3 * i + a] = wrap(P, a, xk[3 * i + a] + 0.5 * dtau * vtil[3 * i + a]);
            if (P->move == 2) {
                nlist_free(&L);
                build_nlist(P, nf, nw, xh, method, &L);
            }
            xe = xh;
        }
        /* walls from (V^k, p^{k+1/2}); velocities of walls are the prescribed ones */
        for (int i = nf; i < n; ++i)
            for (int a = 0; a < 3; ++a) vk[3 * i + a] = vn[3 * i + a];
        wall_pass(P, nf, nw, xe, vk, phalf, &L, pw, vg);
        assemble(nf, n, vk, phalf, vn, pw, vg, vdiv, vvis, pall);
        rates(P, nf, xe, vdiv, vvis, pall, &L, vtil, D, R);
        /* stage 2 */
        for (int i = 0; i < nf; ++i) {
            double nv = 0.0;
            for (int a = 0; a < 3; ++a) {
                double bdf = P->steady ? 0.0
                                       : (3.0 * vk[3 * i + a] - 4.0 * vn[3 * i + a] + vnm1[3 * i + a]) / (2.0 * dt);
                double dvdtau = (R[3 * i + a] - bdf) * gamma;
                vk[3 * i + a] += dtau * dvdtau;
                double t = dt * dvdtau; /* eq. vtilde */
                nv += t * t;
                if (P->move) { /* eq. rkp1: r^{k+1} = r^{k+1/2} + dtau/2 Vtilde^{k+1} */
                    vtil[3 * i + a] = t;
                    xk[3 * i + a] = wrap(P, a, xh[3 * i + a] + 0.5 * dtau * t);
                }
            }
            vt[i] = sqrt(nv);
            pk[i] = phalf[i] + 0.5 * dtau * D[i];
            dk[i] = D[i];
        }
        for (int i = nf; i < n; ++i) pk[i] = pw[i];
        /* residuals (sequential sums: deterministic) */
        double sp = 0, sv = 0, mp = 0, mv = 0;
        for (int i = 0; i < nf; ++i) {
            double ad = fabs(D[i]);
            sp += ad;
            sv += vt[i];
            if (ad > mp || ad != ad) mp = ad;
            if (vt[i] > mv || vt[i] != vt[i]) mv = vt[i];
        }
        double scale_p = dt / (P->rho0 * c * c);
        double nfd = nf > 0 ? (double)nf : 1.0;
        hp[k] = sp / nfd * scale_p;
        hv[k] = sv / nfd / P->vref;
        hpx[k] = mp * scale_p;
        hvx[k] = mv / P->vref;
        ++k;
        if (fixed_iters > 0) {
            if (!isfinite(hp[k - 1]) || !isfinite(hv[k - 1])) reason = OR_NONFINITE;
            else if (k >= fixed_iters) reason = OR_FIXED;
        } else {
            reason = P->conv_norm == 1 ? stop_reason(P, hpx, hvx, k) : stop_reason(P, hp, hv, k);
        }
    }
    if (rep) {
        rep->iters = k;
        rep->reason = reason;
        rep->rp_mean = hp[k - 1];
        rep->rv_mean = hv[k - 1];
        rep->rp_max = hpx[k - 1];
        rep->rv_max = hvx[k - 1];
        rep->pairs = fluid_pairs(&L, nf);
    }
    free(hp); free(hv); free(hpx); free(hvx); free(phalf); free(pw); free(vg);
    free(vdiv); free(vvis); free(pall); free(D); free(R); free(vt);
    free(xk); free(xh); free(vtil);
    nlist_free(&L);
    return reason == OR_NONFINITE ? -4 : (reason == OR_MAXITER ? 1 : 0);
}

/* ---- corrector (eq. r-update) ------------------------------------------------
 * r^{n+1} = r^n + dt/2 (V^n + V^{n+1}) (wrapped); V^{n-1} <- V^n; V^n <- V^{n+1};
 * p^n <- p^{n+1}. Walls keep position and velocity; their p is the last p_w. */
void or_correct(const or_params *P, int nf, int nw, double *x, double *v, double *v_prev,
                double *p, const double *vk, const double *pk)
{
    int n = nf + nw;
    for (int i = 0; i < nf; ++i)
        for (int a = 0; a < 3; ++a) {
            x[3 * i + a] = wrap(P, a, x[3 * i + a] + 0.5 * P->dt * (v[3 * i + a] + vk[3 * i + a]));
            v_prev[3 * i + a] = v[3 * i + a];
            v[3 * i + a] = vk[3 * i + a];
        }
    for (int i = 0; i < n; ++i) p[i] = pk[i];
}

/* ---- particle shifting (section 3.5: eq. shift, eq. shift-deltar, eq.
 * shift-correct, free-surface test; R-shift) ---------------------------------
 * For every fluid particle i, with neighbours at the current positions:
 *   div_r = -sum_j V_j r_ij . gradW_ij                   (fluid and walls)
 *   dr    = -(h^2/2) sum_j V_j (1 + R (W_ij/W(h))^n) gradW_ij   (fluid and walls)
 *   dr    = 0 if div_r < dim - 1/2 (free surface)
 *   grad p, grad V = sum_j V_j (phi_j - phi_i) gradW_ij  (fluid)
 * then r_i += dr (wrapped), p_i += grad p . dr, V_i += grad V . dr. Outputs
 * dr and the free-surface flag per fluid particle when the pointers are given. */
void or_shift(const or_params *P, int nf, int nw, double *x, double *v, double *p, double *dr_out,
              int32_t *fs_out)
{
    int n = nf + nw;
    nlist L;
    build_nlist(P, nf, nw, x, 1, &L);
    const double vol = P->mass / P->rho0;
    const double w0 = or_w(P->dim, P->h, P->h);
    double *dr = (double *)calloc(3 * (size_t)nf + 3, sizeof(double));
    double *dp = (double *)calloc((size_t)nf + 1, sizeof(double));
    double *dv = (double *)calloc(3 * (size_t)nf + 3, sizeof(double));
    int32_t *fs = (int32_t *)calloc((size_t)nf + 1, sizeof(int32_t));
    (void)n;
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < nf; ++i) {
        double divr = 0.0, s[3] = {0, 0, 0}, gp[3] = {0, 0, 0}, gv[3][3] = {{0}};
        for (int64_t e = L.off[i]; e < L.off[i + 1]; ++e) {
            const int j = L.idx[e];
            double d[3];
            separation(P, x + 3 * i, x + 3 * j, d);
            const double r = sqrt(norm2(d));
            if (r <= 0.0) continue;
            const double f = or_dwdr(P->dim, P->h, r) / r; /* gradW = f d */
            divr -= vol * f * ((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
            double ratio = or_w(P->dim, P->h, r) / w0, pw = 1.0;
            for (int k = 0; k < P->shift_n; ++k) pw *= ratio;
            const double c = vol * (1.0 + P->shift_r * pw) * f;
            for (int a = 0; a < 3; ++a) s[a] += c * d[a];
            if (j < nf) {
                const double cp = vol * (p[j] - p[i]) * f;
                for (int a = 0; a < 3; ++a) gp[a] += cp * d[a];
                for (int b = 0; b < 3; ++b) {
                    const double cv = vol * (v[3 * j + b] - v[3 * i + b]) * f;
                    for (int a = 0; a < 3; ++a) gv[b][a] += cv * d[a];
                }
            }
        }
        fs[i] = divr < P->dim - 0.5;
        double del[3] = {0, 0, 0};
        if (!fs[i])
            for (int a = 0; a < P->dim; ++a) del[a] = -0.5 * P->h * P->h * s[a];
        for (int a = 0; a < 3; ++a) dr[3 * i + a] = del[a];
        dp[i] = (gp[0] * del[0] + gp[1] * del[1]) + gp[2] * del[2];
        for (int b = 0; b < 3; ++b) dv[3 * i + b] = (gv[b][0] * del[0] + gv[b][1] * del[1]) + gv[b][2] * del[2];
    }
    for (int i = 0; i < nf; ++i) {
        for (int a = 0; a < 3; ++a) {
            x[3 * i + a] = wrap(P, a, x[3 * i + a] + dr[3 * i + a]);
            v[3 * i + a] += dv[3 * i + a];
            if (dr_out) dr_out[3 * i + a] = dr[3 * i + a];
        }
        p[i] += dp[i];
        if (fs_out) fs_out[i] = fs[i];
    }
    free(dr); free(dp); free(dv); free(fs);
    nlist_free(&L);
}

/* ---- steady-state segment (sections 2.3 and 3.3; R-steady) -------------------
 * D^0 is the steady pressure rate at (x, V, p); the pseudo-time loop runs from
 * there with the particles fixed; V^{n-1} <- V^n, V^n <- V^K, p <- p^K.       */
int or_steady_segment(const or_params *P, int nf, int nw, const double *x, double *v, double *v_prev,
                      double *p, int fixed_iters, or_report *rep)
{
    int n = nf + nw;
    size_t b3 = sizeof(double) * (3 * (size_t)n + 3), b1 = sizeof(double) * ((size_t)n + 1);
    double *vk = (double *)malloc(b3), *R = (double *)calloc(1, b3);
    double *pk = (double *)malloc(b1), *dk = (double *)calloc(1, b1), *pw = (double *)calloc(1, b1);
    or_rates(P, nf, nw, x, v, p, 1, dk, R, pw, NULL);
    for (int i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) vk[3 * i + a] = v[3 * i + a];
        pk[i] = i < nf ? p[i] : pw[i];
        if (i >= nf) dk[i] = 0.0;
    }
    int st = or_pseudo_loop(P, nf, nw, x, v, v_prev, vk, pk, dk, fixed_iters, 1, rep);
    for (int i = 0; i < nf; ++i)
        for (int a = 0; a < 3; ++a) {
            v_prev[3 * i + a] = v[3 * i + a];
            v[3 * i + a] = vk[3 * i + a];
        }
    for (int i = 0; i < n; ++i) p[i] = pk[i];
    free(vk); free(R); free(pk); free(dk); free(pw);
    return st;
}

/* ---- one or more real steps (Algorithm 2; shifting when P->shift; a steady
 *      solve when P->steady) --------------------------------------------------- */
int or_step(const or_params *P, int nf, int nw, double *x, double *v, double *v_prev,
            double *p, int n_steps, int fixed_iters, or_report *reps)
{
    int n = nf + nw, status = 0;
    size_t b3 = sizeof(double) * (3 * (size_t)n + 3), b1 = sizeof(double) * ((size_t)n + 1);
    double *x0 = (double *)malloc(b3), *v0 = (double *)malloc(b3);
    double *p0 = (double *)malloc(b1), *d0 = (double *)malloc(b1);
    for (int s = 0; s < n_steps; ++s) {
        if (P->steady) { /* R-steady: one loop from the current state, particles fixed */
            int st = or_steady_segment(P, nf, nw, x, v, v_prev, p, fixed_iters, reps ? reps + s : NULL);
            if (st < 0) { status = st; break; }
            if (st > 0) status = st;
            continue;
        }
        or_predict(P, nf, nw, x, v, p, x0, v0, p0, d0, NULL);
        int st = or_pseudo_loop(P, nf, nw, x0, v, v_prev, v0, p0, d0, fixed_iters, 1,
                                reps ? reps + s : NULL);
        if (st < 0) { status = st; break; }
        if (st > 0) status = st;
        or_correct(P, nf, nw, x, v, v_prev, p, v0, p0);
        if (P->shift) or_shift(P, nf, nw, x, v, p, NULL, NULL);
    }
    free(x0); free(v0); free(p0); free(d0);
    return status;
}

/* ---- sampled evaluation for large inputs ---------------------------------------
 * The quantities of selected fluid rows only, with neighbours found by brute
 * force over all particles, so that large problems can be checked one row at a
 * time. mode 0: predictor outputs V^(0) and D^n at (x, v, p) (v holds V^n for
 * fluid, prescribed velocity for walls). mode 1: one pseudo-iteration from the
 * in-loop state (x frozen, vk = V^k, pk = p^k, dk = (dp/dtau)^k, vn = V^n,
 * vnm1 = V^{n-1}); outputs V^1, p^1, D^{1/2}.                                  */
static int64_t brute_row(const or_params *P, int nf, int n, int i, const double *x, int32_t **out)
{
    int cap = 64, len = 0;
    int32_t *row = (int32_t *)malloc(sizeof(int32_t) * cap);
    for (int j = 0; j < n; ++j) {
        if (!allowed(nf, i, j) || !is_neighbor(P, x + 3 * i, x + 3 * j)) continue;
        if (len == cap) { cap *= 2; row = (int32_t *)realloc(row, sizeof(int32_t) * cap); }
        row[len++] = j;
    }
    *out = row;
    return len;
}

void or_rows(const or_params *P, int nf, int nw, int mode, const double *x, const double *vk,
             const double *pk, const double *dk, const double *vn, const double *vnm1,
             int nrows, const int32_t *rows, double *v_out, double *p_out, double *d_out)
{
    int n = nf + nw;
    const double dt = P->dt, dtau = pseudo_dt(P);
    const double gamma = P->steady ? 1.0 : 2.0 * dt / (2.0 * dt + 3.0 * dtau);
#pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < nrows; ++r) {
        int i = rows[r];
        int32_t *nb;
        int64_t nnb = brute_row(P, nf, n, i, x, &nb);
        /* local copies: entry 0 is i, then its neighbours */
        int m = (int)nnb + 1;
        double *lx = (double *)malloc(sizeof(double) * 3 * m);
        double *lvd = (double *)malloc(sizeof(double) * 3 * m);
        double *lvv = (double *)malloc(sizeof(double) * 3 * m);
        double *lp = (double *)malloc(sizeof(double) * m);
        int32_t *lnb = (int32_t *)malloc(sizeof(int32_t) * m);
        for (int e = 0; e < m; ++e) {
            int j = e == 0 ? i : nb[e - 1];
            lnb[e] = e;
            for (int a = 0; a < 3; ++a) lx[3 * e + a] = x[3 * j + a];
            double pj = 0;
            if (j < nf) {
                pj = mode == 0 ? pk[j] : pk[j] + 0.5 * dtau * dk[j];
                for (int a = 0; a < 3; ++a) lvd[3 * e + a] = lvv[3 * e + a] = vk[3 * j + a];
            } else {
                /* wall j: its own wall pass over its fluid neighbours */
                int32_t *wn;
                int64_t nwn = brute_row(P, nf, n, j, x, &wn);
                double S0 = 0, Sp = 0, Srr[3] = {0, 0, 0}, Sv[3] = {0, 0, 0};
                for (int64_t q = 0; q < nwn; ++q) {
                    int f = wn[q];
                    double d[3];
                    separation(P, x + 3 * j, x + 3 * f, d);
                    double W = or_w(P->dim, P->h, sqrt(norm2(d)));
                    double pf = mode == 0 ? pk[f] : pk[f] + 0.5 * dtau * dk[f];
                    S0 += W;
                    Sp += pf * W;
                    for (int a = 0; a < 3; ++a) {
                        Srr[a] += P->rho0 * d[a] * W;
                        Sv[a] += vk[3 * f + a] * W;
                    }
                }
                free(wn);
                const double *vwall = mode == 0 ? vk : vn;
                for (int a = 0; a < 3; ++a) lvd[3 * e + a] = vwall[3 * j + a];
                if (S0 > 0) {
                    double pv = (Sp + P->g[0] * Srr[0] + P->g[1] * Srr[1] + P->g[2] * Srr[2]) / S0;
                    pj = pv > 0 ? pv : 0.0;
                    for (int a = 0; a < 3; ++a) lvv[3 * e + a] = 2.0 * vwall[3 * j + a] - Sv[a] / S0;
                } else {
                    for (int a = 0; a < 3; ++a) lvv[3 * e + a] = vwall[3 * j + a];
                }
            }
            lp[e] = pj;
        }
        double D, R[3];
        rates_one(P, 0, lx, lvd, lvv, lp, lnb + 1, nnb, NULL, &D, R);
        for (int a = 0; a < 3; ++a) {
            if (mode == 0) {
                v_out[3 * r + a] = vk[3 * i + a] + dt * R[a];
            } else {
                double bdf = P->steady ? 0.0
                                       : (3.0 * vk[3 * i + a] - 4.0 * vn[3 * i + a] + vnm1[3 * i + a]) / (2.0 * dt);
                v_out[3 * r + a] = vk[3 * i + a] + dtau * (R[a] - bdf) * gamma;
            }
        }
        p_out[r] = mode == 0 ? pk[i] : lp[0] + 0.5 * dtau * D;
        d_out[r] = D;
        free(lx); free(lvd); free(lvv); free(lp); free(lnb); free(nb);
    }
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
