// Pair-pass launches of the frozen-particle dual-time EDAC SPH step, and the
// per-particle kernels around them (records, corrector, particle shifting,
// state transfer). The pair pass, wall pass and residual reduction themselves
// are in dtsph_pass_dev.h.
#include <hip/hip_ext.h>

#include <type_traits>

#include "dtsph_pass_dev.h"

namespace dtsph {

namespace {

// ---- per-particle kernels -------------------------------------------------------

// {V, p} records of the fluid; at the start of a loop (reset) also the reset of
// every sim's loop state and, unless the pressure master already holds it
// (add_half = 0), the stage-1 half step of p.
template <typename T, int DIM>
__global__ void k_records(int Nf, const int *__restrict__ simid, const SimDev *__restrict__ sims,
                          const T *__restrict__ vn, const T *__restrict__ w, double *__restrict__ pm,
                          const T *__restrict__ dp, typename V4<T>::type *__restrict__ vout, int reset,
                          int add_half, SimIter *__restrict__ iters, int n_sims, int fixed)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (reset && i < n_sims) {
        SimIter z{};
        z.fixed = fixed;
        for (int k = 0; k < kHist; ++k) { z.hp[k] = 0.0; z.hv[k] = 0.0; }
        iters[i] = z;
    }
    if (i >= Nf) return;
    double p = pm[i];
    if (add_half) {  // p^{k+1/2} = p^k + dtau/2 (dp/dtau)^k
        p += 0.5 * sims[simid[i]].dtau * (double)dp[i];
        pm[i] = p;
    }
    T v[3] = {0, 0, 0};
    for (int d = 0; d < DIM; ++d) v[d] = vn[d * Nf + i] + (w ? w[d * Nf + i] : T(0));
    vout[i] = make_rec<T, DIM>(v, (T)p);
}

// Corrector (eq. r-update) fused with the end of the loop and the set-up of the
// next rate pass: p^K = p^{K+1/2} - dtau/2 (dp/dtau)^K (when pending), positions
// r^{n+1} = r^n + dt/2 (V^n + V^{n+1}) with periodic wrap, history rotation,
// position records and the {V^{n+1}, p^{n+1}} records of buffer `vrec`.
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_correct(int N, int Nf, const int *__restrict__ simid,
                                                 const SimDev *__restrict__ sims, double *__restrict__ x,
                                                 const double *__restrict__ xn, T *__restrict__ vn,
                                                 T *__restrict__ dv, T *__restrict__ w, void *__restrict__ xr,
                                                 double *__restrict__ pm, const T *__restrict__ dp, int half,
                                                 void *__restrict__ prec, typename V4<T>::type *__restrict__ vrec,
                                                 int gated, int n_sims, const SimIter *__restrict__ iters)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Nf) return;
    // the particle's own state first: these loads depend on nothing, so they are
    // in flight while the gate and the sim's constants are read
    const int sid = simid[i];
    double p = pm[i];
    const T dpi = half ? dp[i] : T(0);
    T v0[DIM], wk[DIM];
    double xnd[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        v0[d] = vn[d * Nf + i];
        wk[d] = w[d * Nf + i];
        xnd[d] = xn[d * N + i];
    }
    if (gated && !spec_gate(n_sims, iters, sims)) return;
    const SimDev &S = sims[sid];
    if (half) {
        p -= 0.5 * S.dtau * (double)dpi;
        pm[i] = p;
    }
    double xo[3] = {0.0, 0.0, 0.0};
    T vr[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const T v1 = v0[d] + wk[d];
        vr[d] = v1;
        double xv = S.steady ? xnd[d] : xnd[d] + 0.5 * S.dt * ((double)v0[d] + (double)v1);
        if (S.periodic[d]) {
            if (xv >= S.hi[d]) xv -= S.L[d];
            else if (xv < S.lo[d]) xv += S.L[d];
        }
        x[d * N + i] = xv;
        xo[d] = xv;
        dv[d * Nf + i] = v1 - v0[d];
        vn[d * Nf + i] = v1;
        w[d * Nf + i] = T(0);
    }
    if (DIM == 2) ((double2 *)xr)[i] = make_double2(xo[0], xo[1]);
    else ((double4 *)xr)[i] = make_double4(xo[0], xo[1], xo[2], 0.0);
    write_pos_record<T>(S, prec, i, xo);
    vrec[i] = make_rec<T, DIM>(vr, (T)p);
}

// ---- particle shifting (section 3.5: eqs. shift, shift-deltar, shift-correct) ---
// After the corrector, for fluid particles of sims with shifting on, over the
// neighbour lists at the corrected positions (fluid and wall entries; a list
// entry beyond the support adds nothing):
//   div r = -sum_j V_j r_ij . gradW_ij; free surface if div r < dim - 1/2
//   dr = -(h^2/2) sum_j V_j (1 + R (W_ij / W(h))^n) gradW_ij (0 on the free surface)
//   grad phi = sum_j V_j (phi_j - phi_i) gradW_ij over fluid j, phi in {p, V}
// k_shift_sums evaluates these from the unshifted records into scratch arrays;
// k_shift_apply then moves the particles and adds the Taylor corrections
// grad phi . dr to p^{n+1} and V^{n+1} (and to V^{n+1} - V^n).
template <typename T> struct ShiftArgs {
    using Q = typename V4<T>::type;
    int N, Nf, Nw;
    const int *simid;
    const SimDev *sims;
    const int *nbr;
    const uint32_t *cnt;
    void *prec;
    Q *vrec;            // {V, p} records of buffer cur (read by the sums, rewritten by apply)
    double *dr, *dp;    // per fluid particle: shift (3 x Nf), pressure correction
    T *dv;              // velocity correction (3 x Nf)
    double *part;       // per workgroup: max |dr|^2
    double *x;          // active positions (3 x N)
    void *xr;
    T *vn, *vdiff;      // V^{n+1}; V^{n+1} - V^n
    double *pm;
    int gated, n_sims;  // gated: run only if spec_gate holds (speculative launch)
    const SimIter *iters;
};

// SL lanes share one particle (list entries sub, sub + SL, ...), combined by
// butterfly shuffles.
template <typename T, int DIM, int SL>
__global__ void __launch_bounds__(256) k_shift_sums(ShiftArgs<T> A)
{
    using Q = typename V4<T>::type;
    using PosT = Pos<T, DIM>;
    using Rec = typename PosT::Rec;
    __shared__ double lds[4];
    const int sub = (int)threadIdx.x & (SL - 1);
    const int i = (blockIdx.x * blockDim.x + threadIdx.x) / SL;
    const bool own = i < A.Nf;  // uniform in each group of SL lanes
    // the particle's own records, count and sim first: in flight while the gate
    // and the sim's constants are read
    const Rec *__restrict__ prec = (const Rec *)A.prec;
    Rec ri{};
    Q me{};
    uint32_t cn = 0u;
    int sid = 0;
    if (own) {
        ri = prec[i];
        me = A.vrec[i];
        cn = A.cnt[i];
        sid = A.simid[i];
    }
    if (A.gated && !spec_gate(A.n_sims, A.iters, A.sims)) return;  // uniform in the grid
    double m2 = 0.0;
    if (own) {
        const SimDev &S = A.sims[sid];
        double del[3] = {0.0, 0.0, 0.0}, dpi = 0.0;
        T dvi[3] = {T(0), T(0), T(0)};
        if (S.shift) {
            const PosT pos(S);
            const T pi = pres<DIM>(me);
            const T vi[3] = {me.x, me.y, DIM == 3 ? me.z : T(0)};
            const T inv_h = (T)S.inv_h, kg = (T)S.kg, vol = (T)S.vol, rco = (T)S.shift_r;
            const int nexp = S.shift_n;
            T divr = 0, sd[3] = {0, 0, 0}, gp[3] = {0, 0, 0}, gv[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
            const int total = (int)(cn & 0xffffu) + (int)(cn >> 16);
            const int *__restrict__ nb = A.nbr + i;
            // neighbours in batches of U per lane: U index loads, then 2U record
            // gathers in flight, then U pair evaluations (each lane keeps its
            // own summation order: entries sub, sub + SL, ...)
            constexpr int U = sizeof(T) == 4 ? 4 : 2;
            for (int k0 = sub; k0 < total; k0 += U * SL) {
                int jj[U];
#pragma unroll
                for (int m = 0; m < U; ++m) {
                    const int k = k0 + m * SL;
                    jj[m] = k < total ? nb[(size_t)k * A.N] : i;
                }
                Rec rj[U];
                Q vq[U];
#pragma unroll
                for (int m = 0; m < U; ++m) {
                    rj[m] = prec[jj[m]];
                    vq[m] = A.vrec[jj[m]];
                }
#pragma unroll
                for (int m = 0; m < U; ++m) {
                    const int j = jj[m];
                    T r[3];
                    pos.delta(ri, rj[m], r);
                    T r2 = r[0] * r[0] + r[1] * r[1];
                    if (DIM == 3) r2 += r[2] * r[2];
                    if (!(r2 > T(0))) continue;  // itself (padding) or a coincident particle
                    const T rinv = rsq<T>(r2);
                    const T q = r2 * rinv * inv_h;
                    T t3 = T(3) - q, t2 = T(2) - q, t1 = T(1) - q;
                    t3 = t3 > T(0) ? t3 : T(0);
                    t2 = t2 > T(0) ? t2 : T(0);
                    t1 = t1 > T(0) ? t1 : T(0);
                    const T a4 = t3 * t3 * t3 * t3, b4 = t2 * t2 * t2 * t2, c4 = t1 * t1 * t1 * t1;
                    const T f = kg * (T(15) * c4 + (T(-6) * b4 + a4)) * rinv;  // dW/dr / r
                    const T w5 = T(15) * c4 * t1 + (T(-6) * b4 * t2 + a4 * t3);
                    divr -= vol * f * r2;
                    const T ratio = w5 * T(1.0 / 26.0);  // W / W(h): w(1) = 2^5 - 6 = 26
                    T pw = T(1);
                    for (int e = 0; e < nexp; ++e) pw *= ratio;
                    const T cf = vol * (T(1) + rco * pw) * f;
                    for (int a = 0; a < DIM; ++a) sd[a] += cf * r[a];
                    if (j < A.Nf) {
                        const Q vj = vq[m];
                        const T cp = vol * (pres<DIM>(vj) - pi) * f;
                        const T vjv[3] = {vj.x, vj.y, DIM == 3 ? vj.z : T(0)};
                        for (int a = 0; a < DIM; ++a) gp[a] += cp * r[a];
                        for (int b = 0; b < DIM; ++b) {
                            const T cv = vol * (vjv[b] - vi[b]) * f;
                            for (int a = 0; a < DIM; ++a) gv[b][a] += cv * r[a];
                        }
                    }
                }
            }
            if (SL > 1) {
                lane_sum(divr, SL);
                for (int a = 0; a < DIM; ++a) {
                    lane_sum(sd[a], SL);
                    lane_sum(gp[a], SL);
                    for (int b = 0; b < DIM; ++b) lane_sum(gv[b][a], SL);
                }
            }
            if (!(divr < T(S.dim) - T(0.5)))  // not on the free surface
                for (int a = 0; a < DIM; ++a) del[a] = -0.5 * S.h * S.h * (double)sd[a];
            for (int a = 0; a < DIM; ++a) dpi += (double)gp[a] * del[a];
            for (int b = 0; b < DIM; ++b) {
                double acc = 0.0;
                for (int a = 0; a < DIM; ++a) acc += (double)gv[b][a] * del[a];
                dvi[b] = (T)acc;
            }
        }
        if (sub == 0) {
            for (int a = 0; a < 3; ++a) {
                A.dr[a * A.Nf + i] = del[a];
                A.dv[a * A.Nf + i] = dvi[a];
            }
            A.dp[i] = dpi;
            m2 = (del[0] * del[0] + del[1] * del[1]) + del[2] * del[2];
        }
    }
    for (int o = 32; o > 0; o >>= 1) m2 = fmax(m2, __shfl_xor(m2, o, 64));
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = m2;
    __syncthreads();
    if (threadIdx.x == 0) A.part[blockIdx.x] = fmax(fmax(lds[0], lds[1]), fmax(lds[2], lds[3]));
}

template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_shift_apply(ShiftArgs<T> A)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.Nf) return;
    const int N = A.N, Nf = A.Nf;
    // the particle's state first: in flight while the gate and the sim's
    // constants are read
    const int sid = A.simid[i];
    double xa[DIM], dra[DIM];
    T dva[DIM], vna[DIM], vda[DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        xa[a] = A.x[a * N + i];
        dra[a] = A.dr[a * Nf + i];
        dva[a] = A.dv[a * Nf + i];
        vna[a] = A.vn[a * Nf + i];
        vda[a] = A.vdiff[a * Nf + i];
    }
    const double pmi = A.pm[i], dpi = A.dp[i];
    if (A.gated && !spec_gate(A.n_sims, A.iters, A.sims)) return;
    const SimDev &S = A.sims[sid];
    if (!S.shift) return;
    double xo[3] = {0.0, 0.0, 0.0};
    T v[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        double xv = xa[a] + dra[a];
        if (S.periodic[a]) {
            if (xv >= S.hi[a]) xv -= S.L[a];
            else if (xv < S.lo[a]) xv += S.L[a];
        }
        A.x[a * N + i] = xv;
        xo[a] = xv;
        const T d = dva[a];
        v[a] = vna[a] + d;
        A.vn[a * Nf + i] = v[a];
        A.vdiff[a * Nf + i] = vda[a] + d;
    }
    const double p = pmi + dpi;
    A.pm[i] = p;
    if (DIM == 2) ((double2 *)A.xr)[i] = make_double2(xo[0], xo[1]);
    else ((double4 *)A.xr)[i] = make_double4(xo[0], xo[1], xo[2], 0.0);
    write_pos_record<T>(S, A.prec, i, xo);
    A.vrec[i] = make_rec<T, DIM>(v, (T)p);
}

// Largest shift of the launch into mapped memory (one workgroup).
__global__ void __launch_bounds__(256) k_shift_max(const double *__restrict__ part, int n, double *out, int gated,
                                                   int n_sims, const SimIter *__restrict__ iters,
                                                   const SimDev *__restrict__ sims)
{
    if (gated && !spec_gate(n_sims, iters, sims)) return;
    __shared__ double lds[4];
    double m = 0.0;
    for (int k = threadIdx.x; k < n; k += 256) m = fmax(m, part[k]);
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = sqrt(fmax(fmax(lds[0], lds[1]), fmax(lds[2], lds[3])));
}

template <typename T>
struct StateArgs {
    int N, Nf, Nw, in_loop, p_half;
    const SimDev *sims;
    int *flags;
    const int *init_slot, *init_sim;
    int *orig, *simid;
    double *x, *xn;
    T *vn, *dv, *w, *dp, *vw, *pw;
    double *pm, *pn;
    double *cx, *cv, *cvp, *cp, *cxi, *cvi, *cpi, *cdp;  // caller arrays
};

template <typename T>
__global__ void k_set_state(StateArgs<T> A)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= A.N) return;
    const int N = A.N, Nf = A.Nf, Nw = A.Nw;
    const int i = A.init_slot[c];
    A.orig[i] = c;
    A.simid[i] = A.init_sim[c];
    const bool lp = A.in_loop != 0;
    const SimDev &S = A.sims[A.init_sim[c]];
    bool outside = false;  // positions on periodic axes must lie in [lo, hi)
    for (int d = 0; d < S.dim; ++d) {
        if (!S.periodic[d]) continue;
        const double a = A.cx[3 * c + d], b = lp ? A.cxi[3 * c + d] : a;
        outside = outside || !(a >= S.lo[d] && a < S.hi[d]) || !(b >= S.lo[d] && b < S.hi[d]);
    }
    if (outside) atomicOr(&A.flags[F_OUTSIDE], 1);
    for (int d = 0; d < 3; ++d) {
        A.x[d * N + i] = lp ? A.cxi[3 * c + d] : A.cx[3 * c + d];
        A.xn[d * N + i] = A.cx[3 * c + d];
    }
    if (i < Nf) {
        for (int d = 0; d < 3; ++d) {
            const double v = A.cv[3 * c + d];
            A.vn[d * Nf + i] = (T)v;
            A.dv[d * Nf + i] = (T)(v - A.cvp[3 * c + d]);
            A.w[d * Nf + i] = lp ? (T)(A.cvi[3 * c + d] - v) : T(0);
        }
        A.pn[i] = A.cp[c];
        A.pm[i] = lp ? A.cpi[c] : A.cp[c];
        A.dp[i] = lp ? (T)A.cdp[c] : T(0);
    } else {
        const int iw = i - Nf;
        for (int d = 0; d < 3; ++d) A.vw[d * Nw + iw] = (T)A.cv[3 * c + d];
        A.pw[iw] = T(0);
    }
}

template <typename T>
__global__ void k_get_state(StateArgs<T> A)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.N) return;
    const int N = A.N, Nf = A.Nf, Nw = A.Nw;
    const int c = A.orig[i];
    const bool lp = A.in_loop != 0;
    for (int d = 0; d < 3; ++d) {
        const double xa = A.x[d * N + i];
        if (A.cx) A.cx[3 * c + d] = (lp && i < Nf) ? A.xn[d * N + i] : xa;
        if (A.cxi) A.cxi[3 * c + d] = xa;
    }
    if (i < Nf) {
        for (int d = 0; d < 3; ++d) {
            const T vn = A.vn[d * Nf + i];
            if (A.cv) A.cv[3 * c + d] = (double)vn;
            if (A.cvp) A.cvp[3 * c + d] = (double)(vn - A.dv[d * Nf + i]);
            if (A.cvi) A.cvi[3 * c + d] = (double)(vn + A.w[d * Nf + i]);
        }
        if (A.cp) A.cp[c] = lp ? A.pn[i] : A.pm[i];
        if (A.cpi) A.cpi[c] = A.p_half ? A.pm[i] - 0.5 * A.sims[A.simid[i]].dtau * (double)A.dp[i] : A.pm[i];
        if (A.cdp) A.cdp[c] = (double)A.dp[i];
    } else {
        const int iw = i - Nf;
        for (int d = 0; d < 3; ++d) {
            const double v = (double)A.vw[d * Nw + iw];
            if (A.cv) A.cv[3 * c + d] = v;
            if (A.cvp) A.cvp[3 * c + d] = 0.0;
            if (A.cvi) A.cvi[3 * c + d] = v;
        }
        if (A.cp) A.cp[c] = (double)A.pw[iw];
        if (A.cpi) A.cpi[c] = (double)A.pw[iw];
        if (A.cdp) A.cdp[c] = 0.0;
    }
}

inline int grid_for(int n, int b = 256) { return n > 0 ? ceil_div(n, b) : 1; }


// A timed pair pass goes through hipExtLaunchKernelGGL, whose events take the
// kernel's own start and end timestamps (no queue gaps in the interval).
// Pseudo-iterations of a context with steady sims take the variant with the
// convective sum (zero coefficient for the time-accurate sims).
template <typename T, int DIM, bool WALLS, bool AV, bool SEPDEN, int LPP, bool CONV, int CACHE, bool MOVE = false>
void launch_pseudo(Ctx &c, const PassArgs<T> &a, dim3 grid)
{
    if (c.ext_start)
        hipExtLaunchKernelGGL((k_pass<T, DIM, WALLS, AV, SEPDEN, MODE_PSEUDO, LPP, CONV, CACHE, MOVE>), grid,
                              dim3(c.block), 0, c.stream, c.ext_start, c.ext_stop, 0, a);
    else
        DTSPH_LAUNCH(c, (k_pass<T, DIM, WALLS, AV, SEPDEN, MODE_PSEUDO, LPP, CONV, CACHE, MOVE>), grid,
                     dim3(c.block), 0, c.stream, a);
}

// Cached pair coefficients hold one regulariser: contexts with separate EDAC
// or artificial-viscosity regularisers always recompute.
template <typename T, int DIM, bool WALLS, bool AV, bool SEPDEN, int LPP, bool CONV>
void dispatch_pseudo(Ctx &c, const PassArgs<T> &a, dim3 grid)
{
    if (SEPDEN || c.cache_phase == 0) launch_pseudo<T, DIM, WALLS, AV, SEPDEN, LPP, CONV, 0>(c, a, grid);
    else if (c.cache_phase == 1) launch_pseudo<T, DIM, WALLS, AV, false, LPP, CONV, 1>(c, a, grid);
    else launch_pseudo<T, DIM, WALLS, AV, false, LPP, CONV, 2>(c, a, grid);
}

template <typename T, int DIM, bool WALLS, bool AV, bool SEPDEN, int LPP>
void dispatch_mode(Ctx &c, int mode, const PassArgs<T> &a, dim3 grid)
{
    if (mode == MODE_PRE)
        DTSPH_LAUNCH(c, (k_pass<T, DIM, WALLS, AV, SEPDEN, MODE_PRE, LPP, false>), grid, dim3(c.block), 0, c.stream,
                     a);
    else if (c.any_move)  // moving particles: advective sums, no coefficient cache
        launch_pseudo<T, DIM, WALLS, AV, SEPDEN, LPP, true, 0, true>(c, a, grid);
    else if (c.any_steady)
        dispatch_pseudo<T, DIM, WALLS, AV, SEPDEN, LPP, true>(c, a, grid);
    else
        dispatch_pseudo<T, DIM, WALLS, AV, SEPDEN, LPP, false>(c, a, grid);
}

template <typename T, int DIM, bool WALLS, bool AV, bool SEPDEN>
void dispatch_lpp(Ctx &c, int mode, const PassArgs<T> &a, dim3 grid)
{
    switch (c.lpp) {
    case 1: dispatch_mode<T, DIM, WALLS, AV, SEPDEN, 1>(c, mode, a, grid); break;
    case 2: dispatch_mode<T, DIM, WALLS, AV, SEPDEN, 2>(c, mode, a, grid); break;
    case 4: dispatch_mode<T, DIM, WALLS, AV, SEPDEN, 4>(c, mode, a, grid); break;
    default: dispatch_mode<T, DIM, WALLS, AV, SEPDEN, 8>(c, mode, a, grid); break;
    }
}

template <typename T, int DIM, bool WALLS, bool AV>
void dispatch_sep(Ctx &c, int mode, const PassArgs<T> &a, dim3 grid)
{
    if (c.sep_den) dispatch_lpp<T, DIM, WALLS, AV, true>(c, mode, a, grid);
    else dispatch_lpp<T, DIM, WALLS, AV, false>(c, mode, a, grid);
}

template <typename T, int DIM, bool WALLS>
void dispatch_av(Ctx &c, int mode, const PassArgs<T> &a, dim3 grid)
{
    if (c.any_av) dispatch_sep<T, DIM, WALLS, true>(c, mode, a, grid);
    else dispatch_sep<T, DIM, WALLS, false>(c, mode, a, grid);
}

template <typename T, int DIM>
void dispatch_walls(Ctx &c, int mode, const PassArgs<T> &a, dim3 grid)
{
    if (c.any_walls) dispatch_av<T, DIM, true>(c, mode, a, grid);
    else dispatch_av<T, DIM, false>(c, mode, a, grid);
}

}  // namespace

template <typename T>
void launch_pass(Ctx &c, int mode, bool cand_lists)
{
    PassArgs<T> a = pass_args<T>(c, mode, cand_lists);
    if (a.n_tiles == 0) return;
    const int grid = c.xcd_remap ? 8 * ((a.n_tiles + 7) / 8) : a.n_tiles;
    const int t0 = mode == MODE_PSEUDO ? timer_slot(c, 0) : -1;
    if (t0 >= 0) {
        c.ext_start = c.ev_pool[t0];
        c.ext_stop = c.ev_pool[t0 + 1];
    }
    if (c.max_dim == 2) dispatch_walls<T, 2>(c, mode, a, dim3(grid));
    else dispatch_walls<T, 3>(c, mode, a, dim3(grid));
    c.ext_start = c.ext_stop = nullptr;
    DTSPH_HIP_CHECK(hipGetLastError());
    timer_book(c, t0, 0);
}


template <typename T>
void launch_wall(Ctx &c, int mode, bool cand_lists)
{
    if (c.Nw == 0) return;
    const WallArgs<T> a = wall_args<T>(c, mode, cand_lists);
    int t0 = mode == MODE_PSEUDO ? timer_begin(c, 1) : -1;
    if (c.max_dim == 2) DTSPH_LAUNCH(c, (k_wall<T, 2>), dim3(grid_for(c.Nw)), dim3(256), 0, c.stream, a);
    else DTSPH_LAUNCH(c, (k_wall<T, 3>), dim3(grid_for(c.Nw)), dim3(256), 0, c.stream, a);
    DTSPH_HIP_CHECK(hipGetLastError());
    if (mode == MODE_PSEUDO) timer_end(c, t0, 1);
}

void launch_gate(Ctx &c)
{
    DTSPH_LAUNCH(c, k_gate, dim3(1), dim3(256), 0, c.stream, c.n_sims, c.iters, c.sims);
    DTSPH_HIP_CHECK(hipGetLastError());
}

void launch_publish(Ctx &c)
{
    const int n = F_COUNT + c.n_sims;
    DTSPH_LAUNCH(c, k_publish, dim3(grid_for(n)), dim3(256), 0, c.stream, c.n_sims, c.flags, c.iters,
                       c.m_flags_d, c.m_reps_d, c.m_pairs_d);
    DTSPH_HIP_CHECK(hipGetLastError());
}


void launch_finalize(Ctx &c, bool publish)
{
    const FinArgs a = fin_args(c, publish);
    DTSPH_LAUNCH(c, k_finalize, dim3(c.n_segs), dim3(kFinThreads), 0, c.stream, a);
    DTSPH_HIP_CHECK(hipGetLastError());
}

template <typename T>
void launch_finalize_wall(Ctx &c, bool publish, int next)
{
    const FinArgs f = fin_args(c, publish);
    const WallArgs<T> w = wall_args<T>(c, MODE_PSEUDO, false);
    const dim3 grid(c.n_segs + ceil_div(c.Nw, kFinThreads));
    if (c.max_dim == 2) DTSPH_LAUNCH(c, (k_finalize_wall<T, 2>), grid, dim3(kFinThreads), 0, c.stream, f, w, c.n_segs, next);
    else DTSPH_LAUNCH(c, (k_finalize_wall<T, 3>), grid, dim3(kFinThreads), 0, c.stream, f, w, c.n_segs, next);
    DTSPH_HIP_CHECK(hipGetLastError());
}

template <typename T>
void launch_wall_pressure(Ctx &c)
{
    using Q = typename V4<T>::type;
    const int b = c.buf;
    DTSPH_LAUNCH(c, k_wall_pressure<T>, dim3(grid_for(c.Nw)), dim3(256), 0, c.stream, c.Nw, c.Nf, c.simid[b], c.iters,
                 (const Q *)c.vp[0], (const Q *)c.vp[1], c.cur, c.max_dim, (T *)c.pw[b]);
    DTSPH_HIP_CHECK(hipGetLastError());
}

template <typename T>
void launch_pre_records(Ctx &c)
{
    using Q = typename V4<T>::type;
    const int b = c.buf;
    if (c.max_dim == 2)
        DTSPH_LAUNCH(c, (k_records<T, 2>), dim3(grid_for(c.Nf)), dim3(256), 0, c.stream, c.Nf, c.simid[b], c.sims,
                           (const T *)c.vn[b], (const T *)nullptr, c.pm[b], (const T *)c.dp[b], (Q *)c.vp[c.cur], 0,
                           0, c.iters, c.n_sims, 0);
    else
        DTSPH_LAUNCH(c, (k_records<T, 3>), dim3(grid_for(c.Nf)), dim3(256), 0, c.stream, c.Nf, c.simid[b], c.sims,
                           (const T *)c.vn[b], (const T *)nullptr, c.pm[b], (const T *)c.dp[b], (Q *)c.vp[c.cur], 0,
                           0, c.iters, c.n_sims, 0);
    DTSPH_HIP_CHECK(hipGetLastError());
}

// Loop start of sims moving in pseudo-time (Algorithm 1): r^{1/2} = r^(0),
// Vtilde^0 = 0, and the second position-record buffer equal to the first (wall
// and frozen entries are only ever read there).
template <typename T, int DIM>
__global__ void k_move_begin(int N, int Nf, const int *__restrict__ simid, const SimDev *__restrict__ sims,
                             const double *__restrict__ x, const void *__restrict__ prec, void *__restrict__ prec2,
                             double *__restrict__ xm, T *__restrict__ vt)
{
    using Rec = typename Pos<T, DIM>::Rec;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    ((Rec *)prec2)[i] = ((const Rec *)prec)[i];
    if (i < Nf && sims[simid[i]].move)
        for (int d = 0; d < DIM; ++d) {
            xm[d * Nf + i] = x[d * N + i];
            vt[d * Nf + i] = T(0);
        }
}

template <typename T>
void launch_move_begin(Ctx &c)
{
    if (!c.any_move) return;
    const int b = c.buf;
    if (c.max_dim == 2)
        DTSPH_LAUNCH(c, (k_move_begin<T, 2>), dim3(grid_for(c.N)), dim3(256), 0, c.stream, c.N, c.Nf, c.simid[b],
                     c.sims, c.x[c.xb], c.prec, c.prec2, c.xm, (T *)c.vt);
    else
        DTSPH_LAUNCH(c, (k_move_begin<T, 3>), dim3(grid_for(c.N)), dim3(256), 0, c.stream, c.N, c.Nf, c.simid[b],
                     c.sims, c.x[c.xb], c.prec, c.prec2, c.xm, (T *)c.vt);
    DTSPH_HIP_CHECK(hipGetLastError());
}

template <typename T>
void launch_loop_begin(Ctx &c, int fixed_iters)
{
    using Q = typename V4<T>::type;
    const int b = c.buf;
    if (c.max_dim == 2)
        DTSPH_LAUNCH(c, (k_records<T, 2>), dim3(grid_for(c.Nf)), dim3(256), 0, c.stream, c.Nf, c.simid[b], c.sims,
                           (const T *)c.vn[b], (const T *)c.w[b], c.pm[b], (const T *)c.dp[b], (Q *)c.vp[c.cur], 1,
                           c.p_half ? 0 : 1, c.iters, c.n_sims, fixed_iters);
    else
        DTSPH_LAUNCH(c, (k_records<T, 3>), dim3(grid_for(c.Nf)), dim3(256), 0, c.stream, c.Nf, c.simid[b], c.sims,
                           (const T *)c.vn[b], (const T *)c.w[b], c.pm[b], (const T *)c.dp[b], (Q *)c.vp[c.cur], 1,
                           c.p_half ? 0 : 1, c.iters, c.n_sims, fixed_iters);
    DTSPH_HIP_CHECK(hipGetLastError());
}

template <typename T>
void launch_correct(Ctx &c)
{
    const int b = c.buf;
    using Q = typename V4<T>::type;
    auto kern = c.max_dim == 2 ? k_correct<T, 2> : k_correct<T, 3>;
    DTSPH_LAUNCH(c, kern, dim3(grid_for(c.Nf)), dim3(256), 0, c.stream, c.N, c.Nf, c.simid[b], c.sims,
                       c.x[c.xb], c.xn[b], (T *)c.vn[b], (T *)c.dv[b], (T *)c.w[b], c.xr, c.pm[b],
                       (const T *)c.dp[b], c.p_half ? 1 : 0, c.prec, (Q *)c.vp[c.cur], c.gated ? 1 : 0, c.n_sims,
                       c.iters);
    DTSPH_HIP_CHECK(hipGetLastError());
}

template <typename T>
void launch_shift(Ctx &c, bool cand_lists)
{
    using Q = typename V4<T>::type;
    const int b = c.buf;
    ShiftArgs<T> a;
    a.N = c.N; a.Nf = c.Nf; a.Nw = c.Nw;
    a.simid = c.simid[b]; a.sims = c.sims;
    a.nbr = cand_lists ? c.cand : c.nbr;
    a.cnt = cand_lists ? c.ccnt : c.cnt;
    a.prec = c.prec;
    a.vrec = (Q *)c.vp[c.cur];
    a.dr = c.sh_dr; a.dp = c.sh_dp; a.dv = (T *)c.sh_dv; a.part = c.sh_part;
    a.x = c.x[c.xb]; a.xr = c.xr;
    a.vn = (T *)c.vn[b]; a.vdiff = (T *)c.dv[b]; a.pm = c.pm[b];
    a.gated = c.gated ? 1 : 0; a.n_sims = c.n_sims; a.iters = c.iters;
    // lanes per particle: 4 for the ~110 neighbours of 3D, 2 for the ~26 of 2D
    const int nblk = grid_for(c.Nf), nsum = grid_for(c.Nf * (c.max_dim == 2 ? 2 : 4));
    if (c.max_dim == 2) {
        DTSPH_LAUNCH(c, (k_shift_sums<T, 2, 2>), dim3(nsum), dim3(256), 0, c.stream, a);
        DTSPH_LAUNCH(c, (k_shift_apply<T, 2>), dim3(nblk), dim3(256), 0, c.stream, a);
    } else {
        DTSPH_LAUNCH(c, (k_shift_sums<T, 3, 4>), dim3(nsum), dim3(256), 0, c.stream, a);
        DTSPH_LAUNCH(c, (k_shift_apply<T, 3>), dim3(nblk), dim3(256), 0, c.stream, a);
    }
    DTSPH_LAUNCH(c, k_shift_max, dim3(1), dim3(256), 0, c.stream, c.sh_part, nsum, c.sh_max_d, c.gated ? 1 : 0,
                 c.n_sims, c.iters, c.sims);
    DTSPH_HIP_CHECK(hipGetLastError());
}

template <typename T>
static StateArgs<T> state_args(Ctx &c, const dtsph_state_view &s, bool in_loop)
{
    const int b = c.buf;
    StateArgs<T> a;
    a.N = c.N; a.Nf = c.Nf; a.Nw = c.Nw; a.in_loop = in_loop ? 1 : 0;
    a.p_half = in_loop && c.p_half ? 1 : 0;
    a.sims = c.sims;
    a.flags = c.flags;
    a.init_slot = c.init_slot; a.init_sim = c.init_slot + c.N;
    a.orig = c.orig[b]; a.simid = c.simid[b];
    a.x = c.x[c.xb]; a.xn = c.xn[b];
    a.vn = (T *)c.vn[b]; a.dv = (T *)c.dv[b]; a.w = (T *)c.w[b]; a.dp = (T *)c.dp[b];
    a.vw = (T *)c.vw[b]; a.pw = (T *)c.pw[b];
    a.pm = c.pm[b]; a.pn = c.pn[b];
    a.cx = s.x; a.cv = s.v; a.cvp = s.v_prev; a.cp = s.p;
    a.cxi = s.x_iter; a.cvi = s.v_iter; a.cpi = s.p_iter; a.cdp = s.dpdtau;
    return a;
}

template <typename T>
void launch_set_state(Ctx &c, const dtsph_state_view &s, bool in_loop)
{
    StateArgs<T> a = state_args<T>(c, s, in_loop);
    DTSPH_LAUNCH(c, k_set_state<T>, dim3(grid_for(c.N)), dim3(256), 0, c.stream, a);
    DTSPH_HIP_CHECK(hipGetLastError());
}

template <typename T>
void launch_get_state(Ctx &c, const dtsph_state_view &s, bool in_loop)
{
    StateArgs<T> a = state_args<T>(c, s, in_loop);
    DTSPH_LAUNCH(c, k_get_state<T>, dim3(grid_for(c.N)), dim3(256), 0, c.stream, a);
    DTSPH_HIP_CHECK(hipGetLastError());
}

#define DTSPH_INSTANTIATE(T)                                                   \
    template void launch_pass<T>(Ctx &, int, bool);                            \
    template void launch_wall<T>(Ctx &, int, bool);                            \
    template void launch_finalize_wall<T>(Ctx &, bool, int);                   \
    template void launch_wall_pressure<T>(Ctx &);                              \
    template void launch_pre_records<T>(Ctx &);                                \
    template void launch_loop_begin<T>(Ctx &, int);                            \
    template void launch_move_begin<T>(Ctx &);                                 \
    template void launch_correct<T>(Ctx &);                                    \
    template void launch_shift<T>(Ctx &, bool);                                \
    template void launch_set_state<T>(Ctx &, const dtsph_state_view &, bool);  \
    template void launch_get_state<T>(Ctx &, const dtsph_state_view &, bool);
DTSPH_INSTANTIATE(float)
DTSPH_INSTANTIATE(double)

}  // namespace dtsph
