// Device code of the pair passes of the frozen-particle dual-time EDAC SPH step
// (pair pass, wall pass, residual reduction), shared by the plain launches and
// the persistent tail launch. Everything sits in an anonymous namespace: each
// source that includes it compiles its own copies.
//
// Pair passes:
//
// k_pass (the hot kernel) evaluates, for every fluid particle i over its exact
// neighbour list (paper section 3.2):
//   D_i = sum_j (m rho_i/rho_j) c^2 V_ij . gradW_ij
//       + sum_j 4 m/(rho_i+rho_j) nu_e p_ij gradW_ij . r_ij / (r^2 + reg_e)
//                                                      (eq. dp-dtau-frozen-edac)
//   R_i = -sum_j m (p_i/rho^2 + p_j/rho^2 + Pi_ij) gradW_ij
//       + sum_j m 4 nu gradW_ij . r_ij / ((rho_i+rho_j)(r^2 + eta h^2)) V_ij + g
//                                                      (eq. mom-sph-frozen,
//                                                       eq. mom-av, eq. av-phiij)
// With the quintic spline, dW/dr = kg * poly(q), poly = (3-q)^4 - 6(2-q)^4 +
// 15(1-q)^4 (terms clipped at zero), kg = -5 sigma / h, so per pair
//   gradW = kg * G * r_vec with G = poly / r,
//   gradW . r / (r^2 + reg) = kg * poly * r / (r^2 + reg),
// and all constant factors move out of the sums. The density is uniform.
//
// MODE_PSEUDO fuses the pseudo-time update (eqs. pkstar_frozen, vkp1_frozen,
// pkp1_frozen with the frozen eq. dv_dtau_exact) and the per-block float64
// residual partials of eq. conv. MODE_PRE is the rate pass before the loop
// fused with the predictor (eq. v0, eq. r0).
//
// Work distribution: one thread per fluid particle; a workgroup is a "tile" of
// consecutive cell-ordered slots of one sim (tiles never straddle sims, so each
// sim's residual is a fixed-order sum of its own partials and a batch member
// computes bit-for-bit what it computes alone). Consecutive tiles are mapped to
// the same XCD so that neighbouring tiles share that XCD's L2.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "dtsph_internal.h"

namespace dtsph {

namespace {

template <typename T> struct V4;
template <> struct V4<float> { using type = float4; };
template <> struct V4<double> { using type = double4; };

template <typename T> __device__ inline T rsq(T x);
template <> __device__ inline float rsq<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <> __device__ inline double rsq<double>(double x) { return 1.0 / sqrt(x); }
template <typename T> __device__ inline T rcp(T x);
template <> __device__ inline float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ inline double rcp<double>(double x) { return 1.0 / x; }

// component access of the {V, p} record: 2D {vx, vy, p, -}, 3D {vx, vy, vz, p}
template <typename Q> __device__ inline auto comp(const Q &v, int k) { return k == 0 ? v.x : k == 1 ? v.y : k == 2 ? v.z : v.w; }

template <int DIM, typename Q> __device__ inline auto pres(const Q &v) { return DIM == 2 ? v.z : v.w; }

template <typename T, int DIM> __device__ inline typename V4<T>::type make_rec(const T v[3], T p)
{
    typename V4<T>::type r;
    r.x = v[0];
    r.y = v[1];
    if (DIM == 2) { r.z = p; r.w = T(0); }
    else { r.z = v[2]; r.w = p; }
    return r;
}

// Position records and separations r_i - r_j. In 2D a record is two words
// (8 B in FP32, 16 B in FP64), so a gather touches half as many cache lines.
template <typename T, int DIM> struct Pos;

template <int DIM> struct Pos<float, DIM> {
    using Rec = typename std::conditional<DIM == 2, uint2, uint4>::type;
    float step[3];
    __device__ explicit Pos(const SimDev &S)
    {
        for (int a = 0; a < 3; ++a) step[a] = (float)(S.q_len[a] * 0x1p-32);
    }
    __device__ inline void delta(const Rec &a, const Rec &b, float r[3]) const
    {
        r[0] = (float)(int)(a.x - b.x) * step[0];
        r[1] = (float)(int)(a.y - b.y) * step[1];
        if constexpr (DIM == 3) r[2] = (float)(int)(a.z - b.z) * step[2];
        else r[2] = 0.0f;
    }
};

template <int DIM> struct Pos<double, DIM> {
    using Rec = typename std::conditional<DIM == 2, double2, double4>::type;
    double L[3], halfL[3];
    int per[3];
    __device__ explicit Pos(const SimDev &S)
    {
        for (int a = 0; a < 3; ++a) { L[a] = S.L[a]; halfL[a] = S.halfL[a]; per[a] = S.periodic[a]; }
    }
    __device__ inline double mi(double s, int a) const
    {
        if (per[a]) {
            if (s > halfL[a]) s -= L[a];
            else if (s < -halfL[a]) s += L[a];
        }
        return s;
    }
    __device__ inline void delta(const Rec &a, const Rec &b, double r[3]) const
    {
        r[0] = mi(a.x - b.x, 0);
        r[1] = mi(a.y - b.y, 1);
        if constexpr (DIM == 3) r[2] = mi(a.z - b.z, 2);
        else r[2] = 0.0;
    }
};

// Gate of the speculative end of step, evaluated by each gated workgroup from
// the loop states: every sim stopped without a non-finite residual and every
// sim's candidate lists still hold all neighbours at r^{n+1} (the rule the host
// applies to the same, published, values).
__device__ inline bool spec_gate(int n_sims, const SimIter *__restrict__ iters, const SimDev *__restrict__ sims)
{
    (void)sims;
    return iters[n_sims].done != 0;  // evaluated once by k_gate before the gated launches
}

// The speculative gate, once per speculative end of step (one workgroup,
// before the gated launches): every sim stopped, no non-finite residual, and
// the candidate lists still cover r^{n+1}. Written to the loop-state slot after
// the sims' own (a word each gated workgroup reads instead of every sim's state).
__global__ void __launch_bounds__(256) k_gate(int n_sims, SimIter *__restrict__ iters, const SimDev *__restrict__ sims)
{
    __shared__ int ok;
    if (threadIdx.x == 0) ok = 1;
    __syncthreads();
    for (int s = threadIdx.x; s < n_sims; s += blockDim.x) {
        const SimIter &It = iters[s];
        if (!(It.done && It.reason != DTSPH_NONFINITE && sims[s].skin > 0 && It.disp < 0.4 * sims[s].skin))
            atomicAnd(&ok, 0);
    }
    __syncthreads();
    if (threadIdx.x == 0) iters[n_sims].done = ok;
}

template <typename T> struct PassConst {
    T inv_h, tiny, den_v, den_e, den_a, k_av;
    __device__ explicit PassConst(const SimDev &S)
        : inv_h((T)S.inv_h), tiny((T)S.tiny_r2), den_v((T)S.den_v), den_e((T)S.den_e),
          den_a((T)S.den_a), k_av((T)S.k_av) {}
};

// Cached artificial-viscosity factor per list entry: r_ij / (r^2 + eps h^2).
template <typename T, int DIM> struct AvC { using type = typename V4<T>::type; };
template <> struct AvC<float, 2> { using type = float2; };
template <> struct AvC<double, 2> { using type = double2; };

template <typename T> struct Acc {
    T div = 0, lap = 0, grad[3] = {0, 0, 0}, vis[3] = {0, 0, 0}, conv[3] = {0, 0, 0}, padv = 0;
};

// One neighbour's contribution. vd: V_ij for the divergence term; vv: V_ij for
// the viscous and artificial-viscosity terms (they differ only for walls).
// CONV adds the advective sums (a . gradW)(V_i + V_j) and (a . gradW)(p_i + p_j)
// with V_j = V_i - vv (a wall's ghost velocity): a = V_i for the convective
// term of eq. mom-steady, a = Vtilde_i for eq. discrete_ME and eq. dp-dtau.
// With CACHE_OUT the pair's geometric coefficients {G r_ij, F_ij} (see
// pair_cached) are stored at `out`, with artificial viscosity also
// r_ij / (r^2 + eps h^2) at `out_av`.
template <typename T, int DIM, bool AV, bool SEPDEN, bool CONV, bool CACHE_OUT = false>
__device__ __forceinline__ void pair_terms(const PassConst<T> &K, const T r[3], const T vd[3], const T vv[3],
                                           const T vi[3], const T av[3], T pi, T pj, Acc<T> &acc,
                                           typename V4<T>::type *out = nullptr,
                                           typename AvC<T, DIM>::type *out_av = nullptr)
{
    T r2 = r[0] * r[0] + r[1] * r[1];
    if (DIM == 3) r2 += r[2] * r[2];
    const T r2s = r2 > K.tiny ? r2 : K.tiny;
    const T rinv = rsq<T>(r2s);
    const T rr = r2s * rinv;
    const T q = rr * K.inv_h;
    T t3 = T(3) - q, t2 = T(2) - q, t1 = T(1) - q;
    t3 = t3 > T(0) ? t3 : T(0);
    t2 = t2 > T(0) ? t2 : T(0);
    t1 = t1 > T(0) ? t1 : T(0);
    T a = t3 * t3, b = t2 * t2, c = t1 * t1;
    a *= a;
    b *= b;
    c *= c;
    const T poly = T(15) * c + (T(-6) * b + a);
    const T G = poly * rinv;
    const T rden = rcp<T>(r2 + K.den_v);
    const T pr = poly * rr;
    const T Fv = pr * rden;
    const T Fe = SEPDEN ? pr * rcp<T>(r2 + K.den_e) : Fv;
    T dotd = vd[0] * r[0] + vd[1] * r[1];
    if (DIM == 3) dotd += vd[2] * r[2];
    acc.div += G * dotd;
    acc.lap += Fe * (pi - pj);
    T P = pi + pj;
    T sG = 0;
    if (CONV) {
        T dvi = av[0] * r[0] + av[1] * r[1];
        if (DIM == 3) dvi += av[2] * r[2];
        sG = G * dvi;
        acc.padv += sG * P;
    }
    if (AV) {
        T dotv = vv[0] * r[0] + vv[1] * r[1];
        if (DIM == 3) dotv += vv[2] * r[2];
        const T phi = dotv * (SEPDEN ? rcp<T>(r2 + K.den_a) : rden);
        P += K.k_av * (phi < T(0) ? phi : T(0));
    }
    const T PG = P * G;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        acc.vis[d] += Fv * vv[d];
        acc.grad[d] += PG * r[d];
    }
    if (CONV) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) acc.conv[d] += sG * (T(2) * vi[d] - vv[d]);
    }
    if (CACHE_OUT) {
        typename V4<T>::type c;
        c.x = G * r[0];
        c.y = G * r[1];
        c.z = DIM == 3 ? G * r[2] : T(0);
        c.w = Fv;
        *out = c;
        if (AV) {
            typename AvC<T, DIM>::type u;
            u.x = r[0] * rden;
            u.y = r[1] * rden;
            if constexpr (DIM == 3) {
                u.z = r[2] * rden;
                u.w = T(0);
            }
            *out_av = u;
        }
    }
}

// One neighbour's contribution from cached coefficients (the performance part of
// section 4 suggests caching kernel values in pseudo-time): c = {G r_ij, F_ij} with
// kernel factor G = poly / r and F_ij = poly r / (r^2 + eta h^2). Only for
// sims with a single regulariser (eta h^2 for the viscous, EDAC and
// artificial-viscosity terms), where these and u = r_ij / (r^2 + eta h^2)
// carry every geometric factor of the pass.
template <typename T, int DIM, bool AV, bool CONV>
__device__ __forceinline__ void pair_cached(const PassConst<T> &K, const typename V4<T>::type &c,
                                            const typename AvC<T, DIM>::type &u, const T vd[3], const T vv[3],
                                            const T vi[3], const T av[3], T pi, T pj, Acc<T> &acc)
{
    const T g[3] = {c.x, c.y, c.z};
    T dotd = vd[0] * g[0] + vd[1] * g[1];
    if (DIM == 3) dotd += vd[2] * g[2];
    acc.div += dotd;
    acc.lap += c.w * (pi - pj);
    T P = pi + pj;
    T sG = 0;
    if (CONV) {
        sG = av[0] * g[0] + av[1] * g[1];
        if (DIM == 3) sG += av[2] * g[2];
        acc.padv += sG * P;
    }
    if (AV) {
        T phi = vv[0] * u.x + vv[1] * u.y;
        if constexpr (DIM == 3) phi += vv[2] * u.z;
        P += K.k_av * (phi < T(0) ? phi : T(0));
    }
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        acc.vis[d] += c.w * vv[d];
        acc.grad[d] += P * g[d];
    }
    if (CONV) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) acc.conv[d] += sG * (T(2) * vi[d] - vv[d]);
    }
}

__device__ inline int tile_of_block(int n_tiles, int remap)
{
    const int b = blockIdx.x;
    if (!remap) return b < n_tiles ? b : -1;
    const int per = (n_tiles + 7) >> 3;
    const int t = (b & 7) * per + (b >> 3);
    return t < n_tiles ? t : -1;
}

template <typename T> struct PassArgs {
    using Q = typename V4<T>::type;
    int N, Nf, Nw, n_tiles, remap;  // n_tiles: tiles this launch covers
    int cur, n_ranges;
    // when n_ranges > 0 the launch covers only these tile ranges (sims whose loop
    // is still running): (first tile, index of that tile within the launch)
    int2 ranges[kMaxRanges];
    const int2 *tiles;
    const SimDev *sims;
    const SimIter *iters;
    const int *nbr;
    const uint32_t *cnt;
    const void *prec;
    Q *vp0, *vp1;   // {V, p} records, ping-ponged per sim
    const T *vwall;
    const T *vn, *dv;
    T *w, *w0, *dp;
    double *pm, *pn;
    const double *x;
    double *x_alt, *xn;
    double4 *partials;
    double2 *partials2;   // per tile: {max |V^{k+1} - V^(0)|^2, neighbour pairs}
    Q *coef;              // cached pair coefficients, entry k of slot i at k*N + i
    void *coef_av;        // cached artificial-viscosity factors, same layout
    // particles moving in pseudo-time: second position-record buffer, r^{k+1/2}
    // and Vtilde^k of the fluid, packed positions for the list filter, flags
    void *prec2;
    double *xm;
    T *vt;
    void *xr;
    int *flags;
    int gated, n_sims;  // gated: run only if spec_gate holds (speculative launch)
};

template <typename T> __device__ inline int launch_tile(const PassArgs<T> &A, int v)
{
    if (A.n_ranges == 0) return v;
    int first = A.ranges[0].x, at = A.ranges[0].y;
#pragma unroll
    for (int q = 1; q < kMaxRanges; ++q) {  // static indices: kernel-argument loads
        const bool take = q < A.n_ranges && A.ranges[q].y <= v;
        first = take ? A.ranges[q].x : first;
        at = take ? A.ranges[q].y : at;
    }
    return first + (v - at);
}

template <typename T> __device__ inline void lane_sum(T &v, int lpp)
{
    for (int o = lpp >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
}

// LPP lanes share one particle: lane `sub` takes neighbour entries sub, sub+LPP,
// ... and the partial sums are combined with butterfly shuffles, so that small
// problems still put enough waves on every SIMD to hide the gather latency.
// Occupancy target (waves per SIMD) of the pair pass: the gathers are latency
// bound, so the register budget is capped where that costs no spills.
template <typename T, int DIM, bool HEAVY> struct PassWaves {
    static constexpr int value = sizeof(T) == 4 ? (DIM == 2 ? 6 : 4) : (DIM == 2 && !HEAVY ? 5 : 4);
};

// CACHE (pseudo-iterations): 0 recompute every pair's geometry; 1 recompute and
// store {G r_ij, F_ij} per list entry (first iteration of a loop); 2 read them
// back instead of the position records. MOVE (with CONV): sims with particles
// moving in pseudo-time read the position records of their iteration's parity,
// add the advective terms with Vtilde^k and write r^{k+3/2} to the other buffer.
// Tile t of a pair pass (the whole workgroup; one tile per call). Record
// buffers: the rate pass reads buffer `cur`; iteration k of sim s reads buffer
// par = (cur + k) & 1 and writes the other (ppar = k & 1 picks the position
// records of moving sims), so a sim whose loop has stopped simply drops out.
// The tile's record tl = tiles[t] and its sim's constants S are the caller's
// (a persistent caller keeps them on chip); the tile's residual partials go to
// part4[t], part2[t]. With PRED (latency-bound callers) a list's last partial
// batch is issued at once, slots past the list masked, instead of one neighbour
// after the other; the sums are the same, in the same order.
template <typename T, int DIM, bool WALLS, bool AV, bool SEPDEN, int MODE, int LPP, bool CONV, int CACHE, bool MOVE,
          bool PRED = false>
__device__ __forceinline__ void pass_tile_at(const PassArgs<T> &A, const SimDev &S, int t, int2 tl, int par, int ppar,
                                             double4 *__restrict__ part4, double2 *__restrict__ part2)
{
    using Q = typename V4<T>::type;
    using PosT = Pos<T, DIM>;
    using Rec = typename PosT::Rec;
    const int sub = (int)threadIdx.x & (LPP - 1);
    const int i = tl.y + (int)threadIdx.x / LPP;
    const bool active = i < S.fluid_begin + S.nf;
    const bool owner = active && sub == 0;
    const int N = A.N, Nf = A.Nf;

    const Q *__restrict__ vin = par ? A.vp1 : A.vp0;
    Q *__restrict__ vout = par ? A.vp0 : A.vp1;

    const PassConst<T> K(S);
    const PosT pos(S);
    // moving sims ping-pong their position records with the iteration parity
    const bool moving = MOVE && MODE == MODE_PSEUDO && S.move;
    const Rec *__restrict__ prec = (const Rec *)((moving && ppar) ? A.prec2 : A.prec);

    Acc<T> acc;
    T pi = 0, vi[3] = {0, 0, 0};
    int npairs = 0;
    // the owner's own state for the update, loaded before the neighbour loop so
    // that its latency hides behind the gathers
    T st_w[3] = {0, 0, 0}, st_dv[3] = {0, 0, 0}, st_w0[3] = {0, 0, 0}, st_vn[3] = {0, 0, 0};
    double st_pm = 0.0;
    if (MODE == MODE_PSEUDO && owner) {
        for (int d = 0; d < DIM; ++d) {
            st_w[d] = A.w[d * Nf + i];
            st_dv[d] = A.dv[d * Nf + i];
            st_w0[d] = A.w0[d * Nf + i];
            st_vn[d] = A.vn[d * Nf + i];
        }
        st_pm = A.pm[i];
    }
    T av[3] = {0, 0, 0};  // dot vector of the advective sums: V_i (steady) or Vtilde_i
    if (active) {
        const Rec ri = prec[i];
        const Q me = vin[i];
        vi[0] = me.x;
        vi[1] = me.y;
        vi[2] = DIM == 3 ? me.z : T(0);
        pi = pres<DIM>(me);
        if (CONV) {
            for (int d = 0; d < 3; ++d) av[d] = vi[d];
            if (moving)
                for (int d = 0; d < DIM; ++d) av[d] = A.vt[d * Nf + i];
        }
        const uint32_t cn = A.cnt[i];
        const int nfl = (int)(cn & 0xffffu), nwl = (int)(cn >> 16);
        npairs = nfl + nwl;
        const int *__restrict__ nb = A.nbr + i;
        using AvT = typename AvC<T, DIM>::type;
        Q *__restrict__ cf = CACHE ? A.coef + i : nullptr;  // cached coefficients
        AvT *__restrict__ cu = (CACHE && AV) ? (AvT *)A.coef_av + i : nullptr;
        const AvT u0{};
        // fluid neighbours in batches of U: U index loads, then 2U record
        // gathers (or U coefficient loads and U gathers) in flight, then U pair
        // evaluations
        // one lane per particle in the plain pseudo pass: 8 deep (the register
        // budget holds it there without spills; the variants with more state
        // stay at 4)
        constexpr bool kDeep = LPP == 1 && MODE == MODE_PSEUDO && !CONV && CACHE == 0 && !MOVE && !SEPDEN;
        constexpr int U = sizeof(T) == 4 ? (kDeep ? 8 : 4) : 2;
        int k = sub;
        for (; k + (U - 1) * LPP < nfl; k += U * LPP) {
            int jj[U];
#pragma unroll
            for (int m = 0; m < U; ++m) jj[m] = nb[(size_t)(k + m * LPP) * N];
            Rec rj[U];
            Q vj[U], cc[U];
            AvT ua[U];
#pragma unroll
            for (int m = 0; m < U; ++m) {
                if (CACHE == 2) {
                    cc[m] = cf[(size_t)(k + m * LPP) * N];
                    ua[m] = AV ? cu[(size_t)(k + m * LPP) * N] : u0;
                } else {
                    rj[m] = prec[jj[m]];
                }
                vj[m] = vin[jj[m]];
            }
#pragma unroll
            for (int m = 0; m < U; ++m) {
                T r[3], vd[3];
                vd[0] = vi[0] - vj[m].x;
                vd[1] = vi[1] - vj[m].y;
                vd[2] = DIM == 3 ? vi[2] - vj[m].z : T(0);
                if (CACHE == 2) {
                    pair_cached<T, DIM, AV, CONV>(K, cc[m], ua[m], vd, vd, vi, av, pi, pres<DIM>(vj[m]), acc);
                } else {
                    pos.delta(ri, rj[m], r);
                    const size_t e = (size_t)(k + m * LPP) * N;
                    pair_terms<T, DIM, AV, SEPDEN, CONV, CACHE == 1>(K, r, vd, vd, vi, av, pi, pres<DIM>(vj[m]), acc,
                                                                     CACHE ? cf + e : nullptr,
                                                                     (CACHE && AV) ? cu + e : nullptr);
                }
            }
        }
        if constexpr (PRED && CACHE == 0) {
            if (k < nfl) {  // the last, partial batch (U - 1 entries at most)
                int jj[U];
#pragma unroll
                for (int m = 0; m < U; ++m) {
                    const int km = k + m * LPP;
                    jj[m] = km < nfl ? nb[(size_t)km * N] : i;
                }
                Rec rj[U];
                Q vj[U];
#pragma unroll
                for (int m = 0; m < U; ++m) {
                    rj[m] = prec[jj[m]];
                    vj[m] = vin[jj[m]];
                }
#pragma unroll
                for (int m = 0; m < U; ++m) {
                    if (k + m * LPP < nfl) {
                        T r[3], vd[3];
                        vd[0] = vi[0] - vj[m].x;
                        vd[1] = vi[1] - vj[m].y;
                        vd[2] = DIM == 3 ? vi[2] - vj[m].z : T(0);
                        pos.delta(ri, rj[m], r);
                        pair_terms<T, DIM, AV, SEPDEN, CONV, false>(K, r, vd, vd, vi, av, pi, pres<DIM>(vj[m]), acc);
                    }
                }
                k = nfl;
            }
        }
        for (; k < nfl; k += LPP) {
            const int j = nb[(size_t)k * N];
            const Q vj = vin[j];
            T r[3], vd[3];
            vd[0] = vi[0] - vj.x;
            vd[1] = vi[1] - vj.y;
            vd[2] = DIM == 3 ? vi[2] - vj.z : T(0);
            if (CACHE == 2) {
                pair_cached<T, DIM, AV, CONV>(K, cf[(size_t)k * N], AV ? cu[(size_t)k * N] : u0, vd, vd, vi, av, pi,
                                              pres<DIM>(vj), acc);
            } else {
                const Rec rj = prec[j];
                pos.delta(ri, rj, r);
                pair_terms<T, DIM, AV, SEPDEN, CONV, CACHE == 1>(K, r, vd, vd, vi, av, pi, pres<DIM>(vj), acc,
                                                                 CACHE ? cf + (size_t)k * N : nullptr,
                                                                 (CACHE && AV) ? cu + (size_t)k * N : nullptr);
            }
        }
        if (WALLS) {
            // wall neighbours in batches too (UW index loads, then their ghost
            // records, position records and wall velocities in flight), summed
            // in list order like the rest; FP32 plain passes only (the FP64 and
            // the heavier variants would spill registers)
            constexpr int UW = sizeof(T) == 4 && !CONV && CACHE == 0 && !MOVE && !SEPDEN ? 4 : 1;
            const int nend = nfl + nwl;
            int k = nfl + sub;
            for (; UW > 1 && k + (UW - 1) * LPP < nend; k += UW * LPP) {
                int jj[UW];
#pragma unroll
                for (int m = 0; m < UW; ++m) jj[m] = nb[(size_t)(k + m * LPP) * N];
                Q gj[UW], cc[UW];
                Rec rj[UW];
                AvT ua[UW];
                T vw[UW][3];
#pragma unroll
                for (int m = 0; m < UW; ++m) {
                    gj[m] = vin[jj[m]];  // ghost velocity and wall pressure
                    const int jw = jj[m] - Nf;
                    for (int d = 0; d < 3; ++d) vw[m][d] = d < DIM ? A.vwall[d * A.Nw + jw] : T(0);
                    if (CACHE == 2) {
                        cc[m] = cf[(size_t)(k + m * LPP) * N];
                        ua[m] = AV ? cu[(size_t)(k + m * LPP) * N] : u0;
                    } else {
                        rj[m] = prec[jj[m]];
                    }
                }
#pragma unroll
                for (int m = 0; m < UW; ++m) {
                    T r[3], vd[3], vv[3];
                    for (int d = 0; d < 3; ++d) vd[d] = vi[d] - vw[m][d];
                    vv[0] = vi[0] - gj[m].x;
                    vv[1] = vi[1] - gj[m].y;
                    vv[2] = DIM == 3 ? vi[2] - gj[m].z : T(0);
                    if (CACHE == 2) {
                        pair_cached<T, DIM, AV, CONV>(K, cc[m], ua[m], vd, vv, vi, av, pi, pres<DIM>(gj[m]), acc);
                    } else {
                        pos.delta(ri, rj[m], r);
                        const size_t e = (size_t)(k + m * LPP) * N;
                        pair_terms<T, DIM, AV, SEPDEN, CONV, CACHE == 1>(K, r, vd, vv, vi, av, pi, pres<DIM>(gj[m]), acc,
                                                                         CACHE ? cf + e : nullptr,
                                                                         (CACHE && AV) ? cu + e : nullptr);
                    }
                }
            }
            if constexpr (PRED && CACHE == 0 && UW > 1) {
                if (k < nend) {  // the last, partial batch of walls
                    int jj[UW];
#pragma unroll
                    for (int m = 0; m < UW; ++m) {
                        const int km = k + m * LPP;
                        jj[m] = km < nend ? nb[(size_t)km * N] : -1;
                    }
                    Q gj[UW];
                    Rec rj[UW];
                    T vw[UW][3];
#pragma unroll
                    for (int m = 0; m < UW; ++m) {
                        const int j = jj[m] >= 0 ? jj[m] : Nf;  // a valid wall slot for the masked ones
                        gj[m] = vin[j];
                        for (int d = 0; d < 3; ++d) vw[m][d] = d < DIM ? A.vwall[d * A.Nw + (j - Nf)] : T(0);
                        rj[m] = prec[j];
                    }
#pragma unroll
                    for (int m = 0; m < UW; ++m) {
                        if (jj[m] >= 0) {
                            T r[3], vd[3], vv[3];
                            for (int d = 0; d < 3; ++d) vd[d] = vi[d] - vw[m][d];
                            vv[0] = vi[0] - gj[m].x;
                            vv[1] = vi[1] - gj[m].y;
                            vv[2] = DIM == 3 ? vi[2] - gj[m].z : T(0);
                            pos.delta(ri, rj[m], r);
                            pair_terms<T, DIM, AV, SEPDEN, CONV, false>(K, r, vd, vv, vi, av, pi, pres<DIM>(gj[m]), acc);
                        }
                    }
                    k = nend;
                }
            }
            for (; k < nend; k += LPP) {
                const int j = nb[(size_t)k * N];
                const Q gj = vin[j];  // ghost velocity and wall pressure
                const int jw = j - Nf;
                T r[3], vd[3], vv[3];
                for (int d = 0; d < 3; ++d) vd[d] = d < DIM ? vi[d] - A.vwall[d * A.Nw + jw] : T(0);
                vv[0] = vi[0] - gj.x;
                vv[1] = vi[1] - gj.y;
                vv[2] = DIM == 3 ? vi[2] - gj.z : T(0);
                if (CACHE == 2) {
                    pair_cached<T, DIM, AV, CONV>(K, cf[(size_t)k * N], AV ? cu[(size_t)k * N] : u0, vd, vv, vi, av, pi,
                                                  pres<DIM>(gj), acc);
                } else {
                    const Rec rj = prec[j];
                    pos.delta(ri, rj, r);
                    pair_terms<T, DIM, AV, SEPDEN, CONV, CACHE == 1>(K, r, vd, vv, vi, av, pi, pres<DIM>(gj), acc,
                                                                     CACHE ? cf + (size_t)k * N : nullptr,
                                                                     (CACHE && AV) ? cu + (size_t)k * N : nullptr);
                }
            }
        }
    }
    if (LPP > 1) {
        lane_sum(acc.div, LPP);
        lane_sum(acc.lap, LPP);
        for (int d = 0; d < DIM; ++d) {
            lane_sum(acc.grad[d], LPP);
            lane_sum(acc.vis[d], LPP);
            if (CONV) lane_sum(acc.conv[d], LPP);
        }
        if (CONV) lane_sum(acc.padv, LPP);
    }

    T Dv = 0, R[3] = {0, 0, 0}, vt2 = 0, dw2 = 0;
    if (owner) {
        Dv = (T)S.k_div * acc.div + (T)S.k_lap * acc.lap;
        for (int d = 0; d < DIM; ++d) R[d] = (T)S.k_grad * acc.grad[d] + (T)S.k_visc * acc.vis[d] + (T)S.g[d];
        if (CONV) {
            for (int d = 0; d < DIM; ++d) R[d] += (T)S.k_conv * acc.conv[d];
            Dv += (T)S.k_padv * acc.padv;
        }

        if (MODE == MODE_PSEUDO) {
            const T inv2dt = (T)S.inv2dt, gamma = (T)S.gamma, dtau = (T)S.dtau, dt = (T)S.dt;
            T vnew[3] = {0, 0, 0}, vtn[3] = {0, 0, 0};
            for (int d = 0; d < DIM; ++d) {
                const T wk = st_w[d];
                const T bdf = (T(3) * wk - st_dv[d]) * inv2dt;
                const T dvdtau = (R[d] - bdf) * gamma;
                const T wn = wk + dtau * dvdtau;
                const T vt = dt * dvdtau;
                vtn[d] = vt;
                vt2 += vt * vt;
                const T dw = wn - st_w0[d];
                dw2 += dw * dw;
                A.w[d * Nf + i] = wn;
                vnew[d] = st_vn[d] + wn;
            }
            const double pm = st_pm + S.dtau * (double)Dv;
            A.pm[i] = pm;
            A.dp[i] = Dv;
            vout[i] = make_rec<T, DIM>(vnew, (T)pm);
            if (moving) {
                // eq. vtilde and eq. rkp1, then the next eq. rkstar: r^{k+1} = r^{k+1/2}
                // + dtau/2 Vtilde^{k+1}, r^{k+3/2} = r^{k+1} + dtau/2 Vtilde^{k+1}
                double xo[3] = {0.0, 0.0, 0.0}, e2 = 0.0;
                for (int d = 0; d < DIM; ++d) {
                    const double hv = 0.5 * S.dtau * (double)vtn[d];
                    double x1 = A.xm[d * Nf + i] + hv;
                    if (S.periodic[d]) x1 = x1 >= S.hi[d] ? x1 - S.L[d] : (x1 < S.lo[d] ? x1 + S.L[d] : x1);
                    double x2 = x1 + hv;
                    if (S.periodic[d]) x2 = x2 >= S.hi[d] ? x2 - S.L[d] : (x2 < S.lo[d] ? x2 + S.L[d] : x2);
                    A.xm[d * Nf + i] = x2;
                    A.vt[d * Nf + i] = vtn[d];
                    xo[d] = x2;
                    double e = x2 - A.x[d * N + i];  // from r^(0), minimum image
                    if (S.periodic[d]) e = e > S.halfL[d] ? e - S.L[d] : (e < -S.halfL[d] ? e + S.L[d] : e);
                    e2 += e * e;
                }
                write_pos_record<T>(S, ppar ? const_cast<void *>(A.prec) : A.prec2, i, xo);
                if (DIM == 2) ((double2 *)A.xr)[i] = make_double2(xo[0], xo[1]);
                else ((double4 *)A.xr)[i] = make_double4(xo[0], xo[1], xo[2], 0.0);
                const double lim = 0.45 * S.skin;
                if (S.move == 2 && e2 > lim * lim) atomicOr(&A.flags[F_SKIN], 1);
            }
        } else {
            // a steady solve keeps its particles where they are and starts from V^n
            const double dt = S.steady ? 0.0 : S.dt, hdt2 = 0.5 * dt * dt;
            for (int d = 0; d < DIM; ++d) {
                const double xv = A.x[d * N + i];
                const double vv = (double)A.vn[d * Nf + i];
                double x0 = (xv + dt * vv) + hdt2 * (double)R[d];
                if (S.periodic[d]) {
                    if (x0 >= S.hi[d]) x0 -= S.L[d];
                    else if (x0 < S.lo[d]) x0 += S.L[d];
                }
                A.x_alt[d * N + i] = x0;
                A.xn[d * N + i] = xv;
                const T w0 = (T)(dt * (double)R[d]);
                A.w[d * Nf + i] = w0;
                A.w0[d * Nf + i] = w0;
            }
            if (DIM == 2) { A.x_alt[2 * N + i] = 0.0; A.xn[2 * N + i] = 0.0; }
            A.dp[i] = Dv;
            A.pn[i] = A.pm[i];
        }
    }

    if (MODE == MODE_PSEUDO) {
        // fixed-order block reduction of {sum |D|, sum |Vtilde|, max |D|, max |Vtilde|}
        __shared__ double lds[kMaxBlock / 64][6];
        double sd = owner ? fabs((double)Dv) : 0.0;
        double sv = owner ? sqrt((double)vt2) : 0.0;
        double md = sd, mv = sv, mw = owner ? (double)dw2 : 0.0;
        double np = owner ? (double)npairs : 0.0;
        for (int o = 32; o > 0; o >>= 1) {
            sd += __shfl_xor(sd, o, 64);
            sv += __shfl_xor(sv, o, 64);
            np += __shfl_xor(np, o, 64);
            md = fmax(md, __shfl_xor(md, o, 64));
            mv = fmax(mv, __shfl_xor(mv, o, 64));
            mw = fmax(mw, __shfl_xor(mw, o, 64));
        }
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        if (lane == 0) {
            lds[wave][0] = sd; lds[wave][1] = sv; lds[wave][2] = md; lds[wave][3] = mv; lds[wave][4] = mw;
            lds[wave][5] = np;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0, a5 = 0;
            for (int wv = 0; wv < (int)(blockDim.x >> 6); ++wv) {
                a0 += lds[wv][0];
                a1 += lds[wv][1];
                a2 = fmax(a2, lds[wv][2]);
                a3 = fmax(a3, lds[wv][3]);
                a4 = fmax(a4, lds[wv][4]);
                a5 += lds[wv][5];
            }
            part4[t] = make_double4(a0, a1, a2, a3);
            part2[t] = make_double2(a4, a5);
        }
    }
}

template <typename T, int DIM, bool WALLS, bool AV, bool SEPDEN, int MODE, int LPP, bool CONV, int CACHE, bool MOVE>
__device__ __forceinline__ void pass_tile(const PassArgs<T> &A, int t, int par, int ppar)
{
    const int2 tl = A.tiles[t];
    pass_tile_at<T, DIM, WALLS, AV, SEPDEN, MODE, LPP, CONV, CACHE, MOVE>(A, A.sims[tl.x], t, tl, par, ppar, A.partials,
                                                                          A.partials2);
}

template <typename T, int DIM, bool WALLS, bool AV, bool SEPDEN, int MODE, int LPP, bool CONV, int CACHE = 0,
          bool MOVE = false>
__global__ void __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(PassWaves<T, DIM, WALLS && AV && SEPDEN>::value)))
k_pass(PassArgs<T> A)
{
    const int v = tile_of_block(A.n_tiles, A.remap);
    if (v < 0) return;
    if (A.gated && !spec_gate(A.n_sims, A.iters, A.sims)) return;
    const int t = launch_tile(A, v);
    int par = A.cur, ppar = 0;
    if (MODE == MODE_PSEUDO) {
        const SimIter &It = A.iters[A.tiles[t].x];
        if (It.done) return;  // uniform per workgroup
        par = (A.cur + It.iters) & 1;
        ppar = It.iters & 1;
    }
    pass_tile<T, DIM, WALLS, AV, SEPDEN, MODE, LPP, CONV, CACHE, MOVE>(A, t, par, ppar);
}

// ---- wall pass (Adami et al. 2012, pressure clipped at zero) -----------------
template <typename T> struct WallArgs {
    using Q = typename V4<T>::type;
    int N, Nf, Nw, mode;
    const int *simid;
    const SimDev *sims;
    const SimIter *iters;
    const int *nbr;
    const uint32_t *cnt;
    const void *prec;
    Q *vp0, *vp1;    // reads fluid records, writes wall records (same buffer)
    const void *prec2;  // position records of odd iterations of moving sims
    int gated, n_sims;  // gated: run only if spec_gate holds (speculative launch)
    int cur;
    const T *vwall;
    T *pwall;
    const double *x;
    double *x_alt;   // MODE_PRE: walls keep their position
};

// Wall particle iw of sim S from the fluid records of buffer `par` (position
// records of buffer `ppar` for moving sims): its record (ghost velocity and
// pressure) into the same buffer and, with write_pw, the wall-pressure array.
template <typename T, int DIM>
__device__ __forceinline__ void wall_particle(const WallArgs<T> &A, const SimDev &S, int iw, int par, int ppar,
                                              bool write_pw)
{
    using Q = typename V4<T>::type;
    using PosT = Pos<T, DIM>;
    using Rec = typename PosT::Rec;
    const int i = A.Nf + iw;
    const int N = A.N;
    Q *__restrict__ vin = par ? A.vp1 : A.vp0;
    const PosT pos(S);
    const Rec *__restrict__ prec = (const Rec *)(ppar ? A.prec2 : A.prec);
    const Rec ri = prec[i];
    const T inv_h = (T)S.inv_h, rho = (T)S.rho0;
    const uint32_t cn = A.cnt[i];
    const int nfl = (int)(cn & 0xffffu);
    const int *__restrict__ nb = A.nbr + i;
    T S0 = 0, Sp = 0, Srr[3] = {0, 0, 0}, Sv[3] = {0, 0, 0};
    // fluid neighbours U at a time: U index loads, then 2U record gathers in
    // flight (slots past the count gather the particle's own records and are
    // skipped), then the sums in entry order
    constexpr int U = sizeof(T) == 4 ? 8 : 4;
    for (int k0 = 0; k0 < nfl; k0 += U) {
        bool ok[U];
        int jj[U];
#pragma unroll
        for (int m = 0; m < U; ++m) {
            ok[m] = k0 + m < nfl;
            jj[m] = ok[m] ? nb[(size_t)(k0 + m) * N] : i;
        }
        Rec rj[U];
        Q vj[U];
#pragma unroll
        for (int m = 0; m < U; ++m) {
            rj[m] = prec[jj[m]];
            vj[m] = vin[jj[m]];
        }
#pragma unroll
        for (int m = 0; m < U; ++m) {
            if (!ok[m]) continue;
            T r[3];
            pos.delta(ri, rj[m], r);
            T r2 = r[0] * r[0] + r[1] * r[1];
            if (DIM == 3) r2 += r[2] * r[2];
            const T q = sqrt(r2) * inv_h;
            T t3 = T(3) - q, t2 = T(2) - q, t1 = T(1) - q;
            t3 = t3 > T(0) ? t3 : T(0);
            t2 = t2 > T(0) ? t2 : T(0);
            t1 = t1 > T(0) ? t1 : T(0);
            const T a5 = t3 * t3 * t3 * t3 * t3, b5 = t2 * t2 * t2 * t2 * t2, c5 = t1 * t1 * t1 * t1 * t1;
            const T W = T(15) * c5 + (T(-6) * b5 + a5);  // sigma cancels in the ratios
            S0 += W;
            Sp += pres<DIM>(vj[m]) * W;
            for (int d = 0; d < DIM; ++d) {
                Srr[d] += rho * r[d] * W;
                Sv[d] += comp(vj[m], d) * W;
            }
        }
    }
    T vw[3] = {0, 0, 0}, ghost[3] = {0, 0, 0};
    for (int d = 0; d < DIM; ++d) vw[d] = A.vwall[d * A.Nw + iw];
    T pw = 0;
    if (S0 > T(0)) {
        T gr = 0;
        for (int d = 0; d < DIM; ++d) gr += (T)S.g[d] * Srr[d];
        const T pv = (Sp + gr) / S0;
        pw = pv > T(0) ? pv : T(0);
        for (int d = 0; d < DIM; ++d) ghost[d] = T(2) * vw[d] - Sv[d] / S0;
    } else {
        for (int d = 0; d < DIM; ++d) ghost[d] = vw[d];
    }
    vin[i] = make_rec<T, DIM>(ghost, pw);
    if (write_pw) A.pwall[iw] = pw;
}

template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_wall(WallArgs<T> A)
{
    const int iw = blockIdx.x * blockDim.x + threadIdx.x;
    if (iw >= A.Nw) return;
    if (A.gated && !spec_gate(A.n_sims, A.iters, A.sims)) return;
    const int i = A.Nf + iw;
    const int N = A.N;
    const int s = A.simid[i];
    const SimDev &S = A.sims[s];
    int par = A.cur, ppar = 0;
    if (A.mode == MODE_PRE) {
        for (int d = 0; d < 3; ++d) A.x_alt[d * N + i] = A.x[d * N + i];
    } else {
        const SimIter &It = A.iters[s];
        if (It.done) return;
        par = (A.cur + It.iters) & 1;
        ppar = S.move ? It.iters & 1 : 0;  // moving fluid: records at r^{k+1/2}
    }
    wall_particle<T, DIM>(A, S, iw, par, ppar, true);
}

// ---- residual reduction and stop test (section 3.4) --------------------------
// Two levels in one launch: workgroup g reduces the partials of segment g (up to
// kSegTiles tiles of one sim, fixed order); the last segment of a sim to arrive
// (per-sim ticket) reduces that sim's segment sums in segment order, applies the
// stop test and writes the sim's report and stop flag into mapped host memory
// (moving any build flag there too), so the host only needs a stream sync.
// Which workgroup arrives last does not change any sum.
struct FinArgs {
    const SimDev *sims;
    SimIter *iters;
    const double4 *partials;
    const double2 *partials2;
    const int4 *segs;
    double4 *seg_p;
    double2 *seg_p2;
    uint32_t *tickets;
    int *done_out, *flags;
    int n_sims;
    int *h_flags;
    MirrorRep *h_reps;
    unsigned long long *h_pairs;
    int *h_seq;      // per sim: its count of published reports, once this one is visible
    uint32_t *pubcount;
    int publish;     // 0: device state only (not the last iteration of a chunk)
};

constexpr int kFinThreads = kSegTiles;

// Build flags move to mapped memory with sim 0's report (same thread, before
// its sequence word).
__device__ inline void move_build_flags(const FinArgs &A)
{
    for (int k = 0; k < F_COUNT; ++k) {
        const int f = A.flags[k];
        if (f) {
            A.h_flags[k] = f;
            A.flags[k] = 0;
        }
    }
}

// Fixed-order workgroup reduction of {sum, sum, max, max, max, sum}; result in
// thread 0.
__device__ inline void fin_block_reduce(double v[6])
{
    __shared__ double lds[kFinThreads / 64][6];
    for (int o = 32; o > 0; o >>= 1) {
        v[0] += __shfl_xor(v[0], o, 64);
        v[1] += __shfl_xor(v[1], o, 64);
        v[5] += __shfl_xor(v[5], o, 64);
        v[2] = fmax(v[2], __shfl_xor(v[2], o, 64));
        v[3] = fmax(v[3], __shfl_xor(v[3], o, 64));
        v[4] = fmax(v[4], __shfl_xor(v[4], o, 64));
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
        for (int k = 0; k < 6; ++k) lds[wave][k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kFinThreads / 64; ++w) {
            v[0] += lds[w][0];
            v[1] += lds[w][1];
            v[2] = fmax(v[2], lds[w][2]);
            v[3] = fmax(v[3], lds[w][3]);
            v[4] = fmax(v[4], lds[w][4]);
            v[5] += lds[w][5];
        }
    }
    __syncthreads();
}

// Sim s's report and stop flag (and, with sim 0, the build flags) into mapped
// memory, then its sequence word behind a system-scope fence.
__device__ inline void publish_report(const FinArgs &A, int s, const SimIter &It)
{
    A.h_flags[F_COUNT + s] = It.done;
    MirrorRep r;
    r.iters = It.iters;
    r.reason = It.reason;
    r.rp_mean = It.rp_mean;
    r.rv_mean = It.rv_mean;
    r.rp_max = It.rp_max;
    r.rv_max = It.rv_max;
    r.disp = It.disp;
    A.h_reps[s] = r;
    A.h_pairs[s] = (unsigned long long)It.pairs;
    if (s == 0) move_build_flags(A);
    const uint32_t q = A.pubcount[s] + 1u;  // one publishing thread per sim and launch
    A.pubcount[s] = q;
    __threadfence_system();
    A.h_seq[s] = (int)q;
}

// What the closing thread needs, read by thread 0 of every workgroup at the
// start (only the last one to arrive uses it), so these reads overlap the
// partial sums instead of following the arrival ticket one by one.
struct FinState {
    int iters, fixed, conv_norm, stall_window, max_iter, steady, seg_begin, seg_count;
    double hp[kHist], hv[kHist];
    double dt, pscale, res_p, res_v, vref, tol, stall_rel;
};

__device__ inline void load_fin_state(FinState &F, const SimIter &It, const SimDev &S)
{
    F.iters = It.iters;
    F.fixed = It.fixed;
#pragma unroll
    for (int e = 0; e < kHist; ++e) {
        F.hp[e] = It.hp[e];
        F.hv[e] = It.hv[e];
    }
    F.conv_norm = S.conv_norm;
    F.stall_window = S.stall_window;
    F.max_iter = S.max_iter;
    F.steady = S.steady;
    F.seg_begin = S.seg_begin;
    F.seg_count = S.seg_count;
    F.dt = S.dt;
    F.pscale = S.dt / (S.rho0 * S.c * S.c);
    F.res_p = S.res_p;
    F.res_v = S.res_v;
    F.vref = S.vref;
    F.tol = S.tol;
    F.stall_rel = S.stall_rel;
}

// Iteration F.iters of a sim from its reduced partials red = {sum |D|, sum
// |Vtilde|, max |D|, max |Vtilde|, max |V - V^(0)|^2, pairs} (one thread): the
// residuals of eq. conv, the stop test and the loop state It, whose done flag
// the caller publishes.
__device__ inline void close_iteration(SimIter &It, const FinState &F, const double red[6])
{
    const double sd = red[0], sv = red[1], md = red[2], mv = red[3], mw = red[4], np = red[5];
    It.disp = F.steady ? 0.0 : 0.5 * F.dt * sqrt(mw);  // steady sims never move
    It.pairs = (long long)np;
    const double rp = sd * F.res_p, rv = sv * F.res_v;
    const double rpx = md * F.pscale, rvx = mv / F.vref;
    const int k = F.iters;
    const int slot = k % kHist;
    const double xp = F.conv_norm == 1 ? rpx : rp, xv = F.conv_norm == 1 ? rvx : rv;
    It.hp[slot] = xp;
    It.hv[slot] = xv;
    It.rp_mean = rp;
    It.rv_mean = rv;
    It.rp_max = rpx;
    It.rv_max = rvx;
    const int count = k + 1;
    It.iters = count;
    int reason = 0;
    if (!isfinite(xp) || !isfinite(xv)) {
        reason = DTSPH_NONFINITE;
    } else if (F.fixed > 0) {
        reason = count >= F.fixed ? DTSPH_FIXED : 0;
    } else {
        bool stalled[2] = {false, false};
        const int W = F.stall_window;
        if (W > 0 && count >= W) {
            // the window holds iterations count-W .. count-1: ring entries whose
            // age (slot - e mod kHist) is below W, the newest being this one
            double mn[2] = {INFINITY, INFINITY}, mx[2] = {-INFINITY, -INFINITY};
#pragma unroll
            for (int e = 0; e < kHist; ++e) {
                const int age = (slot - e + kHist) % kHist;
                if (age < W) {
                    const double vp = e == slot ? xp : F.hp[e], vv = e == slot ? xv : F.hv[e];
                    mn[0] = vp < mn[0] ? vp : mn[0];
                    mx[0] = vp > mx[0] ? vp : mx[0];
                    mn[1] = vv < mn[1] ? vv : mn[1];
                    mx[1] = vv > mx[1] ? vv : mx[1];
                }
            }
            for (int ser = 0; ser < 2; ++ser) stalled[ser] = (mx[ser] - mn[ser]) < F.stall_rel * mx[ser];
        }
        const bool bp = xp < F.tol, bv = xv < F.tol;
        if ((bp || stalled[0]) && (bv || stalled[1])) reason = (bp && bv) ? DTSPH_CONVERGED : DTSPH_STALLED;
        else if (count >= F.max_iter) reason = DTSPH_MAXITER;
    }
    if (reason) {
        It.done = 1;
        It.reason = reason;
    }
}

// Segment g of the residual reduction; the last segment of a sim to arrive
// closes the sim's iteration (stop test, report).
__device__ __forceinline__ void finalize_segment(const FinArgs &A, int g)
{
    __shared__ int last;
    const int4 sg = A.segs[g];
    const int s = sg.x;
    SimIter &It = A.iters[s];
    if (It.done) {
        if (sg.w == 0 && threadIdx.x == 0) {
            A.done_out[s] = 1;
            if (A.publish) publish_report(A, s, It);
        }
        return;
    }
    const SimDev &S = A.sims[s];
    FinState F;
    if (threadIdx.x == 0) load_fin_state(F, It, S);
    double red[6] = {0, 0, 0, 0, 0, 0};
    const int t = sg.y + (int)threadIdx.x;
    if (t < sg.z) {
        const double4 p = A.partials[t];
        const double2 p2 = A.partials2[t];
        red[0] = p.x; red[1] = p.y; red[2] = p.z; red[3] = p.w; red[4] = p2.x; red[5] = p2.y;
    }
    fin_block_reduce(red);
    if (threadIdx.x == 0) {
        A.seg_p[g] = make_double4(red[0], red[1], red[2], red[3]);
        A.seg_p2[g] = make_double2(red[4], red[5]);
        __threadfence();  // segment sums visible before the arrival is counted
        last = atomicAdd(&A.tickets[s], 1u) == (uint32_t)(S.seg_count - 1);
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    for (int k = 0; k < 6; ++k) red[k] = 0.0;
    const int seg_begin = S.seg_begin, seg_count = S.seg_count;
    for (int q = (int)threadIdx.x; q < seg_count; q += kFinThreads) {
        const double4 p = A.seg_p[seg_begin + q];
        const double2 p2 = A.seg_p2[seg_begin + q];
        if (q == (int)threadIdx.x) {
            red[0] = p.x; red[1] = p.y; red[2] = p.z; red[3] = p.w; red[4] = p2.x; red[5] = p2.y;
        } else {
            red[0] += p.x; red[1] += p.y; red[2] = fmax(red[2], p.z); red[3] = fmax(red[3], p.w);
            red[4] = fmax(red[4], p2.x); red[5] += p2.y;
        }
    }
    fin_block_reduce(red);
    if (threadIdx.x != 0) return;
    A.tickets[s] = 0u;
    close_iteration(It, F, red);
    A.done_out[s] = It.done;
    if (A.publish) publish_report(A, s, It);
}

__global__ void __launch_bounds__(kFinThreads) k_finalize(FinArgs A) { finalize_segment(A, blockIdx.x); }

// Iteration k's residual reduction and stop test (the first n_segs
// workgroups) together with the wall pass of iteration k + 1 (the others): the
// wall pass needs only the fluid records that iteration k's pair pass wrote,
// so both run in one launch. The walls of every sim still iterating are
// computed, also of a sim that stops in this launch (their records are then
// never read); the wall-pressure array keeps the values the last pair pass
// used (k_wall_pressure writes it at the end of the loop). `next` = k + 1.
template <typename T, int DIM>
__global__ void __launch_bounds__(kFinThreads) k_finalize_wall(FinArgs F, WallArgs<T> W, int n_segs, int next)
{
    if ((int)blockIdx.x < n_segs) {
        finalize_segment(F, blockIdx.x);
        return;
    }
    const int iw = ((int)blockIdx.x - n_segs) * kFinThreads + (int)threadIdx.x;
    if (iw >= W.Nw) return;
    const int s = W.simid[W.Nf + iw];
    if (W.iters[s].done) return;  // stopped before iteration k (or just now: either way unused)
    const SimDev &S = W.sims[s];
    wall_particle<T, DIM>(W, S, iw, (W.cur + next) & 1, S.move ? next & 1 : 0, false);
}

// End of a loop whose wall passes ran with the residual reductions: each wall
// pressure from the record of the last iteration its sim ran.
template <typename T>
__global__ void __launch_bounds__(256) k_wall_pressure(int Nw, int Nf, const int *__restrict__ simid,
                                                       const SimIter *__restrict__ iters,
                                                       const typename V4<T>::type *__restrict__ vp0,
                                                       const typename V4<T>::type *__restrict__ vp1, int cur,
                                                       int dim, T *__restrict__ pwall)
{
    const int iw = blockIdx.x * blockDim.x + threadIdx.x;
    if (iw >= Nw) return;
    const int i = Nf + iw;
    const int k = iters[simid[i]].iters;
    if (k < 1) return;
    const typename V4<T>::type r = ((cur + k - 1) & 1) ? vp1[i] : vp0[i];
    pwall[iw] = dim == 2 ? r.z : r.w;
}

// Copy the host-visible control words (build flags, stop flags, per-sim reports
// and pair counts) into mapped host memory, so one stream sync makes them
// readable without a separate copy.
__global__ void k_publish(int n_sims, int *__restrict__ flags, const SimIter *__restrict__ iters,
                          int *__restrict__ h_flags, MirrorRep *__restrict__ h_reps,
                          unsigned long long *__restrict__ h_pairs)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < F_COUNT && flags[i]) {  // build flags are moved to the host once
        h_flags[i] = flags[i];
        flags[i] = 0;
    }
    if (i >= F_COUNT && i < F_COUNT + n_sims) h_flags[i] = flags[i];
    if (i < n_sims) {
        const SimIter &It = iters[i];
        MirrorRep r;
        r.iters = It.iters;
        r.reason = It.reason;
        r.rp_mean = It.rp_mean;
        r.rv_mean = It.rv_mean;
        r.rp_max = It.rp_max;
        r.rv_max = It.rv_max;
        r.disp = It.disp;
        h_reps[i] = r;
        h_pairs[i] = (unsigned long long)It.pairs;
    }
}

// ---- launch arguments ----------------------------------------------------------

template <typename T> PassArgs<T> pass_args(Ctx &c, int mode, bool cand_lists)
{
    using Q = typename V4<T>::type;
    const int b = c.buf;
    PassArgs<T> a;
    a.N = c.N; a.Nf = c.Nf; a.Nw = c.Nw; a.remap = c.xcd_remap;
    a.n_tiles = c.n_tiles;
    a.n_ranges = 0;
    if (mode == MODE_PSEUDO && c.n_ranges > 0) {
        a.n_tiles = c.n_act_tiles;
        a.n_ranges = c.n_ranges;
        for (int q = 0; q < c.n_ranges; ++q) a.ranges[q] = c.ranges[q];
    }
    for (int q = a.n_ranges; q < kMaxRanges; ++q) a.ranges[q] = make_int2(0, 0);
    a.cur = c.cur;
    a.tiles = c.tiles; a.sims = c.sims; a.iters = c.iters; a.prec = c.prec;
    a.nbr = cand_lists ? c.cand : c.nbr;
    a.cnt = cand_lists ? c.ccnt : c.cnt;
    a.vp0 = (Q *)c.vp[0];
    a.vp1 = (Q *)c.vp[1];
    a.vwall = (const T *)c.vw[b];
    a.vn = (const T *)c.vn[b]; a.dv = (const T *)c.dv[b];
    a.w = (T *)c.w[b]; a.w0 = (T *)c.w0[b]; a.dp = (T *)c.dp[b];
    a.pm = c.pm[b]; a.pn = c.pn[b];
    a.x = c.x[c.xb]; a.x_alt = c.x[c.xb ^ 1]; a.xn = c.xn[b];
    a.partials = c.partials;
    a.partials2 = c.partials2;
    a.coef = (Q *)c.coef;
    a.coef_av = c.coef_av;
    a.prec2 = c.prec2; a.xm = c.xm; a.vt = (T *)c.vt; a.xr = c.xr; a.flags = c.flags;
    a.gated = c.gated ? 1 : 0;
    a.n_sims = c.n_sims;
    return a;
}

template <typename T> WallArgs<T> wall_args(Ctx &c, int mode, bool cand_lists)
{
    using Q = typename V4<T>::type;
    const int b = c.buf;
    WallArgs<T> a;
    a.N = c.N; a.Nf = c.Nf; a.Nw = c.Nw; a.mode = mode;
    a.simid = c.simid[b]; a.sims = c.sims; a.iters = c.iters; a.prec = c.prec;
    a.nbr = cand_lists ? c.cand : c.nbr;
    a.cnt = cand_lists ? c.ccnt : c.cnt;
    a.vp0 = (Q *)c.vp[0];
    a.vp1 = (Q *)c.vp[1];
    a.prec2 = c.prec2;
    a.gated = c.gated ? 1 : 0;
    a.n_sims = c.n_sims;
    a.cur = c.cur;
    a.vwall = (const T *)c.vw[b];
    a.pwall = (T *)c.pw[b];
    a.x = c.x[c.xb]; a.x_alt = c.x[c.xb ^ 1];
    return a;
}

FinArgs fin_args(Ctx &c, bool publish)
{
    FinArgs a;
    a.sims = c.sims; a.iters = c.iters; a.partials = c.partials; a.partials2 = c.partials2;
    a.segs = c.segs; a.seg_p = c.seg_p; a.seg_p2 = c.seg_p2; a.tickets = c.tickets;
    a.done_out = c.done_dev; a.flags = c.flags; a.n_sims = c.n_sims;
    a.h_flags = c.m_flags_d; a.h_reps = c.m_reps_d; a.h_pairs = c.m_pairs_d;
    a.h_seq = c.m_seq_d;
    a.pubcount = c.pubcount;
    a.publish = publish ? 1 : 0;
    if (publish) ++c.seq;  // every sim's count advances once per publishing launch
    return a;
}

}  // namespace

}  // namespace dtsph
