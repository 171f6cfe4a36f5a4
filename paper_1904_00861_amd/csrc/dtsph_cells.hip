// Cell-linked list and neighbour lists (HBM-bound streaming kernels).
//
// Per build:  k_keys (cell key; per-cell counts by integer atomics, one atomic
//             per run of equal keys in a wavefront)
//          -> three-kernel exclusive scan of the per-key counts (= cell-start table)
//          -> k_scatter (provisional slot: cell start + arrival order)
//          -> k_rank_gather (final slot: cell start + rank of the caller index
//             among the cell's particles; every state array moved there)
//          -> k_nbr (exact neighbour lists, candidate lists of radius kappa h +
//             skin, position records, pair counts).
// Between builds, k_filter re-derives the exact lists from the candidate lists
// at new positions, valid while no particle has moved more than skin/2 since
// the build (checked by the caller).
// The sort is a counting sort over the whole key (one radix digit holding the
// cell id): keys are dense and each cell holds a handful of particles, so one
// histogram + scan + scatter moves the data once instead of once per 8-bit digit.
#include <algorithm>

#include "dtsph_internal.h"

namespace dtsph {

namespace {

constexpr int kThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kThreads * kScanItems;  // 4096 keys per block

__device__ inline int cell_coord(double x, double lo, double inv_cs, int n)
{
    double f = floor((x - lo) * inv_cs);
    int c = 0;
    if (f >= 0.0) c = f > (double)(n - 1) ? n - 1 : (int)f;
    return c;
}

// DIM: the context's dimension, so the particle's coordinates are read together
// with its sim index instead of after the sim's constants.
template <int DIM>
__global__ void __launch_bounds__(kThreads) k_keys(int N, int Nf, int C, const double *__restrict__ x,
                                                   const int *__restrict__ simid, const SimDev *__restrict__ sims,
                                                   uint32_t *__restrict__ key, uint32_t *__restrict__ rank,
                                                   uint32_t *__restrict__ count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = i < N;
    uint32_t k = 0xffffffffu;
    if (active) {
        double p[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) p[a] = x[a * N + i];
        const SimDev &S = sims[simid[i]];
        int c[3] = {0, 0, 0};
#pragma unroll
        for (int a = 0; a < DIM; ++a) c[a] = cell_coord(p[a], S.lo[a], S.inv_cs[a], S.ncell[a]);
        k = (uint32_t)(S.key_base + (c[2] * S.ncell[1] + c[1]) * S.ncell[0] + c[0] + (i >= Nf ? C : 0));
        key[i] = k;
    }
    // Slots are in the previous build's cell order, so equal keys sit in runs of
    // consecutive lanes: the first lane of each run reserves the whole run.
    const int lane = threadIdx.x & 63;
    const uint32_t prev = __shfl_up(k, 1, 64);
    const bool head = active && (lane == 0 || prev != k);
    const unsigned long long heads = __ballot(head);
    const unsigned long long act = __ballot(active);
    const unsigned long long below = heads & ((2ull << lane) - 1ull);  // heads at lanes <= lane
    const int my_head = 63 - __builtin_clzll(below | 1ull);
    const unsigned long long above = heads & ~((2ull << lane) - 1ull);
    const int next_head = above ? __builtin_ctzll(above) : 64 - __builtin_clzll(act);
    uint32_t base = 0;
    if (head) base = atomicAdd(&count[k], (uint32_t)(next_head - lane));
    base = __shfl(base, my_head, 64);
    if (active) rank[i] = base + (uint32_t)(lane - my_head);
}

// Block-wide exclusive scan of one value per thread (wave64 shuffles + LDS).
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *lds_waves, uint32_t &total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    uint32_t inc = v;
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
    }
    if (lane == 63) lds_waves[wave] = inc;
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (int w = 0; w < nwaves; ++w) {
        uint32_t s = lds_waves[w];
        if (w < wave) before += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return before + inc - v;
}

// Per-block totals of the counts; reads are coalesced (the order of an integer
// sum does not matter).
__global__ void __launch_bounds__(kThreads) k_scan_reduce(const uint32_t *__restrict__ in, int n,
                                                          uint32_t *__restrict__ sums)
{
    __shared__ uint32_t lds[kThreads / 64];
    const int base = blockIdx.x * kScanTile + threadIdx.x;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k * kThreads < n) s += in[base + k * kThreads];
    uint32_t tot;
    block_exclusive_scan(s, lds, tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Block b adds the sums of blocks 0..b-1 (read directly: there are at most a few
// hundred), scans its own tile, writes the cell-start table, and leaves the
// counts zeroed for the next build. The tile passes through LDS so that global
// reads and writes are coalesced while each thread scans 16 consecutive counts
// (row padding of one word per 16 keeps the LDS accesses conflict-free).
__global__ void __launch_bounds__(kThreads) k_scan_down(uint32_t *__restrict__ in, int n,
                                                        const uint32_t *__restrict__ sums,
                                                        uint32_t *__restrict__ out)
{
    __shared__ uint32_t lds[kThreads / 64];
    __shared__ uint32_t tile[kScanTile + kScanTile / kScanItems];
    const int t = threadIdx.x;
    const int base = blockIdx.x * kScanTile;
    auto pad = [](int j) { return j + j / kScanItems; };
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int j = k * kThreads + t;
        uint32_t v = 0u;
        if (base + j < n) {
            v = in[base + j];
            in[base + j] = 0u;
        }
        tile[pad(j)] = v;
    }
    uint32_t before = 0;
    for (int q = t; q < (int)blockIdx.x; q += blockDim.x) before += sums[q];
    uint32_t block_off;
    block_exclusive_scan(before, lds, block_off);  // block total = sum of preceding blocks
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = tile[pad(t * kScanItems + k)];
        s += v[k];
    }
    uint32_t tot;
    uint32_t run = block_exclusive_scan(s, lds, tot) + block_off;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        tile[pad(t * kScanItems + k)] = run;
        run += v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int j = k * kThreads + t;
        if (base + j < n) out[base + j] = tile[pad(j)];
    }
    if (blockIdx.x == gridDim.x - 1 && t == blockDim.x - 1) out[n] = run;
}

__global__ void k_scatter(int N, const uint32_t *__restrict__ key, const uint32_t *__restrict__ rank,
                          const uint32_t *__restrict__ cell_start, uint32_t *__restrict__ perm)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    perm[cell_start[key[i]] + rank[i]] = (uint32_t)i;
}

template <typename T>
struct GatherArgs {
    int N, Nf, Nw;
    const uint32_t *perm;      // provisional order from k_scatter
    const uint32_t *key;
    const uint32_t *cell_start;
    uint32_t *src_of;          // final order: source slot of each slot
    int *flags;
    const int *orig_in, *simid_in;
    int *orig_out, *simid_out;
    const double *x_in, *xn_in;
    double *x_out, *xn_out;
    void *xr;
    int dim;
    const T *vn_in, *dv_in, *w_in, *w0_in, *dp_in;
    T *vn_out, *dv_out, *w_out, *w0_out, *dp_out;
    const double *pm_in, *pn_in;
    double *pm_out, *pn_out;
    const T *vw_in, *pw_in;
    T *vw_out, *pw_out;
    // loop set-up fused into the gather (loop >= 0): reset of every sim's loop
    // state (fixed iterations = loop), stage-1 half step of p unless pending,
    // and the {V^k, p^{k+1/2}} records of buffer `rec`
    int loop, add_half, n_sims;
    const SimDev *sims;
    SimIter *iters;
    void *rec;
};

template <typename T> struct RecT;
template <> struct RecT<float> { using type = float4; };
template <> struct RecT<double> { using type = double4; };

// Final slot = cell start + number of the cell's particles with a smaller caller
// index (ties in caller order, independent of atomic arrival order); every
// state array is copied from the old slot to the final one.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_rank_gather(GatherArgs<T> A)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (A.loop >= 0 && m < A.n_sims) {
        SimIter z{};
        z.fixed = A.loop;
        for (int k = 0; k < kHist; ++k) { z.hp[k] = 0.0; z.hv[k] = 0.0; }
        A.iters[m] = z;
    }
    if (m >= A.N) return;
    const int N = A.N, Nf = A.Nf, Nw = A.Nw;
    const int s = (int)A.perm[m];
    // the particle's state is read as soon as its source slot is known, so these
    // loads are in flight while the rank among the cell's members is counted
    const int os = A.orig_in[s];
    const int sid = A.simid_in[s];
    // in 2D the third component is zero everywhere: written, not read
    const int dim = A.dim;
    double xs[3] = {0.0, 0.0, 0.0}, xns[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < dim; ++a) {
        xs[a] = A.x_in[a * N + s];
        xns[a] = A.xn_in[a * N + s];
    }
    const bool fl = s < Nf;  // slots keep their kind (fluid keys precede wall keys)
    T vn[3] = {T(0), T(0), T(0)}, dvv[3] = {T(0), T(0), T(0)}, ww[3] = {T(0), T(0), T(0)},
      w0[3] = {T(0), T(0), T(0)};
    T dp = T(0);
    double pmv = 0.0, pnv = 0.0;
    if (fl) {
        for (int a = 0; a < dim; ++a) {
            vn[a] = A.vn_in[a * Nf + s];
            dvv[a] = A.dv_in[a * Nf + s];
            ww[a] = A.w_in[a * Nf + s];
            w0[a] = A.w0_in[a * Nf + s];
        }
        dp = A.dp_in[s];
        pmv = A.pm_in[s];
        pnv = A.pn_in[s];
    }
    const uint32_t k = A.key[s];
    const int b = (int)A.cell_start[k], e = (int)A.cell_start[k + 1];
    if (e - b > kMaxCellOccupancy) {
        atomicOr(&A.flags[F_CELL_OVERFLOW], 1);
        return;
    }
    int r = 0;
    for (int q0 = b; q0 < e; q0 += 8) {  // 8 members in flight at a time
        uint32_t pm[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) pm[m] = A.perm[q0 + m < e ? q0 + m : b];
#pragma unroll
        for (int m = 0; m < 8; ++m) r += (q0 + m < e) && A.orig_in[pm[m]] < os;
    }
    const int d = b + r;
    A.src_of[d] = (uint32_t)s;
    A.orig_out[d] = os;
    A.simid_out[d] = sid;
    for (int a = 0; a < 3; ++a) {
        A.x_out[a * N + d] = xs[a];
        A.xn_out[a * N + d] = xns[a];
    }
    if (A.dim == 2) ((double2 *)A.xr)[d] = make_double2(xs[0], xs[1]);
    else ((double4 *)A.xr)[d] = make_double4(xs[0], xs[1], xs[2], 0.0);
    if (d < Nf) {
        T v[3];
        for (int a = 0; a < 3; ++a) {
            A.vn_out[a * Nf + d] = vn[a];
            A.dv_out[a * Nf + d] = dvv[a];
            A.w_out[a * Nf + d] = ww[a];
            A.w0_out[a * Nf + d] = w0[a];
            v[a] = vn[a] + ww[a];
        }
        double p = pmv;
        if (A.loop >= 0 && A.add_half) p += 0.5 * A.sims[sid].dtau * (double)dp;
        A.pm_out[d] = p;
        A.pn_out[d] = pnv;
        A.dp_out[d] = dp;
        if (A.loop >= 0) {
            using Q = typename RecT<T>::type;
            Q rec;
            rec.x = v[0];
            rec.y = v[1];
            if (A.dim == 2) { rec.z = (T)p; rec.w = T(0); }
            else { rec.z = v[2]; rec.w = (T)p; }
            ((Q *)A.rec)[d] = rec;
        }
    } else {
        const int dw = d - Nf, sw = s - Nf;
        for (int a = 0; a < 3; ++a) A.vw_out[a * Nw + dw] = A.vw_in[a * Nw + sw];
        A.pw_out[dw] = A.pw_in[sw];
    }
}

// Exact neighbour predicate: minimum-image separation, squared length summed
// as (dx*dx + dy*dy) + dz*dz in float64 without contraction, strict < (kh)^2.
__device__ inline double min_image(double s, int per, double L, double halfL)
{
    // s - L, s + L or s, selected without branches (same roundings as the
    // conditional subtraction/addition)
    const double sh = s > halfL ? -L : (s < -halfL ? L : 0.0);
    return s + (per ? sh : 0.0);
}

// packed positions: xr[i] = (x, y) in 2D, (x, y, z, 0) in 3D
template <int DIM> struct XR;
template <> struct XR<2> {
    using type = double2;
    __device__ static double z(const double2 &) { return 0.0; }
    __device__ static double2 make(double x, double y, double) { return make_double2(x, y); }
};
template <> struct XR<3> {
    using type = double4;
    __device__ static double z(const double4 &v) { return v.z; }
    __device__ static double4 make(double x, double y, double z) { return make_double4(x, y, z, 0.0); }
};

// Cells along one axis whose particles can be neighbours of a particle in cell
// c: c-m .. c+m, wrapped on periodic axes, clipped on others; a periodic axis
// with fewer than 2m+1 cells visits each of its cells once.
struct AxisRange {
    int first, count, n, per;
    __device__ AxisRange(int c, int n_, int per_, int m) : n(n_), per(per_)
    {
        if (per && n < 2 * m + 1) { first = 0; count = n; }
        else if (per) { first = c - m; count = 2 * m + 1; }
        else {
            first = c > m ? c - m : 0;
            const int last = c < n - 1 - m ? c + m : n - 1;
            count = last - first + 1;
        }
    }
    __device__ int at(int k) const
    {
        int v = first + k;
        if (per) v = v < 0 ? v + n : (v >= n ? v - n : v);
        return v;
    }
    // Periodic image of cell k of the block: a particle there, seen from the
    // block's centre cell, is shifted by +L (wrapped from below) or -L.
    __device__ double shift(int k, double L) const
    {
        if (!per) return 0.0;
        const int v = first + k;
        return v < 0 ? L : (v >= n ? -L : 0.0);
    }
};

template <typename T>
struct NbrArgs {
    int N, Nf, C, cap;
    const double *x;
    const void *xr;
    const int *simid;
    const SimDev *sims;
    const uint32_t *cell_start;
    int *nbr;
    uint32_t *cnt;
    int capc;
    int *cand;
    uint32_t *ccnt;
    void *prec;

    int *flags;
};

// G consecutive lanes share one particle and test its candidates G at a time;
// a wave ballot gives each lane the number of accepted candidates before it in
// the group, so the list keeps the sequential scan order.
template <int G> struct Group {
    int sub, g0;
    __device__ Group() : sub((int)threadIdx.x & (G - 1)), g0((int)(threadIdx.x & 63) & ~(G - 1)) {}
    // bits of the group's lanes for which pred holds (bit k = lane sub k)
    __device__ unsigned bits(bool pred) const
    {
        const unsigned long long b = __ballot(pred);
        return G == 64 ? 0u : (unsigned)(b >> g0) & ((1u << G) - 1u);
    }
    __device__ int before(unsigned gb) const { return __popc(gb & ((1u << sub) - 1u)); }
};

// Candidates are taken U at a time per lane: all U position loads are in
// flight before the first test, and list writes happen after the batch.
constexpr int kBatch = 8;   // the filter
constexpr int kBatchNbr = 4;  // the neighbour kernel (more in flight costs occupancy)

template <int DIM> struct Probe {
    double xi, yi, zi, kh2;
    int px, py, pz;
    double Lx, Ly, Lz, hx, hy, hz;
    // squared separation with the minimum image decided per candidate
    __device__ double r2(const typename XR<DIM>::type &q) const
    {
#pragma clang fp contract(off)
        const double dx = min_image(xi - q.x, px, Lx, hx);
        const double dy = min_image(yi - q.y, py, Ly, hy);
        const double dz = DIM == 3 ? min_image(zi - XR<DIM>::z(q), pz, Lz, hz) : 0.0;
        return (dx * dx + dy * dy) + dz * dz;
    }
    // squared separation with the periodic shift of the candidate's cell run
    // (the same roundings: s - L is s + (-L))
    __device__ double r2s(const typename XR<DIM>::type &q, double sx, double sy, double sz) const
    {
#pragma clang fp contract(off)
        const double dx = (xi - q.x) + sx;
        const double dy = (yi - q.y) + sy;
        const double dz = DIM == 3 ? (zi - XR<DIM>::z(q)) + sz : 0.0;
        return (dx * dx + dy * dy) + dz * dz;
    }
};

template <int DIM> __device__ inline Probe<DIM> make_probe(const SimDev &S, double xi, double yi, double zi)
{
    Probe<DIM> P;
    P.xi = xi; P.yi = yi; P.zi = zi; P.kh2 = S.kh2;
    P.px = S.periodic[0]; P.py = S.periodic[1]; P.pz = DIM == 3 ? S.periodic[2] : 0;
    P.Lx = S.L[0]; P.Ly = S.L[1]; P.Lz = S.L[2];
    P.hx = S.halfL[0]; P.hy = S.halfL[1]; P.hz = S.halfL[2];
    return P;
}

// Running state of one particle's list build.
struct ListCursor {
    int total = 0, ctotal = 0;   // entries found so far (exact, candidate)
};

// Tests the candidates in slots [jb, je) (one run of consecutive cells), G
// lanes at a time with kBatchNbr positions per lane in flight, and appends the
// hits to the exact and candidate lists in scan order. GENERAL: minimum image
// per candidate (needed when a periodic axis has fewer than 2m+3 cells);
// otherwise the run's periodic shift (sx, sy, sz) applies to all of it.
template <int DIM, int G, bool GENERAL>
__device__ __forceinline__ void scan_run(const typename XR<DIM>::type *__restrict__ xr, int jb, int je, int i,
                                         const Probe<DIM> &P, double sx, double sy, double sz, double cr2,
                                         int *__restrict__ nbr, int *__restrict__ cand, int N, int cap, int capc,
                                         const Group<G> &grp, ListCursor &cur)
{
    using Q = typename XR<DIM>::type;
    constexpr int kB = kBatchNbr;
    if (jb >= je) return;
    // software pipeline: the next batch's positions are in flight while the
    // current batch is tested
    Q q[kB];
#pragma unroll
    for (int m = 0; m < kB; ++m) {
        const int j = jb + m * G + grp.sub;
        q[m] = xr[j < je ? j : jb];
    }
    for (int j0 = jb; j0 < je; j0 += G * kB) {  // uniform in the group
        Q qn[kB];
        const int jn = j0 + G * kB;
        if (jn < je) {
#pragma unroll
            for (int m = 0; m < kB; ++m) {
                const int j = jn + m * G + grp.sub;
                qn[m] = xr[j < je ? j : jb];
            }
        }
#pragma unroll
        for (int m = 0; m < kB; ++m) {
            const int j = j0 + m * G + grp.sub;
            const double r2 = GENERAL ? P.r2(q[m]) : P.r2s(q[m], sx, sy, sz);
            const bool ok = j < je && j != i;
            const bool in_c = ok && r2 < cr2, in_x = ok && r2 < P.kh2;
            if (G == 1) {
                if (in_c && cur.ctotal < capc) cand[(size_t)cur.ctotal * N] = j;
                if (in_x && cur.total < cap) nbr[(size_t)cur.total * N] = j;
                cur.ctotal += in_c;
                cur.total += in_x;
            } else if (G == 2) {
                // the partner lane's two hits by one lane swap (DPP quad_perm 1,0,3,2);
                // both lanes of a group are always active here
                const int h = (int)in_c | ((int)in_x << 1);
                const int o = __builtin_amdgcn_update_dpp(0, h, 0xB1, 0xF, 0xF, false);
                const int oc = o & 1, ox = o >> 1;
                if (in_c) {  // entry offsets are non-negative: one 32 x 32 -> 64 bit multiply
                    const int qq = cur.ctotal + (grp.sub ? oc : 0);
                    if (qq < capc) cand[(size_t)(unsigned)qq * (unsigned)N] = j;
                }
                if (in_x) {
                    const int qq = cur.total + (grp.sub ? ox : 0);
                    if (qq < cap) nbr[(size_t)(unsigned)qq * (unsigned)N] = j;
                }
                cur.ctotal += (int)in_c + oc;
                cur.total += (int)in_x + ox;
            } else {
                const unsigned bc = grp.bits(in_c), bx = grp.bits(in_x);
                if (in_c) {
                    const int qq = cur.ctotal + grp.before(bc);
                    if (qq < capc) cand[(size_t)qq * N] = j;
                }
                if (in_x) {
                    const int qq = cur.total + grp.before(bx);
                    if (qq < cap) nbr[(size_t)qq * N] = j;
                }
                cur.ctotal += __popc(bc);
                cur.total += __popc(bx);
            }
        }
        if (jn < je) {
#pragma unroll
            for (int m = 0; m < kB; ++m) q[m] = qn[m];
        }
    }
}

// Cell rows of one particle's search block, visited in order (type, plane,
// row); each row is at most two runs of consecutive cell keys along x. The
// bounds of the next row are loaded while the current one is scanned.
// Off the GENERAL path a row's x-run is trimmed to the cells the candidate
// sphere reaches there: with d the distance from the particle to the row's
// y (and z) slab, only |x_j - x_i| <= sqrt(R^2 - d^2) can hold a candidate.
// The trimming runs in float in cell units relative to the particle's cell,
// widened by 1e-5 cells (far above its rounding), so it never drops a cell
// the float64 predicate could accept. Edge cells of a non-periodic axis hold
// the particles clamped into them, so their extent is open on the outer side.
template <typename T, int DIM, int G, bool GENERAL>
__device__ __forceinline__ void scan_block(const NbrArgs<T> &A, const SimDev &S, int i, const Probe<DIM> &P,
                                           int cx, int cy, int cz, bool fluid, int &cf, int &cw, int &ccf,
                                           int &ccw, ListCursor &cur, const Group<G> &grp)
{
    using Q = typename XR<DIM>::type;
    const Q *__restrict__ xr = (const Q *)A.xr;
    const uint32_t *__restrict__ cstart = A.cell_start;
    const int N = A.N;
    const int nx = S.ncell[0], ny = S.ncell[1], nz = DIM == 3 ? S.ncell[2] : 1;
    const int md = S.cell_div;
    // x cells cx-m .. cx+m as at most two contiguous runs of keys
    int xa0, xb0, xa1 = 0, xb1 = -1;
    double sx1 = 0.0;
    if (P.px && nx < 2 * md + 1) { xa0 = 0; xb0 = nx - 1; }
    else if (P.px && cx - md < 0) { xa0 = 0; xb0 = cx + md; xa1 = nx + cx - md; xb1 = nx - 1; sx1 = P.Lx; }
    else if (P.px && cx + md > nx - 1) { xa0 = cx - md; xb0 = nx - 1; xa1 = 0; xb1 = cx + md - nx; sx1 = -P.Lx; }
    else { xa0 = cx > md ? cx - md : 0; xb0 = cx < nx - 1 - md ? cx + md : nx - 1; }
    const AxisRange ry(cy, ny, P.py, md), rz(cz, nz, P.pz, DIM == 3 ? md : 0);
    const int ntp = (fluid && S.nw > 0) ? 2 : 1;  // wall cells only where walls exist
    const int nrows = ntp * rz.count * ry.count;
    int *__restrict__ nbr = A.nbr + i;
    int *__restrict__ cand = A.cand + i;
    const double cr2 = S.cand_r2;
    // the particle in cell units from the low corner of its own cell, clamped to
    // a range that decides every row and window the same way as the exact value
    auto frac = [&](double p, int a, int c) {
        const double f = (p - S.lo[a]) * S.inv_cs[a] - (double)c;
        const double lim = (double)md + 3.0;
        return (float)(f < -lim ? -lim : (f > lim + 1.0 ? lim + 1.0 : f));
    };
    const float fx = GENERAL ? 0.f : frac(P.xi, 0, cx);
    const float fy = GENERAL ? 0.f : frac(P.yi, 1, cy);
    const float fz = (GENERAL || DIM == 2) ? 0.f : frac(P.zi, 2, cz);
    const float csy = (float)S.cs[1], csz = (float)S.cs[2], icsx = (float)S.inv_cs[0];
    const float cr2f = (float)cr2;
    // distance (physical units, shortened by 1e-5 cells) from the particle to
    // the slab of block row k along an axis
    auto slab_d = [&](const AxisRange &ra, int k, int c_own, float f, int per, float cs) {
        const int c = ra.at(k);
        const float o = (float)(ra.first + k - c_own);  // the slab is [o, o + 1) in cell units
        const float below = (!per && c == 0) ? 0.f : o - f;
        const float above = (!per && c == ra.n - 1) ? 0.f : f - (o + 1.f);
        const float d = fmaxf(below, above) - 1e-5f;
        return d > 0.f ? d * cs : 0.f;
    };
    // the row's runs: [a0, b0] unshifted, [a1, b1] with shift s1 (b < a: empty)
    auto row_runs = [&](int u, int v, int &a0, int &b0, int &a1, int &b1, double &s1) {
        a0 = xa0; b0 = xb0; a1 = xa1; b1 = xb1; s1 = sx1;
        if (GENERAL) return;
        const float dy = slab_d(ry, v, cy, fy, P.py, csy);
        const float dz = DIM == 3 ? slab_d(rz, u, cz, fz, P.pz, csz) : 0.f;
        const float rem = cr2f - (dy * dy + dz * dz);
        if (rem < 0.f) { b0 = a0 - 1; b1 = a1 - 1; return; }
        // hardware square root (about 1 ulp, far inside the 1e-5-cell margin)
        const float wc = __builtin_amdgcn_sqrtf(rem) * icsx + 1e-5f;
        int lo_c = cx + (int)floorf(fx - wc);
        int hi_c = cx + (int)floorf(fx + wc);
        lo_c = lo_c > cx - md ? lo_c : cx - md;
        hi_c = hi_c < cx + md ? hi_c : cx + md;
        if (P.px) {
            a0 = lo_c > 0 ? lo_c : 0;
            b0 = hi_c < nx - 1 ? hi_c : nx - 1;
            a1 = 0; b1 = -1; s1 = 0.0;
            if (lo_c < 0) { a1 = nx + lo_c; b1 = nx - 1; s1 = P.Lx; }
            else if (hi_c > nx - 1) { a1 = 0; b1 = hi_c - nx; s1 = -P.Lx; }
        } else {
            // edge cells extend outwards: a window beyond the grid still meets them
            a0 = lo_c < 0 ? 0 : (lo_c > nx - 1 ? nx - 1 : lo_c);
            b0 = hi_c < 0 ? 0 : (hi_c > nx - 1 ? nx - 1 : hi_c);
        }
    };
    auto row_key = [&](int u, int v, int tp) {
        return S.key_base + (tp ? A.C : 0) + (rz.at(u) * ny + ry.at(v)) * nx;
    };
    auto advance = [&](int &u, int &v, int &tp) {
        if (++v == ry.count) {
            v = 0;
            if (++u == rz.count) { u = 0; ++tp; }
        }
    };
    if constexpr (G == 2 && !GENERAL) {
        // The two lanes of a particle prepare alternate rows (lane `sub` the rows
        // 2q + sub: window, bounds) and swap them by a lane swap (DPP quad_perm
        // 1,0,3,2), so each row's window is computed once; both lanes then scan
        // the pair's rows in order, as below. The next pair is prepared while
        // this one is scanned.
        auto swap = [](int x) { return __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false); };
        const int sub = grp.sub;
        int mu = 0, mv = 0, mtp = 0;  // this lane's row
        if (sub) advance(mu, mv, mtp);
        int b0, e0, b1, e1, f1;  // its bounds and the shift sign of its second run
        auto prep = [&](int r) {
            b0 = e0 = b1 = e1 = f1 = 0;
            if (r >= nrows) return;
            int a0, c0, a1, c1;
            double s1;
            const int row = row_key(mu, mv, mtp);
            row_runs(mu, mv, a0, c0, a1, c1, s1);
            if (c0 >= a0) { b0 = (int)cstart[row + a0]; e0 = (int)cstart[row + c0 + 1]; }
            if (c1 >= a1) { b1 = (int)cstart[row + a1]; e1 = (int)cstart[row + c1 + 1]; }
            f1 = s1 > 0.0 ? 1 : (s1 < 0.0 ? -1 : 0);
        };
        prep(sub);
        cf = -1;
        for (int r0 = 0; r0 < nrows; r0 += 2) {  // uniform in the group
            const int o[8] = {swap(b0), swap(e0), swap(b1), swap(e1), swap(f1), swap(mu), swap(mv), swap(mtp)};
            const int m[8] = {b0, e0, b1, e1, f1, mu, mv, mtp};
            int ra[8], rb[8];  // row r0 (lane 0's) and row r0 + 1 (lane 1's)
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                ra[q] = sub ? o[q] : m[q];
                rb[q] = sub ? m[q] : o[q];
            }
            if (r0 + 2 < nrows) {
                advance(mu, mv, mtp);
                advance(mu, mv, mtp);
                prep(r0 + 2 + sub);
            }
            for (int h = 0; h < 2 && r0 + h < nrows; ++h) {
                const int *d = h ? rb : ra;
                if (d[7] == 1 && cf < 0) { cf = cur.total; ccf = cur.ctotal; }
                const double sy = ry.shift(d[6], P.Ly), sz = DIM == 3 ? rz.shift(d[5], P.Lz) : 0.0;
                const double rs1 = (double)d[4] * P.Lx;
                const int nrun = d[2] < d[3] ? 2 : 1;
                for (int k = 0; k < nrun; ++k)
                    scan_run<DIM, G, GENERAL>(xr, k ? d[2] : d[0], k ? d[3] : d[1], i, P, k ? rs1 : 0.0, sy, sz, cr2,
                                              nbr, cand, N, A.cap, A.capc, grp, cur);
            }
        }
        if (cf < 0) { cf = cur.total; ccf = cur.ctotal; }
        cw = cur.total - cf;
        ccw = cur.ctotal - ccf;
        return;
    }
    int u = 0, v = 0, tp = 0;
    int row = row_key(u, v, tp);
    int a0, c0, a1, c1;
    double s1;
    row_runs(u, v, a0, c0, a1, c1, s1);
    int b0 = 0, e0 = 0, b1 = 0, e1 = 0;
    if (c0 >= a0) { b0 = (int)cstart[row + a0]; e0 = (int)cstart[row + c0 + 1]; }
    if (c1 >= a1) { b1 = (int)cstart[row + a1]; e1 = (int)cstart[row + c1 + 1]; }
    cf = -1;
    for (int r = 0; r < nrows; ++r) {
        const int cu = u, cv = v, ctp = tp;
        const int jb0 = b0, je0 = e0, jb1 = b1, je1 = e1;
        const double rs1 = s1;
        if (r + 1 < nrows) {  // prefetch the next row's bounds
            advance(u, v, tp);
            row = row_key(u, v, tp);
            row_runs(u, v, a0, c0, a1, c1, s1);
            b0 = e0 = b1 = e1 = 0;
            if (c0 >= a0) { b0 = (int)cstart[row + a0]; e0 = (int)cstart[row + c0 + 1]; }
            if (c1 >= a1) { b1 = (int)cstart[row + a1]; e1 = (int)cstart[row + c1 + 1]; }
        }
        if (ctp == 1 && cf < 0) { cf = cur.total; ccf = cur.ctotal; }
        const double sy = ry.shift(cv, P.Ly), sz = DIM == 3 ? rz.shift(cu, P.Lz) : 0.0;
        const int nrun = jb1 < je1 ? 2 : 1;
        for (int k = 0; k < nrun; ++k)  // one code copy for both runs
            scan_run<DIM, G, GENERAL>(xr, k ? jb1 : jb0, k ? je1 : je0, i, P, k ? rs1 : 0.0, sy, sz, cr2, nbr,
                                      cand, N, A.cap, A.capc, grp, cur);
    }
    if (cf < 0) { cf = cur.total; ccf = cur.ctotal; }
    cw = cur.total - cf;
    ccw = cur.ctotal - ccf;
}

template <typename T, int DIM, int G>
__global__ void __launch_bounds__(kThreads) k_nbr(NbrArgs<T> A)
{
    using Q = typename XR<DIM>::type;
    const Group<G> grp;
    const int i = (blockIdx.x * blockDim.x + threadIdx.x) / G;
    if (i >= A.N) return;  // whole groups leave together
    const int s = A.simid[i];
    const bool fluid = i < A.Nf;
    const SimDev &S = A.sims[s];
    const Q me = ((const Q *)A.xr)[i];
    const Probe<DIM> P = make_probe<DIM>(S, me.x, me.y, XR<DIM>::z(me));
    if (grp.sub == 0) {
        const double pos3[3] = {P.xi, P.yi, P.zi};
        write_pos_record<T>(S, A.prec, i, pos3);
    }
    const int nx = S.ncell[0], ny = S.ncell[1], nz = DIM == 3 ? S.ncell[2] : 1;
    const int cx = cell_coord(P.xi, S.lo[0], S.inv_cs[0], nx);
    const int cy = cell_coord(P.yi, S.lo[1], S.inv_cs[1], ny);
    const int cz = DIM == 3 ? cell_coord(P.zi, S.lo[2], S.inv_cs[2], nz) : 0;
    // per-run shifts are exact when every periodic axis has at least 2m+3 cells
    // (then a block's cells lie within half a period of its centre, by a margin
    // of half a cell) and positions lie in [lo, hi)
    const int m3 = 2 * S.cell_div + 3;
    const bool general = (P.px && nx < m3) || (P.py && ny < m3) || (DIM == 3 && P.pz && nz < m3);
    ListCursor cur;
    int cf, cw, ccf, ccw;
    if (general) scan_block<T, DIM, G, true>(A, S, i, P, cx, cy, cz, fluid, cf, cw, ccf, ccw, cur, grp);
    else scan_block<T, DIM, G, false>(A, S, i, P, cx, cy, cz, fluid, cf, cw, ccf, ccw, cur, grp);
    const int cap = A.cap, capc = A.capc;
    if (cur.total > cap || cur.ctotal > capc) {
        if (grp.sub == 0) {
            atomicOr(&A.flags[F_NBR_OVERFLOW], 1);
            atomicMax(&A.flags[F_NBR_NEEDED], cur.total > cur.ctotal ? cur.total : cur.ctotal);
        }
        cf = cf < cap ? cf : cap;
        cw = cap - cf < cw ? cap - cf : cw;
        ccf = ccf < capc ? ccf : capc;
        ccw = capc - ccf < ccw ? capc - ccf : ccw;
    }
    if (grp.sub == 0) {
        A.cnt[i] = (uint32_t)cf | ((uint32_t)cw << 16);
        A.ccnt[i] = (uint32_t)ccf | ((uint32_t)ccw << 16);
    }
}

// Exact lists at the current positions from the candidate lists of the last
// build (same predicate, same order), plus new position records.
template <typename T, int DIM, int G>
__global__ void __launch_bounds__(kThreads) k_filter(NbrArgs<T> A)
{
    using Q = typename XR<DIM>::type;
    const Group<G> grp;
    const int i = (blockIdx.x * blockDim.x + threadIdx.x) / G;
    const bool active = i < A.N;
    const int N = A.N;
    const int s = active ? A.simid[i] : -1;
    int cf = 0, cw = 0;
    if (active) {
        const SimDev &S = A.sims[s];
        const Q *__restrict__ xr = (const Q *)A.xr;
        const Q me = xr[i];
        const Probe<DIM> P = make_probe<DIM>(S, me.x, me.y, XR<DIM>::z(me));
        const int *__restrict__ cand = A.cand + i;
        int *__restrict__ nbr = A.nbr + i;
        if (grp.sub == 0) {
            const double pos3[3] = {P.xi, P.yi, P.zi};
            write_pos_record<T>(S, A.prec, i, pos3);
        }
        const uint32_t cc = A.ccnt[i];
        const int ncf = (int)(cc & 0xffffu), nct = ncf + (int)(cc >> 16);
        int total = 0;
        for (int k0 = 0; k0 < nct; k0 += G * kBatch) {  // same trip count for the whole group
            int jj[kBatch];
            Q q[kBatch];
#pragma unroll
            for (int m = 0; m < kBatch; ++m) {
                const int k = k0 + m * G + grp.sub;
                jj[m] = k < nct ? cand[(size_t)k * N] : i;
            }
#pragma unroll
            for (int m = 0; m < kBatch; ++m) q[m] = xr[jj[m]];
#pragma unroll
            for (int m = 0; m < kBatch; ++m) {
                const int k = k0 + m * G + grp.sub;
                const bool in_x = k < nct && P.r2(q[m]) < P.kh2;
                const unsigned bx = grp.bits(in_x), bf = grp.bits(in_x && k < ncf);
                // the exact list is a subset of the candidates, so it fits the capacity
                if (in_x) nbr[(size_t)(total + grp.before(bx)) * N] = jj[m];
                total += __popc(bx);
                cf += __popc(bf);
            }
        }
        cw = total - cf;
        if (grp.sub == 0) A.cnt[i] = (uint32_t)cf | ((uint32_t)cw << 16);
    }
}

// ---- staged-tile neighbour kernel (2D) ---------------------------------------
// One workgroup per strip of tile_w x tile_h cells of one type (fluid or wall
// cells) of one sim. Every particle that a particle of the strip can reach sits
// in the strip's cells widened by cell_div cells on each side: fluid cells, and
// for the fluid particles of a sim with walls also wall cells. Their positions
// and slots are staged in LDS once, in (cell type, row, column) order with the
// periodic images as separate columns, and each particle then visits the same
// rows and trimmed windows as k_nbr, in the same order, with the same float64
// predicate and appends, reading its candidates from LDS: the lists are the
// same. A strip whose neighbourhood holds more than pmax particles reads them
// from global memory instead. The candidate loop has no global loads, so the
// list stores never hold it up.
constexpr int kTileThreads = 256;

template <typename T>
__global__ void __launch_bounds__(kTileThreads) k_nbr_tile(NbrArgs<T> A, const int4 *__restrict__ strips, int pmax)
{
    extern __shared__ double2 tile_lds[];
    __shared__ int s_pb[kMaxTileRows + 1], s_sb[kMaxTileRows], s_scan[kTileThreads / 64 + 1];
    const int4 st = strips[blockIdx.x];
    const int s = st.x, tp = st.y, y0 = st.z, x0 = st.w;
    const SimDev &S = A.sims[s];
    const int nx = S.ncell[0], ny = S.ncell[1], md = S.cell_div;
    const int xe = min(x0 + S.tile_w, nx), ye = min(y0 + S.tile_h, ny), nys = ye - y0;
    const uint32_t *__restrict__ cstart = A.cell_start;
    const int tid = threadIdx.x;
    // the strip's particles: one contiguous run of slots per cell row
    if (tid < nys) {
        const int row = S.key_base + (tp ? A.C : 0) + (y0 + tid) * nx;
        const int b = (int)cstart[row + x0], e = (int)cstart[row + xe];
        s_sb[tid] = b;
        s_pb[tid + 1] = e - b;
    }
    __syncthreads();
    if (tid == 0) {
        s_pb[0] = 0;
        for (int t = 0; t < nys; ++t) s_pb[t + 1] += s_pb[t];
    }
    __syncthreads();
    const int np = s_pb[nys];
    if (np == 0) return;  // an empty strip (uniform)

    // staged columns: virtual cells x0 - m .. x0 + tile_w - 1 + m of virtual rows
    // y0 - m .. y0 + tile_h - 1 + m, per staged cell type
    const int ntp = (tp == 0 && S.nw > 0) ? 2 : 1;
    const int VX = S.tile_w + 2 * md, VY = S.tile_h + 2 * md;
    const int NC = ntp * VY * VX;
    double2 *lpos = tile_lds;
    int *lslot = (int *)(lpos + pmax);
    int *off = lslot + pmax;  // NC + 1 entries: first staged index of each cell
    auto phys = [](int v, int n, int per) { return per ? (v < 0 ? v + n : (v >= n ? v - n : v)) : v; };
    for (int q = tid; q < NC; q += kTileThreads) {
        const int r = q / VX, c = q - r * VX;
        const int t = r / VY;
        const int vy = y0 - md + (r - t * VY), vx = x0 - md + c;
        const bool ok = (S.periodic[1] || (vy >= 0 && vy < ny)) && (S.periodic[0] || (vx >= 0 && vx < nx));
        int n = 0;
        if (ok) {
            const int key = S.key_base + (t ? A.C : 0) + phys(vy, ny, S.periodic[1]) * nx + phys(vx, nx, S.periodic[0]);
            n = (int)cstart[key + 1] - (int)cstart[key];
        }
        off[q] = n;
    }
    __syncthreads();
    {   // exclusive scan of the counts in place; off[NC] = the total
        const int per = (NC + kTileThreads - 1) / kTileThreads;
        const int b = min(tid * per, NC), e = min(b + per, NC);
        int sum = 0;
        for (int k = b; k < e; ++k) sum += off[k];
        const int lane = tid & 63, wave = tid >> 6;
        int incl = sum;
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(incl, o, 64);
            if (lane >= o) incl += y;
        }
        if (lane == 63) s_scan[wave] = incl;
        __syncthreads();
        if (tid == 0) {
            int acc = 0;
            for (int w = 0; w < kTileThreads / 64; ++w) {
                const int v = s_scan[w];
                s_scan[w] = acc;
                acc += v;
            }
            s_scan[kTileThreads / 64] = acc;
        }
        __syncthreads();
        int run = s_scan[wave] + incl - sum;
        for (int k = b; k < e; ++k) {
            const int v = off[k];
            off[k] = run;
            run += v;
        }
        if (tid == 0) off[NC] = s_scan[kTileThreads / 64];
        __syncthreads();
    }
    const int nst = off[NC];
    const bool staged = nst <= pmax;  // uniform
    const double2 *__restrict__ xr = (const double2 *)A.xr;
    if (staged) {
        for (int q = tid; q < nst; q += kTileThreads) {
            int lo = 0, hi = NC - 1;  // the cell holding staged particle q: last k with off[k] <= q
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (off[mid] <= q) lo = mid;
                else hi = mid - 1;
            }
            const int r = lo / VX, c = lo - r * VX;
            const int t = r / VY;
            const int vy = y0 - md + (r - t * VY), vx = x0 - md + c;
            const int key = S.key_base + (t ? A.C : 0) + phys(vy, ny, S.periodic[1]) * nx + phys(vx, nx, S.periodic[0]);
            const int j = (int)cstart[key] + (q - off[lo]);
            lpos[q] = xr[j];
            lslot[q] = j;
        }
    }
    __syncthreads();

    const int N = A.N, cap = A.cap, capc = A.capc;
    const double cr2 = S.cand_r2;
    for (int pi = tid; pi < np; pi += kTileThreads) {
        int t = 0;
        while (t + 1 < nys && s_pb[t + 1] <= pi) ++t;
        const int i = s_sb[t] + (pi - s_pb[t]);
        const double2 me = xr[i];
        const Probe<2> P = make_probe<2>(S, me.x, me.y, 0.0);
        {
            const double pos3[3] = {P.xi, P.yi, 0.0};
            write_pos_record<T>(S, A.prec, i, pos3);
        }
        const int cx = cell_coord(P.xi, S.lo[0], S.inv_cs[0], nx);
        const int cy = cell_coord(P.yi, S.lo[1], S.inv_cs[1], ny);
        // the row windows of k_nbr's trimmed path (float, cell units relative
        // to the particle's cell, widened by 1e-5 cells)
        auto frac = [&](double p, int a, int c) {
            const double f = (p - S.lo[a]) * S.inv_cs[a] - (double)c;
            const double lim = (double)md + 3.0;
            return (float)(f < -lim ? -lim : (f > lim + 1.0 ? lim + 1.0 : f));
        };
        const float fx = frac(P.xi, 0, cx), fy = frac(P.yi, 1, cy);
        const float csy = (float)S.cs[1], icsx = (float)S.inv_cs[0], cr2f = (float)cr2;
        // next free entries of the two lists (column-major: one column per entry)
        int *__restrict__ pn = A.nbr + i;
        int *__restrict__ pc = A.cand + i;
        ListCursor cur;
        int cf = -1, ccf = 0;
        auto test = [&](const double2 &q, int j, double sx, double sy) {
            const double r2 = P.r2s(q, sx, sy, 0.0);
            const bool ok = j != i;
            const bool in_c = ok && r2 < cr2, in_x = ok && r2 < P.kh2;
            if (in_c && cur.ctotal < capc) *pc = j;
            if (in_x && cur.total < cap) *pn = j;
            if (in_c) { ++cur.ctotal; pc += N; }
            if (in_x) { ++cur.total; pn += N; }
        };
        for (int tt = 0; tt < ntp; ++tt) {
            if (tt == 1 && cf < 0) { cf = cur.total; ccf = cur.ctotal; }
            for (int v = 0; v <= 2 * md; ++v) {
                const int vy = cy - md + v;
                if (!P.py && (vy < 0 || vy >= ny)) continue;
                const int py = phys(vy, ny, P.py);
                const double sy = P.py ? (vy < 0 ? P.Ly : (vy >= ny ? -P.Ly : 0.0)) : 0.0;
                const float o = (float)(vy - cy);  // the row's slab is [o, o + 1) in cell units
                const float below = (!P.py && py == 0) ? 0.f : o - fy;
                const float above = (!P.py && py == ny - 1) ? 0.f : fy - (o + 1.f);
                const float dd = fmaxf(below, above) - 1e-5f;
                const float dy = dd > 0.f ? dd * csy : 0.f;
                const float rem = cr2f - dy * dy;
                if (rem < 0.f) continue;
                const float wc = __builtin_amdgcn_sqrtf(rem) * icsx + 1e-5f;
                int lo_c = cx + (int)floorf(fx - wc);
                int hi_c = cx + (int)floorf(fx + wc);
                lo_c = lo_c > cx - md ? lo_c : cx - md;
                hi_c = hi_c < cx + md ? hi_c : cx + md;
                // runs in virtual columns: [a0, b0] unshifted, then [a1, b1] with shift s1
                int a0, b0, a1 = 0, b1 = -1;
                double s1 = 0.0;
                if (P.px) {
                    a0 = lo_c > 0 ? lo_c : 0;
                    b0 = hi_c < nx - 1 ? hi_c : nx - 1;
                    if (lo_c < 0) { a1 = lo_c; b1 = -1; s1 = P.Lx; }
                    else if (hi_c > nx - 1) { a1 = nx; b1 = hi_c; s1 = -P.Lx; }
                } else {
                    // edge cells extend outwards: a window beyond the grid still meets them
                    a0 = lo_c < 0 ? 0 : (lo_c > nx - 1 ? nx - 1 : lo_c);
                    b0 = hi_c < 0 ? 0 : (hi_c > nx - 1 ? nx - 1 : hi_c);
                }
                const int rr = (tt * VY + (vy - (y0 - md))) * VX - (x0 - md);
                const int kb = S.key_base + (tt ? A.C : 0) + py * nx;
                for (int k = 0; k < 2; ++k) {
                    const int va = k ? a1 : a0, vb = k ? b1 : b0;
                    if (vb < va) continue;
                    const double sx = k ? s1 : 0.0;
                    if (staged) {
                        // a run's cells are consecutive keys, so its slots are
                        // consecutive: slot = first slot + offset in the run;
                        // four candidates' positions are read before the tests
                        const int qa = off[rr + va], qb = off[rr + vb + 1];
                        if (qa < qb) {
                            const int j0 = lslot[qa] - qa;
                            for (int q0 = qa; q0 < qb; q0 += 4) {
                                double2 pq[4];
#pragma unroll
                                for (int u = 0; u < 4; ++u) pq[u] = lpos[q0 + u < qb ? q0 + u : qb - 1];
#pragma unroll
                                for (int u = 0; u < 4; ++u)
                                    if (q0 + u < qb) test(pq[u], j0 + q0 + u, sx, sy);
                            }
                        }
                    } else {
                        const int ja = (int)cstart[kb + phys(va, nx, P.px)];
                        const int jb = (int)cstart[kb + phys(vb, nx, P.px) + 1];
                        for (int j = ja; j < jb; ++j) test(xr[j], j, sx, sy);
                    }
                }
            }
        }
        if (cf < 0) { cf = cur.total; ccf = cur.ctotal; }
        int cw = cur.total - cf, ccw = cur.ctotal - ccf;
        if (cur.total > cap || cur.ctotal > capc) {
            atomicOr(&A.flags[F_NBR_OVERFLOW], 1);
            atomicMax(&A.flags[F_NBR_NEEDED], cur.total > cur.ctotal ? cur.total : cur.ctotal);
            cf = cf < cap ? cf : cap;
            cw = cap - cf < cw ? cap - cf : cw;
            ccf = ccf < capc ? ccf : capc;
            ccw = capc - ccf < ccw ? capc - ccf : ccw;
        }
        A.cnt[i] = (uint32_t)cf | ((uint32_t)cw << 16);
        A.ccnt[i] = (uint32_t)ccf | ((uint32_t)ccw << 16);
    }
}

inline int grid_for(int n) { return n > 0 ? ceil_div(n, kThreads) : 1; }

template <typename T, int DIM, int G> void launch_g(Ctx &c, const NbrArgs<T> &a, bool filter)
{
    const dim3 grid(grid_for((int)std::min<int64_t>((int64_t)a.N * G, INT32_MAX)));
    if (filter) DTSPH_LAUNCH(c, (k_filter<T, DIM, G>), grid, dim3(kThreads), 0, c.stream, a);
    else DTSPH_LAUNCH(c, (k_nbr<T, DIM, G>), grid, dim3(kThreads), 0, c.stream, a);
}

// lanes per particle in the neighbour kernels: the autotuner's choice, else
// enough threads for ~8 waves per SIMD
template <typename T> void launch_grouped(Ctx &c, const NbrArgs<T> &a, bool filter)
{
    if (!filter && c.nbr_tiles && c.n_strips > 0) {
        const size_t lds = (size_t)c.tile_pmax * (sizeof(double2) + sizeof(int)) + (size_t)c.tile_offmax * sizeof(int);
        DTSPH_LAUNCH(c, k_nbr_tile<T>, dim3(c.n_strips), dim3(kTileThreads), lds, c.stream, a, c.strips, c.tile_pmax);
        return;
    }
    int g = filter ? c.g_filter : c.g_nbr;
    if (g <= 0) {
        g = 1;
        while (g < 8 && (int64_t)g * a.N < (int64_t)256 * 2048) g *= 2;
    }
    if (c.max_dim == 2) {
        if (g == 1) launch_g<T, 2, 1>(c, a, filter);
        else if (g == 2) launch_g<T, 2, 2>(c, a, filter);
        else if (g == 4) launch_g<T, 2, 4>(c, a, filter);
        else launch_g<T, 2, 8>(c, a, filter);
    } else {
        if (g == 1) launch_g<T, 3, 1>(c, a, filter);
        else if (g == 2) launch_g<T, 3, 2>(c, a, filter);
        else if (g == 4) launch_g<T, 3, 4>(c, a, filter);
        else launch_g<T, 3, 8>(c, a, filter);
    }
}

}  // namespace

template <typename T>
void build_cells(Ctx &c, int loop_fixed)
{
    c.tstats.full_builds++;
    hipStream_t st = c.stream;
    const int N = c.N, nkeys = 2 * c.C;
    const int b = c.buf, o = c.buf ^ 1;
    int t0 = timer_begin(c, 2);
    auto keys = c.max_dim == 2 ? k_keys<2> : k_keys<3>;
    DTSPH_LAUNCH(c, keys, dim3(grid_for(N)), dim3(kThreads), 0, st, N, c.Nf, c.C, c.x[c.xb], c.simid[b],
                       c.sims, c.key, c.rank, c.count);
    const int nblk = ceil_div(nkeys, kScanTile);
    DTSPH_LAUNCH(c, k_scan_reduce, dim3(nblk), dim3(kThreads), 0, st, c.count, nkeys, c.scan_tmp);
    DTSPH_LAUNCH(c, k_scan_down, dim3(nblk), dim3(kThreads), 0, st, c.count, nkeys, c.scan_tmp,
                       c.cell_start);
    DTSPH_LAUNCH(c, k_scatter, dim3(grid_for(N)), dim3(kThreads), 0, st, N, c.key, c.rank, c.cell_start,
                       c.perm);
    GatherArgs<T> g;
    g.N = N; g.Nf = c.Nf; g.Nw = c.Nw;
    g.perm = c.perm; g.key = c.key; g.cell_start = c.cell_start;
    g.src_of = c.rank;  // the arrival ranks are consumed by k_scatter
    g.flags = c.flags;
    g.orig_in = c.orig[b]; g.orig_out = c.orig[o];
    g.simid_in = c.simid[b]; g.simid_out = c.simid[o];
    g.x_in = c.x[c.xb]; g.x_out = c.x[c.xb ^ 1];
    g.xn_in = c.xn[b]; g.xn_out = c.xn[o];
    g.xr = c.xr; g.dim = c.max_dim;
    g.vn_in = (const T *)c.vn[b]; g.vn_out = (T *)c.vn[o];
    g.dv_in = (const T *)c.dv[b]; g.dv_out = (T *)c.dv[o];
    g.w_in = (const T *)c.w[b]; g.w_out = (T *)c.w[o];
    g.w0_in = (const T *)c.w0[b]; g.w0_out = (T *)c.w0[o];
    g.dp_in = (const T *)c.dp[b]; g.dp_out = (T *)c.dp[o];
    g.pm_in = c.pm[b]; g.pm_out = c.pm[o];
    g.pn_in = c.pn[b]; g.pn_out = c.pn[o];
    g.vw_in = (const T *)c.vw[b]; g.vw_out = (T *)c.vw[o];
    g.pw_in = (const T *)c.pw[b]; g.pw_out = (T *)c.pw[o];
    g.loop = loop_fixed;
    g.add_half = c.p_half ? 0 : 1;
    g.n_sims = c.n_sims;
    g.sims = c.sims;
    g.iters = c.iters;
    g.rec = c.vp[c.cur];
    DTSPH_LAUNCH(c, k_rank_gather<T>, dim3(grid_for(N)), dim3(kThreads), 0, st, g);
    c.buf = o;
    c.xb ^= 1;
    c.records_fresh = false;  // the slots moved
    launch_nbr_lists<T>(c, false);
    timer_end(c, t0, 2);
}

// Exact lists from the candidate lists (no sort).
template <typename T>
void filter_lists(Ctx &c)
{
    c.tstats.list_filters++;
    int t0 = timer_begin(c, 3);
    launch_nbr_lists<T>(c, true);
    timer_end(c, t0, 3);
}

// The neighbour-list kernel alone (filter = false; needs a valid cell table) or
// the filter (needs candidate lists covering the current positions).
template <typename T>
void launch_nbr_lists(Ctx &c, bool filter)
{
    NbrArgs<T> a;
    a.N = c.N; a.Nf = c.Nf; a.C = c.C; a.cap = c.cap;
    a.x = c.x[c.xb]; a.simid = c.simid[c.buf]; a.sims = c.sims; a.cell_start = c.cell_start;
    a.nbr = c.nbr; a.cnt = c.cnt; a.prec = c.prec; a.flags = c.flags;
    a.capc = c.capc; a.cand = c.cand; a.ccnt = c.ccnt; a.xr = c.xr;
    c.coef_valid = false;  // cached pair coefficients belong to the old lists
    launch_grouped<T>(c, a, filter);
    DTSPH_HIP_CHECK(hipGetLastError());
}

template void filter_lists<float>(Ctx &);
template void filter_lists<double>(Ctx &);
template void launch_nbr_lists<float>(Ctx &, bool);
template void launch_nbr_lists<double>(Ctx &, bool);
template void build_cells<float>(Ctx &, int);
template void build_cells<double>(Ctx &, int);

}  // namespace dtsph
