// Cell-linked list and neighbour lists (HBM-bound streaming kernels).
//
// Per build:  k_keys (cell key + rank within cell by integer atomics)
//          -> three-kernel exclusive scan of the per-key counts (= cell-start table)
//          -> k_scatter (slot of each particle) -> k_cell_sort (ties by caller index)
//          -> k_gather (all state arrays into the new order)
//          -> k_nbr (exact neighbour lists, position records, pair counts).
// The sort is a counting sort over the whole key (one radix digit holding the
// cell id): keys are dense and each cell holds a handful of particles, so one
// histogram + scan + scatter moves the data once instead of once per 8-bit digit.
#include "dtsph_internal.h"

namespace dtsph {

namespace {

constexpr int kThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kThreads * kScanItems;  // 4096 keys per block

__global__ void k_fill_u32(uint32_t *p, int n, uint32_t v)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u64(unsigned long long *p, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

__device__ inline int cell_coord(double x, double lo, double inv_cs, int n)
{
    double f = floor((x - lo) * inv_cs);
    int c = 0;
    if (f >= 0.0) c = f > (double)(n - 1) ? n - 1 : (int)f;
    return c;
}

__device__ inline int cell_linear(const SimDev &S, const double *x, int N, int i, int c3[3])
{
    c3[0] = c3[1] = c3[2] = 0;
    for (int a = 0; a < S.dim; ++a) c3[a] = cell_coord(x[a * N + i], S.lo[a], S.inv_cs[a], S.ncell[a]);
    return (c3[2] * S.ncell[1] + c3[1]) * S.ncell[0] + c3[0];
}

__global__ void k_keys(int N, int Nf, int C, const double *__restrict__ x, const int *__restrict__ simid,
                       const SimDev *__restrict__ sims, uint32_t *__restrict__ key,
                       uint32_t *__restrict__ rank, uint32_t *__restrict__ count)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const SimDev &S = sims[simid[i]];
    int c3[3];
    uint32_t k = (uint32_t)(S.key_base + cell_linear(S, x, N, i, c3) + (i >= Nf ? C : 0));
    key[i] = k;
    rank[i] = atomicAdd(&count[k], 1u);
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

__global__ void k_scan_reduce(const uint32_t *__restrict__ in, int n, uint32_t *__restrict__ sums)
{
    __shared__ uint32_t lds[kThreads / 64];
    int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    uint32_t s = 0;
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) s += in[base + k];
    uint32_t tot;
    block_exclusive_scan(s, lds, tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Single block: exclusive scan of the block sums (n <= kScanTile).
__global__ void k_scan_top(uint32_t *__restrict__ sums, int n)
{
    __shared__ uint32_t lds[kThreads / 64];
    int base = threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = base + k < n ? sums[base + k] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t run = block_exclusive_scan(s, lds, tot);
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) sums[base + k] = run;
        run += v[k];
    }
}

__global__ void k_scan_down(const uint32_t *__restrict__ in, int n, const uint32_t *__restrict__ sums,
                            uint32_t *__restrict__ out)
{
    __shared__ uint32_t lds[kThreads / 64];
    int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = base + k < n ? in[base + k] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t run = block_exclusive_scan(s, lds, tot) + sums[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    // the total lands one past the end
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == blockDim.x - 1) out[n] = run;
}

__global__ void k_scatter(int N, const uint32_t *__restrict__ key, const uint32_t *__restrict__ rank,
                          const uint32_t *__restrict__ cell_start, uint32_t *__restrict__ perm)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    perm[cell_start[key[i]] + rank[i]] = (uint32_t)i;
}

// Order each cell's slots by caller index (insertion sort; cells are small).
__global__ void k_cell_sort(int nkeys, const uint32_t *__restrict__ cell_start, uint32_t *__restrict__ perm,
                            const int *__restrict__ orig, int *__restrict__ flags)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nkeys) return;
    int b = (int)cell_start[k], e = (int)cell_start[k + 1];
    if (e - b > kMaxCellOccupancy) {
        atomicOr(&flags[F_CELL_OVERFLOW], 1);
        return;
    }
    for (int m = b + 1; m < e; ++m) {
        uint32_t v = perm[m];
        int ov = orig[v];
        int j = m - 1;
        while (j >= b && orig[perm[j]] > ov) {
            perm[j + 1] = perm[j];
            --j;
        }
        perm[j + 1] = v;
    }
}

template <typename T>
struct GatherArgs {
    int N, Nf, Nw;
    const uint32_t *perm;
    const int *orig_in, *simid_in;
    int *orig_out, *simid_out;
    const double *x_in, *xn_in;
    double *x_out, *xn_out;
    const T *vn_in, *dv_in, *w_in, *dp_in;
    T *vn_out, *dv_out, *w_out, *dp_out;
    const double *pm_in, *pn_in;
    double *pm_out, *pn_out;
    const T *vw_in, *pw_in;
    T *vw_out, *pw_out;
};

template <typename T>
__global__ void k_gather(GatherArgs<T> A)
{
    int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= A.N) return;
    const int N = A.N, Nf = A.Nf, Nw = A.Nw;
    int s = (int)A.perm[d];
    A.orig_out[d] = A.orig_in[s];
    A.simid_out[d] = A.simid_in[s];
    for (int a = 0; a < 3; ++a) {
        A.x_out[a * N + d] = A.x_in[a * N + s];
        A.xn_out[a * N + d] = A.xn_in[a * N + s];
    }
    if (d < Nf) {
        for (int a = 0; a < 3; ++a) {
            A.vn_out[a * Nf + d] = A.vn_in[a * Nf + s];
            A.dv_out[a * Nf + d] = A.dv_in[a * Nf + s];
            A.w_out[a * Nf + d] = A.w_in[a * Nf + s];
        }
        A.pm_out[d] = A.pm_in[s];
        A.pn_out[d] = A.pn_in[s];
        A.dp_out[d] = A.dp_in[s];
    } else {
        int dw = d - Nf, sw = s - Nf;
        for (int a = 0; a < 3; ++a) A.vw_out[a * Nw + dw] = A.vw_in[a * Nw + sw];
        A.pw_out[dw] = A.pw_in[sw];
    }
}

// Exact neighbour predicate: minimum-image separation, squared length summed
// as (dx*dx + dy*dy) + dz*dz in float64 without contraction, strict < (kh)^2.
__device__ inline bool exact_neighbor(const SimDev &S, const double xi[3], const double xj[3])
{
#pragma clang fp contract(off)
    double d[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < S.dim; ++a) {
        double s = xi[a] - xj[a];
        if (S.periodic[a]) {
            if (s > S.halfL[a]) s -= S.L[a];
            else if (s < -S.halfL[a]) s += S.L[a];
        }
        d[a] = s;
    }
    double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    return r2 < S.kh2;
}

// Distinct neighbouring cell indices along one axis, ascending.
__device__ inline int axis_cells(int c, int n, int periodic, int out[3])
{
    int m = 0;
    for (int o = -1; o <= 1; ++o) {
        int v = c + o;
        if (periodic) v = (v + n) % n;
        else if (v < 0 || v >= n) continue;
        bool dup = false;
        for (int k = 0; k < m; ++k) dup |= out[k] == v;
        if (!dup) out[m++] = v;
    }
    for (int a = 1; a < m; ++a)  // sort (m <= 3)
        for (int b = a; b > 0 && out[b - 1] > out[b]; --b) {
            int t = out[b];
            out[b] = out[b - 1];
            out[b - 1] = t;
        }
    return m;
}

template <typename T>
struct NbrArgs {
    int N, Nf, C, cap;
    const double *x;
    const int *simid;
    const SimDev *sims;
    const uint32_t *cell_start;
    int *nbr;
    uint32_t *cnt;
    void *prec;
    unsigned long long *pairs;
    int *flags;
};

template <typename T>
__device__ inline void write_record(const SimDev &S, void *prec, int i, const double xi[3]);

template <>
__device__ inline void write_record<float>(const SimDev &S, void *prec, int i, const double xi[3])
{
    uint32_t q[4] = {0u, 0u, 0u, 0u};
    for (int a = 0; a < S.dim; ++a) {
        double v = floor((xi[a] - S.lo[a]) * S.q_inv[a]);
        q[a] = (uint32_t)(unsigned long long)(long long)v;
    }
    ((uint4 *)prec)[i] = make_uint4(q[0], q[1], q[2], 0u);
}

template <>
__device__ inline void write_record<double>(const SimDev &S, void *prec, int i, const double xi[3])
{
    (void)S;
    ((double4 *)prec)[i] = make_double4(xi[0], xi[1], xi[2], 0.0);
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_nbr(NbrArgs<T> A)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.N) return;
    const int N = A.N;
    const int s = A.simid[i];
    const SimDev &S = A.sims[s];
    const bool fluid = i < A.Nf;
    double xi[3] = {A.x[i], A.x[N + i], A.x[2 * N + i]};
    if (S.dim < 3) xi[2] = 0.0;
    write_record<T>(S, A.prec, i, xi);

    int c3[3];
    cell_linear(S, A.x, N, i, c3);
    int ax[3][3], na[3];
    for (int a = 0; a < 3; ++a) {
        if (a < S.dim) na[a] = axis_cells(c3[a], S.ncell[a], S.periodic[a], ax[a]);
        else { na[a] = 1; ax[a][0] = 0; }
    }
    const int cap = A.cap;
    int count[2] = {0, 0};
    int total = 0;
    for (int tp = 0; tp < (fluid ? 2 : 1); ++tp) {
        const int base = S.key_base + (tp ? A.C : 0);
        for (int u = 0; u < na[2]; ++u)
            for (int v = 0; v < na[1]; ++v) {
                const int row = base + (ax[2][u] * S.ncell[1] + ax[1][v]) * S.ncell[0];
                int k = 0;
                while (k < na[0]) {  // contiguous runs of x cells
                    int xa = ax[0][k], xb = xa;
                    while (k + 1 < na[0] && ax[0][k + 1] == xb + 1) { ++k; ++xb; }
                    ++k;
                    const int jb = (int)A.cell_start[row + xa], je = (int)A.cell_start[row + xb + 1];
                    for (int j = jb; j < je; ++j) {
                        if (j == i) continue;
                        double xj[3] = {A.x[j], A.x[N + j], S.dim == 3 ? A.x[2 * N + j] : 0.0};
                        if (!exact_neighbor(S, xi, xj)) continue;
                        if (total < cap) A.nbr[(size_t)total * N + i] = j;
                        ++total;
                        ++count[tp];
                    }
                }
            }
    }
    if (total > cap) {
        atomicOr(&A.flags[F_NBR_OVERFLOW], 1);
        atomicMax(&A.flags[F_NBR_NEEDED], total);
        count[0] = count[0] < cap ? count[0] : cap;
        count[1] = cap - count[0] < count[1] ? cap - count[0] : count[1];
    }
    A.cnt[i] = (uint32_t)count[0] | ((uint32_t)count[1] << 16);
    if (fluid) atomicAdd(&A.pairs[s], (unsigned long long)(count[0] + count[1]));
}

inline int grid_for(int n) { return n > 0 ? ceil_div(n, kThreads) : 1; }

}  // namespace

template <typename T>
void build_cells(Ctx &c)
{
    hipStream_t st = c.stream;
    const int N = c.N, nkeys = 2 * c.C;
    const int b = c.buf, o = c.buf ^ 1;
    int t0 = timer_begin(c);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(nkeys)), dim3(kThreads), 0, st, c.count, nkeys, 0u);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(kThreads), 0, st, (uint32_t *)c.flags, (int)F_COUNT, 0u);
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(c.n_sims)), dim3(kThreads), 0, st, c.pairs, c.n_sims);
    hipLaunchKernelGGL(k_keys, dim3(grid_for(N)), dim3(kThreads), 0, st, N, c.Nf, c.C, c.x[c.xb], c.simid[b],
                       c.sims, c.key, c.rank, c.count);
    const int nblk = ceil_div(nkeys, kScanTile);
    hipLaunchKernelGGL(k_scan_reduce, dim3(nblk), dim3(kThreads), 0, st, c.count, nkeys, c.scan_tmp);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kThreads), 0, st, c.scan_tmp, nblk);
    hipLaunchKernelGGL(k_scan_down, dim3(nblk), dim3(kThreads), 0, st, c.count, nkeys, c.scan_tmp,
                       c.cell_start);
    hipLaunchKernelGGL(k_scatter, dim3(grid_for(N)), dim3(kThreads), 0, st, N, c.key, c.rank, c.cell_start,
                       c.perm);
    hipLaunchKernelGGL(k_cell_sort, dim3(grid_for(nkeys)), dim3(kThreads), 0, st, nkeys, c.cell_start, c.perm,
                       c.orig[b], c.flags);
    GatherArgs<T> g;
    g.N = N; g.Nf = c.Nf; g.Nw = c.Nw;
    g.perm = c.perm;
    g.orig_in = c.orig[b]; g.orig_out = c.orig[o];
    g.simid_in = c.simid[b]; g.simid_out = c.simid[o];
    g.x_in = c.x[c.xb]; g.x_out = c.x[c.xb ^ 1];
    g.xn_in = c.xn[b]; g.xn_out = c.xn[o];
    g.vn_in = (const T *)c.vn[b]; g.vn_out = (T *)c.vn[o];
    g.dv_in = (const T *)c.dv[b]; g.dv_out = (T *)c.dv[o];
    g.w_in = (const T *)c.w[b]; g.w_out = (T *)c.w[o];
    g.dp_in = (const T *)c.dp[b]; g.dp_out = (T *)c.dp[o];
    g.pm_in = c.pm[b]; g.pm_out = c.pm[o];
    g.pn_in = c.pn[b]; g.pn_out = c.pn[o];
    g.vw_in = (const T *)c.vw[b]; g.vw_out = (T *)c.vw[o];
    g.pw_in = (const T *)c.pw[b]; g.pw_out = (T *)c.pw[o];
    hipLaunchKernelGGL(k_gather<T>, dim3(grid_for(N)), dim3(kThreads), 0, st, g);
    c.buf = o;
    c.xb ^= 1;
    NbrArgs<T> a;
    a.N = N; a.Nf = c.Nf; a.C = c.C; a.cap = c.cap;
    a.x = c.x[c.xb]; a.simid = c.simid[o]; a.sims = c.sims; a.cell_start = c.cell_start;
    a.nbr = c.nbr; a.cnt = c.cnt; a.prec = c.prec; a.pairs = c.pairs; a.flags = c.flags;
    hipLaunchKernelGGL(k_nbr<T>, dim3(grid_for(N)), dim3(kThreads), 0, st, a);
    DTSPH_HIP_CHECK(hipGetLastError());
    timer_end(c, t0, 2);
}

template void build_cells<float>(Ctx &);
template void build_cells<double>(Ctx &);

}  // namespace dtsph
