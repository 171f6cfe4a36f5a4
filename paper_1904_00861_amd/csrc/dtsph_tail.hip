// Persistent tail of a pseudo-time loop (Algorithm 2, the loop over k, for the
// sims of a batch still iterating once most have stopped).
//
// In a batch whose sims need very different iteration counts, the last
// iterations of a loop involve a few small sims: each iteration is then a
// handful of workgroups, and plain launches (pair pass, residual reduction with
// the next wall pass) cost their launch and dependency floors, several times
// the work. Once a report shows that the sims still iterating cover few tiles,
// one cooperative launch runs the rest of their loop: each workgroup owns one
// tile and keeps its sim's constants and loop state on chip, and the
// workgroups of a sim meet at a barrier of their own after each pair pass (two
// levels: groups of kTailGroup workgroups count on a word of their own, the
// last of each group on the sim's word). Every workgroup then closes the
// iteration itself (residual reduction and stop test, from the sim's partials),
// so all of them take the same stop decision without a second round trip; the
// sim's first workgroup stores the loop state and the report. The partials
// alternate between two buffers with the iteration's parity, so a workgroup
// that starts the next pass never overwrites partials another is still
// reading. A sim with walls computes them for the next iteration after the
// close and meets again before the next pass. Sims never wait for each other.
//
// Results are bit-identical to plain launches: the same pair-pass code per
// tile, the residual reduction in the same order as k_finalize (per segment,
// then over the segments, with the same per-wave butterflies and wave order for
// any workgroup size), the same stop test and wall pass.
//
// Every barrier wait is bounded: a wait that gives up sets an error word and its
// workgroup leaves; the sims involved then never publish their reports, which
// the host's wait turns into an error once the launch has ended.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "dtsph_pass_dev.h"

namespace dtsph {

namespace {

struct TailArgs {
    int k0;              // iterations every sim in the launch has run
    uint32_t *arrive;    // per sim: group arrivals at its barrier (zero at launch)
    uint32_t *group;     // per group of a sim's workgroups (tile_begin / kTailGroup + sim + group)
    int *err;            // set when a wait gives up
    long long spin;      // polls of a barrier word before a wait gives up
    double4 *part4[2];   // residual partials by iteration parity ([0]: the plain launches' buffer)
    double2 *part2[2];
    uint32_t outside[kTailMaxSims / 32];  // sims not in the launch (stopped before it)
};

// A workgroup's place in its sim's barrier.
struct TailSeat {
    uint32_t *group;     // its group's word
    uint32_t *sim;       // the sim's word (sims of several groups)
    uint32_t gsize;      // workgroups in its group
    uint32_t ngroups;    // groups of the sim
};

// fin_block_reduce's reduction of kFinThreads values for a workgroup of any
// multiple of 64 threads: value vt comes from load(vt, v); the waves take the
// same 64-value groups in turn, with the same butterflies, and thread 0 adds the
// group sums in the same order, so the result (thread 0) is bit-identical.
// Values from n on are zero: their groups are not loaded, and thread 0 combines
// +0.0 for them (which is what their butterflies give).
template <typename L> __device__ inline void fin_reduce_any(double out[6], int n, L load)
{
    constexpr int G = kFinThreads / 64;
    __shared__ double lds[G][6];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int gn = (n + 63) / 64;  // groups holding values
    for (int w0 = 0; w0 < gn; w0 += nw) {
        const int w = w0 + wave;
        if (w < gn) {  // uniform per wave
            double v[6];
            load(w * 64 + lane, v);
            for (int o = 32; o > 0; o >>= 1) {
                v[0] += __shfl_xor(v[0], o, 64);
                v[1] += __shfl_xor(v[1], o, 64);
                v[5] += __shfl_xor(v[5], o, 64);
                v[2] = fmax(v[2], __shfl_xor(v[2], o, 64));
                v[3] = fmax(v[3], __shfl_xor(v[3], o, 64));
                v[4] = fmax(v[4], __shfl_xor(v[4], o, 64));
            }
            if (lane == 0)
                for (int k = 0; k < 6; ++k) lds[w][k] = v[k];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < 6; ++k) out[k] = gn > 0 ? lds[0][k] : 0.0;
        for (int w = 1; w < G; ++w) {
            double g[6];
            for (int k = 0; k < 6; ++k) g[k] = w < gn ? lds[w][k] : 0.0;
            out[0] += g[0];
            out[1] += g[1];
            out[2] = fmax(out[2], g[2]);
            out[3] = fmax(out[3], g[3]);
            out[4] = fmax(out[4], g[4]);
            out[5] += g[5];
        }
    }
    __syncthreads();
}

// This thread's values of the first round of the residual reduction of a
// tail sim (fin_reduce_any's value wave * 64 + lane), all issued at once right
// after the barrier.
__device__ inline void prefetch_partials(double v[6], const SimDev &S, const double4 *p4, const double2 *p2)
{
    const int b = S.tile_begin, n = S.tile_end - S.tile_begin;
    const int vt = (int)threadIdx.x;  // wave * 64 + lane
    for (int k = 0; k < 6; ++k) v[k] = 0.0;
    if (vt < n) {
        const double4 p = p4[b + vt];
        const double2 q = p2[b + vt];
        v[0] = p.x; v[1] = p.y; v[2] = p.z; v[3] = p.w; v[4] = q.x; v[5] = q.y;
    }
}

// Closes iteration It.iters of sim s in the calling workgroup (every thread;
// after sim_meet, so that every tile's partials p4, p2 are visible; pre holds
// this thread's first-round values from prefetch_partials): a tail sim is one
// residual segment (kTailSimTiles <= kSegTiles), reduced as k_finalize reduces
// it, then the sum over the one segment (on thread 0: the same operations that
// k_finalize's reduction applies to it), and the stop test on the workgroup's
// own copy of the loop state It; every workgroup of the sim computes the same.
// When the sim stops, the writer (its first workgroup) stores the loop state,
// the stop flag and the report. Returns the stop flag.
__device__ inline int tail_close(const FinArgs &F, int s, const SimDev &S, SimIter &It, const double pre[6],
                                 const double4 *p4, const double2 *p2, bool writer)
{
    static_assert(kTailSimTiles <= kSegTiles, "a tail sim is a single residual segment");
    __shared__ int s_stop;
    const int b = S.tile_begin, n = S.tile_end - S.tile_begin;
    double red[6];
    fin_reduce_any(red, n, [&](int vt, double v[6]) {
        if (vt == (int)threadIdx.x) {  // the first round: already loaded
            for (int k = 0; k < 6; ++k) v[k] = pre[k];
            return;
        }
        for (int k = 0; k < 6; ++k) v[k] = 0.0;
        if (vt < n) {
            const double4 p = p4[b + vt];
            const double2 q = p2[b + vt];
            v[0] = p.x; v[1] = p.y; v[2] = p.z; v[3] = p.w; v[4] = q.x; v[5] = q.y;
        }
    });
    if (threadIdx.x == 0) {
        // The sum over the segments: with one segment, k_finalize's butterflies
        // and group sums combine it only with +0.0 (the other threads' and
        // groups' values), which leaves a sum s as s + 0.0 and a maximum m as
        // fmax(m, 0.0) (the partials are non-negative or NaN).
        red[0] += 0.0;
        red[1] += 0.0;
        red[5] += 0.0;
        red[2] = fmax(red[2], 0.0);
        red[3] = fmax(red[3], 0.0);
        red[4] = fmax(red[4], 0.0);
        FinState st;
        load_fin_state(st, It, S);
        close_iteration(It, st, red);
        if (writer && It.done) {  // no one reads the device loop state of a sim still iterating
            F.iters[s] = It;
            F.done_out[s] = 1;
            publish_report(F, s, It);
        }
        s_stop = It.done;
    }
    __syncthreads();
    const int stop = s_stop;
    __syncthreads();
    return stop;
}

// The workgroups of a sim meet. Every wave waits for its own stores, then
// thread 0 makes them visible device-wide with a release-only arrival on its
// group's word (an L2 write-back, no invalidation: workgroups still computing
// keep their cached data); in a sim of several groups the last of each group
// acquires and arrives on the sim's word. Every workgroup polls the word that
// counts the whole sim (its group's word when the group is the sim) until all
// have arrived, then acquires. Phases count the sim's barriers. Returns false
// when the wait gave up.
__device__ inline bool sim_meet(const TailArgs &L, const TailSeat &seat, uint32_t &phase)
{
    __shared__ int s_ok;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    ++phase;
    if (threadIdx.x == 0) {
        const uint32_t a = __hip_atomic_fetch_add(seat.group, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t *word = seat.group;
        uint32_t target = phase * seat.gsize;
        if (seat.ngroups > 1) {
            if (a + 1u == target) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                __hip_atomic_fetch_add(seat.sim, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
            word = seat.sim;
            target = phase * seat.ngroups;
        }
        int ok = 1;
        for (long spins = 0; __hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target; ++spins) {
            if (spins >= L.spin) {
                atomicOr(L.err, 1);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_ok = ok;
    }
    __syncthreads();
    const bool ok = s_ok;
    __syncthreads();
    return ok;
}

// Copy of `bytes` (a multiple of 4) from global memory into LDS, whole workgroup.
__device__ inline void copy_words(void *dst, const void *src, int bytes)
{
    for (int w = (int)threadIdx.x; w < bytes / 4; w += (int)blockDim.x)
        ((uint32_t *)dst)[w] = ((const uint32_t *)src)[w];
}

// Blocks 0 .. n_tiles-1: one tile each (through the launch's tile ranges); the
// last block publishes the reports of the sims outside the launch. A tail
// launch holds few workgroups, so the register budget is set for no spills
// (FP64 and 3D: 2 waves per SIMD, FP32 2D: 3) rather than for occupancy.
template <typename T, int DIM, bool WALLS, bool AV, int LPP>
__global__ void __launch_bounds__(kMaxBlock)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 || DIM == 3 ? 2 : 3)))
k_tail(PassArgs<T> A, FinArgs F, WallArgs<T> W, TailArgs L)
{
    static_assert(sizeof(SimDev) % 4 == 0 && sizeof(SimIter) % 4 == 0, "word copies");
    const int v = blockIdx.x;
    if (v >= A.n_tiles) {
        for (int s = threadIdx.x; s < F.n_sims; s += blockDim.x)
            if ((L.outside[s >> 5] >> (s & 31)) & 1u) {
                F.done_out[s] = 1;
                publish_report(F, s, F.iters[s]);
            }
        return;
    }
    __shared__ SimDev S;   // the sim's constants
    __shared__ SimIter It; // this workgroup's copy of the sim's loop state
    const int t = launch_tile(A, v);
    const int2 tl = A.tiles[t];
    const int s = tl.x;
    copy_words(&S, &A.sims[s], (int)sizeof(SimDev));
    copy_words(&It, &F.iters[s], (int)sizeof(SimIter));
    __syncthreads();
    const int nt = S.tile_end - S.tile_begin;
    const int bi = t - S.tile_begin;  // this workgroup's place among the sim's
    const int gi = bi / kTailGroup;
    TailSeat seat;
    seat.group = L.group + S.tile_begin / kTailGroup + s + gi;
    seat.sim = L.arrive + s;
    seat.gsize = (uint32_t)min(kTailGroup, nt - gi * kTailGroup);
    seat.ngroups = (uint32_t)((nt + kTailGroup - 1) / kTailGroup);
    const bool walls = WALLS && S.nw > 0;
    uint32_t phase = 0;
    double pre[6];
    for (int k = L.k0;; ++k) {
        const int q = k & 1;
        // the last partial batch of a list issued at once (2D: in 3D the masked
        // batch compiles to a different fusion of multiplies and adds, so its
        // sums would round differently from the plain launches')
        pass_tile_at<T, DIM, WALLS, AV, false, MODE_PSEUDO, LPP, false, 0, false, DIM == 2>(
            A, S, t, tl, (A.cur + k) & 1, k & 1, L.part4[q], L.part2[q]);
        if (!sim_meet(L, seat, phase)) return;
        prefetch_partials(pre, S, L.part4[q], L.part2[q]);
        const int stop = tail_close(F, s, S, It, pre, L.part4[q], L.part2[q], bi == 0);
        if (walls) {  // the sim's walls for iteration k + 1 (records of its fluid at k + 1)
            const int end = S.wall_begin + S.nw, stride = nt * (int)blockDim.x;
            for (int iw = S.wall_begin + bi * (int)blockDim.x + (int)threadIdx.x; iw < end; iw += stride)
                wall_particle<T, DIM>(W, S, iw, (W.cur + k + 1) & 1, 0, false);
            if (stop) return;
            if (!sim_meet(L, seat, phase)) return;
        } else if (stop) {
            return;
        }
    }
}

__global__ void k_tail_zero(uint32_t *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Workgroups of a kernel that fit on the device at once (cached per kernel and
// workgroup size).
int coresident(const void *fn, int block)
{
    static std::mutex mu;
    static std::map<std::pair<const void *, int>, int> cache;
    std::lock_guard<std::mutex> lock(mu);
    const auto key = std::make_pair(fn, block);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int dev = 0, cus = 0, per = 0;
    DTSPH_HIP_CHECK(hipGetDevice(&dev));
    DTSPH_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    DTSPH_HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, block, 0));
    const int n = per * cus;
    cache[key] = n;
    return n;
}

template <typename T, int DIM, bool WALLS, bool AV> const void *tail_kernel(int lpp)
{
    switch (lpp) {
    case 1: return (const void *)k_tail<T, DIM, WALLS, AV, 1>;
    case 2: return (const void *)k_tail<T, DIM, WALLS, AV, 2>;
    case 4: return (const void *)k_tail<T, DIM, WALLS, AV, 4>;
    default: return (const void *)k_tail<T, DIM, WALLS, AV, 8>;
    }
}

template <typename T> const void *tail_kernel(const Ctx &c)
{
    if (c.max_dim == 2) {
        if (c.any_walls) return c.any_av ? tail_kernel<T, 2, true, true>(c.lpp) : tail_kernel<T, 2, true, false>(c.lpp);
        return c.any_av ? tail_kernel<T, 2, false, true>(c.lpp) : tail_kernel<T, 2, false, false>(c.lpp);
    }
    if (c.any_walls) return c.any_av ? tail_kernel<T, 3, true, true>(c.lpp) : tail_kernel<T, 3, true, false>(c.lpp);
    return c.any_av ? tail_kernel<T, 3, false, true>(c.lpp) : tail_kernel<T, 3, false, false>(c.lpp);
}

}  // namespace

// Tail launches run the plain pseudo pass only: no moving or steady sims, one
// regulariser, no cached coefficients, no speculative gate, not a static
// context (whose callers may not allow a cooperative launch).
bool tail_kind(const Ctx &c)
{
    return c.tail_loop == 1 && !c.static_mode && !c.any_move && !c.any_steady && !c.sep_den && c.pair_cache == 0 &&
           c.n_sims <= kTailMaxSims && c.block <= kMaxBlock;
}

// Can the sims still iterating (stop flags from the last report, tile ranges
// from set_active_ranges) run the rest of their loop in one tail launch? Each
// must be small, and the launch's tile ranges must cover exactly them.
bool tail_fits(const Ctx &c)
{
    if (!tail_kind(c) || c.loop_cached || c.gated || c.replay) return false;
    int64_t tiles = 0;
    for (int s = 0; s < c.n_sims; ++s) {
        if (c.flags_host[F_COUNT + s]) continue;
        const int nt = c.sims_h[s].tile_end - c.sims_h[s].tile_begin;
        if (nt <= 0 || nt > kTailSimTiles) return false;
        tiles += nt;
    }
    // a small remainder of a batch (a single sim runs its loop with plain
    // launches: inside a launch a device-wide barrier costs about what a kernel
    // boundary does, so a persistent loop gains nothing there)
    if (tiles == 0 || 4 * tiles > c.n_tiles || tiles + 1 > tail_capacity(c)) return false;
    return tiles == c.n_act_tiles;  // not every tile of a context in which some sims stopped
}

int tail_capacity(const Ctx &c)
{
    const void *fn = c.precision == DTSPH_FP32 ? tail_kernel<float>(c) : tail_kernel<double>(c);
    return coresident(fn, c.block);
}

template <typename T> bool launch_tail(Ctx &c, int k0)
{
    if (!tail_fits(c)) return false;
    const void *fn = tail_kernel<T>(c);
    const int grid = c.n_act_tiles + 1;
    PassArgs<T> a = pass_args<T>(c, MODE_PSEUDO, false);
    FinArgs f = fin_args(c, true);
    WallArgs<T> w = wall_args<T>(c, MODE_PSEUDO, false);
    TailArgs L;
    L.k0 = k0;
    L.spin = c.tail_spin;
    L.arrive = c.tail_words;
    L.err = (int *)(c.tail_words + c.n_sims);
    L.group = c.tail_words + c.n_sims + 1;
    L.part4[0] = c.partials;
    L.part2[0] = c.partials2;
    L.part4[1] = c.tail_part4;
    L.part2[1] = c.tail_part2;
    for (int q = 0; q < kTailMaxSims / 32; ++q) L.outside[q] = 0u;
    for (int s = 0; s < c.n_sims; ++s)
        if (c.flags_host[F_COUNT + s]) L.outside[s >> 5] |= 1u << (s & 31);
    const int nw = c.n_sims + 1 + c.n_tiles / kTailGroup + c.n_sims + 1;  // arrivals, error, groups
    hipLaunchKernelGGL(k_tail_zero, dim3((nw + 255) / 256), dim3(256), 0, c.stream, c.tail_words, nw);
    DTSPH_HIP_CHECK(hipGetLastError());
    void *args[] = {&a, &f, &w, &L};
    DTSPH_HIP_CHECK(hipLaunchCooperativeKernel(fn, dim3(grid), dim3(c.block), args, 0, c.stream));
    c.tstats.tail_launches++;
    return true;
}

template bool launch_tail<float>(Ctx &, int);
template bool launch_tail<double>(Ctx &, int);

}  // namespace dtsph
