// Internal declarations of libdtsph (not part of the C-ABI).
//
// Layout on the device (one context, all sims):
//   * "slots" are the cell-ordered particle positions in memory. Keys put every
//     fluid particle of every sim before every wall particle, and within each
//     type sim by sim, cell by cell, caller index by caller index. Hence fluid
//     slots [0, Nf) hold sim s's fluid at [fluid_begin[s], fluid_begin[s]+nf[s])
//     (fixed for the context's life) and wall slots are [Nf, N).
//   * Structure-of-arrays, one array per component ([a*n + i]), float64 master
//     copies of positions and pressure; velocity-like arrays in the pass type T.
//   * The pair pass reads neighbours through two gathered records per slot: a
//     position record (32-bit fixed point for FP32, float64 for FP64) built with
//     the neighbour list, and a T4 {V, p} record ping-ponged between passes.
//   * Neighbour lists are column-major (ELL): entry k of slot i at nbr[k*N + i],
//     so lanes of a wavefront read consecutive words. Fluid neighbours come
//     first, then wall neighbours; cnt[i] = n_fluid_nbrs | n_wall_nbrs << 16.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <array>
#include <map>
#include <string>
#include <vector>

#include "dtsph.h"

namespace dtsph {

constexpr int kHist = 8;             // residual history ring (stall window <= 8)
constexpr int kMaxCellOccupancy = 4096;
constexpr int kMaxBlock = 256;
constexpr int kMaxRanges = 32;       // active tile ranges passed to the pair pass
constexpr int kSegTiles = 256;       // tiles per residual segment (one finalize workgroup)
constexpr int kMaxTileRows = 32;     // cell rows per strip of the staged neighbour kernel
constexpr int kTailMaxSims = 256;    // sims of a context that may use tail launches
constexpr int64_t kTailSpinDefault = 1LL << 22;  // polls of a tail barrier word before a wait gives up
constexpr int kTailSimTiles = 128;   // tiles of one sim in a tail launch (its barrier's workgroups)
constexpr int kTailGroup = 32;       // workgroups per first-level barrier word of a tail launch

enum PassMode { MODE_PRE = 0, MODE_PSEUDO = 1 };

// Device flag words
enum Flag { F_NBR_OVERFLOW = 0, F_NBR_NEEDED = 1, F_CELL_OVERFLOW = 2, F_OUTSIDE = 3, F_SKIN = 4, F_COUNT = 5 };

// Per-sim constants (device). Everything the kernels need, precomputed on the
// host in float64; FP32 kernels convert once per thread.
struct SimDev {
    int dim, nf, nw;
    int fluid_begin;     // first fluid slot
    int wall_begin;      // first wall (index among the walls: slot Nf + wall_begin)
    int key_base;        // first fluid key; wall keys add the total cell count
    int tile_begin, tile_end;  // fluid tiles of this sim (residual partials)
    int seg_begin, seg_count;  // residual segments (runs of up to kSegTiles tiles)
    int ncell[3];
    int cell_div;        // cells of side >= (kappa h + skin) / cell_div; blocks of +-cell_div cells
    int tile_w, tile_h;  // cells per strip of the staged neighbour kernel (2D)
    int periodic[3];
    int edac_reg_literal;
    double lo[3], hi[3], L[3], halfL[3], cs[3], inv_cs[3];
    double kh2;          // (kappa h)^2, exact neighbour predicate
    double skin, cand_r2; // candidate lists reach kappa h + skin (squared radius)
    double h, inv_h, rho0, mass, c, nu, nu_e;
    double g[3];
    double dt, dtau, gamma, inv2dt, tol, vref;
    int max_iter, stall_window, conv_norm;
    int abs32;           // ablation: pair passes see float32-rounded absolute coordinates
    double stall_rel;
    // pass coefficients: dW/dr = kg * poly(q); see the pass kernel
    double sigma, kg;
    double k_div, k_lap, k_grad, k_visc, k_av;
    double den_v, den_e, den_a;   // eta h^2, EDAC regulariser, eps_av h^2
    double tiny_r2;
    // 32-bit fixed-point frame of the FP32 pass: x_q = (x - lo) * q_inv mod 2^32
    double q_inv[3], q_len[3];
    double res_p, res_v;          // residual scales incl. 1/nf
    // particle shifting (section 3.5): on/off, coefficient 1 + shift_r (W/W(h))^shift_n
    int shift, shift_n;
    double shift_r, vol;          // vol = m / rho0
    // steady-state solve (sections 2.3, 3.3): no real-time term (gamma = 1,
    // inv2dt = 0), no EDAC term (k_lap = 0), convective sum with k_conv
    int steady;
    // moving particles in pseudo-time (Algorithm 1): 0 frozen, 1 moving, 2
    // moving with neighbour updates; k_padv: pressure advection coefficient
    int move;
    double k_conv, k_padv;
};

// Per-sim pseudo-time loop state (device).
struct SimIter {
    int iters, done, reason, fixed;
    double hp[kHist], hv[kHist];
    double rp_mean, rv_mean, rp_max, rv_max;
    double disp;   // max |r^{n+1} - r^(0)| = dt/2 max |V^{k} - V^(0)| at the last iteration
    long long pairs;  // fluid-row neighbour pairs of the last iteration
};

// Per-sim report as published to mapped host memory.
struct MirrorRep {
    int iters, reason;
    double rp_mean, rv_mean, rp_max, rv_max, disp;
};

// Context (host object owning device memory).
struct Ctx {
    int precision = DTSPH_FP32;
    int n_sims = 0;
    int N = 0, Nf = 0, Nw = 0;
    int C = 0;               // fluid cells of all sims; keys 0..2C-1
    int C_max = 0;           // C at the finest subdivision (sizes the key tables)
    int cell_div = 2;
    int cap = 0;             // neighbour-list capacity per particle
    int block = 256;
    int lpp = 1;             // lanes per particle in the pair pass
    int g_nbr = 0, g_filter = 0;  // lanes per particle in the neighbour kernels (0: heuristic)
    // staged-tile neighbour kernel (2D contexts): 1 use it where it applies;
    // strip table {sim, cell type, first row, first column} for the current
    // subdivision, its capacity (the most strips of any subdivision), and the
    // particles one strip may stage in LDS
    int nbr_tiles = 0;
    int4 *strips = nullptr;
    int n_strips = 0, strip_cap = 0, tile_pmax = 0, tile_offmax = 0;
    int chunk = 0;           // 0 = adaptive
    int xcd_remap = 1;
    int max_dim = 2;
    bool any_walls = false, any_av = false, sep_den = false, any_shift = false;
    bool any_steady = false, all_steady = true;  // steady-state sims (fixed particles)
    bool any_move = false, any_move2 = false;   // sims moving in pseudo-time (any / with list updates)
    void *prec2 = nullptr;   // second position-record buffer (moving sims ping-pong)
    double *xm = nullptr;    // r^{k+1/2} of the fluid in the loop, float64 [3][Nf]
    void *vt = nullptr;      // Vtilde^k of the fluid [3][Nf] (pass type)
    // cached pair coefficients (DTSPH_OPT_PAIR_CACHE): 0 off, 1 on, 2 automatic;
    // cache_phase of the next pseudo-iteration launch: 0 none, 1 write, 2 read
    int pair_cache = 0, cache_phase = 0;
    bool loop_cached = false;
    bool coef_valid = false;  // coef holds the coefficients of the current lists
    void *coef = nullptr, *coef_av = nullptr;
    hipStream_t stream = nullptr;
    int device = 0;

    std::vector<dtsph_sim_desc> desc;
    std::vector<int64_t> nf, nw;
    std::vector<SimDev> sims_h;
    std::vector<double> skin_default;  // per sim: candidate skin chosen at creation
    std::vector<int> fluid_begin, wall_begin_caller, caller_begin;

    // phase
    bool in_loop = false;
    bool cells_valid = false;  // exact lists match the current positions
    bool cand_ok = false;      // candidate lists cover the current positions
    bool cand_next = false;    // ... will cover r^{n+1} (decided by the loop)
    int cur = 0;             // vp buffer read by the rate pass and the first
                             // iteration; sim s then alternates by its own
                             // iteration count (buffer (cur + iters_s) & 1)
    bool p_half = false;     // pm holds p^{K+1/2} (the half step back to p^K
                             // is applied by the corrector / state readout)
    bool records_fresh = false;  // vp[cur] and the position records hold the
                                 // state at the current positions (corrector)
    int last_iters = 4;      // adaptive chunking
    std::vector<int> prev_iters;  // per sim: iterations of its last loop (-1: none yet)
    // loop schedule (DTSPH_OPT_TAIL_LOOP): 0 plain chunks, 1 cut first chunk
    // and tail launches, 2 cut first chunk and plain chunks; per sim arrival
    // words of the sims' barriers, an error word, then the words of the
    // workgroup groups (tiles / kTailGroup + n_sims + 1); the tail launches'
    // second buffer of residual partials (odd iterations)
    int tail_loop = 1;
    int64_t tail_spin = kTailSpinDefault;  // polls of a tail barrier before a wait gives up
    uint32_t *tail_words = nullptr;
    double4 *tail_part4 = nullptr;
    double2 *tail_part2 = nullptr;
    // pair-pass launches inside a loop cover only sims still iterating: tile
    // ranges (first tile, index within the launch); n_ranges == 0: every tile
    int n_ranges = 0, n_act_tiles = 0;
    int2 ranges[kMaxRanges];

    // device memory: every device array of the context is registered with the
    // address of the field that points to it, so that the whole set can move into
    // (or out of) a caller-supplied workspace.
    struct DevArray {
        void **slot;
        size_t bytes;
    };
    std::vector<DevArray> arrays;
    std::vector<void *> owned;            // library allocations (empty while a workspace is set)
    char *workspace = nullptr;            // caller-owned, or nullptr
    size_t workspace_size = 0;
    // context of dtsph_create_static: every device array is carved from the
    // library's static device scratch (bump offset below), the report mirror is
    // device memory copied to a static host buffer after each stream sync
    bool static_mode = false;
    char *bump = nullptr;
    size_t bump_off = 0, bump_cap = 0;
    char *mirror_dev = nullptr;           // static mode: device copy of the mirror
    size_t mirror_bytes = 0;
    int64_t device_bytes = 0;
    SimDev *sims = nullptr;
    SimIter *iters = nullptr;             // per sim, then the speculative gate (k_gate)
    int *orig[2] = {nullptr, nullptr};
    int *simid[2] = {nullptr, nullptr};
    double *x[2] = {nullptr, nullptr};    // active positions (3 x N SoA)
    double *xn[2] = {nullptr, nullptr};   // r^n during the loop (3 x N)
    void *xr = nullptr;                   // packed float64 positions for the neighbour
                                          // kernels (double2 in 2D, double4 in 3D)
    void *vn[2] = {nullptr, nullptr};     // V^n (3 x Nf, type T)
    void *dv[2] = {nullptr, nullptr};     // V^n - V^{n-1}
    void *w[2] = {nullptr, nullptr};      // V^k - V^n
    void *w0[2] = {nullptr, nullptr};     // V^(0) - V^n (predictor), for the skin test
    double *pm[2] = {nullptr, nullptr};   // p^n, or p^{k+1/2} inside the loop
    double *pn[2] = {nullptr, nullptr};   // p^n kept during the loop
    void *dp[2] = {nullptr, nullptr};     // (dp/dtau)^k (type T)
    void *vw[2] = {nullptr, nullptr};     // prescribed wall velocity (3 x Nw)
    void *pw[2] = {nullptr, nullptr};     // last wall pressure (Nw)
    int buf = 0;                          // which gathered buffer set is live
    int xb = 0;                           // live buffer of x (also swapped by the predictor)
    void *vp[2] = {nullptr, nullptr};     // T4 {V, p} records (N)
    void *prec = nullptr;                 // position records (N): uint4 or double4
    uint32_t *key = nullptr, *rank = nullptr, *perm = nullptr;
    uint32_t *count = nullptr, *cell_start = nullptr, *scan_tmp = nullptr;
    int *nbr = nullptr;
    uint32_t *cnt = nullptr;
    int *cand = nullptr;                  // candidate lists (radius kappa h + skin)
    uint32_t *ccnt = nullptr;
    int capc = 0;
    int2 *tiles = nullptr;
    int n_tiles = 0;
    int4 *segs = nullptr;                 // per segment: sim, first tile, end tile, index in sim
    int n_segs = 0;
    double4 *seg_p = nullptr;             // per segment: partial sums of the residual terms
    double2 *seg_p2 = nullptr;
    uint32_t *tickets = nullptr;          // per sim: segments of the running finalize done
    // speculative end of step (dtsph_step): the corrector and the next rate pass
    // are queued behind a device gate before the host reads the loop's reports
    bool gated = false;                   // the next launches are speculative
    bool speculate = false, spec_ready = false;  // DTSPH_OPT_SPECULATE (off by default)
    int spec_score = 4, spec_idle = 0;    // recent success of speculation (adaptive)
    // after shifting: skip the read-back of the largest shift while shifts keep
    // leaving the candidate skin (checked later, at the next wait)
    int shift_miss = 0;
    bool shift_nosync = false, shift_pending = false, shift_pending_cand = false;
    std::vector<double> shift_disp;
    double4 *partials = nullptr;
    double2 *partials2 = nullptr;         // per tile: max |V^{k+1} - V^(0)|^2, pairs
    int *flags = nullptr;
    int *done_dev = nullptr;
    int *init_slot = nullptr;             // caller index -> slot before any sort

    // mapped host memory written by k_publish (host and device views)
    void *mirror_h = nullptr;
    int *flags_host = nullptr;             // F_COUNT flags then n_sims stop flags
    MirrorRep *reps_host = nullptr;
    unsigned long long *pairs_host = nullptr;
    int *m_flags_d = nullptr;
    MirrorRep *m_reps_d = nullptr;
    unsigned long long *m_pairs_d = nullptr;
    int *seq_host = nullptr;              // per sim: sequence number of the last finalize
    int *m_seq_d = nullptr;
    int seq = 0;                          // last finalize launched

    // timing
    bool timing = false;
    int timing_every = 1;                 // time every n-th launch of each kind
    bool timing_first = false;            // time the first pair and wall pass of each loop (and every build)
    long long timer_count[4] = {0, 0, 0, 0};  // pair pass, wall pass, full build, list filter
    int pass_index = 0;                   // launch index of the next pair pass in the loop
    hipEvent_t ext_start = nullptr, ext_stop = nullptr;  // events of a timed pass launch
    std::vector<std::pair<int, double>> pass_times;  // this loop's timed pair passes (index, ms)
    dtsph_timing tstats{};
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::array<int, 3>> ev_pending;  // (start event, kind, pass index)
    size_t ev_used = 0;

    // HIP graphs of the step segment from the rate pass to the first chunk of
    // pseudo-iterations, keyed by everything that changes its launches
    bool graphs = false;
    bool replay = false;       // host logic of a cached segment: launch nothing
    bool in_segment = false;   // inside a captured or replayed segment
    hipStream_t cap_stream = nullptr;
    std::map<uint64_t, hipGraphExec_t> graph_cache;
    uint32_t *pubcount = nullptr;  // per sim: reports published so far (device)

    // particle shifting: per fluid particle shift and corrections, per-block
    // maximum |shift|^2, and the last maximum read back by the host
    double *sh_dr = nullptr, *sh_dp = nullptr;
    void *sh_dv = nullptr;
    double *sh_part = nullptr;
    double *sh_max_h = nullptr, *sh_max_d = nullptr;  // mapped host memory
    std::vector<double> last_disp;    // per sim: max |r^{n+1} - r^(0)| of the last loop

    std::string err;
};

// Every kernel launch of the library goes through this gate: while the host
// logic of a cached graph segment runs (replay), it launches nothing.
#define DTSPH_LAUNCH(ctx, ...)                                                             \
    do {                                                                                   \
        if (!(ctx).replay) hipLaunchKernelGGL(__VA_ARGS__);                                \
    } while (0)

// ---- launchers (defined in the .hip files) ---------------------------------
// build_cells(c, loop_fixed): with loop_fixed >= 0 the gather also performs the
// set-up of a pseudo-time loop (what launch_loop_begin does) for fixed = loop_fixed
template <typename T> void build_cells(Ctx &c, int loop_fixed = -1);  // dtsph_cells.hip
template <typename T> void filter_lists(Ctx &c);
template <typename T> void launch_nbr_lists(Ctx &c, bool filter);
template <typename T> void launch_pre_records(Ctx &c);
template <typename T> void launch_wall(Ctx &c, int mode, bool cand_lists = false);
template <typename T> void launch_pass(Ctx &c, int mode, bool cand_lists = false);
void launch_finalize(Ctx &c, bool publish);
// iteration next-1's residual reduction together with iteration next's wall pass
template <typename T> void launch_finalize_wall(Ctx &c, bool publish, int next);
// wall pressures of the last iteration each sim ran (after a loop of fused wall passes)
template <typename T> void launch_wall_pressure(Ctx &c);
void launch_gate(Ctx &c);  // the speculative gate, before gated launches
// The rest of a pseudo-time loop in one persistent launch when the sims still
// iterating are few and small (dtsph_tail.hip); false: not launched (the caller
// goes on with plain chunks). k0 = iterations every such sim has run.
bool tail_kind(const Ctx &c);  // the context's kind allows tail launches at all
bool tail_fits(const Ctx &c);  // ... and the sims still iterating fit one now
int tail_capacity(const Ctx &c);  // workgroups of a tail launch that fit on the device at once
template <typename T> bool launch_tail(Ctx &c, int k0);
void launch_publish(Ctx &c);
template <typename T> void launch_loop_begin(Ctx &c, int fixed_iters);
template <typename T> void launch_move_begin(Ctx &c);
template <typename T> void launch_correct(Ctx &c);
template <typename T> void launch_shift(Ctx &c, bool cand_lists);  // sums, apply, max
template <typename T> void launch_set_state(Ctx &c, const dtsph_state_view &s, bool in_loop);
template <typename T> void launch_get_state(Ctx &c, const dtsph_state_view &s, bool in_loop);

// timing helpers (dtsph_api.hip); timer_slot reserves the two events of a
// launch timed by the runtime itself (hipExtLaunchKernel), timer_book queues them
int timer_begin(Ctx &c, int kind);
int timer_slot(Ctx &c, int kind);
void timer_book(Ctx &c, int slot, int kind);
void timer_end(Ctx &c, int slot, int kind);

#define DTSPH_HIP_CHECK(expr)                                                              \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) throw HipError(e_, #expr, __FILE__, __LINE__);               \
    } while (0)

struct HipError {
    hipError_t code;
    std::string what;
    HipError(hipError_t c, const char *expr, const char *file, int line)
        : code(c), what(std::string(hipGetErrorString(c)) + " in " + expr + " at " + file + ":" +
                        std::to_string(line)) {}
};

struct ApiError {
    int status;
    std::string what;
    ApiError(int s, std::string w) : status(s), what(std::move(w)) {}
};

inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Position record of slot i read by the pair passes: FP32 path 32-bit fixed
// point per axis, x_q = floor((x - lo) * q_inv) mod 2^32 (exact wrap on periodic
// axes, whose q_len divides the period); FP64 path the float64 coordinates. Two
// components in 2D (uint2 / double2), four in 3D (uint4 / double4).
template <typename T>
__device__ inline void write_pos_record(const SimDev &S, void *prec, int i, const double xi[3]);

template <>
__device__ inline void write_pos_record<float>(const SimDev &S, void *prec, int i, const double xi[3])
{
    uint32_t q[4] = {0u, 0u, 0u, 0u};
    for (int a = 0; a < S.dim; ++a) {
        // ablation (DTSPH_OPT_ABS32_POSITIONS): the coordinate rounded to float32 first;
        // the fixed-point difference of two such values is the float32 difference
        // (exact for neighbours, Sterbenz) rounded once, as in a float32 pipeline
        const double xa = S.abs32 ? (double)(float)xi[a] : xi[a];
        double v = floor((xa - S.lo[a]) * S.q_inv[a]);
        q[a] = (uint32_t)(unsigned long long)(long long)v;
    }
    if (S.dim == 2) ((uint2 *)prec)[i] = make_uint2(q[0], q[1]);
    else ((uint4 *)prec)[i] = make_uint4(q[0], q[1], q[2], 0u);
}

template <>
__device__ inline void write_pos_record<double>(const SimDev &S, void *prec, int i, const double xi[3])
{
    if (S.dim == 2) ((double2 *)prec)[i] = make_double2(xi[0], xi[1]);
    else ((double4 *)prec)[i] = make_double4(xi[0], xi[1], xi[2], 0.0);
}

}  // namespace dtsph
