// C-ABI of libdtsph: context set-up, argument checking, and the host side of
// Algorithm 2 (predict -> pseudo-time loop -> correct). All arithmetic on
// particle data happens in the kernels of dtsph_cells.hip and dtsph_pass.hip;
// the host only orders launches and reads back per-sim stop flags.
#include <algorithm>
#include <cmath>
#include <array>
#include <map>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <atomic>

#include "dtsph_internal.h"

using namespace dtsph;

struct dtsph_ctx {
    Ctx c;
};

// Device scratch of dtsph_create_static: the whole context of one static
// context per GPU lives here. In host code this name is only a stand-in for the
// device symbol; its device address comes from hipGetSymbolAddress (per device).
static __device__ __align__(256) char scratch[DTSPH_STATIC_SCRATCH_BYTES];

namespace {

std::string g_create_error = "no error";

// autotuner choices of this process: key -> (pass lanes, pass block, neighbour-kernel
// lanes, filter lanes, cell subdivision)
std::mutex g_tune_mu;
std::map<std::string, std::array<int, 6>> g_tune_cache;

std::string tune_key(const Ctx &c)
{
    int bucket = 0;
    while ((1ll << (bucket + 1)) <= (long long)c.Nf) ++bucket;
    return std::to_string(c.max_dim) + "/" + std::to_string(c.precision) + "/" + std::to_string(c.any_walls) +
           "/" + std::to_string(c.any_av) + "/" + std::to_string(c.sep_den) + "/" + std::to_string(bucket);
}

template <typename F> int guarded(dtsph_ctx *ctx, F &&f)
{
    if (!ctx) return DTSPH_EINVAL;
    try {
        DTSPH_HIP_CHECK(hipSetDevice(ctx->c.device));
        return f(ctx->c);
    } catch (const ApiError &e) {
        ctx->c.err = e.what;
        return e.status;
    } catch (const HipError &e) {
        ctx->c.err = e.what;
        return DTSPH_EHIP;
    } catch (const std::exception &e) {
        ctx->c.err = e.what();
        return DTSPH_EHIP;
    } catch (...) {
        ctx->c.err = "unknown error";
        return DTSPH_EHIP;
    }
}

constexpr size_t kWsAlign = 256;

size_t ws_round(size_t b) { return (std::max<size_t>(b, 16) + kWsAlign - 1) / kWsAlign * kWsAlign; }

void *raw_alloc(size_t bytes)
{
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, std::max<size_t>(bytes, 16));
    if (e != hipSuccess) throw ApiError(DTSPH_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " +
                                                          hipGetErrorString(e));
    return p;
}

// Allocate a device array owned by the library and register the field that
// holds it (see Ctx::arrays). A static context carves it from the static
// scratch instead (no allocation).
template <typename P> void dev_alloc(Ctx &c, P *&slot, size_t bytes)
{
    void *p;
    if (c.static_mode) {
        const size_t b = ws_round(bytes);
        if (c.bump_off + b > c.bump_cap)
            throw ApiError(DTSPH_ENOMEM, "the static scratch of " + std::to_string(c.bump_cap) +
                                             " bytes cannot hold this context (needs more than " +
                                             std::to_string(c.bump_off + b) + ")");
        p = c.bump + c.bump_off;
        c.bump_off += b;
    } else {
        p = raw_alloc(bytes);
        c.owned.push_back(p);
    }
    c.arrays.push_back({(void **)&slot, bytes});
    c.device_bytes += (int64_t)bytes;
    slot = (P *)p;
}

size_t workspace_need(const Ctx &c)
{
    size_t total = 0;
    for (const auto &a : c.arrays) total += ws_round(a.bytes);
    return total;
}

// Move every device array to `base` (a caller workspace of workspace_need(c)
// bytes) or, with base == nullptr, to fresh library allocations; contents are
// copied on the context's stream, old library allocations freed.
void clear_graphs(Ctx &c)
{
    for (auto &kv : c.graph_cache) (void)hipGraphExecDestroy(kv.second);
    c.graph_cache.clear();
}

void relocate(Ctx &c, char *base, size_t size)
{
    clear_graphs(c);  // they hold the old addresses
    std::vector<void *> fresh(c.arrays.size(), nullptr);
    std::vector<void *> fresh_owned;
    try {
        size_t off = 0;
        for (size_t i = 0; i < c.arrays.size(); ++i) {
            if (base) {
                fresh[i] = base + off;
                off += ws_round(c.arrays[i].bytes);
            } else {
                fresh[i] = raw_alloc(c.arrays[i].bytes);
                fresh_owned.push_back(fresh[i]);
            }
        }
        DTSPH_HIP_CHECK(hipStreamSynchronize(c.stream));
        for (size_t i = 0; i < c.arrays.size(); ++i)
            DTSPH_HIP_CHECK(hipMemcpyAsync(fresh[i], *c.arrays[i].slot, c.arrays[i].bytes, hipMemcpyDeviceToDevice,
                                           c.stream));
        DTSPH_HIP_CHECK(hipStreamSynchronize(c.stream));
    } catch (...) {
        for (void *p : fresh_owned) (void)hipFree(p);
        throw;
    }
    for (void *p : c.owned) (void)hipFree(p);
    c.owned = std::move(fresh_owned);
    for (size_t i = 0; i < c.arrays.size(); ++i) *c.arrays[i].slot = fresh[i];
    c.done_dev = c.flags + F_COUNT;
    c.workspace = base;
    c.workspace_size = base ? size : 0;
}

// Per-device state of the static scratch: its device address (looked up once
// per device) and whether a static context holds it; the host copy of a static
// context's report mirror.
constexpr int kMaxDevices = 64;
constexpr size_t kStaticMirrorBytes = 16384;
std::mutex g_static_mu;
void *g_scratch_ptr[kMaxDevices] = {};
bool g_scratch_busy[kMaxDevices] = {};
alignas(64) char g_static_mirror[kMaxDevices][kStaticMirrorBytes];

void *static_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) throw ApiError(DTSPH_EINVAL, "device index out of range");
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) throw HipError(e, "hipGetSymbolAddress(scratch)", __FILE__, __LINE__);
        g_scratch_ptr[device] = ptr;
    }
    return g_scratch_ptr[device];
}

// Static contexts: bring the device copy of the mirror to the host (after the
// stream has been synchronised), and the cleared build flags back.
void mirror_pull(Ctx &c)
{
    if (c.static_mode)
        DTSPH_HIP_CHECK(hipMemcpy(c.mirror_h, c.mirror_dev, c.mirror_bytes, hipMemcpyDeviceToHost));
}

void mirror_push_flags(Ctx &c)
{
    if (c.static_mode)
        DTSPH_HIP_CHECK(hipMemcpy(c.m_flags_d, c.flags_host, sizeof(int) * F_COUNT, hipMemcpyHostToDevice));
}

void free_all(Ctx &c)
{
    if (c.static_mode) {  // nothing was allocated: give the scratch back
        std::lock_guard<std::mutex> lk(g_static_mu);
        g_scratch_busy[c.device] = false;
        c.static_mode = false;
        c.mirror_h = nullptr;
    }
    clear_graphs(c);
    if (c.cap_stream) (void)hipStreamDestroy(c.cap_stream);
    c.cap_stream = nullptr;
    for (void *p : c.owned) (void)hipFree(p);
    c.owned.clear();
    c.arrays.clear();
    if (c.mirror_h) (void)hipHostFree(c.mirror_h);
    c.mirror_h = nullptr;
    c.flags_host = nullptr;
    for (hipEvent_t e : c.ev_pool) (void)hipEventDestroy(e);
    c.ev_pool.clear();
}

void check_desc(const dtsph_sim_desc &d, int s, int64_t nf, int64_t nw)
{
    auto bad = [s](const std::string &m) { throw ApiError(DTSPH_EINVAL, "sim " + std::to_string(s) + ": " + m); };
    if (d.dim != 2 && d.dim != 3) bad("dim must be 2 or 3");
    if (nf < 1) bad("n_fluid must be >= 1");
    if (nw < 0) bad("n_wall must be >= 0");
    if (!(d.h > 0) || !(d.kappa > 0)) bad("h and kappa must be > 0");
    if (!(d.rho0 > 0) || !(d.mass > 0)) bad("rho0 and mass must be > 0");
    if (!(d.vref > 0) || !(d.beta > 0)) bad("vref and beta must be > 0");
    if (!(d.dt > 0)) bad("dt must be > 0");
    if (d.dtau < 0 || !std::isfinite(d.dtau)) bad("dtau must be >= 0 (0 selects dt/beta)");
    if (d.nu < 0 || d.alpha < 0 || d.eta < 0 || d.eps_av < 0) bad("nu, alpha, eta, eps_av must be >= 0");
    if (!(d.tol >= 0)) bad("tol must be >= 0");
    if (d.max_iter < 1) bad("max_iter must be >= 1");
    if (d.stall_window < 0 || d.stall_window > kHist) bad("stall_window must be in [0, 8]");
    if (d.conv_norm != 0 && d.conv_norm != 1) bad("conv_norm must be 0 or 1");
    if (d.max_neighbors < 0 || d.max_neighbors > 8000) bad("max_neighbors must be in [0, 8000]");
    if (d.shift != 0 && d.shift != 1) bad("shift must be 0 or 1");
    if (d.shift && (d.shift_n < 1 || d.shift_n > 8)) bad("shift_n must be in [1, 8]");
    if (d.shift && !(d.shift_r >= 0 && std::isfinite(d.shift_r))) bad("shift_r must be finite and >= 0");
    if (d.steady != 0 && d.steady != 1) bad("steady must be 0 or 1");
    if (d.steady && d.shift) bad("a steady solve keeps its particles fixed: shift must be 0");
    if (d.move < 0 || d.move > 2) bad("move must be 0, 1 or 2");
    if (d.move && d.steady) bad("a steady solve keeps its particles fixed: move must be 0");
    for (int a = 0; a < d.dim; ++a) {
        if (!(d.hi[a] > d.lo[a])) bad("hi must exceed lo on every axis");
        if (d.periodic[a] && !(d.kappa * d.h < 0.5 * (d.hi[a] - d.lo[a])))
            bad("kappa*h must be below half the period on periodic axes");
    }
}

// Cell grid: cells no smaller than (kappa h + skin) / m (small margin against
// rounding), so every candidate of a particle lies within m cells of its own.
void set_grid(SimDev &S, int m)
{
    const double kc = std::sqrt(S.cand_r2);
    S.cell_div = m;
    for (int a = 0; a < 3; ++a) {
        if (a < S.dim) {
            const int n = (int)std::floor(S.L[a] / (kc / m * (1.0 + 1e-6)));
            S.ncell[a] = std::max(1, n);
            S.cs[a] = S.L[a] / S.ncell[a];
            S.inv_cs[a] = 1.0 / S.cs[a];
        } else {
            S.ncell[a] = 1;
            S.cs[a] = S.inv_cs[a] = 1.0;
        }
    }
    // strips of the staged neighbour kernel (2D): about 256 particles at the
    // lattice density, three times wider than tall (a strip row is one run of
    // consecutive keys)
    S.tile_w = S.tile_h = 0;
    if (S.dim == 2) {
        const double ppc = S.cs[0] * S.cs[1] / (S.mass / S.rho0);  // particles per cell
        const double target = std::max(16.0, 256.0 / ppc);          // cells per strip
        int th = (int)std::lround(std::sqrt(target / 3.0));
        th = std::max(1, std::min(std::min(th, S.ncell[1]), kMaxTileRows));
        int tw = (int)std::ceil(target / th);
        tw = std::max(1, std::min(tw, S.ncell[0]));
        S.tile_w = tw;
        S.tile_h = th;
    }
}

// Strips of the staged neighbour kernel at the sims' current grids: per sim its
// fluid-cell strips and, with walls, its wall-cell strips (0 unless every sim is 2D).
int64_t count_strips(const std::vector<SimDev> &sims)
{
    int64_t n = 0;
    for (const SimDev &S : sims) {
        if (S.dim != 2) return 0;
        n += (int64_t)ceil_div(S.ncell[0], S.tile_w) * ceil_div(S.ncell[1], S.tile_h) * (S.nw > 0 ? 2 : 1);
    }
    return n;
}

// The strip table and LDS sizes for the current subdivision. The staged kernel
// applies when every sim is 2D and every periodic axis has at least 2m+3 cells
// (one image shift per staged column, as in k_nbr's trimmed path); otherwise
// n_strips stays 0 and builds use the per-particle kernel.
void setup_strips(Ctx &c)
{
    c.n_strips = 0;
    if (!c.strips) return;
    std::vector<int4> v;
    int pmax = 0, offmax = 0;
    for (int s = 0; s < c.n_sims; ++s) {
        const SimDev &S = c.sims_h[s];
        const int m = S.cell_div, m3 = 2 * m + 3;
        if (S.dim != 2 || (S.periodic[0] && S.ncell[0] < m3) || (S.periodic[1] && S.ncell[1] < m3)) return;
        const int ntp = S.nw > 0 ? 2 : 1;
        for (int tp = 0; tp < ntp; ++tp)
            for (int y0 = 0; y0 < S.ncell[1]; y0 += S.tile_h)
                for (int x0 = 0; x0 < S.ncell[0]; x0 += S.tile_w) v.push_back(make_int4(s, tp, y0, x0));
        const int vx = S.tile_w + 2 * m, vy = S.tile_h + 2 * m;
        offmax = std::max(offmax, ntp * vx * vy + 1);
        // staged particles at the lattice density (fluid cells; wall cells hold
        // a few layers), with room for 2.5 times that
        const double ppc = S.cs[0] * S.cs[1] / (S.mass / S.rho0);
        pmax = std::max(pmax, (int)std::ceil(2.5 * vx * vy * ppc) + 64);
    }
    // LDS per workgroup: pmax positions (16 B) and slots (4 B), offmax cell offsets
    const int room = (65536 - 1024 - 4 * offmax) / 20;
    if ((int64_t)v.size() > c.strip_cap || room < 64) return;
    c.tile_pmax = std::min(pmax, room);
    c.tile_offmax = offmax;
    DTSPH_HIP_CHECK(hipMemcpy(c.strips, v.data(), sizeof(int4) * v.size(), hipMemcpyHostToDevice));
    c.n_strips = (int)v.size();
}

// Key bases for the current subdivision: sim s's fluid cells are keys
// [key_base, key_base + cells); wall cells add the total C.
void setup_keys(Ctx &c, int m)
{
    int64_t C = 0;
    for (int s = 0; s < c.n_sims; ++s) {
        set_grid(c.sims_h[s], m);
        c.sims_h[s].key_base = (int)C;
        C += (int64_t)c.sims_h[s].ncell[0] * c.sims_h[s].ncell[1] * c.sims_h[s].ncell[2];
    }
    if (C > c.C_max) throw ApiError(DTSPH_EINVAL, "cell grid exceeds the key tables sized at creation");
    c.C = (int)C;
    c.cell_div = m;
    setup_strips(c);
}

SimDev make_simdev(const dtsph_sim_desc &d, int64_t nf, int64_t nw)
{
    SimDev S;
    std::memset(&S, 0, sizeof(S));
    S.dim = d.dim;
    S.nf = (int)nf;
    S.nw = (int)nw;
    S.edac_reg_literal = d.edac_reg_literal;
    const double kh = d.kappa * d.h;
    // candidate lists reach kappa h + skin: skin = 0.3 h (0.25 h with particle
    // shifting, whose moves of a few hundredths of h add to the loop's), reduced
    // so that the candidate radius stays below half of every period. A context
    // rebuilds its lists whenever any sim moved beyond 0.4 skin, so a batch needs
    // the margin of its most mobile member: on the 64-sim batch 0.1 h rebuilt
    // 1.51 times per step, 0.3 h 1.02 times (2.70 -> 2.46 ms per step), for about
    // 12% longer candidate lists (a single 160k vortex: 0.142 -> 0.146 ms)
    double skin = (d.shift ? 0.25 : 0.3) * d.h;
    for (int a = 0; a < d.dim; ++a)
        if (d.periodic[a]) skin = std::min(skin, 0.5 * (0.5 * (d.hi[a] - d.lo[a]) - kh));
    S.skin = std::max(0.0, skin);
    const double kc = kh + S.skin;
    S.cand_r2 = kc * kc;
    for (int a = 0; a < 3; ++a) {
        if (a < d.dim) {
            S.lo[a] = d.lo[a];
            S.hi[a] = d.hi[a];
            S.L[a] = d.hi[a] - d.lo[a];
            S.halfL[a] = 0.5 * S.L[a];
            S.periodic[a] = d.periodic[a] ? 1 : 0;
            // fixed-point frame: a length q_len maps onto 2^32 units; on periodic
            // axes q_len divides the period so wrap-around is exact
            if (S.periodic[a]) {
                double m = std::max(1.0, std::floor(S.L[a] / (4.0 * kh)));
                S.q_len[a] = S.L[a] / m;
            } else {
                S.q_len[a] = 4.0 * kh;
            }
            S.q_inv[a] = 4294967296.0 / S.q_len[a];
        } else {
            S.ncell[a] = 1;
            S.cs[a] = S.inv_cs[a] = 1.0;
            S.L[a] = S.halfL[a] = 1.0;
            S.q_len[a] = 1.0;
            S.q_inv[a] = 0.0;
        }
    }
    S.kh2 = kh * kh;
    S.h = d.h;
    S.inv_h = 1.0 / d.h;
    S.rho0 = d.rho0;
    S.mass = d.mass;
    // section 3.4: c = beta V_ref, dtau = dt / beta; eq. nu_edac: nu_e = h c / 16
    S.c = d.beta * d.vref;
    S.nu = d.nu;
    S.nu_e = d.nu_e > 0 ? d.nu_e : d.h * S.c / 16.0;
    for (int a = 0; a < 3; ++a) S.g[a] = a < d.dim ? d.g[a] : 0.0;
    S.dt = d.dt;
    S.dtau = d.dtau > 0 ? d.dtau : d.dt / d.beta;
    // frozen eq. dv_dtau_exact: factor 2 dt / (2 dt + 3 dtau)
    S.gamma = 2.0 * S.dt / (2.0 * S.dt + 3.0 * S.dtau);
    S.inv2dt = 1.0 / (2.0 * S.dt);
    S.tol = d.tol;
    S.vref = d.vref;
    S.max_iter = d.max_iter;
    S.stall_window = d.stall_window;
    S.stall_rel = d.stall_rel;
    S.conv_norm = d.conv_norm;
    // quintic spline normalisation; dW/dr = (sigma/h) w'(q) = kg * poly(q)
    const double pi = 3.14159265358979323846;
    S.sigma = d.dim == 2 ? 7.0 / (478.0 * pi * d.h * d.h) : 1.0 / (120.0 * pi * d.h * d.h * d.h);
    S.kg = -5.0 * S.sigma / d.h;
    const double rho = d.rho0, m = d.mass;
    S.k_div = S.c * S.c * m * S.kg;                     // (m rho_i/rho_j) c^2, rho uniform
    double ecoef = 4.0 * m / (2.0 * rho);                // 4 m_j / (rho_i + rho_j)
    if (d.edac_rho_literal) ecoef /= rho;
    S.k_lap = ecoef * S.nu_e * S.kg;
    S.k_grad = -(m / (rho * rho)) * S.kg;
    S.k_visc = 4.0 * m * d.nu / (2.0 * rho) * S.kg;
    S.k_av = -d.alpha * d.h * S.c * rho;                 // rho^2 Pi = k_av * min(phi, 0)
    if (d.steady) {
        // eq. dp-dtau-frozen and eq. mom-steady: no EDAC term, no real-time term,
        // minus sum_j (V_i . gradW_ij)(V_i + V_j) m/rho with gradW = kg G r_ij
        S.steady = 1;
        S.k_lap = 0.0;
        S.gamma = 1.0;
        S.inv2dt = 0.0;
        S.k_conv = -(m / rho) * S.kg;
    }
    if (d.move) {
        // Algorithm 1: + sum_j (Vtilde_i . gradW_ij)(V_i + V_j) m/rho in the momentum
        // rate, + rho_i Vtilde_i . sum_j m (p_i + p_j)/rho^2 gradW_ij in the pressure rate
        S.move = d.move;
        S.k_conv = (m / rho) * S.kg;
        S.k_padv = (m / rho) * S.kg;
    }
    S.den_v = d.eta * d.h * d.h;
    S.den_e = d.edac_reg_literal ? d.h * d.h : d.eta * d.h * d.h;
    S.den_a = d.eps_av * d.h * d.h;
    S.tiny_r2 = 1e-12 * d.h * d.h;
    S.res_p = S.dt / (rho * S.c * S.c) / (double)nf;
    S.res_v = 1.0 / (d.vref * (double)nf);
    S.shift = d.shift ? 1 : 0;
    S.shift_n = d.shift_n;
    S.shift_r = d.shift_r;
    S.vol = m / rho;
    return S;
}

void setup_tiles(Ctx &c)
{
    std::vector<int2> tiles;
    std::vector<int4> segs;
    for (int s = 0; s < c.n_sims; ++s) {
        SimDev &S = c.sims_h[s];
        S.tile_begin = (int)tiles.size();
        const int per = c.block / c.lpp;  // particles per tile
        for (int off = 0; off < (int)c.nf[s]; off += per) tiles.push_back(make_int2(s, c.fluid_begin[s] + off));
        S.tile_end = (int)tiles.size();
        S.seg_begin = (int)segs.size();
        for (int t = S.tile_begin, k = 0; t < S.tile_end; t += kSegTiles, ++k)
            segs.push_back(make_int4(s, t, std::min(t + kSegTiles, S.tile_end), k));
        S.seg_count = (int)segs.size() - S.seg_begin;
    }
    c.n_tiles = (int)tiles.size();
    c.n_segs = (int)segs.size();
    DTSPH_HIP_CHECK(hipMemcpy(c.tiles, tiles.data(), sizeof(int2) * tiles.size(), hipMemcpyHostToDevice));
    DTSPH_HIP_CHECK(hipMemcpy(c.segs, segs.data(), sizeof(int4) * segs.size(), hipMemcpyHostToDevice));
    DTSPH_HIP_CHECK(hipMemcpy(c.sims, c.sims_h.data(), sizeof(SimDev) * c.n_sims, hipMemcpyHostToDevice));
}

template <typename T> void alloc_state(Ctx &c)
{
    const size_t N = c.N, Nf = c.Nf, Nw = std::max(c.Nw, 1);
    for (int b = 0; b < 2; ++b) {
        dev_alloc(c, c.orig[b], 4 * N);
        dev_alloc(c, c.simid[b], 4 * N);
        dev_alloc(c, c.x[b], 8 * 3 * N);
        dev_alloc(c, c.xn[b], 8 * 3 * N);
        dev_alloc(c, c.vn[b], sizeof(T) * 3 * Nf);
        dev_alloc(c, c.dv[b], sizeof(T) * 3 * Nf);
        dev_alloc(c, c.w[b], sizeof(T) * 3 * Nf);
        dev_alloc(c, c.w0[b], sizeof(T) * 3 * Nf);
        dev_alloc(c, c.pm[b], 8 * Nf);
        dev_alloc(c, c.pn[b], 8 * Nf);
        dev_alloc(c, c.dp[b], sizeof(T) * Nf);
        dev_alloc(c, c.vw[b], sizeof(T) * 3 * Nw);
        dev_alloc(c, c.pw[b], sizeof(T) * Nw);
        dev_alloc(c, c.vp[b], sizeof(T) * 4 * N);
    }
    dev_alloc(c, c.prec, (sizeof(T) == 4 ? 16 : 32) * N);
    dev_alloc(c, c.xr, 32 * N);
    if (c.any_move) {  // loop state of particles moving in pseudo-time
        dev_alloc(c, c.prec2, (sizeof(T) == 4 ? 16 : 32) * N);
        dev_alloc(c, c.xm, 8 * 3 * Nf);
        dev_alloc(c, c.vt, sizeof(T) * 3 * Nf);
    }
}

// ---- timing -------------------------------------------------------------------
hipEvent_t pool_event(Ctx &c, size_t k)
{
    while (c.ev_pool.size() <= k) {
        hipEvent_t e;
        DTSPH_HIP_CHECK(hipEventCreate(&e));
        c.ev_pool.push_back(e);
    }
    return c.ev_pool[k];
}

void resolve_timers(Ctx &c)
{
    for (auto &pr : c.ev_pending) {
        float ms = 0.f;
        DTSPH_HIP_CHECK(hipEventSynchronize(c.ev_pool[pr[0] + 1]));
        DTSPH_HIP_CHECK(hipEventElapsedTime(&ms, c.ev_pool[pr[0]], c.ev_pool[pr[0] + 1]));
        // pair passes are booked at the end of their loop, with their pairs
        if (pr[1] == 0) c.pass_times.emplace_back(pr[2], (double)ms);
        else if (pr[1] == 1) { c.tstats.wall_launches++; c.tstats.wall_ms += ms; }
        else if (pr[1] == 2) { c.tstats.build_launches++; c.tstats.build_ms += ms; c.tstats.build_particles += c.N; }
        else { c.tstats.filter_launches++; c.tstats.filter_ms += ms; }
    }
    c.ev_pending.clear();
    c.ev_used = 0;
}

// ---- flags / sync -------------------------------------------------------------
// Build flags moved to mapped host memory by k_finalize / k_publish; the host
// clears them after reading.
void check_host_flags(Ctx &c)
{
    if (c.timing) resolve_timers(c);
    const int over = c.flags_host[F_NBR_OVERFLOW], need = c.flags_host[F_NBR_NEEDED];
    const int cell = c.flags_host[F_CELL_OVERFLOW], outside = c.flags_host[F_OUTSIDE];
    const int skin = c.flags_host[F_SKIN];
    for (int k = 0; k < F_COUNT; ++k) c.flags_host[k] = 0;
    mirror_push_flags(c);
    if (skin)
        throw ApiError(DTSPH_EOVERFLOW, "a particle moving in pseudo-time (move = 2) left the candidate-list skin "
                                        "of its loop; lower dtau or dt");
    if (outside)
        throw ApiError(DTSPH_EINVAL, "a position on a periodic axis lies outside [lo, hi); the state was not "
                                     "accepted (set it again)");
    if (over)
        throw ApiError(DTSPH_EOVERFLOW, "neighbour list capacity " + std::to_string(c.cap) + " exceeded; needs " +
                                            std::to_string(need) + " (set max_neighbors); particle state is undefined");
    if (cell)
        throw ApiError(DTSPH_EOVERFLOW, "a cell holds more than 4096 particles (particles far outside the grid "
                                        "box or clumped); particle state is undefined");
}

// Wait until the last finalize has published every sim's report: spin on the
// per-sim sequence words in mapped memory (each written after its report, behind
// a system-scope fence), asking the stream for errors now and then.
void wait_reports(Ctx &c)
{
    const volatile int *seq = c.seq_host;
    auto seen = [&]() {
        for (int s = 0; s < c.n_sims; ++s)
            if (seq[s] != c.seq) return false;
        return true;
    };
    if (c.static_mode) {  // no mapped memory: wait for the stream, then copy
        DTSPH_HIP_CHECK(hipStreamSynchronize(c.stream));
        mirror_pull(c);
        if (!seen()) throw ApiError(DTSPH_EHIP, "finalize completed without publishing its reports");
        return;
    }
    for (long spins = 1;; ++spins) {
        if (seen()) break;
        __builtin_ia32_pause();
        if ((spins & 1023) == 0) {
            const hipError_t e = hipStreamQuery(c.stream);
            if (e == hipSuccess) {
                if (seen()) break;
                throw ApiError(DTSPH_EHIP, "the loop's launches completed without publishing every report "
                                           "(a tail launch's barrier wait gave up, or a kernel failed)");
            }
            if (e != hipErrorNotReady) throw HipError(e, "hipStreamQuery", __FILE__, __LINE__);
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
}

void readback_flags(Ctx &c)
{
    launch_publish(c);
    DTSPH_HIP_CHECK(hipStreamSynchronize(c.stream));
    mirror_pull(c);
    check_host_flags(c);
}

// Exact neighbour lists for the current positions: a filter of the candidate
// lists when every particle is known to be within skin/2 of where the lists
// were built, else a full cell build.
template <typename T> void ensure_cells(Ctx &c)
{
    if (!c.cells_valid) {
        if (c.cand_ok) filter_lists<T>(c);
        else build_cells<T>(c);
        c.cells_valid = true;
    }
}

// Rate pass at r^n and predictor. When the candidate lists of the last build
// still cover every neighbour at r^n, the pass runs over them directly: a
// candidate beyond the support adds exactly zero (every clipped kernel term is
// zero there), so no filtered list is needed for this one pass.
template <typename T> void do_predict(Ctx &c)
{
    if (c.in_loop) throw ApiError(DTSPH_EINVAL, "dtsph_predict: already inside a step (call dtsph_correct)");
    bool use_cand = false;
    if (!c.cells_valid) {
        if (c.cand_ok) use_cand = true;
        else ensure_cells<T>(c);
    }
    if (!c.records_fresh) launch_pre_records<T>(c);
    launch_wall<T>(c, MODE_PRE, use_cand);
    launch_pass<T>(c, MODE_PRE, use_cand);
    c.xb ^= 1;
    c.in_loop = true;
    // steady sims keep their particles where they are: their lists stay exact
    c.cells_valid = c.all_steady && c.cells_valid;
    c.cand_ok = false;
    c.records_fresh = false;
    c.p_half = false;
}

// Tile ranges of the sims whose loop is still running (from the stop flags in
// mapped memory); every tile when all run or the ranges do not fit.
void set_active_ranges(Ctx &c, bool all)
{
    c.n_ranges = 0;
    c.n_act_tiles = c.n_tiles;
    if (all) return;
    int n = 0, at = 0;
    int2 r[kMaxRanges];
    for (int s = 0; s < c.n_sims; ++s) {
        if (c.flags_host[F_COUNT + s]) continue;
        const int tb = c.sims_h[s].tile_begin, te = c.sims_h[s].tile_end;
        if (te <= tb) continue;
        if (n > 0 && r[n - 1].x + (at - r[n - 1].y) == tb) {
            at += te - tb;
            continue;
        }
        if (n == kMaxRanges) return;  // too fragmented: launch every tile
        r[n++] = make_int2(tb, at);
        at += te - tb;
    }
    if (at == c.n_tiles) return;
    c.n_ranges = n;
    c.n_act_tiles = at;
    for (int q = 0; q < n; ++q) c.ranges[q] = r[q];
}

// Do the candidate lists cover the shifted positions? (the loop's move plus the
// largest shift within 0.4 skin for every sim)
bool shift_cand_ok(const Ctx &c, double mx, bool use_cand, const std::vector<double> &disp)
{
    bool ok = true;
    for (int s = 0; s < c.n_sims; ++s) {
        const double moved = (use_cand ? disp[s] : 0.0) + mx;
        ok = ok && c.sims_h[s].skin > 0 && moved < 0.4 * c.sims_h[s].skin;
    }
    return ok;
}

void shift_outcome(Ctx &c, bool ok)
{
    c.shift_miss = ok ? 0 : c.shift_miss + 1;
    c.shift_nosync = c.shift_miss >= 3;
}

// After the shift kernels: the next rate pass may run on the candidate lists
// only if they cover the shifted positions, which needs the largest shift read
// back (a stream sync). After three steps in a row whose shifts left the skin,
// the sync is skipped and a rebuild taken; the value is read at the next wait
// (free by then), and a shift back inside the skin resumes the check.
void shift_decision(Ctx &c, bool use_cand)
{
    if (c.shift_nosync) {
        c.cand_ok = false;
        c.shift_pending = true;
        c.shift_pending_cand = use_cand;
        c.shift_disp = c.last_disp;
    } else {
        DTSPH_HIP_CHECK(hipStreamSynchronize(c.stream));
        mirror_pull(c);
        const double mx = *(volatile double *)c.sh_max_h;
        c.tstats.last_max_shift = mx;
        c.cand_ok = shift_cand_ok(c, mx, use_cand, c.last_disp);
        shift_outcome(c, c.cand_ok);
    }
    c.cells_valid = false;
    c.records_fresh = true;  // k_shift_apply rewrote the records
}

// A pseudo-time loop: set-up, chunks of iterations with a stop check after each,
// and the bookkeeping at its end.
struct LoopRun {
    int fixed = 0, max_it = 0, launched = 0, chunk = 1;
    bool spec = false, spec_next = false;  // speculative end of step after each chunk
    bool queued = false;  // the speculative launches follow the latest chunk
    bool split = false;   // the first chunk ends early for a tail launch
    int tries = 0;
};

// Length of a loop's first chunk: the last loop's longest (at most 64). A
// batch whose sims needed very different counts last time (cut schedule, see
// DTSPH_OPT_TAIL_LOOP) stops it at the first iteration k after which, by those
// counts, the sims still iterating hold at most a quarter of the tiles, if at
// least 4 iterations would remain: the host reads the reports there and cuts
// the launches down to those sims' tiles (or hands them to a tail launch),
// instead of launching every tile for a few sims.
int first_chunk(const Ctx &c, int max_it, bool *split = nullptr)
{
    const int n = std::min(c.chunk > 0 ? c.chunk : std::max(1, std::min(c.last_iters, 64)), max_it);
    if (split) *split = false;
    if (c.chunk > 0 || c.tail_loop == 0 || c.n_sims < 2) return n;
    for (int k = 1; k + 4 <= n; ++k) {
        int64_t tiles = 0;
        for (int s = 0; s < c.n_sims; ++s)
            if (c.prev_iters[s] < 0 || c.prev_iters[s] > k) tiles += c.sims_h[s].tile_end - c.sims_h[s].tile_begin;
        if (4 * tiles <= c.n_tiles) {
            if (split) *split = true;
            return k;
        }
    }
    return n;
}

template <typename T> void launch_speculation(Ctx &c, bool next_pre);

// Automatic pair-coefficient caching: the first iteration of a loop writes the
// coefficients (16 B per pair in FP32) and later ones read them. Streaming them
// from HBM is slower than recomputing (measured: the 518k-particle dam break's
// pass takes 2.5x as long), so it pays only when they stay in the last-level
// cache and the loop runs several iterations.
constexpr int kCacheMinIters = 3;
constexpr double kCacheMaxBytes = 32.0 * 1048576.0;

bool cache_usable(const Ctx &c) { return c.coef && !c.sep_den && !c.any_move && (!c.any_av || c.coef_av); }

template <typename T> void loop_prologue(Ctx &c, int fixed, LoopRun &L)
{
    if (!c.in_loop) throw ApiError(DTSPH_EINVAL, "dtsph_pseudo_iterate: not inside a step (call dtsph_predict)");
    if (fixed < 0) throw ApiError(DTSPH_EINVAL, "fixed_iters must be >= 0");
    if (c.any_move2) c.cand_ok = false;  // list updates filter candidates centred at r^(0)
    if (!c.cells_valid && !c.cand_ok) {
        // full build at the frozen positions, with the loop set-up in its gather
        build_cells<T>(c, fixed);
        c.cells_valid = true;
    } else {
        ensure_cells<T>(c);
        launch_loop_begin<T>(c, fixed);
    }
    launch_move_begin<T>(c);
    set_active_ranges(c, true);
    c.pass_times.clear();
    L.fixed = fixed;
    L.max_it = fixed;
    if (fixed == 0)
        for (auto &d : c.desc) L.max_it = std::max(L.max_it, (int)d.max_iter);
    L.launched = 0;
    L.chunk = first_chunk(c, L.max_it, &L.split);
    const int expect = fixed > 0 ? fixed : c.last_iters;
    bool fits = false;
    if (c.pair_cache == 2) {
        double entries = 0.0;  // list entries of the fluid, from the last reports
        for (int s = 0; s < c.n_sims; ++s) entries += (double)c.pairs_host[s];
        const double per = (c.precision == DTSPH_FP32 ? 16.0 : 32.0) * (c.any_av ? 1.5 : 1.0);
        fits = entries > 0 && entries * per <= kCacheMaxBytes;
    }
    c.loop_cached = cache_usable(c) && (c.pair_cache == 1 || (c.pair_cache == 2 && expect >= kCacheMinIters && fits));
}

// Wall passes of a loop run with the previous iteration's residual reduction
// (one launch less per iteration), except for the first iteration and in
// contexts whose lists change between iterations (moving sims with list
// updates filter the lists before each wall pass).
bool fused_walls(const Ctx &c) { return c.Nw > 0 && !c.any_move2; }

// The next chunk of iterations (its size: L.chunk, capped by the iteration limit).
template <typename T> void launch_chunk(Ctx &c, LoopRun &L)
{
    const int n = std::min(L.chunk, L.max_it - L.launched);
    const bool fuse = fused_walls(c);
    for (int k = 0; k < n; ++k) {
        c.pass_index = L.launched + k;
        // moving sims with neighbour updates: exact lists at r^{k+1/2}
        if (c.any_move2 && L.launched + k > 0) filter_lists<T>(c);
        if (!fuse || L.launched + k == 0) launch_wall<T>(c, MODE_PSEUDO);
        // with cached coefficients the loop's first pass stores them, later ones
        // read; steady contexts keep them from loop to loop (lists and positions
        // do not change)
        c.cache_phase = c.loop_cached ? (c.coef_valid ? 2 : 1) : 0;
        launch_pass<T>(c, MODE_PSEUDO);
        if (c.cache_phase == 1) c.coef_valid = true;
        c.cache_phase = 0;
        // the chunk's last one publishes the reports
        if (fuse) launch_finalize_wall<T>(c, k == n - 1, L.launched + k + 1);
        else launch_finalize(c, k == n - 1);
    }
    L.launched += n;
}

// Waits for the chunk in flight, launches more until every sim has stopped, and
// books the loop's reports.
template <typename T> int loop_finish(Ctx &c, LoopRun &L, dtsph_iter_report *rep)
{
    for (;;) {
        wait_reports(c);  // k_finalize wrote the mapped reports
        check_host_flags(c);
        if (c.shift_pending) {  // the last shift has finished: book its size
            c.shift_pending = false;
            const double mx = *(volatile double *)c.sh_max_h;
            c.tstats.last_max_shift = mx;
            shift_outcome(c, shift_cand_ok(c, mx, c.shift_pending_cand, c.shift_disp));
        }
        bool all = true;
        for (int s = 0; s < c.n_sims; ++s) all = all && c.flags_host[F_COUNT + s];
        if (all || L.launched >= L.max_it) break;
        // more iterations than the last loop needed: chunks grow with the loop
        // (sims that stop inside a chunk leave only no-op launches behind)
        set_active_ranges(c, false);
        if (c.tail_loop == 1 && launch_tail<T>(c, L.launched)) {
            L.launched = L.max_it;  // every sim of the launch stops in it
        } else {
            L.chunk = c.chunk > 0 ? c.chunk : std::max(2, std::min(L.launched / 2, 32));
            launch_chunk<T>(c, L);
        }
        L.queued = L.spec;
        if (L.spec) {
            launch_speculation<T>(c, L.spec_next);
            L.tries++;
        }
    }
    set_active_ranges(c, true);
    if (fused_walls(c)) launch_wall_pressure<T>(c);
    c.p_half = true;  // p^K = p^{K+1/2} - dtau/2 (dp/dtau)^K is applied lazily
    int status = DTSPH_OK, most = 1;
    bool cand = true;
    for (int s = 0; s < c.n_sims; ++s) {
        const MirrorRep &it = c.reps_host[s];
        // r^{n+1} - r^(0) = dt/2 (V^{n+1} - V^(0)): within skin/2 (with margin) the
        // candidate lists built at r^(0) still hold every neighbour at r^{n+1}
        cand = cand && c.sims_h[s].skin > 0 && it.disp < 0.4 * c.sims_h[s].skin;
        c.last_disp[s] = it.disp;
        c.tstats.last_disp = s == 0 ? it.disp : std::max(c.tstats.last_disp, it.disp);
        const int64_t pairs = (int64_t)c.pairs_host[s];
        most = std::max(most, it.iters);
        if (rep) {
            rep[s].iters = it.iters;
            rep[s].reason = it.reason;
            rep[s].rp_mean = it.rp_mean;
            rep[s].rv_mean = it.rv_mean;
            rep[s].rp_max = it.rp_max;
            rep[s].rv_max = it.rv_max;
            rep[s].pairs = pairs;
        }
        if (it.reason == DTSPH_NONFINITE) status = DTSPH_ENONFINITE;
        else if (it.reason == DTSPH_MAXITER && status == DTSPH_OK) status = DTSPH_WARN_MAXITER;
    }
    c.last_iters = most;
    for (int s = 0; s < c.n_sims; ++s) c.prev_iters[s] = c.reps_host[s].iters;
    for (const auto &pt : c.pass_times) {  // timed launches with the sims that took part
        int64_t pairs = 0, parts = 0;
        for (int s = 0; s < c.n_sims; ++s)
            if (pt.first < c.reps_host[s].iters) {
                pairs += (int64_t)c.pairs_host[s];
                parts += c.nf[s];
            }
        if (pairs == 0) continue;  // a launch after every sim had stopped
        c.tstats.pass_launches++;
        c.tstats.pass_ms += pt.second;
        c.tstats.pass_pairs += pairs;
        c.tstats.pass_particles += parts;
    }
    c.pass_times.clear();
    c.cand_next = cand;
    if (status == DTSPH_ENONFINITE) c.err = "non-finite residual in the pseudo-time loop";
    return status;
}

template <typename T> int do_loop(Ctx &c, int fixed, dtsph_iter_report *rep)
{
    LoopRun L;
    loop_prologue<T>(c, fixed, L);
    launch_chunk<T>(c, L);
    return loop_finish<T>(c, L, rep);
}

// Particle shifting after the corrector (section 3.5) for the sims that ask
// for it. The sums run over the candidate lists when they cover r^{n+1}, else
// over lists of a fresh build there; the largest shift is read back to decide
// whether the candidate lists still cover the shifted positions.
template <typename T> void do_shift(Ctx &c)
{
    const bool use_cand = c.cand_ok;
    if (!use_cand) {
        build_cells<T>(c);
        c.cells_valid = true;
        launch_pre_records<T>(c);
    }
    launch_shift<T>(c, use_cand);
    shift_decision(c, use_cand);
}

template <typename T> void do_correct(Ctx &c)
{
    if (!c.in_loop) throw ApiError(DTSPH_EINVAL, "dtsph_correct: not inside a step (call dtsph_predict)");
    launch_correct<T>(c);
    c.in_loop = false;
    c.cells_valid = c.all_steady && c.cells_valid;
    c.cand_ok = c.cand_next;
    c.p_half = false;
    c.records_fresh = true;
    if (c.any_shift) do_shift<T>(c);
}

// Would the timer sample one of the next n pair-pass launches?
bool pass_timer_fires(const Ctx &c, int n)
{
    if (!c.timing) return false;
    if (c.timing_first) return true;  // the segment holds the loop's first pass
    for (int k = 0; k < n; ++k)
        if ((c.timer_count[0] + k) % c.timing_every == 0) return true;
    return false;
}

// The segment of a real step that runs without host decisions: rate pass and
// predictor, the build at the frozen positions with the loop set-up, and the
// first chunk of pseudo-iterations. With graphs on (and no timed launch in it)
// it is captured once per key into a HIP graph and replayed afterwards; the
// host logic still runs (launching nothing) to keep the context's bookkeeping.
template <typename T> void step_segment(Ctx &c, LoopRun &L)
{
    auto body = [&]() {
        do_predict<T>(c);
        loop_prologue<T>(c, 0, L);
        launch_chunk<T>(c, L);
    };
    int max_it = 0;
    for (auto &d : c.desc) max_it = std::max(max_it, (int)d.max_iter);
    const int n = first_chunk(c, max_it);
    if (!c.graphs || pass_timer_fires(c, n)) {
        body();
        return;
    }
    const bool use_cand = !c.cells_valid && c.cand_ok;
    const uint64_t key = (uint64_t)c.buf | (uint64_t)c.xb << 1 | (uint64_t)use_cand << 2 |
                         (uint64_t)c.cells_valid << 3 | (uint64_t)c.records_fresh << 4 | (uint64_t)c.cur << 5 |
                         (uint64_t)n << 8;
    constexpr size_t kMaxGraphs = 16;  // recording is costly: past this many keys, launch plainly
    if (c.graph_cache.size() >= kMaxGraphs && c.graph_cache.find(key) == c.graph_cache.end()) {
        body();
        return;
    }
    struct SegmentFlags {  // restores the mode flags however the body ends
        Ctx &c;
        hipStream_t stream;
        ~SegmentFlags() { c.replay = false; c.in_segment = false; c.stream = stream; }
    } guard{c, c.stream};
    c.in_segment = true;
    auto hit = c.graph_cache.find(key);
    if (hit != c.graph_cache.end()) {
        c.replay = true;
        body();
        c.replay = false;
        DTSPH_HIP_CHECK(hipGraphLaunch(hit->second, guard.stream));
        return;
    }
    DTSPH_HIP_CHECK(hipStreamBeginCapture(c.cap_stream, hipStreamCaptureModeRelaxed));
    c.stream = c.cap_stream;
    hipGraph_t g = nullptr;
    try {
        body();
    } catch (...) {
        (void)hipStreamEndCapture(c.cap_stream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    c.stream = guard.stream;
    DTSPH_HIP_CHECK(hipStreamEndCapture(c.cap_stream, &g));
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) throw HipError(e, "hipGraphInstantiate", __FILE__, __LINE__);
    c.graph_cache[key] = ex;
    DTSPH_HIP_CHECK(hipGraphLaunch(ex, c.stream));
}

// Speculative end of step: behind a device gate (every sim stopped, no
// non-finite residual, candidate lists still cover r^{n+1}; evaluated once by
// k_gate into a word every gated workgroup reads) queue the corrector
// and, when another step follows, the next rate pass on the candidate lists, so
// the GPU works while the host waits for the reports. When the gate is closed
// these launches return at once and the host proceeds as without them.
template <typename T> void launch_speculation(Ctx &c, bool next_pre)
{
    c.tstats.spec_tries++;
    launch_gate(c);
    c.gated = true;
    const bool p_half = c.p_half;
    c.p_half = true;  // state at the end of a loop: p^K is still pending
    launch_correct<T>(c);
    c.p_half = p_half;
    if (c.any_shift) launch_shift<T>(c, true);  // the gate implies valid candidate lists
    if (next_pre) {
        // after the corrector the records are fresh; the lists are those of
        // r^(0) (candidates) or, for steady contexts, still exact
        const bool use_cand = !(c.all_steady && c.cells_valid);
        launch_wall<T>(c, MODE_PRE, use_cand);
        launch_pass<T>(c, MODE_PRE, use_cand);
    }
    c.gated = false;
}

// The host's reading of the gate, from the published reports.
bool gate_open(const Ctx &c)
{
    if (!c.cand_next) return false;
    for (int s = 0; s < c.n_sims; ++s)
        if (!c.flags_host[F_COUNT + s] || c.reps_host[s].reason == DTSPH_NONFINITE) return false;
    return true;
}

template <typename T> int do_step(Ctx &c, int n_steps, dtsph_iter_report *reps)
{
    if (n_steps < 0) throw ApiError(DTSPH_EINVAL, "n_steps must be >= 0");
    if (c.in_loop) throw ApiError(DTSPH_EINVAL, "dtsph_step: inside a step (call dtsph_correct first)");
    int status = DTSPH_OK;
    c.spec_ready = false;
    for (int s = 0; s < n_steps; ++s) {
        LoopRun L;
        if (c.spec_ready) {  // this step's rate pass and predictor already ran
            c.spec_ready = false;
            loop_prologue<T>(c, 0, L);
            launch_chunk<T>(c, L);
        } else {
            step_segment<T>(c, L);
        }
        // speculate while it mostly pays (a closed gate costs a few no-op
        // launches); after a run of misses, probe again every 16 steps
        L.spec = c.speculate && !c.graphs && c.n_sims <= 64 && (c.spec_score > 0 || ++c.spec_idle % 16 == 0);
        L.spec_next = s + 1 < n_steps && !c.any_shift;  // shifting: the rate pass waits for the shift's size
        // (not after a first chunk cut for a tail launch: the loop rarely ends there)
        L.queued = L.spec && !L.split;
        if (L.queued) {
            launch_speculation<T>(c, L.spec_next);
            L.tries++;
        }
        int st = loop_finish<T>(c, L, reps ? reps + (size_t)s * c.n_sims : nullptr);
        // the gated launches ran only if they followed the loop's last chunk
        const bool hit = L.queued && gate_open(c);
        if (L.spec) {
            c.spec_score = std::min(8, c.spec_score + (hit ? 1 : 0) - 2 * (L.tries - (hit ? 1 : 0)));
            if (c.spec_score > 0) c.spec_idle = 0;
        }
        if (hit) {
            c.tstats.spec_hits++;
            // book what the gated launches did: do_correct, then do_predict
            c.in_loop = false;
            c.cells_valid = c.all_steady && c.cells_valid;
            c.cand_ok = c.cand_next;
            c.p_half = false;
            c.records_fresh = true;
            if (c.any_shift) shift_decision(c, true);  // the gated shift ran on the candidate lists
            if (L.spec_next) {
                c.xb ^= 1;
                c.in_loop = true;
                c.cells_valid = c.all_steady && c.cells_valid;
                c.cand_ok = false;
                c.records_fresh = false;
                c.spec_ready = true;
            }
        } else {
            do_correct<T>(c);
        }
        if (st < 0) return st;
        if (st > 0) status = st;
    }
    return status;
}

template <typename F> auto by_precision(Ctx &c, F &&f)
{
    if (c.precision == DTSPH_FP32) return f(float());
    return f(double());
}

}  // namespace

namespace dtsph {

// The first-pass mode samples the first pair and wall pass of every loop (every
// sim takes part: the launch covers the whole workload, and it is queued behind
// the build, so its events hold the kernel alone) and every build.
bool timer_skips(Ctx &c, int kind)
{
    if (c.timing_first) return kind <= 1 && c.pass_index != 0;
    return c.timer_count[kind]++ % c.timing_every != 0;
}

int timer_begin(Ctx &c, int kind)
{
    if (!c.timing) return -1;
    if (c.in_segment && kind != 0) return -1;  // graph segments time pair passes only
    if (timer_skips(c, kind)) return -1;
    size_t k = c.ev_used;
    c.ev_used += 2;
    DTSPH_HIP_CHECK(hipEventRecord(pool_event(c, k), c.stream));
    pool_event(c, k + 1);
    return (int)k;
}

int timer_slot(Ctx &c, int kind)
{
    if (!c.timing) return -1;
    if (c.in_segment && kind != 0) return -1;
    if (timer_skips(c, kind)) return -1;
    size_t k = c.ev_used;
    c.ev_used += 2;
    pool_event(c, k + 1);
    return (int)k;
}

void timer_book(Ctx &c, int slot, int kind)
{
    if (slot < 0) return;
    c.ev_pending.push_back({slot, kind, kind == 0 ? c.pass_index : -1});
}

void timer_end(Ctx &c, int slot, int kind)
{
    if (slot < 0) return;
    DTSPH_HIP_CHECK(hipEventRecord(c.ev_pool[slot + 1], c.stream));
    c.ev_pending.push_back({slot, kind, kind == 0 ? c.pass_index : -1});
}

}  // namespace dtsph

extern "C" {

static int create_impl(const dtsph_sim_desc *sims, const int64_t *n_fluid, const int64_t *n_wall, int32_t n_sims,
                       int32_t precision, void *hip_stream, dtsph_ctx **out, bool static_mode)
{
    if (out) *out = nullptr;
    dtsph_ctx *ctx = nullptr;
    try {
        if (!sims || !n_fluid || !n_wall || !out) throw ApiError(DTSPH_EINVAL, "NULL argument");
        if (n_sims < 1) throw ApiError(DTSPH_EINVAL, "n_sims must be >= 1");
        if (precision != DTSPH_FP32 && precision != DTSPH_FP64)
            throw ApiError(DTSPH_EINVAL, "precision must be DTSPH_FP32 or DTSPH_FP64");
        int64_t N = 0, Nf = 0, Nw = 0, C = 0;
        for (int s = 0; s < n_sims; ++s) {
            check_desc(sims[s], s, n_fluid[s], n_wall[s]);
            if (sims[s].dim != sims[0].dim) throw ApiError(DTSPH_EINVAL, "all sims of a context must share dim");
            Nf += n_fluid[s];
            Nw += n_wall[s];
        }
        N = Nf + Nw;
        if (N >= (int64_t)1 << 31) throw ApiError(DTSPH_EINVAL, "too many particles for one context");

        ctx = new dtsph_ctx();
        Ctx &c = ctx->c;
        DTSPH_HIP_CHECK(hipGetDevice(&c.device));
        c.stream = (hipStream_t)hip_stream;
        if (static_mode) {
            std::lock_guard<std::mutex> lk(g_static_mu);
            char *base = (char *)static_scratch(c.device);
            if (g_scratch_busy[c.device])
                throw ApiError(DTSPH_EINVAL, "the static scratch of this device is held by another static context");
            g_scratch_busy[c.device] = true;
            c.static_mode = true;
            c.bump = base;
            c.bump_cap = DTSPH_STATIC_SCRATCH_BYTES;
        } else {
            DTSPH_HIP_CHECK(hipStreamCreateWithFlags(&c.cap_stream, hipStreamNonBlocking));
        }
        c.precision = precision;
        c.n_sims = n_sims;
        c.N = (int)N;
        c.Nf = (int)Nf;
        c.Nw = (int)Nw;
        c.desc.assign(sims, sims + n_sims);
        c.nf.assign(n_fluid, n_fluid + n_sims);
        c.nw.assign(n_wall, n_wall + n_sims);
        c.max_dim = sims[0].dim;
        c.sims_h.resize(n_sims);
        c.skin_default.resize(n_sims);
        c.prev_iters.assign(n_sims, -1);
        c.fluid_begin.resize(n_sims);
        int64_t fb = 0, wb = 0;
        double cap_est = 0;
        std::vector<int> init_slot(2 * N);
        int64_t caller = 0;
        for (int s = 0; s < n_sims; ++s) {
            const dtsph_sim_desc &d = sims[s];
            SimDev S = make_simdev(d, n_fluid[s], n_wall[s]);
            S.fluid_begin = (int)fb;
            S.wall_begin = (int)wb;
            // the finest subdivision at the smallest skin (0, see DTSPH_OPT_SKIN) has
            // the most cells: it sizes the key tables
            SimDev S0 = S;
            S0.cand_r2 = S0.kh2;
            set_grid(S0, 3);
            int64_t cells = (int64_t)S0.ncell[0] * S0.ncell[1] * S0.ncell[2];
            C += cells;
            if (2 * C > (int64_t)4096 * 4096)
                throw ApiError(DTSPH_EINVAL, "cell grid too large (more than 8M cells); enlarge h or shrink the box");
            c.sims_h[s] = S;
            c.skin_default[s] = S.skin;
            c.fluid_begin[s] = (int)fb;
            for (int64_t k = 0; k < n_fluid[s]; ++k, ++caller) {
                init_slot[caller] = (int)(fb + k);
                init_slot[N + caller] = s;
            }
            for (int64_t k = 0; k < n_wall[s]; ++k, ++caller) {
                init_slot[caller] = (int)(Nf + wb + k);
                init_slot[N + caller] = s;
            }
            fb += n_fluid[s];
            wb += n_wall[s];
            c.any_walls = c.any_walls || n_wall[s] > 0;
            c.any_av = c.any_av || d.alpha > 0;
            c.any_shift = c.any_shift || d.shift;
            c.any_steady = c.any_steady || d.steady;
            c.any_move = c.any_move || d.move;
            c.any_move2 = c.any_move2 || d.move == 2;
            c.all_steady = c.all_steady && d.steady;
            c.sep_den = c.sep_den || S.den_e != S.den_v || (d.alpha > 0 && S.den_a != S.den_v);
            double est;
            if (d.max_neighbors > 0) {
                est = d.max_neighbors;
            } else {
                const double dx = std::pow(d.mass / d.rho0, 1.0 / d.dim), kh = d.kappa * d.h * 1.04;
                const double lat = d.dim == 2 ? 3.14159265358979 * kh * kh / (dx * dx)
                                              : 4.0 / 3.0 * 3.14159265358979 * kh * kh * kh / (dx * dx * dx);
                est = 1.5 * lat + 8.0;
            }
            cap_est = std::max(cap_est, est);
        }
        c.C_max = (int)C;
        setup_keys(c, 2);
        c.cap = std::min(8000, ((int)std::ceil(cap_est) + 3) / 4 * 4);

        // device memory
        dev_alloc(c, c.sims, sizeof(SimDev) * n_sims);
        dev_alloc(c, c.iters, sizeof(SimIter) * (n_sims + 1));  // + the speculative gate
        if (precision == DTSPH_FP32) alloc_state<float>(c);
        else alloc_state<double>(c);
        dev_alloc(c, c.key, 4 * (size_t)N);
        dev_alloc(c, c.rank, 4 * (size_t)N);
        dev_alloc(c, c.perm, 4 * (size_t)N);
        dev_alloc(c, c.count, 4 * (size_t)(2 * c.C_max));
        dev_alloc(c, c.cell_start, 4 * (size_t)(2 * c.C_max + 1));
        dev_alloc(c, c.scan_tmp, 4 * (size_t)(4096 + 1));
        dev_alloc(c, c.nbr, 4 * (size_t)c.cap * (size_t)N);
        dev_alloc(c, c.cnt, 4 * (size_t)N);
        c.capc = c.cap;
        dev_alloc(c, c.cand, 4 * (size_t)c.capc * (size_t)N);
        dev_alloc(c, c.ccnt, 4 * (size_t)N);
        {   // strip table: room for the most strips of any subdivision
            int64_t most = 0;
            for (int m = 1; m <= 3; ++m) {
                std::vector<SimDev> g = c.sims_h;
                for (SimDev &S : g) set_grid(S, m);
                most = std::max(most, count_strips(g));
            }
            if (most > 0 && most < INT32_MAX) {
                c.strip_cap = (int)most;
                dev_alloc(c, c.strips, sizeof(int4) * (size_t)most);
            }
        }
        setup_keys(c, c.cell_div);
        // lanes per particle: enough threads for ~8 waves per SIMD on 256 CUs
        {
            int lpp = 1;
            while (lpp < 8 && (int64_t)lpp * Nf < (int64_t)256 * 2048) lpp *= 2;
            c.lpp = lpp;
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tune_cache.find(tune_key(c));
            if (it != g_tune_cache.end()) {
                c.lpp = it->second[0];
                c.block = it->second[1];
                c.g_nbr = it->second[2];
                c.g_filter = it->second[3];
                c.nbr_tiles = c.strips ? it->second[5] : 0;
                setup_keys(c, it->second[4]);
            }
        }
        const size_t max_tiles = (size_t)(Nf + n_sims + 8);
        dev_alloc(c, c.tiles, sizeof(int2) * max_tiles);
        dev_alloc(c, c.partials, sizeof(double4) * max_tiles);
        const size_t max_segs = max_tiles / kSegTiles + (size_t)n_sims + 1;
        if (!c.static_mode) {  // tail launches: arrivals, error word, group words; odd iterations' partials
            dev_alloc(c, c.tail_words, sizeof(uint32_t) * (2 * (size_t)n_sims + 2 + max_tiles / kTailGroup));
            dev_alloc(c, c.tail_part4, sizeof(double4) * max_tiles);
            dev_alloc(c, c.tail_part2, sizeof(double2) * max_tiles);
        }
        dev_alloc(c, c.segs, sizeof(int4) * max_segs);
        dev_alloc(c, c.seg_p, sizeof(double4) * max_segs);
        dev_alloc(c, c.seg_p2, sizeof(double2) * max_segs);
        dev_alloc(c, c.tickets, sizeof(uint32_t) * n_sims);
        dev_alloc(c, c.pubcount, sizeof(uint32_t) * n_sims);
        dev_alloc(c, c.partials2, sizeof(double2) * max_tiles);
        dev_alloc(c, c.flags, sizeof(int) * (F_COUNT + n_sims));
        c.done_dev = c.flags + F_COUNT;
        dev_alloc(c, c.init_slot, sizeof(int) * 2 * (size_t)N);
        if (c.any_shift) {
            dev_alloc(c, c.sh_dr, 8 * 3 * (size_t)Nf);
            dev_alloc(c, c.sh_dp, 8 * (size_t)Nf);
            dev_alloc(c, c.sh_dv, 8 * 3 * (size_t)Nf);
            dev_alloc(c, c.sh_part, 8 * ((size_t)Nf * 4 / 256 + 2));  // per shift-sum workgroup
        }
        c.last_disp.assign(n_sims, 0.0);
        {
            const size_t fb_bytes = (sizeof(int) * (F_COUNT + n_sims) + 15) / 16 * 16;
            const size_t pb_bytes = 8 * (size_t)n_sims;
            const size_t rb_bytes = (sizeof(MirrorRep) * n_sims + 15) / 16 * 16;
            const size_t sq_bytes = (sizeof(int) * n_sims + 15) / 16 * 16;
            const size_t bytes = fb_bytes + pb_bytes + rb_bytes + sq_bytes + 16;
            void *md = nullptr;
            if (c.static_mode) {
                // device memory in the scratch, copied to a static host buffer after each sync
                if (bytes > kStaticMirrorBytes)
                    throw ApiError(DTSPH_EINVAL, "too many sims for a static context");
                c.mirror_h = g_static_mirror[c.device];
                c.mirror_bytes = bytes;
                std::memset(c.mirror_h, 0, bytes);
                const size_t b = ws_round(bytes);
                if (c.bump_off + b > c.bump_cap) throw ApiError(DTSPH_ENOMEM, "the static scratch is too small");
                c.mirror_dev = c.bump + c.bump_off;
                c.bump_off += b;
                DTSPH_HIP_CHECK(hipMemset(c.mirror_dev, 0, bytes));
                md = c.mirror_dev;
            } else {
                DTSPH_HIP_CHECK(hipHostMalloc(&c.mirror_h, bytes, hipHostMallocMapped));
                std::memset(c.mirror_h, 0, bytes);
                DTSPH_HIP_CHECK(hipHostGetDevicePointer(&md, c.mirror_h, 0));
            }
            char *hb = (char *)c.mirror_h, *db = (char *)md;
            c.flags_host = (int *)hb;
            c.pairs_host = (unsigned long long *)(hb + fb_bytes);
            c.reps_host = (MirrorRep *)(hb + fb_bytes + pb_bytes);
            c.m_flags_d = (int *)db;
            c.m_pairs_d = (unsigned long long *)(db + fb_bytes);
            c.m_reps_d = (MirrorRep *)(db + fb_bytes + pb_bytes);
            c.seq_host = (int *)(hb + fb_bytes + pb_bytes + rb_bytes);
            c.m_seq_d = (int *)(db + fb_bytes + pb_bytes + rb_bytes);
            c.sh_max_h = (double *)(hb + fb_bytes + pb_bytes + rb_bytes + sq_bytes);
            c.sh_max_d = (double *)(db + fb_bytes + pb_bytes + rb_bytes + sq_bytes);
        }
        DTSPH_HIP_CHECK(hipMemcpy(c.init_slot, init_slot.data(), sizeof(int) * 2 * N, hipMemcpyHostToDevice));
        DTSPH_HIP_CHECK(hipMemset(c.flags, 0, sizeof(int) * (F_COUNT + n_sims)));
        DTSPH_HIP_CHECK(hipMemset(c.tickets, 0, sizeof(uint32_t) * n_sims));
        DTSPH_HIP_CHECK(hipMemset(c.pubcount, 0, sizeof(uint32_t) * n_sims));
        DTSPH_HIP_CHECK(hipMemset(c.cell_start, 0, 4 * (size_t)(2 * c.C_max + 1)));
        DTSPH_HIP_CHECK(hipMemset(c.count, 0, 4 * (size_t)(2 * c.C_max)));
        DTSPH_HIP_CHECK(hipMemset(c.cnt, 0, 4 * (size_t)N));
        setup_tiles(c);
        DTSPH_HIP_CHECK(hipDeviceSynchronize());
        *out = ctx;
        return DTSPH_OK;
    } catch (const ApiError &e) {
        g_create_error = e.what;
        if (ctx) { free_all(ctx->c); delete ctx; }
        return e.status;
    } catch (const HipError &e) {
        g_create_error = e.what;
        if (ctx) { free_all(ctx->c); delete ctx; }
        return DTSPH_EHIP;
    } catch (...) {
        g_create_error = "unknown error in dtsph_create";
        if (ctx) { free_all(ctx->c); delete ctx; }
        return DTSPH_EHIP;
    }
}

int dtsph_create(const dtsph_sim_desc *sims, const int64_t *n_fluid, const int64_t *n_wall, int32_t n_sims,
                 int32_t precision, void *hip_stream, dtsph_ctx **out)
{
    return create_impl(sims, n_fluid, n_wall, n_sims, precision, hip_stream, out, false);
}

int dtsph_create_static(const dtsph_sim_desc *sims, const int64_t *n_fluid, const int64_t *n_wall, int32_t n_sims,
                        int32_t precision, void *hip_stream, dtsph_ctx **out)
{
    return create_impl(sims, n_fluid, n_wall, n_sims, precision, hip_stream, out, true);
}

void dtsph_destroy(dtsph_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->c.device);
    (void)hipStreamSynchronize(ctx->c.stream);
    free_all(ctx->c);
    delete ctx;
}

const char *dtsph_last_error(const dtsph_ctx *ctx)
{
    if (!ctx) return g_create_error.c_str();
    return ctx->c.err.empty() ? "no error" : ctx->c.err.c_str();
}

int dtsph_set_state(dtsph_ctx *ctx, const dtsph_state_view *s)
{
    return guarded(ctx, [&](Ctx &c) {
        if (!s || !s->x || !s->v || !s->v_prev || !s->p) throw ApiError(DTSPH_EINVAL, "x, v, v_prev, p are required");
        const bool lp = s->x_iter != nullptr;
        if (lp && (!s->v_iter || !s->p_iter || !s->dpdtau))
            throw ApiError(DTSPH_EINVAL, "in-loop state needs x_iter, v_iter, p_iter and dpdtau");
        by_precision(c, [&](auto t) {
            using T = decltype(t);
            launch_set_state<T>(c, *s, lp);
            return 0;
        });
        c.in_loop = lp;
        c.cells_valid = false;
        c.coef_valid = false;
        c.cand_ok = false;
        c.cand_next = false;
        c.cur = 0;
        c.p_half = false;
        c.records_fresh = false;
        readback_flags(c);
        return DTSPH_OK;
    });
}

int dtsph_get_state(dtsph_ctx *ctx, const dtsph_state_view *s)
{
    return guarded(ctx, [&](Ctx &c) {
        if (!s) throw ApiError(DTSPH_EINVAL, "NULL view");
        const bool want_loop = s->x_iter || s->v_iter || s->p_iter || s->dpdtau;
        if (want_loop && !c.in_loop) throw ApiError(DTSPH_EINVAL, "in-loop fields requested outside a step");
        by_precision(c, [&](auto t) {
            using T = decltype(t);
            launch_get_state<T>(c, *s, c.in_loop);
            return 0;
        });
        DTSPH_HIP_CHECK(hipStreamSynchronize(c.stream));
        return DTSPH_OK;
    });
}

int dtsph_build_cells(dtsph_ctx *ctx, const dtsph_cells_view *out)
{
    return guarded(ctx, [&](Ctx &c) {
        by_precision(c, [&](auto t) {
            using T = decltype(t);
            ensure_cells<T>(c);
            return 0;
        });
        readback_flags(c);
        if (!out) return DTSPH_OK;
        const size_t N = c.N, K = 2 * (size_t)c.C + 1;
        if (out->keys) {
            std::vector<uint32_t> key(N), perm(N);
            DTSPH_HIP_CHECK(hipMemcpy(key.data(), c.key, 4 * N, hipMemcpyDeviceToHost));
            DTSPH_HIP_CHECK(hipMemcpy(perm.data(), c.rank, 4 * N, hipMemcpyDeviceToHost));
            for (size_t d = 0; d < N; ++d) out->keys[d] = (int32_t)key[perm[d]];
        }
        if (out->caller_index)
            DTSPH_HIP_CHECK(hipMemcpy(out->caller_index, c.orig[c.buf], 4 * N, hipMemcpyDeviceToHost));
        if (out->cell_start) {
            std::vector<uint32_t> cs(K);
            DTSPH_HIP_CHECK(hipMemcpy(cs.data(), c.cell_start, 4 * K, hipMemcpyDeviceToHost));
            for (size_t k = 0; k < K; ++k) out->cell_start[k] = cs[k];
        }
        return DTSPH_OK;
    });
}

int dtsph_predict(dtsph_ctx *ctx)
{
    return guarded(ctx, [&](Ctx &c) {
        by_precision(c, [&](auto t) {
            using T = decltype(t);
            do_predict<T>(c);
            return 0;
        });
        readback_flags(c);
        return DTSPH_OK;
    });
}

int dtsph_pseudo_iterate(dtsph_ctx *ctx, int32_t fixed_iters, dtsph_iter_report *rep)
{
    return guarded(ctx, [&](Ctx &c) {
        return by_precision(c, [&](auto t) {
            using T = decltype(t);
            return do_loop<T>(c, fixed_iters, rep);
        });
    });
}

int dtsph_correct(dtsph_ctx *ctx)
{
    return guarded(ctx, [&](Ctx &c) {
        by_precision(c, [&](auto t) {
            using T = decltype(t);
            do_correct<T>(c);
            return 0;
        });
        DTSPH_HIP_CHECK(hipStreamSynchronize(c.stream));
        return DTSPH_OK;
    });
}

int dtsph_step(dtsph_ctx *ctx, int32_t n_steps, dtsph_iter_report *reps)
{
    return guarded(ctx, [&](Ctx &c) {
        return by_precision(c, [&](auto t) {
            using T = decltype(t);
            return do_step<T>(c, n_steps, reps);
        });
    });
}

int dtsph_neighbor_list(dtsph_ctx *ctx, int32_t sim, int64_t *offsets, int32_t *nbrs, int64_t cap,
                        int64_t *needed)
{
    return guarded(ctx, [&](Ctx &c) {
        if (!offsets || !needed) throw ApiError(DTSPH_EINVAL, "offsets and needed are required");
        if (sim < -1 || sim >= c.n_sims) throw ApiError(DTSPH_EINVAL, "sim must be -1 or a sim index");
        by_precision(c, [&](auto t) {
            using T = decltype(t);
            ensure_cells<T>(c);
            return 0;
        });
        readback_flags(c);
        const size_t N = c.N;
        std::vector<uint32_t> cnt(N);
        std::vector<int> orig(N), nb((size_t)c.cap * N);
        DTSPH_HIP_CHECK(hipMemcpy(cnt.data(), c.cnt, 4 * N, hipMemcpyDeviceToHost));
        DTSPH_HIP_CHECK(hipMemcpy(orig.data(), c.orig[c.buf], 4 * N, hipMemcpyDeviceToHost));
        DTSPH_HIP_CHECK(hipMemcpy(nb.data(), c.nbr, 4 * (size_t)c.cap * N, hipMemcpyDeviceToHost));
        std::vector<int64_t> len(N + 1, 0);
        std::vector<size_t> slot_of(N);
        for (size_t i = 0; i < N; ++i) {
            len[orig[i] + 1] = (cnt[i] & 0xffffu) + (cnt[i] >> 16);
            slot_of[orig[i]] = i;
        }
        for (size_t k = 0; k < N; ++k) len[k + 1] += len[k];
        // caller range [cb, ce) of the requested rows
        size_t cb = 0, ce = N;
        if (sim >= 0) {
            for (int s = 0; s < sim; ++s) cb += (size_t)(c.nf[s] + c.nw[s]);
            ce = cb + (size_t)(c.nf[sim] + c.nw[sim]);
        }
        const int64_t base = len[cb];
        *needed = len[ce] - base;
        for (size_t k = cb; k <= ce; ++k) offsets[k - cb] = len[k] - base;
        if (nbrs && cap >= *needed) {
            for (size_t cidx = cb; cidx < ce; ++cidx) {
                const size_t i = slot_of[cidx];
                const int n = (int)((cnt[i] & 0xffffu) + (cnt[i] >> 16));
                int32_t *row = nbrs + (len[cidx] - base);
                for (int k = 0; k < n; ++k) row[k] = orig[nb[(size_t)k * N + i]] - (int32_t)cb;
                std::sort(row, row + n);
            }
        }
        return DTSPH_OK;
    });
}

int dtsph_set_option(dtsph_ctx *ctx, int32_t option, int64_t value)
{
    return guarded(ctx, [&](Ctx &c) {
        // a static context allocates nothing: no coefficient cache, graphs or timing events
        if (c.static_mode && value != 0 &&
            (option == DTSPH_OPT_PAIR_CACHE || option == DTSPH_OPT_GRAPHS || option == DTSPH_OPT_TIMING))
            throw ApiError(DTSPH_EINVAL, "option not available in a static context (it would allocate)");
        // launch shapes, grids and lists change: recorded graphs are stale
        if (option != DTSPH_OPT_TIMING && option != DTSPH_OPT_RESET_TIMING && option != DTSPH_OPT_CHUNK)
            clear_graphs(c);
        switch (option) {
        case DTSPH_OPT_TIMING:
            if (value < -1) throw ApiError(DTSPH_EINVAL, "timing sample interval must be >= -1");
            c.timing = value != 0;
            c.timing_first = value == -1;
            c.timing_every = value > 0 ? (int)std::min<int64_t>(value, 1 << 20) : 1;
            c.timer_count[0] = c.timer_count[1] = c.timer_count[2] = c.timer_count[3] = 0;
            break;
        case DTSPH_OPT_RESET_TIMING:
            DTSPH_HIP_CHECK(hipStreamSynchronize(c.stream));
            resolve_timers(c);
            c.tstats = dtsph_timing{};
            break;
        case DTSPH_OPT_CHUNK:
            if (value < 0 || value > 1000) throw ApiError(DTSPH_EINVAL, "chunk must be in [0, 1000] (0 = adaptive)");
            c.chunk = (int)value;
            break;
        case DTSPH_OPT_BLOCK:
            if (value != 64 && value != 128 && value != 256) throw ApiError(DTSPH_EINVAL, "block must be 64, 128 or 256");
            DTSPH_HIP_CHECK(hipStreamSynchronize(c.stream));
            c.block = (int)value;
            setup_tiles(c);
            break;
        case DTSPH_OPT_XCD_REMAP:
            c.xcd_remap = value != 0;
            break;
        case DTSPH_OPT_SKIN: {
            if (value < 0) throw ApiError(DTSPH_EINVAL, "skin must be >= 0");
            for (int s = 0; s < c.n_sims; ++s) {
                SimDev &S = c.sims_h[s];
                const double kh = std::sqrt(S.kh2);
                S.skin = std::min(c.skin_default[s], 1e-3 * (double)value * S.h);
                S.cand_r2 = (kh + S.skin) * (kh + S.skin);
            }
            DTSPH_HIP_CHECK(hipStreamSynchronize(c.stream));
            DTSPH_HIP_CHECK(hipMemcpy(c.sims, c.sims_h.data(), sizeof(SimDev) * c.n_sims, hipMemcpyHostToDevice));
            c.cand_ok = c.cand_next = false;
            c.cells_valid = false;
            break;
        }
        case DTSPH_OPT_CELL_DIV:
            if (value < 1 || value > 3) throw ApiError(DTSPH_EINVAL, "cell subdivision must be 1, 2 or 3");
            DTSPH_HIP_CHECK(hipStreamSynchronize(c.stream));
            setup_keys(c, (int)value);
            DTSPH_HIP_CHECK(hipMemcpy(c.sims, c.sims_h.data(), sizeof(SimDev) * c.n_sims, hipMemcpyHostToDevice));
            c.cells_valid = false;
            c.cand_ok = c.cand_next = false;
            break;
        case DTSPH_OPT_PAIR_CACHE:
            if (value < 0 || value > 2) throw ApiError(DTSPH_EINVAL, "pair cache must be 0, 1 or 2");
            if (value != 0 && !c.coef) {
                if (c.in_loop) throw ApiError(DTSPH_EINVAL, "enable the pair cache between steps");
                const size_t f = c.precision == DTSPH_FP32 ? 4 : 8, entries = (size_t)c.cap * (size_t)c.N;
                dev_alloc(c, c.coef, 4 * f * entries);
                if (c.any_av) dev_alloc(c, c.coef_av, (c.max_dim == 2 ? 2 : 4) * f * entries);
                c.coef_valid = false;
            }
            c.pair_cache = (int)value;
            break;
        case DTSPH_OPT_SPECULATE:
            if (value != 0 && value != 1) throw ApiError(DTSPH_EINVAL, "speculate must be 0 or 1");
            c.speculate = value != 0;
            break;
        case DTSPH_OPT_GRAPHS:
            if (value != 0 && value != 1) throw ApiError(DTSPH_EINVAL, "graphs must be 0 or 1");
            clear_graphs(c);
            c.graphs = value != 0;
            break;
        case DTSPH_OPT_NBR_LANES:
            if (value != 0 && value != 1 && value != 2 && value != 4 && value != 8)
                throw ApiError(DTSPH_EINVAL, "neighbour-build lanes must be 0, 1, 2, 4 or 8");
            c.g_nbr = (int)value;
            break;
        case DTSPH_OPT_ABS32_POSITIONS: {
            if (value != 0 && value != 1) throw ApiError(DTSPH_EINVAL, "abs32 positions must be 0 or 1");
            for (int s = 0; s < c.n_sims; ++s) c.sims_h[s].abs32 = (int)value;
            DTSPH_HIP_CHECK(hipStreamSynchronize(c.stream));
            DTSPH_HIP_CHECK(hipMemcpy(c.sims, c.sims_h.data(), sizeof(SimDev) * c.n_sims, hipMemcpyHostToDevice));
            c.cells_valid = false;  // records are rewritten by the next build
            c.cand_ok = c.cand_next = false;
            break;
        }
        case DTSPH_OPT_FILTER_LANES:
            if (value != 0 && value != 1 && value != 2 && value != 4 && value != 8)
                throw ApiError(DTSPH_EINVAL, "filter lanes must be 0, 1, 2, 4 or 8");
            c.g_filter = (int)value;
            break;
        case DTSPH_OPT_TAIL_LOOP:
            if (value < 0 || value > 2) throw ApiError(DTSPH_EINVAL, "loop schedule must be 0, 1 or 2");
            c.tail_loop = (int)value;
            break;
        case DTSPH_OPT_TAIL_SPIN:
            if (value < 0) throw ApiError(DTSPH_EINVAL, "tail barrier polls must be >= 0");
            c.tail_spin = value > 0 ? value : kTailSpinDefault;
            break;
        case DTSPH_OPT_NBR_TILES:
            if (value != 0 && value != 1) throw ApiError(DTSPH_EINVAL, "neighbour tiles must be 0 or 1");
            c.nbr_tiles = c.strips ? (int)value : 0;
            break;
        case DTSPH_OPT_LANES:
            if (value != 1 && value != 2 && value != 4 && value != 8)
                throw ApiError(DTSPH_EINVAL, "lanes per particle must be 1, 2, 4 or 8");
            DTSPH_HIP_CHECK(hipStreamSynchronize(c.stream));
            c.lpp = (int)value;
            setup_tiles(c);
            break;
        default:
            throw ApiError(DTSPH_EINVAL, "unknown option " + std::to_string(option));
        }
        return DTSPH_OK;
    });
}

int dtsph_autotune(dtsph_ctx *ctx, int32_t repeats, dtsph_tune_report *out)
{
    return guarded(ctx, [&](Ctx &c) {
        if (c.in_loop) throw ApiError(DTSPH_EINVAL, "dtsph_autotune: only between steps");
        if (c.static_mode) throw ApiError(DTSPH_EINVAL, "dtsph_autotune times with HIP events: not in a static context");
        clear_graphs(c);
        const int reps = repeats > 0 ? repeats : 5;
        const bool timing = c.timing;
        c.timing = false;
        by_precision(c, [&](auto t) {
            using T = decltype(t);
            ensure_cells<T>(c);
            launch_pre_records<T>(c);
            launch_wall<T>(c, MODE_PRE);
            return 0;
        });
        hipEvent_t e0, e1;
        DTSPH_HIP_CHECK(hipEventCreate(&e0));
        DTSPH_HIP_CHECK(hipEventCreate(&e1));
        // time per launch: the best of three windows of `reps` launches (one
        // window can be stretched by other work on the device)
        auto time_us = [&](auto &&launch) {
            double best_us = 1e300;
            for (int w = 0; w < 3; ++w) {
                float ms = 0.f;
                DTSPH_HIP_CHECK(hipEventRecord(e0, c.stream));
                for (int r = 0; r < reps; ++r) launch();
                DTSPH_HIP_CHECK(hipEventRecord(e1, c.stream));
                DTSPH_HIP_CHECK(hipEventSynchronize(e1));
                DTSPH_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
                best_us = std::min(best_us, 1e3 * (double)ms / reps);
            }
            return best_us;
        };
        dtsph_tune_report rep{};
        // cell subdivision and neighbour-kernel lanes together: time full builds
        // (sort + lists; they only reorder the state) for every pair, since the
        // best lane count depends on the subdivision
        {
            double best = 1e300;
            int best_m = c.cell_div, best_g = 1, best_t = 0;
            for (int m = 1; m <= 3; ++m) {
                setup_keys(c, m);
                DTSPH_HIP_CHECK(hipMemcpy(c.sims, c.sims_h.data(), sizeof(SimDev) * c.n_sims, hipMemcpyHostToDevice));
                // g = 0: the staged-tile kernel (where it applies), else lanes per particle
                for (int g = 0; g <= 8; g = g ? 2 * g : 1) {
                    if (g == 0 && c.n_strips == 0) continue;
                    c.nbr_tiles = g == 0 ? 1 : 0;
                    if (g > 0) c.g_nbr = g;
                    const double us = by_precision(c, [&](auto t) {
                        using T = decltype(t);
                        build_cells<T>(c);
                        return time_us([&] { build_cells<T>(c); });
                    });
                    if (us < best) { best = us; best_m = m; best_g = g; best_t = c.nbr_tiles; }
                }
            }
            // the per-particle kernel stays the fallback of a tiled context
            // (3D or small periodic grids at another subdivision)
            c.g_nbr = best_g > 0 ? best_g : 1;
            c.nbr_tiles = best_t;
            setup_keys(c, best_m);
            DTSPH_HIP_CHECK(hipMemcpy(c.sims, c.sims_h.data(), sizeof(SimDev) * c.n_sims, hipMemcpyHostToDevice));
            by_precision(c, [&](auto t) {
                using T = decltype(t);
                build_cells<T>(c);
                launch_pre_records<T>(c);
                launch_wall<T>(c, MODE_PRE);
                return 0;
            });
            c.cells_valid = true;
            c.cand_ok = c.cand_next = false;
            rep.cell_div = best_m;
            rep.build_us = best;
        }
        rep.us = 1e300;
        const int lanes[4] = {1, 2, 4, 8}, blocks[3] = {64, 128, 256};
        for (int li = 0; li < 4; ++li)
            for (int bi = 0; bi < 3; ++bi) {
                c.lpp = lanes[li];
                c.block = blocks[bi];
                setup_tiles(c);
                const double us = by_precision(c, [&](auto t) {
                    using T = decltype(t);
                    launch_pass<T>(c, MODE_PRE);  // warm-up
                    return time_us([&] { launch_pass<T>(c, MODE_PRE); });
                });
                rep.entries[rep.n_entries++] = dtsph_tune_entry{c.lpp, c.block, us};
                if (us < rep.us) {
                    rep.us = us;
                    rep.lanes = c.lpp;
                    rep.block = c.block;
                }
            }
        c.lpp = rep.lanes;
        c.block = rep.block;
        setup_tiles(c);
        // the chosen neighbour kernel alone, and the lanes per particle of the
        // filter (both rewrite lists at unchanged positions, so repeats are
        // harmless)
        rep.nbr_us = by_precision(c, [&](auto t) {
            using T = decltype(t);
            return time_us([&] { launch_nbr_lists<T>(c, false); });
        });
        {
            double best = 1e300;
            int best_g = 1;
            for (int g = 1; g <= 8; g *= 2) {
                c.g_filter = g;
                const double us = by_precision(c, [&](auto t) {
                    using T = decltype(t);
                    launch_nbr_lists<T>(c, true);
                    return time_us([&] { launch_nbr_lists<T>(c, true); });
                });
                if (us < best) { best = us; best_g = g; }
            }
            c.g_filter = best_g;
            rep.filter_us = best;
        }
        rep.nbr_lanes = c.g_nbr;
        rep.nbr_tiles = c.nbr_tiles && c.n_strips > 0 ? 1 : 0;
        rep.filter_lanes = c.g_filter;
        readback_flags(c);  // a capacity overflow in the trials surfaces here
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        c.timing = timing;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune_cache[tune_key(c)] = {c.lpp, c.block, c.g_nbr, c.g_filter, c.cell_div, c.nbr_tiles};
        }
        if (out) *out = rep;
        return DTSPH_OK;
    });
}

int dtsph_get_timing(const dtsph_ctx *ctx, dtsph_timing *out)
{
    if (!ctx || !out) return DTSPH_EINVAL;
    dtsph_ctx *m = const_cast<dtsph_ctx *>(ctx);
    return guarded(m, [&](Ctx &c) {
        DTSPH_HIP_CHECK(hipStreamSynchronize(c.stream));
        resolve_timers(c);
        *out = c.tstats;
        return DTSPH_OK;
    });
}

int dtsph_get_info(const dtsph_ctx *ctx, dtsph_info *out)
{
    if (!ctx || !out) return DTSPH_EINVAL;
    const Ctx &c = ctx->c;
    out->n = c.N;
    out->n_fluid = c.Nf;
    out->n_wall = c.Nw;
    out->n_cells = c.C;
    out->n_sims = c.n_sims;
    out->precision = c.precision;
    out->nbr_capacity = c.cap;
    out->block = c.block;
    out->lanes = c.lpp;
    out->reserved = 0;
    out->device_bytes = c.device_bytes;
    return DTSPH_OK;
}

int dtsph_workspace_bytes(const dtsph_ctx *ctx, size_t *bytes)
{
    if (!ctx || !bytes) return DTSPH_EINVAL;
    *bytes = workspace_need(ctx->c);
    return DTSPH_OK;
}

int dtsph_set_workspace(dtsph_ctx *ctx, void *dev, size_t bytes)
{
    return guarded(ctx, [&](Ctx &c) {
        if (c.static_mode) throw ApiError(DTSPH_EINVAL, "a static context keeps its arrays in the static scratch");
        char *base = (char *)dev;
        if (base == c.workspace && (base == nullptr || bytes == c.workspace_size)) return DTSPH_OK;
        if (base) {
            const size_t need = workspace_need(c);
            if ((uintptr_t)base % kWsAlign)
                throw ApiError(DTSPH_EINVAL, "workspace must be 256-byte aligned");
            if (bytes < need)
                throw ApiError(DTSPH_ENOMEM, "workspace of " + std::to_string(bytes) + " bytes is smaller than the " +
                                                 std::to_string(need) + " bytes needed");
            if (c.workspace && base < c.workspace + c.workspace_size && c.workspace < base + need)
                throw ApiError(DTSPH_EINVAL, "the new workspace overlaps the current one");
            hipPointerAttribute_t attr{};
            if (hipPointerGetAttributes(&attr, dev) != hipSuccess || attr.type != hipMemoryTypeDevice ||
                attr.device != c.device) {
                (void)hipGetLastError();
                throw ApiError(DTSPH_EINVAL, "workspace is not device memory of the context's device");
            }
        }
        relocate(c, base, bytes);
        return DTSPH_OK;
    });
}

}  // extern "C"
