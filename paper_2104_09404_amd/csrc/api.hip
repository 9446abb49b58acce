// api.hip -- the C ABI (include/mgrit.h): argument validation, kernel
// configuration choice, workspace layout and the MGRIT cycle driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mgrit.h"
#include "sweep.h"

using mgk::KernelCfg;
using mgk::SweepArgs;

// synchronisation scratch of split-line launches outside a workspace-taking
// call (device_tile_scratch); host code uses only its hipGetSymbolAddress
static __device__ __align__(256) char split_scratch[mgk::kTileScratchBytes];

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* where)
{
    return fail(MGRIT_EHIP, "%s: %s", where, hipGetErrorString(e));
}

#define HIP_TRY(expr, where)                 \
    do {                                     \
        hipError_t e_ = (expr);              \
        if (e_ != hipSuccess) return hip_fail(e_, where); \
    } while (0)

// ---------------------------------------------------------------------------
// kernel configuration: smallest compiled (cells per thread, waves) whose
// capacity 64*waves*cpt covers the line, among those that keep the WENO5 /
// SSPRK3 kernel free of register spills
// ---------------------------------------------------------------------------
const KernelCfg kCfgs[] = {
#define MGK_ENTRY(C, W) {C, W},
    MGK_CFG_LIST(MGK_ENTRY)
#undef MGK_ENTRY
};
const int kNumCfgs = (int)(sizeof(kCfgs) / sizeof(kCfgs[0]));
const int kMaxLine = 64 * 8 * 8;  // (8 cells, 8 waves): the largest spill-free WENO5 configuration

struct Override {
    int nx_lo, nx_hi;
    bool latency;
    KernelCfg cfg;
};
std::vector<Override> g_overrides;

bool batch_cfg_compiled(const KernelCfg& c)
{
#define MGK_ENTRY(C, W) \
    if (c.cpt == C && c.nw == W) return true;
    MGK_BATCH_CFG_LIST(MGK_ENTRY)
#undef MGK_ENTRY
    return false;
}

bool cfg_compiled(int cpt, int nw)
{
    for (int i = 0; i < kNumCfgs; ++i)
        if (kCfgs[i].cpt == cpt && kCfgs[i].nw == nw) return true;
    return false;
}

// Lines per launch below which a launch counts as latency bound (it cannot
// fill the 256 compute units with one workgroup per line).
const int kLatencyLines = 256;

// systems (flux 2: shallow water, 3: Euler): D components per cell, one cell
// per thread; lines of at most kMaxSysLine cells on one workgroup, longer ones
// split (choose_sys_tiled)
const int kMaxSysLine = 512;
int ncomp(const mgrit_scheme* s) { return s->flux == 2 ? 2 : (s->flux == 3 ? 3 : 1); }
bool is_system(const mgrit_scheme* s) { return s->flux >= 2; }
// doubles per time node of the scheme's arrays
int64_t line_len(const mgrit_scheme* s) { return (int64_t)ncomp(s) * s->nx; }

bool choose_cfg_default(int nx, int nlines, KernelCfg* out);

bool choose_cfg(int nx, int nlines, KernelCfg* out)
{
    const bool latency = nlines < kLatencyLines;
    for (const Override& o : g_overrides)
        if (nx >= o.nx_lo && nx <= o.nx_hi && latency == o.latency && o.cfg.cpt * o.cfg.nw * 64 >= nx) {
            *out = o.cfg;
            return true;
        }
    return choose_cfg_default(nx, nlines, out);
}

// the measured preference tables, without overrides
bool choose_cfg_default(int nx, int nlines, KernelCfg* out)
{
    const bool latency = nlines < kLatencyLines;
    if (nx > kMaxLine) return false;
    if (latency) {
        // per-step latency of a single line, measured on MI355X (1024 cells:
        // 1.08 us per stage with 4 cells x 4 waves, 1.13 with 2 x 8, 1.58 with
        // 1 x 16): few cells per thread do not pay for the extra waves
        static const KernelCfg pref[] = {{1, 1}, {1, 2}, {2, 2}, {2, 4}, {4, 4}, {4, 8}, {8, 8}};
        for (const KernelCfg& c : pref)
            if (c.cpt * c.nw * 64 >= nx) {
                *out = c;
                return true;
            }
        return false;
    }
    // throughput: fill one wave first, then widen to 4 cells per thread and
    // more waves, then 8 cells per thread
    static const KernelCfg pref[] = {{1, 1}, {2, 1}, {4, 1}, {4, 2}, {4, 4}, {4, 8}, {8, 8}};
    for (const KernelCfg& c : pref)
        if (c.cpt * c.nw * 64 >= nx) {
            *out = c;
            return true;
        }
    return false;
}

// ---------------------------------------------------------------------------
// tiled lines (several workgroups per line): lines longer than one workgroup
// holds, or any range set by mgrit_set_tiled_config
// ---------------------------------------------------------------------------
const KernelCfg kTiledCfgs[] = {
#define MGK_ENTRY(C, W) {C, W},
    MGK_TILED_CFG_LIST(MGK_ENTRY)
#undef MGK_ENTRY
};

struct TiledOverride {
    int nx_lo, nx_hi;
    KernelCfg cfg;
};
std::vector<TiledOverride> g_tiled_overrides;

const KernelCfg kTiledPairCfgs[] = {
#define MGK_ENTRY(C, W) {C, W, 2},
    MGK_TILED_PAIR_CFG_LIST(MGK_ENTRY)
#undef MGK_ENTRY
};

bool tiled_compiled(int cpt, int nw, int intervals = 1)
{
    if (intervals == 2) {
        for (const KernelCfg& c : kTiledPairCfgs)
            if (c.cpt == cpt && c.nw == nw) return true;
        return false;
    }
    if (intervals != 1) return false;
    for (const KernelCfg& c : kTiledCfgs)
        if (c.cpt == cpt && c.nw == nw) return true;
    return false;
}

// fewest tiles of configuration c that hold a line of nx cells (balanced in
// whole threads, mgk::tiles_fit)
int tiles_for(int nx, const KernelCfg& c)
{
    const int T = 64 * c.nw * c.cpt;
    int G = (nx + T - 1) / T;
    while (G < nx && !mgk::tiles_fit(nx, G, c.cpt, c.nw)) ++G;
    return G;
}

// Configuration and number of tiles for lines of nx cells, or false when a
// line of nx cells runs in one workgroup.  Default: tiles of whole threads;
// lines of at least kWideTileLine cells that 16 divides take 8192-cell tiles
// of 16 cells per thread and 8 waves (2 waves per SIMD, 254 VGPRs): twice the
// work per tile between two exchanges, measured 13.4 against 16.3 ms for the
// level-0 sweep of the 65536-cell problem.  Otherwise 4 cells per thread (up
// to 4096 cells) when 4 divides nx, else 2 cells per thread (up to 2048
// cells, 16 waves) when nx is even; odd lines take 2048-cell tiles of 4 cells
// per thread and 8 waves, whose ragged variant the compiler holds free of
// register spills.
// Longest split line: 2^20 cells (128 tiles of 8192 cells, or 256 of 4096);
// lines of 2 cells per thread up to 2^19 cells (256 tiles of 2048).
const int kMaxTiledLine = 1 << 20;
const int kWideTileLine = 32768;

bool choose_tiled(int nx, KernelCfg* out, int* tiles)
{
    if (nx > kMaxTiledLine) return false;
    for (const TiledOverride& o : g_tiled_overrides)
        if (nx >= o.nx_lo && nx <= o.nx_hi) {
            *out = o.cfg;
            *tiles = tiles_for(nx, o.cfg);
            return mgk::tiles_fit(nx, *tiles, o.cfg.cpt, o.cfg.nw);
        }
    if (nx <= kMaxLine) return false;
    if (nx % 16 == 0 && nx >= kWideTileLine) *out = KernelCfg{16, 8};
    else if (nx % 4 == 0) *out = KernelCfg{4, 16};
    else if (nx % 2 == 0 && nx <= kMaxTiledLine / 2) *out = KernelCfg{2, 16};
    else *out = KernelCfg{4, 8};
    *tiles = tiles_for(nx, *out);
    return true;
}

// Split-line launches of few chunks (serial stepping, the coarsest solve,
// the coarse levels of a cycle) are bound by the latency of one RK stage, not
// by throughput.  Measured on one line (WENO5 + LF + SSPRK3, per stage):
// 65536 cells take 8.07 us on 8 tiles of (16, 8), 4.98 on 16 tiles of
// (4, 16) and 3.85 on 64 tiles of 1024 cells (2 cells per thread, 8 waves);
// from 8192 to 131072 cells the 1024-cell tiles stay within 12 % of the
// fastest compiled shape.  An even line of at most kLatencyTiledLine cells
// takes them when the default shape would occupy fewer than kLatencyLines
// workgroups (chunks x tiles) and no override covers its length.  Launches
// that write residual partials keep the default shape: its tile count sizes
// the partial buffer.  Results are bitwise those of every other shape.
const int kLatencyTiledLine = 131072;

void latency_tiled(int nx, int64_t nchunks, bool resid, KernelCfg* cfg, int* tiles)
{
    if (resid || nx % 2 != 0 || nx > kLatencyTiledLine) return;
    for (const TiledOverride& o : g_tiled_overrides)
        if (nx >= o.nx_lo && nx <= o.nx_hi) return;
    if (nchunks * (int64_t)*tiles >= kLatencyLines) return;
    const KernelCfg c{2, 8};
    const int G = tiles_for(nx, c);
    if (!mgk::tiles_fit(nx, G, c.cpt, c.nw)) return;
    *cfg = c;
    *tiles = G;
}

// Synchronisation scratch of tiled launches: mgrit_cycle takes it from its
// workspace (set for the duration of the call on the calling thread); the
// other entry points use the static device array split_scratch (one per
// device, in the library's code object: nothing is allocated), whose address
// hipGetSymbolAddress gives once per device.
thread_local char* tl_tile_scratch = nullptr;
std::mutex g_tile_mutex;
std::vector<char*> g_tile_scratch;

int device_tile_scratch(char** out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    std::lock_guard<std::mutex> lock(g_tile_mutex);
    if ((int)g_tile_scratch.size() <= dev) g_tile_scratch.resize(dev + 1, nullptr);
    if (g_tile_scratch[dev] == nullptr) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(split_scratch)), "hipGetSymbolAddress of the split-line scratch");
        if (p == nullptr || ((uintptr_t)p & 255) != 0)
            return fail(MGRIT_EHIP, "split-line scratch has no 256-byte aligned device address");
        g_tile_scratch[dev] = (char*)p;
    }
    *out = g_tile_scratch[dev];
    return MGRIT_OK;
}

// Systems: lines of up to kMaxSysLine cells run on one workgroup, longer ones
// on tiles of at most kSysTile cells (one cell per thread and two spare
// threads in a workgroup of at most 512), as few tiles as hold the line, up to
// kMaxSysTiledLine cells.  mgrit_set_sys_tiles sets the tile count for a
// range of line lengths (also below kMaxSysLine).
const int kSysTile = 510;
const int kMaxSysTiledLine = 1 << 16;

struct SysTileOverride {
    int nx_lo, nx_hi, tiles;
};
std::vector<SysTileOverride> g_sys_tile_overrides;

bool sys_tiles_ok(int n, int G, int k)
{
    const int ng = (k == 3) ? 4 : 3;
    return G >= 1 && (n + G - 1) / G + 2 <= 512 && n / G >= ng;
}

// tiles and threads per workgroup for a system line of s->nx cells, or false
// when it runs on one workgroup
bool choose_sys_tiled(const mgrit_scheme* s, int* tiles, int* threads)
{
    const int n = s->nx;
    int G = 0;
    for (const SysTileOverride& o : g_sys_tile_overrides)
        if (n >= o.nx_lo && n <= o.nx_hi) {
            if (sys_tiles_ok(n, o.tiles, s->k)) G = o.tiles;
            break;
        }
    if (G == 0) {
        if (n <= kMaxSysLine || n > kMaxSysTiledLine) return false;
        G = (n + kSysTile - 1) / kSysTile;
        if (!sys_tiles_ok(n, G, s->k)) return false;
    }
    *tiles = G;
    *threads = 64 * (((n + G - 1) / G + 2 + 63) / 64);
    return true;
}

// Adjoint configurations (no register spills): the line must be a multiple of
// the cells per thread and fit one workgroup.
const int kMaxAdjLine = 64 * 8 * 2;

bool choose_adj_cfg(int nx, KernelCfg* out)
{
    static const KernelCfg pref[] = {{1, 1}, {1, 2}, {1, 4}, {1, 8}, {2, 4}, {2, 8}};
    for (const KernelCfg& c : pref)
        if (c.cpt * c.nw * 64 >= nx && nx % c.cpt == 0) {
            *out = c;
            return true;
        }
    return false;
}

// Adjoint of split lines: a split-line setting (mgrit_set_tiled_config) whose
// pair is compiled for the adjoint applies to it too; otherwise lines that no
// single-workgroup adjoint configuration covers use tiles of at most 512
// cells, one cell per thread.
const KernelCfg kTiledAdjCfgs[] = {
#define MGK_ENTRY(C, W) {C, W},
    MGK_TADJ_CFG_LIST(MGK_ENTRY)
#undef MGK_ENTRY
};

bool tiled_adj_ok(int nx, const KernelCfg& c, int G)
{
    if (G < 1 || nx / G < 6) return false;
    if (c.cpt > 1 && (nx % G != 0 || (nx / G) % c.cpt != 0)) return false;
    return (nx + G - 1) / G <= 64 * c.nw * c.cpt;
}

bool choose_tiled_adj(int nx, KernelCfg* out, int* tiles)
{
    if (nx > kMaxTiledLine) return false;
    for (const TiledOverride& o : g_tiled_overrides)
        if (nx >= o.nx_lo && nx <= o.nx_hi) {
            for (const KernelCfg& c : kTiledAdjCfgs)
                if (c.cpt == o.cfg.cpt && c.nw == o.cfg.nw) {
                    const int G = tiles_for(nx, c);
                    if (!tiled_adj_ok(nx, c, G)) return false;
                    *out = c;
                    *tiles = G;
                    return true;
                }
            break;
        }
    KernelCfg single;
    if (choose_adj_cfg(nx, &single)) return false;
    const KernelCfg c{1, 8};
    const int G = tiles_for(nx, c);
    if (!tiled_adj_ok(nx, c, G)) return false;
    *out = c;
    *tiles = G;
    return true;
}

// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------
int check_scheme(const mgrit_scheme* s)
{
    if (s == nullptr) return fail(MGRIT_EINVAL, "scheme is NULL");
    if (s->flux < 0 || s->flux > 3)
        return fail(MGRIT_EINVAL, "flux must be 0 (Burgers), 1 (advection), 2 (shallow water) or 3 (Euler), got %d",
                    s->flux);
    if (s->k < 0 || s->k > 3) return fail(MGRIT_EINVAL, "k must be 0, 1, 2 or 3, got %d", s->k);
    if (s->stepper < 1 || s->stepper > 3) return fail(MGRIT_EINVAL, "stepper must be 1, 2 or 3, got %d", s->stepper);
    if (s->nx < 8) return fail(MGRIT_EINVAL, "nx must be >= 8, got %d", s->nx);
    if (!(s->L > 0.0) || !std::isfinite(s->L)) return fail(MGRIT_EINVAL, "L must be positive and finite");
    if (s->k > 0 && (!(s->eps > 0.0) || !std::isfinite(s->eps))) return fail(MGRIT_EINVAL, "eps must be positive");
    if (s->flux == 1 && !std::isfinite(s->a)) return fail(MGRIT_EINVAL, "advection speed must be finite");
    if (!(s->alpha_fixed >= 0.0) || !std::isfinite(s->alpha_fixed)) return fail(MGRIT_EINVAL, "alpha_fixed must be >= 0");
    if (s->lf_dx_dt != 0 && s->lf_dx_dt != 1) return fail(MGRIT_EINVAL, "lf_dx_dt must be 0 or 1");
    if (s->numflux != 0 && s->numflux != 1) return fail(MGRIT_EINVAL, "numflux must be 0 (LF) or 1 (Roe), got %d", s->numflux);
    if (s->numflux == 1 && (s->alpha_fixed > 0.0 || s->lf_dx_dt != 0))
        return fail(MGRIT_EINVAL, "alpha_fixed and lf_dx_dt apply to the Lax-Friedrichs flux only");
    if (is_system(s)) {
        if (s->flux == 2 && !(s->a > 0.0 && std::isfinite(s->a)))
            return fail(MGRIT_EINVAL, "shallow water: a is the gravitational constant and must be positive");
        if (s->flux == 3 && !(s->a > 1.0 && std::isfinite(s->a)))
            return fail(MGRIT_EINVAL, "Euler: a is the ratio of specific heats and must exceed 1");
        int G = 0, threads = 0;
        if (s->nx > kMaxSysLine && !choose_sys_tiled(s, &G, &threads))
            return fail(MGRIT_EUNSUPPORTED, "systems run on lines of at most %d cells, nx = %d", kMaxSysTiledLine,
                        s->nx);
        return MGRIT_OK;
    }
    KernelCfg c;
    int tiles = 0;
    const bool split = choose_tiled(s->nx, &c, &tiles);
    if (!split && !choose_cfg(s->nx, kLatencyLines, &c))
        return fail(MGRIT_EUNSUPPORTED, "no kernel configuration for nx = %d", s->nx);
    return MGRIT_OK;
}

// the discrete adjoint covers the LF flux with k = 0 or 2
int check_adjoint_scheme(const mgrit_scheme* s)
{
    if (is_system(s)) return fail(MGRIT_EUNSUPPORTED, "the adjoint covers scalar conservation laws only");
    if ((s->k != 0 && s->k != 2) || s->numflux != 0)
        return fail(MGRIT_EUNSUPPORTED, "the adjoint covers the Lax-Friedrichs flux with k = 0 or 2 (k = %d, numflux = %d)",
                    s->k, s->numflux);
    return MGRIT_OK;
}

int check_dt(double dt)
{
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(MGRIT_EINVAL, "dt must be positive and finite");
    return MGRIT_OK;
}

mgk::PhiConst phi_const(const mgrit_scheme* s, double dt = 0.0)
{
    mgk::PhiConst pc;
    if (s->flux == 0) {
        pc.fa = 0.5;
        pc.fb = 0.0;
    } else {
        pc.fa = 0.0;
        pc.fb = s->a;
    }
    pc.half_inv_dx = 0.5 / (s->L / (double)s->nx);
    pc.eps = s->eps;
    pc.alpha_fixed = s->alpha_fixed;
    if (s->lf_dx_dt && dt > 0.0) pc.alpha_fixed = (s->L / (double)s->nx) / dt;
    pc.roe = s->numflux;
    pc.pad_ = 0;
    return pc;
}

SweepArgs base_args(const mgrit_scheme* s)
{
    SweepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.nx = (int)line_len(s);
    a.ncomp = ncomp(s);
    a.pc = phi_const(s);
    return a;
}

// ---------------------------------------------------------------------------
// profiling
// ---------------------------------------------------------------------------
struct PendingEvent {
    int kc;
    hipEvent_t e0, e1;
    double phi_lines, cells;
};
bool g_prof = false;
uint32_t g_prof_mask = 0xffffffffu;  // kernel classes whose launches are bracketed by events
mgrit_profile_entry g_prof_acc[MGRIT_KC_COUNT];
std::vector<PendingEvent> g_pending;

// Profiling of one launch: every class counts launches, Phi lines and cell
// steps; only the classes in g_prof_mask are bracketed by HIP events (the
// events themselves cost stream time, so a timing run can keep them to the
// kernel it measures).
// Set for the duration of an allocation-free call on the calling thread:
// launches are then counted without events (creating one may allocate).
thread_local bool tl_no_alloc = false;

struct ProfLaunch {
    PendingEvent pe;
    bool timed = false;
    int begin(int kc, double phi_lines, double cells, hipStream_t st)
    {
        if (!g_prof) return MGRIT_OK;
        pe.kc = kc;
        pe.phi_lines = phi_lines;
        pe.cells = cells;
        timed = !tl_no_alloc && ((g_prof_mask >> kc) & 1u) != 0;
        if (!timed) return MGRIT_OK;
        HIP_TRY(hipEventCreate(&pe.e0), "hipEventCreate");
        HIP_TRY(hipEventCreate(&pe.e1), "hipEventCreate");
        HIP_TRY(hipEventRecord(pe.e0, st), "hipEventRecord");
        return MGRIT_OK;
    }
    int end(hipStream_t st)
    {
        if (!g_prof) return MGRIT_OK;
        if (timed) {
            HIP_TRY(hipEventRecord(pe.e1, st), "hipEventRecord");
            g_pending.push_back(pe);
        } else {
            mgrit_profile_entry& acc = g_prof_acc[pe.kc];
            acc.launches += 1;
            acc.phi_lines += pe.phi_lines;
            acc.cell_steps += pe.cells;
        }
        return MGRIT_OK;
    }
};

// A batch records the sweeps of one cycle per problem instead of launching them
struct Recorded {
    int kc;
    SweepArgs a;
    double phi_lines;
};
thread_local std::vector<Recorded>* tl_recorder = nullptr;

// the scheme of eq fineLF: the LF coefficient of every step is dx/dt
void lf_dx_dt_args(SweepArgs& a, const mgrit_scheme* s)
{
    if (!s->lf_dx_dt) return;
    const double dx = s->L / (double)s->nx;
    a.pc.alpha_fixed = dx / a.dt;
    if (a.dt_next > 0.0) a.alpha_next = dx / a.dt_next;
}

int launch(int kc, const SweepArgs& a_in, const mgrit_scheme* s, hipStream_t st, double phi_lines)
{
    SweepArgs a0 = a_in;
    lf_dx_dt_args(a0, s);
    if (tl_recorder != nullptr) {
        tl_recorder->push_back(Recorded{kc, a0, phi_lines});
        return MGRIT_OK;
    }
    KernelCfg cfg;
    int tiles = 0;
    SweepArgs a = a0;
    if (is_system(s)) {
        int threads = ((s->nx + 63) / 64) * 64;
        const bool split = choose_sys_tiled(s, &tiles, &threads);
        if (split) {
            if (a0.coarse_split || a0.gc_sub != nullptr)
                return fail(MGRIT_EUNSUPPORTED, "a scheme per level does not run on split lines");
            char* scratch = tl_tile_scratch;
            if (scratch == nullptr) {
                int rc = device_tile_scratch(&scratch);
                if (rc) return rc;
            }
            a.tiles = tiles;
            a.tile_sync = (unsigned long long*)scratch;
            a.tile_pub = (double*)(scratch + mgk::tile_sync_bytes());
        }
        ProfLaunch pl;
        int rc = pl.begin(kc, phi_lines, phi_lines * (double)s->nx, st);
        if (rc) return rc;
        hipError_t e = split ? mgk::launch_sys_tiled(a, threads, s->flux, s->k, s->stepper, st)
                             : mgk::launch_sys(a, threads, s->flux, s->k, s->stepper, st);
        if (e != hipSuccess) return hip_fail(e, split ? "split-line system sweep kernel launch" : "system sweep kernel launch");
        return pl.end(st);
    }
    const bool tiled = choose_tiled(s->nx, &cfg, &tiles);
    if (tiled) latency_tiled(s->nx, a.nchunks, a.resid_partial != nullptr, &cfg, &tiles);
    if (tiled && (a0.coarse_split || a0.gc_sub != nullptr))
        return fail(MGRIT_EUNSUPPORTED, "a scheme per level does not run on split lines");
    if (tiled) {
        char* scratch = tl_tile_scratch;
        if (scratch == nullptr) {
            int rc = device_tile_scratch(&scratch);
            if (rc) return rc;
        }
        a.tiles = tiles;
        a.tile_sync = (unsigned long long*)scratch;
        a.tile_pub = (double*)(scratch + mgk::tile_sync_bytes());
    } else if (!choose_cfg(s->nx, a.nchunks, &cfg)) {
        return fail(MGRIT_EUNSUPPORTED, "no kernel configuration for nx = %d", s->nx);
    }
    ProfLaunch pl;
    int rc = pl.begin(kc, phi_lines, phi_lines * (double)s->nx, st);
    if (rc) return rc;
    hipError_t e = tiled ? mgk::launch_tiled(a, cfg, s->k, s->stepper, st)
                         : mgk::launch_sweep(a, cfg, s->k, s->stepper, st);
    if (e != hipSuccess) return hip_fail(e, tiled ? "tiled sweep kernel launch" : "sweep kernel launch");
    return pl.end(st);
}

int launch_adj(int kc, const mgk::AdjArgs& a, const mgrit_scheme* s, int store_mode, hipStream_t st, double cells)
{
    KernelCfg cfg;
    if (!choose_adj_cfg(s->nx, &cfg))
        return fail(MGRIT_EUNSUPPORTED, "adjoint: nx = %d is not supported (at most %d cells, even above 512)", s->nx,
                    kMaxAdjLine);
    ProfLaunch pl;
    int rc = pl.begin(kc, cells / (double)s->nx, cells, st);
    if (rc) return rc;
    hipError_t e = mgk::launch_adjoint(a, cfg, s->k, s->stepper, store_mode, st);
    if (e != hipSuccess) return hip_fail(e, "adjoint kernel launch");
    return pl.end(st);
}

// Two ints of pinned host memory per calling thread, allocated on the thread's
// first mgrit_cycle and kept until the process ends: the stop flag and the
// residual count are read back through it without a per-call allocation.
int* pinned_flags()
{
    thread_local int* buf = nullptr;
    if (!buf && hipHostMalloc((void**)&buf, sizeof(int) * 2, hipHostMallocDefault) != hipSuccess) buf = nullptr;
    return buf;
}

template <class F>
int launch_aux(F&& f, hipStream_t st)
{
    ProfLaunch pl;
    int rc = pl.begin(MGRIT_KC_AUX, 0.0, 0.0, st);
    if (rc) return rc;
    hipError_t e = f();
    if (e != hipSuccess) return hip_fail(e, "auxiliary kernel launch");
    return pl.end(st);
}

int drain_profile()
{
    for (PendingEvent& pe : g_pending) {
        HIP_TRY(hipEventSynchronize(pe.e1), "hipEventSynchronize");
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, pe.e0, pe.e1), "hipEventElapsedTime");
        mgrit_profile_entry& acc = g_prof_acc[pe.kc];
        acc.launches += 1;
        acc.ms += ms;
        acc.phi_lines += pe.phi_lines;
        acc.cell_steps += pe.cells;
        (void)hipEventDestroy(pe.e0);
        (void)hipEventDestroy(pe.e1);
    }
    g_pending.clear();
    return MGRIT_OK;
}

// ---------------------------------------------------------------------------
// workspace layout of mgrit_cycle
// ---------------------------------------------------------------------------
struct Layout {
    int L;
    int N[16];          // steps per level
    size_t u_off[16];   // level arrays, l >= 1 (bytes)
    size_t g_off[16];
    size_t side_off, partial_off, hist_off, ints_off, tile_off, total;
    int tiles;          // workgroups per line (1: one workgroup per line)
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int check_params(const mgrit_scheme* s, const mgrit_params* p)
{
    if (p == nullptr) return fail(MGRIT_EINVAL, "params is NULL");
    if (p->nt < 1) return fail(MGRIT_EINVAL, "nt must be >= 1");
    if (p->levels < 1 || p->levels > 16) return fail(MGRIT_EINVAL, "levels must be in 1..16");
    if (p->levels > 1 && p->m < 2) return fail(MGRIT_EINVAL, "m must be >= 2");
    if (p->relax != 0 && p->relax != 1) return fail(MGRIT_EINVAL, "relax must be 0 (F) or 1 (FCF)");
    if (p->cycle != 0 && p->cycle != 1) return fail(MGRIT_EINVAL, "cycle must be 0 (V) or 1 (F)");
    if (p->max_iter < 0) return fail(MGRIT_EINVAL, "max_iter must be >= 0");
    if (p->init != 0 && p->init != 1) return fail(MGRIT_EINVAL, "init must be 0 or 1");
    if (p->coarse_guess != 0 && p->coarse_guess != 1) return fail(MGRIT_EINVAL, "coarse_guess must be 0 or 1");
    if (p->storage != 0 && p->storage != 1) return fail(MGRIT_EINVAL, "storage must be 0 or 1");
    if (p->levels == 1 && p->storage != 0) return fail(MGRIT_EINVAL, "levels == 1 needs storage 0");
    if (p->sync_every < 1) return fail(MGRIT_EINVAL, "sync_every must be >= 1");
    if (p->coarse_integrator < 0 || p->coarse_integrator > 2)
        return fail(MGRIT_EINVAL, "coarse_integrator must be 0, 1 or 2");
    if (p->coarse_integrator != 0) {
        if (s->k != 0 || s->stepper != 1 || s->lf_dx_dt != 1 || is_system(s))
            return fail(MGRIT_EINVAL, "fine-integrator matching needs the scheme of eq fineLF (k = 0, stepper 1, lf_dx_dt 1)");
    }
    if (!(p->tol == p->tol)) return fail(MGRIT_EINVAL, "tol is NaN");
    int rc = check_dt(p->dt);
    if (rc) return rc;
    long long div = 1;
    for (int l = 1; l < p->levels; ++l) {
        div *= p->m;
        if (div > p->nt) return fail(MGRIT_EINVAL, "m^(levels-1) exceeds nt");
    }
    if (p->nt % div != 0) return fail(MGRIT_EINVAL, "nt = %d is not divisible by m^(levels-1) = %lld", p->nt, div);
    return MGRIT_OK;
}

Layout make_layout(const mgrit_scheme* s, const mgrit_params* p)
{
    Layout ly;
    std::memset(&ly, 0, sizeof(ly));
    ly.L = p->levels;
    const size_t line = sizeof(double) * (size_t)line_len(s);
    int N = p->nt;
    size_t off = 0;
    for (int l = 0; l < ly.L; ++l) {
        ly.N[l] = N;
        if (l >= 1) {
            ly.u_off[l] = off;
            off = align256(off + line * (size_t)(N + 1));
            ly.g_off[l] = off;
            off = align256(off + line * (size_t)(N + 1));
        }
        if (l + 1 < ly.L) N /= p->m;
    }
    const int nch0 = (ly.L > 1) ? p->nt / p->m : 1;
    KernelCfg tc;
    int tiles = 0;
    int threads = 0;
    if (is_system(s)) ly.tiles = choose_sys_tiled(s, &tiles, &threads) ? tiles : 1;
    else ly.tiles = choose_tiled(s->nx, &tc, &tiles) ? tiles : 1;
    ly.side_off = off;
    off = align256(off + line * (size_t)(nch0 + 1));
    ly.partial_off = off;
    off = align256(off + sizeof(double) * (size_t)nch0 * (size_t)ly.tiles);
    ly.hist_off = off;
    off = align256(off + sizeof(double) * (size_t)(p->max_iter + 2));
    ly.ints_off = off;
    off = align256(off + 4 * sizeof(int));
    ly.tile_off = off;
    if (ly.tiles > 1) off = align256(off + mgk::tile_scratch_bytes());
    ly.total = off;
    return ly;
}

// ---------------------------------------------------------------------------
// the cycle driver
// ---------------------------------------------------------------------------
// two schemes that compute the same Phi
bool same_scheme(const mgrit_scheme* a, const mgrit_scheme* b)
{
    return a == b || (a->flux == b->flux && a->k == b->k && a->stepper == b->stepper && a->nx == b->nx &&
                      a->a == b->a && a->eps == b->eps && a->L == b->L && a->alpha_fixed == b->alpha_fixed &&
                      a->lf_dx_dt == b->lf_dx_dt && a->numflux == b->numflux);
}

struct Cycle {
    const mgrit_scheme* s;        // level 0
    const mgrit_scheme* sl[16];   // the scheme of level l (sl[l] == s unless a scheme per level is given)
    const mgrit_params* p;
    Layout ly;
    char* ws;
    double* u0_level;     // level-0 array (caller's u)
    int64_t cstride0;     // lines between level-0 C-points in u
    bool fstore0;
    const int* flag;
    double dtl[16];
    hipStream_t st;

    // fine-integrator matching: matched fine steps M of level l (0: Phi_l)
    int psiM(int l)
    {
        if (l < 1 || p->coarse_integrator == 0) return 0;
        int M = 1;
        for (int j = 0; j < l; ++j) M *= p->m;
        return M;
    }
    void psi_args(SweepArgs& a, int l)
    {
        a.psi_order = p->coarse_integrator;
        a.psi_M = psiM(l);
        a.psi_M_next = psiM(l + 1);
        a.dt_fine = p->dt;
    }

    double* U(int l) { return l == 0 ? u0_level : (double*)(ws + ly.u_off[l]); }
    double* G(int l) { return l == 0 ? nullptr : (double*)(ws + ly.g_off[l]); }
    double* side() { return (double*)(ws + ly.side_off); }
    double* partial() { return (double*)(ws + ly.partial_off); }
    int64_t cstride(int l) { return l == 0 ? cstride0 : p->m; }
    double* fout(int l) { return (l == 0 && !fstore0) ? nullptr : U(l); }
    int kc(int l, int base0, int basec) { return l == 0 ? base0 : basec; }
    const mgrit_scheme* S(int l) { return sl[l]; }
    // the FAS restriction from level l applies Phi_{l+1} inside the level-l
    // kernel when both levels have the same scheme; otherwise a second launch
    // with the level-(l+1) scheme subtracts it
    bool fused_restrict(int l) { return same_scheme(sl[l], sl[l + 1]); }

    // F + C-step into the side buffer (first half of FCF); residual at level 0
    int sweep_fc(int l, bool resid)
    {
        SweepArgs a = base_args(S(l));
        psi_args(a, l);
        a.nchunks = ly.N[l] / p->m;
        a.m = p->m;
        a.nsteps = p->m - 1;
        a.end_mode = mgk::END_CSTEP;
        a.dt = dtl[l];
        a.ustart = U(l);
        a.ustart_stride = cstride(l);
        a.fout = fout(l);
        a.g = G(l);
        a.side_out = side();
        a.cref = U(l);
        a.cref_stride = cstride(l);
        a.resid_partial = resid ? partial() : nullptr;
        a.flag = flag;
        return launch(kc(l, MGRIT_KC_RELAX_FC, MGRIT_KC_RELAX_FC_C), a, S(l), st, (double)a.nchunks * p->m);
    }

    // F-relaxation (from the side buffer after a C-relaxation) + FAS restriction to level l+1
    int sweep_fr(int l, bool from_side, bool resid)
    {
        SweepArgs a = base_args(S(l));
        psi_args(a, l);
        a.nchunks = ly.N[l] / p->m;
        a.m = p->m;
        a.nsteps = p->m - 1;
        a.end_mode = mgk::END_RESTRICT;
        a.coarse_injection = p->coarse_guess;
        a.dt = dtl[l];
        a.dt_next = dtl[l + 1];
        a.ustart = U(l);
        a.ustart_stride = cstride(l);
        a.cref = U(l);
        a.cref_stride = cstride(l);
        if (from_side) {
            // after the C-relaxation the C-points live in the side buffer; commit them
            a.side_in = side();
            a.ucommit = U(l);
            a.ucommit_stride = cstride(l);
            a.inject_last = 1;
            a.cref = side();
            a.cref_stride = 1;
        }
        a.fout = fout(l);
        a.g = G(l);
        a.uc_out = U(l + 1);
        a.gc_out = G(l + 1);
        a.resid_partial = resid ? partial() : nullptr;
        a.flag = flag;
        const bool fused = fused_restrict(l);
        a.coarse_split = fused ? 0 : 1;
        int rc = launch(kc(l, MGRIT_KC_RELAX_FR, MGRIT_KC_RELAX_FR_C), a, S(l), st, (double)a.nchunks * (p->m + 1));
        if (rc || fused) return rc;
        // g_c^{i+1} -= Phi_{l+1}(u_l^{mi}) with the level-(l+1) scheme; the chunk
        // starts are the committed C-points of level l
        SweepArgs b = base_args(S(l + 1));
        b.nchunks = ly.N[l] / p->m;
        b.m = p->m;
        b.nsteps = 0;
        b.end_mode = mgk::END_PHI;
        b.dt = dtl[l + 1];
        b.ustart = U(l);
        b.ustart_stride = cstride(l);
        b.gc_sub = G(l + 1);
        b.flag = flag;
        return launch(MGRIT_KC_RELAX_FR_C, b, S(l + 1), st, (double)b.nchunks);
    }

    // ideal interpolation: inject level l+1 into the C-points of level l, then F-relax
    int interp(int l, bool relax_f)
    {
        SweepArgs a = base_args(S(l));
        psi_args(a, l);
        a.nchunks = ly.N[l] / p->m;
        a.m = p->m;
        a.nsteps = relax_f ? p->m - 1 : 0;
        a.end_mode = mgk::END_NONE;
        a.inject_last = 1;
        a.dt = dtl[l];
        a.ustart = U(l + 1);
        a.ustart_stride = 1;
        a.ucommit = U(l);
        a.ucommit_stride = cstride(l);
        a.fout = relax_f ? fout(l) : nullptr;
        a.g = G(l);
        a.flag = flag;
        return launch(MGRIT_KC_INTERP, a, S(l), st, (double)a.nchunks * a.nsteps);
    }

    // serial solve on level l: v^0 = g^0, v^n = Phi(v^{n-1}) + g^n
    int coarse(int l)
    {
        SweepArgs a = base_args(S(l));
        psi_args(a, l);
        a.nchunks = 1;
        a.m = 0;
        a.nsteps = ly.N[l];
        a.end_mode = mgk::END_NONE;
        a.dt = dtl[l];
        a.ustart = G(l);
        a.ustart_stride = 0;
        a.ucommit = U(l);
        a.ucommit_stride = 0;
        a.fout = U(l);
        a.g = G(l);
        a.flag = flag;
        return launch(MGRIT_KC_COARSE, a, S(l), st, (double)ly.N[l]);
    }

    int relax(int l)  // F or FCF on level l >= 1, then restriction
    {
        int rc;
        if (p->relax == 1) {
            if ((rc = sweep_fc(l, false))) return rc;
            return sweep_fr(l, true, false);
        }
        return sweep_fr(l, false, false);
    }

    int vcycle(int l)
    {
        int rc;
        if (l == ly.L - 1) return coarse(l);
        if ((rc = relax(l))) return rc;
        if ((rc = vcycle(l + 1))) return rc;
        return interp(l, true);
    }

    int fcycle(int l)
    {
        int rc;
        if (l == ly.L - 1) return coarse(l);
        if ((rc = relax(l))) return rc;
        if ((rc = fcycle(l + 1))) return rc;
        if ((rc = interp(l, true))) return rc;
        if (l > 0) return vcycle(l);
        return MGRIT_OK;
    }
};

}  // namespace

// ===========================================================================
// exported C ABI
// ===========================================================================
// ---------------------------------------------------------------------------
// allocation-free cycle: the workspace is a static device array; host code
// uses only the per-device address that hipGetSymbolAddress returns for it
// (the array's name on the host is a stand-in, not a device address)
// ---------------------------------------------------------------------------
static __device__ __align__(256) char scratch[MGRIT_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mutex;
char* g_noalloc_ptr[kMaxDevices] = {};

// address of `scratch` on the current device, looked up once per device
int noalloc_scratch(char** out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(MGRIT_EUNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_noalloc_mutex);
    if (g_noalloc_ptr[dev] == nullptr) {
        void* ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress of the allocation-free workspace");
        if (ptr == nullptr || ((uintptr_t)ptr & 255) != 0)
            return fail(MGRIT_EHIP, "allocation-free workspace has no 256-byte aligned device address");
        g_noalloc_ptr[dev] = (char*)ptr;
    }
    *out = g_noalloc_ptr[dev];
    return MGRIT_OK;
}

}  // namespace

extern "C" {

const char* mgrit_last_error(void) { return g_err.c_str(); }

void mgrit_set_profiling(int on)
{
    g_prof = on != 0;
    std::memset(g_prof_acc, 0, sizeof(g_prof_acc));
    for (PendingEvent& pe : g_pending) {
        (void)hipEventDestroy(pe.e0);
        (void)hipEventDestroy(pe.e1);
    }
    g_pending.clear();
}

void mgrit_set_profiling_mask(uint32_t classes) { g_prof_mask = classes; }

int mgrit_get_profile(mgrit_profile_entry* out, int cap)
{
    int rc = drain_profile();
    if (rc) return rc;
    const int n = cap < MGRIT_KC_COUNT ? cap : MGRIT_KC_COUNT;
    for (int i = 0; i < n; ++i) out[i] = g_prof_acc[i];
    return MGRIT_KC_COUNT;
}

int mgrit_kernel_config(int32_t nx, int32_t nlines, int32_t* cells_per_thread, int32_t* waves)
{
    KernelCfg c;
    if (!choose_cfg(nx, nlines, &c)) return fail(MGRIT_EUNSUPPORTED, "no kernel configuration for nx = %d", nx);
    if (cells_per_thread) *cells_per_thread = c.cpt;
    if (waves) *waves = c.nw;
    return MGRIT_OK;
}

size_t mgrit_autotune_scratch_bytes(int32_t nx, int32_t nlines)
{
    if (nx < 8 || nlines < 1) return 0;
    return align256(sizeof(double) * (size_t)nx * (size_t)nlines);
}

int mgrit_autotune(const mgrit_scheme* s, int32_t nlines, int32_t nsteps, void* scratch, size_t scratch_bytes,
                   int32_t install, int32_t* cells_per_thread, int32_t* waves, float* ms_best, void* stream)
{
    int rc = check_scheme(s);
    if (rc) return rc;
    if (is_system(s)) return fail(MGRIT_EUNSUPPORTED, "systems run one cell per thread: nothing to tune");
    if (nlines < 1 || nsteps < 1) return fail(MGRIT_EINVAL, "nlines and nsteps must be >= 1");
    if (scratch == nullptr || scratch_bytes < mgrit_autotune_scratch_bytes(s->nx, nlines))
        return fail(MGRIT_EINVAL, "scratch must hold nlines x nx doubles");
    hipStream_t st = (hipStream_t)stream;
    double* lines = (double*)scratch;
    HIP_TRY(mgk::launch_fill_wave(lines, s->nx, nlines, st), "fill kernel launch");
    // CFL 0.5 for the data's speed 0.75 (Burgers) or |a| (advection)
    const double dx = s->L / (double)s->nx;
    const double speed = (s->flux == 0) ? 0.75 : (std::fabs(s->a) > 0.0 ? std::fabs(s->a) : 1.0);
    const double dt = 0.5 * dx / speed;
    SweepArgs a = base_args(s);
    a.nchunks = nlines;
    a.m = 0;
    a.nsteps = nsteps;
    a.end_mode = mgk::END_NONE;
    a.dt = dt;
    a.ustart = lines;
    a.ustart_stride = 1;  // nothing is stored: the lines stay as filled
    a.pc = phi_const(s, dt);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
    HIP_TRY(hipEventCreate(&e1), "hipEventCreate");
    float best = -1.f;
    KernelCfg best_cfg{0, 0};
    for (int i = 0; i < kNumCfgs && rc == MGRIT_OK; ++i) {
        const KernelCfg c = kCfgs[i];
        const int cap = 64 * c.cpt * c.nw;
        if (cap < s->nx || cap > 4 * (s->nx > 64 ? s->nx : 64)) continue;  // covers the line, not mostly idle
        float t[3];
        for (int r = 0; r < 4 && rc == MGRIT_OK; ++r) {  // one warm-up, three timed
            hipError_t e = hipEventRecord(e0, st);
            if (e == hipSuccess) e = mgk::launch_sweep(a, c, s->k, s->stepper, st);
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) rc = hip_fail(e, "autotune launch");
            else if (r > 0) t[r - 1] = ms;
        }
        if (rc) break;
        std::sort(t, t + 3);
        if (best < 0.f || t[1] < best) {
            best = t[1];
            best_cfg = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (best < 0.f) return fail(MGRIT_EUNSUPPORTED, "no one-workgroup configuration covers nx = %d", s->nx);
    if (install) {
        const bool latency = nlines < kLatencyLines;
        g_overrides.insert(g_overrides.begin(), Override{s->nx, s->nx, latency, best_cfg});
    }
    if (cells_per_thread) *cells_per_thread = best_cfg.cpt;
    if (waves) *waves = best_cfg.nw;
    if (ms_best) *ms_best = best;
    return MGRIT_OK;
}

int mgrit_autotune_tiled(const mgrit_scheme* s, int32_t nlines, int32_t nsteps, void* scratch, size_t scratch_bytes,
                         int32_t install, int32_t* cells_per_thread, int32_t* waves, int32_t* intervals,
                         float* ms_best, void* stream)
{
    int rc = check_scheme(s);
    if (rc) return rc;
    if (is_system(s)) return fail(MGRIT_EUNSUPPORTED, "systems do not run on split lines");
    if (nlines < 1 || nsteps < 1) return fail(MGRIT_EINVAL, "nlines and nsteps must be >= 1");
    if (scratch == nullptr || scratch_bytes < mgrit_autotune_scratch_bytes(s->nx, nlines))
        return fail(MGRIT_EINVAL, "scratch must hold nlines x nx doubles");
    char* tscratch = nullptr;
    if ((rc = device_tile_scratch(&tscratch))) return rc;
    hipStream_t st = (hipStream_t)stream;
    double* lines = (double*)scratch;
    HIP_TRY(mgk::launch_fill_wave(lines, s->nx, nlines, st), "fill kernel launch");
    const double dx = s->L / (double)s->nx;
    const double speed = (s->flux == 0) ? 0.75 : (std::fabs(s->a) > 0.0 ? std::fabs(s->a) : 1.0);
    const double dt = 0.5 * dx / speed;
    SweepArgs a = base_args(s);
    a.nchunks = nlines;
    a.m = 0;
    a.nsteps = nsteps;
    a.end_mode = mgk::END_NONE;
    a.dt = dt;
    a.ustart = lines;
    a.ustart_stride = 1;  // nothing is stored: the lines stay as filled
    a.pc = phi_const(s, dt);
    a.tile_sync = (unsigned long long*)tscratch;
    a.tile_pub = (double*)(tscratch + mgk::tile_sync_bytes());
    std::vector<KernelCfg> cands(std::begin(kTiledCfgs), std::end(kTiledCfgs));
    cands.insert(cands.end(), std::begin(kTiledPairCfgs), std::end(kTiledPairCfgs));
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
    HIP_TRY(hipEventCreate(&e1), "hipEventCreate");
    float best = -1.f;
    KernelCfg best_cfg{0, 0};
    for (const KernelCfg& c : cands) {
        const int G = tiles_for(s->nx, c);
        if (!mgk::tiles_fit(s->nx, G, c.cpt, c.nw) || G > 256) continue;
        a.tiles = G;
        float t[3] = {0.f, 0.f, 0.f};
        bool fits = true;
        for (int r = 0; r < 4 && rc == MGRIT_OK && fits; ++r) {  // one warm-up, three timed
            hipError_t e = hipEventRecord(e0, st);
            if (e == hipSuccess) e = mgk::launch_tiled(a, c, s->k, s->stepper, st);
            if (e == hipErrorCooperativeLaunchTooLarge) {  // the tiles of a line cannot be resident at once
                fits = false;
                break;
            }
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) rc = hip_fail(e, "autotune launch");
            else if (r > 0) t[r - 1] = ms;
        }
        if (rc) break;
        if (!fits) continue;
        std::sort(t, t + 3);
        if (best < 0.f || t[1] < best) {
            best = t[1];
            best_cfg = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    unsigned long long w = 0;
    HIP_TRY(hipMemcpy(&w, tscratch, sizeof(w), hipMemcpyDeviceToHost), "hipMemcpy");
    if (w != 0) return fail(MGRIT_EHIP, "split-line autotune: workgroups of a line failed to synchronise");
    if (best < 0.f) return fail(MGRIT_EUNSUPPORTED, "no split-line configuration holds nx = %d", s->nx);
    if (install)
        g_tiled_overrides.insert(g_tiled_overrides.begin(), TiledOverride{s->nx, s->nx, best_cfg});
    if (cells_per_thread) *cells_per_thread = best_cfg.cpt;
    if (waves) *waves = best_cfg.nw;
    if (intervals) *intervals = best_cfg.intervals;
    if (ms_best) *ms_best = best;
    return MGRIT_OK;
}

int mgrit_tiled_config(int32_t nx, int32_t* cells_per_thread, int32_t* waves, int32_t* tiles)
{
    KernelCfg c{0, 0};
    int G = 1;
    if (!choose_tiled(nx, &c, &G)) {
        c = KernelCfg{0, 0};
        G = 1;
    }
    if (cells_per_thread) *cells_per_thread = c.cpt;
    if (waves) *waves = c.nw;
    if (tiles) *tiles = G;
    return MGRIT_OK;
}

int mgrit_tiled_launch_config(int32_t nx, int64_t nchunks, int32_t residual, int32_t* cells_per_thread,
                              int32_t* waves, int32_t* tiles)
{
    if (nchunks < 0) return fail(MGRIT_EINVAL, "nchunks must be >= 0");
    KernelCfg c{0, 0};
    int G = 1;
    if (choose_tiled(nx, &c, &G)) {
        latency_tiled(nx, nchunks, residual != 0, &c, &G);
    } else {
        c = KernelCfg{0, 0};
        G = 1;
    }
    if (cells_per_thread) *cells_per_thread = c.cpt;
    if (waves) *waves = c.nw;
    if (tiles) *tiles = G;
    return MGRIT_OK;
}

int mgrit_tiled_intervals(int32_t nx, int32_t* intervals)
{
    KernelCfg c{0, 0};
    int G = 1;
    if (intervals) *intervals = choose_tiled(nx, &c, &G) ? c.intervals : 1;
    return MGRIT_OK;
}

int mgrit_set_tiled_intervals(int32_t nx_lo, int32_t nx_hi, int32_t cpt, int32_t waves, int32_t intervals)
{
    if (intervals != 1 && intervals != 2) return fail(MGRIT_EINVAL, "intervals per workgroup must be 1 or 2");
    if (nx_lo > nx_hi || nx_lo < 8) return fail(MGRIT_EINVAL, "empty range or nx_lo < 8");
    if (!tiled_compiled(cpt, waves, intervals))
        return fail(MGRIT_EINVAL, "split-line configuration (%d, %d) with %d interval(s) per workgroup is not compiled",
                    cpt, waves, intervals);
    g_tiled_overrides.insert(g_tiled_overrides.begin(), TiledOverride{nx_lo, nx_hi, KernelCfg{cpt, waves, intervals}});
    return MGRIT_OK;
}

int mgrit_set_tiled_config(int32_t nx_lo, int32_t nx_hi, int32_t cpt, int32_t waves)
{
    if (cpt == 0) {
        g_tiled_overrides.clear();
        return MGRIT_OK;
    }
    if (!tiled_compiled(cpt, waves)) return fail(MGRIT_EINVAL, "tiled configuration (%d, %d) is not compiled", cpt, waves);
    if (nx_lo > nx_hi || nx_lo < 8) return fail(MGRIT_EINVAL, "empty range or nx_lo < 8");
    g_tiled_overrides.insert(g_tiled_overrides.begin(), TiledOverride{nx_lo, nx_hi, KernelCfg{cpt, waves}});
    return MGRIT_OK;
}

int mgrit_set_sys_tiles(int32_t nx_lo, int32_t nx_hi, int32_t tiles)
{
    if (tiles == 0) {
        g_sys_tile_overrides.clear();
        return MGRIT_OK;
    }
    if (tiles < 1) return fail(MGRIT_EINVAL, "tiles must be >= 1 (0 clears)");
    if (nx_lo > nx_hi || nx_lo < 8) return fail(MGRIT_EINVAL, "empty range or nx_lo < 8");
    if ((nx_hi + tiles - 1) / tiles + 2 > 512 || nx_lo / tiles < 4)
        return fail(MGRIT_EINVAL, "%d tiles do not split lines of %d..%d cells into 4..510 cells each", tiles, nx_lo,
                    nx_hi);
    g_sys_tile_overrides.insert(g_sys_tile_overrides.begin(), SysTileOverride{nx_lo, nx_hi, tiles});
    return MGRIT_OK;
}

int mgrit_sys_tiles(const mgrit_scheme* s, int32_t* tiles)
{
    int rc = check_scheme(s);
    if (rc) return rc;
    if (!is_system(s)) return fail(MGRIT_EINVAL, "not a system (flux 2 or 3)");
    int G = 1, threads = 0;
    if (!choose_sys_tiled(s, &G, &threads)) G = 1;
    if (tiles) *tiles = G;
    return MGRIT_OK;
}

int mgrit_set_kernel_config(int32_t nx_lo, int32_t nx_hi, int32_t latency, int32_t cpt, int32_t waves)
{
    if (cpt == 0) {
        g_overrides.clear();
        return MGRIT_OK;
    }
    if (!cfg_compiled(cpt, waves)) return fail(MGRIT_EINVAL, "configuration (%d, %d) is not compiled", cpt, waves);
    if (nx_lo > nx_hi) return fail(MGRIT_EINVAL, "empty range");
    if (cpt * waves * 64 < nx_hi) return fail(MGRIT_EINVAL, "configuration (%d, %d) does not cover nx = %d", cpt, waves, nx_hi);
    g_overrides.insert(g_overrides.begin(), Override{nx_lo, nx_hi, latency != 0, KernelCfg{cpt, waves}});
    return MGRIT_OK;
}

int mgrit_phi(const mgrit_scheme* s, double dt, const double* u_in, double* u_out, int64_t nlines, void* stream)
{
    int rc = check_scheme(s);
    if (rc) return rc;
    if ((rc = check_dt(dt))) return rc;
    if (nlines < 0 || nlines > 2147483647LL) return fail(MGRIT_EINVAL, "nlines out of range");
    if (nlines == 0) return MGRIT_OK;
    if (u_in == nullptr || u_out == nullptr) return fail(MGRIT_EINVAL, "NULL array");
    SweepArgs a = base_args(s);
    a.nchunks = (int)nlines;
    a.nsteps = 0;
    a.end_mode = mgk::END_PHI;
    a.dt = dt;
    a.ustart = u_in;
    a.ustart_stride = 1;
    a.side_out = u_out;
    return launch(MGRIT_KC_PHI, a, s, (hipStream_t)stream, (double)nlines);
}

int mgrit_serial(const mgrit_scheme* s, double dt, int32_t nt, const double* u0, double* traj, void* stream)
{
    int rc = check_scheme(s);
    if (rc) return rc;
    if ((rc = check_dt(dt))) return rc;
    if (nt < 0) return fail(MGRIT_EINVAL, "nt must be >= 0");
    if (u0 == nullptr || traj == nullptr) return fail(MGRIT_EINVAL, "NULL array");
    SweepArgs a = base_args(s);
    a.nchunks = 1;
    a.nsteps = nt;
    a.end_mode = mgk::END_NONE;
    a.dt = dt;
    a.ustart = u0;
    a.ucommit = traj;
    a.fout = traj;
    return launch(MGRIT_KC_PHI, a, s, (hipStream_t)stream, (double)nt);
}

int mgrit_relax(const mgrit_scheme* s, double dt, int32_t m, int32_t kind, double* u, const double* g, int32_t n,
                void* stream)
{
    int rc = check_scheme(s);
    if (rc) return rc;
    if ((rc = check_dt(dt))) return rc;
    if (m < 2) return fail(MGRIT_EINVAL, "m must be >= 2");
    if (n < 1 || n % m != 0) return fail(MGRIT_EINVAL, "n must be a positive multiple of m");
    if (kind < 0 || kind > 2) return fail(MGRIT_EINVAL, "kind must be 0 (F), 1 (C) or 2 (FCF)");
    if (u == nullptr) return fail(MGRIT_EINVAL, "NULL array");
    hipStream_t st = (hipStream_t)stream;
    const int nch = n / m;
    auto F = [&]() {
        SweepArgs a = base_args(s);
        a.nchunks = nch;
        a.m = m;
        a.nsteps = m - 1;
        a.end_mode = mgk::END_NONE;
        a.dt = dt;
        a.ustart = u;
        a.ustart_stride = m;
        a.fout = u;
        a.g = g;
        return launch(MGRIT_KC_RELAX_FR_C, a, s, st, (double)nch * (m - 1));
    };
    auto Cr = [&]() {
        // chunk c (c = 0..nch-1) steps from F-point cm+m-1 to C-point (c+1)m
        SweepArgs a = base_args(s);
        a.nchunks = nch;
        a.m = m;
        a.nsteps = 1;
        a.end_mode = mgk::END_NONE;
        a.dt = dt;
        a.ustart = u + (size_t)(m - 1) * line_len(s);
        a.ustart_stride = m;
        a.fout = u + (size_t)(m - 1) * line_len(s);  // node c*m + 1 relative to the shifted base = (c+1) m
        a.g = g ? g + (size_t)(m - 1) * line_len(s) : nullptr;
        return launch(MGRIT_KC_RELAX_FC_C, a, s, st, (double)nch);
    };
    if (kind == 0) return F();
    if (kind == 1) return Cr();
    if ((rc = F())) return rc;
    if ((rc = Cr())) return rc;
    return F();
}

int mgrit_residual(const mgrit_scheme* s, double dt, int32_t m, const double* u, const double* g, int32_t n,
                   int32_t coarse_guess, double* r, double* u_coarse, double* g_coarse, double* norm, void* stream)
{
    int rc = check_scheme(s);
    if (rc) return rc;
    if ((rc = check_dt(dt))) return rc;
    if (m < 2) return fail(MGRIT_EINVAL, "m must be >= 2");
    if (n < 1 || n % m != 0) return fail(MGRIT_EINVAL, "n must be a positive multiple of m");
    if (u == nullptr) return fail(MGRIT_EINVAL, "NULL array");
    if (coarse_guess != 0 && coarse_guess != 1) return fail(MGRIT_EINVAL, "coarse_guess must be 0 or 1");
    if ((u_coarse == nullptr) != (g_coarse == nullptr))
        return fail(MGRIT_EINVAL, "u_coarse and g_coarse must both be given or both be NULL");
    if (norm != nullptr && r == nullptr) return fail(MGRIT_EINVAL, "norm needs r");
    if (r == nullptr && u_coarse == nullptr) return MGRIT_OK;
    hipStream_t st = (hipStream_t)stream;
    const int nch = n / m;
    const int64_t nx = line_len(s);
    // chunk c starts at its last F-point cm+m-1 and takes the step to C-point (c+1)m
    SweepArgs a = base_args(s);
    a.nchunks = nch;
    a.m = m;
    a.nsteps = 0;
    a.dt = dt;
    a.dt_next = dt * (double)m;
    a.g = g;
    a.ustart = u + (size_t)(m - 1) * nx;
    a.ustart_stride = m;
    a.cref = u;
    a.cref_stride = m;
    a.r_out = r;
    if (u_coarse != nullptr) {
        a.end_mode = mgk::END_RESTRICT;
        a.coarse_injection = coarse_guess;
        a.uc_out = u_coarse;
        a.gc_out = g_coarse;
        a.ystart = u;  // Phi_{l+1} acts on the C-point u^{m(i-1)}
        a.ystart_stride = m;
        rc = launch(MGRIT_KC_RELAX_FR_C, a, s, st, (double)nch * 2);
    } else {
        a.end_mode = mgk::END_CSTEP;
        a.side_out = nullptr;
        rc = launch(MGRIT_KC_RELAX_FC_C, a, s, st, (double)nch);
    }
    if (rc) return rc;
    if (norm != nullptr) {
        rc = launch_aux([&] { return mgk::launch_sumsq_norm(r, (int64_t)nch * nx, norm, st); }, st);
        if (rc) return rc;
    }
    return MGRIT_OK;
}

int mgrit_phi_vjp(const mgrit_scheme* s, double dt, const double* u, const double* lam_in, double* lam_out,
                  int64_t nlines, void* stream)
{
    int rc = check_scheme(s);
    if (rc) return rc;
    if ((rc = check_adjoint_scheme(s))) return rc;
    {
        KernelCfg c;
        if (!choose_adj_cfg(s->nx, &c))
            return fail(MGRIT_EUNSUPPORTED, "mgrit_phi_vjp: nx = %d needs a split line; use mgrit_adjoint", s->nx);
    }
    if ((rc = check_dt(dt))) return rc;
    if (nlines < 0 || nlines > 2147483647LL) return fail(MGRIT_EINVAL, "nlines out of range");
    if (nlines == 0) return MGRIT_OK;
    if (u == nullptr || lam_in == nullptr || lam_out == nullptr) return fail(MGRIT_EINVAL, "NULL array");
    mgk::AdjArgs a;
    std::memset(&a, 0, sizeof(a));
    a.nx = s->nx;
    a.nlines = (int)nlines;
    a.nsteps = 1;
    a.stored = 0;
    a.dt = dt;
    a.pc = phi_const(s, dt);
    a.u = u;
    a.lam_in = lam_in;
    a.lam_out = lam_out;
    return launch_adj(MGRIT_KC_ADJOINT, a, s, 0, (hipStream_t)stream, (double)nlines * s->nx);
}

int mgrit_checkpoints(const mgrit_scheme* s, double dt, int32_t nt, int32_t every, const double* u0, double* ckpt,
                      void* stream)
{
    int rc = check_scheme(s);
    if (rc) return rc;
    if ((rc = check_dt(dt))) return rc;
    if (nt < 1 || every < 1 || nt % every != 0) return fail(MGRIT_EINVAL, "nt must be a positive multiple of every");
    if (u0 == nullptr || ckpt == nullptr) return fail(MGRIT_EINVAL, "NULL array");
    SweepArgs a = base_args(s);
    a.nchunks = 1;
    a.nsteps = nt;
    a.end_mode = mgk::END_NONE;
    a.dt = dt;
    a.ustart = u0;
    a.ucommit = ckpt;
    a.fout = ckpt;
    a.fout_every = every;
    return launch(MGRIT_KC_PHI, a, s, (hipStream_t)stream, (double)nt);
}

size_t mgrit_adjoint_workspace_bytes(const mgrit_scheme* s, int32_t nt, int32_t every, int32_t parallel_segments)
{
    if (check_scheme(s) != MGRIT_OK || check_adjoint_scheme(s) != MGRIT_OK) return 0;
    if (nt < 1 || every < 1 || nt % every != 0 || parallel_segments < 1) {
        fail(MGRIT_EINVAL, "nt must be a positive multiple of every, parallel_segments >= 1");
        return 0;
    }
    const int nseg = nt / every;
    const int P = parallel_segments < nseg ? parallel_segments : nseg;
    const size_t traj = sizeof(double) * (size_t)P * (size_t)every * (size_t)s->stepper * (size_t)s->nx;
    KernelCfg c;
    int tiles = 0;
    size_t tile = 0;
    if (choose_tiled_adj(s->nx, &c, &tiles) || choose_tiled(s->nx, &c, &tiles)) tile = align256(mgk::tile_scratch_bytes());
    return align256(traj) + align256(sizeof(double) * (size_t)s->nx) + tile;
}

int mgrit_adjoint(const mgrit_scheme* s, double dt, int32_t nt, int32_t every, int32_t parallel_segments,
                  const double* ckpt, const double* lambda_T, double* lambda_0, void* workspace, size_t ws_bytes,
                  void* stream)
{
    int rc = check_scheme(s);
    if (rc) return rc;
    if ((rc = check_adjoint_scheme(s))) return rc;
    if ((rc = check_dt(dt))) return rc;
    const size_t need = mgrit_adjoint_workspace_bytes(s, nt, every, parallel_segments);
    if (need == 0) return MGRIT_EINVAL;
    if (ckpt == nullptr || lambda_T == nullptr || lambda_0 == nullptr || workspace == nullptr)
        return fail(MGRIT_EINVAL, "NULL array");
    if (ws_bytes < need) return fail(MGRIT_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, need);
    if (((uintptr_t)workspace & 255) != 0) return fail(MGRIT_EINVAL, "workspace must be 256-byte aligned");
    KernelCfg cfg;
    int tiles = 0;
    const bool split = choose_tiled_adj(s->nx, &cfg, &tiles);
    if (!split && !choose_adj_cfg(s->nx, &cfg))
        return fail(MGRIT_EUNSUPPORTED, "adjoint: nx = %d is not supported", s->nx);
    hipStream_t st = (hipStream_t)stream;
    const int64_t nx = s->nx;
    const int nseg = nt / every;
    const int P = parallel_segments < nseg ? parallel_segments : nseg;
    const int ST = s->stepper;
    double* traj = (double*)workspace;
    const size_t traj_bytes = align256(sizeof(double) * (size_t)P * every * ST * nx);
    double* lamw = (double*)((char*)workspace + traj_bytes);
    char* tscratch = (char*)workspace + traj_bytes + align256(sizeof(double) * (size_t)nx);
    // the forward recompute of split lines (split for the forward sweep) and
    // the split reverse sweep synchronise through the workspace
    struct ScratchScope {
        explicit ScratchScope(char* p) { tl_tile_scratch = p; }
        ~ScratchScope() { tl_tile_scratch = nullptr; }
    } scope(split ? tscratch : nullptr);
    auto tile_args = [&](mgk::AdjArgs& a) {
        a.tiles = tiles;
        a.tile_sync = (unsigned long long*)tscratch;
        a.tile_pub = (double*)(tscratch + mgk::tile_sync_bytes());
    };
    auto run = [&](int kc, mgk::AdjArgs& a, int store_mode, double cells) -> int {
        if (!split) return launch_adj(kc, a, s, store_mode, st, cells);
        tile_args(a);
        ProfLaunch pl;
        int prc = pl.begin(kc, cells / (double)nx, cells, st);
        if (prc) return prc;
        hipError_t e = mgk::launch_tiled_adjoint(a, cfg, s->k, s->stepper, store_mode, st);
        if (e != hipSuccess) return hip_fail(e, "split-line adjoint kernel launch");
        return pl.end(st);
    };
    const int nbatch = (nseg + P - 1) / P;
    const double* lam_cur = lambda_T;
    int batch = 0;
    for (int hi = nseg - 1; hi >= 0; hi -= P, ++batch) {
        const int lo = hi - P + 1 > 0 ? hi - P + 1 : 0;
        const int nb = hi - lo + 1;
        // recompute the batch's segments in parallel, keeping every stage input
        mgk::AdjArgs f;
        std::memset(&f, 0, sizeof(f));
        f.nx = s->nx;
        f.nlines = nb;
        f.nsteps = every;
        f.dt = dt;
        f.pc = phi_const(s, dt);
        f.u = ckpt + (int64_t)lo * nx;
        f.u_stride = 1;
        f.traj_out = traj;
        f.traj_stride = (int64_t)every * ST * nx;
        if ((rc = run(MGRIT_KC_ADJOINT_RECOMPUTE, f, 1, (double)nb * every * nx))) return rc;
        // reverse sweep over the batch (one line, nb*every steps)
        double* out = ((nbatch - 1 - batch) % 2 == 0) ? lambda_0 : lamw;
        mgk::AdjArgs r;
        std::memset(&r, 0, sizeof(r));
        r.nx = s->nx;
        r.nlines = 1;
        r.nsteps = nb * every;
        r.stored = 1;
        r.dt = dt;
        r.pc = phi_const(s, dt);
        r.traj = traj;
        r.traj_stride = 0;
        r.lam_in = lam_cur;
        r.lam_out = out;
        if ((rc = run(MGRIT_KC_ADJOINT, r, 0, (double)nb * every * nx))) return rc;
        lam_cur = out;
    }
    if (split) {
        unsigned long long w = 0;
        HIP_TRY(hipMemcpyAsync(&w, tscratch, sizeof(w), hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
        HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
        if (w != 0) return fail(MGRIT_EHIP, "split-line adjoint: workgroups of a line failed to synchronise");
    }
    return MGRIT_OK;
}

size_t mgrit_workspace_bytes(const mgrit_scheme* s, const mgrit_params* p)
{
    if (check_scheme(s) != MGRIT_OK || check_params(s, p) != MGRIT_OK) return 0;
    return make_layout(s, p).total;
}

// the solve of mgrit_cycle and mgrit_cycle_levels (arguments validated):
// sl[l] is the scheme of level l
static int run_cycle(const mgrit_scheme* const* sl, const mgrit_params* p, const double* u0, double* u,
                     void* workspace, size_t ws_bytes, double* res_hist, int32_t* iters, void* stream)
{
    const mgrit_scheme* s = sl[0];
    int rc = MGRIT_OK;
    if (u0 == nullptr || u == nullptr || workspace == nullptr) return fail(MGRIT_EINVAL, "NULL array");
    if (res_hist == nullptr || iters == nullptr) return fail(MGRIT_EINVAL, "NULL host output");
    if (((uintptr_t)workspace & 255) != 0) return fail(MGRIT_EINVAL, "workspace must be 256-byte aligned");
    Cycle cy;
    cy.s = s;
    for (int l = 0; l < 16; ++l) cy.sl[l] = sl[l];
    cy.p = p;
    cy.ly = make_layout(s, p);
    if (ws_bytes < cy.ly.total)
        return fail(MGRIT_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, cy.ly.total);
    cy.ws = (char*)workspace;
    cy.u0_level = u;
    cy.st = (hipStream_t)stream;
    const int64_t nx = line_len(s);
    const int L = p->levels;
    cy.cstride0 = (p->storage == 0) ? (L > 1 ? p->m : 1) : 1;
    cy.fstore0 = p->storage == 0;
    double dtl = p->dt;
    for (int l = 0; l < L; ++l) {
        cy.dtl[l] = dtl;
        dtl *= (double)p->m;
    }
    int* ints = (int*)(cy.ws + cy.ly.ints_off);
    int* flag = ints;
    int* counter = ints + 1;
    double* hist = (double*)(cy.ws + cy.ly.hist_off);
    hipStream_t st = cy.st;
    // tiled launches of this call synchronise through the workspace
    struct ScratchScope {
        explicit ScratchScope(char* p) { tl_tile_scratch = p; }
        ~ScratchScope() { tl_tile_scratch = nullptr; }
    } scope(cy.ly.tiles > 1 ? cy.ws + cy.ly.tile_off : nullptr);
    // a tiled line whose workgroups failed to meet (cannot happen with the
    // cooperative launch; the kernels' spins are bounded) leaves its error word set
    auto tile_error = [&]() -> int {
        if (cy.ly.tiles <= 1) return MGRIT_OK;
        unsigned long long w = 0;
        HIP_TRY(hipMemcpy(&w, cy.ws + cy.ly.tile_off, sizeof(w), hipMemcpyDeviceToHost), "hipMemcpy");
        if (w != 0) return fail(MGRIT_EHIP, "tiled sweep: workgroups of a line failed to synchronise");
        return MGRIT_OK;
    };

    // initial iterate
    const int64_t nlines0 = (p->storage == 0) ? (int64_t)p->nt + 1 : (int64_t)(p->nt / p->m) + 1;
    if (p->init == 0) {
        if ((rc = launch_aux([&] { return mgk::launch_broadcast(u0, u, nx, nlines0, st); }, st))) return rc;
    } else {
        if ((rc = launch_aux([&] { return mgk::launch_broadcast(u0, u, nx, 1, st); }, st))) return rc;
    }
    if ((rc = launch_aux([&] { return mgk::launch_clear_ints(ints, 4, st); }, st))) return rc;

    if (L == 1) {
        // serial time stepping: the coarse solve on level 0, from g^0 = u0
        SweepArgs a = base_args(s);
        a.nchunks = 1;
        a.nsteps = p->nt;
        a.end_mode = mgk::END_NONE;
        a.dt = p->dt;
        a.ustart = u0;
        a.ucommit = u;
        a.fout = u;
        if ((rc = launch(MGRIT_KC_COARSE, a, s, st, (double)p->nt))) return rc;
        HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
        if ((rc = tile_error())) return rc;
        res_hist[0] = 0.0;
        *iters = 1;
        return MGRIT_OK;
    }

    cy.flag = flag;
    const int nch0 = p->nt / p->m;
    int host_flag = 0;
    // an allocation-free call reads the flags into stack memory (a pageable
    // copy, which the runtime stages itself)
    int stack_flags[2] = {0, 0};
    int* pinned = tl_no_alloc ? stack_flags : pinned_flags();
    if (!pinned) return fail(MGRIT_EHIP, "hipHostMalloc of the stop-flag buffer failed");
    int k = 0;
    for (;; ++k) {
        // first level-0 sweep of the next cycle: F-relaxation and the residual r_k
        if (p->relax == 1) rc = cy.sweep_fc(0, true);
        else rc = cy.sweep_fr(0, false, true);
        if (rc) break;
        rc = launch_aux([&] { return mgk::launch_reduce_norm(cy.partial(), nch0 * cy.ly.tiles, hist, counter, flag, p->tol, st); }, st);
        if (rc) break;
        if (k == p->max_iter) break;
        // rest of the cycle
        if (p->relax == 1) {
            if ((rc = cy.sweep_fr(0, true, false))) break;
        }
        if (p->cycle == 1) rc = cy.fcycle(1);
        else rc = cy.vcycle(1);
        if (rc) break;
        if ((rc = cy.interp(0, false))) break;
        if ((k + 1) % p->sync_every == 0) {
            hipError_t e = hipMemcpyAsync(pinned, flag, sizeof(int), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) {
                rc = hip_fail(e, "convergence check");
                break;
            }
            host_flag = pinned[0];
            if (host_flag) break;
        }
    }
    if (rc) {
        return rc;
    }
    hipError_t e = hipMemcpyAsync(pinned, ints, sizeof(int) * 2, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        return hip_fail(e, "final readback");
    }
    host_flag = pinned[0];
    const int nres = pinned[1];
    if (nres < 1 || nres > p->max_iter + 1) return fail(MGRIT_EHIP, "inconsistent residual counter %d", nres);
    HIP_TRY(hipMemcpy(res_hist, hist, sizeof(double) * (size_t)nres, hipMemcpyDeviceToHost), "hipMemcpy");
    if ((rc = tile_error())) return rc;
    *iters = nres - 1;
    return host_flag ? MGRIT_OK : MGRIT_NOT_CONVERGED;
}

int mgrit_cycle(const mgrit_scheme* s, const mgrit_params* p, const double* u0, double* u, void* workspace,
                size_t ws_bytes, double* res_hist, int32_t* iters, void* stream)
{
    int rc = check_scheme(s);
    if (rc) return rc;
    if ((rc = check_params(s, p))) return rc;
    const mgrit_scheme* sl[16];
    for (int l = 0; l < 16; ++l) sl[l] = s;
    return run_cycle(sl, p, u0, u, workspace, ws_bytes, res_hist, iters, stream);
}

int mgrit_cycle_noalloc(const mgrit_scheme* s, const mgrit_params* p, const double* u0, double* u,
                        double* res_hist, int32_t* iters, void* stream)
{
    int rc = check_scheme(s);
    if (rc) return rc;
    if ((rc = check_params(s, p))) return rc;
    const size_t need = make_layout(s, p).total;
    if (need > MGRIT_NOALLOC_SCRATCH_BYTES)
        return fail(MGRIT_EINVAL, "mgrit_cycle_noalloc: the problem needs %zu workspace bytes, more than the %zu of "
                                  "the static workspace; use mgrit_cycle with a caller workspace",
                    need, (size_t)MGRIT_NOALLOC_SCRATCH_BYTES);
    char* ws = nullptr;
    if ((rc = noalloc_scratch(&ws))) return rc;
    struct NoAllocScope {
        NoAllocScope() { tl_no_alloc = true; }
        ~NoAllocScope() { tl_no_alloc = false; }
    } scope;
    const mgrit_scheme* sl[16];
    for (int l = 0; l < 16; ++l) sl[l] = s;
    return run_cycle(sl, p, u0, u, ws, MGRIT_NOALLOC_SCRATCH_BYTES, res_hist, iters, stream);
}

int mgrit_cycle_levels(const mgrit_scheme* schemes, const mgrit_params* p, const double* u0, double* u,
                       void* workspace, size_t ws_bytes, double* res_hist, int32_t* iters, void* stream)
{
    if (schemes == nullptr) return fail(MGRIT_EINVAL, "schemes is NULL");
    int rc = check_scheme(&schemes[0]);
    if (rc) return rc;
    if ((rc = check_params(&schemes[0], p))) return rc;
    if (p->coarse_integrator != 0)
        return fail(MGRIT_EINVAL, "coarse_integrator replaces the coarse schemes: use mgrit_cycle");
    const mgrit_scheme* s0 = &schemes[0];
    bool mixed = false;
    for (int l = 1; l < p->levels; ++l) {
        const mgrit_scheme* sl = &schemes[l];
        if ((rc = check_scheme(sl))) return rc;
        if (sl->nx != s0->nx || sl->L != s0->L || sl->flux != s0->flux || (s0->flux >= 1 && sl->a != s0->a))
            return fail(MGRIT_EINVAL, "level %d: every level must have the same nx, L and conservation law", l);
        if (!same_scheme(&schemes[l - 1], sl)) mixed = true;
    }
    KernelCfg c;
    int tiles = 0;
    int threads = 0;
    if (mixed && (is_system(s0) ? choose_sys_tiled(s0, &tiles, &threads) : choose_tiled(s0->nx, &c, &tiles)))
        return fail(MGRIT_EUNSUPPORTED, "a scheme per level runs on lines of one workgroup");
    const mgrit_scheme* sl[16];
    for (int l = 0; l < 16; ++l) sl[l] = &schemes[l < p->levels ? l : p->levels - 1];
    return run_cycle(sl, p, u0, u, workspace, ws_bytes, res_hist, iters, stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batches of independent problems
// ---------------------------------------------------------------------------
namespace {

// longest line whose serial solve a batch runs on one workgroup

struct BatchBucket {
    KernelCfg cfg;
    int ragged;
    int roe;                 // numerical flux of every problem in the bucket
    std::vector<int> probs;  // problem indices
    std::vector<int> offset;
    int nblocks;             // workgroups (one line each), or work items of split lines
    size_t dev_off;          // offset / problem arrays in the workspace
    int tiles;               // split lines: workgroups per line (0: one workgroup per line)
    int wide;                // lines of one workgroup with several cell blocks per thread (cfg.intervals)
};

struct BatchPhase {
    int kc;
    int end_mode;
    size_t args_off;                 // count SweepArgs in the workspace
    std::vector<BatchBucket> buckets;
    std::vector<int> split;          // problems on split lines (own launches)
    double cells;                    // cell steps of the phase over the batch
};

struct BatchPlan {
    int count;
    std::vector<Layout> ly;
    std::vector<size_t> ly_off;      // per-problem workspace base
    std::vector<BatchPhase> phA, phB;
    size_t norm_off, conv_off, tile_off, tables_off, total;
    bool any_split;
    std::vector<SweepArgs> host_args;  // [phase][problem], A phases first
    std::vector<double> host_phi;      // Phi applications of each entry of host_args
    std::vector<int> host_ints;        // bucket offset / problem arrays
    std::vector<mgk::BatchNorm> host_norm;
};

mgrit_params problem_params(const mgrit_params* p, const mgrit_problem* q)
{
    mgrit_params pp = *p;
    pp.nt = q->nt;
    pp.dt = q->dt;
    return pp;
}

int check_batch(const mgrit_problem* probs, int32_t count, const mgrit_params* p)
{
    if (probs == nullptr || p == nullptr) return fail(MGRIT_EINVAL, "NULL problem table or params");
    if (count < 1) return fail(MGRIT_EINVAL, "count must be >= 1");
    if (p->levels < 2) return fail(MGRIT_EINVAL, "a batch needs levels >= 2");
    for (int i = 0; i < count; ++i) {
        const mgrit_problem& q = probs[i];
        int rc = check_scheme(&q.scheme);
        if (rc) return fail(rc, "problem %d: %s", i, mgrit_last_error());
        if (is_system(&q.scheme))
            return fail(MGRIT_EUNSUPPORTED, "problem %d: batches hold scalar conservation laws only", i);
        const mgrit_params pp = problem_params(p, &q);
        if ((rc = check_params(&q.scheme, &pp))) return fail(rc, "problem %d: %s", i, mgrit_last_error());
        if (q.scheme.k != probs[0].scheme.k || q.scheme.stepper != probs[0].scheme.stepper)
            return fail(MGRIT_EINVAL, "problem %d: every problem of a batch needs the same k and stepper", i);
    }
    return MGRIT_OK;
}

// Record the sweeps of one cycle of every problem, group them into buckets and
// lay out the workspace.  With ws == nullptr only the sizes are computed.
// tiles of the serial solves of split-line problems in a batch
const int kBatchSerialTiles = 4;

// Lines of 4097..8192 cells that are a multiple of 4, with the LF flux and
// Phi steps (no matching integrator), run the many-chunk phases of a batch on
// one workgroup per line (wide_impl.h): no per-stage exchange between
// workgroups.  Serial solves stay split (latency), and so do other lines.
const KernelCfg kBatchWideCfg{4, 8, 4};
const int kBatchWideMax = 8192;

const KernelCfg kBatchWideCfg2{2, 8, 8};  // even lines that 4 does not divide

bool batch_wide(const mgrit_scheme& s, const SweepArgs& a, bool serial, KernelCfg* c)
{
    if (serial || s.nx <= kMaxLine || s.nx > kBatchWideMax || s.numflux != 0 || s.k > 2 || a.psi_order != 0)
        return false;
    if (s.nx % kBatchWideCfg.cpt == 0) *c = kBatchWideCfg;
    else if (s.nx % kBatchWideCfg2.cpt == 0) *c = kBatchWideCfg2;
    else return false;
    return true;
}

int plan_batch(const mgrit_problem* probs, int32_t count, const mgrit_params* p, char* ws, BatchPlan* bp)
{
    bp->count = count;
    bp->ly.resize(count);
    bp->ly_off.resize(count);
    bp->any_split = false;
    size_t off = 0;
    for (int i = 0; i < count; ++i) {
        const mgrit_params pp = problem_params(p, &probs[i]);
        bp->ly[i] = make_layout(&probs[i].scheme, &pp);
        bp->ly_off[i] = off;
        off = align256(off + bp->ly[i].total);
        KernelCfg c;
        int t = 0;
        if (choose_tiled(probs[i].scheme.nx, &c, &t)) bp->any_split = true;
    }
    bp->norm_off = off;
    off = align256(off + sizeof(mgk::BatchNorm) * (size_t)count);
    bp->conv_off = off;
    off = align256(off + 256);
    bp->tile_off = off;
    if (bp->any_split) off = align256(off + mgk::tile_scratch_bytes());
    // record one cycle per problem
    std::vector<std::vector<Recorded>> recA(count), recB(count);
    for (int i = 0; i < count; ++i) {
        const mgrit_problem& q = probs[i];
        const mgrit_params pp = problem_params(p, &q);
        Cycle cy;
        cy.s = &q.scheme;
        for (int l = 0; l < 16; ++l) cy.sl[l] = &q.scheme;
        cy.p = &pp;
        cy.ly = bp->ly[i];
        cy.ws = (ws != nullptr ? ws : (char*)nullptr) + bp->ly_off[i];
        cy.u0_level = q.u;
        cy.st = nullptr;
        const int L = pp.levels;
        cy.cstride0 = (pp.storage == 0) ? pp.m : 1;
        cy.fstore0 = pp.storage == 0;
        double dtl = pp.dt;
        for (int l = 0; l < L; ++l) {
            cy.dtl[l] = dtl;
            dtl *= (double)pp.m;
        }
        cy.flag = (int*)(cy.ws + cy.ly.ints_off);
        int rc;
        tl_recorder = &recA[i];
        rc = (pp.relax == 1) ? cy.sweep_fc(0, true) : cy.sweep_fr(0, false, true);
        tl_recorder = &recB[i];
        if (!rc && pp.relax == 1) rc = cy.sweep_fr(0, true, false);
        if (!rc) rc = (pp.cycle == 1) ? cy.fcycle(1) : cy.vcycle(1);
        if (!rc) rc = cy.interp(0, false);
        tl_recorder = nullptr;
        if (rc) return rc;
        if (recA[i].size() != recA[0].size() || recB[i].size() != recB[0].size())
            return fail(MGRIT_EINVAL, "problem %d: cycle structure differs", i);
    }
    // phases and buckets
    const size_t nA = recA[0].size(), nB = recB[0].size();
    bp->host_args.assign((nA + nB) * (size_t)count, SweepArgs());
    bp->host_phi.assign((nA + nB) * (size_t)count, 0.0);
    bp->host_ints.clear();
    size_t args_off = 0;  // relative to tables_off
    auto build = [&](std::vector<std::vector<Recorded>>& rec, size_t nph, size_t base, std::vector<BatchPhase>& out) -> int {
        out.resize(nph);
        for (size_t ph = 0; ph < nph; ++ph) {
            BatchPhase& P = out[ph];
            P.kc = rec[0][ph].kc;
            P.end_mode = rec[0][ph].a.end_mode;
            P.args_off = args_off;
            args_off += sizeof(SweepArgs) * (size_t)count;
            P.cells = 0.0;
            long long total_lines = 0;
            for (int i = 0; i < count; ++i) total_lines += rec[i][ph].a.nchunks;
            for (int i = 0; i < count; ++i) {
                const Recorded& r = rec[i][ph];
                bp->host_args[(base + ph) * count + i] = r.a;
                bp->host_phi[(base + ph) * count + i] = r.phi_lines;
                P.cells += r.phi_lines * (double)probs[i].scheme.nx;
                KernelCfg c;
                int t = 0;
                const bool serial = r.a.nchunks == 1 && r.a.end_mode == mgk::END_NONE;
                int tiles = 0, wide = 0;
                if (batch_wide(probs[i].scheme, r.a, serial, &c)) {
                    wide = c.intervals;
                    // the chunk's residual partial sits in the first of the
                    // layout's per-tile slots, the others are zero
                    bp->host_args[(base + ph) * count + i].tiles = bp->ly[i].tiles;
                } else if (choose_tiled(probs[i].scheme.nx, &c, &t)) {
                    if (serial && mgk::tiles_fit(probs[i].scheme.nx, kBatchSerialTiles, 2, 16)) {
                        // serial solves (no residual partials, so any tiling) share one
                        // shape: every split-line problem's solve runs at once, each on
                        // 4 tiles, which also shortens its step
                        c = KernelCfg{2, 16};
                        t = kBatchSerialTiles;
                    }
                    if (!mgk::tiled_batch_compiled(c)) {
                        // a split shape not compiled for batches: the problem's own launches
                        P.split.push_back(i);
                        continue;
                    }
                    // every split-line problem of the phase with this shape and tile
                    // count in one persistent launch
                    tiles = t;
                } else {
                    // serial solves (one chunk per problem) take the latency configuration
                    const int nl = serial ? 1 : (int)std::min<long long>(total_lines, 1 << 30);
                    if (!choose_cfg(probs[i].scheme.nx, nl, &c))
                        return fail(MGRIT_EUNSUPPORTED, "problem %d: no kernel configuration", i);
                    // an override outside the configurations compiled for batches
                    // gives way to the measured default
                    if (!batch_cfg_compiled(c) && !choose_cfg_default(probs[i].scheme.nx, nl, &c))
                        return fail(MGRIT_EUNSUPPORTED, "problem %d: no kernel configuration", i);
                }
                const int rag = (c.cpt > 1 && probs[i].scheme.nx % c.cpt != 0) ? 1 : 0;
                const int roe = probs[i].scheme.numflux;
                BatchBucket* bk = nullptr;
                for (BatchBucket& b : P.buckets)
                    if (b.cfg.cpt == c.cpt && b.cfg.nw == c.nw && b.ragged == rag && b.roe == roe && b.tiles == tiles &&
                        b.wide == wide)
                        bk = &b;
                if (bk == nullptr) {
                    P.buckets.push_back(BatchBucket{c, rag, roe, {}, {}, 0, 0, tiles, wide});
                    bk = &P.buckets.back();
                }
                bk->offset.push_back(bk->nblocks);
                bk->probs.push_back(i);
                bk->nblocks += r.a.nchunks;
            }
            // serial solves of split lines (one work item per problem): line group
            // g runs items g, g + groups, ... one after the other, so with the
            // longest solves first the groups that run a second solve get short ones
            for (BatchBucket& b : P.buckets) {
                if (b.tiles == 0 || b.nblocks != (int)b.probs.size()) continue;
                bool serial_all = true;
                for (int i : b.probs)
                    serial_all = serial_all && rec[i][ph].a.nchunks == 1 && rec[i][ph].a.end_mode == mgk::END_NONE;
                if (serial_all)
                    std::stable_sort(b.probs.begin(), b.probs.end(),
                                     [&](int x, int y) { return rec[x][ph].a.nsteps > rec[y][ph].a.nsteps; });
            }
            for (BatchBucket& b : P.buckets) {
                b.dev_off = sizeof(int) * bp->host_ints.size();
                bp->host_ints.insert(bp->host_ints.end(), b.offset.begin(), b.offset.end());
                bp->host_ints.insert(bp->host_ints.end(), b.probs.begin(), b.probs.end());
            }
        }
        return MGRIT_OK;
    };
    int rc = build(recA, nA, 0, bp->phA);
    if (!rc) rc = build(recB, nB, nA, bp->phB);
    if (rc) return rc;
    bp->tables_off = off;
    const size_t ints_rel = align256(args_off);
    off = align256(off + ints_rel + sizeof(int) * bp->host_ints.size());
    bp->total = off;
    // fix the int-array offsets (relative to tables_off)
    for (auto* v : {&bp->phA, &bp->phB})
        for (BatchPhase& P : *v)
            for (BatchBucket& b : P.buckets) b.dev_off += ints_rel;
    // residual reduction table
    bp->host_norm.resize(count);
    for (int i = 0; i < count; ++i) {
        const Layout& l = bp->ly[i];
        char* base = (ws != nullptr ? ws : (char*)nullptr) + bp->ly_off[i];
        mgk::BatchNorm& e = bp->host_norm[i];
        e.partial = (const double*)(base + l.partial_off);
        e.n = (probs[i].nt / p->m) * l.tiles;
        e.pad_ = 0;
        e.hist = (double*)(base + l.hist_off);
        e.counter = (int*)(base + l.ints_off) + 1;
        e.flag = (int*)(base + l.ints_off);
    }
    return MGRIT_OK;
}

}  // namespace

extern "C" {

size_t mgrit_batched_workspace_bytes(const mgrit_problem* probs, int32_t count, const mgrit_params* p)
{
    if (check_batch(probs, count, p) != MGRIT_OK) return 0;
    BatchPlan bp;
    if (plan_batch(probs, count, p, nullptr, &bp) != MGRIT_OK) return 0;
    return bp.total;
}

int mgrit_cycle_batched(const mgrit_problem* probs, int32_t count, const mgrit_params* p, void* workspace,
                        size_t ws_bytes, double* res_hist, int32_t* iters, int32_t* status, void* stream)
{
    int rc = check_batch(probs, count, p);
    if (rc) return rc;
    if (workspace == nullptr || res_hist == nullptr || iters == nullptr || status == nullptr)
        return fail(MGRIT_EINVAL, "NULL workspace or host output");
    if (((uintptr_t)workspace & 255) != 0) return fail(MGRIT_EINVAL, "workspace must be 256-byte aligned");
    for (int i = 0; i < count; ++i)
        if (probs[i].u0 == nullptr || probs[i].u == nullptr) return fail(MGRIT_EINVAL, "problem %d: NULL array", i);
    char* ws = (char*)workspace;
    BatchPlan bp;
    if ((rc = plan_batch(probs, count, p, ws, &bp))) return rc;
    if (ws_bytes < bp.total) return fail(MGRIT_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, bp.total);
    hipStream_t st = (hipStream_t)stream;
    struct ScratchScope {
        explicit ScratchScope(char* q) { tl_tile_scratch = q; }
        ~ScratchScope() { tl_tile_scratch = nullptr; }
    } scope(bp.any_split ? ws + bp.tile_off : nullptr);

    // tables
    char* tables = ws + bp.tables_off;
    HIP_TRY(hipMemcpyAsync(tables, bp.host_args.data(), sizeof(SweepArgs) * bp.host_args.size(),
                           hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    const size_t args_bytes = sizeof(SweepArgs) * bp.host_args.size();
    if (!bp.host_ints.empty()) {
        HIP_TRY(hipMemcpyAsync(tables + align256(args_bytes), bp.host_ints.data(), sizeof(int) * bp.host_ints.size(),
                               hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    }
    HIP_TRY(hipMemcpyAsync(ws + bp.norm_off, bp.host_norm.data(), sizeof(mgk::BatchNorm) * (size_t)count,
                           hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    int* converged = (int*)(ws + bp.conv_off);
    if ((rc = launch_aux([&] { return mgk::launch_clear_ints(converged, 1, st); }, st))) return rc;
    // initial iterates
    for (int i = 0; i < count; ++i) {
        const mgrit_problem& q = probs[i];
        const int64_t nl0 = (p->storage == 0) ? (int64_t)q.nt + 1 : (int64_t)(q.nt / p->m) + 1;
        int* ints = (int*)(ws + bp.ly_off[i] + bp.ly[i].ints_off);
        if ((rc = launch_aux([&] { return mgk::launch_broadcast(q.u0, q.u, q.scheme.nx, p->init == 0 ? nl0 : 1, st); },
                             st)))
            return rc;
        if ((rc = launch_aux([&] { return mgk::launch_clear_ints(ints, 4, st); }, st))) return rc;
    }
    // HIP's host-to-device copies above come from pageable memory: finish them
    // before the host vectors go out of scope
    HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");

    const int k0 = probs[0].scheme.k, st0 = probs[0].scheme.stepper;
    auto run_phases = [&](const std::vector<BatchPhase>& phases, size_t base_index) -> int {
        for (size_t ph = 0; ph < phases.size(); ++ph) {
            const BatchPhase& P = phases[ph];
            const SweepArgs* dargs = (const SweepArgs*)(tables + P.args_off);
            for (const BatchBucket& b : P.buckets) {
                mgk::BatchLaunch t;
                t.args = dargs;
                t.offset = (const int*)(tables + b.dev_off);
                t.problem = t.offset + b.offset.size();
                t.nprob = (int)b.probs.size();
                t.nblocks = b.nblocks;
                t.end_mode = P.end_mode;
                t.ragged = b.ragged;
                t.roe = b.roe;
                t.pad_ = 0;
                double phi_lines = 0.0, cells = 0.0;
                if (g_prof) {
                    for (int i : b.probs) {
                        const double phi = bp.host_phi[(base_index + ph) * count + i];
                        phi_lines += phi;
                        cells += phi * (double)probs[i].scheme.nx;
                    }
                }
                t.tiles = b.tiles > 0 ? b.tiles : 1;
                t.tile_sync = nullptr;
                t.tile_pub = nullptr;
                t.groups = 0;
                if (b.tiles > 0) {
                    char* scratch = ws + bp.tile_off;
                    t.tile_sync = (unsigned long long*)scratch;
                    t.tile_pub = (double*)(scratch + mgk::tile_sync_bytes());
                }
                ProfLaunch pl;
                int prc = pl.begin(P.kc, phi_lines, cells, st);
                if (prc) return prc;
                hipError_t e = (b.tiles > 0) ? mgk::launch_tiled_batch(t, b.cfg, k0, st0, st)
                               : (b.wide > 0) ? mgk::launch_wide_batch(t, b.cfg, k0, st0, st)
                                              : mgk::launch_batch(t, b.cfg, k0, st0, st);
                if (e != hipSuccess)
                    return hip_fail(e, b.tiles > 0 ? "batched split-line launch"
                                       : b.wide > 0 ? "batched wide-line launch" : "batched sweep kernel launch");
                if ((prc = pl.end(st))) return prc;
            }
            for (int i : P.split) {
                const SweepArgs& a = bp.host_args[(base_index + ph) * count + i];
                int r = launch(P.kc, a, &probs[i].scheme, st, bp.host_phi[(base_index + ph) * count + i]);
                if (r) return r;
            }
        }
        return MGRIT_OK;
    };
    int* pinned = pinned_flags();
    if (!pinned) return fail(MGRIT_EHIP, "hipHostMalloc of the stop-flag buffer failed");
    const mgk::BatchNorm* dnorm = (const mgk::BatchNorm*)(ws + bp.norm_off);
    for (int k = 0;; ++k) {
        if ((rc = run_phases(bp.phA, 0))) return rc;
        if ((rc = launch_aux([&] { return mgk::launch_reduce_norm_batch(dnorm, count, p->tol, converged, st); }, st)))
            return rc;
        if (k == p->max_iter) break;
        if ((rc = run_phases(bp.phB, bp.phA.size()))) return rc;
        if ((k + 1) % p->sync_every == 0) {
            HIP_TRY(hipMemcpyAsync(pinned, converged, sizeof(int), hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
            HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
            if (pinned[0] >= count) break;
        }
    }
    HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
    if (bp.any_split) {
        unsigned long long w = 0;
        HIP_TRY(hipMemcpy(&w, ws + bp.tile_off, sizeof(w), hipMemcpyDeviceToHost), "hipMemcpy");
        if (w != 0) return fail(MGRIT_EHIP, "tiled sweep: workgroups of a line failed to synchronise");
    }
    const int H = p->max_iter + 1;
    for (int i = 0; i < count; ++i) {
        int ints[2];
        HIP_TRY(hipMemcpy(ints, bp.host_norm[i].flag, sizeof(int) * 2, hipMemcpyDeviceToHost), "hipMemcpy");
        const int nres = ints[1];
        if (nres < 1 || nres > H) return fail(MGRIT_EHIP, "problem %d: inconsistent residual counter %d", i, nres);
        for (int j = 0; j < H; ++j) res_hist[(size_t)i * H + j] = 0.0;
        HIP_TRY(hipMemcpy(res_hist + (size_t)i * H, bp.host_norm[i].hist, sizeof(double) * (size_t)nres,
                          hipMemcpyDeviceToHost), "hipMemcpy");
        iters[i] = nres - 1;
        status[i] = ints[0] ? MGRIT_OK : MGRIT_NOT_CONVERGED;
    }
    return MGRIT_OK;
}

}  // extern "C"
