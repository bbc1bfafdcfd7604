// fk_api.hip -- C ABI of libfk.so: argument validation, host-side planning
// (cost-ordered node tables, level constants, launch shape) and the launch
// sequence of the Monte-Carlo interface solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "fk.h"
#include "fk_accum.hpp"
#include "fk_internal.hpp"

namespace fk {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what) { return fail(FK_E_DEVICE, "%s: %s", what, hipGetErrorString(e)); }

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

int64_t step_count(double t, double dt) {
    if (t <= 0.0) return 0;
    return (int64_t)std::ceil(t / dt - 1e-9);
}

static bool kind_supported(int32_t kind) {
    return kind == FK_DENSITY_CONST || kind == FK_DENSITY_BUMP || kind == FK_DENSITY_MOVING_BUMP ||
           kind == FK_DENSITY_TWO_BUMPS || kind == FK_DENSITY_RING || kind == FK_DENSITY_RIDGE ||
           kind == FK_DENSITY_GRID;
}

int validate_density(const fk_density *w) {
    if (!w) return fail(FK_E_INVAL, "density is NULL");
    if (!kind_supported(w->kind)) return fail(FK_E_INVAL, "unknown density kind %d", w->kind);
    if (w->time_mode != FK_TIME_BACKWARD && w->time_mode != FK_TIME_FROZEN)
        return fail(FK_E_INVAL, "unknown time mode %d", w->time_mode);
    const double v[] = {w->amp, w->width2, w->cx, w->cy, w->orbit_r, w->omega, w->t_freeze};
    for (double x : v)
        if (!std::isfinite(x)) return fail(FK_E_INVAL, "density parameter is not finite");
    if (w->kind == FK_DENSITY_GRID) {
        if (w->grid_n < 2 || w->grid_n > 65535) return fail(FK_E_INVAL, "grid density needs 2 <= grid_n <= 65535");
        if (!w->grid_w || !w->grid_b) return fail(FK_E_INVAL, "grid density needs grid_w and grid_b");
        if (((uintptr_t)w->grid_b & 7u) != 0) return fail(FK_E_INVAL, "grid_b must be 8-byte aligned");
    } else if (w->kind == FK_DENSITY_RING) {
        if (!(w->amp >= 0.0)) return fail(FK_E_INVAL, "ring amplitude (alpha) must be >= 0");
        if (!(w->width2 <= 0.0)) return fail(FK_E_INVAL, "ring exponent (beta) must be <= 0");
    } else if (w->kind != FK_DENSITY_CONST) {
        if (!(w->width2 > 0.0)) return fail(FK_E_INVAL, "density width2 must be > 0");
        if (!(w->amp > -1.0)) return fail(FK_E_INVAL, "density amplitude must be > -1 (w > 0)");
    }
    return FK_OK;
}

int validate_data(const fk_data *d) {
    if (!d) return fail(FK_E_INVAL, "data is NULL");
    if (d->init_kind < 0 || d->init_kind > FK_DATA_GRID) return fail(FK_E_INVAL, "unknown init kind %d", d->init_kind);
    if (d->bdry_kind < 0 || d->bdry_kind > FK_DATA_GRID)
        return fail(FK_E_INVAL, "unknown boundary kind %d", d->bdry_kind);
    if (d->score_mode != FK_SCORE_UNCLAMPED && d->score_mode != FK_SCORE_PROJECT && d->score_mode != FK_SCORE_EXTEND &&
        d->score_mode != FK_SCORE_BRIDGE && d->score_mode != FK_SCORE_EXPONENTIAL)
        return fail(FK_E_INVAL, "unknown score mode %d", d->score_mode);
    if (d->bdry_kind == FK_DATA_GRID &&
        (d->init_kind != FK_DATA_GRID || (d->score_mode != FK_SCORE_PROJECT && d->score_mode != FK_SCORE_BRIDGE &&
                                          d->score_mode != FK_SCORE_EXPONENTIAL)))
        return fail(FK_E_INVAL, "grid boundary data needs grid initial data and a projecting score mode");
    if (d->score_mode == FK_SCORE_EXTEND && d->init_kind != FK_DATA_GRID)
        return fail(FK_E_INVAL, "score mode EXTEND needs grid initial data");
    if (!std::isfinite(d->t_init)) return fail(FK_E_INVAL, "t_init is not finite");
    if (d->init_kind == FK_DATA_GRID) {
        if (d->grid_n < 1 || !d->grid_xi || !d->grid_eta)
            return fail(FK_E_INVAL, "grid initial data needs grid_n >= 1 and both grids");
    }
    return FK_OK;
}

int validate_common(int64_t n_paths, double dt) {
    if (n_paths < 2 || n_paths > 0x7fffffff) return fail(FK_E_INVAL, "n_paths must be in [2, 2^31)");
    if (!std::isfinite(dt) || !(dt > 0.0)) return fail(FK_E_INVAL, "dt must be finite and > 0");
    return FK_OK;
}

int validate_horizon(double t, double t_init, double dt, uint32_t level_id) {
    if (!std::isfinite(t) || t < 0.0) return fail(FK_E_INVAL, "t must be finite and >= 0");
    if (!std::isfinite(t_init)) return fail(FK_E_INVAL, "t_init is not finite");
    if (level_id >= (1u << 28)) return fail(FK_E_INVAL, "level_id must be < 2^28");
    if (step_count(t, dt) > 0x7ffffffe) return fail(FK_E_INVAL, "t/dt too large");
    return FK_OK;
}

int validate_device_points(const double *pts, int64_t n) {
    if (n < 0) return fail(FK_E_INVAL, "negative node count");
    if (n > 0 && !pts) return fail(FK_E_INVAL, "pts is NULL");
    if (n > 0xffffffffLL) return fail(FK_E_INVAL, "too many nodes");
    if (((uintptr_t)pts & 7u) != 0) return fail(FK_E_INVAL, "pts must be 8-byte aligned");
    return FK_OK;
}

int validate_points(const double *pts, int64_t n) {
    if (n < 0) return fail(FK_E_INVAL, "negative node count");
    if (n > 0 && !pts) return fail(FK_E_INVAL, "pts is NULL");
    for (int64_t i = 0; i < n; ++i) {
        const double x = pts[2 * i], y = pts[2 * i + 1];
        if (!(x >= 0.0 && x <= 1.0 && y >= 0.0 && y <= 1.0))
            return fail(FK_E_INVAL, "node %lld (%g, %g) is not in the closed unit square", (long long)i, x, y);
    }
    return FK_OK;
}

int resolve_plan(const fk_plan *plan, fk_plan *out) {
    fk_plan pl{256, 0, 128, 1};
    if (plan) {
        if (plan->block) pl.block = plan->block;
        if (plan->blocks_per_cu) pl.blocks_per_cu = plan->blocks_per_cu;
        if (plan->chunk) pl.chunk = plan->chunk;
        if (plan->node_tile) pl.node_tile = plan->node_tile;
    }
    if (pl.node_tile < 1 || pl.node_tile > 256 || (pl.node_tile & (pl.node_tile - 1)))
        return fail(FK_E_INVAL, "plan node_tile must be a power of two in [1, 256]");
    if (pl.block < 64 || pl.block > 256 || pl.block % 64)
        return fail(FK_E_INVAL, "plan block must be 64, 128, 192 or 256");
    if (pl.chunk < 1 || pl.chunk > (int)kMaxChunk) return fail(FK_E_INVAL, "plan chunk must be in [1, %u]", kMaxChunk);
    if (pl.blocks_per_cu < 0 || pl.blocks_per_cu > 64) return fail(FK_E_INVAL, "plan blocks_per_cu out of range");
    *out = pl;
    return FK_OK;
}

// Level constants in the FP32 form the path kernel uses.
LevelDev make_level(const fk_density *w, double t_init, double t, double dt, uint32_t level_id, uint32_t stream) {
    LevelDev L{};
    const int64_t K = step_count(t, dt);
    const double dl = K > 0 ? t - (double)(K - 1) * dt : dt;
    const double ln2 = 0.69314718055994530942;
    const double log2e = 1.44269504088896340736;
    const double orev = w->omega / (2.0 * 3.14159265358979323846);
    L.tend = (float)(t_init + t);
    L.horizon = (float)t;
    L.dt = (float)dt;
    L.dt_last = (float)dl;
    L.cbm = (float)(-4.0 * ln2 * dt);
    L.cbm_last = (float)(-4.0 * ln2 * dl);
    L.K = (int32_t)K;
    L.ctr3 = (level_id << 4) | (stream & 15u);
    L.amp = (float)w->amp;
    if (w->kind == FK_DENSITY_RING) {
        L.nscale = (float)(w->width2 * log2e);
        L.a2s = (float)(2.0 * w->amp * w->width2);
    } else {
        L.nscale = w->kind == FK_DENSITY_CONST ? 0.f : (float)(-log2e / w->width2);
        L.a2s = w->kind == FK_DENSITY_CONST ? 0.f : (float)(2.0 * w->amp / w->width2);
    }
    L.cx = (float)w->cx;
    L.cy = (float)w->cy;
    L.orbit_r = (float)w->orbit_r;
    L.omega_rev = (float)orev;
    L.t_freeze = (float)w->t_freeze;
    L.rev0 = (float)((t_init + t) * orev);
    L.drev = (float)(dt * orev);
    L.cos_d = (float)std::cos(dt * w->omega);
    L.sin_d = (float)std::sin(dt * w->omega);
    if (w->kind == FK_DENSITY_GRID) {
        L.gb = (const float2 *)w->grid_b;
        L.gn = w->grid_n;
        L.fn = (float)w->grid_n;
        L.nscale = L.a2s = 0.f;
    }
    return L;
}

// Expected relative cost of a node: a proxy of its mean exit time, capped by
// the horizon.  Only the order matters.
double node_cost(double x, double y, double t) {
    const double ax = x * (1.0 - x), ay = y * (1.0 - y);
    if (ax <= 0.0 || ay <= 0.0) return 0.0;
    const double tau = 1.0 / (2.0 / ax + 2.0 / ay);
    return std::min(t, tau);
}

int build_tables(const LevelSpec *lv, int n_levels, const double *pts, int64_t n_total, const fk_data *d, double dt,
                 Tables &T) {
    T.levels.resize((size_t)n_levels);
    T.nodes.resize((size_t)n_total);
    T.outs.resize((size_t)n_total);
    T.shift = (d->init_kind == FK_DATA_IDENTITY && d->bdry_kind == FK_DATA_IDENTITY);
    T.kind = lv[0].w.kind;
    T.time_mode = lv[0].w.time_mode;
    T.uniform = true;
    std::vector<double> cost((size_t)n_total);
    std::vector<int32_t> level_of((size_t)n_total, -1);
    for (int l = 0; l < n_levels; ++l) {
        T.levels[(size_t)l] = make_level(&lv[l].w, lv[l].t_init, lv[l].t, dt, lv[l].level_id, 0u);
        const LevelDev &L = T.levels[(size_t)l];
        if (!(L.dt_last == L.dt && L.cbm_last == L.cbm)) T.uniform = false;
        for (int64_t i = 0; i < lv[l].n_nodes; ++i) {
            const int64_t g = lv[l].node_offset + i;
            if (level_of[(size_t)g] >= 0) return fail(FK_E_INVAL, "levels overlap at node %lld", (long long)g);
            level_of[(size_t)g] = l;
            cost[(size_t)g] = node_cost(pts[2 * g], pts[2 * g + 1], lv[l].t);
        }
    }
    for (int64_t g = 0; g < n_total; ++g)
        if (level_of[(size_t)g] < 0) return fail(FK_E_INVAL, "node %lld belongs to no level", (long long)g);
    std::vector<int64_t> order((size_t)n_total);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return cost[(size_t)a] > cost[(size_t)b]; });
    for (int64_t s = 0; s < n_total; ++s) {
        const int64_t g = order[(size_t)s];
        const int l = level_of[(size_t)g];
        NodeDev &nd = T.nodes[(size_t)s];
        // Start point as an FP32 (hi, lo) pair holding the FP64 node to ~2^-48.
        nd.x = (float)pts[2 * g];
        nd.y = (float)pts[2 * g + 1];
        nd.xlo = (float)(pts[2 * g] - (double)nd.x);
        nd.ylo = (float)(pts[2 * g + 1] - (double)nd.y);
        nd.nid = (uint32_t)(g - lv[l].node_offset);
        nd.level = (uint32_t)l;
        nd.out = (uint64_t)g;
        OutDev &od = T.outs[(size_t)g];
        // The kernel stores scores minus the hi part of the start point; the
        // shift adds that same value back.
        od.shift_x = T.shift ? (double)nd.x : 0.0;
        od.shift_y = T.shift ? (double)nd.y : 0.0;
        od.K = T.levels[(size_t)l].K;
    }
    return FK_OK;
}

int device_cus(int *n_cu) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(FK_E_NODEVICE, "no HIP device: %s", hipGetErrorString(e));
    e = hipDeviceGetAttribute(n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    return FK_OK;
}

// Optional per-kernel event timing of the calling thread.
struct Timing {
    bool enabled = false;
    bool recorded = false;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
};
thread_local Timing g_timing;

static hipError_t timing_mark(bool on, int i, hipStream_t s) {
    if (!on) return hipSuccess;
    return hipEventRecord(g_timing.ev[i], s);
}

hipError_t timing_record(int i, hipStream_t s) {
    hipError_t e = timing_mark(g_timing.enabled, i, s);
    if (e == hipSuccess && i == 2 && g_timing.enabled) g_timing.recorded = true;
    return e;
}

int short_chunk(int64_t n_nodes, int64_t n_paths, int n_cu, bool masked) {
    if (masked) return 256;   // the active count is known on the device only
    const int64_t want = 8LL * 28 * n_cu;
    for (int c = 2048; c > 256; c >>= 1)
        if (n_nodes * ((n_paths + c - 1) / c) >= want) return c;
    return 256;
}

int few_paths_chunk(int64_t n_nodes, int64_t n_paths, int n_cu) {
    // 64 chunks per CU: at least eight per resident wavefront of the
    // network kernels (two waves per SIMD)
    const int64_t want = 64LL * n_cu;
    for (int c = 128; c > 32; c >>= 1)
        if (n_nodes * ((n_paths + c - 1) / c) >= want) return c;
    return 32;
}

int check_chunks(int64_t n_nodes, int64_t n_paths, const fk_plan &pl) {
    const int64_t cpn = (n_paths + pl.chunk - 1) / pl.chunk;
    // chunk indices run past the last chunk by up to two grid-fulls of
    // wavefronts (each wavefront's first chunk, and its final failed grab)
    if (n_nodes * cpn >= 0xff000000LL) return fail(FK_E_INVAL, "too many work chunks; raise plan chunk");
    return FK_OK;
}

int enqueue_solve(const SolveLaunch &S, hipStream_t stream, bool allow_timing) {
    int n_cu = 0;
    int rc;
    if ((rc = device_cus(&n_cu)) != FK_OK) return rc;
    if ((rc = check_chunks(S.n_nodes, S.n_paths, S.plan)) != FK_OK) return rc;
    const bool timed = allow_timing && g_timing.enabled;
    hipError_t e;
    const int64_t cpn = (S.n_paths + S.plan.chunk - 1) / S.plan.chunk;
    if ((e = launch_counters_init(S.counters, (uint32_t)(S.n_nodes * cpn), stream)) != hipSuccess)
        return hip_fail(e, "zero counters");
    if ((e = launch_zero_u32((uint32_t *)S.args.acc, (int)(acc_bytes(S.n_nodes) / 4), stream)) != hipSuccess)
        return hip_fail(e, "zero estimator sums");
    if (S.tables) {
        // node tables from the device coordinates (they also set the chunk count)
        TableArgs t = *S.tables;
        t.counters = S.counters;
        t.cpn = (uint32_t)cpn;
        if ((e = launch_tables(t, stream)) != hipSuccess) return hip_fail(e, "node table kernels");
    }
    PathArgs a = S.args;
    if (S.total_steps) {
        if ((e = launch_zero_u32((uint32_t *)S.total_steps, 2, stream)) != hipSuccess)
            return hip_fail(e, "zero total_steps");
        a.total_steps = (unsigned long long *)S.total_steps;
    } else {
        // nobody asked for the count: short horizons skip it (the kernels
        // skip a null count), others keep it in the counters block
        a.total_steps = S.first_by_index ? nullptr : (unsigned long long *)(S.counters + 2);
    }
    a.queue = S.counters;
    a.n_paths = (uint32_t)S.n_paths;
    a.chunk = (uint32_t)S.plan.chunk;
    a.cpn = (uint32_t)cpn;
    a.total_chunks = (uint32_t)(S.n_nodes * cpn);
    a.tile_shift = (uint32_t)__builtin_ctz((unsigned)S.plan.node_tile);
    int bpc = S.plan.blocks_per_cu;
    const bool expo = a.score_mode == FK_SCORE_EXPONENTIAL;
    const int occ = expo ? expo_kernel_max_blocks_per_cu(S.kind, S.time_mode, S.plan.block)
                         : path_kernel_max_blocks_per_cu(S.kind, S.time_mode, S.uniform,
                                                         a.score_mode == FK_SCORE_BRIDGE, S.first_by_index,
                                                         S.plan.block);
    if (bpc == 0 || (occ > 0 && bpc > occ)) bpc = occ > 0 ? occ : 1;
    const int grid = cap_grid(n_cu * bpc, a.total_chunks, S.plan.block);
    if ((e = timing_mark(timed, 0, stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    e = expo ? launch_expo_paths(S.kind, S.time_mode, a, grid, S.plan.block, stream)
             : launch_paths(S.kind, S.time_mode, S.uniform, S.first_by_index, a, grid, S.plan.block, stream);
    if (e != hipSuccess) return hip_fail(e, "path kernel launch");
    if ((e = timing_mark(timed, 1, stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    FinalArgs f = S.fin;
    f.acc = a.acc;
    f.n_paths = S.n_paths;
    f.n_out = S.n_nodes;
    if ((e = launch_finalize(f, stream)) != hipSuccess) return hip_fail(e, "finalize kernel launch");
    if ((e = timing_mark(timed, 2, stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    if (timed) g_timing.recorded = true;
    return FK_OK;
}

void fill_common_args(SolveLaunch &S, const fk_data *d, bool shift, uint64_t seed) {
    PathArgs &a = S.args;
    a.grid_xi = d->grid_xi;
    a.grid_eta = d->grid_eta;
    a.grid_n = d->grid_n;
    a.init_kind = d->init_kind;
    a.bdry_kind = d->bdry_kind;
    a.score_mode = d->score_mode;
    a.shift = shift ? 1 : 0;
    a.key0 = (uint32_t)seed;
    a.key1 = (uint32_t)(seed >> 32);
}

// Workspace layout of one single-call interface solve: queue counters, the
// level and node tables and the per-node estimator sums (no per-path data).
struct WsLayout {
    size_t counters, levels, nodes, outs, acc, total;
};

static WsLayout ws_layout(int64_t n_levels, int64_t n_nodes) {
    WsLayout L{};
    size_t off = 0;
    L.counters = off;
    off += 256;
    L.levels = off;
    off += align256(sizeof(LevelDev) * (size_t)n_levels);
    L.nodes = off;
    off += align256(sizeof(NodeDev) * (size_t)n_nodes);
    L.outs = off;
    off += align256(sizeof(OutDev) * (size_t)n_nodes);
    L.acc = off;
    off += align256(acc_bytes(n_nodes));
    L.total = off;
    return L;
}

// ---- device scratch of fk_interface_solve_noalloc ---------------------------
// A fixed device array in the library's code object (each GPU holds its own
// copy until the process ends).  Host code never uses the array's name as a
// device address: its address on each device is looked up once, with that
// device current, and kept here.
constexpr size_t kScratchBytes = (size_t)8 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

static int scratch_address(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(FK_E_NODEVICE, "no HIP device: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(FK_E_UNSUPPORTED, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress of the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return FK_OK;
}

}  // namespace fk

using namespace fk;

extern "C" {

int fk_version(void) { return 100; }

const char *fk_last_error(void) { return g_last_error.c_str(); }

size_t fk_interface_workspace_bytes(int64_t n_nodes, int64_t n_paths) {
    if (n_nodes < 0 || n_paths < 2) return 0;
    return ws_layout(1, n_nodes).total;
}

int fk_timing_enable(int enable) {
    g_last_error.clear();
    if (enable && !g_timing.ev[0]) {
        for (hipEvent_t &e : g_timing.ev) {
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return hip_fail(r, "hipEventCreate");
        }
    }
    g_timing.enabled = enable != 0;
    g_timing.recorded = false;
    return FK_OK;
}

int fk_timing_last(double *path_kernel_ms, double *reduce_kernel_ms) {
    g_last_error.clear();
    if (!g_timing.recorded) return fail(FK_E_INVAL, "no timed solve recorded");
    hipError_t e = hipEventSynchronize(g_timing.ev[2]);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float a = 0.f, b = 0.f;
    if ((e = hipEventElapsedTime(&a, g_timing.ev[0], g_timing.ev[1])) != hipSuccess)
        return hip_fail(e, "hipEventElapsedTime");
    if ((e = hipEventElapsedTime(&b, g_timing.ev[1], g_timing.ev[2])) != hipSuccess)
        return hip_fail(e, "hipEventElapsedTime");
    if (path_kernel_ms) *path_kernel_ms = a;
    if (reduce_kernel_ms) *reduce_kernel_ms = b;
    return FK_OK;
}

int fk_sync(hipStream_t stream) {
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "queued work");
    return FK_OK;
}

int fk_interface_solve(const fk_density *w, const fk_data *d, const double *pts, const uint8_t *mask,
                       int64_t n_nodes, double t, double dt, int64_t n_paths, uint64_t seed, uint32_t level_id,
                       double *xi, double *eta, double *se_xi, double *se_eta, int32_t *exit_step, float *scores,
                       int64_t *steps, uint64_t *total_steps, const fk_plan *plan, void *workspace,
                       size_t workspace_bytes, hipStream_t stream) {
    g_last_error.clear();
    int rc;
    if ((rc = validate_density(w)) != FK_OK) return rc;
    if ((rc = validate_data(d)) != FK_OK) return rc;
    if ((rc = validate_common(n_paths, dt)) != FK_OK) return rc;
    if ((rc = validate_horizon(t, d->t_init, dt, level_id)) != FK_OK) return rc;
    if ((rc = validate_device_points(pts, n_nodes)) != FK_OK) return rc;
    if (n_nodes > 0 && (!xi || !eta || !se_xi || !se_eta)) return fail(FK_E_INVAL, "an output pointer is NULL");
    fk_plan pl;
    if ((rc = resolve_plan(plan, &pl)) != FK_OK) return rc;
    if ((rc = check_chunks(n_nodes, n_paths, pl)) != FK_OK) return rc;
    const WsLayout lay = ws_layout(1, n_nodes);
    if (!workspace || workspace_bytes < lay.total)
        return fail(FK_E_NOMEM, "workspace too small: need %zu bytes", lay.total);
    if (((uintptr_t)workspace & 255u) != 0) return fail(FK_E_INVAL, "workspace must be 256-byte aligned");
    if (n_nodes == 0) return FK_OK;

    char *ws = (char *)workspace;
    const LevelDev level = make_level(w, d->t_init, t, dt, level_id, 0u);
    const bool shift = (d->init_kind == FK_DATA_IDENTITY && d->bdry_kind == FK_DATA_IDENTITY);
    SolveLaunch S{};
    S.kind = w->kind;
    S.time_mode = w->time_mode;
    S.uniform = (level.dt_last == level.dt && level.cbm_last == level.cbm);
    S.plan = pl;
    // Short paths (a mesh step of a few tens of sub-steps): each wavefront's
    // first chunk by its grid index, and by default short_chunk paths per
    // grab, which cuts the wavefronts' fixed costs per path; long ones 128,
    // for the balance of the tail.
    S.first_by_index = level.K <= 64 && d->score_mode != FK_SCORE_EXPONENTIAL;
    if ((!plan || plan->chunk == 0) && S.first_by_index) {
        int n_cu = 0;
        if ((rc = device_cus(&n_cu)) != FK_OK) return rc;
        S.plan.chunk = short_chunk(n_nodes, n_paths, n_cu, mask != nullptr);
    }
    S.n_nodes = n_nodes;
    S.n_paths = n_paths;
    S.counters = (uint32_t *)(ws + lay.counters);
    S.total_steps = total_steps;
    fill_common_args(S, d, shift, seed);
    S.args.levels = (const LevelDev *)(ws + lay.levels);
    S.args.nodes = (const NodeDev *)(ws + lay.nodes);
    S.args.acc = (NodeAcc *)(ws + lay.acc);
    S.args.scores = (float2 *)scores;
    S.args.exit_step = exit_step;
    TableArgs tab{};
    tab.pts = pts;
    tab.mask = mask;
    tab.n = n_nodes;
    tab.level = level;
    tab.levels_out = (LevelDev *)(ws + lay.levels);
    tab.nodes_out = (NodeDev *)(ws + lay.nodes);
    tab.outs_out = (OutDev *)(ws + lay.outs);
    tab.acc = S.args.acc;
    tab.shift = shift ? 1 : 0;
    tab.sort = S.first_by_index ? 0 : 1;   // every node of a short horizon costs about the same
    tab.horizon = (float)t;
    S.tables = &tab;
    S.fin.outs = (const OutDev *)(ws + lay.outs);
    S.fin.xi = xi;
    S.fin.eta = eta;
    S.fin.se_xi = se_xi;
    S.fin.se_eta = se_eta;
    S.fin.steps = steps;
    S.fin.mask = mask;
    return enqueue_solve(S, stream, true);
}

size_t fk_interface_noalloc_max_bytes(void) { return kScratchBytes; }

int fk_interface_solve_noalloc(const fk_density *w, const fk_data *d, const double *pts, const uint8_t *mask,
                               int64_t n_nodes, double t, double dt, int64_t n_paths, uint64_t seed,
                               uint32_t level_id, double *xi, double *eta, double *se_xi, double *se_eta,
                               int32_t *exit_step, float *scores, int64_t *steps, uint64_t *total_steps,
                               const fk_plan *plan, hipStream_t stream) {
    g_last_error.clear();
    const size_t need = fk_interface_workspace_bytes(n_nodes, n_paths);
    if (need > kScratchBytes)
        return fail(FK_E_NOMEM, "%lld nodes need %zu bytes of scratch; the static scratch holds %zu (about %lld nodes)",
                    (long long)n_nodes, need, kScratchBytes,
                    (long long)(kScratchBytes / (need / (size_t)std::max<int64_t>(n_nodes, 1))));
    void *ws = nullptr;
    int rc;
    if ((rc = scratch_address(&ws)) != FK_OK) return rc;
    return fk_interface_solve(w, d, pts, mask, n_nodes, t, dt, n_paths, seed, level_id, xi, eta, se_xi, se_eta,
                              exit_step, scores, steps, total_steps, plan, ws, kScratchBytes, stream);
}

}  // extern "C"
