// fk_batch.hip -- batched interface solves: many time levels and sub-domain
// layouts (uneven node counts) in one persistent launch, with a plan object
// that keeps the tables on the device, an autotuner over launch shapes, and
// hipGraph capture of the whole launch sequence.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fk.h"
#include "fk_accum.hpp"
#include "fk_internal.hpp"

struct fk_batch {
    int device = 0;
    fk::Tables T;
    void *dev_tables = nullptr;
    const fk::LevelDev *d_levels = nullptr;
    const fk::NodeDev *d_nodes = nullptr;
    const fk::OutDev *d_outs = nullptr;
    fk_data data{};
    double dt = 0.0;
    int64_t n_total = 0, n_paths = 0;
    uint64_t seed = 0;
    fk_plan plan{256, 0, 128, 0};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace fk {

// Workspace of a batch run: queue counters and the per-node estimator sums.
static size_t batch_ws_bytes(const fk_batch *b) { return 256 + align256(acc_bytes(b->n_total)); }

static int batch_launch(fk_batch *b, int64_t n_paths, const fk_plan &pl, double *xi, double *eta, double *se_xi,
                        double *se_eta, int32_t *exit_step, float *scores, uint64_t *total_steps, void *workspace,
                        size_t workspace_bytes, hipStream_t stream, bool allow_timing) {
    if (b->n_total > 0 && (!xi || !eta || !se_xi || !se_eta)) return fail(FK_E_INVAL, "an output pointer is NULL");
    const size_t need = batch_ws_bytes(b);
    if (!workspace || workspace_bytes < need) return fail(FK_E_NOMEM, "workspace too small: need %zu bytes", need);
    if (((uintptr_t)workspace & 255u) != 0) return fail(FK_E_INVAL, "workspace must be 256-byte aligned");
    if (b->n_total == 0) return FK_OK;
    char *ws = (char *)workspace;
    SolveLaunch S{};
    S.kind = b->T.kind;
    S.time_mode = b->T.time_mode;
    S.uniform = b->T.uniform;
    S.plan = pl;
    S.n_nodes = b->n_total;
    S.n_paths = n_paths;
    S.counters = (uint32_t *)ws;
    S.total_steps = total_steps;
    fill_common_args(S, &b->data, b->T.shift, b->seed);
    S.args.levels = b->d_levels;
    S.args.nodes = b->d_nodes;
    S.args.acc = (NodeAcc *)(ws + 256);
    S.args.scores = (float2 *)scores;
    S.args.exit_step = exit_step;
    S.fin.outs = b->d_outs;
    S.fin.xi = xi;
    S.fin.eta = eta;
    S.fin.se_xi = se_xi;
    S.fin.se_eta = se_eta;
    S.fin.steps = nullptr;
    return enqueue_solve(S, stream, allow_timing);
}

// The batch's shape for the tuned-plan cache: the device and a hash of the
// kinds, modes, level count, nodes, paths and probe size.
static std::string tune_key(const fk_batch *b, int64_t probe) {
    struct {
        int32_t kind, time_mode, uniform, score_mode;
        int64_t levels, n_total, n_paths, probe;
    } shape{b->T.kind, b->T.time_mode, (int32_t)b->T.uniform, b->data.score_mode, (int64_t)b->T.levels.size(),
            b->n_total, b->n_paths, probe};
    char hex[32];
    std::snprintf(hex, sizeof hex, "%016llx", (unsigned long long)fnv1a(&shape, sizeof shape, 0xcbf29ce484222325ull));
    return "batch/" + device_signature(b->device) + "/" + hex;
}

}  // namespace fk

using namespace fk;

extern "C" {

int fk_batch_create(const fk_level *levels, int32_t n_levels, const double *pts, int64_t n_total, const fk_data *d,
                    double dt, int64_t n_paths, uint64_t seed, fk_batch_t *out) {
    g_last_error.clear();
    if (!out) return fail(FK_E_INVAL, "out is NULL");
    *out = nullptr;
    int rc;
    if (n_levels < 1 || !levels) return fail(FK_E_INVAL, "need at least one level");
    if ((rc = validate_data(d)) != FK_OK) return rc;
    if (d->score_mode == FK_SCORE_EXPONENTIAL)
        return fail(FK_E_UNSUPPORTED, "exponential time-stepping is for single plain solves only");
    if ((rc = validate_common(n_paths, dt)) != FK_OK) return rc;
    if ((rc = validate_points(pts, n_total)) != FK_OK) return rc;
    std::vector<LevelSpec> spec((size_t)n_levels);
    for (int l = 0; l < n_levels; ++l) {
        const fk_level &L = levels[l];
        if ((rc = validate_density(&L.w)) != FK_OK) return rc;
        if (L.w.kind != levels[0].w.kind || L.w.time_mode != levels[0].w.time_mode)
            return fail(FK_E_UNSUPPORTED, "all levels of a batch must share the density kind and time mode");
        if ((rc = validate_horizon(L.t, L.t_init, dt, L.level_id)) != FK_OK) return rc;
        if (L.node_offset < 0 || L.n_nodes < 0 || L.node_offset + L.n_nodes > n_total)
            return fail(FK_E_INVAL, "level %d node range is outside the node list", l);
        spec[(size_t)l] = LevelSpec{L.w, L.t, L.t_init, L.node_offset, L.n_nodes, L.level_id};
    }
    fk_batch *b = new fk_batch();
    if ((rc = build_tables(spec.data(), n_levels, pts, n_total, d, dt, b->T)) != FK_OK) {
        delete b;
        return rc;
    }
    hipError_t e = hipGetDevice(&b->device);
    if (e != hipSuccess) {
        delete b;
        return fail(FK_E_NODEVICE, "no HIP device: %s", hipGetErrorString(e));
    }
    const size_t lb = align256(sizeof(LevelDev) * b->T.levels.size());
    const size_t nb = align256(sizeof(NodeDev) * b->T.nodes.size());
    const size_t ob = align256(sizeof(OutDev) * b->T.outs.size());
    if ((e = hipMalloc(&b->dev_tables, lb + nb + ob + 256)) != hipSuccess) {
        delete b;
        return fail(FK_E_NOMEM, "hipMalloc of batch tables: %s", hipGetErrorString(e));
    }
    char *p = (char *)b->dev_tables;
    b->d_levels = (const LevelDev *)p;
    b->d_nodes = (const NodeDev *)(p + lb);
    b->d_outs = (const OutDev *)(p + lb + nb);
    if ((e = hipMemcpy(p, b->T.levels.data(), sizeof(LevelDev) * b->T.levels.size(), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(p + lb, b->T.nodes.data(), sizeof(NodeDev) * b->T.nodes.size(), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(p + lb + nb, b->T.outs.data(), sizeof(OutDev) * b->T.outs.size(), hipMemcpyHostToDevice)) != hipSuccess) {
        hipFree(b->dev_tables);
        delete b;
        return hip_fail(e, "upload batch tables");
    }
    b->data = *d;
    b->dt = dt;
    b->n_total = n_total;
    b->n_paths = n_paths;
    b->seed = seed;
    *out = b;
    return FK_OK;
}

size_t fk_batch_workspace_bytes(fk_batch_t b) { return b ? batch_ws_bytes(b) : 0; }

int fk_batch_set_plan(fk_batch_t b, const fk_plan *plan) {
    g_last_error.clear();
    if (!b) return fail(FK_E_INVAL, "batch is NULL");
    fk_plan pl;
    int rc;
    if ((rc = resolve_plan(plan, &pl)) != FK_OK) return rc;
    if ((rc = check_chunks(b->n_total, b->n_paths, pl)) != FK_OK) return rc;
    b->plan = pl;
    return FK_OK;
}

int fk_batch_get_plan(fk_batch_t b, fk_plan *plan) {
    g_last_error.clear();
    if (!b || !plan) return fail(FK_E_INVAL, "NULL argument");
    *plan = b->plan;
    return FK_OK;
}

int fk_batch_run(fk_batch_t b, double *xi, double *eta, double *se_xi, double *se_eta, int32_t *exit_step,
                 float *scores, uint64_t *total_steps, void *workspace, size_t workspace_bytes, hipStream_t stream) {
    g_last_error.clear();
    if (!b) return fail(FK_E_INVAL, "batch is NULL");
    return batch_launch(b, b->n_paths, b->plan, xi, eta, se_xi, se_eta, exit_step, scores, total_steps, workspace,
                        workspace_bytes, stream, true);
}

int fk_batch_autotune(fk_batch_t b, int64_t probe_paths, void *workspace, size_t workspace_bytes, hipStream_t stream,
                      fk_plan *chosen) {
    g_last_error.clear();
    if (!b) return fail(FK_E_INVAL, "batch is NULL");
    if (probe_paths < 2 || probe_paths > b->n_paths) return fail(FK_E_INVAL, "probe_paths must be in [2, n_paths]");
    const std::string key = tune_key(b, probe_paths);
    fk_plan cached;
    if (tune_cache_get(key, &cached)) {
        b->plan = cached;
        if (chosen) *chosen = b->plan;
        return FK_OK;
    }
    if (b->n_total == 0) {
        if (chosen) *chosen = b->plan;
        return FK_OK;
    }
    double *out = nullptr;
    hipError_t e = hipMalloc(&out, sizeof(double) * 4 * (size_t)b->n_total);
    if (e != hipSuccess) return fail(FK_E_NOMEM, "hipMalloc of probe outputs: %s", hipGetErrorString(e));
    const int occ = path_kernel_max_blocks_per_cu(b->T.kind, b->T.time_mode, b->T.uniform,
                                                  b->data.score_mode == FK_SCORE_BRIDGE, false, 256);
    fk_plan best = b->plan;
    // Each grab costs one atomic on the queue counter.  A probe much shorter
    // than the full launch does not show that cost, which grows with the
    // path count: grabs below 128 paths are only tried when the full launch
    // has less than 16 times the probe's paths.
    const int min_chunk = b->n_paths >= 16 * probe_paths ? 128 : 1;
    const int rc = tune_sweep(
        occ,
        [&](const fk_plan &pl) {
            return batch_launch(b, probe_paths, pl, out, out + b->n_total, out + 2 * b->n_total,
                                out + 3 * b->n_total, nullptr, nullptr, nullptr, workspace, workspace_bytes, stream,
                                false);
        },
        [&](const fk_plan &pl) { return check_chunks(b->n_total, probe_paths, pl) == FK_OK; }, stream, &best,
        min_chunk);
    hipFree(out);
    if (rc != FK_OK) return rc;
    b->plan = best;
    tune_cache_put(key, best);
    if (chosen) *chosen = best;
    return FK_OK;
}

int fk_batch_capture(fk_batch_t b, double *xi, double *eta, double *se_xi, double *se_eta, int32_t *exit_step,
                     float *scores, uint64_t *total_steps, void *workspace, size_t workspace_bytes,
                     hipStream_t stream) {
    g_last_error.clear();
    if (!b) return fail(FK_E_INVAL, "batch is NULL");
    if (stream == nullptr) return fail(FK_E_INVAL, "graph capture needs a non-default stream");
    hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    int rc = batch_launch(b, b->n_paths, b->plan, xi, eta, se_xi, se_eta, exit_step, scores, total_steps, workspace,
                          workspace_bytes, stream, false);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(stream, &g);
    if (rc != FK_OK) {
        if (g) hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t x = nullptr;
    if ((e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0)) != hipSuccess) {
        hipGraphDestroy(g);
        return hip_fail(e, "hipGraphInstantiate");
    }
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    b->graph = g;
    b->exec = x;
    return FK_OK;
}

int fk_batch_replay(fk_batch_t b, hipStream_t stream) {
    g_last_error.clear();
    if (!b || !b->exec) return fail(FK_E_INVAL, "no captured graph");
    hipError_t e = hipGraphLaunch(b->exec, stream);
    return e == hipSuccess ? FK_OK : hip_fail(e, "hipGraphLaunch");
}

void fk_batch_destroy(fk_batch_t b) {
    if (!b) return;
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    if (b->dev_tables) hipFree(b->dev_tables);
    delete b;
}

}  // extern "C"
