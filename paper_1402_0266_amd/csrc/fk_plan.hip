// fk_plan.hip -- launch plans: the autotuner of the path kernel's launch
// shape (shared by single solves and batches), its cache, and the plan
// handle that also holds a captured HIP graph.
//
// The tuner times candidate shapes of the persistent path kernel (workgroup
// size x paths per queue grab x resident workgroups x node tile) on the
// caller's own problem and keeps the fastest.  Every candidate computes the
// same result: the plan only changes the schedule.  Results are cached per
// process under a key made of the device's signature (name, architecture,
// compute units) and a hash of the problem's shape; with the environment
// variable FK_TUNE_CACHE naming a file, also in that file (one "key block
// blocks_per_cu chunk node_tile" line per entry), so a later process skips
// the sweep.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fk.h"
#include "fk_internal.hpp"

namespace fk {

namespace {
std::mutex g_cache_mu;
std::map<std::string, fk_plan> g_cache;
bool g_file_loaded = false;

const char *cache_file() {
    const char *f = std::getenv("FK_TUNE_CACHE");
    return (f && *f) ? f : nullptr;
}

void load_file_locked() {
    if (g_file_loaded) return;
    g_file_loaded = true;
    const char *path = cache_file();
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char key[256];
    fk_plan p{};
    while (std::fscanf(f, "%255s %d %d %d %d", key, &p.block, &p.blocks_per_cu, &p.chunk, &p.node_tile) == 5)
        g_cache[key] = p;
    std::fclose(f);
}
}  // namespace

uint64_t fnv1a(const void *data, size_t n, uint64_t h) {
    const unsigned char *p = (const unsigned char *)data;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

std::string device_signature(int dev) {
    hipDeviceProp_t prop{};
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    char buf[160];
    std::snprintf(buf, sizeof buf, "%s/%s/%dcu", prop.gcnArchName, prop.name, prop.multiProcessorCount);
    for (char *c = buf; *c; ++c)
        if (*c == ' ') *c = '_';
    return buf;
}

bool tune_cache_get(const std::string &key, fk_plan *out) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    load_file_locked();
    auto it = g_cache.find(key);
    if (it == g_cache.end()) return false;
    *out = it->second;
    return true;
}

void tune_cache_put(const std::string &key, const fk_plan &p) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    load_file_locked();
    g_cache[key] = p;
    if (const char *path = cache_file()) {
        if (FILE *f = std::fopen(path, "a")) {
            std::fprintf(f, "%s %d %d %d %d\n", key.c_str(), p.block, p.blocks_per_cu, p.chunk, p.node_tile);
            std::fclose(f);
        }
    }
}

int tune_sweep(int occ_full, const std::function<int(const fk_plan &)> &launch,
               const std::function<bool(const fk_plan &)> &admissible, hipStream_t stream, fk_plan *best_out,
               int min_chunk) {
    static const int blocks[] = {64, 128, 256};
    static const int chunks[] = {32, 128, 512};
    static const int divs[] = {1, 2};
    static const int tiles[] = {1, 8};
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        hipEventDestroy(e0);
        return hip_fail(e, "hipEventCreate");
    }
    fk_plan best = *best_out;
    float best_ms = 1e30f;
    // one untimed launch loads the code object and warms the caches
    int rc = launch(best);
    for (int bl : blocks) {
        for (int ch : chunks) {
            if (ch < min_chunk) continue;
            for (int dv : divs) {
                for (int nt : tiles) {
                    if (rc != FK_OK) break;
                    const int occ = occ_full > 0 ? occ_full * 256 / bl : 0;
                    fk_plan pl{bl, occ > 0 ? (occ + dv - 1) / dv : 0, ch, nt};
                    if (!admissible(pl)) continue;
                    hipEventRecord(e0, stream);
                    rc = launch(pl);
                    hipEventRecord(e1, stream);
                    if (rc != FK_OK) break;
                    if ((e = hipEventSynchronize(e1)) != hipSuccess) {
                        rc = hip_fail(e, "autotune probe");
                        break;
                    }
                    float ms = 0.f;
                    hipEventElapsedTime(&ms, e0, e1);
                    if (ms < best_ms) {
                        best_ms = ms;
                        best = pl;
                    }
                }
            }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc == FK_OK) *best_out = best;
    return rc;
}

}  // namespace fk

using namespace fk;

// The plan handle: a launch plan, and the executable graph of the last
// capture on it.
struct fk_plan_handle {
    fk_plan plan{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int updates = 0;       // captures applied to the existing executable graph in place
};

extern "C" {

int fk_plan_create(const fk_plan *initial, fk_plan_t *out) {
    g_last_error.clear();
    if (!out) return fail(FK_E_INVAL, "out is NULL");
    *out = nullptr;
    fk_plan pl;
    int rc;
    if ((rc = resolve_plan(initial, &pl)) != FK_OK) return rc;
    fk_plan_handle *h = new fk_plan_handle();
    h->plan = pl;
    *out = h;
    return FK_OK;
}

int fk_plan_get(fk_plan_t p, fk_plan *out) {
    g_last_error.clear();
    if (!p || !out) return fail(FK_E_INVAL, "NULL argument");
    *out = p->plan;
    return FK_OK;
}

int fk_plan_set(fk_plan_t p, const fk_plan *plan) {
    g_last_error.clear();
    if (!p) return fail(FK_E_INVAL, "plan handle is NULL");
    fk_plan pl;
    int rc;
    if ((rc = resolve_plan(plan, &pl)) != FK_OK) return rc;
    p->plan = pl;
    return FK_OK;
}

int fk_plan_autotune(fk_plan_t p, const fk_density *w, const fk_data *d, const double *pts, const uint8_t *mask,
                     int64_t n_nodes, double t, double dt, int64_t probe_paths, uint64_t seed, void *workspace,
                     size_t workspace_bytes, hipStream_t stream) {
    g_last_error.clear();
    if (!p) return fail(FK_E_INVAL, "plan handle is NULL");
    int rc;
    if ((rc = validate_density(w)) != FK_OK) return rc;
    if ((rc = validate_data(d)) != FK_OK) return rc;
    if ((rc = validate_common(probe_paths, dt)) != FK_OK) return rc;
    if ((rc = validate_horizon(t, d->t_init, dt, 0)) != FK_OK) return rc;
    if ((rc = validate_device_points(pts, n_nodes)) != FK_OK) return rc;
    if (n_nodes == 0) return FK_OK;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(FK_E_NODEVICE, "no HIP device: %s", hipGetErrorString(e));
    // the key: the device, and the problem's shape (not its values)
    struct {
        int32_t kind, time_mode, score_mode, init_kind, bdry_kind, masked;
        int64_t n_nodes, probe, K;
    } shape{w->kind, w->time_mode, d->score_mode, d->init_kind, d->bdry_kind, mask ? 1 : 0, n_nodes, probe_paths,
            (int64_t)step_count(t, dt)};
    char hex[32];
    std::snprintf(hex, sizeof hex, "%016llx", (unsigned long long)fnv1a(&shape, sizeof shape, 0xcbf29ce484222325ull));
    const std::string key = "solve/" + device_signature(dev) + "/" + hex;
    fk_plan cached;
    if (tune_cache_get(key, &cached)) {
        p->plan = cached;
        return FK_OK;
    }
    double *out = nullptr;
    if ((e = hipMalloc(&out, sizeof(double) * 4 * (size_t)n_nodes)) != hipSuccess)
        return fail(FK_E_NOMEM, "hipMalloc of probe outputs: %s", hipGetErrorString(e));
    const bool expo = d->score_mode == FK_SCORE_EXPONENTIAL;
    const bool first = step_count(t, dt) <= 64 && !expo;
    const int occ = expo ? expo_kernel_max_blocks_per_cu(w->kind, w->time_mode, 256)
                         : path_kernel_max_blocks_per_cu(w->kind, w->time_mode, true,
                                                         d->score_mode == FK_SCORE_BRIDGE, first, 256);
    fk_plan best = p->plan;
    rc = tune_sweep(
        occ,
        [&](const fk_plan &pl) {
            return fk_interface_solve(w, d, pts, mask, n_nodes, t, dt, probe_paths, seed, 0, out, out + n_nodes,
                                      out + 2 * n_nodes, out + 3 * n_nodes, nullptr, nullptr, nullptr, nullptr, &pl,
                                      workspace, workspace_bytes, stream);
        },
        [&](const fk_plan &pl) { return check_chunks(n_nodes, probe_paths, pl) == FK_OK; }, stream, &best);
    hipFree(out);
    if (rc != FK_OK) return rc;
    p->plan = best;
    tune_cache_put(key, best);
    return FK_OK;
}

int fk_plan_capture_begin(fk_plan_t p, hipStream_t stream) {
    g_last_error.clear();
    if (!p) return fail(FK_E_INVAL, "plan handle is NULL");
    if (stream == nullptr) return fail(FK_E_INVAL, "graph capture needs a non-default stream");
    hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed);
    return e == hipSuccess ? FK_OK : hip_fail(e, "hipStreamBeginCapture");
}

int fk_plan_capture_end(fk_plan_t p, hipStream_t stream) {
    g_last_error.clear();
    if (!p) return fail(FK_E_INVAL, "plan handle is NULL");
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(stream, &g);
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    if (p->exec) {
        // the same sequence with other arguments: update the executable graph
        // in place when its topology allows it
        hipGraphNode_t err_node = nullptr;
        hipGraphExecUpdateResult res = hipGraphExecUpdateError;
        if (hipGraphExecUpdate(p->exec, g, &err_node, &res) == hipSuccess && res == hipGraphExecUpdateSuccess) {
            if (p->graph) hipGraphDestroy(p->graph);
            p->graph = g;
            ++p->updates;
            return FK_OK;
        }
        (void)hipGetLastError();
        hipGraphExecDestroy(p->exec);
        p->exec = nullptr;
    }
    hipGraphExec_t x = nullptr;
    if ((e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0)) != hipSuccess) {
        hipGraphDestroy(g);
        return hip_fail(e, "hipGraphInstantiate");
    }
    if (p->graph) hipGraphDestroy(p->graph);
    p->graph = g;
    p->exec = x;
    return FK_OK;
}

int fk_plan_replay(fk_plan_t p, hipStream_t stream) {
    g_last_error.clear();
    if (!p) return fail(FK_E_INVAL, "plan handle is NULL");
    if (!p->exec) return fail(FK_E_INVAL, "nothing captured on this plan");
    hipError_t e = hipGraphLaunch(p->exec, stream);
    return e == hipSuccess ? FK_OK : hip_fail(e, "hipGraphLaunch");
}

int fk_plan_graph_updates(fk_plan_t p) { return p ? p->updates : -1; }

void fk_plan_destroy(fk_plan_t p) {
    if (!p) return;
    if (p->exec || p->graph) hipDeviceSynchronize();
    if (p->exec) hipGraphExecDestroy(p->exec);
    if (p->graph) hipGraphDestroy(p->graph);
    delete p;
}

}  // extern "C"
