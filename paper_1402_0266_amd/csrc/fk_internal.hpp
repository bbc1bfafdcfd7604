// fk_internal.hpp -- device-side tables and kernel arguments shared by the
// library's own translation units (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <functional>

#include <string>
#include <vector>

#include "fk.h"

namespace fk {

// Per time level: horizon, step sizes and density parameters, pre-folded into
// the FP32 constants the path kernel uses.
struct alignas(16) LevelDev {
    float tend;        // PDE time at path start: t_init + t
    float horizon;     // t: elapsed time since the initial data at path start
    float dt;          // step size of all steps but the last
    float dt_last;     // t - (K-1) dt
    float cbm;         // -4 ln2 dt: sqrt(cbm * log2(u1)) = sqrt(2 dt) * sqrt(-2 ln u1)
    float cbm_last;    // same for dt_last
    int32_t K;         // number of steps
    uint32_t ctr3;     // Philox counter word 3: (level_id << 4) | stream
    float amp;         // density amplitude A
    float nscale;      // -log2(e) / width2 (argument scale of exp2)
    float a2s;         // 2 A / width2
    float cx, cy;      // centre (static) or orbit centre (moving)
    float orbit_r;     // orbit radius
    float omega_rev;   // omega / (2 pi): angular speed in revolutions per unit time
    float t_freeze;    // frozen density time
    float rev0;        // (t_init + t) omega_rev: orbit angle at path start, in revolutions
    float drev;        // dt omega_rev: orbit angle step
    float cos_d, sin_d;  // cos / sin of the orbit angle step (2 pi drev)
    const float2 *gb;  // grid density: nodal drift table [(gn+1)^2], else nullptr
    int32_t gn;        // grid density: cells per side
    float fn;          // (float) gn
};

// One interface node, in launch (cost-sorted) order.
struct alignas(16) NodeDev {
    float x, y;        // start point, hi parts
    float xlo, ylo;    // start point, lo parts (x + xlo is the FP64 node to ~2^-48)
    uint32_t nid;      // Philox counter word 2: index of the node in its level
    uint32_t level;    // index into the level table
    uint64_t out;      // output row: per-path records live at out * n_paths + path
};

// One output row: the shift the per-path records are stored relative to.
struct alignas(16) OutDev {
    double shift_x, shift_y;
    int64_t K;
    int64_t pad;
};

struct NodeAcc;

// The 64 32-bit words of a launch's counters (zeroed before it).
constexpr int kCtrQueue = 0;     // work-chunk counter
constexpr int kCtrSteps = 2;     // [2..3] 64-bit step count (when the caller gives no buffer)
constexpr int kCtrActive = 4;    // nodes in the launch
constexpr int kCtrTotal = 5;     // work chunks in the launch (the path kernels read it here)
constexpr int kCtrHist = 16;     // [16..48) per cost bucket: node count, then the bucket's next slot
constexpr int kCostBuckets = 32;

struct PathArgs {
    const LevelDev *levels;
    const NodeDev *nodes;
    NodeAcc *acc;                    // [n_out] estimator sums (zeroed before launch)
    float2 *scores;                  // [n_out * n_paths] per-path scores, or nullptr
    int32_t *exit_step;              // [n_out * n_paths] or nullptr
    uint32_t *queue;                 // chunk counter (zeroed before launch)
    unsigned long long *total_steps; // accumulated Euler-Maruyama steps
    const double *grid_xi;
    const double *grid_eta;
    int32_t grid_n;
    int32_t init_kind, bdry_kind, score_mode;
    int32_t shift;                   // identity data: store scores minus the start point
    uint32_t key0, key1;
    uint32_t n_paths;                // paths per node
    uint32_t chunk;                  // paths per queue grab
    uint32_t cpn;                    // chunks per node
    uint32_t total_chunks;           // host bound on the work chunks (grid size); the kernels
                                     // read the launch's own count from queue[kCtrTotal]
    uint32_t tile_shift;             // chunk order: interleave the chunks of 2^tile_shift nodes (0: node by node)
};

// The estimator's last step: node sums -> means, standard errors, steps.
struct FinalArgs {
    const NodeAcc *acc;
    const OutDev *outs;
    int64_t n_out;
    int64_t n_paths;
    double *xi, *eta, *se_xi, *se_eta;
    int64_t *steps;                  // or nullptr
    const uint8_t *mask;             // nodes solved (others' outputs untouched), or nullptr: all
};

// Node tables of a single-level solve built on the device from its node
// coordinates (device memory): the level constants, one NodeDev per node in
// the solve (in decreasing expected cost when `sort`), one OutDev per node.
struct TableArgs {
    const double *pts;       // [n][2] FP64
    const uint8_t *mask;     // [n]: nodes to solve, or nullptr: all
    int64_t n;
    LevelDev level;
    LevelDev *levels_out;    // [1]
    NodeDev *nodes_out;      // [n] (the first counters[kCtrActive] used)
    OutDev *outs_out;        // [n]: shift (FP32 rounding of the node when `shift`), K
    OutDev *outs_zero_out;   // [n] or nullptr: the same with zero shift (control-variate estimates)
    NodeAcc *acc;            // [n]: a node outside the closed square (or NaN) is flagged bad
    NodeAcc *acc2;           // [n] or nullptr: flagged too
    uint32_t *counters;
    uint32_t cpn;            // work chunks per node
    int shift;
    int sort;
    float horizon;           // t: caps the expected cost
};

// ---- host-side planning (fk_api.hip) ---------------------------------------

// One time level of a solve: density, horizon and its slice of the node list.
struct LevelSpec {
    fk_density w;
    double t;
    double t_init;
    int64_t node_offset;
    int64_t n_nodes;
    uint32_t level_id;
};

// Device tables of a solve, built on the host.
struct Tables {
    std::vector<LevelDev> levels;
    std::vector<NodeDev> nodes;  // launch (cost) order
    std::vector<OutDev> outs;    // output order
    int kind = 0, time_mode = 0;
    bool uniform = true;         // every step has length dt
    bool shift = false;          // scores stored relative to the start point
};

// Everything one enqueue of the solve sequence needs.
struct SolveLaunch {
    PathArgs args;       // tables, accumulators, data; counters and sizes filled by enqueue_solve
    FinalArgs fin;       // outputs; sizes filled by enqueue_solve
    int kind, time_mode;
    bool uniform;
    bool first_by_index;  // short horizons: each wavefront's first chunk by its grid index
    const TableArgs *tables;  // device-built tables (filled in by enqueue_solve), or nullptr: host tables
    fk_plan plan;
    int64_t n_nodes, n_paths;
    uint32_t *counters;  // 256 B of device scratch (queue, step count)
    uint64_t *total_steps;
};

extern thread_local std::string g_last_error;
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int hip_fail(hipError_t e, const char *what);
size_t align256(size_t n);
int64_t step_count(double t, double dt);
int validate_density(const fk_density *w);
int validate_data(const fk_data *d);
int validate_common(int64_t n_paths, double dt);
int validate_horizon(double t, double t_init, double dt, uint32_t level_id);
int validate_points(const double *pts, int64_t n);         // host coordinates
int validate_device_points(const double *pts, int64_t n);  // device coordinates (checked in the kernels)
LevelDev make_level(const fk_density *w, double t_init, double t, double dt, uint32_t level_id, uint32_t stream);
int resolve_plan(const fk_plan *plan, fk_plan *out);
int check_chunks(int64_t n_nodes, int64_t n_paths, const fk_plan &pl);
// Default paths per grab for short horizons: 256, or the largest of 512 ..
// 2048 that still leaves 8 chunks per resident wavefront (28 per CU); 256
// for masked solves.  The chunk only changes the schedule, never a result.
int short_chunk(int64_t n_nodes, int64_t n_paths, int n_cu, bool masked);
// Default grab of the network and gradient-table forms on long horizons:
// the largest of 128, 64, 32 paths that leaves at least 64 chunks per CU
// (few paths per node leave the grid part-empty with larger grabs).
int few_paths_chunk(int64_t n_nodes, int64_t n_paths, int n_cu);

// Launch-plan tuning (fk_plan.hip): a 64-bit FNV-1a hash, the device's
// signature, the tuned-plan cache (per process; FK_TUNE_CACHE names a file
// that persists it), and the sweep over candidate plans: `launch` enqueues
// one run with a plan, `admissible` filters the candidates, occ_full is the
// kernel's occupancy at 256 threads; best_out holds the starting plan and
// receives the fastest; grab sizes below min_chunk are not tried.
uint64_t fnv1a(const void *data, size_t n, uint64_t h);
std::string device_signature(int dev);
bool tune_cache_get(const std::string &key, fk_plan *out);
void tune_cache_put(const std::string &key, const fk_plan &p);
int tune_sweep(int occ_full, const std::function<int(const fk_plan &)> &launch,
               const std::function<bool(const fk_plan &)> &admissible, hipStream_t stream, fk_plan *best_out,
               int min_chunk = 1);
// A persistent grid of `grid` blocks cut to no more wavefronts than there
// are work chunks (small solves: a wavefront with no chunk only costs its
// launch).
inline int cap_grid(int grid, uint32_t total_chunks, int block) {
    const int64_t wpb = block / 64;
    const int64_t need = ((int64_t)total_chunks + wpb - 1) / wpb;
    return (int)std::max<int64_t>(1, std::min<int64_t>(grid, need));
}
int build_tables(const LevelSpec *lv, int n_levels, const double *pts, int64_t n_total, const fk_data *d, double dt,
                 Tables &T);
void fill_common_args(SolveLaunch &S, const fk_data *d, bool shift, uint64_t seed);
int device_cus(int *n_cu);
// Queues zero-counters, path kernel and reduction on the stream.  With
// allow_timing, records the timing events when timing is enabled.
int enqueue_solve(const SolveLaunch &S, hipStream_t stream, bool allow_timing);
// Timing events of the calling thread (no-ops while timing is disabled):
// 0 before the path kernels, 1 after them, 2 after the reductions.
hipError_t timing_record(int i, hipStream_t s);

// Launch helpers implemented in fk_paths.hip.
hipError_t launch_zero_u32(uint32_t *p, int n_words, hipStream_t s);
hipError_t launch_paths(int kind, int time_mode, bool uniform, bool first_by_index, const PathArgs &a, int grid,
                        int block, hipStream_t s);
hipError_t launch_finalize(const FinalArgs &a, hipStream_t s);
// Device node tables (three small kernels; after the counters and sums are zeroed).
hipError_t launch_tables(const TableArgs &t, hipStream_t s);
// Zeroes a launch's 64 counter words and sets counters[kCtrTotal] (host tables).
hipError_t launch_counters_init(uint32_t *counters, uint32_t total_chunks, hipStream_t s);
// Bytes of the per-node estimator sums of n_out rows.
size_t acc_bytes(int64_t n_out);
int path_kernel_max_blocks_per_cu(int kind, int time_mode, bool uniform, bool bridge, bool first_by_index, int block);
// Exponential time-stepping (FK_SCORE_EXPONENTIAL): its own path kernel.
hipError_t launch_expo_paths(int kind, int time_mode, const PathArgs &a, int grid, int block, hipStream_t s);
int expo_kernel_max_blocks_per_cu(int kind, int time_mode, int block);

}  // namespace fk
