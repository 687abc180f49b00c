// Internal declarations shared by the host API and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pbf {

// Per-scene constants on the device.  Derived on the host in double and
// rounded once to float.
struct SceneDev {
    float lo[3], hi[3];
    float h, h2, h6;
    float c_rho;   // m * 315 / (64 pi h^9) / rho0: rho_i / rho0 = c_rho * sum (h^2 - r^2)^3
    float c_grad;  // 45 / (pi h^6): |grad W_spiky| = c_grad (h - r)^2
    float c_s;     // m / rho0^2: factor of lambda's denominator
    float inv_rho0, eps, dt, inv_dt;
    float g[3];
    int32_t dims[3];
    uint32_t cell_off;  // first global cell index of the scene
    uint32_t pid_off;   // first global particle ID of the scene
    int32_t n_min, n_max;
    int32_t lod_mode;
    float cam[3], d_near, d_far;
};

// Device fault bits, latched in a device word.
enum : uint32_t {
    ERR_NEIGHBOUR_CAP = 1u,
    ERR_CELL_CAP = 2u,
    ERR_NONFINITE = 4u,
};

// Kernel classes (launch shape and profiling unit).
enum Kernel : int {
    K_FILL = 0,
    K_LOD_PREDICT,
    K_SCAN_REDUCE,
    K_SCAN_TOP,
    K_SCAN_APPLY,
    K_SORT_SCATTER,
    K_SORT_FINISH,
    K_NEIGHBOURS,
    K_LEVEL_COUNT,
    K_LEVEL_SCAN,
    K_LEVEL_SCATTER,
    K_LAMBDA,
    K_UPDATE,
    K_COMMIT,
    K_COUNT
};

extern const char *const kKernelNames[K_COUNT];
extern const int kDefaultBlock[K_COUNT];

constexpr int kLevelBlock = 256;  // slots per level-bucketing block (fixed: 4 waves)
constexpr int kScanItems = 8;     // items per thread in the cell-count scan
constexpr int kScanBlock = 256;   // threads of a scan block (2048 items)

// Every buffer one step touches.  Storage ("slot") order is the cell order
// of the last counting sort; "t" order is the level-bucketed order of the
// active sets (descending level, then slot).
struct StepBuffers {
    int64_t n;              // particles, all scenes
    uint32_t n_cells;       // cells, all scenes
    int32_t n_iters;        // loop bound (largest n_max)
    int32_t nbr_cap;        // neighbour capacity
    int32_t n_level_blocks; // ceil(n / kLevelBlock)
    int32_t n_scan_blocks;  // ceil(n_cells / (kScanBlock * kScanItems))
    const SceneDev *scenes;
    uint8_t *lev_by_id;        // explicit levels, global-ID order

    // ping-pong particle state (slot order): [0] = current, [1] = after reorder
    float4 *x[2], *v[2];
    uint32_t *id[2];
    uint8_t *lvl[2];
    float4 *xs[2];          // x* ping-pong inside a step; .w carries lambda
    float4 *xs_pred;        // x* right after prediction, pre-sort order
    uint32_t *key_pre, *ticket, *key;
    uint32_t *tmp_src, *tmp_id;
    uint32_t *cell_count, *cell_start, *scan_part;
    uint32_t *level_counts;  // n_iters * n_level_blocks, scanned in place
    uint32_t *count_ge;      // [PBF_MAX_ITERS + 2]: |{i : N_i >= L}|
    uint32_t *order;         // t -> slot
    uint32_t *nbr;           // [nbr_cap][n] column-major, indexed by t
    uint32_t *nmeta;         // [n] by t: (scene << 16) | |N_i|
    uint32_t *err;
    unsigned long long *totals;  // [0] sum of N_i over steps, [1] steps
};

struct LaunchShape {
    int block[K_COUNT];
};

struct Timer;  // per-launch profiling hook (host side)
void timer_begin(Timer *tm, int kernel, hipStream_t s);
void timer_end(Timer *tm, int kernel, hipStream_t s);

// Enqueue one full step on stream s: LOD + predict, counting sort and
// reorder, neighbour lists, level buckets, n_iters x (lambda, update),
// commit.  `cur` selects which ping-pong half holds the current state; after
// the step the current state is in half cur ^ 1.
hipError_t enqueue_step(const StepBuffers &b, int cur, const LaunchShape &ls, hipStream_t s,
                        Timer *tm);

}  // namespace pbf

namespace pbf {
// Scatter slot-ordered positions (or velocities) into ID order for the IDs
// [id_lo, id_hi): out[3 (id - id_lo) + c].
hipError_t enqueue_unpermute(int64_t n, const float4 *x, const uint32_t *id, float *out,
                             uint32_t id_lo, uint32_t id_hi, hipStream_t s);
}  // namespace pbf
