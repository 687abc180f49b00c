// Internal declarations shared by the host API and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pbf {

constexpr int PBF_MAX_ITERS_INTERNAL = 32;  // equals PBF_MAX_ITERS of the public header

// Spatial tiles: blocks of kTileEdge^3 grid cells.  A tile's workgroup stages
// the (kTileEdge + 2)^3 cells around it -- kStageRows x-rows of
// kStageEdge cells each -- into LDS and evaluates every pair of its own
// particles from there.
constexpr int kTileEdge = 4;
constexpr int kStageEdge = kTileEdge + 2;
constexpr int kStageRows = kStageEdge * kStageEdge;
constexpr int kOwnRows = kTileEdge * kTileEdge;
// float4 entries staged in LDS: a third above the rest occupancy of eight
// particles per cell (2304 entries, 36 KiB, for 6^3 cells), in whole waves
constexpr int kStageCap = kStageEdge * kStageEdge * kStageEdge * 32 / 3 / 64 * 64;
constexpr int kTileThreads = 512;  // threads of a solver-pass tile workgroup (at most)
constexpr int kNbrThreads = 512;   // threads of a neighbour-build tile workgroup (at most)
constexpr int kDecodeThreads = 256;  // threads of a workgroup decoding a tile's codes (reverse pass)
constexpr int kBndWords = kStageRows * (kStageEdge + 1);  // cell bounds of the staged rows
constexpr int kRowWords = kBndWords + kStageRows + 1;     // saved tables per tile
constexpr uint32_t kXcds = 8;       // accelerator complex dies of an MI355X (own L2 each)
constexpr int kSegOffBits = 10;    // fallback neighbour code: row << 10 | offset
static_assert(kStageRows <= 64 && kOwnRows <= 64, "staged row in six bits, an own row per lane");
// LDS stage entry kStageCap (one past the staged particles) holds a point
// this far away; its code pads the last group of a neighbour list
constexpr uint32_t kFarCode = kStageCap;
constexpr float kFar = 1e18f;
// LDS stage array: the staged particles, the far entry, and spare entries so
// that the neighbour scan may read up to three entries past any window
constexpr int kStageSlack = 3;
constexpr int kStageEntries = kStageCap + 1 + kStageSlack;
// pmeta bit fields: neighbour count (13 bits), level (6 bits), and the
// particle's own index in its tile's LDS stage (13 bits; 0 when the stage
// does not fit)
constexpr uint32_t kMetaCountBits = 13;
constexpr uint32_t kMetaCount = (1u << kMetaCountBits) - 1u;
constexpr uint32_t kMetaLevelShift = kMetaCountBits;
constexpr uint32_t kMetaSelfShift = kMetaCountBits + 6;
__host__ __device__ inline uint32_t meta_level(uint32_t m) { return (m >> kMetaLevelShift) & 63u; }
__host__ __device__ inline uint32_t meta_self(uint32_t m) { return m >> kMetaSelfShift; }
__host__ __device__ inline uint32_t make_meta(uint32_t count, uint32_t level, uint32_t self)
{
    return count | (level << kMetaLevelShift) | (self << kMetaSelfShift);
}

// Per-scene constants on the device.  Derived on the host in double and
// rounded once to float.
// A solid obstacle (PBF_OBSTACLE_*): centre and sizes as in pbf_obstacle.
struct ObstacleDev {
    int32_t kind;
    float c[3];
    float a[3];
};
constexpr int kMaxObstacles = 4;  // PBF_MAX_OBSTACLES
constexpr int kMaxCameras = 4;    // PBF_MAX_CAMERAS

struct SceneDev {
    float lo[3], hi[3];
    float h, h2, h6;
    float c_rho;   // m * 315 / (64 pi h^9) / rho0: rho_i / rho0 = c_rho * sum (h^2 - r^2)^3
    float c_grad;  // 45 / (pi h^6): |grad W_spiky| = c_grad (h - r)^2
    float c_s;     // m / rho0^2: factor of lambda's denominator
    float inv_rho0, eps, dt, inv_dt;
    float g[3];
    int32_t dims[3];
    int32_t tiles[3];   // tiles per axis: ceil(dims / kTileEdge)
    uint32_t cell_off;  // first global cell index of the scene
    uint32_t tile_off;  // first global tile index of the scene
    uint32_t pid_off;   // first global particle ID of the scene
    int32_t n_min, n_max;
    int32_t lod_mode;
    float cam[3], d_near, d_far;
    // distance to the visible surface: camera frame, focal length, image
    // and splat radius; the scene's depth image starts at depth_off
    float fwd[3], up[3], focal, splat;
    int32_t img_w, img_h;
    uint32_t depth_off;
    // solid obstacles and pre-stabilisation (particles with N_i < stab_s)
    int32_t n_obst, stab_iters, stab_s;
    ObstacleDev obst[kMaxObstacles];
    // distance-to-camera cameras (cams[0] = cam) with their ranges; with
    // auto_range the ranges are found every step, into the range words at
    // range_off (min, max float bits per camera)
    int32_t n_cam, auto_range;
    float cams[kMaxCameras][3];
    float rng[kMaxCameras][2];
    uint32_t range_off;
    float c_floor;  // lower bound of C_i: 0 (unilateral) or -infinity
    // force-based cohesion: gamma, and the factor gamma m 32 dt^2 / (pi h^9)
    // of the prediction's shift (0: none)
    float cohesion, c_coh;
};

// Device fault bits, latched in a device word.
enum : uint32_t {
    ERR_NEIGHBOUR_CAP = 1u,
    ERR_CELL_CAP = 2u,
    ERR_NONFINITE = 4u,
};

// Kernel classes (launch shape and profiling unit).
enum Kernel : int {
    K_DEPTH = 0,
    K_LOD_PREDICT,
    K_SCAN_REDUCE,
    K_SCAN_TOP,
    K_SCAN_APPLY,
    K_SORT_SCATTER,
    K_SORT_FINISH,
    K_TILE_PREPARE,
    K_LEVEL_COUNT,
    K_LEVEL_SCAN,
    K_LEVEL_SCATTER,
    K_TILE_TABLES,
    K_NEIGHBOURS,
    K_LAMBDA,
    K_UPDATE,
    K_COMMIT,
    K_CONTACTS,
    K_LOD_RANGE,
    K_COHESION,
    K_COUNT
};

extern const char *const kKernelNames[K_COUNT];
extern const int kDefaultBlock[K_COUNT];

constexpr int kLevelBlock = 256;  // items per level-bucketing block (fixed: 4 waves)
constexpr int kScanItems = 8;     // items per thread in the exclusive scans
constexpr int kScanBlock = 256;   // threads of a scan block (2048 items)
constexpr int kScanDirect = 1024;  // scans of up to this many blocks skip the top-level pass
constexpr uint32_t kFusedTiles = 16384;  // up to this many tiles, one workgroup does the tile tables
constexpr uint32_t kSplitTarget = 1024;  // tile workgroups that fill the chip (4 per CU)
constexpr uint32_t kMaxSplit = 8;        // at most this many workgroups per tile (64 particles each)

// Workgroups per tile for a grid of `tiles` tiles: with few tiles, each
// tile's own particles are split over up to kMaxSplit workgroups so that the
// grid still fills the chip.
inline uint32_t tile_split(uint32_t tiles)
{
    return tiles >= kSplitTarget ? 1u : (kSplitTarget / tiles < kMaxSplit ? kSplitTarget / tiles : kMaxSplit);
}

// Part `sub` of `parts` of a tile's nown own particles, cut at wave
// boundaries: [first, last); false when the part is empty.
__device__ __forceinline__ bool split_part(uint32_t nown, uint32_t sub, uint32_t parts, uint32_t &first,
                                           uint32_t &last)
{
    const uint32_t chunk = ((nown + parts - 1) / parts + 63u) & ~63u;
    first = sub * chunk;
    last = nown < first + chunk ? nown : first + chunk;
    return first < last;
}

// Every buffer one step touches.  Storage ("slot") order is the cell order
// of the last counting sort.  Per-particle solver data ("p" order) is laid
// out tile by tile: p = tile_start[tile] + rank inside the tile (descending
// level, ties in cell order), so each iteration's active particles come first.
struct StepBuffers {
    int64_t n;               // particles, all scenes
    uint32_t n_cells;        // cells, all scenes
    uint32_t n_tiles;        // tiles, all scenes
    int32_t n_iters;         // loop bound (largest n_max)
    int32_t nbr_cap;         // neighbour capacity
    int32_t nbr_stride;      // codes per particle in nbr: nbr_cap rounded up to 8
    int32_t n_level_blocks;  // ceil(n_tiles / kLevelBlock)
    int32_t n_scan_blocks;   // scan blocks for max(n_cells, n_tiles)
    const SceneDev *scenes;
    uint8_t *lev_by_id;      // explicit levels, global-ID order
    const uint32_t *tile_scene;  // scene of each tile
    const uint32_t *id_scene;    // scene of each global particle ID

    // ping-pong particle state (slot order): [cur] -> reorder -> [cur ^ 1]
    float4 *x[2], *v[2];
    uint32_t *id[2];
    uint8_t *lvl[2];
    float4 *xs[2];           // x* ping-pong inside a step; .w carries lambda
    float4 *xs_pred;         // x* right after prediction, pre-sort order
    uint32_t *key_pre, *ticket, *key;
    uint32_t *tmp_src, *tmp_id;
    uint32_t *cell_count, *cell_start, *scan_part;
    // tiles
    uint32_t *tile_count;    // own particles per tile
    uint32_t *tile_start;    // exclusive scan of tile_count (n_tiles + 1)
    uint8_t *tile_lvl;       // largest level among own particles (0: empty)
    uint32_t *level_counts;  // (n_iters + 1) * n_level_blocks, scanned in place
    uint32_t *tile_ge;       // [PBF_MAX_ITERS + 2]: tiles with level >= L
    uint32_t *tile_order;    // tiles by descending level, ties by tile index
    uint32_t *tile_rows;     // [n_tiles][kRowWords] stage layout of each tile, by its
                             // slot in tile_order
    uint4 *tile_rec;         // [n_tiles] by slot in tile_order: tile, first p, own
                             // particles, scene (written by the neighbour build)
    // per particle, p order
    uint4 *nbr;              // [nbr_stride / 8][n] groups of eight u16 neighbour codes
    uint32_t *pmeta;         // neighbour count, level, own stage index (see make_meta)
    uint32_t *pslot;         // slot of particle p
    uint32_t *err;
    uint32_t *level_part;    // per lod_predict block: sum of N_i
    unsigned long long *totals;  // [0] sum of N_i over steps, [1] steps
    uint32_t *depth;         // depth images of the DTVS scenes (float bits)
    uint32_t n_depth;        // their pixels in total (0: no DTVS scene)
    uint8_t *contact;        // [n] contacts found this step, slot order (bit o: obstacle o)
    bool contacts_on;        // some scene has obstacles or pre-stabilisation
    bool cohesion_on;        // some scene has force-based cohesion
    bool poison;             // debug: NaN-fill the float buffers each step writes before it reads them
    uint32_t *range;         // automatic distance ranges (min, max float bits per camera)
    uint32_t n_range;        // their words (0: no scene with an automatic range)
};

struct LaunchShape {
    int block[K_COUNT];
};

// What the reverse pass needs of one forward step: its sorted IDs and
// levels, its neighbour structure, and the positions (with the lambda used)
// before every iteration's correction plus the final positions.
struct StepRecord {
    uint32_t *id;        // slot -> ID after the step's counting sort
    uint8_t *lvl;        // level per slot
    uint4 *nbr;
    uint32_t *pmeta, *pslot;
    uint32_t *tile_rows, *tile_order, *tile_start, *tile_count, *tile_ge;
    uint4 *tile_rec;
    float4 *snap[PBF_MAX_ITERS_INTERNAL + 1];  // (z^k, lambda^k) for k < K; snap[K] = z^K
};

// scratch of the reverse pass, slot order of the step being reversed
struct AdjointScratch {
    uint32_t *nslot;     // [nbr_cap][n] neighbour slots (decoded codes)
    float4 *zb, *xb, *dpb, *gc;
    float *lb, *sb;
};

struct Timer;  // per-launch profiling hook (host side)
void timer_begin(Timer *tm, int kernel, hipStream_t s);
void timer_end(Timer *tm, int kernel, hipStream_t s);

// Enqueue one full step on stream s: levels + prediction, counting sort and
// reorder, tiles and their level buckets, neighbour lists, n_iters x
// (lambda, update), commit.  `cur` selects the ping-pong half that holds the
// current state; after the step the current state is in half cur ^ 1.
hipError_t enqueue_step(const StepBuffers &b, int cur, const LaunchShape &ls, hipStream_t s,
                        Timer *tm, const StepRecord *rec = nullptr);

// Reverse of one recorded step: ID-order adjoints of the step's outputs (x',
// v') in, of its inputs (x, v) out (in and out may alias).
hipError_t enqueue_adjoint_step(const StepBuffers &b, const StepRecord &r, const float *ax_in,
                                const float *av_in, float *ax_out, float *av_out,
                                const AdjointScratch &w, hipStream_t s);

// Storage order = ID order, state from float[3n] arrays in ID order.
hipError_t enqueue_load_state(int64_t n, const float *x3, const float *v3,
                              const uint32_t *id_scene, float4 *x, float4 *v, uint32_t *id,
                              hipStream_t s);

// Buffers of the average-density measure: a fresh neighbour structure of the
// current positions (sizes as in StepBuffers), its own fault word and
// totals, and the results.
struct DensityBuffers {
    float4 *xs;              // current positions in the fresh cell order
    uint32_t *key;
    uint4 *nbr;
    uint32_t *pmeta, *pslot;
    uint32_t *tile_rows, *tile_order, *tile_start, *tile_count, *tile_ge;
    uint4 *tile_rec;
    uint8_t *tile_lvl;
    uint32_t *err;
    unsigned long long *totals;
    float *rho_slot;         // rho_i / rho0 per fresh slot
    double *part_sum;        // per tile workgroup (n_tiles rounded up to kXcds)
    float *part_max;
    double *out;             // [0] mean, [1] max
};

// rho_i / rho0 of every particle at the positions of half `cur` (Eqs. 5-6)
// over neighbour sets found afresh at those positions; half cur ^ 1 is used
// as scratch.  rho_id (if not null): float[n] in ID order.
hipError_t enqueue_density(const StepBuffers &b, int cur, const LaunchShape &ls,
                           const DensityBuffers &d, float *rho_id, hipStream_t s);

// Scatter slot-ordered positions (or velocities) into ID order for the IDs
// [id_lo, id_hi): out[3 (id - id_lo) + c].
hipError_t enqueue_unpermute(int64_t n, const float4 *x, const uint32_t *id, float *out,
                             uint32_t id_lo, uint32_t id_hi, hipStream_t s);

}  // namespace pbf
