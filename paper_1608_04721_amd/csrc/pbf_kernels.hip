// gfx950 kernels of one adaptive PBF step (Section 5, Fig. 7 of the paper).
//
// Data layout in HBM (all scenes of a context concatenated):
//   x, v        float4[n]  slot order (cell-sorted); x.w holds the scene index bits
//   xs[2]       float4[n]  predicted positions x*, ping-pong across solver
//                          iterations; .w holds lambda_i
//   id, lvl     u32/u8[n]  particle ID and level N_i per slot
//   key         u32[n]     global cell key per slot (scene cell offset + local
//                          key, x fastest)
//   cell_start  u32[G+1]   first slot of every cell (exclusive scan of counts)
//   tiles       blocks of 4^3 cells; tile_start is the exclusive scan of their
//               particle counts, tile_order lists them by descending largest
//               level, so the tiles holding active particles of iteration k
//               are a prefix of tile_order (Eqs. 9-10: the active sets nest)
//   nbr         neighbour codes in p order (p = tile_start[tile] + the
//               particle's rank in its tile by descending level, see rank_part),
//               u16 codes packed eight per 16-byte group, group-major:
//               group g of particle p at [g * n + p]; a code is the
//               neighbour's index in the tile's LDS stage, or row << 10 |
//               offset when the stage does not fit in LDS
//   pmeta/pslot u32[n]     neighbour count, level and own index in the LDS
//                          stage (13, 6 and 13 bits), and slot, per p
//
// A tile's workgroup stages the 6^3 cells around its 4^3 cells (36 x-rows of
// 6 cells, contiguous slot ranges) into LDS once per pass and evaluates all
// pairs of its own particles from there.  Every sum is a gather in a fixed
// order (no floating-point atomics), so a step is deterministic; integer
// atomics only count cell occupancy, and the resulting tickets are replaced
// by the rank of the particle ID inside its cell.
#include "pbf_internal.h"

#include <algorithm>
#include <limits>
#include "../../include/pbf.h"

namespace pbf {

const char *const kKernelNames[K_COUNT] = {
    "depth",        "lod_predict",  "scan_reduce", "scan_top",     "scan_apply",  "sort_scatter",
    "sort_finish",  "tile_prepare", "level_count", "level_scan",  "level_scatter",
    "tile_tables",  "neighbours",  "lambda",       "update",      "commit",       "contacts",
    "lod_range",    "cohesion"};

const int kDefaultBlock[K_COUNT] = {256,          256,          kScanBlock,   1024,         kScanBlock,
                                    256,          256,          256,          kLevelBlock,
                                    1024,         kLevelBlock,  1024,         kNbrThreads,
                                    kTileThreads, kTileThreads, 256,          256,
                                    256,          kTileThreads};

namespace {

__device__ __forceinline__ uint32_t block_exclusive_sum(uint32_t v, uint32_t *lds,
                                                        uint32_t *block_total)
{
    // lds: at least blockDim.x / 64 + 1 words; blockDim.x is a multiple of 64
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint32_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t u = __shfl_up(inc, o, 64);
        if (lane >= o) inc += u;
    }
    if (lane == 63) lds[wave] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int w = 0; w < nw; ++w) {
            uint32_t c = lds[w];
            lds[w] = run;
            run += c;
        }
        lds[nw] = run;
    }
    __syncthreads();
    uint32_t r = lds[wave] + inc - v;
    if (block_total) *block_total = lds[nw];
    __syncthreads();
    return r;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ int cell_coord(float p, float lo, float h, int dims)
{
    int c = (int)floorf((p - lo) / h);
    return min(max(c, 0), dims - 1);
}

__device__ __forceinline__ float clampf(float v, float lo, float hi)
{
    return fminf(fmaxf(v, lo), hi);
}

// Level from a distance (linear map of the distance range onto the level
// range, Section 4.1).  The level is an integer chosen by floating point, so
// the operations are fixed: float32, no contraction into FMAs, correctly
// rounded square root and division, in this order.
__device__ __forceinline__ int level_of_distance(float d, float d_near, float d_far, int nmin, int nmax)
{
#pragma clang fp contract(off)
    float t = (d - d_near) / (d_far - d_near);
    t = fminf(fmaxf(t, 0.f), 1.f);  // not a number (zero-width range) -> 0
    const int L = nmax - (int)floorf(t * (float)(nmax - nmin + 1));
    return min(max(L, nmin), nmax);
}

// Distance to a camera, float32 in a fixed order
__device__ __forceinline__ float camera_distance(float x, float y, float z, const float *c)
{
#pragma clang fp contract(off)
    const float dx = x - c[0], dy = y - c[1], dz = z - c[2];
    float d2 = dx * dx;
    d2 = d2 + dy * dy;
    d2 = d2 + dz * dz;
    return sqrtf(d2);
}

// The distance range of camera c of a scene: given, or found this step
// (min, max over the particles; [0, 0] when nothing was found)
__device__ __forceinline__ void camera_range(const SceneDev &S, const uint32_t *__restrict__ range, int c,
                                             float &d_near, float &d_far)
{
    if (S.auto_range) {
        d_near = __uint_as_float(range[S.range_off + 2 * c]);
        d_far = __uint_as_float(range[S.range_off + 2 * c + 1]);
        if (d_far < d_near) d_near = d_far = 0.f;
    } else {
        d_near = S.rng[c][0];
        d_far = S.rng[c][1];
    }
}

// Distance-to-camera level (DTC): the highest level over the scene's cameras
__device__ __forceinline__ int dtc_level(const SceneDev &S, const uint32_t *__restrict__ range, float x,
                                         float y, float z)
{
    int L = 0;
    for (int c = 0; c < S.n_cam; ++c) {
        float dn, df;
        camera_range(S, range, c, dn, df);
        L = max(L, level_of_distance(camera_distance(x, y, z, S.cams[c]), dn, df, S.n_min, S.n_max));
    }
    return L;
}

// Pinhole projection for the distance-to-the-visible-surface model (DTVS):
// pixel, splat radius in pixels and distance to the camera, in float32 with
// a fixed order of operations (pixels and depth minima are decided by
// floating point).  False when the particle is not in front of the camera
// by more than its splat radius or its pixel is far outside the image.
struct Proj {
    int pu, pv, rad;
    float dist;
};

__device__ __forceinline__ bool dtvs_project(const SceneDev &S, float x, float y, float z, Proj &o)
{
#pragma clang fp contract(off)
    const float f0 = S.fwd[0], f1 = S.fwd[1], f2 = S.fwd[2];
    const float u0 = S.up[0], u1 = S.up[1], u2 = S.up[2];
    const float r0 = f1 * u2 - f2 * u1, r1 = f2 * u0 - f0 * u2, r2 = f0 * u1 - f1 * u0;
    const float qx = x - S.cam[0], qy = y - S.cam[1], qz = z - S.cam[2];
    float zd = qx * f0;
    zd = zd + qy * f1;
    zd = zd + qz * f2;
    if (!(zd > S.splat)) return false;
    float xr = qx * r0;
    xr = xr + qy * r1;
    xr = xr + qz * r2;
    float yu = qx * u0;
    yu = yu + qy * u1;
    yu = yu + qz * u2;
    float u = S.focal * xr;
    u = u / zd;
    u = u + 0.5f * (float)S.img_w;
    float v = S.focal * yu;
    v = v / zd;
    v = v + 0.5f * (float)S.img_h;
    const float lim = (float)PBF_MAX_SPLAT + 1.0f;
    if (!(u > -lim && u < (float)S.img_w + lim && v > -lim && v < (float)S.img_h + lim)) return false;
    o.pu = (int)floorf(u);
    o.pv = (int)floorf(v);
    float rf = S.focal * S.splat;
    rf = rf / zd;
    o.rad = min((int)ceilf(rf), PBF_MAX_SPLAT);
    float d2 = qx * qx;
    d2 = d2 + qy * qy;
    d2 = d2 + qz * qz;
    o.dist = sqrtf(d2);
    return true;
}

// DTVS distance: the particle's distance to the camera minus the depth of
// the visible surface at its pixel; false when it is not seen
__device__ __forceinline__ bool dtvs_distance(const SceneDev &S, const uint32_t *__restrict__ depth,
                                              float x, float y, float z, float &d)
{
#pragma clang fp contract(off)
    Proj o;
    if (!(dtvs_project(S, x, y, z, o) && o.pu >= 0 && o.pu < S.img_w && o.pv >= 0 && o.pv < S.img_h))
        return false;
    d = o.dist - __uint_as_float(depth[S.depth_off + (uint32_t)o.pv * (uint32_t)S.img_w + (uint32_t)o.pu]);
    return true;
}

// DTVS level; the lowest level when the particle is not seen
__device__ __forceinline__ int dtvs_level(const SceneDev &S, const uint32_t *__restrict__ depth,
                                          const uint32_t *__restrict__ range, float x, float y, float z)
{
    float d;
    if (!dtvs_distance(S, depth, x, y, z, d)) d = 3.402823466e38f;  // largest float
    float dn, df;
    camera_range(S, range, 0, dn, df);
    return level_of_distance(d, dn, df, S.n_min, S.n_max);
}

// Automatic distance ranges (Section 4.1): clear to (+infinity, 0), then
// every particle of such a scene lowers the minimum and raises the maximum
// of each of its cameras' distances (unsigned order of the float bits, which
// orders non-negative floats; order-independent).  A wave whose particles
// all belong to one scene combines its values first.
__global__ void k_range_clear(uint32_t m, uint32_t *__restrict__ range)
{
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m) range[e] = (e & 1u) ? 0u : 0x7f800000u;
}

__global__ void k_lod_range(int64_t n, const SceneDev *__restrict__ sc, const float4 *__restrict__ x,
                            const uint32_t *__restrict__ depth, uint32_t *__restrict__ range)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = s < n;
    const float4 xi = valid ? x[s] : make_float4(0.f, 0.f, 0.f, __int_as_float(0));
    const int scene = __float_as_int(xi.w);
    const SceneDev &S = sc[scene];
    const bool on = valid && S.auto_range && (S.lod_mode == PBF_LOD_DTC || S.lod_mode == PBF_LOD_DTVS);
    // one scene for the whole wave (lanes past the end count as that scene)
    const int first = __shfl(scene, 0, 64);
    const bool uniform = __all(!valid || scene == first);
    const int ncam = on ? (S.lod_mode == PBF_LOD_DTC ? S.n_cam : 1) : 0;
    const int nloop = uniform ? __shfl(ncam, 0, 64) : ncam;
    for (int c = 0; c < nloop; ++c) {
        float lo = __uint_as_float(0x7f800000u), hi = 0.f;
        if (on && c < ncam) {
            float d;
            bool seen = true;
            if (S.lod_mode == PBF_LOD_DTC) d = camera_distance(xi.x, xi.y, xi.z, S.cams[c]);
            else seen = dtvs_distance(S, depth, xi.x, xi.y, xi.z, d);
            if (seen) lo = hi = d;
        }
        if (uniform) {
            for (int o = 32; o > 0; o >>= 1) {
                lo = fminf(lo, __shfl_xor(lo, o, 64));
                hi = fmaxf(hi, __shfl_xor(hi, o, 64));
            }
            if ((threadIdx.x & 63) != 0) continue;
            if (!(sc[first].auto_range)) continue;
        } else if (!(on && c < ncam)) {
            continue;
        }
        const SceneDev &T = uniform ? sc[first] : S;
        uint32_t *w = &range[T.range_off + 2 * c];
        const uint32_t bl = __float_as_uint(lo), bh = __float_as_uint(hi);
        if (bl < w[0]) atomicMin(&w[0], bl);  // values only move outwards: a stale read is safe
        if (bh > w[1]) atomicMax(&w[1], bh);
    }
}

// Depth images of the DTVS scenes: clear to +infinity, then every particle
// of such a scene keeps the minimum of its distance over its splat square
// (an unsigned minimum of the float bits, which orders non-negative floats;
// the result does not depend on the order of the atomics)
__global__ void k_depth_clear(uint32_t m, uint32_t *__restrict__ depth)
{
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m) depth[e] = 0x7f800000u;
}

// Lower depth[idx[q]] to val[q] where on[q]: the current values are read
// first, all together, and an atomic is issued only where it can still
// lower the value (a stale read costs one needless atomic; the minimum is
// the same, since values only fall)
template <int B>
__device__ __forceinline__ void lower_pixels(uint32_t *__restrict__ depth, const uint32_t (&idx)[B],
                                             const uint32_t (&val)[B], const bool (&on)[B])
{
    uint32_t cur[B];
#pragma unroll
    for (int q = 0; q < B; ++q) cur[q] = on[q] ? depth[idx[q]] : 0u;
#pragma unroll
    for (int q = 0; q < B; ++q)
        if (on[q] && val[q] < cur[q]) atomicMin(&depth[idx[q]], val[q]);
}

constexpr int kSplatThreads = 256;  // particles per splat workgroup
constexpr int kSplatTile = 4096;    // pixels of a workgroup's LDS depth tile (16 KB)
constexpr int kSplatWaves = kSplatThreads / 64;

__global__ __launch_bounds__(kSplatThreads) void k_depth_splat(int64_t n, const SceneDev *__restrict__ sc,
                                                             const float4 *__restrict__ x,
                                                             uint32_t *__restrict__ depth)
{
    // Consecutive particles (cell order) splat overlapping squares, about
    // five per pixel for a workgroup.  Their minimum is taken in an LDS tile
    // over the workgroup's bounding box first, so the depth image gets one
    // read (and at most one atomic) per pixel the workgroup touches; a
    // workgroup spanning scenes or a box larger than the tile writes each
    // particle's square to the image directly.  The whole tile is cleared
    // while the positions load, and the box is combined from one entry per
    // wave, so the workgroup waits at two barriers only.
    __shared__ __align__(16) uint32_t img[kSplatTile];
    __shared__ int wbox[kSplatWaves][6];  // per wave: a0, b0, -a1, -b1 (minima), scenes min, max
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const float4 xi = s < n ? x[s] : make_float4(0.f, 0.f, 0.f, 0.f);
    static_assert(kSplatTile % (4 * kSplatThreads) == 0, "tile clear");
    for (int e = 4 * threadIdx.x; e < kSplatTile; e += 4 * kSplatThreads)
        *reinterpret_cast<uint4 *>(&img[e]) = make_uint4(0x7f800000u, 0x7f800000u, 0x7f800000u, 0x7f800000u);
    bool ok = false;
    int scene = 0, a0 = 0, a1 = -1, b0 = 0, b1 = -1;
    uint32_t bits = 0;
    if (s < n) {
        scene = __float_as_int(xi.w);
        const SceneDev &S = sc[scene];
        Proj o;
        if (S.lod_mode == PBF_LOD_DTVS && dtvs_project(S, xi.x, xi.y, xi.z, o)) {
            bits = __float_as_uint(o.dist);
            a0 = max(o.pu - o.rad, 0);
            a1 = min(o.pu + o.rad, S.img_w - 1);
            b0 = max(o.pv - o.rad, 0);
            b1 = min(o.pv + o.rad, S.img_h - 1);
            ok = a0 <= a1 && b0 <= b1;
        }
    }
    // the wave's box by shuffles (LDS atomics of all lanes on one address
    // would run one lane at a time), one LDS entry per wave
    int bx[6] = {ok ? a0 : INT_MAX, ok ? b0 : INT_MAX, ok ? -a1 : INT_MAX, ok ? -b1 : INT_MAX,
                 ok ? scene : INT_MAX, ok ? scene : -1};
    for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
        for (int q = 0; q < 5; ++q) bx[q] = min(bx[q], __shfl_xor(bx[q], o, 64));
        bx[5] = max(bx[5], __shfl_xor(bx[5], o, 64));
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int q = 0; q < 6; ++q) wbox[wave][q] = bx[q];
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < kSplatWaves; ++w) {
        if (w == wave) continue;
#pragma unroll
        for (int q = 0; q < 5; ++q) bx[q] = min(bx[q], wbox[w][q]);
        bx[5] = max(bx[5], wbox[w][5]);
    }
    const int x0 = bx[0], y0 = bx[1], bw = -bx[2] - x0 + 1, bh = -bx[3] - y0 + 1;
    const bool any = bx[5] >= 0;
    const bool tiled = any && bx[4] == bx[5] && (int64_t)bw * bh <= kSplatTile;  // uniform
    if (!tiled) {
        // each particle's square straight into the image, eight pixels at a
        // time (the particles along one ray all land on the same pixels, so
        // most of them find the value already lower)
        if (ok) {
            const SceneDev &S = sc[scene];
            int a = a0, b = b0;
            while (b <= b1) {
                uint32_t idx[8], val[8];
                bool on[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    on[q] = b <= b1;
                    idx[q] = on[q] ? S.depth_off + (uint32_t)b * (uint32_t)S.img_w + (uint32_t)a
                                   : S.depth_off;  // in bounds even when unused
                    val[q] = bits;
                    if (++a > a1) {
                        a = a0;
                        ++b;
                    }
                }
                lower_pixels(depth, idx, val, on);
            }
        }
        return;
    }
    if (ok)
        for (int b = b0; b <= b1; ++b)
            for (int a = a0; a <= a1; ++a) atomicMin(&img[(b - y0) * bw + (a - x0)], bits);
    __syncthreads();
    // the touched pixels of the tile into the image, four per thread at a time
    const SceneDev &T = sc[bx[4]];
    const int m = bw * bh;
    for (int e0 = threadIdx.x; e0 < m; e0 += 4 * kSplatThreads) {
        uint32_t idx[4], val[4];
        bool on[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = e0 + q * kSplatThreads;
            val[q] = e < m ? img[e] : 0x7f800000u;
            on[q] = val[q] != 0x7f800000u;
            const int r = e / bw, c = e - r * bw;
            idx[q] = on[q] ? T.depth_off + (uint32_t)(y0 + r) * (uint32_t)T.img_w + (uint32_t)(x0 + c)
                           : T.depth_off;
        }
        lower_pixels(depth, idx, val, on);
    }
}

// Ticket of a particle inside its cell from the counting-sort histogram (all
// lanes of the wave call; valid lanes form a prefix of the wave).  Runs of
// lanes with equal keys (consecutive slots usually share a cell) take their
// tickets with one atomic issued by the run's first lane; all run heads of
// the wave issue together.
__device__ __forceinline__ uint32_t cell_ticket(uint32_t k, bool valid, uint32_t *__restrict__ cell_count)
{
    const int lane = threadIdx.x & 63;
    const uint32_t kprev = __shfl_up(k, 1, 64);
    const bool head = valid && (lane == 0 || kprev != k);
    const uint64_t heads = __ballot(head);
    const uint64_t upto = heads & ((2ull << lane) - 1ull);              // heads at or below lane
    const int my_head = 63 - __clzll((long long)upto);                  // valid lanes have one
    const uint64_t above = heads & ~((2ull << lane) - 1ull);
    const uint64_t valid_mask = __ballot(valid);
    const int run_end = above ? (__ffsll((unsigned long long)above) - 1)
                              : (64 - __clzll((long long)valid_mask));  // one past the last valid lane
    uint32_t base = 0;
    if (head) base = atomicAdd(&cell_count[k], (uint32_t)(run_end - lane));
    base = __shfl(base, valid ? my_head : lane, 64);
    return base + (uint32_t)(lane - my_head);
}

// --------------------------------------------- levels + forces + prediction
// Fig. 7 first loop for every particle, plus the level N_i (Eq. 8, adaption
// model of Section 4.1) from the position at the start of the step, the cell
// key of x*, and a ticket inside its cell from the counting-sort histogram.
// Lanes of a wave that share a cell take one atomic for all of them.
__global__ void k_lod_predict(int64_t n, const SceneDev *__restrict__ sc,
                              const float4 *__restrict__ x, const float4 *__restrict__ v,
                              const uint32_t *__restrict__ id, const uint8_t *__restrict__ lev_by_id,
                              const uint32_t *__restrict__ depth, const uint32_t *__restrict__ range,
                              float4 *__restrict__ xs_pred, uint8_t *__restrict__ lvl,
                              uint32_t *__restrict__ key, uint32_t *__restrict__ ticket,
                              uint32_t *__restrict__ cell_count,
                              uint32_t *__restrict__ level_part)
{
    __shared__ uint32_t wsum[1024 / 64];
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool valid = s < n;
    uint32_t k = 0xffffffffu;
    int L = 0;
    if (valid) {
        const float4 xi = x[s];
        const SceneDev &S = sc[__float_as_int(xi.w)];
        const int nmax = S.n_max;
        if (S.lod_mode == PBF_LOD_EXPLICIT) {
            L = lev_by_id[id[s]];
        } else if (S.lod_mode == PBF_LOD_DTC) {
            L = dtc_level(S, range, xi.x, xi.y, xi.z);
        } else if (S.lod_mode == PBF_LOD_DTVS) {
            L = dtvs_level(S, depth, range, xi.x, xi.y, xi.z);
        } else {
            L = nmax;
        }
        const float dt = S.dt;
        float4 vi = v[s];  // v + dt g is only needed for x*: the commit recomputes v
        vi.x += dt * S.g[0];
        vi.y += dt * S.g[1];
        vi.z += dt * S.g[2];
        const float px = clampf(xi.x + dt * vi.x, S.lo[0], S.hi[0]);
        const float py = clampf(xi.y + dt * vi.y, S.lo[1], S.hi[1]);
        const float pz = clampf(xi.z + dt * vi.z, S.lo[2], S.hi[2]);
        xs_pred[s] = make_float4(px, py, pz, 0.f);
        lvl[s] = (uint8_t)L;
        const float h = S.h;
        const int cx = cell_coord(px, S.lo[0], h, S.dims[0]);
        const int cy = cell_coord(py, S.lo[1], h, S.dims[1]);
        const int cz = cell_coord(pz, S.lo[2], h, S.dims[2]);
        k = S.cell_off + (uint32_t)(((int64_t)cz * S.dims[1] + cy) * S.dims[0] + cx);
        key[s] = k;
    }
    const uint32_t tk = cell_ticket(k, valid, cell_count);
    if (valid) ticket[s] = tk;
    // sum of N_i over the block, for the running particle-iteration count
    const uint32_t lsum = wave_sum((uint32_t)L);
    if (lane == 0) wsum[threadIdx.x >> 6] = lsum;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += wsum[w];
        level_part[blockIdx.x] = t;
    }
}

// --------------------------------------------------- exclusive scans
__global__ void k_scan_reduce(const uint32_t *__restrict__ in, uint32_t G,
                              uint32_t *__restrict__ part)
{
    __shared__ uint32_t lds[1024 / 64 + 1];
    const uint32_t base = blockIdx.x * (uint32_t)(blockDim.x * kScanItems);
    uint32_t sum = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        uint32_t e = base + q * blockDim.x + threadIdx.x;
        if (e < G) sum += in[e];
    }
    uint32_t tot;
    block_exclusive_sum(sum, lds, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// single workgroup: exclusive scan of the per-block sums, in place
__global__ void k_scan_top(uint32_t *__restrict__ part, uint32_t nb)
{
    __shared__ uint32_t lds[1024 / 64 + 1];
    uint32_t carry = 0;
    for (uint32_t b0 = 0; b0 < nb; b0 += blockDim.x) {
        uint32_t i = b0 + threadIdx.x;
        uint32_t v = i < nb ? part[i] : 0u;
        uint32_t tot;
        uint32_t ex = block_exclusive_sum(v, lds, &tot);
        if (i < nb) part[i] = carry + ex;
        carry += tot;
    }
}

// clear: if not null (the same array as in), each count is zeroed once read,
// which leaves the cell histogram ready for the next step.  sum_parts: part
// holds the per-block sums themselves (no k_scan_top), and each block adds
// up those before it.
__global__ void k_scan_apply(const uint32_t *in, uint32_t G, const uint32_t *__restrict__ part,
                             uint32_t *__restrict__ out, uint32_t *clear, bool sum_parts)
{
    __shared__ uint32_t lds[1024 / 64 + 1];
    uint32_t off = 0;
    if (sum_parts) {  // uniform
        uint32_t v = 0;
        for (uint32_t i = threadIdx.x; i < blockIdx.x; i += blockDim.x) v += part[i];
        block_exclusive_sum(v, lds, &off);
    } else {
        off = part[blockIdx.x];
    }
    // each thread owns kScanItems consecutive cells
    const uint32_t base = blockIdx.x * (uint32_t)(blockDim.x * kScanItems) +
                          threadIdx.x * (uint32_t)kScanItems;
    uint32_t vals[kScanItems];
    uint32_t sum = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        uint32_t e = base + q;
        vals[q] = e < G ? in[e] : 0u;
        sum += vals[q];
    }
    if (clear) {
#pragma unroll
        for (int q = 0; q < kScanItems; ++q)
            if (base + q < G) clear[base + q] = 0u;
    }
    uint32_t run = off + block_exclusive_sum(sum, lds, nullptr);
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        uint32_t e = base + q;
        if (e < G) {
            out[e] = run;
            if (e == G - 1) out[G] = run + vals[q];
        }
        run += vals[q];
    }
}

// ------------------------------------------------ counting-sort scatter
// Slot inside the cell from the histogram ticket (arbitrary order among
// equal keys); k_sort_finish replaces it by the rank by particle ID.
__global__ void k_sort_scatter(int64_t n, const uint32_t *__restrict__ key,
                               const uint32_t *__restrict__ ticket,
                               const uint32_t *__restrict__ cell_start,
                               const uint32_t *__restrict__ id, uint32_t *__restrict__ tmp_src,
                               uint32_t *__restrict__ tmp_id)
{
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    uint32_t t = cell_start[key[s]] + ticket[s];
    tmp_src[t] = (uint32_t)s;
    tmp_id[t] = id[s];
}

// Final slot = cell start + rank of the particle ID inside its cell (ties of
// the counting sort in particle-ID order), then move the particle there.
// Velocities are not moved: the commit recomputes every one from x and x*.
__global__ void k_sort_finish(int64_t n, const uint32_t *__restrict__ tmp_src,
                              const uint32_t *__restrict__ tmp_id,
                              const uint32_t *__restrict__ key_pre,
                              const uint32_t *__restrict__ cell_start,
                              const float4 *__restrict__ x, const float4 *__restrict__ xs_pred,
                              const uint8_t *__restrict__ lvl_in, float4 *__restrict__ x_out,
                              float4 *__restrict__ xs_out,
                              uint32_t *__restrict__ id_out, uint8_t *__restrict__ lvl_out,
                              uint32_t *__restrict__ key_out, uint32_t *__restrict__ err)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const uint32_t s = tmp_src[t];
    const uint32_t k = key_pre[s];
    const uint32_t lo = cell_start[k], hi = cell_start[k + 1];
    const uint32_t my = tmp_id[t];
    uint32_t f;
    if (hi - lo > (uint32_t)PBF_MAX_CELL) {
        f = (uint32_t)t;
        if (t == lo) atomicOr(err, ERR_CELL_CAP);
    } else {
        uint32_t r = 0;
        for (uint32_t u = lo; u < hi; ++u) r += tmp_id[u] < my ? 1u : 0u;
        f = lo + r;
    }
    x_out[f] = x[s];
    xs_out[f] = xs_pred[s];
    id_out[f] = my;
    lvl_out[f] = lvl_in[s];
    key_out[f] = k;
}


// ------------------------------------------------------------------ obstacles
// Contact finding (Fig. 7, second loop): obstacle o is a contact when its
// bounding volume grown by the margin m holds the predicted position;
// decided in float32 with one rounding per operation.
__device__ __forceinline__ bool contact_found(const ObstacleDev &o, float px, float py, float pz,
                                              float m)
{
#pragma clang fp contract(off)
    const float dx = px - o.c[0], dy = py - o.c[1], dz = pz - o.c[2];
    if (o.kind == PBF_OBSTACLE_SPHERE) {
        const float r = o.a[0] + m;
        return dx * dx + dy * dy + dz * dz < r * r;
    }
    if (o.kind == PBF_OBSTACLE_CONE) {  // the slant moved out by m
        const float rho = sqrtf(dx * dx + dz * dz);
        const float L = sqrtf(o.a[1] * o.a[1] + o.a[0] * o.a[0]);
        return rho * o.a[1] + dy * o.a[0] < o.a[1] * o.a[0] + m * L;
    }
    return fabsf(dx) < o.a[0] + m && fabsf(dy) < o.a[1] + m && fabsf(dz) < o.a[2] + m;
}

// Moves (x, y, z) to the closest point of the obstacle's surface when it
// lies inside the solid (the contact's projection); returns whether it did.
// Sphere: radially (straight up from the centre).  Box: through the face of
// least penetration (first axis on ties).  Cone (standing on the floor, its
// slant continued below the base circle): in the plane of the axis and the
// point, to the foot of the perpendicular on the slant line (+x on the
// axis).
__device__ __forceinline__ bool obstacle_project(const ObstacleDev &o, float &x, float &y, float &z)
{
    const float d0 = x - o.c[0], d1 = y - o.c[1], d2 = z - o.c[2];
    if (o.kind == PBF_OBSTACLE_SPHERE) {
        const float R = o.a[0];
        const float r2 = d0 * d0 + d1 * d1 + d2 * d2;
        if (!(r2 < R * R)) return false;
        if (r2 > 0.f) {
            const float s = R / sqrtf(r2);
            x = o.c[0] + s * d0;
            y = o.c[1] + s * d1;
            z = o.c[2] + s * d2;
        } else {
            y = o.c[1] + R;
        }
        return true;
    }
    if (o.kind == PBF_OBSTACLE_CONE) {
        const float R = o.a[0], H = o.a[1];
        float rho = sqrtf(d0 * d0 + d2 * d2), yb = d1;
        if (!(rho * H + yb * R < H * R)) return false;
        const float L = sqrtf(H * H + R * R);
        const float ds = (H * R - rho * H - yb * R) / L;  // distance to the slant line
        const float ux = rho > 0.f ? d0 / rho : 1.f, uz = rho > 0.f ? d2 / rho : 0.f;
        rho += ds * H / L;
        yb += ds * R / L;
        x = o.c[0] + rho * ux;
        y = o.c[1] + yb;
        z = o.c[2] + rho * uz;
        return true;
    }
    const float q0 = fabsf(d0) - o.a[0], q1 = fabsf(d1) - o.a[1], q2 = fabsf(d2) - o.a[2];
    if (!(q0 < 0.f && q1 < 0.f && q2 < 0.f)) return false;
    if (q0 >= q1 && q0 >= q2) x = o.c[0] + (d0 >= 0.f ? o.a[0] : -o.a[0]);
    else if (q1 >= q2) y = o.c[1] + (d1 >= 0.f ? o.a[1] : -o.a[1]);
    else z = o.c[2] + (d2 >= 0.f ? o.a[2] : -o.a[2]);
    return true;
}

// Contact response of an update: out of every found obstacle, in order.
__device__ __forceinline__ void contact_response(const SceneDev &S, uint32_t mask, float &x, float &y,
                                                 float &z)
{
    for (int o = 0; o < S.n_obst; ++o)
        if ((mask >> o) & 1u) obstacle_project(S.obst[o], x, y, z);
}

// Contact finding for every particle from its predicted position, then
// pre-stabilisation (Section 4.3, Fig. 6) of the particles with N_i <
// stab_s: x* of a particle inside a found obstacle goes to the obstacle's
// surface (clamped to the walls) and x moves by the same amount.  Runs after
// the neighbour search, which used x* before these moves (Fig. 7 order).
__global__ void k_contacts(int64_t n, const SceneDev *__restrict__ sc, float4 *__restrict__ x,
                           float4 *__restrict__ xs, const uint8_t *__restrict__ lvl,
                           uint8_t *__restrict__ contact)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const float4 xi = x[s];
    const SceneDev &S = sc[__float_as_int(xi.w)];
    float4 p = xs[s];
    uint32_t mask = 0;
    for (int o = 0; o < S.n_obst; ++o)
        if (contact_found(S.obst[o], p.x, p.y, p.z, S.h)) mask |= 1u << o;
    contact[s] = (uint8_t)mask;
    if (!mask || !((int)lvl[s] < S.stab_s)) return;
    float mx = 0.f, my = 0.f, mz = 0.f;
    bool moved = false;
    for (int it = 0; it < S.stab_iters; ++it)
        for (int o = 0; o < S.n_obst; ++o) {
            float qx = p.x, qy = p.y, qz = p.z;
            if (!((mask >> o) & 1u) || !obstacle_project(S.obst[o], qx, qy, qz)) continue;
            qx = clampf(qx, S.lo[0], S.hi[0]);
            qy = clampf(qy, S.lo[1], S.hi[1]);
            qz = clampf(qz, S.lo[2], S.hi[2]);
            mx += qx - p.x;
            my += qy - p.y;
            mz += qz - p.z;
            p.x = qx;
            p.y = qy;
            p.z = qz;
            moved = true;
        }
    if (!moved) return;
    xs[s] = p;
    x[s] = make_float4(xi.x + mx, xi.y + my, xi.z + mz, xi.w);
}


// ------------------------------------------------------------------ tiles
struct TileLoc {
    const SceneDev *S;
    int tx, ty, tz;
};

__device__ __forceinline__ TileLoc tile_locate(uint32_t tile, const uint32_t *__restrict__ tile_scene,
                                               const SceneDev *__restrict__ sc)
{
    TileLoc t;
    t.S = &sc[tile_scene[tile]];
    const uint32_t local = tile - t.S->tile_off;
    const uint32_t nx = (uint32_t)t.S->tiles[0], ny = (uint32_t)t.S->tiles[1];
    t.tx = (int)(local % nx);
    t.ty = (int)((local / nx) % ny);
    t.tz = (int)(local / (nx * ny));
    return t;
}

// The entry of tile_order that workgroup b handles when the first `active`
// entries are listed.  Workgroups are dealt to the XCDs round robin (b %
// kXcds), so each XCD is given one contiguous run of the list: tiles next to
// each other, whose LDS stages share halo cells, then meet in the same L2.
// False for workgroups past the list (the grid is rounded up to kXcds).
__device__ __forceinline__ bool xcd_slot(uint32_t b, uint32_t active, uint32_t &slot)
{
    const uint32_t per = (active + kXcds - 1) / kXcds;
    const uint32_t j = b / kXcds;
    slot = (b % kXcds) * per + j;
    return j < per && slot < active;
}

// Slot where staged cell x (0..kStageEdge; kStageEdge = end) of staged row
// (sy, sz) begins.  Staged cells run from one cell before the tile to one
// after it; cells left or right of the grid are empty ranges, and rows above,
// below, in front of or behind the grid are empty.
__device__ __forceinline__ uint32_t row_bound(const TileLoc &t, const uint32_t *__restrict__ cell_start,
                                              int sy, int sz, int x)
{
    const SceneDev &S = *t.S;
    const int cy = t.ty * kTileEdge - 1 + sy, cz = t.tz * kTileEdge - 1 + sz;
    if (cy < 0 || cy >= S.dims[1] || cz < 0 || cz >= S.dims[2]) return 0u;
    const int cx = min(max(t.tx * kTileEdge - 1 + x, 0), S.dims[0]);
    return cell_start[S.cell_off + ((uint32_t)cz * (uint32_t)S.dims[1] + (uint32_t)cy) *
                                       (uint32_t)S.dims[0] + (uint32_t)cx];
}

// LDS tables of one tile: cell bounds of the 36 staged rows, LDS offset of
// each row, and the prefix of own particles over the 16 own rows.
struct TileTables {
    uint32_t bnd[kStageRows][kStageEdge + 1];
    uint32_t base[kStageRows + 1];
    uint32_t own[kOwnRows + 1];
};

// fills tb (all threads call; ends with a barrier); returns whether the stage fits in LDS
__device__ bool tile_tables(const TileLoc &t, const uint32_t *__restrict__ cell_start, TileTables &tb)
{
    for (int e = threadIdx.x; e < kStageRows * (kStageEdge + 1); e += blockDim.x) {
        const int r = e / (kStageEdge + 1), x = e % (kStageEdge + 1);
        tb.bnd[r][x] = row_bound(t, cell_start, r % kStageEdge, r / kStageEdge, x);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int r = 0; r < kStageRows; ++r) {
            tb.base[r] = run;
            run += tb.bnd[r][kStageEdge] - tb.bnd[r][0];
        }
        tb.base[kStageRows] = run;
        run = 0;
        for (int o = 0; o < kOwnRows; ++o) {
            const int r = (1 + o / kTileEdge) * kStageEdge + 1 + o % kTileEdge;
            tb.own[o] = run;
            run += tb.bnd[r][kTileEdge + 1] - tb.bnd[r][1];
        }
        tb.own[kOwnRows] = run;
    }
    __syncthreads();
    return tb.base[kStageRows] <= (uint32_t)kStageCap;
}

// copy the staged rows of `src` into LDS, plus the far-away entry at
// kFarCode that pads neighbour groups (all threads; ends with a barrier).
// Wave w copies rows w, w + nw, ...: every 64-entry piece of a row is one
// global-to-LDS load (gfx950 global_load_lds_dwordx4: lane L of the piece
// lands 16 L bytes past the piece's LDS base), all of a wave's pieces are
// issued before it waits once, and no data passes through registers.  The
// caller has checked that the rows fit (tb.base[kStageRows] <= kStageCap),
// so every written entry lies inside the stage.
using lds_void = __attribute__((address_space(3))) void;
__device__ __forceinline__ void tile_stage(const TileTables &tb, const float4 *__restrict__ src,
                                           float4 *__restrict__ stage)
{
    const uint32_t lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (threadIdx.x == 0) stage[kFarCode] = make_float4(kFar, kFar, kFar, 0.f);
    for (int r = wave; r < kStageRows; r += nw) {
        const uint32_t g0 = tb.bnd[r][0], len = tb.bnd[r][kStageEdge] - g0, b0 = tb.base[r];
        for (uint32_t c = 0; c < len; c += 64) {
            if (c + lane < len)
                __builtin_amdgcn_global_load_lds(static_cast<const void *>(src + g0 + c + lane),
                                                 (lds_void *)(stage + b0 + c), 16, 0, 0);
        }
    }
    __builtin_amdgcn_s_waitcnt(0);  // this wave's pieces are in LDS
    __syncthreads();
}

// Own particles and largest level of every tile: one wave per tile.
__global__ void k_tile_prepare(uint32_t n_tiles, const SceneDev *__restrict__ sc,
                               const uint32_t *__restrict__ tile_scene,
                               const uint32_t *__restrict__ cell_start,
                               const uint8_t *__restrict__ lvl, uint32_t *__restrict__ tile_count,
                               uint8_t *__restrict__ tile_lvl)
{
    const int lane = threadIdx.x & 63;
    const uint32_t tile = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (tile >= n_tiles) return;  // whole wave leaves together
    const TileLoc t = tile_locate(tile, tile_scene, sc);
    uint32_t a = 0, b = 0;
    if (lane < kOwnRows) {
        const int sy = 1 + lane % kTileEdge, sz = 1 + lane / kTileEdge;
        a = row_bound(t, cell_start, sy, sz, 1);
        b = row_bound(t, cell_start, sy, sz, kTileEdge + 1);
    }
    const uint32_t count = wave_sum(b - a);
    // kPrepLanes lanes per own row, each taking every kPrepLanes-th particle
    // of it, with eight loads issued together (longer rows take another round)
    constexpr int kPrepLanes = 64 / kOwnRows;
    static_assert(kPrepLanes >= 1, "an own row per lane at least");
    const int o = min(lane / kPrepLanes, kOwnRows - 1);
    const uint32_t ao = __shfl(a, o, 64), bsh = __shfl(b, o, 64);
    const uint32_t bo = lane < kOwnRows * kPrepLanes ? bsh : ao;
    uint32_t mx = 0;
    for (uint32_t e0 = ao + (uint32_t)(lane % kPrepLanes); e0 < bo; e0 += 8 * kPrepLanes) {
        uint32_t v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q)
            v[q] = e0 + kPrepLanes * q < bo ? (uint32_t)lvl[e0 + kPrepLanes * q] : 0u;
#pragma unroll
        for (int q = 0; q < 8; ++q) mx = max(mx, v[q]);
    }
    mx = wave_max(mx);
    if (lane == 0) {
        tile_count[tile] = count;
        tile_lvl[tile] = (uint8_t)(count ? mx : 0u);
    }
}

// ------------------------------------------------------- level buckets
// Stable bucketing of tiles by descending level 0..K (the active sets nest,
// Eqs. 9-10, so one bucketing per step makes the tiles with active particles
// of every iteration a prefix).  counts: [(K - L) * nb + block].
__global__ void k_level_count(uint32_t m, const uint8_t *__restrict__ lvl,
                              uint32_t *__restrict__ counts, int nb, int K)
{
    __shared__ uint32_t hist[PBF_MAX_ITERS + 1];
    for (int i = threadIdx.x; i <= K; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    const uint32_t s = blockIdx.x * kLevelBlock + threadIdx.x;
    if (s < m) atomicAdd(&hist[lvl[s]], 1u);
    __syncthreads();
    for (int L = threadIdx.x; L <= K; L += blockDim.x)
        counts[(size_t)(K - L) * nb + blockIdx.x] = hist[L];
}

// single workgroup: exclusive scan of the bucket counts; ge[L] = number of
// items with level >= L for L = 0..K+1; also counts the steps.
__global__ void k_level_scan(uint32_t *__restrict__ counts, int nb, int K,
                             uint32_t *__restrict__ ge, const uint32_t *__restrict__ level_part,
                             uint32_t n_part, unsigned long long *__restrict__ totals)
{
    __shared__ uint32_t lds[1024 / 64 + 1];
    const uint32_t M = (uint32_t)nb * (uint32_t)(K + 1);
    uint32_t carry = 0;
    for (uint32_t b0 = 0; b0 < M; b0 += blockDim.x) {
        const uint32_t i = b0 + threadIdx.x;
        const uint32_t v = i < M ? counts[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_exclusive_sum(v, lds, &tot);
        if (i < M) counts[i] = carry + ex;
        carry += tot;
    }
    // running count of particle-iterations (sum_i N_i) and of steps
    uint32_t part = 0;
    for (uint32_t e = threadIdx.x; e < n_part; e += blockDim.x) part += level_part[e];
    part = wave_sum(part);
    __shared__ uint32_t psum[1024 / 64];
    if ((threadIdx.x & 63) == 0) psum[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
        ge[0] = carry;
        ge[K + 1] = 0;
        unsigned long long pit = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) pit += psum[w];
        totals[0] += pit;
        totals[1] += 1ull;
    }
    for (int L = 1 + threadIdx.x; L <= K; L += blockDim.x)
        ge[L] = counts[(size_t)(K - L + 1) * nb];
}

// Rank of each item among equal levels inside its wave by ballots, then
// across the block's waves, then the bucket offset of the block.
__global__ void k_level_scatter(uint32_t m, const uint8_t *__restrict__ lvl,
                                const uint32_t *__restrict__ offs, int nb, int K,
                                uint32_t *__restrict__ order)
{
    __shared__ uint32_t wc[kLevelBlock / 64][PBF_MAX_ITERS + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < (kLevelBlock / 64) * (PBF_MAX_ITERS + 1); i += blockDim.x)
        (&wc[0][0])[i] = 0;
    __syncthreads();
    const uint32_t s = blockIdx.x * kLevelBlock + threadIdx.x;
    const bool valid = s < m;
    const int L = valid ? (int)lvl[s] : 0;
    uint64_t rem = __ballot(valid);
    uint32_t rank = 0;
    while (rem) {
        const int leader = __ffsll((unsigned long long)rem) - 1;
        const int L0 = __shfl(L, leader, 64);
        const uint64_t mm = __ballot(valid && L == L0);
        if (valid && L == L0) rank = (uint32_t)__popcll(mm & ((1ull << lane) - 1ull));
        if (lane == leader) wc[wave][L0] = (uint32_t)__popcll(mm);
        rem &= ~mm;
    }
    __syncthreads();
    if (valid) {
        uint32_t base = 0;
        for (int w = 0; w < wave; ++w) base += wc[w][L];
        order[offs[(size_t)(K - L) * nb + blockIdx.x] + base + rank] = s;
    }
}

// One workgroup of 1024 threads for contexts with few tiles (T <=
// kFusedTiles): the exclusive scan of the tile counts, the stable bucketing
// of the tiles by descending level with the prefix counts ge[L] (tiles with
// level >= L), and the running totals -- what k_scan_* and k_level_* do in
// six launches.  The order is the same: descending level, ties by tile index.
// Each wave owns a contiguous chunk of tiles, held in registers: it scans
// the counts and ranks the levels of its chunk by itself (lane L keeps the
// running count of level L), so the waves meet at one barrier only.
constexpr int kTableWaves = 16;                                  // 1024 threads
constexpr int kTablePer = kFusedTiles / (kTableWaves * 64);      // tiles per lane, at most
__global__ __launch_bounds__(1024) void k_tile_tables(
    uint32_t T, int K, const uint32_t *__restrict__ tile_count, const uint8_t *__restrict__ tile_lvl,
    uint32_t *__restrict__ tile_start, uint32_t *__restrict__ order, uint32_t *__restrict__ ge,
    const uint32_t *__restrict__ level_part, uint32_t n_part,
    unsigned long long *__restrict__ totals)
{
    __shared__ uint32_t wlev[kTableWaves][PBF_MAX_ITERS + 1];  // per wave: tiles per level
    __shared__ uint32_t wown[kTableWaves];                     // per wave: own particles
    __shared__ uint32_t wpit[kTableWaves];                     // per wave: particle-iterations
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t J = (T + kTableWaves * 64 - 1) / (kTableWaves * 64);  // rounds of 64 per wave
    const uint32_t t0 = (uint32_t)wave * J * 64u;                        // first tile of the chunk
    // every global load first
    uint32_t cnt[kTablePer];
    int lv[kTablePer];  // -1: past the last tile
#pragma unroll
    for (int r = 0; r < kTablePer; ++r) {
        const uint32_t s = t0 + (uint32_t)r * 64u + (uint32_t)lane;
        const bool ok = (uint32_t)r < J && s < T;
        cnt[r] = ok ? tile_count[s] : 0u;
        lv[r] = ok ? (int)tile_lvl[s] : -1;
    }
    uint32_t part = 0;
    for (uint32_t e = threadIdx.x; e < n_part; e += blockDim.x) part += level_part[e];
    // the chunk's exclusive count scan and level ranks
    uint32_t cex[kTablePer], rk[kTablePer];
    uint32_t run = 0, lrun = 0;  // particles so far (uniform); tiles of level `lane` so far
#pragma unroll
    for (int r = 0; r < kTablePer; ++r) {
        if ((uint32_t)r >= J) break;
        uint32_t inc = cnt[r];
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t u = __shfl_up(inc, o, 64);
            if (lane >= o) inc += u;
        }
        cex[r] = run + inc - cnt[r];
        run += __shfl(inc, 63, 64);
        const int L = lv[r];
        rk[r] = 0;
        uint64_t rem = __ballot(L >= 0);
        while (rem) {
            const int leader = __ffsll((unsigned long long)rem) - 1;
            const int L0 = __shfl(L, leader, 64);
            const uint64_t mm = __ballot(L == L0);
            const uint32_t base = __shfl(lrun, L0, 64);
            if (L == L0) rk[r] = base + (uint32_t)__popcll(mm & ((1ull << lane) - 1ull));
            if (lane == L0) lrun += (uint32_t)__popcll(mm);
            rem &= ~mm;
        }
    }
    part = wave_sum(part);
    if (lane <= K) wlev[wave][lane] = lrun;
    if (lane == 0) {
        wown[wave] = run;
        wpit[wave] = part;
    }
    __syncthreads();
    // level `lane`: tiles in all waves and in the waves before this one;
    // particles before this wave's chunk
    uint32_t tot = 0, pre = 0, own_pre = 0, own_tot = 0;
#pragma unroll
    for (int w = 0; w < kTableWaves; ++w) {
        const uint32_t c = lane <= K ? wlev[w][lane] : 0u;
        const uint32_t o = wown[w];
        tot += c;
        own_tot += o;
        if (w < wave) {
            pre += c;
            own_pre += o;
        }
    }
    // tiles of higher levels: a suffix sum over the lanes
    uint32_t suf = tot;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_down(suf, o, 64);
        if (lane + o < 64) suf += u;
    }
    const uint32_t above = suf - tot;  // first position of level `lane`
    if (wave == 0 && lane <= K + 1) ge[lane] = lane <= K ? suf : 0u;
    const uint32_t first = above + pre;  // this wave's first position of level `lane`
#pragma unroll
    for (int r = 0; r < kTablePer; ++r) {
        if ((uint32_t)r >= J) break;
        const int L = lv[r];
        const uint32_t f = __shfl(first, L >= 0 ? L : 0, 64);
        if (L >= 0) {
            const uint32_t s = t0 + (uint32_t)r * 64u + (uint32_t)lane;
            order[f + rk[r]] = s;
            tile_start[s] = own_pre + cex[r];
        }
    }
    if (threadIdx.x == 0) {
        tile_start[T] = own_tot;
        unsigned long long pit = 0;
#pragma unroll
        for (int w = 0; w < kTableWaves; ++w) pit += wpit[w];
        totals[0] += pit;  // running count of particle-iterations (sum_i N_i)
        totals[1] += 1ull;
    }
}

// Order of the own particles of a tile part in p (the order of the solver
// passes): by descending level, ties in cell order.  The active particles
// of every iteration then form a prefix of the part (Eqs. 9-10), so
// finished particles leave whole waves idle rather than single lanes.  Each
// particle's sums keep their neighbour-list order, so no result depends on
// this order.
//
// A stable counting sort by level, before the stage is loaded (its LDS is
// the scratch): each wave counts the levels of each round of blockDim.x
// particles by ballots, and a particle's rank is the number of particles
// of higher level in the part, plus those of its level in earlier rounds
// and waves, plus those below it in its wave.  Parts of more than kRankHold
// * blockDim.x particles keep cell order.
constexpr int kRankHold = 4;  // particles per thread that carry a rank
constexpr int kRankWaves = kNbrThreads / 64;
constexpr int kRankLevels = PBF_MAX_ITERS + 1;
struct RankLds {
    uint32_t count[kRankHold][kRankWaves][kRankLevels];  // particles per round, wave and level
    uint32_t above[kRankLevels];  // particles of the part with a higher level
};

// Slot of own particle pl of a tile (cell order) and its staged row.
__device__ __forceinline__ uint32_t own_slot(const TileTables &tb, uint32_t pl, int &row)
{
    int o = 0;
    while (tb.own[o + 1] <= pl) ++o;
    row = (1 + o / kTileEdge) * kStageEdge + (1 + o % kTileEdge);
    return tb.bnd[row][1] + (pl - tb.own[o]);
}

// rank[q]: position in the part of own particle first + threadIdx.x + q *
// blockDim.x (all threads call; ends with a barrier).
__device__ void rank_part(RankLds &L, const TileTables &tb, uint32_t first, uint32_t m,
                          const uint8_t *__restrict__ lvl, uint32_t (&rank)[kRankHold])
{
    const uint32_t bd = blockDim.x, t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6, nw = (int)(bd >> 6);
    const int rounds = (int)((m + bd - 1) / bd);  // <= kRankHold
    for (uint32_t e = t; e < (uint32_t)(kRankHold * kRankWaves * kRankLevels); e += bd)
        (&L.count[0][0][0])[e] = 0u;
    __syncthreads();
    int lv[kRankHold];
#pragma unroll
    for (int q = 0; q < kRankHold; ++q) {
        const uint32_t e = t + (uint32_t)q * bd;
        int row;
        lv[q] = e < m ? (int)lvl[own_slot(tb, first + e, row)] : -1;
        rank[q] = 0;
        if (q >= rounds) continue;  // uniform
        // rank inside the wave among equal levels; the lowest lane of each level counts
        uint64_t rem = __ballot(lv[q] >= 0);
        while (rem) {
            const int f = __ffsll((unsigned long long)rem) - 1;
            const int l0 = __shfl(lv[q], f, 64);
            const uint64_t mm = __ballot(lv[q] == l0);
            if (lv[q] == l0) rank[q] = (uint32_t)__popcll(mm & ((1ull << lane) - 1ull));
            if (lane == f) L.count[q][wave][l0] = (uint32_t)__popcll(mm);
            rem &= ~mm;
        }
    }
    __syncthreads();
    if (t < (uint32_t)kRankLevels) {  // particles of each level in the part, then those above it
        uint32_t tot = 0;
        for (int q = 0; q < rounds; ++q)
            for (int w = 0; w < nw; ++w) tot += L.count[q][w][t];
        uint32_t suf = tot;  // suffix sum over the levels (lanes 0..32 of wave 0)
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t u = __shfl_down(suf, o, 64);
            if (lane + o < kRankLevels) suf += u;
        }
        L.above[t] = suf - tot;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kRankHold; ++q) {
        if (lv[q] < 0) continue;
        uint32_t r = L.above[lv[q]] + rank[q];
        for (int q2 = 0; q2 <= q; ++q2)
            for (int w = 0; w < (q2 < q ? nw : wave); ++w) r += L.count[q2][w][lv[q]];
        rank[q] = r;
    }
    __syncthreads();  // the stage may overwrite the tables now
}

// ------------------------------------------------------ neighbour lists
// N_i = { j != i : |x*_i - x*_j|^2 < h^2 } over the 27 cells around x*_i
// (Fig. 7 second loop), kept for every iteration of the step.  The 27 cells
// are nine x-contiguous windows of three cells (rows dz, dy in {-1, 0, 1},
// cells lx-1..lx+1) of the tile's LDS stage.  A neighbour is stored as a
// 16-bit code: its index in the stage, or row << 10 | offset in the row when
// the stage did not fit in LDS.  Codes are packed eight to a 16-byte group,
// groups stored group-major (nbr[g * n + p]): one store per eight
// neighbours here, fully coalesced loads in the solver passes.
// The neighbour list of every own particle of one tile.  FITS: the stage is
// in LDS and codes are stage indices; the unused codes of a particle's last
// group point at the stage's far-away entry, so the solver passes read whole
// groups without tests.
//
// Each window is scanned in chunks of 32 candidates, four candidates per
// round (their loads issued together) into a 32-bit hit mask; the hits then
// become codes in candidate order, each stored as a 16-bit value into its
// slot of the particle's current 16-byte group.
template <bool FITS>
__device__ __forceinline__ uint32_t tile_neighbours(const TileTables &tb, const float4 *__restrict__ stage,
                                                    const float4 *__restrict__ xs, float h2, uint32_t p0,
                                                    int64_t n, int cap, const uint8_t *__restrict__ lvl,
                                                    uint4 *__restrict__ nbr, uint32_t *__restrict__ pmeta,
                                                    uint32_t *__restrict__ pslot, uint32_t first,
                                                    uint32_t last, uint32_t rank01, uint32_t rank23)
{
    uint32_t bad = 0;
    uint32_t q = 0;
    for (uint32_t pl = first + threadIdx.x; pl < last; pl += blockDim.x, ++q) {
        int r;
        const uint32_t i = own_slot(tb, pl, r);
        const int sy = r % kStageEdge, sz = r / kStageEdge;
        // position in the part: its rank (see rank_part), two 16-bit ranks
        // per word for the thread's first four particles
        const uint32_t pr = q < 2u ? ((q ? rank01 >> 16 : rank01) & 0xffffu)
                            : q < 4u ? ((q & 1u ? rank23 >> 16 : rank23) & 0xffffu)
                                     : pl - first;
        int lx = 1;
        while (lx < kTileEdge && tb.bnd[r][lx + 1] <= i) ++lx;  // x-cell of i, 1..kTileEdge
        const float4 xi = FITS ? stage[tb.base[r] + (i - tb.bnd[r][0])] : xs[i];
        // LDS path: the stage holds positions relative to the block's centre
        // with |x|^2 in .w, so |x_i - x_j|^2 - h^2 = |x_j|^2 + (|x_i|^2 - h^2)
        // - 2 x_i.x_j: one add and three FMAs per candidate.  Staged
        // positions lie within 3 h of the centre on each axis, so |x|^2 <=
        // 27 h^2 and the expanded form's rounding stays near 1e-5 of h^2:
        // only pairs at the radius to that precision can be decided
        // differently from the direct form.
        const float ax = -2.f * xi.x, ay = -2.f * xi.y, az = -2.f * xi.z, ci = xi.w - h2;
        const size_t p = (size_t)p0 + first + pr;

        const uint32_t room = ((uint32_t)cap + 7u) >> 3;  // groups that have room
        // The particle's current group of eight codes is built in four
        // registers: each code enters at the top and the group shifts down by
        // 16 bits, so after the eighth the first code found sits in the low
        // half of the first word, the order of the stored u16 array.  A full
        // group is written with one 16-byte store, the particle's next group
        // n groups further on: one write request per eight codes instead of
        // one per code, which bound the build when each 16-bit code was
        // stored as it was found.
        // free: slots left in the current group (8..1); full: groups completed
        uint32_t w0 = 0, w1 = 0, w2 = 0, w3 = 0, free = 8, full = 0;
        auto put = [&](uint32_t code) {
            w0 = __builtin_amdgcn_alignbit(w1, w0, 16);
            w1 = __builtin_amdgcn_alignbit(w2, w1, 16);
            w2 = __builtin_amdgcn_alignbit(w3, w2, 16);
            w3 = __builtin_amdgcn_alignbit(code, w3, 16);
            if (--free == 0u) {
                if (full < room) nbr[p + (size_t)full * (size_t)n] = make_uint4(w0, w1, w2, w3);
                ++full;
                free = 8;
            }
        };
#pragma unroll 1
        for (int win = 0; win < 9; ++win) {
            const int r2 = (sz + win / 3 - 1) * kStageEdge + (sy + win % 3 - 1);
            const uint32_t g0 = tb.bnd[r2][0];
            const uint32_t ja = tb.bnd[r2][lx - 1], len = tb.bnd[r2][lx + 2] - ja;
            const uint32_t l0 = tb.base[r2] + (ja - g0);
            for (uint32_t c0 = 0; c0 < len; c0 += 32) {
                // distance test of up to 32 candidates into a bit mask: the
                // sign of |d|^2 - h^2 (h^2 folded into the first FMA) is
                // shifted into the mask, one instruction per candidate, so
                // the candidate tested last sits in bit 0 ...
                const uint32_t cl = min(len - c0, 32u);
                uint32_t m = 0;
                for (uint32_t c = 0; c < cl; c += 4) {
                    float4 xj[4];
                    // past the window's end: other stage entries (the stage has
                    // kStageSlack spare entries past the far entry), masked below
                    const float4 *sp = stage + (l0 + c0 + c);
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        xj[u] = FITS ? sp[u] : xs[min((int64_t)(ja + c0 + c + u), n - 1)];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        float e;  // < 0: inside
                        if (FITS) {
                            e = fmaf(az, xj[u].z, fmaf(ay, xj[u].y, fmaf(ax, xj[u].x, xj[u].w + ci)));
                        } else {
                            const float dx = xi.x - xj[u].x, dy = xi.y - xj[u].y, dz = xi.z - xj[u].z;
                            e = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, -h2)));
                        }
                        m = __builtin_amdgcn_alignbit(m, __float_as_uint(e), 31);
                    }
                }
                // ... and reversed, so that candidate c is bit c
                const uint32_t tested = (cl + 3u) & ~3u;
                m = __builtin_bitreverse32(m) >> (32u - tested);
                if (cl < 32u) m &= (1u << cl) - 1u;
                if (ja + c0 <= i && i < ja + c0 + cl) m &= ~(1u << (i - ja - c0));  // not itself
                // ... then its hits become codes, in candidate order
                while (m) {
                    const uint32_t c = c0 + (uint32_t)(__ffs(m) - 1);
                    m &= m - 1u;
                    if (FITS) {
                        put(l0 + c);
                    } else {
                        const uint32_t off = ja + c - g0;
                        if (off >= (1u << kSegOffBits)) bad |= ERR_CELL_CAP;
                        put(((uint32_t)r2 << kSegOffBits) | (off & ((1u << kSegOffBits) - 1)));
                    }
                }
            }
        }
        uint32_t cnt = 8u * full + (8u - free);
        if (cnt > (uint32_t)cap) {
            bad |= ERR_NEIGHBOUR_CAP;
            cnt = (uint32_t)cap & ~7u;  // only whole stored groups are valid
        } else if (free != 8u) {
            // complete and store the last group: on the LDS path its unused
            // codes name the far-away entry (the HBM path reads only cnt codes)
            while (free != 8u) put(FITS ? kFarCode : 0u);
        }
        pslot[p] = i;
        pmeta[p] = make_meta(cnt, lvl[i], FITS ? tb.base[r] + (i - tb.bnd[r][0]) : 0u);
    }
    return bad;
}

template <bool SPLIT>
__global__ __launch_bounds__(kNbrThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_neighbours(
    const SceneDev *__restrict__ sc, const uint32_t *__restrict__ tile_scene,
    const uint32_t *__restrict__ tile_order, const uint32_t *__restrict__ tile_ge,
    const uint32_t *__restrict__ tile_start, const uint32_t *__restrict__ cell_start,
    const float4 *__restrict__ xs, const uint8_t *__restrict__ lvl, int64_t n, int cap,
    uint4 *__restrict__ nbr, uint32_t *__restrict__ pmeta, uint32_t *__restrict__ pslot,
    const uint32_t *__restrict__ tile_count, uint32_t *__restrict__ rows,
    uint32_t *__restrict__ err, uint32_t tx, uint4 *__restrict__ tile_rec)
{
    __shared__ TileTables tb;
    __shared__ float4 stage[kStageEntries];
    uint32_t slot;
    if (!xcd_slot(SPLIT ? blockIdx.x % tx : blockIdx.x, tile_ge[1], slot)) return;  // empty tiles last
    const uint32_t tile = tile_order[slot];
    uint32_t first = 0, last = 0;
    if (SPLIT && !split_part(tile_count[tile], blockIdx.x / tx, gridDim.x / tx, first, last)) return;
    const TileLoc t = tile_locate(tile, tile_scene, sc);
    const bool fits = tile_tables(t, cell_start, tb);
    if (!SPLIT) last = tb.own[kOwnRows];
    // keep the tables and the tile's record for the solver passes of this
    // step, at the tile's slot in tile_order (their first loads)
    if (first == 0) {
        for (int e = threadIdx.x; e < kRowWords; e += blockDim.x)
            rows[(size_t)slot * kRowWords + e] = e < kBndWords ? (&tb.bnd[0][0])[e] : tb.base[e - kBndWords];
        if (threadIdx.x == 0)
            tile_rec[slot] = make_uint4(tile, tile_start[tile], SPLIT ? tile_count[tile] : tb.own[kOwnRows],
                                        tile_scene[tile]);
    }
    const float h2 = t.S->h2;
    const uint32_t p0 = tile_start[tile];
    // positions of the own particles in the part (uniform condition); the
    // stage array is the scratch of the ranking until it is loaded
    uint32_t rank[kRankHold];
    const uint32_t m = last - first;
    if (m > 1u && m <= (uint32_t)kRankHold * blockDim.x) {
        static_assert(sizeof(RankLds) <= sizeof(stage), "ranking tables fit in the stage array");
        rank_part(*reinterpret_cast<RankLds *>(stage), tb, first, m, lvl, rank);
    } else {
#pragma unroll
        for (int q = 0; q < kRankHold; ++q) rank[q] = threadIdx.x + (uint32_t)q * blockDim.x;
    }
    static_assert(kRankHold == 4 && kRankHold * kNbrThreads <= 65536, "ranks packed two per word");
    const uint32_t rank01 = rank[0] | (rank[1] << 16), rank23 = rank[2] | (rank[3] << 16);
    uint32_t bad;
    if (fits) {
        tile_stage(tb, xs, stage);
        // positions relative to the centre of the staged block, with their
        // squared length in .w, for the expanded distance test
        const SceneDev &S = *t.S;
        const float c0 = S.lo[0] + (float)(t.tx * kTileEdge + kStageEdge / 2 - 1) * S.h;
        const float c1 = S.lo[1] + (float)(t.ty * kTileEdge + kStageEdge / 2 - 1) * S.h;
        const float c2 = S.lo[2] + (float)(t.tz * kTileEdge + kStageEdge / 2 - 1) * S.h;
        const uint32_t total = tb.base[kStageRows];
        for (uint32_t e = threadIdx.x; e < total; e += blockDim.x) {
            const float4 v = stage[e];
            const float rx = v.x - c0, ry = v.y - c1, rz = v.z - c2;
            stage[e] = make_float4(rx, ry, rz, fmaf(rz, rz, fmaf(ry, ry, rx * rx)));
        }
        __syncthreads();
        bad = tile_neighbours<true>(tb, stage, xs, h2, p0, n, cap, lvl, nbr, pmeta, pslot, first, last,
                                    rank01, rank23);
    } else {
        bad = tile_neighbours<false>(tb, stage, xs, h2, p0, n, cap, lvl, nbr, pmeta, pslot, first,
                                     last, rank01, rank23);
    }
    if (bad) atomicOr(err, bad);
}

// Tables of a tile saved by k_neighbours (cell bounds of the staged rows and
// their LDS offsets): load them and stage `src` (all threads; ends with a
// barrier); returns whether the stage fits in LDS.
__device__ __forceinline__ bool stage_rows(const uint32_t *__restrict__ rows, uint32_t slot,
                                           const float4 *__restrict__ src, TileTables &tb,
                                           float4 *__restrict__ stage)
{
    for (int e = threadIdx.x; e < kRowWords; e += blockDim.x) {
        const uint32_t w = rows[(size_t)slot * kRowWords + e];
        if (e < kBndWords) (&tb.bnd[0][0])[e] = w;
        else tb.base[e - kBndWords] = w;
    }
    __syncthreads();
    const bool fits = tb.base[kStageRows] <= (uint32_t)kStageCap;
    if (fits) tile_stage(tb, src, stage);
    return fits;
}

// The same in two parts, for words of the saved tables that each thread has
// already loaded (words threadIdx.x + q blockDim.x, see saved_row_words):
// the tables depend only on the slot, so their load can leave together with
// the tile's record.  put_rows stores them (before the caller issues loads
// that depend on the record, so that the wait covers only these words);
// stage_tables then stages `src` (all threads; ends with a barrier).
constexpr int kRowHold = (kRowWords + 63) / 64;  // words per thread at 64 threads
struct RowWords {
    uint32_t w[kRowHold];
};

__device__ __forceinline__ RowWords saved_row_words(const uint32_t *__restrict__ rows, uint32_t slot)
{
    RowWords r;
#pragma unroll
    for (int q = 0; q < kRowHold; ++q) {
        const uint32_t e = threadIdx.x + (uint32_t)q * blockDim.x;
        r.w[q] = e < (uint32_t)kRowWords ? rows[(size_t)slot * kRowWords + e] : 0u;
    }
    return r;
}

__device__ __forceinline__ void put_rows(const RowWords &r, TileTables &tb)
{
#pragma unroll
    for (int q = 0; q < kRowHold; ++q) {
        const uint32_t e = threadIdx.x + (uint32_t)q * blockDim.x;
        if (e < (uint32_t)kBndWords) (&tb.bnd[0][0])[e] = r.w[q];
        else if (e < (uint32_t)kRowWords) tb.base[e - kBndWords] = r.w[q];
    }
}

__device__ __forceinline__ bool stage_tables(const float4 *__restrict__ src, TileTables &tb,
                                             float4 *__restrict__ stage)
{
    __syncthreads();
    const bool fits = tb.base[kStageRows] <= (uint32_t)kStageCap;
    if (fits) tile_stage(tb, src, stage);
    return fits;
}

// Walk the neighbour list of particle p in stored order, calling f(position
// and lambda of the neighbour); codes are read eight at a time.  FITS: every
// code of a stored group is an LDS index (padding codes name the far-away
// entry, which no test admits); otherwise codes are row << 10 | offset into
// `src` and the tail of the last group is skipped.
template <bool FITS, class F>
__device__ __forceinline__ void for_each_neighbour(const TileTables &tb,
                                                   const float4 *__restrict__ stage,
                                                   const float4 *__restrict__ src,
                                                   const uint4 *__restrict__ nbr, int64_t n,
                                                   size_t p, uint32_t cnt, uint4 v, F &&f)
{
    // v holds group 0 (loaded by the caller); the next group's codes are
    // loaded while this group is evaluated; the index is clamped to the last
    // group (group 0 exists for every p), so every load is unconditional
    const uint32_t last = cnt ? (cnt - 1u) >> 3 : 0u;
    const uint32_t stride = (uint32_t)n;  // groups of one particle are n entries apart
    auto eval = [&](const uint4 &g, uint32_t q) {
        const uint32_t cc[8] = {g.x & 0xffffu, g.x >> 16, g.y & 0xffffu, g.y >> 16,
                                g.z & 0xffffu, g.z >> 16, g.w & 0xffffu, g.w >> 16};
        float4 xj[8];
        if (FITS) {
#pragma unroll
            for (int u = 0; u < 8; ++u) xj[u] = stage[cc[u]];
#pragma unroll
            for (int u = 0; u < 8; ++u) f(xj[u]);
        } else {
            const uint32_t m = min(cnt - q, 8u);
#pragma unroll
            for (int u = 0; u < 8; ++u)
                xj[u] = (uint32_t)u < m
                            ? src[tb.bnd[cc[u] >> kSegOffBits][0] + (cc[u] & ((1u << kSegOffBits) - 1))]
                            : make_float4(kFar, kFar, kFar, 0.f);
#pragma unroll
            for (int u = 0; u < 8; ++u) f(xj[u]);
        }
    };
    const uint4 *__restrict__ gp = nbr + p + (last ? stride : 0u);  // group min(1, last)
    for (uint32_t q = 0; q < cnt; q += 8) {
        const uint4 vn = *gp;
        gp += (q >> 3) + 2u <= last ? stride : 0u;
        const uint4 g = v;
        v = vn;
        eval(g, q);
    }
}

// ------------------------------------------------ solver iteration k
// Pair terms are evaluated without branches: outside the radius (and for the
// far-away padding entry) the clamped factors are zero.  1/r is the hardware
// reciprocal square root (about 1 ulp) of max(r^2, kTinyR2): coincident
// particles (r = 0, d = 0) then give a finite factor times d = 0, so no
// gradient, as for the exact kernel; distinct float32 positions are never
// that close.  The constant factor -c_grad of the spiky gradient is applied
// once per particle instead of once per pair.
constexpr float kTinyR2 = 1e-20f;

// A thread's first own particle: its metadata, slot and first code group,
// loaded before the tile's stage so that they arrive while it is staged.
struct Head {
    uint32_t meta, slot;
    uint4 g0;
};

__device__ __forceinline__ Head load_head(const uint32_t *__restrict__ pmeta,
                                          const uint32_t *__restrict__ pslot,
                                          const uint4 *__restrict__ nbr, uint32_t p0, uint32_t first,
                                          uint32_t last)
{
    Head hd{0u, 0u, make_uint4(0u, 0u, 0u, 0u)};
    const uint32_t pl = first + threadIdx.x;
    if (pl < last) {
        hd.meta = pmeta[p0 + pl];
        hd.slot = pslot[p0 + pl];
        hd.g0 = nbr[p0 + pl];
    }
    return hd;
}

// lambda_i for the active own particles of a tile (Eqs. 4-6)
// UNIT: h <= 1 (so h^2 - r^2 <= 1 and h - r <= 1), and the clamps at zero of
// the pair terms become the clamp to [0, 1] of the instruction producing
// them (one instruction less each).
template <bool UNIT>
__device__ __forceinline__ float pos_part(float v)
{
    return UNIT ? __builtin_amdgcn_fmed3f(v, 0.f, 1.f) : fmaxf(v, 0.f);
}

template <bool FITS, bool WIDE, bool UNIT>
__device__ __forceinline__ void tile_lambda(int k, const SceneDev &S, const TileTables &tb,
                                            const float4 *__restrict__ stage, float4 *__restrict__ xs,
                                            int64_t n, const uint4 *__restrict__ nbr,
                                            const uint32_t *__restrict__ pmeta,
                                            const uint32_t *__restrict__ pslot, uint32_t p0,
                                            uint32_t nown, uint32_t first, uint32_t last,
                                            const Head &hd)
{
    const float h = S.h, h2 = S.h2, cg = S.c_grad, h6 = S.h6, crho = S.c_rho, cs = S.c_s,
                eps = S.eps, cfloor = S.c_floor;
    for (uint32_t pl = first + threadIdx.x; pl < last; pl += blockDim.x) {
        const bool head = pl == first + threadIdx.x;
        const size_t p = p0 + pl;
        const uint32_t meta = head ? hd.meta : pmeta[p];
        const uint32_t i = head ? hd.slot : pslot[p];  // independent loads, issued together
        if ((int)meta_level(meta) <= k) continue;
        const float4 xi = FITS ? stage[meta_self(meta)] : xs[i];
        float sum6 = h6;  // the particle itself: (h^2 - 0)^3
        float gx = 0.f, gy = 0.f, gz = 0.f, g2 = 0.f;
        for_each_neighbour<FITS>(tb, stage, xs, nbr, n, p, meta & kMetaCount, head ? hd.g0 : nbr[p],
                                 [&](const float4 &xj) {
            // keep the 16-byte LDS read (an empty asm that takes .w): on
            // gfx950 random 12-byte reads conflict more than 16-byte ones
            // (measured 4% on this pass); the split variant would spill
            if (WIDE) asm volatile("" : : "v"(xj.w));
            const float dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
            const float r2 = dx * dx + dy * dy + dz * dz;
            const float w = pos_part<UNIT>(h2 - r2);
            sum6 += w * w * w;
            const float ir = __builtin_amdgcn_rsqf(fmaxf(r2, kTinyR2));
            const float hr = pos_part<UNIT>(h - r2 * ir);
            const float q = hr * hr * ir;  // grad W = -c_grad q d
            gx += q * dx;
            gy += q * dy;
            gz += q * dz;
            g2 += q * q * r2;
        });
        const float C = fmaxf(crho * sum6 - 1.f, cfloor);  // unilateral: C >= 0
        const float denom = cs * cg * cg * (gx * gx + gy * gy + gz * gz + g2) + eps;
        xs[i].w = -C / denom;
    }
}

// lambda_i of the tile's active particles, written to xs[i].w; neighbours
// read only xyz of the same buffer.
template <bool SPLIT>
__global__ __launch_bounds__(kTileThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_lambda(
    int k, const SceneDev *__restrict__ sc, const uint4 *__restrict__ tile_rec,
    const uint32_t *__restrict__ tile_ge, const uint32_t *__restrict__ rows, float4 *__restrict__ xs,
    int64_t n, const uint4 *__restrict__ nbr, const uint32_t *__restrict__ pmeta,
    const uint32_t *__restrict__ pslot, uint32_t tx)
{
    __shared__ TileTables tb;
    __shared__ float4 stage[kStageEntries];
    uint32_t slot;
    if (!xcd_slot(SPLIT ? blockIdx.x % tx : blockIdx.x, tile_ge[k + 1], slot)) return;  // active tiles
    const RowWords row_w = saved_row_words(rows, slot);
    const uint4 rec = tile_rec[slot];  // tile, first p, own particles, scene
    const SceneDev &S = sc[rec.w];
    const uint32_t p0 = rec.y, nown = rec.z;
    uint32_t first = 0, last = nown;
    if (SPLIT && !split_part(nown, blockIdx.x / tx, gridDim.x / tx, first, last)) return;
    put_rows(row_w, tb);
    const Head hd = load_head(pmeta, pslot, nbr, p0, first, last);
    if (!stage_tables(xs, tb, stage))
        tile_lambda<false, !SPLIT, false>(k, S, tb, stage, xs, n, nbr, pmeta, pslot, p0, nown, first, last, hd);
    else if (S.h <= 1.f)
        tile_lambda<true, !SPLIT, true>(k, S, tb, stage, xs, n, nbr, pmeta, pslot, p0, nown, first, last, hd);
    else
        tile_lambda<true, !SPLIT, false>(k, S, tb, stage, xs, n, nbr, pmeta, pslot, p0, nown, first, last, hd);
}

// Delta p_i (Eq. 7) with the wall contact (clamp) for the active own
// particles of a tile
template <bool FITS, bool CONTACTS, bool UNIT>
__device__ __forceinline__ void tile_update(int k, const SceneDev &S, const TileTables &tb,
                                            const float4 *__restrict__ stage,
                                            const float4 *__restrict__ xs_in,
                                            float4 *__restrict__ xs_out, int64_t n,
                                            const uint4 *__restrict__ nbr,
                                            const uint32_t *__restrict__ pmeta,
                                            const uint32_t *__restrict__ pslot,
                                            const uint8_t *__restrict__ contact, uint32_t p0,
                                            uint32_t nown, uint32_t first, uint32_t last,
                                            const Head &hd)
{
    const float h = S.h, cg = S.c_grad, sr = S.inv_rho0;
    const float lo0 = S.lo[0], lo1 = S.lo[1], lo2 = S.lo[2];
    const float hi0 = S.hi[0], hi1 = S.hi[1], hi2 = S.hi[2];
    for (uint32_t pl = first + threadIdx.x; pl < last; pl += blockDim.x) {
        const bool head = pl == first + threadIdx.x;
        const size_t p = p0 + pl;
        const uint32_t meta = head ? hd.meta : pmeta[p];
        const uint32_t i = head ? hd.slot : pslot[p];  // independent loads, issued together
        const int L = (int)meta_level(meta);
        if (L < k) continue;
        const float4 xi = FITS ? stage[meta_self(meta)] : xs_in[i];
        if (L == k) {
            xs_out[i] = xi;
            continue;
        }
        const float li = xi.w;
        float px = 0.f, py = 0.f, pz = 0.f;
        for_each_neighbour<FITS>(tb, stage, xs_in, nbr, n, p, meta & kMetaCount, head ? hd.g0 : nbr[p],
                                 [&](const float4 &xj) {
            const float dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
            const float r2 = dx * dx + dy * dy + dz * dz;
            const float ir = __builtin_amdgcn_rsqf(fmaxf(r2, kTinyR2));
            const float hr = pos_part<UNIT>(h - r2 * ir);
            const float f = hr * hr * ir * (li + xj.w);  // (lambda_i + lambda_j) grad W = -c_grad f d
            px += f * dx;
            py += f * dy;
            pz += f * dz;
        });
        const float s = -cg * sr;
        float nx = xi.x + px * s, ny = xi.y + py * s, nz = xi.z + pz * s;
        if (CONTACTS) {  // found obstacles first, then the walls
            const uint32_t m = contact[i];
            if (m) contact_response(S, m, nx, ny, nz);
        }
        xs_out[i] = make_float4(clampf(nx, lo0, hi0), clampf(ny, lo1, hi1), clampf(nz, lo2, hi2), li);
    }
}

// Corrections of the tile's active particles, written to the other buffer
// (Jacobi).  Particles that finished with this iteration (N_i == k) copy
// position and lambda across, so that both buffers hold their final values
// from now on.
template <bool SPLIT, bool CONTACTS>
__global__ __launch_bounds__(kTileThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_update(
    int k, const SceneDev *__restrict__ sc, const uint4 *__restrict__ tile_rec,
    const uint32_t *__restrict__ tile_ge, const uint32_t *__restrict__ rows,
    const float4 *__restrict__ xs_in, float4 *__restrict__ xs_out, int64_t n,
    const uint4 *__restrict__ nbr, const uint32_t *__restrict__ pmeta,
    const uint32_t *__restrict__ pslot, const uint8_t *__restrict__ contact, uint32_t tx)
{
    __shared__ TileTables tb;
    __shared__ float4 stage[kStageEntries];
    uint32_t slot;  // tiles with a particle of level >= k
    if (!xcd_slot(SPLIT ? blockIdx.x % tx : blockIdx.x, tile_ge[k > 1 ? k : 1], slot)) return;
    const bool copy_only = slot >= tile_ge[k + 1];  // the tile's highest level is k
    RowWords row_w{};
    if (!copy_only) row_w = saved_row_words(rows, slot);
    const uint4 rec = tile_rec[slot];  // tile, first p, own particles, scene
    const SceneDev &S = sc[rec.w];
    const uint32_t p0 = rec.y, nown = rec.z;
    uint32_t first = 0, last = nown;
    if (SPLIT && !split_part(nown, blockIdx.x / tx, gridDim.x / tx, first, last)) return;
    if (copy_only) {
        // its particles only copy across, so its neighbourhood is not staged
        for (uint32_t pl = first + threadIdx.x; pl < last; pl += blockDim.x) {
            const uint32_t meta = pmeta[p0 + pl], i = pslot[p0 + pl];
            if ((int)meta_level(meta) == k) xs_out[i] = xs_in[i];
        }
        return;
    }
    put_rows(row_w, tb);
    const Head hd = load_head(pmeta, pslot, nbr, p0, first, last);
    if (!stage_tables(xs_in, tb, stage))
        tile_update<false, CONTACTS, false>(k, S, tb, stage, xs_in, xs_out, n, nbr, pmeta, pslot, contact,
                                            p0, nown, first, last, hd);
    else if (S.h <= 1.f)
        tile_update<true, CONTACTS, true>(k, S, tb, stage, xs_in, xs_out, n, nbr, pmeta, pslot, contact,
                                          p0, nown, first, last, hd);
    else
        tile_update<true, CONTACTS, false>(k, S, tb, stage, xs_in, xs_out, n, nbr, pmeta, pslot, contact,
                                           p0, nown, first, last, hd);
}

// ------------------------------------------------ force-based cohesion
// The cohesion option's acceleration (see pbf_batch_set_cohesion) of every
// own particle of a tile, at the positions x at the start of the step (slot
// order, staged like x*) over the step's neighbour lists, applied to the
// prediction: x*_i += -c_coh sum_j P(r) d/r, P = (h - r)^3 r^3 (2 r > h) or
// 2 (h - r)^3 r^3 - h^6/64, clamped into the box.  Pair terms are
// branch-free: beyond h (and for the far-away padding entry) h - r clamps to
// zero, and coincident particles (d = 0) give zero.
template <bool FITS>
__device__ __forceinline__ void tile_cohesion(const SceneDev &S, const TileTables &tb,
                                              const float4 *__restrict__ stage,
                                              const float4 *__restrict__ x, float4 *__restrict__ xs,
                                              int64_t n, const uint4 *__restrict__ nbr,
                                              const uint32_t *__restrict__ pmeta,
                                              const uint32_t *__restrict__ pslot, uint32_t p0,
                                              uint32_t first, uint32_t last)
{
    const float h = S.h, half = 0.5f * S.h, q64 = S.h6 * (1.f / 64.f), c = S.c_coh;
    for (uint32_t pl = first + threadIdx.x; pl < last; pl += blockDim.x) {
        const size_t p = p0 + pl;
        const uint32_t meta = pmeta[p];
        const uint32_t i = pslot[p];  // independent loads, issued together
        const float4 xi = FITS ? stage[meta_self(meta)] : x[i];
        float ax = 0.f, ay = 0.f, az = 0.f;
        for_each_neighbour<FITS>(tb, stage, x, nbr, n, p, meta & kMetaCount, nbr[p], [&](const float4 &xj) {
            const float dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
            const float r2 = dx * dx + dy * dy + dz * dz;
            const float ir = __builtin_amdgcn_rsqf(fmaxf(r2, kTinyR2));
            const float r = r2 * ir;
            const float u = fmaxf(h - r, 0.f) * r;  // 0 beyond h (even for the far entry)
            const float t = u * u * u;
            const float P = r > half ? t : 2.f * t - q64;
            const float f = P * ir;
            ax += f * dx;
            ay += f * dy;
            az += f * dz;
        });
        const float4 s = xs[i];
        xs[i] = make_float4(clampf(s.x - c * ax, S.lo[0], S.hi[0]), clampf(s.y - c * ay, S.lo[1], S.hi[1]),
                            clampf(s.z - c * az, S.lo[2], S.hi[2]), s.w);
    }
}

template <bool SPLIT>
__global__ __launch_bounds__(kTileThreads) void k_cohesion(
    const SceneDev *__restrict__ sc, const uint4 *__restrict__ tile_rec,
    const uint32_t *__restrict__ tile_ge, const uint32_t *__restrict__ rows,
    const float4 *__restrict__ x, float4 *__restrict__ xs, int64_t n,
    const uint4 *__restrict__ nbr, const uint32_t *__restrict__ pmeta,
    const uint32_t *__restrict__ pslot, uint32_t tx)
{
    __shared__ TileTables tb;
    __shared__ float4 stage[kStageEntries];
    uint32_t slot;  // every tile with particles
    if (!xcd_slot(SPLIT ? blockIdx.x % tx : blockIdx.x, tile_ge[1], slot)) return;
    const uint4 rec = tile_rec[slot];  // tile, first p, own particles, scene
    const SceneDev &S = sc[rec.w];
    if (!(S.c_coh != 0.f)) return;  // uniform: scenes without cohesion
    const uint32_t p0 = rec.y, nown = rec.z;
    uint32_t first = 0, last = nown;
    if (SPLIT && !split_part(nown, blockIdx.x / tx, gridDim.x / tx, first, last)) return;
    if (stage_rows(rows, slot, x, tb, stage))
        tile_cohesion<true>(S, tb, stage, x, xs, n, nbr, pmeta, pslot, p0, first, last);
    else
        tile_cohesion<false>(S, tb, stage, x, xs, n, nbr, pmeta, pslot, p0, first, last);
}

// ------------------------------------------------ average density
// Cell keys and histogram tickets of the current positions (no prediction):
// the start of a fresh neighbour search for the density measure.
__global__ void k_density_keys(int64_t n, const SceneDev *__restrict__ sc,
                               const float4 *__restrict__ x, float4 *__restrict__ xs,
                               uint32_t *__restrict__ key, uint32_t *__restrict__ ticket,
                               uint32_t *__restrict__ cell_count)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = s < n;
    uint32_t k = 0xffffffffu;
    if (valid) {
        const float4 xi = x[s];
        const SceneDev &S = sc[__float_as_int(xi.w)];
        const int cx = cell_coord(xi.x, S.lo[0], S.h, S.dims[0]);
        const int cy = cell_coord(xi.y, S.lo[1], S.h, S.dims[1]);
        const int cz = cell_coord(xi.z, S.lo[2], S.h, S.dims[2]);
        k = S.cell_off + (uint32_t)(((int64_t)cz * S.dims[1] + cy) * S.dims[0] + cx);
        xs[s] = make_float4(xi.x, xi.y, xi.z, 0.f);
        key[s] = k;
    }
    const uint32_t tk = cell_ticket(k, valid, cell_count);
    if (valid) ticket[s] = tk;
}

// rho_i / rho0 (Eqs. 5-6, the particle itself included) of every particle at
// the positions after the last step, over neighbour sets found afresh at
// those positions (enqueue_density sorts and searches them anew); the
// quality measure of the paper's evaluation is the average over all
// particles.  Per workgroup: the sum (double, reduced in a fixed order) and
// the maximum; k_density_finish adds the workgroups up, again in a fixed
// order, so the result is deterministic.
template <bool FITS>
__device__ __forceinline__ void tile_density(const SceneDev &S, const TileTables &tb,
                                             const float4 *__restrict__ stage,
                                             const float4 *__restrict__ x, int64_t n,
                                             const uint4 *__restrict__ nbr,
                                             const uint32_t *__restrict__ pmeta,
                                             const uint32_t *__restrict__ pslot, uint32_t p0,
                                             uint32_t nown, float *__restrict__ rho, double &sum,
                                             float &mx)
{
    const float h2 = S.h2, h6 = S.h6, crho = S.c_rho;
    for (uint32_t pl = threadIdx.x; pl < nown; pl += blockDim.x) {
        const size_t p = p0 + pl;
        const uint32_t meta = pmeta[p];
        const uint32_t i = pslot[p];
        const float4 xi = FITS ? stage[meta_self(meta)] : x[i];
        float sum6 = h6;
        for_each_neighbour<FITS>(tb, stage, x, nbr, n, p, meta & kMetaCount, nbr[p], [&](const float4 &xj) {
            const float dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
            const float w = fmaxf(h2 - (dx * dx + dy * dy + dz * dz), 0.f);
            sum6 += w * w * w;
        });
        const float r = crho * sum6;
        rho[i] = r;
        sum += (double)r;
        mx = fmaxf(mx, r);
    }
}

__global__ __launch_bounds__(kTileThreads) void k_density(
    const SceneDev *__restrict__ sc, const uint4 *__restrict__ tile_rec,
    const uint32_t *__restrict__ tile_ge, const uint32_t *__restrict__ rows,
    const float4 *__restrict__ x, int64_t n, const uint4 *__restrict__ nbr,
    const uint32_t *__restrict__ pmeta, const uint32_t *__restrict__ pslot,
    float *__restrict__ rho, double *__restrict__ part_sum, float *__restrict__ part_max)
{
    __shared__ TileTables tb;
    __shared__ float4 stage[kStageEntries];
    __shared__ double dsum[kTileThreads / 64];
    __shared__ float dmax[kTileThreads / 64];
    double sum = 0.0;
    float mx = 0.f;
    uint32_t slot;
    if (xcd_slot(blockIdx.x, tile_ge[1], slot)) {  // uniform per workgroup
        const uint4 rec = tile_rec[slot];  // tile, first p, own particles, scene
        const SceneDev &S = sc[rec.w];
        const uint32_t p0 = rec.y, nown = rec.z;
        if (stage_rows(rows, slot, x, tb, stage))
            tile_density<true>(S, tb, stage, x, n, nbr, pmeta, pslot, p0, nown, rho, sum, mx);
        else
            tile_density<false>(S, tb, stage, x, n, nbr, pmeta, pslot, p0, nown, rho, sum, mx);
    }
    // fixed-order reduction: lanes by a butterfly, then waves in order
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        sum += __shfl_xor(sum, o, 64);
        mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        dsum[threadIdx.x >> 6] = sum;
        dmax[threadIdx.x >> 6] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        float m = 0.f;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            s += dsum[w];
            m = fmaxf(m, dmax[w]);
        }
        part_sum[blockIdx.x] = s;
        part_max[blockIdx.x] = m;
    }
}

// one workgroup: out[0] = sum of the parts / n, out[1] = their maximum
__global__ __launch_bounds__(1024) void k_density_finish(uint32_t parts, int64_t n,
                                                        const double *__restrict__ part_sum,
                                                        const float *__restrict__ part_max,
                                                        double *__restrict__ out)
{
    __shared__ double dsum[1024 / 64];
    __shared__ float dmax[1024 / 64];
    double sum = 0.0;
    float mx = 0.f;
    for (uint32_t e = threadIdx.x; e < parts; e += blockDim.x) {
        sum += part_sum[e];
        mx = fmaxf(mx, part_max[e]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        sum += __shfl_xor(sum, o, 64);
        mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        dsum[threadIdx.x >> 6] = sum;
        dmax[threadIdx.x >> 6] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        float m = 0.f;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            s += dsum[w];
            m = fmaxf(m, dmax[w]);
        }
        out[0] = n ? s / (double)n : 0.0;
        out[1] = (double)m;
    }
}

// out[id] = v[s] for a per-slot float
__global__ void k_unpermute_scalar(int64_t n, const float *__restrict__ v,
                                   const uint32_t *__restrict__ id, float *__restrict__ out)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) out[id[s]] = v[s];
}

// --------------------------------------------- velocity and position update
// Each thread takes kCommitPer slots, blockDim.x apart, loaded together.
constexpr int kCommitPer = 2;

__global__ void k_commit(int64_t n, const SceneDev *__restrict__ sc, float4 *__restrict__ x,
                         float4 *__restrict__ v, const float4 *__restrict__ xs,
                         uint32_t *__restrict__ err)
{
    const int64_t base = (int64_t)blockIdx.x * blockDim.x * kCommitPer + threadIdx.x;
    float4 xi[kCommitPer], p[kCommitPer];
#pragma unroll
    for (int q = 0; q < kCommitPer; ++q) {
        const int64_t s = base + (int64_t)q * blockDim.x;
        if (s < n) {
            xi[q] = x[s];
            p[q] = xs[s];
        }
    }
#pragma unroll
    for (int q = 0; q < kCommitPer; ++q) {
        const int64_t s = base + (int64_t)q * blockDim.x;
        if (s >= n) continue;
        const float dt = sc[__float_as_int(xi[q].w)].dt;
        if (!(isfinite(p[q].x) && isfinite(p[q].y) && isfinite(p[q].z))) atomicOr(err, ERR_NONFINITE);
        v[s] = make_float4((p[q].x - xi[q].x) / dt, (p[q].y - xi[q].y) / dt, (p[q].z - xi[q].z) / dt, 0.f);
        x[s] = make_float4(p[q].x, p[q].y, p[q].z, xi[q].w);
    }
}


// out[3 (id - id_lo) + c] = x[s].c for particles with id in [id_lo, id_hi)
__global__ void k_unpermute(int64_t n, const float4 *__restrict__ x,
                            const uint32_t *__restrict__ id, float *__restrict__ out,
                            uint32_t id_lo, uint32_t id_hi)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint32_t g = id[s];
    if (g < id_lo || g >= id_hi) return;
    const float4 p = x[s];
    const size_t o = 3 * (size_t)(g - id_lo);
    out[o] = p.x;
    out[o + 1] = p.y;
    out[o + 2] = p.z;
}

inline unsigned blocks_for(int64_t n, int block)
{
    return (unsigned)((n + block - 1) / block);
}

}  // namespace

#define LAUNCH(KID, GRID, BLOCK, KERNEL, ...)                                   \
    do {                                                                        \
        if (tm) timer_begin(tm, KID, s);                                        \
        hipLaunchKernelGGL(KERNEL, dim3(GRID), dim3(BLOCK), 0, s, __VA_ARGS__); \
        if (tm) timer_end(tm, KID, s);                                          \
        hipError_t e_ = hipGetLastError();                                      \
        if (e_ != hipSuccess) return e_;                                        \
    } while (0)

// Debug fill of one float4 buffer (a kernel, not a memset, so that a
// captured step replays it like its other launches).
__global__ void k_poison(int64_t n, float4 *__restrict__ p, float4 v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static hipError_t enqueue_poison(const StepBuffers &b, int nxt, hipStream_t s)
{
    // quiet NaN in every float; x.w holds the scene index, so the free
    // position buffer gets scene 0 there: a stray read then gives a NaN
    // position and never an out-of-range scene
    const float qn = std::numeric_limits<float>::quiet_NaN();
    const float4 all = make_float4(qn, qn, qn, qn), pos = make_float4(qn, qn, qn, 0.f);  // 0.f: all bits 0
    const int64_t n = b.n;
    const unsigned grid = (unsigned)std::min<int64_t>(blocks_for(n, 256), 4096);
    float4 *const fill[] = {b.xs_pred, b.xs[0], b.xs[1], b.v[nxt]};
    for (float4 *p : fill) {
        hipLaunchKernelGGL(k_poison, dim3(grid), dim3(256), 0, s, n, p, all);
        if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_poison, dim3(grid), dim3(256), 0, s, n, b.x[nxt], pos);
    return hipGetLastError();
}

static hipError_t enqueue_scan(uint32_t *in, uint32_t count, uint32_t *part, uint32_t *out,
                               bool clear_in, hipStream_t s, Timer *tm)
{
    const unsigned nb = blocks_for(count, kScanBlock * kScanItems);
    // up to kScanDirect blocks, each block of the apply pass adds up the
    // block sums before it (a few loads per thread) instead of a third launch
    const bool direct = nb <= (unsigned)kScanDirect;
    LAUNCH(K_SCAN_REDUCE, nb, kScanBlock, k_scan_reduce, in, count, part);
    if (!direct) LAUNCH(K_SCAN_TOP, 1, 1024, k_scan_top, part, nb);
    LAUNCH(K_SCAN_APPLY, nb, kScanBlock, k_scan_apply, in, count, part, out,
           clear_in ? in : nullptr, direct);
    return hipSuccess;
}

hipError_t enqueue_step(const StepBuffers &b0, int cur, const LaunchShape &ls, hipStream_t s,
                        Timer *tm, const StepRecord *rec)
{
    StepBuffers b = b0;
    if (rec) {  // a recorded step keeps its neighbour structure in the record
        b.nbr = rec->nbr;
        b.pmeta = rec->pmeta;
        b.pslot = rec->pslot;
        b.tile_rows = rec->tile_rows;
        b.tile_rec = rec->tile_rec;
        b.tile_order = rec->tile_order;
        b.tile_start = rec->tile_start;
        b.tile_count = rec->tile_count;
        b.tile_ge = rec->tile_ge;
    }
    const int64_t n = b.n;
    if (n == 0) return hipSuccess;
    const int nxt = cur ^ 1;
    const int K = b.n_iters;
    const uint32_t G = b.n_cells, T = b.n_tiles;
    const uint32_t TX = (T + kXcds - 1) / kXcds * kXcds;  // tile grids, see xcd_slot
    const uint32_t SPLIT = tile_split(TX);
    const int *bs = ls.block;
    hipError_t e;

    if (b.poison && (e = enqueue_poison(b, nxt, s)) != hipSuccess) return e;
    if (b.n_depth) {  // depth images of the distance-to-the-visible-surface scenes
        LAUNCH(K_DEPTH, blocks_for(b.n_depth, 256), 256, k_depth_clear, b.n_depth, b.depth);
        LAUNCH(K_DEPTH, blocks_for(n, kSplatThreads), kSplatThreads, k_depth_splat, n, b.scenes, b.x[cur],
               b.depth);
    }
    if (b.n_range) {  // automatic distance ranges
        LAUNCH(K_LOD_RANGE, blocks_for(b.n_range, 256), 256, k_range_clear, b.n_range, b.range);
        LAUNCH(K_LOD_RANGE, blocks_for(n, bs[K_LOD_RANGE]), bs[K_LOD_RANGE], k_lod_range, n, b.scenes,
               b.x[cur], b.depth, b.range);
    }
    // cell_count is all zero here: cleared at creation, and by the cell scan
    // of every step once it has read the counts
    LAUNCH(K_LOD_PREDICT, blocks_for(n, bs[K_LOD_PREDICT]), bs[K_LOD_PREDICT], k_lod_predict, n,
           b.scenes, b.x[cur], b.v[cur], b.id[cur], b.lev_by_id, b.depth, b.range, b.xs_pred, b.lvl[cur],
           b.key_pre, b.ticket, b.cell_count, b.level_part);
    if ((e = enqueue_scan(b.cell_count, G, b.scan_part, b.cell_start, true, s, tm)) != hipSuccess)
        return e;
    LAUNCH(K_SORT_SCATTER, blocks_for(n, bs[K_SORT_SCATTER]), bs[K_SORT_SCATTER], k_sort_scatter,
           n, b.key_pre, b.ticket, b.cell_start, b.id[cur], b.tmp_src, b.tmp_id);
    LAUNCH(K_SORT_FINISH, blocks_for(n, bs[K_SORT_FINISH]), bs[K_SORT_FINISH], k_sort_finish, n,
           b.tmp_src, b.tmp_id, b.key_pre, b.cell_start, b.x[cur], b.xs_pred, b.lvl[cur],
           b.x[nxt], b.xs[0], b.id[nxt], b.lvl[nxt], b.key, b.err);
    // tiles: own counts and levels, their prefix, and the level buckets
    LAUNCH(K_TILE_PREPARE, blocks_for((int64_t)T * 64, bs[K_TILE_PREPARE]), bs[K_TILE_PREPARE],
           k_tile_prepare, T, b.scenes, b.tile_scene, b.cell_start, b.lvl[nxt], b.tile_count,
           b.tile_lvl);
    if (T <= kFusedTiles) {
        LAUNCH(K_TILE_TABLES, 1, 1024, k_tile_tables, T, K, b.tile_count, b.tile_lvl, b.tile_start,
               b.tile_order, b.tile_ge, b.level_part, blocks_for(n, bs[K_LOD_PREDICT]), b.totals);
    } else {
        if ((e = enqueue_scan(b.tile_count, T, b.scan_part, b.tile_start, false, s, tm)) != hipSuccess)
            return e;
        LAUNCH(K_LEVEL_COUNT, b.n_level_blocks, kLevelBlock, k_level_count, T, b.tile_lvl,
               b.level_counts, b.n_level_blocks, K);
        LAUNCH(K_LEVEL_SCAN, 1, 1024, k_level_scan, b.level_counts, b.n_level_blocks, K, b.tile_ge,
               b.level_part, blocks_for(n, bs[K_LOD_PREDICT]), b.totals);
        LAUNCH(K_LEVEL_SCATTER, b.n_level_blocks, kLevelBlock, k_level_scatter, T, b.tile_lvl,
               b.level_counts, b.n_level_blocks, K, b.tile_order);
    }
    // the split variants only where the grid has room for them (the plain
    // ones need not wait for the tile's count before staging); contact
    // responses only in contexts with obstacles
    const bool split = SPLIT > 1, ct = b.contacts_on;
    const auto nbr_kernel = split ? k_neighbours<true> : k_neighbours<false>;
    const auto lam_kernel = split ? k_lambda<true> : k_lambda<false>;
    const auto upd_kernel = split ? (ct ? k_update<true, true> : k_update<true, false>)
                                  : (ct ? k_update<false, true> : k_update<false, false>);
    LAUNCH(K_NEIGHBOURS, TX * SPLIT, bs[K_NEIGHBOURS], nbr_kernel, b.scenes, b.tile_scene,
           b.tile_order, b.tile_ge, b.tile_start, b.cell_start, b.xs[0], b.lvl[nxt], n, b.nbr_cap,
           b.nbr, b.pmeta, b.pslot, b.tile_count, b.tile_rows, b.err, TX, b.tile_rec);
    if (b.cohesion_on)  // the cohesion force, before contact finding (it is part of the prediction)
        LAUNCH(K_COHESION, TX * SPLIT, bs[K_COHESION], split ? k_cohesion<true> : k_cohesion<false>,
               b.scenes, b.tile_rec, b.tile_ge, b.tile_rows, b.x[nxt], b.xs[0], n, b.nbr, b.pmeta,
               b.pslot, TX);
    if (ct)
        LAUNCH(K_CONTACTS, blocks_for(n, bs[K_CONTACTS]), bs[K_CONTACTS], k_contacts, n, b.scenes,
               b.x[nxt], b.xs[0], b.lvl[nxt], b.contact);
    for (int k = 0; k < K; ++k) {
        float4 *xin = b.xs[k & 1], *xout = b.xs[(k + 1) & 1];
        LAUNCH(K_LAMBDA, TX * SPLIT, bs[K_LAMBDA], lam_kernel, k, b.scenes, b.tile_rec, b.tile_ge,
               b.tile_rows, xin, n, b.nbr, b.pmeta, b.pslot, TX);
        if (rec && (e = hipMemcpyAsync(rec->snap[k], xin, sizeof(float4) * n,
                                       hipMemcpyDeviceToDevice, s)) != hipSuccess)
            return e;
        LAUNCH(K_UPDATE, TX * SPLIT, bs[K_UPDATE], upd_kernel, k, b.scenes, b.tile_rec, b.tile_ge,
               b.tile_rows, xin, xout, n, b.nbr, b.pmeta, b.pslot, b.contact, TX);
    }
    if (rec) {
        if ((e = hipMemcpyAsync(rec->snap[K], b.xs[K & 1], sizeof(float4) * n,
                                hipMemcpyDeviceToDevice, s)) != hipSuccess ||
            (e = hipMemcpyAsync(rec->id, b.id[nxt], sizeof(uint32_t) * n, hipMemcpyDeviceToDevice,
                                s)) != hipSuccess ||
            (e = hipMemcpyAsync(rec->lvl, b.lvl[nxt], n, hipMemcpyDeviceToDevice, s)) != hipSuccess)
            return e;
    }
    LAUNCH(K_COMMIT, blocks_for(n, bs[K_COMMIT] * kCommitPer), bs[K_COMMIT], k_commit, n, b.scenes, b.x[nxt],
           b.v[nxt], b.xs[K & 1], b.err);
    return hipSuccess;
}

hipError_t enqueue_density(const StepBuffers &b0, int cur, const LaunchShape &ls,
                           const DensityBuffers &d, float *rho_id, hipStream_t s)
{
    // A fresh counting sort and neighbour search of the current positions
    // into the free ping-pong half and the density buffers; the step's own
    // structure, error word and running totals are left alone.
    StepBuffers b = b0;
    b.nbr = d.nbr;
    b.pmeta = d.pmeta;
    b.pslot = d.pslot;
    b.tile_rows = d.tile_rows;
    b.tile_rec = d.tile_rec;
    b.tile_order = d.tile_order;
    b.tile_start = d.tile_start;
    b.tile_count = d.tile_count;
    b.tile_ge = d.tile_ge;
    b.tile_lvl = d.tile_lvl;
    b.key = d.key;
    b.err = d.err;
    b.totals = d.totals;
    const int64_t n = b.n;
    if (n == 0) return hipErrorInvalidValue;
    const int nxt = cur ^ 1;
    const int K = b.n_iters;
    const uint32_t G = b.n_cells, T = b.n_tiles;
    const uint32_t TX = (T + kXcds - 1) / kXcds * kXcds;
    const int *bs = ls.block;
    Timer *tm = nullptr;
    hipError_t e;
    LAUNCH(K_LOD_PREDICT, blocks_for(n, 256), 256, k_density_keys, n, b.scenes, b.x[cur],
           b.xs_pred, b.key_pre, b.ticket, b.cell_count);
    if ((e = enqueue_scan(b.cell_count, G, b.scan_part, b.cell_start, true, s, tm)) != hipSuccess)
        return e;
    LAUNCH(K_SORT_SCATTER, blocks_for(n, bs[K_SORT_SCATTER]), bs[K_SORT_SCATTER], k_sort_scatter,
           n, b.key_pre, b.ticket, b.cell_start, b.id[cur], b.tmp_src, b.tmp_id);
    LAUNCH(K_SORT_FINISH, blocks_for(n, bs[K_SORT_FINISH]), bs[K_SORT_FINISH], k_sort_finish, n,
           b.tmp_src, b.tmp_id, b.key_pre, b.cell_start, b.x[cur], b.xs_pred, b.lvl[cur],
           b.x[nxt], d.xs, b.id[nxt], b.lvl[nxt], b.key, b.err);
    LAUNCH(K_TILE_PREPARE, blocks_for((int64_t)T * 64, bs[K_TILE_PREPARE]), bs[K_TILE_PREPARE],
           k_tile_prepare, T, b.scenes, b.tile_scene, b.cell_start, b.lvl[nxt], b.tile_count,
           b.tile_lvl);
    if (T <= kFusedTiles) {
        LAUNCH(K_TILE_TABLES, 1, 1024, k_tile_tables, T, K, b.tile_count, b.tile_lvl, b.tile_start,
               b.tile_order, b.tile_ge, b.level_part, 0u, b.totals);
    } else {
        if ((e = enqueue_scan(b.tile_count, T, b.scan_part, b.tile_start, false, s, tm)) != hipSuccess)
            return e;
        LAUNCH(K_LEVEL_COUNT, b.n_level_blocks, kLevelBlock, k_level_count, T, b.tile_lvl,
               b.level_counts, b.n_level_blocks, K);
        LAUNCH(K_LEVEL_SCAN, 1, 1024, k_level_scan, b.level_counts, b.n_level_blocks, K, b.tile_ge,
               b.level_part, 0u, b.totals);
        LAUNCH(K_LEVEL_SCATTER, b.n_level_blocks, kLevelBlock, k_level_scatter, T, b.tile_lvl,
               b.level_counts, b.n_level_blocks, K, b.tile_order);
    }
    LAUNCH(K_NEIGHBOURS, TX, bs[K_NEIGHBOURS], k_neighbours<false>, b.scenes, b.tile_scene,
           b.tile_order, b.tile_ge, b.tile_start, b.cell_start, d.xs, b.lvl[nxt], n, b.nbr_cap,
           b.nbr, b.pmeta, b.pslot, b.tile_count, b.tile_rows, b.err, TX, b.tile_rec);
    LAUNCH(K_LAMBDA, TX, kTileThreads, k_density, b.scenes, b.tile_rec, b.tile_ge, b.tile_rows,
           d.xs, n, b.nbr, b.pmeta, b.pslot, d.rho_slot, d.part_sum, d.part_max);
    LAUNCH(K_COMMIT, 1, 1024, k_density_finish, TX, n, d.part_sum, d.part_max, d.out);
    if (rho_id)
        LAUNCH(K_COMMIT, blocks_for(n, 256), 256, k_unpermute_scalar, n, d.rho_slot, b.id[nxt],
               rho_id);
    return hipSuccess;
}

hipError_t enqueue_unpermute(int64_t n, const float4 *x, const uint32_t *id, float *out,
                             uint32_t id_lo, uint32_t id_hi, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_unpermute, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, x, id, out,
                       id_lo, id_hi);
    return hipGetLastError();
}

}  // namespace pbf
