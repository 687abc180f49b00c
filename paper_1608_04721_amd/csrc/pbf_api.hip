// Host side of libpbf: contexts, argument checks, device buffers, graph
// capture, profiling and the ID-order debug exports declared in pbf.h.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "../../include/pbf.h"
#include "pbf_internal.h"

namespace pbf {

struct Timer {
    struct Rec {
        int kernel;
        hipEvent_t a, b;
    };
    std::vector<Rec> pool;
    size_t used = 0;
    double total_ms[K_COUNT] = {};
    int64_t launches[K_COUNT] = {};
    hipError_t status = hipSuccess;
};

void timer_begin(Timer *tm, int kernel, hipStream_t s)
{
    if (tm->used == tm->pool.size()) {
        Timer::Rec r{kernel, nullptr, nullptr};
        if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) {
            tm->status = hipErrorOutOfMemory;
            return;
        }
        tm->pool.push_back(r);
    }
    Timer::Rec &r = tm->pool[tm->used];
    r.kernel = kernel;
    hipError_t e = hipEventRecord(r.a, s);
    if (e != hipSuccess) tm->status = e;
}

void timer_end(Timer *tm, int kernel, hipStream_t s)
{
    if (tm->used >= tm->pool.size()) return;
    Timer::Rec &r = tm->pool[tm->used];
    (void)kernel;
    hipError_t e = hipEventRecord(r.b, s);
    if (e != hipSuccess) tm->status = e;
    tm->used++;
}

static hipError_t timer_collect(Timer *tm, hipStream_t s)
{
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    for (size_t i = 0; i < tm->used; ++i) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, tm->pool[i].a, tm->pool[i].b);
        if (e != hipSuccess) return e;
        tm->total_ms[tm->pool[i].kernel] += ms;
        tm->launches[tm->pool[i].kernel] += 1;
    }
    tm->used = 0;
    return hipSuccess;
}

// Device memory of the library.  Every allocation and free goes through
// dev_malloc / dev_free, which keep the bytes held by all contexts of the
// process and enforce the limit set with pbf_set_memory_limit.
namespace {
std::mutex g_mem_mu;
std::unordered_map<void *, size_t> g_mem_size;
int64_t g_mem_held = 0;
int64_t g_mem_limit = 0;  // 0: none
}  // namespace

hipError_t dev_malloc(void **p, size_t bytes)
{
    bytes = std::max<size_t>(bytes, 1);
    std::lock_guard<std::mutex> lk(g_mem_mu);
    *p = nullptr;
    if (g_mem_limit > 0 && g_mem_held + (int64_t)bytes > g_mem_limit) return hipErrorOutOfMemory;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return e;
    }
    g_mem_size[*p] = bytes;
    g_mem_held += (int64_t)bytes;
    return hipSuccess;
}

void dev_free(void *p)
{
    if (!p) return;
    {
        std::lock_guard<std::mutex> lk(g_mem_mu);
        auto it = g_mem_size.find(p);
        if (it != g_mem_size.end()) {
            g_mem_held -= (int64_t)it->second;
            g_mem_size.erase(it);
        }
    }
    (void)hipFree(p);
}

}  // namespace pbf

using namespace pbf;

struct pbf_ctx {
    int32_t n_scenes = 0;
    int64_t n_total = 0;
    std::vector<pbf_params> params;
    std::vector<int64_t> pid_off;  // n_scenes + 1
    std::vector<SceneDev> scenes;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    StepBuffers b{};
    int cur = 0;
    int64_t step = 0;
    bool stepped = false;
    LaunchShape ls{};
    bool graph = false;
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    bool profiling = false;
    Timer timer;
    float *staging = nullptr;  // float[3 n_total], device
    std::vector<void *> allocs;
    std::string err;
    // differentiable rollout: checkpoints of (x, v) in ID order, float[3 n] each
    std::vector<float *> ckpt;  // x0, v0, x1, v1, ... (pairs)
    int32_t roll_steps = 0, roll_every = 0;
    bool roll_valid = false;
    size_t depth_cap = 0;  // pixels allocated in b.depth (DTVS depth images)
    uint32_t range_cap = 0;  // words allocated in b.range (automatic distance ranges)
    // b.depth and b.range are owned here (not in allocs): they are replaced
    // when a larger layout is needed
    // average-density buffers (allocated by the first pbf_density)
    pbf::DensityBuffers dens{};
    float *dens_rho_id = nullptr;
    // work buffers of the reverse pass, kept for the next call of the same shape
    struct {
        std::vector<void *> bufs;
        int32_t seg_len = 0;
        float *ax = nullptr, *av = nullptr, *fx = nullptr, *fv = nullptr;
        unsigned long long *tot = nullptr;
        pbf::AdjointScratch w{};
        std::vector<pbf::StepRecord> recs;
    } rs;
};

namespace {

pbf_status fail(pbf_ctx *c, pbf_status s, const std::string &msg)
{
    if (c) c->err = msg;
    return s;
}

pbf_status hip_fail(pbf_ctx *c, hipError_t e, const char *what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fail(c, PBF_ERR_OUT_OF_MEMORY, m);
    return fail(c, PBF_ERR_DEVICE, m);
}

#define HIPCHK(C, EXPR, WHAT)                         \
    do {                                              \
        hipError_t e_ = (EXPR);                       \
        if (e_ != hipSuccess) return hip_fail(C, e_, WHAT); \
    } while (0)

bool finite3(const float *p)
{
    return std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]);
}

// ceil(extent / h) with a relative slack of 1e-9, at least 1
int32_t auto_dim(float lo, float hi, float h)
{
    double q = ((double)hi - (double)lo) / (double)h;
    double d = std::ceil(q * (1.0 - 1e-9));
    return d < 1.0 ? 1 : (int32_t)d;
}

pbf_status check_params(const pbf_params &p, int32_t idx, std::string &msg, int32_t dims[3])
{
    char buf[256];
    auto bad = [&](const char *what) {
        std::snprintf(buf, sizeof buf, "scene %d: %s", idx, what);
        msg = buf;
        return PBF_ERR_INVALID_ARG;
    };
    if (p.n < 0) return bad("n < 0");
    if (p.n_min < 1 || p.n_max < p.n_min || p.n_max > PBF_MAX_ITERS)
        return bad("need 1 <= n_min <= n_max <= PBF_MAX_ITERS");
    const float fs[] = {p.h, p.rho0, p.mass, p.eps, p.dt, p.gravity[0], p.gravity[1],
                        p.gravity[2], p.box_lo[0], p.box_lo[1], p.box_lo[2], p.box_hi[0],
                        p.box_hi[1], p.box_hi[2]};
    for (float f : fs)
        if (!std::isfinite(f)) return bad("non-finite parameter");
    if (!(p.h > 0.f) || !(p.rho0 > 0.f) || !(p.mass > 0.f) || !(p.eps >= 0.f) || !(p.dt > 0.f))
        return bad("need h, rho0, mass, dt > 0 and eps >= 0");
    if (p.flags & ~PBF_FLAG_UNILATERAL) return bad("unknown flags");
    if (p.max_neighbours < 0 || p.max_neighbours > 4096) return bad("max_neighbours outside [0, 4096]");
    for (int d = 0; d < 3; ++d) {
        if (!(p.box_hi[d] >= p.box_lo[d])) return bad("box_hi < box_lo");
        if (p.grid_dims[d] < 0) return bad("grid_dims < 0");
        dims[d] = p.grid_dims[d] ? p.grid_dims[d] : auto_dim(p.box_lo[d], p.box_hi[d], p.h);
        if (dims[d] > (1 << 20)) return bad("grid too large");
    }
    return PBF_OK;
}

SceneDev make_scene(const pbf_params &p, const int32_t dims[3], uint32_t cell_off,
                    uint32_t tile_off, uint32_t pid_off)
{
    SceneDev s{};
    const double h = p.h, pi = 3.14159265358979323846;
    for (int d = 0; d < 3; ++d) {
        s.lo[d] = p.box_lo[d];
        s.hi[d] = p.box_hi[d];
        s.g[d] = p.gravity[d];
        s.dims[d] = dims[d];
        s.tiles[d] = (dims[d] + kTileEdge - 1) / kTileEdge;
        s.cam[d] = 0.f;
    }
    s.h = p.h;
    s.h2 = (float)(h * h);
    s.h6 = (float)std::pow(h, 6);
    s.c_rho = (float)((double)p.mass * 315.0 / (64.0 * pi * std::pow(h, 9)) / (double)p.rho0);
    s.c_grad = (float)(45.0 / (pi * std::pow(h, 6)));
    s.c_s = (float)((double)p.mass / ((double)p.rho0 * (double)p.rho0));
    s.inv_rho0 = (float)(1.0 / (double)p.rho0);
    s.eps = p.eps;
    s.dt = p.dt;
    s.inv_dt = (float)(1.0 / (double)p.dt);
    s.cell_off = cell_off;
    s.tile_off = tile_off;
    s.pid_off = pid_off;
    s.n_min = p.n_min;
    s.n_max = p.n_max;
    s.lod_mode = PBF_LOD_UNIFORM;
    s.d_near = 0.f;
    s.d_far = 1.f;
    s.n_cam = 1;
    s.rng[0][0] = 0.f;
    s.rng[0][1] = 1.f;
    s.stab_s = 1;
    s.c_floor = (p.flags & PBF_FLAG_UNILATERAL) ? 0.f : -INFINITY;
    return s;
}

template <class T>
hipError_t dalloc(pbf_ctx *c, T **p, size_t count)
{
    void *q = nullptr;
    hipError_t e = dev_malloc(&q, std::max<size_t>(count, 1) * sizeof(T));
    if (e == hipSuccess) {
        c->allocs.push_back(q);
        *p = (T *)q;
    }
    return e;
}

void drop_graphs(pbf_ctx *c)
{
    for (auto &g : c->exec)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
}

bool fixed_shape(int k)
{
    return k == K_DEPTH || k == K_SCAN_REDUCE || k == K_SCAN_TOP || k == K_SCAN_APPLY || k == K_LEVEL_COUNT ||
           k == K_LEVEL_SCAN || k == K_LEVEL_SCATTER || k == K_TILE_TABLES;
}

// tile kernels are compiled for a bounded block size
int max_block(int k)
{
    if (k == K_NEIGHBOURS) return kNbrThreads;
    if (k == K_LAMBDA || k == K_UPDATE || k == K_COHESION) return kTileThreads;
    return 1024;
}

pbf_status latched(pbf_ctx *c)
{
    uint32_t e = 0;
    HIPCHK(c, hipMemcpyAsync(&e, c->b.err, sizeof e, hipMemcpyDeviceToHost, c->stream),
           "read fault word");
    HIPCHK(c, hipStreamSynchronize(c->stream), "stream synchronize");
    if (e & ERR_NONFINITE) return fail(c, PBF_ERR_NONFINITE, "positions became non-finite");
    if (e & ERR_NEIGHBOUR_CAP)
        return fail(c, PBF_ERR_CAPACITY, "a particle exceeded the neighbour capacity");
    if (e & ERR_CELL_CAP)
        return fail(c, PBF_ERR_CAPACITY, "a grid cell held more than PBF_MAX_CELL particles, or "
                                          "six cells of a grid row more than 1024");
    return PBF_OK;
}

// Upload x, v (float[3 n_total], ID order, host) as the current state with
// storage order = ID order.
pbf_status upload_state(pbf_ctx *c, const float *x, const float *v)
{
    const int64_t n = c->n_total;
    std::vector<float4> hx((size_t)n), hv((size_t)n);
    std::vector<uint32_t> hid((size_t)n);
    for (int32_t s = 0; s < c->n_scenes; ++s) {
        float sbits;
        int32_t si = s;
        std::memcpy(&sbits, &si, sizeof sbits);
        for (int64_t g = c->pid_off[s]; g < c->pid_off[s + 1]; ++g) {
            hx[g] = make_float4(x[3 * g], x[3 * g + 1], x[3 * g + 2], sbits);
            hv[g] = make_float4(v[3 * g], v[3 * g + 1], v[3 * g + 2], 0.f);
            hid[g] = (uint32_t)g;
        }
    }
    c->cur = 0;
    HIPCHK(c, hipMemcpyAsync(c->b.x[0], hx.data(), n * sizeof(float4), hipMemcpyHostToDevice, c->stream), "upload x");
    HIPCHK(c, hipMemcpyAsync(c->b.v[0], hv.data(), n * sizeof(float4), hipMemcpyHostToDevice, c->stream), "upload v");
    HIPCHK(c, hipMemcpyAsync(c->b.id[0], hid.data(), n * sizeof(uint32_t), hipMemcpyHostToDevice, c->stream), "upload id");
    HIPCHK(c, hipStreamSynchronize(c->stream), "stream synchronize");
    return PBF_OK;
}

// Copy a caller buffer (host or device) of `bytes` into host memory.
pbf_status fetch_input(pbf_ctx *c, const void *src, size_t bytes, int on_device, void *dst)
{
    if (bytes == 0) return PBF_OK;
    if (!on_device) {
        std::memcpy(dst, src, bytes);
        return PBF_OK;
    }
    HIPCHK(c, hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost), "copy device input");
    return PBF_OK;
}

pbf_status check_levels(pbf_ctx *c, int32_t scene, const uint8_t *lv)
{
    const pbf_params &p = c->params[scene];
    for (int32_t i = 0; i < p.n; ++i)
        if (lv[i] < p.n_min || lv[i] > p.n_max)
            return fail(c, PBF_ERR_INVALID_ARG, "explicit level outside [n_min, n_max]");
    return PBF_OK;
}

pbf_status read_by_id(pbf_ctx *c, const float4 *src, float *out, int on_device, int64_t id_lo,
                      int64_t id_hi)
{
    float *dst = on_device ? out : c->staging;
    HIPCHK(c, enqueue_unpermute(c->n_total, src, c->b.id[c->cur], dst, (uint32_t)id_lo,
                                (uint32_t)id_hi, c->stream), "unpermute");
    if (!on_device) {
        HIPCHK(c, hipMemcpyAsync(out, c->staging, (size_t)(id_hi - id_lo) * 3 * sizeof(float),
                                 hipMemcpyDeviceToHost, c->stream), "copy out");
        HIPCHK(c, hipStreamSynchronize(c->stream), "stream synchronize");
        return latched(c);
    }
    return PBF_OK;
}

template <class T>
pbf_status d2h(pbf_ctx *c, std::vector<T> &dst, const T *src, size_t count)
{
    dst.resize(count);
    if (count == 0) return PBF_OK;
    HIPCHK(c, hipMemcpyAsync(dst.data(), src, count * sizeof(T), hipMemcpyDeviceToHost, c->stream),
           "copy to host");
    HIPCHK(c, hipStreamSynchronize(c->stream), "stream synchronize");
    return PBF_OK;
}

// Work space of pbf_density_noalloc: one fixed array per GPU (this code
// object's copy on each device), so that entry point allocates nothing.
// Host code never uses the array's name as an address: static_scratch gives
// the device address, looked up once per device.
constexpr long long kStaticScratchBytes = PBF_STATIC_SCRATCH_BYTES;
}  // namespace
static __device__ __align__(256) unsigned char scratch[PBF_STATIC_SCRATCH_BYTES];
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (made current for the lookup).
hipError_t static_scratch(int device, unsigned char **ptr)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int prev = 0;
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess) return e;
        if (prev != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *q = nullptr;
        e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
        if (prev != device) {
            hipError_t e2 = hipSetDevice(prev);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        if (!q) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = (unsigned char *)q;
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
}

// Carve the density buffers of context c out of the work space at `base`
// (256-byte aligned pieces); returns the bytes needed.  base = nullptr only
// sizes.
size_t static_density_layout(const pbf_ctx *c, unsigned char *base, DensityBuffers &d,
                             float *&rho_stage)
{
    const size_t n = (size_t)c->n_total, T = c->b.n_tiles;
    const size_t parts = (T + kXcds - 1) / kXcds * kXcds;
    size_t off = 0;
    auto take = [&](auto **ptr, size_t count) {
        off = (off + 255) & ~(size_t)255;
        *ptr = base ? (std::remove_reference_t<decltype(*ptr)>)(base + off) : nullptr;
        off += std::max<size_t>(count, 1) * sizeof(**ptr);
    };
    take(&d.xs, n);
    take(&d.key, n);
    take(&d.nbr, n * (size_t)(c->b.nbr_stride / 8));
    take(&d.pmeta, n);
    take(&d.pslot, n);
    take(&d.tile_rows, T * kRowWords);
    take(&d.tile_rec, T);
    take(&d.tile_order, T);
    take(&d.tile_start, T + 1);
    take(&d.tile_count, T);
    take(&d.tile_ge, (size_t)PBF_MAX_ITERS + 2);
    take(&d.tile_lvl, T);
    take(&d.err, 1);
    take(&d.totals, 2);
    take(&d.rho_slot, n);
    take(&d.part_sum, parts);
    take(&d.part_max, parts);
    take(&rho_stage, n);
    take(&d.out, 2);
    return off;
}

__global__ void k_clear_words(uint32_t *__restrict__ p, uint32_t count)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0u;
}

// Zero `count` words on stream s with a kernel (no memset node).
hipError_t clear_words(uint32_t *p, uint32_t count, hipStream_t s)
{
    hipLaunchKernelGGL(k_clear_words, dim3((count + 255) / 256), dim3(256), 0, s, p, count);
    return hipGetLastError();
}

// The density measure with its buffers in d (err already cleared on the
// stream): enqueue, copy the results out, synchronise, report faults.
// rho_stage: n floats of device memory for a host rho_rel.
pbf_status density_run(pbf_ctx *c, const DensityBuffers &d, float *rho_stage, double *out,
                       float *rho_rel, int32_t on_device)
{
    const int64_t n = c->n_total;
    float *rho_id = rho_rel ? (on_device ? rho_rel : rho_stage) : nullptr;
    HIPCHK(c, enqueue_density(c->b, c->cur, c->ls, d, rho_id, c->stream), "density");
    uint32_t bad = 0;
    HIPCHK(c, hipMemcpyAsync(out, d.out, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream),
           "density out");
    HIPCHK(c, hipMemcpyAsync(&bad, d.err, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream),
           "density faults");
    if (rho_rel && !on_device)
        HIPCHK(c, hipMemcpyAsync(rho_rel, rho_id, (size_t)n * sizeof(float), hipMemcpyDeviceToHost,
                                 c->stream),
               "density out");
    HIPCHK(c, hipStreamSynchronize(c->stream), "stream synchronize");
    if (bad & ERR_NEIGHBOUR_CAP)
        return fail(c, PBF_ERR_CAPACITY, "pbf_density: a particle exceeded the neighbour capacity");
    if (bad & ERR_CELL_CAP)
        return fail(c, PBF_ERR_CAPACITY, "pbf_density: a cell or staged row exceeded its capacity");
    return latched(c);
}

pbf_status step_n(pbf_ctx *c, int32_t n_steps);

pbf_status need_step(pbf_ctx *c)
{
    if (!c->stepped) return fail(c, PBF_ERR_INVALID_ARG, "no step has run since the state was set");
    return PBF_OK;
}

}  // namespace

extern "C" {

const char *pbf_status_string(pbf_status s)
{
    switch (s) {
    case PBF_OK: return "ok";
    case PBF_ERR_INVALID_ARG: return "invalid argument";
    case PBF_ERR_NONFINITE: return "non-finite value";
    case PBF_ERR_OUT_OF_MEMORY: return "out of memory";
    case PBF_ERR_DEVICE: return "device error";
    case PBF_ERR_CAPACITY: return "capacity exceeded";
    }
    return "unknown status";
}

const char *pbf_last_error(const pbf_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : "null context";
}

pbf_status pbf_set_memory_limit(int64_t bytes)
{
    if (bytes < 0) return PBF_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_mem_mu);
    g_mem_limit = bytes;
    return PBF_OK;
}

int64_t pbf_device_bytes(void)
{
    std::lock_guard<std::mutex> lk(g_mem_mu);
    return g_mem_held;
}

int32_t pbf_kernel_count(void) { return K_COUNT; }

const char *pbf_kernel_name(int32_t k)
{
    return (k >= 0 && k < K_COUNT) ? kKernelNames[k] : nullptr;
}

void pbf_destroy(pbf_ctx *c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    for (auto &r : c->timer.pool) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (void *p : c->allocs) dev_free(p);
    for (float *p : c->ckpt) dev_free(p);
    for (void *p : c->rs.bufs) dev_free(p);
    dev_free(c->b.depth);
    dev_free(c->b.range);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

pbf_status pbf_batch_create(int32_t n_scenes, const pbf_params *params, const float *x0,
                            const float *v0, int32_t inputs_on_device, void *hip_stream,
                            pbf_ctx **out)
{
    if (!out) return PBF_ERR_INVALID_ARG;
    *out = nullptr;
    if (n_scenes < 1 || n_scenes > PBF_MAX_SCENES || !params) return PBF_ERR_INVALID_ARG;
    // ---- host-side checks, before any HIP call
    std::vector<std::array<int32_t, 3>> dims((size_t)n_scenes);
    int64_t n_total = 0, cells = 0, tiles = 0;
    int32_t cap = 0, kmax = 1;
    std::string msg;
    for (int32_t s = 0; s < n_scenes; ++s) {
        if (check_params(params[s], s, msg, dims[s].data()) != PBF_OK) return PBF_ERR_INVALID_ARG;
        n_total += params[s].n;
        cells += (int64_t)dims[s][0] * dims[s][1] * dims[s][2];
        tiles += (int64_t)((dims[s][0] + kTileEdge - 1) / kTileEdge) *
                 ((dims[s][1] + kTileEdge - 1) / kTileEdge) *
                 ((dims[s][2] + kTileEdge - 1) / kTileEdge);
        cap = std::max(cap, params[s].max_neighbours ? params[s].max_neighbours
                                                     : PBF_DEFAULT_NEIGHBOURS);
        kmax = std::max(kmax, params[s].n_max);
    }
    if (n_total >= ((int64_t)1 << 31) || cells >= ((int64_t)1 << 32) - 2 ||
        tiles >= ((int64_t)1 << 31))
        return PBF_ERR_INVALID_ARG;
    if (n_total > 0 && (!x0 || !v0)) return PBF_ERR_INVALID_ARG;

    pbf_ctx *c = new (std::nothrow) pbf_ctx();
    if (!c) return PBF_ERR_OUT_OF_MEMORY;
    c->n_scenes = n_scenes;
    c->n_total = n_total;
    c->params.assign(params, params + n_scenes);
    c->pid_off.assign((size_t)n_scenes + 1, 0);
    for (int32_t s = 0; s < n_scenes; ++s) c->pid_off[s + 1] = c->pid_off[s] + params[s].n;
    for (int k = 0; k < K_COUNT; ++k) c->ls.block[k] = kDefaultBlock[k];

    std::vector<float> hx((size_t)n_total * 3), hv((size_t)n_total * 3);
    pbf_status st = fetch_input(c, x0, hx.size() * sizeof(float), inputs_on_device, hx.data());
    if (st == PBF_OK) st = fetch_input(c, v0, hv.size() * sizeof(float), inputs_on_device, hv.data());
    if (st != PBF_OK) {
        pbf_status r = st;
        pbf_destroy(c);
        return r;
    }
    for (int64_t i = 0; i < n_total; ++i)
        if (!finite3(&hx[3 * i]) || !finite3(&hv[3 * i])) {
            pbf_destroy(c);
            return PBF_ERR_NONFINITE;
        }

    auto bail = [&](pbf_status s) {
        pbf_destroy(c);
        return s;
    };
    if (hipGetDevice(&c->device) != hipSuccess) return bail(PBF_ERR_DEVICE);
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess)
            return bail(PBF_ERR_DEVICE);
        c->own_stream = true;
    }

    uint32_t coff = 0, toff = 0;
    std::vector<uint32_t> tile_scene((size_t)tiles), id_scene((size_t)n_total);
    for (int32_t s = 0; s < n_scenes; ++s)
        for (int64_t g = c->pid_off[s]; g < c->pid_off[s + 1]; ++g) id_scene[g] = (uint32_t)s;
    for (int32_t s = 0; s < n_scenes; ++s) {
        c->scenes.push_back(make_scene(params[s], dims[s].data(), coff, toff,
                                       (uint32_t)c->pid_off[s]));
        const SceneDev &sd = c->scenes.back();
        const uint32_t nt = (uint32_t)sd.tiles[0] * (uint32_t)sd.tiles[1] * (uint32_t)sd.tiles[2];
        for (uint32_t t = 0; t < nt; ++t) tile_scene[toff + t] = (uint32_t)s;
        coff += (uint32_t)((int64_t)dims[s][0] * dims[s][1] * dims[s][2]);
        toff += nt;
    }

    StepBuffers &b = c->b;
    const size_t n = (size_t)n_total;
    b.n = n_total;
    b.n_cells = (uint32_t)cells;
    b.n_tiles = (uint32_t)tiles;
    b.n_iters = kmax;
    b.nbr_cap = cap;
    b.nbr_stride = (cap + 7) / 8 * 8;
    b.n_level_blocks = (int32_t)((tiles + kLevelBlock - 1) / kLevelBlock);
    b.n_scan_blocks = (int32_t)((std::max(cells, tiles) + kScanBlock * kScanItems - 1) /
                                (kScanBlock * kScanItems));
    SceneDev *dsc = nullptr;
    uint8_t *dlev = nullptr;
    uint32_t *dtile_scene = nullptr, *did_scene = nullptr;
    hipError_t e = hipSuccess;
#define AL(P, N) if (e == hipSuccess) e = dalloc(c, &(P), (N))
    AL(dsc, (size_t)n_scenes);
    AL(dlev, n);
    for (int h = 0; h < 2; ++h) {
        AL(b.x[h], n);
        AL(b.v[h], n);
        AL(b.id[h], n);
        AL(b.lvl[h], n);
        AL(b.xs[h], n);
    }
    AL(b.xs_pred, n);
    AL(b.key_pre, n);
    AL(b.ticket, n);
    AL(b.key, n);
    AL(b.tmp_src, n);
    AL(b.tmp_id, n);
    AL(b.cell_count, (size_t)cells);
    if (e == hipSuccess) e = hipMemset(b.cell_count, 0, sizeof(uint32_t) * std::max<size_t>(cells, 1));
    AL(b.cell_start, (size_t)cells + 1);
    AL(b.scan_part, (size_t)b.n_scan_blocks);
    AL(dtile_scene, (size_t)tiles);
    AL(did_scene, n);
    AL(b.tile_count, (size_t)tiles);
    AL(b.tile_start, (size_t)tiles + 1);
    AL(b.tile_lvl, (size_t)tiles);
    AL(b.level_counts, (size_t)b.n_level_blocks * (kmax + 1));
    AL(b.tile_ge, (size_t)PBF_MAX_ITERS + 2);
    AL(b.tile_order, (size_t)tiles);
    AL(b.tile_rows, (size_t)tiles * kRowWords);
    AL(b.tile_rec, (size_t)tiles);
    AL(b.nbr, n * (size_t)(b.nbr_stride / 8));
    AL(b.pmeta, n);
    AL(b.pslot, n);
    AL(b.err, 1);
    AL(b.totals, 2);
    AL(b.level_part, (n + 63) / 64);
    AL(c->staging, n * 3);
#undef AL
    if (e != hipSuccess) return bail(hip_fail(c, e, "allocate") );
    b.scenes = dsc;
    b.lev_by_id = dlev;
    b.tile_scene = dtile_scene;
    b.id_scene = did_scene;
    if (hipMemcpy(dsc, c->scenes.data(), sizeof(SceneDev) * n_scenes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(did_scene, id_scene.data(), sizeof(uint32_t) * n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dtile_scene, tile_scene.data(), sizeof(uint32_t) * tile_scene.size(),
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(b.err, 0, sizeof(uint32_t)) != hipSuccess ||
        hipMemset(b.totals, 0, 2 * sizeof(unsigned long long)) != hipSuccess ||
        hipMemset(dlev, 0, n ? n : 1) != hipSuccess)
        return bail(PBF_ERR_DEVICE);
    if (upload_state(c, hx.data(), hv.data()) != PBF_OK) return bail(PBF_ERR_DEVICE);
    *out = c;
    return PBF_OK;
}

pbf_status pbf_create(const pbf_params *params, const float *x0, const float *v0,
                      int32_t inputs_on_device, void *hip_stream, pbf_ctx **out)
{
    return pbf_batch_create(1, params, x0, v0, inputs_on_device, hip_stream, out);
}

pbf_status pbf_batch_set_lod(pbf_ctx *c, int32_t scene, const pbf_lod_desc *lod)
{
    if (!c) return PBF_ERR_INVALID_ARG;
    if (!lod || scene < 0 || scene >= c->n_scenes)
        return fail(c, PBF_ERR_INVALID_ARG, "bad scene index or null descriptor");
    SceneDev s = c->scenes[scene];
    const pbf_params &p = c->params[scene];
    std::vector<uint8_t> lv;
    if (lod->mode == PBF_LOD_EXPLICIT) {
        if (p.n > 0 && !lod->levels) return fail(c, PBF_ERR_INVALID_ARG, "levels is NULL");
        lv.resize((size_t)p.n);
        pbf_status st = fetch_input(c, lod->levels, lv.size(), lod->levels_on_device, lv.data());
        if (st != PBF_OK) return st;
        st = check_levels(c, scene, lv.data());
        if (st != PBF_OK) return st;
    } else if (lod->mode == PBF_LOD_DTC) {
        if (lod->auto_range != 0 && lod->auto_range != 1)
            return fail(c, PBF_ERR_INVALID_ARG, "auto_range must be 0 or 1");
        if (lod->n_extra_cameras < 0 || lod->n_extra_cameras > PBF_MAX_CAMERAS - 1)
            return fail(c, PBF_ERR_INVALID_ARG, "n_extra_cameras outside [0, PBF_MAX_CAMERAS - 1]");
        const auto range_ok = [&](float dn, float df) {
            return std::isfinite(dn) && std::isfinite(df) && (lod->auto_range || df > dn);
        };
        if (!finite3(lod->camera) || !range_ok(lod->d_near, lod->d_far))
            return fail(c, PBF_ERR_INVALID_ARG, "DTC needs a finite camera and d_far > d_near");
        for (int k = 0; k < lod->n_extra_cameras; ++k)
            if (!finite3(lod->extra_camera[k]) ||
                !range_ok(lod->extra_range[k][0], lod->extra_range[k][1]))
                return fail(c, PBF_ERR_INVALID_ARG, "DTC needs finite cameras and d_far > d_near");
        for (int d = 0; d < 3; ++d) s.cam[d] = lod->camera[d];
        s.d_near = lod->d_near;
        s.d_far = lod->d_far;
        s.n_cam = 1 + lod->n_extra_cameras;
        for (int k = 0; k < s.n_cam; ++k) {
            for (int d = 0; d < 3; ++d) s.cams[k][d] = k ? lod->extra_camera[k - 1][d] : lod->camera[d];
            s.rng[k][0] = k ? lod->extra_range[k - 1][0] : lod->d_near;
            s.rng[k][1] = k ? lod->extra_range[k - 1][1] : lod->d_far;
        }
        s.auto_range = lod->auto_range;
    } else if (lod->mode == PBF_LOD_DTVS) {
        const auto fin = [](float v) { return std::isfinite(v); };
        if (lod->auto_range != 0 && lod->auto_range != 1)
            return fail(c, PBF_ERR_INVALID_ARG, "auto_range must be 0 or 1");
        if (lod->n_extra_cameras != 0)
            return fail(c, PBF_ERR_INVALID_ARG, "further cameras are for DTC only");
        if (!finite3(lod->camera) || !finite3(lod->forward) || !finite3(lod->up) ||
            !fin(lod->focal) || !(lod->focal > 0.f) || !fin(lod->splat) || !(lod->splat >= 0.f) ||
            !fin(lod->d_near) || !fin(lod->d_far) || !(lod->auto_range || lod->d_far > lod->d_near))
            return fail(c, PBF_ERR_INVALID_ARG, "DTVS needs a finite camera frame, focal > 0, "
                                                "splat >= 0 and d_far > d_near");
        s.n_cam = 1;
        s.rng[0][0] = lod->d_near;
        s.rng[0][1] = lod->d_far;
        s.auto_range = lod->auto_range;
        if (lod->width < 1 || lod->height < 1 || lod->width > PBF_MAX_IMAGE ||
            lod->height > PBF_MAX_IMAGE)
            return fail(c, PBF_ERR_INVALID_ARG, "DTVS image size outside [1, PBF_MAX_IMAGE]");
        for (int d = 0; d < 3; ++d) {
            s.cam[d] = lod->camera[d];
            s.fwd[d] = lod->forward[d];
            s.up[d] = lod->up[d];
        }
        s.d_near = lod->d_near;
        s.d_far = lod->d_far;
        s.focal = lod->focal;
        s.splat = lod->splat;
        s.img_w = lod->width;
        s.img_h = lod->height;
    } else if (lod->mode != PBF_LOD_UNIFORM) {
        return fail(c, PBF_ERR_INVALID_ARG, "unknown LOD mode");
    }
    s.lod_mode = lod->mode;
    // The new scene table with the layout of the depth images of all DTVS
    // scenes (one after another) and of the automatic-range words.  Nothing
    // of the context changes until every check and allocation has passed.
    std::vector<SceneDev> ns = c->scenes;
    ns[scene] = s;
    size_t pixels = 0;
    for (auto &sd : ns) {
        sd.depth_off = (uint32_t)pixels;
        if (sd.lod_mode == PBF_LOD_DTVS) pixels += (size_t)sd.img_w * (size_t)sd.img_h;
        if (pixels > 0xffffffffull) return fail(c, PBF_ERR_INVALID_ARG, "DTVS images too large in total");
    }
    uint32_t words = 0;
    for (auto &sd : ns) {
        sd.range_off = words;
        if (sd.auto_range && (sd.lod_mode == PBF_LOD_DTC || sd.lod_mode == PBF_LOD_DTVS))
            words += 2u * (uint32_t)sd.n_cam;
    }
    uint32_t *new_depth = nullptr, *new_range = nullptr;
    if (pixels > c->depth_cap) {
        hipError_t e = dev_malloc((void **)&new_depth, pixels * sizeof(uint32_t));
        if (e != hipSuccess) return hip_fail(c, e, "depth images");
    }
    if (words > c->range_cap) {
        hipError_t e = dev_malloc((void **)&new_range, (size_t)words * sizeof(uint32_t));
        if (e != hipSuccess) {
            dev_free(new_depth);
            return hip_fail(c, e, "range words");
        }
    }
    // commit: the stream is idle before buffers that captured steps use change
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        dev_free(new_depth);
        dev_free(new_range);
        return hip_fail(c, e, "stream synchronize");
    }
    if (new_depth || new_range || pixels != c->b.n_depth || words != c->b.n_range)
        drop_graphs(c);  // the step's launches or their buffers change
    if (new_depth) {
        dev_free(c->b.depth);
        c->b.depth = new_depth;
        c->depth_cap = pixels;
    }
    if (new_range) {
        dev_free(c->b.range);
        c->b.range = new_range;
        c->range_cap = words;
    }
    c->b.n_depth = (uint32_t)pixels;
    c->b.n_range = words;
    c->scenes = ns;
    c->roll_valid = false;  // a recorded rollout no longer replays the same steps
    if (!lv.empty())
        HIPCHK(c, hipMemcpyAsync(c->b.lev_by_id + c->pid_off[scene], lv.data(), lv.size(),
                                 hipMemcpyHostToDevice, c->stream), "upload levels");
    HIPCHK(c, hipMemcpyAsync((void *)c->b.scenes, c->scenes.data(), sizeof(SceneDev) * c->scenes.size(),
                             hipMemcpyHostToDevice, c->stream), "upload scenes");
    HIPCHK(c, hipStreamSynchronize(c->stream), "stream synchronize");
    return PBF_OK;
}

pbf_status pbf_set_lod(pbf_ctx *c, const pbf_lod_desc *lod)
{
    return pbf_batch_set_lod(c, 0, lod);
}

pbf_status pbf_batch_set_obstacles(pbf_ctx *c, int32_t scene, const pbf_contact_desc *desc)
{
    if (!c) return PBF_ERR_INVALID_ARG;
    if (!desc || scene < 0 || scene >= c->n_scenes)
        return fail(c, PBF_ERR_INVALID_ARG, "bad scene index or null descriptor");
    const pbf_params &p = c->params[scene];
    if (desc->count < 0 || desc->count > PBF_MAX_OBSTACLES)
        return fail(c, PBF_ERR_INVALID_ARG, "obstacle count outside [0, PBF_MAX_OBSTACLES]");
    if (desc->stab_iters < 0 || desc->stab_iters > PBF_MAX_ITERS)
        return fail(c, PBF_ERR_INVALID_ARG, "stab_iters outside [0, PBF_MAX_ITERS]");
    if (desc->stab_set < 1 || desc->stab_set > p.n_max)
        return fail(c, PBF_ERR_INVALID_ARG, "stab_set outside [1, n_max]");
    SceneDev s = c->scenes[scene];
    for (int o = 0; o < desc->count; ++o) {
        const pbf_obstacle &ob = desc->obstacles[o];
        const int used = ob.kind == PBF_OBSTACLE_SPHERE ? 1 : ob.kind == PBF_OBSTACLE_CONE ? 2 : 3;
        if (ob.kind < PBF_OBSTACLE_SPHERE || ob.kind > PBF_OBSTACLE_BOX)
            return fail(c, PBF_ERR_INVALID_ARG, "unknown obstacle kind");
        if (!finite3(ob.centre) || !finite3(ob.a))
            return fail(c, PBF_ERR_INVALID_ARG, "non-finite obstacle");
        for (int d = 0; d < used; ++d)
            if (!(ob.a[d] > 0.f)) return fail(c, PBF_ERR_INVALID_ARG, "obstacle sizes must be > 0");
        s.obst[o].kind = ob.kind;
        for (int d = 0; d < 3; ++d) {
            s.obst[o].c[d] = ob.centre[d];
            s.obst[o].a[d] = ob.a[d];
        }
    }
    for (int o = desc->count; o < kMaxObstacles; ++o) s.obst[o] = ObstacleDev{};
    s.n_obst = desc->count;
    s.stab_iters = desc->stab_iters;
    s.stab_s = desc->stab_set;
    HIPCHK(c, hipStreamSynchronize(c->stream), "stream synchronize");
    bool on = false;
    for (int k = 0; k < c->n_scenes; ++k) {
        const SceneDev &sd = k == scene ? s : c->scenes[k];
        on = on || sd.n_obst > 0;
    }
    if (on && !c->b.contact) {
        hipError_t e = dalloc(c, &c->b.contact, (size_t)c->n_total);
        if (e != hipSuccess) {
            c->b.contact = nullptr;
            return hip_fail(c, e, "contact buffer");
        }
        HIPCHK(c, hipMemsetAsync(c->b.contact, 0, (size_t)std::max<int64_t>(c->n_total, 1), c->stream),
               "clear contacts");
    }
    c->scenes[scene] = s;
    c->roll_valid = false;
    if (on != c->b.contacts_on) drop_graphs(c);  // the step's launches change
    c->b.contacts_on = on;
    HIPCHK(c, hipMemcpyAsync((void *)c->b.scenes, c->scenes.data(), sizeof(SceneDev) * c->scenes.size(),
                             hipMemcpyHostToDevice, c->stream), "upload scenes");
    HIPCHK(c, hipStreamSynchronize(c->stream), "stream synchronize");
    return PBF_OK;
}

pbf_status pbf_batch_set_cohesion(pbf_ctx *c, int32_t scene, float gamma)
{
    if (!c) return PBF_ERR_INVALID_ARG;
    if (scene < 0 || scene >= c->n_scenes) return fail(c, PBF_ERR_INVALID_ARG, "bad scene index");
    if (!(gamma >= 0.f) || !std::isfinite(gamma))
        return fail(c, PBF_ERR_INVALID_ARG, "cohesion must be finite and >= 0");
    const pbf_params &p = c->params[scene];
    SceneDev s = c->scenes[scene];
    const double h = p.h, pi = 3.14159265358979323846;
    s.cohesion = gamma;
    s.c_coh = (float)((double)gamma * p.mass * 32.0 * (double)p.dt * p.dt / (pi * std::pow(h, 9)));
    if (gamma > 0.f && !(std::isfinite(s.c_coh) && s.c_coh > 0.f))
        return fail(c, PBF_ERR_INVALID_ARG, "cohesion factor out of float range for this scene");
    HIPCHK(c, hipStreamSynchronize(c->stream), "stream synchronize");
    bool on = false;
    for (int k = 0; k < c->n_scenes; ++k) on = on || (k == scene ? s : c->scenes[k]).c_coh > 0.f;
    c->scenes[scene] = s;
    c->roll_valid = false;
    if (on != c->b.cohesion_on) drop_graphs(c);  // the step's launches change
    c->b.cohesion_on = on;
    HIPCHK(c, hipMemcpyAsync((void *)c->b.scenes, c->scenes.data(), sizeof(SceneDev) * c->scenes.size(),
                             hipMemcpyHostToDevice, c->stream), "upload scenes");
    HIPCHK(c, hipStreamSynchronize(c->stream), "stream synchronize");
    return PBF_OK;
}

pbf_status pbf_step(pbf_ctx *c, int32_t n_steps)
{
    if (!c) return PBF_ERR_INVALID_ARG;
    if (n_steps < 0) return fail(c, PBF_ERR_INVALID_ARG, "n_steps < 0");
    if (n_steps > 0) c->roll_valid = false;
    return step_n(c, n_steps);
}

}  // extern "C"

namespace {
pbf_status step_n(pbf_ctx *c, int32_t n_steps)
{
    for (int32_t k = 0; k < n_steps; ++k) {
        if (c->graph && !c->profiling && c->n_total > 0) {
            hipGraphExec_t &g = c->exec[c->cur];
            if (!g) {
                hipGraph_t graph = nullptr;
                HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal),
                       "begin capture");
                hipError_t e = enqueue_step(c->b, c->cur, c->ls, c->stream, nullptr);
                hipError_t e2 = hipStreamEndCapture(c->stream, &graph);
                if (e != hipSuccess) return hip_fail(c, e, "capture step");
                if (e2 != hipSuccess) return hip_fail(c, e2, "end capture");
                e = hipGraphInstantiate(&g, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (e != hipSuccess) {
                    g = nullptr;
                    return hip_fail(c, e, "instantiate graph");
                }
            }
            HIPCHK(c, hipGraphLaunch(g, c->stream), "launch graph");
        } else {
            HIPCHK(c, enqueue_step(c->b, c->cur, c->ls, c->stream,
                                   c->profiling ? &c->timer : nullptr), "enqueue step");
            if (c->profiling) {
                if (c->timer.status != hipSuccess) return hip_fail(c, c->timer.status, "profiling events");
                HIPCHK(c, timer_collect(&c->timer, c->stream), "collect timings");
            }
        }
        c->cur ^= 1;
        c->step += 1;
        c->stepped = true;
    }
    return PBF_OK;
}
}  // namespace

extern "C" {

pbf_status pbf_sync(pbf_ctx *c)
{
    if (!c) return PBF_ERR_INVALID_ARG;
    HIPCHK(c, hipStreamSynchronize(c->stream), "stream synchronize");
    return latched(c);
}

pbf_status pbf_read_positions(pbf_ctx *c, float *out, int32_t on_device)
{
    if (!c) return PBF_ERR_INVALID_ARG;
    if (!out && c->n_total) return fail(c, PBF_ERR_INVALID_ARG, "out is NULL");
    return read_by_id(c, c->b.x[c->cur], out, on_device, 0, c->n_total);
}

pbf_status pbf_read_velocities(pbf_ctx *c, float *out, int32_t on_device)
{
    if (!c) return PBF_ERR_INVALID_ARG;
    if (!out && c->n_total) return fail(c, PBF_ERR_INVALID_ARG, "out is NULL");
    return read_by_id(c, c->b.v[c->cur], out, on_device, 0, c->n_total);
}

pbf_status pbf_batch_read_positions(pbf_ctx *c, int32_t scene, float *out, int32_t on_device)
{
    if (!c) return PBF_ERR_INVALID_ARG;
    if (scene < 0 || scene >= c->n_scenes) return fail(c, PBF_ERR_INVALID_ARG, "bad scene index");
    if (!out && c->params[scene].n) return fail(c, PBF_ERR_INVALID_ARG, "out is NULL");
    return read_by_id(c, c->b.x[c->cur], out, on_device, c->pid_off[scene], c->pid_off[scene + 1]);
}

pbf_status pbf_get_counts(const pbf_ctx *c, int32_t *n_scenes, int64_t *n_total)
{
    if (!c) return PBF_ERR_INVALID_ARG;
    if (n_scenes) *n_scenes = c->n_scenes;
    if (n_total) *n_total = c->n_total;
    return PBF_OK;
}

pbf_status pbf_set_graph(pbf_ctx *c, int32_t enable)
{
    if (!c) return PBF_ERR_INVALID_ARG;
    c->graph = enable != 0;
    if (!c->graph) {
        HIPCHK(c, hipStreamSynchronize(c->stream), "stream synchronize");
        drop_graphs(c);
    }
    return PBF_OK;
}

pbf_status pbf_set_block_size(pbf_ctx *c, int32_t kernel, int32_t threads)
{
    if (!c) return PBF_ERR_INVALID_ARG;
    if (kernel < 0 || kernel >= K_COUNT) return fail(c, PBF_ERR_INVALID_ARG, "bad kernel index");
    if (threads == 0) threads = kDefaultBlock[kernel];
    if (threads < 64 || threads > max_block(kernel) || threads % 64)
        return fail(c, PBF_ERR_INVALID_ARG, "threads must be a multiple of 64 in [64, 1024] "
                                            "(at most 512 for neighbours, lambda and update)");
    if (fixed_shape(kernel) && threads != kDefaultBlock[kernel])
        return fail(c, PBF_ERR_INVALID_ARG, "this kernel has a fixed launch shape");
    if (c->ls.block[kernel] != threads) {
        HIPCHK(c, hipStreamSynchronize(c->stream), "stream synchronize");
        drop_graphs(c);
        c->ls.block[kernel] = threads;
    }
    return PBF_OK;
}

pbf_status pbf_profile_enable(pbf_ctx *c, int32_t enable)
{
    if (!c) return PBF_ERR_INVALID_ARG;
    c->profiling = enable != 0;
    for (int k = 0; k < K_COUNT; ++k) {
        c->timer.total_ms[k] = 0.0;
        c->timer.launches[k] = 0;
    }
    c->timer.used = 0;
    c->timer.status = hipSuccess;
    return PBF_OK;
}

pbf_status pbf_profile_read(pbf_ctx *c, double *total_ms, int64_t *launches, int32_t count)
{
    if (!c) return PBF_ERR_INVALID_ARG;
    if (count < 0 || count > K_COUNT || (count && (!total_ms || !launches)))
        return fail(c, PBF_ERR_INVALID_ARG, "bad output arrays");
    HIPCHK(c, hipStreamSynchronize(c->stream), "stream synchronize");
    for (int k = 0; k < count; ++k) {
        total_ms[k] = c->timer.total_ms[k];
        launches[k] = c->timer.launches[k];
    }
    return PBF_OK;
}

pbf_status pbf_stats(pbf_ctx *c, pbf_step_stats *o)
{
    if (!c || !o) return PBF_ERR_INVALID_ARG;
    std::memset(o, 0, sizeof *o);
    pbf_status st = need_step(c);
    if (st != PBF_OK) return st;
    std::vector<uint32_t> meta;
    std::vector<uint8_t> lv;
    std::vector<unsigned long long> tot;
    if ((st = d2h(c, tot, c->b.totals, 2)) != PBF_OK) return st;
    o->total_particle_iterations = (int64_t)tot[0];
    o->total_steps = (int64_t)tot[1];
    if ((st = d2h(c, lv, (const uint8_t *)c->b.lvl[c->cur], (size_t)c->n_total)) != PBF_OK) return st;
    if ((st = d2h(c, meta, c->b.pmeta, (size_t)c->n_total)) != PBF_OK) return st;
    o->n_iters = c->b.n_iters;
    for (uint8_t L : lv) {
        for (int k = 0; k < (int)L && k < PBF_MAX_ITERS; ++k) o->active[k] += 1;
        o->particle_iterations += L;
    }
    for (uint32_t m : meta) {
        int32_t cnt = (int32_t)(m & kMetaCount);
        o->neighbour_pairs += cnt;
        o->max_neighbours = std::max(o->max_neighbours, cnt);
    }
    // staged neighbourhood of every tile with particles (saved stage tables,
    // by slot in the tile order; the tiles with particles come first)
    std::vector<uint32_t> tcount, rows, order;
    const size_t T = c->b.n_tiles;
    if ((st = d2h(c, tcount, c->b.tile_count, T)) != PBF_OK) return st;
    if ((st = d2h(c, order, c->b.tile_order, T)) != PBF_OK) return st;
    if ((st = d2h(c, rows, c->b.tile_rows, T * (size_t)kRowWords)) != PBF_OK) return st;
    for (size_t t = 0; t < T; ++t) {
        if (!tcount[order[t]]) continue;
        const uint32_t staged = rows[t * (size_t)kRowWords + kBndWords + kStageRows];
        o->max_stage = std::max(o->max_stage, (int32_t)staged);
        if (staged > (uint32_t)kStageCap) o->tiles_unstaged += 1;
    }
    return latched(c);
}

pbf_status pbf_debug_keys(pbf_ctx *c, uint32_t *keys)
{
    if (!c || (!keys && c->n_total)) return PBF_ERR_INVALID_ARG;
    pbf_status st = need_step(c);
    if (st != PBF_OK) return st;
    std::vector<uint32_t> k, id;
    std::vector<float4> x;
    if ((st = d2h(c, k, c->b.key, (size_t)c->n_total)) != PBF_OK) return st;
    if ((st = d2h(c, id, c->b.id[c->cur], (size_t)c->n_total)) != PBF_OK) return st;
    for (size_t s = 0; s < k.size(); ++s) {
        // scene of the particle from its global ID
        int32_t sc = (int32_t)(std::upper_bound(c->pid_off.begin(), c->pid_off.end(), (int64_t)id[s]) -
                               c->pid_off.begin()) - 1;
        keys[id[s]] = k[s] - c->scenes[sc].cell_off;
    }
    return PBF_OK;
}

pbf_status pbf_debug_permutation(pbf_ctx *c, int32_t *ids)
{
    if (!c || (!ids && c->n_total)) return PBF_ERR_INVALID_ARG;
    pbf_status st = need_step(c);
    if (st != PBF_OK) return st;
    std::vector<uint32_t> id;
    if ((st = d2h(c, id, c->b.id[c->cur], (size_t)c->n_total)) != PBF_OK) return st;
    for (size_t s = 0; s < id.size(); ++s) ids[s] = (int32_t)id[s];
    return PBF_OK;
}

pbf_status pbf_debug_neighbours(pbf_ctx *c, int32_t *counts, int32_t *ids, int64_t cap,
                                int64_t *total)
{
    if (!c || (!counts && c->n_total) || !total) return PBF_ERR_INVALID_ARG;
    pbf_status st = need_step(c);
    if (st != PBF_OK) return st;
    const size_t n = (size_t)c->n_total;
    std::vector<uint32_t> meta, slot, id;
    if ((st = d2h(c, meta, c->b.pmeta, n)) != PBF_OK) return st;
    if ((st = d2h(c, slot, c->b.pslot, n)) != PBF_OK) return st;
    if ((st = d2h(c, id, c->b.id[c->cur], n)) != PBF_OK) return st;
    std::vector<int64_t> off(n + 1, 0);
    for (size_t p = 0; p < n; ++p) counts[id[slot[p]]] = (int32_t)(meta[p] & kMetaCount);
    for (size_t g = 0; g < n; ++g) off[g + 1] = off[g] + counts[g];
    *total = off[n];
    if (!ids || cap < off[n] || n == 0) return PBF_OK;
    // decode the codes with each tile's saved tables (host side; the tables
    // are stored by the tile's slot in the tile order)
    const size_t T = c->b.n_tiles, stride = (size_t)c->b.nbr_stride;
    std::vector<uint32_t> tstart, tcount, rows, order;
    std::vector<uint16_t> codes;
    if ((st = d2h(c, tstart, c->b.tile_start, T + 1)) != PBF_OK) return st;
    if ((st = d2h(c, tcount, c->b.tile_count, T)) != PBF_OK) return st;
    if ((st = d2h(c, order, c->b.tile_order, T)) != PBF_OK) return st;
    if ((st = d2h(c, rows, c->b.tile_rows, T * (size_t)kRowWords)) != PBF_OK) return st;
    if ((st = d2h(c, codes, (const uint16_t *)c->b.nbr, n * stride)) != PBF_OK) return st;
    // group g of particle p holds codes 8g..8g+7 at u16 offset 8 (g n + p)
    auto code_at = [&](size_t p, int32_t q) -> uint32_t {
        return codes[8 * ((size_t)(q / 8) * n + p) + (size_t)(q % 8)];
    };
    for (size_t sl = 0; sl < T; ++sl) {
        const uint32_t t = order[sl];
        if (!tcount[t]) continue;  // no tables saved
        const uint32_t *bnd = rows.data() + sl * (size_t)kRowWords;  // [row][x], then LDS bases
        const uint32_t *base = bnd + kBndWords;
        const bool fits = base[kStageRows] <= (uint32_t)kStageCap;
        for (uint32_t pl = 0; pl < tcount[t]; ++pl) {
            const size_t p = (size_t)tstart[t] + pl;
            const int32_t cnt = (int32_t)(meta[p] & kMetaCount);
            int32_t *dst = ids + off[id[slot[p]]];
            for (int32_t q = 0; q < cnt; ++q) {
                const uint32_t code = code_at(p, q);
                uint32_t s;
                if (fits) {
                    int r = 0;
                    while (base[r + 1] <= code) ++r;
                    s = bnd[r * (kStageEdge + 1)] + (code - base[r]);
                } else {
                    s = bnd[(code >> kSegOffBits) * (kStageEdge + 1)] +
                        (code & ((1u << kSegOffBits) - 1));
                }
                dst[q] = (int32_t)id[s];
            }
            std::sort(dst, dst + cnt);
        }
    }
    return PBF_OK;
}

pbf_status pbf_debug_lambda(pbf_ctx *c, float *lambda)
{
    if (!c || (!lambda && c->n_total)) return PBF_ERR_INVALID_ARG;
    pbf_status st = need_step(c);
    if (st != PBF_OK) return st;
    std::vector<float4> xs;
    std::vector<uint32_t> id;
    if ((st = d2h(c, xs, (const float4 *)c->b.xs[c->b.n_iters & 1], (size_t)c->n_total)) != PBF_OK) return st;
    if ((st = d2h(c, id, c->b.id[c->cur], (size_t)c->n_total)) != PBF_OK) return st;
    for (size_t s = 0; s < id.size(); ++s) lambda[id[s]] = xs[s].w;
    return PBF_OK;
}

pbf_status pbf_density(pbf_ctx *c, double *out, float *rho_rel, int32_t on_device)
{
    if (!c || !out) return PBF_ERR_INVALID_ARG;
    pbf_status st = need_step(c);
    if (st != PBF_OK) return st;
    const int64_t n = c->n_total;
    if (n == 0) {
        out[0] = out[1] = 0.0;
        return PBF_OK;
    }
    DensityBuffers &d = c->dens;
    if (!d.out) {
        // allocated by the first call and kept; a failed attempt frees what
        // it allocated and leaves the context as it was
        const size_t T = c->b.n_tiles, parts = (T + kXcds - 1) / kXcds * kXcds;
        DensityBuffers nd{};
        float *rho_id_buf = nullptr;
        std::vector<void *> got;
        hipError_t e = hipSuccess;
        auto al = [&](auto **ptr, size_t count) {
            if (e != hipSuccess) return;
            void *q = nullptr;
            e = dev_malloc(&q, std::max<size_t>(count, 1) * sizeof(**ptr));
            if (e == hipSuccess) {
                got.push_back(q);
                *ptr = (std::remove_reference_t<decltype(*ptr)>)q;
            }
        };
        al(&nd.xs, (size_t)n);
        al(&nd.key, (size_t)n);
        al(&nd.nbr, (size_t)n * (size_t)(c->b.nbr_stride / 8));
        al(&nd.pmeta, (size_t)n);
        al(&nd.pslot, (size_t)n);
        al(&nd.tile_rows, T * kRowWords);
        al(&nd.tile_rec, T);
        al(&nd.tile_order, T);
        al(&nd.tile_start, T + 1);
        al(&nd.tile_count, T);
        al(&nd.tile_ge, (size_t)PBF_MAX_ITERS + 2);
        al(&nd.tile_lvl, T);
        al(&nd.err, 1);
        al(&nd.totals, 2);
        al(&nd.rho_slot, (size_t)n);
        al(&nd.part_sum, parts);
        al(&nd.part_max, parts);
        al(&rho_id_buf, (size_t)n);
        al(&nd.out, 2);
        if (e != hipSuccess) {
            for (void *q : got) dev_free(q);
            return hip_fail(c, e, "density buffers");
        }
        c->allocs.insert(c->allocs.end(), got.begin(), got.end());
        d = nd;
        c->dens_rho_id = rho_id_buf;
    }
    HIPCHK(c, hipMemsetAsync(d.err, 0, sizeof(uint32_t), c->stream), "clear faults");
    return density_run(c, d, c->dens_rho_id, out, rho_rel, on_device);
}

pbf_status pbf_density_noalloc(pbf_ctx *c, double *out, float *rho_rel, int32_t on_device)
{
    if (!c || !out) return PBF_ERR_INVALID_ARG;
    pbf_status st = need_step(c);
    if (st != PBF_OK) return st;
    const int64_t n = c->n_total;
    if (n == 0) {
        out[0] = out[1] = 0.0;
        return PBF_OK;
    }
    DensityBuffers d{};
    float *rho_stage = nullptr;
    const size_t need = static_density_layout(c, nullptr, d, rho_stage);
    if (need > (size_t)kStaticScratchBytes) {
        char msg[192];
        std::snprintf(msg, sizeof msg,
                      "pbf_density_noalloc: needs %zu bytes of work space, the static array "
                      "holds %lld",
                      need, (long long)kStaticScratchBytes);
        return fail(c, PBF_ERR_INVALID_ARG, msg);
    }
    unsigned char *base = nullptr;
    HIPCHK(c, static_scratch(c->device, &base), "static scratch address");
    static_density_layout(c, base, d, rho_stage);
    HIPCHK(c, clear_words(d.err, 1, c->stream), "clear faults");
    return density_run(c, d, rho_stage, out, rho_rel, on_device);
}

pbf_status pbf_debug_levels(pbf_ctx *c, uint8_t *levels)
{
    if (!c || (!levels && c->n_total)) return PBF_ERR_INVALID_ARG;
    pbf_status st = need_step(c);
    if (st != PBF_OK) return st;
    std::vector<uint8_t> lv;
    std::vector<uint32_t> id;
    if ((st = d2h(c, lv, (const uint8_t *)c->b.lvl[c->cur], (size_t)c->n_total)) != PBF_OK) return st;
    if ((st = d2h(c, id, c->b.id[c->cur], (size_t)c->n_total)) != PBF_OK) return st;
    for (size_t s = 0; s < id.size(); ++s) levels[id[s]] = lv[s];
    return PBF_OK;
}

pbf_status pbf_debug_contacts(pbf_ctx *c, uint8_t *mask)
{
    if (!c || (!mask && c->n_total)) return PBF_ERR_INVALID_ARG;
    pbf_status st = need_step(c);
    if (st != PBF_OK) return st;
    if (!c->b.contacts_on) {
        std::fill(mask, mask + c->n_total, (uint8_t)0);
        return PBF_OK;
    }
    std::vector<uint8_t> m;
    std::vector<uint32_t> id;
    if ((st = d2h(c, m, (const uint8_t *)c->b.contact, (size_t)c->n_total)) != PBF_OK) return st;
    if ((st = d2h(c, id, c->b.id[c->cur], (size_t)c->n_total)) != PBF_OK) return st;
    for (size_t s = 0; s < id.size(); ++s) mask[id[s]] = m[s];
    return PBF_OK;
}

pbf_status pbf_debug_poison(pbf_ctx *c, int32_t enable)
{
    if (!c) return PBF_ERR_INVALID_ARG;
    if (enable != 0 && enable != 1) return fail(c, PBF_ERR_INVALID_ARG, "enable must be 0 or 1");
    const bool on = enable != 0;
    if (on != c->b.poison) {
        HIPCHK(c, hipStreamSynchronize(c->stream), "stream synchronize");
        drop_graphs(c);  // the step's launches change
    }
    c->b.poison = on;
    return PBF_OK;
}

pbf_status pbf_get_state(pbf_ctx *c, float *x, float *v, int64_t *step)
{
    if (!c || ((!x || !v) && c->n_total)) return PBF_ERR_INVALID_ARG;
    pbf_status st = read_by_id(c, c->b.x[c->cur], x, 0, 0, c->n_total);
    if (st != PBF_OK) return st;
    st = read_by_id(c, c->b.v[c->cur], v, 0, 0, c->n_total);
    if (st != PBF_OK) return st;
    if (step) *step = c->step;
    return PBF_OK;
}

pbf_status pbf_set_state(pbf_ctx *c, const float *x, const float *v, int64_t step)
{
    if (!c || ((!x || !v) && c->n_total) || step < 0) return PBF_ERR_INVALID_ARG;
    for (int64_t i = 0; i < c->n_total; ++i)
        if (!finite3(x + 3 * i) || !finite3(v + 3 * i))
            return fail(c, PBF_ERR_NONFINITE, "non-finite state");
    HIPCHK(c, hipStreamSynchronize(c->stream), "stream synchronize");
    pbf_status st = upload_state(c, x, v);
    if (st != PBF_OK) return st;
    HIPCHK(c, hipMemsetAsync(c->b.err, 0, sizeof(uint32_t), c->stream), "clear faults");
    HIPCHK(c, hipMemsetAsync(c->b.totals, 0, 2 * sizeof(unsigned long long), c->stream),
           "clear totals");
    HIPCHK(c, hipStreamSynchronize(c->stream), "stream synchronize");
    c->step = step;
    c->stepped = false;
    c->roll_valid = false;
    return PBF_OK;
}

pbf_status pbf_rollout_forward(pbf_ctx *c, int32_t n_steps, int32_t ckpt_every)
{
    if (!c) return PBF_ERR_INVALID_ARG;
    if (n_steps < 1 || ckpt_every < 1)
        return fail(c, PBF_ERR_INVALID_ARG, "need n_steps >= 1 and ckpt_every >= 1");
    if (c->b.contacts_on)
        return fail(c, PBF_ERR_INVALID_ARG, "the rollout does not differentiate obstacle contacts");
    if (c->b.cohesion_on)
        return fail(c, PBF_ERR_INVALID_ARG, "the rollout does not differentiate the cohesion force");
    for (const pbf_params &p : c->params)
        if (p.flags & PBF_FLAG_UNILATERAL)
            return fail(c, PBF_ERR_INVALID_ARG,
                        "the rollout does not differentiate the unilateral constraint");
    HIPCHK(c, hipStreamSynchronize(c->stream), "stream synchronize");
    c->roll_valid = false;
    const size_t n3 = (size_t)c->n_total * 3;
    const int32_t nck = (n_steps + ckpt_every - 1) / ckpt_every;
    if (c->ckpt.size() != (size_t)(2 * nck)) {  // kept from the last rollout if the count matches
        for (float *p : c->ckpt) dev_free(p);
        c->ckpt.clear();
        for (int32_t k = 0; k < 2 * nck; ++k) {
            float *p = nullptr;
            hipError_t e = dev_malloc((void **)&p, std::max<size_t>(n3, 1) * sizeof(float));
            if (e != hipSuccess) {
                for (float *q : c->ckpt) dev_free(q);
                c->ckpt.clear();
                return hip_fail(c, e, "checkpoint buffers");
            }
            c->ckpt.push_back(p);
        }
    }
    for (int32_t s = 0; s < n_steps; ++s) {
        if (s % ckpt_every == 0) {
            const int32_t k = s / ckpt_every;
            HIPCHK(c, enqueue_unpermute(c->n_total, c->b.x[c->cur], c->b.id[c->cur], c->ckpt[2 * k],
                                        0, (uint32_t)c->n_total, c->stream), "checkpoint x");
            HIPCHK(c, enqueue_unpermute(c->n_total, c->b.v[c->cur], c->b.id[c->cur],
                                        c->ckpt[2 * k + 1], 0, (uint32_t)c->n_total, c->stream),
                   "checkpoint v");
        }
        pbf_status st = step_n(c, 1);
        if (st != PBF_OK) return st;
    }
    c->roll_steps = n_steps;
    c->roll_every = ckpt_every;
    c->roll_valid = true;
    return PBF_OK;
}

pbf_status pbf_rollout_backward(pbf_ctx *c, const float *dl_dx, const float *dl_dv, float *dl_dx0,
                                float *dl_dv0, int32_t on_device)
{
    if (!c) return PBF_ERR_INVALID_ARG;
    if (!c->roll_valid)
        return fail(c, PBF_ERR_INVALID_ARG, "no rollout to reverse (pbf_rollout_forward, then no "
                                            "other step or state change)");
    const int64_t n = c->n_total;
    const size_t n3 = (size_t)n * 3;
    if (n && (!dl_dx || !dl_dv || !dl_dx0 || !dl_dv0))
        return fail(c, PBF_ERR_INVALID_ARG, "null gradient buffer");
    if (n == 0) return PBF_OK;
    const int K = c->b.n_iters;
    const int32_t T = c->roll_steps, C = c->roll_every;
    const int32_t seg_len = std::min(C, T);
    auto &rs = c->rs;
    if (rs.seg_len != seg_len) {  // (re)allocate the work buffers for this segment length
        for (void *p : rs.bufs) dev_free(p);
        rs.bufs.clear();
        rs.seg_len = 0;
        auto alloc = [&](size_t bytes) -> void * {
            void *p = nullptr;
            if (dev_malloc(&p, bytes) != hipSuccess) return nullptr;
            rs.bufs.push_back(p);
            return p;
        };
        // adjoint state (ID order), the final state to restore afterwards, and
        // the running totals (the recomputed steps must not count in them)
        rs.ax = (float *)alloc(n3 * 4);
        rs.av = (float *)alloc(n3 * 4);
        rs.fx = (float *)alloc(n3 * 4);
        rs.fv = (float *)alloc(n3 * 4);
        rs.tot = (unsigned long long *)alloc(2 * sizeof(unsigned long long));
        AdjointScratch &w = rs.w;
        w.nslot = (uint32_t *)alloc((size_t)n * c->b.nbr_cap * 4);
        w.zb = (float4 *)alloc((size_t)n * 16);
        w.xb = (float4 *)alloc((size_t)n * 16);
        w.dpb = (float4 *)alloc((size_t)n * 16);
        w.gc = (float4 *)alloc((size_t)n * 16);
        w.lb = (float *)alloc((size_t)n * 4);
        w.sb = (float *)alloc((size_t)n * 4);
        rs.recs.assign((size_t)seg_len, StepRecord{});
        const size_t T_t = c->b.n_tiles;
        bool ok = rs.ax && rs.av && rs.fx && rs.fv && rs.tot && w.nslot && w.zb && w.xb && w.dpb &&
                  w.gc && w.lb && w.sb;
        for (auto &r : rs.recs) {
            if (!ok) break;
            r.id = (uint32_t *)alloc((size_t)n * 4);
            r.lvl = (uint8_t *)alloc((size_t)n);
            r.nbr = (uint4 *)alloc((size_t)n * (c->b.nbr_stride / 8) * 16);
            r.pmeta = (uint32_t *)alloc((size_t)n * 4);
            r.pslot = (uint32_t *)alloc((size_t)n * 4);
            r.tile_rows = (uint32_t *)alloc(T_t * kRowWords * 4);
            r.tile_rec = (uint4 *)alloc(T_t * 16);
            r.tile_order = (uint32_t *)alloc(T_t * 4);
            r.tile_start = (uint32_t *)alloc((T_t + 1) * 4);
            r.tile_count = (uint32_t *)alloc(T_t * 4);
            r.tile_ge = (uint32_t *)alloc((PBF_MAX_ITERS + 2) * 4);
            ok = r.id && r.lvl && r.nbr && r.pmeta && r.pslot && r.tile_rows && r.tile_rec && r.tile_order &&
                 r.tile_start && r.tile_count && r.tile_ge;
            for (int k = 0; k <= K && ok; ++k) ok = (r.snap[k] = (float4 *)alloc((size_t)n * 16)) != nullptr;
        }
        if (!ok) {
            for (void *p : rs.bufs) dev_free(p);
            rs.bufs.clear();
            return fail(c, PBF_ERR_OUT_OF_MEMORY, "rollout backward buffers");
        }
        rs.seg_len = seg_len;
    }
    float *ax = rs.ax, *av = rs.av, *fx = rs.fx, *fv = rs.fv;
    unsigned long long *tot = rs.tot;
    const AdjointScratch &w = rs.w;
    std::vector<StepRecord> &recs = rs.recs;
    hipError_t e = hipSuccess;
    const hipMemcpyKind kin = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    const hipMemcpyKind kout = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
#define BCHK(X, WHAT)                                  \
    do {                                               \
        if ((e = (X)) != hipSuccess) {                 \
            pbf_status r_ = hip_fail(c, e, WHAT);      \
            (void)hipStreamSynchronize(c->stream);     \
            return r_;                                 \
        }                                              \
    } while (0)
    BCHK(hipMemcpyAsync(tot, c->b.totals, 2 * sizeof(unsigned long long), hipMemcpyDeviceToDevice,
                        c->stream), "save totals");
    BCHK(hipMemcpyAsync(ax, dl_dx, n3 * 4, kin, c->stream), "gradient in");
    BCHK(hipMemcpyAsync(av, dl_dv, n3 * 4, kin, c->stream), "gradient in");
    BCHK(enqueue_unpermute(n, c->b.x[c->cur], c->b.id[c->cur], fx, 0, (uint32_t)n, c->stream), "save state");
    BCHK(enqueue_unpermute(n, c->b.v[c->cur], c->b.id[c->cur], fv, 0, (uint32_t)n, c->stream), "save state");
    const int32_t nseg = (T + C - 1) / C;
    for (int32_t seg = nseg - 1; seg >= 0; --seg) {
        const int32_t s0 = seg * C, s1 = std::min(s0 + C, T);
        // recompute the segment from its checkpoint, recording every step
        BCHK(enqueue_load_state(n, c->ckpt[2 * seg], c->ckpt[2 * seg + 1], c->b.id_scene,
                                c->b.x[0], c->b.v[0], c->b.id[0], c->stream), "load checkpoint");
        c->cur = 0;
        for (int32_t j = 0; j < s1 - s0; ++j) {
            BCHK(enqueue_step(c->b, c->cur, c->ls, c->stream, nullptr, &recs[j]), "recompute step");
            c->cur ^= 1;
        }
        for (int32_t j = s1 - s0 - 1; j >= 0; --j)
            BCHK(enqueue_adjoint_step(c->b, recs[j], ax, av, ax, av, w, c->stream), "adjoint step");
    }
    BCHK(hipMemcpyAsync(dl_dx0, ax, n3 * 4, kout, c->stream), "gradient out");
    BCHK(hipMemcpyAsync(dl_dv0, av, n3 * 4, kout, c->stream), "gradient out");
    // back to the final state of the rollout (storage order = ID order)
    BCHK(enqueue_load_state(n, fx, fv, c->b.id_scene, c->b.x[0], c->b.v[0], c->b.id[0], c->stream),
         "restore state");
    BCHK(hipMemcpyAsync(c->b.totals, tot, 2 * sizeof(unsigned long long), hipMemcpyDeviceToDevice,
                        c->stream), "restore totals");
    c->cur = 0;
    c->stepped = false;
    BCHK(hipStreamSynchronize(c->stream), "stream synchronize");
#undef BCHK
    return latched(c);
}

}  // extern "C"
