// gfx950 kernels of one adaptive PBF step (Section 5, Fig. 7 of the paper).
//
// Data layout in HBM (all scenes of a context concatenated):
//   x, v      float4[n]  slot order (cell-sorted); x.w holds the scene index bits
//   xs[2]     float4[n]  predicted positions x*, ping-pong across solver
//                        iterations; .w holds lambda_i
//   id, lvl   u32/u8[n]  particle ID and level N_i per slot
//   key       u32[n]     global cell key per slot (scene cell offset + local key)
//   cell_start u32[G+1]  first slot of every cell (exclusive scan of counts)
//   order     u32[n]     level buckets: t -> slot, descending N_i, ties by slot,
//                        so the active set P_k of iteration k is order[0, |P_k|)
//   nbr       u32[cap][n] neighbour slots, column-major by t (coalesced)
//   nmeta     u32[n]     by t: scene << 16 | neighbour count
//
// Every kernel is gather-only (no floating-point atomics), so a step is
// deterministic; integer atomics are used only for cell counts and tickets,
// and the tickets are replaced by a rank by particle ID before use.
#include "pbf_internal.h"
#include "../../include/pbf.h"

namespace pbf {

const char *const kKernelNames[K_COUNT] = {
    "fill",         "lod_predict",  "scan_reduce",   "scan_top",     "scan_apply",
    "sort_scatter", "sort_finish",  "neighbours",    "level_count",  "level_scan",
    "level_scatter", "lambda",      "update",        "commit"};

const int kDefaultBlock[K_COUNT] = {256, 256, kScanBlock, 1024, kScanBlock, 256, 256,
                                    256, kLevelBlock, 1024, kLevelBlock, 256, 256, 256};

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

__device__ __forceinline__ int cell_coord(float p, float lo, float h, int dims)
{
    int c = (int)floorf((p - lo) / h);
    return min(max(c, 0), dims - 1);
}

__device__ __forceinline__ float clampf(float v, float lo, float hi)
{
    return fminf(fmaxf(v, lo), hi);
}

// Distance-to-camera level (linear map of the distance to the level range,
// Section 4.1).  The level is an integer chosen by floating point, so the
// operations are fixed: float32, no contraction into FMAs, correctly rounded
// square root and division, in this order.
__device__ __forceinline__ int dtc_level(float x, float y, float z, float cx, float cy, float cz,
                                         float d_near, float d_far, int nmin, int nmax)
{
#pragma clang fp contract(off)
    const float dx = x - cx, dy = y - cy, dz = z - cz;
    float d2 = dx * dx;
    d2 = d2 + dy * dy;
    d2 = d2 + dz * dz;
    const float d = sqrtf(d2);
    float t = (d - d_near) / (d_far - d_near);
    t = fminf(fmaxf(t, 0.f), 1.f);
    const int L = nmax - (int)floorf(t * (float)(nmax - nmin + 1));
    return min(max(L, nmin), nmax);
}

// ------------------------------------------------------------------ fill
__global__ void k_fill(uint32_t *__restrict__ p, uint32_t n, uint32_t value)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = value;
}

// --------------------------------------------- levels + forces + prediction
// Fig. 7 first loop for every particle, plus the level N_i (Eq. 8, adaption
// model of Section 4.1) from the position at the start of the step, the cell
// key of x*, and a ticket inside its cell from the counting-sort histogram.
__global__ void k_lod_predict(int64_t n, const SceneDev *__restrict__ sc,
                              const float4 *__restrict__ x, float4 *__restrict__ v,
                              const uint32_t *__restrict__ id, const uint8_t *__restrict__ lev_by_id,
                              float4 *__restrict__ xs_pred, uint8_t *__restrict__ lvl,
                              uint32_t *__restrict__ key, uint32_t *__restrict__ ticket,
                              uint32_t *__restrict__ cell_count)
{
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    float4 xi = x[s];
    const SceneDev &S = sc[__float_as_int(xi.w)];
    const int nmin = S.n_min, nmax = S.n_max;
    int L;
    if (S.lod_mode == PBF_LOD_EXPLICIT) {
        L = lev_by_id[id[s]];
    } else if (S.lod_mode == PBF_LOD_DTC) {
        L = dtc_level(xi.x, xi.y, xi.z, S.cam[0], S.cam[1], S.cam[2], S.d_near, S.d_far, nmin,
                      nmax);
    } else {
        L = nmax;
    }
    const float dt = S.dt;
    float4 vi = v[s];
    vi.x += dt * S.g[0];
    vi.y += dt * S.g[1];
    vi.z += dt * S.g[2];
    float px = clampf(xi.x + dt * vi.x, S.lo[0], S.hi[0]);
    float py = clampf(xi.y + dt * vi.y, S.lo[1], S.hi[1]);
    float pz = clampf(xi.z + dt * vi.z, S.lo[2], S.hi[2]);
    v[s] = vi;
    xs_pred[s] = make_float4(px, py, pz, 0.f);
    lvl[s] = (uint8_t)L;
    const float h = S.h;
    int cx = cell_coord(px, S.lo[0], h, S.dims[0]);
    int cy = cell_coord(py, S.lo[1], h, S.dims[1]);
    int cz = cell_coord(pz, S.lo[2], h, S.dims[2]);
    uint32_t k = S.cell_off + (uint32_t)(((int64_t)cz * S.dims[1] + cy) * S.dims[0] + cx);
    key[s] = k;
    ticket[s] = atomicAdd(&cell_count[k], 1u);
}

// --------------------------------------------------- exclusive scan of cells
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

__global__ void k_scan_apply(const uint32_t *__restrict__ in, uint32_t G,
                             const uint32_t *__restrict__ part, uint32_t *__restrict__ out)
{
    __shared__ uint32_t lds[1024 / 64 + 1];
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
    uint32_t run = part[blockIdx.x] + block_exclusive_sum(sum, lds, nullptr);
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
__global__ void k_sort_finish(int64_t n, const uint32_t *__restrict__ tmp_src,
                              const uint32_t *__restrict__ tmp_id,
                              const uint32_t *__restrict__ key_pre,
                              const uint32_t *__restrict__ cell_start,
                              const float4 *__restrict__ x, const float4 *__restrict__ v,
                              const float4 *__restrict__ xs_pred,
                              const uint8_t *__restrict__ lvl_in, float4 *__restrict__ x_out,
                              float4 *__restrict__ v_out, float4 *__restrict__ xs_out,
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
    v_out[f] = v[s];
    xs_out[f] = xs_pred[s];
    id_out[f] = my;
    lvl_out[f] = lvl_in[s];
    key_out[f] = k;
}

// ------------------------------------------------------ neighbour lists
// N_i = { j != i : |x*_i - x*_j|^2 < h^2 } over the 27 cells around x*_i:
// nine x-contiguous slot ranges (rows dz, dy in {-1, 0, 1}), Fig. 7 second
// loop.  Lists are written at the particle's level-bucket position t.
__global__ void k_neighbours(int64_t n, const SceneDev *__restrict__ sc,
                             const uint32_t *__restrict__ order, const float4 *__restrict__ xs,
                             const float4 *__restrict__ x, const uint32_t *__restrict__ key,
                             const uint32_t *__restrict__ cell_start, int cap,
                             uint32_t *__restrict__ nbr, uint32_t *__restrict__ nmeta,
                             uint32_t *__restrict__ err)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const uint32_t i = order[t];
    const int scn = __float_as_int(x[i].w);
    const SceneDev &S = sc[scn];
    const float h2 = S.h2;
    const int gx = S.dims[0], gy = S.dims[1], gz = S.dims[2];
    const uint32_t coff = S.cell_off;
    const float4 xi = xs[i];
    const uint32_t kl = key[i] - coff;
    const int cx = (int)(kl % (uint32_t)gx);
    const int cy = (int)((kl / (uint32_t)gx) % (uint32_t)gy);
    const int cz = (int)(kl / ((uint32_t)gx * (uint32_t)gy));
    const int x0 = max(cx - 1, 0), x1 = min(cx + 1, gx - 1);
    uint32_t cnt = 0;
    for (int zz = max(cz - 1, 0); zz <= min(cz + 1, gz - 1); ++zz) {
        for (int yy = max(cy - 1, 0); yy <= min(cy + 1, gy - 1); ++yy) {
            const uint32_t row = coff + (uint32_t)(((int64_t)zz * gy + yy) * gx);
            const uint32_t j0 = cell_start[row + x0], j1 = cell_start[row + x1 + 1];
            for (uint32_t j = j0; j < j1; ++j) {
                if (j == i) continue;
                const float4 xj = xs[j];
                const float dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
                const float r2 = dx * dx + dy * dy + dz * dz;
                if (r2 < h2) {
                    if (cnt < (uint32_t)cap) nbr[(size_t)cnt * n + t] = j;
                    ++cnt;
                }
            }
        }
    }
    if (cnt > (uint32_t)cap) {
        atomicOr(err, ERR_NEIGHBOUR_CAP);
        cnt = (uint32_t)cap;
    }
    nmeta[t] = ((uint32_t)scn << 16) | cnt;
}

// ------------------------------------------------------- level buckets
// Stable bucketing of slots by descending level (Eqs. 9-10: the active sets
// are nested, so one bucketing per step makes every P_k a prefix).
// counts layout: [(n_iters - L) * nb + block] for L = n_iters..1.
__global__ void k_level_count(int64_t n, const uint8_t *__restrict__ lvl,
                              uint32_t *__restrict__ counts, int nb, int K)
{
    __shared__ uint32_t hist[PBF_MAX_ITERS + 1];
    for (int i = threadIdx.x; i <= K; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    int64_t s = (int64_t)blockIdx.x * kLevelBlock + threadIdx.x;
    if (s < n) atomicAdd(&hist[lvl[s]], 1u);
    __syncthreads();
    for (int L = threadIdx.x + 1; L <= K; L += blockDim.x)
        counts[(size_t)(K - L) * nb + blockIdx.x] = hist[L];
}

// single workgroup: exclusive scan of the bucket counts; count_ge[L] =
// |{i : N_i >= L}| for L = 0..K+1 (count_ge[k + 1] = |P_k|).
__global__ void k_level_scan(uint32_t *__restrict__ counts, int nb, int K,
                             uint32_t *__restrict__ count_ge,
                             unsigned long long *__restrict__ totals)
{
    __shared__ uint32_t lds[1024 / 64 + 1];
    const uint32_t M = (uint32_t)nb * (uint32_t)K;
    uint32_t carry = 0;
    for (uint32_t b0 = 0; b0 < M; b0 += blockDim.x) {
        uint32_t i = b0 + threadIdx.x;
        uint32_t v = i < M ? counts[i] : 0u;
        uint32_t tot;
        uint32_t ex = block_exclusive_sum(v, lds, &tot);
        if (i < M) counts[i] = carry + ex;
        carry += tot;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        count_ge[0] = carry;
        count_ge[1] = carry;
        count_ge[K + 1] = 0;
    }
    for (int L = 2 + threadIdx.x; L <= K; L += blockDim.x)
        count_ge[L] = counts[(size_t)(K - L + 1) * nb];
    // running particle-iteration count: sum_L |{N_i >= L}| = sum_i N_i
    if (threadIdx.x == 0) {
        unsigned long long pit = carry;
        for (int L = 2; L <= K; ++L) pit += counts[(size_t)(K - L + 1) * nb];
        totals[0] += pit;
        totals[1] += 1ull;
    }
}

// Rank of each slot among equal levels inside its wave by ballots, then
// across the block's waves, then the bucket offset of the block.
__global__ void k_level_scatter(int64_t n, const uint8_t *__restrict__ lvl,
                                const uint32_t *__restrict__ offs, int nb, int K,
                                uint32_t *__restrict__ order)
{
    __shared__ uint32_t wc[kLevelBlock / 64][PBF_MAX_ITERS + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < (kLevelBlock / 64) * (PBF_MAX_ITERS + 1); i += blockDim.x)
        (&wc[0][0])[i] = 0;
    __syncthreads();
    const int64_t s = (int64_t)blockIdx.x * kLevelBlock + threadIdx.x;
    const bool valid = s < n;
    const int L = valid ? (int)lvl[s] : 0;
    uint64_t rem = __ballot(valid);
    uint32_t rank = 0;
    while (rem) {
        const int leader = __ffsll((unsigned long long)rem) - 1;
        const int L0 = __shfl(L, leader, 64);
        const uint64_t m = __ballot(valid && L == L0);
        if (valid && L == L0) rank = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
        if (lane == leader) wc[wave][L0] = (uint32_t)__popcll(m);
        rem &= ~m;
    }
    __syncthreads();
    if (valid) {
        uint32_t base = 0;
        for (int w = 0; w < wave; ++w) base += wc[w][L];
        order[offs[(size_t)(K - L) * nb + blockIdx.x] + base + rank] = (uint32_t)s;
    }
}

// ------------------------------------------------ solver iteration k
// lambda_i for i in P_k (Eqs. 4-6), written to xs[i].w.  Neighbours read
// only xyz of the same buffer, so the 4-byte write of w does not disturb them.
__global__ void k_lambda(int k, int64_t n, const SceneDev *__restrict__ sc,
                         const uint32_t *__restrict__ count_ge,
                         const uint32_t *__restrict__ order, float4 *__restrict__ xs,
                         const uint32_t *__restrict__ nbr, const uint32_t *__restrict__ nmeta)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)count_ge[k + 1]) return;
    const uint32_t i = order[t];
    const uint32_t meta = nmeta[t];
    const int cnt = (int)(meta & 0xffffu);
    const SceneDev &S = sc[meta >> 16];
    const float h = S.h, h2 = S.h2, cg = S.c_grad;
    const float4 xi = xs[i];
    float sum6 = S.h6;  // the particle itself: (h^2 - 0)^3
    float gx = 0.f, gy = 0.f, gz = 0.f, g2 = 0.f;
    for (int q = 0; q < cnt; ++q) {
        const uint32_t j = nbr[(size_t)q * n + t];
        const float4 xj = xs[j];
        const float dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
        const float r2 = dx * dx + dy * dy + dz * dz;
        if (r2 < h2) {
            const float w = h2 - r2;
            sum6 += w * w * w;
            if (r2 > 0.f) {
                const float ir = rsqrtf(r2);
                const float hr = h - r2 * ir;
                const float f = -cg * hr * hr * ir;  // grad W = f d
                gx += f * dx;
                gy += f * dy;
                gz += f * dz;
                g2 += f * f * r2;
            }
        }
    }
    const float C = S.c_rho * sum6 - 1.f;
    const float denom = S.c_s * (gx * gx + gy * gy + gz * gz + g2) + S.eps;
    xs[i].w = -C / denom;
}

// Delta p_i for i in P_k (Eq. 7) with the wall contact (clamp), written to
// the other buffer (Jacobi).  Particles that finished with this iteration
// (N_i == k) copy position and lambda across, so that from now on both
// buffers hold their final values and they need no further work.
__global__ void k_update(int k, int64_t n, const SceneDev *__restrict__ sc,
                         const uint32_t *__restrict__ count_ge,
                         const uint32_t *__restrict__ order, const float4 *__restrict__ xs_in,
                         float4 *__restrict__ xs_out, const uint32_t *__restrict__ nbr,
                         const uint32_t *__restrict__ nmeta)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)count_ge[k]) return;
    const uint32_t i = order[t];
    const float4 xi = xs_in[i];
    if (t >= (int64_t)count_ge[k + 1]) {
        xs_out[i] = xi;
        return;
    }
    const uint32_t meta = nmeta[t];
    const int cnt = (int)(meta & 0xffffu);
    const SceneDev &S = sc[meta >> 16];
    const float h = S.h, h2 = S.h2, cg = S.c_grad;
    const float li = xi.w;
    float px = 0.f, py = 0.f, pz = 0.f;
    for (int q = 0; q < cnt; ++q) {
        const uint32_t j = nbr[(size_t)q * n + t];
        const float4 xj = xs_in[j];
        const float dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
        const float r2 = dx * dx + dy * dy + dz * dz;
        if (r2 < h2 && r2 > 0.f) {
            const float ir = rsqrtf(r2);
            const float hr = h - r2 * ir;
            const float f = -cg * hr * hr * ir * (li + xj.w);
            px += f * dx;
            py += f * dy;
            pz += f * dz;
        }
    }
    const float s = S.inv_rho0;
    xs_out[i] = make_float4(clampf(xi.x + px * s, S.lo[0], S.hi[0]),
                            clampf(xi.y + py * s, S.lo[1], S.hi[1]),
                            clampf(xi.z + pz * s, S.lo[2], S.hi[2]), li);
}

// --------------------------------------------- velocity and position update
__global__ void k_commit(int64_t n, const SceneDev *__restrict__ sc, float4 *__restrict__ x,
                         float4 *__restrict__ v, const float4 *__restrict__ xs,
                         uint32_t *__restrict__ err)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const float4 xi = x[s];
    const float4 p = xs[s];
    const float dt = sc[__float_as_int(xi.w)].dt;
    if (!(isfinite(p.x) && isfinite(p.y) && isfinite(p.z))) atomicOr(err, ERR_NONFINITE);
    v[s] = make_float4((p.x - xi.x) / dt, (p.y - xi.y) / dt, (p.z - xi.z) / dt, 0.f);
    x[s] = make_float4(p.x, p.y, p.z, xi.w);
}

inline unsigned blocks_for(int64_t n, int block)
{
    return (unsigned)((n + block - 1) / block);
}

}  // namespace

#define LAUNCH(KID, GRID, BLOCK, KERNEL, ...)                              \
    do {                                                                   \
        if (tm) timer_begin(tm, KID, s);                                   \
        hipLaunchKernelGGL(KERNEL, dim3(GRID), dim3(BLOCK), 0, s, __VA_ARGS__); \
        if (tm) timer_end(tm, KID, s);                                     \
        hipError_t e_ = hipGetLastError();                                 \
        if (e_ != hipSuccess) return e_;                                   \
    } while (0)

hipError_t enqueue_step(const StepBuffers &b, int cur, const LaunchShape &ls, hipStream_t s,
                        Timer *tm)
{
    const int64_t n = b.n;
    if (n == 0) return hipSuccess;
    const int nxt = cur ^ 1;
    const int K = b.n_iters;
    const uint32_t G = b.n_cells;
    const int *bs = ls.block;

    LAUNCH(K_FILL, blocks_for(G, bs[K_FILL]), bs[K_FILL], k_fill, b.cell_count, G, 0u);
    LAUNCH(K_LOD_PREDICT, blocks_for(n, bs[K_LOD_PREDICT]), bs[K_LOD_PREDICT], k_lod_predict, n,
           b.scenes, b.x[cur], b.v[cur], b.id[cur], b.lev_by_id, b.xs_pred, b.lvl[cur],
           b.key_pre, b.ticket, b.cell_count);
    LAUNCH(K_SCAN_REDUCE, b.n_scan_blocks, kScanBlock, k_scan_reduce, b.cell_count, G,
           b.scan_part);
    LAUNCH(K_SCAN_TOP, 1, 1024, k_scan_top, b.scan_part, (uint32_t)b.n_scan_blocks);
    LAUNCH(K_SCAN_APPLY, b.n_scan_blocks, kScanBlock, k_scan_apply, b.cell_count, G, b.scan_part,
           b.cell_start);
    LAUNCH(K_SORT_SCATTER, blocks_for(n, bs[K_SORT_SCATTER]), bs[K_SORT_SCATTER], k_sort_scatter,
           n, b.key_pre, b.ticket, b.cell_start, b.id[cur], b.tmp_src, b.tmp_id);
    LAUNCH(K_SORT_FINISH, blocks_for(n, bs[K_SORT_FINISH]), bs[K_SORT_FINISH], k_sort_finish, n,
           b.tmp_src, b.tmp_id, b.key_pre, b.cell_start, b.x[cur], b.v[cur], b.xs_pred,
           b.lvl[cur], b.x[nxt], b.v[nxt], b.xs[0], b.id[nxt], b.lvl[nxt], b.key, b.err);
    LAUNCH(K_LEVEL_COUNT, b.n_level_blocks, kLevelBlock, k_level_count, n, b.lvl[nxt],
           b.level_counts, b.n_level_blocks, K);
    LAUNCH(K_LEVEL_SCAN, 1, 1024, k_level_scan, b.level_counts, b.n_level_blocks, K, b.count_ge,
           b.totals);
    LAUNCH(K_LEVEL_SCATTER, b.n_level_blocks, kLevelBlock, k_level_scatter, n, b.lvl[nxt],
           b.level_counts, b.n_level_blocks, K, b.order);
    LAUNCH(K_NEIGHBOURS, blocks_for(n, bs[K_NEIGHBOURS]), bs[K_NEIGHBOURS], k_neighbours, n,
           b.scenes, b.order, b.xs[0], b.x[nxt], b.key, b.cell_start, b.nbr_cap, b.nbr, b.nmeta,
           b.err);
    for (int k = 0; k < K; ++k) {
        float4 *xin = b.xs[k & 1], *xout = b.xs[(k + 1) & 1];
        LAUNCH(K_LAMBDA, blocks_for(n, bs[K_LAMBDA]), bs[K_LAMBDA], k_lambda, k, n, b.scenes,
               b.count_ge, b.order, xin, b.nbr, b.nmeta);
        LAUNCH(K_UPDATE, blocks_for(n, bs[K_UPDATE]), bs[K_UPDATE], k_update, k, n, b.scenes,
               b.count_ge, b.order, xin, xout, b.nbr, b.nmeta);
    }
    LAUNCH(K_COMMIT, blocks_for(n, bs[K_COMMIT]), bs[K_COMMIT], k_commit, n, b.scenes, b.x[nxt],
           b.v[nxt], b.xs[K & 1], b.err);
    return hipSuccess;
}

}  // namespace pbf

namespace pbf {
namespace {
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
}  // namespace

hipError_t enqueue_unpermute(int64_t n, const float4 *x, const uint32_t *id, float *out,
                             uint32_t id_lo, uint32_t id_hi, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_unpermute, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, x, id, out,
                       id_lo, id_hi);
    return hipGetLastError();
}
}  // namespace pbf
