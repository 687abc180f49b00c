// Reverse mode of the adaptive PBF step (training form): the adjoint of the
// projection loop of Fig. 7 (Eqs. 4-7, gated by Eqs. 9-11), of the
// prediction and of the velocity/position update, with each step's levels,
// neighbour sets and wall contacts held fixed.
//
// Forward step (per particle, slot order of the step's counting sort):
//   v1 = v + dt g;  z0 = clamp(x + dt v1)
//   iteration k, i active (k < N_i):
//     lambda_i = -C_i / (S_i + eps),  C_i = c_rho sum_q (h^2 - r^2)^3 - 1,
//     S_i = c_s (|G_i|^2 + sum_q |g_iq|^2),  g_iq = grad W(z_i - z_q), G_i = sum_q g_iq
//     dp_i = (1/rho0) sum_q (lambda_i + lambda_q) g_iq
//     z_i <- clamp(z_i + dp_i)          (finished particles keep z and lambda)
//   v' = (zK - x) / dt;  x' = zK
// Reverse iteration k (bars are adjoints, dpb = 0 for finished particles,
// M = 1 where the clamp did not act, H = Hessian of the spiky kernel):
//   dpb_i = M ⊙ zb_i;  zb_i <- M ⊙ zb_i                                  (a)
//   lb_p += (1/rho0) sum_q (dpb_p - dpb_q) . g_pq
//   zb_p += (1/rho0) sum_q (lambda_p + lambda_q) H_pq (dpb_p - dpb_q)     (b)
//   active p: Cb = -lb/(S+eps), Sb = -lb lambda/(S+eps), lb <- 0          (c)
//   zb_p += sum_q -6 c_rho w_pq^2 d_pq (Cb_p + Cb_q)
//                 + 2 c_s H_pq (Sb_p (G_p + g_pq) - Sb_q (G_q - g_pq))    (d)
// A finished particle's lb keeps accumulating over the iterations that use
// its frozen lambda and is spent at its last active iteration.  Every sum is
// a gather over the particle's own neighbour list (the sets are symmetric),
// so there are no atomics and the result is deterministic.
#include "pbf_internal.h"
#include "../../include/pbf.h"

namespace pbf {
namespace {

inline unsigned blocks(int64_t n, int b)
{
    return (unsigned)((n + b - 1) / b);
}

__device__ __forceinline__ float3 f3(const float4 &a)
{
    return make_float3(a.x, a.y, a.z);
}

// spiky-gradient factor f (grad W = f d) and Hessian coefficient e
// (H = f I + e d d^T) at distance r = |d| > 0, r < h
__device__ __forceinline__ void spiky(float r2, float h, float cg, float &f, float &e)
{
    const float ir = rsqrtf(r2);
    const float r = r2 * ir;
    const float hr = h - r;
    f = -cg * hr * hr * ir;
    e = cg * hr * (h + r) * ir * ir * ir;
}

// H v for H = f I + e d d^T
__device__ __forceinline__ float3 hess(float f, float e, float3 d, float3 v)
{
    const float dv = d.x * v.x + d.y * v.y + d.z * v.z;
    return make_float3(f * v.x + e * dv * d.x, f * v.y + e * dv * d.y, f * v.z + e * dv * d.z);
}

__device__ __forceinline__ uint32_t level_of(uint32_t meta)
{
    return meta_level(meta);
}

// The gather kernels below give each particle L consecutive lanes of a wave
// (L divides 64): lane `sub` takes neighbours sub, sub + L, ..., and the L
// partial sums are combined in a fixed butterfly order, so the result is
// deterministic.  Lane 0 of the group writes.
template <int L>
__device__ __forceinline__ float group_sum(float v)
{
    for (int o = 1; o < L; o <<= 1) v += __shfl_xor(v, o);
    return v;
}

template <int L>
__device__ __forceinline__ bool group_of(int64_t n, int64_t &p, uint32_t &sub)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    p = t / L;
    sub = (uint32_t)(t % L);
    return p < n;
}

// Decode the step's neighbour codes into slots, slot[q * n + p] (a tile's
// own particles over gridDim.x / tiles workgroups, same tables as the
// forward kernels).  A thread takes one group of 8 codes of one particle;
// a staged code is an LDS stage index, turned into its slot by a table of
// the whole stage built first.
__global__ __launch_bounds__(kDecodeThreads) void k_adj_decode(
    uint32_t tiles, const uint32_t *__restrict__ tile_order, const uint32_t *__restrict__ tile_ge,
    const uint32_t *__restrict__ tile_start, const uint32_t *__restrict__ tile_count,
    const uint32_t *__restrict__ rows, int64_t n, uint32_t groups, const uint4 *__restrict__ nbr,
    const uint32_t *__restrict__ pmeta, uint32_t *__restrict__ slot)
{
    __shared__ uint32_t bnd[kBndWords];
    __shared__ uint32_t base[kStageRows + 1];
    __shared__ uint32_t table[kStageCap];
    const uint32_t b = blockIdx.x % tiles;
    if (b >= tile_ge[1]) return;
    const uint32_t tile = tile_order[b];
    const uint32_t p0 = tile_start[tile], nown = tile_count[tile];
    uint32_t first, last;
    if (!split_part(nown, blockIdx.x / tiles, gridDim.x / tiles, first, last)) return;
    for (int e = threadIdx.x; e < kRowWords; e += blockDim.x) {
        const uint32_t w = rows[(size_t)b * kRowWords + e];  // by slot
        if (e < kBndWords) bnd[e] = w;
        else base[e - kBndWords] = w;
    }
    __syncthreads();
    const bool fits = base[kStageRows] <= (uint32_t)kStageCap;
    if (fits) {
        for (int r = 0; r < kStageRows; ++r)
            for (uint32_t c = base[r] + threadIdx.x; c < base[r + 1]; c += blockDim.x)
                table[c] = bnd[r * (kStageEdge + 1)] + (c - base[r]);
        __syncthreads();
    }
    const uint32_t m = last - first;
    for (uint32_t t = threadIdx.x; t < m * groups; t += blockDim.x) {
        const uint32_t g = t / m;
        const size_t p = p0 + first + (t - g * m);
        const uint32_t cnt = pmeta[p] & kMetaCount;
        if (8 * g >= cnt) continue;
        const uint4 v = nbr[(size_t)g * n + p];
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
        const uint32_t top = cnt - 8 * g < 8 ? cnt - 8 * g : 8;
        for (uint32_t u = 0; u < top; ++u) {
            const uint32_t c = (u & 1u) ? (w[u >> 1] >> 16) : (w[u >> 1] & 0xffffu);
            const uint32_t s = fits ? table[c]
                                    : bnd[(c >> kSegOffBits) * (kStageEdge + 1)] +
                                          (c & ((1u << kSegOffBits) - 1));
            slot[(size_t)(8 * g + u) * n + p] = s;
        }
    }
}

// commit: zb = xb' + vb'/dt, xb (partial) = -vb'/dt; slot order from ID order
__global__ void k_adj_commit(int64_t n, const SceneDev *__restrict__ sc,
                             const uint32_t *__restrict__ id_scene, const uint32_t *__restrict__ id,
                             const float *__restrict__ ax, const float *__restrict__ av,
                             float4 *__restrict__ zb, float4 *__restrict__ xb,
                             float *__restrict__ lb)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint32_t g = id[s];
    const float idt = 1.f / sc[id_scene[g]].dt;
    const float vx = av[3 * (size_t)g], vy = av[3 * (size_t)g + 1], vz = av[3 * (size_t)g + 2];
    zb[s] = make_float4(ax[3 * (size_t)g] + vx * idt, ax[3 * (size_t)g + 1] + vy * idt,
                        ax[3 * (size_t)g + 2] + vz * idt, 0.f);
    xb[s] = make_float4(-vx * idt, -vy * idt, -vz * idt, 0.f);
    lb[s] = 0.f;
}

// (a): split zb of the positions after iteration k into the correction's
// adjoint and the identity part, for active particles
__global__ void k_adj_clamp(int k, int64_t n, const SceneDev *__restrict__ sc,
                            const uint32_t *__restrict__ id_scene, const uint32_t *__restrict__ id,
                            const uint8_t *__restrict__ lvl, const float4 *__restrict__ znext,
                            float4 *__restrict__ zb, float4 *__restrict__ dpb)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    if ((int)lvl[s] <= k) {
        dpb[s] = make_float4(0.f, 0.f, 0.f, 0.f);
        return;
    }
    const SceneDev &S = sc[id_scene[id[s]]];
    const float4 z = znext[s];
    const float4 b = zb[s];
    const float mx = (z.x > S.lo[0] && z.x < S.hi[0]) ? 1.f : 0.f;
    const float my = (z.y > S.lo[1] && z.y < S.hi[1]) ? 1.f : 0.f;
    const float mz = (z.z > S.lo[2] && z.z < S.hi[2]) ? 1.f : 0.f;
    const float4 m = make_float4(mx * b.x, my * b.y, mz * b.z, 0.f);
    dpb[s] = m;
    zb[s] = m;
}

// (b): lambda and position adjoints from the corrections
template <int L>
__global__ void k_adj_dp(int64_t n, const SceneDev *__restrict__ sc,
                         const uint32_t *__restrict__ id_scene, const uint32_t *__restrict__ id,
                         const uint32_t *__restrict__ pslot, const uint32_t *__restrict__ pmeta,
                         const uint32_t *__restrict__ nslot, const float4 *__restrict__ zl,
                         const float4 *__restrict__ dpb, float4 *__restrict__ zb,
                         float *__restrict__ lb)
{
    int64_t p;
    uint32_t sub;
    if (!group_of<L>(n, p, sub)) return;
    const uint32_t i = pslot[p];
    const SceneDev &S = sc[id_scene[id[i]]];
    const float h = S.h, h2 = S.h2, cg = S.c_grad, ir0 = S.inv_rho0;
    const uint32_t cnt = pmeta[p] & kMetaCount;
    const float4 zi = zl[i];
    const float3 di = f3(dpb[i]);
    float lsum = 0.f;
    float3 acc = make_float3(0.f, 0.f, 0.f);
    for (uint32_t q = sub; q < cnt; q += L) {
        const uint32_t j = nslot[(size_t)q * n + p];
        const float4 zj = zl[j];
        const float3 d = make_float3(zi.x - zj.x, zi.y - zj.y, zi.z - zj.z);
        const float r2 = d.x * d.x + d.y * d.y + d.z * d.z;
        if (!(r2 < h2 && r2 > 0.f)) continue;
        float f, e;
        spiky(r2, h, cg, f, e);
        const float3 dj = f3(dpb[j]);
        const float3 u = make_float3(di.x - dj.x, di.y - dj.y, di.z - dj.z);
        lsum += f * (u.x * d.x + u.y * d.y + u.z * d.z);
        const float3 hu = hess(f, e, d, u);
        const float s = zi.w + zj.w;
        acc.x += s * hu.x;
        acc.y += s * hu.y;
        acc.z += s * hu.z;
    }
    lsum = group_sum<L>(lsum);
    acc.x = group_sum<L>(acc.x);
    acc.y = group_sum<L>(acc.y);
    acc.z = group_sum<L>(acc.z);
    if (sub) return;
    lb[i] += ir0 * lsum;
    float4 b = zb[i];
    b.x += ir0 * acc.x;
    b.y += ir0 * acc.y;
    b.z += ir0 * acc.z;
    zb[i] = b;
}

// (c): constraint adjoints of the active particles (G, Cb in gc; Sb in sb)
template <int L>
__global__ void k_adj_lambda(int k, int64_t n, const SceneDev *__restrict__ sc,
                             const uint32_t *__restrict__ id_scene, const uint32_t *__restrict__ id,
                             const uint32_t *__restrict__ pslot, const uint32_t *__restrict__ pmeta,
                             const uint32_t *__restrict__ nslot, const float4 *__restrict__ zl,
                             float *__restrict__ lb, float4 *__restrict__ gc,
                             float *__restrict__ sb)
{
    int64_t p;
    uint32_t sub;
    if (!group_of<L>(n, p, sub)) return;
    const uint32_t i = pslot[p];
    const uint32_t meta = pmeta[p];
    if ((int)level_of(meta) <= k) {
        if (sub == 0) {
            gc[i] = make_float4(0.f, 0.f, 0.f, 0.f);
            sb[i] = 0.f;
        }
        return;
    }
    const SceneDev &S = sc[id_scene[id[i]]];
    const float h = S.h, h2 = S.h2, cg = S.c_grad;
    const uint32_t cnt = meta & kMetaCount;
    const float4 zi = zl[i];
    float gx = 0.f, gy = 0.f, gz = 0.f, g2 = 0.f;
    for (uint32_t q = sub; q < cnt; q += L) {
        const float4 zj = zl[nslot[(size_t)q * n + p]];
        const float dx = zi.x - zj.x, dy = zi.y - zj.y, dz = zi.z - zj.z;
        const float r2 = dx * dx + dy * dy + dz * dz;
        if (r2 < h2 && r2 > 0.f) {
            float f, e;
            spiky(r2, h, cg, f, e);
            gx += f * dx;
            gy += f * dy;
            gz += f * dz;
            g2 += f * f * r2;
        }
    }
    gx = group_sum<L>(gx);
    gy = group_sum<L>(gy);
    gz = group_sum<L>(gz);
    g2 = group_sum<L>(g2);
    if (sub) return;
    const float denom = S.c_s * (gx * gx + gy * gy + gz * gz + g2) + S.eps;
    const float l = lb[i];
    gc[i] = make_float4(gx, gy, gz, -l / denom);
    sb[i] = -l * zi.w / denom;
    lb[i] = 0.f;
}

// (d): position adjoints from the constraints C and S
template <int L>
__global__ void k_adj_constraint(int64_t n, const SceneDev *__restrict__ sc,
                                 const uint32_t *__restrict__ id_scene,
                                 const uint32_t *__restrict__ id, const uint32_t *__restrict__ pslot,
                                 const uint32_t *__restrict__ pmeta,
                                 const uint32_t *__restrict__ nslot, const float4 *__restrict__ zl,
                                 const float4 *__restrict__ gc, const float *__restrict__ sb,
                                 float4 *__restrict__ zb)
{
    int64_t p;
    uint32_t sub;
    if (!group_of<L>(n, p, sub)) return;
    const uint32_t i = pslot[p];
    const SceneDev &S = sc[id_scene[id[i]]];
    const float h = S.h, h2 = S.h2, cg = S.c_grad, c6 = 6.f * S.c_rho, c2 = 2.f * S.c_s;
    const uint32_t cnt = pmeta[p] & kMetaCount;
    const float4 zi = zl[i];
    const float4 gi = gc[i];
    const float si = sb[i];
    float3 acc = make_float3(0.f, 0.f, 0.f);
    for (uint32_t q = sub; q < cnt; q += L) {
        const uint32_t j = nslot[(size_t)q * n + p];
        const float4 zj = zl[j];
        const float3 d = make_float3(zi.x - zj.x, zi.y - zj.y, zi.z - zj.z);
        const float r2 = d.x * d.x + d.y * d.y + d.z * d.z;
        if (!(r2 < h2)) continue;
        const float4 gj = gc[j];
        const float w = h2 - r2;
        const float cc = -c6 * w * w * (gi.w + gj.w);  // density terms of C_p and C_q
        acc.x += cc * d.x;
        acc.y += cc * d.y;
        acc.z += cc * d.z;
        if (r2 > 0.f) {
            float f, e;
            spiky(r2, h, cg, f, e);
            const float3 g = make_float3(f * d.x, f * d.y, f * d.z);
            const float sj = sb[j];
            const float3 v = make_float3(si * (gi.x + g.x) - sj * (gj.x - g.x),
                                         si * (gi.y + g.y) - sj * (gj.y - g.y),
                                         si * (gi.z + g.z) - sj * (gj.z - g.z));
            const float3 hv = hess(f, e, d, v);
            acc.x += c2 * hv.x;
            acc.y += c2 * hv.y;
            acc.z += c2 * hv.z;
        }
    }
    acc.x = group_sum<L>(acc.x);
    acc.y = group_sum<L>(acc.y);
    acc.z = group_sum<L>(acc.z);
    if (sub) return;
    float4 b = zb[i];
    b.x += acc.x;
    b.y += acc.y;
    b.z += acc.z;
    zb[i] = b;
}

// prediction: yb = M0 ⊙ zb; xb_in = xb + yb, vb_in = dt yb (ID order out)
__global__ void k_adj_predict(int64_t n, const SceneDev *__restrict__ sc,
                              const uint32_t *__restrict__ id_scene, const uint32_t *__restrict__ id,
                              const float4 *__restrict__ z0, const float4 *__restrict__ zb,
                              const float4 *__restrict__ xb, float *__restrict__ ax,
                              float *__restrict__ av)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint32_t g = id[s];
    const SceneDev &S = sc[id_scene[g]];
    const float4 z = z0[s];
    const float4 b = zb[s];
    const float yx = (z.x > S.lo[0] && z.x < S.hi[0]) ? b.x : 0.f;
    const float yy = (z.y > S.lo[1] && z.y < S.hi[1]) ? b.y : 0.f;
    const float yz = (z.z > S.lo[2] && z.z < S.hi[2]) ? b.z : 0.f;
    const float4 x = xb[s];
    ax[3 * (size_t)g] = x.x + yx;
    ax[3 * (size_t)g + 1] = x.y + yy;
    ax[3 * (size_t)g + 2] = x.z + yz;
    av[3 * (size_t)g] = S.dt * yx;
    av[3 * (size_t)g + 1] = S.dt * yy;
    av[3 * (size_t)g + 2] = S.dt * yz;
}

// restore a state saved in ID order (float[3n] each) with storage order = ID
__global__ void k_load_state(int64_t n, const float *__restrict__ x3, const float *__restrict__ v3,
                             const uint32_t *__restrict__ id_scene, float4 *__restrict__ x,
                             float4 *__restrict__ v, uint32_t *__restrict__ id)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    x[g] = make_float4(x3[3 * g], x3[3 * g + 1], x3[3 * g + 2], __int_as_float((int)id_scene[g]));
    v[g] = make_float4(v3[3 * g], v3[3 * g + 1], v3[3 * g + 2], 0.f);
    id[g] = (uint32_t)g;
}

}  // namespace

#define ACHK(X)                                   \
    do {                                          \
        hipError_t e_ = (X);                      \
        if (e_ != hipSuccess) return e_;          \
    } while (0)

hipError_t enqueue_load_state(int64_t n, const float *x3, const float *v3,
                              const uint32_t *id_scene, float4 *x, float4 *v, uint32_t *id,
                              hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_load_state, dim3(blocks(n, 256)), dim3(256), 0, s, n, x3, v3, id_scene,
                       x, v, id);
    return hipGetLastError();
}

hipError_t enqueue_adjoint_step(const StepBuffers &b, const StepRecord &r, const float *ax_in,
                                const float *av_in, float *ax_out, float *av_out,
                                const AdjointScratch &w, hipStream_t s)
{
    const int64_t n = b.n;
    if (n == 0) return hipSuccess;
    const int K = b.n_iters;
    const int tb = 256;
    const unsigned gb = blocks(n, tb);
    // lanes per particle of the gather kernels: enough for about 2^19 threads
    const int lanes = n >= (int64_t(1) << 19) ? 1 : n >= (int64_t(1) << 18) ? 2 : n >= (int64_t(1) << 17) ? 4 : 8;
    const unsigned gl = blocks(n * lanes, tb);
    hipLaunchKernelGGL(k_adj_decode, dim3(b.n_tiles * tile_split(b.n_tiles)), dim3(kDecodeThreads), 0,
                       s, b.n_tiles, r.tile_order, r.tile_ge, r.tile_start, r.tile_count,
                       r.tile_rows, n, (uint32_t)(b.nbr_cap + 7) / 8, r.nbr, r.pmeta, w.nslot);
    ACHK(hipGetLastError());
    hipLaunchKernelGGL(k_adj_commit, dim3(gb), dim3(tb), 0, s, n, b.scenes, b.id_scene, r.id,
                       ax_in, av_in, w.zb, w.xb, w.lb);
    ACHK(hipGetLastError());
    for (int k = K - 1; k >= 0; --k) {
        hipLaunchKernelGGL(k_adj_clamp, dim3(gb), dim3(tb), 0, s, k, n, b.scenes, b.id_scene,
                           r.id, r.lvl, r.snap[k + 1], w.zb, w.dpb);
        ACHK(hipGetLastError());
#define GATHER(KERNEL, ...)                                                                      \
    switch (lanes) {                                                                             \
    case 1: hipLaunchKernelGGL(KERNEL<1>, dim3(gl), dim3(tb), 0, s, __VA_ARGS__); break;          \
    case 2: hipLaunchKernelGGL(KERNEL<2>, dim3(gl), dim3(tb), 0, s, __VA_ARGS__); break;          \
    case 4: hipLaunchKernelGGL(KERNEL<4>, dim3(gl), dim3(tb), 0, s, __VA_ARGS__); break;          \
    default: hipLaunchKernelGGL(KERNEL<8>, dim3(gl), dim3(tb), 0, s, __VA_ARGS__); break;         \
    }                                                                                            \
    ACHK(hipGetLastError())
        GATHER(k_adj_dp, n, b.scenes, b.id_scene, r.id, r.pslot, r.pmeta, w.nslot, r.snap[k], w.dpb,
               w.zb, w.lb);
        GATHER(k_adj_lambda, k, n, b.scenes, b.id_scene, r.id, r.pslot, r.pmeta, w.nslot, r.snap[k],
               w.lb, w.gc, w.sb);
        GATHER(k_adj_constraint, n, b.scenes, b.id_scene, r.id, r.pslot, r.pmeta, w.nslot,
               r.snap[k], w.gc, w.sb, w.zb);
#undef GATHER
    }
    hipLaunchKernelGGL(k_adj_predict, dim3(gb), dim3(tb), 0, s, n, b.scenes, b.id_scene, r.id,
                       r.snap[0], w.zb, w.xb, ax_out, av_out);
    return hipGetLastError();
}

}  // namespace pbf
