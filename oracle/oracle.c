/*
 * FP64 CPU oracle of one adaptive position-based-fluids (APBF) time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The product
 * path (the HIP library) never calls it and shares no code with it.
 *
 * Plain, slow, obviously-correct loops in double precision, following the
 * paper step by step:
 *   - constraint projection with a scaling factor (Eqs. 1-4),
 *   - density constraint and SPH density estimate (Eqs. 5-6),
 *   - position correction (Eq. 7),
 *   - levels, active predicate, active set and finished set (Eqs. 8-11),
 *   - the simulation loop of Section 5 (Fig. 7): apply forces and predict,
 *     find neighbours, then per solver iteration compute lambda, compute the
 *     correction with contact response, and update, for active particles
 *     only; finally update velocity and position of every particle,
 *   - neighbour discovery by counting sort of uniform-grid cell keys
 *     (Section 6).
 *
 * Readings where the paper is silent (they are the same in the HIP path):
 *   - W is the poly6 kernel, grad W the spiky-kernel gradient (Mueller et
 *     al. 2003); the density includes the particle itself.
 *   - Uniform mass m: Eq. 7 carries the weight w_i = 1/m of Eq. 3 and the
 *     m_j of Eq. 6, so Delta p_i = (1/rho0) sum_j (lambda_i + lambda_j) grad W.
 *   - Eq. 4's denominator gets a relaxation eps, lambda = -C / (S + eps).
 *   - Neighbour sets are found once per step from the predicted positions,
 *     with the strict test |x_i - x_j|^2 < h^2, and kept for all iterations.
 *   - A finished particle keeps its position and its last lambda; active
 *     particles use that lambda in their corrections (Fig. 5).
 *   - Contacts are the box walls: positions are clamped to [lo, hi] after
 *     prediction and after each update.  Optional solid obstacles (sphere,
 *     cone with a vertical axis standing on the floor, axis-aligned box;
 *     signed-distance shapes, Section 6) add the contacts of Fig. 7: contact
 *     finding once per step from the predicted positions (the obstacles
 *     that, grown by h, hold x*, decided in float32 like the kernel), then
 *     pre-stabilisation (Section 4.3, Fig. 6) of the particles with
 *     N_i < S: each iteration moves x* of a particle found inside an
 *     obstacle to the closest point of its surface (clamped into the box)
 *     and moves x by the same amount; finally, in every update of an active
 *     particle, x* + Delta p is moved out of each found obstacle it lies
 *     in, before the wall clamp.
 *   - Iterations k = 0 .. n_max-1 (the paper's l = k + 1); particle i is
 *     active while k < N_i.
 *   - Grid cells have edge h from lo, keys are x-fastest, coordinates are
 *     clamped into the grid; ties in the counting sort keep particle-ID
 *     order (a stable counting sort of the particles listed by ID).
 *   - Distance-to-camera levels: t = clamp((d - d_near)/(d_far - d_near)),
 *     N = clamp(n_max - floor(t (n_max - n_min + 1)), n_min, n_max), in
 *     FP64; a particle whose t (n_max - n_min + 1) lies within
 *     ORC_LEVEL_GUARD of an interior bin edge is reported as near the edge,
 *     where an evaluation in lower precision may take the neighbouring
 *     level.  A t that is not a number (a range of zero width) counts as 0.  Several
 *     cameras blend by taking the highest level; an automatic range is the
 *     min/max of the distances over the particles at the step's start
 *     (Section 4.1).
 *   - Unilateral density constraint (an option; the variant named at the
 *     end of Section 7's setup): C_i = max(rho_i/rho0 - 1, 0).
 *   - Force-based cohesion (an option named beside it, taken from the
 *     works the paper cites there: the cohesion kernel of Akinci et al.
 *     2013).  Particle i gets the acceleration
 *       a_i = -gamma m sum_j C(|x_i - x_j|) (x_i - x_j) / |x_i - x_j|
 *     with C(r) = 32/(pi h^9) (h - r)^3 r^3 for h/2 < r <= h,
 *     32/(pi h^9) (2 (h - r)^3 r^3 - h^6/64) for 0 < r <= h/2, else 0.
 *     It is an external force of Fig. 7's first loop, evaluated at the
 *     positions x at the start of the step over the neighbour sets N_i
 *     that the second loop finds (the sets at x are not known before the
 *     search); once the sets are known it is applied to the prediction,
 *     x*_i += dt^2 a_i (clamped into the box), which is what adding dt a_i
 *     to v_i in the first loop would have given.  The keys and the sets
 *     come from x* before this shift.
 * Neighbour sums run in ascending particle-ID order, so results do not
 * depend on any storage order.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef struct {
    int32_t n, n_min, n_max;
    int32_t dims[3];
    double lo[3], hi[3];
    double h, rho0, mass, eps, dt;
    double g[3];
    int32_t unilateral;     /* 1: C_i = max(rho_i / rho0 - 1, 0) (resists compression only) */
    double cohesion;        /* gamma >= 0 of the force-based cohesion; 0: none */
} orc_params;

typedef struct {
    int32_t mode;           /* 0 uniform (N_i = n_max), 1 explicit, 2 distance to camera,
                               3 distance to the visible surface */
    const int32_t *levels;  /* explicit: n levels in particle-ID order */
    double camera[3];
    double d_near, d_far;
    /* distance to the visible surface: the camera frame (unit forward and up
     * vectors, right = forward x up), focal length in pixels, image size in
     * pixels and the splat radius of a particle */
    double forward[3], up[3];
    double focal;
    int32_t width, height;
    double splat;
    /* distance to camera with several cameras: the level is the highest of
     * the levels the cameras give (the particle gets the detail the nearest
     * view asks for); camera 0 is `camera` with d_near/d_far */
    int32_t n_extra;        /* further cameras, 0..3 */
    double extra_camera[3][3];
    double extra_range[3][2];  /* d_near, d_far of each */
    int32_t auto_range;     /* 1: each camera's range is the min/max of its distances over
                               the particles (DTVS: over the particles seen), every step */
} orc_lod;

typedef struct {
    int32_t *levels;        /* [n]  N_i used this step */
    uint32_t *keys;         /* [n]  cell key of the predicted position */
    int32_t *perm;          /* [n]  sorted order as a list of particle IDs */
    int32_t *nbr_count;     /* [n]  |N_i| */
    int32_t *nbr_ids;       /* [nbr_cap] neighbour IDs, particle by particle, ascending */
    int64_t nbr_cap;
    int64_t nbr_total;      /* out: total entries (written even when nbr_ids is too small) */
    double *xs_iter;        /* [(n_max+1)*n*3] x* after prediction (the keys and neighbours
                               come from it; pre-stabilisation follows) and after each iteration */
    double *lambda_iter;    /* [n_max*n] lambda after the lambda pass of each iteration */
    uint8_t *contacts;      /* [n]  obstacles found for each particle (bit o = obstacle o) */
} orc_trace;

/* Solid obstacles and the pre-stabilisation set (Section 4.3, Fig. 7). */
enum { ORC_MAX_OBST = 4 };
enum { ORC_OB_SPHERE = 1, ORC_OB_CONE = 2, ORC_OB_BOX = 3 };

typedef struct {
    int32_t kind;  /* ORC_OB_* */
    double c[3];   /* sphere: centre; cone: centre of the base circle; box: centre */
    double a[3];   /* sphere: a[0] radius; cone: a[0] base radius, a[1] height
                      (apex above the base, +y; the slant continues below the
                      base); box: half extents */
} orc_obstacle;

typedef struct {
    int32_t count;                   /* 0 .. ORC_MAX_OBST */
    orc_obstacle ob[ORC_MAX_OBST];
    int32_t stab_iters;              /* pre-stabilisation iterations */
    int32_t stab_s;                  /* S: particles with N_i < S are pre-stabilised */
} orc_contacts;

enum { ORC_OK = 0, ORC_ERR_ARG = -1, ORC_ERR_MEM = -3 };

/* ------------------------------------------------------------------ */
/* smoothing kernels                                                   */
/* ------------------------------------------------------------------ */

/* poly6: W(r) = 315 / (64 pi h^9) (h^2 - r^2)^3 for r < h, else 0. */
double orc_poly6(double r2, double h)
{
    if (r2 >= h * h) return 0.0;
    double t = h * h - r2;
    return 315.0 / (64.0 * M_PI * pow(h, 9)) * t * t * t;
}

/* Gradient with respect to p_i of the spiky kernel 15/(pi h^6) (h - r)^3,
 * evaluated at d = p_i - p_j:  -45/(pi h^6) (h - r)^2 d / r for 0 < r < h. */
void orc_spiky_grad(const double d[3], double h, double out[3])
{
    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    out[0] = out[1] = out[2] = 0.0;
    if (r <= 0.0 || r >= h) return;
    double c = -45.0 / (M_PI * pow(h, 6)) * (h - r) * (h - r) / r;
    out[0] = c * d[0];
    out[1] = c * d[1];
    out[2] = c * d[2];
}

/* ------------------------------------------------------------------ */
/* grid                                                                */
/* ------------------------------------------------------------------ */

static int64_t n_cells(const orc_params *p)
{
    return (int64_t)p->dims[0] * p->dims[1] * p->dims[2];
}

static void cell_of(const orc_params *p, const double *x, int32_t c[3])
{
    for (int d = 0; d < 3; ++d) {
        double q = floor((x[d] - p->lo[d]) / p->h);
        if (q < 0) q = 0;
        if (q > p->dims[d] - 1) q = p->dims[d] - 1;
        c[d] = (int32_t)q;
    }
}

static uint32_t key_of(const orc_params *p, const int32_t c[3])
{
    return (uint32_t)(((int64_t)c[2] * p->dims[1] + c[1]) * p->dims[0] + c[0]);
}

void orc_cell_keys(const orc_params *p, const double *xs, uint32_t *keys)
{
    for (int32_t i = 0; i < p->n; ++i) {
        int32_t c[3];
        cell_of(p, xs + 3 * (int64_t)i, c);
        keys[i] = key_of(p, c);
    }
}

/* Counting sort of particle IDs by cell key (Section 6): histogram,
 * exclusive prefix sum, then scatter in ID order, which keeps ties in ID
 * order.  start[] has n_cells + 1 entries. */
int orc_counting_sort(const orc_params *p, const uint32_t *keys, int32_t *perm,
                      int64_t *start)
{
    int64_t G = n_cells(p);
    int64_t *fill = (int64_t *)calloc((size_t)G + 1, sizeof(int64_t));
    if (!fill) return ORC_ERR_MEM;
    for (int64_t c = 0; c <= G; ++c) start[c] = 0;
    for (int32_t i = 0; i < p->n; ++i) start[keys[i] + 1] += 1;
    for (int64_t c = 0; c < G; ++c) start[c + 1] += start[c];
    for (int32_t i = 0; i < p->n; ++i) {
        uint32_t k = keys[i];
        perm[start[k] + fill[k]] = i;
        fill[k] += 1;
    }
    free(fill);
    return ORC_OK;
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Neighbour sets N_i = { j != i : |x_i - x_j|^2 < h^2 } by scanning the 27
 * cells around the cell of x_i (Fig. 7, neighbour step); each set is sorted
 * by ascending ID.  Returns CSR arrays (caller frees). */
static int find_neighbours(const orc_params *p, const double *xs, const int32_t *perm,
                           const int64_t *start, int64_t **off_out, int32_t **ids_out)
{
    const int32_t n = p->n;
    const double h2 = p->h * p->h;
    int64_t *off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!off) return ORC_ERR_MEM;

    for (int pass = 0; pass < 2; ++pass) {
        int32_t *ids = NULL;
        if (pass == 1) {
            for (int32_t i = 0; i < n; ++i) off[i + 1] += off[i];
            ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)(off[n] > 0 ? off[n] : 1));
            if (!ids) { free(off); return ORC_ERR_MEM; }
            *ids_out = ids;
        }
#pragma omp parallel for schedule(dynamic, 256)
        for (int32_t i = 0; i < n; ++i) {
            const double *xi = xs + 3 * (int64_t)i;
            int32_t c[3];
            cell_of(p, xi, c);
            int64_t cnt = 0;
            for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int32_t q[3] = {c[0] + dx, c[1] + dy, c[2] + dz};
                if (q[0] < 0 || q[1] < 0 || q[2] < 0 || q[0] >= p->dims[0] ||
                    q[1] >= p->dims[1] || q[2] >= p->dims[2])
                    continue;
                uint32_t k = key_of(p, q);
                for (int64_t t = start[k]; t < start[k + 1]; ++t) {
                    int32_t j = perm[t];
                    if (j == i) continue;
                    const double *xj = xs + 3 * (int64_t)j;
                    double dxv = xi[0] - xj[0], dyv = xi[1] - xj[1], dzv = xi[2] - xj[2];
                    if (dxv * dxv + dyv * dyv + dzv * dzv < h2) {
                        if (pass == 1) ids[off[i] + cnt] = j;
                        ++cnt;
                    }
                }
            }
            if (pass == 0) off[i + 1] = cnt;
            else qsort(ids + off[i], (size_t)cnt, sizeof(int32_t), cmp_i32);
        }
    }
    *off_out = off;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* per-particle solver terms                                           */
/* ------------------------------------------------------------------ */

/* lambda_i of Eq. 4 for the density constraint of Eq. 5 with the density
 * estimate of Eq. 6 (self term included).  The gradient of C_i with respect
 * to p_i is (m/rho0) sum_j grad W_ij and with respect to p_j it is
 * -(m/rho0) grad W_ij; each is weighted by w = 1/m. */
static double lambda_of(const orc_params *p, const double *xs, int32_t i,
                        const int32_t *nb, int64_t cnt, double *rho_out, double *s_out)
{
    const double *xi = xs + 3 * (int64_t)i;
    const double w = 1.0 / p->mass;
    double rho = p->mass * orc_poly6(0.0, p->h);
    double gi[3] = {0.0, 0.0, 0.0};
    double sum_wj = 0.0;
    for (int64_t q = 0; q < cnt; ++q) {
        const double *xj = xs + 3 * (int64_t)nb[q];
        double d[3] = {xi[0] - xj[0], xi[1] - xj[1], xi[2] - xj[2]};
        rho += p->mass * orc_poly6(d[0] * d[0] + d[1] * d[1] + d[2] * d[2], p->h);
        double gw[3];
        orc_spiky_grad(d, p->h, gw);
        double gj[3] = {-p->mass / p->rho0 * gw[0], -p->mass / p->rho0 * gw[1],
                        -p->mass / p->rho0 * gw[2]};
        sum_wj += w * (gj[0] * gj[0] + gj[1] * gj[1] + gj[2] * gj[2]);
        gi[0] += p->mass / p->rho0 * gw[0];
        gi[1] += p->mass / p->rho0 * gw[1];
        gi[2] += p->mass / p->rho0 * gw[2];
    }
    double C = rho / p->rho0 - 1.0;
    if (p->unilateral && C < 0.0) C = 0.0;
    double denom = w * (gi[0] * gi[0] + gi[1] * gi[1] + gi[2] * gi[2]) + sum_wj;
    if (rho_out) *rho_out = rho;
    if (s_out) *s_out = denom;
    return -C / (denom + p->eps);
}

/* Delta p_i of Eq. 7 (uniform mass): (1/rho0) sum_j (lambda_i + lambda_j) grad W_ij. */
static void delta_p_of(const orc_params *p, const double *xs, const double *lam, int32_t i,
                       const int32_t *nb, int64_t cnt, double dp[3])
{
    const double *xi = xs + 3 * (int64_t)i;
    dp[0] = dp[1] = dp[2] = 0.0;
    for (int64_t q = 0; q < cnt; ++q) {
        int32_t j = nb[q];
        const double *xj = xs + 3 * (int64_t)j;
        double d[3] = {xi[0] - xj[0], xi[1] - xj[1], xi[2] - xj[2]};
        double gw[3];
        orc_spiky_grad(d, p->h, gw);
        double s = lam[i] + lam[j];
        dp[0] += s * gw[0];
        dp[1] += s * gw[1];
        dp[2] += s * gw[2];
    }
    dp[0] /= p->rho0;
    dp[1] /= p->rho0;
    dp[2] /= p->rho0;
}

/* Contact response with the box walls: clamp each coordinate to [lo, hi]. */
static void clamp_box(const orc_params *p, double *x)
{
    for (int d = 0; d < 3; ++d) {
        if (x[d] < p->lo[d]) x[d] = p->lo[d];
        if (x[d] > p->hi[d]) x[d] = p->hi[d];
    }
}

/* ------------------------------------------------------------------ */
/* obstacles (contact lines of Fig. 7)                                 */
/* ------------------------------------------------------------------ */

/* Contact finding (Fig. 7, second loop): obstacle o is a contact of a
 * particle when the obstacle grown by the margin holds x* (sphere: radius
 * + m; box: half extents + m; cone: its slant moved out by m; for the box
 * this is its bounding box grown by m, a superset of the points within m).
 * Decided in float32 with one rounding per operation, like the kernel. */
int orc_contact_found(const orc_obstacle *o, const double *x, double margin_d)
{
    const float m = (float)margin_d;
    const float dx = (float)x[0] - (float)o->c[0];
    const float dy = (float)x[1] - (float)o->c[1];
    const float dz = (float)x[2] - (float)o->c[2];
    const float a0 = (float)o->a[0], a1 = (float)o->a[1], a2 = (float)o->a[2];
    if (o->kind == ORC_OB_SPHERE) {
        const float r = a0 + m;
        return dx * dx + dy * dy + dz * dz < r * r;
    }
    if (o->kind == ORC_OB_CONE) {
        /* the cone grown by m: its slant moved out by m along the normal */
        const float rho = sqrtf(dx * dx + dz * dz);
        const float L = sqrtf(a1 * a1 + a0 * a0);
        return rho * a1 + dy * a0 < a1 * a0 + m * L;
    }
    if (o->kind == ORC_OB_BOX)
        return fabsf(dx) < a0 + m && fabsf(dy) < a1 + m && fabsf(dz) < a2 + m;
    return 0;
}

/* If x lies inside the solid obstacle, write the closest point of the
 * obstacle's surface to y and return 1 (the contact constraint's
 * projection: the signed distance becomes zero); otherwise return 0.
 *   sphere: radially out from the centre (straight up from the centre
 *     itself);
 *   box: through the face of least penetration (first axis on ties);
 *   cone (apex H above the centre c, radius R at the height of c, and its
 *     slant continued below that circle: a cone standing on the floor, so
 *     fluid pressed into it leaves through the slant, never under it): in
 *     the plane of the axis and x, to the foot of the perpendicular on the
 *     slant line; on the axis the plane is taken through +x. */
int orc_obstacle_project(const orc_obstacle *o, const double *x, double *y)
{
    const double d0 = x[0] - o->c[0], d1 = x[1] - o->c[1], d2 = x[2] - o->c[2];
    if (o->kind == ORC_OB_SPHERE) {
        const double R = o->a[0];
        const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
        if (!(r2 < R * R)) return 0;
        const double r = sqrt(r2);
        if (r > 0.0) {
            y[0] = o->c[0] + R * d0 / r;
            y[1] = o->c[1] + R * d1 / r;
            y[2] = o->c[2] + R * d2 / r;
        } else {
            y[0] = o->c[0];
            y[1] = o->c[1] + R;
            y[2] = o->c[2];
        }
        return 1;
    }
    if (o->kind == ORC_OB_CONE) {
        const double R = o->a[0], H = o->a[1];
        double rho = sqrt(d0 * d0 + d2 * d2), yb = d1;
        if (!(rho * H + yb * R < H * R)) return 0;
        const double L = sqrt(H * H + R * R);
        const double ds = (H * R - rho * H - yb * R) / L;  /* distance to the slant line */
        const double ux = rho > 0.0 ? d0 / rho : 1.0, uz = rho > 0.0 ? d2 / rho : 0.0;
        rho += ds * H / L;
        yb += ds * R / L;
        y[0] = o->c[0] + rho * ux;
        y[1] = o->c[1] + yb;
        y[2] = o->c[2] + rho * uz;
        return 1;
    }
    if (o->kind == ORC_OB_BOX) {
        const double d[3] = {d0, d1, d2};
        double q[3];
        for (int a = 0; a < 3; ++a) {
            q[a] = fabs(d[a]) - o->a[a];
            if (!(q[a] < 0.0)) return 0;
        }
        int m = 0;
        for (int a = 1; a < 3; ++a)
            if (q[a] > q[m]) m = a;
        y[0] = x[0];
        y[1] = x[1];
        y[2] = x[2];
        y[m] = o->c[m] + (d[m] >= 0.0 ? o->a[m] : -o->a[m]);
        return 1;
    }
    return 0;
}

/* Contact response of an active particle's update: x* + Delta p is moved
 * out of every found obstacle it lies in, in obstacle order, then clamped
 * to the walls. */
static void contact_response(const orc_params *p, const orc_contacts *oc, uint32_t mask, double *x)
{
    if (oc)
        for (int o = 0; o < oc->count; ++o) {
            double y[3];
            if ((mask >> o) & 1u && orc_obstacle_project(&oc->ob[o], x, y)) {
                x[0] = y[0];
                x[1] = y[1];
                x[2] = y[2];
            }
        }
    clamp_box(p, x);
}

/* ------------------------------------------------------------------ */
/* levels (Eq. 8, adaption model of Section 4.1)                       */
/* ------------------------------------------------------------------ */

/* Level from a distance (DTC and DTVS, Section 4.1): linear map of the
 * distance range [d_near, d_far] onto the levels n_max .. n_min, in FP64.
 * With u = t (n_max - n_min + 1), the level changes at the integers
 * 1 .. n_max - n_min; *near_edge (if given) is set when u lies within
 * ORC_LEVEL_GUARD of one of them.  (A float32 evaluation of u from the same
 * inputs errs by a few units in the last place, below 1e-5 for u <= 32.) */
#define ORC_LEVEL_GUARD 2e-5
static int32_t level_of_distance(const orc_params *p, double d, double d_near, double d_far,
                                 uint8_t *near_edge)
{
    double t = (d - d_near) / (d_far - d_near);
    if (!(t >= 0.0)) t = 0.0;  /* negative, or not a number */
    if (t > 1.0) t = 1.0;
    const int32_t nb = p->n_max - p->n_min + 1;
    const double u = t * (double)nb;
    const double f = floor(u);
    int32_t L = p->n_max - (int32_t)f;
    if (L < p->n_min) L = p->n_min;
    if (L > p->n_max) L = p->n_max;
    if (near_edge) {
        const double below = u - f, above = f + 1.0 - u;  /* to the edges f and f + 1 */
        if ((below < ORC_LEVEL_GUARD && f >= 1.0 && f <= (double)(nb - 1)) ||
            (above < ORC_LEVEL_GUARD && f + 1.0 <= (double)(nb - 1)))
            *near_edge = 1;
    }
    return L;
}

enum { ORC_MAX_SPLAT = 16 };  /* largest splat radius in pixels */

/* Pinhole projection of x for the DTVS model, in float32 with a fixed
 * order of operations (the pixel and the depth are integers and minima
 * decided by floating point).  Returns 0 when the particle is not in front
 * of the camera by more than its splat radius or its pixel is far outside
 * the image. */
typedef struct { int32_t pu, pv, rad; float dist; } orc_proj;

static int dtvs_project(const orc_lod *lod, const double *xi, orc_proj *o)
{
    const float f0 = (float)lod->forward[0], f1 = (float)lod->forward[1], f2 = (float)lod->forward[2];
    const float u0 = (float)lod->up[0], u1 = (float)lod->up[1], u2 = (float)lod->up[2];
    const float r0 = f1 * u2 - f2 * u1, r1 = f2 * u0 - f0 * u2, r2 = f0 * u1 - f1 * u0;
    const float qx = (float)xi[0] - (float)lod->camera[0];
    const float qy = (float)xi[1] - (float)lod->camera[1];
    const float qz = (float)xi[2] - (float)lod->camera[2];
    float z = qx * f0;
    z = z + qy * f1;
    z = z + qz * f2;
    const float splat = (float)lod->splat, focal = (float)lod->focal;
    if (!(z > splat)) return 0;
    float xr = qx * r0;
    xr = xr + qy * r1;
    xr = xr + qz * r2;
    float yu = qx * u0;
    yu = yu + qy * u1;
    yu = yu + qz * u2;
    float u = focal * xr;
    u = u / z;
    u = u + 0.5f * (float)lod->width;
    float v = focal * yu;
    v = v / z;
    v = v + 0.5f * (float)lod->height;
    const float lim = (float)ORC_MAX_SPLAT + 1.0f;
    if (!(u > -lim && u < (float)lod->width + lim && v > -lim && v < (float)lod->height + lim)) return 0;
    o->pu = (int32_t)floorf(u);
    o->pv = (int32_t)floorf(v);
    float rf = focal * splat;
    rf = rf / z;
    int32_t rad = (int32_t)ceilf(rf);
    o->rad = rad < ORC_MAX_SPLAT ? rad : ORC_MAX_SPLAT;
    float d2 = qx * qx;
    d2 = d2 + qy * qy;
    d2 = d2 + qz * qz;
    o->dist = sqrtf(d2);
    return 1;
}

/* Distance to the visible surface (DTVS, Section 4.1): every particle in
 * front of the camera is splatted into a depth image as a square of
 * (2 rad + 1)^2 pixels around its pixel, keeping the smallest distance to
 * the camera per pixel; the particles seen at a pixel are the surface, and a
 * particle's distance to the visible surface is its own distance minus the
 * depth at its pixel.  Particles behind the camera or outside the image get
 * the largest distance (lowest level). */
static int levels_dtvs(const orc_params *p, const orc_lod *lod, const double *x, int32_t *lev,
                       uint8_t *near_edge)
{
    const int32_t W = lod->width, H = lod->height;
    if (W < 1 || H < 1) return ORC_ERR_ARG;
    float *depth = (float *)malloc(sizeof(float) * (size_t)W * (size_t)H);
    if (!depth) return ORC_ERR_MEM;
    for (int64_t e = 0; e < (int64_t)W * H; ++e) depth[e] = INFINITY;
    for (int32_t j = 0; j < p->n; ++j) {
        orc_proj o;
        if (!dtvs_project(lod, x + 3 * (int64_t)j, &o)) continue;
        for (int32_t b = o.pv - o.rad; b <= o.pv + o.rad; ++b)
            for (int32_t a = o.pu - o.rad; a <= o.pu + o.rad; ++a)
                if (a >= 0 && a < W && b >= 0 && b < H && o.dist < depth[(int64_t)b * W + a])
                    depth[(int64_t)b * W + a] = o.dist;
    }
    float *dist = (float *)malloc(sizeof(float) * (size_t)(p->n ? p->n : 1));
    if (!dist) { free(depth); return ORC_ERR_MEM; }
    float dn = (float)lod->d_near, df = (float)lod->d_far;
    if (lod->auto_range) { dn = FLT_MAX; df = 0.0f; }
    for (int32_t i = 0; i < p->n; ++i) {
        orc_proj o;
        float d = FLT_MAX;
        if (dtvs_project(lod, x + 3 * (int64_t)i, &o) && o.pu >= 0 && o.pu < W && o.pv >= 0 && o.pv < H) {
            d = o.dist - depth[(int64_t)o.pv * W + o.pu];
            if (lod->auto_range) {  /* over the particles seen */
                if (d < dn) dn = d;
                if (d > df) df = d;
            }
        }
        dist[i] = d;
    }
    if (df < dn) dn = df = 0.0f;  /* automatic range with no particle seen */
    for (int32_t i = 0; i < p->n; ++i)
        lev[i] = level_of_distance(p, dist[i], dn, df, near_edge ? near_edge + i : NULL);
    free(dist);
    free(depth);
    return ORC_OK;
}

/* Distance of a particle to a camera. */
static double camera_distance(const double *xi, const double *cam)
{
    const double dx = xi[0] - cam[0], dy = xi[1] - cam[1], dz = xi[2] - cam[2];
    return sqrt(dx * dx + dy * dy + dz * dz);
}

/* Distance-to-camera levels over 1 + n_extra cameras: each camera maps its
 * distance through its range (given, or the min/max over the particles);
 * the particle takes the highest of the levels. */
static int levels_dtc(const orc_params *p, const orc_lod *lod, const double *x, int32_t *lev,
                      uint8_t *near_edge)
{
    const int nc = 1 + lod->n_extra;
    if (lod->n_extra < 0 || lod->n_extra > 3) return ORC_ERR_ARG;
    const double *cam[4] = {lod->camera, lod->extra_camera[0], lod->extra_camera[1], lod->extra_camera[2]};
    double dn[4], df[4];
    dn[0] = lod->d_near;
    df[0] = lod->d_far;
    for (int c = 1; c < nc; ++c) {
        dn[c] = lod->extra_range[c - 1][0];
        df[c] = lod->extra_range[c - 1][1];
    }
    if (lod->auto_range)
        for (int c = 0; c < nc; ++c) {
            dn[c] = DBL_MAX;
            df[c] = 0.0;
            for (int32_t i = 0; i < p->n; ++i) {
                const double d = camera_distance(x + 3 * (int64_t)i, cam[c]);
                if (d < dn[c]) dn[c] = d;
                if (d > df[c]) df[c] = d;
            }
        }
    for (int32_t i = 0; i < p->n; ++i) {
        int32_t L = 0;
        for (int c = 0; c < nc; ++c) {
            const int32_t Lc = level_of_distance(p, camera_distance(x + 3 * (int64_t)i, cam[c]), dn[c], df[c],
                                                 near_edge ? near_edge + i : NULL);
            if (Lc > L) L = Lc;
        }
        lev[i] = L;
    }
    return ORC_OK;
}

int orc_levels_guarded(const orc_params *p, const orc_lod *lod, const double *x, int32_t *lev,
                       uint8_t *near_edge)
{
    if (near_edge)
        for (int32_t i = 0; i < p->n; ++i) near_edge[i] = 0;
    if (lod->mode == 3) {
        int rc = levels_dtvs(p, lod, x, lev, near_edge);
        if (rc) return rc;
        for (int32_t i = 0; i < p->n; ++i)
            if (lev[i] < 1 || lev[i] < p->n_min || lev[i] > p->n_max) return ORC_ERR_ARG;
        return ORC_OK;
    }
    if (lod->mode == 2) {
        int rc = levels_dtc(p, lod, x, lev, near_edge);
        if (rc) return rc;
        for (int32_t i = 0; i < p->n; ++i)
            if (lev[i] < 1 || lev[i] < p->n_min || lev[i] > p->n_max) return ORC_ERR_ARG;
        return ORC_OK;
    }
    for (int32_t i = 0; i < p->n; ++i) {
        int32_t L = lod->mode == 0 ? p->n_max : lod->levels[i];
        if (L < 1 || L < p->n_min || L > p->n_max) return ORC_ERR_ARG;
        lev[i] = L;
    }
    return ORC_OK;
}

int orc_levels(const orc_params *p, const orc_lod *lod, const double *x, int32_t *lev)
{
    return orc_levels_guarded(p, lod, x, lev, NULL);
}

static int check_params(const orc_params *p)
{
    if (p->n < 0 || p->n_min < 1 || p->n_max < p->n_min || !(p->h > 0) || !(p->rho0 > 0) ||
        !(p->mass > 0) || !(p->eps >= 0) || !(p->dt > 0) || !(p->cohesion >= 0) ||
        !(p->cohesion < INFINITY))
        return ORC_ERR_ARG;
    for (int d = 0; d < 3; ++d)
        if (p->dims[d] < 1 || !(p->hi[d] >= p->lo[d])) return ORC_ERR_ARG;
    return ORC_OK;
}

/* Cohesion kernel C(r) of the force-based cohesion (see the readings). */
double orc_cohesion_spline(double r, double h)
{
    if (!(r > 0.0) || r > h) return 0.0;
    const double c = 32.0 / (M_PI * pow(h, 9));
    const double t = (h - r) * (h - r) * (h - r) * r * r * r;
    return 2.0 * r > h ? c * t : c * (2.0 * t - pow(h, 6) / 64.0);
}

/* Cohesion acceleration of particle i at the positions x over its
 * neighbour set ids[0..cnt) (ascending IDs). */
static void cohesion_of(const orc_params *p, const double *x, int32_t i, const int32_t *ids,
                        int64_t cnt, double a[3])
{
    a[0] = a[1] = a[2] = 0.0;
    const double *xi = x + 3 * (int64_t)i;
    for (int64_t e = 0; e < cnt; ++e) {
        const double *xj = x + 3 * (int64_t)ids[e];
        const double d[3] = {xi[0] - xj[0], xi[1] - xj[1], xi[2] - xj[2]};
        const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (!(r > 0.0)) continue;  /* coincident particles: no direction, no force */
        const double f = -p->cohesion * p->mass * orc_cohesion_spline(r, p->h) / r;
        for (int k = 0; k < 3; ++k) a[k] += f * d[k];
    }
}

/* The accelerations themselves (test access): a[n*3] from x over the
 * CSR sets (off[n+1], ids). */
int orc_cohesion_accel(const orc_params *p, const double *x, const int64_t *off, const int32_t *ids,
                       double *a)
{
    if (!p || p->n < 0 || !(p->h > 0) || !(p->mass > 0) || !(p->cohesion >= 0)) return ORC_ERR_ARG;
    for (int32_t i = 0; i < p->n; ++i) cohesion_of(p, x, i, ids + off[i], off[i + 1] - off[i], a + 3 * (int64_t)i);
    return ORC_OK;
}

/* Shared front half of a step: forces + prediction + clamp (Fig. 7, first
 * loop), cell keys, counting sort and neighbour sets (second loop). */
static int predict_and_neighbours(const orc_params *p, const double *x, double *v, double *xs,
                                  uint32_t *keys, int32_t *perm, int64_t **off, int32_t **ids)
{
    const int32_t n = p->n;
    for (int32_t i = 0; i < n; ++i) {
        for (int d = 0; d < 3; ++d) {
            v[3 * (int64_t)i + d] += p->dt * p->g[d];
            xs[3 * (int64_t)i + d] = x[3 * (int64_t)i + d] + p->dt * v[3 * (int64_t)i + d];
        }
        clamp_box(p, xs + 3 * (int64_t)i);
    }
    orc_cell_keys(p, xs, keys);
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_cells(p) + 1));
    if (!start) return ORC_ERR_MEM;
    int rc = orc_counting_sort(p, keys, perm, start);
    if (rc == ORC_OK) rc = find_neighbours(p, xs, perm, start, off, ids);
    free(start);
    return rc;
}

static void copy_trace_neighbours(const orc_params *p, orc_trace *tr, const int64_t *off,
                                  const int32_t *ids)
{
    if (!tr) return;
    tr->nbr_total = off[p->n];
    if (tr->nbr_count)
        for (int32_t i = 0; i < p->n; ++i) tr->nbr_count[i] = (int32_t)(off[i + 1] - off[i]);
    if (tr->nbr_ids && tr->nbr_cap >= off[p->n])
        memcpy(tr->nbr_ids, ids, sizeof(int32_t) * (size_t)off[p->n]);
}

/* ------------------------------------------------------------------ */
/* one APBF step (Fig. 7)                                              */
/* ------------------------------------------------------------------ */

static int check_contacts(const orc_params *p, const orc_contacts *oc)
{
    if (!oc) return ORC_OK;
    if (oc->count < 0 || oc->count > ORC_MAX_OBST || oc->stab_iters < 0 || oc->stab_s < 1 ||
        oc->stab_s > p->n_max)
        return ORC_ERR_ARG;
    for (int o = 0; o < oc->count; ++o) {
        const orc_obstacle *b = &oc->ob[o];
        if (b->kind < ORC_OB_SPHERE || b->kind > ORC_OB_BOX || !(b->a[0] > 0)) return ORC_ERR_ARG;
        if (b->kind != ORC_OB_SPHERE && !(b->a[1] > 0)) return ORC_ERR_ARG;
        if (b->kind == ORC_OB_BOX && !(b->a[2] > 0)) return ORC_ERR_ARG;
    }
    return ORC_OK;
}

int orc_apbf_step_contacts(const orc_params *p, const orc_lod *lod, const orc_contacts *oc,
                           double *x, double *v, orc_trace *tr);

/* x, v: n*3 doubles in particle-ID order, advanced in place by one step.
 * tr may be NULL; any of its pointers may be NULL. */
int orc_apbf_step(const orc_params *p, const orc_lod *lod, double *x, double *v, orc_trace *tr)
{
    return orc_apbf_step_contacts(p, lod, NULL, x, v, tr);
}

/* The same step with solid obstacles (oc may be NULL: walls only). */
int orc_apbf_step_contacts(const orc_params *p, const orc_lod *lod, const orc_contacts *oc,
                           double *x, double *v, orc_trace *tr)
{
    int rc = check_params(p);
    if (rc) return rc;
    if ((rc = check_contacts(p, oc))) return rc;
    const int32_t n = p->n;
    const int32_t K = p->n_max;
    size_t n3 = (size_t)n * 3;
    int32_t *lev = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    double *xs = (double *)malloc(sizeof(double) * (n3 ? n3 : 1));
    double *dp = (double *)malloc(sizeof(double) * (n3 ? n3 : 1));
    double *lam = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
    uint32_t *keys = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    uint8_t *cmask = (uint8_t *)calloc((size_t)(n ? n : 1), 1);
    int64_t *off = NULL;
    int32_t *ids = NULL;
    if (!lev || !xs || !dp || !lam || !keys || !perm || !cmask) { rc = ORC_ERR_MEM; goto done; }

    /* levels from the positions at the start of the step */
    rc = orc_levels(p, lod, x, lev);
    if (rc) goto done;

    rc = predict_and_neighbours(p, x, v, xs, keys, perm, &off, &ids);
    if (rc) goto done;

    if (tr) {
        if (tr->levels) memcpy(tr->levels, lev, sizeof(int32_t) * (size_t)n);
        if (tr->keys) memcpy(tr->keys, keys, sizeof(uint32_t) * (size_t)n);
        if (tr->perm) memcpy(tr->perm, perm, sizeof(int32_t) * (size_t)n);
        copy_trace_neighbours(p, tr, off, ids);
        if (tr->xs_iter) memcpy(tr->xs_iter, xs, sizeof(double) * n3);
    }

    if (p->cohesion > 0.0) {
        /* the cohesion force of the first loop, at x over the sets just found */
        double *acc = (double *)malloc(sizeof(double) * (n3 ? n3 : 1));
        if (!acc) { rc = ORC_ERR_MEM; goto done; }
#pragma omp parallel for schedule(dynamic, 256)
        for (int32_t i = 0; i < n; ++i) cohesion_of(p, x, i, ids + off[i], off[i + 1] - off[i], acc + 3 * (int64_t)i);
        for (int32_t i = 0; i < n; ++i) {
            for (int d = 0; d < 3; ++d) xs[3 * (int64_t)i + d] += p->dt * p->dt * acc[3 * (int64_t)i + d];
            clamp_box(p, xs + 3 * (int64_t)i);
        }
        free(acc);
    }

    if (oc && oc->count > 0) {
        /* contact finding from the predicted positions */
        for (int32_t i = 0; i < n; ++i)
            for (int o = 0; o < oc->count; ++o)
                if (orc_contact_found(&oc->ob[o], xs + 3 * (int64_t)i, p->h)) cmask[i] |= (uint8_t)(1u << o);
        /* pre-stabilisation of the particles with N_i < S: x* to the
         * obstacle's surface, x moved along (no velocity is gained) */
        for (int32_t it = 0; it < oc->stab_iters; ++it)
            for (int32_t i = 0; i < n; ++i) {
                if (!(lev[i] < oc->stab_s)) continue;
                double *xi = x + 3 * (int64_t)i, *si = xs + 3 * (int64_t)i;
                for (int o = 0; o < oc->count; ++o) {
                    double y[3];
                    if (!((cmask[i] >> o) & 1u) || !orc_obstacle_project(&oc->ob[o], si, y)) continue;
                    clamp_box(p, y);
                    for (int d = 0; d < 3; ++d) {
                        xi[d] += y[d] - si[d];
                        si[d] = y[d];
                    }
                }
            }
    }
    if (tr && tr->contacts) memcpy(tr->contacts, cmask, (size_t)n);

    /* solver iterations: particle i is active in iteration k while k < N_i */
    for (int32_t k = 0; k < K; ++k) {
#pragma omp parallel for schedule(dynamic, 256)
        for (int32_t i = 0; i < n; ++i)
            if (lev[i] > k) lam[i] = lambda_of(p, xs, i, ids + off[i], off[i + 1] - off[i], NULL, NULL);
#pragma omp parallel for schedule(dynamic, 256)
        for (int32_t i = 0; i < n; ++i)
            if (lev[i] > k) delta_p_of(p, xs, lam, i, ids + off[i], off[i + 1] - off[i], dp + 3 * (int64_t)i);
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i)
            if (lev[i] > k) {
                for (int d = 0; d < 3; ++d) xs[3 * (int64_t)i + d] += dp[3 * (int64_t)i + d];
                contact_response(p, oc, cmask[i], xs + 3 * (int64_t)i);
            }
        if (tr && tr->lambda_iter) memcpy(tr->lambda_iter + (size_t)k * n, lam, sizeof(double) * (size_t)n);
        if (tr && tr->xs_iter) memcpy(tr->xs_iter + (size_t)(k + 1) * n3, xs, sizeof(double) * n3);
    }

    /* velocity and position update for every particle */
    for (size_t e = 0; e < n3; ++e) {
        v[e] = (xs[e] - x[e]) / p->dt;
        x[e] = xs[e];
    }
done:
    free(lev); free(xs); free(dp); free(lam); free(keys); free(perm); free(cmask); free(off); free(ids);
    return rc;
}

/* ------------------------------------------------------------------ */
/* one APBF step with given neighbour sets and levels                  */
/* ------------------------------------------------------------------ */

/* The step of Fig. 7 with the discrete structure held fixed: levels
 * lev[n] and neighbour sets as CSR (off[n+1], ids, particle-ID order)
 * are inputs instead of being found.  With them fixed the step is a smooth
 * function of (x, v) away from wall contacts; its finite differences are
 * what an adjoint that keeps the neighbour sets constant differentiates. */
int orc_apbf_step_fixed(const orc_params *p, const int32_t *lev, const int64_t *off,
                        const int32_t *ids, double *x, double *v)
{
    int rc = check_params(p);
    if (rc) return rc;
    const int32_t n = p->n;
    const int32_t K = p->n_max;
    size_t n3 = (size_t)n * 3;
    double *xs = (double *)malloc(sizeof(double) * (n3 ? n3 : 1));
    double *dp = (double *)malloc(sizeof(double) * (n3 ? n3 : 1));
    double *lam = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
    if (!xs || !dp || !lam) { rc = ORC_ERR_MEM; goto done; }
    for (int32_t i = 0; i < n; ++i) {
        if (lev[i] < p->n_min || lev[i] > p->n_max) { rc = ORC_ERR_ARG; goto done; }
        for (int d = 0; d < 3; ++d) {
            v[3 * (int64_t)i + d] += p->dt * p->g[d];
            xs[3 * (int64_t)i + d] = x[3 * (int64_t)i + d] + p->dt * v[3 * (int64_t)i + d];
        }
        clamp_box(p, xs + 3 * (int64_t)i);
    }
    for (int32_t k = 0; k < K; ++k) {
#pragma omp parallel for schedule(dynamic, 256)
        for (int32_t i = 0; i < n; ++i)
            if (lev[i] > k) lam[i] = lambda_of(p, xs, i, ids + off[i], off[i + 1] - off[i], NULL, NULL);
#pragma omp parallel for schedule(dynamic, 256)
        for (int32_t i = 0; i < n; ++i)
            if (lev[i] > k) delta_p_of(p, xs, lam, i, ids + off[i], off[i + 1] - off[i], dp + 3 * (int64_t)i);
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i)
            if (lev[i] > k) {
                for (int d = 0; d < 3; ++d) xs[3 * (int64_t)i + d] += dp[3 * (int64_t)i + d];
                clamp_box(p, xs + 3 * (int64_t)i);
            }
    }
    for (size_t e = 0; e < n3; ++e) {
        v[e] = (xs[e] - x[e]) / p->dt;
        x[e] = xs[e];
    }
done:
    free(xs); free(dp); free(lam);
    return rc;
}

/* ------------------------------------------------------------------ */
/* reverse mode of the fixed-structure step                            */
/* ------------------------------------------------------------------ */

/* Hessian of the spiky kernel with respect to p_i at d = p_i - p_j, i.e. the
 * Jacobian of orc_spiky_grad: with grad W = phi(r) d and
 * phi(r) = -45/(pi h^6) (h - r)^2 / r, it is phi I + (phi'(r) / r) d d^T,
 * phi'(r) = 45/(pi h^6) (h - r)(h + r) / r^2.  Zero outside 0 < r < h. */
void orc_spiky_hess(const double d[3], double h, double H[9])
{
    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int e = 0; e < 9; ++e) H[e] = 0.0;
    if (r <= 0.0 || r >= h) return;
    double k = 45.0 / (M_PI * pow(h, 6));
    double phi = -k * (h - r) * (h - r) / r;
    double dphi_r = k * (h - r) * (h + r) / (r * r * r);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) H[3 * a + b] = (a == b ? phi : 0.0) + dphi_r * d[a] * d[b];
}

/* Gradient of the poly6 kernel with respect to p_i at d = p_i - p_j:
 * -6 * 315/(64 pi h^9) (h^2 - r^2)^2 d for r < h. */
static void poly6_grad(const double d[3], double h, double out[3])
{
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    out[0] = out[1] = out[2] = 0.0;
    if (r2 >= h * h) return;
    double t = h * h - r2;
    double c = -6.0 * 315.0 / (64.0 * M_PI * pow(h, 9)) * t * t;
    out[0] = c * d[0];
    out[1] = c * d[1];
    out[2] = c * d[2];
}

static void mat_vec_add(const double H[9], const double u[3], double s, double *acc)
{
    for (int a = 0; a < 3; ++a) acc[a] += s * (H[3 * a] * u[0] + H[3 * a + 1] * u[1] + H[3 * a + 2] * u[2]);
}

/* Vector-Jacobian product of orc_apbf_step_fixed: given (x, v) at the start
 * of the step and the adjoints gx, gv of the step's outputs (x', v'), both
 * float[3n] by particle ID, overwrite gx, gv with the adjoints of (x, v).
 * Levels, neighbour sets and the wall contacts of the forward step are held
 * fixed (the chain rule through Eqs. 4-7 with the gating of Eqs. 9-11 and the
 * prediction and update of Fig. 7).  Each pair's contribution is scattered
 * to both of its particles, following the forward formulas term by term:
 * the forward pass is recomputed and kept per iteration, then the iterations
 * are reversed. */
int orc_apbf_step_fixed_vjp(const orc_params *p, const int32_t *lev, const int64_t *off,
                            const int32_t *ids, const double *x, const double *v, double *gx,
                            double *gv)
{
    int rc = check_params(p);
    if (rc) return rc;
    const int32_t n = p->n;
    const int32_t K = p->n_max;
    const size_t n3 = (size_t)n * 3, nn = (size_t)(n ? n : 1);
    const double m = p->mass, rho0 = p->rho0, dt = p->dt;
    double *z = (double *)malloc(sizeof(double) * (K + 1) * (n3 ? n3 : 1));  /* z^k, k = 0..K */
    double *u = (double *)malloc(sizeof(double) * (K + 1) * (n3 ? n3 : 1));  /* pre-clamp values */
    double *lam = (double *)calloc((size_t)(K ? K : 1) * nn, sizeof(double)); /* lambda used at k */
    double *Cv = (double *)calloc((size_t)(K ? K : 1) * nn, sizeof(double));
    double *Sv = (double *)calloc((size_t)(K ? K : 1) * nn, sizeof(double));
    double *bz = (double *)calloc(n3 ? n3 : 1, sizeof(double));
    double *bdp = (double *)calloc(n3 ? n3 : 1, sizeof(double));
    double *bl = (double *)calloc(nn, sizeof(double));
    if (!z || !u || !lam || !Cv || !Sv || !bz || !bdp || !bl) { rc = ORC_ERR_MEM; goto done; }
    for (int32_t i = 0; i < n; ++i) {
        if (lev[i] < p->n_min || lev[i] > p->n_max) { rc = ORC_ERR_ARG; goto done; }
        for (int d = 0; d < 3; ++d) {
            double v1 = v[3 * (int64_t)i + d] + dt * p->g[d];
            u[3 * (int64_t)i + d] = x[3 * (int64_t)i + d] + dt * v1;
            z[3 * (int64_t)i + d] = u[3 * (int64_t)i + d];
        }
        clamp_box(p, z + 3 * (int64_t)i);
    }
    /* forward, keeping z^k, the unclamped values, lambda, C and S per iteration */
    for (int32_t k = 0; k < K; ++k) {
        const double *zk = z + (size_t)k * n3;
        double *zn = z + (size_t)(k + 1) * n3, *un = u + (size_t)(k + 1) * n3;
        double *lk = lam + (size_t)k * nn;
        if (k > 0) memcpy(lk, lam + (size_t)(k - 1) * nn, sizeof(double) * n);
        for (int32_t i = 0; i < n; ++i) {
            if (lev[i] <= k) continue;
            double rho;
            lk[i] = lambda_of(p, zk, i, ids + off[i], off[i + 1] - off[i], &rho,
                              Sv + (size_t)k * nn + i);
            Cv[(size_t)k * nn + i] = rho / rho0 - 1.0;
        }
        for (int32_t i = 0; i < n; ++i) {
            for (int d = 0; d < 3; ++d) zn[3 * (int64_t)i + d] = zk[3 * (int64_t)i + d];
            if (lev[i] <= k) continue;
            double dp[3];
            delta_p_of(p, zk, lk, i, ids + off[i], off[i + 1] - off[i], dp);
            for (int d = 0; d < 3; ++d) un[3 * (int64_t)i + d] = zk[3 * (int64_t)i + d] + dp[d];
            for (int d = 0; d < 3; ++d) zn[3 * (int64_t)i + d] = un[3 * (int64_t)i + d];
            clamp_box(p, zn + 3 * (int64_t)i);
        }
    }
    /* x' = z^K, v' = (z^K - x) / dt */
    for (size_t e = 0; e < n3; ++e) {
        bz[e] = gx[e] + gv[e] / dt;
        gx[e] = -gv[e] / dt;
    }
    for (int32_t k = K - 1; k >= 0; --k) {
        const double *zk = z + (size_t)k * n3, *un = u + (size_t)(k + 1) * n3;
        const double *lk = lam + (size_t)k * nn;
        /* clamp of the active particles' update */
        for (int32_t i = 0; i < n; ++i)
            for (int d = 0; d < 3; ++d) {
                size_t e = 3 * (size_t)i + d;
                if (lev[i] <= k) { bdp[e] = 0.0; continue; }
                if (!(un[e] > p->lo[d] && un[e] < p->hi[d])) bz[e] = 0.0;
                bdp[e] = bz[e];
            }
        /* Delta p_i = (1/rho0) sum_j (lambda_i + lambda_j) grad W(z_i - z_j) */
        for (int32_t i = 0; i < n; ++i) {
            if (lev[i] <= k) continue;
            const double *bi = bdp + 3 * (size_t)i;
            for (int64_t q = off[i]; q < off[i + 1]; ++q) {
                int32_t j = ids[q];
                double d[3], gw[3], H[9];
                for (int a = 0; a < 3; ++a) d[a] = zk[3 * (size_t)i + a] - zk[3 * (size_t)j + a];
                orc_spiky_grad(d, p->h, gw);
                orc_spiky_hess(d, p->h, H);
                double dl = (bi[0] * gw[0] + bi[1] * gw[1] + bi[2] * gw[2]) / rho0;
                bl[i] += dl;
                bl[j] += dl;
                double s = (lk[i] + lk[j]) / rho0;
                double t[3] = {0.0, 0.0, 0.0};
                mat_vec_add(H, bi, s, t);
                for (int a = 0; a < 3; ++a) {
                    bz[3 * (size_t)i + a] += t[a];
                    bz[3 * (size_t)j + a] -= t[a];
                }
            }
        }
        /* lambda_i = -C_i / (S_i + eps) of the particles active at k: the
         * adjoint collected over every later iteration that used this value
         * is spent here */
        for (int32_t i = 0; i < n; ++i) {
            if (lev[i] <= k) continue;
            const double C = Cv[(size_t)k * nn + i], S = Sv[(size_t)k * nn + i];
            const double bC = -bl[i] / (S + p->eps);
            const double bS = bl[i] * C / ((S + p->eps) * (S + p->eps));
            bl[i] = 0.0;
            /* C_i = rho_i / rho0 - 1, rho_i = m W(0) + m sum_j W(z_i - z_j);
             * S_i = (1/m) (|G_i|^2 + sum_j |g_ij|^2), G_i = (m/rho0) sum_j grad W_ij,
             * g_ij = -(m/rho0) grad W_ij */
            double G[3] = {0.0, 0.0, 0.0};
            for (int64_t q = off[i]; q < off[i + 1]; ++q) {
                int32_t j = ids[q];
                double d[3], gw[3];
                for (int a = 0; a < 3; ++a) d[a] = zk[3 * (size_t)i + a] - zk[3 * (size_t)j + a];
                orc_spiky_grad(d, p->h, gw);
                for (int a = 0; a < 3; ++a) G[a] += m / rho0 * gw[a];
            }
            for (int64_t q = off[i]; q < off[i + 1]; ++q) {
                int32_t j = ids[q];
                double d[3], gw[3], gp[3], H[9];
                for (int a = 0; a < 3; ++a) d[a] = zk[3 * (size_t)i + a] - zk[3 * (size_t)j + a];
                orc_spiky_grad(d, p->h, gw);
                orc_spiky_hess(d, p->h, H);
                poly6_grad(d, p->h, gp);
                /* adjoint of grad W_ij: from G_i and from g_ij */
                double bg[3];
                for (int a = 0; a < 3; ++a) {
                    double gij = -m / rho0 * gw[a];
                    bg[a] = (m / rho0) * (2.0 * bS * G[a] / m) - (m / rho0) * (2.0 * bS * gij / m);
                }
                double t[3] = {0.0, 0.0, 0.0};
                mat_vec_add(H, bg, 1.0, t);
                for (int a = 0; a < 3; ++a) {
                    double c = bC * m / rho0 * gp[a];
                    bz[3 * (size_t)i + a] += t[a] + c;
                    bz[3 * (size_t)j + a] -= t[a] + c;
                }
            }
        }
    }
    /* prediction: z^0 = clamp(x + dt (v + dt g)) */
    for (int32_t i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            size_t e = 3 * (size_t)i + d;
            double b = (u[e] > p->lo[d] && u[e] < p->hi[d]) ? bz[e] : 0.0;
            gx[e] += b;
            gv[e] = dt * b;
        }
done:
    free(z); free(u); free(lam); free(Cv); free(Sv); free(bz); free(bdp); free(bl);
    return rc;
}

/* ------------------------------------------------------------------ */
/* one plain PBF step, its own loop without gating                     */
/* ------------------------------------------------------------------ */

int orc_pbf_step(const orc_params *p, int32_t iters, double *x, double *v)
{
    int rc = check_params(p);
    if (rc) return rc;
    if (iters < 0) return ORC_ERR_ARG;
    const int32_t n = p->n;
    size_t n3 = (size_t)n * 3;
    double *xs = (double *)malloc(sizeof(double) * (n3 ? n3 : 1));
    double *dp = (double *)malloc(sizeof(double) * (n3 ? n3 : 1));
    double *lam = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
    uint32_t *keys = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int64_t *off = NULL;
    int32_t *ids = NULL;
    if (!xs || !dp || !lam || !keys || !perm) { rc = ORC_ERR_MEM; goto done; }
    rc = predict_and_neighbours(p, x, v, xs, keys, perm, &off, &ids);
    if (rc) goto done;
    for (int32_t it = 0; it < iters; ++it) {
#pragma omp parallel for schedule(dynamic, 256)
        for (int32_t i = 0; i < n; ++i)
            lam[i] = lambda_of(p, xs, i, ids + off[i], off[i + 1] - off[i], NULL, NULL);
#pragma omp parallel for schedule(dynamic, 256)
        for (int32_t i = 0; i < n; ++i)
            delta_p_of(p, xs, lam, i, ids + off[i], off[i + 1] - off[i], dp + 3 * (int64_t)i);
#pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i) {
            for (int d = 0; d < 3; ++d) xs[3 * (int64_t)i + d] += dp[3 * (int64_t)i + d];
            clamp_box(p, xs + 3 * (int64_t)i);
        }
    }
    for (size_t e = 0; e < n3; ++e) {
        v[e] = (xs[e] - x[e]) / p->dt;
        x[e] = xs[e];
    }
done:
    free(xs); free(dp); free(lam); free(keys); free(perm); free(off); free(ids);
    return rc;
}

/* ------------------------------------------------------------------ */
/* SPH density of every particle at given positions (Eq. 6), for the   */
/* average-density report; neighbours by the same grid search.         */
/* ------------------------------------------------------------------ */

int orc_density(const orc_params *p, const double *x, double *rho)
{
    int rc = check_params(p);
    if (rc) return rc;
    const int32_t n = p->n;
    uint32_t *keys = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_cells(p) + 1));
    int64_t *off = NULL;
    int32_t *ids = NULL;
    if (!keys || !perm || !start) { rc = ORC_ERR_MEM; goto done; }
    orc_cell_keys(p, x, keys);
    rc = orc_counting_sort(p, keys, perm, start);
    if (rc) goto done;
    rc = find_neighbours(p, x, perm, start, &off, &ids);
    if (rc) goto done;
#pragma omp parallel for schedule(dynamic, 256)
    for (int32_t i = 0; i < n; ++i) {
        double r = p->mass * orc_poly6(0.0, p->h);
        const double *xi = x + 3 * (int64_t)i;
        for (int64_t q = off[i]; q < off[i + 1]; ++q) {
            const double *xj = x + 3 * (int64_t)ids[q];
            double d0 = xi[0] - xj[0], d1 = xi[1] - xj[1], d2 = xi[2] - xj[2];
            r += p->mass * orc_poly6(d0 * d0 + d1 * d1 + d2 * d2, p->h);
        }
        rho[i] = r;
    }
done:
    free(keys); free(perm); free(start); free(off); free(ids);
    return rc;
}

void orc_set_threads(int32_t t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

int32_t orc_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
