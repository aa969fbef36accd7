/*
 * FP64 CPU oracle for ray-traced solar-radiation-pressure (SRP) force and
 * torque on an articulated, triangulated spacecraft.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * statement of what the method computes.  It is used by the tests, by the
 * smoke check and by the CPU-baseline leg of the benchmark; the GPU library
 * never calls it, links it or shares code with it.
 *
 * What it follows, step by step (paper sections):
 *   - Articulation (Sec. 4.4.1 tree G=(N,E,L), edge labels (p,A,I);
 *     Sec. 4.4.2 steps 1, 4 and 5): every node's triangles are moved by the
 *     composition of the rotations on the path from the root, each a rotation
 *     about the edge's pivot and axes, with angles clamped to the intervals.
 *   - Per-pixel independent rays over a discretised image plane (Sec. 4.3):
 *     an N x N grid of parallel rays travelling along the photon direction,
 *     one ray per pixel centre, over the tight projected window of the mesh.
 *   - First hit along each ray = self-shadowing (Sec. 1, ray tracing with
 *     self-shadowing and multiple reflections).
 *   - Momentum transfer at a hit by the flat-plate absorbed / specular /
 *     diffuse law (the paper keeps the SRP formulation of its predecessor,
 *     Sec. 4.3; per-part rho_s, rho_d, rho_a with rho_s+rho_d+rho_a = 1,
 *     Sec. 5.1 table of spacecraft models).
 *   - Secondary rays followed iteratively for a given number of levels
 *     (Sec. 4.3; two levels in Sec. 6.1).
 *   - Compensated summation of all contributions (Kahan, Sec. 1 and 4.3),
 *     here the Kahan-Babuska-Neumaier variant in FP64.
 *
 * Readings of points the paper leaves open (each one stated where used):
 *   R1 photon direction d = -s/|s| with s the spacecraft->Sun direction.
 *   R2 image-plane basis: helper h = e_z if |d_z| < 0.9 else e_x;
 *      u = normalize(h x d), v = d x u.
 *   R3 window: tight bounds of the articulated vertices projected on u and v;
 *      pixel (i,j) centre at u_min + (i+1/2) W_u/N, v_min + (j+1/2) W_v/N;
 *      ray origins on the plane h_min - 1e-3 L - 1e-3 along d, L = max(W_u,W_v);
 *      pixel area A_pix = W_u W_v / N^2.  A window of zero area gives zero.
 *   R4 triangles are two-sided; the shading normal faces the incoming ray.
 *   R5 watertight ray/triangle test (Woop, Benthin, Wald 2013), inclusive
 *      edges; a triangle whose projection along the ray has zero area (zero-
 *      area triangles, exactly edge-on triangles) is never hit.
 *   R6 closest hit: smallest t; on an exact tie the smallest triangle index.
 *   R7 the specular chain: at a hit with rho_s > 0 the ray continues along
 *      d' = d + 2 c n with weight w rho_s, from the hit point, excluding the
 *      source triangle and requiring t > 1e-6 L; a miss ends the chain.
 *      Without diffuse rays (R10) diffuse re-emission is not traced: its
 *      Lambertian recoil is the rho_d/3 term of the law.
 *   R8 per hit: dF = w P A_pix [(1-rho_s) d - 2 (rho_s c + rho_d/3) n],
 *      c = -n.d, dtau = (x - ref) x dF.
 *   R9 summation order: pixels in row-major order (j outer, i inner), within
 *      a pixel its chain in generation order, each emitting hit followed by
 *      its diffuse rays in set order.
 *   R10 diffuse secondary rays (Sec. 4.3: the number of secondary rays made
 *      at each interaction sets the level of scattering; Sec. 6.1 uses 16
 *      diffuse rays with two secondary levels).  With K > 0, a chain hit of
 *      generation g < B on a material with rho_d > 0 also emits K diffuse
 *      rays of weight w rho_d / K each, from the hit point (same exclusion
 *      and t > 1e-6 L as R7).  Their directions are a fixed cosine-weighted
 *      set: ray k has u = (k + 1/2)/K, phi = 2 pi frac(k (sqrt(5) - 1)/2) and
 *      local direction (sqrt(u) cos phi, sqrt(u) sin phi, sqrt(1 - u)) (a
 *      Fibonacci point set on the unit disk lifted to the hemisphere, which
 *      makes the lifted directions cosine distributed), placed in the hit's
 *      frame (t, b, n): t = normalize(h x n) with h = (1, 2, 3) (e_x if
 *      h x n = 0), b = n x t.  The emitting hit's diffuse recoil is the
 *      exact mean m of the K emitted world directions instead of 2/3 n:
 *      dF = w P A_pix [(1 - rho_s) d - 2 rho_s c n - rho_d m], so the fan's
 *      momentum is accounted for exactly.  A diffuse ray that hits deposits
 *      at its first hit by the R8 law with its own weight and direction and
 *      spawns nothing; one that misses leaves.  Diffuse rays count as
 *      secondary rays.
 *
 * Units: metres, N/m^2 for the pressure, newtons and newton-metres out.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#ifdef _OPENMP
#include <omp.h>
#endif

/* Number of OpenMP threads the pixel loops use. */
int32_t orc_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------- vectors */
static void v_sub(const double *a, const double *b, double *o) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
static double v_dot(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void v_cross(const double *a, const double *b, double *o)
{
    double x = a[1] * b[2] - a[2] * b[1];
    double y = a[2] * b[0] - a[0] * b[2];
    double z = a[0] * b[1] - a[1] * b[0];
    o[0] = x; o[1] = y; o[2] = z;
}
static double v_norm(const double *a) { return sqrt(v_dot(a, a)); }

/* 3x3 row-major matrices */
static void m_mul(const double *A, const double *B, double *C)
{
    double T[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            T[3 * r + c] = A[3 * r + 0] * B[0 * 3 + c] + A[3 * r + 1] * B[1 * 3 + c] + A[3 * r + 2] * B[2 * 3 + c];
    memcpy(C, T, sizeof T);
}
static void m_vec(const double *A, const double *x, double *y)
{
    double t0 = A[0] * x[0] + A[1] * x[1] + A[2] * x[2];
    double t1 = A[3] * x[0] + A[4] * x[1] + A[5] * x[2];
    double t2 = A[6] * x[0] + A[7] * x[1] + A[8] * x[2];
    y[0] = t0; y[1] = t1; y[2] = t2;
}

/* Rotation by angle th about unit axis a (Rodrigues). */
static void rodrigues(const double *a_in, double th, double *R)
{
    double n = v_norm(a_in);
    double a[3] = {a_in[0] / n, a_in[1] / n, a_in[2] / n};
    double c = cos(th), s = sin(th), C = 1.0 - c;
    R[0] = c + a[0] * a[0] * C;        R[1] = a[0] * a[1] * C - a[2] * s; R[2] = a[0] * a[2] * C + a[1] * s;
    R[3] = a[1] * a[0] * C + a[2] * s; R[4] = c + a[1] * a[1] * C;        R[5] = a[1] * a[2] * C - a[0] * s;
    R[6] = a[2] * a[0] * C - a[1] * s; R[7] = a[2] * a[1] * C + a[0] * s; R[8] = c + a[2] * a[2] * C;
}

/* ------------------------------------------------------------ compensated */
typedef struct { double s, c; } ksum;
static void ks_add(ksum *k, double x)
{
    double t = k->s + x;
    if (fabs(k->s) >= fabs(x)) k->c += (k->s - t) + x;
    else k->c += (x - t) + k->s;
    k->s = t;
}
static double ks_val(const ksum *k) { return k->s + k->c; }

/* ------------------------------------------------------------ validation */
int orc_validate(const orc_scene *S)
{
    if (!S || S->nt < 0 || S->nv < 0 || S->nn < 1 || S->nm < 1) return ORC_ERR_ARG;
    if (S->parent[0] != -1 || S->n_axes[0] != 0) return ORC_ERR_ARG;
    for (int32_t k = 1; k < S->nn; ++k) {
        if (S->parent[k] < 0 || S->parent[k] >= k) return ORC_ERR_ARG;
        if (S->n_axes[k] < 0 || S->n_axes[k] > 3) return ORC_ERR_ARG;
    }
    for (int32_t m = 0; m < S->nm; ++m) {
        double rs = S->mats[2 * m], rd = S->mats[2 * m + 1];
        if (!(rs >= 0 && rd >= 0 && rs + rd <= 1.0 + 1e-12)) return ORC_ERR_ARG;
    }
    for (int64_t t = 0; t < S->nt; ++t) {
        for (int c = 0; c < 3; ++c)
            if (S->tris[3 * t + c] < 0 || S->tris[3 * t + c] >= S->nv) return ORC_ERR_ARG;
        if (S->tri_mat[t] < 0 || S->tri_mat[t] >= S->nm) return ORC_ERR_ARG;
        if (S->tri_node[t] < 0 || S->tri_node[t] >= S->nn) return ORC_ERR_ARG;
    }
    return ORC_OK;
}

int32_t orc_n_dof(const orc_scene *S)
{
    int32_t n = 0;
    for (int32_t k = 0; k < S->nn; ++k) n += S->n_axes[k];
    return n;
}

/* ------------------------------------------------------------ articulation
 * Sec. 4.4.1-4.4.2: node transform M_k = M_parent o T(p) R(a1,th1) R(a2,th2).. T(-p)
 * with pivot p and axes a in the rest-pose body frame (axes composed from the
 * first to the last), each angle clamped to its interval; M_root = identity.
 * xf[12*k]: R (row-major 3x3) then t, so x_world = R x_rest + t.
 */
int orc_node_transforms(const orc_scene *S, const double *angles, double *xf)
{
    int32_t dof = 0;
    for (int32_t k = 0; k < S->nn; ++k) {
        double *X = xf + 12 * k;
        if (k == 0) {
            memset(X, 0, 12 * sizeof(double));
            X[0] = X[4] = X[8] = 1.0;
            continue;
        }
        double Rl[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
        for (int32_t a = 0; a < S->n_axes[k]; ++a, ++dof) {
            double th = angles ? angles[dof] : 0.0;
            double lo = S->lo[3 * k + a], hi = S->hi[3 * k + a];
            if (th < lo) th = lo;
            if (th > hi) th = hi;
            double Ra[9];
            rodrigues(S->axes + 9 * k + 3 * a, th, Ra);
            m_mul(Rl, Ra, Rl);
        }
        const double *p = S->pivot + 3 * k;
        double Rp[3], tl[3];
        m_vec(Rl, p, Rp);
        v_sub(p, Rp, tl);                       /* local: x -> Rl x + (p - Rl p) */
        const double *P = xf + 12 * S->parent[k];
        m_mul(P, Rl, X);                        /* R = R_par Rl */
        double Pt[3];
        m_vec(P, tl, Pt);                       /* t = R_par tl + t_par */
        X[9] = Pt[0] + P[9];
        X[10] = Pt[1] + P[10];
        X[11] = Pt[2] + P[11];
    }
    return ORC_OK;
}

int orc_articulate(const orc_scene *S, const double *angles, double *wtri)
{
    double *xf = (double *)malloc(sizeof(double) * 12 * (size_t)S->nn);
    if (!xf) return ORC_ERR_OOM;
    orc_node_transforms(S, angles, xf);
    for (int64_t t = 0; t < S->nt; ++t) {
        const double *X = xf + 12 * S->tri_node[t];
        for (int c = 0; c < 3; ++c) {
            const double *x = S->verts + 3 * (int64_t)S->tris[3 * t + c];
            double y[3];
            m_vec(X, x, y);
            wtri[9 * t + 3 * c + 0] = y[0] + X[9];
            wtri[9 * t + 3 * c + 1] = y[1] + X[10];
            wtri[9 * t + 3 * c + 2] = y[2] + X[11];
        }
    }
    free(xf);
    return ORC_OK;
}

/* ------------------------------------------------------------ ray grid (R1-R3) */
static int grid_setup(const orc_scene *S, const double *wtri, const orc_params *P, orc_grid *g)
{
    double sn = v_norm(P->sun_dir);
    if (!(sn > 0) || !isfinite(sn)) return ORC_ERR_ARG;
    for (int c = 0; c < 3; ++c) g->d[c] = -P->sun_dir[c] / sn;
    double h[3] = {0, 0, 1};
    if (!(fabs(g->d[2]) < 0.9)) { h[0] = 1; h[2] = 0; }
    v_cross(h, g->d, g->u);
    double un = v_norm(g->u);
    for (int c = 0; c < 3; ++c) g->u[c] /= un;
    v_cross(g->d, g->u, g->v);
    double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY, hmin = INFINITY;
    for (int64_t k = 0; k < 3 * S->nt; ++k) {
        const double *x = wtri + 3 * k;
        double a = v_dot(x, g->u), b = v_dot(x, g->v), c = v_dot(x, g->d);
        if (a < umin) umin = a;
        if (a > umax) umax = a;
        if (b < vmin) vmin = b;
        if (b > vmax) vmax = b;
        if (c < hmin) hmin = c;
    }
    if (S->nt == 0) umin = umax = vmin = vmax = hmin = 0;
    g->umin = umin; g->umax = umax; g->vmin = vmin; g->vmax = vmax; g->hmin = hmin;
    g->wu = umax - umin;
    g->wv = vmax - vmin;
    g->L = g->wu > g->wv ? g->wu : g->wv;
    g->a_pix = g->wu * g->wv / ((double)P->n * (double)P->n);
    g->h0 = hmin - 1e-3 * g->L - 1e-3;
    return ORC_OK;
}

/* Origin of the ray through pixel (i, j). */
static void pixel_origin(const orc_grid *g, int32_t n, int64_t i, int64_t j, double *o)
{
    double a = g->umin + ((double)i + 0.5) * g->wu / (double)n;
    double b = g->vmin + ((double)j + 0.5) * g->wv / (double)n;
    for (int c = 0; c < 3; ++c) o[c] = a * g->u[c] + b * g->v[c] + g->h0 * g->d[c];
}

/* ------------------------------------------------------------ intersection (R5)
 * Watertight ray/triangle test (Woop, Benthin and Wald, JCGT 2013): the ray
 * becomes the +z axis of a sheared frame, the triangle's corners are
 * projected into that frame and the three 2-D edge functions decide the hit.
 * A shared edge gets the same edge function (negated) in both triangles, so
 * a ray can never pass between two triangles that share an edge.  Edges are
 * inclusive; a triangle whose projection has zero signed area (det == 0) is
 * never hit.
 */
static int wt_hit(const double *o, const double *d, const double *tv, double *t_out)
{
    int kz = 0;
    if (fabs(d[1]) > fabs(d[kz])) kz = 1;
    if (fabs(d[2]) > fabs(d[kz])) kz = 2;
    int kx = (kz + 1) % 3, ky = (kx + 1) % 3;
    if (d[kz] < 0.0) { int s = kx; kx = ky; ky = s; }     /* keep the winding */
    double Sx = d[kx] / d[kz], Sy = d[ky] / d[kz], Sz = 1.0 / d[kz];
    double A[3], B[3], Cv[3];
    v_sub(tv, o, A);
    v_sub(tv + 3, o, B);
    v_sub(tv + 6, o, Cv);
    double Ax = A[kx] - Sx * A[kz], Ay = A[ky] - Sy * A[kz];
    double Bx = B[kx] - Sx * B[kz], By = B[ky] - Sy * B[kz];
    double Cx = Cv[kx] - Sx * Cv[kz], Cy = Cv[ky] - Sy * Cv[kz];
    double U = Cx * By - Cy * Bx;
    double V = Ax * Cy - Ay * Cx;
    double W = Bx * Ay - By * Ax;
    if ((U < 0.0 || V < 0.0 || W < 0.0) && (U > 0.0 || V > 0.0 || W > 0.0)) return 0;
    double det = U + V + W;
    if (det == 0.0) return 0;
    double T = U * (Sz * A[kz]) + V * (Sz * B[kz]) + W * (Sz * Cv[kz]);
    *t_out = T / det;
    return 1;
}

/* Closest-hit update with the tie rule R6. */
static void consider(const double *o, const double *d, const double *wtri, int64_t t_idx,
                     double tmin, int64_t exclude, double *best_t, int64_t *best)
{
    if (t_idx == exclude) return;
    double t;
    if (!wt_hit(o, d, wtri + 9 * t_idx, &t)) return;
    if (!(t > tmin)) return;
    if (t < *best_t || (t == *best_t && t_idx < *best)) {
        *best_t = t;
        *best = t_idx;
    }
}

/* ------------------------------------------------------------ oracle BVH
 * A plain median-split bounding-volume hierarchy over the articulated
 * triangles, used only to make large cases finish; it must (and is tested
 * to) return exactly what the brute-force loop returns.  Boxes are padded so
 * that rounding in the slab test can never drop a triangle.
 */
typedef struct { double lo[3], hi[3]; int64_t left, right, first, count; } bnode;
typedef struct { bnode *n; int64_t nn; int64_t *idx; } bvh;

static void tri_box(const double *tv, double *lo, double *hi)
{
    for (int c = 0; c < 3; ++c) {
        lo[c] = fmin(tv[c], fmin(tv[3 + c], tv[6 + c]));
        hi[c] = fmax(tv[c], fmax(tv[3 + c], tv[6 + c]));
    }
}

static int cmp_axis;
static const double *cmp_cent;
static int cmp_fn(const void *a, const void *b)
{
    double x = cmp_cent[3 * *(const int64_t *)a + cmp_axis], y = cmp_cent[3 * *(const int64_t *)b + cmp_axis];
    if (x < y) return -1;
    if (x > y) return 1;
    int64_t ia = *(const int64_t *)a, ib = *(const int64_t *)b;
    return ia < ib ? -1 : ia > ib;
}

static int64_t bvh_build_rec(bvh *B, const double *wtri, const double *cent, int64_t first, int64_t count, double pad)
{
    int64_t me = B->nn++;
    bnode *n = &B->n[me];
    for (int c = 0; c < 3; ++c) { n->lo[c] = INFINITY; n->hi[c] = -INFINITY; }
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t k = first; k < first + count; ++k) {
        double lo[3], hi[3];
        tri_box(wtri + 9 * B->idx[k], lo, hi);
        for (int c = 0; c < 3; ++c) {
            n->lo[c] = fmin(n->lo[c], lo[c] - pad);
            n->hi[c] = fmax(n->hi[c], hi[c] + pad);
            clo[c] = fmin(clo[c], cent[3 * B->idx[k] + c]);
            chi[c] = fmax(chi[c], cent[3 * B->idx[k] + c]);
        }
    }
    n->left = n->right = -1;
    n->first = first;
    n->count = count;
    if (count <= 4) return me;
    int ax = 0;
    for (int c = 1; c < 3; ++c)
        if (chi[c] - clo[c] > chi[ax] - clo[ax]) ax = c;
    cmp_axis = ax;
    cmp_cent = cent;
    qsort(B->idx + first, (size_t)count, sizeof(int64_t), cmp_fn);
    int64_t half = count / 2;
    int64_t l = bvh_build_rec(B, wtri, cent, first, half, pad);
    int64_t r = bvh_build_rec(B, wtri, cent, first + half, count - half, pad);
    B->n[me].left = l;
    B->n[me].right = r;
    B->n[me].count = 0;
    return me;
}

static int bvh_build(bvh *B, const double *wtri, int64_t nt, double pad)
{
    B->n = (bnode *)malloc(sizeof(bnode) * (size_t)(2 * nt + 1));
    B->idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nt + 1));
    double *cent = (double *)malloc(sizeof(double) * 3 * (size_t)(nt + 1));
    if (!B->n || !B->idx || !cent) { free(cent); return ORC_ERR_OOM; }
    B->nn = 0;
    for (int64_t t = 0; t < nt; ++t) {
        B->idx[t] = t;
        for (int c = 0; c < 3; ++c)
            cent[3 * t + c] = (wtri[9 * t + c] + wtri[9 * t + 3 + c] + wtri[9 * t + 6 + c]) / 3.0;
    }
    if (nt > 0) bvh_build_rec(B, wtri, cent, 0, nt, pad);
    free(cent);
    return ORC_OK;
}

static void bvh_free(bvh *B) { free(B->n); free(B->idx); }

static int box_hit(const bnode *n, const double *o, const double *d, double tmin, double tmax)
{
    double t0 = tmin, t1 = tmax;
    for (int c = 0; c < 3; ++c) {
        if (d[c] == 0.0) {
            if (o[c] < n->lo[c] || o[c] > n->hi[c]) return 0;
            continue;
        }
        double a = (n->lo[c] - o[c]) / d[c], b = (n->hi[c] - o[c]) / d[c];
        if (a > b) { double s = a; a = b; b = s; }
        if (a > t0) t0 = a;
        if (b < t1) t1 = b;
        if (t0 > t1) return 0;
    }
    return 1;
}

/* Closest hit along o + t d with t > tmin, skipping triangle `exclude`.
 * cnt (may be NULL) accumulates the box and triangle tests made (a count of
 * work only: the result does not depend on it). */
static void closest_hit(const bvh *B, const double *wtri, int64_t nt, const double *o, const double *d,
                        double tmin, int64_t exclude, double *best_t, int64_t *best, int64_t *cnt)
{
    *best_t = INFINITY;
    *best = -1;
    if (!B) {
        for (int64_t t = 0; t < nt; ++t) consider(o, d, wtri, t, tmin, exclude, best_t, best);
        if (cnt) cnt[1] += nt;
        return;
    }
    if (B->nn == 0) return;
    int64_t stack[256];
    int sp = 0;
    stack[sp++] = 0;
    while (sp) {
        const bnode *n = &B->n[stack[--sp]];
        if (cnt) cnt[0]++;
        if (!box_hit(n, o, d, tmin, *best_t)) continue;
        if (n->count) {
            if (cnt) cnt[1] += n->count;
            for (int64_t k = n->first; k < n->first + n->count; ++k)
                consider(o, d, wtri, B->idx[k], tmin, exclude, best_t, best);
        } else {
            stack[sp++] = n->left;
            stack[sp++] = n->right;
        }
    }
}

/* ------------------------------------------------------------ momentum law (R4, R8) */
/* Unit geometric normal of triangle tv (not oriented). */
static void tri_normal(const double *tv, double *n)
{
    double e1[3], e2[3];
    v_sub(tv + 3, tv, e1);
    v_sub(tv + 6, tv, e2);
    v_cross(e1, e2, n);
    double l = v_norm(n);
    n[0] /= l; n[1] /= l; n[2] /= l;
}

/* Normal nf oriented against the incoming direction d (R4); returns c = -n.d. */
static double orient(const double *nf, const double *d, double *n)
{
    double sgn = v_dot(nf, d) > 0 ? -1.0 : 1.0;
    for (int c = 0; c < 3; ++c) n[c] = sgn * nf[c];
    return -v_dot(n, d);
}

/* Contribution of one hit (R8): ray weight w, incoming direction d, oriented
 * normal n with c = -n.d, material (rs, rd), hit point x, scale = P A_pix.
 * mdiff = NULL: the law's Lambertian recoil 2/3 rho_d n; else the emitted
 * diffuse rays' mean direction m replaces 2/3 n (R10).  Writes dF and dtau. */
static void shade(double scale, double w, const double *d, const double *n, double cth, double rs,
                  double rd, const double *mdiff, const double *x, const double *ref, double *dF, double *dT)
{
    double a = w * scale * (1.0 - rs);
    if (!mdiff) {
        double b = -2.0 * w * scale * (rs * cth + rd / 3.0);
        for (int c = 0; c < 3; ++c) dF[c] = a * d[c] + b * n[c];
    } else {
        double b = -2.0 * w * scale * rs * cth, e = -w * scale * rd;
        for (int c = 0; c < 3; ++c) dF[c] = a * d[c] + b * n[c] + e * mdiff[c];
    }
    double r[3];
    v_sub(x, ref, r);
    v_cross(r, dF, dT);
}

/* ------------------------------------------------------------ diffuse set (R10) */
static const double ORC_PI = 3.14159265358979323846;

/* Local direction of diffuse ray k of K. */
static void diffuse_local(int32_t K, int32_t k, double *l)
{
    double g = (sqrt(5.0) - 1.0) / 2.0;
    double u = ((double)k + 0.5) / (double)K;
    double f = (double)k * g;
    f -= floor(f);
    double phi = 2.0 * ORC_PI * f;
    double r = sqrt(u);
    l[0] = r * cos(phi);
    l[1] = r * sin(phi);
    l[2] = sqrt(1.0 - u);
}

int orc_diffuse_set(int32_t K, double *l)
{
    if (K < 1 || !l) return ORC_ERR_ARG;
    for (int32_t k = 0; k < K; ++k) diffuse_local(K, k, l + 3 * k);
    return ORC_OK;
}

/* Tangent frame of unit normal n: t = normalize(h x n), b = n x t. */
static void tangent_frame(const double *n, double *t, double *b)
{
    const double h[3] = {1.0, 2.0, 3.0}, ex[3] = {1.0, 0.0, 0.0};
    v_cross(h, n, t);
    double l = v_norm(t);
    if (!(l > 0)) {
        v_cross(ex, n, t);
        l = v_norm(t);
    }
    t[0] /= l; t[1] /= l; t[2] /= l;
    v_cross(n, t, b);
}

/* World directions of the K diffuse rays at a hit with oriented normal n
 * (dirs: K x 3) and their mean m. */
static void diffuse_fan(int32_t K, const double *n, double *dirs, double *m)
{
    double t[3], b[3];
    tangent_frame(n, t, b);
    m[0] = m[1] = m[2] = 0.0;
    for (int32_t k = 0; k < K; ++k) {
        double l[3];
        diffuse_local(K, k, l);
        for (int c = 0; c < 3; ++c) {
            dirs[3 * k + c] = l[0] * t[c] + l[1] * b[c] + l[2] * n[c];
            m[c] += dirs[3 * k + c];
        }
    }
    for (int c = 0; c < 3; ++c) m[c] /= (double)K;
}

int32_t orc_record_slots(const orc_params *P)
{
    return P->bounces + 1 + P->bounces * (P->n_diffuse > 0 ? P->n_diffuse : 0);
}

/* ------------------------------------------------------------ evaluation */
typedef struct { double f[6]; int64_t hits, sec, sec_hits, dif, dif_hits, tests[2]; } pix_out;

static void trace_pixel(const orc_scene *S, const double *wtri, const bvh *B, const orc_params *P,
                        const orc_grid *g, int64_t pix, pix_out *po, int32_t *ids, double *ts,
                        double *fan /* K x 3 scratch */)
{
    int32_t n = P->n, K = P->n_diffuse > 0 ? P->n_diffuse : 0;
    int64_t i = pix % n, j = pix / n;
    double o[3], d[3] = {g->d[0], g->d[1], g->d[2]};
    pixel_origin(g, n, i, j, o);
    ksum acc[6];
    memset(acc, 0, sizeof acc);
    memset(po, 0, sizeof *po);
    double w = 1.0, tmin = 0.0;
    int64_t exclude = -1;
    double scale = P->pressure * g->a_pix;
    for (int32_t gen = 0; gen <= P->bounces; ++gen) {
        double bt;
        int64_t bi;
        closest_hit(B, wtri, S->nt, o, d, tmin, exclude, &bt, &bi, po->tests);
        if (bi < 0) break;
        if (ids) ids[gen] = (int32_t)bi;
        if (ts) ts[gen] = bt;
        if (gen == 0) po->hits++;
        else po->sec_hits++;
        double x[3] = {o[0] + bt * d[0], o[1] + bt * d[1], o[2] + bt * d[2]};
        double nf[3], nn[3], dF[3], dT[3], m[3];
        tri_normal(wtri + 9 * bi, nf);
        double cth = orient(nf, d, nn);
        int32_t mt = S->tri_mat[bi];
        double rs = S->mats[2 * mt], rd = S->mats[2 * mt + 1];
        int emit = gen < P->bounces && K > 0 && rd > 0.0;   /* R10 */
        if (emit) diffuse_fan(K, nn, fan, m);
        shade(scale, w, d, nn, cth, rs, rd, emit ? m : NULL, x, P->ref, dF, dT);
        for (int c = 0; c < 3; ++c) { ks_add(&acc[c], dF[c]); ks_add(&acc[3 + c], dT[c]); }
        if (emit) {
            double wd = w * rd / (double)K;
            for (int32_t k = 0; k < K; ++k) {
                const double *e = fan + 3 * k;
                double et;
                int64_t ei;
                po->sec++;
                po->dif++;
                closest_hit(B, wtri, S->nt, x, e, 1e-6 * g->L, bi, &et, &ei, po->tests);
                int32_t slot = P->bounces + 1 + gen * K + k;
                if (ei < 0) continue;
                if (ids) ids[slot] = (int32_t)ei;
                if (ts) ts[slot] = et;
                po->sec_hits++;
                po->dif_hits++;
                double y[3] = {x[0] + et * e[0], x[1] + et * e[1], x[2] + et * e[2]};
                double mf[3], mn[3], eF[3], eT[3];
                tri_normal(wtri + 9 * ei, mf);
                double ce = orient(mf, e, mn);
                int32_t me = S->tri_mat[ei];
                shade(scale, wd, e, mn, ce, S->mats[2 * me], S->mats[2 * me + 1], NULL, y, P->ref, eF, eT);
                for (int c = 0; c < 3; ++c) { ks_add(&acc[c], eF[c]); ks_add(&acc[3 + c], eT[c]); }
            }
        }
        if (gen == P->bounces || !(rs > 0.0)) break;
        /* R7: specular continuation */
        for (int c = 0; c < 3; ++c) { o[c] = x[c]; d[c] = d[c] + 2.0 * cth * nn[c]; }
        w *= rs;
        tmin = 1e-6 * g->L;
        exclude = bi;
        po->sec++;
    }
    for (int c = 0; c < 6; ++c) po->f[c] = ks_val(&acc[c]);
}

static void finish(const orc_scene *S, const orc_params *P, const orc_grid *g, const pix_out *po,
                   int64_t np, orc_result *out)
{
    ksum acc[6];
    memset(acc, 0, sizeof acc);
    memset(out, 0, sizeof *out);
    for (int64_t k = 0; k < np; ++k) {
        for (int c = 0; c < 6; ++c) ks_add(&acc[c], po[k].f[c]);
        out->n_hits += po[k].hits;
        out->n_secondary += po[k].sec;
        out->n_secondary_hits += po[k].sec_hits;
        out->n_diffuse += po[k].dif;
        out->n_diffuse_hits += po[k].dif_hits;
        out->n_box_tests += po[k].tests[0];
        out->n_tri_tests += po[k].tests[1];
    }
    for (int c = 0; c < 3; ++c) { out->force[c] = ks_val(&acc[c]); out->torque[c] = ks_val(&acc[3 + c]); }
    out->n_rays = np;
    out->grid = *g;
    (void)S; (void)P;
}

int orc_eval(const orc_scene *S, const double *angles, const orc_params *P, int32_t use_bvh,
             const int64_t *pixels, int64_t n_pixels, orc_result *out, int32_t *ids, double *ts)
{
    int rc = orc_validate(S);
    if (rc) return rc;
    if (!P || P->n < 1 || P->bounces < 0 || P->bounces > 8 || P->n_diffuse < 0 || !out) return ORC_ERR_ARG;
    double *wtri = (double *)malloc(sizeof(double) * 9 * (size_t)(S->nt + 1));
    if (!wtri) return ORC_ERR_OOM;
    orc_articulate(S, angles, wtri);
    orc_grid g;
    rc = grid_setup(S, wtri, P, &g);
    if (rc) { free(wtri); return rc; }
    int64_t np = pixels ? n_pixels : (int64_t)P->n * P->n;
    int32_t G = orc_record_slots(P);
    if (ids) for (int64_t k = 0; k < np * G; ++k) ids[k] = -1;
    if (ts) for (int64_t k = 0; k < np * G; ++k) ts[k] = 0.0;
    if (!(g.wu * g.wv > 0)) {               /* R3: empty window */
        memset(out, 0, sizeof *out);
        out->n_rays = np;
        out->grid = g;
        free(wtri);
        return ORC_OK;
    }
    bvh B;
    int have_bvh = 0;
    if (use_bvh) {
        rc = bvh_build(&B, wtri, S->nt, 1e-9 * (g.L + 1.0));
        if (rc) { free(wtri); return rc; }
        have_bvh = 1;
    }
    pix_out *po = (pix_out *)malloc(sizeof(pix_out) * (size_t)(np + 1));
    if (!po) { if (have_bvh) bvh_free(&B); free(wtri); return ORC_ERR_OOM; }
    int oom = 0;
#pragma omp parallel
    {
        double *fan = (double *)malloc(sizeof(double) * 3 * (size_t)(P->n_diffuse + 1));
        if (!fan) {
#pragma omp atomic write
            oom = 1;
        }
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < np; ++k) {
            if (!fan) continue;
            int64_t pix = pixels ? pixels[k] : k;
            trace_pixel(S, wtri, have_bvh ? &B : NULL, P, &g, pix, &po[k],
                        ids ? ids + k * G : NULL, ts ? ts + k * G : NULL, fan);
        }
        free(fan);
    }
    if (oom) { free(po); if (have_bvh) bvh_free(&B); free(wtri); return ORC_ERR_OOM; }
    finish(S, P, &g, po, np, out);
    free(po);
    if (have_bvh) bvh_free(&B);
    free(wtri);
    return ORC_OK;
}

int orc_grid_of(const orc_scene *S, const double *angles, const orc_params *P, orc_grid *g)
{
    int rc = orc_validate(S);
    if (rc) return rc;
    double *wtri = (double *)malloc(sizeof(double) * 9 * (size_t)(S->nt + 1));
    if (!wtri) return ORC_ERR_OOM;
    orc_articulate(S, angles, wtri);
    rc = grid_setup(S, wtri, P, g);
    free(wtri);
    return rc;
}

/* ------------------------------------------------------------ frozen visibility
 * Re-shades every ray chain for given hit ids (all generations and, with
 * diffuse rays, every fan's rays, in the orc_eval record layout) on a frozen
 * grid (window, pixel area, origins), after articulating with `angles` and
 * using the materials in S.  Hit points are the intersections of each chain's
 * rays with the planes of its frozen triangles.  At the angles the ids were
 * recorded with this reproduces orc_eval; perturbing angles or materials gives
 * the fixed-visibility variation whose derivative the adjoint computes.
 *
 * angles_ref (may be NULL): the angles the ids were recorded at.  With it,
 * the recorded state is held as the direction re-shade below holds it:
 *   - every hit keeps the face the recorded ray met (the normal's orientation
 *     is taken from the recorded chain, followed through the triangles at
 *     angles_ref), so the law varies smoothly even where a bounce meets its
 *     triangle near edge-on;
 *   - every primary ray keeps its share of its triangle's visible surface, so
 *     the projected area it carries scales with the primary cosine: the
 *     pixel's whole contribution is multiplied by c0(angles) / c0(angles_ref),
 *     c0 = -n0 . d with that orientation.
 * For a fully visible plate the variation is then the flat-plate law's own,
 * P A cos(theta) [...], including the cos(theta) prefactor.  Diffuse fan rays
 * are re-shaded as without it.  Without angles_ref the pixel area is held
 * (factor 1) and each hit faces the ray it is re-shaded with.
 */
int orc_shade_frozen(const orc_scene *S, const double *angles, const double *angles_ref, const orc_params *P,
                     const orc_grid *g, const int32_t *ids, orc_result *out)
{
    int rc = orc_validate(S);
    if (rc) return rc;
    if (!P || P->n < 1 || P->bounces < 0 || P->n_diffuse < 0 || !ids || !out) return ORC_ERR_ARG;
    double *wtri = (double *)malloc(sizeof(double) * 9 * (size_t)(S->nt + 1));
    if (!wtri) return ORC_ERR_OOM;
    orc_articulate(S, angles, wtri);
    double *wref = NULL;
    if (angles_ref) {
        wref = (double *)malloc(sizeof(double) * 9 * (size_t)(S->nt + 1));
        if (!wref) { free(wtri); return ORC_ERR_OOM; }
        orc_articulate(S, angles_ref, wref);
    }
    int64_t np = (int64_t)P->n * P->n;
    int32_t G = orc_record_slots(P), K = P->n_diffuse;
    pix_out *po = (pix_out *)malloc(sizeof(pix_out) * (size_t)(np + 1));
    if (!po) { free(wref); free(wtri); return ORC_ERR_OOM; }
    double scale = P->pressure * g->a_pix;
    int oom = 0;
#pragma omp parallel
    {
        double *fan = (double *)malloc(sizeof(double) * 3 * (size_t)(K + 1));
        if (!fan) {
#pragma omp atomic write
            oom = 1;
        }
#pragma omp for schedule(static)
        for (int64_t k = 0; k < np; ++k) {
            if (!fan) continue;
            int64_t i = k % P->n, j = k / P->n;
            double o[3], d[3] = {g->d[0], g->d[1], g->d[2]};
            pixel_origin(g, P->n, i, j, o);
            ksum acc[6];
            memset(acc, 0, sizeof acc);
            memset(&po[k], 0, sizeof po[k]);
            double w = 1.0;
            double dref[3] = {g->d[0], g->d[1], g->d[2]};   /* the recorded chain's direction */
            for (int32_t gen = 0; gen <= P->bounces; ++gen) {
                int32_t tri = ids[k * G + gen];
                if (tri < 0) break;
                const double *tv = wtri + 9 * (int64_t)tri;
                double nf[3], nn[3], dF[3], dT[3], r0[3], m[3];
                tri_normal(tv, nf);
                double cth;
                if (wref) {
                    /* the face the recorded ray met, and (primary) the surface share */
                    double nr[3], nro[3];
                    tri_normal(wref + 9 * (int64_t)tri, nr);
                    double cref = orient(nr, dref, nro);
                    double sgn = v_dot(nro, nr) > 0 ? 1.0 : -1.0;
                    for (int c = 0; c < 3; ++c) nn[c] = sgn * nf[c];
                    cth = -v_dot(nn, d);
                    if (gen == 0) w = cth / cref;
                    for (int c = 0; c < 3; ++c) dref[c] += 2.0 * cref * nro[c];
                } else {
                    cth = orient(nf, d, nn);
                }
                v_sub(tv, o, r0);
                double t = v_dot(r0, nf) / v_dot(d, nf);
                double x[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
                int32_t mt = S->tri_mat[tri];
                double rs = S->mats[2 * mt], rd = S->mats[2 * mt + 1];
                int emit = gen < P->bounces && K > 0 && rd > 0.0;
                if (emit) diffuse_fan(K, nn, fan, m);
                shade(scale, w, d, nn, cth, rs, rd, emit ? m : NULL, x, P->ref, dF, dT);
                for (int c = 0; c < 3; ++c) { ks_add(&acc[c], dF[c]); ks_add(&acc[3 + c], dT[c]); }
                if (gen == 0) po[k].hits++;
                else po[k].sec_hits++;
                if (emit) {
                    for (int32_t q = 0; q < K; ++q) {
                        int32_t et = ids[k * G + P->bounces + 1 + gen * K + q];
                        po[k].sec++;
                        po[k].dif++;
                        if (et < 0) continue;
                        const double *e = fan + 3 * q, *ev = wtri + 9 * (int64_t)et;
                        double mf[3], mn[3], eF[3], eT[3], r1[3];
                        tri_normal(ev, mf);
                        v_sub(ev, x, r1);
                        double te = v_dot(r1, mf) / v_dot(e, mf);
                        double y[3] = {x[0] + te * e[0], x[1] + te * e[1], x[2] + te * e[2]};
                        double ce = orient(mf, e, mn);
                        int32_t me = S->tri_mat[et];
                        shade(scale, w * rd / (double)K, e, mn, ce, S->mats[2 * me], S->mats[2 * me + 1], NULL,
                              y, P->ref, eF, eT);
                        for (int c = 0; c < 3; ++c) { ks_add(&acc[c], eF[c]); ks_add(&acc[3 + c], eT[c]); }
                        po[k].sec_hits++;
                        po[k].dif_hits++;
                    }
                }
                for (int c = 0; c < 3; ++c) { o[c] = x[c]; d[c] = d[c] + 2.0 * cth * nn[c]; }
                w *= rs;
            }
            for (int c = 0; c < 6; ++c) po[k].f[c] = ks_val(&acc[c]);
        }
        free(fan);
    }
    if (!oom) finish(S, P, g, po, np, out);
    free(po);
    free(wref);
    free(wtri);
    return oom ? ORC_ERR_OOM : ORC_OK;
}

/* ------------------------------------------------------------ frozen visibility, new direction
 * Force of the recorded chains (chain generations only, no diffuse fans) when
 * the photon direction becomes dnew (any 3-vector, not normalised): every
 * primary ray keeps its triangle and its share of that triangle's visible
 * area, whose projected size scales with c0 = -n0.d, so the chain's force is
 * multiplied by c0(dnew) / c0(g->d); the chain follows dnew through its
 * specular reflections on the frozen triangles (d' = d - 2 (n.d) n) with the
 * weights of the law.  The normal orientation is the one that faces the
 * recorded direction.  At dnew = g->d this reproduces orc_shade_frozen's
 * force.  Only the force is written (torque zero).
 */
int orc_shade_frozen_dir(const orc_scene *S, const double *angles, const orc_params *P, const orc_grid *g,
                         const int32_t *ids, const double *dnew, orc_result *out)
{
    int rc = orc_validate(S);
    if (rc) return rc;
    if (!P || P->n < 1 || P->bounces < 0 || P->n_diffuse != 0 || !ids || !dnew || !out) return ORC_ERR_ARG;
    double *wtri = (double *)malloc(sizeof(double) * 9 * (size_t)(S->nt + 1));
    if (!wtri) return ORC_ERR_OOM;
    orc_articulate(S, angles, wtri);
    int64_t np = (int64_t)P->n * P->n;
    int32_t G = P->bounces + 1;
    pix_out *po = (pix_out *)malloc(sizeof(pix_out) * (size_t)(np + 1));
    if (!po) { free(wtri); return ORC_ERR_OOM; }
    double scale = P->pressure * g->a_pix;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < np; ++k) {
        ksum acc[3];
        memset(acc, 0, sizeof acc);
        memset(&po[k], 0, sizeof po[k]);
        double dref[3] = {g->d[0], g->d[1], g->d[2]}, d[3] = {dnew[0], dnew[1], dnew[2]};
        double w = 1.0, area = 1.0;
        for (int32_t gen = 0; gen < G; ++gen) {
            int32_t tri = ids[k * G + gen];
            if (tri < 0) break;
            double nf[3], n[3], nr[3], dF[3], dT[3], x[3] = {0, 0, 0}, zero[3] = {0, 0, 0};
            tri_normal(wtri + 9 * (int64_t)tri, nf);
            double cref = orient(nf, dref, nr);       /* orientation from the recorded ray */
            for (int c = 0; c < 3; ++c) n[c] = nr[c];
            double cth = -v_dot(n, d);
            if (gen == 0) area = cth / cref;
            int32_t m = S->tri_mat[tri];
            double rs = S->mats[2 * m], rd = S->mats[2 * m + 1];
            shade(scale, w * area, d, n, cth, rs, rd, NULL, x, zero, dF, dT);
            for (int c = 0; c < 3; ++c) ks_add(&acc[c], dF[c]);
            if (gen == 0) po[k].hits++;
            for (int c = 0; c < 3; ++c) {
                d[c] = d[c] + 2.0 * cth * n[c];
                dref[c] = dref[c] + 2.0 * cref * n[c];
            }
            w *= rs;
        }
        for (int c = 0; c < 3; ++c) po[k].f[c] = ks_val(&acc[c]);
    }
    finish(S, P, g, po, np, out);
    for (int c = 0; c < 3; ++c) out->torque[c] = 0.0;
    free(po);
    free(wtri);
    return ORC_OK;
}
