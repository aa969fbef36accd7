/*
 * FP64 CPU oracle for ray-traced SRP — TEST INFRASTRUCTURE ONLY.
 * Declarations for oracle.c; see that file for the method and the readings.
 */
#ifndef SRP_ORACLE_H
#define SRP_ORACLE_H
#include <stdint.h>

#define ORC_OK 0
#define ORC_ERR_ARG -1
#define ORC_ERR_OOM -2

typedef struct {
    int64_t nv;
    const double *verts;      /* nv x 3, rest pose, body frame */
    int64_t nt;
    const int32_t *tris;      /* nt x 3 */
    const int32_t *tri_mat;   /* nt */
    const int32_t *tri_node;  /* nt */
    int32_t nm;
    const double *mats;       /* nm x 2: rho_s, rho_d */
    int32_t nn;
    const int32_t *parent;    /* nn; parent[0] = -1, parent[k] < k */
    const double *pivot;      /* nn x 3 */
    const int32_t *n_axes;    /* nn, 0..3 (root 0) */
    const double *axes;       /* nn x 3 x 3 */
    const double *lo;         /* nn x 3, radians */
    const double *hi;         /* nn x 3 */
} orc_scene;

typedef struct {
    double sun_dir[3];        /* spacecraft -> Sun, any nonzero length */
    double pressure;          /* N/m^2 */
    int32_t n;                /* N x N rays */
    int32_t bounces;          /* secondary generations */
    double ref[3];            /* torque reference point */
    int32_t n_diffuse;        /* diffuse rays per emitting hit (R10), 0 = none */
    int32_t pad_;
} orc_params;

typedef struct {
    double u[3], v[3], d[3];  /* image-plane basis and photon direction */
    double umin, umax, vmin, vmax, hmin;
    double wu, wv, L, a_pix, h0;
} orc_grid;

typedef struct {
    double force[3], torque[3];
    int64_t n_rays, n_hits, n_secondary, n_secondary_hits;
    int64_t n_diffuse, n_diffuse_hits;   /* the diffuse part of the secondary counts */
    int64_t n_box_tests, n_tri_tests;    /* work of the evaluation (orc_eval only): box and triangle tests */
    orc_grid grid;
} orc_result;

int32_t orc_threads(void);
int orc_validate(const orc_scene *S);
int32_t orc_n_dof(const orc_scene *S);
int orc_node_transforms(const orc_scene *S, const double *angles, double *xf /* nn x 12 */);
int orc_articulate(const orc_scene *S, const double *angles, double *wtri /* nt x 9 */);
int orc_grid_of(const orc_scene *S, const double *angles, const orc_params *P, orc_grid *g);
int orc_eval(const orc_scene *S, const double *angles, const orc_params *P, int32_t use_bvh,
             const int64_t *pixels, int64_t n_pixels, orc_result *out,
             int32_t *ids /* n_pix x R or NULL */, double *ts /* same or NULL */);
int orc_shade_frozen(const orc_scene *S, const double *angles, const double *angles_ref /* or NULL */,
                     const orc_params *P, const orc_grid *g, const int32_t *ids /* N*N x R */,
                     orc_result *out);
int orc_shade_frozen_dir(const orc_scene *S, const double *angles, const orc_params *P,
                         const orc_grid *g, const int32_t *ids /* N*N x (B+1) */, const double *dnew,
                         orc_result *out);
/* R = record slots per pixel: B + 1 chain generations, then B fans of K
 * diffuse rays (fan of generation g at slot B + 1 + g K). */
int32_t orc_record_slots(const orc_params *P);
/* Diffuse set (R10): the K local directions, K x 3. */
int orc_diffuse_set(int32_t K, double *l);
#endif
