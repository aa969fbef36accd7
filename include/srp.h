/*
 * srp.h — C ABI of the MI355X (gfx950) ray-traced solar-radiation-pressure
 * library.
 *
 * The library evaluates the SRP force and torque on a triangulated,
 * articulated spacecraft by casting a uniform grid of parallel sun-direction
 * rays over the mesh's projected footprint (one independent ray per pixel of
 * a discretised image plane, Sec. 4.3 of the paper), finding each ray's first
 * hit (self-shadowing, Sec. 1), applying the absorbed / specular / diffuse
 * momentum-transfer law of the hit facet's material, following specular
 * secondary rays iteratively (Sec. 4.3), and reducing everything on the GPU to
 * a total force and torque (GPU-side reduction, Sec. 4.3 and Sec. 8.2).
 * Articulated solar panels follow the paper's rooted kinematic tree
 * G = (N, E, L) with edge labels (pivot, axes, intervals) (Sec. 4.4.1) and the
 * clamp-to-interval rule of the panel update (Sec. 4.4.2).
 *
 * Conventions for every entry point:
 *   - Return value: SRP_OK (0) or a negative SRP_ERR_* code; srp_last_error()
 *     then gives a thread-local, human-readable message.  On error no output
 *     is written except where stated.
 *   - Units: metres, radians, N/m^2 for pressure; forces in N, torques in N m.
 *   - Frames: everything is in the spacecraft body frame (rest pose for the
 *     mesh and the tree).
 *   - Ownership: inputs are copied during the call; the caller keeps its
 *     buffers.  Opaque handles are owned by the library until destroyed.
 *   - Device: the library uses the HIP device current at srp_build_scene;
 *     a scene's calls are ordered on the stream given (or the null stream).
 *     Calls on one scene must not overlap from several host threads.
 *   - Precision: rays, traversal and intersection in FP32; force and torque
 *     contributions are summed in FP64.  The adjoint's per-hit gradient
 *     terms are first summed over a wavefront in FP32 (at most 64 terms per
 *     sum) and then accumulated in FP64 across hits and patches.
 */
#ifndef SRP_MI355X_H
#define SRP_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SRP_OK 0
#define SRP_ERR_ARG -1     /* invalid argument (null pointer, range, topology, shape) */
#define SRP_ERR_OOM -2     /* host or device allocation failed */
#define SRP_ERR_DEVICE -3  /* a HIP runtime call failed; message has its text */
#define SRP_ERR_DEPTH -4   /* a hierarchy deeper than the traversal stack */

/* srp_eval_params.flags */
#define SRP_F_COUNT 1u     /* also count box and triangle tests (slower kernel variant) */
#define SRP_F_GRAD_DIR 2u  /* gradient calls: also dF/dd (photon direction); without it those
                              9 outputs are 0.  srp_eval_grad sets it when dF_ddir is non-NULL */

#define SRP_MAX_N 8192     /* largest ray grid side */
#define SRP_MAX_BOUNCES 4  /* largest number of secondary generations */
#define SRP_MAX_DIFFUSE 64 /* largest number of diffuse rays per emitting hit */
#define SRP_MAX_NODES 128  /* largest number of tree nodes */
#define SRP_MAX_MATS 64    /* largest number of materials */

typedef struct srp_scene srp_scene;

/* Optical coefficients of one material: rho_s specular, rho_d diffuse,
 * rho_a = 1 - rho_s - rho_d absorbed (Sec. 5.1 table of spacecraft models).
 * Valid when rho_s >= 0, rho_d >= 0, rho_s + rho_d <= 1. */
typedef struct {
    double rho_s, rho_d;
} srp_material;

/* One node of the kinematic tree (Sec. 4.4.1): a rigid group of mesh parts.
 * Node 0 is the root (parent = -1, n_axes = 0); every other node's parent has
 * a smaller index.  The edge from the parent carries the label (p, A, I):
 * pivot p, unit axes axis[0..n_axes-1] and intervals [lo, hi] (radians), all in
 * the rest-pose body frame.  The node's world transform is
 *   M = M_parent * T(p) * R(axis[0], th0) * ... * R(axis[k-1], th_{k-1}) * T(-p). */
typedef struct {
    int32_t parent;
    int32_t is_panel;      /* 1 if the node is a solar panel (Sec. 4.4.1 flag t_n) */
    double pivot[3];
    int32_t n_axes;        /* 0..3 */
    int32_t reserved;
    double axis[3][3];
    double lo[3], hi[3];
} srp_node;

/* Per-evaluation parameters. */
typedef struct {
    double sun_dir[3];     /* spacecraft -> Sun, body frame; finite, nonzero, any length */
    double pressure;       /* N/m^2 at the spacecraft (caller scales P0 (AU/r)^2) */
    int32_t n;             /* ray grid N (N x N rays), 1..SRP_MAX_N */
    int32_t bounces;       /* specular secondary generations B, 0..SRP_MAX_BOUNCES */
    double ref[3];         /* torque reference point, body frame */
    uint32_t flags;        /* SRP_F_* */
    /* Diffuse rays K per emitting hit, 0..SRP_MAX_DIFFUSE (Sec. 4.3: the
     * secondary rays made at each interaction set the level of scattering;
     * Sec. 6.1 uses 16).  0: diffuse re-emission is the law's Lambertian
     * recoil only.  K > 0: a chain hit of generation g < B on a material
     * with rho_d > 0 also emits K rays of weight w rho_d / K along a fixed
     * cosine-weighted set (u = (k + 1/2)/K, phi = 2 pi frac(k (sqrt5 - 1)/2),
     * local (sqrt(u) cos phi, sqrt(u) sin phi, sqrt(1 - u)) in the frame
     * t = normalize((1,2,3) x n), b = n x t); its recoil is the set's mean
     * direction; each diffuse ray deposits at its first hit (flat-plate
     * law) and spawns nothing.  Diffuse rays count as secondary rays. */
    int32_t n_diffuse;
} srp_eval_params;

/* Result of one evaluation.  n_box_tests / n_tri_tests are filled only with
 * SRP_F_COUNT (else 0). */
typedef struct {
    double force[3];
    double torque[3];
    int64_t n_rays;            /* primary rays cast (N^2) */
    int64_t n_hits;            /* primary rays that hit */
    int64_t n_secondary;       /* secondary rays spawned */
    int64_t n_secondary_hits;  /* secondary rays that hit */
    int64_t n_box_tests;       /* ray-box tests (SRP_F_COUNT) */
    int64_t n_tri_tests;       /* ray-triangle tests (SRP_F_COUNT) */
    uint32_t status;           /* 0, or SRP_STATUS_* bits (the evaluation is then invalid) */
    uint32_t n_clamped;        /* hinge angles of this evaluation that lay outside their
                                  intervals and were clamped (Sec. 4.4.2; the item's angles,
                                  or the scene's current ones as srp_set_panel_angles
                                  counted them); not an error */
} srp_result;

/* srp_result.status bits */
#define SRP_STATUS_STACK 1u   /* a traversal stack overflowed (cannot happen for scenes
                                 accepted by srp_build_scene; reported, never silent) */

/* One item of a batch.  Items may use different scenes, grid sizes, bounce
 * counts and angles. */
typedef struct {
    srp_scene *scene;
    const double *angles;  /* host, scene's n_dof values; NULL = scene's current angles */
    srp_eval_params p;
} srp_batch_item;

/* Build a scene: mesh (rest pose), per-triangle material and node, material
 * table and kinematic tree (Sec. 4.4.1; the triangles of a node form its mesh
 * parts O_n and every triangle belongs to exactly one node).
 *   verts:  n_verts x 3 (double);  tris: n_tris x 3 vertex indices;
 *   tri_material, tri_node: n_tris each;  mats: n_mats;  nodes: n_nodes.
 * Builds one bounding-volume hierarchy per node in rest-pose coordinates and
 * uploads everything to the current device; all angles start at 0 (clamped).
 * Errors: SRP_ERR_ARG for null pointers, out-of-range indices, invalid
 * coefficients, a tree whose parent indices are not increasing from a single
 * root, n_axes outside 0..3 or a root with axes, n_nodes > SRP_MAX_NODES,
 * n_mats > SRP_MAX_MATS, non-finite coordinates; SRP_ERR_OOM; SRP_ERR_DEPTH if
 * a hierarchy cannot be kept within the traversal stack; SRP_ERR_DEVICE.
 * *out is set only on success. */
int srp_build_scene(const double *verts, int64_t n_verts, const int32_t *tris, int64_t n_tris,
                    const int32_t *tri_material, const int32_t *tri_node,
                    const srp_material *mats, int32_t n_mats,
                    const srp_node *nodes, int32_t n_nodes, srp_scene **out);

/* Release a scene and its device memory (waits for its pending work).
 * NULL is accepted and ignored. */
int srp_destroy_scene(srp_scene *scene);

/* Number of hinge degrees of freedom (sum of n_axes), or a negative error. */
int32_t srp_scene_n_dof(const srp_scene *scene);

/* Replace the material table (same count).  Cheap; for coefficient fitting. */
int srp_set_materials(srp_scene *scene, const srp_material *mats, int32_t n_mats);

/* Set the hinge angles (Sec. 4.4.2): angles[n_dof] in node order, then axis
 * order; each is clamped to its interval (not an error).  Only the per-node
 * instance transforms and the boxes of the top-level hierarchy over the nodes
 * change (its topology is built once, over the rest pose, and refitted); the
 * per-node hierarchies are untouched.  Returns the number of clamped
 * angles (>= 0) on success.  Errors: SRP_ERR_ARG (null, n_dof mismatch,
 * non-finite angle). */
int srp_set_panel_angles(srp_scene *scene, const double *angles, int32_t n_dof);

/* One evaluation at the scene's current angles; blocks until the result is
 * on the host.  Optional per-ray records (host buffers, may be NULL):
 *   hit_ids: N*N*R int32 with R = (B+1) + B*K rays per pixel, pixel
 *            p = j*N + i (row j, column i) major; within a pixel the chain's
 *            generations 0..B, then generation g's fan of K diffuse rays at
 *            B+1+g*K..; the original triangle index, or -1 for a miss or a
 *            ray not traced;
 *   hit_t:   same layout, ray parameter of the hit (0 where none).
 * Errors: SRP_ERR_ARG (null scene/params/out, N, B or K out of range,
 * non-finite or zero sun_dir, non-finite pressure/ref), SRP_ERR_OOM (record
 * buffer), SRP_ERR_DEVICE. */
int srp_eval(srp_scene *scene, const srp_eval_params *params, srp_result *out,
             int32_t *hit_ids, float *hit_t);

/* A batch of evaluations in one persistent launch (plus a window pass and a
 * fixed-order reduction).  out_dev: device array of n_items srp_result,
 * written in stream order on hip_stream (a hipStream_t; NULL = null stream).
 * The call returns once the work is queued; host inputs may be reused then.
 * Items with angles get one articulation slot per distinct angle vector
 * (equal bits), built on the device from the cosine and sine of each clamped
 * angle: the same bits as srp_set_panel_angles gives for those angles, so an
 * item's result equals the single evaluation after srp_set_panel_angles.
 * A batch whose device workspace (about 64 bytes per 8x8-pixel patch, plus
 * gradient partials) would exceed 16 GiB runs as consecutive sub-batches; the
 * call may then block while earlier sub-batches run.  Results are bitwise
 * independent of scheduling and of that split.  Errors as srp_eval, checked
 * for every item before anything is queued. */
int srp_eval_batch(const srp_batch_item *items, int64_t n_items, srp_result *out_dev,
                   void *hip_stream);

/* One evaluation plus the gradient of the force at fixed visibility (hit
 * triangles of every generation, the face of each that the ray met, window
 * and ray origins frozen; every primary ray keeps its triangle and its share
 * of that triangle's visible surface, whose projected area scales with
 * c0 = -n0.d of the primary hit):
 *   dF_drho_s: n_mats x 3, dF_drho_d: n_mats x 3, dF_dtheta: n_dof x 3,
 *   dF_ddir: 3 x 3, dF_i/dd_j (row-major) with respect to the photon
 *   direction d = -sun_dir/|sun_dir| (host).
 * dF_dtheta is with respect to the clamped angles; a turned primary
 * triangle changes its rays' projected area with c0 (for a fully visible
 * plate the result is the derivative of the flat-plate law
 * P A cos(theta) [...]), and the specular chain follows the turned normals.
 * dF_ddir is computed when the pointer is non-NULL (SRP_F_GRAD_DIR); the
 * specular chain follows d through its reflections.  d is varied as a free 3-vector; a
 * rotation of the Sun direction or of the attitude takes the component
 * orthogonal to d.  Any gradient pointer may be NULL.  Blocks until the
 * results are on the host.  Errors as srp_eval; SRP_ERR_ARG for
 * n_diffuse > 0 (the adjoint covers the specular chain only) and for a scene
 * with 9*nodes + 6*materials + 9 > 960. */
int srp_eval_grad(srp_scene *scene, const srp_eval_params *params, srp_result *out,
                  double *dF_drho_s, double *dF_drho_d, double *dF_dtheta, double *dF_ddir);

/* srp_eval_batch for callers that cannot allocate memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * kernels and the same results, bitwise, but the call makes no device or
 * pinned-host allocation (no hipMalloc, hipHostMalloc, hipFree).  Its device
 * workspace is a fixed array of SRP_NOALLOC_SCRATCH_BYTES per GPU, held by
 * every GPU the library runs on until the process ends; its host staging
 * image is a fixed buffer of SRP_NOALLOC_STAGE_BYTES.  A batch whose
 * workspace does not fit (after reducing the persistent grid) or whose
 * staging image exceeds the buffer is rejected with SRP_ERR_ARG and a
 * message giving both sizes; it is never split.  Every call on one GPU uses
 * that GPU's array: calls ordered on one stream are safe, calls that overlap
 * on one GPU (other streams, other threads' streams) race and give wrong
 * results.  The array keeps the last call's contents; the launch sequence
 * rewrites everything it reads (counters are zeroed by its first kernel).
 * Items, out_dev and errors as srp_eval_batch; stream-ordered on hip_stream. */
#define SRP_NOALLOC_SCRATCH_BYTES (64ll << 20)
#define SRP_NOALLOC_STAGE_BYTES (4ll << 20)
int srp_eval_batch_noalloc(const srp_batch_item *items, int64_t n_items, srp_result *out_dev, void *hip_stream);

/* Batched form of srp_eval_grad.  grad_dev: device array, item k's gradients
 * at grad_dev + k*grad_stride doubles, laid out as rho_s (M x 3), rho_d
 * (M x 3), theta (J x 3), dF/dd (3 x 3, zeros unless the item's flags hold
 * SRP_F_GRAD_DIR) with that item's M and J;
 * grad_stride must be at least 3*(2M+J) + 9 for every item.  Stream-ordered
 * like srp_eval_batch. */
int srp_eval_grad_batch(const srp_batch_item *items, int64_t n_items, srp_result *out_dev,
                        double *grad_dev, int64_t grad_stride, void *hip_stream);

/* ---- captured launches, schedules and the autotuner ---- */

#define SRP_PLAN_GRAD 1   /* plan / autotune flag: forward + fixed-visibility adjoint */

/* A plan captures one batch launch (staging upload, window pass, persistent
 * trace, reduction) in a HIP graph for repeated replays, e.g. the chunks of a
 * precomputed table or the stages of many propagations.  The items fix the
 * layout: scenes, grid sizes, bounce counts, flags and the number of distinct
 * angle vectors; srp_plan_update may change Sun directions, pressures,
 * references and angle values (a changed layout is recaptured).  out_dev
 * (n_items srp_result) and, with SRP_PLAN_GRAD, grad_dev (as
 * srp_eval_grad_batch) are device buffers that must outlive the plan.  Items
 * with NULL angles read the scene's current angles at launch time: do not
 * change them while a launch is in flight.  Errors as srp_eval_batch,
 * SRP_ERR_DEVICE for graph capture failures. */
typedef struct srp_plan srp_plan;
int srp_plan_create(const srp_batch_item *items, int64_t n_items, int32_t flags, srp_result *out_dev,
                    double *grad_dev, int64_t grad_stride, srp_plan **out);
int srp_plan_update(srp_plan *plan, const srp_batch_item *items, int64_t n_items);
int srp_plan_launch(srp_plan *plan, void *hip_stream);   /* stream-ordered; returns once queued */
int srp_plan_destroy(srp_plan *plan);

/* Launch schedule of batched evaluations: 8x8-pixel patches per work chunk
 * (1..64; a chunk is one wave's work item) and resident blocks per compute
 * unit of the persistent grid (1..64, capped at the kernel's occupancy);
 * 0 = automatic (autotuned value for the batch's size class if any, else a
 * heuristic).  Forces and torques do not depend on the schedule (every patch
 * keeps its own partial sum).  The adjoint's chunks are fixed groups of an
 * evaluation's patches (8 to 64, the smallest power of two whose gradient
 * partials for that evaluation fit 8 MiB), so it takes only the blocks per
 * CU from the schedule and its gradients do not depend on the schedule
 * either.  Errors: SRP_ERR_ARG (out of range). */
int srp_set_schedule(int32_t patches_per_chunk, int32_t blocks_per_cu);

/* Times the batch under candidate schedules (patches per chunk 1..64 in powers
 * of two, full and half occupancy; with SRP_PLAN_GRAD the occupancy only, the
 * adjoint's chunks being its evaluations' fixed patch groups; the best of four
 * timed runs after a warm-up each) and keeps the fastest for batches of the
 * same size class (total primary rays to a power of two, bounce count,
 * gradient flag).  Outputs the choice and its time (ms); any output pointer
 * may be NULL.  Blocks.  Errors as srp_eval_batch. */
int srp_autotune(const srp_batch_item *items, int64_t n_items, int32_t flags, int32_t *patches_per_chunk,
                 int32_t *blocks_per_cu, double *best_ms);

/* ---- orbit propagation (Sec. 3) and panel sun tracking (Sec. 4.4.2) ---- */

/* Sun tracking of the wing roots (panel nodes whose parent is not a panel),
 * the panel-update steps 2-4: for each of the node's axes, outer to inner,
 * the angle that turns the node's rest-pose area-weighted normal as close as
 * possible to the Sun direction (either face, the smaller rotation), clamped
 * to the interval.  Other angles are returned unchanged.  angles: in/out, n_dof
 * values.  Host only.  Errors: SRP_ERR_ARG (null, n_dof mismatch, zero or
 * non-finite sun_dir). */
int srp_sun_tracking_angles(const srp_scene *scene, const double *sun_dir, double *angles, int32_t n_dof);

/* Acceleration callback for srp_rk4: a(t, r, v) into a[3]; returns 0 or a
 * negative error code that aborts the integration. */
typedef int (*srp_accel_fn)(double t, const double *r, const double *v, double *a, void *user);

/* Classical fixed-step fourth-order Runge-Kutta for y = [r; v],
 * y' = [v; a(t, r, v)] (Sec. 3 equations of motion).  traj: caller-owned,
 * (n_steps + 1) x 7 doubles per row (t, r, v), row 0 = the initial state.
 * Host only.  Errors: SRP_ERR_ARG, or the callback's code. */
int srp_rk4(const double *y0, double t0, double h, int64_t n_steps, srp_accel_fn accel, void *user,
            double *traj);

/* Step control of srp_rk78. */
typedef struct {
    double h0;          /* fixed step, or the first trial step (s), > 0 */
    int32_t adaptive;   /* 0: fixed steps t0 + k*h0, the last one ending at t1; 1: adaptive */
    int32_t reserved;
    double rtol;        /* adaptive: relative tolerance, >= 0 */
    double atol[6];     /* adaptive: absolute tolerances of x, y, z (m), vx, vy, vz (m/s), >= 0 */
    double h_min;       /* adaptive: error when a rejected step would shrink below this (s), >= 0 */
    double h_max;       /* adaptive: largest step (s); 0 = no limit */
} srp_rk78_opts;

/* Explicit Runge-Kutta 7(8) (the paper's RK78, Sec. 3; Fehlberg's 13-stage
 * embedded pair) for y = [r; v], y' = [v; a(t, r, v)] from t0 to t1 > t0,
 * advancing the 8th-order solution.  Adaptive steps are accepted when
 * max_i |err_i| / (atol_i + rtol max(|y_i|, |y_new_i|)) <= 1 (err = the
 * embedded 7th-order error estimate; a component with zero error counts 0)
 * and every trial step is the previous one
 * times 0.9 err^(-1/8) within [0.2, 5] (capped at h_max), shortened to end at
 * t1.  traj: caller-owned, max_rows x 7 doubles (t, r, v), row 0 = t0; the
 * accepted steps follow.  *n_rows = rows written; *n_evals (may be NULL) =
 * derivative evaluations (13 per trial step).  Host only.  Errors:
 * SRP_ERR_ARG (invalid argument, more than max_rows rows, a step below h_min,
 * a non-finite state), or the callback's code. */
int srp_rk78(const double *y0, double t0, double t1, const srp_rk78_opts *opts, srp_accel_fn accel,
             void *user, double *traj, int64_t max_rows, int64_t *n_rows, int64_t *n_evals);

typedef struct {
    double mu;          /* gravitational parameter of the central body (Sun), m^3/s^2 */
    double mass;        /* spacecraft mass, kg */
    double p_ref;       /* radiation pressure at distance r_ref, N/m^2 */
    double r_ref;       /* m */
    int32_t n;          /* SRP ray grid N */
    int32_t bounces;    /* SRP secondary generations */
    int32_t track_sun;  /* 1: wing roots track the Sun (srp_sun_tracking_angles) every stage */
    int32_t n_diffuse;  /* SRP diffuse rays per emitting hit (srp_eval_params.n_diffuse) */
    double ref[3];      /* torque reference point */
} srp_orbit_params;

typedef struct {
    int64_t n_evals;      /* SRP evaluations (4 per step) */
    double srp_seconds;   /* host wall time spent in them */
} srp_prop_stats;

/* Heliocentric two-body + ray-traced SRP propagation with RK4 (one SRP
 * evaluation per stage, Sec. 3): the Sun is at the origin, the attitude is
 * inertially fixed (body frame = inertial frame, Sec. 5.1), the Sun direction
 * of a stage is -r/|r| and its pressure p_ref (r_ref/|r|)^2; a = -mu r/|r|^3 +
 * F/mass.  angles0: initial hinge angles (NULL = zeros); y0: r (m), v (m/s);
 * traj as srp_rk4.  Leaves the scene at the last stage's angles.  Errors as
 * srp_eval, SRP_ERR_ARG for invalid orbit parameters. */
int srp_propagate(srp_scene *scene, const srp_orbit_params *op, const double *angles0, const double *y0,
                  double t0, double h, int64_t n_steps, double *traj, srp_prop_stats *stats);

/* ---- SPAD tables (Sec. 2 and Sec. 4.2: SRP precomputed over attitudes and
 * interpolated during propagation; Sec. 6.1: 20 azimuth x 10 elevation grids
 * from -180 / -90 deg, and a copy shifted by 5 deg) ---- */

/* Grid of Sun directions in the body frame: az_j = az0 + j*daz (j < n_az),
 * el_i = el0 + i*del (i < n_el), radians; node (i, j) is the direction
 * s = (cos el cos az, cos el sin az, sin el).  Azimuth wraps around when
 * n_az*daz is a full turn (within 1e-9 rad). */
typedef struct {
    int32_t n_az, n_el;   /* 1..2^24 nodes in total */
    double az0, el0;      /* first azimuth and elevation, finite */
    double daz, del;      /* spacings, > 0 */
} srp_spad_grid;

/* Builds a table: force and torque at every node direction with the scene at
 * `angles` (host, n_dof values; NULL = the scene's current angles) and the
 * params' n, bounces, n_diffuse, pressure, ref and flags (its sun_dir is
 * ignored), in one batched launch.  table: host, n_el x n_az x 6 doubles
 * (force, torque), elevation-major; caller-owned.  Blocks.  Errors: as
 * srp_eval_batch, SRP_ERR_ARG for an invalid grid, SRP_ERR_OOM,
 * SRP_ERR_DEPTH. */
int srp_spad_build(srp_scene *scene, const srp_eval_params *params, const double *angles,
                   const srp_spad_grid *grid, double *table);

/* Bilinear interpolation of a table at Sun direction sun_dir (body frame, any
 * nonzero length): azimuth atan2(s_y, s_x), elevation atan2(s_z, hypot(s_x,
 * s_y)); between the four surrounding nodes; azimuth held at the first / last
 * column unless the grid wraps; elevations beyond the first / last row take
 * that row.  out: 6 doubles (force, torque).  Host only.  Errors:
 * SRP_ERR_ARG (null, invalid grid, zero or non-finite sun_dir). */
int srp_spad_interp(const srp_spad_grid *grid, const double *table, const double *sun_dir, double *out);

/* Propagation as srp_propagate with the SRP force interpolated from a table
 * built at pressure p_table, scaled to the stage's pressure
 * p_ref (r_ref/|r|)^2: F = interp(-r/|r|) p / p_table.  Uses mu, mass, p_ref and
 * r_ref of op (track_sun must be 0: the table has fixed hinge angles).  traj as
 * srp_rk4.  Host only.  Errors: SRP_ERR_ARG. */
int srp_propagate_spad(const srp_spad_grid *grid, const double *table, double p_table,
                       const srp_orbit_params *op, const double *y0, double t0, double h,
                       int64_t n_steps, double *traj);

/* srp_propagate with srp_rk78 from t0 to t1 (13 SRP evaluations per trial
 * step; sun tracking per stage when op->track_sun).  traj, max_rows and
 * n_rows as srp_rk78.  Errors as srp_propagate and srp_rk78. */
int srp_propagate_rk78(srp_scene *scene, const srp_orbit_params *op, const double *angles0, const double *y0,
                       double t0, double t1, const srp_rk78_opts *opts, double *traj, int64_t max_rows,
                       int64_t *n_rows, srp_prop_stats *stats);

/* srp_propagate_spad with srp_rk78.  Errors as srp_propagate_spad and srp_rk78. */
int srp_propagate_spad_rk78(const srp_spad_grid *grid, const double *table, double p_table,
                            const srp_orbit_params *op, const double *y0, double t0, double t1,
                            const srp_rk78_opts *opts, double *traj, int64_t max_rows, int64_t *n_rows);

/* ---- N-plate model: the analytical model of Sec. 1, one of the strategies
 * compared in Sec. 6.1 and 7.1 ----
 *
 * The spacecraft as flat plates, each lit on the side its normal points to
 * (or on either side when two-sided), with no shadowing and no secondary
 * rays.  Per lit plate, with s the unit Sun direction, d = -s the photon
 * direction, n the plate normal turned towards the Sun and c = n . s > 0:
 *   F = P A c [(1 - rho_s) d - 2 (rho_s c + rho_d / 3) n],
 *   tau = (center - ref) x F.
 * Body frame throughout. */
typedef struct {
    double normal[3];  /* unit; a one-sided plate is lit only when normal . s > 0 */
    double center[3];  /* area-weighted centroid (torque lever) */
    double area;       /* m^2, > 0 */
    double rho_s, rho_d;
    int32_t two_sided; /* 1: lit from either side */
    int32_t reserved;
} srp_plate;

/* The plates of a scene at `angles` (NULL = its current angles; clamped as in
 * srp_set_panel_angles): the articulated triangles grouped by node, material
 * and normal direction (normals equal to 1e-6 per component share a plate;
 * the grouping is made once, by srp_build_scene, in each node's frame, and
 * the plates move rigidly with their nodes);
 * the triangle winding gives the normal; plates of panel nodes are
 * two-sided (single-layer panels), the others one-sided (closed bodies wound
 * outward).  Zero-area triangles are skipped.  plates: caller-owned,
 * max_plates entries; *n_plates = plates needed (written also when
 * max_plates is too small, with SRP_ERR_ARG).  Host only. */
int srp_nplate_from_scene(srp_scene *scene, const double *angles, srp_plate *plates, int32_t max_plates,
                          int32_t *n_plates);

/* The same plates straight from the arrays srp_build_scene takes (same
 * meaning, layout and validation), at `angles` (NULL = all zero; clamped),
 * without building a scene: for callers that want the N-plate model of a
 * mesh, also on a machine without a GPU.  plates, max_plates and *n_plates as
 * srp_nplate_from_scene.  Host only.  Errors: those of srp_build_scene's
 * validation (SRP_ERR_ARG, SRP_ERR_DEPTH), SRP_ERR_OOM, SRP_ERR_ARG for
 * max_plates. */
int srp_nplate_from_mesh(const double *verts, int64_t n_verts, const int32_t *tris, int64_t n_tris,
                         const int32_t *tri_material, const int32_t *tri_node, const srp_material *mats,
                         int32_t n_mats, const srp_node *nodes, int32_t n_nodes, const double *angles,
                         srp_plate *plates, int32_t max_plates, int32_t *n_plates);

/* N-plate force and torque for Sun direction sun_dir (body frame, need not
 * be unit) at pressure P (N/m^2) about ref.  force, torque: 3 doubles each.
 * Host only.  Errors: SRP_ERR_ARG (null pointer, n_plates < 0, a zero or
 * non-finite sun_dir, a plate with a non-unit normal, a non-positive area or
 * reflectivities outside [0, 1]). */
int srp_nplate_eval(const srp_plate *plates, int32_t n_plates, const double *sun_dir, double pressure,
                    const double *ref, double *force, double *torque);

/* Two-body + N-plate SRP propagation with the attitude fixed (the body frame
 * is the inertial frame, the Sun direction at r is -r / |r|, the pressure
 * op->p_ref (op->r_ref / |r|)^2; op->n, bounces, n_diffuse and ref unused;
 * track_sun must be 0): srp_rk4 with step h (traj as srp_rk4), or srp_rk78
 * from t0 to t1 (traj, max_rows, n_rows as srp_rk78).  Host only.  Errors:
 * SRP_ERR_ARG, or those of the integrator. */
int srp_propagate_nplate(const srp_plate *plates, int32_t n_plates, const srp_orbit_params *op, const double *y0,
                         double t0, double h, int64_t n_steps, double *traj);
int srp_propagate_nplate_rk78(const srp_plate *plates, int32_t n_plates, const srp_orbit_params *op,
                              const double *y0, double t0, double t1, const srp_rk78_opts *opts, double *traj,
                              int64_t max_rows, int64_t *n_rows);

/* Measurement hook (not part of an evaluation): srp_profile(1) starts timing
 * every launch's ray-tracing kernels (the trace kernel, then the diffuse fan
 * kernel when n_diffuse > 0) with a pair of HIP events recorded on the launch
 * stream, srp_profile(0) stops; both reset the totals.  srp_profile_read waits
 * for the recorded launches and returns the summed kernel time (ms) and the
 * launch count since the last reset. */
int srp_profile(int enable);
int srp_profile_read(double *trace_ms, int64_t *launches);
/* The same timing for each whole launch: HIP events on the launch stream
 * around its staging upload, articulation, window, trace, fan, reduction
 * kernels and result copy.  Returns the summed milliseconds and the launch
 * count since the last reset (a host that cannot keep the device fed shows
 * as wall time above this sum).  SRP_ERR_ARG for a null output. */
int srp_profile_read_launch(double *launch_ms, int64_t *launches);

/* Thread-local message of the last error ("" if none). */
/* ---- measurement ---- */

/* The measured issue rate of non-packed FP32 fused multiply-adds on the
 * current GPU: a kernel of 8 waves per SIMD, each lane running 8 independent
 * FMA chains, timed with HIP events after a warm-up launch.  Writes the
 * lane-FMAs per second (*lane_fma_per_s), the shader clock the timed launch
 * ran at (*shader_ghz: its clock counter over its constant-rate wall clock)
 * and the compute-unit count (*n_cu).  Allocates and frees a few MB of
 * device memory; SRP_ERR_DEVICE on a HIP failure. */
int srp_valu_peak(double *lane_fma_per_s, double *shader_ghz, int32_t *n_cu);

const char *srp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
