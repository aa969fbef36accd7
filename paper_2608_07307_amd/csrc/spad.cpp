// SPAD tables: the SRP force and torque precomputed over a grid of Sun
// directions in the body frame and interpolated during propagation instead of
// tracing rays at every stage (Sec. 2 and Sec. 4.2; Sec. 6.1 uses grids of
// 20 azimuth x 10 elevation values).  The table is built by one batched GPU
// launch (srp_eval_batch); interpolation and propagation run on the host.
//
// Grid: az_j = az0 + j daz, el_i = el0 + i del; node (i, j) holds the result
// for s = (cos el cos az, cos el sin az, sin el).  Interpolation is bilinear
// in (az, el) with az = atan2(s_y, s_x), el = atan2(s_z, hypot(s_x, s_y));
// azimuth wraps when the grid spans a full turn, otherwise it is held at the
// first / last column, and elevations beyond the first / last row take that
// row.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "host.h"

namespace srp {
void set_error(const std::string &msg);
}

using namespace srp;

namespace {

constexpr double TWO_PI = 6.283185307179586476925;

int check_grid(const srp_spad_grid *g) {
    if (!g) { set_error("null grid"); return SRP_ERR_ARG; }
    if (g->n_az < 1 || g->n_el < 1 || (int64_t)g->n_az * g->n_el > (int64_t(1) << 24)) {
        set_error("grid size out of range (1..2^24 nodes)");
        return SRP_ERR_ARG;
    }
    if (!std::isfinite(g->az0) || !std::isfinite(g->el0) || !(g->daz > 0) || !(g->del > 0) ||
        !std::isfinite(g->daz) || !std::isfinite(g->del)) {
        set_error("grid origin or spacing invalid");
        return SRP_ERR_ARG;
    }
    return SRP_OK;
}

void node_dir(const srp_spad_grid &g, int i, int j, double s[3]) {
    const double az = g.az0 + j * g.daz, el = g.el0 + i * g.del;
    s[0] = std::cos(el) * std::cos(az);
    s[1] = std::cos(el) * std::sin(az);
    s[2] = std::sin(el);
}

// Lower node index and weight of the upper one along one axis.
void axis_cell(double u, int n, bool wrap, int *k0, int *k1, double *f) {
    if (wrap) {
        double q = std::floor(u / n);
        u -= q * n;                           // [0, n], n only by rounding
        int k = (int)std::floor(u);
        *f = u - k;
        if (k >= n) { k = 0; *f = 0.0; }
        *k0 = k;
        *k1 = (k + 1) % n;
        return;
    }
    u = std::fmin(std::fmax(u, 0.0), (double)(n - 1));
    int k = std::min((int)std::floor(u), std::max(n - 2, 0));
    *f = u - k;
    *k0 = k;
    *k1 = std::min(k + 1, n - 1);
}

void interp(const srp_spad_grid &g, const double *table, const double *s, double *out) {
    const double az = std::atan2(s[1], s[0]), el = std::atan2(s[2], std::hypot(s[0], s[1]));
    const bool wrap = std::fabs(g.n_az * g.daz - TWO_PI) <= 1e-9;
    int j0, j1, i0, i1;
    double fu, fv;
    axis_cell((az - g.az0) / g.daz, g.n_az, wrap, &j0, &j1, &fu);
    axis_cell((el - g.el0) / g.del, g.n_el, false, &i0, &i1, &fv);
    const double *t00 = table + 6 * ((size_t)i0 * g.n_az + j0), *t01 = table + 6 * ((size_t)i0 * g.n_az + j1);
    const double *t10 = table + 6 * ((size_t)i1 * g.n_az + j0), *t11 = table + 6 * ((size_t)i1 * g.n_az + j1);
    for (int c = 0; c < 6; ++c)
        out[c] = (1 - fu) * (1 - fv) * t00[c] + fu * (1 - fv) * t01[c] + (1 - fu) * fv * t10[c] + fu * fv * t11[c];
}

struct SpadCtx {
    const srp_spad_grid *g;
    const double *table;
    double p_table;
    const srp_orbit_params *op;
};

int spad_accel(double, const double *r, const double *, double *a, void *user) {
    const SpadCtx &C = *reinterpret_cast<const SpadCtx *>(user);
    const srp_orbit_params &O = *C.op;
    const double rn = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    if (!(rn > 0)) { set_error("spacecraft at the Sun"); return SRP_ERR_ARG; }
    const double s[3] = {-r[0] / rn, -r[1] / rn, -r[2] / rn};
    double f[6];
    interp(*C.g, C.table, s, f);
    const double scale = O.p_ref * (O.r_ref / rn) * (O.r_ref / rn) / C.p_table;
    const double gk = -O.mu / (rn * rn * rn);
    for (int i = 0; i < 3; ++i) a[i] = gk * r[i] + scale * f[i] / O.mass;
    return SRP_OK;
}

}  // namespace

extern "C" {

int srp_spad_build(srp_scene *scene, const srp_eval_params *params, const double *angles, const srp_spad_grid *grid,
                   double *table) {
    if (!scene || !params || !table) { set_error("null argument"); return SRP_ERR_ARG; }
    int rc = check_grid(grid);
    if (rc) return rc;
    const int64_t n = (int64_t)grid->n_az * grid->n_el;
    std::vector<srp_batch_item> items((size_t)n);
    for (int i = 0; i < grid->n_el; ++i)
        for (int j = 0; j < grid->n_az; ++j) {
            srp_batch_item &it = items[(size_t)i * grid->n_az + j];
            it.scene = scene;
            it.angles = angles;
            it.p = *params;
            node_dir(*grid, i, j, it.p.sun_dir);
        }
    srp_result *d_out = nullptr;
    if (hipMalloc(&d_out, sizeof(srp_result) * (size_t)n) != hipSuccess) {
        (void)hipGetLastError();
        set_error("SPAD result allocation failed");
        return SRP_ERR_OOM;
    }
    std::vector<srp_result> res((size_t)n);
    rc = srp_eval_batch(items.data(), n, d_out, nullptr);   // null stream: ordered before the copy
    if (!rc && hipMemcpy(res.data(), d_out, sizeof(srp_result) * (size_t)n, hipMemcpyDeviceToHost) != hipSuccess) {
        set_error(std::string("SPAD result copy: ") + hipGetErrorString(hipGetLastError()));
        rc = SRP_ERR_DEVICE;
    }
    (void)hipFree(d_out);
    if (rc) return rc;
    for (int64_t k = 0; k < n; ++k) {
        if (res[k].status & SRP_STATUS_STACK) { set_error("traversal stack overflow"); return SRP_ERR_DEPTH; }
        std::memcpy(table + 6 * k, res[k].force, 3 * sizeof(double));
        std::memcpy(table + 6 * k + 3, res[k].torque, 3 * sizeof(double));
    }
    return SRP_OK;
}

int srp_spad_interp(const srp_spad_grid *grid, const double *table, const double *sun_dir, double *out) {
    if (!table || !sun_dir || !out) { set_error("null argument"); return SRP_ERR_ARG; }
    int rc = check_grid(grid);
    if (rc) return rc;
    const double sn = std::sqrt(sun_dir[0] * sun_dir[0] + sun_dir[1] * sun_dir[1] + sun_dir[2] * sun_dir[2]);
    if (!(sn > 0) || !std::isfinite(sn)) { set_error("zero or non-finite sun_dir"); return SRP_ERR_ARG; }
    interp(*grid, table, sun_dir, out);
    return SRP_OK;
}

int srp_propagate_spad(const srp_spad_grid *grid, const double *table, double p_table, const srp_orbit_params *op,
                       const double *y0, double t0, double h, int64_t n_steps, double *traj) {
    if (!table || !op || !y0 || !traj) { set_error("null argument"); return SRP_ERR_ARG; }
    int rc = check_grid(grid);
    if (rc) return rc;
    if (!(p_table > 0) || !std::isfinite(p_table) || !(op->mass > 0) || !std::isfinite(op->mu) ||
        !std::isfinite(op->p_ref) || !(op->r_ref > 0)) {
        set_error("invalid table pressure or orbit parameters");
        return SRP_ERR_ARG;
    }
    if (op->track_sun) { set_error("a SPAD table is built at fixed hinge angles: track_sun must be 0"); return SRP_ERR_ARG; }
    SpadCtx C{grid, table, p_table, op};
    return srp_rk4(y0, t0, h, n_steps, spad_accel, &C, traj);
}

int srp_propagate_spad_rk78(const srp_spad_grid *grid, const double *table, double p_table,
                            const srp_orbit_params *op, const double *y0, double t0, double t1,
                            const srp_rk78_opts *opts, double *traj, int64_t max_rows, int64_t *n_rows) {
    if (!table || !op || !y0 || !traj || !opts || !n_rows) { set_error("null argument"); return SRP_ERR_ARG; }
    int rc = check_grid(grid);
    if (rc) return rc;
    if (!(p_table > 0) || !std::isfinite(p_table) || !(op->mass > 0) || !std::isfinite(op->mu) ||
        !std::isfinite(op->p_ref) || !(op->r_ref > 0)) {
        set_error("invalid table pressure or orbit parameters");
        return SRP_ERR_ARG;
    }
    if (op->track_sun) { set_error("a SPAD table is built at fixed hinge angles: track_sun must be 0"); return SRP_ERR_ARG; }
    SpadCtx C{grid, table, p_table, op};
    return srp_rk78(y0, t0, t1, opts, spad_accel, &C, traj, max_rows, n_rows, nullptr);
}

}  // extern "C"
