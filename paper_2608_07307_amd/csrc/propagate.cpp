// Host orbit propagation (Sec. 3: two-body + SRP equations of motion,
// y = [x; v], y' = [v; a_g + a_SRP]) and sun tracking of the solar panels
// (Sec. 4.4.2 steps 2-4: panel normal, rotate towards the Sun, clamp).
//
// The integrators are the classical fixed-step fourth-order Runge-Kutta scheme
// and the paper's RK78 (Fehlberg's 7(8) pair, fixed or adaptive steps); every
// stage requests one SRP acceleration (Sec. 3), which srp_propagate obtains
// from the GPU evaluation with the Sun direction and pressure of the stage's
// position.  The spacecraft attitude is inertially fixed (Sec. 5.1),
// so the body frame is the heliocentric inertial frame and the Sun is at the
// origin.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "host.h"

namespace srp {
int scene_rest_normal(const srp_scene *sc, int node, double n0[3]);
const SceneHost &scene_host(const srp_scene *sc);
void set_error(const std::string &msg);
}  // namespace srp

using namespace srp;

namespace {

void rot(const double *a, double th, double *R) {
    double c = std::cos(th), s = std::sin(th), C = 1 - c;
    double x = a[0], y = a[1], z = a[2];
    double M[9] = {c + x * x * C, x * y * C - z * s, x * z * C + y * s, y * x * C + z * s, c + y * y * C,
                   y * z * C - x * s, z * x * C - y * s, z * y * C + x * s, c + z * z * C};
    std::memcpy(R, M, sizeof M);
}
void mv(const double *R, const double *x, double *y) {
    double t[3];
    for (int i = 0; i < 3; ++i) t[i] = R[3 * i] * x[0] + R[3 * i + 1] * x[1] + R[3 * i + 2] * x[2];
    std::memcpy(y, t, sizeof t);
}
void mtv(const double *R, const double *x, double *y) {   // R^T x
    double t[3];
    for (int i = 0; i < 3; ++i) t[i] = R[i] * x[0] + R[3 + i] * x[1] + R[6 + i] * x[2];
    std::memcpy(y, t, sizeof t);
}
void mm(const double *A, const double *B, double *C) {
    double T[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) T[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
    std::memcpy(C, T, sizeof T);
}
double dot(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
void cross(const double *a, const double *b, double *c) {
    double t[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    std::memcpy(c, t, sizeof t);
}

// Angle about unit axis a that turns m as close as possible to s:
// m(th) = m_par + cos th m_perp + sin th (a x m), so m(th).s is largest at
// th = atan2((a x m).s, m_perp.s).  A panel is two-sided, so the opposite face
// (th -/+ pi) is taken when that needs the smaller rotation.  Returns false
// when s is parallel to a (every angle is equally good).
bool track_angle(const double *a, const double *m, const double *s, double *th) {
    double am[3];
    cross(a, m, am);
    double ma = dot(m, a);
    double mp[3] = {m[0] - ma * a[0], m[1] - ma * a[1], m[2] - ma * a[2]};
    double y = dot(am, s), x = dot(mp, s);
    if (std::hypot(x, y) <= 1e-12 * (std::sqrt(dot(mp, mp)) + 1e-300)) return false;
    double t = std::atan2(y, x);
    double alt = t > 0 ? t - M_PI : t + M_PI;
    *th = std::fabs(alt) < std::fabs(t) ? alt : t;
    return true;
}

}  // namespace

extern "C" {

// Sun tracking (Sec. 4.4.2 steps 2-4) of every wing root: a panel node whose
// parent is not a panel.  Its axes are set outer to inner, each to the angle
// that turns the node's rest-pose area-weighted normal as close as possible to
// the Sun direction given the other angles, then clamped to its interval.
// Other angles are left as given.  angles: n_dof values in and out.
int srp_sun_tracking_angles(const srp_scene *scene, const double *sun_dir, double *angles, int32_t n_dof) {
    if (!scene || !sun_dir || (n_dof > 0 && !angles)) { set_error("null argument"); return SRP_ERR_ARG; }
    const SceneHost &S = scene_host(scene);
    if (n_dof != S.n_dof) { set_error("n_dof differs from the scene's"); return SRP_ERR_ARG; }
    double sn = std::sqrt(dot(sun_dir, sun_dir));
    if (!(sn > 0) || !std::isfinite(sn)) { set_error("zero or non-finite sun_dir"); return SRP_ERR_ARG; }
    double s[3] = {sun_dir[0] / sn, sun_dir[1] / sn, sun_dir[2] / sn};
    // world rotations of the nodes at the current angles (clamped)
    std::vector<double> Rw(9 * (size_t)S.n_nodes);
    double I[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    std::memcpy(&Rw[0], I, sizeof I);
    for (int k = 1; k < S.n_nodes; ++k) {
        const NodeInfo &nd = S.nodes[k];
        double R[9];
        std::memcpy(R, &Rw[9 * (size_t)nd.parent], sizeof R);
        bool root_wing = nd.is_panel && !S.nodes[nd.parent].is_panel && nd.n_axes > 0;
        if (root_wing) {
            double n0[3];
            scene_rest_normal(scene, k, n0);
            double sp[3];
            mtv(R, s, sp);                       // Sun direction in the parent frame
            for (int a = 0; a < nd.n_axes; ++a) {
                // normal after the inner axes at their current angles
                double m[3] = {n0[0], n0[1], n0[2]};
                for (int b = nd.n_axes - 1; b > a; --b) {
                    double Rb[9];
                    double th = std::fmin(std::fmax(angles[nd.dof_offset + b], nd.lo[b]), nd.hi[b]);
                    rot(nd.axis[b], th, Rb);
                    mv(Rb, m, m);
                }
                double th;
                if (track_angle(nd.axis[a], m, sp, &th)) angles[nd.dof_offset + a] = th;
                double tc = std::fmin(std::fmax(angles[nd.dof_offset + a], nd.lo[a]), nd.hi[a]);
                angles[nd.dof_offset + a] = tc;
                double Ra[9];
                rot(nd.axis[a], tc, Ra);
                mtv(Ra, sp, sp);                 // into the frame after this axis
            }
        }
        for (int a = 0; a < nd.n_axes; ++a) {
            double th = std::fmin(std::fmax(angles[nd.dof_offset + a], nd.lo[a]), nd.hi[a]);
            double Ra[9];
            rot(nd.axis[a], th, Ra);
            mm(R, Ra, R);
        }
        std::memcpy(&Rw[9 * (size_t)k], R, sizeof R);
    }
    return SRP_OK;
}

// Fixed-step classical RK4 for y = [r; v], y' = [v; a(t, r, v)].
// traj: (n_steps + 1) x 7 rows (t, r, v).  accel returns 0 or an error code.

int srp_rk4(const double *y0, double t0, double h, int64_t n_steps, srp_accel_fn accel, void *user, double *traj) {
    if (!y0 || !accel || !traj || n_steps < 0 || !std::isfinite(h) || !std::isfinite(t0)) {
        set_error("srp_rk4: invalid argument");
        return SRP_ERR_ARG;
    }
    double y[6];
    std::memcpy(y, y0, sizeof y);
    double t = t0;
    auto f = [&](double tt, const double *yy, double *dy) -> int {
        std::memcpy(dy, yy + 3, 3 * sizeof(double));
        return accel(tt, yy, yy + 3, dy + 3, user);
    };
    traj[0] = t;
    std::memcpy(traj + 1, y, sizeof y);
    for (int64_t k = 0; k < n_steps; ++k) {
        double k1[6], k2[6], k3[6], k4[6], yt[6];
        int rc;
        if ((rc = f(t, y, k1))) return rc;
        for (int i = 0; i < 6; ++i) yt[i] = y[i] + 0.5 * h * k1[i];
        if ((rc = f(t + 0.5 * h, yt, k2))) return rc;
        for (int i = 0; i < 6; ++i) yt[i] = y[i] + 0.5 * h * k2[i];
        if ((rc = f(t + 0.5 * h, yt, k3))) return rc;
        for (int i = 0; i < 6; ++i) yt[i] = y[i] + h * k3[i];
        if ((rc = f(t + h, yt, k4))) return rc;
        for (int i = 0; i < 6; ++i) y[i] += h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
        t = t0 + (double)(k + 1) * h;
        traj[7 * (k + 1)] = t;
        std::memcpy(traj + 7 * (k + 1) + 1, y, sizeof y);
    }
    return SRP_OK;
}

// Fehlberg's embedded Runge-Kutta 7(8) pair (13 stages; NASA TR R-287, 1968),
// the paper's RK78 (Sec. 3): nodes, coefficients (row i uses stages 0..i-1),
// 8th-order weights and the weight of the local error estimate
// (k0 + k10 - k11 - k12) h of the embedded 7th-order solution.
namespace {
constexpr double RK_C[13] = {0.0, 2.0 / 27, 1.0 / 9, 1.0 / 6, 5.0 / 12, 1.0 / 2, 5.0 / 6, 1.0 / 6, 2.0 / 3, 1.0 / 3, 1.0, 0.0, 1.0};
constexpr double RK_A[13][12] = {
    {},
    {2.0 / 27},
    {1.0 / 36, 1.0 / 12},
    {1.0 / 24, 0, 1.0 / 8},
    {5.0 / 12, 0, -25.0 / 16, 25.0 / 16},
    {1.0 / 20, 0, 0, 1.0 / 4, 1.0 / 5},
    {-25.0 / 108, 0, 0, 125.0 / 108, -65.0 / 27, 125.0 / 54},
    {31.0 / 300, 0, 0, 0, 61.0 / 225, -2.0 / 9, 13.0 / 900},
    {2.0, 0, 0, -53.0 / 6, 704.0 / 45, -107.0 / 9, 67.0 / 90, 3.0},
    {-91.0 / 108, 0, 0, 23.0 / 108, -976.0 / 135, 311.0 / 54, -19.0 / 60, 17.0 / 6, -1.0 / 12},
    {2383.0 / 4100, 0, 0, -341.0 / 164, 4496.0 / 1025, -301.0 / 82, 2133.0 / 4100, 45.0 / 82, 45.0 / 164, 18.0 / 41},
    {3.0 / 205, 0, 0, 0, 0, -6.0 / 41, -3.0 / 205, -3.0 / 41, 3.0 / 41, 6.0 / 41, 0},
    {-1777.0 / 4100, 0, 0, -341.0 / 164, 4496.0 / 1025, -289.0 / 82, 2193.0 / 4100, 51.0 / 82, 33.0 / 164, 12.0 / 41, 0, 1.0},
};
constexpr double RK_B8[13] = {0, 0, 0, 0, 0, 34.0 / 105, 9.0 / 35, 9.0 / 35, 9.0 / 280, 9.0 / 280, 0, 41.0 / 840, 41.0 / 840};
constexpr double RK_ERR = 41.0 / 840;

// One 8th-order step: y8 and the error estimate err.
int rk78_step(srp_accel_fn accel, void *user, double t, const double *y, double h, double *y8, double *err) {
    double k[13][6];
    for (int i = 0; i < 13; ++i) {
        double yi[6];
        for (int c = 0; c < 6; ++c) {
            double acc = y[c];
            for (int j = 0; j < i; ++j)
                if (RK_A[i][j] != 0.0) acc += h * RK_A[i][j] * k[j][c];
            yi[c] = acc;
        }
        std::memcpy(k[i], yi + 3, 3 * sizeof(double));
        int rc = accel(t + RK_C[i] * h, yi, yi + 3, k[i] + 3, user);
        if (rc) return rc;
    }
    for (int c = 0; c < 6; ++c) {
        double acc = y[c];
        for (int i = 0; i < 13; ++i)
            if (RK_B8[i] != 0.0) acc += h * RK_B8[i] * k[i][c];
        y8[c] = acc;
        err[c] = RK_ERR * h * (k[0][c] + k[10][c] - k[11][c] - k[12][c]);
    }
    return SRP_OK;
}
}  // namespace

// RK7(8) from t0 to t1 (srp.h): fixed steps t0 + k h0 (the last ending at t1),
// or adaptive steps accepted when max_i |err_i| / (atol_i + rtol max(|y_i|,
// |y8_i|)) <= 1 (a zero error counts 0) and resized by 0.9 err^(-1/8) within
// [0.2, 5].
int srp_rk78(const double *y0, double t0, double t1, const srp_rk78_opts *o, srp_accel_fn accel, void *user,
             double *traj, int64_t max_rows, int64_t *n_rows, int64_t *n_evals) {
    if (!y0 || !o || !accel || !traj || !n_rows || max_rows < 1 || !std::isfinite(t0) || !std::isfinite(t1) ||
        !(t1 > t0) || !(o->h0 > 0) || !std::isfinite(o->h0)) {
        set_error("srp_rk78: invalid argument");
        return SRP_ERR_ARG;
    }
    double tol_sum = o->rtol;
    for (int c = 0; c < 6; ++c) {
        if (!(o->atol[c] >= 0) || !std::isfinite(o->atol[c])) { set_error("srp_rk78: invalid atol"); return SRP_ERR_ARG; }
        tol_sum += o->atol[c];
    }
    if (o->adaptive && (!(o->rtol >= 0) || !(tol_sum > 0) || !(o->h_min >= 0))) {
        set_error("srp_rk78: adaptive steps need rtol >= 0, some tolerance > 0 and h_min >= 0");
        return SRP_ERR_ARG;
    }
    double y[6], y8[6], err[6];
    std::memcpy(y, y0, sizeof y);
    int64_t rows = 1, evals = 0;
    traj[0] = t0;
    std::memcpy(traj + 1, y, sizeof y);
    auto emit = [&](double t) -> int {
        if (rows >= max_rows) { set_error("srp_rk78: more steps than max_rows"); return SRP_ERR_ARG; }
        traj[7 * rows] = t;
        std::memcpy(traj + 7 * rows + 1, y, sizeof y);
        ++rows;
        return SRP_OK;
    };
    int rc = SRP_OK;
    if (!o->adaptive) {
        const double q = std::ceil((t1 - t0) / o->h0 * (1 - 1e-12));
        if (!(q >= 1) || q > 1e12) { set_error("srp_rk78: step count out of range"); return SRP_ERR_ARG; }
        const int64_t n = (int64_t)q;
        for (int64_t k = 0; k < n && !rc; ++k) {
            const double tk = t0 + (double)k * o->h0, hs = k == n - 1 ? t1 - tk : o->h0;
            if ((rc = rk78_step(accel, user, tk, y, hs, y8, err))) break;
            evals += 13;
            std::memcpy(y, y8, sizeof y);
            rc = emit(k == n - 1 ? t1 : t0 + (double)(k + 1) * o->h0);
        }
    } else {
        double t = t0, h = o->h0;
        while (t < t1 && !rc) {
            const bool last = h >= t1 - t;
            const double hs = last ? t1 - t : h;
            if ((rc = rk78_step(accel, user, t, y, hs, y8, err))) break;
            evals += 13;
            double e = 0;
            for (int c = 0; c < 6; ++c) {
                const double sc = o->atol[c] + o->rtol * std::fmax(std::fabs(y[c]), std::fabs(y8[c]));
                if (!std::isfinite(y8[c]) || std::isnan(err[c])) { e = NAN; break; }
                if (err[c] != 0.0) e = std::fmax(e, std::fabs(err[c]) / sc);   // zero error counts 0, also where sc = 0
            }
            if (std::isnan(e)) { set_error("srp_rk78: non-finite state or error estimate"); rc = SRP_ERR_ARG; break; }
            const double fac = e == 0 ? 5.0 : std::fmin(5.0, std::fmax(0.2, 0.9 * std::pow(e, -1.0 / 8.0)));
            if (e > 1.0) {
                h = hs * fac;
                if (h < o->h_min) { set_error("srp_rk78: step below h_min"); rc = SRP_ERR_ARG; }
                continue;
            }
            t = last ? t1 : t + hs;
            std::memcpy(y, y8, sizeof y);
            h = hs * fac;
            if (o->h_max > 0) h = std::fmin(h, o->h_max);
            rc = emit(t);
        }
    }
    *n_rows = rows;
    if (n_evals) *n_evals = evals;
    return rc;
}

}  // extern "C"

namespace {
struct PropCtx {
    srp_scene *sc;
    const srp_orbit_params *op;
    std::vector<double> angles;
    int64_t evals = 0;
    double secs = 0;
};

int prop_accel(double, const double *r, const double *, double *a, void *user) {
    PropCtx &C = *reinterpret_cast<PropCtx *>(user);
    const srp_orbit_params &O = *C.op;
    double rn = std::sqrt(dot(r, r));
    if (!(rn > 0)) { set_error("spacecraft at the Sun"); return SRP_ERR_ARG; }
    double s[3] = {-r[0] / rn, -r[1] / rn, -r[2] / rn};   // spacecraft -> Sun
    struct timespec t0, t1;
    clock_gettime(CLOCK_MONOTONIC, &t0);
    int rc;
    if (O.track_sun) {
        if ((rc = srp_sun_tracking_angles(C.sc, s, C.angles.data(), (int32_t)C.angles.size()))) return rc;
    }
    srp_eval_params p;
    std::memset(&p, 0, sizeof p);
    std::memcpy(p.sun_dir, s, sizeof s);
    p.pressure = O.p_ref * (O.r_ref / rn) * (O.r_ref / rn);
    p.n = O.n;
    p.bounces = O.bounces;
    p.n_diffuse = O.n_diffuse;
    std::memcpy(p.ref, O.ref, sizeof p.ref);
    srp_result res;
    // tracking: this stage's angles go with the evaluation (the slot is built on the
    // device inside the captured launch); the scene takes the last ones at the end
    if ((rc = eval_single(C.sc, &p, O.track_sun ? C.angles.data() : nullptr, &res, nullptr, nullptr))) return rc;
    clock_gettime(CLOCK_MONOTONIC, &t1);
    C.secs += (t1.tv_sec - t0.tv_sec) + 1e-9 * (t1.tv_nsec - t0.tv_nsec);
    C.evals++;
    double g = -O.mu / (rn * rn * rn);
    for (int i = 0; i < 3; ++i) a[i] = g * r[i] + res.force[i] / O.mass;
    return SRP_OK;
}
}  // namespace

extern "C" int srp_propagate_rk78(srp_scene *scene, const srp_orbit_params *op, const double *angles0,
                                  const double *y0, double t0, double t1, const srp_rk78_opts *opts, double *traj,
                                  int64_t max_rows, int64_t *n_rows, srp_prop_stats *stats) {
    if (!scene || !op || !y0 || !traj || !opts || !n_rows) { set_error("null argument"); return SRP_ERR_ARG; }
    if (!(op->mass > 0) || !std::isfinite(op->mu) || !std::isfinite(op->p_ref) || !(op->r_ref > 0)) {
        set_error("invalid orbit parameters");
        return SRP_ERR_ARG;
    }
    const SceneHost &S = scene_host(scene);
    PropCtx C{scene, op, std::vector<double>(S.n_dof, 0.0)};
    if (angles0 && S.n_dof) std::memcpy(C.angles.data(), angles0, sizeof(double) * S.n_dof);
    int rc = srp_set_panel_angles(scene, C.angles.data(), S.n_dof);
    if (rc < 0) return rc;
    rc = srp_rk78(y0, t0, t1, opts, prop_accel, &C, traj, max_rows, n_rows, nullptr);
    if (stats) { stats->n_evals = C.evals; stats->srp_seconds = C.secs; }
    if (rc == SRP_OK && op->track_sun) {
        const int r2 = srp_set_panel_angles(scene, C.angles.data(), S.n_dof);   // the last stage's angles
        if (r2 < 0) return r2;
    }
    return rc;
}

extern "C" int srp_propagate(srp_scene *scene, const srp_orbit_params *op, const double *angles0, const double *y0,
                             double t0, double h, int64_t n_steps, double *traj, srp_prop_stats *stats) {
    if (!scene || !op || !y0 || !traj) { set_error("null argument"); return SRP_ERR_ARG; }
    if (!(op->mass > 0) || !std::isfinite(op->mu) || !std::isfinite(op->p_ref) || !(op->r_ref > 0)) {
        set_error("invalid orbit parameters");
        return SRP_ERR_ARG;
    }
    const SceneHost &S = scene_host(scene);
    PropCtx C{scene, op, std::vector<double>(S.n_dof, 0.0)};
    if (angles0 && S.n_dof) std::memcpy(C.angles.data(), angles0, sizeof(double) * S.n_dof);
    int rc = srp_set_panel_angles(scene, C.angles.data(), S.n_dof);
    if (rc < 0) return rc;
    rc = srp_rk4(y0, t0, h, n_steps, prop_accel, &C, traj);
    if (stats) { stats->n_evals = C.evals; stats->srp_seconds = C.secs; }
    if (rc == SRP_OK && op->track_sun) {
        const int r2 = srp_set_panel_angles(scene, C.angles.data(), S.n_dof);   // the last stage's angles
        if (r2 < 0) return r2;
    }
    return rc;
}
