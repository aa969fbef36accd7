// N-plate SRP model: the analytical model the paper compares its ray tracer
// and its SPAD tables against (Sec. 1; one of the strategies of Sec. 6.1 and
// 7.1).  The spacecraft is a set of flat plates, each lit on the side its
// normal points to (either side when two-sided), with no shadowing and no
// secondary rays.  Per lit plate, s the unit Sun direction, d = -s the photon
// direction, n the normal turned towards the Sun and c = n . s > 0, the
// flat-plate law
//   F = P A c [(1 - rho_s) d - 2 (rho_s c + rho_d / 3) n],  tau = (x - ref) x F.
// Host code; the propagation uses the library's RK4 / RK7(8) integrators.
#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <new>
#include <string>

#include "host.h"

namespace srp {
void set_error(const std::string &msg);
}

using namespace srp;

namespace {

int check_plates(const srp_plate *p, int32_t n) {
    if (n < 0 || (n > 0 && !p)) { set_error("null plates or negative count"); return SRP_ERR_ARG; }
    for (int32_t k = 0; k < n; ++k) {
        const srp_plate &q = p[k];
        const double nn = q.normal[0] * q.normal[0] + q.normal[1] * q.normal[1] + q.normal[2] * q.normal[2];
        if (!(std::fabs(nn - 1.0) <= 1e-9) || !(q.area > 0) || !std::isfinite(q.area) ||
            !std::isfinite(q.center[0]) || !std::isfinite(q.center[1]) || !std::isfinite(q.center[2]) ||
            !(q.rho_s >= 0 && q.rho_s <= 1) || !(q.rho_d >= 0 && q.rho_d <= 1)) {
            set_error("plate " + std::to_string(k) + ": non-unit normal, non-positive area or bad reflectivity");
            return SRP_ERR_ARG;
        }
    }
    return SRP_OK;
}

// Force and torque of the plates for unit Sun direction s.
void nplate_force(const srp_plate *p, int32_t n, const double s[3], double P, const double ref[3], double F[3],
                  double T[3]) {
    for (int i = 0; i < 3; ++i) F[i] = T[i] = 0.0;
    for (int32_t k = 0; k < n; ++k) {
        const srp_plate &q = p[k];
        double nv[3] = {q.normal[0], q.normal[1], q.normal[2]};
        double c = nv[0] * s[0] + nv[1] * s[1] + nv[2] * s[2];
        if (c < 0 && q.two_sided) {
            for (int i = 0; i < 3; ++i) nv[i] = -nv[i];
            c = -c;
        }
        if (!(c > 0)) continue;
        const double a = P * q.area * c;
        double f[3];
        for (int i = 0; i < 3; ++i) f[i] = a * ((1.0 - q.rho_s) * (-s[i]) - 2.0 * (q.rho_s * c + q.rho_d / 3.0) * nv[i]);
        const double r[3] = {q.center[0] - ref[0], q.center[1] - ref[1], q.center[2] - ref[2]};
        F[0] += f[0];
        F[1] += f[1];
        F[2] += f[2];
        T[0] += r[1] * f[2] - r[2] * f[1];
        T[1] += r[2] * f[0] - r[0] * f[2];
        T[2] += r[0] * f[1] - r[1] * f[0];
    }
}

struct NplateCtx {
    const srp_plate *p;
    int32_t n;
    const srp_orbit_params *op;
};

int nplate_accel(double, const double *r, const double *, double *a, void *user) {
    const NplateCtx &C = *reinterpret_cast<const NplateCtx *>(user);
    const srp_orbit_params &O = *C.op;
    const double rn = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    if (!(rn > 0)) { set_error("spacecraft at the Sun"); return SRP_ERR_ARG; }
    const double s[3] = {-r[0] / rn, -r[1] / rn, -r[2] / rn};
    const double P = O.p_ref * (O.r_ref / rn) * (O.r_ref / rn);
    const double zero[3] = {0, 0, 0};
    double F[3], T[3];
    nplate_force(C.p, C.n, s, P, zero, F, T);
    const double gk = -O.mu / (rn * rn * rn);
    for (int i = 0; i < 3; ++i) a[i] = gk * r[i] + F[i] / O.mass;
    return SRP_OK;
}

int check_orbit(const srp_orbit_params *op) {
    if (!(op->mass > 0) || !std::isfinite(op->mu) || !std::isfinite(op->p_ref) || !(op->r_ref > 0)) {
        set_error("invalid orbit parameters");
        return SRP_ERR_ARG;
    }
    if (op->track_sun) { set_error("the N-plate model has fixed plates: track_sun must be 0"); return SRP_ERR_ARG; }
    return SRP_OK;
}

}  // namespace

namespace srp {

void plates_build(SceneHost *S) {
    // per triangle: area, unit normal and centroid in its node's frame, and a
    // grouping key (node, material, normal rounded to 1e-6)
    struct Tri {
        std::array<int64_t, 5> key;
        int32_t id;
        double a, n[3], c[3];
    };
    std::vector<Tri> t;
    t.reserve(S->tris.size());
    for (const TriRec &T : S->tris) {
        double e1[3], e2[3];
        for (int i = 0; i < 3; ++i) {
            e1[i] = (double)T.v1[i] - (double)T.v0[i];
            e2[i] = (double)T.v2[i] - (double)T.v0[i];
        }
        const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                              e1[0] * e2[1] - e1[1] * e2[0]};
        const double len = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        if (!(len > 0)) continue;   // zero-area triangle
        Tri q;
        q.id = T.id;
        q.a = 0.5 * len;
        for (int i = 0; i < 3; ++i) {
            q.n[i] = cr[i] / len;
            q.c[i] = ((double)T.v0[i] + (double)T.v1[i] + (double)T.v2[i]) / 3.0;
        }
        q.key = {T.node, T.mat, std::llround(q.n[0] * 1e6), std::llround(q.n[1] * 1e6), std::llround(q.n[2] * 1e6)};
        t.push_back(q);
    }
    // groups are runs of equal keys; within a group the sums run in triangle
    // order, so the result does not depend on the leaf order
    std::sort(t.begin(), t.end(), [](const Tri &x, const Tri &y) { return x.key != y.key ? x.key < y.key : x.id < y.id; });
    std::vector<std::pair<int32_t, PlateLocal>> g;   // (first triangle, plate)
    for (size_t k = 0; k < t.size(); ++k) {
        if (k == 0 || t[k].key != t[k - 1].key) {
            PlateLocal P;
            P.node = (int32_t)t[k].key[0];
            P.mat = (int32_t)t[k].key[1];
            g.emplace_back(t[k].id, P);
        }
        PlateLocal &P = g.back().second;
        P.area += t[k].a;
        for (int i = 0; i < 3; ++i) {
            P.n[i] += t[k].a * t[k].n[i];
            P.c[i] += t[k].a * t[k].c[i];
        }
    }
    std::sort(g.begin(), g.end(), [](const std::pair<int32_t, PlateLocal> &x, const std::pair<int32_t, PlateLocal> &y) {
        return x.first < y.first;
    });
    S->plates.clear();
    S->plates.reserve(g.size());
    for (auto &e : g) {
        for (int i = 0; i < 3; ++i) e.second.c[i] /= e.second.area;
        S->plates.push_back(e.second);
    }
}

void plates_world(const SceneHost &S, const SlotHost &slot, srp_plate *out) {
    for (size_t k = 0; k < S.plates.size(); ++k) {
        const PlateLocal &P = S.plates[k];
        const double *X = slot.xf.data() + 12 * (size_t)P.node;
        srp_plate &q = out[k];
        double nw[3];
        for (int i = 0; i < 3; ++i) {
            nw[i] = X[3 * i] * P.n[0] + X[3 * i + 1] * P.n[1] + X[3 * i + 2] * P.n[2];
            q.center[i] = X[3 * i] * P.c[0] + X[3 * i + 1] * P.c[1] + X[3 * i + 2] * P.c[2] + X[9 + i];
        }
        const double nl = std::sqrt(nw[0] * nw[0] + nw[1] * nw[1] + nw[2] * nw[2]);
        for (int i = 0; i < 3; ++i) q.normal[i] = nw[i] / nl;
        q.area = P.area;
        q.rho_s = S.mats[2 * (size_t)P.mat];
        q.rho_d = S.mats[2 * (size_t)P.mat + 1];
        q.two_sided = S.nodes[P.node].is_panel ? 1 : 0;
        q.reserved = 0;
    }
}

}  // namespace srp

extern "C" {

int srp_nplate_from_mesh(const double *verts, int64_t n_verts, const int32_t *tris, int64_t n_tris,
                         const int32_t *tri_material, const int32_t *tri_node, const srp_material *mats,
                         int32_t n_mats, const srp_node *nodes, int32_t n_nodes, const double *angles,
                         srp_plate *plates, int32_t max_plates, int32_t *n_plates) {
    if (!n_plates || (max_plates > 0 && !plates) || max_plates < 0) {
        set_error("null plates or count");
        return SRP_ERR_ARG;
    }
    std::string err;
    try {
        SceneHost h;
        int rc = scene_build(verts, n_verts, tris, n_tris, tri_material, tri_node, mats, n_mats, nodes, n_nodes, &h,
                             &err);
        SlotHost slot;
        if (!rc) rc = slot_build(h, angles, &slot, &err);
        if (rc) { set_error(err); return rc; }
        plates_build(&h);
        if (h.plates.size() > (size_t)INT32_MAX) { set_error("too many plates"); return SRP_ERR_ARG; }
        *n_plates = (int32_t)h.plates.size();
        if ((int64_t)h.plates.size() > max_plates) {
            set_error("max_plates too small: " + std::to_string(h.plates.size()) + " plates");
            return SRP_ERR_ARG;
        }
        plates_world(h, slot, plates);
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return SRP_ERR_OOM;
    }
    return SRP_OK;
}


int srp_nplate_eval(const srp_plate *plates, int32_t n_plates, const double *sun_dir, double pressure,
                    const double *ref, double *force, double *torque) {
    if (!sun_dir || !ref || !force || !torque) { set_error("null argument"); return SRP_ERR_ARG; }
    int rc = check_plates(plates, n_plates);
    if (rc) return rc;
    const double sn = std::sqrt(sun_dir[0] * sun_dir[0] + sun_dir[1] * sun_dir[1] + sun_dir[2] * sun_dir[2]);
    if (!(sn > 0) || !std::isfinite(sn) || !std::isfinite(pressure)) {
        set_error("zero or non-finite sun_dir, or non-finite pressure");
        return SRP_ERR_ARG;
    }
    const double s[3] = {sun_dir[0] / sn, sun_dir[1] / sn, sun_dir[2] / sn};
    nplate_force(plates, n_plates, s, pressure, ref, force, torque);
    return SRP_OK;
}

int srp_propagate_nplate(const srp_plate *plates, int32_t n_plates, const srp_orbit_params *op, const double *y0,
                         double t0, double h, int64_t n_steps, double *traj) {
    if (!op || !y0 || !traj) { set_error("null argument"); return SRP_ERR_ARG; }
    int rc = check_plates(plates, n_plates);
    if (rc || (rc = check_orbit(op))) return rc;
    NplateCtx C{plates, n_plates, op};
    return srp_rk4(y0, t0, h, n_steps, nplate_accel, &C, traj);
}

int srp_propagate_nplate_rk78(const srp_plate *plates, int32_t n_plates, const srp_orbit_params *op,
                              const double *y0, double t0, double t1, const srp_rk78_opts *opts, double *traj,
                              int64_t max_rows, int64_t *n_rows) {
    if (!op || !y0 || !traj || !opts || !n_rows) { set_error("null argument"); return SRP_ERR_ARG; }
    int rc = check_plates(plates, n_plates);
    if (rc || (rc = check_orbit(op))) return rc;
    NplateCtx C{plates, n_plates, op};
    return srp_rk78(y0, t0, t1, opts, nplate_accel, &C, traj, max_rows, n_rows, nullptr);
}

}  // extern "C"
