// Scene construction on the host: input validation, one bounding-volume
// hierarchy per kinematic-tree node in rest-pose coordinates, the window
// point set, the top-level topology, and the per-angle articulation slot
// (instance transforms and the top level refitted to them).
//
// The paper moves the triangles of each articulated subtree on the CPU before
// every evaluation (Sec. 4.4.2, step 5).  Here each node's triangles stay in
// their rest pose inside their own hierarchy; a hinge rotation only changes
// the node's rigid transform, so an angle update builds nothing: it refits
// the boxes of a top level of at most SRP_MAX_NODES instances whose topology
// was built once, over the rest pose.  The articulation kernel
// (articulate.hip) does the same for a batch's angle vectors with the same
// separately rounded FP64 operations, so both give the same bits; floating-
// point contraction stays off in both files for that reason.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "host.h"

#pragma clang fp contract(off)

namespace srp {

namespace {

constexpr int BINS = 16;
// Surface-area cost of a binary node's traversal relative to one triangle test.
// Measured on the ~50k-triangle craft at 1024^2, B = 2: 1.0 beats 0.3, 0.6, 1.5,
// 2.0 and 3.0 for the batched forward + adjoint launch; larger values (bigger
// leaves) favour single evaluations and smaller ones nothing.
constexpr double C_TRAV = 1.0;

struct Prim {
    float lo[3], hi[3];
    float c[3];
    int32_t tri;
};

// Binary node of the build (host only); the device gets the 4-wide collapse.
struct BNode2 {
    float lo[2][3], hi[2][3];
    uint32_t ref[2];
};

struct Box {
    float lo[3], hi[3];
    Box() {
        for (int a = 0; a < 3; ++a) { lo[a] = INFINITY; hi[a] = -INFINITY; }
    }
    void grow(const Box &b) {
        for (int a = 0; a < 3; ++a) { lo[a] = std::min(lo[a], b.lo[a]); hi[a] = std::max(hi[a], b.hi[a]); }
    }
    void grow(const float *p) {
        for (int a = 0; a < 3; ++a) { lo[a] = std::min(lo[a], p[a]); hi[a] = std::max(hi[a], p[a]); }
    }
    double area() const {
        double dx = (double)hi[0] - lo[0], dy = (double)hi[1] - lo[1], dz = (double)hi[2] - lo[2];
        if (!(dx >= 0) || !(dy >= 0) || !(dz >= 0)) return 0;
        return 2.0 * (dx * dy + dy * dz + dz * dx);
    }
};

int ceil_log2(int64_t x) {
    int k = 0;
    while ((int64_t(1) << k) < x) ++k;
    return k;
}

struct BlasBuilder {
    std::vector<Prim> &P;
    const std::vector<TriRec> &rec;   // by original triangle index
    std::vector<BNode2> &nodes;
    std::vector<TriRec> &out;
    float pad;
    int max_depth = 0;
    bool depth_error = false;

    uint32_t leaf(int b, int e) {
        uint32_t first = (uint32_t)out.size();
        for (int k = b; k < e; ++k) out.push_back(rec[P[k].tri]);
        return make_ref(REF_BLAS_LEAF, (first << 3) | (uint32_t)(e - b - 1));
    }

    // Builds prims [b, e) at `depth` internal levels below the root; returns its
    // reference and writes its (unpadded) bounds.
    uint32_t build(int b, int e, int depth, Box &bounds) {
        Box cb;
        bounds = Box();
        for (int k = b; k < e; ++k) {
            Box pb;
            std::memcpy(pb.lo, P[k].lo, sizeof pb.lo);
            std::memcpy(pb.hi, P[k].hi, sizeof pb.hi);
            bounds.grow(pb);
            cb.grow(P[k].c);
        }
        int n = e - b;
        if (n <= 1) return leaf(b, e);
        int remaining = BLAS_MAX_DEPTH - depth;                // internal levels still allowed
        int needed = ceil_log2((n + LEAF_MAX - 1) / LEAF_MAX); // levels a balanced split needs
        if (needed > remaining) { depth_error = true; return leaf(b, std::min(e, b + LEAF_MAX)); }

        int split = -1, axis = -1;
        double best = INFINITY;
        bool sah = remaining > needed + 1;
        double leaf_cost = n;
        if (sah) {
            double pa = bounds.area();
            for (int a = 0; a < 3; ++a) {
                double ext = (double)cb.hi[a] - cb.lo[a];
                if (!(ext > 0)) continue;
                Box bb[BINS];
                int cnt[BINS] = {0};
                double scale = BINS / ext;
                for (int k = b; k < e; ++k) {
                    int bi = std::min(BINS - 1, (int)((P[k].c[a] - cb.lo[a]) * scale));
                    Box pb;
                    std::memcpy(pb.lo, P[k].lo, sizeof pb.lo);
                    std::memcpy(pb.hi, P[k].hi, sizeof pb.hi);
                    bb[bi].grow(pb);
                    cnt[bi]++;
                }
                double la[BINS], ra[BINS];
                int lc[BINS], rc[BINS];
                Box acc;
                int c = 0;
                for (int i = 0; i < BINS; ++i) { acc.grow(bb[i]); c += cnt[i]; la[i] = acc.area(); lc[i] = c; }
                acc = Box();
                c = 0;
                for (int i = BINS - 1; i >= 0; --i) { acc.grow(bb[i]); c += cnt[i]; ra[i] = acc.area(); rc[i] = c; }
                for (int i = 0; i < BINS - 1; ++i) {
                    if (lc[i] == 0 || rc[i + 1] == 0) continue;
                    double cost = C_TRAV + (pa > 0 ? (la[i] * lc[i] + ra[i + 1] * rc[i + 1]) / pa : n);
                    if (cost < best) { best = cost; split = i; axis = a; }
                }
            }
            if (n <= LEAF_MAX && leaf_cost <= best) return leaf(b, e);
        } else if (n <= LEAF_MAX && n <= 4) {
            return leaf(b, e);
        }

        int mid;
        if (split >= 0) {
            double ext = (double)cb.hi[axis] - cb.lo[axis];
            double scale = BINS / ext;
            float lo = cb.lo[axis];
            auto it = std::partition(P.begin() + b, P.begin() + e, [&](const Prim &p) {
                return std::min(BINS - 1, (int)((p.c[axis] - lo) * scale)) <= split;
            });
            mid = (int)(it - P.begin());
        } else {
            // object median along the widest centroid axis (or by index when all coincide)
            int a = 0;
            for (int k = 1; k < 3; ++k)
                if ((double)cb.hi[k] - cb.lo[k] > (double)cb.hi[a] - cb.lo[a]) a = k;
            mid = b + n / 2;
            std::nth_element(P.begin() + b, P.begin() + mid, P.begin() + e, [&](const Prim &x, const Prim &y) {
                return x.c[a] < y.c[a] || (x.c[a] == y.c[a] && x.tri < y.tri);
            });
        }
        if (mid <= b || mid >= e) mid = b + n / 2;

        uint32_t me = (uint32_t)nodes.size();
        nodes.push_back(BNode2{});
        max_depth = std::max(max_depth, depth + 1);
        Box lb, rb;
        uint32_t l = build(b, mid, depth + 1, lb);
        uint32_t r = build(mid, e, depth + 1, rb);
        BNode2 &nd = nodes[me];
        for (int a = 0; a < 3; ++a) {
            nd.lo[0][a] = lb.lo[a] - pad; nd.hi[0][a] = lb.hi[a] + pad;
            nd.lo[1][a] = rb.lo[a] - pad; nd.hi[1][a] = rb.hi[a] + pad;
        }
        nd.ref[0] = l;
        nd.ref[1] = r;
        return make_ref(REF_BLAS_NODE, me);
    }
};

// Collapses a binary hierarchy into 4-wide nodes: a node takes the children
// of its binary node and keeps replacing its largest-area inner child by that
// child's two children until it has four (or only leaves).  References of
// `inner` type are rewritten; leaves pass through.
struct Collapser {
    const std::vector<BNode2> &bin;
    std::vector<BNode4> &out;
    uint32_t inner;      // REF_BLAS_NODE or REF_TLAS_NODE
    const std::vector<NodeInfo> *leaf_info = nullptr;   // top level: an instance leaf's node (for its worst case)
    int max_depth = 0;   // 4-wide levels
    int worst = 0;       // most stack entries any ray can hold below the root: on every path, a
                         // node with n children pushes at most n - 1 (plus, at the top level,
                         // what the entered instance's hierarchy can push)
    std::vector<int> node_worst;   // per node this collapse emitted: out[base + i]
    size_t base = 0;

    int worst_of(uint32_t ref) const {
        if (ref == REF_NONE) return 0;
        if (ref_type(ref) == inner) return node_worst[ref_index(ref) - base];
        if (leaf_info && ref_type(ref) == REF_TLAS_LEAF) return (*leaf_info)[ref_index(ref)].blas_worst;
        return 0;
    }
    uint32_t root(uint32_t ref) {
        base = out.size();
        node_worst.clear();
        const uint32_t r = run(ref, 0);
        worst = worst_of(r);
        return r;
    }

    struct Child {
        uint32_t ref;
        float lo[3], hi[3];
        double area() const {
            double dx = (double)hi[0] - lo[0], dy = (double)hi[1] - lo[1], dz = (double)hi[2] - lo[2];
            return dx * dy + dy * dz + dz * dx;
        }
    };

    uint32_t run(uint32_t ref, int depth) {
        if (ref == REF_NONE || ref_type(ref) != inner) return ref;
        Child ch[4];
        int n = 0;
        auto take = [&](const BNode2 &b, int k) {
            Child c;
            c.ref = b.ref[k];
            for (int a = 0; a < 3; ++a) { c.lo[a] = b.lo[k][a]; c.hi[a] = b.hi[k][a]; }
            return c;
        };
        const BNode2 &b = bin[ref_index(ref)];
        ch[n++] = take(b, 0);
        ch[n++] = take(b, 1);
        while (n < 4) {
            int best = -1;
            double ba = -1;
            for (int k = 0; k < n; ++k)
                if (ch[k].ref != REF_NONE && ref_type(ch[k].ref) == inner && ch[k].area() > ba) {
                    ba = ch[k].area();
                    best = k;
                }
            if (best < 0) break;
            const BNode2 &c = bin[ref_index(ch[best].ref)];
            ch[best] = take(c, 0);
            ch[n++] = take(c, 1);
        }
        const uint32_t me = (uint32_t)out.size();
        BNode4 e;
        for (int k = 0; k < 4; ++k) {
            e.lox[k] = e.loy[k] = e.loz[k] = INFINITY;
            e.hix[k] = e.hiy[k] = e.hiz[k] = INFINITY;
            e.ref[k] = REF_NONE;
            e.pad[k] = 0;
        }
        out.push_back(e);
        node_worst.push_back(0);   // index me - base
        max_depth = std::max(max_depth, depth + 1);
        uint32_t refs[4];
        int below = 0;
        for (int k = 0; k < n; ++k) {
            refs[k] = run(ch[k].ref, depth + 1);
            below = std::max(below, worst_of(refs[k]));
        }
        node_worst[me - base] = n - 1 + below;
        BNode4 &nd = out[me];
        for (int k = 0; k < n; ++k) {
            nd.lox[k] = ch[k].lo[0]; nd.loy[k] = ch[k].lo[1]; nd.loz[k] = ch[k].lo[2];
            nd.hix[k] = ch[k].hi[0]; nd.hiy[k] = ch[k].hi[1]; nd.hiz[k] = ch[k].hi[2];
            nd.ref[k] = refs[k];
        }
        return make_ref(inner, me);
    }
};

// Rotation by the angle of cosine c and sine s about the unit axis u (Rodrigues).
void rot_unit(const double *u, double c, double s, double *R) {
    const double x = u[0], y = u[1], z = u[2], C = 1 - c;
    double M[9] = {c + x * x * C,     x * y * C - z * s, x * z * C + y * s,
                   y * x * C + z * s, c + y * y * C,     y * z * C - x * s,
                   z * x * C - y * s, z * y * C + x * s, c + z * z * C};
    std::memcpy(R, M, sizeof M);
}

void mat3_mul(const double *A, const double *B, double *C) {
    double T[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) T[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
    std::memcpy(C, T, sizeof T);
}

void mat3_vec(const double *A, const double *x, double *y) {
    double t[3];
    for (int i = 0; i < 3; ++i) t[i] = A[3 * i] * x[0] + A[3 * i + 1] * x[1] + A[3 * i + 2] * x[2];
    std::memcpy(y, t, sizeof t);
}

bool finite3(const double *v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

}  // namespace

int validate_materials(const srp_material *mats, int32_t n_mats, std::string *err) {
    if (!mats || n_mats < 1 || n_mats > SRP_MAX_MATS) {
        *err = "materials: need 1.." + std::to_string(SRP_MAX_MATS) + " entries";
        return SRP_ERR_ARG;
    }
    for (int32_t m = 0; m < n_mats; ++m) {
        double s = mats[m].rho_s, d = mats[m].rho_d;
        if (!(s >= 0 && d >= 0 && s + d <= 1.0 + 1e-12) || !std::isfinite(s) || !std::isfinite(d)) {
            *err = "material " + std::to_string(m) + ": need rho_s >= 0, rho_d >= 0, rho_s + rho_d <= 1";
            return SRP_ERR_ARG;
        }
    }
    return SRP_OK;
}

namespace {
int tlas_topology(SceneHost *S, std::string *err);
}

int scene_build(const double *verts, int64_t n_verts, const int32_t *tris, int64_t n_tris,
                const int32_t *tri_material, const int32_t *tri_node, const srp_material *mats,
                int32_t n_mats, const srp_node *nodes, int32_t n_nodes, SceneHost *S,
                std::string *err) {
    if ((n_verts > 0 && !verts) || (n_tris > 0 && (!tris || !tri_material || !tri_node)) || !nodes ||
        n_verts < 0 || n_tris < 0) {
        *err = "srp_build_scene: null or negative-size input";
        return SRP_ERR_ARG;
    }
    if (n_tris >= (int64_t(1) << 27)) { *err = "srp_build_scene: too many triangles"; return SRP_ERR_ARG; }
    if (n_nodes < 1 || n_nodes > SRP_MAX_NODES) {
        *err = "srp_build_scene: need 1.." + std::to_string(SRP_MAX_NODES) + " nodes";
        return SRP_ERR_ARG;
    }
    int rc = validate_materials(mats, n_mats, err);
    if (rc) return rc;
    if (nodes[0].parent != -1 || nodes[0].n_axes != 0) {
        *err = "srp_build_scene: node 0 must be the root (parent -1, no axes)";
        return SRP_ERR_ARG;
    }
    S->nodes.assign(n_nodes, NodeInfo{});
    S->parent.assign(n_nodes, -1);
    int32_t dof = 0;
    for (int32_t k = 0; k < n_nodes; ++k) {
        const srp_node &in = nodes[k];
        NodeInfo &o = S->nodes[k];
        if (k > 0 && (in.parent < 0 || in.parent >= k)) {
            *err = "node " + std::to_string(k) + ": parent must be in [0, k) (single root, topological order)";
            return SRP_ERR_ARG;
        }
        if (in.n_axes < 0 || in.n_axes > 3) { *err = "node " + std::to_string(k) + ": n_axes must be 0..3"; return SRP_ERR_ARG; }
        o.parent = in.parent;
        o.is_panel = in.is_panel;
        o.n_axes = in.n_axes;
        o.dof_offset = dof;
        dof += in.n_axes;
        if (!finite3(in.pivot)) { *err = "node " + std::to_string(k) + ": non-finite pivot"; return SRP_ERR_ARG; }
        std::memcpy(o.pivot, in.pivot, sizeof o.pivot);
        for (int a = 0; a < in.n_axes; ++a) {
            double nrm = std::sqrt(in.axis[a][0] * in.axis[a][0] + in.axis[a][1] * in.axis[a][1] + in.axis[a][2] * in.axis[a][2]);
            if (!(nrm > 0) || !std::isfinite(nrm) || !(in.lo[a] <= in.hi[a]) || !std::isfinite(in.lo[a]) ||
                !std::isfinite(in.hi[a])) {
                *err = "node " + std::to_string(k) + ": invalid axis or interval";
                return SRP_ERR_ARG;
            }
            for (int c = 0; c < 3; ++c) o.axis[a][c] = in.axis[a][c] / nrm;
            const double *ax = o.axis[a];
            const double n2 = std::sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]);
            for (int c = 0; c < 3; ++c) o.unit[a][c] = ax[c] / n2;
            o.lo[a] = in.lo[a];
            o.hi[a] = in.hi[a];
        }
        S->parent[k] = in.parent;
    }
    S->n_nodes = n_nodes;
    S->n_dof = dof;
    S->n_mats = n_mats;
    S->n_tris = n_tris;
    S->mats.resize(2 * n_mats);
    for (int m = 0; m < n_mats; ++m) { S->mats[2 * m] = (float)mats[m].rho_s; S->mats[2 * m + 1] = (float)mats[m].rho_d; }

    // triangles: validate, FP32 records, per-node lists, scene scale
    std::vector<TriRec> rec(n_tris);
    std::vector<std::vector<int32_t>> per_node(n_nodes);
    double scale = 0;
    for (int64_t t = 0; t < n_tris; ++t) {
        for (int c = 0; c < 3; ++c) {
            int32_t vi = tris[3 * t + c];
            if (vi < 0 || vi >= n_verts) { *err = "triangle " + std::to_string(t) + ": vertex index out of range"; return SRP_ERR_ARG; }
            if (!finite3(verts + 3 * (int64_t)vi)) { *err = "non-finite vertex"; return SRP_ERR_ARG; }
        }
        if (tri_material[t] < 0 || tri_material[t] >= n_mats) { *err = "triangle " + std::to_string(t) + ": material out of range"; return SRP_ERR_ARG; }
        if (tri_node[t] < 0 || tri_node[t] >= n_nodes) { *err = "triangle " + std::to_string(t) + ": node out of range"; return SRP_ERR_ARG; }
        TriRec &r = rec[t];
        const double *p0 = verts + 3 * (int64_t)tris[3 * t];
        const double *p1 = verts + 3 * (int64_t)tris[3 * t + 1];
        const double *p2 = verts + 3 * (int64_t)tris[3 * t + 2];
        for (int a = 0; a < 3; ++a) {
            r.v0[a] = (float)p0[a]; r.v1[a] = (float)p1[a]; r.v2[a] = (float)p2[a];
            scale = std::max(scale, std::max(std::fabs(p0[a]), std::max(std::fabs(p1[a]), std::fabs(p2[a]))));
        }
        r.id = (int32_t)t;
        r.mat = tri_material[t];
        r.node = tri_node[t];
        per_node[tri_node[t]].push_back((int32_t)t);
        double e1[3], e2[3];
        for (int a = 0; a < 3; ++a) { e1[a] = p1[a] - p0[a]; e2[a] = p2[a] - p0[a]; }
        double *nn = S->nodes[tri_node[t]].n0;
        nn[0] += e1[1] * e2[2] - e1[2] * e2[1];
        nn[1] += e1[2] * e2[0] - e1[0] * e2[2];
        nn[2] += e1[0] * e2[1] - e1[1] * e2[0];
    }
    S->pad = 4e-6 * scale + 1e-9;
    for (auto &nd : S->nodes) {
        double l = std::sqrt(nd.n0[0] * nd.n0[0] + nd.n0[1] * nd.n0[1] + nd.n0[2] * nd.n0[2]);
        for (int a = 0; a < 3; ++a) nd.n0[a] = l > 0 ? nd.n0[a] / l : 0.0;
    }
    // planar nodes: every vertex of the node's triangles within 1e-9 x scale of
    // the plane through its first vertex with the unit normal n0 (a flat panel
    // segment; a ray leaving such a node cannot meet it again)
    for (int32_t k = 0; k < n_nodes; ++k) {
        NodeInfo &nd = S->nodes[k];
        const auto &lst = per_node[k];
        nd.planar = 0;
        if (lst.empty() || (nd.n0[0] == 0.0 && nd.n0[1] == 0.0 && nd.n0[2] == 0.0)) continue;
        const double *q = verts + 3 * (int64_t)tris[3 * lst[0]];
        double dev = 0.0;
        for (int32_t t : lst)
            for (int c = 0; c < 3; ++c) {
                const double *p = verts + 3 * (int64_t)tris[3 * t + c];
                dev = std::max(dev, std::fabs(nd.n0[0] * (p[0] - q[0]) + nd.n0[1] * (p[1] - q[1]) +
                                              nd.n0[2] * (p[2] - q[2])));
            }
        nd.planar = dev <= 1e-9 * scale ? 1 : 0;
    }

    // one hierarchy per node
    S->tris.clear();
    S->tris.reserve(n_tris);
    S->blas.clear();
    S->max_blas_depth = 0;
    for (int32_t k = 0; k < n_nodes; ++k) {
        NodeInfo &o = S->nodes[k];
        const auto &lst = per_node[k];
        if (lst.empty()) { o.blas_root = REF_NONE; continue; }
        std::vector<Prim> P(lst.size());
        for (size_t i = 0; i < lst.size(); ++i) {
            const TriRec &r = rec[lst[i]];
            Prim &p = P[i];
            for (int a = 0; a < 3; ++a) {
                p.lo[a] = std::min(r.v0[a], std::min(r.v1[a], r.v2[a]));
                p.hi[a] = std::max(r.v0[a], std::max(r.v1[a], r.v2[a]));
                p.c[a] = 0.5f * (p.lo[a] + p.hi[a]);
            }
            p.tri = lst[i];
        }
        std::vector<BNode2> bin;
        BlasBuilder B{P, rec, bin, S->tris, (float)S->pad};
        Box root;
        const uint32_t broot = B.build(0, (int)P.size(), 0, root);
        if (B.depth_error) {
            *err = "node " + std::to_string(k) + ": hierarchy exceeds the traversal stack";
            return SRP_ERR_DEPTH;
        }
        Collapser Cl{bin, S->blas, REF_BLAS_NODE};
        o.blas_root = Cl.root(broot);
        o.blas_depth = Cl.max_depth;
        o.blas_worst = Cl.worst;
        S->max_blas_depth = std::max(S->max_blas_depth, Cl.max_depth);
        if (Cl.worst > STACK_DEPTH) {
            *err = "node " + std::to_string(k) + ": hierarchy exceeds the traversal stack";
            return SRP_ERR_DEPTH;
        }
        for (int a = 0; a < 3; ++a) { o.blo[a] = (double)root.lo[a] - S->pad; o.bhi[a] = (double)root.hi[a] + S->pad; }
    }
    if ((int64_t)S->blas.size() >= (int64_t(1) << 30)) { *err = "srp_build_scene: hierarchy too large"; return SRP_ERR_ARG; }

    // window points: distinct (vertex, node) pairs used by triangles
    std::vector<std::pair<int32_t, int32_t>> vn;
    vn.reserve(3 * n_tris);
    for (int64_t t = 0; t < n_tris; ++t)
        for (int c = 0; c < 3; ++c) vn.emplace_back(tri_node[t], tris[3 * t + c]);
    std::sort(vn.begin(), vn.end());
    vn.erase(std::unique(vn.begin(), vn.end()), vn.end());
    S->wpts.resize(vn.size());
    for (size_t i = 0; i < vn.size(); ++i) {
        const double *p = verts + 3 * (int64_t)vn[i].second;
        S->wpts[i] = WPoint{p[0], p[1], p[2], vn[i].first, 0};
    }
    return tlas_topology(S, err);
}

SlotLayout slot_layout(int n_nodes, int n_tlas, int n_dof) {
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    SlotLayout L;
    L.inst = 0;
    L.tlas = al(L.inst + sizeof(Inst) * (size_t)n_nodes);
    L.xf = al(L.tlas + sizeof(BNode4) * (size_t)std::max(n_tlas, 1));
    L.axw = al(L.xf + sizeof(double) * 12 * (size_t)n_nodes);
    L.dof_node = al(L.axw + sizeof(double) * 3 * (size_t)std::max(n_dof, 1));
    L.bytes = al(L.dof_node + sizeof(int32_t) * (size_t)std::max(n_dof, 1));
    return L;
}

void slot_pack(const SlotHost &s, const SlotLayout &L, char *dst) {
    std::memcpy(dst + L.inst, s.inst.data(), sizeof(Inst) * s.inst.size());
    if (!s.tlas.empty()) std::memcpy(dst + L.tlas, s.tlas.data(), sizeof(BNode4) * s.tlas.size());
    std::memcpy(dst + L.xf, s.xf.data(), sizeof(double) * s.xf.size());
    if (!s.axw.empty()) std::memcpy(dst + L.axw, s.axw.data(), sizeof(double) * s.axw.size());
    if (!s.dof_node.empty()) std::memcpy(dst + L.dof_node, s.dof_node.data(), sizeof(int32_t) * s.dof_node.size());
}

double clamp_angle(const NodeInfo &nd, int a, double th, int *clamped) {
    if (th < nd.lo[a]) { th = nd.lo[a]; ++*clamped; }
    if (th > nd.hi[a]) { th = nd.hi[a]; ++*clamped; }
    return th;
}

std::vector<ArtNode> art_nodes(const SceneHost &S) {
    std::vector<ArtNode> v(S.n_nodes);
    for (int k = 0; k < S.n_nodes; ++k) {
        const NodeInfo &nd = S.nodes[k];
        ArtNode &a = v[k];
        std::memset(&a, 0, sizeof a);
        std::memcpy(a.pivot, nd.pivot, sizeof a.pivot);
        std::memcpy(a.axis, nd.axis, sizeof a.axis);
        std::memcpy(a.unit, nd.unit, sizeof a.unit);
        std::memcpy(a.blo, nd.blo, sizeof a.blo);
        std::memcpy(a.bhi, nd.bhi, sizeof a.bhi);
        a.parent = nd.parent;
        a.n_axes = nd.n_axes;
        a.dof_offset = nd.dof_offset;
        a.blas_root = nd.blas_root;
        a.depth = k == 0 ? 0 : v[nd.parent].depth + 1;   // parents precede their children
    }
    return v;
}

namespace {

// Node transforms, instances and world hinge axes for `angles` (NULL = all
// zero), each angle clamped to its interval.  Node k's transform is its
// parent's times the local x -> R_l (x - p) + p, with R_l the product of the
// axis rotations in axis order.
int slot_compose(const SceneHost &S, const double *angles, SlotHost *out, std::string *err) {
    const int K = S.n_nodes, J = S.n_dof;
    out->inst.assign(K, Inst{});
    out->xf.assign(12 * (size_t)K, 0.0);
    out->axw.assign(3 * (size_t)J, 0.0);
    out->dof_node.assign(J, 0);
    out->n_clamped = 0;
    for (int k = 0; k < K; ++k) {
        const NodeInfo &nd = S.nodes[k];
        double *X = &out->xf[12 * (size_t)k];
        if (k == 0) {
            double I[12] = {1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0};
            std::memcpy(X, I, sizeof I);
        } else {
            const double *Pm = &out->xf[12 * (size_t)nd.parent];
            double prefix[9];
            std::memcpy(prefix, Pm, sizeof prefix);   // R_parent * R(a_0) ... R(a_{j-1})
            double Rl[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
            for (int a = 0; a < nd.n_axes; ++a) {
                int j = nd.dof_offset + a;
                double th = angles ? angles[j] : 0.0;
                if (!std::isfinite(th)) { *err = "non-finite hinge angle"; return SRP_ERR_ARG; }
                th = clamp_angle(nd, a, th, &out->n_clamped);
                mat3_vec(prefix, nd.axis[a], &out->axw[3 * (size_t)j]);
                out->dof_node[j] = k;
                double Ra[9];
                rot_unit(nd.unit[a], std::cos(th), std::sin(th), Ra);
                mat3_mul(Rl, Ra, Rl);
                mat3_mul(prefix, Ra, prefix);
            }
            // local: x -> Rl (x - p) + p ; world: R_par * local + t_par
            double Rp[3], tl[3], tw[3];
            mat3_vec(Rl, nd.pivot, Rp);
            for (int c = 0; c < 3; ++c) tl[c] = nd.pivot[c] - Rp[c];
            mat3_vec(Pm, tl, tw);
            mat3_mul(Pm, Rl, X);
            for (int c = 0; c < 3; ++c) X[9 + c] = tw[c] + Pm[9 + c];
        }
        Inst &I = out->inst[k];
        for (int c = 0; c < 9; ++c) I.R[c] = (float)X[c];
        for (int c = 0; c < 3; ++c) I.t[c] = (float)X[9 + c];
        I.root = nd.blas_root;
        I.node = k;
    }
    return SRP_OK;
}

// World box (FP64) of node nd's padded rest-pose box under transform X: the
// extremes of its eight transformed corners.
void world_box(const NodeInfo &nd, const double *X, double lo[3], double hi[3]) {
    for (int a = 0; a < 3; ++a) { lo[a] = INFINITY; hi[a] = -INFINITY; }
    for (int c = 0; c < 8; ++c) {
        double p[3] = {(c & 1) ? nd.bhi[0] : nd.blo[0], (c & 2) ? nd.bhi[1] : nd.blo[1], (c & 4) ? nd.bhi[2] : nd.blo[2]};
        double w[3];
        mat3_vec(X, p, w);
        for (int a = 0; a < 3; ++a) {
            w[a] += X[9 + a];
            lo[a] = std::min(lo[a], w[a]);
            hi[a] = std::max(hi[a], w[a]);
        }
    }
}

// The instance's top-level box: the world box grown by the padding and
// rounded outward to FP32.
void inst_box(const NodeInfo &nd, const double *X, double pad, float lo[3], float hi[3]) {
    double l[3], h[3];
    world_box(nd, X, l, h);
    for (int a = 0; a < 3; ++a) {
        lo[a] = std::nextafter((float)(l[a] - pad), -INFINITY);
        hi[a] = std::nextafter((float)(h[a] + pad), INFINITY);
    }
}

struct TItem {
    float lo[3], hi[3];
    double c[3];
    int32_t inst;
};

uint32_t tlas_build(std::vector<TItem> &it, int b, int e, std::vector<BNode2> &nodes, int depth, int &maxd,
                    float lo[3], float hi[3]) {
    for (int a = 0; a < 3; ++a) { lo[a] = INFINITY; hi[a] = -INFINITY; }
    for (int k = b; k < e; ++k)
        for (int a = 0; a < 3; ++a) { lo[a] = std::min(lo[a], it[k].lo[a]); hi[a] = std::max(hi[a], it[k].hi[a]); }
    if (e - b == 1) return make_ref(REF_TLAS_LEAF, (uint32_t)it[b].inst);
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int k = b; k < e; ++k)
        for (int a = 0; a < 3; ++a) { clo[a] = std::min(clo[a], it[k].c[a]); chi[a] = std::max(chi[a], it[k].c[a]); }
    int ax = 0;
    for (int a = 1; a < 3; ++a)
        if (chi[a] - clo[a] > chi[ax] - clo[ax]) ax = a;
    int mid = b + (e - b) / 2;
    std::nth_element(it.begin() + b, it.begin() + mid, it.begin() + e, [&](const TItem &x, const TItem &y) {
        return x.c[ax] < y.c[ax] || (x.c[ax] == y.c[ax] && x.inst < y.inst);
    });
    uint32_t me = (uint32_t)nodes.size();
    nodes.push_back(BNode2{});
    maxd = std::max(maxd, depth + 1);
    float llo[3], lhi[3], rlo[3], rhi[3];
    uint32_t l = tlas_build(it, b, mid, nodes, depth + 1, maxd, llo, lhi);
    uint32_t r = tlas_build(it, mid, e, nodes, depth + 1, maxd, rlo, rhi);
    BNode2 &n = nodes[me];
    for (int a = 0; a < 3; ++a) { n.lo[0][a] = llo[a]; n.hi[0][a] = lhi[a]; n.lo[1][a] = rlo[a]; n.hi[1][a] = rhi[a]; }
    n.ref[0] = l;
    n.ref[1] = r;
    return make_ref(REF_TLAS_NODE, me);
}

// The top level over the rest pose: median splits of the non-empty nodes'
// world-box centres along the widest axis, collapsed to 4-wide nodes.  Its
// references are kept for every pose; its stack bound holds for every pose
// (it depends on the references alone).
int tlas_topology(SceneHost *S, std::string *err) {
    SlotHost rest;
    int rc = slot_compose(*S, nullptr, &rest, err);
    if (rc) return rc;
    std::vector<TItem> items;
    for (int k = 0; k < S->n_nodes; ++k) {
        const NodeInfo &nd = S->nodes[k];
        if (nd.blas_root == REF_NONE) continue;
        const double *X = &rest.xf[12 * (size_t)k];
        double lo[3], hi[3];
        world_box(nd, X, lo, hi);
        TItem ti;
        inst_box(nd, X, S->pad, ti.lo, ti.hi);
        for (int a = 0; a < 3; ++a) ti.c[a] = 0.5 * (lo[a] + hi[a]);
        ti.inst = k;
        items.push_back(ti);
    }
    S->tlas_topo.clear();
    S->tlas_root = REF_NONE;
    S->tlas_depth = 0;
    S->stack_worst = 0;
    if (!items.empty()) {
        float lo[3], hi[3];
        std::vector<BNode2> bin;
        int bdepth = 0;
        const uint32_t broot = tlas_build(items, 0, (int)items.size(), bin, 0, bdepth, lo, hi);
        Collapser Cl{bin, S->tlas_topo, REF_TLAS_NODE};
        Cl.leaf_info = &S->nodes;
        S->tlas_root = Cl.root(broot);
        S->tlas_depth = Cl.max_depth;
        S->stack_worst = Cl.worst;
    }
    if (S->stack_worst > STACK_DEPTH) {
        *err = "hierarchy depth exceeds the traversal stack";
        return SRP_ERR_DEPTH;
    }
    if (S->tlas_topo.size() > (size_t)SRP_MAX_NODES) {   // (at most 127 for 128 instances)
        *err = "top level: too many nodes";
        return SRP_ERR_ARG;
    }
    // the refit visits nodes last to first: every child must follow its parent
    for (size_t i = 0; i < S->tlas_topo.size(); ++i)
        for (int k = 0; k < 4; ++k) {
            const uint32_t r = S->tlas_topo[i].ref[k];
            if (r != REF_NONE && ref_type(r) == REF_TLAS_NODE && ref_index(r) <= i) {
                *err = "top level: a child precedes its parent";
                return SRP_ERR_ARG;
            }
        }
    // each node's height (inner-node levels below it) in pad[0]: the device refit
    // runs level by level from height 0 up
    S->tlas_max_height = 0;
    for (size_t i = S->tlas_topo.size(); i-- > 0;) {
        BNode4 &nd = S->tlas_topo[i];
        uint32_t hgt = 0;
        for (int k = 0; k < 4; ++k) {
            const uint32_t r = nd.ref[k];
            if (r != REF_NONE && ref_type(r) == REF_TLAS_NODE)
                hgt = std::max(hgt, S->tlas_topo[ref_index(r)].pad[0] + 1);
        }
        nd.pad[0] = hgt;
        S->tlas_max_height = std::max(S->tlas_max_height, (int)hgt);
    }
    S->tree_max_depth = 0;
    {
        std::vector<int> depth(S->n_nodes, 0);
        for (int k = 1; k < S->n_nodes; ++k) {
            depth[k] = depth[S->nodes[k].parent] + 1;
            S->tree_max_depth = std::max(S->tree_max_depth, depth[k]);
        }
    }
    return SRP_OK;
}

}  // namespace

int slot_build(const SceneHost &S, const double *angles, SlotHost *out, std::string *err) {
    int rc = slot_compose(S, angles, out, err);
    if (rc) return rc;
    // refit the top level, children before parents: an instance leaf takes its
    // world box, an inner child the union of its node's non-empty boxes
    out->tlas = S.tlas_topo;
    for (size_t i = out->tlas.size(); i-- > 0;) {
        BNode4 &nd = out->tlas[i];
        for (int k = 0; k < 4; ++k) {
            const uint32_t r = nd.ref[k];
            if (r == REF_NONE) continue;
            float lo[3], hi[3];
            if (ref_type(r) == REF_TLAS_LEAF) {
                const uint32_t q = ref_index(r);
                inst_box(S.nodes[q], &out->xf[12 * (size_t)q], S.pad, lo, hi);
            } else {
                const BNode4 &c = out->tlas[ref_index(r)];
                for (int a = 0; a < 3; ++a) { lo[a] = INFINITY; hi[a] = -INFINITY; }
                for (int m = 0; m < 4; ++m) {
                    if (c.ref[m] == REF_NONE) continue;
                    lo[0] = std::min(lo[0], c.lox[m]); hi[0] = std::max(hi[0], c.hix[m]);
                    lo[1] = std::min(lo[1], c.loy[m]); hi[1] = std::max(hi[1], c.hiy[m]);
                    lo[2] = std::min(lo[2], c.loz[m]); hi[2] = std::max(hi[2], c.hiz[m]);
                }
            }
            nd.lox[k] = lo[0]; nd.loy[k] = lo[1]; nd.loz[k] = lo[2];
            nd.hix[k] = hi[0]; nd.hiy[k] = hi[1]; nd.hiz[k] = hi[2];
        }
    }
    out->root_ref = S.tlas_root;
    out->tlas_depth = S.tlas_depth;
    out->stack_worst = S.stack_worst;
    return SRP_OK;
}

}  // namespace srp
