// Host build of the library's ray traversal (csrc/trace.h) for a CPU check
// under AddressSanitizer and UndefinedBehaviorSanitizer: the scene and its
// articulation slot are built by the library's own host code (csrc/scene.cpp),
// the per-lane stack is a ring of exactly SRP_STACK_LDS entries plus a spill
// array of exactly STACK_DEPTH - SRP_STACK_LDS entries (so any access outside
// them is reported), and every ray is traced one at a time.
//
//   trace_check <input> <output>
//
// Input (little-endian, written by tests/test_trace_host.py):
//   int64 nv, nt; int32 nm, nn, n_dof, n_rays
//   f64 verts[nv][3]; i32 tris[nt][3]; i32 tri_mat[nt]; i32 tri_node[nt]
//   srp_material mats[nm]; srp_node nodes[nn]; f64 angles[n_dof]
//   per ray: f32 o[3], d[3], tmin; i32 exclude (original triangle id or -1);
//   i32 skip (the instance the ray leaves, skipped whole, or -1)
// Output: int32 status (0, or the library's error code), int32 stack_worst
// (the builder's bound for this slot), int32 n_nodes, int32 planar[n_nodes]
// (the builder's flag: every triangle of the node in one plane), then per ray:
//   i32 ok (1, or 0 when trace_closest reported an overflow), i32 id (-1 =
//   miss), f32 t, u32 box tests, u32 triangle tests, i32 deepest stack.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "host.h"
#include "trace.h"

using namespace srp;

namespace {

template <class T>
bool rd(FILE *f, T *p, size_t n) {
    return n == 0 || fread(p, sizeof(T), n, f) == n;
}

struct Ray {
    float o[3], d[3], tmin;
    int32_t exclude, skip;
};

}  // namespace

int main(int argc, char **argv) {
    if (argc != 3) {
        fprintf(stderr, "usage: trace_check <input> <output>\n");
        return 2;
    }
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t nv = 0, nt = 0;
    int32_t nm = 0, nn = 0, n_dof = 0, n_rays = 0;
    if (!rd(f, &nv, 1) || !rd(f, &nt, 1) || !rd(f, &nm, 1) || !rd(f, &nn, 1) || !rd(f, &n_dof, 1) ||
        !rd(f, &n_rays, 1))
        return 3;
    std::vector<double> verts(3 * nv), angles(n_dof);
    std::vector<int32_t> tris(3 * nt), tmat(nt), tnode(nt);
    std::vector<srp_material> mats(nm);
    std::vector<srp_node> nodes(nn);
    std::vector<Ray> rays(n_rays);
    if (!rd(f, verts.data(), verts.size()) || !rd(f, tris.data(), tris.size()) || !rd(f, tmat.data(), tmat.size()) ||
        !rd(f, tnode.data(), tnode.size()) || !rd(f, mats.data(), mats.size()) || !rd(f, nodes.data(), nodes.size()) ||
        !rd(f, angles.data(), angles.size()) || !rd(f, rays.data(), rays.size()))
        return 3;
    fclose(f);

    FILE *g = fopen(argv[2], "wb");
    if (!g) return 2;
    SceneHost S;
    SlotHost slot;
    std::string err;
    int32_t status = scene_build(verts.data(), nv, tris.data(), nt, tmat.data(), tnode.data(), mats.data(), nm,
                                 nodes.data(), nn, &S, &err);
    if (!status) status = slot_build(S, n_dof ? angles.data() : nullptr, &slot, &err);
    int32_t worst = slot.stack_worst;
    fwrite(&status, sizeof status, 1, g);
    fwrite(&worst, sizeof worst, 1, g);
    fwrite(&nn, sizeof nn, 1, g);
    for (int32_t k = 0; k < nn; ++k) {
        const int32_t pl = (!status && k < (int32_t)S.nodes.size()) ? S.nodes[k].planar : 0;
        fwrite(&pl, sizeof pl, 1, g);
    }
    if (status) {
        fprintf(stderr, "scene: %s\n", err.c_str());
        fclose(g);
        return 0;
    }
    TraceCtx C;
    C.blas = S.blas.data();
    C.tlas = slot.tlas.data();
    C.tris = S.tris.data();
    C.inst = slot.inst.data();
    C.root = slot.root_ref;
    // the ring and the spill array at exactly their sizes (heap, so that the
    // sanitizer sees their bounds)
    std::vector<uint32_t> ring(STACK_LDS), spill(STACK_DEPTH - STACK_LDS);
    LaneStack st;
    st.ring = ring.data();
    st.stride = 1;
    st.spill = spill.data();
    st.sstride = 1;
    for (const Ray &r : rays) {
        Hit h;
        uint32_t nbox = 0, ntri = 0;
        int deepest = 0;
        const bool ok = trace_closest<true>(C, r.o, r.d, r.tmin, r.exclude, r.skip, st, h, nbox, ntri, nullptr, &deepest);
        const int32_t rec[2] = {ok ? 1 : 0, h.tri >= 0 ? h.id : -1};
        const float t = h.tri >= 0 ? h.t : 0.0f;
        const uint32_t cnt[2] = {nbox, ntri};
        fwrite(rec, sizeof rec, 1, g);
        fwrite(&t, sizeof t, 1, g);
        fwrite(cnt, sizeof cnt, 1, g);
        fwrite(&deepest, sizeof deepest, 1, g);
    }
    fclose(g);
    return 0;
}
