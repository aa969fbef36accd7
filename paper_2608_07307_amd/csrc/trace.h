// Ray traversal and intersection shared by the gfx950 kernels and a host
// build of the same code (used to check the traversal on the CPU).
//
// trace_closest: closest hit of one ray in a two-level hierarchy (top level
// over the kinematic-tree nodes in world coordinates; per node a bottom level
// in rest-pose coordinates entered through the node's rigid transform, which
// preserves the ray parameter t), with a per-lane traversal stack (LaneStack).
#pragma once
#include <math.h>
#include <stdint.h>

#include "srp_internal.h"

namespace srp {

constexpr float T_INF = 3.0e38f;

// Reciprocal for the ray-frame constants and the hit distance: on the GPU the
// single-instruction hardware approximation (within 1 ulp; an IEEE division
// costs a dozen instructions), in a host build of this code a division.  The
// hierarchy's boxes are padded far beyond the resulting rounding of entry and
// exit distances, and one frame serves every triangle of an instance, so the
// triangle test stays watertight.
SRP_HD inline float frame_rcp(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}

SRP_HD inline float safe_inv(float x) {
    // reciprocal of a direction component, finite for zero components
    float ax = fabsf(x) < 1e-30f ? copysignf(1e-30f, x) : x;
    return frame_rcp(ax);
}

// An orthonormal basis (bx, by) orthogonal to unit d (Duff et al., JCGT 2017).
SRP_HD inline void onb(const float d[3], float bx[3], float by[3]) {
    float s = copysignf(1.0f, d[2]);
    float a = -frame_rcp(s + d[2]);
    float b = d[0] * d[1] * a;
    bx[0] = 1.0f + s * d[0] * d[0] * a;
    bx[1] = s * b;
    bx[2] = -s * d[0];
    by[0] = b;
    by[1] = s + d[1] * d[1] * a;
    by[2] = -d[1];
}

// Ray state in one frame: slab-test constants and the watertight-test frame
// (x, y axes orthogonal to the direction, z = direction, offsets = axes . o).
struct Frame {
    float ix, iy, iz;      // 1 / d
    float oix, oiy, oiz;   // o / d
    float mx[3], my[3], mz[3];
    float cx, cy, cz;
    int nx, ny, nz;        // float4 index of the near-plane array per axis in a node
};

// Near-plane arrays of a 4-wide node for a direction with inverse (ix, iy, iz):
// lo (0, 1, 2) where the component is positive, hi (3, 4, 5) where negative;
// the far plane's index is the near one's XOR 3, 5, 7.  With lo <= hi and a
// monotone rounded fma, the near plane gives min(t_lo, t_hi) exactly.
SRP_HD inline void near_planes(float ix, float iy, float iz, int &nx, int &ny, int &nz) {
    nx = ix < 0.0f ? 3 : 0;
    ny = iy < 0.0f ? 4 : 1;
    nz = iz < 0.0f ? 5 : 2;
}

SRP_HD inline void frame_setup(const float o[3], const float d[3], Frame &F) {
    F.ix = safe_inv(d[0]);
    F.iy = safe_inv(d[1]);
    F.iz = safe_inv(d[2]);
    F.oix = o[0] * F.ix;
    F.oiy = o[1] * F.iy;
    F.oiz = o[2] * F.iz;
    near_planes(F.ix, F.iy, F.iz, F.nx, F.ny, F.nz);
    onb(d, F.mx, F.my);
    F.mz[0] = d[0]; F.mz[1] = d[1]; F.mz[2] = d[2];
    F.cx = F.mx[0] * o[0] + F.mx[1] * o[1] + F.mx[2] * o[2];
    F.cy = F.my[0] * o[0] + F.my[1] * o[1] + F.my[2] * o[2];
    F.cz = F.mz[0] * o[0] + F.mz[1] * o[1] + F.mz[2] * o[2];
}

// Slab test of one box against [tmin, tmax] with its planes already ordered
// per axis (near, far): returns 1 when the ray enters the box, with t = the
// entry distance (at most tmax, which never exceeds T_INF), else 0 with
// t = +infinity, so that sorting puts every entered child before every other.
// (A node visit counts its hit children from these flags, so the compiler
// needs the full sort of the children only when a lane has two or more.)
SRP_HD inline int box_enter(float nx, float ny, float nz, float fx, float fy, float fz,
                            float ix, float iy, float iz, float oix, float oiy, float oiz,
                            float tmin, float tmax, float &t) {
    float tn = fmaxf(fmaxf(fmaf(nx, ix, -oix), fmaf(ny, iy, -oiy)), fmaxf(fmaf(nz, iz, -oiz), tmin));
    float tf = fminf(fminf(fmaf(fx, ix, -oix), fmaf(fy, iy, -oiy)), fminf(fmaf(fz, iz, -oiz), tmax));
    const bool in = tn <= tf;
    t = in ? tn : INFINITY;
    return in ? 1 : 0;
}

SRP_HD inline float xf_dot(const float m[3], float c, const float v[3]) {
    return fmaf(m[0], v[0], fmaf(m[1], v[1], fmaf(m[2], v[2], -c)));
}

// Watertight ray/triangle test in the ray frame: 2-D edge functions of the
// projected corners (products rounded separately, so a shared edge gets the
// exact negated value in both triangles: no ray passes between them), then
// the hit distance.  Returns t or a negative value for a miss.
SRP_HD inline float tri_hit(const Frame &F, const float a[3], const float b[3], const float c[3]) {
#pragma clang fp contract(off)
    float ax = xf_dot(F.mx, F.cx, a), ay = xf_dot(F.my, F.cy, a);
    float bx = xf_dot(F.mx, F.cx, b), by = xf_dot(F.my, F.cy, b);
    float cx = xf_dot(F.mx, F.cx, c), cy = xf_dot(F.my, F.cy, c);
    float U = cx * by - cy * bx;
    float V = ax * cy - ay * cx;
    float W = bx * ay - by * ax;
    float mn = fminf(fminf(U, V), W), mx = fmaxf(fmaxf(U, V), W);
    if (mn < 0.0f && mx > 0.0f) return -1.0f;
    float det = U + V + W;
    if (det == 0.0f) return -1.0f;
    float az = xf_dot(F.mz, F.cz, a), bz = xf_dot(F.mz, F.cz, b), cz = xf_dot(F.mz, F.cz, c);
    float T = U * az + V * bz + W * cz;
    return T * frame_rcp(det);
}

SRP_HD inline int32_t f2i(float x) {
    union { float f; int32_t i; } u;
    u.f = x;
    return u.i;
}

struct Hit {
    float t;
    int32_t tri;    // leaf-order index into the scene's triangle records
    int32_t inst;
    int32_t id;     // original triangle index
};

// Hard bound on the nodes and leaves one ray may visit: far above what any
// hierarchy accepted by the builder needs (each node is visited at most once),
// so reaching it means corrupted data and the ray reports an error instead of
// looping.
constexpr uint32_t MAX_VISITS = 1u << 22;

// Device loads through these pointers are global-memory loads (the pointers
// come from a descriptor in memory, which would otherwise make them generic).
#if defined(__HIP_DEVICE_COMPILE__)
#define SRP_GLOBAL __attribute__((address_space(1)))
#else
#define SRP_GLOBAL
#endif

// What one traversal needs from an evaluation's descriptor, held in registers.
struct TraceCtx {
    const BNode4 SRP_GLOBAL *blas;
    const BNode4 SRP_GLOBAL *tlas;
    const TriRec SRP_GLOBAL *tris;
    const Inst SRP_GLOBAL *inst;
    uint32_t root;
};

SRP_HD inline TraceCtx trace_ctx(const EvalDesc &D) {
    TraceCtx c;
    c.blas = (const BNode4 SRP_GLOBAL *)D.blas;
    c.tlas = (const BNode4 SRP_GLOBAL *)D.tlas;
    c.tris = (const TriRec SRP_GLOBAL *)D.tris;
    c.inst = (const Inst SRP_GLOBAL *)D.inst;
    c.root = D.root_ref;
    return c;
}

// Orders (t[i], r[i]) so that t[i] <= t[j] for i < j (five compare-exchanges).
SRP_HD inline void sort4(float t[4], uint32_t r[4]) {
    auto cx = [&](int i, int j) {
        const bool sw = t[j] < t[i];
        const float ti = sw ? t[j] : t[i], tj = sw ? t[i] : t[j];
        const uint32_t ri = sw ? r[j] : r[i], rj = sw ? r[i] : r[j];
        t[i] = ti; t[j] = tj; r[i] = ri; r[j] = rj;
    };
    cx(0, 1); cx(2, 3); cx(0, 2); cx(1, 3); cx(1, 2);
}

// Per-lane traversal stack of up to STACK_DEPTH entries.  The newest entry
// is held in a register (`top`); below it the next STACK_LDS entries sit in a
// ring (entry s in slot s mod STACK_LDS, slots `stride` words apart, in LDS on
// the GPU), and pushing past that evicts the oldest ring entry to the lane's
// spill array (entry e at spill[e * sstride], global memory on the GPU) while
// popping brings it back.  A pop therefore never waits for memory: the ring
// read that refills `top` is needed only by the next pop.  Rays rarely hold
// more than a handful of entries, so the spill path is almost never taken,
// but any hierarchy the builder accepts still traverses exactly.
struct LaneStack {
    uint32_t *ring;
    int stride;
    uint32_t SRP_GLOBAL *spill;
    int sstride;
};

// Entry e (0-based from the bottom) of the ring/spill part.  e = -1 is the
// slot below the bottom: storing or loading it touches ring slot
// STACK_LDS - 1, which holds no live entry while the stack is that short, so
// callers need not test for an empty stack.
SRP_HD inline void st_store(const LaneStack &S, int e, uint32_t v) {
    const int slot = (e & (STACK_LDS - 1)) * S.stride;
    if (e >= STACK_LDS) S.spill[(e - STACK_LDS) * S.sstride] = S.ring[slot];
    S.ring[slot] = v;
}
SRP_HD inline uint32_t st_load(const LaneStack &S, int e) {
    // entry e is the newest of the ring part: read it, then refill its slot
    // with the entry STACK_LDS below it if that one was spilled
    const int slot = (e & (STACK_LDS - 1)) * S.stride;
    const uint32_t v = S.ring[slot];
    if (e >= STACK_LDS) S.ring[slot] = S.spill[(e - STACK_LDS) * S.sstride];
    return v;
}

// Closest hit along o + t d, t > tmin, skipping triangle `exclude_id` and,
// when skip_inst >= 0, the whole instance skip_inst.  A caller passes the
// instance a ray leaves when every triangle of that instance lies in one
// plane: the ray then has a nonzero component along the plane's normal, so
// no point of it beyond its origin lies in that plane and the instance holds
// no hit for it (the first hit is the same as without the skip, up to the
// rounding of a grazing ray's origin).
// Both levels are 4-wide: a node visit tests the four child boxes, descends
// into the nearest hit child and pushes the other hit children far to near.
// Top-level nodes are tested in the world frame; a top-level leaf enters its
// instance (the ray in the node's rest-pose frame; t is preserved) and the
// instance's bottom-level nodes are tested in that frame.  One stack holds
// both kinds of reference, so a popped reference's type says which frame it
// belongs to and leaving an instance needs no bookkeeping.  The loop is
// "descend, then test leaves": every lane steps through inner nodes and
// instance entries until it holds a leaf (or is done), then the lanes test
// their leaves together; lanes in different instances advance in the same
// steps.  The descent loop has a single exit (stack overflow and the visit
// bound are reported after it).  Returns false only when the stack or the
// visit bound is exceeded (corrupted data).
// (steps, deepest: optional instrumentation of a host build, the node and
// leaf visits and the most entries the stack held.)
template <bool COUNT>
SRP_HD inline bool trace_closest(const TraceCtx &C, const float o[3], const float d[3], float tmin,
                                 int32_t exclude_id, int32_t skip_inst, const LaneStack &stack, Hit &h,
                                 uint32_t &nbox, uint32_t &ntri, uint32_t *steps = nullptr,
                                 int *deepest = nullptr) {
    h.t = T_INF;
    h.tri = -1;
    h.inst = -1;
    h.id = 0x7FFFFFFF;
    if (C.root == REF_NONE) return true;
    const float wix = safe_inv(d[0]), wiy = safe_inv(d[1]), wiz = safe_inv(d[2]);
    const float woix = o[0] * wix, woiy = o[1] * wiy, woiz = o[2] * wiz;
    // The level being traversed: its box-test constants (F.ix .. F.oiz) and its
    // node array.  Entering an instance switches to the instance's frame and
    // the bottom-level nodes; popping a top-level node switches back.  (Entries
    // of the bottom level on the stack always belong to the current instance,
    // so those are the only transitions.)
    Frame F;
    F.ix = wix; F.iy = wiy; F.iz = wiz;
    F.oix = woix; F.oiy = woiy; F.oiz = woiz;
    near_planes(wix, wiy, wiz, F.nx, F.ny, F.nz);
    const BNode4 SRP_GLOBAL *nodes = C.tlas;
    int inst = -1;
    uint32_t visits = 0;
    bool overflow = false;
    int sp = 0;              // entries on the stack; the newest is `top`
    uint32_t top = REF_NONE;
    uint32_t ref = C.root;
    for (;;) {
        // ---- descend: inner nodes of either level and instance entries
        while (ref_type(ref) != REF_BLAS_LEAF && ref != REF_NONE && visits < MAX_VISITS) {
            ++visits;
            if (steps) ++*steps;
            if (ref_type(ref) == REF_TLAS_LEAF) {
              inst = (int)ref_index(ref);
              if (inst == skip_inst) {
                // the instance the ray leaves (planar): nothing to enter; the next
                // entry is popped (always a top-level one: this leaf was on the
                // top level, so the stack holds no bottom-level entries)
                if (sp > 0) {
                    ref = top;
                    --sp;
                    top = st_load(stack, sp - 1);
                } else {
                    ref = REF_NONE;
                }
              } else {
                // enter the instance: the ray in the node's rest-pose frame
                const Inst SRP_GLOBAL &I = C.inst[inst];
                float lo[3], ld[3];
                const float r0 = o[0] - I.t[0], r1 = o[1] - I.t[1], r2 = o[2] - I.t[2];
                lo[0] = I.R[0] * r0 + I.R[3] * r1 + I.R[6] * r2;
                lo[1] = I.R[1] * r0 + I.R[4] * r1 + I.R[7] * r2;
                lo[2] = I.R[2] * r0 + I.R[5] * r1 + I.R[8] * r2;
                ld[0] = I.R[0] * d[0] + I.R[3] * d[1] + I.R[6] * d[2];
                ld[1] = I.R[1] * d[0] + I.R[4] * d[1] + I.R[7] * d[2];
                ld[2] = I.R[2] * d[0] + I.R[5] * d[1] + I.R[8] * d[2];
                frame_setup(lo, ld, F);
                nodes = C.blas;
                ref = I.root;
              }
            } else {
                const float4 SRP_GLOBAL *q = (const float4 SRP_GLOBAL *)(nodes + ref_index(ref));
                const float4 NX = q[F.nx], NY = q[F.ny], NZ = q[F.nz];
                const float4 FX = q[F.nx ^ 3], FY = q[F.ny ^ 5], FZ = q[F.nz ^ 7];
                const uint4 NR = ((const uint4 SRP_GLOBAL *)q)[6];
                const float ix = F.ix, iy = F.iy, iz = F.iz, oix = F.oix, oiy = F.oiy, oiz = F.oiz;
                float t[4];
                const int hits = box_enter(NX.x, NY.x, NZ.x, FX.x, FY.x, FZ.x, ix, iy, iz, oix, oiy, oiz, tmin, h.t, t[0]) +
                                 box_enter(NX.y, NY.y, NZ.y, FX.y, FY.y, FZ.y, ix, iy, iz, oix, oiy, oiz, tmin, h.t, t[1]) +
                                 box_enter(NX.z, NY.z, NZ.z, FX.z, FY.z, FZ.z, ix, iy, iz, oix, oiy, oiz, tmin, h.t, t[2]) +
                                 box_enter(NX.w, NY.w, NZ.w, FX.w, FY.w, FZ.w, ix, iy, iz, oix, oiy, oiz, tmin, h.t, t[3]);
                uint32_t r[4] = {NR.x, NR.y, NR.z, NR.w};
                if (COUNT) nbox += (r[0] != REF_NONE) + (r[1] != REF_NONE) + (r[2] != REF_NONE) + (r[3] != REF_NONE);
                sort4(t, r);   // the hit children first, nearest first
                if (hits > 1) {
                    // push the other hit children far to near: afterwards the ring holds
                    // ..., old top (entry sp - 1), r[np], ..., r[2] and r[1] is the top
                    const int np = hits - 1;
                    if (sp + np > STACK_DEPTH) {
                        overflow = true;
                    } else if (sp + 2 < STACK_LDS) {
                        // nothing reaches the spill part: three fixed-slot stores (the ones
                        // past the new top write free slots)
                        const int m = STACK_LDS - 1;
                        stack.ring[((sp - 1) & m) * stack.stride] = top;
                        stack.ring[(sp & m) * stack.stride] = np == 3 ? r[3] : r[2];
                        stack.ring[((sp + 1) & m) * stack.stride] = r[2];
                        top = r[1];
                        sp += np;
                    } else {
                        for (int k = np; k >= 1; --k) {
                            st_store(stack, sp - 1, top);
                            top = r[k];
                            ++sp;
                        }
                    }
                }
                if (deepest && sp > *deepest) *deepest = sp;
                if (hits > 0) {
                    ref = r[0];   // descend into the nearest
                } else if (sp > 0) {
                    ref = top;
                    --sp;
                    top = st_load(stack, sp - 1);
                    if (ref_type(ref) == REF_TLAS_NODE) {
                        F.ix = wix; F.iy = wiy; F.iz = wiz;
                        F.oix = woix; F.oiy = woiy; F.oiz = woiz;
                        near_planes(wix, wiy, wiz, F.nx, F.ny, F.nz);
                        nodes = C.tlas;
                    }
                } else {
                    ref = REF_NONE;
                }
            }
        }
        if (overflow || visits >= MAX_VISITS) return false;
        if (ref == REF_NONE) return true;
        // ---- leaf: test its triangles (in the current instance's frame)
        ++visits;
        if (steps) ++*steps;
        const uint32_t p = ref_index(ref);
        const uint32_t first = p >> 3, cnt = (p & 7u) + 1u;
        for (uint32_t k = 0; k < cnt; ++k) {
            const float4 SRP_GLOBAL *q = (const float4 SRP_GLOBAL *)(C.tris + first + k);
            const float4 A = q[0], B = q[1], Cc = q[2];
            const int32_t id = f2i(A.w);
            if (COUNT) ntri++;
            // the excluded triangle is tested too and rejected here: skipping it
            // before the test would hold the third corner's load back until the
            // id had arrived (two memory round trips per triangle instead of one)
            const float va[3] = {A.x, A.y, A.z}, vb[3] = {B.x, B.y, B.z}, vc[3] = {Cc.x, Cc.y, Cc.z};
            const float t = tri_hit(F, va, vb, vc);
            if (id != exclude_id && t > tmin && (t < h.t || (t == h.t && id < h.id))) {
                h.t = t;
                h.tri = (int32_t)(first + k);
                h.inst = inst;
                h.id = id;
            }
        }
        if (sp > 0) {
            ref = top;
            --sp;
            top = st_load(stack, sp - 1);
            if (ref_type(ref) == REF_TLAS_NODE) {
                F.ix = wix; F.iy = wiy; F.iz = wiz;
                F.oix = woix; F.oiy = woiy; F.oiz = woiz;
                near_planes(wix, wiy, wiz, F.nx, F.ny, F.nz);
                nodes = C.tlas;
            }
        } else {
            ref = REF_NONE;
        }
    }
}
}  // namespace srp
