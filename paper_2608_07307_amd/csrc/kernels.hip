// gfx950 kernels of the ray-traced SRP library.
//
//   k_window  per evaluation, the tight projected window of the articulated
//             mesh (FP64 bounds of every (vertex, node) point on the image
//             axes u, v and the photon direction d), merged across blocks with
//             order-preserving 64-bit atomic min.
//   k_trace   persistent: every wave takes chunks (runs of 8x8-pixel patches
//             of one evaluation) from per-XCD work queues until none is left,
//             with no block barrier; one ray per lane; two-level traversal (top level over
//             the kinematic-tree nodes, rigid instance transform, bottom level
//             in rest-pose coordinates) with a per-lane stack (LDS ring, global
//             spill); watertight FP32 triangle test; momentum law at each hit;
//             specular secondary rays iteratively; FP64 per-lane sums, a wave
//             reduction, one partial per patch (no floating-point atomics, so
//             results do not depend on scheduling).  With diffuse rays a chain
//             hit that emits a fan writes an emitter record; for big batches
//             the kernel then traces the patch's fan passes itself.  The GRAD
//             variant also differentiates each ray's hit chain at fixed
//             visibility.
//   k_fans    small diffuse batches: the patches' fan passes as a separate
//             persistent launch, each patch split into several work units.
//   k_slices  one block per range sum (up to 16 per evaluation, numbered
//             through the batch), summing a contiguous range of its evaluation's
//             patch, fan-pass and gradient partials in a fixed order.
//   k_reduce  per evaluation, adds the ranges in order, scales by P * A_pix and
//             writes the srp_result (and assembles the gradients).
//
// The per-pixel structure, the iterative secondary rays and the GPU-side
// reduction follow Sec. 4.3 of the paper; the articulation follows Sec. 4.4.
#include <float.h>

#include "srp.h"
#include "srp_internal.h"
#include "trace.h"

namespace srp {

namespace {

constexpr int WAVE = 64;
constexpr int HWREG_XCC_ID = 20;   // hardware register holding the wave's XCD (accelerator complex die)

// Occupancy targets of the trace kernels (waves per SIMD): the register
// budget the compiler keeps to.
#ifndef SRP_WPE_FWD
#define SRP_WPE_FWD 4
#endif
#ifndef SRP_WPE_GRAD
#define SRP_WPE_GRAD 4
#endif
constexpr int MAX_CHAIN = SRP_MAX_BOUNCES + 1;

// x from another lane of the same 16-lane row (data-parallel primitive move,
// one per 32-bit half).  Every lane of the wave must be active.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double readlane_f64(double x, int lane) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), lane),
                            __builtin_amdgcn_readlane(__double2loint(x), lane));
}

// Wave-wide sum, OR and maximum of 32-bit integers, returned to every lane
// (quads, then rows by rotation, then the rows' first lanes).  Every lane of
// the wave must be active.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t rows_u32(uint32_t x, int k) {
    return (uint32_t)__builtin_amdgcn_readlane((int)x, k);
}
__device__ __forceinline__ uint32_t wave_add_u32(uint32_t x) {
    x += dpp_u32<0xB1>(x);
    x += dpp_u32<0x4E>(x);
    x += dpp_u32<0x124>(x);
    x += dpp_u32<0x128>(x);
    return rows_u32(x, 0) + rows_u32(x, 16) + rows_u32(x, 32) + rows_u32(x, 48);
}
__device__ __forceinline__ uint32_t wave_or_u32(uint32_t x) {
    x |= dpp_u32<0xB1>(x);
    x |= dpp_u32<0x4E>(x);
    x |= dpp_u32<0x124>(x);
    x |= dpp_u32<0x128>(x);
    return rows_u32(x, 0) | rows_u32(x, 16) | rows_u32(x, 32) | rows_u32(x, 48);
}
__device__ __forceinline__ int wave_max_i32(int x) {
    x = max(x, (int)dpp_u32<0xB1>((uint32_t)x));
    x = max(x, (int)dpp_u32<0x4E>((uint32_t)x));
    x = max(x, (int)dpp_u32<0x124>((uint32_t)x));
    x = max(x, (int)dpp_u32<0x128>((uint32_t)x));
    return max(max((int)rows_u32((uint32_t)x, 0), (int)rows_u32((uint32_t)x, 16)),
               max((int)rows_u32((uint32_t)x, 32), (int)rows_u32((uint32_t)x, 48)));
}

// The FP32 sum of x over the wave's 64 lanes, returned to every lane, in the
// same fixed order as wave_sum.  Every lane of the wave must be active.
__device__ __forceinline__ float wave_sum_f32(float x) {
    x += __int_as_float((int)dpp_u32<0xB1>((uint32_t)__float_as_int(x)));
    x += __int_as_float((int)dpp_u32<0x4E>((uint32_t)__float_as_int(x)));
    x += __int_as_float((int)dpp_u32<0x124>((uint32_t)__float_as_int(x)));
    x += __int_as_float((int)dpp_u32<0x128>((uint32_t)__float_as_int(x)));
    const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 0));
    const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 16));
    const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 32));
    const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 48));
    return (r0 + r1) + (r2 + r3);
}

// The sum of x over the wave's 64 lanes, returned to every lane, in a fixed
// order: quads (lane ^ 1, then lane ^ 2), the four quads of each row (row
// rotations by 4 and 8), then the four rows' totals as read from their first
// lanes, ((r0 + r1) + (r2 + r3)).  Every lane of the wave must be active.
__device__ __forceinline__ double wave_sum(double x) {
    x += dpp_f64<0xB1>(x);    // quad_perm (1, 0, 3, 2)
    x += dpp_f64<0x4E>(x);    // quad_perm (2, 3, 0, 1)
    x += dpp_f64<0x124>(x);   // row_ror 4
    x += dpp_f64<0x128>(x);   // row_ror 8
    return (readlane_f64(x, 0) + readlane_f64(x, 16)) + (readlane_f64(x, 32) + readlane_f64(x, 48));
}

// The adjoint keeps one word per hit of a lane's chain in LDS: the triangle's
// leaf-order index, with the top bit set when the geometric normal was flipped
// to face the incoming ray.  The reverse sweep recomputes the normal from it
// bit for bit and recovers each incoming direction and weight backwards from
// the last ones (a mirror reflection is its own inverse).
constexpr uint32_t CHAIN_FLIP = 0x80000000u;

// Adds per-lane vectors into per-wave FP64 LDS accumulators
// acc[key * stride + 0..n), one wave-wide sum per distinct key (keys processed
// lowest lane first).  The wave sum of the (at most 64) FP32 terms is taken in
// FP32 (relative rounding below 64 ulp of FP32, far under the adjoint's 1e-4
// tolerance), the accumulation across a chunk's patches in FP64.
__device__ void wave_scatter_add(double *acc, int key, bool active, const float *vals, int n, int stride) {
    const int lane = threadIdx.x & (WAVE - 1);
    uint64_t pending = __ballot(active);
    while (pending) {
        int leader = __ffsll((unsigned long long)pending) - 1;
        int k = __shfl(key, leader, WAVE);
        bool sel = active && key == k;
        uint64_t m = __ballot(sel);
        for (int c = 0; c < n; ++c) {
            const float s = wave_sum_f32(sel ? vals[c] : 0.0f);
            if (lane == c) acc[k * stride + c] += (double)s;
        }
        pending &= ~m;
    }
}

// 3x3 helpers (row-major)
__device__ __forceinline__ void m3_zero(float *M) {
#pragma unroll
    for (int i = 0; i < 9; ++i) M[i] = 0.0f;
}

// lane-private LDS accumulator: *p += v as one LDS add (the order of one
// lane's adds is its program order)
__device__ __forceinline__ void lds_add(double *p, double v) {
    (void)__hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// A wave-uniform float held in a scalar register.
__device__ __forceinline__ float uniform_f32(float x) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

// Orders this wave's earlier LDS accesses before its later ones across lanes
// (one wave's LDS operations execute in issue order; this keeps the compiler
// from reordering them).
__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Whether every triangle of node k lies in one plane (a ray leaving one of
// them cannot meet the node again, so its traversal skips the node).
__device__ __forceinline__ bool planar_node(const EvalDesc &D, int k) {
    const uint64_t m = k < 64 ? D.planar[0] : D.planar[1];
    return ((m >> (k & 63)) & 1ull) != 0;
}

// The byte per emitter record that follows an evaluation's records: the
// planar instance the record's diffuse rays leave, or -1.
__device__ __forceinline__ int8_t SRP_GLOBAL *emit_skip(const EvalDesc &D) {
    return (int8_t SRP_GLOBAL *)(D.emit + (size_t)D.n_patches * D.bounces * WAVE);
}

// Hit record -> unit normal n facing the incoming direction d, c = -n.d, the
// material's (rho_s, rho_d) and the original triangle index; returns whether
// the geometric normal was flipped.
__device__ __forceinline__ bool hit_normal(const TraceCtx &TC, const EvalDesc &D, const Hit &h, const float d[3],
                                           float n[3], float &c, float &rs, float &rd, int32_t &id) {
    // the instance's rotation does not depend on the triangle: read it first
    const Inst SRP_GLOBAL &I = TC.inst[h.inst];
    const float4 Ra = *(const float4 SRP_GLOBAL *)&I.R[0], Rb = *(const float4 SRP_GLOBAL *)&I.R[4];
    const float R8 = I.R[8];
    const float IR[9] = {Ra.x, Ra.y, Ra.z, Ra.w, Rb.x, Rb.y, Rb.z, Rb.w, R8};
    const TriRec SRP_GLOBAL &T = TC.tris[h.tri];
    float e1[3] = {T.v1[0] - T.v0[0], T.v1[1] - T.v0[1], T.v1[2] - T.v0[2]};
    float e2[3] = {T.v2[0] - T.v0[0], T.v2[1] - T.v0[1], T.v2[2] - T.v0[2]};
    float nl[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    for (int k = 0; k < 3; ++k) n[k] = IR[3 * k] * nl[0] + IR[3 * k + 1] * nl[1] + IR[3 * k + 2] * nl[2];
    float inv = rsqrtf(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    const float nd = (n[0] * d[0] + n[1] * d[1] + n[2] * d[2]) * inv;
    const bool flip = nd > 0.0f;
    if (flip) inv = -inv;
    for (int k = 0; k < 3; ++k) n[k] *= inv;
    c = -(n[0] * d[0] + n[1] * d[1] + n[2] * d[2]);
    const float SRP_GLOBAL *mats = (const float SRP_GLOBAL *)D.mats;
    rs = mats[2 * T.mat];
    rd = mats[2 * T.mat + 1];
    id = T.id;
    return flip;
}

// Adds force f at point x (and its torque about ref) to the lane's FP64 sums.
__device__ __forceinline__ void deposit(double *lacc, const float f[3], const float x[3], const double ref[3]) {
    float rr[3];
    for (int k = 0; k < 3; ++k) rr[k] = x[k] - (float)ref[k];
    lds_add(lacc, (double)f[0]);
    lds_add(lacc + BLOCK, (double)f[1]);
    lds_add(lacc + 2 * BLOCK, (double)f[2]);
    lds_add(lacc + 3 * BLOCK, (double)(rr[1] * f[2] - rr[2] * f[1]));
    lds_add(lacc + 4 * BLOCK, (double)(rr[2] * f[0] - rr[0] * f[2]));
    lds_add(lacc + 5 * BLOCK, (double)(rr[0] * f[1] - rr[1] * f[0]));
}

// Tangent frame of a diffuse fan about unit normal n: t = normalize(h x n)
// with the fixed helper h = (1, 2, 3) (e_x when h x n vanishes), b = n x t.
// A generic helper keeps the frame smooth for every normal but +-h.
__device__ __forceinline__ void fan_frame(const float n[3], float t[3], float b[3]) {
    float c0 = 2.0f * n[2] - 3.0f * n[1], c1 = 3.0f * n[0] - n[2], c2 = n[1] - 2.0f * n[0];
    float l2 = c0 * c0 + c1 * c1 + c2 * c2;
    if (!(l2 > 0.0f)) {
        c0 = 0.0f;
        c1 = -n[2];
        c2 = n[1];
        l2 = c1 * c1 + c2 * c2;
    }
    const float il = rsqrtf(l2);
    t[0] = c0 * il;
    t[1] = c1 * il;
    t[2] = c2 * il;
    b[0] = n[1] * t[2] - n[2] * t[1];
    b[1] = n[2] * t[0] - n[0] * t[2];
    b[2] = n[0] * t[1] - n[1] * t[0];
}

// World direction of the fan ray with local direction l about normal n.
__device__ __forceinline__ void fan_dir(const float n[3], const float4 l, float d[3]) {
    float t[3], b[3];
    fan_frame(n, t, b);
    for (int k = 0; k < 3; ++k) d[k] = l.x * t[k] + l.y * b[k] + l.z * n[k];
}

// Takes the next work item from the per-XCD queues: queue r hands out items
// r, r + N_QUEUES, r + 2 N_QUEUES, ... in order; a wave drains the queue of its
// own XCD, then helps with the others; a relaxed load skips drained queues
// without an atomic.  Lane 0 talks to the counters and broadcasts, so the
// result is wave-uniform.  Returns -1 once every queue is drained.
__device__ __forceinline__ int64_t take_work(uint32_t *queue, uint32_t &r, int &tried, int64_t &n_r, int64_t total,
                                             int lane) {
    int64_t c;
    #pragma unroll 1
    for (;;) {
        uint32_t v = 0;
        if (lane == 0) {
            uint32_t *qr = queue + r * QUEUE_STRIDE;
            v = __hip_atomic_load(qr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (v < (uint32_t)n_r) v = atomicAdd(qr, 1u);
        }
        c = (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)v);
        if (c < n_r || tried == N_QUEUES) break;
        r = (r + 1) & (N_QUEUES - 1);
        ++tried;
        n_r = (total - r + N_QUEUES - 1) / N_QUEUES;
    }
    return c < n_r ? (int64_t)r + c * N_QUEUES : -1;
}

// Position of the (j+1)-th set bit of m (j < popcount(m)).
__device__ __forceinline__ int nth_set_bit(uint64_t m, int j) {
    int pos = 0;
    #pragma unroll
    for (int w = 32; w >= 1; w >>= 1) {
        const uint64_t low = m & ((1ull << w) - 1ull);
        const int c = __popcll(low);
        if (j >= c) {
            j -= c;
            m >>= w;
            pos += w;
        } else {
            m = low;
        }
    }
    return pos;
}

// The diffuse fans of one patch's recorded emitters.  The patch's fan work is
// split into tasks (emitter, slice of FAN_SLICE consecutive fan-ray indices),
// slice-major, packed 64 to a pass, so lanes idle only in the patch's last
// pass.  Every pass writes its own partial sums (force, torque, diffuse rays
// and hits) to its slot of the patch's B * ceil(K / FAN_SLICE) slots (passes
// past the patch's tasks write zeros), so the result depends neither on the
// schedule nor on which kernel, or how many work units, traced the passes.
// This call traces passes pass0, pass0 + step, ...; m[g] = the patch's
// emitters of generation g (bit = lane of the trace kernel's patch).
template <bool COUNT>
__device__ __forceinline__ void fan_passes(const EvalDesc &D, const TraceCtx &TC, int64_t p, uint64_t m0, uint64_t m1,
                                           uint64_t m2, uint64_t m3, int pass0, int step, float tmin2,
                                           LaneStack &stack, double *lacc, int lane, PatchOut *fan_out,
                                           uint64_t *fan_counts) {
    const int KD = D.n_diffuse, B = D.bounces, N = D.n;
    const int S = (KD + FAN_SLICE - 1) / FAN_SLICE;
    const int PM = B * S;               // pass slots per patch
    const int R = B + 1 + B * KD;
    const float4 SRP_GLOBAL *dset = (const float4 SRP_GLOBAL *)D.dset;
    // emitters packed in generation-then-lane order
    const int c0 = __popcll(m0), c1 = c0 + __popcll(m1), c2 = c1 + __popcll(m2), total = c2 + __popcll(m3);
    const int tasks = total * S;
    const int tile = (int)(p >> 2), q = (int)(p & 3);
    #pragma unroll 1
    for (int pass = pass0; pass < PM; pass += step) {
        const int64_t slot_out = D.fan_base + p * PM + pass;
        uint32_t rays = 0, hits = 0, nbox = 0, ntri = 0, status = 0;
        double tot[6] = {0, 0, 0, 0, 0, 0};
        if (pass * WAVE < tasks) {
            for (int k = 0; k < 6; ++k) lacc[k * BLOCK] = 0.0;
            const int t = pass * WAVE + lane;
            if (t < tasks) {
                const int sl = t / total;
                const int j = t - sl * total;
                const int k0 = sl * FAN_SLICE, k1 = min(k0 + FAN_SLICE, KD);
                const int g = j >= c0 ? (j >= c1 ? (j >= c2 ? 3 : 2) : 1) : 0;
                const uint64_t mg = g == 0 ? m0 : g == 1 ? m1 : g == 2 ? m2 : m3;
                const int base = g == 0 ? 0 : g == 1 ? c0 : g == 2 ? c1 : c2;
                const int bl = nth_set_bit(mg, j - base);   // the emitting lane of the trace kernel's patch
                const float4 SRP_GLOBAL *er =
                    (const float4 SRP_GLOBAL *)(D.emit + ((size_t)(p * B + g) * WAVE + bl));
                const float4 ea = er[0], eb = er[1];
                const int32_t skip = emit_skip(D)[(size_t)(p * B + g) * WAVE + bl];
                const float x[3] = {ea.x, ea.y, ea.z}, n[3] = {eb.x, eb.y, eb.z};
                const float wd = ea.w;
                const int32_t excl = __float_as_int(eb.w);
                const int px = (tile % D.tiles_x) * TILE + (q & 1) * PATCH + (bl & 7);
                const int py = (tile / D.tiles_x) * TILE + (q >> 1) * PATCH + (bl >> 3);
                const int64_t pix = (int64_t)py * N + px;
                #pragma unroll 1
                for (int k = k0; k < k1; ++k) {
                    float d[3];
                    fan_dir(n, dset[k], d);
                    Hit h;
                    if (!trace_closest<COUNT>(TC, x, d, tmin2, excl, skip, stack, h, nbox, ntri)) {
                        status |= SRP_STATUS_STACK;
                        break;
                    }
                    ++rays;
                    if (D.hit_ids) {
                        const int64_t slot = pix * R + (B + 1 + g * KD + k);
                        ((int32_t SRP_GLOBAL *)D.hit_ids)[slot] = h.tri >= 0 ? h.id : -1;
                        ((float SRP_GLOBAL *)D.hit_t)[slot] = h.tri >= 0 ? h.t : 0.0f;
                    }
                    if (h.tri >= 0) {
                        ++hits;
                        float nh[3], ch, rs, rd;
                        int32_t id;
                        hit_normal(TC, D, h, d, nh, ch, rs, rd, id);
                        const float a = wd * (1.0f - rs), bb = -2.0f * wd * (rs * ch + rd * (1.0f / 3.0f));
                        float f[3], y[3];
                        for (int i = 0; i < 3; ++i) {
                            f[i] = a * d[i] + bb * nh[i];
                            y[i] = fmaf(h.t, d[i], x[i]);
                        }
                        deposit(lacc, f, y, D.ref);
                    }
                }
            }
            for (int k = 0; k < 6; ++k) tot[k] = wave_sum(lacc[k * BLOCK]);
            rays = wave_add_u32(rays);
            hits = wave_add_u32(hits);
            status = wave_or_u32(status);
            if (COUNT) {
                nbox = wave_add_u32(nbox);
                ntri = wave_add_u32(ntri);
            }
        }
        if (lane == 0) {
            PatchOut co;
            for (int k = 0; k < 6; ++k) co.f[k] = tot[k];
            co.hits = 0;
            co.sec = rays;
            co.sec_hits = hits;
            co.flags = status;
            fan_out[slot_out] = co;
            if (COUNT) {
                fan_counts[2 * slot_out] = nbox;
                fan_counts[2 * slot_out + 1] = ntri;
            }
        }
    }
}

// WPE = 0: registers for the occupancy targets above (batches); WPE = 2: for
// launches of at most 2 blocks per CU (single evaluations), which lose no
// occupancy by it and keep every value in registers.
template <bool COUNT, bool GRAD, bool DIR, int WPE = 0>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(WPE ? WPE : GRAD ? SRP_WPE_GRAD : SRP_WPE_FWD))) void k_trace(
    const EvalDesc *__restrict__ descs, const int64_t *__restrict__ chunk_base, int n_evals,
    const uint64_t *__restrict__ win, int grid_blocks, int64_t total_chunks, uint32_t *queue, uint32_t *spill,
    PatchOut *__restrict__ patches, uint64_t *__restrict__ counts, int lds_grad_doubles, int fans_inline,
    PatchOut *__restrict__ fan_out, uint64_t *__restrict__ fan_counts, int4 *__restrict__ fan_units,
    const uint32_t *__restrict__ order, uint32_t *__restrict__ cost) {
    extern __shared__ char smem[];
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid >> 6;
    LaneStack stack;
    stack.ring = reinterpret_cast<uint32_t *>(smem) + tid;   // slot k at [k * BLOCK]
    stack.stride = BLOCK;
    stack.spill = (uint32_t SRP_GLOBAL *)spill + (size_t)blockIdx.x * BLOCK + tid;
    stack.sstride = grid_blocks * BLOCK;
    // per-lane FP64 force/torque sums of the current patch (component k at [k * BLOCK]):
    // kept in LDS and updated with LDS adds, out of the traversal's registers
    double *lacc = reinterpret_cast<double *>(smem + sizeof(uint32_t) * STACK_LDS * BLOCK) + tid;
    // adjoint only: the hit chains (hit k at [k * BLOCK]), then per-wave gradient sums
    uint32_t *lchain = reinterpret_cast<uint32_t *>(smem + sizeof(uint32_t) * STACK_LDS * BLOCK +
                                                    sizeof(double) * 6 * BLOCK) + tid;
    double *gw = reinterpret_cast<double *>(smem + sizeof(uint32_t) * STACK_LDS * BLOCK + sizeof(double) * 6 * BLOCK +
                                            sizeof(uint32_t) * MAX_CHAIN * BLOCK) +
                 (size_t)wv * lds_grad_doubles;

    // Every wave is persistent on its own and takes chunks from work queues:
    // queue r (one per XCD, each counter on its own 256-byte line) hands out
    // chunks r, r + N_QUEUES, r + 2 N_QUEUES, ... in order.  A wave drains the
    // queue of the XCD it runs on and then helps with the others; a relaxed
    // load skips drained queues without an atomic.  Every queue walks the whole
    // batch in order, so expensive image regions spread over the grid and over
    // time, and each counter sees an eighth of the traffic.  Lane 0 talks to
    // the counters and broadcasts the chunk, so the loop control is
    // wave-uniform, and there is no block barrier anywhere.
    uint32_t r = __builtin_amdgcn_s_getreg((HWREG_XCC_ID << 0) | (0 << 6) | (3 << 11)) & (N_QUEUES - 1);
    int tried = 1;
    int64_t n_r = (total_chunks - r + N_QUEUES - 1) / N_QUEUES;   // chunks of queue r
    int cur = -1;                          // evaluation of the previous chunk
    int64_t cur_begin = 0, cur_end = -1;   // its chunk range
    float o0[3], su[3], sv[3], dd[3];      // its ray grid (FP32 constants)
    float tmin2 = 0.0f;
    bool empty = true;
    #pragma unroll 1
    for (;;) {
        const int64_t c = take_work(queue, r, tried, n_r, total_chunks, lane);
        if (c < 0) break;   // every queue drained

        if (c < cur_begin || c >= cur_end) {
            // evaluation owning chunk c (chunk_base is increasing; chunk_base[n_evals] = total)
            int lo = (cur >= 0 && c >= cur_end) ? cur : 0, hi = n_evals - 1;
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (chunk_base[mid] <= c) lo = mid; else hi = mid - 1;
            }
            cur = lo;
            cur_begin = chunk_base[lo];
            cur_end = chunk_base[lo + 1];
            const EvalDesc &D = descs[lo];
            // window -> ray grid (FP64 -> FP32 constants)
            const uint64_t *W = win + (size_t)lo * WIN_STRIDE;
            const double umin = dec_f64(W[0]), umax = -dec_f64(W[1]);
            const double vmin = dec_f64(W[2]), vmax = -dec_f64(W[3]), hmin = dec_f64(W[4]);
            const double wu = umax - umin, wv_ = vmax - vmin;
            empty = !(wu * wv_ > 0.0) || !(wu < INFINITY) || !(wv_ < INFINITY) || D.root_ref == REF_NONE;
            const double L = fmax(wu, wv_);
            const double h0 = hmin - 1e-3 * L - 1e-3;
            const double du = wu / D.n, dv = wv_ / D.n;
            // (wave-uniform values computed on the vector unit: moved to scalar registers)
            for (int k = 0; k < 3; ++k) {
                o0[k] = uniform_f32((float)((umin + 0.5 * du) * D.u[k] + (vmin + 0.5 * dv) * D.v[k] + h0 * D.d[k]));
                su[k] = uniform_f32((float)(du * D.u[k]));
                sv[k] = uniform_f32((float)(dv * D.v[k]));
                dd[k] = uniform_f32((float)D.d[k]);
            }
            tmin2 = uniform_f32((float)(1e-6 * L));
            empty = __builtin_amdgcn_readfirstlane((int)empty) != 0;
        }
        const EvalDesc &D = descs[cur];
        const int64_t kc = c - D.chunk_base;
        const int N = D.n;

        int64_t p0 = kc * D.ppc, p1 = min(p0 + D.ppc, D.n_patches);
        // (patch order and costs: only in the 2-wave build, which the ordered
        // launches use, so the batch builds keep their registers)
        constexpr bool ORDERED = !GRAD && WPE == 2;
        if (ORDERED && order) {
            // a captured forward plan of one patch per chunk hands out its patches
            // heaviest first, in the order its previous launch measured; any order
            // gives the same result, since every patch writes its own partial slot
            p0 = ((const uint32_t SRP_GLOBAL *)order)[D.patch_base + kc];
            p1 = p0 < D.n_patches ? p0 + 1 : p0;
        }
        const int B = D.bounces;
        const int KD = GRAD ? 0 : D.n_diffuse;          // diffuse rays per emitting hit
        const int R = B + 1 + B * KD;                   // recorded rays per pixel
        const float4 SRP_GLOBAL *dset = (const float4 SRP_GLOBAL *)D.dset;   // KD directions, then their mean
        const TraceCtx TC = trace_ctx(D);

        const int gK = D.n_nodes;
        if (GRAD) {
            for (int i = lane; i < D.grad_n; i += WAVE) gw[i] = 0.0;
            wave_lds_fence();
        }

        #pragma unroll 1
        for (int64_t pt = p0; pt < p1; ++pt) {
            // one 8x8 patch per iteration, one ray per lane; its sums go to the
            // patch's own slot, so the forward result does not depend on the
            // chunking or on which wave runs it
            const int tile = (int)(pt >> 2), q = (int)(pt & 3);
            const int px = (tile % D.tiles_x) * TILE + (q & 1) * PATCH + (lane & 7);
            const int py = (tile / D.tiles_x) * TILE + (q >> 1) * PATCH + (lane >> 3);
            const uint64_t clock0 = (ORDERED && cost) ? wall_clock64() : 0;
            for (int k = 0; k < 6; ++k) lacc[k * BLOCK] = 0.0;
            // hit counts packed in 10-bit fields (primary hits, specular secondary rays and
            // their hits; a patch sums at most 64 * SRP_MAX_BOUNCES of each), the status
            // separately (the diffuse rays are counted by the fan kernel)
            uint32_t hcnt = 0, nbox = 0, ntri = 0, status = 0;
            uint64_t em[SRP_MAX_BOUNCES] = {};   // the patch's fan emitters per generation
            {
                const bool inside = px < N && py < N;
                const bool valid = !empty && inside;
                const int64_t pix = (int64_t)py * N + px;
                int K = 0;
                float d[3] = {dd[0], dd[1], dd[2]}, w = 1.0f;   // the current ray's direction and weight
                bool cont = false;                              // the last chain hit spawned a specular ray
                uint32_t emitted = 0;                           // generations whose hit emitted a fan
                if (inside && D.hit_ids) {   // rays that are not traced or miss stay "no hit"
                    for (int s = 0; s < R; ++s) {
                        ((int32_t SRP_GLOBAL *)D.hit_ids)[pix * R + s] = -1;
                        ((float SRP_GLOBAL *)D.hit_t)[pix * R + s] = 0.0f;
                    }
                }
                if (valid) {
                    float o[3];
                    for (int k = 0; k < 3; ++k) o[k] = fmaf((float)py, sv[k], fmaf((float)px, su[k], o0[k]));
                    float tmin = 0.0f;
                    int32_t excl = -1, skip = -1;   // the triangle and the planar instance the ray leaves
                    int gen = 0;   // chain generation
                    #pragma unroll 1
                    for (;;) {
                        Hit h;
                        if (!trace_closest<COUNT>(TC, o, d, tmin, excl, skip, stack, h, nbox, ntri)) {
                            status |= SRP_STATUS_STACK;
                            break;
                        }
                        if (D.hit_ids) {
                            ((int32_t SRP_GLOBAL *)D.hit_ids)[pix * R + gen] = h.tri >= 0 ? h.id : -1;
                            ((float SRP_GLOBAL *)D.hit_t)[pix * R + gen] = h.tri >= 0 ? h.t : 0.0f;
                        }
                        if (h.tri < 0) break;
                        hcnt += gen == 0 ? 1u : (1u << 20);
                        float n[3], cth, rs, rd;
                        int32_t id;
                        const bool flip = hit_normal(TC, D, h, d, n, cth, rs, rd, id);
                        const bool emit = !GRAD && KD > 0 && gen < B && rd > 0.0f;
                        const bool spec = gen < B && rs > 0.0f;
                        const float a = w * (1.0f - rs);
                        float f[3], x[3];
                        if (emit) {
                            // the fan's exact mean direction replaces the Lambertian 2/3 n recoil
                            float ft[3], fb[3];
                            fan_frame(n, ft, fb);
                            const float4 m = dset[KD];
                            const float b = -2.0f * w * rs * cth - w * rd * m.z, e = -w * rd;
                            for (int k = 0; k < 3; ++k) f[k] = a * d[k] + b * n[k] + e * (m.x * ft[k] + m.y * fb[k]);
                        } else {
                            const float b = -2.0f * w * (rs * cth + rd * (1.0f / 3.0f));
                            for (int k = 0; k < 3; ++k) f[k] = a * d[k] + b * n[k];
                        }
                        for (int k = 0; k < 3; ++k) x[k] = fmaf(h.t, d[k], o[k]);
                        deposit(lacc, f, x, D.ref);
                        if (emit) {
                            // the fan kernel traces this hit's diffuse rays from its record
                            // (slot gen * 64 + lane of the patch's region)
                            float4 SRP_GLOBAL *er = (float4 SRP_GLOBAL *)(D.emit + ((size_t)(pt * B + gen) * WAVE + lane));
                            er[0] = make_float4(x[0], x[1], x[2], w * rd / (float)KD);
                            er[1] = make_float4(n[0], n[1], n[2], __int_as_float(id));
                            emit_skip(D)[(size_t)(pt * B + gen) * WAVE + lane] =
                                (int8_t)(planar_node(D, h.inst) ? h.inst : -1);
                            emitted |= 1u << gen;
                        }
                        if (GRAD) lchain[K * BLOCK] = (uint32_t)h.tri | (flip ? CHAIN_FLIP : 0u);
                        ++K;
                        cont = false;
                        if (!spec) break;
                        for (int k = 0; k < 3; ++k) {
                            o[k] = x[k];
                            d[k] = fmaf(2.0f * cth, n[k], d[k]);   // the specular direction
                        }
                        w *= rs;
                        tmin = tmin2;
                        excl = id;
                        skip = planar_node(D, h.inst) ? h.inst : -1;
                        ++gen;
                        cont = true;
                        hcnt += 1u << 10;
                    }
                }
                if (!GRAD && KD > 0) {
                    // which slots of the patch's emitter region hold records, per generation
                    #pragma unroll
                    for (int g = 0; g < SRP_MAX_BOUNCES; ++g) {
                        if (g >= B) break;
                        em[g] = __ballot((emitted >> g) & 1u);
                        if (lane == 0) ((uint64_t SRP_GLOBAL *)D.emit_mask)[(size_t)pt * B + g] = em[g];
                    }
                }
                if (GRAD) {
                    // Reverse sweep over the chain at fixed visibility.
                    //   A  = d(sum of later contributions)/d(incoming direction)   (3x3)
                    //   Tn = later contributions divided by the weight after this hit
                    const int Kmax = wave_max_i32(K);
                    float A[9], Tn[3] = {0, 0, 0};
                    float n0[3] = {0, 0, 0}, c0 = 1.0f;   // the primary hit's normal and cosine (DIR)
                    m3_zero(A);
                    for (int k = Kmax - 1; k >= 0; --k) {
                        const bool act = k < K;
                        float Hm[9], gmat[6];
                        int node = 0, mat = 0;
                        if (act) {
                            // hit k's normal exactly as the forward pass computed it
                            // the triangle record in one round trip, then its instance's
                            // rotation and its material together
                            const uint32_t ew = lchain[k * BLOCK];
                            const float4 SRP_GLOBAL *tq = (const float4 SRP_GLOBAL *)(TC.tris + (ew & ~CHAIN_FLIP));
                            const float4 T0 = tq[0], T1 = tq[1], T2 = tq[2];
                            const int tnode = f2i(T2.w), tmat = f2i(T1.w);
                            const Inst SRP_GLOBAL &I = TC.inst[tnode];
                            const float4 Ra = *(const float4 SRP_GLOBAL *)&I.R[0], Rb = *(const float4 SRP_GLOBAL *)&I.R[4];
                            const float R8 = I.R[8];
                            const float2 rm = ((const float2 SRP_GLOBAL *)D.mats)[tmat];
                            const float IR[9] = {Ra.x, Ra.y, Ra.z, Ra.w, Rb.x, Rb.y, Rb.z, Rb.w, R8};
                            float e1[3] = {T1.x - T0.x, T1.y - T0.y, T1.z - T0.z};
                            float e2[3] = {T2.x - T0.x, T2.y - T0.y, T2.z - T0.z};
                            float nl[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                                           e1[0] * e2[1] - e1[1] * e2[0]};
                            float n[3];
                            for (int i = 0; i < 3; ++i)
                                n[i] = IR[3 * i] * nl[0] + IR[3 * i + 1] * nl[1] + IR[3 * i + 2] * nl[2];
                            float inv = rsqrtf(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
                            if (ew & CHAIN_FLIP) inv = -inv;
                            for (int i = 0; i < 3; ++i) n[i] *= inv;
                            const float rs = rm.x, rd = rm.y;
                            // (d, w) hold the ray after hit k when hit k spawned one: undo the
                            // reflection and the weight factor to get hit k's incoming ray
                            if (k < K - 1 || cont) {
                                const float dn = n[0] * d[0] + n[1] * d[1] + n[2] * d[2];
                                for (int i = 0; i < 3; ++i) d[i] = fmaf(-2.0f * dn, n[i], d[i]);
                                w = w / rs;
                            }
                            const float cc = -(n[0] * d[0] + n[1] * d[1] + n[2] * d[2]);
                            const float sc = rs * cc + rd * (1.0f / 3.0f);
                            if (DIR && k == 0) {
                                for (int i = 0; i < 3; ++i) n0[i] = n[i];
                                c0 = cc;
                            }
                            // material terms
                            for (int i = 0; i < 3; ++i) {
                                gmat[i] = w * (-d[i] - 2.0f * cc * n[i] + Tn[i]);
                                gmat[3 + i] = w * (-2.0f / 3.0f) * n[i];
                            }
                            // G = dF/dn (explicit) + A (2c I - 2 n d^T)
                            float G[9];
                            for (int i = 0; i < 3; ++i)
                                for (int j = 0; j < 3; ++j) {
                                    float e = w * (2.0f * rs * n[i] * d[j] - (i == j ? 2.0f * sc : 0.0f));
                                    float an = A[3 * i] * n[0] + A[3 * i + 1] * n[1] + A[3 * i + 2] * n[2];
                                    e += 2.0f * cc * A[3 * i + j] - 2.0f * an * d[j];
                                    G[3 * i + j] = e;
                                }
                            if (k == 0) {
                                // the primary ray keeps its share of the triangle's visible surface,
                                // whose projected area scales with c0 = -n0.d: the whole chain's
                                // contribution S (per unit weight) adds dF/dn0 = -S d^T / c0
                                float S[3];
                                for (int i = 0; i < 3; ++i) S[i] = (1.0f - rs) * d[i] - 2.0f * sc * n[i] + rs * Tn[i];
                                const float ws = w / cc;
                                for (int i = 0; i < 3; ++i)
                                    for (int j = 0; j < 3; ++j) G[3 * i + j] -= ws * S[i] * d[j];
                            }
                            // H = -G [n]x
                            for (int i = 0; i < 3; ++i) {
                                const float g0 = G[3 * i], g1 = G[3 * i + 1], g2 = G[3 * i + 2];
                                Hm[3 * i + 0] = -(g1 * n[2] - g2 * n[1]);
                                Hm[3 * i + 1] = -(g2 * n[0] - g0 * n[2]);
                                Hm[3 * i + 2] = -(g0 * n[1] - g1 * n[0]);
                            }
                            // A <- dF_k/dd + A (I - 2 n n^T);  Tn <- f_k + rs Tn
                            float An[3];
                            for (int i = 0; i < 3; ++i) An[i] = A[3 * i] * n[0] + A[3 * i + 1] * n[1] + A[3 * i + 2] * n[2];
                            for (int i = 0; i < 3; ++i)
                                for (int j = 0; j < 3; ++j)
                                    A[3 * i + j] = A[3 * i + j] - 2.0f * An[i] * n[j] +
                                                   w * ((i == j ? 1.0f - rs : 0.0f) + 2.0f * rs * n[i] * n[j]);
                            for (int i = 0; i < 3; ++i) Tn[i] = (1.0f - rs) * d[i] - 2.0f * sc * n[i] + rs * Tn[i];
                            node = tnode;
                            mat = tmat;
                        }
                        wave_scatter_add(gw, node, act, Hm, 9, 9);
                        wave_scatter_add(gw + 9 * gK, mat, act, gmat, 6, 6);
                    }
                    // Photon-direction Jacobian of the ray's whole chain, each primary ray
                    // keeping its triangle and its share of that triangle's visible area
                    // (the share's projected area scales with c = -n0.d):
                    //   dF/dd = A - S n0^T / c0,  S = chain contribution per unit weight (Tn)
                    if (DIR && (D.flags & SRP_F_GRAD_DIR)) {
                        float Jd[9];
                        for (int i = 0; i < 3; ++i)
                            for (int j = 0; j < 3; ++j) Jd[3 * i + j] = A[3 * i + j] - Tn[i] * n0[j] / c0;
                        wave_scatter_add(gw + 9 * gK + 6 * D.n_mats, 0, K > 0, Jd, 9, 9);
                    }
                }
            }

            // the patch's sums: wave reductions (every lane ends with the total), lane 0
            // stores; a patch without a hit has zero sums (secondary hits need a primary)
            double tot[6] = {0, 0, 0, 0, 0, 0};
            if (__ballot((hcnt & 1023u) != 0))
                for (int k = 0; k < 6; ++k) tot[k] = wave_sum(lacc[k * BLOCK]);
            hcnt = wave_add_u32(hcnt);
            status = wave_or_u32(status);
            if (COUNT) {
                nbox = wave_add_u32(nbox);
                ntri = wave_add_u32(ntri);
            }
            const uint32_t cnts[6] = {hcnt & 1023u, (hcnt >> 10) & 1023u, hcnt >> 20, nbox, ntri, status};
            if (lane == 0) {
                PatchOut co;
                for (int k = 0; k < 6; ++k) co.f[k] = tot[k];
                co.hits = cnts[0];
                co.sec = cnts[1];
                co.sec_hits = cnts[2];
                co.flags = cnts[5];
                const int64_t t = D.patch_base + pt;
                patches[t] = co;
                if (COUNT) {
                    counts[2 * t] = cnts[3];
                    counts[2 * t + 1] = cnts[4];
                }
            }
            if (!GRAD && KD > 0 && fans_inline) {
                // the patch's fans right away, from the records its lanes just wrote
                __threadfence_block();
                fan_passes<COUNT>(D, TC, pt, em[0], em[1], em[2], em[3], 0, 1, tmin2, stack, lacc, lane, fan_out,
                                  fan_counts);
            } else if (!GRAD && KD > 0 && fan_units) {
                // a fan launch follows: list the patch's non-empty fan passes as its
                // work units (one pass each), and write the empty passes' zero
                // partials here, as a pass with no task writes them
                const int S = (KD + FAN_SLICE - 1) / FAN_SLICE, PM = B * S;
                int ne = 0;
                for (int g = 0; g < B; ++g) ne += __popcll(em[g]);
                const int np = (ne * S + WAVE - 1) / WAVE;
                uint32_t ubase = 0;
                if (lane == 0 && np > 0) ubase = atomicAdd(queue + FAN_UNITS_AT, (uint32_t)np);
                ubase = (uint32_t)__builtin_amdgcn_readfirstlane((int)ubase);
                for (int l = lane; l < PM; l += WAVE) {
                    if (l < np) {
                        ((int4 SRP_GLOBAL *)fan_units)[ubase + l] = make_int4(cur, (int)pt, l, 0);
                    } else {
                        const int64_t slot = D.fan_base + pt * PM + l;
                        PatchOut co = {};
                        fan_out[slot] = co;
                        if (COUNT) {
                            fan_counts[2 * slot] = 0;
                            fan_counts[2 * slot + 1] = 0;
                        }
                    }
                }
            }
            if (ORDERED && cost && lane == 0) {
                const uint64_t dt = wall_clock64() - clock0;
                ((uint32_t SRP_GLOBAL *)cost)[D.patch_base + pt] = dt < 0xFFFFFFFFull ? (uint32_t)dt : 0xFFFFFFFFu;
            }
        }
        if (GRAD) {
            wave_lds_fence();
            double SRP_GLOBAL *dst = (double SRP_GLOBAL *)(D.grad_part + (size_t)kc * D.grad_n);
            for (int i = lane; i < D.grad_n; i += WAVE) dst[i] = gw[i];
        }
    }
}

// Fan work of the trace kernel's recorded emitters as a separate launch, for
// batches too small to fill the GPU with whole patches: one unit per
// non-empty fan pass, as the trace kernel listed them (evaluation, patch,
// pass), so that one heavy patch's passes run side by side on as many waves
// and no wave claims an empty pass.  Persistent waves and work queues as in
// k_trace.
template <bool COUNT>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(SRP_WPE_FWD))) void k_fans(
    const EvalDesc *__restrict__ descs, const uint64_t *__restrict__ win, int grid_blocks,
    const int4 *__restrict__ units, int64_t max_units, uint32_t *queue, uint32_t *spill,
    PatchOut *__restrict__ fan_out, uint64_t *__restrict__ fan_counts) {
    extern __shared__ char smem[];
    const int tid = threadIdx.x, lane = tid & (WAVE - 1);
    LaneStack stack;
    stack.ring = reinterpret_cast<uint32_t *>(smem) + tid;
    stack.stride = BLOCK;
    stack.spill = (uint32_t SRP_GLOBAL *)spill + (size_t)blockIdx.x * BLOCK + tid;
    stack.sstride = grid_blocks * BLOCK;
    double *lacc = reinterpret_cast<double *>(smem + sizeof(uint32_t) * STACK_LDS * BLOCK) + tid;

    // the units the trace kernel listed (it finished before this launch)
    const int64_t listed = (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)queue[FAN_UNITS_AT]);
    const int64_t total = min(listed, max_units);
    uint32_t *fq = queue + N_QUEUES * QUEUE_STRIDE;   // the fan kernel's own counters
    uint32_t r = __builtin_amdgcn_s_getreg((HWREG_XCC_ID << 0) | (0 << 6) | (3 << 11)) & (N_QUEUES - 1);
    int tried = 1;
    int64_t n_r = (total - r + N_QUEUES - 1) / N_QUEUES;
    int cur = -1;
    float tmin2 = 0.0f;
    #pragma unroll 1
    for (;;) {
        const int64_t c = take_work(fq, r, tried, n_r, total, lane);
        if (c < 0) break;
        const int4 U = ((const int4 SRP_GLOBAL *)units)[c];
        if (U.x != cur) {
            cur = U.x;
            const uint64_t *W = win + (size_t)cur * WIN_STRIDE;
            const double wu = -dec_f64(W[1]) - dec_f64(W[0]), wv_ = -dec_f64(W[3]) - dec_f64(W[2]);
            tmin2 = uniform_f32((float)(1e-6 * fmax(wu, wv_)));
        }
        const EvalDesc &D = descs[cur];
        const int B = D.bounces, PM = B * ((D.n_diffuse + FAN_SLICE - 1) / FAN_SLICE);
        const int64_t p = U.y;   // the patch
        const uint64_t SRP_GLOBAL *em = (const uint64_t SRP_GLOBAL *)(D.emit_mask + (size_t)p * B);
        const uint64_t m0 = em[0], m1 = B > 1 ? em[1] : 0ull, m2 = B > 2 ? em[2] : 0ull, m3 = B > 3 ? em[3] : 0ull;
        // exactly pass U.z (a step of PM ends the pass loop after it)
        fan_passes<COUNT>(D, trace_ctx(D), p, m0, m1, m2, m3, U.z, PM, tmin2, stack, lacc, lane, fan_out, fan_counts);
    }
}

constexpr int WBLOCK = 256;   // threads per block of the window kernel

// Loop strides use compile-time block sizes and an explicit grid-width
// argument, so termination never depends on runtime-filled dispatch values.
__global__ __launch_bounds__(WBLOCK) void k_window(const EvalDesc *__restrict__ descs, uint64_t *win, int blocks_x,
                                                  uint32_t *queue) {
    const EvalDesc &D = descs[blockIdx.y];
    // the trace and fan kernels' work counters and the count of listed fan
    // units start at zero
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x <= 2 * N_QUEUES) queue[threadIdx.x * QUEUE_STRIDE] = 0u;
    double mn[5] = {INFINITY, INFINITY, INFINITY, INFINITY, INFINITY};
    const int64_t stride = (int64_t)blocks_x * WBLOCK;
    for (int64_t i = (int64_t)blockIdx.x * WBLOCK + threadIdx.x; i < D.n_wpts; i += stride) {
        const WPoint p = D.wpts[i];
        const double *X = D.xf + 12 * p.node;
        double x = X[0] * p.x + X[1] * p.y + X[2] * p.z + X[9];
        double y = X[3] * p.x + X[4] * p.y + X[5] * p.z + X[10];
        double z = X[6] * p.x + X[7] * p.y + X[8] * p.z + X[11];
        double a = x * D.u[0] + y * D.u[1] + z * D.u[2];
        double b = x * D.v[0] + y * D.v[1] + z * D.v[2];
        double h = x * D.d[0] + y * D.d[1] + z * D.d[2];
        mn[0] = fmin(mn[0], a);
        mn[1] = fmin(mn[1], -a);
        mn[2] = fmin(mn[2], b);
        mn[3] = fmin(mn[3], -b);
        mn[4] = fmin(mn[4], h);
    }
    __shared__ double s[WBLOCK / WAVE][5];
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x >> 6;
    for (int k = 0; k < 5; ++k) {
        double x = mn[k];
        for (int m = 32; m >= 1; m >>= 1) x = fmin(x, __shfl_xor(x, m, WAVE));
        if (lane == 0) s[wv][k] = x;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        double x = s[0][threadIdx.x];
        for (int w = 1; w < WBLOCK / WAVE; ++w) x = fmin(x, s[w][threadIdx.x]);
        if (x != INFINITY) atomicMin((unsigned long long *)(win + (size_t)blockIdx.y * WIN_STRIDE + threadIdx.x),
                                     (unsigned long long)enc_f64(x));
    }
}

constexpr int RBLOCK = 1024;   // threads per block of the reduction kernels
constexpr uint32_t ORDER_EVERY = 8;   // launches of a plan per rebuild of its patch order

// Reduction, first stage: block (q, e) sums the q-th of n_slices contiguous
// ranges of evaluation e's patch partials (patches np q / Q .. np (q + 1) / Q),
// then the same range of its fan pass slots, with per-thread strided sums,
// wave butterflies and the waves in order; with GRAD also the q-th range of its
// per-chunk gradient partials (the range split again into P contiguous slices,
// P threads per component when the components fit the block several times,
// each summed with eight interleaved accumulators, the slices added in order).
// Q depends only on the evaluation's own size, so every result depends only on
// the evaluation (and, for gradients, on the patches per chunk), not on the
// batch around it.
template <bool COUNT, bool GRAD>
__global__ __launch_bounds__(RBLOCK) void k_slices(const EvalDesc *__restrict__ descs,
                                                const uint32_t *__restrict__ slice_eval,
                                                const PatchOut *__restrict__ patches,
                                                const uint64_t *__restrict__ counts,
                                                const PatchOut *__restrict__ fan_out,
                                                const uint64_t *__restrict__ fan_counts) {
    const int64_t b = blockIdx.x;
    const int e = (int)slice_eval[b], tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid >> 6;
    const EvalDesc &D = descs[e];
    const int Q = D.n_slices, q = (int)(b - D.slice_base);
    if (q < 0 || q >= Q) return;
    double f[6] = {0, 0, 0, 0, 0, 0};
    unsigned long long cn[5] = {0, 0, 0, 0, 0};
    uint32_t st = 0;
    {
        const int64_t np = D.n_patches;
        const int64_t c0 = D.patch_base + np * q / Q, c1 = D.patch_base + np * (q + 1) / Q;
        for (int64_t c = c0 + tid; c < c1; c += RBLOCK) {
            const PatchOut &co = patches[c];
            for (int k = 0; k < 6; ++k) f[k] += co.f[k];
            cn[0] += co.hits;
            cn[1] += co.sec;
            cn[2] += co.sec_hits;
            st |= co.flags;
            if (COUNT) { cn[3] += counts[2 * c]; cn[4] += counts[2 * c + 1]; }
        }
    }
    if (!GRAD && D.emit) {
        // the fan pass slots (diffuse rays): B ceil(K / FAN_SLICE) per patch
        const int64_t nf = D.n_patches * D.bounces * ((D.n_diffuse + FAN_SLICE - 1) / FAN_SLICE);
        const int64_t u0 = D.fan_base + nf * q / Q, u1 = D.fan_base + nf * (q + 1) / Q;
        for (int64_t c = u0 + tid; c < u1; c += RBLOCK) {
            const PatchOut &co = fan_out[c];
            for (int k = 0; k < 6; ++k) f[k] += co.f[k];
            cn[1] += co.sec;
            cn[2] += co.sec_hits;
            st |= co.flags;
            if (COUNT) { cn[3] += fan_counts[2 * c]; cn[4] += fan_counts[2 * c + 1]; }
        }
    }
    for (int k = 0; k < 6; ++k) f[k] = wave_sum(f[k]);
    for (int m = 32; m >= 1; m >>= 1) {
        for (int k = 0; k < 5; ++k) cn[k] += __shfl_xor(cn[k], m, WAVE);
        st |= __shfl_xor(st, m, WAVE);
    }
    __shared__ double sf[RBLOCK / WAVE][6];
    __shared__ unsigned long long sc[RBLOCK / WAVE][5];
    __shared__ uint32_t ss[RBLOCK / WAVE];
    if (lane == 0) {
        for (int k = 0; k < 6; ++k) sf[wid][k] = f[k];
        for (int k = 0; k < 5; ++k) sc[wid][k] = cn[k];
        ss[wid] = st;
    }
    __syncthreads();
    if (tid == 0) {
        SliceOut o = {};
        for (int w = 0; w < RBLOCK / WAVE; ++w) {
            for (int k = 0; k < 6; ++k) o.f[k] += sf[w][k];
            for (int k = 0; k < 5; ++k) o.cnt[k] += sc[w][k];
            o.flags |= ss[w];
        }
        D.pslice[q] = o;
    }
    if (GRAD) {
        const int G = D.grad_n;
        const double *gp = D.grad_part;
        const int64_t NC = D.n_chunks, r0 = NC * q / Q, r1 = NC * (q + 1) / Q;
        const int P = (G > 0 && G <= RBLOCK) ? RBLOCK / G : 1;
        __shared__ double sl[RBLOCK];
        auto slice_sum = [&](int i, int64_t a0, int64_t a1) {
            double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            int64_t c = a0;
            for (; c + 8 <= a1; c += 8)
                for (int u = 0; u < 8; ++u) a[u] += gp[(size_t)(c + u) * G + i];
            for (; c < a1; ++c) a[0] += gp[(size_t)c * G + i];
            return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
        };
        double *gs = D.gslice + (size_t)q * G;
        if (P > 1) {
            const int i = tid % G, p = tid / G;
            if (p < P) sl[p * G + i] = slice_sum(i, r0 + (r1 - r0) * p / P, r0 + (r1 - r0) * (p + 1) / P);
            __syncthreads();
            for (int j = tid; j < G; j += RBLOCK) {
                double t = 0.0;
                for (int k = 0; k < P; ++k) t += sl[k * G + j];
                gs[j] = t;
            }
        } else {
            for (int j = tid; j < G; j += RBLOCK) gs[j] = slice_sum(j, r0, r1);
        }
    }
}

// Heaviest-first patch order for the next launch of a captured forward plan
// (run by the reduction's block of the evaluation, all RBLOCK threads): the
// patches grouped by the bit length of their measured cost (trace time on
// the constant-rate clock, so groups differ by factors of two), groups in
// decreasing cost.  Positions inside a group come from LDS atomics and may
// differ between launches; that changes which wave traces a patch and when,
// never the result.  Every count is exact, so the positions form a
// permutation of the evaluation's patches.
__device__ void patch_order(const EvalDesc &D, uint32_t *order_all, const uint32_t *cost_all, int tid) {
    uint32_t SRP_GLOBAL *ord = (uint32_t SRP_GLOBAL *)order_all + D.patch_base;
    const uint32_t SRP_GLOBAL *cost = (const uint32_t SRP_GLOBAL *)cost_all + D.patch_base;
    const int64_t n = D.n_patches;
    constexpr int NG = 33;   // bit lengths 0..32
    __shared__ uint32_t cnt[NG];
    if (tid < NG) cnt[tid] = 0;
    __syncthreads();
    for (int64_t i = tid; i < n; i += RBLOCK) atomicAdd(&cnt[32 - __clz(cost[i])], 1u);
    __syncthreads();
    if (tid == 0) {
        uint32_t run = 0;
        for (int g = NG - 1; g >= 0; --g) {
            const uint32_t c = cnt[g];
            cnt[g] = run;
            run += c;
        }
    }
    __syncthreads();
    for (int64_t i = tid; i < n; i += RBLOCK) ord[atomicAdd(&cnt[32 - __clz(cost[i])], 1u)] = (uint32_t)i;
}

// Reduction, second stage (one block per evaluation): the first stage's
// range sums added in order, scaled to newtons; with GRAD the gradient range
// sums likewise, then assembled per material and hinge DOF.  A captured
// forward plan's block also orders the patches for the plan's next launch.
template <bool COUNT, bool GRAD>
__global__ __launch_bounds__(RBLOCK) void k_reduce(const EvalDesc *__restrict__ descs,
                                                const uint64_t *__restrict__ win, srp_result *out,
                                                uint32_t *order, const uint32_t *cost, uint32_t *order_launch) {
    const int e = blockIdx.x, tid = threadIdx.x;
    const EvalDesc &D = descs[e];
    const int Q = D.n_slices;
    const uint64_t *W = win + (size_t)e * WIN_STRIDE;
    const double umin = dec_f64(W[0]), umax = -dec_f64(W[1]);
    const double vmin = dec_f64(W[2]), vmax = -dec_f64(W[3]);
    const double wu = umax - umin, wv = vmax - vmin;
    const bool empty = !(wu * wv > 0.0) || !(wu < INFINITY) || !(wv < INFINITY) || D.root_ref == REF_NONE;
    const double scale = empty ? 0.0 : D.pressure * (wu * wv / ((double)D.n * (double)D.n));
    if (tid == 0) {
        double F[6] = {0, 0, 0, 0, 0, 0};
        unsigned long long N[5] = {0, 0, 0, 0, 0};
        uint32_t S = 0;
        for (int q = 0; q < Q; ++q) {
            const SliceOut &o = D.pslice[q];
            for (int k = 0; k < 6; ++k) F[k] += o.f[k];
            for (int k = 0; k < 5; ++k) N[k] += o.cnt[k];
            S |= o.flags;
        }
        srp_result r;
        for (int k = 0; k < 3; ++k) {
            r.force[k] = scale * F[k];
            r.torque[k] = scale * F[3 + k];
        }
        r.n_rays = (int64_t)D.n * D.n;
        r.n_hits = (int64_t)N[0];
        r.n_secondary = (int64_t)N[1];
        r.n_secondary_hits = (int64_t)N[2];
        r.n_box_tests = COUNT ? (int64_t)N[3] : 0;
        r.n_tri_tests = COUNT ? (int64_t)N[4] : 0;
        r.status = S;
        r.n_clamped = (uint32_t)D.n_clamped;
        out[e] = r;
    }
    if (!GRAD && order && cost) {   // (the same for the whole block)
        // rebuilt on every ORDER_EVERY-th launch of the plan: the order stays
        // useful while consecutive launches see similar images, and the pass
        // costs as much as the reduction itself (its LDS counters are hot)
        __shared__ uint32_t s_launch;
        if (tid == 0) s_launch = *order_launch;
        __syncthreads();
        const uint32_t launch = s_launch;
        if (launch % ORDER_EVERY == 0) patch_order(D, order, cost, tid);
        // (one increment per launch; another evaluation's block may read either
        // value, which only moves the launch its order is rebuilt on)
        if (e == 0 && tid == 0) *order_launch = launch + 1;
    }
    if (GRAD) {
        const int G = D.grad_n, K = D.n_nodes, M = D.n_mats, J = D.n_dof;
        __shared__ double sg[MAX_GRAD_SLOTS];
        __shared__ int spar[SRP_MAX_NODES];   // the tree, for the subtree walks below
        for (int j = tid; j < G; j += RBLOCK) {
            double t = 0.0;
            for (int q = 0; q < Q; ++q) t += D.gslice[(size_t)q * G + j];
            sg[j] = t;
        }
        for (int q = tid; q < K; q += RBLOCK) spar[q] = D.parent[q];
        __syncthreads();
        double *g = D.grad_out;
        if (g) {
            // rho_s (M x 3), rho_d (M x 3)
            for (int i = tid; i < 6 * M; i += RBLOCK) {
                int m = i / 6, k = i % 6;
                double v = scale * sg[9 * K + i];
                if (k < 3) g[3 * m + k] = v;
                else g[3 * M + 3 * m + (k - 3)] = v;
            }
            // theta: (sum of S_q over the subtree of the joint's node) * world axis
            for (int j = tid; j < J; j += RBLOCK) {
                const int p = D.dof_node[j];
                double S[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
                for (int q = 0; q < K; ++q) {
                    int a = q;
                    while (a > p) a = spar[a];
                    if (a != p) continue;
                    for (int i = 0; i < 9; ++i) S[i] += sg[9 * q + i];
                }
                const double *ax = D.axw + 3 * j;
                for (int i = 0; i < 3; ++i)
                    g[6 * M + 3 * j + i] = scale * (S[3 * i] * ax[0] + S[3 * i + 1] * ax[1] + S[3 * i + 2] * ax[2]);
            }
            // photon-direction Jacobian dF_i/dd_j (row-major); zeros when the item
            // did not ask for it (its partials then have no direction slots)
            const bool has_dir = G >= 9 * K + 6 * M + 9;
            for (int i = tid; i < 9; i += RBLOCK) g[6 * M + 3 * J + i] = has_dir ? scale * sg[9 * K + 6 * M + i] : 0.0;
        }
    }
}

int check(hipError_t e) { return e == hipSuccess ? 0 : (int)e; }

}  // namespace

// The device workspace of srp_eval_batch_noalloc.  Its name is a host-side
// stand-in in host code: only the address looked up on each device is passed
// to kernels and copies.
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

static char *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

int noalloc_scratch_init() {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return (int)hipErrorInvalidDevice;
    if (g_scratch_ptr[dev]) return 0;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    g_scratch_ptr[dev] = static_cast<char *>(p);
    return 0;
}

char *noalloc_scratch(int device) {
    return (device >= 0 && device < NOALLOC_MAX_DEVICES) ? g_scratch_ptr[device] : nullptr;
}

int launch_window(const EvalDesc *d_desc, int n_evals, int blocks_x, uint64_t *d_win, uint32_t *d_queue,
                  void *stream) {
    if (n_evals <= 0) return 0;
    hipLaunchKernelGGL(k_window, dim3(blocks_x, n_evals), dim3(WBLOCK), 0, (hipStream_t)stream, d_desc, d_win, blocks_x,
                       d_queue);
    return check(hipGetLastError());
}

size_t trace_lds_bytes(bool grad, int lds_grad_doubles) {
    return sizeof(uint32_t) * STACK_LDS * BLOCK + sizeof(double) * 6 * BLOCK +
           (grad ? sizeof(uint32_t) * MAX_CHAIN * BLOCK + sizeof(double) * (BLOCK / 64) * lds_grad_doubles : 0);
}

int launch_trace(const EvalDesc *d_desc, const int64_t *d_chunk_base, int n_evals, const uint64_t *d_win,
                 int64_t total_chunks, uint32_t *d_queue, uint32_t *d_spill, PatchOut *d_chunks,
                 uint64_t *d_counts, bool count, bool grad, bool dir, int grid_blocks, int lds_grad_doubles,
                 PatchOut *d_fan_out, uint64_t *d_fan_counts, bool fans_inline_, int4 *d_fan_units,
                 int blocks_per_cu, const uint32_t *d_order, uint32_t *d_cost, void *stream) {
    if (total_chunks <= 0) return 0;
    const size_t lds = trace_lds_bytes(grad, lds_grad_doubles);
    const int lgd = grad ? lds_grad_doubles : 0;
    const int fans_inline = (!grad && d_fan_out && fans_inline_) ? 1 : 0;
    int4 *fan_units = (!grad && d_fan_out && !fans_inline_) ? d_fan_units : nullptr;
    hipStream_t s = (hipStream_t)stream;
#define SRP_LAUNCH_TRACE(C, G, R, W)                                                                              \
    hipLaunchKernelGGL((k_trace<C, G, R, W>), dim3(grid_blocks), dim3(BLOCK), lds, s, d_desc, d_chunk_base, n_evals, \
                       d_win, grid_blocks, total_chunks, d_queue, d_spill, d_chunks, d_counts, lgd, fans_inline,  \
                       d_fan_out, d_fan_counts, fan_units, d_order, d_cost)
    // (the counting variants serve tests and the benchmark's work counts: one
    // instantiation each; both instantiations compute the same bits)
    const bool lean = blocks_per_cu <= 2;
    if (count && grad && dir) SRP_LAUNCH_TRACE(true, true, true, 0);
    else if (count && grad) SRP_LAUNCH_TRACE(true, true, false, 0);
    else if (count) SRP_LAUNCH_TRACE(true, false, false, 0);
    else if (grad && dir && lean) SRP_LAUNCH_TRACE(false, true, true, 2);
    else if (grad && dir) SRP_LAUNCH_TRACE(false, true, true, 0);
    else if (grad && lean) SRP_LAUNCH_TRACE(false, true, false, 2);
    else if (grad) SRP_LAUNCH_TRACE(false, true, false, 0);
    else if (lean) SRP_LAUNCH_TRACE(false, false, false, 2);
    else SRP_LAUNCH_TRACE(false, false, false, 0);
#undef SRP_LAUNCH_TRACE
    return check(hipGetLastError());
}

int launch_fans(const EvalDesc *d_desc, const uint64_t *d_win, int64_t max_units, uint32_t *d_queue,
                uint32_t *d_spill, PatchOut *d_fan_out, uint64_t *d_fan_counts, const int4 *d_fan_units, bool count,
                int grid_blocks, void *stream) {
    if (max_units <= 0) return 0;
    const size_t lds = trace_lds_bytes(false, 0);   // the same ring and accumulators as the forward trace
    hipStream_t s = (hipStream_t)stream;
    if (count)
        hipLaunchKernelGGL((k_fans<true>), dim3(grid_blocks), dim3(BLOCK), lds, s, d_desc, d_win, grid_blocks,
                           d_fan_units, max_units, d_queue, d_spill, d_fan_out, d_fan_counts);
    else
        hipLaunchKernelGGL((k_fans<false>), dim3(grid_blocks), dim3(BLOCK), lds, s, d_desc, d_win, grid_blocks,
                           d_fan_units, max_units, d_queue, d_spill, d_fan_out, d_fan_counts);
    return check(hipGetLastError());
}

int launch_reduce(const EvalDesc *d_desc, int n_evals, const uint64_t *d_win, const PatchOut *d_patches,
                  const uint64_t *d_counts, const PatchOut *d_fan_out, const uint64_t *d_fan_counts, bool count,
                  bool grad, const uint32_t *d_slice_eval, int64_t total_slices, void *d_out, uint32_t *d_order,
                  const uint32_t *d_cost, uint32_t *d_order_launch, void *stream) {
    if (n_evals <= 0) return 0;
    if (total_slices < n_evals || total_slices > INT32_MAX) return (int)hipErrorInvalidValue;
    hipStream_t s = (hipStream_t)stream;
    srp_result *out = (srp_result *)d_out;
#define SRP_LAUNCH_REDUCE(C, G)                                                                                 \
    do {                                                                                                        \
        hipLaunchKernelGGL((k_slices<C, G>), dim3((uint32_t)total_slices), dim3(RBLOCK), 0, s, d_desc,          \
                           d_slice_eval, d_patches, d_counts, d_fan_out, d_fan_counts);                         \
        hipLaunchKernelGGL((k_reduce<C, G>), dim3(n_evals), dim3(RBLOCK), 0, s, d_desc, d_win, out, d_order,    \
                           d_cost, d_order_launch);                                                             \
    } while (0)
    if (count && grad) SRP_LAUNCH_REDUCE(true, true);
    else if (count) SRP_LAUNCH_REDUCE(true, false);
    else if (grad) SRP_LAUNCH_REDUCE(false, true);
    else SRP_LAUNCH_REDUCE(false, false);
#undef SRP_LAUNCH_REDUCE
    return check(hipGetLastError());
}

int trace_blocks_per_cu(bool count, bool grad, bool dir, int lds_grad_doubles) {
    const size_t lds = trace_lds_bytes(grad, lds_grad_doubles);
    int nb = 0;
    hipError_t e;
    if (count && grad && dir) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_trace<true, true, true>, BLOCK, lds);
    else if (count && grad) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_trace<true, true, false>, BLOCK, lds);
    else if (count) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_trace<true, false, false>, BLOCK, lds);
    else if (grad && dir) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_trace<false, true, true>, BLOCK, lds);
    else if (grad) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_trace<false, true, false>, BLOCK, lds);
    else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_trace<false, false, false>, BLOCK, lds);
    if (e != hipSuccess || nb < 1) nb = 1;
    return nb;
}

int fan_blocks_per_cu(bool count) {
    const size_t lds = trace_lds_bytes(false, 0);
    int nb = 0;
    hipError_t e = count ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fans<true>, BLOCK, lds)
                         : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fans<false>, BLOCK, lds);
    if (e != hipSuccess || nb < 1) nb = 1;
    return nb;
}

}  // namespace srp
