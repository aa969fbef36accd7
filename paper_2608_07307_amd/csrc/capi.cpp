// C ABI entry points: argument checks, articulation slots, the per-call
// upload and the window -> trace -> reduce launch sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>
#include <new>
#include <string>
#include <vector>

#include "host.h"

using namespace srp;

struct PlanImpl;

struct srp_scene {
    int device = 0;
    SceneHost h;
    TriRec *d_tris = nullptr;
    BNode4 *d_blas = nullptr;
    float *d_mats = nullptr;
    WPoint *d_wpts = nullptr;
    int32_t *d_parent = nullptr;
    ArtNode *d_art = nullptr;      // the tree as the articulation kernel reads it
    BNode4 *d_topo = nullptr;      // top-level topology (references; boxes refitted per slot)
    char *d_slot = nullptr;        // current articulation slot
    SlotLayout slot_L{};
    SlotHost cur;
    std::vector<double> angles;    // current (clamped) angles
    // captured single-evaluation launches keyed by (n, diffuse rays, bounces, flags)
    std::map<uint64_t, PlanImpl *> eval_plans;
    srp_result *d_res = nullptr;   // device result of those launches
    srp_result *h_res = nullptr;   // pinned host copy
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(x)                                                                              \
    do {                                                                                       \
        hipError_t e_ = (x);                                                                   \
        if (e_ != hipSuccess) return fail(SRP_ERR_DEVICE, std::string(#x ": ") + hipGetErrorString(e_)); \
    } while (0)

size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) & ~(a - 1); }

// Per-process workspace: one growing device buffer, one pinned staging
// buffer, the library stream, and the upload and completion events of the
// last batch.
struct Workspace {
    std::mutex mu;
    bool init = false;
    int device = -1;
    int n_cu = 256;
    char *d_buf = nullptr;
    size_t d_cap = 0;
    char *h_stage = nullptr;
    size_t h_cap = 0;
    srp_result *h_res = nullptr;   // pinned result readback
    size_t h_res_cap = 0;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;     // the last batch's device work finished
    hipEvent_t copied = nullptr;   // its staging image was uploaded
    bool pending = false;
    float *d_dset = nullptr;       // diffuse direction sets, K = 1..SRP_MAX_DIFFUSE
};
Workspace g_ws;

// Diffuse direction sets: for K = 1..SRP_MAX_DIFFUSE, K entries (x, y, z, 0)
// then their mean; set K starts at entry (K - 1)(K + 2)/2.  Ray k of K has
// u = (k + 1/2)/K, phi = 2 pi frac(k (sqrt5 - 1)/2) and local direction
// (sqrt(u) cos phi, sqrt(u) sin phi, sqrt(1 - u)): Fibonacci points on the
// unit disk lifted to the hemisphere, so the directions are cosine
// distributed about the normal.  Computed in FP64, stored as FP32.
size_t dset_entry(int K) { return (size_t)(K - 1) * (size_t)(K + 2) / 2; }

std::vector<float> diffuse_sets() {
    std::vector<float> t(4 * dset_entry(SRP_MAX_DIFFUSE + 1), 0.0f);
    const double g = (std::sqrt(5.0) - 1.0) / 2.0, two_pi = 6.283185307179586476925;
    for (int K = 1; K <= SRP_MAX_DIFFUSE; ++K) {
        float *e = &t[4 * dset_entry(K)];
        double m[3] = {0, 0, 0};
        for (int k = 0; k < K; ++k) {
            const double u = (k + 0.5) / K;
            double f = k * g;
            f -= std::floor(f);
            const double r = std::sqrt(u), ph = two_pi * f;
            const double l[3] = {r * std::cos(ph), r * std::sin(ph), std::sqrt(1.0 - u)};
            for (int c = 0; c < 3; ++c) {
                e[4 * k + c] = (float)l[c];
                m[c] += l[c];
            }
        }
        for (int c = 0; c < 3; ++c) e[4 * K + c] = (float)(m[c] / K);
    }
    return t;
}

// Optional timing of the trace-kernel launches (HIP events on the launch stream),
// and of each whole launch: from its staging upload through its result copy.
struct Profile {
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pairs;   // recorded, not yet read
    std::vector<std::pair<hipEvent_t, hipEvent_t>> whole;   // the same for whole launches
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
    double ms = 0, whole_ms = 0;
    int64_t launches = 0;
};
Profile g_prof;

int prof_event_pair(std::pair<hipEvent_t, hipEvent_t> *p) {
    if (!g_prof.pool.empty()) {
        *p = g_prof.pool.back();
        g_prof.pool.pop_back();
        return SRP_OK;
    }
    HIPCHK(hipEventCreate(&p->first));
    HIPCHK(hipEventCreate(&p->second));
    return SRP_OK;
}

int prof_collect() {
    for (auto &pr : g_prof.pairs) {
        HIPCHK(hipEventSynchronize(pr.second));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, pr.first, pr.second));
        g_prof.ms += ms;
        g_prof.launches++;
        g_prof.pool.push_back(pr);
    }
    g_prof.pairs.clear();
    for (auto &pr : g_prof.whole) {
        HIPCHK(hipEventSynchronize(pr.second));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, pr.first, pr.second));
        g_prof.whole_ms += ms;
        g_prof.pool.push_back(pr);
    }
    g_prof.whole.clear();
    return SRP_OK;
}

int ws_init() {
    if (g_ws.init) return SRP_OK;
    HIPCHK(hipGetDevice(&g_ws.device));
    HIPCHK(hipDeviceGetAttribute(&g_ws.n_cu, hipDeviceAttributeMultiprocessorCount, g_ws.device));
    HIPCHK(hipStreamCreateWithFlags(&g_ws.stream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&g_ws.done, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&g_ws.copied, hipEventDisableTiming));
    {
        const std::vector<float> t = diffuse_sets();
        if (hipMalloc(&g_ws.d_dset, t.size() * sizeof(float)) != hipSuccess) {
            (void)hipGetLastError();
            g_ws.d_dset = nullptr;
            return fail(SRP_ERR_OOM, "diffuse set allocation failed");
        }
        HIPCHK(hipMemcpy(g_ws.d_dset, t.data(), t.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    // the fixed workspace of srp_eval_batch_noalloc on this device
    int e = noalloc_scratch_init();
    if (e) return fail(SRP_ERR_DEVICE, std::string("scratch address lookup: ") + hipGetErrorString((hipError_t)e));
    g_ws.init = true;
    return SRP_OK;
}

int ws_wait() {
    if (g_ws.pending) HIPCHK(hipEventSynchronize(g_ws.done));
    g_ws.pending = false;
    return SRP_OK;
}

int ws_reserve(size_t dev_bytes, size_t host_bytes) {
    if (dev_bytes > g_ws.d_cap) {
        int rc = ws_wait();
        if (rc) return rc;
        if (g_ws.d_buf) HIPCHK(hipFree(g_ws.d_buf));
        g_ws.d_buf = nullptr;
        size_t cap = std::max(dev_bytes, g_ws.d_cap + g_ws.d_cap / 2);
        if (hipMalloc(&g_ws.d_buf, cap) != hipSuccess) {
            g_ws.d_cap = 0;
            (void)hipGetLastError();
            return fail(SRP_ERR_OOM, "device workspace allocation failed (" + std::to_string(cap) + " bytes)");
        }
        g_ws.d_cap = cap;
    }
    if (host_bytes > g_ws.h_cap) {
        int rc = ws_wait();
        if (rc) return rc;
        if (g_ws.h_stage) HIPCHK(hipHostFree(g_ws.h_stage));
        g_ws.h_stage = nullptr;
        size_t cap = std::max(host_bytes, g_ws.h_cap + g_ws.h_cap / 2);
        if (hipHostMalloc(&g_ws.h_stage, cap, hipHostMallocDefault) != hipSuccess) {
            g_ws.h_cap = 0;
            (void)hipGetLastError();
            return fail(SRP_ERR_OOM, "pinned staging allocation failed");
        }
        g_ws.h_cap = cap;
    }
    return SRP_OK;
}

bool finite3(const double *v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

int check_params(const srp_eval_params *p) {
    if (!p) return fail(SRP_ERR_ARG, "null params");
    if (p->n < 1 || p->n > SRP_MAX_N) return fail(SRP_ERR_ARG, "n must be in 1.." + std::to_string(SRP_MAX_N));
    if (p->bounces < 0 || p->bounces > SRP_MAX_BOUNCES)
        return fail(SRP_ERR_ARG, "bounces must be in 0.." + std::to_string(SRP_MAX_BOUNCES));
    if (!finite3(p->sun_dir)) return fail(SRP_ERR_ARG, "non-finite sun_dir");
    double s = std::sqrt(p->sun_dir[0] * p->sun_dir[0] + p->sun_dir[1] * p->sun_dir[1] + p->sun_dir[2] * p->sun_dir[2]);
    if (!(s > 0) || !std::isfinite(s)) return fail(SRP_ERR_ARG, "zero sun_dir");
    if (!std::isfinite(p->pressure) || !finite3(p->ref)) return fail(SRP_ERR_ARG, "non-finite pressure or ref");
    if (p->flags & ~(uint32_t)(SRP_F_COUNT | SRP_F_GRAD_DIR)) return fail(SRP_ERR_ARG, "unknown flags");
    if (p->n_diffuse < 0 || p->n_diffuse > SRP_MAX_DIFFUSE)
        return fail(SRP_ERR_ARG, "n_diffuse must be in 0.." + std::to_string(SRP_MAX_DIFFUSE));
    return SRP_OK;
}

// Image-plane basis for photon direction d = -s/|s|: helper e_z unless
// |d_z| >= 0.9 (then e_x), u = normalize(h x d), v = d x u.
void basis(const double *s, double *u, double *v, double *d) {
    double n = std::sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
    for (int k = 0; k < 3; ++k) d[k] = -s[k] / n;
    double h[3] = {0, 0, 1};
    if (!(std::fabs(d[2]) < 0.9)) { h[0] = 1; h[2] = 0; }
    u[0] = h[1] * d[2] - h[2] * d[1];
    u[1] = h[2] * d[0] - h[0] * d[2];
    u[2] = h[0] * d[1] - h[1] * d[0];
    double un = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    for (int k = 0; k < 3; ++k) u[k] /= un;
    v[0] = d[1] * u[2] - d[2] * u[1];
    v[1] = d[2] * u[0] - d[0] * u[2];
    v[2] = d[0] * u[1] - d[1] * u[0];
}

struct BatchOut {
    srp_result *d_out = nullptr;     // device results (n items)
    double *d_grad = nullptr;        // device gradients or null
    int64_t grad_stride = 0;
    int32_t *d_hit_ids = nullptr;    // single item only
    float *d_hit_t = nullptr;
    srp_result *h_copy = nullptr;    // optional pinned host copy of the results (graph plans)
};

// Schedule of a batch launch: 8x8-pixel patches per chunk (a chunk is one
// wave's work item) and resident blocks per compute unit of the persistent
// grid.  0 = automatic.
struct Schedule {
    int ppc = 0;
    int bpc = 0;
};
Schedule g_override;                    // srp_set_schedule
std::map<uint64_t, Schedule> g_tuned;   // autotuner results

int ilog2(int64_t x) {
    int k = 0;
    while (x > 1) { x >>= 1; ++k; }
    return k;
}

// Autotuner key: total primary rays (power-of-two bucket), bounces, diffuse
// rays, gradient.
uint64_t tune_key(const srp_batch_item *items, int64_t n, bool grad) {
    int64_t rays = 0;
    int b = 0, kd = 0;
    for (int64_t k = 0; k < n; ++k) {
        rays += (int64_t)items[k].p.n * items[k].p.n;
        b = std::max(b, (int)items[k].p.bounces);
        kd = std::max(kd, (int)items[k].p.n_diffuse);
    }
    return ((uint64_t)ilog2(std::max<int64_t>(rays, 1)) << 16) | ((uint64_t)kd << 8) | ((uint64_t)b << 1) |
           (grad ? 1u : 0u);
}

// A batch's articulation slot: built on the device by k_articulate from the
// angles of its first item (`item`); `next` chains slots of equal angle hash.
struct SlotRec {
    const srp_scene *sc;
    int64_t item;
    int next;
    size_t cs_off;   // its cosines and sines: doubles from Layout::o_cs
    SlotLayout L;
    size_t off;      // device offset of the slot
};

// Everything about a batch that does not change when only Sun directions,
// pressures, references or hinge-angle values change.
struct Layout {
    int64_t n = 0;
    bool grad = false, count = false, dir = false;
    Schedule sch;
    std::vector<int64_t> chunk_base, patch_base;
    std::vector<int64_t> fan_base;    // first fan partial slot of every item, then the total
    std::vector<int> tiles_x, tiles_y;
    std::vector<int> item_slot;
    std::vector<SlotRec> slots;
    int max_grad_n = 0;
    int64_t total_chunks = 0, total_patches = 0, max_wpts = 0, total_units = 0, total_fan_slots = 0;
    size_t o_desc = 0, o_cbase = 0, o_win = 0, o_seval = 0, o_jobs = 0, o_cs = 0, stage_bytes = 0;
    size_t o_slots = 0, total_cs = 0;
    size_t o_patches = 0, o_counts = 0, o_emask = 0, o_fanout = 0, o_fancnt = 0, o_units = 0, o_gpart = 0, o_queue = 0;
    size_t o_spill = 0, dev_bytes = 0;
    std::vector<size_t> gpart_off, gslice_off, pslice_off;
    std::vector<int> n_slices;    // reduction range sums per item (first stage)
    std::vector<int64_t> slice_base;   // first range sum of every item, then the total
    std::vector<size_t> emit_off;   // emitter records of each item with diffuse fans (0: none)
    std::vector<int> grad_n;   // gradient partial doubles per chunk of each item (allocation and kernel)
    std::vector<int> item_ppc;   // patches per chunk of each item (the adjoint: its gradient group)
    int grid = 1, fan_grid = 0, wb = 1;
    bool fans_inline = false;   // the trace kernel traces the fans itself (no fan launch)
    // captured forward plans of one patch per chunk: the patch order of the next
    // launch and the per-patch costs it is made from (layout_add_order)
    bool ordered = false;
    size_t o_order = 0, o_cost = 0;
};

// Gradient partial slots per chunk: 9 per node (rotation sensitivities), 6
// per material, and 9 for the photon-direction Jacobian when the item asks
// for it (SRP_F_GRAD_DIR).
int grad_slots(const srp_scene *sc, uint32_t flags) {
    return 9 * sc->h.n_nodes + 6 * sc->h.n_mats + ((flags & SRP_F_GRAD_DIR) ? 9 : 0);
}
// Gradient outputs per evaluation: rho_s (M x 3), rho_d (M x 3), theta (J x 3), dF/dd (3 x 3).
int64_t grad_out_size(const srp_scene *sc) { return 3 * (2 * (int64_t)sc->h.n_mats + sc->h.n_dof) + 9; }

int check_items(const srp_batch_item *items, int64_t n, bool grad, const BatchOut &bo) {
    if (n > (1 << 30)) return fail(SRP_ERR_ARG, "too many items");
    for (int64_t k = 0; k < n; ++k) {
        const srp_batch_item &it = items[k];
        if (!it.scene) return fail(SRP_ERR_ARG, "item " + std::to_string(k) + ": null scene");
        int rc = check_params(&it.p);
        if (rc) return fail(rc, "item " + std::to_string(k) + ": " + g_err);
        if (it.scene->device != g_ws.device) return fail(SRP_ERR_ARG, "scene built on another device");
        if (it.angles)
            for (int j = 0; j < it.scene->h.n_dof; ++j)
                if (!std::isfinite(it.angles[j])) return fail(SRP_ERR_ARG, "item " + std::to_string(k) + ": non-finite angle");
        if (grad && it.p.n_diffuse > 0)
            return fail(SRP_ERR_ARG, "item " + std::to_string(k) + ": the adjoint does not cover diffuse rays (n_diffuse must be 0)");
        if (grad) {
            int gn = grad_slots(it.scene, it.p.flags);
            if (gn > MAX_GRAD_SLOTS) return fail(SRP_ERR_ARG, "gradient needs 9*nodes + 6*materials + 9 <= 960");
            if (bo.d_grad && bo.grad_stride < grad_out_size(it.scene))
                return fail(SRP_ERR_ARG, "grad_stride too small");
        }
    }
    return SRP_OK;
}

// The adjoint's gradient partials are per chunk, and an adjoint chunk is a
// fixed group of an evaluation's patches whose size depends on that
// evaluation alone (grad_group), never on the schedule: gradient bits then do
// not depend on the autotuner, the blocks per CU or the batch around an
// evaluation.  The group is the smallest power of two from GRAD_GROUP_MIN up
// to MAX_PPC patches whose partials for the evaluation fit GRAD_PART_EVAL
// bytes.  A batch whose whole device workspace would exceed WORKSPACE_CAP
// runs as consecutive sub-batches.
constexpr int GRAD_GROUP_MIN = 8;
constexpr size_t GRAD_PART_EVAL = (size_t)8 << 20;
constexpr size_t WORKSPACE_CAP = (size_t)16 << 30;   // of the MI355X's 288 GB: the 32,768-evaluation table at 512^2 (8.6 GB of patch partials) runs as one launch

int grad_group(int64_t n_patches, int grad_n) {
    int g = GRAD_GROUP_MIN;
    while (g < MAX_PPC && (size_t)((n_patches + g - 1) / g) * grad_n * sizeof(double) > GRAD_PART_EVAL) g *= 2;
    return g;
}

Schedule pick_schedule(const srp_batch_item *items, int64_t n, bool grad, int64_t total_patches, int occ,
                       int max_grad_n) {
    Schedule s = g_override;
    if (!s.ppc || !s.bpc) {
        auto f = g_tuned.find(tune_key(items, n, grad));
        if (f != g_tuned.end()) {
            if (!s.ppc) s.ppc = f->second.ppc;
            if (!s.bpc) s.bpc = f->second.bpc;
        }
    }
    if (!s.bpc) {
        // a launch with few patches per resident wave (a single evaluation) ends on a
        // few long patches, which run faster at half occupancy (measured on the ~50k
        // craft, B = 2: one evaluation at 1024^2 4 % faster, at 512^2 5 %)
        s.bpc = occ;
        if (total_patches < 16 * (int64_t)g_ws.n_cu * occ * (BLOCK / 64)) s.bpc = std::min(occ, 2);
    }
    if (!s.ppc) {
        // largest patches-per-chunk (up to 4) that still leaves >= 16 chunks per
        // resident wave: small chunks spread expensive image regions best
        int64_t resident = (int64_t)g_ws.n_cu * s.bpc * (BLOCK / 64);
        s.ppc = 1;
        while (s.ppc < 4 && total_patches / (2 * s.ppc) >= 16 * resident) s.ppc *= 2;
    }
    s.bpc = std::max(1, std::min(s.bpc, occ));
    return s;
}

int layout_build(const srp_batch_item *items, int64_t n, bool grad, Schedule force, Layout *Lp) {
    Layout &L = *Lp;
    L = Layout();
    L.n = n;
    L.grad = grad;
    L.chunk_base.assign(n + 1, 0);
    L.patch_base.assign(n + 1, 0);
    L.tiles_x.assign(n, 0);
    L.tiles_y.assign(n, 0);
    for (int64_t k = 0; k < n; ++k) {
        const srp_batch_item &it = items[k];
        L.count |= (it.p.flags & SRP_F_COUNT) != 0;
        L.tiles_x[k] = (it.p.n + TILE - 1) / TILE;
        L.tiles_y[k] = (it.p.n + TILE - 1) / TILE;
        L.patch_base[k] = L.total_patches;
        L.total_patches += 4 * (int64_t)L.tiles_x[k] * L.tiles_y[k];
        if (grad) L.max_grad_n = std::max(L.max_grad_n, grad_slots(it.scene, it.p.flags));
        L.dir |= grad && (it.p.flags & SRP_F_GRAD_DIR);
        L.max_wpts = std::max<int64_t>(L.max_wpts, (int64_t)it.scene->h.wpts.size());
    }
    L.patch_base[n] = L.total_patches;
    // the reduction's first stage: range sums of about 1,024 patches each (at most
    // MAX_SLICES), a function of the item's own size, so an item's results do not
    // depend on its batch
    L.n_slices.assign(n, 0);
    L.slice_base.assign(n + 1, 0);
    for (int64_t k = 0; k < n; ++k) {
        const int64_t np = L.patch_base[k + 1] - L.patch_base[k];
        L.n_slices[k] = (int)std::min<int64_t>(MAX_SLICES, std::max<int64_t>(1, np / 1024));
        L.slice_base[k + 1] = L.slice_base[k] + L.n_slices[k];
    }
    if (L.slice_base[n] > INT32_MAX) return fail(SRP_ERR_ARG, "batch too large: more than 2^31 range sums (split it)");
    int occ = trace_blocks_per_cu(L.count, grad, L.dir, L.max_grad_n);
    L.sch = (force.ppc && force.bpc) ? force : pick_schedule(items, n, grad, L.total_patches, occ, L.max_grad_n);
    if (force.ppc) L.sch.ppc = force.ppc;
    if (force.bpc) L.sch.bpc = std::min(force.bpc, occ);
    // patches per chunk: the schedule's for the forward launch, each evaluation's
    // own gradient group for the adjoint
    L.item_ppc.assign(n, L.sch.ppc);
    for (int64_t k = 0; k < n; ++k) {
        const int64_t np = L.patch_base[k + 1] - L.patch_base[k];
        if (grad) L.item_ppc[k] = grad_group(np, grad_slots(items[k].scene, items[k].p.flags));
        L.chunk_base[k] = L.total_chunks;
        L.total_chunks += (np + L.item_ppc[k] - 1) / L.item_ppc[k];
    }
    L.chunk_base[n] = L.total_chunks;
    // diffuse fans (forward only; emitters are chain hits of generation < bounces).
    // Many patches with fans: the trace kernel traces each patch's fans right after
    // its chains.  Few: the trace kernel lists every patch's non-empty fan passes and
    // a fan kernel follows with one unit per listed pass, so that a small batch
    // still fills the GPU and a heavy patch's passes run side by side.  Both give
    // the same bits.
    int64_t fan_patches = 0;
    for (int64_t k = 0; k < n; ++k)
        if (!grad && items[k].p.bounces > 0 && items[k].p.n_diffuse > 0)
            fan_patches += L.patch_base[k + 1] - L.patch_base[k];
    if (fan_patches > 0) {
        const int64_t resident = (int64_t)g_ws.n_cu * fan_blocks_per_cu(L.count) * (BLOCK / 64);
        L.fans_inline = fan_patches >= 2 * resident;
    }
    // partial slots: one per pass of 64 tasks (emitter, slice of FAN_SLICE fan rays), at
    // most bounces x ceil(n_diffuse / FAN_SLICE) per patch
    L.fan_base.assign(n + 1, 0);
    for (int64_t k = 0; k < n; ++k) {
        L.fan_base[k] = L.total_fan_slots;
        const srp_eval_params &p = items[k].p;
        if (!grad && p.bounces > 0 && p.n_diffuse > 0) {
            const int64_t np = L.patch_base[k + 1] - L.patch_base[k];
            L.total_fan_slots += np * p.bounces * ((p.n_diffuse + FAN_SLICE - 1) / FAN_SLICE);
        }
    }
    L.fan_base[n] = L.total_fan_slots;
    // the fan launch's unit list: room for every pass slot (each patch lists at
    // most its slots)
    L.total_units = L.fans_inline ? 0 : L.total_fan_slots;
    // the work counters are 32-bit and overshoot their range by at most one per wave
    if (L.total_chunks > ((int64_t)1 << 31))
        return fail(SRP_ERR_ARG, "batch too large: more than 2^31 chunks (split it or raise patches per chunk)");
    if (L.total_units > ((int64_t)1 << 31))
        return fail(SRP_ERR_ARG, "batch too large: more than 2^31 diffuse work units (split it)");

    // articulation slots: the scene's current slot, or one per distinct angle
    // vector (equal bits), built on the device
    std::unordered_map<uint64_t, int> head;   // angle hash -> newest slot with it
    L.item_slot.assign(n, -1);
    for (int64_t k = 0; k < n; ++k) {
        const srp_batch_item &it = items[k];
        if (!it.angles) continue;
        const int J = it.scene->h.n_dof;
        uint64_t h = 1469598103934665603ull;   // FNV-1a over the scene address and the angle bytes
        auto mix = [&h](const void *p, size_t len) {
            const unsigned char *b = static_cast<const unsigned char *>(p);
            for (size_t i = 0; i < len; ++i) h = (h ^ b[i]) * 1099511628211ull;
        };
        mix(&it.scene, sizeof it.scene);
        mix(it.angles, sizeof(double) * J);
        auto f = head.find(h);
        int found = -1;
        for (int q = (f == head.end()) ? -1 : f->second; q >= 0; q = L.slots[q].next)
            if (L.slots[q].sc == it.scene && std::memcmp(items[L.slots[q].item].angles, it.angles, sizeof(double) * J) == 0) {
                found = q;
                break;
            }
        if (found < 0) {
            SlotRec r;
            r.sc = it.scene;
            r.item = k;
            r.next = (f == head.end()) ? -1 : f->second;
            r.cs_off = L.total_cs;
            L.total_cs += 2 * (size_t)J;
            r.L = it.scene->slot_L;
            r.off = 0;
            L.slots.push_back(r);
            found = (int)L.slots.size() - 1;
            head[h] = found;
        }
        L.item_slot[k] = found;
    }

    // staging (uploaded every launch): descs | chunk_base | win |
    // evaluation of every range sum | articulation jobs | their cosines and sines
    L.o_desc = 0;
    L.o_cbase = align_up(sizeof(EvalDesc) * n);
    L.o_win = align_up(L.o_cbase + sizeof(int64_t) * (n + 1));
    L.o_seval = align_up(L.o_win + sizeof(uint64_t) * WIN_STRIDE * n);
    L.o_jobs = align_up(L.o_seval + sizeof(uint32_t) * L.slice_base[n]);
    L.o_cs = align_up(L.o_jobs + sizeof(ArtJob) * L.slots.size());
    L.stage_bytes = align_up(L.o_cs + sizeof(double) * L.total_cs);
    // device-only: articulation slots | patch partials | counts | emitter masks
    L.o_slots = L.stage_bytes;
    size_t off = L.o_slots;
    for (auto &sl : L.slots) { sl.off = off; off = align_up(off + sl.L.bytes); }
    // ... | fan pass partials | their counts | emitter records (per item) |
    // gradient partials (per chunk)
    L.o_patches = align_up(off);
    L.o_counts = align_up(L.o_patches + sizeof(PatchOut) * L.total_patches);
    L.o_emask = align_up(L.o_counts + (L.count ? sizeof(uint64_t) * 2 * L.total_patches : 0));
    L.emit_off.assign(n, 0);
    size_t eoff = L.o_emask;
    if (L.total_fan_slots > 0) {
        // masks: SRP_MAX_BOUNCES per patch of every item (only items with fans use theirs)
        L.o_fanout = align_up(L.o_emask + sizeof(uint64_t) * SRP_MAX_BOUNCES * L.total_patches);
        L.o_fancnt = align_up(L.o_fanout + sizeof(PatchOut) * L.total_fan_slots);
        L.o_units = align_up(L.o_fancnt + (L.count ? sizeof(uint64_t) * 2 * L.total_fan_slots : 0));
        eoff = align_up(L.o_units + sizeof(int4) * (size_t)L.total_units);
        for (int64_t k = 0; k < n; ++k) {
            if (L.fan_base[k + 1] == L.fan_base[k]) continue;
            // the records, then one byte per record: the planar instance its rays leave, or -1
            L.emit_off[k] = eoff;
            eoff = align_up(eoff + (sizeof(FanRec) + 1) * 64 * (size_t)items[k].p.bounces *
                                       (L.patch_base[k + 1] - L.patch_base[k]));
        }
    }
    L.o_gpart = eoff;
    L.gpart_off.assign(n, 0);
    L.grad_n.assign(n, 0);
    L.gslice_off.assign(n, 0);
    L.pslice_off.assign(n, 0);
    size_t goff = L.o_gpart;
    for (int64_t k = 0; k < n; ++k) {
        L.pslice_off[k] = goff;
        goff = align_up(goff + sizeof(SliceOut) * L.n_slices[k]);
        if (!grad) continue;
        const int64_t nc = L.chunk_base[k + 1] - L.chunk_base[k];
        L.gpart_off[k] = goff;
        L.grad_n[k] = grad_slots(items[k].scene, items[k].p.flags);
        goff = align_up(goff + sizeof(double) * L.grad_n[k] * nc);
        L.gslice_off[k] = goff;
        goff = align_up(goff + sizeof(double) * L.grad_n[k] * L.n_slices[k]);
    }
    // persistent grids: one chunk (fan unit) per wave at a time, at most bpc resident
    // blocks per CU (the fan kernel: as many as fit)
    const int64_t waves = BLOCK / 64;
    L.grid = (int)std::max<int64_t>(1, std::min<int64_t>((L.total_chunks + waves - 1) / waves,
                                                         (int64_t)g_ws.n_cu * L.sch.bpc));
    if (L.total_units > 0)
        L.fan_grid = (int)std::max<int64_t>(1, std::min<int64_t>((L.total_units + waves - 1) / waves,
                                                                 (int64_t)g_ws.n_cu * fan_blocks_per_cu(L.count)));
    // the work counters (trace kernel's, then fan kernel's, then the count of
    // listed fan units), then the traversal stacks' spill area (per thread of
    // the larger grid: the kernels run one after the other)
    L.o_queue = align_up(goff);
    L.o_spill = align_up(L.o_queue + sizeof(uint32_t) * QUEUE_WORDS);
    L.dev_bytes = align_up(L.o_spill + sizeof(uint32_t) * STACK_SPILL * (size_t)BLOCK * std::max(L.grid, L.fan_grid));
    L.wb = (int)std::min<int64_t>(64, std::max<int64_t>(1, (L.max_wpts + 2047) / 2048));
    return SRP_OK;
}

// Gives a captured forward launch of one patch per chunk its patch order and
// cost arrays (one 32-bit word per patch each, after the rest of the device
// workspace): each launch traces the patches heaviest first by the costs the
// previous launch measured, which shortens the launch's tail when consecutive
// launches see similar images (a propagation's stages; replays of one batch).
// The results do not depend on the order.
void layout_add_order(Layout &L) {
    // (launches of at most 2 blocks per CU: the kernel build that orders its work)
    if (L.grad || L.count || L.sch.bpc > 2 || L.total_patches <= 0) return;
    for (int64_t k = 0; k < L.n; ++k)
        if (L.item_ppc[k] != 1) return;
    L.ordered = true;
    L.o_order = align_up(L.dev_bytes);
    L.o_cost = align_up(L.o_order + sizeof(uint32_t) * (size_t)(L.total_patches + 1));   // (+ launch count)
    L.dev_bytes = align_up(L.o_cost + sizeof(uint32_t) * (size_t)L.total_patches);
}

// Writes the per-launch staging image for device buffer Dv.
void staging_fill(const Layout &L, const srp_batch_item *items, const BatchOut &bo, char *H, char *Dv) {
    const int64_t n = L.n;
    EvalDesc *desc = reinterpret_cast<EvalDesc *>(H + L.o_desc);
    std::memcpy(H + L.o_cbase, L.chunk_base.data(), sizeof(int64_t) * (n + 1));
    uint64_t *win = reinterpret_cast<uint64_t *>(H + L.o_win);
    for (int64_t k = 0; k < WIN_STRIDE * n; ++k) win[k] = enc_f64(INFINITY);
    uint32_t *seval = reinterpret_cast<uint32_t *>(H + L.o_seval);
    for (int64_t k = 0; k < n; ++k)
        for (int64_t q = L.slice_base[k]; q < L.slice_base[k + 1]; ++q) seval[q] = (uint32_t)k;
    ArtJob *jobs = reinterpret_cast<ArtJob *>(H + L.o_jobs);
    double *cs = reinterpret_cast<double *>(H + L.o_cs);
    std::vector<int> slot_clamped(L.slots.size(), 0);
    for (size_t q = 0; q < L.slots.size(); ++q) {
        const SlotRec &sl = L.slots[q];
        const SceneHost &S = sl.sc->h;
        const double *a = items[sl.item].angles;
        double *o = cs + sl.cs_off;
        for (int k = 0; k < S.n_nodes; ++k) {
            const NodeInfo &nd = S.nodes[k];
            for (int x = 0; x < nd.n_axes; ++x) {
                const int j = nd.dof_offset + x;
                const double th = clamp_angle(nd, x, a[j], &slot_clamped[q]);
                o[2 * j] = std::cos(th);
                o[2 * j + 1] = std::sin(th);
            }
        }
        char *base = Dv + sl.off;
        ArtJob &J = jobs[q];
        J.nodes = sl.sc->d_art;
        J.topo = sl.sc->d_topo;
        J.cs = reinterpret_cast<const double *>(Dv + L.o_cs) + sl.cs_off;
        J.inst = reinterpret_cast<Inst *>(base + sl.L.inst);
        J.tlas = reinterpret_cast<BNode4 *>(base + sl.L.tlas);
        J.xf = reinterpret_cast<double *>(base + sl.L.xf);
        J.axw = reinterpret_cast<double *>(base + sl.L.axw);
        J.dof_node = reinterpret_cast<int32_t *>(base + sl.L.dof_node);
        J.pad = S.pad;
        J.n_nodes = S.n_nodes;
        J.n_tlas = (int32_t)S.tlas_topo.size();
        J.max_depth = S.tree_max_depth;
        J.max_height = S.tlas_max_height;
        J.pad_[0] = J.pad_[1] = 0;
    }
    for (int64_t k = 0; k < n; ++k) {
        const srp_batch_item &it = items[k];
        const srp_scene *sc = it.scene;
        EvalDesc &D = desc[k];
        std::memset(&D, 0, sizeof D);
        D.tris = sc->d_tris;
        D.blas = sc->d_blas;
        D.mats = sc->d_mats;
        D.wpts = sc->d_wpts;
        D.n_wpts = (int64_t)sc->h.wpts.size();
        const char *slot_base = (L.item_slot[k] >= 0) ? Dv + L.slots[L.item_slot[k]].off : sc->d_slot;
        const SlotLayout &SL = sc->slot_L;
        const uint32_t root = sc->h.tlas_root;   // every pose shares the topology
        D.inst = reinterpret_cast<const Inst *>(slot_base + SL.inst);
        D.tlas = reinterpret_cast<const BNode4 *>(slot_base + SL.tlas);
        D.xf = reinterpret_cast<const double *>(slot_base + SL.xf);
        D.axw = reinterpret_cast<const double *>(slot_base + SL.axw);
        D.dof_node = reinterpret_cast<const int32_t *>(slot_base + SL.dof_node);
        D.parent = sc->d_parent;
        D.root_ref = root;
        D.n_nodes = sc->h.n_nodes;
        for (int32_t j = 0; j < sc->h.n_nodes; ++j)
            if (sc->h.nodes[j].planar) D.planar[j >> 6] |= 1ull << (j & 63);
        D.n_mats = sc->h.n_mats;
        D.n_dof = sc->h.n_dof;
        basis(it.p.sun_dir, D.u, D.v, D.d);
        D.pressure = it.p.pressure;
        for (int c = 0; c < 3; ++c) D.ref[c] = it.p.ref[c];
        D.n = it.p.n;
        D.bounces = it.p.bounces;
        D.flags = it.p.flags;
        D.n_diffuse = it.p.n_diffuse;
        D.dset = it.p.n_diffuse > 0 ? g_ws.d_dset + 4 * dset_entry(it.p.n_diffuse) : nullptr;
        D.tiles_x = L.tiles_x[k];
        D.tiles_y = L.tiles_y[k];
        D.ppc = L.item_ppc[k];
        D.chunk_base = L.chunk_base[k];
        D.n_chunks = L.chunk_base[k + 1] - L.chunk_base[k];
        D.patch_base = L.patch_base[k];
        D.n_patches = L.patch_base[k + 1] - L.patch_base[k];
        const bool fans = L.fan_base[k + 1] > L.fan_base[k];
        D.emit = fans ? reinterpret_cast<FanRec *>(Dv + L.emit_off[k]) : nullptr;
        D.emit_mask = fans ? reinterpret_cast<uint64_t *>(Dv + L.o_emask) + SRP_MAX_BOUNCES * D.patch_base : nullptr;
        D.fan_base = L.fan_base[k];
        D.grad_n = L.grad ? L.grad_n[k] : 0;   // the per-chunk size the partials were allocated with
        D.grad_part = L.grad ? reinterpret_cast<double *>(Dv + L.gpart_off[k]) : nullptr;
        D.n_slices = L.n_slices[k];
        D.slice_base = L.slice_base[k];
        D.n_clamped = L.item_slot[k] >= 0 ? slot_clamped[L.item_slot[k]] : sc->cur.n_clamped;
        D.pslice = reinterpret_cast<SliceOut *>(Dv + L.pslice_off[k]);
        D.gslice = L.grad ? reinterpret_cast<double *>(Dv + L.gslice_off[k]) : nullptr;
        D.grad_out = (L.grad && bo.d_grad) ? bo.d_grad + k * bo.grad_stride : nullptr;
        D.hit_ids = (n == 1) ? bo.d_hit_ids : nullptr;
        D.hit_t = (n == 1) ? bo.d_hit_t : nullptr;
    }
}

// Upload + window + trace + reduce (+ optional result copy) on `stream`.
int enqueue(const Layout &L, char *Dv, const char *H, size_t copy_bytes, const BatchOut &bo, hipStream_t stream,
            bool profile, hipEvent_t copied = nullptr) {
    std::pair<hipEvent_t, hipEvent_t> whole{};
    if (profile) {
        int rc = prof_event_pair(&whole);
        if (rc) return rc;
        HIPCHK(hipEventRecord(whole.first, stream));
    }
    HIPCHK(hipMemcpyAsync(Dv, H, copy_bytes, hipMemcpyHostToDevice, stream));
    if (copied) HIPCHK(hipEventRecord(copied, stream));
    if (!L.slots.empty()) {
        int e = launch_articulate(reinterpret_cast<const ArtJob *>(Dv + L.o_jobs), (int)L.slots.size(), stream);
        if (e) return fail(SRP_ERR_DEVICE, std::string("articulation kernel: ") + hipGetErrorString((hipError_t)e));
    }
    const EvalDesc *d_desc = reinterpret_cast<const EvalDesc *>(Dv + L.o_desc);
    const int64_t *d_cbase = reinterpret_cast<const int64_t *>(Dv + L.o_cbase);
    uint64_t *d_win = reinterpret_cast<uint64_t *>(Dv + L.o_win);
    PatchOut *d_patches = reinterpret_cast<PatchOut *>(Dv + L.o_patches);
    uint64_t *d_counts = L.count ? reinterpret_cast<uint64_t *>(Dv + L.o_counts) : nullptr;
    uint32_t *d_queue = reinterpret_cast<uint32_t *>(Dv + L.o_queue);
    uint32_t *d_spill = reinterpret_cast<uint32_t *>(Dv + L.o_spill);
    uint32_t *d_order = L.ordered ? reinterpret_cast<uint32_t *>(Dv + L.o_order) : nullptr;
    uint32_t *d_cost = L.ordered ? reinterpret_cast<uint32_t *>(Dv + L.o_cost) : nullptr;
    int e = launch_window(d_desc, (int)L.n, L.wb, d_win, d_queue, stream);
    if (e) return fail(SRP_ERR_DEVICE, std::string("window kernel: ") + hipGetErrorString((hipError_t)e));
    std::pair<hipEvent_t, hipEvent_t> ev{};
    if (profile) {
        int rc = prof_event_pair(&ev);
        if (rc) return rc;
        HIPCHK(hipEventRecord(ev.first, stream));
    }
    PatchOut *d_fan_out = nullptr;
    uint64_t *d_fan_counts = nullptr;
    if (L.total_fan_slots > 0) {
        d_fan_out = reinterpret_cast<PatchOut *>(Dv + L.o_fanout);
        d_fan_counts = L.count ? reinterpret_cast<uint64_t *>(Dv + L.o_fancnt) : nullptr;
    }
    int4 *d_units = L.total_units > 0 ? reinterpret_cast<int4 *>(Dv + L.o_units) : nullptr;
    e = launch_trace(d_desc, d_cbase, (int)L.n, d_win, L.total_chunks, d_queue, d_spill, d_patches, d_counts, L.count,
                     L.grad, L.dir, L.grid, L.max_grad_n, d_fan_out, d_fan_counts, L.fans_inline, d_units, L.sch.bpc,
                     d_order, d_cost, stream);
    if (e) return fail(SRP_ERR_DEVICE, std::string("trace kernel: ") + hipGetErrorString((hipError_t)e));
    if (L.total_units > 0) {
        e = launch_fans(d_desc, d_win, L.total_units, d_queue, d_spill, d_fan_out, d_fan_counts, d_units, L.count,
                        L.fan_grid, stream);
        if (e) return fail(SRP_ERR_DEVICE, std::string("fan kernel: ") + hipGetErrorString((hipError_t)e));
    }
    if (profile) {   // the ray-tracing kernels: trace, then fans
        HIPCHK(hipEventRecord(ev.second, stream));
        g_prof.pairs.push_back(ev);
    }
    e = launch_reduce(d_desc, (int)L.n, d_win, d_patches, d_counts, d_fan_out, d_fan_counts, L.count, L.grad,
                      reinterpret_cast<const uint32_t *>(Dv + L.o_seval), L.slice_base[L.n], bo.d_out, d_order, d_cost,
                      d_order ? d_order + L.total_patches : nullptr, stream);
    if (e) return fail(SRP_ERR_DEVICE, std::string("reduce kernel: ") + hipGetErrorString((hipError_t)e));
    if (bo.h_copy) HIPCHK(hipMemcpyAsync(bo.h_copy, bo.d_out, sizeof(srp_result) * L.n, hipMemcpyDeviceToHost, stream));
    if (profile) {
        HIPCHK(hipEventRecord(whole.second, stream));
        g_prof.whole.push_back(whole);
    }
    return SRP_OK;
}

// Queues one batch on `stream` through the shared workspace.  Caller holds g_ws.mu.
// A batch whose device workspace would exceed WORKSPACE_CAP is split into
// halves, run one after the other (results land at their items' offsets).
int run_batch(const srp_batch_item *items, int64_t n, bool grad, const BatchOut &bo, hipStream_t stream,
              Schedule force = Schedule()) {
    if (n <= 0) return SRP_OK;
    int rc = check_items(items, n, grad, bo);
    if (rc) return rc;
    Layout L;
    if ((rc = layout_build(items, n, grad, force, &L))) return rc;
    if (L.dev_bytes > WORKSPACE_CAP && n > 1) {
        const int64_t h = n / 2;
        BatchOut b2 = bo;
        b2.d_out = bo.d_out + h;
        if (bo.d_grad) b2.d_grad = bo.d_grad + h * bo.grad_stride;
        if (bo.h_copy) b2.h_copy = bo.h_copy + h;
        if ((rc = run_batch(items, h, grad, bo, stream, force))) return rc;
        return run_batch(items + h, n - h, grad, b2, stream, force);
    }
    if (g_ws.pending) {
        // the pinned staging image may be rewritten once the last batch's upload is
        // done (the host prepares this batch while that one runs); the device
        // workspace is reused on `stream` only after the last batch finished
        HIPCHK(hipEventSynchronize(g_ws.copied));
        HIPCHK(hipStreamWaitEvent(stream, g_ws.done, 0));
    }
    if ((rc = ws_reserve(L.dev_bytes, L.stage_bytes))) return rc;   // (waits for the last batch to grow)
    staging_fill(L, items, bo, g_ws.h_stage, g_ws.d_buf);
    if ((rc = enqueue(L, g_ws.d_buf, g_ws.h_stage, L.stage_bytes, bo, stream, g_prof.on, g_ws.copied))) return rc;
    HIPCHK(hipEventRecord(g_ws.done, stream));
    g_ws.pending = true;
    return SRP_OK;
}

// Host staging image of srp_eval_batch_noalloc (descriptors, chunk bases,
// window slots, articulation slots): a fixed buffer, uploaded from pageable
// memory (the copy has consumed it when hipMemcpyAsync returns).
constexpr size_t NOALLOC_STAGE_BYTES = (size_t)4 << 20;
alignas(256) char g_noalloc_stage[NOALLOC_STAGE_BYTES];

// Shrinks the persistent grids of L until its device workspace fits `cap`
// bytes (only the traversal stacks' spill area depends on the grid size);
// fails when even one block does not fit.
int layout_fit(Layout *Lp, size_t cap) {
    Layout &L = *Lp;
    const size_t per_block = sizeof(uint32_t) * STACK_SPILL * (size_t)BLOCK;
    if (L.o_spill + per_block > cap)
        return fail(SRP_ERR_ARG, "batch too large for the fixed workspace: it needs " +
                                     std::to_string(L.o_spill + per_block) + " bytes of the " +
                                     std::to_string(cap) + " available (split it)");
    const int max_blocks = (int)std::min<size_t>((cap - L.o_spill) / per_block, 1 << 30);
    if (L.grid > max_blocks) L.grid = max_blocks;
    if (L.fan_grid > max_blocks) L.fan_grid = max_blocks;
    L.dev_bytes = align_up(L.o_spill + per_block * (size_t)std::max(L.grid, L.fan_grid));
    return SRP_OK;
}

}  // namespace

// A captured launch sequence (upload, window, trace, reduce, result copy)
// for a fixed batch layout, replayed with new Sun directions, pressures and
// angle values by rewriting its pinned staging image.
struct PlanImpl {
    Layout L;
    BatchOut bo;
    int64_t grad_stride = 0;
    char *d_buf = nullptr;
    char *h_stage = nullptr;
    hipStream_t cs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
    bool pending = false;
};

namespace {

void plan_free(PlanImpl *P) {
    if (!P) return;
    if (P->pending && P->done) (void)hipEventSynchronize(P->done);
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    if (P->cs) (void)hipStreamDestroy(P->cs);
    if (P->done) (void)hipEventDestroy(P->done);
    if (P->d_buf) (void)hipFree(P->d_buf);
    if (P->h_stage) (void)hipHostFree(P->h_stage);
    delete P;
}

// Builds buffers and captures the graph.  Caller holds g_ws.mu.
int plan_make(const srp_batch_item *items, int64_t n, bool grad, const BatchOut &bo, PlanImpl **out) {
    int rc = check_items(items, n, grad, bo);
    if (rc) return rc;
    PlanImpl *P = new (std::nothrow) PlanImpl();
    if (!P) return fail(SRP_ERR_OOM, "host allocation failed");
    P->bo = bo;
    if ((rc = layout_build(items, n, grad, Schedule(), &P->L))) { plan_free(P); return rc; }
    layout_add_order(P->L);
    if (hipMalloc(&P->d_buf, std::max<size_t>(P->L.dev_bytes, 256)) != hipSuccess) {
        (void)hipGetLastError();
        plan_free(P);
        return fail(SRP_ERR_OOM, "plan device allocation failed");
    }
    if (P->L.ordered) {
        // the first launch traces every evaluation's patches in image order (the
        // word after the order counts the plan's launches)
        std::vector<uint32_t> ident((size_t)P->L.total_patches + 1, 0u);
        for (int64_t k = 0; k < n; ++k)
            for (int64_t q = P->L.patch_base[k]; q < P->L.patch_base[k + 1]; ++q)
                ident[(size_t)q] = (uint32_t)(q - P->L.patch_base[k]);
        hipError_t e1 = hipMemcpy(P->d_buf + P->L.o_order, ident.data(), sizeof(uint32_t) * ident.size(),
                                  hipMemcpyHostToDevice);
        hipError_t e2 = hipMemset(P->d_buf + P->L.o_cost, 0, sizeof(uint32_t) * (size_t)P->L.total_patches);
        if (e1 != hipSuccess || e2 != hipSuccess) {
            plan_free(P);
            return fail(SRP_ERR_DEVICE, std::string("plan order setup: ") +
                                            hipGetErrorString(e1 != hipSuccess ? e1 : e2));
        }
    }
    if (hipHostMalloc(&P->h_stage, std::max<size_t>(P->L.stage_bytes, 256), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        plan_free(P);
        return fail(SRP_ERR_OOM, "plan staging allocation failed");
    }
    staging_fill(P->L, items, P->bo, P->h_stage, P->d_buf);
    auto dev = [&](hipError_t e, const char *what) {
        if (e == hipSuccess) return SRP_OK;
        return fail(SRP_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    };
    if ((rc = dev(hipStreamCreateWithFlags(&P->cs, hipStreamNonBlocking), "hipStreamCreate")) ||
        (rc = dev(hipEventCreateWithFlags(&P->done, hipEventDisableTiming), "hipEventCreate")) ||
        (rc = dev(hipStreamBeginCapture(P->cs, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture"))) {
        plan_free(P);
        return rc;
    }
    rc = enqueue(P->L, P->d_buf, P->h_stage, P->L.stage_bytes, P->bo, P->cs, false);
    hipGraph_t g = nullptr;
    hipError_t ee = hipStreamEndCapture(P->cs, &g);
    P->graph = g;
    if (rc) { plan_free(P); return rc; }
    if ((rc = dev(ee, "hipStreamEndCapture")) ||
        (rc = dev(hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0), "hipGraphInstantiate"))) {
        plan_free(P);
        return rc;
    }
    *out = P;
    return SRP_OK;
}

// Rewrites the staging image for new item values; false if the layout differs.
int plan_refill(PlanImpl *P, const srp_batch_item *items, int64_t n, bool *compatible) {
    *compatible = false;
    int rc = check_items(items, n, P->L.grad, P->bo);
    if (rc) return rc;
    Layout L2;
    if ((rc = layout_build(items, n, P->L.grad, P->L.sch, &L2))) return rc;
    if (P->L.ordered) layout_add_order(L2);
    const Layout &L = P->L;
    if (L2.n != L.n || L2.stage_bytes != L.stage_bytes || L2.dev_bytes > L.dev_bytes || L2.grid != L.grid ||
        L2.wb != L.wb || L2.count != L.count || L2.dir != L.dir || L2.max_grad_n != L.max_grad_n ||
        L2.grad_n != L.grad_n || L2.chunk_base != L.chunk_base ||
        L2.patch_base != L.patch_base || L2.o_patches != L.o_patches || L2.o_counts != L.o_counts ||
        L2.total_units != L.total_units || L2.fan_base != L.fan_base || L2.fan_grid != L.fan_grid ||
        L2.o_units != L.o_units || L2.fans_inline != L.fans_inline ||
        L2.emit_off != L.emit_off ||
        L2.o_emask != L.o_emask || L2.o_fanout != L.o_fanout || L2.o_fancnt != L.o_fancnt ||
        L2.o_queue != L.o_queue || L2.o_spill != L.o_spill || L2.slots.size() != L.slots.size() ||
        L2.o_jobs != L.o_jobs || L2.o_cs != L.o_cs || L2.o_slots != L.o_slots || L2.ordered != L.ordered ||
        L2.o_order != L.o_order || L2.o_cost != L.o_cost)
        return SRP_OK;
    for (size_t q = 0; q < L.slots.size(); ++q)
        if (L2.slots[q].off != L.slots[q].off || L2.slots[q].sc != L.slots[q].sc) return SRP_OK;
    if (P->pending) HIPCHK(hipEventSynchronize(P->done));
    P->pending = false;
    P->L = std::move(L2);
    staging_fill(P->L, items, P->bo, P->h_stage, P->d_buf);
    *compatible = true;
    return SRP_OK;
}

int upload_slot(srp_scene *sc) {
    std::vector<char> buf(sc->slot_L.bytes, 0);
    slot_pack(sc->cur, sc->slot_L, buf.data());
    HIPCHK(hipMemcpy(sc->d_slot, buf.data(), buf.size(), hipMemcpyHostToDevice));
    return SRP_OK;
}

void free_scene(srp_scene *sc) {
    if (!sc) return;
    for (auto &kv : sc->eval_plans) plan_free(kv.second);
    sc->eval_plans.clear();
    if (sc->d_res) (void)hipFree(sc->d_res);
    if (sc->h_res) (void)hipHostFree(sc->h_res);
    (void)hipFree(sc->d_tris);
    (void)hipFree(sc->d_blas);
    (void)hipFree(sc->d_mats);
    (void)hipFree(sc->d_wpts);
    (void)hipFree(sc->d_parent);
    (void)hipFree(sc->d_art);
    (void)hipFree(sc->d_topo);
    (void)hipFree(sc->d_slot);
    delete sc;
}

template <typename T>
int dev_upload(T **dst, const std::vector<T> &src) {
    size_t bytes = std::max<size_t>(sizeof(T) * src.size(), 256);
    if (hipMalloc(dst, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *dst = nullptr;
        return fail(SRP_ERR_OOM, "device allocation failed");
    }
    if (!src.empty()) HIPCHK(hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice));
    return SRP_OK;
}

}  // namespace

namespace srp {
// One evaluation (srp_eval) with explicit hinge angles for this evaluation
// only (NULL: the scene's current angles): the item's articulation slot is
// built by the articulation kernel inside the captured launch, so a caller
// that changes the angles at every evaluation (a sun-tracking propagation)
// needs no host slot build and no synchronous upload.  The scene's current
// angles are not changed.
int eval_single(srp_scene *scene, const srp_eval_params *params, const double *angles, srp_result *out,
                int32_t *hit_ids, float *hit_t) {
    if (!scene || !params || !out) return fail(SRP_ERR_ARG, "null scene, params or out");
    int rc = check_params(params);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_ws.mu);
    if ((rc = ws_init())) return rc;
    srp_batch_item it{scene, angles, *params};
    if ((rc = check_items(&it, 1, false, BatchOut()))) return rc;
    if (!scene->d_res) {
        if (hipMalloc(&scene->d_res, sizeof(srp_result)) != hipSuccess) { (void)hipGetLastError(); return fail(SRP_ERR_OOM, "result allocation failed"); }
        if (hipHostMalloc(&scene->h_res, sizeof(srp_result), hipHostMallocDefault) != hipSuccess) { (void)hipGetLastError(); return fail(SRP_ERR_OOM, "pinned result allocation failed"); }
    }
    const size_t R = (size_t)params->bounces + 1 + (size_t)params->bounces * params->n_diffuse;
    size_t nrec = (hit_ids || hit_t) ? (size_t)params->n * params->n * R : 0;
    if (nrec) {
        // recorded evaluations (tests, fixed-visibility checks) take the direct path
        static char *d_rec = nullptr;
        static size_t rec_cap = 0;
        if (nrec * 8 > rec_cap) {
            if ((rc = ws_wait())) return rc;
            if (d_rec) HIPCHK(hipFree(d_rec));
            d_rec = nullptr;
            if (hipMalloc(&d_rec, nrec * 8) != hipSuccess) {
                (void)hipGetLastError();
                rec_cap = 0;
                return fail(SRP_ERR_OOM, "record buffer allocation failed");
            }
            rec_cap = nrec * 8;
        }
        BatchOut bo;
        bo.d_out = scene->d_res;
        bo.h_copy = scene->h_res;
        bo.d_hit_ids = reinterpret_cast<int32_t *>(d_rec);
        bo.d_hit_t = reinterpret_cast<float *>(d_rec + nrec * 4);
        if ((rc = run_batch(&it, 1, false, bo, g_ws.stream))) return rc;
        HIPCHK(hipStreamSynchronize(g_ws.stream));
        g_ws.pending = false;
        *out = *scene->h_res;
        if (hit_ids) HIPCHK(hipMemcpy(hit_ids, d_rec, nrec * 4, hipMemcpyDeviceToHost));
        if (hit_t) HIPCHK(hipMemcpy(hit_t, d_rec + nrec * 4, nrec * 4, hipMemcpyDeviceToHost));
    } else {
        // replay of a captured single-evaluation launch (one graph launch + one sync)
        uint64_t key = ((uint64_t)params->n << 24) | ((uint64_t)params->n_diffuse << 16) |
                       ((uint64_t)params->bounces << 8) | params->flags | (angles ? (1ull << 63) : 0);
        PlanImpl *P = nullptr;
        auto f = scene->eval_plans.find(key);
        if (f != scene->eval_plans.end()) {
            P = f->second;
            bool ok = false;
            if ((rc = plan_refill(P, &it, 1, &ok))) return rc;
            if (!ok) {
                plan_free(P);
                scene->eval_plans.erase(f);
                P = nullptr;
            }
        }
        if (!P) {
            if ((rc = ws_wait())) return rc;
            BatchOut bo;
            bo.d_out = scene->d_res;
            bo.h_copy = scene->h_res;
            if ((rc = plan_make(&it, 1, false, bo, &P))) return rc;
            scene->eval_plans[key] = P;
        }
        HIPCHK(hipGraphLaunch(P->exec, g_ws.stream));
        HIPCHK(hipStreamSynchronize(g_ws.stream));
        *out = *scene->h_res;
    }
    if (out->status & SRP_STATUS_STACK) return fail(SRP_ERR_DEPTH, "traversal stack overflow");
    return SRP_OK;
}


const SceneHost &scene_host(const srp_scene *sc) { return sc->h; }
int scene_rest_normal(const srp_scene *sc, int node, double n0[3]) {
    for (int a = 0; a < 3; ++a) n0[a] = sc->h.nodes[node].n0[a];
    return SRP_OK;
}
void set_error(const std::string &msg) { g_err = msg; }
}  // namespace srp

extern "C" {

const char *srp_last_error(void) { return g_err.c_str(); }

int srp_build_scene(const double *verts, int64_t n_verts, const int32_t *tris, int64_t n_tris,
                    const int32_t *tri_material, const int32_t *tri_node, const srp_material *mats,
                    int32_t n_mats, const srp_node *nodes, int32_t n_nodes, srp_scene **out) {
    g_err.clear();
    if (!out) return fail(SRP_ERR_ARG, "null out");
    srp_scene *sc = new (std::nothrow) srp_scene();
    if (!sc) return fail(SRP_ERR_OOM, "host allocation failed");
    int rc;
    try {
        // host-side validation and hierarchy build first: no device call before the inputs pass
        rc = scene_build(verts, n_verts, tris, n_tris, tri_material, tri_node, mats, n_mats, nodes, n_nodes, &sc->h,
                         &g_err);
        if (!rc) rc = slot_build(sc->h, nullptr, &sc->cur, &g_err);
        if (!rc) plates_build(&sc->h);
    } catch (const std::bad_alloc &) {
        rc = fail(SRP_ERR_OOM, "host allocation failed");
    }
    if (rc) { free_scene(sc); return rc; }
    std::lock_guard<std::mutex> lk(g_ws.mu);
    if ((rc = ws_init())) { free_scene(sc); return rc; }
    sc->device = g_ws.device;
    sc->angles.assign(sc->h.n_dof, 0.0);
    sc->slot_L = slot_layout(sc->h.n_nodes, std::max((int)sc->h.tlas_topo.size(), 1), sc->h.n_dof);
    if ((rc = dev_upload(&sc->d_tris, sc->h.tris)) || (rc = dev_upload(&sc->d_blas, sc->h.blas)) ||
        (rc = dev_upload(&sc->d_mats, sc->h.mats)) || (rc = dev_upload(&sc->d_wpts, sc->h.wpts)) ||
        (rc = dev_upload(&sc->d_parent, sc->h.parent)) || (rc = dev_upload(&sc->d_art, art_nodes(sc->h))) ||
        (rc = dev_upload(&sc->d_topo, sc->h.tlas_topo))) {
        free_scene(sc);
        return rc;
    }
    if (hipMalloc(&sc->d_slot, sc->slot_L.bytes) != hipSuccess) {
        (void)hipGetLastError();
        free_scene(sc);
        return fail(SRP_ERR_OOM, "device allocation failed");
    }
    if ((rc = upload_slot(sc))) { free_scene(sc); return rc; }
    // the host copies of the large arrays are no longer needed
    std::vector<TriRec>().swap(sc->h.tris);
    std::vector<BNode4>().swap(sc->h.blas);
    sc->h.wpts.shrink_to_fit();
    *out = sc;
    return SRP_OK;
}

int srp_destroy_scene(srp_scene *scene) {
    g_err.clear();
    if (!scene) return SRP_OK;
    std::lock_guard<std::mutex> lk(g_ws.mu);
    int rc = ws_wait();
    free_scene(scene);
    return rc;
}

int32_t srp_scene_n_dof(const srp_scene *scene) {
    if (!scene) return fail(SRP_ERR_ARG, "null scene");
    return scene->h.n_dof;
}

int srp_set_materials(srp_scene *scene, const srp_material *mats, int32_t n_mats) {
    g_err.clear();
    if (!scene) return fail(SRP_ERR_ARG, "null scene");
    int rc = validate_materials(mats, n_mats, &g_err);
    if (rc) return rc;
    if (n_mats != scene->h.n_mats) return fail(SRP_ERR_ARG, "material count differs from the scene's");
    std::lock_guard<std::mutex> lk(g_ws.mu);
    if ((rc = ws_wait())) return rc;
    for (int m = 0; m < n_mats; ++m) {
        scene->h.mats[2 * m] = (float)mats[m].rho_s;
        scene->h.mats[2 * m + 1] = (float)mats[m].rho_d;
    }
    HIPCHK(hipMemcpy(scene->d_mats, scene->h.mats.data(), sizeof(float) * scene->h.mats.size(), hipMemcpyHostToDevice));
    return SRP_OK;
}

int srp_set_panel_angles(srp_scene *scene, const double *angles, int32_t n_dof) {
    g_err.clear();
    if (!scene) return fail(SRP_ERR_ARG, "null scene");
    if (n_dof != scene->h.n_dof) return fail(SRP_ERR_ARG, "n_dof differs from the scene's");
    if (n_dof > 0 && !angles) return fail(SRP_ERR_ARG, "null angles");
    SlotHost s;
    int rc = slot_build(scene->h, angles, &s, &g_err);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_ws.mu);
    if ((rc = ws_wait())) return rc;
    scene->cur = std::move(s);
    scene->angles.assign(angles, angles + n_dof);
    if ((rc = upload_slot(scene))) return rc;
    return scene->cur.n_clamped;
}

int srp_nplate_from_scene(srp_scene *scene, const double *angles, srp_plate *plates, int32_t max_plates,
                          int32_t *n_plates) {
    g_err.clear();
    if (!scene || !n_plates || (max_plates > 0 && !plates) || max_plates < 0)
        return fail(SRP_ERR_ARG, "null scene, plates or count");
    SlotHost own;
    const SlotHost *slot = &scene->cur;
    if (angles) {
        int rc = slot_build(scene->h, angles, &own, &g_err);
        if (rc) return rc;
        slot = &own;
    }
    // the scene's plates, moved rigidly with their nodes
    const std::vector<PlateLocal> &pl = scene->h.plates;
    if (pl.size() > (size_t)INT32_MAX) return fail(SRP_ERR_ARG, "too many plates");
    *n_plates = (int32_t)pl.size();
    if ((int64_t)pl.size() > max_plates)
        return fail(SRP_ERR_ARG, "max_plates too small: " + std::to_string(pl.size()) + " plates");
    plates_world(scene->h, *slot, plates);
    return SRP_OK;
}

int srp_eval(srp_scene *scene, const srp_eval_params *params, srp_result *out, int32_t *hit_ids, float *hit_t) {
    g_err.clear();
    return eval_single(scene, params, nullptr, out, hit_ids, hit_t);
}

int srp_eval_batch(const srp_batch_item *items, int64_t n_items, srp_result *out_dev, void *hip_stream) {
    g_err.clear();
    if (n_items < 0 || (n_items > 0 && (!items || !out_dev))) return fail(SRP_ERR_ARG, "null items or out_dev");
    std::lock_guard<std::mutex> lk(g_ws.mu);
    int rc = ws_init();
    if (rc) return rc;
    BatchOut bo;
    bo.d_out = out_dev;
    return run_batch(items, n_items, false, bo, (hipStream_t)hip_stream);
}

int srp_eval_batch_noalloc(const srp_batch_item *items, int64_t n_items, srp_result *out_dev, void *hip_stream) {
    g_err.clear();
    if (n_items < 0 || (n_items > 0 && (!items || !out_dev))) return fail(SRP_ERR_ARG, "null items or out_dev");
    if (n_items == 0) return SRP_OK;
    std::lock_guard<std::mutex> lk(g_ws.mu);
    // every item's scene was built, so the library is initialised on its device
    // (scratch address looked up); nothing here allocates
    if (!g_ws.init) return fail(SRP_ERR_ARG, "no scene has been built");
    char *scr = noalloc_scratch(g_ws.device);
    if (!scr) return fail(SRP_ERR_DEVICE, "no scratch address for this device");
    BatchOut bo;
    bo.d_out = out_dev;
    int rc = check_items(items, n_items, false, bo);
    if (rc) return rc;
    Layout L;
    if ((rc = layout_build(items, n_items, false, Schedule(), &L))) return rc;
    if ((rc = layout_fit(&L, NOALLOC_SCRATCH_BYTES))) return rc;
    if (L.stage_bytes > NOALLOC_STAGE_BYTES)
        return fail(SRP_ERR_ARG, "batch too large for the fixed staging area: " + std::to_string(L.stage_bytes) +
                                     " bytes of " + std::to_string(NOALLOC_STAGE_BYTES) + " (split it)");
    staging_fill(L, items, bo, g_noalloc_stage, scr);
    return enqueue(L, scr, g_noalloc_stage, L.stage_bytes, bo, (hipStream_t)hip_stream, false);
}

int srp_eval_grad_batch(const srp_batch_item *items, int64_t n_items, srp_result *out_dev, double *grad_dev,
                        int64_t grad_stride, void *hip_stream) {
    g_err.clear();
    if (n_items < 0 || (n_items > 0 && (!items || !out_dev || !grad_dev)))
        return fail(SRP_ERR_ARG, "null items, out_dev or grad_dev");
    std::lock_guard<std::mutex> lk(g_ws.mu);
    int rc = ws_init();
    if (rc) return rc;
    BatchOut bo;
    bo.d_out = out_dev;
    bo.d_grad = grad_dev;
    bo.grad_stride = grad_stride;
    return run_batch(items, n_items, true, bo, (hipStream_t)hip_stream);
}

int srp_eval_grad(srp_scene *scene, const srp_eval_params *params, srp_result *out, double *dF_drho_s,
                  double *dF_drho_d, double *dF_dtheta, double *dF_ddir) {
    g_err.clear();
    if (!scene || !params || !out) return fail(SRP_ERR_ARG, "null scene, params or out");
    int rc = check_params(params);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_ws.mu);
    if ((rc = ws_init())) return rc;
    const int M = scene->h.n_mats, J = scene->h.n_dof;
    const size_t gsz = (size_t)grad_out_size(scene);
    static char *d_buf = nullptr;
    static size_t cap = 0;
    size_t need = sizeof(srp_result) + sizeof(double) * gsz + 256;
    if (need > cap) {
        if ((rc = ws_wait())) return rc;
        if (d_buf) HIPCHK(hipFree(d_buf));
        d_buf = nullptr;
        if (hipMalloc(&d_buf, need) != hipSuccess) {
            (void)hipGetLastError();
            cap = 0;
            return fail(SRP_ERR_OOM, "gradient buffer allocation failed");
        }
        cap = need;
    }
    srp_batch_item it{scene, nullptr, *params};
    if (dF_ddir) it.p.flags |= SRP_F_GRAD_DIR;
    else it.p.flags &= ~(uint32_t)SRP_F_GRAD_DIR;
    BatchOut bo;
    bo.d_out = reinterpret_cast<srp_result *>(d_buf);
    bo.d_grad = reinterpret_cast<double *>(d_buf + 256);
    bo.grad_stride = (int64_t)gsz;
    if ((rc = run_batch(&it, 1, true, bo, g_ws.stream))) return rc;
    std::vector<double> g(gsz);
    HIPCHK(hipStreamSynchronize(g_ws.stream));
    g_ws.pending = false;
    HIPCHK(hipMemcpy(out, d_buf, sizeof(srp_result), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(g.data(), d_buf + 256, sizeof(double) * gsz, hipMemcpyDeviceToHost));
    if (dF_drho_s) std::memcpy(dF_drho_s, g.data(), sizeof(double) * 3 * M);
    if (dF_drho_d) std::memcpy(dF_drho_d, g.data() + 3 * M, sizeof(double) * 3 * M);
    if (dF_dtheta) std::memcpy(dF_dtheta, g.data() + 6 * M, sizeof(double) * 3 * J);
    if (dF_ddir) std::memcpy(dF_ddir, g.data() + 6 * M + 3 * J, sizeof(double) * 9);
    if (out->status & SRP_STATUS_STACK) return fail(SRP_ERR_DEPTH, "traversal stack overflow");
    return SRP_OK;
}

struct srp_plan {
    PlanImpl *impl;
};

int srp_plan_create(const srp_batch_item *items, int64_t n_items, int32_t flags, srp_result *out_dev,
                    double *grad_dev, int64_t grad_stride, srp_plan **out) {
    g_err.clear();
    if (!out || n_items <= 0 || !items || !out_dev) return fail(SRP_ERR_ARG, "null or empty arguments");
    bool grad = (flags & SRP_PLAN_GRAD) != 0;
    if (grad && !grad_dev) return fail(SRP_ERR_ARG, "gradient plan without grad_dev");
    if (flags & ~(int32_t)SRP_PLAN_GRAD) return fail(SRP_ERR_ARG, "unknown plan flags");
    std::lock_guard<std::mutex> lk(g_ws.mu);
    int rc = ws_init();
    if (rc) return rc;
    BatchOut bo;
    bo.d_out = out_dev;
    bo.d_grad = grad ? grad_dev : nullptr;
    bo.grad_stride = grad_stride;
    PlanImpl *P = nullptr;
    if ((rc = plan_make(items, n_items, grad, bo, &P))) return rc;
    srp_plan *h = new (std::nothrow) srp_plan{P};
    if (!h) { plan_free(P); return fail(SRP_ERR_OOM, "host allocation failed"); }
    *out = h;
    return SRP_OK;
}

int srp_plan_update(srp_plan *plan, const srp_batch_item *items, int64_t n_items) {
    g_err.clear();
    if (!plan || !items) return fail(SRP_ERR_ARG, "null argument");
    std::lock_guard<std::mutex> lk(g_ws.mu);
    bool ok = false;
    int rc = plan_refill(plan->impl, items, n_items, &ok);
    if (rc) return rc;
    if (!ok) {
        // layout changed (item count, grid sizes, scenes or number of distinct angle sets): recapture
        PlanImpl *P = nullptr;
        if ((rc = plan_make(items, n_items, plan->impl->L.grad, plan->impl->bo, &P))) return rc;
        plan_free(plan->impl);
        plan->impl = P;
    }
    return SRP_OK;
}

int srp_plan_launch(srp_plan *plan, void *hip_stream) {
    g_err.clear();
    if (!plan) return fail(SRP_ERR_ARG, "null plan");
    std::lock_guard<std::mutex> lk(g_ws.mu);
    PlanImpl *P = plan->impl;
    if (P->pending) HIPCHK(hipEventSynchronize(P->done));   // staging may have been rewritten
    HIPCHK(hipGraphLaunch(P->exec, (hipStream_t)hip_stream));
    HIPCHK(hipEventRecord(P->done, (hipStream_t)hip_stream));
    P->pending = true;
    return SRP_OK;
}

int srp_plan_destroy(srp_plan *plan) {
    g_err.clear();
    if (!plan) return SRP_OK;
    std::lock_guard<std::mutex> lk(g_ws.mu);
    plan_free(plan->impl);
    delete plan;
    return SRP_OK;
}

int srp_set_schedule(int32_t patches_per_chunk, int32_t blocks_per_cu) {
    g_err.clear();
    if (patches_per_chunk < 0 || patches_per_chunk > MAX_PPC || blocks_per_cu < 0 || blocks_per_cu > 64)
        return fail(SRP_ERR_ARG, "schedule out of range");
    std::lock_guard<std::mutex> lk(g_ws.mu);
    g_override.ppc = patches_per_chunk;
    g_override.bpc = blocks_per_cu;
    return SRP_OK;
}

int srp_autotune(const srp_batch_item *items, int64_t n_items, int32_t flags, int32_t *patches_per_chunk,
                 int32_t *blocks_per_cu, double *best_ms) {
    g_err.clear();
    if (!items || n_items <= 0) return fail(SRP_ERR_ARG, "null or empty batch");
    bool grad = (flags & SRP_PLAN_GRAD) != 0;
    std::lock_guard<std::mutex> lk(g_ws.mu);
    int rc = ws_init();
    if (rc) return rc;
    srp_result *d_out = nullptr;
    double *d_grad = nullptr;
    int64_t stride = 0;
    for (int64_t k = 0; k < n_items; ++k)
        if (items[k].scene) stride = std::max<int64_t>(stride, grad_out_size(items[k].scene));
    if (hipMalloc(&d_out, sizeof(srp_result) * n_items) != hipSuccess ||
        (grad && hipMalloc(&d_grad, sizeof(double) * std::max<int64_t>(stride, 1) * n_items) != hipSuccess)) {
        (void)hipGetLastError();
        if (d_out) (void)hipFree(d_out);
        return fail(SRP_ERR_OOM, "autotune buffers");
    }
    BatchOut bo;
    bo.d_out = d_out;
    bo.d_grad = d_grad;
    bo.grad_stride = stride;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    bool cnt = false, dir = false;
    int mg = 0;
    for (int64_t k = 0; k < n_items; ++k) {
        cnt |= (items[k].p.flags & SRP_F_COUNT) != 0;
        dir |= grad && (items[k].p.flags & SRP_F_GRAD_DIR);
        if (grad && items[k].scene) mg = std::max(mg, grad_slots(items[k].scene, items[k].p.flags));
    }
    int occ = trace_blocks_per_cu(cnt, grad, dir, mg);
    Schedule best;
    double best_t = INFINITY;
    int64_t total_patches = 0;
    for (int64_t k = 0; k < n_items; ++k) {
        const int64_t t = (items[k].p.n + TILE - 1) / TILE;
        total_patches += 4 * t * t;
    }
    // candidates: patches per chunk 1..64 (powers of two) that give every
    // resident wave at least one chunk and at most 64, at full and half
    // occupancy; the adjoint's chunks are its evaluations' gradient groups, so
    // only the occupancy is tuned for it
    std::vector<Schedule> cands;
    for (int b : {occ, std::max(1, occ / 2)}) {
        const int64_t resident = (int64_t)g_ws.n_cu * b * (BLOCK / 64);
        for (int ppc = 1; ppc <= MAX_PPC; ppc *= 2) {
            const int64_t chunks = (total_patches + ppc - 1) / ppc;
            if (!grad && ((chunks < resident && ppc > 1) || chunks > 64 * resident)) continue;
            Schedule sc;
            sc.ppc = grad ? GRAD_GROUP_MIN : ppc;
            sc.bpc = b;
            cands.push_back(sc);
            if (grad) break;
        }
        if (b == 1) break;
    }
    if (cands.empty()) cands.push_back(pick_schedule(items, n_items, grad, total_patches, occ, mg));
    for (const Schedule &sc : cands) {
        double tmin = INFINITY;
        for (int rep = 0; rep < 5 && rc == 0; ++rep) {   // one warm-up, the best of four
            if ((rc = run_batch(items, n_items, grad, bo, g_ws.stream, sc))) break;
            HIPCHK(hipStreamSynchronize(g_ws.stream));
            g_ws.pending = false;
            if (rep == 0) continue;   // warm-up
            HIPCHK(hipEventRecord(e0, g_ws.stream));
            if ((rc = run_batch(items, n_items, grad, bo, g_ws.stream, sc))) break;
            HIPCHK(hipEventRecord(e1, g_ws.stream));
            HIPCHK(hipEventSynchronize(e1));
            g_ws.pending = false;
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            tmin = std::min(tmin, (double)ms);
        }
        if (rc) break;
        if (tmin < best_t) { best_t = tmin; best = sc; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(d_out);
    if (d_grad) (void)hipFree(d_grad);
    if (rc) return rc;
    g_tuned[tune_key(items, n_items, grad)] = best;
    if (patches_per_chunk) *patches_per_chunk = best.ppc;
    if (blocks_per_cu) *blocks_per_cu = best.bpc;
    if (best_ms) *best_ms = best_t;
    return SRP_OK;
}

int srp_profile(int enable) {
    g_err.clear();
    std::lock_guard<std::mutex> lk(g_ws.mu);
    int rc = prof_collect();
    if (rc) return rc;
    g_prof.on = enable != 0;
    g_prof.ms = 0;
    g_prof.whole_ms = 0;
    g_prof.launches = 0;
    return SRP_OK;
}

int srp_profile_read(double *trace_ms, int64_t *launches) {
    g_err.clear();
    if (!trace_ms || !launches) return fail(SRP_ERR_ARG, "null output");
    std::lock_guard<std::mutex> lk(g_ws.mu);
    int rc = prof_collect();
    if (rc) return rc;
    *trace_ms = g_prof.ms;
    *launches = g_prof.launches;
    return SRP_OK;
}

int srp_profile_read_launch(double *launch_ms, int64_t *launches) {
    g_err.clear();
    if (!launch_ms || !launches) return fail(SRP_ERR_ARG, "null output");
    std::lock_guard<std::mutex> lk(g_ws.mu);
    int rc = prof_collect();
    if (rc) return rc;
    *launch_ms = g_prof.whole_ms;
    *launches = g_prof.launches;
    return SRP_OK;
}

}  // extern "C"
