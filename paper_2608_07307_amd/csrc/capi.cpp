// C ABI entry points: argument checks, articulation slots, the per-call
// upload and the window -> trace -> reduce launch sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "host.h"

using namespace srp;

struct srp_scene {
    int device = 0;
    SceneHost h;
    TriRec *d_tris = nullptr;
    BNode *d_blas = nullptr;
    float *d_mats = nullptr;
    WPoint *d_wpts = nullptr;
    int32_t *d_parent = nullptr;
    char *d_slot = nullptr;        // current articulation slot
    SlotLayout slot_L{};
    SlotHost cur;
    std::vector<double> angles;    // current (clamped) angles
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
// buffer, the library stream and the completion event of the last batch.
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
    hipEvent_t done = nullptr;
    bool pending = false;
};
Workspace g_ws;

// Optional timing of the trace-kernel launches (HIP events on the launch stream).
struct Profile {
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pairs;   // recorded, not yet read
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
    double ms = 0;
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
    return SRP_OK;
}

int ws_init() {
    if (g_ws.init) return SRP_OK;
    HIPCHK(hipGetDevice(&g_ws.device));
    HIPCHK(hipDeviceGetAttribute(&g_ws.n_cu, hipDeviceAttributeMultiprocessorCount, g_ws.device));
    HIPCHK(hipStreamCreateWithFlags(&g_ws.stream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&g_ws.done, hipEventDisableTiming));
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
    if (p->flags & ~(uint32_t)SRP_F_COUNT) return fail(SRP_ERR_ARG, "unknown flags");
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

int choose_rpt(int n) { return n >= 1024 ? 4 : (n >= 512 ? 2 : 1); }

struct BatchOut {
    srp_result *d_out = nullptr;     // device results (n items)
    double *d_grad = nullptr;        // device gradients or null
    int64_t grad_stride = 0;
    int32_t *d_hit_ids = nullptr;    // single item only
    float *d_hit_t = nullptr;
};

// Queues one batch on `stream`.  Caller holds g_ws.mu.
int run_batch(const srp_batch_item *items, int64_t n, bool grad, const BatchOut &bo, hipStream_t stream) {
    if (n <= 0) return SRP_OK;
    if (n > (1 << 30)) return fail(SRP_ERR_ARG, "too many items");
    bool count = false;
    int64_t total_chunks = 0;
    int max_grad_n = 0;
    std::vector<int64_t> base(n + 1);
    std::vector<int> rpt(n), tiles_x(n);
    int64_t max_wpts = 0;
    for (int64_t k = 0; k < n; ++k) {
        const srp_batch_item &it = items[k];
        if (!it.scene) return fail(SRP_ERR_ARG, "item " + std::to_string(k) + ": null scene");
        int rc = check_params(&it.p);
        if (rc) return fail(rc, "item " + std::to_string(k) + ": " + g_err);
        if (it.scene->device != g_ws.device) return fail(SRP_ERR_ARG, "scene built on another device");
        if (it.angles)
            for (int j = 0; j < it.scene->h.n_dof; ++j)
                if (!std::isfinite(it.angles[j])) return fail(SRP_ERR_ARG, "item " + std::to_string(k) + ": non-finite angle");
        count |= (it.p.flags & SRP_F_COUNT) != 0;
        const int N = it.p.n;
        rpt[k] = choose_rpt(N);
        tiles_x[k] = (N + TILE - 1) / TILE;
        int tiles_y = (N + TILE * rpt[k] - 1) / (TILE * rpt[k]);
        base[k] = total_chunks;
        total_chunks += (int64_t)tiles_x[k] * tiles_y;
        if (grad) {
            int gn = 9 * it.scene->h.n_nodes + 6 * it.scene->h.n_mats;
            if (gn > MAX_GRAD_SLOTS) return fail(SRP_ERR_ARG, "gradient needs 9*nodes + 6*materials <= 960");
            if (bo.d_grad && bo.grad_stride < 3 * (2 * it.scene->h.n_mats + it.scene->h.n_dof))
                return fail(SRP_ERR_ARG, "grad_stride too small");
            max_grad_n = std::max(max_grad_n, gn);
        }
        max_wpts = std::max<int64_t>(max_wpts, (int64_t)it.scene->h.wpts.size());
    }
    base[n] = total_chunks;

    // articulation slots: the scene's current slot, or one per distinct angle vector
    struct SlotRec {
        const srp_scene *sc;
        std::vector<double> ang;
        SlotHost s;
        SlotLayout L;
        size_t off;
    };
    std::vector<SlotRec> slots;
    std::map<std::pair<const srp_scene *, std::vector<double>>, int> slot_of;
    std::vector<int> item_slot(n, -1);
    for (int64_t k = 0; k < n; ++k) {
        const srp_batch_item &it = items[k];
        if (!it.angles) continue;
        std::vector<double> a(it.angles, it.angles + it.scene->h.n_dof);
        auto key = std::make_pair((const srp_scene *)it.scene, a);
        auto f = slot_of.find(key);
        if (f != slot_of.end()) { item_slot[k] = f->second; continue; }
        SlotRec r;
        r.sc = it.scene;
        r.ang = a;
        int rc = slot_build(it.scene->h, a.data(), &r.s, &g_err);
        if (rc) return rc;
        r.L = slot_layout(it.scene->h.n_nodes, std::max<int>(it.scene->h.n_nodes, 1), it.scene->h.n_dof);
        slots.push_back(std::move(r));
        item_slot[k] = (int)slots.size() - 1;
        slot_of.emplace(key, item_slot[k]);
    }

    // staging layout (uploaded): descs | chunk_base | win | (spare) | slots
    size_t o_desc = 0;
    size_t o_base = align_up(o_desc + sizeof(EvalDesc) * n);
    size_t o_win = align_up(o_base + sizeof(int64_t) * (n + 1));
    size_t o_cnt = align_up(o_win + sizeof(uint64_t) * WIN_STRIDE * n);
    size_t o_slots = align_up(o_cnt + 256);
    size_t off = o_slots;
    for (auto &s : slots) { s.off = off; off = align_up(off + s.L.bytes); }
    size_t stage_bytes = off;
    // device-only regions: chunk partials | counts | gradient partials
    size_t o_chunks = align_up(stage_bytes);
    size_t o_counts = align_up(o_chunks + sizeof(ChunkOut) * total_chunks);
    size_t o_gpart = align_up(o_counts + (count ? sizeof(uint64_t) * 2 * total_chunks : 0));
    std::vector<size_t> gpart_off(n, 0);
    size_t goff = o_gpart;
    if (grad)
        for (int64_t k = 0; k < n; ++k) {
            gpart_off[k] = goff;
            int gn = 9 * items[k].scene->h.n_nodes + 6 * items[k].scene->h.n_mats;
            goff = align_up(goff + sizeof(double) * gn * (base[k + 1] - base[k]));
        }
    size_t dev_bytes = align_up(goff);

    int rc = ws_wait();   // staging buffer reuse
    if (rc) return rc;
    rc = ws_reserve(dev_bytes, stage_bytes);
    if (rc) return rc;
    char *H = g_ws.h_stage, *Dv = g_ws.d_buf;
    EvalDesc *desc = reinterpret_cast<EvalDesc *>(H + o_desc);
    std::memcpy(H + o_base, base.data(), sizeof(int64_t) * (n + 1));
    uint64_t *win = reinterpret_cast<uint64_t *>(H + o_win);
    for (int64_t k = 0; k < WIN_STRIDE * n; ++k) win[k] = enc_f64(INFINITY);
    std::memset(H + o_cnt, 0, 256);
    for (auto &s : slots) slot_pack(s.s, s.L, H + s.off);

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
        const char *slot_base;
        SlotLayout L;
        uint32_t root;
        if (item_slot[k] >= 0) {
            const SlotRec &s = slots[item_slot[k]];
            slot_base = Dv + s.off;
            L = s.L;
            root = s.s.root_ref;
        } else {
            slot_base = sc->d_slot;
            L = sc->slot_L;
            root = sc->cur.root_ref;
        }
        D.inst = reinterpret_cast<const Inst *>(slot_base + L.inst);
        D.tlas = reinterpret_cast<const BNode *>(slot_base + L.tlas);
        D.xf = reinterpret_cast<const double *>(slot_base + L.xf);
        D.axw = reinterpret_cast<const double *>(slot_base + L.axw);
        D.dof_node = reinterpret_cast<const int32_t *>(slot_base + L.dof_node);
        D.parent = sc->d_parent;
        D.root_ref = root;
        D.n_nodes = sc->h.n_nodes;
        D.n_mats = sc->h.n_mats;
        D.n_dof = sc->h.n_dof;
        basis(it.p.sun_dir, D.u, D.v, D.d);
        D.pressure = it.p.pressure;
        for (int c = 0; c < 3; ++c) D.ref[c] = it.p.ref[c];
        D.n = it.p.n;
        D.bounces = it.p.bounces;
        D.flags = it.p.flags;
        D.tiles_x = tiles_x[k];
        D.rpt = rpt[k];
        D.chunk_base = base[k];
        D.n_chunks = base[k + 1] - base[k];
        D.grad_n = grad ? 9 * sc->h.n_nodes + 6 * sc->h.n_mats : 0;
        D.grad_part = grad ? reinterpret_cast<double *>(Dv + gpart_off[k]) : nullptr;
        D.grad_out = (grad && bo.d_grad) ? bo.d_grad + k * bo.grad_stride : nullptr;
        D.hit_ids = (n == 1) ? bo.d_hit_ids : nullptr;
        D.hit_t = (n == 1) ? bo.d_hit_t : nullptr;
    }

    // the previous batch has completed (ws_wait above), so the staging
    // buffer and the workspace are free on every stream
    HIPCHK(hipMemcpyAsync(Dv, H, stage_bytes, hipMemcpyHostToDevice, stream));
    const EvalDesc *d_desc = reinterpret_cast<const EvalDesc *>(Dv + o_desc);
    const int64_t *d_base = reinterpret_cast<const int64_t *>(Dv + o_base);
    uint64_t *d_win = reinterpret_cast<uint64_t *>(Dv + o_win);
    ChunkOut *d_chunks = reinterpret_cast<ChunkOut *>(Dv + o_chunks);
    uint64_t *d_counts = count ? reinterpret_cast<uint64_t *>(Dv + o_counts) : nullptr;

    int wb = (int)std::min<int64_t>(64, std::max<int64_t>(1, (max_wpts + 2047) / 2048));
    int e = launch_window(d_desc, (int)n, wb, d_win, stream);
    if (e) return fail(SRP_ERR_DEVICE, std::string("window kernel: ") + hipGetErrorString((hipError_t)e));
    int bpc = trace_blocks_per_cu(count, grad, max_grad_n);
    int64_t grid = std::min<int64_t>(total_chunks, (int64_t)g_ws.n_cu * bpc);
    std::pair<hipEvent_t, hipEvent_t> ev{};
    if (g_prof.on) {
        if ((rc = prof_event_pair(&ev))) return rc;
        HIPCHK(hipEventRecord(ev.first, stream));
    }
    e = launch_trace(d_desc, d_base, (int)n, d_win, total_chunks, d_chunks, d_counts, count, grad,
                     (int)std::max<int64_t>(grid, 1), max_grad_n, stream);
    if (e) return fail(SRP_ERR_DEVICE, std::string("trace kernel: ") + hipGetErrorString((hipError_t)e));
    if (g_prof.on) {
        HIPCHK(hipEventRecord(ev.second, stream));
        g_prof.pairs.push_back(ev);
    }
    e = launch_reduce(d_desc, d_base, (int)n, d_win, d_chunks, d_counts, count, grad, bo.d_out, stream);
    if (e) return fail(SRP_ERR_DEVICE, std::string("reduce kernel: ") + hipGetErrorString((hipError_t)e));
    HIPCHK(hipEventRecord(g_ws.done, stream));
    g_ws.pending = true;
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
    (void)hipFree(sc->d_tris);
    (void)hipFree(sc->d_blas);
    (void)hipFree(sc->d_mats);
    (void)hipFree(sc->d_wpts);
    (void)hipFree(sc->d_parent);
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
    } catch (const std::bad_alloc &) {
        rc = fail(SRP_ERR_OOM, "host allocation failed");
    }
    if (rc) { free_scene(sc); return rc; }
    std::lock_guard<std::mutex> lk(g_ws.mu);
    if ((rc = ws_init())) { free_scene(sc); return rc; }
    sc->device = g_ws.device;
    sc->angles.assign(sc->h.n_dof, 0.0);
    sc->slot_L = slot_layout(sc->h.n_nodes, std::max(sc->h.n_nodes, 1), sc->h.n_dof);
    if ((rc = dev_upload(&sc->d_tris, sc->h.tris)) || (rc = dev_upload(&sc->d_blas, sc->h.blas)) ||
        (rc = dev_upload(&sc->d_mats, sc->h.mats)) || (rc = dev_upload(&sc->d_wpts, sc->h.wpts)) ||
        (rc = dev_upload(&sc->d_parent, sc->h.parent))) {
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
    std::vector<BNode>().swap(sc->h.blas);
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

int srp_eval(srp_scene *scene, const srp_eval_params *params, srp_result *out, int32_t *hit_ids, float *hit_t) {
    g_err.clear();
    if (!scene || !params || !out) return fail(SRP_ERR_ARG, "null scene, params or out");
    int rc = check_params(params);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_ws.mu);
    if ((rc = ws_init())) return rc;
    srp_batch_item it{scene, nullptr, *params};
    size_t nrec = (hit_ids || hit_t) ? (size_t)params->n * params->n * (params->bounces + 1) : 0;
    // results and records live in a second device buffer so the workspace can be reused
    static srp_result *d_res = nullptr;
    static char *d_rec = nullptr;
    static size_t rec_cap = 0;
    if (!d_res) HIPCHK(hipMalloc(&d_res, sizeof(srp_result)));
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
    bo.d_out = d_res;
    if (nrec) {
        bo.d_hit_ids = reinterpret_cast<int32_t *>(d_rec);
        bo.d_hit_t = reinterpret_cast<float *>(d_rec + nrec * 4);
    }
    if ((rc = run_batch(&it, 1, false, bo, g_ws.stream))) return rc;
    if (!g_ws.h_res) HIPCHK(hipHostMalloc(&g_ws.h_res, sizeof(srp_result), hipHostMallocDefault));
    HIPCHK(hipMemcpyAsync(g_ws.h_res, d_res, sizeof(srp_result), hipMemcpyDeviceToHost, g_ws.stream));
    HIPCHK(hipStreamSynchronize(g_ws.stream));
    g_ws.pending = false;
    *out = *g_ws.h_res;
    if (nrec) {
        if (hit_ids) HIPCHK(hipMemcpy(hit_ids, d_rec, nrec * 4, hipMemcpyDeviceToHost));
        if (hit_t) HIPCHK(hipMemcpy(hit_t, d_rec + nrec * 4, nrec * 4, hipMemcpyDeviceToHost));
    }
    if (out->status & SRP_STATUS_STACK) return fail(SRP_ERR_DEPTH, "traversal stack overflow");
    return SRP_OK;
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
                  double *dF_drho_d, double *dF_dtheta) {
    g_err.clear();
    if (!scene || !params || !out) return fail(SRP_ERR_ARG, "null scene, params or out");
    int rc = check_params(params);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_ws.mu);
    if ((rc = ws_init())) return rc;
    const int M = scene->h.n_mats, J = scene->h.n_dof;
    const size_t gsz = 3 * (size_t)(2 * M + J);
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
    if (out->status & SRP_STATUS_STACK) return fail(SRP_ERR_DEPTH, "traversal stack overflow");
    return SRP_OK;
}

int srp_profile(int enable) {
    g_err.clear();
    std::lock_guard<std::mutex> lk(g_ws.mu);
    int rc = prof_collect();
    if (rc) return rc;
    g_prof.on = enable != 0;
    g_prof.ms = 0;
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

}  // extern "C"
