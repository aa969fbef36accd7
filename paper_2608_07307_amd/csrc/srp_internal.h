// Internal data layout shared by the host runtime and the gfx950 kernels.
//
// Device memory of a scene (built once, Sec. 4.4.1: one rigid node = one
// bottom-level hierarchy in rest-pose coordinates):
//   TriRec  tris[T]   triangles in leaf order, 48 B each (3 corners + ids)
//   BNode4  blas[..]  4-wide hierarchy nodes of all tree nodes, 128 B each
//   float2  mats[M]   (rho_s, rho_d)
//   WPoint  wpts[..]  distinct (vertex, tree node) pairs, for the window pass
// Device memory of an articulation slot (one per distinct hinge-angle vector,
// Sec. 4.4.2 steps 1, 4, 5 as rigid instance transforms; built by the host for
// a scene's current angles, by k_articulate for a batch's angle vectors):
//   Inst    inst[K]   local->world transform + bottom-level root, 64 B each
//   BNode4  tlas[..]  the scene's top-level topology refitted to the instances'
//                     world boxes
//   double  xf[K][12] FP64 transforms (window pass)
//   double  axw[J][3] world-frame hinge axes (gradient)
//   int32   dof_node[J]
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace srp {

// ---- references stored in hierarchy nodes and on the traversal stack ----
// bits 31..30 type; BLAS leaf payload = (first_tri << 3) | (count - 1).
constexpr uint32_t REF_BLAS_NODE = 0u;
constexpr uint32_t REF_BLAS_LEAF = 1u;
constexpr uint32_t REF_TLAS_NODE = 2u;
constexpr uint32_t REF_TLAS_LEAF = 3u;
constexpr uint32_t REF_NONE = 0xFFFFFFFFu;
constexpr int LEAF_MAX = 8;
#ifndef SRP_STACK_DEPTH
#define SRP_STACK_DEPTH 64                  // (a host build of the traversal may lower it to check overflow reporting)
#endif
constexpr int STACK_DEPTH = SRP_STACK_DEPTH;   // per-lane traversal stack entries (the build checks each hierarchy's worst case)
#ifndef SRP_STACK_LDS
#define SRP_STACK_LDS 16                    // (a host build may shrink it to exercise the spill path)
#endif
constexpr int STACK_LDS = SRP_STACK_LDS;    // of which the newest live in LDS (a ring)
constexpr int STACK_SPILL = STACK_DEPTH - STACK_LDS;   // older ones: per-lane global spill area
static_assert((STACK_LDS & (STACK_LDS - 1)) == 0, "the LDS ring size is a power of two");
constexpr int BLAS_MAX_DEPTH = 24;          // binary internal nodes on any root-to-leaf path (build)
constexpr int TLAS_MAX_DEPTH = 7;           // <= 128 instances, median split (build)
constexpr int BLOCK = 256;                  // threads per block of the trace kernel (4 waves)
constexpr int PATCH = 8;                    // a patch is PATCH x PATCH pixels: one ray per lane of a wave
constexpr int TILE = 16;                    // patches are numbered by 16x16 tile (row-major), 4 per tile
constexpr int MAX_PPC = 64;                 // patches per chunk (one wave's work item) at most
constexpr int MAX_GRAD_SLOTS = 960;         // doubles per wave for gradient partials (LDS <= 64 KB)

#define SRP_HD __host__ __device__

SRP_HD inline uint32_t make_ref(uint32_t type, uint32_t idx) { return (type << 30) | idx; }
SRP_HD inline uint32_t ref_type(uint32_t r) { return r >> 30; }
SRP_HD inline uint32_t ref_index(uint32_t r) { return r & 0x3FFFFFFFu; }

// 4-wide hierarchy node: the boxes of up to four children as structure of
// arrays inside the node (one 16-byte load gives one bound of all four), their
// references, 128 B.  An empty slot has reference REF_NONE and a box with
// every coordinate +inf, which no ray enters.
struct alignas(128) BNode4 {
    float lox[4], loy[4], loz[4];
    float hix[4], hiy[4], hiz[4];
    uint32_t ref[4];
    uint32_t pad[4];
};
static_assert(sizeof(BNode4) == 128, "BNode4 is 128 bytes");

struct alignas(16) TriRec {
    float v0[3];
    int32_t id;     // original triangle index
    float v1[3];
    int32_t mat;
    float v2[3];
    int32_t node;
};
static_assert(sizeof(TriRec) == 48, "TriRec is 48 bytes");

struct alignas(64) Inst {
    float R[9];       // local -> world rotation, row-major
    float t[3];       // local -> world translation
    uint32_t root;    // bottom-level root reference
    int32_t node;
    float pad[2];
};
static_assert(sizeof(Inst) == 64, "Inst is 64 bytes");

struct alignas(32) WPoint {
    double x, y, z;
    int32_t node;
    int32_t pad;
};

// Per-patch partial sums (unscaled: multiply by P * A_pix).
struct alignas(64) PatchOut {
    double f[6];        // force (3), torque (3)
    uint32_t hits, sec, sec_hits, flags;
};

// A fan emitter (a chain hit that emits diffuse rays), written by the trace
// kernel at slot gen * 64 + lane of its patch's region and read by the fan
// kernel: hit point, weight w rho_d / K of each diffuse ray, oriented normal,
// original index of the hit triangle (excluded from the fan's rays).
struct alignas(16) FanRec {
    float x[3];
    float wd;
    float n[3];
    int32_t id;
};
static_assert(sizeof(FanRec) == 32, "FanRec is 32 bytes");

// Diffuse rays per fan task: the fan kernel's lane task is one emitter times
// one slice of FAN_SLICE consecutive fan-ray indices.
constexpr int FAN_SLICE = 2;   // (4 and 1 measured: 2 gives single evaluations at the paper's
                                //  setting 3 % with batches unchanged; 1 costs batches 2 %)
static_assert(SRP_MAX_BOUNCES == 4, "fan emitter masks: four generations");
// Most range sums per evaluation in the reduction's first stage (separate
// blocks, added in order by the second).
constexpr int MAX_SLICES = 16;

// A range sum of an evaluation's patch (and fan) partials: force and torque
// (FP64, before scaling), hit and test counts, status flags.
struct alignas(16) SliceOut {
    double f[6];
    uint64_t cnt[5];   // primary hits, secondary rays, secondary hits, box tests, triangle tests
    uint32_t flags;
    uint32_t pad_;
};
static_assert(sizeof(SliceOut) == 96, "SliceOut is 96 bytes");

// One kinematic-tree node as the articulation kernel reads it (built once per
// scene): the edge label (pivot, axes as given and renormalised for the
// rotation), the padded rest-pose box of the node's triangles and its
// bottom-level root.
struct alignas(16) ArtNode {
    double pivot[3];
    double axis[3][3];
    double unit[3][3];
    double blo[3], bhi[3];
    int32_t parent, n_axes, dof_offset;
    uint32_t blas_root;
    int32_t depth;      // edges from the root
    int32_t pad_;
};
static_assert(sizeof(ArtNode) == 240, "ArtNode layout");

// One articulation slot to build on the device: the scene's nodes and top-level
// topology (each node's height, the most inner-node levels below it, in
// pad[0]), the cosine and sine of each clamped hinge angle (2 per degree of
// freedom), and where the slot's arrays go.
struct alignas(16) ArtJob {
    const ArtNode *nodes;
    const BNode4 *topo;
    const double *cs;
    Inst *inst;
    BNode4 *tlas;
    double *xf;
    double *axw;
    int32_t *dof_node;
    double pad;
    int32_t n_nodes, n_tlas;
    int32_t max_depth, max_height;
    int32_t pad_[2];
};
static_assert(sizeof(ArtJob) == 96, "ArtJob layout");

// One evaluation, as the kernels see it.
struct alignas(64) EvalDesc {
    // scene
    const TriRec *tris;
    const BNode4 *blas;
    const float *mats;       // 2 floats per material
    const WPoint *wpts;
    int64_t n_wpts;
    // articulation slot
    const Inst *inst;
    const BNode4 *tlas;
    const double *xf;        // K x 12
    const double *axw;       // J x 3
    const int32_t *dof_node; // J
    const int32_t *parent;   // K (device copy of the tree)
    uint32_t root_ref;
    int32_t n_nodes, n_mats, n_dof;
    // parameters (basis in FP64 from the host)
    double u[3], v[3], d[3];
    double pressure;
    double ref[3];
    int32_t n, bounces;
    uint32_t flags;
    int32_t tiles_x;        // 16-pixel tile columns
    int32_t ppc;            // patches per chunk
    int32_t grad_n;         // doubles per chunk gradient partial (0 = no gradient)
    int64_t chunk_base;     // first chunk of this evaluation
    int64_t n_chunks;
    int64_t patch_base;     // first patch of this evaluation (partial sums are per patch)
    int64_t n_patches;      // 4 * tiles_x * tiles_y
    int32_t tiles_y;        // 16-pixel tile rows
    int32_t n_diffuse;      // diffuse rays per emitting hit (0 = none)
    // optional outputs
    int32_t *hit_ids;       // N*N*R (R = B+1 + B*n_diffuse) or null
    float *hit_t;
    double *grad_part;      // n_chunks x grad_n (gradient partials)
    double *grad_out;       // 3*(2M+J) final gradient or null
    const float *dset;      // n_diffuse > 0: the diffuse set, 4 floats per ray (x, y, z, 0), then its mean
    FanRec *emit;           // n_diffuse > 0, forward: emitter records, n_patches x bounces x 64, then as
                            // many bytes: the planar instance each record's rays leave, or -1
    uint64_t *emit_mask;    // which of them are filled: n_patches x bounces masks of 64 lanes
    int32_t n_slices;       // reduction: contiguous ranges summed by separate blocks (1..MAX_SLICES)
    int64_t fan_base;       // first fan partial slot (n_patches x bounces x ceil(n_diffuse / FAN_SLICE))
    double *gslice;         // gradient: n_slices x grad_n range sums
    SliceOut *pslice;       // n_slices range sums of the patch (and fan) partials
    int64_t slice_base;     // the batch's number of this evaluation's first range sum
    int32_t n_clamped;      // hinge angles of this evaluation clamped to their intervals
    int32_t pad_;
    uint64_t planar[2];     // bit k: every triangle of node k lies in one plane (rays leaving it skip it)
};

// The host writes these records and the kernels read them: both compilation
// passes (host and gfx950) must agree on every offset.
static_assert(sizeof(EvalDesc) == 448, "EvalDesc layout");
static_assert(offsetof(EvalDesc, tris) == 0, "EvalDesc layout");
static_assert(offsetof(EvalDesc, blas) == 8, "EvalDesc layout");
static_assert(offsetof(EvalDesc, mats) == 16, "EvalDesc layout");
static_assert(offsetof(EvalDesc, wpts) == 24, "EvalDesc layout");
static_assert(offsetof(EvalDesc, n_wpts) == 32, "EvalDesc layout");
static_assert(offsetof(EvalDesc, inst) == 40, "EvalDesc layout");
static_assert(offsetof(EvalDesc, tlas) == 48, "EvalDesc layout");
static_assert(offsetof(EvalDesc, xf) == 56, "EvalDesc layout");
static_assert(offsetof(EvalDesc, axw) == 64, "EvalDesc layout");
static_assert(offsetof(EvalDesc, dof_node) == 72, "EvalDesc layout");
static_assert(offsetof(EvalDesc, parent) == 80, "EvalDesc layout");
static_assert(offsetof(EvalDesc, root_ref) == 88, "EvalDesc layout");
static_assert(offsetof(EvalDesc, n_nodes) == 92, "EvalDesc layout");
static_assert(offsetof(EvalDesc, n_mats) == 96, "EvalDesc layout");
static_assert(offsetof(EvalDesc, n_dof) == 100, "EvalDesc layout");
static_assert(offsetof(EvalDesc, u) == 104, "EvalDesc layout");
static_assert(offsetof(EvalDesc, v) == 128, "EvalDesc layout");
static_assert(offsetof(EvalDesc, d) == 152, "EvalDesc layout");
static_assert(offsetof(EvalDesc, pressure) == 176, "EvalDesc layout");
static_assert(offsetof(EvalDesc, ref) == 184, "EvalDesc layout");
static_assert(offsetof(EvalDesc, n) == 208, "EvalDesc layout");
static_assert(offsetof(EvalDesc, bounces) == 212, "EvalDesc layout");
static_assert(offsetof(EvalDesc, flags) == 216, "EvalDesc layout");
static_assert(offsetof(EvalDesc, tiles_x) == 220, "EvalDesc layout");
static_assert(offsetof(EvalDesc, ppc) == 224, "EvalDesc layout");
static_assert(offsetof(EvalDesc, grad_n) == 228, "EvalDesc layout");
static_assert(offsetof(EvalDesc, chunk_base) == 232, "EvalDesc layout");
static_assert(offsetof(EvalDesc, n_chunks) == 240, "EvalDesc layout");
static_assert(offsetof(EvalDesc, patch_base) == 248, "EvalDesc layout");
static_assert(offsetof(EvalDesc, n_patches) == 256, "EvalDesc layout");
static_assert(offsetof(EvalDesc, tiles_y) == 264, "EvalDesc layout");
static_assert(offsetof(EvalDesc, n_diffuse) == 268, "EvalDesc layout");
static_assert(offsetof(EvalDesc, hit_ids) == 272, "EvalDesc layout");
static_assert(offsetof(EvalDesc, hit_t) == 280, "EvalDesc layout");
static_assert(offsetof(EvalDesc, grad_part) == 288, "EvalDesc layout");
static_assert(offsetof(EvalDesc, grad_out) == 296, "EvalDesc layout");
static_assert(offsetof(EvalDesc, dset) == 304, "EvalDesc layout");
static_assert(offsetof(EvalDesc, emit) == 312, "EvalDesc layout");
static_assert(offsetof(EvalDesc, emit_mask) == 320, "EvalDesc layout");
static_assert(offsetof(EvalDesc, n_slices) == 328, "EvalDesc layout");
static_assert(offsetof(EvalDesc, fan_base) == 336, "EvalDesc layout");
static_assert(offsetof(EvalDesc, gslice) == 344, "EvalDesc layout");
static_assert(offsetof(EvalDesc, pslice) == 352, "EvalDesc layout");
static_assert(offsetof(EvalDesc, slice_base) == 360, "EvalDesc layout");
static_assert(offsetof(EvalDesc, n_clamped) == 368, "EvalDesc layout");
static_assert(offsetof(EvalDesc, planar) == 376, "EvalDesc layout");
static_assert(sizeof(PatchOut) == 64, "PatchOut layout");
static_assert(offsetof(PatchOut, f) == 0, "PatchOut layout");
static_assert(offsetof(PatchOut, hits) == 48, "PatchOut layout");
static_assert(offsetof(PatchOut, flags) == 60, "PatchOut layout");
static_assert(sizeof(WPoint) == 32, "WPoint layout");
static_assert(offsetof(WPoint, node) == 24, "WPoint layout");
static_assert(offsetof(Inst, t) == 36, "Inst layout");
static_assert(offsetof(Inst, root) == 48, "Inst layout");
static_assert(offsetof(BNode4, ref) == 96, "BNode4 layout");
static_assert(offsetof(TriRec, id) == 12, "TriRec layout");
static_assert(offsetof(TriRec, mat) == 28, "TriRec layout");
static_assert(offsetof(TriRec, node) == 44, "TriRec layout");

// Order-preserving map of doubles to unsigned 64-bit integers (for
// atomic min/max of the window bounds).
SRP_HD inline uint64_t enc_f64(double x) {
    union { double d; uint64_t u; } c;
    c.d = x;
    return (c.u >> 63) ? ~c.u : (c.u | 0x8000000000000000ull);
}
SRP_HD inline double dec_f64(uint64_t e) {
    union { double d; uint64_t u; } c;
    c.u = (e >> 63) ? (e & 0x7FFFFFFFFFFFFFFFull) : ~e;
    return c.d;
}

// window slots per evaluation: enc(umin), enc(-umax), enc(vmin), enc(-vmax), enc(hmin)
constexpr int WIN_STRIDE = 8;

// Kernel launchers (kernels.hip)
// Work queues of the trace kernel (and, after them, of the fan kernel): N_QUEUES
// counters QUEUE_STRIDE words apart; after both sets, the count of fan units
// the trace kernel listed (FAN_UNITS_AT)
// (launch_window zeroes them).
constexpr int N_QUEUES = 8;
constexpr int QUEUE_STRIDE = 64;
constexpr int FAN_UNITS_AT = 2 * N_QUEUES * QUEUE_STRIDE;
constexpr int QUEUE_WORDS = FAN_UNITS_AT + QUEUE_STRIDE;
int launch_window(const EvalDesc *d_desc, int n_evals, int blocks_x, uint64_t *d_win, uint32_t *d_queue,
                  void *stream);
// Builds n_jobs articulation slots, one thread each (articulate.hip); the
// window kernel reads them, so it runs first on the same stream.
int launch_articulate(const ArtJob *d_jobs, int n_jobs, void *stream);
// d_spill: grid_blocks * BLOCK * STACK_SPILL words; chunk counts below 2^31.
// d_fan_out, d_fan_counts (forward, diffuse rays on): the fan pass partial
// slots.  With fans_inline the trace kernel also traces every patch's diffuse
// fans into them (no fan launch follows); otherwise it lists each patch's
// non-empty passes in d_fan_units (capacity: one entry per pass slot; their
// number at d_queue[FAN_UNITS_AT]) for the fan launch and writes the empty
// passes' zero partials itself.  blocks_per_cu <= 2 (grid_blocks = that times the CU count) launches the
// kernel compiled for 2 waves per SIMD.  d_order, d_cost (such forward
// launches of one patch per chunk, else null; other launches ignore them):
// one word per patch of the batch (at each evaluation's patch_base); chunk c
// of an evaluation traces its patch d_order[c], and d_cost receives every
// patch's trace time (constant-rate clock ticks).
int launch_trace(const EvalDesc *d_desc, const int64_t *d_chunk_base, int n_evals,
                 const uint64_t *d_win, int64_t total_chunks, uint32_t *d_queue, uint32_t *d_spill,
                 PatchOut *d_patches, uint64_t *d_counts, bool count, bool grad, bool dir, int grid_blocks,
                 int lds_grad_doubles, PatchOut *d_fan_out, uint64_t *d_fan_counts, bool fans_inline,
                 int4 *d_fan_units, int blocks_per_cu, const uint32_t *d_order, uint32_t *d_cost, void *stream);
// Diffuse fans of the recorded emitters: one work unit per non-empty fan pass,
// as the trace kernel listed them in d_fan_units (at most max_units); uses the
// second set of queue counters and the same spill area as the trace kernel.
int launch_fans(const EvalDesc *d_desc, const uint64_t *d_win, int64_t max_units, uint32_t *d_queue,
                uint32_t *d_spill, PatchOut *d_fan_out, uint64_t *d_fan_counts, const int4 *d_fan_units, bool count,
                int grid_blocks, void *stream);
// d_slice_eval: the evaluation of each of the batch's total_slices range sums
// (one block each; an evaluation's are consecutive, from its slice_base).
// With d_order and d_cost (as for launch_trace) the second stage also
// rewrites every evaluation's patch order from the costs, heaviest first, for
// the next launches, on every eighth launch as counted in *d_order_launch.
int launch_reduce(const EvalDesc *d_desc, int n_evals, const uint64_t *d_win, const PatchOut *d_patches,
                  const uint64_t *d_counts, const PatchOut *d_fan_out, const uint64_t *d_fan_counts, bool count,
                  bool grad, const uint32_t *d_slice_eval, int64_t total_slices, void *d_out, uint32_t *d_order,
                  const uint32_t *d_cost, uint32_t *d_order_launch, void *stream);
// Resident blocks per compute unit of the trace kernel variant.
int trace_blocks_per_cu(bool count, bool grad, bool dir, int lds_grad_doubles);
// Resident blocks per compute unit of the fan kernel variant.
int fan_blocks_per_cu(bool count);

// Fixed device workspace of the entry point that allocates nothing: a
// file-scope static device array in kernels.hip, NOALLOC_SCRATCH_BYTES per
// GPU, held until the process ends.  noalloc_scratch_init looks up its address
// on the current device (once per device; the library's init calls it);
// noalloc_scratch returns that address (nullptr before the lookup).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
int noalloc_scratch_init();
char *noalloc_scratch(int device);

}  // namespace srp
