// Host-side scene and articulation structures of the SRP library.
#pragma once
#include <string>
#include <vector>

#include "srp.h"
#include "srp_internal.h"

namespace srp {

// One kinematic-tree node (Sec. 4.4.1) plus its bottom-level hierarchy.
struct NodeInfo {
    int32_t parent = -1;
    int32_t is_panel = 0;
    double pivot[3] = {0, 0, 0};
    int32_t n_axes = 0;
    double axis[3][3] = {{0}};       // unit axes (world hinge axes are R_parent times these)
    double unit[3][3] = {{0}};       // the same axes renormalised, as the rotation matrices use them
    double lo[3] = {0}, hi[3] = {0};
    int32_t dof_offset = 0;
    uint32_t blas_root = REF_NONE;   // REF_NONE when the node has no triangles
    int32_t blas_depth = 0;          // 4-wide levels
    int32_t blas_worst = 0;          // most traversal-stack entries a ray can hold in this hierarchy
    double blo[3] = {0}, bhi[3] = {0};  // padded rest-pose bounds of the node's triangles
    double n0[3] = {0, 0, 0};           // area-weighted rest-pose normal (unit, or 0 if none)
    int32_t planar = 0;                 // every triangle within 1e-9 x the mesh scale of one plane
};

// One plate of the N-plate model in its node's frame: the node's triangles of
// one material whose unit normals agree to 1e-6 (rounded components), merged;
// n is the area-weighted sum of their unit normals, c their area-weighted
// centroid.  Articulation moves a plate rigidly with its node.
struct PlateLocal {
    double n[3] = {0, 0, 0}, c[3] = {0, 0, 0}, area = 0;
    int32_t node = 0, mat = 0;
};

// Host image of one articulation slot (see srp_internal.h for the layout).
struct SlotHost {
    std::vector<Inst> inst;
    std::vector<BNode4> tlas;
    uint32_t root_ref = REF_NONE;
    int tlas_depth = 0;
    int stack_worst = 0;           // most traversal-stack entries a ray can hold
    std::vector<double> xf;        // K x 12: R (row-major) then t
    std::vector<double> axw;       // J x 3
    std::vector<int32_t> dof_node; // J
    int n_clamped = 0;
};

struct SlotLayout {
    size_t inst, tlas, xf, axw, dof_node, bytes;
};
SlotLayout slot_layout(int n_nodes, int n_tlas, int n_dof);
void slot_pack(const SlotHost &s, const SlotLayout &L, char *dst);

struct SceneHost {
    int32_t n_nodes = 0, n_mats = 0, n_dof = 0;
    int64_t n_tris = 0;
    std::vector<NodeInfo> nodes;
    std::vector<float> mats;        // 2 per material
    std::vector<TriRec> tris;       // leaf order
    std::vector<BNode4> blas;
    std::vector<WPoint> wpts;
    std::vector<int32_t> parent;
    std::vector<PlateLocal> plates; // N-plate model, in the order of each plate's first triangle
    double pad = 0;                 // box padding (metres)
    int max_blas_depth = 0;
    // top level: 4-wide nodes over the non-empty nodes' instances, built once over
    // the rest pose; a slot copies the references and refits the boxes (children
    // follow their parent in this array)
    std::vector<BNode4> tlas_topo;  // pad[0] of each node: its height (inner-node levels below it)
    uint32_t tlas_root = REF_NONE;
    int tlas_depth = 0;
    int tlas_max_height = 0;
    int tree_max_depth = 0;         // kinematic tree: most edges from the root
    int stack_worst = 0;            // most traversal-stack entries a ray can hold (any pose)
};

// Validates the inputs and builds the host image.  Returns SRP_OK or an
// error code with a message in *err.
int scene_build(const double *verts, int64_t n_verts, const int32_t *tris, int64_t n_tris,
                const int32_t *tri_material, const int32_t *tri_node, const srp_material *mats,
                int32_t n_mats, const srp_node *nodes, int32_t n_nodes, SceneHost *out,
                std::string *err);

int validate_materials(const srp_material *mats, int32_t n_mats, std::string *err);

// Composes the node transforms for `angles` (NULL = all zero), clamping each
// angle to its interval (Sec. 4.4.2 step 4), and builds the instances, the
// world hinge axes and the top level refitted to the instances' world boxes.
int slot_build(const SceneHost &S, const double *angles, SlotHost *out, std::string *err);

// Angle `th` of axis a of node nd clamped to its interval; *clamped counts a clamp.
double clamp_angle(const NodeInfo &nd, int a, double th, int *clamped);

// The articulation kernel's view of the scene's nodes (same order).
std::vector<ArtNode> art_nodes(const SceneHost &S);

// srp_eval with hinge angles for this evaluation only (NULL: the scene's
// current angles), the slot built on the device inside the captured launch;
// the scene's current angles are unchanged (capi.cpp).
int eval_single(srp_scene *scene, const srp_eval_params *params, const double *angles, srp_result *out,
                int32_t *hit_ids, float *hit_t);

// Fills S->plates from S->tris (which the library frees once they are on the
// device).
void plates_build(SceneHost *S);

// S's plates moved by the node transforms of `slot` into out[0 .. S.plates.size()).
void plates_world(const SceneHost &S, const SlotHost &slot, srp_plate *out);

}  // namespace srp
