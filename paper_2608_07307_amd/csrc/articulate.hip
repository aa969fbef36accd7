// Articulation slots on the GPU (Sec. 4.4.2 steps 1, 4 and 5 as rigid
// instance transforms; Sec. 4.4.1 for the tree): one wave per slot, one lane
// per tree node.  The nodes are composed level by level down the tree (a node
// reads its parent's FP64 transform from LDS), then every instance's world box
// is computed in parallel and the scene's fixed top-level topology is refitted
// level by level from the bottom.  The host computes the cosine and sine of
// every clamped angle (the same library calls as its own slot build); every
// node's and box's arithmetic after that is the host build's sequence of
// separately rounded FP64 operations (contraction is off in this file and in
// the host's), so a slot built here holds the same bits as one built on the
// host for the same angles.
#include <hip/hip_runtime.h>

#include "srp.h"
#include "srp_internal.h"

#pragma clang fp contract(off)

namespace srp {
namespace {

constexpr int ART_BLOCK = 64;

// std::min and std::max as the host build calls them (the first argument on ties)
template <typename T>
__device__ inline T lmin(T a, T b) { return (b < a) ? b : a; }
template <typename T>
__device__ inline T lmax(T a, T b) { return (a < b) ? b : a; }

__device__ inline void mat3_mul(const double *A, const double *B, double *C) {
    double T[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) T[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
    for (int i = 0; i < 9; ++i) C[i] = T[i];
}

__device__ inline void mat3_vec(const double *A, const double *x, double *y) {
    double t[3];
    for (int i = 0; i < 3; ++i) t[i] = A[3 * i] * x[0] + A[3 * i + 1] * x[1] + A[3 * i + 2] * x[2];
    for (int i = 0; i < 3; ++i) y[i] = t[i];
}

// Rotation by the angle of cosine c and sine s about the unit axis u (Rodrigues).
__device__ inline void rot_unit(const double *u, double c, double s, double *R) {
    const double x = u[0], y = u[1], z = u[2], C = 1 - c;
    R[0] = c + x * x * C;
    R[1] = x * y * C - z * s;
    R[2] = x * z * C + y * s;
    R[3] = y * x * C + z * s;
    R[4] = c + y * y * C;
    R[5] = y * z * C - x * s;
    R[6] = z * x * C - y * s;
    R[7] = z * y * C + x * s;
    R[8] = c + z * z * C;
}

// The instance's top-level box: its padded rest-pose box's eight corners under
// X, their extremes grown by the padding and rounded outward to FP32.
__device__ inline void inst_box(const ArtNode &nd, const double *X, double pad, float lo[3], float hi[3]) {
    double l[3] = {INFINITY, INFINITY, INFINITY}, h[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int c = 0; c < 8; ++c) {
        const double p[3] = {(c & 1) ? nd.bhi[0] : nd.blo[0], (c & 2) ? nd.bhi[1] : nd.blo[1],
                             (c & 4) ? nd.bhi[2] : nd.blo[2]};
        double w[3];
        mat3_vec(X, p, w);
        for (int a = 0; a < 3; ++a) {
            w[a] += X[9 + a];
            l[a] = lmin(l[a], w[a]);
            h[a] = lmax(h[a], w[a]);
        }
    }
    for (int a = 0; a < 3; ++a) {
        lo[a] = nextafterf((float)(l[a] - pad), -INFINITY);
        hi[a] = nextafterf((float)(h[a] + pad), INFINITY);
    }
}

// Node k's world transform X (rotation row-major, then translation) from its
// parent's in sX, with its axes' cosines and sines cs; writes the world hinge
// axes, the DOF-to-node map, X (LDS and the slot) and the instance.
__device__ inline void compose(const ArtJob &J, int k, const ArtNode &nd, const double *cs, double *sX) {
    double X[12];
    if (k == 0) {
        for (int c = 0; c < 12; ++c) X[c] = (c == 0 || c == 4 || c == 8) ? 1.0 : 0.0;
    } else {
        double Pm[12];
        for (int c = 0; c < 12; ++c) Pm[c] = sX[12 * nd.parent + c];
        double prefix[9], Rl[9];
        for (int c = 0; c < 9; ++c) {
            prefix[c] = Pm[c];   // R_parent * R(a_0) ... R(a_{i-1})
            Rl[c] = (c == 0 || c == 4 || c == 8) ? 1.0 : 0.0;
        }
        #pragma unroll
        for (int a = 0; a < 3; ++a) {   // (unrolled: the node stays in registers)
            if (a >= nd.n_axes) break;
            const int q = nd.dof_offset + a;
            double w[3];
            mat3_vec(prefix, nd.axis[a], w);
            for (int c = 0; c < 3; ++c) J.axw[3 * q + c] = w[c];
            J.dof_node[q] = k;
            double Ra[9];
            rot_unit(nd.unit[a], cs[2 * a], cs[2 * a + 1], Ra);
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
    for (int c = 0; c < 12; ++c) {
        sX[12 * k + c] = X[c];
        J.xf[12 * k + c] = X[c];
    }
    Inst I;
    for (int c = 0; c < 9; ++c) I.R[c] = (float)X[c];
    for (int c = 0; c < 3; ++c) I.t[c] = (float)X[9 + c];
    I.root = nd.blas_root;
    I.node = k;
    I.pad[0] = I.pad[1] = 0.0f;
    J.inst[k] = I;
}

// Top-level node tp refitted from the instance boxes sB and the already
// refitted nodes sT: an instance leaf takes its world box, an inner child
// the union of its node's non-empty boxes.
__device__ inline void refit(BNode4 nd, int i, const ArtJob &J, const float *sB, BNode4 *sT) {
    for (int k = 0; k < 4; ++k) {
        const uint32_t r = nd.ref[k];
        if (r == REF_NONE) continue;
        float lo[3], hi[3];
        if (ref_type(r) == REF_TLAS_LEAF) {
            const uint32_t q = ref_index(r);
            for (int a = 0; a < 3; ++a) { lo[a] = sB[6 * q + a]; hi[a] = sB[6 * q + 3 + a]; }
        } else {
            const BNode4 &c = sT[ref_index(r)];
            for (int a = 0; a < 3; ++a) { lo[a] = INFINITY; hi[a] = -INFINITY; }
            for (int m = 0; m < 4; ++m) {
                if (c.ref[m] == REF_NONE) continue;
                lo[0] = lmin(lo[0], c.lox[m]); hi[0] = lmax(hi[0], c.hix[m]);
                lo[1] = lmin(lo[1], c.loy[m]); hi[1] = lmax(hi[1], c.hiy[m]);
                lo[2] = lmin(lo[2], c.loz[m]); hi[2] = lmax(hi[2], c.hiz[m]);
            }
        }
        nd.lox[k] = lo[0]; nd.loy[k] = lo[1]; nd.loz[k] = lo[2];
        nd.hix[k] = hi[0]; nd.hiy[k] = hi[1]; nd.hiz[k] = hi[2];
    }
    sT[i] = nd;
    J.tlas[i] = nd;
}

static_assert(SRP_MAX_NODES <= 2 * ART_BLOCK, "at most two tree nodes and two top-level nodes per lane");

__global__ __launch_bounds__(ART_BLOCK) void k_articulate(const ArtJob *__restrict__ jobs, int n_jobs) {
    __shared__ double sX[SRP_MAX_NODES * 12];   // node transforms
    __shared__ float sB[SRP_MAX_NODES * 6];     // instance boxes (lo, hi)
    __shared__ BNode4 sT[SRP_MAX_NODES];        // refitted top-level nodes
    if ((int)blockIdx.x >= n_jobs) return;
    const ArtJob J = jobs[blockIdx.x];
    const int lane = threadIdx.x;
    // Each lane's tree nodes (lane and lane + ART_BLOCK), their axes' cosines
    // and sines, and its top-level nodes, read once: the level loops below then
    // wait on LDS only, not on a memory round trip per level.
    ArtNode nd[2];
    double cs[2][6];
    BNode4 tp[2];
    #pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int k = lane + s * ART_BLOCK;
        if (k < J.n_nodes) nd[s] = J.nodes[k];
        if (k < J.n_tlas) tp[s] = J.topo[k];
    }
    #pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int k = lane + s * ART_BLOCK;
        #pragma unroll
        for (int a = 0; a < 3; ++a)
            if (k < J.n_nodes && a < nd[s].n_axes) {
                cs[s][2 * a] = J.cs[2 * (nd[s].dof_offset + a)];
                cs[s][2 * a + 1] = J.cs[2 * (nd[s].dof_offset + a) + 1];
            }
    }
    // node transforms, one tree level after the other
    for (int L = 0; L <= J.max_depth; ++L) {
        #pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int k = lane + s * ART_BLOCK;
            if (k < J.n_nodes && nd[s].depth == L) compose(J, k, nd[s], cs[s], sX);
        }
        __syncthreads();
    }
    // the instances' world boxes
    #pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int k = lane + s * ART_BLOCK;
        if (k < J.n_nodes && nd[s].blas_root != REF_NONE) inst_box(nd[s], sX + 12 * k, J.pad, sB + 6 * k, sB + 6 * k + 3);
    }
    __syncthreads();
    // refit, one height after the other
    for (int hgt = 0; hgt <= J.max_height; ++hgt) {
        #pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int i = lane + s * ART_BLOCK;
            if (i < J.n_tlas && (int)tp[s].pad[0] == hgt) refit(tp[s], i, J, sB, sT);
        }
        __syncthreads();
    }
}

}  // namespace

int launch_articulate(const ArtJob *d_jobs, int n_jobs, void *stream) {
    if (n_jobs <= 0) return 0;
    hipLaunchKernelGGL(k_articulate, dim3(n_jobs), dim3(ART_BLOCK), 0, (hipStream_t)stream, d_jobs, n_jobs);
    return (int)hipGetLastError();
}

}  // namespace srp
