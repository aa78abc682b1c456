// The P2-P1 (Taylor-Hood) pair of the paper (quadratic velocity, linear
// pressure; Sec. 2.3 allows FE degree 1 or 2 on tetrahedra): host set-up and
// device kernels of its split block system.
//
// Velocity nodes are the vertices (ids 0..nv-1, RCM order) followed by the
// edge midpoints (nv + k, edges ordered by their vertex pair).  Vectors keep
// the [node][4] layout of the P1 path: (u_x, u_y, u_z, p) on vertex nodes and
// (u_x, u_y, u_z, 0) on edge nodes, so the Krylov kernels are shared.  The
// matrix is stored as four block-CSR parts: F over node pairs (9 planes), G
// node x vertex (3 planes), B vertex x node (3 planes) and C on the vertex
// pattern of the P1 path (1 plane).
#pragma once

#include <vector>

#include "lx_common.h"
#include "lx_kernels.h"

namespace lx {

struct P2Setup {
    int64_t ne = 0, nu = 0;
    std::vector<uint64_t> edge_key;   // [ne] (lower << 32 | higher) new vertex ids, sorted
    std::vector<int32_t> nodes;       // [10][nt] P2 node ids of each element (vertices, then edges
                                      //  (0,1) (0,2) (0,3) (1,2) (1,3) (2,3))
    std::vector<double> xnode;        // [nu][3] reference coordinates of the nodes
    std::vector<int32_t> fptr, fcol, fdiag, finc_ptr, finc;   // F pattern and incidence
    std::vector<int32_t> gptr, gcol, ginc_ptr, ginc;          // G pattern and incidence
    std::vector<int32_t> bptr, bcol, binc_ptr, binc;          // B pattern and incidence
    // incidence codes: 128 e + 10 a + b with local indices a, b (velocity 0..9, pressure 0..3)
};

lx_status build_setup_p2(const HostSetup &hs, P2Setup &p2);
// node id of the edge between new vertex ids a and b, or -1
int32_t p2_edge_node(const P2Setup &p2, int64_t nv, int32_t a, int32_t b);

// Quadrature of the P2 element (degree 5): 27-point conical product rule on the
// unit simplex (barycentric [q][4], weights summing to 1/6), and the 9-point
// degree-5 rule on the unit triangle for the boundary traction (barycentric
// [q][3], weights summing to 1/2).  Generated on the host from Gauss-Jacobi
// points.
constexpr int kP2Q = 27, kP2FQ = 9;
struct P2Rules {
    double lam[kP2Q][4], w[kP2Q];
    double flam[kP2FQ][3], fw[kP2FQ];
};
void p2_rules(P2Rules &R);

// Element record of the P2 assembly: the 34 x 34 element matrix (rows and
// columns: velocity 3a + c, a = 0..9, then pressure 30 + a, a = 0..3) and the
// 34-entry right-hand side.
constexpr int kP2Rec = 34 * 34 + 34;

// Device view of the split system.
template <typename T>
struct P2Sys {
    int64_t nv, nu, nt;
    const int32_t *fptr, *fcol, *gptr, *gcol, *bptr, *bcol, *cptr, *ccol;
    int64_t nf, ng, nb, nc;            // slot counts (plane strides)
    T *F, *G, *B, *C;                  // planes: F[9][nf], G[3][ng], B[3][nb], C[nc]
};

struct P2AsmArgs {
    int64_t nt, nv, nu;
    const int32_t *tet, *nodes;        // [4][nt], [10][nt]
    const double *x, *xh;              // vertex coordinates (current = reference: no ALE)
    const double *h0, *h1, *h2;        // history [nu][4]
    const double *f;                   // [nu][3] or null
    const P2Rules *rules;              // device copy
    double *rec;                       // [nt][kP2Rec]
    const int32_t *finc_ptr, *finc, *ginc_ptr, *ginc, *binc_ptr, *binc, *cinc_ptr, *cinc;
    const int32_t *fdiag, *cdiag;      // diagonal slots (node rows of F, vertex rows of C)
};

void launch_assemble_p2(const P2AsmArgs &a, const StepCoef &c, const P2Sys<double> &S, double *rhs,
                        hipStream_t s);
// Dirichlet rows at velocity nodes: F rows keep only their diagonal, G rows are
// cleared, rhs = a_ii g (rhs may be null).
template <typename T>
void launch_dirichlet_rows_p2(int64_t n_dir, const int32_t *dir_node, const double *g, const P2Sys<T> &S,
                              const int32_t *fdiag, T *rhs, hipStream_t s);
// Neumann traction on the 6-node boundary triangles (vertices, then the edge
// nodes (0,1) (1,2) (2,0)); nodal traction [nu][3] or a constant vector.
void launch_neumann_p2(int64_t nf, const int32_t *faces6, const double *xnode, const double *hn,
                       const double hconst[3], const P2Rules *rules, double *out, hipStream_t s);
template <typename T>
void launch_simple_setup_p2(const P2Sys<T> &S, const int32_t *fdiag, T *Finv, T *Dinv, hipStream_t s);
template <typename T>
void launch_spmv_p2(const P2Sys<T> &S, const T *x, T *y, const int32_t *done, hipStream_t s,
                    hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// dst = (float) src over the four parts
void launch_round_p2(const P2Sys<double> &S64, const P2Sys<float> &S32, hipStream_t s);

}  // namespace lx
