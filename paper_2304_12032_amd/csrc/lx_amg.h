// Block approximations of the SIMPLE preconditioner built on device every step:
// an algebraic multigrid hierarchy for the Schur block S~ = C - B D^{-1} G and a
// Chebyshev-accelerated nodal block Jacobi iteration for the velocity block F.
//
// The paper's solver applies SIMPLE with its velocity and Schur blocks
// approximated by AMG, additive Schwarz or block Jacobi (Sec. 2.4).  Here the
// Schur block is formed explicitly (its pattern is the vertex 2-ring) and
// approximated by one cycle of unsmoothed-aggregation AMG with Chebyshev
// smoothing (a W-cycle below the finest level by default); the aggregates depend on the mesh only, so the host builds the
// hierarchy's patterns once and the device refreshes every level's values at
// each step (Galerkin products with piecewise-constant prolongation are plain
// sums over fixed index lists).  The coarsest level is inverted densely.
#pragma once

#include <vector>

#include "lx_common.h"
#include "lx_kernels.h"

namespace lx {

constexpr int kAmgMaxLevels = 8;    // smoothed levels above the dense coarsest one
constexpr int kAmgDenseMax = 256;   // size limit of the dense coarsest level

// Patterns of one level and its link to the next (host side, set-up only).
struct AmgLevelHost {
    int64_t n = 0;
    std::vector<int32_t> rowptr, col, diag;   // CSR pattern, sorted columns
    std::vector<int32_t> agg;                 // [n] aggregate (next-level row) of each row
    std::vector<int32_t> mptr, mem;           // members of each aggregate
    std::vector<int32_t> cptr, cidx;          // next-level entry c sums entries cidx[cptr[c]..cptr[c+1])
};

struct AmgHost {
    std::vector<AmgLevelHost> lev;   // lev[0]: S~ on the vertices; lev.back(): dense coarsest
};

// Builds the Schur pattern (2-ring of the block pattern) and the aggregation
// hierarchy.  Deterministic: depends only on the pattern.
lx_status amg_build_host(const HostSetup &hs, AmgHost &H);

template <typename T>
struct AmgLevel {
    int64_t n = 0, nnz = 0;
    int32_t *rowptr = nullptr, *col = nullptr, *diag = nullptr;
    T *val = nullptr, *dinv = nullptr;
    int32_t *agg = nullptr, *mptr = nullptr, *mem = nullptr, *cptr = nullptr, *cidx = nullptr;
    T *r = nullptr, *x0 = nullptr, *x1 = nullptr, *res = nullptr, *d0 = nullptr, *d1 = nullptr;
    int lpr = 16;
};

// Device state of the two block approximations.  Scalar slots of lam:
// [0, kAmgMaxLevels) Gershgorin bounds of diag(A_l)^{-1} A_l, kLamF the
// Chebyshev bound of F~^{-1} F, kNormA/kNormB the power-iteration norms.
constexpr int kLamF = kAmgMaxLevels, kNormA = kAmgMaxLevels + 1, kNormB = kAmgMaxLevels + 2, kLamSlots = 16;

template <typename T>
struct Amg {
    int nlev = 0;                       // smoothed levels; level nlev is the dense one
    AmgLevel<T> L[kAmgMaxLevels + 1];
    int64_t nc = 0;                     // dense size
    int32_t *crow = nullptr;            // row of each entry of level nlev
    double *dense = nullptr;            // [nc][2 nc] augmented matrix; right half = inverse
    double *lam = nullptr;              // [kLamSlots]
    double *partial = nullptr;
    uint32_t *counter = nullptr;
    int nb = 1;                         // reduction blocks
    int degree = 2;                     // Chebyshev smoothing degree (pre and post)
    int cycle = 1;                      // coarse corrections per level below the finest (1 V, 2 W)
    double ratio = 30.0;                // smoothing interval [lam / ratio, lam]
    int f_degree = 3;                   // Chebyshev degree on F (1: plain block Jacobi)
    double f_ratio = 10.0;
    int f_pow_first = 16, f_pow_iters = 6;   // power iterations for the bound of F~^{-1} F
    double f_safety = 1.15;
    bool f_warm = false;                // fv holds the last power-iteration vector
    T *fr = nullptr, *fd0 = nullptr, *fd1 = nullptr, *fv = nullptr;   // [nv][4]
};

// Per-step numeric set-up: forms S~, every coarse level, the dense inverse and
// the Chebyshev bounds.  Finv / Dinv come from launch_simple_setup.
template <typename T>
void launch_amg_setup(const RowPattern &P, const T *val, const T *Finv, const T *Dinv, Amg<T> &A,
                      hipStream_t s);

// z <- M^{-1} (scale * r) for the SIMPLE preconditioner with the AMG Schur block
// and the Chebyshev velocity block.
template <typename T>
void launch_simple_amg_apply(const RowPattern &P, const T *val, const T *Finv, const T *Dinv, Amg<T> &A,
                             const T *r, const double *scale_ptr, T *z, const int32_t *done, hipStream_t s);

}  // namespace lx
