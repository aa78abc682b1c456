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
    // Sliced-ELL storage (the finest level): rows in slices of 64, entry j of row i
    // at soff[i / 64] + 64 j + i % 64, slices as wide as their longest row, the
    // padding a zero value in the row's own column.  val and scol then hold
    // that layout (rowptr/col keep the CSR pattern); soff = null: plain CSR.
    // Columns are stored as 16-bit offsets from the row (sdel) when every one
    // fits, else as 32-bit indices (scol).
    int32_t *soff = nullptr, *swid = nullptr, *scol = nullptr;
    int16_t *sdel = nullptr;
    int64_t nsell = 0;
};

// Position of CSR entry e of row i in the sliced-ELL layout.
inline int64_t sell_pos(const std::vector<int32_t> &soff, const std::vector<int32_t> &rowptr, int64_t i, int64_t e)
{
    return (int64_t)soff[i >> 6] + (e - rowptr[i]) * 64 + (i & 63);
}

// The coarse end of the hierarchy (from level `first` down to the dense level)
// runs as one workgroup out of LDS.  Its arrays sit in one device buffer laid
// out exactly as the LDS image (offsets in bytes, 16-byte aligned): the dense
// augmented matrix, the member lists of level first - 1 (for the restriction
// onto level first; left in global memory when they would not fit), then per level the values, dinv, row pointers, columns,
// aggregate map and member lists; the set-up kernels write values, dinv and the
// dense inverse there, and the cycle copies the image into LDS in one pass.
// The level vectors follow the image in LDS only.
constexpr int kTailDepth = 3;          // smoothed levels the one-workgroup cycle may hold
constexpr int kTailThreads = 1024;
constexpr int kTailMaxRows = 1024;

struct TailLevelLds {
    int32_t n = 0, nnz = 0, nn = 0, lanes = 1;   // rows, entries, rows of the next level, lanes per row
    int32_t o_val = 0, o_dinv = 0, o_rowptr = 0, o_col = 0, o_agg = 0, o_mptr = 0, o_mem = 0;
    int32_t o_r = 0, o_res = 0, o_x0 = 0, o_x1 = 0, o_d0 = 0, o_d1 = 0;
};

struct TailLayout {
    int first = 0, nlev = 0, nc = 0;   // first: 0 = no one-workgroup cycle
    int32_t o_dense = 0, o_rc = 0, o_xc = 0;
    int32_t o_fmptr = -1, o_fmem = -1; // member lists of level first - 1 in the image (-1: read globally)
    int32_t o_fstage = -1;             // LDS copy of level first - 1's residual in member order (-1: none)
    int32_t img_bytes = 0, lds_bytes = 0;
    TailLevelLds lv[kTailDepth];
};

// Device state of the two block approximations.  Scalar slots of lam:
// [0, kAmgMaxLevels) Gershgorin bounds of diag(A_l)^{-1} A_l, kLamF the
// Chebyshev bound of F~^{-1} F, kNormA/kNormB the power-iteration norms.
constexpr int kLamF = kAmgMaxLevels, kNormA = kAmgMaxLevels + 1, kNormB = kAmgMaxLevels + 2, kLamSlots = 16;
// Most lanes per row any row kernel of the preconditioner runs with (LXNS_LPR and
// LXNS_AMG_LPR accept 4..32): sizes the per-workgroup partial sums (Amg::partial).
constexpr int kMaxRowLanes = 32;

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
    int cycle_coarse = 1;               // the same on the levels from coarse_from on
    int coarse_from = 1 << 20;          // first level that fits one workgroup's LDS
    double ratio = 30.0;                // smoothing interval [lam / ratio, lam]
    int f_degree = 3;                   // Chebyshev degree on F (1: plain block Jacobi)
    double f_ratio = 10.0;
    int f_pow_first = 16, f_pow_iters = 2;   // power iterations for the bound of F~^{-1} F (first step; later, warm)
    double f_safety = 1.15;
    bool f_warm = false;                // fv holds the last power-iteration vector
    T *fr = nullptr, *fd0 = nullptr, *fd1 = nullptr, *fv = nullptr;   // [nv][4]
    TailLayout tail;                    // one-workgroup coarse cycle (tail.first = 0: none)
    unsigned char *tail_img = nullptr;  // [tail.img_bytes]
    // The one-workgroup cycle is linear in the restricted residual it starts
    // from, so each step its operator is tabulated, column j = the cycle applied
    // to the unit vector e_j ([n][n], column-major, n the rows of level
    // tail.first), and every visit is then the restriction and one dense
    // product instead of a chain of workgroup barriers (null: cycle each visit).
    T *tail_op = nullptr;
    T *tail_rc = nullptr;               // [n] the restricted residual a tabulated visit starts from
};

// Chooses the first level of the one-workgroup coarse cycle and its LDS layout
// from the level sizes (n[l], nnz[l] for l = 0..nlev; level nlev dense) for a
// value size vbytes; tail.first = 0 if no suffix of the hierarchy fits max_lds.
TailLayout amg_tail_layout(int nlev, const int64_t *n, const int64_t *nnz, int vbytes, int64_t max_lds);

// Lets the one-workgroup cycle kernel use lds_bytes of dynamic LDS.
template <typename T>
lx_status amg_tail_prepare(int lds_bytes);

// The blocks of the saddle-point matrix as the preconditioner sees them: F as a
// 3x3 block-CSR over the velocity nodes (9 planes of stride Fp.nblk), G (rows:
// velocity nodes, columns: pressure rows; 3 planes of stride gs), B (rows:
// pressure rows, columns: velocity nodes; 3 planes of stride bs) and C (pressure
// pattern).  For P1-P1 all four share the vertex block pattern; for P2-P1 they
// are the split parts.  Vectors are [nu][4] with the pressure in component 3
// of the first np nodes (0 elsewhere).
template <typename T>
struct SimpleView {
    int64_t nu, np;
    RowPattern Fp;
    const T *F;
    const int32_t *gptr, *gcol;
    const T *Gv;
    int64_t gs;
    const int32_t *bptr, *bcol;
    const T *Bv;
    int64_t bs;
    const int32_t *cptr, *ccol;
    const T *Cv;
};

// View of the P1-P1 block pattern with planes F 0-8, G 9-11, B 12-14, C 15.
template <typename T>
inline SimpleView<T> simple_view_p1(const RowPattern &P, const T *val)
{
    SimpleView<T> V;
    V.nu = V.np = P.nv;
    V.Fp = P;
    V.F = val;
    V.gptr = V.bptr = V.cptr = P.rowptr;
    V.gcol = V.bcol = V.ccol = P.col;
    V.Gv = val + 9 * P.nblk;
    V.Bv = val + 12 * P.nblk;
    V.Cv = val + 15 * P.nblk;
    V.gs = V.bs = P.nblk;
    return V;
}

// Per-step numeric set-up: forms S~, every coarse level, the dense inverse and
// the Chebyshev bounds.  Finv / Dinv come from the SIMPLE set-up.
template <typename T>
void launch_amg_setup(const SimpleView<T> &V, const T *Finv, const T *Dinv, Amg<T> &A, hipStream_t s);

// z <- M^{-1} (scale * r) for the SIMPLE preconditioner with the AMG Schur block
// and the Chebyshev velocity block.
// start_done: z.u, z.p and the Chebyshev start of the velocity block were
// already written (by the Gram-Schmidt pass that formed r, see amg_fz_start).
template <typename T>
void launch_simple_amg_apply(const SimpleView<T> &V, const T *Finv, const T *Dinv, Amg<T> &A, const T *r,
                             const double *scale_ptr, T *z, const int32_t *done, hipStream_t s,
                             bool start_done = false);

// The velocity block's start for a direction whose preconditioned vector goes to z.
template <typename T>
inline FzStart<T> amg_fz_start(const Amg<T> &A, const T *Finv, T *z)
{
    FzStart<T> f;
    f.Finv = Finv;
    f.z = z;
    f.fr = A.fr;
    f.fd = A.fd0;
    f.lamF = &A.lam[kLamF];
    f.ratio = A.f_ratio;
    f.degree = A.f_degree;
    return f;
}

}  // namespace lx
