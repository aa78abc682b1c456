// Device kernels of the step and their host launchers.
#pragma once

#include "lx_common.h"

namespace lx {

// Block values are stored as 16 planes of length nblk ("SoA" block-CSR):
// plane 3c+d holds F[c][d] (velocity-velocity), 9+c holds G[c] (velocity row,
// pressure column), 12+d holds B[d] (pressure row, velocity column), 15 holds
// C.  Vectors are [nv][4] = (u_x, u_y, u_z, p) per vertex.
constexpr int kPlanes = 16;

// Per-element record written by the element pass of the P1 assembly and read
// by the slot gather (kRec values of T per element in all: the records, then
// the elements' right-hand side blocks).
constexpr int kRec = 72;

template <typename T>
struct AsmArgs {
    int64_t nt, nblk;
    const int32_t *tet;    // [4][nt]
    const int32_t *sinc_ptr, *sinc;   // slot incidence (codes 16 e + 4a + b)
    T *rec;                // [kRec nt] element records and right-hand side blocks
    const double *x;       // [nv][3] current coordinates
    const double *xh;      // [nv][3] reference coordinates
    const double *h0, *h1, *h2;  // history levels [nv][4]
    const double *uA;      // [nv][3] ALE velocity or null
    const double *f;       // [nv][3] forcing or null
    T *val;                // planes
    T *rhs;                // [nv][4] or null
};

// Contributions of the FP64 residual, one per (element, local vertex), stored in
// vertex-incidence order: r [4 nt][4], then b [4 nt][4], then the Dirichlet
// diagonal [4 nt][4] (3 used): kRRec doubles per element in all.
constexpr int kRRec = 48;

struct ResArgs {
    int64_t nt, nv;
    const int32_t *tet;
    const int32_t *vinc_ptr, *vpos;   // vertex incidence ranges; position of (element, local vertex)
    double *rec;             // [3][4 nt][4]
    const double *x, *xh, *h0, *h1, *h2, *uA, *f;
    const double *xs;        // iterate [nv][4]
    const int32_t *dir_index;  // [nv] Dirichlet index or -1
    double *r;               // [nv][4] accumulates b - A xs (non-Dirichlet rows)
    double *b;               // [nv][4] accumulates b, or null
    double *dg;              // [n_dir][3] accumulates FP64 diagonal of Dirichlet rows, or null
};

struct RowPattern {
    int64_t nv, nblk;
    const int32_t *rowptr, *col, *diag, *tslot;
    int32_t remap = 1;   // die-contiguous workgroup ranges (0: rows of very unequal length, as P2's)
};

template <typename T>
void launch_assemble_p1(const AsmArgs<T> &a, const StepCoef &c, hipStream_t s);
void launch_residual_p1(const ResArgs &a, const StepCoef &c, hipStream_t s);

void launch_dirichlet_values(int64_t n_dir, const int32_t *dir_node, const int32_t *dir_bc,
                             const BCSet &bcs, const double *x, const double *uA,
                             const double *gnodal, double *g, hipStream_t s);
template <typename T>
void launch_dirichlet_rows(int64_t n_dir, const int32_t *dir_node, const double *g,
                           const RowPattern &P, T *val, T *rhs, hipStream_t s);
void launch_dirichlet_residual(int64_t n_dir, const int32_t *dir_node, const double *g,
                               const double *dg, const double *xs, double *r, double *b,
                               hipStream_t s);
void launch_neumann(int64_t nf, const int32_t *faces, const double *x, const double *hnodal,
                    const double hconst[3], double *out0, double *out1, float *out32,
                    hipStream_t s);

template <typename T>
void launch_simple_setup(const RowPattern &P, const T *val, T *Finv, T *Dinv, T *Sinv, hipStream_t s);
// st->lam_max = Gershgorin bound of diag(S~)^{-1} S~, S~ = C - B D^{-1} G (not formed);
// work: 4 nv entries of T.
template <typename T>
void launch_schur_bound(const RowPattern &P, const T *val, const T *Dinv, const T *Sinv, T *work,
                        GmState *st, double *partial, int nb, hipStream_t s);

// The SIMPLE preconditioner's operands.  degree = 0: S~^{-1} ~ diag(S~)^{-1};
// degree k > 0: k-step Chebyshev iteration on S~ z = t with diagonal scaling on
// [lam_max / ratio, lam_max] (work: 9 nv entries of T).
template <typename T>
struct Simple {
    const T *val, *Finv, *Dinv, *Sinv;
    int degree;
    double ratio;
    T *work;
    const GmState *st;
};
// z <- SIMPLE^{-1} (scale * r), scale = *scale_ptr (or 1 if null)
template <typename T>
void launch_simple_apply(const RowPattern &P, const Simple<T> &S, const T *r, const double *scale_ptr, T *z,
                         const int32_t *done, hipStream_t s);
template <typename T>
void launch_spmv(const RowPattern &P, const T *val, const T *x, T *y, const int32_t *done,
                 hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// GMRES building blocks (vectors of length n = 4 nv, basis stride ldv).  Each
// reduction writes per-block partial sums into partial (gm_partial_size(n)
// doubles) and a one-block kernel finishes it.
constexpr int kDotChunk = 4096;
int64_t gm_partial_size(int64_t n);
// r = b - Ax (Ax null: r = b), V0 = r, beta = ||r||; starts a cycle or marks it done
template <typename T>
void launch_gm_start(int64_t n, const T *b, const T *Ax, T *V0, GmState *st, double *partial, hipStream_t s);
// The first pass of the velocity block's Chebyshev iteration on the next Arnoldi
// direction r = V_{k+1}, done by the Gram-Schmidt pass that completes it:
// z.u = F~^{-1} r.u / theta with fr = r.u and fd = z.u (degree > 1), or
// z.u = F~^{-1} r.u (degree 1); z.p = r.p.  Vectors [nv][4], Finv [9][nv].
template <typename T>
struct FzStart {
    const T *Finv = nullptr;
    T *z = nullptr, *fr = nullptr, *fd = nullptr;
    const double *lamF = nullptr;   // Chebyshev bound of F~^{-1} F
    double ratio = 1.0;
    int degree = 1;
};
// CGS2 of w against Vhat_0..Vhat_k, Vhat_{k+1}, Hessenberg column k and its Givens
// update; fz (optional): also the velocity block's start on V_{k+1}
template <typename T>
void launch_gm_orth(int64_t n, int k, T *V, int64_t ldv, T *w, GmState *st, double *partial, hipStream_t s,
                    const FzStart<T> *fz = nullptr);
void launch_gm_solve_y(GmState *st, hipStream_t s);
// x += sum_j y_j Z_j (flexible GMRES solution update)
template <typename T>
void launch_gm_update(int64_t n, const T *Z, int64_t ldz, const GmState *st, T *x, hipStream_t s);
// st->norms[slot] = ||x||; if rtol > 0, st->tol_abs = rtol * ||x||
template <typename T>
void launch_norm(int64_t n, const T *x, GmState *st, double rtol, double *partial, int slot, hipStream_t s);

// vector utilities
template <typename T>
void launch_fill(int64_t n, T *x, T v, hipStream_t s);
// out[0..2] = squared 2-norm errors of the BDF (gamma), quadratic (nk >= 2) and
// cubic (nk >= 3) extrapolations of h[0..3] against x; all four h are read
// (allocated, finite); partial: 3 * 256 doubles.
constexpr int kGuessErrPartial = 3 * 256;
void launch_guess_err(int64_t n, int nk, const double *x, const double *const *h, const double *gamma,
                      double *partial, double *out, hipStream_t s);

// x = g0 h0 + g1 h1 + g2 h2 + g3 h3 (null levels left out)
void launch_extrapolate(int64_t n, double *x, const double *h0, const double *h1, const double *h2, double g0,
                        double g1, double g2, hipStream_t s, const double *h3 = nullptr, double g3 = 0.0);
template <typename TD, typename TS>
void launch_axpy(int64_t n, TD *y, const TS *x, const double *scale_ptr, double scale, hipStream_t s);
// dst = (TD)(src * factor)
template <typename TD, typename TS>
void launch_scale_copy(int64_t n, TD *dst, const TS *src, double factor, hipStream_t s);
void launch_set_dirichlet_x(int64_t n_dir, const int32_t *dir_node, const double *g, double *xs,
                            hipStream_t s);

}  // namespace lx
