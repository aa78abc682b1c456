// Outflow boundary terms (resistance, backflow stabilisation) of P1-P1
// problems and boundary integrals: device data and launchers.
#pragma once

#include "lx_common.h"

namespace lx {

// One Neumann or resistance condition with a backflow or resistance term.
// Vertex ids are the library's numbering; faces are the condition's boundary
// triangles in mesh order.
struct OutflowDev {
    int bc = -1;
    double dir[3] = {0, 0, 0};   // outward direction that orients the face normals
    double cr = 0.0;             // C_R (0: no resistance term)
    double beta = 0.0;           // backflow beta (0: none)
    int64_t nf = 0, nbv = 0, npair = 0, nrow = 0;
    const int32_t *faces = nullptr;   // [nf][3]
    double *geom = nullptr;           // [nf][4] unit normal, area
    int32_t *bv = nullptr;            // [nbv] boundary vertices, ascending
    int32_t *vptr = nullptr, *vinc = nullptr;   // per boundary vertex: codes 3 f + l, ascending f
    int32_t *keep = nullptr;          // [nbv] 1: the vertex's rows take the terms (not Dirichlet)
    double *w = nullptr;              // [nbv][3] int phi_v n
    // backflow pairs (a, b), a kept, sorted by (a, b): block of (a, b), column b,
    // incidences (f << 4 | la << 2 | lb) in ascending f, coefficient
    int32_t *pblk = nullptr, *pcol = nullptr, *pptr = nullptr, *pinc = nullptr;
    double *pcoef = nullptr;
    int32_t *rptr = nullptr, *rvert = nullptr;   // pairs grouped by row: [nrow + 1], row vertex
};

// Face geometry, flux weights and backflow coefficients of the coming step
// (x: configuration x^{n+1}; h0..h2 and gamma: u_EXT).
void launch_outflow_prepare(const OutflowDev &o, const double *x, const double *h0, const double *h1,
                            const double *h2, const double gamma[3], double rho, hipStream_t s);
// Backflow coefficients into the assembled planes.
template <typename T>
void launch_backflow_add(const OutflowDev &o, int64_t nblk, T *val, hipStream_t s);
// Matrix-free FP64 residual: r -= backflow x + C_R (w . x) w; r (and b) += the
// resistance right-hand side.
void launch_outflow_residual(const OutflowDev &o, double p0, const double *uA, const double *xs, double *r, double *b,
                             hipStream_t s);
// Resistance right-hand side into an assembled FP64 right-hand side.
void launch_outflow_rhs(const OutflowDev &o, double p0, const double *uA, double *rhs, hipStream_t s);
// y += C_R (w . x) w (after the sparse product; skipped when *done is set).
template <typename T>
void launch_rank1(const OutflowDev &o, const T *x, T *y, const int32_t *done, hipStream_t s);
// (int (u - u_ALE) . n, int p, area) over faces into out[3] (device).
void launch_boundary_integrals(int64_t nf, const int32_t *faces, const double *x, const double dir[3],
                               const double *u, const double *uA, double *out, hipStream_t s);

}  // namespace lx
