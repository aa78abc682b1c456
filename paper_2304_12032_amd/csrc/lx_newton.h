// Fully implicit P1-P1 formulation: Newton systems (Jacobian and residual per
// element, gathered per block) and the Dirichlet values of the Newton update.
#pragma once

#include "lx_common.h"

namespace lx {

// Per element: the 16 x 16 Jacobian (row-major, local index 3a+c then 12+a) and
// the 16-entry residual.
constexpr int kNewtonRec = 272;

struct NewtonArgs {
    int64_t nt, nblk;
    const int32_t *tet;                // [4][nt]
    const int32_t *sinc_ptr, *sinc;    // slot incidence (codes 16 e + 4a + b)
    const double *x, *xh;              // [nv][3] current and reference coordinates
    const double *xs;                  // [nv][4] Newton iterate
    const double *h0, *h1, *h2;        // history levels [nv][4] (u_BDF)
    const double *uA, *f;              // [nv][3] or null
    double *rec;                       // [nt][kNewtonRec]
    double *val;                       // 16 planes [nblk]
    double *rhs;                       // [nv][4]: -R
};

// Element Jacobians and residuals at the iterate, then the block planes and -R.
void launch_newton_p1(const NewtonArgs &a, const StepCoef &c, hipStream_t s);
// gd = g - xs on the Dirichlet velocity entries.
void launch_dirichlet_delta(int64_t n_dir, const int32_t *node, const double *g, const double *xs, double *gd,
                            hipStream_t s);

}  // namespace lx
