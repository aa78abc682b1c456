// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lxns.h"

namespace lx {

constexpr int kMaxValves = 8;
constexpr int kMaxBC = 16;
constexpr int kMaxRestart = 64;
// Earlier lifting solutions kept to project the next lifting's initial guess on.
constexpr int kProjMax = 8;

// Per-step scalar coefficients passed by value to the element kernels.
struct StepCoef {
    double alpha;          // BDF alpha at this step
    double sigma;          // BDF order used at this step (tau_M first term)
    double dt, rho, mu, C_r;
    double beta[3];        // u_BDF = sum_l beta[l] u^{n-l}
    double gamma[3];       // u_EXT = sum_l gamma[l] u^{n-l} (same weights for p_EXT)
    int32_t nlev;          // history levels combined
    int32_t stab;          // LX_STAB_*
    int32_t symgrad;       // 1: symmetric-gradient diffusion
    int32_t n_valves;
    // valves at t^{n+1}: center[3], unit normal[3], r_in, r_out, R, eps
    double valve[kMaxValves][10];
};

// Boundary data of one Dirichlet/no-slip condition at t^{n+1}.
struct BCVal {
    int32_t type;          // LX_BC_*
    int32_t profile;       // LX_PROFILE_*
    double scale;          // theta * g(t^{n+1})
    double center[3], normal[3], radius;
};
struct BCSet {
    int32_t n;
    int32_t ale;
    BCVal bc[kMaxBC];
};

// Device-side GMRES state (one per solver instance).
struct GmState {
    double H[(kMaxRestart + 1) * kMaxRestart];  // Hessenberg, row-major [i][j], stride kMaxRestart
    double cs[kMaxRestart], sn[kMaxRestart];
    double g[kMaxRestart + 1];
    double s[kMaxRestart + 1];      // V_j = s[j] * Vhat_j
    double y[kMaxRestart];          // least-squares solution of the cycle
    double tol_abs;                 // stop when |g_{k+1}| <= tol_abs
    double resid;                   // current residual estimate (or true at start)
    double norms[4];                // result slots of plain norm kernels
    double lam_max;                 // Gershgorin bound of diag(S~)^{-1} S~ (Chebyshev interval)
    int32_t kused;                  // Arnoldi columns completed in this cycle
    int32_t done;                   // 1: no further work this cycle
    int32_t converged;
    int32_t breakdown;
    uint32_t counter;               // last-block arrival counter (reset by the last block)
    double reorth_frac;             // second pass when the first removed more than this share of ||w||^2
    int32_t reorth;                 // 1: the current Arnoldi step takes a second Gram-Schmidt pass
    int32_t n_reorth;               // second passes taken in this cycle
    int32_t pad;
};

// Host error reporting.
void set_error(const char *fmt, ...);
lx_status fail(lx_status st, const char *fmt, ...);

#define LX_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t _e = (call);                                                        \
        if (_e != hipSuccess)                                                          \
            return ::lx::fail(LX_EDEVICE, "%s failed: %s (%s:%d)", #call,              \
                              hipGetErrorString(_e), __FILE__, __LINE__);              \
    } while (0)

// ---------------------------------------------------------------- host setup
struct HostSetup {
    int64_t nv = 0, nt = 0;
    std::vector<int32_t> perm_v;    // new -> old vertex
    std::vector<int32_t> iperm_v;   // old -> new vertex
    std::vector<int64_t> perm_e;    // new -> old element
    std::vector<double> xh;         // [nv][3] reference coordinates, new numbering
    std::vector<int32_t> tet_soa;   // [4][nt] new numbering, local order kept
    std::vector<int32_t> rowptr;    // [nv+1] block rows
    std::vector<int32_t> col;       // [nblk]
    std::vector<int32_t> diag;      // [nv] slot of the diagonal block
    std::vector<int32_t> tslot;     // [nblk] slot of the transposed block
    std::vector<int32_t> eslot;     // [16][nt] slot of block (a,b), index (4a+b)*nt + e
    std::vector<int32_t> sinc_ptr;  // [nblk+1] incidence of each slot ...
    std::vector<int32_t> sinc;      // [16 nt]  ... as codes 16 e + 4a + b, by element then (a, b)
    std::vector<int32_t> vinc_ptr;  // [nv+1] vertex incidence: the diagonal slots' lists in vertex order
    std::vector<int32_t> vpos;      // [4][nt] position of (element, local vertex) in that order
    double hmin = 0;
};

// Validates, renumbers (RCM) and builds the pattern.  Returns LX_OK or an error.
lx_status build_setup(const lx_mesh *mesh, HostSetup &hs);

}  // namespace lx
