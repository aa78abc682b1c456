/*
 * lxns.h -- C ABI of the MI355X (gfx950) library for one semi-implicit BDF time
 * step of the VMS-LES-stabilised incompressible Navier-Stokes equations on
 * tetrahedral meshes, with RIIS resistive immersed valves and ALE mesh motion
 * (Africa et al., "lifex-cfd", arXiv 2304.12032).
 *
 * Every call returns an lx_status; nothing throws or aborts across the ABI.
 * On a negative status, lx_last_error() returns a thread-local message that is
 * valid until the next call on the same thread.
 *
 * Conventions for all calls:
 *   - All array arguments are HOST pointers to caller-owned memory.  Inputs are
 *     copied before the call returns; the caller may free them afterwards.
 *     Outputs are written into caller buffers whose sizes follow lx_sim_query.
 *   - Layouts: coordinates and vector fields are node-major [n][3] doubles;
 *     pressure is [n_vertices] doubles; connectivity is [n_tets][4] int32,
 *     0-based.  Vertex ids are the caller's; the library renumbers internally
 *     and maps back on output.
 *   - The library owns all device memory it allocates (hipMalloc on the
 *     device named in lx_device) and frees it in the matching destroy call.
 *   - Work is queued on the stream given in lx_device (NULL: the library
 *     creates its own); calls that return host data synchronise that stream.
 *   - Units are the caller's, used consistently (the synthetic vascular cases
 *     are in CGS).
 */
#ifndef LXNS_H
#define LXNS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LX_OK = 0,
    LX_EINVAL = -1,    /* bad argument or unsupported option                         */
    LX_ENOMEM = -2,    /* host or device allocation failed                           */
    LX_EDEVICE = -3,   /* HIP runtime error                                          */
    LX_ENOCONV = -4,   /* GMRES / refinement missed its tolerance; state NOT advanced */
    LX_EMESH = -5,     /* degenerate tetrahedron (|det J| <= 1e-14 h^3) or bad ids    */
    LX_EBUSY = -6,     /* request exceeds the server's device-memory budget           */
    LX_ESTATE = -7     /* call not valid in the object's current state               */
} lx_status;

const char *lx_last_error(void);

/* ------------------------------------------------------------------ inputs */

/* Where an object runs: the device, the stream its work is queued on, and
 * optionally the caller's device allocator (PyTorch's caching allocator plugs
 * in here).  With alloc/free set, every device buffer of the object comes from
 * alloc(bytes, ctx) -- device memory on `device`, usable on hip_stream, at
 * least 256-byte aligned, NULL on failure (the call then returns LX_ENOMEM) --
 * and goes back through free(ptr, ctx) when the object is destroyed; both are
 * called from the thread that makes the library call (for a server: its worker
 * threads).  With both NULL the library uses hipMalloc / hipFree.  Pinned host
 * staging (a few hundred bytes per object) always comes from hipHostMalloc. */
typedef struct {
    int32_t device;      /* HIP device ordinal                                       */
    void *hip_stream;    /* hipStream_t to queue work on, or NULL                    */
    void *(*alloc)(size_t bytes, void *ctx);   /* optional device allocator          */
    void (*free)(void *ptr, void *ctx);        /* its release; both or neither       */
    void *ctx;                                 /* passed back to alloc / free        */
} lx_device;

/* Mesh (the paper's mesh input, Sec. 3.1): reference configuration x^ and a
 * labelled boundary. */
typedef struct {
    int64_t n_vertices, n_tets, n_bfaces;
    const double *coords;     /* [n_vertices][3] reference coordinates x^       */
    const int32_t *tets;      /* [n_tets][4]; the local vertex order is kept and
                                 defines the element map of the unit simplex     */
    const int32_t *bfaces;    /* [n_bfaces][3] vertex ids of boundary triangles  */
    const int32_t *bface_tag; /* [n_bfaces] boundary tags                       */
} lx_mesh;

/* Time laws g(t) of Sec. 2.2.1. */
enum {
    LX_LAW_CONSTANT = 0,  /* p = {g}                                                  */
    LX_LAW_PULSATILE = 1, /* p = {gmin, gmax, period}: gmin + (gmax-gmin)(1-cos 2pi t/T)/2 */
    LX_LAW_RAMP = 2,      /* p = {g0, g1, t0, tL}: sinusoidal ramp from g0 to g1         */
    LX_LAW_RAMP2 = 3,     /* p = {g0, g1, t_open, dur_open, t_close, dur_close, period}:
                             ramp up then back down, repeated every period if > 0      */
    LX_LAW_LINEAR = 4,    /* p = {g0, g1}: g0 + g1 t (rigid mesh translation)           */
    LX_LAW_SINE = 5       /* p = {A, w, phi}: A sin(w t + phi) (the time factor of the
                             ALE verification displacement, Appendix A)                 */
};
typedef struct {
    int32_t kind;
    int32_t pad;
    double p[8];
} lx_time_law;

/* Space profiles s(x) of Sec. 2.2.1. */
enum {
    LX_PROFILE_UNIFORM = 0,   /* s = -n                                               */
    LX_PROFILE_PARABOLIC = 1, /* s = -2 (R^2 - r^2)/(pi R^4) n, unit flow rate        */
    LX_PROFILE_NODAL = 2      /* values supplied per step (lx_sim_set_dirichlet_values /
                                 lx_sim_set_neumann_traction)                          */
};
typedef struct {
    int32_t kind;
    int32_t pad;
    double center[3];         /* r = |x - center|                                     */
    double normal[3];         /* outward unit normal n of the boundary portion        */
    double radius;            /* R of the parabolic profile                           */
} lx_profile;

/* Boundary conditions, Sec. 2.2: no-slip u = u_ALE (or 0), Dirichlet
 * u = theta g(t) s(x), Neumann sigma(u,p) n = -theta h(t) n (uniform profile)
 * or a nodal traction vector (nodal profile).  Where conditions share a
 * vertex, no-slip wins, then the first Dirichlet condition in the list.
 *
 * Resistance (Sec. 2.2, resistance boundary conditions; P1-P1):
 *   sigma(u,p) n = -(theta p0(t) + C_R int_Gamma (u - u_ALE) . n) n,
 * p0 = law, C_R = resistance >= 0, taken implicitly: the flux functional
 * w . u (w_v = int_Gamma phi_v n, face normals oriented along profile.normal)
 * couples the condition's vertices through the rank-1 term C_R w w^T, applied
 * beside the sparse matrix in every operator product (rows of Dirichlet
 * vertices excluded), and lx_sim_debug_export leaves it out.
 * Inertial backflow stabilisation (Sec. 2.2, Neumann conditions; P1-P1):
 * backflow = beta > 0 on a Neumann or resistance condition adds
 * beta rho/2 min(u . n, 0) u to the traction, semi-implicitly as
 * min(u_EXT . n, 0) u^{n+1} (a boundary mass term, edge-midpoint rule), to the
 * rows of its non-Dirichlet vertices. */
enum { LX_BC_NOSLIP = 0, LX_BC_DIRICHLET = 1, LX_BC_NEUMANN = 2, LX_BC_RESISTANCE = 3 };
typedef struct {
    int32_t type;
    int32_t n_tags;
    const int32_t *tags;
    double theta;
    lx_time_law law;
    lx_profile profile;
    double resistance;       /* C_R of a resistance condition                        */
    double backflow;         /* beta of the backflow stabilisation (0: off)          */
} lx_boundary;

/* RIIS immersed surface (Sec. 2.1.2, eq. (riis)): an annular disc (center, unit
 * normal, outer radius, central orifice radius following a time law) with
 * resistance R and half-thickness eps.  The distance is measured at the
 * reference position of each quadrature point, so the surface moves with the
 * mesh; the surface velocity u_Sigma is zero. */
typedef struct {
    double center[3];
    double normal[3];
    double outer_radius;
    lx_time_law orifice_radius;
    double R, eps;
} lx_riis;

enum { LX_P1P1 = 1, LX_P2P1 = 2 };
enum { LX_DIFF_GRADGRAD = 0, LX_DIFF_SYMGRAD = 1 };              /* eq. (diffusion-term) */
enum { LX_STAB_NONE = 0, LX_STAB_SUPG_PSPG = 1, LX_STAB_VMS_LES = 2 };

/* Lifting problem of the ALE displacement (Sec. 2.1.1, eq. (lifting)):
 * -div(alpha sigma_L(d)) = 0 on the reference mesh, d given on the vertices of
 * the ale_tags faces, zero traction elsewhere.  sigma_L = grad d (harmonic) or
 * E/(1+nu) sym grad d + E nu/((1+nu)(1-2nu)) div d I (linear elasticity,
 * moduli lift_E > 0, 0 <= lift_nu < 1/2).  Stiffening alpha, constant per
 * element: 1; (J0/J)^chi with J = |det| of the map from the unit simplex to
 * the element (stiff_p = {J0, chi}); or max(d, beta)^-gamma with d the distance
 * from the element's centroid to the ale_tags faces (stiff_p = {beta, gamma}). */
enum { LX_LIFT_HARMONIC = 0, LX_LIFT_ELASTIC = 1 };
enum { LX_STIFF_NONE = 0, LX_STIFF_JACOBIAN = 1, LX_STIFF_BOUNDARY = 2 };

/* The problem of Sec. 2.1-2.3: FE pair, BDF order (1..3) and time step (eq. (bdf)),
 * density and viscosity, diffusion form, stabilisation with constant C_r of
 * tau_M, semi-implicit advection (the only mode), ALE on/off with the boundary
 * displacement d^ = ale_law(t) * D^(x^) on the vertices of faces tagged ale_tags
 * (D^ set by lx_sim_set_ale_displacement) and its lifting, nodal forcing on/off. */
typedef struct {
    int32_t fe, bdf_order;
    double dt, t0, rho, mu;
    int32_t diffusion, stab;
    double C_r;
    int32_t semi_implicit;   /* 1: u* = u_EXT - u_ALE, semi-implicit LES term (one
                                linear solve per step); 0: the fully implicit
                                formulation (u* = u^{n+1} - u_ALE, implicit LES term,
                                Sec. 2.3) solved by Newton's method with the consistent
                                Jacobian (Sec. 2.4): P1-P1 (resistance and backflow
                                terms join the Jacobian as in the semi-implicit
                                system, the backflow coefficient at u_EXT);
                                lx_solver.max_ir caps the Newton updates and
                                ir_rtol is their tolerance (||R|| <= ir_rtol ||R_0||,
                                or an update below ir_rtol ||x||); rtol is each
                                update's linear tolerance.  LX_FP32_IR: the FP64
                                Jacobian and residual rounded, each update solved in
                                FP32 (to no tighter than inner_rtol)               */
    int32_t ale;             /* 0 | 1                                                */
    int32_t forcing;         /* 0: f = 0; 1: nodal f from lx_sim_set_forcing        */
    int32_t n_bc;
    const lx_boundary *bc;
    int32_t n_riis;
    int32_t n_ale_tags;
    const lx_riis *riis;
    const int32_t *ale_tags;
    lx_time_law ale_law;
    int32_t lifting;         /* LX_LIFT_*                                            */
    int32_t stiffening;      /* LX_STIFF_*                                           */
    double lift_E, lift_nu;  /* elasticity moduli (LX_LIFT_ELASTIC)                  */
    double stiff_p[2];       /* {J0, chi} or {beta, gamma}                           */
} lx_problem;

enum { LX_FP64 = 0, LX_FP32_IR = 1 };
enum { LX_PC_AMG = 0, LX_PC_CHEB_SCHUR = 1 };
/* Linear solver (Sec. 2.4): right-preconditioned (flexible) restarted
 * GMRES(restart) with the SIMPLE block preconditioner (D = diag(F), F~ = nodal
 * 3x3 diagonal blocks of F, S~ = C - B D^{-1} G); stop when
 * ||b - A x|| <= rtol ||b||.  The paper approximates the velocity and Schur
 * blocks of SIMPLE by AMG, additive Schwarz or block Jacobi; the two choices
 * here are
 *   LX_PC_AMG (default): S~ is formed explicitly and approximated by one
 *     multigrid cycle of aggregation AMG (amg_cycle coarse corrections on
 *     every level below the finest) with Chebyshev smoothing of degree
 *     amg_degree over [lam / amg_ratio, lam] on every level (lam the
 *     Gershgorin bound of diag(A_l)^{-1} A_l) and a dense coarsest solve; F is
 *     approximated by a Chebyshev iteration of degree f_degree on F~^{-1} F
 *     over [lam_F / f_ratio, lam_F] (lam_F from power iterations; f_degree 1
 *     is plain block Jacobi F~^{-1});
 *   LX_PC_CHEB_SCHUR: F by F~^{-1}; S~ (not formed) by diag(S~)^{-1}
 *     (schur_degree = 0) or a Chebyshev iteration of degree schur_degree with
 *     diagonal scaling over [lam / schur_ratio, lam].
 * A zero in f_degree, amg_degree, amg_cycle, f_ratio, amg_ratio or amg_coarse_cycle selects its
 * default (f_degree 3 for P1-P1 and 12 for P2-P1, amg_degree 2, amg_cycle 2,
 * f_ratio 5 for P1-P1 and 300 for P2-P1, amg_ratio 30, amg_coarse_cycle 3).  LX_FP32_IR: FP32 matrix and FP32 inner GMRES inside an
 * FP64 iterative refinement loop that stops when the FP64 residual satisfies
 * ir_rtol; inner solves aim at one more refinement step but never tighter
 * than inner_rtol. */
typedef struct {
    int32_t precision, restart, max_iters, max_ir;
    double rtol, ir_rtol, inner_rtol;
    int32_t deterministic;   /* reserved: the assembly gathers element records in
                                a fixed order (no atomics) and every reduction
                                has a fixed order already                          */
    int32_t collect_timing;  /* n >= 1: HIP events stamped by every n-th SpMV
                                launch of the solves (Arnoldi steps and cycle
                                starts alike; a timed Arnoldi step launches its
                                product outside the step's HIP graph) and around
                                every assembly and FP64 residual pass; 0: none  */
    int32_t schur_degree;    /* 0..32                                               */
    int32_t asm_fp64;        /* LX_FP32_IR only: 1 = build the FP32 matrix by FP64
                                element arithmetic and scatter, rounded to FP32;
                                0 = FP32 element arithmetic and FP32 scatter       */
    double schur_ratio;      /* > 1                                                  */
    int32_t precond;         /* LX_PC_AMG | LX_PC_CHEB_SCHUR                         */
    int32_t f_degree;        /* LX_PC_AMG: 0..16 (0: default, see above)             */
    int32_t amg_degree;      /* LX_PC_AMG: 0..8 (0: default 2)                       */
    int32_t amg_cycle;       /* LX_PC_AMG: coarse corrections per level below the
                                finest, 0..3 (0: default 2, a W-cycle there)        */
    double f_ratio;          /* LX_PC_AMG: 0 (default, see above) or > 1             */
    double amg_ratio;        /* LX_PC_AMG: 0 (default 30) or > 1                     */
    int32_t amg_coarse_cycle;   /* LX_PC_AMG: coarse corrections per level on the
                                   coarse levels that fit one workgroup's LDS, 0..6
                                   (0: default 3); amg_cycle applies above them      */
} lx_solver;

/* ---------------------------------------------------------------- outputs */

typedef struct {
    int64_t n_vertices, n_tets;
    int64_t n_u_nodes;       /* velocity nodes: n_vertices (P1-P1) or n_vertices +
                                n_edges (P2-P1)                                     */
    int64_t n_dofs;          /* 3 n_u_nodes + n_vertices                            */
    int64_t n_blocks;        /* stored block slots: vertex pairs of the 4x4 block
                                pattern (P1-P1) or F + G + B + C slots (P2-P1)      */
    int64_t device_bytes;    /* device memory held by the simulation              */
    int64_t n_edges;         /* P2-P1: edge nodes (0 for P1-P1)                     */
    int64_t n_scalar_nnz;    /* scalar entries of the stored matrix                 */
    int32_t amg_levels;      /* LX_PC_AMG: levels of the Schur-block hierarchy, the
                                dense coarsest included (0 for LX_PC_CHEB_SCHUR)    */
    int32_t amg_tail_level;  /* LX_PC_AMG: first level cycled by one workgroup out
                                of LDS, down to the dense level (0: none; the
                                environment variable LXNS_AMG_TAIL=0 turns it off) */
    int64_t amg_level_rows[8];   /* LX_PC_AMG: rows of levels 0..7 (0 past the last)   */
    int64_t amg_level_nnz[8];    /* LX_PC_AMG: stored entries of levels 0..7           */
} lx_sizes;

typedef struct {
    int32_t gmres_iters;      /* total (inner) GMRES iterations of the step           */
    int32_t ir_iters;         /* refinement iterations (0 for FP64)                   */
    int32_t restarts;
    int32_t converged;
    double rel_residual;      /* final true FP64 ||b - A x|| / ||b||                  */
    double t_step_ms;         /* wall time of the step on the stream (HIP events)     */
    double t_assembly_ms;     /* assembly + scatter + Dirichlet + SIMPLE setup        */
    double t_solve_ms;
    double spmv_ms;           /* summed time of the timed SpMV launches (collect_timing) */
    int64_t spmv_calls;
    double asm_ms;            /* assembly-kernel time (collect_timing >= 1)           */
    int64_t asm_calls;
    double resid_ms;          /* FP64 matrix-free residual kernel time                */
    int64_t resid_calls;
    int32_t newton_iters;     /* Newton updates of an implicit step (0 semi-implicit)  */
    int32_t lift_iters;       /* lifting CG iterations of the step (0 when the step
                                 solved no lifting problem)                       */
} lx_step_stats;

typedef struct lx_sim lx_sim;

/* Create a simulation: validates the mesh (LX_EMESH on a degenerate tet or an
 * id out of range), renumbers vertices (reverse Cuthill-McKee) and elements,
 * builds the shared block-CSR pattern, element->slot maps and boundary lists,
 * and uploads everything to the device.  History starts at rest (u = p = 0)
 * at time problem->t0. */
lx_status lx_sim_create(const lx_device *dev, const lx_mesh *mesh, const lx_problem *problem,
                        const lx_solver *solver, lx_sim **out);

lx_status lx_sim_query(const lx_sim *sim, lx_sizes *out);

/* P2-P1 velocity nodes: rows [0, n_vertices) of every velocity-node array are
 * the vertices (caller ids), rows n_vertices + k are the midpoints of the edges
 * listed here, edges [n_edges][2] as caller vertex ids (Sec. 2.3's quadratic
 * Lagrange element).  Nothing is written for P1-P1. */
lx_status lx_sim_get_edges(const lx_sim *sim, int32_t *edges);

/* Set history level `level` (0 = u^n, 1 = u^{n-1}, ...): u [n_u_nodes][3],
 * p [n_vertices], optional ALE displacement d [n_vertices][3] (NULL: 0).
 * The BDF order used at a step is min(bdf_order, levels set or computed). */
lx_status lx_sim_set_state(lx_sim *sim, int32_t level, const double *u, const double *p,
                           const double *d);
lx_status lx_sim_set_time(lx_sim *sim, double t);

/* Nodal data for a boundary condition with a nodal profile, at t^{n+1} of the
 * next step: Dirichlet values or Neumann traction vectors, [n_u_nodes][3]
 * (only the rows of that condition's nodes are read). */
lx_status lx_sim_set_dirichlet_values(lx_sim *sim, int32_t bc_index, const double *g);
lx_status lx_sim_set_neumann_traction(lx_sim *sim, int32_t bc_index, const double *h);
/* Forcing f at t^{n+1}, [n_u_nodes][3] (problem.forcing = 1). */
lx_status lx_sim_set_forcing(lx_sim *sim, const double *f);
/* ALE boundary-displacement shape D^ [n_vertices][3] (rows of ALE boundary
 * vertices are read); the displacement at t is ale_law(t) * D^ (Sec. 2.1.1). */
lx_status lx_sim_set_ale_displacement(lx_sim *sim, const double *d);
/* Boundary displacement d^ at t^{n+1} of the coming step, [n_vertices][3] (rows
 * of ALE boundary vertices are read; Sec. 2.1.1's data on the moving boundary).
 * From this call on, every step solves the lifting problem for the values last
 * set (CG on the reference-mesh lifting operator to a relative residual of 1e-13,
 * started from the extrapolation of the displacement history corrected by its
 * projection onto up to 8 earlier lifting solutions) instead of scaling the
 * extension of a shape; lx_sim_set_ale_displacement switches back. */
lx_status lx_sim_set_boundary_displacement(lx_sim *sim, const double *d);

/* Advance one time step (paper's fully discrete problem, Sec. 2.3): boundary
 * data at t^{n+1}, ALE lifting and mesh velocity, element assembly and
 * scatter, Dirichlet rows, SIMPLE setup, GMRES (or FP32 GMRES inside FP64
 * refinement), history rotation.  The solve starts from an extrapolation of
 * the last solutions to t^{n+1} (the BDF extrapolation weights, or the
 * quadratic or cubic through the last three or four solutions, whichever
 * predicted the previous step's solution best); the stopping test does not
 * depend on it.  Levels set by lx_sim_set_state count as history; older
 * computed levels are then dropped.  Transactional: on LX_ENOCONV the state
 * and time are left unchanged.  stats may be NULL. */
lx_status lx_sim_step(lx_sim *sim, lx_step_stats *stats);

/* Checkpoint and restore (stop-and-restart serialisation of Sec. 3.1).  The
 * state is everything the next step reads besides the mesh, problem and solver
 * given at creation: time and step counters, every stored solution level (the
 * BDF history and the levels the initial guess extrapolates from) and the
 * choice of extrapolation order, the ALE displacement history and lifting,
 * the nodal boundary data, forcing and displacement last set, and the warm
 * start of the preconditioner's power iterations.  lx_sim_state_size gives the
 * byte count; lx_sim_get_state writes an opaque blob of exactly that size into
 * caller memory (synchronising the stream); lx_sim_restore_state loads it into a
 * simulation created with the same mesh, problem and solver (LX_EINVAL on a size
 * or fingerprint mismatch, the simulation unchanged).  A restored simulation
 * continues bitwise as the saved one would have. */
lx_status lx_sim_state_size(const lx_sim *sim, int64_t *bytes);
lx_status lx_sim_get_state(const lx_sim *sim, void *blob, int64_t bytes);
lx_status lx_sim_restore_state(lx_sim *sim, const void *blob, int64_t bytes);

/* Copy the current solution to caller buffers: u [n_u_nodes][3], p
 * [n_vertices], t (any may be NULL).  Synchronises the stream. */
lx_status lx_sim_get_solution(const lx_sim *sim, double *u, double *p, double *t);

/* Parity export (tests only): assemble the system of the coming step without
 * solving and copy it out in the caller's numbering as block COO with 4x4
 * blocks (row-major within the block: rows u_x,u_y,u_z,p; cols likewise):
 * brow/bcol [n_blocks], vals [n_blocks][16], rhs [n_vertices][4].  Values are
 * FP64 (FP32 matrices are widened).  rhs is zero for FP32 precision.  With the
 * implicit formulation: the Newton system (Jacobian and -R, Dirichlet rows set
 * to the update g - x) at the last solution. */
lx_status lx_sim_debug_export(lx_sim *sim, int32_t *brow, int32_t *bcol, double *vals, double *rhs);

/* P2-P1 parity export (tests only): the system of the coming step as scalar
 * COO (n_scalar_nnz entries) in the caller's dof numbering -- velocity dof
 * 3 node + c over the velocity nodes, pressure dof 3 n_u_nodes + vertex -- and
 * rhs [n_dofs] in the same numbering; FP64 in both precisions. */
lx_status lx_sim_debug_export_p2(lx_sim *sim, int32_t *rows, int32_t *cols, double *vals, double *rhs);

/* FP64 matrix-free residual b - A x of the coming step at the caller's state
 * x = (u [n][3], p [n]), written to r [n_vertices][4] (tests only; P1-P1). */
lx_status lx_sim_debug_residual(lx_sim *sim, const double *u, const double *p, double *r);

/* Allocation-free variant of lx_sim_debug_residual, for callers that cannot
 * allocate device memory (code under stream or graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same FP64 matrix-free residual
 * b - A x of the coming step (P1-P1), with u [n_vertices][3], p [n_vertices] and
 * the output r [n_vertices][4] as DEVICE pointers on the simulation's device in
 * the caller's numbering.  The work is queued on the simulation's stream (the
 * call returns without waiting, except that an ALE lifting solve waits for its
 * own convergence checks); read r after synchronising that stream.  The iterate,
 * residual, right-hand side and element contributions live in a fixed 64 MiB
 * device array that the library holds on every device it runs on until the
 * process ends: meshes needing more (96 n_vertices + 384 n_tets bytes; about
 * 160k tets) are rejected with LX_EINVAL.  All calls on one device share that
 * array, which keeps the last call's contents: calls that overlap on one device
 * (other streams, other threads) race and must be serialised by the caller.
 * Nothing is allocated: no hipMalloc, hipFree or caller allocator call. */
lx_status lx_sim_residual_noalloc(lx_sim *sim, const double *u, const double *p, double *r);

/* Flow rate and pressure over the faces of condition `bc` (any type; Sec. 4's
 * section diagnostics), on the configuration and with the solution of the
 * last step: out[0] = int (u - u_ALE) . n (the flux through the moving
 * surface; normals oriented along the condition's profile.normal, or as the
 * faces are listed where that is zero), out[1] = int p, out[2] = area (the
 * mean pressure is out[1] / out[2]).  P1-P1; host array of 3; synchronises
 * the simulation's stream.  LX_EINVAL for a bad index or a P2-P1 problem. */
lx_status lx_sim_boundary_integrals(lx_sim *sim, int32_t bc, double *out);

void lx_sim_destroy(lx_sim *sim);

/* ---------------------------------------------------------------- serving */

/* A continuous-batching server: requests (mesh + problem + solver + step
 * count) are admitted in arrival order while the device-memory budget and the
 * active-slot limit allow, set up by a pool of host threads on streams of their
 * own, then stepped by one persistent worker thread per stream (each worker
 * steps its simulations in turn, one time step each, so that the device work of
 * the streams overlaps), and retired by their worker when done; new requests
 * are admitted as memory and slots free up.  Every simulation's arithmetic is
 * independent of what else runs (fixed-order reductions), so a served result
 * is bitwise the one the same request gives alone.  The server's simulations
 * allocate with hipMalloc (cfg.device.alloc / free must be NULL). */
typedef struct {
    lx_device device;
    int64_t hbm_budget_bytes;   /* admission limit on summed simulation footprints */
    int32_t max_active;         /* slot limit                                        */
    int32_t n_streams;          /* streams the active simulations are spread over    */
} lx_server_cfg;

typedef struct {
    lx_mesh mesh;
    lx_problem problem;
    lx_solver solver;
    int32_t n_steps;
    int32_t pad;
} lx_request;

/* QUEUED: waiting for admission; SETUP: admitted (memory reserved), being set up;
 * RUNNING: stepping; DONE / FAILED: final, until lx_server_result releases it. */
enum { LX_REQ_QUEUED = 0, LX_REQ_RUNNING = 1, LX_REQ_DONE = 2, LX_REQ_FAILED = 3, LX_REQ_SETUP = 4 };
typedef struct {
    int32_t state;
    int32_t steps_done;
    int64_t footprint_bytes;
} lx_request_status;

typedef struct {
    double admit_wait_ms;       /* submission to admission                          */
    double setup_ms;            /* admission to the first step's eligibility (set-up) */
    double total_ms;            /* submission to completion                         */
    double step_p50_ms, step_p99_ms;  /* per step: eligible -> completed            */
    int32_t n_steps;
    int32_t gmres_iters;
} lx_latency_stats;

typedef struct lx_server lx_server;

lx_status lx_server_create(const lx_server_cfg *cfg, lx_server **out);
/* Copies the request's arrays; returns a ticket.  LX_EBUSY if the request's
 * footprint estimate alone exceeds the budget; LX_EINVAL for a P2-P1 problem
 * (the server runs P1-P1).  Admission reserves the estimate; once the
 * simulation exists its measured footprint replaces it, and if that breaks the
 * budget the simulation is released and the request queued again at the front
 * with the measured figure (FAILED if that alone exceeds the budget).  All
 * lx_server_* calls are thread-safe and return LX_ENOMEM / LX_EDEVICE on a host
 * exception instead of throwing. */
lx_status lx_server_submit(lx_server *srv, const lx_request *req, int64_t *ticket);
/* The first tick starts the server's streams and threads.  A tick admits what
 * fits, then waits until a step, set-up or retirement completes (at most 20 ms;
 * with nothing admitted it returns at once) and admits again.  Stepping does not
 * wait for ticks.  *n_active gets the admitted count (set-up + running). */
lx_status lx_server_tick(lx_server *srv, int32_t *n_active);
lx_status lx_server_poll(lx_server *srv, int64_t ticket, lx_request_status *st);
/* Copy a finished request's solution (u [n][3], p [n], caller numbering) and
 * latency statistics, then release it.  LX_ESTATE if not done. */
lx_status lx_server_result(lx_server *srv, int64_t ticket, double *u, double *p,
                           lx_latency_stats *lat);
void lx_server_destroy(lx_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* LXNS_H */
