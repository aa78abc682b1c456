// The simulation object behind lx_sim*.
#pragma once

#include <utility>
#include <vector>

#include "lx_amg.h"
#include "lx_common.h"
#include "lx_kernels.h"
#include "lx_newton.h"
#include "lx_outflow.h"
#include "lx_p2.h"

namespace lx {

double law_value(const lx_time_law &L, double t);

struct BCDesc {
    lx_boundary spec{};
    std::vector<int32_t> tags;
    int64_t nf = 0;                 // Neumann faces
    std::vector<int32_t> h_faces;   // [nf][3] new numbering (P2-P1: [nf][6] with the edge nodes)
    int32_t *d_faces = nullptr;
    double *d_hnodal = nullptr;     // [nu][3] nodal traction (nodal profile)
    bool nodal_set = false;
};

struct GmResult {
    int iters = 0;
    int restarts = 0;
    bool converged = false;
    double resid = 0;
    double bnorm = 0;
};

struct Sim {
    int device = -1;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    HostSetup hs;
    lx_problem prob{};
    lx_solver solver{};
    std::vector<BCDesc> bcs;
    std::vector<lx_riis> valves;
    std::vector<int32_t> ale_tags;
    std::vector<int32_t> h_ale_nodes;
    int64_t nv = 0, nt = 0, nblk = 0, N = 0, n_dir = 0;
    // P2-P1: velocity nodes (vertices, then edges); nu = nv for P1-P1
    bool p2 = false;
    int64_t nu = 0;
    P2Setup p2h;
    int32_t *d_nodes = nullptr, *d_fptr = nullptr, *d_fcol = nullptr, *d_fdiag = nullptr, *d_gptr = nullptr,
            *d_gcol = nullptr, *d_bptr = nullptr, *d_bcol = nullptr, *d_finc_ptr = nullptr, *d_finc = nullptr,
            *d_ginc_ptr = nullptr, *d_ginc = nullptr, *d_binc_ptr = nullptr, *d_binc = nullptr;
    double *d_xnode = nullptr;      // [nu][3]
    P2Rules *d_rules = nullptr;
    double *d_rec2 = nullptr;       // [nt][kP2Rec] element records
    P2Sys<double> s64{};            // FP64 split system (both precisions for P2-P1)
    P2Sys<float> s32{};             // FP32 copy (FP32 + refinement)
    // caller row of internal node i (vertices are renumbered, edge nodes keep the library order)
    int64_t caller_node(int64_t i) const { return i < nv ? (int64_t)hs.perm_v[i] : i; }
    std::vector<int32_t> h_dir_index, h_dir_node, h_dir_bc;
    std::vector<double> h_gnodal;
    bool dirty_gnodal = false;
    // outflow conditions with a resistance or backflow term (P1-P1), and the
    // device result of lx_sim_boundary_integrals
    std::vector<OutflowDev> outflow;
    double *d_bint = nullptr;

    // device arrays (new numbering)
    double *d_xh = nullptr, *d_x = nullptr;
    int32_t *d_sinc_ptr = nullptr, *d_sinc = nullptr;             // slot incidence of the assembly gather
    int32_t *d_vinc_ptr = nullptr, *d_vpos = nullptr;             // vertex incidence of the residual pass
    double *d_rec64 = nullptr;                                    // element records (FP64 assembly)
    float *d_rec32 = nullptr;                                     // element records (FP32 assembly)
    int32_t *d_tet = nullptr, *d_rowptr = nullptr, *d_col = nullptr, *d_diag = nullptr,
            *d_tslot = nullptr;
    int32_t *d_dir_index = nullptr, *d_dir_node = nullptr, *d_dir_bc = nullptr;
    int32_t *d_perm = nullptr;                                    // [nv] caller id of internal vertex i
    double *d_g = nullptr, *d_gnodal = nullptr, *d_dg = nullptr;
    double *d_hist[4] = {nullptr, nullptr, nullptr, nullptr};   // [nv][4] u^n, u^{n-1}, ...
    double *d_xs = nullptr;                                      // solution of the step in progress
    double *d_f = nullptr, *d_uA = nullptr;
    // ALE
    double *d_dhist[4] = {nullptr, nullptr, nullptr, nullptr};  // [nv][3] displacement history
    double *d_dnew = nullptr;                                    // displacement at t^{n+1}
    double *d_ale_shape = nullptr;                               // [nv][3] D^
    // lifting stiffness on x^: [nblk] scalars (harmonic) or [9][nblk] 3x3 blocks (elasticity),
    // as assembled (full) and with the boundary rows and columns eliminated; its (block) Jacobi
    // inverse [nv] or [nv][9]
    bool lift_vec = false;
    double *d_lap = nullptr;
    double *d_lapfull = nullptr;
    double *d_lapdinv = nullptr;
    std::vector<int32_t> h_ale_faces;                            // [n][3] faces with the ALE tags
    int32_t *d_ale_nodes = nullptr;
    int32_t *d_ale_mark = nullptr;                               // [nv] 1 on ALE boundary
    double *d_cg = nullptr;                                      // CG work: 6 vectors [nv][3] + state
    double *d_cg_partial = nullptr;
    bool ale_ext_valid = false;
    double *d_dbnd = nullptr;                                    // [nv][3] nodal boundary displacement at t^{n+1}
    bool ale_nodal = false;                                      // lifting of d_dbnd solved every step
    int ale_iters = 0;                                           // CG iterations of the step's lifting solves
    bool lift_solved = false;                                    // the step solved the lifting for nodal data
    // projection of the lifting's initial guess onto earlier solutions (nodal data)
    double *d_projQ = nullptr;                                   // [kProjMax][nv][3], K-orthonormal
    double *d_proj_coef = nullptr;                               // [2 kProjMax]
    int32_t proj_n = 0;                                          // vectors in use
    bool lift_proj = true;                                       // LXNS_LIFT_PROJ=0: off
    // FP64 system
    double *d_val64 = nullptr, *d_rhs64 = nullptr, *d_Finv64 = nullptr, *d_Dinv64 = nullptr, *d_Sinv64 = nullptr;
    double *d_V64 = nullptr, *d_w64 = nullptr, *d_sw64 = nullptr, *d_Z64 = nullptr;
    // FP32 system + refinement
    float *d_val32 = nullptr, *d_Finv32 = nullptr, *d_Dinv32 = nullptr, *d_Sinv32 = nullptr;
    float *d_V32 = nullptr, *d_w32 = nullptr, *d_x32 = nullptr, *d_r32 = nullptr, *d_sw32 = nullptr,
          *d_Z32 = nullptr;
    double *d_r64 = nullptr, *d_b64 = nullptr;
    double *d_rrec = nullptr;                                    // element records of the FP64 residual
    // implicit formulation: element Newton records [nt][kNewtonRec], the update, its Dirichlet values
    double *d_nrec = nullptr, *d_dx = nullptr, *d_gdelta = nullptr;
    // SIMPLE block approximations of LX_PC_AMG (one of the two, by precision)
    AmgHost amgh;
    Amg<double> amg64;
    Amg<float> amg32;
    // reductions
    GmState *d_st = nullptr;
    GmState *h_st = nullptr;
    double *d_partial = nullptr;
    int nb_red = 1;

    std::vector<void *> allocs;
    int64_t device_bytes = 0;

    // timing
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
    std::vector<std::pair<int, int>> ev_tag;
    size_t ev_used = 0;
    int64_t spmv_seq = 0;   // SpMV launches of the solves so far (every collect_timing-th one is timed)
    hipEvent_t ev_step0 = nullptr, ev_step1 = nullptr, ev_asm1 = nullptr;
    // P1-P1 FP32 + refinement on meshes of 2^19 tets and more: a second stream on which the FP64
    // residual of the initial guess runs while the FP32 system is assembled
    hipStream_t stream_aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // the norms of b and of the guess's residual, formed on the second stream behind the
    // residual (partial sums of their own) and copied to pinned memory, so that the host
    // has them while the set-up still runs on the first
    double *d_partial_aux = nullptr, *h_norms0 = nullptr;
    // convergence checks inside an Arnoldi cycle: the scalar part of the state (done
    // flag, columns used, residual estimate) copied to pinned host memory behind an
    // event, one check in flight (ping-pong slots)
    GmState *h_chk = nullptr;
    double *h_gerr = nullptr;  // pinned: errors of the guess orders on the last step
    double *d_gerr = nullptr;  // their partial sums, then the three sums
    int x_order = 4;           // extrapolation order of the next guess (2: BDF weights, 3, 4)
    hipEvent_t ev_chk[2] = {nullptr, nullptr};
    // HIP graphs of the Arnoldi steps: step k's preconditioner apply, product and
    // Gram-Schmidt pass, one graph per (k, whether the step ends the cycle),
    // captured on a private stream the first time it is needed and replayed on
    // every later solve (their launches take fixed buffers); LXNS_GRAPH=0 launches
    // the kernels one by one instead.  Steps whose product is timed replay the
    // apply (slot 2 kMaxRestart + k) and the Gram-Schmidt pass (4 kMaxRestart + key)
    // as graphs of their own and launch the product between them
    bool use_graphs = true;
    hipStream_t cap_stream = nullptr;
    std::vector<hipGraph_t> g_step;
    std::vector<hipGraphExec_t> gx_step;   // [6 kMaxRestart]
    // columns used by cycle c of the last solve of each kind (0: unknown), where
    // the next solve of that kind starts checking every step
    int32_t k_hint[8][8] = {};

    // caller allocator for device memory (lx_device.alloc / free); NULL: hipMalloc / hipFree
    void *(*alloc_fn)(size_t, void *) = nullptr;
    void (*free_fn)(void *, void *) = nullptr;
    void *alloc_ctx = nullptr;

    double t = 0;
    int nlev = 0;
    int nhist = 0;   // valid solution levels in d_hist (up to max(bdf_order, 4); the guess may use four)
    int64_t step_index = 0;

    ~Sim();
    lx_status dalloc(void **p, size_t bytes);
    lx_status create(const lx_device *dev, const lx_mesh *mesh, const lx_problem *pr, const lx_solver *sv);
    RowPattern pattern() const;
    const double *hist(int l) const { return (l < prob.bdf_order && d_hist[l]) ? d_hist[l] : d_hist[0]; }

    std::pair<hipEvent_t, hipEvent_t> *timer_begin(int kind, int iter, bool record = true);
    void timer_end(std::pair<hipEvent_t, hipEvent_t> *p);
    void timer_flush(int kused, lx_step_stats &acc);
    lx_status read_state();

    template <typename T>
    lx_status setup_amg(Amg<T> &A);
    template <typename T>
    SimpleView<T> view();
    template <typename T>
    void spmv(const T *x, T *y, const int32_t *done, std::pair<hipEvent_t, hipEvent_t> *tm,
              hipStream_t s = nullptr);
    template <typename T>
    lx_status gmres(const T *b, T *x, bool x_zero, double rtol, int max_iters, GmResult &res,
                    lx_step_stats &tstats, bool inner = false, int kind = 0);
    void coefficients(double t1, StepCoef &C, BCSet &B) const;
    lx_status prepare(double t1, StepCoef &C);
    lx_status newton(double t1, const StepCoef &C, lx_step_stats &S);
    void newton_system(double t1, const StepCoef &C);
    lx_status build_system(double t1, StepCoef &C, lx_step_stats &tstats);
    lx_status assemble_system(double t1, StepCoef &C, bool fork_residual = false);
    lx_status build_system_p2(double t1, StepCoef &C);
    void add_neumann(double t1, double *out0, double *out1);
    lx_status outflow_setup();
    double outflow_p0(const OutflowDev &o, double t1) const;
    lx_status residual64(const StepCoef &C, const double *xs, bool first, double t1);
    lx_status residual64_into(const StepCoef &C, const double *xs, bool first, double t1, double *rec, double *r,
                              double *b, bool timed);
    lx_status step(lx_step_stats *out);

    // checkpoint of everything the next step reads besides mesh, problem and solver
    int64_t state_bytes() const;
    lx_status save_state(void *blob, int64_t bytes);
    lx_status load_state(const void *blob, int64_t bytes);

    lx_status ale_setup();
    lx_status ale_boundary_distance(std::vector<double> &dist);
    lx_status ale_extend(const double *data);
    lx_status ale_update(double t1, const StepCoef &C);
    void ale_commit();
    void ale_add_solution();
};

}  // namespace lx

namespace lx {
// Resolves, once per device (that device current), the device address of the
// allocation-free entry point's static scratch array.
lx_status noalloc_init(int device);
}  // namespace lx

struct lx_sim : public lx::Sim {};
