// Continuous-batching server for many simulations on one device.
//
// Requests queue in arrival order.  Admission (first come, first served: a
// request that does not fit blocks the ones behind it) reserves a request's
// device-footprint estimate and a slot and hands it to a pool of set-up
// threads, which create the simulation on a private stream of their own, so
// the host set-up (renumbering, patterns, aggregation) never holds up the
// stepping.  Each of the server's streams has one persistent worker thread that
// steps its simulations in turn, one time step each, for as long as they have
// steps left; the device work of different streams overlaps.  A worker retires
// a finished simulation itself (solution copied back, memory freed) and admits
// what the freed memory lets in.  lx_server_tick does the admission on the
// caller's thread and then waits for the next completed step or set-up.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "lx_sim.h"

using lx::fail;
using Clock = std::chrono::steady_clock;

namespace {

// internal request state: set-up in progress (reported through the ABI as its own state)
constexpr int32_t kReqSetup = LX_REQ_SETUP;

struct Request {
    // deep copies of the caller's request
    std::vector<double> coords;
    std::vector<int32_t> tets, bfaces, btags;
    std::vector<lx_boundary> bc;
    std::vector<std::vector<int32_t>> bc_tags;
    std::vector<lx_riis> riis;
    std::vector<int32_t> ale_tags;
    lx_problem problem{};
    lx_solver solver{};
    int32_t n_steps = 0;
    int64_t ticket = 0;
    // runtime (guarded by the server's mutex, except sim, which only the thread
    // that currently owns the request touches: a set-up thread, then the worker)
    int32_t state = LX_REQ_QUEUED;
    int32_t steps_done = 0;
    int64_t footprint = 0;     // estimate until set-up, then what the simulation allocated
    bool measured = false;     // footprint is the measured one
    int worker = 0;
    int64_t load = 0;          // unknowns charged to the worker
    lx_sim *sim = nullptr;
    Clock::time_point t_submit, t_admit, t_ready, t_eligible, t_done;
    std::vector<double> step_ms;
    int32_t gmres_iters = 0;
    std::vector<double> u, p;
    std::string error;

    lx_mesh mesh() const
    {
        lx_mesh m;
        m.n_vertices = (int64_t)coords.size() / 3;
        m.n_tets = (int64_t)tets.size() / 4;
        m.n_bfaces = (int64_t)btags.size();
        m.coords = coords.data();
        m.tets = tets.data();
        m.bfaces = bfaces.data();
        m.bface_tag = btags.data();
        return m;
    }
};

// Device-memory estimate of a simulation before it is created: block count from
// the edge count of a tetrahedral mesh (about 1.3 edges per tet), 16 block planes,
// pattern and slot maps, Krylov basis and work vectors.  Meant as an upper bound;
// a simulation that allocates more is checked again once it exists.
int64_t estimate_footprint(const Request &r)
{
    const int64_t nv = (int64_t)r.coords.size() / 3, nt = (int64_t)r.tets.size() / 4;
    const int64_t nblk = nv + (int64_t)(2.6 * (double)nt);
    const int64_t s = (r.solver.precision == LX_FP64) ? 8 : 4;
    const int64_t N = 4 * nv;
    const int64_t L = std::max<int64_t>(r.problem.bdf_order, 4);
    int64_t b = 0;
    b += nblk * (16 * s + 8);                 // planes + col + tslot
    b += nt * (16 + 64) + 4 * nblk;           // connectivity + slot incidence
    b += nt * 16 + 4 * (nv + 1);              // vertex incidence of the residual pass
    b += nt * lx::kRec * ((r.solver.precision == LX_FP64 || r.solver.asm_fp64) ? 8 : 4);   // element records
    b += nv * (48 + 16 + 12 * s + 4);         // coords, rowptr/diag/dir index, SIMPLE blocks
    b += N * 8 * (L + 2);                     // history levels (at least four: the guess
                                              // extrapolates), solution, right-hand side
    b += N * s * (2 * r.solver.restart + 3);  // basis, preconditioned directions, work
    if (r.solver.precond == LX_PC_AMG)
        // S~ on the vertex 2-ring (about 4x the block count) with its coarsening
        // lists and formation tables, level vectors, velocity-block Chebyshev
        // work, coarse levels and the tabulated coarse operator
        // (the finest level also in sliced-ELL order: about 10% padding)
        b += 4 * nblk * (s + s / 4 + 18) + nv * (22 * s + 24) + (5 << 20);
    else
        b += nv * s * 9;                      // Schur Chebyshev work
    if (r.solver.precision != LX_FP64) b += N * (8 * 2 + 4 * 2) + nt * lx::kRRec * 8;
    if (r.problem.ale)   // lifting: stiffness as assembled and eliminated (9 planes when elastic), CG work
        b += nv * 8 * 3 * (12 + lx::kProjMax) + nblk * 16 * (r.problem.lifting == LX_LIFT_ELASTIC ? 9 : 1) +
             (r.problem.lifting == LX_LIFT_ELASTIC ? nv * 72 : 0);
    return b + (1 << 20);
}

// Host threads that set up admitted simulations concurrently.
constexpr int kSetupThreads = 8;

}  // namespace

struct lx_server {
    lx_server_cfg cfg{};
    double est_scale = 1.0;                // LXNS_SERVER_EST_SCALE: scales the estimates
                                           // (tests of the post-set-up budget check)
    std::mutex mu;
    std::condition_variable cv_progress;   // a step, set-up or retirement completed
    std::condition_variable cv_setup;      // work for the set-up threads
    std::vector<std::unique_ptr<std::condition_variable>> cv_worker;
    std::map<int64_t, std::unique_ptr<Request>> reqs;
    std::deque<int64_t> queue;             // waiting for admission
    std::deque<Request *> setup_q;         // admitted, waiting for a set-up thread
    std::vector<std::deque<Request *>> runq;   // per worker: simulations with steps left
    std::vector<int64_t> load;             // per worker: unknowns of its simulations
    int n_admitted = 0;                    // in set-up or stepping
    int64_t next_ticket = 1;
    int64_t used_bytes = 0;
    int64_t progress = 0;
    bool stop = false;
    bool started = false;
    std::vector<hipStream_t> streams, setup_streams;
    std::vector<std::thread> threads;
};

static double ms_between(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::milli>(b - a).count();
}

// Admit queued requests while a slot is free and the reservation fits (mu held).
static void admit_locked(lx_server *srv)
{
    while (!srv->queue.empty() && srv->n_admitted < srv->cfg.max_active) {
        Request &r = *srv->reqs[srv->queue.front()];
        if (srv->used_bytes + r.footprint > srv->cfg.hbm_budget_bytes) break;
        srv->queue.pop_front();
        srv->used_bytes += r.footprint;
        srv->n_admitted++;
        r.state = kReqSetup;
        r.t_admit = Clock::now();
        srv->setup_q.push_back(&r);
        srv->cv_setup.notify_one();
    }
}

// A request leaves the device: solution copied back (ok), simulation destroyed.
// Called by the thread that owns the request, without mu.
static void finish(Request &r, bool ok)
{
    if (r.sim) {
        if (ok) {
            const int64_t nv = r.sim->nv;
            r.u.resize(3 * nv);
            r.p.resize(nv);
            if (lx_sim_get_solution(r.sim, r.u.data(), r.p.data(), nullptr) != LX_OK) r.error = lx_last_error();
        }
        lx_sim_destroy(r.sim);
        r.sim = nullptr;
    }
}

// Book a finished request (mu held): memory and slot released, state final.
static void retire_locked(lx_server *srv, Request &r, bool ok)
{
    srv->used_bytes -= r.footprint;
    srv->n_admitted--;
    srv->load[r.worker] -= r.load;
    r.load = 0;
    r.state = (ok && r.error.empty()) ? LX_REQ_DONE : LX_REQ_FAILED;
    r.t_done = Clock::now();
    srv->progress++;
    admit_locked(srv);
    srv->cv_progress.notify_all();
}

static void setup_thread(lx_server *srv, int k)
{
    (void)hipSetDevice(srv->cfg.device.device);
    std::unique_lock<std::mutex> lk(srv->mu);
    for (;;) {
        srv->cv_setup.wait(lk, [&] { return srv->stop || !srv->setup_q.empty(); });
        if (srv->stop) return;
        Request &r = *srv->setup_q.front();
        srv->setup_q.pop_front();
        lk.unlock();
        // set-up on this thread's own stream, then the simulation moves to its worker's
        // stream; the set-up ends with its stream drained, so nothing of it is in flight
        lx_device dev{srv->cfg.device.device, (void *)srv->setup_streams[k], nullptr, nullptr, nullptr};
        lx_mesh m = r.mesh();
        lx_status st = LX_OK;
        try {
            st = lx_sim_create(&dev, &m, &r.problem, &r.solver, &r.sim);
            if (st != LX_OK) r.error = lx_last_error();
            else if (hipStreamSynchronize(srv->setup_streams[k]) != hipSuccess) {
                st = LX_EDEVICE;
                r.error = "set-up stream synchronisation failed";
            }
        } catch (const std::exception &e) {
            st = LX_ENOMEM;
            r.error = std::string("set-up failed: ") + e.what();
        }
        if (st != LX_OK && r.sim) {
            lx_sim_destroy(r.sim);
            r.sim = nullptr;
        }
        const int64_t real = st == LX_OK ? r.sim->device_bytes : 0;
        lk.lock();
        if (st != LX_OK) {
            retire_locked(srv, r, false);
            continue;
        }
        // the reservation was an estimate: if what the simulation holds breaks the
        // budget, release it and queue the request again at the front, with the
        // measured footprint (alone over the budget: it fails)
        if (srv->used_bytes - r.footprint + real > srv->cfg.hbm_budget_bytes) {
            lk.unlock();
            lx_sim_destroy(r.sim);
            r.sim = nullptr;
            lk.lock();
            srv->used_bytes -= r.footprint;
            srv->n_admitted--;
            r.footprint = real;
            r.measured = true;
            if (real > srv->cfg.hbm_budget_bytes) {
                r.state = LX_REQ_FAILED;
                r.error = "measured footprint " + std::to_string(real) + " exceeds the budget";
                r.t_done = Clock::now();
            } else {
                r.state = LX_REQ_QUEUED;
                srv->queue.push_front(r.ticket);
            }
            srv->progress++;
            admit_locked(srv);
            srv->cv_progress.notify_all();
            continue;
        }
        srv->used_bytes += real - r.footprint;
        r.footprint = real;
        r.measured = true;
        r.t_ready = r.t_eligible = Clock::now();
        // the worker whose simulations hold the fewest unknowns takes it
        int w = 0;
        for (int i = 1; i < (int)srv->runq.size(); ++i)
            if (srv->load[i] < srv->load[w]) w = i;
        r.worker = w;
        r.load = 4 * (int64_t)(r.coords.size() / 3);
        srv->load[w] += r.load;
        r.sim->stream = srv->streams[w];
        r.state = LX_REQ_RUNNING;
        srv->progress++;
        if (r.n_steps == 0) {
            lk.unlock();
            finish(r, true);
            lk.lock();
            retire_locked(srv, r, true);
            continue;
        }
        srv->runq[w].push_back(&r);
        srv->cv_worker[w]->notify_one();
        srv->cv_progress.notify_all();
    }
}

// One worker per stream: steps its simulations in turn, one step each.
static void worker_thread(lx_server *srv, int w)
{
    (void)hipSetDevice(srv->cfg.device.device);
    std::unique_lock<std::mutex> lk(srv->mu);
    for (;;) {
        srv->cv_worker[w]->wait(lk, [&] { return srv->stop || !srv->runq[w].empty(); });
        if (srv->stop) return;
        Request &r = *srv->runq[w].front();
        srv->runq[w].pop_front();
        lk.unlock();
        lx_step_stats stt{};
        lx_status st;
        std::string err;
        try {
            st = lx_sim_step(r.sim, &stt);
            if (st != LX_OK) err = lx_last_error();
        } catch (const std::exception &e) {
            st = LX_ENOMEM;
            err = std::string("step failed: ") + e.what();
        }
        const Clock::time_point now = Clock::now();
        const bool last = st != LX_OK || r.steps_done + 1 >= r.n_steps;
        if (st != LX_OK) r.error = err;
        if (last) finish(r, st == LX_OK);
        lk.lock();
        r.step_ms.push_back(ms_between(r.t_eligible, now));
        r.gmres_iters += stt.gmres_iters;
        if (st == LX_OK) r.steps_done++;
        if (last) {
            retire_locked(srv, r, st == LX_OK);
            continue;
        }
        r.t_eligible = now;
        srv->runq[w].push_back(&r);
        srv->progress++;
        srv->cv_progress.notify_all();
    }
}

// Streams and threads start with the first tick, so that queueing and admission
// decisions can be exercised without touching the device.
static lx_status ensure_started(lx_server *srv)
{
    if (srv->started) return LX_OK;
    const int ns = std::max(1, srv->cfg.n_streams);
    if (hipSetDevice(srv->cfg.device.device) != hipSuccess) return fail(LX_EDEVICE, "hipSetDevice failed");
    for (int i = 0; i < ns + kSetupThreads; ++i) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
            return fail(LX_EDEVICE, "hipStreamCreate failed");
        (i < ns ? srv->streams : srv->setup_streams).push_back(st);
    }
    srv->runq.assign(ns, {});
    srv->load.assign(ns, 0);
    for (int i = 0; i < ns; ++i) srv->cv_worker.emplace_back(new std::condition_variable());
    srv->started = true;
    for (int i = 0; i < ns; ++i) srv->threads.emplace_back(worker_thread, srv, i);
    for (int k = 0; k < kSetupThreads; ++k) srv->threads.emplace_back(setup_thread, srv, k);
    return LX_OK;
}

extern "C" lx_status lx_server_create(const lx_server_cfg *cfg, lx_server **out)
{
    if (!cfg || !out) return fail(LX_EINVAL, "NULL argument");
    if (cfg->max_active < 1 || cfg->hbm_budget_bytes <= 0) return fail(LX_EINVAL, "bad server limits");
    if (cfg->device.alloc || cfg->device.free)
        return fail(LX_EINVAL, "the server allocates with hipMalloc: lx_device.alloc/free must be NULL");
    auto *s = new (std::nothrow) lx_server();
    if (!s) return fail(LX_ENOMEM, "host allocation failed");
    s->cfg = *cfg;
    if (const char *e = getenv("LXNS_SERVER_EST_SCALE")) {
        const double v = atof(e);
        if (v > 0) s->est_scale = v;
    }
    *out = s;
    return LX_OK;
}

extern "C" lx_status lx_server_submit(lx_server *srv, const lx_request *req, int64_t *ticket)
{
    if (!srv || !req || !ticket) return fail(LX_EINVAL, "NULL argument");
    const lx_mesh &m = req->mesh;
    if (m.n_vertices <= 0 || m.n_tets <= 0 || !m.coords || !m.tets) return fail(LX_EINVAL, "empty mesh");
    if (req->n_steps < 0) return fail(LX_EINVAL, "n_steps < 0");
    if (req->problem.fe != LX_P1P1) return fail(LX_EINVAL, "the server runs P1-P1 requests");
    try {
        auto r = std::make_unique<Request>();
        r->coords.assign(m.coords, m.coords + 3 * m.n_vertices);
        r->tets.assign(m.tets, m.tets + 4 * m.n_tets);
        if (m.n_bfaces > 0) {
            r->bfaces.assign(m.bfaces, m.bfaces + 3 * m.n_bfaces);
            r->btags.assign(m.bface_tag, m.bface_tag + m.n_bfaces);
        }
        r->problem = req->problem;
        r->bc.assign(req->problem.bc, req->problem.bc + req->problem.n_bc);
        for (auto &b : r->bc) r->bc_tags.emplace_back(b.tags, b.tags + b.n_tags);
        for (size_t i = 0; i < r->bc.size(); ++i) r->bc[i].tags = r->bc_tags[i].data();
        r->problem.bc = r->bc.data();
        r->riis.assign(req->problem.riis, req->problem.riis + req->problem.n_riis);
        r->problem.riis = r->riis.data();
        if (req->problem.ale && req->problem.n_ale_tags > 0)
            r->ale_tags.assign(req->problem.ale_tags, req->problem.ale_tags + req->problem.n_ale_tags);
        r->problem.ale_tags = r->ale_tags.data();
        r->solver = req->solver;
        r->n_steps = req->n_steps;
        r->footprint = (int64_t)(srv->est_scale * (double)estimate_footprint(*r));
        if (r->footprint > srv->cfg.hbm_budget_bytes)
            return fail(LX_EBUSY, "request footprint %lld exceeds the budget %lld", (long long)r->footprint,
                        (long long)srv->cfg.hbm_budget_bytes);
        r->t_submit = Clock::now();
        std::lock_guard<std::mutex> lk(srv->mu);
        r->ticket = *ticket = srv->next_ticket++;
        srv->queue.push_back(*ticket);
        srv->reqs[*ticket] = std::move(r);
        return LX_OK;
    } catch (const std::exception &e) {
        return fail(LX_ENOMEM, "submit: %s", e.what());
    }
}

extern "C" lx_status lx_server_tick(lx_server *srv, int32_t *n_active)
{
    if (!srv) return fail(LX_EINVAL, "server is NULL");
    try {
        std::unique_lock<std::mutex> lk(srv->mu);
        lx_status es = ensure_started(srv);
        if (es != LX_OK) return es;
        admit_locked(srv);
        // wait for the next completed step, set-up or retirement (none outstanding:
        // return at once; a bounded wait, so that the caller can submit meanwhile)
        const int64_t seen = srv->progress;
        if (srv->n_admitted > 0)
            srv->cv_progress.wait_for(lk, std::chrono::milliseconds(20),
                                      [&] { return srv->progress != seen || srv->n_admitted == 0; });
        admit_locked(srv);
        if (n_active) *n_active = srv->n_admitted;
        return LX_OK;
    } catch (const std::exception &e) {
        return fail(LX_EDEVICE, "tick: %s", e.what());
    }
}

extern "C" lx_status lx_server_poll(lx_server *srv, int64_t ticket, lx_request_status *st)
{
    if (!srv || !st) return fail(LX_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return fail(LX_EINVAL, "unknown ticket %lld", (long long)ticket);
    st->state = it->second->state;
    st->steps_done = it->second->steps_done;
    st->footprint_bytes = it->second->footprint;
    return LX_OK;
}

static double percentile(std::vector<double> v, double q)
{
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (double)(v.size() - 1);
    const size_t lo = (size_t)std::floor(pos), hi = std::min(lo + 1, v.size() - 1);
    return v[lo] + (pos - (double)lo) * (v[hi] - v[lo]);
}

extern "C" lx_status lx_server_result(lx_server *srv, int64_t ticket, double *u, double *p, lx_latency_stats *lat)
{
    if (!srv) return fail(LX_EINVAL, "server is NULL");
    try {
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->reqs.find(ticket);
        if (it == srv->reqs.end()) return fail(LX_EINVAL, "unknown ticket %lld", (long long)ticket);
        Request &r = *it->second;
        if (r.state == LX_REQ_FAILED) {
            lx_status s = fail(LX_ENOCONV, "request failed: %s", r.error.c_str());
            srv->reqs.erase(it);
            return s;
        }
        if (r.state != LX_REQ_DONE) return fail(LX_ESTATE, "request %lld is not finished", (long long)ticket);
        if (u) std::memcpy(u, r.u.data(), sizeof(double) * r.u.size());
        if (p) std::memcpy(p, r.p.data(), sizeof(double) * r.p.size());
        if (lat) {
            lat->admit_wait_ms = ms_between(r.t_submit, r.t_admit);
            lat->setup_ms = ms_between(r.t_admit, r.t_ready);
            lat->total_ms = ms_between(r.t_submit, r.t_done);
            lat->step_p50_ms = percentile(r.step_ms, 0.50);
            lat->step_p99_ms = percentile(r.step_ms, 0.99);
            lat->n_steps = r.steps_done;
            lat->gmres_iters = r.gmres_iters;
        }
        srv->reqs.erase(it);
        return LX_OK;
    } catch (const std::exception &e) {
        return fail(LX_ENOMEM, "result: %s", e.what());
    }
}

extern "C" void lx_server_destroy(lx_server *srv)
{
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        srv->cv_setup.notify_all();
        for (auto &cv : srv->cv_worker) cv->notify_all();
    }
    // every thread finishes the step or set-up it is in and leaves
    for (auto &t : srv->threads) t.join();
    for (auto &kv : srv->reqs)
        if (kv.second->sim) lx_sim_destroy(kv.second->sim);
    for (auto v : {&srv->streams, &srv->setup_streams})
        for (auto st : *v) {
            (void)hipStreamSynchronize(st);
            (void)hipStreamDestroy(st);
        }
    delete srv;
}
