// Continuous-batching server for many simulations on one device.
//
// Requests queue in arrival order.  Every tick admits queued requests while
// the summed device footprint stays under the budget and a slot is free (first
// come, first served: a request that does not fit blocks the ones behind it;
// the admitted ones are set up concurrently),
// advances every active simulation by one time step -- each simulation on one
// of a pool of HIP streams, driven by its own host thread so that the device
// work of different simulations overlaps -- and retires finished requests,
// freeing their memory and slot for the next tick.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "lx_sim.h"

using lx::fail;
using Clock = std::chrono::steady_clock;

namespace {

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
    // runtime
    int32_t state = LX_REQ_QUEUED;
    int32_t steps_done = 0;
    int64_t footprint = 0;
    int stream_index = 0;
    lx_sim *sim = nullptr;
    Clock::time_point t_submit, t_admit, t_done;
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
// pattern and slot maps, Krylov basis and work vectors.
int64_t estimate_footprint(const Request &r)
{
    const int64_t nv = (int64_t)r.coords.size() / 3, nt = (int64_t)r.tets.size() / 4;
    const int64_t nblk = nv + (int64_t)(2.6 * (double)nt);
    const int64_t s = (r.solver.precision == LX_FP64) ? 8 : 4;
    const int64_t N = 4 * nv;
    int64_t b = 0;
    b += nblk * (16 * s + 8);                 // planes + col + tslot
    b += nt * (16 + 64) + 4 * nblk;           // connectivity + slot incidence
    b += nt * 16 + 4 * (nv + 1);              // vertex incidence of the residual pass
    b += nt * lx::kRec * ((r.solver.precision == LX_FP64 || r.solver.asm_fp64) ? 8 : 4);   // element records
    b += nv * (48 + 16 + 12 * s + 4);         // coords, rowptr/diag/dir index, SIMPLE blocks
    b += N * 8 * (r.problem.bdf_order + 2);   // history + solution (FP64)
    b += N * s * (2 * r.solver.restart + 3);  // basis, preconditioned directions, work
    if (r.solver.precond == LX_PC_AMG)
        // S~ on the vertex 2-ring (about 4x the block count) with its coarsening
        // lists, level vectors, velocity-block Chebyshev work, coarse levels
        // (the finest level also in sliced-ELL order: about 10% padding)
        b += 4 * nblk * (s + s / 4 + 14) + nv * (22 * s + 24) + (3 << 20);
    else
        b += nv * s * 9;                      // Schur Chebyshev work
    if (r.solver.precision != LX_FP64) b += N * (8 * 2 + 4 * 2) + nt * lx::kRRec * 8;
    if (r.problem.ale) b += nv * 8 * 3 * 12 + nblk * 16;
    return b + (1 << 20);
}

// Host threads that create admitted simulations concurrently.
constexpr int kCreateThreads = 8;

}  // namespace

struct lx_server {
    lx_server_cfg cfg{};
    std::vector<hipStream_t> streams;
    std::map<int64_t, std::unique_ptr<Request>> reqs;
    std::deque<int64_t> queue;
    std::vector<int64_t> active;
    int64_t next_ticket = 1;
    int64_t used_bytes = 0;
    int next_stream = 0;
};

extern "C" lx_status lx_server_create(const lx_server_cfg *cfg, lx_server **out)
{
    if (!cfg || !out) return fail(LX_EINVAL, "NULL argument");
    if (cfg->max_active < 1 || cfg->hbm_budget_bytes <= 0) return fail(LX_EINVAL, "bad server limits");
    auto *s = new (std::nothrow) lx_server();
    if (!s) return fail(LX_ENOMEM, "host allocation failed");
    s->cfg = *cfg;
    *out = s;
    return LX_OK;
}

// Streams are created on the first tick, so that queueing and admission
// decisions can be exercised without touching the device.
static lx_status ensure_streams(lx_server *s)
{
    if (!s->streams.empty()) return LX_OK;
    const int ns = std::max(1, s->cfg.n_streams);
    if (hipSetDevice(s->cfg.device.device) != hipSuccess) return fail(LX_EDEVICE, "hipSetDevice failed");
    for (int i = 0; i < ns; ++i) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
            return fail(LX_EDEVICE, "hipStreamCreate failed");
        s->streams.push_back(st);
    }
    return LX_OK;
}

extern "C" lx_status lx_server_submit(lx_server *srv, const lx_request *req, int64_t *ticket)
{
    if (!srv || !req || !ticket) return fail(LX_EINVAL, "NULL argument");
    const lx_mesh &m = req->mesh;
    if (m.n_vertices <= 0 || m.n_tets <= 0 || !m.coords || !m.tets) return fail(LX_EINVAL, "empty mesh");
    if (req->n_steps < 0) return fail(LX_EINVAL, "n_steps < 0");
    if (req->problem.fe != LX_P1P1) return fail(LX_EINVAL, "the server runs P1-P1 requests");
    auto r = std::make_unique<Request>();
    r->coords.assign(m.coords, m.coords + 3 * m.n_vertices);
    r->tets.assign(m.tets, m.tets + 4 * m.n_tets);
    if (m.n_bfaces > 0) {
        r->bfaces.assign(m.bfaces, m.bfaces + 3 * m.n_bfaces);
        r->btags.assign(m.bface_tag, m.bface_tag + m.n_bfaces);
    }
    r->problem = req->problem;
    r->bc.assign(req->problem.bc, req->problem.bc + req->problem.n_bc);
    for (auto &b : r->bc) {
        r->bc_tags.emplace_back(b.tags, b.tags + b.n_tags);
    }
    for (size_t i = 0; i < r->bc.size(); ++i) r->bc[i].tags = r->bc_tags[i].data();
    r->problem.bc = r->bc.data();
    r->riis.assign(req->problem.riis, req->problem.riis + req->problem.n_riis);
    r->problem.riis = r->riis.data();
    if (req->problem.ale && req->problem.n_ale_tags > 0)
        r->ale_tags.assign(req->problem.ale_tags, req->problem.ale_tags + req->problem.n_ale_tags);
    r->problem.ale_tags = r->ale_tags.data();
    r->solver = req->solver;
    r->n_steps = req->n_steps;
    r->footprint = estimate_footprint(*r);
    if (r->footprint > srv->cfg.hbm_budget_bytes)
        return fail(LX_EBUSY, "request footprint %lld exceeds the budget %lld", (long long)r->footprint,
                    (long long)srv->cfg.hbm_budget_bytes);
    r->t_submit = Clock::now();
    *ticket = srv->next_ticket++;
    srv->queue.push_back(*ticket);
    srv->reqs[*ticket] = std::move(r);
    return LX_OK;
}

static void retire(lx_server *srv, Request &r, bool ok)
{
    if (r.sim) {
        if (ok) {
            const int64_t nv = r.sim->nv;
            r.u.resize(3 * nv);
            r.p.resize(nv);
            if (lx_sim_get_solution(r.sim, r.u.data(), r.p.data(), nullptr) != LX_OK) {
                ok = false;
                r.error = lx_last_error();
            }
        }
        lx_sim_destroy(r.sim);
        r.sim = nullptr;
    }
    srv->used_bytes -= r.footprint;
    r.state = ok ? LX_REQ_DONE : LX_REQ_FAILED;
    r.t_done = Clock::now();
}

extern "C" lx_status lx_server_tick(lx_server *srv, int32_t *n_active)
{
    if (!srv) return fail(LX_EINVAL, "server is NULL");
    lx_status es = ensure_streams(srv);
    if (es != LX_OK) return es;
    // 1. admission, first come first served, by the footprint estimates; the
    // admitted simulations are then created concurrently (their host set-up
    // dominates) and charged their real footprint afterwards
    std::vector<int64_t> admit;
    int64_t planned = srv->used_bytes;
    while (!srv->queue.empty() && (int)(srv->active.size() + admit.size()) < srv->cfg.max_active) {
        Request &r = *srv->reqs[srv->queue.front()];
        if (planned + r.footprint > srv->cfg.hbm_budget_bytes) break;
        planned += r.footprint;
        admit.push_back(srv->queue.front());
        srv->queue.pop_front();
    }
    if (!admit.empty()) {
        std::vector<lx_status> cst(admit.size(), LX_OK);
        std::vector<std::string> cerr(admit.size());
        for (size_t i = 0; i < admit.size(); ++i) {
            Request &r = *srv->reqs[admit[i]];
            r.stream_index = srv->next_stream++ % (int)srv->streams.size();
            srv->used_bytes += r.footprint;
        }
        std::atomic<size_t> next{0};
        auto work = [&]() {
            (void)hipSetDevice(srv->cfg.device.device);
            for (size_t i; (i = next.fetch_add(1)) < admit.size();) {
                Request &r = *srv->reqs[admit[i]];
                lx_device dev{srv->cfg.device.device, (void *)srv->streams[r.stream_index]};
                lx_mesh m = r.mesh();
                cst[i] = lx_sim_create(&dev, &m, &r.problem, &r.solver, &r.sim);
                if (cst[i] != LX_OK) cerr[i] = lx_last_error();
                r.t_admit = Clock::now();
            }
        };
        const size_t nw = std::min(admit.size(), (size_t)kCreateThreads);
        std::vector<std::thread> pool;
        for (size_t w = 1; w < nw; ++w) pool.emplace_back(work);
        work();
        for (auto &t : pool) t.join();
        for (size_t i = 0; i < admit.size(); ++i) {
            Request &r = *srv->reqs[admit[i]];
            if (cst[i] != LX_OK) {
                r.error = cerr[i];
                retire(srv, r, false);
                continue;
            }
            // account the real footprint from now on
            srv->used_bytes += r.sim->device_bytes - r.footprint;
            r.footprint = r.sim->device_bytes;
            r.state = LX_REQ_RUNNING;
            if (r.n_steps == 0) {
                retire(srv, r, true);
                continue;
            }
            srv->active.push_back(admit[i]);
        }
    }
    // 2. one step of every active simulation, concurrently
    const Clock::time_point eligible = Clock::now();
    std::vector<std::thread> th;
    std::vector<lx_status> res(srv->active.size(), LX_OK);
    std::vector<std::string> errs(srv->active.size());
    for (size_t i = 0; i < srv->active.size(); ++i) {
        Request *r = srv->reqs[srv->active[i]].get();
        th.emplace_back([r, i, &res, &errs, eligible, srv]() {
            (void)hipSetDevice(srv->cfg.device.device);
            lx_step_stats stt;
            res[i] = lx_sim_step(r->sim, &stt);
            if (res[i] != LX_OK) errs[i] = lx_last_error();
            r->step_ms.push_back(std::chrono::duration<double, std::milli>(Clock::now() - eligible).count());
            r->gmres_iters += stt.gmres_iters;
        });
    }
    for (auto &t : th) t.join();
    // 3. retirement
    std::vector<int64_t> still;
    for (size_t i = 0; i < srv->active.size(); ++i) {
        Request &r = *srv->reqs[srv->active[i]];
        if (res[i] != LX_OK) {
            r.error = errs[i];
            retire(srv, r, false);
            continue;
        }
        r.steps_done++;
        if (r.steps_done >= r.n_steps) retire(srv, r, true);
        else still.push_back(srv->active[i]);
    }
    srv->active.swap(still);
    if (n_active) *n_active = (int32_t)srv->active.size();
    return LX_OK;
}

extern "C" lx_status lx_server_poll(lx_server *srv, int64_t ticket, lx_request_status *st)
{
    if (!srv || !st) return fail(LX_EINVAL, "NULL argument");
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
        lat->admit_wait_ms = std::chrono::duration<double, std::milli>(r.t_admit - r.t_submit).count();
        lat->total_ms = std::chrono::duration<double, std::milli>(r.t_done - r.t_submit).count();
        lat->step_p50_ms = percentile(r.step_ms, 0.50);
        lat->step_p99_ms = percentile(r.step_ms, 0.99);
        lat->n_steps = r.steps_done;
        lat->gmres_iters = r.gmres_iters;
    }
    srv->reqs.erase(it);
    return LX_OK;
}

extern "C" void lx_server_destroy(lx_server *srv)
{
    if (!srv) return;
    for (auto &kv : srv->reqs)
        if (kv.second->sim) lx_sim_destroy(kv.second->sim);
    for (auto st : srv->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    delete srv;
}
