// Serving loop with continuous batching.
//
// Host threads share the device.  Submitted requests wait in FIFO order.  A pool of set-up
// threads classifies the geometry of the first waiting requests (host work, in parallel:
// that sizes each request's device footprint before any device allocation), admits the
// front request when a slot is free and its footprint fits in the remaining memory budget
// (admission stays FIFO), reserves both, and builds the request's context -- point sets,
// LGF table, boundary data through the caller's callback -- on the context's own stream,
// while the running batch keeps the device busy.  With one set-up thread the host geometry
// of the larger grids limited admission to about 12 requests a second, with most slots idle.
// The scheduler thread owns one batch engine: at each step boundary
// it takes the requests whose set-up has finished into the batch; every step advances all
// running requests by a few GMRES iterations with one launch per phase, so new work
// overlaps with work already on the GPU.  A finished request (FP64 GMRES, or the FP32 inner
// solve of a refinement step followed by its FP64 residual) leaves the batch, its result is
// copied to the host and its memory and slot are released for the requests still waiting.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "batch.hpp"

namespace bae {
namespace {

enum { Q_WAITING = 0, Q_RUNNING = 1, Q_DONE = 2, Q_FAILED = 3 };

struct Req {
    uint64_t ticket = 0;
    bae_grid grid{};
    bae_levelset ls{};
    std::vector<double> phi;
    bae_boundary_fn g = nullptr;
    void* user = nullptr;
    int state = Q_WAITING;
    int status = BAE_OK;
    std::string error;
    std::unique_ptr<Geometry> geo;
    bool sizing = false, sized = false;   // geometry being classified / classified
    int64_t bytes = 0;
    bae_ctx* ctx = nullptr;
    double bnorm = 0.0, relres = 1.0;
    int iters = 0, outer = 0;
    int64_t mv64 = 0, mv32 = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    std::vector<double> q, ug;
    bool fetched = false;
};

using clock_t_ = std::chrono::steady_clock;

}  // namespace
}  // namespace bae

using namespace bae;

struct bae_server {
    bae_server_options opt{};
    BatchEngine* engine = nullptr;
    std::thread thread;
    std::vector<std::thread> setup_threads;
    std::mutex mu;
    std::condition_variable cv_work, cv_setup, cv_done;
    bool stop = false;
    uint64_t next_ticket = 1;
    std::deque<std::shared_ptr<Req>> waiting;
    int in_setup = 0;                                  // admitted, context being built
    std::vector<std::shared_ptr<Req>> ready;           // set up, joining at the next step
    std::vector<std::shared_ptr<Req>> running;
    std::map<uint64_t, std::shared_ptr<Req>> all;
    int64_t used = 0;
    bae_server_stats stats{};
    clock_t_::time_point t0;
    double now() const { return std::chrono::duration<double>(clock_t_::now() - t0).count(); }
};

namespace bae {
namespace {

void fail(bae_server* s, const std::shared_ptr<Req>& r, int status, const std::string& msg) {
    r->state = Q_FAILED;
    r->status = status;
    r->error = msg;
    r->t_done = s->now();
    s->stats.failed++;
}

// Waiting requests whose geometry the set-up threads classify ahead of admission.
constexpr int kSizeAhead = 16;

// A set-up thread: admits the front request when it is classified and a slot and its memory
// are free (both reserved at admission) and builds its context, then hands it to the
// scheduler; otherwise classifies the geometry of one of the first waiting requests.  Every
// failure fails that request only.
void setup_loop(bae_server* s) {
    (void)hipSetDevice(s->opt.device);
    bae_options o{};
    o.device = s->opt.device;
    o.max_rhs = 1;
    o.max_krylov = s->opt.max_krylov;
    for (;;) {
        std::shared_ptr<Req> r, sz;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            auto slot_free = [&] {
                return (int)(s->running.size() + s->ready.size()) + s->in_setup < s->opt.max_slots;
            };
            auto admissible = [&] {
                if (s->waiting.empty()) return false;
                const auto& f = s->waiting.front();
                return f->sized && slot_free() && s->used + f->bytes <= s->opt.hbm_budget;
            };
            auto to_size = [&]() -> std::shared_ptr<Req> {
                int k = 0;
                for (const auto& w : s->waiting) {
                    if (k++ >= kSizeAhead) break;
                    if (!w->sized && !w->sizing) return w;
                }
                return nullptr;
            };
            s->cv_setup.wait(lk, [&] { return s->stop || admissible() || to_size() != nullptr; });
            if (s->stop) return;
            if (admissible()) {
                r = s->waiting.front();
                s->waiting.pop_front();
                s->used += r->bytes;
                s->in_setup++;
                s->stats.admitted++;
                s->stats.peak_bytes = std::max<int64_t>(s->stats.peak_bytes, s->used);
                r->state = Q_RUNNING;
                r->t_admit = s->now();
            } else {
                sz = to_size();
                sz->sizing = true;
            }
        }
        std::string fail_msg;
        int fail_code = BAE_OK;
        if (sz) {
            // the geometry (host) gives the exact footprint before any device allocation
            auto geo = std::make_unique<Geometry>();
            int64_t bytes = 0;
            try {
                bae_levelset ls = sz->ls;
                if (ls.kind == BAE_LS_SAMPLED) ls.phi_samples = sz->phi.data();
                build_geometry(sz->grid, ls, *geo);
                bytes = estimate_context_bytes(*geo, sz->grid.sigma * sz->grid.h * sz->grid.h, &o);
            } catch (const Error& e) {
                fail_code = e.code;
                fail_msg = e.msg;
            } catch (const std::exception& e) {
                fail_code = BAE_ERR_ARG;
                fail_msg = std::string("geometry: ") + e.what();
            }
            std::lock_guard<std::mutex> lk(s->mu);
            sz->sizing = false;
            if (fail_code == BAE_OK && bytes > s->opt.hbm_budget) {
                fail_code = BAE_ERR_ADMISSION;
                fail_msg = "request needs more device memory than the whole budget";
            }
            const auto it = std::find(s->waiting.begin(), s->waiting.end(), sz);
            if (it == s->waiting.end()) continue;   // failed meanwhile (server shut down)
            if (fail_code != BAE_OK) {
                s->waiting.erase(it);
                fail(s, sz, fail_code, fail_msg);
                s->cv_done.notify_all();
            } else {
                sz->geo = std::move(geo);
                sz->bytes = bytes;
                sz->sized = true;
            }
            s->cv_setup.notify_all();
            continue;
        }
        try {
            r->ctx = create_context(r->grid, &o, std::move(*r->geo));
            r->geo.reset();
            const int64_t n = r->ctx->ngm;
            std::vector<double> gx(n);
            r->g(r->user, n, r->ctx->geo.xstar.data(), gx.data());
            if (int rc = bae_set_rhs(r->ctx, 1, gx.data(), nullptr); rc != BAE_OK) throw Error{rc, bae_last_error()};
        } catch (const Error& e) {
            fail_code = e.code;
            fail_msg = e.msg;
        } catch (const std::bad_alloc&) {
            fail_code = BAE_ERR_OOM;
            fail_msg = "host allocation failed during set-up";
        } catch (const std::exception& e) {
            fail_code = BAE_ERR_ARG;
            fail_msg = std::string("set-up: ") + e.what();
        }
        if (fail_code != BAE_OK && r->ctx) {
            bae_destroy(r->ctx);
            r->ctx = nullptr;
        }
        std::lock_guard<std::mutex> lk(s->mu);
        s->in_setup--;
        if (fail_code != BAE_OK) {
            s->used -= r->bytes;
            fail(s, r, fail_code, fail_msg);
            s->cv_done.notify_all();
            s->cv_setup.notify_all();
            continue;
        }
        s->ready.push_back(r);
        s->cv_work.notify_all();
    }
}

void scheduler(bae_server* s) {
    (void)hipSetDevice(s->opt.device);
    const bool refined = s->opt.precision == BAE_SOLVE_FP32_REFINED;
    const int prec = refined ? BAE_PREC_FP32 : BAE_PREC_FP64;
    const double floor_tol = 1e-6;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait_for(lk, std::chrono::milliseconds(20), [&] {
                return (s->stop && s->in_setup == 0) || !s->ready.empty() || !s->running.empty();
            });
            if (s->stop && s->running.empty() && s->ready.empty() && s->in_setup == 0) return;
        }
        std::vector<std::shared_ptr<Req>> fresh, run;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            fresh.swap(s->ready);
            s->running.insert(s->running.end(), fresh.begin(), fresh.end());
            run = s->running;
            s->stats.max_active = std::max<int64_t>(s->stats.max_active, (int64_t)run.size());
        }
        if (run.empty()) continue;
        try {
            if (!fresh.empty()) {
                std::vector<bae_ctx*> members;
                for (auto& r : run) members.push_back(r->ctx);
                batch_set_members(s->engine, members);
                const int np = (int)run.size();
                std::vector<int32_t> mask(np, 0);
                for (int p = 0; p < np; ++p) mask[p] = std::find(fresh.begin(), fresh.end(), run[p]) != fresh.end();
                const std::vector<double> bn = batch_bnorms(s->engine);
                for (int p = 0; p < np; ++p)
                    if (mask[p]) run[p]->bnorm = bn[p];
                batch_vec(s->engine, 1, mask);              // x = 0
                if (refined) batch_vec(s->engine, 2, mask);  // r = b
                std::vector<double> tol(np, s->opt.tol);
                if (refined)
                    for (int p = 0; p < np; ++p) tol[p] = std::min(0.1, std::max(floor_tol, 0.5 * s->opt.tol));
                batch_begin(s->engine, mask, refined ? 1 : 0, tol, std::vector<int>(np, s->opt.maxit));
            }
            batch_iterate(s->engine, prec, s->opt.iters_per_step, false);
            s->stats.steps++;
            const std::vector<int32_t> done = batch_done(s->engine);
            const int np = (int)run.size();
            std::vector<int32_t> fin(np, 0);
            bool any = false;
            for (int p = 0; p < np; ++p) {
                fin[p] = done[p] != 0;
                any |= fin[p] != 0;
            }
            if (!any) continue;
            batch_finish(s->engine, fin, refined);
            const std::vector<int32_t> kd = batch_kdone(s->engine);
            const std::vector<double> rn = batch_residual_norms(s->engine, &fin);
            std::vector<int32_t> complete(np, 0), again(np, 0);
            std::vector<double> tol(np, s->opt.tol);
            for (int p = 0; p < np; ++p) {
                if (!fin[p]) continue;
                Req& r = *run[p];
                r.iters += kd[p];
                (refined ? r.mv32 : r.mv64) += kd[p];
                r.mv64 += 1;
                r.relres = r.bnorm > 0 ? rn[p] / r.bnorm : 0.0;
                if (refined) r.outer++;
                if (refined && r.relres > s->opt.tol && r.outer < 8 && r.iters < 4 * s->opt.maxit) {
                    again[p] = 1;
                    tol[p] = std::min(0.1, std::max(floor_tol, 0.5 * s->opt.tol / r.relres));
                } else {
                    complete[p] = 1;
                }
            }
            if (std::any_of(again.begin(), again.end(), [](int32_t v) { return v != 0; }))
                batch_begin(s->engine, again, 1, tol, std::vector<int>(np, s->opt.maxit));
            if (!std::any_of(complete.begin(), complete.end(), [](int32_t v) { return v != 0; })) continue;
            batch_gamma_values(s->engine, &complete);
            std::vector<std::shared_ptr<Req>> keep;
            for (int p = 0; p < np; ++p) {
                auto& r = run[p];
                if (!complete[p]) {
                    keep.push_back(r);
                    continue;
                }
                bae_ctx* c = r->ctx;
                r->q.resize(c->ngm);
                r->ug.resize(c->nT);
                BAE_HIP_CHECK(hipMemcpy(r->q.data(), c->x.p, sizeof(double) * c->ngm, hipMemcpyDeviceToHost));
                BAE_HIP_CHECK(hipMemcpy(r->ug.data(), c->u_gamma.p, sizeof(double) * c->nT, hipMemcpyDeviceToHost));
                r->ctx = nullptr;
                bae_destroy(c);
                std::lock_guard<std::mutex> lk(s->mu);
                r->state = Q_DONE;
                r->status = r->relres <= s->opt.tol ? BAE_OK : BAE_NOT_CONVERGED;
                r->t_done = s->now();
                s->used -= r->bytes;
                s->stats.completed++;
            }
            s->cv_setup.notify_all();   // slots and memory were released
            std::vector<bae_ctx*> members;
            for (auto& r : keep) members.push_back(r->ctx);
            batch_set_members(s->engine, members);
            {
                std::lock_guard<std::mutex> lk(s->mu);
                s->running = keep;
            }
            s->cv_done.notify_all();
        } catch (const Error& e) {
            // a device error ends every running request; the server keeps serving new ones
            std::lock_guard<std::mutex> lk(s->mu);
            for (auto& r : s->running) {
                if (r->ctx) bae_destroy(r->ctx);
                r->ctx = nullptr;
                s->used -= r->bytes;
                fail(s, r, e.code, e.msg);
            }
            s->running.clear();
            s->cv_done.notify_all();
            s->cv_setup.notify_all();
        }
    }
}

}  // namespace
}  // namespace bae

extern "C" {

int bae_server_create(const bae_server_options* opt, bae_server** out) {
    return guard([&] {
        if (!opt || !out) throw Error{BAE_ERR_ARG, "null argument"};
        if (opt->max_slots < 1 || opt->hbm_budget <= 0) throw Error{BAE_ERR_ARG, "max_slots and hbm_budget must be > 0"};
        if (opt->precision != BAE_SOLVE_FP64 && opt->precision != BAE_SOLVE_FP32_REFINED)
            throw Error{BAE_ERR_ARG, "unknown precision"};
        *out = nullptr;
        auto s = std::make_unique<bae_server>();
        s->opt = *opt;
        if (s->opt.tol <= 0) s->opt.tol = 1e-10;
        if (s->opt.max_krylov <= 0) s->opt.max_krylov = 200;
        if (s->opt.maxit <= 0 || s->opt.maxit > s->opt.max_krylov) s->opt.maxit = s->opt.max_krylov;
        if (s->opt.iters_per_step <= 0) s->opt.iters_per_step = 4;
        if (s->opt.setup_threads <= 0) s->opt.setup_threads = 4;
        s->opt.setup_threads = std::min(s->opt.setup_threads, 16);
        BAE_HIP_CHECK(hipSetDevice(s->opt.device));
        s->engine = batch_engine_new(s->opt.device, nullptr);
        s->t0 = clock_t_::now();
        s->thread = std::thread(scheduler, s.get());
        for (int k = 0; k < s->opt.setup_threads; ++k) s->setup_threads.emplace_back(setup_loop, s.get());
        *out = s.release();
    });
}

int bae_server_submit(bae_server* s, const bae_request* req, uint64_t* ticket) {
    return guard([&] {
        if (!s || !req || !ticket || !req->g) throw Error{BAE_ERR_ARG, "null argument"};
        auto r = std::make_shared<Req>();
        r->grid = req->grid;
        r->ls = req->levelset;
        if (r->ls.kind == BAE_LS_SAMPLED) {
            if (!r->ls.phi_samples) throw Error{BAE_ERR_ARG, "sampled level set without samples"};
            const int64_t n3 = (int64_t)r->grid.n[0] * r->grid.n[1] * r->grid.n[2];
            r->phi.assign(r->ls.phi_samples, r->ls.phi_samples + n3);
        }
        r->ls.phi_samples = nullptr;
        r->g = req->g;
        r->user = req->user;
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) throw Error{BAE_ERR_STATE, "server is shutting down"};
        r->ticket = s->next_ticket++;
        r->t_submit = s->now();
        s->waiting.push_back(r);
        s->all[r->ticket] = r;
        s->stats.submitted++;
        *ticket = r->ticket;
        s->cv_setup.notify_all();
    });
}

int bae_server_wait(bae_server* s, uint64_t ticket, double timeout_s, bae_result* res, bae_request_info* info) {
    int status = BAE_OK;
    int rc = guard([&] {
        if (!s) throw Error{BAE_ERR_ARG, "null server"};
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->all.find(ticket);
        if (it == s->all.end()) throw Error{BAE_ERR_ARG, "unknown ticket"};
        auto r = it->second;
        auto ready = [&] { return r->state == Q_DONE || r->state == Q_FAILED; };
        if (timeout_s < 0) s->cv_done.wait(lk, ready);
        else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready))
            throw Error{BAE_ERR_STATE, "timed out"};
        if (r->state == Q_FAILED) throw Error{r->status, r->error};
        status = r->status;
        if (res) {
            res->status = r->status;
            res->iterations = r->iters;
            res->outer_steps = r->outer;
            res->converged = r->status == BAE_OK;
            res->rel_residual_est = 0.0;
            res->rel_residual_true = r->relres;
            res->seconds = r->t_done - r->t_submit;
            res->matvecs_fp64 = r->mv64;
            res->matvecs_fp32 = r->mv32;
        }
        if (info) {
            info->state = r->state;
            info->n_gamma_minus = (int64_t)r->q.size();
            info->n_targets = (int64_t)r->ug.size();
            info->bytes = r->bytes;
            info->t_submit = r->t_submit;
            info->t_admit = r->t_admit;
            info->t_done = r->t_done;
        }
    });
    return rc != BAE_OK ? rc : status;
}

int bae_server_poll(bae_server* s, uint64_t ticket, int32_t* state) {
    return guard([&] {
        if (!s || !state) throw Error{BAE_ERR_ARG, "null argument"};
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->all.find(ticket);
        if (it == s->all.end()) throw Error{BAE_ERR_ARG, "unknown ticket"};
        *state = it->second->state;
    });
}

int bae_server_fetch(bae_server* s, uint64_t ticket, double* q, int64_t q_cap, double* u_gamma, int64_t u_cap) {
    return guard([&] {
        if (!s) throw Error{BAE_ERR_ARG, "null server"};
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->all.find(ticket);
        if (it == s->all.end()) throw Error{BAE_ERR_ARG, "unknown ticket"};
        auto r = it->second;
        if (r->state != Q_DONE) throw Error{BAE_ERR_STATE, "request not done"};
        if ((q && q_cap < (int64_t)r->q.size()) || (u_gamma && u_cap < (int64_t)r->ug.size()))
            throw Error{BAE_ERR_ARG, "output buffer too small"};
        if (q) std::copy(r->q.begin(), r->q.end(), q);
        if (u_gamma) std::copy(r->ug.begin(), r->ug.end(), u_gamma);
        s->all.erase(it);
    });
}

int bae_server_stats_get(bae_server* s, bae_server_stats* out) {
    return guard([&] {
        if (!s || !out) throw Error{BAE_ERR_ARG, "null argument"};
        std::lock_guard<std::mutex> lk(s->mu);
        *out = s->stats;
        out->bytes_in_use = s->used;
        out->waiting = (int64_t)s->waiting.size();
        out->running = (int64_t)s->running.size();
    });
}

int bae_server_destroy(bae_server* s) {
    if (!s) return BAE_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        // requests that never started are failed; running ones finish
        for (auto& r : s->waiting) fail(s, r, BAE_ERR_STATE, "server shut down");
        s->waiting.clear();
        s->cv_work.notify_all();
        s->cv_setup.notify_all();
        s->cv_done.notify_all();
    }
    for (auto& t : s->setup_threads)   // set-ups in progress finish first
        if (t.joinable()) t.join();
    if (s->thread.joinable()) s->thread.join();
    (void)hipSetDevice(s->opt.device);
    batch_engine_delete(s->engine);
    delete s;
    return BAE_OK;
}

}  // extern "C"
