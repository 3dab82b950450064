// Continuous-batching server: a worker thread admits queued solves while
// their device footprint fits the budget and a slot is free, keeps their
// state resident on the device, advances all active solves together in
// batched ticks (one persistent launch per step per precision group), and
// completes each ticket when its solve has done its steps.  A helper thread
// does the host work of admitting (create, upload, initialise) and of
// completing (read back) while the ticks run.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "lbm3d_batch.h"

namespace {

using Clock = std::chrono::steady_clock;

// ticks a membership must last before its steps are captured as a graph
constexpr int64_t GRAPH_AFTER_TICKS = 8;

struct Ticket {
    uint64_t id = 0;
    lbm3d_params p{};
    std::vector<double> in[5];
    std::vector<double> out[5];
    int64_t nsteps = 0, left = 0;
    size_t footprint = 0;
    lbm3d_solver* h = nullptr;
    enum { QUEUED, ACTIVE, DONE } state = QUEUED;
    bool cancel = false;
    bool waited = false;  // a thread waits on it (a second waiter gets E_STATE)
    int32_t status = LBM3D_OK;
    uint32_t health = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
};

}  // namespace

struct lbm3d_server {
    size_t budget = 0;
    int max_active = 1;
    int64_t tick_steps = 32;
    int device = 0;
    Clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done, cv_help;
    std::deque<Ticket*> queue;
    std::vector<Ticket*> active;
    std::unordered_map<uint64_t, std::unique_ptr<Ticket>> tickets;
    size_t used = 0;
    uint64_t next_id = 1;
    bool stop = false;
    bool membership_changed = true;
    std::thread worker;
    // The helper thread creates and initialises admitted solves and reads
    // back finished ones (on the side stream), so that the worker, which
    // runs the ticks, never holds up the next tick with that host work.
    struct Task {
        Ticket* t;
        int32_t status;
        bool admit;  // admit (create and initialise) or finish (read back)
    };
    std::thread helper;
    std::deque<Task> tasks;       // for the helper, in order
    int helping = 0;              // tasks queued at or running on the helper
    int admitting = 0;            // admit tasks among them (they hold slots)
    bool helper_stop = false;
    std::vector<Ticket*> ready;   // admitted and initialised, to join at the next tick
    // solvers of completed tickets awaiting release (with the footprint each
    // holds against the budget): freed by the worker between ticks, since
    // freeing device memory waits for the whole device
    using Releases = std::vector<std::pair<lbm3d_solver*, size_t>>;
    Releases to_release;
    hipStream_t stream = nullptr;  // the ticks
    hipStream_t side = nullptr;    // the helper's initialisation and read-back
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    lbm3d::BatchPlan plans[3];  // one per precision
    int64_t plan_ticks[3] = {0, 0, 0};  // ticks each plan has run since it was built
    lbm3d_server_counters stats{};  // guarded by mu

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
    void run();
    void help();
    void admit_one(Ticket* t);
    void finish(Ticket* t, int32_t status);
    void to_helper(Ticket* t, int32_t status, bool admit)  // caller holds mu
    {
        tasks.push_back(Task{t, status, admit});
        helping++;
        if (admit) admitting++;
        cv_help.notify_one();
    }
};

static double secs_since(Clock::time_point a) { return std::chrono::duration<double>(Clock::now() - a).count(); }

// Completes a ticket (helper thread): its results are read back on the side
// stream, while a tick may run, and its solver is left to the worker to
// free between ticks.
void lbm3d_server::finish(Ticket* t, int32_t status)
{
    const auto tf = Clock::now();
    if (t->h) {
        if (status == LBM3D_OK || status == LBM3D_E_NONFINITE) {
            const int64_t n = t->h->n;
            for (int c = 0; c < 5; c++) t->out[c].resize((size_t)n);
            int32_t rc = lbm3d_moments(t->h, t->out[0].data(), t->out[1].data(), t->out[2].data(),
                                       t->out[3].data(), t->out[4].data());
            if (status == LBM3D_OK) status = rc;
        }
        uint32_t hw = 0;
        (void)lbm3d_status(t->h, &hw, nullptr);
        t->health = hw;
    }
    std::lock_guard<std::mutex> lk(mu);
    // (a ticket whose create failed still holds its footprint until then)
    to_release.emplace_back(t->h, t->footprint);
    t->h = nullptr;
    t->status = status;
    t->t_done = now();
    t->state = Ticket::DONE;
    stats.completed++;
    stats.finish_s += secs_since(tf);
    cv_done.notify_all();
    cv_work.notify_one();
}

// Creates and initialises an admitted solve (helper thread); it joins the
// active set at the worker's next tick.
void lbm3d_server::admit_one(Ticket* t)
{
    const auto ta = Clock::now();
    lbm3d_solver* h = nullptr;
    int32_t rc = lbm3d_create(&t->p, &h);
    if (rc == LBM3D_OK) rc = lbm3d_set_stream(h, side);
    if (rc == LBM3D_OK)
        rc = lbm3d_init(h, t->in[0].data(), t->in[1].data(), t->in[2].data(), t->in[3].data(), t->in[4].data());
    for (auto& v : t->in) std::vector<double>().swap(v);
    t->h = h;
    if (rc != LBM3D_OK) {
        finish(t, rc);
        return;
    }
    std::lock_guard<std::mutex> lk(mu);
    t->t_admit = now();
    t->state = Ticket::ACTIVE;
    ready.push_back(t);
    stats.admitted++;
    stats.admit_s += secs_since(ta);
    cv_work.notify_one();
}

void lbm3d_server::help()
{
    (void)hipSetDevice(device);
    for (;;) {
        Task task{nullptr, LBM3D_OK, false};
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_help.wait(lk, [&] { return !tasks.empty() || helper_stop; });
            if (tasks.empty()) return;
            task = tasks.front();
            tasks.pop_front();
        }
        if (task.admit)
            admit_one(task.t);
        else
            finish(task.t, task.status);
        std::lock_guard<std::mutex> lk(mu);
        helping--;
        if (task.admit) admitting--;
        cv_work.notify_one();
    }
}

void lbm3d_server::run()
{
    (void)hipSetDevice(device);
    for (;;) {
        std::vector<Ticket*> act;
        bool rebuild = false;
        Releases rel;
        {
            std::unique_lock<std::mutex> lk(mu);
            for (;;) {
                // queued tickets that were cancelled complete right away
                for (auto it = queue.begin(); it != queue.end();) {
                    if ((*it)->cancel) {
                        Ticket* t = *it;
                        t->status = LBM3D_E_CANCELLED;
                        t->t_done = now();
                        t->state = Ticket::DONE;
                        cv_done.notify_all();
                        it = queue.erase(it);
                    } else {
                        ++it;
                    }
                }
                // admission in arrival order, by device footprint and slots
                // (active, ready and being admitted): the helper creates and
                // initialises the solve while the ticks run
                while (!queue.empty() && (int)(active.size() + ready.size()) + admitting < max_active &&
                       used + queue.front()->footprint <= budget) {
                    Ticket* t = queue.front();
                    queue.pop_front();
                    used += t->footprint;
                    to_helper(t, LBM3D_OK, true);
                }
                // admitted solves join
                if (!ready.empty()) {
                    active.insert(active.end(), ready.begin(), ready.end());
                    ready.clear();
                    membership_changed = true;
                }
                // running tickets that were cancelled leave the active set
                for (auto it = active.begin(); it != active.end();) {
                    if ((*it)->cancel) {
                        to_helper(*it, LBM3D_E_CANCELLED, false);
                        it = active.erase(it);
                        membership_changed = true;
                    } else {
                        ++it;
                    }
                }
                rel.swap(to_release);
                if (!active.empty() || !rel.empty()) break;
                if (stop && queue.empty() && helping == 0 && ready.empty()) break;
                cv_work.wait(lk);
            }
            act = active;
            rebuild = membership_changed;
            if (!act.empty()) membership_changed = false;
        }
        // 1. free the solvers of completed tickets: no tick is running
        // (freeing waits for the device) and their footprint returns to the
        // budget
        if (!rel.empty()) {
            const auto tr = Clock::now();
            size_t freed = 0;
            for (auto& r : rel) {
                if (r.first) (void)lbm3d_destroy(r.first);
                freed += r.second;
            }
            std::lock_guard<std::mutex> lk(mu);
            used -= freed;
            stats.finish_s += secs_since(tr);
        }
        if (act.empty()) {
            std::lock_guard<std::mutex> lk(mu);
            if (stop && queue.empty() && helping == 0 && ready.empty() && to_release.empty()) return;
            continue;
        }
        // 2. one tick of the active solves: every precision group runs up
        // to tick_steps launches of the batched step, in which each member
        // takes the steps it still needs (at most tick_steps) and sits out
        // the rest, so a solve that is about to finish does not shorten the
        // tick for the others.  Ticks launch their steps directly; a graph
        // is captured only for a membership that has lasted
        // GRAPH_AFTER_TICKS ticks (capturing takes the worker milliseconds,
        // during which the device waits, and arrivals and completions
        // change the membership every few ticks under load).
        int32_t err = LBM3D_OK;
        double plan_s = 0.0;
        int rebuilds = 0;
        std::vector<Ticket*> members_of[3];
        (void)hipEventRecord(ev0, stream);
        for (int mode = 0; mode < 3 && err == LBM3D_OK; mode++) {
            std::vector<lbm3d_solver*> members;
            std::vector<int64_t> limit;
            int64_t k = 0;
            for (Ticket* t : act)
                if (t->h->mode == mode) {
                    members.push_back(t->h);
                    members_of[mode].push_back(t);
                    limit.push_back(t->left);
                    k = std::max(k, std::min(tick_steps, t->left));
                }
            if (members.empty() || k <= 0) continue;
            const bool fresh = rebuild || plans[mode].ntiles() == 0;
            if (fresh) {
                const auto tp = Clock::now();
                // (tile depth from the launch model for this membership)
                err = plans[mode].build(members, stream, -1);
                plan_s += secs_since(tp);
                rebuilds++;
                plan_ticks[mode] = 0;
            }
            const bool graphs = plan_ticks[mode]++ >= GRAPH_AFTER_TICKS;
            if (err == LBM3D_OK) err = plans[mode].run(k, stream, graphs, &limit);
            if (err == LBM3D_OK)
                for (Ticket* t : members_of[mode]) t->left -= std::min(k, t->left);
        }
        (void)hipEventRecord(ev1, stream);
        // 3. wait for the tick, then the health of every member (one gather
        // per precision): a solve that has gone non-finite stops now instead
        // of running out its steps; finished solves go to the helper
        float busy_ms = 0.0f;
        int nevict = 0;
        if (err == LBM3D_OK && hipStreamSynchronize(stream) != hipSuccess) err = LBM3D_E_DEVICE;
        if (err == LBM3D_OK) (void)hipEventElapsedTime(&busy_ms, ev0, ev1);
        std::vector<uint32_t> hw_of[3];
        for (int mode = 0; mode < 3 && err == LBM3D_OK; mode++)
            if (!members_of[mode].empty()) err = plans[mode].health(hw_of[mode], stream);
        std::lock_guard<std::mutex> lk(mu);
        for (int mode = 0; mode < 3; mode++) {
            for (size_t j = 0; j < members_of[mode].size(); j++) {
                Ticket* t = members_of[mode][j];
                const uint32_t hw = (err == LBM3D_OK && j < hw_of[mode].size()) ? hw_of[mode][j] : 0u;
                const bool bad = (hw & LBM3D_HEALTH_NONFINITE) != 0;
                if (err == LBM3D_OK && t->left > 0 && !bad) continue;
                auto it = std::find(active.begin(), active.end(), t);
                if (it == active.end()) continue;  // (already handed over, cancelled)
                active.erase(it);
                membership_changed = true;
                if (bad && t->left > 0) nevict++;
                to_helper(t, err != LBM3D_OK ? err : (bad ? LBM3D_E_NONFINITE : LBM3D_OK), false);
            }
        }
        stats.ticks++;
        stats.rebuilds += rebuilds;
        stats.plan_s += plan_s;
        stats.busy_s += busy_ms * 1e-3;
        stats.evicted += nevict;
    }
}

extern "C" {

int32_t lbm3d_server_create(size_t hbm_budget_bytes, int32_t max_active, lbm3d_server_t* out)
{
    if (!out || max_active < 1 || hbm_budget_bytes == 0) return LBM3D_E_INVAL;
    *out = nullptr;
    lbm3d_server* s = new (std::nothrow) lbm3d_server();
    if (!s) return LBM3D_E_NOMEM;
    s->budget = hbm_budget_bytes;
    s->max_active = max_active;
    s->t0 = Clock::now();
    if (hipGetDevice(&s->device) != hipSuccess ||
        hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&s->ev0) != hipSuccess || hipEventCreate(&s->ev1) != hipSuccess) {
        if (s->ev0) (void)hipEventDestroy(s->ev0);
        if (s->side) (void)hipStreamDestroy(s->side);
        if (s->stream) (void)hipStreamDestroy(s->stream);
        delete s;
        return LBM3D_E_DEVICE;
    }
    try {
        s->helper = std::thread([s] { s->help(); });
        s->worker = std::thread([s] { s->run(); });
    } catch (...) {
        if (s->helper.joinable()) {
            {
                std::lock_guard<std::mutex> lk(s->mu);
                s->helper_stop = true;
                s->cv_help.notify_one();
            }
            s->helper.join();
        }
        (void)hipEventDestroy(s->ev0);
        (void)hipEventDestroy(s->ev1);
        (void)hipStreamDestroy(s->side);
        (void)hipStreamDestroy(s->stream);
        delete s;
        return LBM3D_E_NOMEM;
    }
    *out = s;
    return LBM3D_OK;
}

int32_t lbm3d_server_set_tick(lbm3d_server_t s, int64_t steps)
{
    if (!s || steps < 1) return LBM3D_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    s->tick_steps = steps;
    return LBM3D_OK;
}

int32_t lbm3d_server_submit(lbm3d_server_t s, const lbm3d_params* p, const double* rho, const double* ux,
                            const double* uy, const double* uz, const double* pr, int64_t nsteps,
                            uint64_t* ticket)
{
    if (!s || !p || !rho || !ux || !uy || !uz || !pr || !ticket || nsteps < 0) return LBM3D_E_INVAL;
    size_t fp = 0;
    int32_t rc = lbm3d_footprint(p, &fp);
    if (rc) return rc;
    if (fp > s->budget) return LBM3D_E_NOMEM;
    // the batched kernel's limits: 32-bit plane offsets, NND only
    if (!lbm3d::tiled_fits(p->precision, lbm3d::make_grid(p)) || (p->flags & LBM3D_UPWIND2)) return LBM3D_E_INVAL;
    const size_t n = (size_t)p->nx * p->ny * p->nz;
    for (size_t k = 0; k < n; k++)
        if (!(rho[k] > 0.0) || !(pr[k] > 0.0)) return LBM3D_E_INVAL;
    std::unique_ptr<Ticket> t(new (std::nothrow) Ticket());
    if (!t) return LBM3D_E_NOMEM;
    t->p = *p;
    const double* src[5] = {rho, ux, uy, uz, pr};
    try {
        for (int c = 0; c < 5; c++) t->in[c].assign(src[c], src[c] + n);
    } catch (...) {
        return LBM3D_E_NOMEM;
    }
    t->nsteps = t->left = nsteps;
    t->footprint = fp;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return LBM3D_E_STATE;
    t->id = s->next_id++;
    t->t_submit = s->now();
    *ticket = t->id;
    s->queue.push_back(t.get());
    s->tickets[t->id] = std::move(t);
    s->cv_work.notify_one();
    return LBM3D_OK;
}

int32_t lbm3d_server_poll(lbm3d_server_t s, uint64_t ticket, int32_t* done)
{
    if (!s || !done) return LBM3D_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return LBM3D_E_NOTFOUND;
    *done = it->second->state == Ticket::DONE ? 1 : 0;
    return LBM3D_OK;
}

int32_t lbm3d_server_wait(lbm3d_server_t s, uint64_t ticket, double* rho, double* ux, double* uy, double* uz,
                          double* p, lbm3d_timing* tm)
{
    if (!s) return LBM3D_E_INVAL;
    std::unique_ptr<Ticket> t;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->tickets.find(ticket);
        if (it == s->tickets.end()) return LBM3D_E_NOTFOUND;
        Ticket* tp = it->second.get();
        // one waiter per ticket: the ticket (and its map entry) is released
        // by the waiter that claimed it
        if (tp->waited) return LBM3D_E_STATE;
        tp->waited = true;
        s->cv_done.wait(lk, [tp] { return tp->state == Ticket::DONE; });
        it = s->tickets.find(ticket);  // (the map may have rehashed meanwhile)
        t = std::move(it->second);
        s->tickets.erase(it);
    }
    double* dst[5] = {rho, ux, uy, uz, p};
    for (int c = 0; c < 5; c++)
        if (dst[c] && !t->out[c].empty()) std::memcpy(dst[c], t->out[c].data(), t->out[c].size() * sizeof(double));
    if (tm) {
        tm->t_submit = t->t_submit;
        tm->t_admit = t->t_admit;
        tm->t_done = t->t_done;
        tm->steps = t->nsteps - t->left;
        tm->health = t->health;
    }
    return t->status;
}

int32_t lbm3d_server_stats(lbm3d_server_t s, lbm3d_server_counters* out)
{
    if (!s || !out) return LBM3D_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->wall_s = s->now();
    return LBM3D_OK;
}

int32_t lbm3d_server_cancel(lbm3d_server_t s, uint64_t ticket)
{
    if (!s) return LBM3D_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return LBM3D_E_NOTFOUND;
    it->second->cancel = true;
    s->cv_work.notify_one();
    return LBM3D_OK;
}

int32_t lbm3d_server_destroy(lbm3d_server_t s)
{
    if (!s) return LBM3D_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (auto& kv : s->tickets) kv.second->cancel = true;
        s->cv_work.notify_one();
    }
    // the worker returns once every ticket is complete and every solver
    // freed (the helper has no task left then)
    if (s->worker.joinable()) s->worker.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->helper_stop = true;
        s->cv_help.notify_one();
    }
    if (s->helper.joinable()) s->helper.join();
    (void)hipStreamSynchronize(s->stream);
    (void)hipStreamSynchronize(s->side);
    for (auto& pl : s->plans) pl.build({}, s->stream);  // drop the plans' graphs and tables first
    (void)hipEventDestroy(s->ev0);
    (void)hipEventDestroy(s->ev1);
    (void)hipStreamDestroy(s->side);
    (void)hipStreamDestroy(s->stream);
    delete s;
    return LBM3D_OK;
}

}  // extern "C"
