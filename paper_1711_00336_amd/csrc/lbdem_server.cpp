// Serving form of the coupled LBM-DEM library: a request loop that admits
// settling solves (the problem of Sec. 4.1) of different grid sizes and
// solid fractions by their HBM footprint, keeps every admitted domain
// resident, and advances all of them in chunks of steps on parallel streams.
// Requests that arrive while others run join at the next chunk boundary
// (continuous batching); finished solves free their memory and slot at once.
#include "../../include/lbdem.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace {

thread_local std::string g_srv_err = "";

double now_s(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

struct Req {
    lbdem_params prm{};
    std::vector<double> x, u, w, d, rho;
    int64_t steps = 0, avg_from = 0;
    size_t footprint = 0;
    int state = 0;  // 0 queued, 1 active, 2 done
    bool cancel = false;
    lbdem_domain_t dom = nullptr;
    int stream = 0;
    int64_t done = 0;
    double ups_sum = 0.0;
    int64_t ups_n = 0;
    lbdem_result res{};
};

}  // namespace

struct lbdem_server {
    size_t budget = 0, used = 0;
    int32_t max_slots = 0, chunk = 20;
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<uint64_t> queue;
    std::map<uint64_t, Req> reqs;
    uint64_t next = 1;
    bool stop = false;
    std::vector<hipStream_t> streams;
    std::thread th;
    int64_t active = 0;
};

namespace {

lbdem_status sfail(lbdem_status st, const std::string &m)
{
    g_srv_err = m;
    return st;
}

// device bytes of one domain: two PDF buffers and 30 field components per
// cell in the storage precision, bins, per-particle state, and the Verlet
// lists (capacity twice the mean neighbour count within d_max + h_c + 0.25,
// plus 24 entries, as the domain sizes them)
size_t footprint_of(const lbdem_params &p, int64_t np, double dmax)
{
    const size_t nc = (size_t)p.n[0] * p.n[1] * p.n[2];
    const size_t rs = p.precision == LBDEM_FP64 ? 8 : 4;
    const double reach = dmax + (p.use_lub ? std::max(p.h_c, 0.0) : 0.0) + 0.25;
    const double nbr = 2.0 * (double)np / (double)nc * (4.0 / 3.0) * M_PI * reach * reach * reach + 28.0;
    const size_t per_particle = 1100 + (p.use_lift ? 48 : 0) + 4 * (size_t)std::max(32.0, nbr);
    return nc * (rs * (2 * 19 + 30 + (p.use_lift ? 4 : 0)) + 12) + (size_t)std::max<int64_t>(np, 64) * per_particle +
           (32u << 20);
}

void finish(lbdem_server_t s, uint64_t t, Req &r, lbdem_status st)
{
    r.res.status = st;
    r.res.steps_done = r.done;
    r.res.t_done = now_s(s->t0);
    if (r.dom) {
        lbdem_diag d{};
        if (st == LBDEM_OK && lbdem_diagnostics(r.dom, &d) == LBDEM_OK) {
            r.res.mean_eps_f = d.mean_eps_f;
            for (int a = 0; a < 3; ++a) r.res.mom[a] = d.mom_fluid[a] + d.mom_part[a];
        }
        r.res.u_ps = r.ups_n ? r.ups_sum / (double)r.ups_n : 0.0;
        lbdem_destroy(r.dom);
        r.dom = nullptr;
    }
    s->used -= r.footprint;
    s->active -= 1;
    r.state = 2;
    (void)t;
}

void loop(lbdem_server_t s)
{
    std::unique_lock<std::mutex> lk(s->mu);
    while (!s->stop) {
        // admission, first come first served, by footprint and slot count
        while (!s->queue.empty()) {
            const uint64_t t = s->queue.front();
            Req &r = s->reqs[t];
            if (r.cancel) {
                s->queue.pop_front();
                r.state = 2;
                r.res.status = LBDEM_E_STATE;
                r.res.t_done = now_s(s->t0);
                continue;
            }
            if (s->active >= s->max_slots || s->used + r.footprint > s->budget) break;
            s->queue.pop_front();
            r.stream = (int)(t % s->streams.size());
            r.res.t_admit = now_s(s->t0);
            s->used += r.footprint;
            s->active += 1;
            r.state = 1;
            lbdem_status st = lbdem_create(&r.prm, (void *)s->streams[r.stream], &r.dom);
            if (st == LBDEM_OK && !r.d.empty())
                st = lbdem_add_particles(r.dom, (int64_t)r.d.size(), r.x.data(), r.u.data(), r.w.data(), r.d.data(),
                                         r.rho.data());
            r.x.clear(); r.u.clear(); r.w.clear(); r.d.clear(); r.rho.clear();
            r.x.shrink_to_fit(); r.u.shrink_to_fit(); r.w.shrink_to_fit(); r.d.shrink_to_fit(); r.rho.shrink_to_fit();
            if (st != LBDEM_OK) finish(s, t, r, st);
        }
        struct Act {
            uint64_t t;
            Req *r;
            bool cancel;
        };
        std::vector<Act> act;
        for (auto &kv : s->reqs)
            if (kv.second.state == 1) act.push_back({kv.first, &kv.second, kv.second.cancel});
        if (act.empty()) {
            s->cv.wait_for(lk, std::chrono::milliseconds(2));
            continue;
        }
        const int32_t chunk = s->chunk;
        lk.unlock();
        // enqueue one chunk of every active solve; they run concurrently
        std::vector<lbdem_status> st(act.size(), LBDEM_OK);
        std::vector<int64_t> adv(act.size(), 0);
        for (size_t k = 0; k < act.size(); ++k) {
            Req &r = *act[k].r;
            if (act[k].cancel) continue;
            adv[k] = std::min<int64_t>(chunk, r.steps - r.done);
            if (adv[k] > 0) st[k] = lbdem_step(r.dom, adv[k]);
        }
        for (size_t k = 0; k < act.size(); ++k) {
            Req &r = *act[k].r;
            if (act[k].cancel || st[k] != LBDEM_OK) continue;
            st[k] = lbdem_sync(r.dom);
            if (st[k] != LBDEM_OK) continue;
            r.done += adv[k];
            if (r.done > r.avg_from || r.done == r.steps) {
                lbdem_diag d{};
                st[k] = lbdem_diagnostics(r.dom, &d);
                if (st[k] == LBDEM_OK && r.done > r.avg_from) {
                    r.ups_sum += d.u_ps;
                    r.ups_n += 1;
                }
            }
        }
        lk.lock();
        for (size_t k = 0; k < act.size(); ++k) {
            Req &r = *act[k].r;
            if (act[k].cancel) finish(s, act[k].t, r, LBDEM_E_STATE);
            else if (st[k] != LBDEM_OK) finish(s, act[k].t, r, st[k]);
            else if (r.done >= r.steps) finish(s, act[k].t, r, LBDEM_OK);
        }
    }
    // drain: free what is still resident
    for (auto &kv : s->reqs)
        if (kv.second.dom) {
            lbdem_destroy(kv.second.dom);
            kv.second.dom = nullptr;
        }
}

}  // namespace

extern "C" {

const char *lbdem_server_last_error(void) { return g_srv_err.c_str(); }

lbdem_status lbdem_server_create(size_t hbm_budget, int32_t max_slots, int32_t chunk_steps, lbdem_server_t *out)
{
    if (!out || hbm_budget == 0 || max_slots < 1 || chunk_steps < 1)
        return sfail(LBDEM_E_INVALID, "bad server arguments");
    *out = nullptr;
    lbdem_server_t s = new lbdem_server();
    s->budget = hbm_budget;
    s->max_slots = max_slots;
    s->chunk = chunk_steps;
    s->t0 = std::chrono::steady_clock::now();
    const int S = std::min<int>(max_slots, 4);
    for (int i = 0; i < S; ++i) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            lbdem_server_destroy(s);
            return sfail(LBDEM_E_DEVICE, "hipStreamCreate failed");
        }
        s->streams.push_back(st);
    }
    s->th = std::thread(loop, s);
    *out = s;
    return LBDEM_OK;
}

lbdem_status lbdem_server_submit(lbdem_server_t s, const lbdem_request *r, uint64_t *ticket)
{
    if (!s || !r || !ticket) return sfail(LBDEM_E_INVALID, "null argument");
    if (r->steps < 1 || r->np < 0 || (r->np > 0 && (!r->x || !r->d || !r->rho_p)))
        return sfail(LBDEM_E_INVALID, "bad request");
    Req q;
    q.prm = r->params;
    q.steps = r->steps;
    q.avg_from = std::max<int64_t>(0, std::min<int64_t>(r->avg_from, r->steps - 1));
    double dmax = 0.0;
    for (int64_t i = 0; i < r->np; ++i) dmax = std::max(dmax, r->d[i]);
    q.footprint = footprint_of(r->params, r->np, dmax);
    if (q.footprint > s->budget) return sfail(LBDEM_E_INVALID, "request exceeds the server's HBM budget");
    const int64_t n = r->np;
    q.x.assign(r->x, r->x + 3 * n);
    if (r->u) q.u.assign(r->u, r->u + 3 * n); else q.u.assign(3 * n, 0.0);
    if (r->omega) q.w.assign(r->omega, r->omega + 3 * n); else q.w.assign(3 * n, 0.0);
    q.d.assign(r->d, r->d + n);
    q.rho.assign(r->rho_p, r->rho_p + n);
    std::lock_guard<std::mutex> lk(s->mu);
    q.res.t_submit = now_s(s->t0);
    const uint64_t t = s->next++;
    s->reqs.emplace(t, std::move(q));
    s->queue.push_back(t);
    *ticket = t;
    s->cv.notify_all();
    return LBDEM_OK;
}

lbdem_status lbdem_server_poll(lbdem_server_t s, uint64_t ticket, lbdem_result *out)
{
    if (!s || !out) return sfail(LBDEM_E_INVALID, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return sfail(LBDEM_E_INVALID, "unknown ticket");
    if (it->second.state != 2) return LBDEM_E_BUSY;
    *out = it->second.res;
    return LBDEM_OK;
}

lbdem_status lbdem_server_cancel(lbdem_server_t s, uint64_t ticket)
{
    if (!s) return sfail(LBDEM_E_INVALID, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return sfail(LBDEM_E_INVALID, "unknown ticket");
    if (it->second.state == 2) return LBDEM_E_STATE;
    it->second.cancel = true;
    return LBDEM_OK;
}

lbdem_status lbdem_server_stats(lbdem_server_t s, int64_t *queued, int64_t *active, size_t *bytes_in_use)
{
    if (!s) return sfail(LBDEM_E_INVALID, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    if (queued) *queued = (int64_t)s->queue.size();
    if (active) *active = s->active;
    if (bytes_in_use) *bytes_in_use = s->used;
    return LBDEM_OK;
}

lbdem_status lbdem_server_destroy(lbdem_server_t s)
{
    if (!s) return LBDEM_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    if (s->th.joinable()) s->th.join();
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    delete s;
    return LBDEM_OK;
}

}  // extern "C"
