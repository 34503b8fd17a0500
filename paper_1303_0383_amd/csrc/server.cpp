// server.cpp -- serving engine behind lagp_server_*: continuous batching of
// prediction requests on one device under an HBM budget.
//
// Requests (host arrays, copied at submission) wait in a FIFO queue.  The
// work is cut into pieces: runs of queued locations of one model (n0, d, g,
// precision), at most `piece` locations, taken from the requests in arrival
// order; a request may span several pieces and a piece may hold several
// requests.  Up to `slots` pieces are in flight at once, each on its own HIP
// stream with its own region of the device arena (first fit), so a request
// that arrives while others run is admitted as soon as a slot and enough of
// the arena are free, and its kernels run beside theirs.  The last slot only
// takes requests that have not started, so a short request never queues
// behind the remaining pieces of a long one.  A thread per slot waits for its
// piece, copies the results into the requests and completes each request
// whose last location is in: every request has its own completion time.
// Locations are independent (Section 4.1) and each location's arithmetic does
// not depend on the piece it runs in, so a request's results are bitwise the
// same alone or mixed with other traffic.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "arena_map.h"
#include "lagp_runtime.h"

using namespace lagp_rt;

namespace {

constexpr int kSlotsDefault = 3;
constexpr int kSlotsMax = 8;
constexpr int32_t kPieceDefault = 1024;

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
    uint64_t ticket = 0;
    int32_t T = 0;
    lagp_params prm{};
    std::vector<double> XX;
    std::vector<int32_t> n, M;   // per location
    int32_t nmax = 0, Mmax = 0;
    int32_t next = 0;            // first location not yet in a piece
    int32_t finished = 0;        // locations whose results are in
    double t_submit = 0.0, t_done = 0.0;
    int rc = LAGP_OK;            // failure code of a piece holding it
    bool done = false;
    std::vector<double> mean, s2, var;
    std::vector<int32_t> df, sel;   // sel: T x nmax
    std::vector<int8_t> status;
};

bool same_model(const lagp_params& a, const lagp_params& b)
{
    return a.n0 == b.n0 && a.d == b.d && a.g == b.g && a.precision == b.precision;
}

size_t a256(size_t b) { return lagp::align256(b); }

// Device bytes of a piece's inputs and outputs beyond its plan workspace.
size_t io_bytes(int64_t T, int32_t nmax, int p)
{
    return a256(T * p * sizeof(double)) + 2 * a256(T * sizeof(int32_t)) + 3 * a256(T * sizeof(double)) +
           a256(T * sizeof(int32_t)) + a256((size_t)T * nmax * sizeof(int32_t)) + a256(T);
}

// Locations [first, first + count) of a request, at offset `at` of a piece.
struct Segment {
    std::shared_ptr<Request> r;
    int32_t first = 0, count = 0;
    int64_t at = 0;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    std::thread th;
    bool express = false;   // takes only requests that have not started
    bool busy = false;      // a piece is enqueued and not yet harvested
    char* pin = nullptr;    // pinned staging: the piece's inputs, then its outputs
    size_t pin_bytes = 0;
    // the piece in flight
    std::vector<Segment> segs;
    int64_t T = 0;
    int32_t nmax = 0;
    size_t off = 0, bytes = 0;   // arena region
    size_t out_at = 0;           // outputs in the staging buffer; offsets from mean:
    size_t o_s2 = 0, o_var = 0, o_df = 0, o_sel = 0, o_status = 0;
    int rc = LAGP_OK;
};

}  // namespace

struct lagp_server {
    lagp_design* design = nullptr;
    size_t budget = 0;
    char* arena = nullptr;
    ArenaMap amap;
    int32_t piece = kPieceDefault;
    std::vector<std::unique_ptr<Slot>> slots;   // the last one is the express slot
    std::thread dispatcher;
    std::mutex mu;
    std::condition_variable cv_work, cv_slot, cv_done;
    bool stop = false, dispatcher_done = false;
    std::deque<std::shared_ptr<Request>> queue;   // requests with locations not yet in a piece
    std::unordered_map<uint64_t, std::shared_ptr<Request>> live;
    uint64_t next_ticket = 1;
    int64_t pieces = 0, locations = 0, requests = 0;
    int inflight = 0;
    double busy_s = 0.0, busy_t0 = 0.0;

    // Exact device footprint of a piece: its plan workspace, work list,
    // inputs and outputs (SIZE_MAX if the plan is rejected).
    size_t footprint(const std::vector<Segment>& segs, Plan* P)
    {
        int64_t T = 0;
        for (const auto& g : segs) T += g.count;
        std::vector<int32_t> hn(T), hm(T);
        for (const auto& g : segs) {
            std::copy(g.r->n.begin() + g.first, g.r->n.begin() + g.first + g.count, hn.begin() + g.at);
            std::copy(g.r->M.begin() + g.first, g.r->M.begin() + g.first + g.count, hm.begin() + g.at);
        }
        *P = Plan();
        // one lane: the pieces in flight already overlap on the device
        if (build_plan(design, &segs[0].r->prm, T, hn.data(), hm.data(), true, true, P, kChunk, 1)) return SIZE_MAX;
        return P->total + a256(T * sizeof(int32_t)) + io_bytes(T, P->nmax, design->dev.p);
    }

    enum class Form { none, ok, failed };
    Form form_piece(bool express, std::vector<Segment>* segs, Plan* P, size_t* bytes);
    int enqueue_piece(Slot& s, const Plan& P);
    void drop(const std::shared_ptr<Request>& r, int rc, double t);
    void dispatch_loop();
    void slot_loop(Slot& s);
};

// The next piece for a slot, under the lock: queued locations of the first
// eligible request's model in arrival order, at most `piece` of them, halved
// until the piece fits the largest free block of the arena.
lagp_server::Form lagp_server::form_piece(bool express, std::vector<Segment>* segs, Plan* P, size_t* bytes)
{
    const Request* head = nullptr;
    for (const auto& r : queue)
        if (!express || r->next == 0) {
            head = r.get();
            break;
        }
    if (!head) return Form::none;
    const size_t room = amap.largest();
    for (int64_t cap = piece;; cap = (cap + 1) / 2) {
        segs->clear();
        int64_t T = 0;
        for (const auto& r : queue) {
            if (T == cap) break;
            if ((express && r->next != 0) || !same_model(r->prm, head->prm)) continue;
            const int32_t c = (int32_t)std::min<int64_t>(r->T - r->next, cap - T);
            segs->push_back({r, r->next, c, T});
            T += c;
        }
        const size_t need = footprint(*segs, P);
        if (need == SIZE_MAX) {
            // every location passed the same checks at submission; fail the
            // requests rather than retry a plan that cannot be built
            for (const auto& g : *segs) drop(g.r, LAGP_E_INVAL, now_s());
            return Form::failed;
        }
        if (need <= room) {
            *bytes = need;
            return Form::ok;
        }
        if (cap == 1) return Form::none;
    }
}

// A request fails: its locations not yet in a piece are dropped, and it
// completes once the pieces holding the rest are harvested.  Under the lock.
void lagp_server::drop(const std::shared_ptr<Request>& r, int rc, double t)
{
    if (r->rc == LAGP_OK) r->rc = rc;
    if (r->next < r->T) {
        r->finished += r->T - r->next;
        r->next = r->T;
        queue.erase(std::remove(queue.begin(), queue.end(), r), queue.end());
    }
    if (r->finished == r->T && !r->done) {
        r->done = true;
        r->t_done = t;
        requests += 1;
    }
}

// Stages the piece's inputs and enqueues copy-in, the plan and copy-out on
// the slot's stream, without host waits.
int lagp_server::enqueue_piece(Slot& s, const Plan& P)
{
    const int p = design->dev.p;
    const int64_t T = P.T;
    const int32_t nmax = P.nmax;
    const size_t order_b = a256(T * sizeof(int32_t));
    int rc = prepare_plan(design, P);
    if (rc) return rc;
    // region: plan workspace | order | XX | n | M | mean | s2 | var | df | sel | status
    char* q = arena + s.off;
    char* ws = q;                      q += P.total;
    int32_t* order = (int32_t*)q;      q += order_b;
    double* XX = (double*)q;           q += a256(T * p * sizeof(double));
    int32_t* n_per = (int32_t*)q;      q += a256(T * sizeof(int32_t));
    int32_t* M_per = (int32_t*)q;      q += a256(T * sizeof(int32_t));
    double* mean = (double*)q;         q += a256(T * sizeof(double));
    double* s2 = (double*)q;           q += a256(T * sizeof(double));
    double* var = (double*)q;          q += a256(T * sizeof(double));
    int32_t* df = (int32_t*)q;         q += a256(T * sizeof(int32_t));
    int32_t* sel = (int32_t*)q;        q += a256((size_t)T * nmax * sizeof(int32_t));
    int8_t* status = (int8_t*)q;
    const size_t in_b = (size_t)((char*)mean - (char*)order);
    const size_t out_b = (size_t)((char*)status + a256(T) - (char*)mean);
    if (in_b + out_b > s.pin_bytes) {
        if (s.pin) (void)hipHostFree(s.pin);
        s.pin = nullptr;
        s.pin_bytes = 0;
        const size_t want = (in_b + out_b) * 3 / 2;
        hipError_t e = hipHostMalloc((void**)&s.pin, want, hipHostMallocDefault);
        if (e != hipSuccess) return hip_fail("pinned staging allocation", e);
        s.pin_bytes = want;
    }
    char* hin = s.pin;
    if (P.uneven) memcpy(hin, P.order.data(), T * sizeof(int32_t));
    else memset(hin, 0, T * sizeof(int32_t));
    double* hXX = (double*)(hin + ((char*)XX - (char*)order));
    int32_t* hn = (int32_t*)(hin + ((char*)n_per - (char*)order));
    int32_t* hm = (int32_t*)(hin + ((char*)M_per - (char*)order));
    for (const auto& g : s.segs) {
        memcpy(hXX + g.at * p, g.r->XX.data() + (size_t)g.first * p, (size_t)g.count * p * sizeof(double));
        memcpy(hn + g.at, g.r->n.data() + g.first, g.count * sizeof(int32_t));
        memcpy(hm + g.at, g.r->M.data() + g.first, g.count * sizeof(int32_t));
    }
    hipError_t e = hipMemcpyAsync(order, hin, in_b, hipMemcpyHostToDevice, s.stream);
    if (e != hipSuccess) return hip_fail("piece input copy", e);
    const Outputs out = {mean, s2, df, var, sel, nmax, status};
    // graph_safe: the kNN runs its fixed pass budget without host waits
    rc = enqueue_plan(design, P, ws, P.uneven ? order : nullptr, n_per, M_per, XX, out, s.stream, true, false);
    if (rc) return rc;
    s.out_at = in_b;
    s.o_s2 = (char*)s2 - (char*)mean;
    s.o_var = (char*)var - (char*)mean;
    s.o_df = (char*)df - (char*)mean;
    s.o_sel = (char*)sel - (char*)mean;
    s.o_status = (char*)status - (char*)mean;
    e = hipMemcpyAsync(s.pin + in_b, mean, out_b, hipMemcpyDeviceToHost, s.stream);
    return e == hipSuccess ? LAGP_OK : hip_fail("piece output copy", e);
}

void lagp_server::dispatch_loop()
{
    (void)hipSetDevice(design->device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        bool progressed = false;
        for (auto& sp : slots) {
            Slot& s = *sp;
            if (s.busy || queue.empty()) continue;
            std::vector<Segment> segs;
            Plan P;
            size_t bytes = 0;
            const Form f = form_piece(s.express, &segs, &P, &bytes);
            if (f == Form::failed) {
                progressed = true;
                cv_done.notify_all();
                continue;
            }
            if (f == Form::none || !amap.alloc(bytes, &s.off)) continue;
            for (const auto& g : segs) g.r->next += g.count;
            queue.erase(std::remove_if(queue.begin(), queue.end(),
                                       [](const std::shared_ptr<Request>& r) { return r->next == r->T; }),
                        queue.end());
            s.segs = std::move(segs);
            s.T = P.T;
            s.nmax = P.nmax;
            s.bytes = bytes;
            s.busy = true;
            if (inflight++ == 0) busy_t0 = now_s();
            pieces += 1;
            s.rc = enqueue_piece(s, P);
            // recorded whatever enqueue_piece managed, so the slot's wait
            // covers every launch made for the piece
            const hipError_t e = hipEventRecord(s.done, s.stream);
            if (e != hipSuccess && s.rc == LAGP_OK) s.rc = hip_fail("hipEventRecord", e);
            progressed = true;
            cv_slot.notify_all();
        }
        if (stop && queue.empty()) break;
        if (!progressed) cv_work.wait(lk);
    }
    dispatcher_done = true;
    cv_slot.notify_all();
}

void lagp_server::slot_loop(Slot& s)
{
    (void)hipSetDevice(design->device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        cv_slot.wait(lk, [&] { return s.busy || dispatcher_done; });
        if (!s.busy) return;
        lk.unlock();
        const hipError_t e = hipEventSynchronize(s.done);
        if (s.rc != LAGP_OK) (void)hipStreamSynchronize(s.stream);
        int rc = s.rc;
        if (rc == LAGP_OK && e != hipSuccess) rc = hip_fail("serving piece", e);
        if (rc == LAGP_OK) {
            // each location belongs to one piece: no other thread writes these ranges
            const char* hout = s.pin + s.out_at;
            const double* hmean = (const double*)hout;
            const double* hs2 = (const double*)(hout + s.o_s2);
            const double* hvar = (const double*)(hout + s.o_var);
            const int32_t* hdf = (const int32_t*)(hout + s.o_df);
            const int32_t* hsel = (const int32_t*)(hout + s.o_sel);
            const int8_t* hst = (const int8_t*)(hout + s.o_status);
            for (const auto& g : s.segs) {
                Request& r = *g.r;
                std::copy(hmean + g.at, hmean + g.at + g.count, r.mean.begin() + g.first);
                std::copy(hs2 + g.at, hs2 + g.at + g.count, r.s2.begin() + g.first);
                std::copy(hvar + g.at, hvar + g.at + g.count, r.var.begin() + g.first);
                std::copy(hdf + g.at, hdf + g.at + g.count, r.df.begin() + g.first);
                std::copy(hst + g.at, hst + g.at + g.count, r.status.begin() + g.first);
                for (int32_t t = 0; t < g.count; ++t)
                    memcpy(&r.sel[(size_t)(g.first + t) * r.nmax], hsel + (size_t)(g.at + t) * s.nmax,
                           r.nmax * sizeof(int32_t));
            }
        }
        lk.lock();
        const double t = now_s();
        for (const auto& g : s.segs) {
            Request& r = *g.r;
            r.finished += g.count;
            locations += g.count;
            if (rc != LAGP_OK) drop(g.r, rc, t);
            if (r.finished == r.T && !r.done) {
                r.done = true;
                r.t_done = t;
                requests += 1;
            }
        }
        s.segs.clear();
        amap.release(s.off, s.bytes);
        s.busy = false;
        if (--inflight == 0) busy_s += t - busy_t0;
        cv_work.notify_one();
        cv_done.notify_all();
    }
}

namespace {

void destroy_server(lagp_server* s)
{
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->dispatcher.joinable()) s->dispatcher.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->dispatcher_done = true;
    }
    s->cv_slot.notify_all();
    for (auto& sp : s->slots) {
        if (sp->th.joinable()) sp->th.join();
        if (sp->stream) {
            (void)hipStreamSynchronize(sp->stream);
            (void)hipStreamDestroy(sp->stream);
        }
        if (sp->done) (void)hipEventDestroy(sp->done);
        if (sp->pin) (void)hipHostFree(sp->pin);
    }
    if (s->arena) (void)hipFree(s->arena);
    delete s;
}

}  // namespace

extern "C" {

int lagp_server_create_ex(const lagp_design* design, size_t hbm_budget_bytes, int32_t slots, int32_t piece_locations,
                          lagp_server** out)
{
    if (!out) return fail(LAGP_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!design) return fail(LAGP_E_INVAL, "design is NULL");
    if (hbm_budget_bytes < ((size_t)1 << 20)) return fail(LAGP_E_INVAL, "budget below 1 MiB");
    if (slots == 0) slots = kSlotsDefault;
    if (slots < 2 || slots > kSlotsMax) return fail(LAGP_E_INVAL, "slots must be 0 (default) or in [2, 8]");
    if (piece_locations == 0) piece_locations = kPieceDefault;
    if (piece_locations < 1 || piece_locations > kChunk)
        return fail(LAGP_E_INVAL, "piece_locations must be 0 (default) or in [1, 131072]");
    int rc = check_device(design);
    if (rc) return rc;
    lagp_server* s = new lagp_server();
    s->design = const_cast<lagp_design*>(design);
    s->budget = hbm_budget_bytes;
    s->piece = piece_locations;
    hipError_t e = hipMalloc(&s->arena, hbm_budget_bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        s->arena = nullptr;
        destroy_server(s);
        return fail(LAGP_E_NOMEM, "serving arena allocation of " + std::to_string(hbm_budget_bytes) + " bytes failed");
    }
    s->amap.reset(hbm_budget_bytes);
    for (int k = 0; k < slots; ++k) {
        auto sl = std::make_unique<Slot>();
        sl->express = k == slots - 1;
        e = hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl->done, hipEventDisableTiming | hipEventBlockingSync);
        s->slots.push_back(std::move(sl));
        if (e != hipSuccess) {
            destroy_server(s);
            return hip_fail("serving stream or event", e);
        }
    }
    for (auto& sp : s->slots) {
        Slot* sl = sp.get();
        sl->th = std::thread([s, sl] { s->slot_loop(*sl); });
    }
    s->dispatcher = std::thread([s] { s->dispatch_loop(); });
    *out = s;
    return LAGP_OK;
}

int lagp_server_create(const lagp_design* design, size_t hbm_budget_bytes, lagp_server** out)
{
    return lagp_server_create_ex(design, hbm_budget_bytes, 0, 0, out);
}

int lagp_server_submit(lagp_server* s, const double* XX, int32_t T, const lagp_params* prm, const int32_t* n_per,
                       const int32_t* ncand_per, uint64_t* ticket)
{
    if (!s || !prm || !ticket) return fail(LAGP_E_INVAL, "NULL argument");
    if (T < 1) return fail(LAGP_E_INVAL, "T must be >= 1");
    if (!XX) return fail(LAGP_E_INVAL, "XX is NULL");
    if (prm->flags) return fail(LAGP_E_INVAL, "no flags are supported for served requests");
    if (is_device_ptr(XX) || (n_per && is_device_ptr(n_per)) || (ncand_per && is_device_ptr(ncand_per)))
        return fail(LAGP_E_INVAL, "served requests take host arrays");
    auto r = std::make_shared<Request>();
    r->T = T;
    r->prm = *prm;
    const int p = s->design->dev.p;
    r->XX.assign(XX, XX + (size_t)T * p);
    r->n.resize(T);
    r->M.resize(T);
    for (int32_t t = 0; t < T; ++t) {
        r->n[t] = n_per ? n_per[t] : prm->n;
        r->M[t] = ncand_per ? ncand_per[t] : prm->ncand;
        r->nmax = std::max(r->nmax, r->n[t]);
        r->Mmax = std::max(r->Mmax, r->M[t]);
    }
    // Full validation (the same checks as lagp_predict), then admission: the
    // whole request must fit the arena as one piece.
    Plan P;
    int rc = build_plan(s->design, prm, T, r->n.data(), r->M.data(), true, true, &P);
    if (rc) return rc;
    const size_t need = s->footprint({Segment{r, 0, T, 0}}, &P);
    if (need > s->budget)
        return fail(LAGP_E_BUDGET, "request needs " + std::to_string(need) + " device bytes, above the budget of " +
                                       std::to_string(s->budget));
    r->mean.resize(T);
    r->s2.resize(T);
    r->var.resize(T);
    r->df.resize(T);
    r->status.resize(T);
    r->sel.resize((size_t)T * r->nmax);
    r->t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        r->ticket = s->next_ticket++;
        s->live[r->ticket] = r;
        s->queue.push_back(r);
    }
    s->cv_work.notify_one();
    *ticket = r->ticket;
    return LAGP_OK;
}

int lagp_server_poll(lagp_server* s, uint64_t ticket, int32_t wait_ms, double* mean, double* s2, int32_t* df,
                     double* var, int32_t* sel, int64_t sel_stride, int8_t* status, double* times)
{
    if (!s) return fail(LAGP_E_INVAL, "server is NULL");
    std::shared_ptr<Request> r;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->live.find(ticket);
        if (it == s->live.end()) return fail(LAGP_E_INVAL, "unknown ticket");
        r = it->second;
        if (!r->done && wait_ms != 0) {
            auto pred = [&] { return r->done; };
            if (wait_ms < 0) s->cv_done.wait(lk, pred);
            else s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), pred);
        }
        if (!r->done) return 0;
        if (sel && sel_stride < r->nmax) return fail(LAGP_E_INVAL, "sel_stride below the request's n");
        s->live.erase(it);
    }
    if (r->rc != LAGP_OK) return fail(r->rc, "a piece holding this request failed");
    const size_t T = r->T;
    if (mean) memcpy(mean, r->mean.data(), T * sizeof(double));
    if (s2) memcpy(s2, r->s2.data(), T * sizeof(double));
    if (var) memcpy(var, r->var.data(), T * sizeof(double));
    if (df) memcpy(df, r->df.data(), T * sizeof(int32_t));
    if (status) memcpy(status, r->status.data(), T);
    if (sel)
        for (size_t t = 0; t < T; ++t)
            memcpy(sel + t * sel_stride, &r->sel[t * r->nmax], r->nmax * sizeof(int32_t));
    if (times) {
        times[0] = r->t_submit;
        times[1] = r->t_done;
    }
    return 1;
}

int lagp_server_stats(lagp_server* s, int64_t* pieces, int64_t* locations, int64_t* requests, double* busy_s)
{
    if (!s) return fail(LAGP_E_INVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (pieces) *pieces = s->pieces;
    if (locations) *locations = s->locations;
    if (requests) *requests = s->requests;
    if (busy_s) *busy_s = s->busy_s + (s->inflight ? now_s() - s->busy_t0 : 0.0);
    return LAGP_OK;
}

double lagp_monotonic_seconds(void) { return now_s(); }

void lagp_server_destroy(lagp_server* s)
{
    if (s) destroy_server(s);
}

}  // extern "C"
