// server.cpp -- serving engine behind lagp_server_*: continuous batching of
// prediction requests on one device under an HBM budget.
//
// Requests (host arrays, copied at submission) wait in a FIFO queue.  A
// worker thread owns a HIP stream and a device arena of the budgeted size.
// Whenever the device is free it forms the next batch from the head of the
// queue: every queued request with the same model parameters, in arrival
// order, while the batch's device footprint (workspace of its plan, inputs
// and outputs) stays within the arena.  The batch runs as one plan (size
// buckets, longest-first work lists) and its results are scattered back to
// the requests.  Locations are independent (Section 4.1) and every
// location's arithmetic is independent of the batch it runs in, so a
// request's results do not depend on the traffic it is mixed with.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "lagp_runtime.h"

using namespace lagp_rt;

namespace {

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
    double t_submit = 0.0, t_done = 0.0;
    int rc = LAGP_OK;            // batch failure code
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

// Device bytes of a batch's inputs and outputs beyond its plan workspace.
size_t io_bytes(int64_t T, int32_t nmax, int p)
{
    return a256(T * p * sizeof(double)) + 2 * a256(T * sizeof(int32_t)) + 3 * a256(T * sizeof(double)) +
           a256(T * sizeof(int32_t)) + a256((size_t)T * nmax * sizeof(int32_t)) + a256(T);
}

}  // namespace

struct lagp_server {
    lagp_design* design = nullptr;
    size_t budget = 0;
    char* arena = nullptr;
    hipStream_t stream = nullptr;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    std::deque<std::shared_ptr<Request>> queue;
    std::unordered_map<uint64_t, std::shared_ptr<Request>> live;
    uint64_t next_ticket = 1;
    int64_t batches = 0, locations = 0, requests = 0;
    double busy_s = 0.0;
    // pinned staging, grown by the worker
    char* pin = nullptr;
    size_t pin_bytes = 0;

    // Device footprint of a quick estimate: the plan with every location at
    // the batch maxima, plus the work list and the inputs and outputs.
    size_t estimate(int64_t T, int32_t nmax, int32_t Mmax, const lagp_params& prm)
    {
        lagp_params q = prm;
        q.n = nmax;
        q.ncand = Mmax;
        q.flags = 0;
        Plan P;
        if (build_plan(design, &q, T, nullptr, nullptr, true, true, &P)) return SIZE_MAX;
        return P.total + a256(T * sizeof(int32_t)) + io_bytes(T, nmax, design->dev.p);
    }

    // Exact footprint of the first k requests of `batch`, with their plan.
    size_t exact(const std::vector<std::shared_ptr<Request>>& batch, size_t k, Plan* P)
    {
        int64_t T = 0;
        int32_t nmax = 0;
        for (size_t i = 0; i < k; ++i) {
            T += batch[i]->T;
            nmax = std::max(nmax, batch[i]->nmax);
        }
        std::vector<int32_t> hn(T), hm(T);
        int64_t o = 0;
        for (size_t i = 0; i < k; ++i) {
            std::copy(batch[i]->n.begin(), batch[i]->n.end(), hn.begin() + o);
            std::copy(batch[i]->M.begin(), batch[i]->M.end(), hm.begin() + o);
            o += batch[i]->T;
        }
        *P = Plan();
        if (build_plan(design, &batch[0]->prm, T, hn.data(), hm.data(), true, true, P)) return SIZE_MAX;
        return P->total + a256(T * sizeof(int32_t)) + io_bytes(T, nmax, design->dev.p);
    }

    void run();
    int run_batch(const std::vector<std::shared_ptr<Request>>& batch, const Plan& P);
};

int lagp_server::run_batch(const std::vector<std::shared_ptr<Request>>& batch, const Plan& P)
{
    const int p = design->dev.p;
    const int64_t T = P.T;
    const int32_t nmax = P.nmax;
    const size_t order_b = a256(T * sizeof(int32_t));
    if (P.total + order_b + io_bytes(T, nmax, p) > budget) return fail(LAGP_E_BUDGET, "batch exceeds the serving budget");
    int rc = prepare_plan(design, P);
    if (rc) return rc;
    // arena: plan workspace | order | XX | n | M | mean | s2 | var | df | sel | status
    char* q = arena;
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
    // pinned staging: inputs then outputs, one copy each way
    const size_t in_b = order_b + a256(T * p * sizeof(double)) + 2 * a256(T * sizeof(int32_t));
    const size_t out_b = (size_t)((char*)status + a256(T) - (char*)mean);
    if (in_b + out_b > pin_bytes) {
        if (pin) (void)hipHostFree(pin);
        pin = nullptr;
        pin_bytes = 0;
        const size_t want = (in_b + out_b) * 3 / 2;
        hipError_t e = hipHostMalloc((void**)&pin, want, hipHostMallocDefault);
        if (e != hipSuccess) return hip_fail("pinned staging allocation", e);
        pin_bytes = want;
    }
    char* hin = pin;
    if (P.uneven) memcpy(hin, P.order.data(), T * sizeof(int32_t));
    else memset(hin, 0, T * sizeof(int32_t));
    int64_t o = 0;
    double* hXX = (double*)(hin + order_b);
    for (auto& r : batch) {
        memcpy(hXX + o * p, r->XX.data(), r->XX.size() * sizeof(double));
        o += r->T;
    }
    o = 0;
    for (auto& r : batch) {
        memcpy(hin + ((char*)n_per - (char*)order) + o * sizeof(int32_t), r->n.data(), r->T * sizeof(int32_t));
        memcpy(hin + ((char*)M_per - (char*)order) + o * sizeof(int32_t), r->M.data(), r->T * sizeof(int32_t));
        o += r->T;
    }
    hipError_t e = hipMemcpyAsync(order, hin, in_b, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_fail("batch input copy", e);
    const Outputs out = {mean, s2, df, var, sel, nmax, status};
    rc = enqueue_plan(design, P, ws, P.uneven ? order : nullptr, n_per, M_per, XX, out, stream, false, false);
    if (rc) return rc;
    char* hout = pin + in_b;
    e = hipMemcpyAsync(hout, mean, out_b, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail("batch", e);
    const double* hmean = (const double*)hout;
    const double* hs2 = (const double*)(hout + ((char*)s2 - (char*)mean));
    const double* hvar = (const double*)(hout + ((char*)var - (char*)mean));
    const int32_t* hdf = (const int32_t*)(hout + ((char*)df - (char*)mean));
    const int32_t* hsel = (const int32_t*)(hout + ((char*)sel - (char*)mean));
    const int8_t* hst = (const int8_t*)(hout + ((char*)status - (char*)mean));
    o = 0;
    for (auto& r : batch) {
        r->mean.assign(hmean + o, hmean + o + r->T);
        r->s2.assign(hs2 + o, hs2 + o + r->T);
        r->var.assign(hvar + o, hvar + o + r->T);
        r->df.assign(hdf + o, hdf + o + r->T);
        r->status.assign(hst + o, hst + o + r->T);
        r->sel.resize((size_t)r->T * r->nmax);
        for (int32_t t = 0; t < r->T; ++t)
            memcpy(&r->sel[(size_t)t * r->nmax], hsel + (size_t)(o + t) * nmax, r->nmax * sizeof(int32_t));
        o += r->T;
    }
    return LAGP_OK;
}

void lagp_server::run()
{
    (void)hipSetDevice(design->device);
    for (;;) {
        std::vector<std::shared_ptr<Request>> batch;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stop || !queue.empty(); });
            if (stop && queue.empty()) return;
            // FIFO admission: the head request and every later one with the
            // same model while the estimated batch footprint fits the arena.
            const lagp_params head = queue.front()->prm;
            int64_t T = 0;
            int32_t nmax = 0, Mmax = 0;
            for (auto it = queue.begin(); it != queue.end();) {
                const Request& r = **it;
                if (!same_model(r.prm, head)) { ++it; continue; }
                const int64_t T2 = T + r.T;
                const int32_t n2 = std::max(nmax, r.nmax), M2 = std::max(Mmax, r.Mmax);
                if (!batch.empty() && (T2 > kChunk || estimate(T2, n2, M2, head) > budget)) break;
                T = T2;
                nmax = n2;
                Mmax = M2;
                batch.push_back(*it);
                it = queue.erase(it);
            }
        }
        // The exact plan decides; if it does not fit, the largest fitting
        // prefix runs and the rest go back to the front of the queue.
        Plan P;
        size_t k = batch.size();
        if (exact(batch, k, &P) > budget) {
            size_t lo = 1, hi = k - 1;   // a single request always fits (checked at submission)
            while (lo < hi) {
                const size_t mid = (lo + hi + 1) / 2;
                Plan Q;
                if (exact(batch, mid, &Q) <= budget) lo = mid;
                else hi = mid - 1;
            }
            k = lo;
            (void)exact(batch, k, &P);
            std::lock_guard<std::mutex> lk(mu);
            for (size_t i = batch.size(); i-- > k;) queue.push_front(batch[i]);
            batch.resize(k);
        }
        const double t0 = now_s();
        int rc = run_batch(batch, P);
        const double t1 = now_s();
        {
            std::lock_guard<std::mutex> lk(mu);
            for (auto& r : batch) {
                r->rc = rc;
                r->done = true;
                r->t_done = t1;
            }
            batches += 1;
            for (auto& r : batch) locations += r->T;
            requests += (int64_t)batch.size();
            busy_s += t1 - t0;
        }
        cv_done.notify_all();
    }
}

extern "C" {

int lagp_server_create(const lagp_design* design, size_t hbm_budget_bytes, lagp_server** out)
{
    if (!out) return fail(LAGP_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!design) return fail(LAGP_E_INVAL, "design is NULL");
    if (hbm_budget_bytes < ((size_t)1 << 20)) return fail(LAGP_E_INVAL, "budget below 1 MiB");
    int rc = check_device(design);
    if (rc) return rc;
    lagp_server* s = new lagp_server();
    s->design = const_cast<lagp_design*>(design);
    s->budget = hbm_budget_bytes;
    hipError_t e = hipMalloc(&s->arena, hbm_budget_bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return fail(LAGP_E_NOMEM, "serving arena allocation of " + std::to_string(hbm_budget_bytes) + " bytes failed");
    }
    e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        (void)hipFree(s->arena);
        delete s;
        return hip_fail("hipStreamCreateWithFlags", e);
    }
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return LAGP_OK;
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
    // Full validation (the same checks as lagp_predict), then admission.
    std::vector<std::shared_ptr<Request>> one{r};
    Plan P;
    int rc = build_plan(s->design, prm, T, r->n.data(), r->M.data(), true, true, &P);
    if (rc) return rc;
    const size_t need = s->exact(one, 1, &P);
    if (need > s->budget)
        return fail(LAGP_E_BUDGET, "request needs " + std::to_string(need) + " device bytes, above the budget of " +
                                       std::to_string(s->budget));
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
    if (r->rc != LAGP_OK) return fail(r->rc, "the batch holding this request failed");
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

int lagp_server_stats(lagp_server* s, int64_t* batches, int64_t* locations, int64_t* requests, double* busy_s)
{
    if (!s) return fail(LAGP_E_INVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (batches) *batches = s->batches;
    if (locations) *locations = s->locations;
    if (requests) *requests = s->requests;
    if (busy_s) *busy_s = s->busy_s;
    return LAGP_OK;
}

double lagp_monotonic_seconds(void) { return now_s(); }

void lagp_server_destroy(lagp_server* s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    if (s->stream) {
        (void)hipStreamSynchronize(s->stream);
        (void)hipStreamDestroy(s->stream);
    }
    if (s->pin) (void)hipHostFree(s->pin);
    if (s->arena) (void)hipFree(s->arena);
    delete s;
}

}  // extern "C"
