// lagp_api.cpp -- host runtime behind include/lagp.h: argument checks, the
// device-resident design, the workspace pool and the launch sequence
// (candidate sets, then greedy local designs with prediction) in chunks of
// locations.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <dlfcn.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "lagp_runtime.h"

namespace lagp_rt {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

int hip_fail(const char* what, hipError_t e)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return LAGP_E_HIP;
}

bool is_device_ptr(const void* p)
{
    if (!p) return false;
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// Rows 0, S, 2S, ... of the row-major design into a row-major sample.
__global__ void sample_rows_kernel(const double* __restrict__ X, double* __restrict__ Xs, int64_t Ns, int p, int S)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= Ns * p) return;
    int64_t j = e / p;
    int k = (int)(e - j * p);
    Xs[e] = X[j * S * p + k];
}

int ensure_ws(lagp_design* d, size_t bytes, hipStream_t stream)
{
    if (bytes <= d->ws_bytes) return LAGP_OK;
    hipError_t e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail("hipStreamSynchronize", e);
    if (d->ws) (void)hipFree(d->ws);
    d->ws = nullptr;
    d->ws_bytes = 0;
    size_t want = std::max(bytes, (size_t)1 << 20);
    e = hipMalloc(&d->ws, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(LAGP_E_NOMEM, "workspace allocation of " + std::to_string(want) + " bytes failed");
    }
    d->ws_bytes = want;
    return LAGP_OK;
}

int check_device(const lagp_design* d)
{
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail("hipGetDevice", e);
    if (cur != d->device) return fail(LAGP_E_INVAL, "the current device is not the design's device");
    return LAGP_OK;
}

}  // namespace lagp_rt

using namespace lagp_rt;

extern "C" {

int lagp_version(void) { return 100; }

const char* lagp_last_error(void) { return g_err.c_str(); }

int lagp_device_count(void)
{
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return n;
}

int lagp_design_create(const double* X, const double* y, int64_t N, int32_t p, uint32_t flags, void* stream,
                       lagp_design** out)
{
    if (!out) return fail(LAGP_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!X || !y) return fail(LAGP_E_INVAL, "X or y is NULL");
    if (N < 1 || N >= ((int64_t)1 << 31)) return fail(LAGP_E_INVAL, "N must be in [1, 2^31)");
    if (p < 1 || p > 32) return fail(LAGP_E_INVAL, "p must be in [1, 32]");
    if (flags & ~LAGP_PTR_HOST) return fail(LAGP_E_INVAL, "unknown flag");
    if (lagp_device_count() == 0) return fail(LAGP_E_NODEVICE, "no HIP device visible");
    const bool host = flags & LAGP_PTR_HOST;
    if (!host && (!is_device_ptr(X) || !is_device_ptr(y)))
        return fail(LAGP_E_INVAL, "X and y must be device pointers (or pass LAGP_PTR_HOST)");
    hipStream_t s = (hipStream_t)stream;

    lagp_design* d = new lagp_design();
    hipError_t e = hipGetDevice(&d->device);
    if (e != hipSuccess) { delete d; return hip_fail("hipGetDevice", e); }
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, d->device);
    if (e != hipSuccess) { delete d; return hip_fail("hipGetDeviceProperties", e); }
    d->num_cu = prop.multiProcessorCount;
    d->arch = prop.gcnArchName;
    d->arch = d->arch.substr(0, d->arch.find(':'));
    d->max_lds = prop.sharedMemPerBlock;
    const size_t bytes = (size_t)N * p * sizeof(double);
    const int64_t Ns = (N + lagp::KNN_SAMPLE_STRIDE - 1) / lagp::KNN_SAMPLE_STRIDE;
    if (hipMalloc(&d->Xaos, bytes) != hipSuccess ||
        hipMalloc(&d->Xaos_s, (size_t)Ns * p * sizeof(double)) != hipSuccess ||
        hipMalloc(&d->y, (size_t)N * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        lagp_design_destroy(d);
        return fail(LAGP_E_NOMEM, "design allocation failed");
    }
    const hipMemcpyKind kind = host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    e = hipMemcpyAsync(d->Xaos, X, bytes, kind, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d->y, y, (size_t)N * sizeof(double), kind, s);
    if (e != hipSuccess) { lagp_design_destroy(d); return hip_fail("design copy", e); }
    hipLaunchKernelGGL(sample_rows_kernel, dim3((unsigned)((Ns * p + 255) / 256)), dim3(256), 0, s, d->Xaos,
                       d->Xaos_s, Ns, p, lagp::KNN_SAMPLE_STRIDE);
    e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) { lagp_design_destroy(d); return hip_fail("design layout", e); }
    d->dev.Xaos = d->Xaos;
    d->dev.Xaos_s = d->Xaos_s;
    d->dev.Ns = Ns;
    d->dev.y = d->y;
    d->dev.N = N;
    d->dev.p = p;
    *out = d;
    return LAGP_OK;
}

void lagp_design_destroy(lagp_design* d)
{
    if (!d) return;
    (void)hipDeviceSynchronize();
    for (hipEvent_t e : d->ev) (void)hipEventDestroy(e);
    for (int l = 0; l + 1 < lagp_design::kLanes; ++l) {
        if (d->lane_stream[l]) (void)hipStreamDestroy(d->lane_stream[l]);
        if (d->lane_join[l]) (void)hipEventDestroy(d->lane_join[l]);
    }
    if (d->lane_fork) (void)hipEventDestroy(d->lane_fork);
    if (d->Xaos) (void)hipFree(d->Xaos);
    if (d->Xaos_s) (void)hipFree(d->Xaos_s);
    if (d->y) (void)hipFree(d->y);
    if (d->ws) (void)hipFree(d->ws);
    delete d;
}

int lagp_knn(const lagp_design* design, const double* XX, int64_t T, int32_t M, int32_t* idx, int64_t idx_stride,
             void* stream)
{
    if (!design) return fail(LAGP_E_INVAL, "design is NULL");
    if (T < 0) return fail(LAGP_E_INVAL, "T < 0");
    if (M < 1 || M > design->dev.N) return fail(LAGP_E_INVAL, "M must be in [1, N]");
    if (M > 4096) return fail(LAGP_E_INVAL, "M above 4096 is not supported");
    if (idx_stride < M) return fail(LAGP_E_INVAL, "idx_stride < M");
    if (T == 0) return LAGP_OK;
    if (!is_device_ptr(XX) || !is_device_ptr(idx)) return fail(LAGP_E_INVAL, "XX and idx must be device pointers");
    int rc = check_device(design);
    if (rc) return rc;
    lagp_design* d = const_cast<lagp_design*>(design);
    hipStream_t s = (hipStream_t)stream;
    for (int64_t t0 = 0; t0 < T; t0 += kChunk) {
        const int64_t tc = std::min(kChunk, T - t0);
        rc = ensure_ws(d, lagp::knn_workspace_bytes(tc, lagp::KNN_BUCKET_MAX), s);
        if (rc) return rc;
        std::string err;
        int r = lagp::knn_run(d->dev, XX + t0 * d->dev.p, tc, M, nullptr, idx + t0 * idx_stride, idx_stride, true,
                              d->ws, d->ws_bytes, s, d->num_cu, d->max_lds, &err);
        if (r) return fail(r == -1 ? LAGP_E_INVAL : LAGP_E_HIP, err);
    }
    return LAGP_OK;
}

}  // extern "C"

// ------------------------------------------------------------ batch planning
//
// A batch is planned once from host-side sizes: every location is checked,
// locations are grouped by size class (candidate-set size rounded up to a
// power of two >= 256, design size rounded up to a power of two >= 32) so
// that each group runs a kernel variant sized for it, and each group is
// ordered by decreasing modelled cost (longest first) so that the persistent
// workgroups finish together.  Enqueueing a plan launches kernels only: no
// allocation, no host synchronisation and no memset, so it can be captured
// into a HIP graph.
namespace lagp_rt {

int size_class(int32_t v, int32_t lo)
{
    int c = lo;
    while (c < v) c <<= 1;
    return c;
}

// ---- tuned kernel variants: text table
// "arch precision mclass nclass threads coords [lds_pct]"
struct TuneEntry {
    std::string arch;
    int prec, mclass, nclass, threads, coords, lds = 100;
};

std::vector<TuneEntry>& tune_table()
{
    static std::vector<TuneEntry> table;
    static std::once_flag once;
    std::call_once(once, [] {
        std::string path;
        if (const char* e = getenv("LAGP_TUNE_TABLE")) {
            path = e;
        } else {
            Dl_info info;
            if (dladdr((const void*)&lagp_version, &info) && info.dli_fname) {
                path = info.dli_fname;
                const size_t k = path.rfind('/');
                path = (k == std::string::npos ? std::string(".") : path.substr(0, k)) + "/tune/table.txt";
            }
        }
        FILE* f = path.empty() ? nullptr : fopen(path.c_str(), "r");
        if (!f) return;
        char line[512];
        while (fgets(line, sizeof line, f)) {
            if (line[0] == '#') continue;
            char arch[64];
            TuneEntry t;
            const int k = sscanf(line, "%63s %d %d %d %d %d %d", arch, &t.prec, &t.mclass, &t.nclass, &t.threads,
                                 &t.coords, &t.lds);
            if (k == 6 || k == 7) {
                t.arch = arch;
                if (k == 6 || t.lds < 0 || t.lds > 100) t.lds = 100;
                table.push_back(t);
            }
        }
        fclose(f);
    });
    return table;
}

void choose_variant(const lagp_design* d, int prec, int32_t nmax, int32_t Mmax, lagp::DesignPlan* plan)
{
    plan->threads = 256;
    plan->coords_pref = -1;
    plan->lds_pct = 100;
    if (d->force_threads || d->force_coords >= 0 || d->force_lds_pct >= 0) {
        if (d->force_threads) plan->threads = d->force_threads;
        plan->coords_pref = d->force_coords;
        if (d->force_lds_pct >= 0) plan->lds_pct = d->force_lds_pct;
        return;
    }
    const int mc = size_class(Mmax, 256), nc = size_class(nmax, 32);
    // a BF16-tile class without its own entry takes the FP32 tile's
    for (const int pr : {prec, prec == LAGP_PREC_SCORE_BF16 ? (int)LAGP_PREC_SCORE_FP32 : prec})
        for (const TuneEntry& t : tune_table())
            if (t.arch == d->arch && t.prec == pr && t.mclass == mc && t.nclass == nc) {
                plan->threads = t.threads;
                plan->coords_pref = t.coords;
                plan->lds_pct = t.lds;
                return;
            }
}

int plan_design(const lagp_design* d, int prec, int32_t nmax, int32_t Mmax, int32_t Mmin, int32_t n0, int64_t count,
                lagp::DesignPlan* plan)
{
    std::string err;
    choose_variant(d, prec, nmax, Mmax, plan);
    if (lagp::design_plan(d->dev, nmax, Mmax, Mmin, n0, prec, d->num_cu, d->max_lds, plan, &err))
        return fail(LAGP_E_INVAL, err);
    // no more persistent workgroups (and scratch slabs) than locations
    plan->blocks = (int)std::max<int64_t>(1, std::min<int64_t>(plan->blocks, count));
    return LAGP_OK;
}

// Checks parameters and per-location sizes (host arrays, nullable) and builds the plan.
int build_plan(const lagp_design* d, const lagp_params* prm, int64_t T, const int32_t* hn, const int32_t* hm,
               bool have_sel, bool have_status, Plan* P, int64_t chunk, int lanes)
{
    if (chunk < 1) return fail(LAGP_E_INVAL, "chunk must be >= 1");
    if (const char* e = getenv("LAGP_BUCKET_LANES")) lanes = std::min(lanes, atoi(e));   // measurement override
    lanes = std::max(1, std::min(lanes, (int)lagp_design::kLanes));
    int max_lanes = 1;
    P->chunk = chunk;
    const int64_t N = d->dev.N;
    if (!(prm->d > 0.0) || !isfinite(prm->d)) return fail(LAGP_E_INVAL, "lengthscale d must be positive and finite");
    if (!(prm->g >= 0.0) || !isfinite(prm->g)) return fail(LAGP_E_INVAL, "nugget g must be >= 0 and finite");
    if (prm->precision != LAGP_PREC_FP64 && prm->precision != LAGP_PREC_SCORE_FP32 &&
        prm->precision != LAGP_PREC_SCORE_BF16)
        return fail(LAGP_E_INVAL, "unsupported precision mode");
    if (prm->flags & ~(uint32_t)LAGP_STRICT) return fail(LAGP_E_INVAL, "unknown flag");
    if (prm->n0 < 1) return fail(LAGP_E_INVAL, "n0 must be >= 1");
    if (!hn && (prm->n < prm->n0)) return fail(LAGP_E_INVAL, "n must be >= n0");
    if (!hm && (prm->ncand < 1 || prm->ncand > N)) return fail(LAGP_E_INVAL, "ncand must be in [1, N]");
    if (!hn && !hm && prm->ncand < prm->n) return fail(LAGP_E_INVAL, "ncand must be >= n");
    P->prm = *prm;
    P->T = T;
    P->uneven = hn || hm;
    P->mix = prm->precision != LAGP_PREC_FP64;
    int32_t nmax = prm->n, Mmax = prm->ncand;
    P->nmin = hn ? INT32_MAX : prm->n;
    if (P->uneven) {
        nmax = 0;
        Mmax = 0;
        for (int64_t t = 0; t < T; ++t) {
            const int32_t nt = hn ? hn[t] : prm->n;
            const int32_t mt = hm ? hm[t] : prm->ncand;
            if (nt < prm->n0 || mt < nt || mt > N)
                return fail(LAGP_E_INVAL, "location " + std::to_string(t) + ": need n0 <= n <= ncand <= N");
            nmax = std::max(nmax, nt);
            P->nmin = std::min(P->nmin, nt);
            Mmax = std::max(Mmax, mt);
        }
    }
    if (Mmax > 4096) return fail(LAGP_E_INVAL, "ncand above 4096 is not supported");
    if (nmax > 1024) return fail(LAGP_E_INVAL, "n above 1024 is not supported");
    if (P->mix && nmax > 128) return fail(LAGP_E_INVAL, "the mixed precision mode supports n <= 128");
    P->nmax = nmax;
    P->Mmax = Mmax;
    P->own_sel = false;
    P->own_status = P->mix && !have_status;
    const int64_t tc_max = std::min(chunk, std::max<int64_t>(T, 1));
    size_t design_b = 0;
    if (P->uneven) P->order.resize(T);
    for (int64_t t0 = 0; t0 < T; t0 += chunk) {
        Chunk c;
        c.t0 = t0;
        c.T = std::min(chunk, T - t0);
        c.nmax = 0;
        c.Mmax = 0;
        if (!P->uneven) {
            Bucket b;
            b.nmax = c.nmax = nmax;
            b.Mmax = c.Mmax = Mmax;
            b.Mmin = c.Mmin = Mmax;
            b.first = 0;
            b.count = c.T;
            c.buckets.push_back(b);
        } else {
            // group by (candidate class, design class), largest classes first
            std::vector<std::pair<int64_t, int64_t>> key(c.T);   // (class key, location)
            for (int64_t k = 0; k < c.T; ++k) {
                const int64_t t = t0 + k;
                const int32_t nt = hn ? hn[t] : prm->n, mt = hm ? hm[t] : prm->ncand;
                c.nmax = std::max(c.nmax, nt);
                c.Mmax = std::max(c.Mmax, mt);
                c.Mmin = std::min(c.Mmin, mt);
                key[k] = {-((int64_t)size_class(mt, 256) << 16 | size_class(nt, 32)), k};
            }
            auto cost = [&](int64_t k) {
                const int64_t t = t0 + k;
                const double nt = hn ? hn[t] : prm->n, mt = hm ? hm[t] : prm->ncand;
                return nt * nt * mt;
            };
            std::stable_sort(key.begin(), key.end(), [&](const auto& a, const auto& b) {
                if (a.first != b.first) return a.first < b.first;
                const double ca = cost(a.second), cb = cost(b.second);
                if (ca != cb) return ca > cb;
                return a.second < b.second;
            });
            for (int64_t k = 0; k < c.T;) {
                int64_t e = k;
                Bucket b;
                while (e < c.T && key[e].first == key[k].first) {
                    const int64_t t = t0 + key[e].second;
                    b.nmax = std::max(b.nmax, hn ? hn[t] : prm->n);
                    b.Mmax = std::max(b.Mmax, hm ? hm[t] : prm->ncand);
                    b.Mmin = std::min(b.Mmin, hm ? hm[t] : prm->ncand);
                    P->order[t0 + e] = (int32_t)key[e].second;
                    ++e;
                }
                b.first = k;
                b.count = e - k;
                c.buckets.push_back(b);
                k = e;
            }
        }
        for (Bucket& b : c.buckets) {
            int rc = plan_design(d, prm->precision, b.nmax, b.Mmax, b.Mmin, prm->n0, b.count, &b.plan);
            if (rc) return rc;
            design_b = std::max(design_b, lagp::design_workspace_bytes(b.plan));
        }
        // Concurrent lanes: each bucket (largest classes first) joins the lane
        // with the least estimated work so far (count x n^2 x N'), so one
        // bucket's tail overlaps the others' work.
        c.lanes = (int)std::min<size_t>((size_t)lanes, c.buckets.size());
        std::vector<double> load(c.lanes, 0.0);
        for (Bucket& b : c.buckets) {
            int best = 0;
            for (int l = 1; l < c.lanes; ++l)
                if (load[l] < load[best]) best = l;
            b.lane = best;
            load[best] += (double)b.count * b.nmax * b.nmax * b.Mmax;
        }
        max_lanes = std::max(max_lanes, c.lanes);
        if (P->mix) {
            int rc = plan_design(d, LAGP_PREC_FP64, c.nmax, c.Mmax, c.Mmin, prm->n0, c.T, &c.redo);
            if (rc) return rc;
            design_b = std::max(design_b, lagp::design_workspace_bytes(c.redo));
        }
        P->chunks.push_back(c);
    }
    P->knn_b = lagp::align256(lagp::knn_workspace_bytes(tc_max, lagp::KNN_BUCKET_MAX));
    P->cand_b = lagp::align256((size_t)tc_max * Mmax * sizeof(int32_t));
    P->lane_b = lagp::align256(design_b);
    P->design_b = P->lane_b * max_lanes;
    P->order_b = P->uneven ? lagp::align256((size_t)T * sizeof(int32_t)) : 0;
    P->sel_b = P->own_sel ? lagp::align256((size_t)tc_max * nmax * sizeof(int32_t)) : 0;
    P->status_b = P->own_status ? lagp::align256((size_t)T) : 0;
    P->redo_b = P->mix ? lagp::align256((size_t)tc_max * sizeof(int32_t)) + 256 : 0;
    P->total = P->knn_b + P->cand_b + P->design_b + P->order_b + P->sel_b + P->status_b + P->redo_b;
    if (getenv("LAGP_VERBOSE"))
        for (const Chunk& c : P->chunks)
            for (const Bucket& b : c.buckets)
                fprintf(stderr,
                        "[lagp] bucket: locations=%lld n<=%d ncand<=%d p=%d threads=%d slots/thread=%d trim=%d rows: reg=%d "
                        "lds=%d global=%d coords_lds=%d lds=%zu B global_row_reads/loc=%lld workspace=%zu B\n",
                        (long long)b.count, b.nmax, b.Mmax, d->dev.p, b.plan.threads, b.plan.cpt, (int)b.plan.trim, b.plan.rreg,
                        b.plan.rlds, b.plan.rglob, (int)b.plan.coords_lds, b.plan.lds_bytes,
                        b.plan.global_row_reads, P->total);
    return LAGP_OK;
}

// Host-side kernel set-up for every variant the plan launches.
int prepare_plan(const lagp_design* dc, const Plan& P)
{
    std::string err;
    lagp_design* d = const_cast<lagp_design*>(dc);
    bool lanes = false;
    for (const Chunk& c : P.chunks) lanes = lanes || c.lanes > 1;
    if (lanes) {
        std::lock_guard<std::mutex> lk(d->lane_mu);
        hipError_t e = hipSuccess;
        if (!d->lane_fork) e = hipEventCreateWithFlags(&d->lane_fork, hipEventDisableTiming);
        for (int l = 0; l + 1 < lagp_design::kLanes && e == hipSuccess; ++l) {
            if (!d->lane_stream[l]) e = hipStreamCreateWithFlags(&d->lane_stream[l], hipStreamNonBlocking);
            if (e == hipSuccess && !d->lane_join[l]) e = hipEventCreateWithFlags(&d->lane_join[l], hipEventDisableTiming);
        }
        if (e != hipSuccess) return hip_fail("bucket lane streams", e);
    }
    if (lagp::knn_prepare(d->dev.p, d->max_lds, &err)) return fail(LAGP_E_HIP, err);
    for (const Chunk& c : P.chunks) {
        for (const Bucket& b : c.buckets)
            if (lagp::design_prepare(b.plan, &err)) return fail(LAGP_E_HIP, err);
        if (P.mix && lagp::design_prepare(c.redo, &err)) return fail(LAGP_E_HIP, err);
    }
    if (P.alc2 && lagp::predict_prepare(P.nmax, d->max_lds, &err)) return fail(LAGP_E_HIP, err);
    if (P.alc2 && lagp::mle_prepare(P.nmax, d->dev.p, d->max_lds, &err)) return fail(LAGP_E_HIP, err);
    return LAGP_OK;
}

int check_mle_params(const lagp_mle_params* m)
{
    if (!m) return fail(LAGP_E_INVAL, "MLE parameters are NULL");
    if (!(m->tmin > 0.0) || !(m->tmax > m->tmin) || !isfinite(m->tmax))
        return fail(LAGP_E_INVAL, "need 0 < tmin < tmax, finite");
    if (m->maxit < 1) return fail(LAGP_E_INVAL, "maxit must be >= 1");
    if (!(m->tol > 0.0) || !isfinite(m->tol)) return fail(LAGP_E_INVAL, "tol must be positive and finite");
    return LAGP_OK;
}

int plan_alc2(const lagp_design* d, const lagp_mle_params* mle, bool have_sel, Plan* P)
{
    int rc = check_mle_params(mle);
    if (rc) return rc;
    if (P->nmin < 2) return fail(LAGP_E_INVAL, "the two-stage scheme needs n >= 2 at every location");
    if (lagp::mle_lds_bytes(P->nmax, d->dev.p, 512) > d->max_lds)
        return fail(LAGP_E_INVAL, "n too large for the likelihood kernel");
    if (lagp::predict_lds_bytes(P->nmax) > d->max_lds) return fail(LAGP_E_INVAL, "n too large for the prediction kernel");
    P->alc2 = true;
    P->mle = *mle;
    const int64_t tc_max = std::min(P->chunk, std::max<int64_t>(P->T, 1));
    if (!have_sel && !P->own_sel) {
        P->own_sel = true;
        P->total -= P->sel_b;
        P->sel_b = lagp::align256((size_t)tc_max * P->nmax * sizeof(int32_t));
        P->total += P->sel_b;
    }
    P->sel1_b = lagp::align256((size_t)tc_max * P->nmax * sizeof(int32_t));
    P->stage_b = 4 * lagp::align256((size_t)tc_max * sizeof(double)) + lagp::align256((size_t)tc_max);
    P->total += P->sel1_b + P->stage_b;
    return LAGP_OK;
}

__global__ void collect_failed_kernel(const int8_t* __restrict__ status, int64_t T, int32_t* __restrict__ list,
                                      uint32_t* __restrict__ count)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < T && status[t] != LAGP_LOC_OK) list[atomicAdd(count, 1u)] = (int32_t)t;
}

// One design pass over chunk c into L's outputs: every bucket's launch, and
// in the mixed mode the FP64 prediction and the FP64 redo of failed locations.
static int enqueue_designs(lagp_design* d, const Plan& P, const Chunk& c, lagp::DesignLaunch L,
                           const int32_t* order_dev, void* des_ws, int32_t* redo_list, uint32_t* redo_count,
                           hipStream_t s)
{
    std::string err;
    // Buckets in several lanes: the lanes' streams wait for the caller's
    // stream, each lane runs its buckets in order in its own workspace, and
    // the caller's stream waits for every lane (in stream capture these are
    // the graph's fork and join).
    const bool fork = c.lanes > 1;
    std::unique_lock<std::mutex> lk(d->lane_mu, std::defer_lock);
    if (fork) {
        lk.lock();
        hipError_t e = hipEventRecord(d->lane_fork, s);
        for (int l = 1; l < c.lanes && e == hipSuccess; ++l) e = hipStreamWaitEvent(d->lane_stream[l - 1], d->lane_fork, 0);
        if (e != hipSuccess) return hip_fail("bucket lanes: fork", e);
    }
    int rb = 0;
    for (const Bucket& b : c.buckets) {
        L.precision = P.prm.precision;
        L.T = b.count;
        L.n = b.nmax;
        L.M = b.Mmax;
        L.order = order_dev ? order_dev + c.t0 + b.first : nullptr;
        hipStream_t ls = b.lane == 0 ? s : d->lane_stream[b.lane - 1];
        void* ws = (char*)des_ws + (size_t)b.lane * P.lane_b;
        rb = lagp::design_run(d->dev, L, b.plan, ws, P.lane_b, ls, &err);
        if (rb) break;
    }
    if (fork) {
        // joined on the error path too: the caller's stream (or the capture)
        // must not end while a lane still has work in flight
        hipError_t e = hipSuccess;
        for (int l = 1; l < c.lanes && e == hipSuccess; ++l) {
            e = hipEventRecord(d->lane_join[l - 1], d->lane_stream[l - 1]);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, d->lane_join[l - 1], 0);
        }
        lk.unlock();
        if (rb) return fail(rb == -1 ? LAGP_E_INVAL : LAGP_E_HIP, err);
        if (e != hipSuccess) return hip_fail("bucket lanes: join", e);
    }
    if (rb) return fail(rb == -1 ? LAGP_E_INVAL : LAGP_E_HIP, err);
    if (P.mix) {
        // A location the mixed mode could not finish (its short list held no
        // candidate with a positive exact variance) is redone in FP64 from a
        // device-side list.
        lagp::fill_u32(redo_count, 1, 0u, s);
        int r;
        hipLaunchKernelGGL(collect_failed_kernel, dim3((unsigned)((c.T + 255) / 256)), dim3(256), 0, s, L.status,
                           c.T, redo_list, redo_count);
        L.precision = LAGP_PREC_FP64;
        L.T = c.T;
        L.n = c.nmax;
        L.M = c.Mmax;
        L.order = redo_list;
        L.count = redo_count;
        r = lagp::design_run(d->dev, L, c.redo, des_ws, P.lane_b, s, &err);
        if (r) return fail(r == -1 ? LAGP_E_INVAL : LAGP_E_HIP, err);
    }
    return LAGP_OK;
}

// The likelihood kernel over a chunk's locations.  Its LDS is sized for the
// largest design of a launch, so with uneven sizes it runs once per size
// bucket (the bucket's part of the work list, LDS for the bucket's largest
// design): small designs then share a CU instead of each taking the space of
// the chunk's largest.
static int mle_by_bucket(lagp::MleArgs m, const Chunk& c, const int32_t* order_dev, size_t max_lds, hipStream_t s)
{
    std::string err;
    if (!order_dev || c.buckets.size() < 2) {
        const int r = lagp::mle_run(m, max_lds, s, &err);
        return r ? fail(r == -1 ? LAGP_E_INVAL : LAGP_E_HIP, err) : 0;
    }
    for (const Bucket& b : c.buckets) {
        if (b.count == 0) continue;
        m.order = order_dev + c.t0 + b.first;
        m.T = b.count;
        m.nmax = b.nmax;
        const int r = lagp::mle_run(m, max_lds, s, &err);
        if (r) return fail(r == -1 ? LAGP_E_INVAL : LAGP_E_HIP, err);
    }
    return 0;
}

// Enqueues the whole plan on stream s.  ws holds P.total bytes; order_dev is
// the uploaded work list (uneven plans); n_per / ncand_per are device arrays.
int enqueue_plan(lagp_design* d, const Plan& P, char* ws, const int32_t* order_dev, const int32_t* n_per,
                 const int32_t* ncand_per, const double* XX, const Outputs& o, hipStream_t s, bool graph_safe,
                 bool timing, const ThetaIO* th)
{
    char* q = ws;
    void* knn_ws = q;                  q += P.knn_b;
    int32_t* cand = (int32_t*)q;       q += P.cand_b;
    void* des_ws = q;                  q += P.design_b;
    q += P.order_b;                    // (order_dev lives here for lagp_predict)
    int32_t* sel_ws = (int32_t*)q;     q += P.sel_b;
    int8_t* st_ws = (int8_t*)q;        q += P.status_b;
    int32_t* redo_list = (int32_t*)q;
    uint32_t* redo_count = (uint32_t*)(q + (P.redo_b ? P.redo_b - 256 : 0));
    q += P.redo_b;
    int32_t* sel1_ws = (int32_t*)q;    q += P.sel1_b;
    const int64_t tc_max = std::min(P.chunk, std::max<int64_t>(P.T, 1));
    const size_t vb = lagp::align256((size_t)tc_max * sizeof(double));
    double* st_mean = (double*)q;
    double* st_s2 = (double*)(q + vb);
    double* th1_ws = (double*)(q + 2 * vb);
    double* th2_ws = (double*)(q + 3 * vb);
    int8_t* st_status = (int8_t*)(q + 4 * vb);
    const int p = d->dev.p;
    const double* d_per = th ? th->d_per : nullptr;
    // With `timing`, an event closes each phase interval on the stream.
    auto mark = [&](int phase, int64_t launches) -> int {
        if (!timing) return LAGP_OK;
        hipEvent_t e = nullptr;
        hipError_t h = hipEventCreate(&e);
        if (h != hipSuccess) return hip_fail("hipEventCreate", h);
        d->ev.push_back(e);
        d->ev_phase.push_back(phase);
        d->ev_launches.push_back(launches);
        h = hipEventRecord(e, s);
        return h == hipSuccess ? LAGP_OK : hip_fail("hipEventRecord", h);
    };
    for (const Chunk& c : P.chunks) {
        std::string err;
        const int64_t launches = (int64_t)c.buckets.size();
        int r = mark(-1, 0);
        if (r) return r;
        const double* xx = XX + c.t0 * p;
        r = lagp::knn_run(d->dev, xx, c.T, P.Mmax, ncand_per ? ncand_per + c.t0 : nullptr, cand, P.Mmax, false,
                          knn_ws, P.knn_b, s, d->num_cu, d->max_lds, &err, graph_safe);
        if (r) return fail(r == -1 ? LAGP_E_INVAL : LAGP_E_HIP, err);
        if ((r = mark(LAGP_PHASE_KNN, 0))) return r;
        lagp::DesignLaunch L;
        L.XX = xx;
        L.cand = cand;
        L.cand_stride = P.Mmax;
        L.n_per = n_per ? n_per + c.t0 : nullptr;
        L.M_per = ncand_per ? ncand_per + c.t0 : nullptr;
        L.n0 = P.prm.n0;
        L.theta = P.prm.d;
        L.theta_per = d_per ? d_per + c.t0 : nullptr;
        if (th && th->start) {
            L.start = th->start + c.t0 * th->start_stride;
            L.start_stride = th->start_stride;
            L.start_n = th->start_n ? th->start_n + c.t0 : nullptr;
        }
        L.vratio = th ? th->vratio : 0.0;
        L.eta = P.prm.g;
        L.mean = o.mean + c.t0;
        L.s2 = o.s2 + c.t0;
        L.df = o.df ? o.df + c.t0 : nullptr;
        L.var = o.var ? o.var + c.t0 : nullptr;
        L.sel = o.sel ? o.sel + c.t0 * o.sel_stride : (P.own_sel ? sel_ws : nullptr);
        L.sel_stride = o.sel ? o.sel_stride : P.nmax;
        L.status = o.status ? o.status + c.t0 : (P.own_status ? st_ws + c.t0 : nullptr);
        if (!P.alc2) {
            r = enqueue_designs(d, P, c, L, order_dev, des_ws, redo_list, redo_count, s);
            if (r) return r;
            if ((r = mark(LAGP_PHASE_DESIGN, launches))) return r;
        } else {
            // Section 4.2, one repetition: designs at theta0, the local MLE
            // theta1, designs at theta1, the local MLE theta2 (started from
            // theta1), and the prediction from the second designs at theta2.
            double* th1 = (th && th->d1) ? th->d1 + c.t0 : th1_ws;
            double* th2 = (th && th->d2) ? th->d2 + c.t0 : th2_ws;
            lagp::DesignLaunch S = L;
            S.mean = st_mean;
            S.s2 = st_s2;
            S.df = nullptr;
            S.var = nullptr;
            S.status = st_status;
            S.sel = sel1_ws;
            S.sel_stride = P.nmax;
            r = enqueue_designs(d, P, c, S, order_dev, des_ws, redo_list, redo_count, s);
            if (r) return r;
            if ((r = mark(LAGP_PHASE_DESIGN, launches))) return r;
            lagp::MleArgs m;
            m.Xaos = d->dev.Xaos;
            m.y = d->dev.y;
            m.p = p;
            m.N = d->dev.N;
            m.T = c.T;
            m.sel = sel1_ws;
            m.sel_stride = P.nmax;
            m.n_per = L.n_per;
            m.n = P.prm.n;
            m.nmax = c.nmax;
            m.theta0_per = L.theta_per;
            m.theta0 = P.prm.d;
            m.eta = P.prm.g;
            m.tmin = P.mle.tmin;
            m.tmax = P.mle.tmax;
            m.maxit = P.mle.maxit;
            m.tol = P.mle.tol;
            m.theta_out = th1;
            if ((r = mle_by_bucket(m, c, order_dev, d->max_lds, s))) return r;
            if ((r = mark(LAGP_PHASE_MLE, 0))) return r;
            S.theta_per = th1;
            S.sel = L.sel;
            S.sel_stride = L.sel_stride;
            r = enqueue_designs(d, P, c, S, order_dev, des_ws, redo_list, redo_count, s);
            if (r) return r;
            if ((r = mark(LAGP_PHASE_DESIGN, launches))) return r;
            m.sel = L.sel;
            m.sel_stride = L.sel_stride;
            m.theta0_per = th1;
            m.theta_out = th2;
            if ((r = mle_by_bucket(m, c, order_dev, d->max_lds, s))) return r;
            if ((r = mark(LAGP_PHASE_MLE, 0))) return r;
            r = lagp::predict_run(d->dev, xx, c.T, L.sel, L.sel_stride, L.n_per, c.nmax, P.prm.d, th2, P.prm.g, L.mean,
                                  L.s2, L.df, L.var, L.status, d->max_lds, s, &err);
            if (r) return fail(r == -1 ? LAGP_E_INVAL : LAGP_E_HIP, err);
            if ((r = mark(LAGP_PHASE_PREDICT, 0))) return r;
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail("launch", e);
    return LAGP_OK;
}

int check_outputs(const Outputs& o, int32_t nmax)
{
    if (!o.mean || !o.s2) return fail(LAGP_E_INVAL, "mean and s2 are required");
    if (o.sel && o.sel_stride < nmax) return fail(LAGP_E_INVAL, "sel_stride must be >= n");
    const void* devptrs[] = {o.mean, o.s2, o.df, o.var, o.sel, o.status};
    for (const void* q : devptrs)
        if (q && !is_device_ptr(q)) return fail(LAGP_E_INVAL, "array arguments must be device pointers");
    return LAGP_OK;
}

}  // namespace lagp_rt

struct lagp_batch {
    lagp_design* design = nullptr;
    Plan plan;
    bool have_sel = false, have_status = false;
    char* mem = nullptr;          // workspace, then the work list and size arrays
    int32_t* order = nullptr;
    int32_t* n_per = nullptr;
    int32_t* ncand_per = nullptr;
    hipStream_t cap = nullptr;    // capture stream
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void* key[8] = {};      // pointers the captured graph was recorded with
};

extern "C" {

int lagp_workspace_bytes(const lagp_design* design, int64_t T, int32_t nmax, int32_t ncand_max, size_t* out)
{
    if (!design || !out) return fail(LAGP_E_INVAL, "NULL argument");
    if (T < 0 || nmax < 1 || ncand_max < nmax) return fail(LAGP_E_INVAL, "bad sizes");
    lagp_params prm = {1, nmax, ncand_max, 1.0, 0.0, 0, 0};
    if (ncand_max > design->dev.N) return fail(LAGP_E_INVAL, "ncand above N");
    Plan P;
    int rc = build_plan(design, &prm, std::max<int64_t>(T, 1), nullptr, nullptr, true, true, &P);
    if (rc) return rc;
    *out = P.total;
    return LAGP_OK;
}

}  // extern "C"

// lagp_predict, lagp_predict_theta and lagp_predict_alc2 (mle non-null).
static int run_predict(const lagp_design* design, const double* XX, int64_t T, const lagp_params* prm,
                       const ThetaIO& th, const lagp_mle_params* mle, const int32_t* n_per, const int32_t* ncand_per,
                       double* mean, double* s2, int32_t* df, double* var, int32_t* sel, int64_t sel_stride,
                       int8_t* status, void* stream)
{
    if (!design || !prm) return fail(LAGP_E_INVAL, "design or params is NULL");
    if (T < 0) return fail(LAGP_E_INVAL, "T < 0");
    if (mle) {
        int rc = check_mle_params(mle);
        if (rc) return rc;
    }
    if (T == 0) {
        Plan P;
        return build_plan(design, prm, 0, nullptr, nullptr, true, true, &P);
    }
    if (!XX || !mean || !s2) return fail(LAGP_E_INVAL, "XX, mean and s2 are required");
    int rc = check_device(design);
    if (rc) return rc;
    const void* devptrs[] = {XX, n_per, ncand_per, th.d_per, th.d1, th.d2, th.start, th.start_n};
    for (const void* q : devptrs)
        if (q && !is_device_ptr(q)) return fail(LAGP_E_INVAL, "array arguments must be device pointers");
    if (!(th.vratio >= 0.0) || !isfinite(th.vratio)) return fail(LAGP_E_INVAL, "vratio must be >= 0 and finite");
    if (th.vratio > 0.0 && !df) return fail(LAGP_E_INVAL, "the stopping rule reports each design size in df: df is required");
    if (th.start_n && !th.start) return fail(LAGP_E_INVAL, "start_n without start");
    const Outputs o = {mean, s2, df, var, sel, sel_stride, status};
    hipStream_t s = (hipStream_t)stream;

    // Per-location sizes come to the host for checking and bucketing.
    std::vector<int32_t> hn(n_per ? T : 0), hm(ncand_per ? T : 0);
    if (n_per || ncand_per) {
        hipError_t e = hipSuccess;
        if (n_per) e = hipMemcpyAsync(hn.data(), n_per, T * sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess && ncand_per)
            e = hipMemcpyAsync(hm.data(), ncand_per, T * sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail("per-location size copy", e);
    }
    Plan P;
    rc = build_plan(design, prm, T, n_per ? hn.data() : nullptr, ncand_per ? hm.data() : nullptr, sel != nullptr,
                    status != nullptr, &P);
    if (rc) return rc;
    if (th.start) {
        // saved starting designs: sizes in [1, n] per location, read from start_stride columns
        int32_t smax = prm->n0;
        if (th.start_n) {
            std::vector<int32_t> hs(T);
            hipError_t e = hipMemcpyAsync(hs.data(), th.start_n, T * sizeof(int32_t), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) return hip_fail("start size copy", e);
            smax = 0;
            for (int64_t t = 0; t < T; ++t) {
                const int32_t nt = n_per ? hn[t] : prm->n;
                if (hs[t] < 1 || hs[t] > nt)
                    return fail(LAGP_E_INVAL, "location " + std::to_string(t) + ": need 1 <= start size <= n");
                smax = std::max(smax, hs[t]);
            }
        }
        if (th.start_stride < smax) return fail(LAGP_E_INVAL, "start_stride must be >= the largest start size");
    }
    rc = check_outputs(o, P.nmax);
    if (rc) return rc;
    if (mle) {
        rc = plan_alc2(design, mle, sel != nullptr, &P);
        if (rc) return rc;
    }
    lagp_design* d = const_cast<lagp_design*>(design);
    rc = ensure_ws(d, P.total, s);
    if (rc) return rc;
    rc = prepare_plan(d, P);
    if (rc) return rc;
    int32_t* order_dev = nullptr;
    if (P.uneven) {
        order_dev = (int32_t*)((char*)d->ws + P.knn_b + P.cand_b + P.design_b);
        hipError_t e = hipMemcpyAsync(order_dev, P.order.data(), T * sizeof(int32_t), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);   // P.order is released on return
        if (e != hipSuccess) return hip_fail("work list copy", e);
    }
    rc = enqueue_plan(d, P, (char*)d->ws, order_dev, n_per, ncand_per, XX, o, s, false, d->timing, &th);
    if (rc) return rc;
    if (prm->flags & LAGP_STRICT) {
        if (!status) return fail(LAGP_E_INVAL, "strict mode needs the status output");
        std::vector<int8_t> hs(T);
        hipError_t e = hipMemcpyAsync(hs.data(), status, T, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail("status copy", e);
        for (int8_t v : hs)
            if (v != LAGP_LOC_OK) return fail(LAGP_E_NOTPD, "some location's local covariance was not positive definite");
    }
    return LAGP_OK;
}

extern "C" {

int lagp_predict(const lagp_design* design, const double* XX, int64_t T, const lagp_params* prm,
                 const int32_t* n_per, const int32_t* ncand_per, double* mean, double* s2, int32_t* df, double* var,
                 int32_t* sel, int64_t sel_stride, int8_t* status, void* stream)
{
    return run_predict(design, XX, T, prm, ThetaIO{}, nullptr, n_per, ncand_per, mean, s2, df, var, sel, sel_stride,
                       status, stream);
}

int lagp_predict_ex(const lagp_design* design, const double* XX, int64_t T, const lagp_params* prm,
                    const lagp_options* opt, const int32_t* n_per, const int32_t* ncand_per, double* mean, double* s2,
                    int32_t* df, double* var, int32_t* sel, int64_t sel_stride, int8_t* status, void* stream)
{
    ThetaIO th;
    if (opt) {
        th.d_per = opt->d_per;
        th.start = opt->start;
        th.start_stride = opt->start_stride;
        th.start_n = opt->start_n;
        th.vratio = opt->vratio;
    }
    return run_predict(design, XX, T, prm, th, nullptr, n_per, ncand_per, mean, s2, df, var, sel, sel_stride, status,
                       stream);
}

int lagp_predict_theta(const lagp_design* design, const double* XX, int64_t T, const lagp_params* prm,
                       const double* d_per, const int32_t* n_per, const int32_t* ncand_per, double* mean, double* s2,
                       int32_t* df, double* var, int32_t* sel, int64_t sel_stride, int8_t* status, void* stream)
{
    if (!d_per && T > 0) return fail(LAGP_E_INVAL, "d_per is required");
    ThetaIO th;
    th.d_per = d_per;
    return run_predict(design, XX, T, prm, th, nullptr, n_per, ncand_per, mean, s2, df, var, sel, sel_stride, status,
                       stream);
}

int lagp_predict_alc2(const lagp_design* design, const double* XX, int64_t T, const lagp_params* prm,
                      const lagp_mle_params* mle, const double* d_per, const int32_t* n_per,
                      const int32_t* ncand_per, double* mean, double* s2, int32_t* df, double* var, int32_t* sel,
                      int64_t sel_stride, int8_t* status, double* d1, double* d2, void* stream)
{
    if (!mle) return fail(LAGP_E_INVAL, "MLE parameters are NULL");
    ThetaIO th;
    th.d_per = d_per;
    th.d1 = d1;
    th.d2 = d2;
    return run_predict(design, XX, T, prm, th, mle, n_per, ncand_per, mean, s2, df, var, sel, sel_stride, status,
                       stream);
}

int lagp_predict_mspe(const lagp_design* design, const double* XX, int64_t T, const lagp_params* prm,
                      const int32_t* n_per, const int32_t* ncand_per, double* mean, double* s2, int32_t* df,
                      double* var, int32_t* sel, int64_t sel_stride, int8_t* status, void* stream)
{
    if (!design || !prm) return fail(LAGP_E_INVAL, "design or params is NULL");
    if (T < 0) return fail(LAGP_E_INVAL, "T < 0");
    const int64_t N = design->dev.N;
    if (!(prm->d > 0.0) || !isfinite(prm->d)) return fail(LAGP_E_INVAL, "lengthscale d must be positive and finite");
    if (!(prm->g >= 0.0) || !isfinite(prm->g)) return fail(LAGP_E_INVAL, "nugget g must be >= 0 and finite");
    if (prm->precision != LAGP_PREC_FP64) return fail(LAGP_E_INVAL, "the MSPE criterion runs in FP64 only");
    if (prm->flags & ~(uint32_t)LAGP_STRICT) return fail(LAGP_E_INVAL, "unknown flag");
    if (prm->n0 < 3) return fail(LAGP_E_INVAL, "the MSPE criterion needs n0 >= 3 (it scales by j - 2)");
    if (T == 0) return LAGP_OK;
    if (!XX || !mean || !s2) return fail(LAGP_E_INVAL, "XX, mean and s2 are required");
    int rc = check_device(design);
    if (rc) return rc;
    const void* devptrs[] = {XX, n_per, ncand_per};
    for (const void* q : devptrs)
        if (q && !is_device_ptr(q)) return fail(LAGP_E_INVAL, "array arguments must be device pointers");
    lagp_design* d = const_cast<lagp_design*>(design);
    hipStream_t s = (hipStream_t)stream;
    // per-location sizes come to the host for checking
    std::vector<int32_t> hn(n_per ? T : 0), hm(ncand_per ? T : 0);
    if (n_per || ncand_per) {
        hipError_t e = hipSuccess;
        if (n_per) e = hipMemcpyAsync(hn.data(), n_per, T * sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess && ncand_per)
            e = hipMemcpyAsync(hm.data(), ncand_per, T * sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail("per-location size copy", e);
    }
    int32_t nmax = 0, Mmax = 0;
    for (int64_t t = 0; t < T; ++t) {
        const int32_t nt = n_per ? hn[t] : prm->n, mt = ncand_per ? hm[t] : prm->ncand;
        if (nt < prm->n0 || mt < nt || mt > N)
            return fail(LAGP_E_INVAL, "location " + std::to_string(t) + ": need n0 <= n <= ncand <= N");
        nmax = std::max(nmax, nt);
        Mmax = std::max(Mmax, mt);
        if (!n_per && !ncand_per) break;
    }
    if (Mmax > 2048) return fail(LAGP_E_INVAL, "the MSPE kernel takes at most 2048 candidates");
    if (lagp::mspe_lds_bytes(nmax, design->dev.p) > design->max_lds)
        return fail(LAGP_E_INVAL, "n too large for the MSPE kernel");
    const Outputs o = {mean, s2, df, var, sel, sel_stride, status};
    rc = check_outputs(o, nmax);
    if (rc) return rc;
    const int p = d->dev.p;
    const int64_t tc_max = std::min(kChunk, T);
    const int blocks = (int)std::min<int64_t>(tc_max, d->num_cu);
    const size_t knn_b = lagp::align256(lagp::knn_workspace_bytes(tc_max, lagp::KNN_BUCKET_MAX));
    const size_t cand_b = lagp::align256((size_t)tc_max * Mmax * sizeof(int32_t));
    const size_t slab = lagp::align256(lagp::mspe_slab_bytes(nmax, Mmax, p));
    const size_t total = knn_b + cand_b + 256 + (size_t)blocks * slab;
    rc = ensure_ws(d, total, s);
    if (rc) return rc;
    std::string err;
    if (lagp::knn_prepare(p, d->max_lds, &err)) return fail(LAGP_E_HIP, err);
    int r = lagp::mspe_prepare(nmax, Mmax, p, d->max_lds, &err);
    if (r) return fail(r == -1 ? LAGP_E_INVAL : LAGP_E_HIP, err);
    char* q = (char*)d->ws;
    void* knn_ws = q;
    int32_t* cand = (int32_t*)(q + knn_b);
    unsigned int* counter = (unsigned int*)(q + knn_b + cand_b);
    double* scratch = (double*)(q + knn_b + cand_b + 256);
    auto mark = [&](int phase) {
        if (!d->timing) return;
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return;
        d->ev.push_back(e);
        d->ev_phase.push_back(phase);
        d->ev_launches.push_back(phase == LAGP_PHASE_DESIGN ? 1 : 0);
        (void)hipEventRecord(e, s);
    };
    for (int64_t t0 = 0; t0 < T; t0 += kChunk) {
        const int64_t tc = std::min(kChunk, T - t0);
        const double* xx = XX + t0 * p;
        const int32_t* mp = ncand_per ? ncand_per + t0 : nullptr;
        mark(-1);
        r = lagp::knn_run(d->dev, xx, tc, Mmax, mp, cand, Mmax, false, knn_ws, knn_b, s, d->num_cu, d->max_lds, &err);
        if (r) return fail(r == -1 ? LAGP_E_INVAL : LAGP_E_HIP, err);
        mark(LAGP_PHASE_KNN);
        lagp::MspeArgs a;
        a.Xaos = d->dev.Xaos;
        a.y = d->dev.y;
        a.p = p;
        a.XX = xx;
        a.T = tc;
        a.cand = cand;
        a.cand_stride = Mmax;
        a.n_per = n_per ? n_per + t0 : nullptr;
        a.M_per = mp;
        a.n0 = prm->n0;
        a.n = prm->n;
        a.M = Mmax;
        a.nmax = nmax;
        a.theta = prm->d;
        a.eta = prm->g;
        a.mean = mean + t0;
        a.s2 = s2 + t0;
        a.df = df ? df + t0 : nullptr;
        a.var = var ? var + t0 : nullptr;
        a.sel = sel ? sel + t0 * sel_stride : nullptr;
        a.sel_stride = sel_stride;
        a.status = status ? status + t0 : nullptr;
        a.scratch = scratch;
        a.scratch_stride = (int64_t)(slab / sizeof(double));
        a.counter = counter;
        r = lagp::mspe_run(a, (int)std::min<int64_t>(tc, blocks), d->max_lds, s, &err);
        if (r) return fail(r == -1 ? LAGP_E_INVAL : LAGP_E_HIP, err);
        mark(LAGP_PHASE_DESIGN);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail("launch", e);
    if (prm->flags & LAGP_STRICT) {
        if (!status) return fail(LAGP_E_INVAL, "strict mode needs the status output");
        std::vector<int8_t> hs(T);
        e = hipMemcpyAsync(hs.data(), status, T, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail("status copy", e);
        for (int8_t v : hs)
            if (v != LAGP_LOC_OK) return fail(LAGP_E_NOTPD, "some location's local covariance was not positive definite");
    }
    return LAGP_OK;
}

int lagp_mle(const lagp_design* design, int64_t T, const int32_t* sel, int64_t sel_stride, const int32_t* n_per,
             int32_t n, const double* d0_per, double d0, double g, const lagp_mle_params* mle, double* d_hat,
             int32_t* iters, int8_t* status, void* stream)
{
    if (!design) return fail(LAGP_E_INVAL, "design is NULL");
    if (T < 0) return fail(LAGP_E_INVAL, "T < 0");
    int rc = check_mle_params(mle);
    if (rc) return rc;
    if (!d0_per && (!(d0 > 0.0) || !isfinite(d0))) return fail(LAGP_E_INVAL, "lengthscale d0 must be positive and finite");
    if (!(g >= 0.0) || !isfinite(g)) return fail(LAGP_E_INVAL, "nugget g must be >= 0 and finite");
    if (T == 0) return LAGP_OK;
    if (!sel || !d_hat) return fail(LAGP_E_INVAL, "sel and d_hat are required");
    const void* devptrs[] = {sel, n_per, d0_per, d_hat, iters, status};
    for (const void* q : devptrs)
        if (q && !is_device_ptr(q)) return fail(LAGP_E_INVAL, "array arguments must be device pointers");
    rc = check_device(design);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    int32_t nmax = n;
    if (n_per) {
        std::vector<int32_t> hn(T);
        hipError_t e = hipMemcpyAsync(hn.data(), n_per, T * sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail("per-location size copy", e);
        nmax = 0;
        for (int64_t t = 0; t < T; ++t) {
            if (hn[t] < 2) return fail(LAGP_E_INVAL, "every n must be >= 2");
            nmax = std::max(nmax, hn[t]);
        }
    }
    if (nmax < 2) return fail(LAGP_E_INVAL, "n must be >= 2");
    if (sel_stride < nmax) return fail(LAGP_E_INVAL, "sel_stride must be >= n");
    if (T > INT32_MAX) return fail(LAGP_E_INVAL, "T above 2^31 - 1");
    std::string err;
    int r = lagp::mle_prepare(nmax, design->dev.p, design->max_lds, &err);
    if (r) return fail(r == -1 ? LAGP_E_INVAL : LAGP_E_HIP, err);
    lagp::MleArgs m;
    m.Xaos = design->dev.Xaos;
    m.y = design->dev.y;
    m.p = design->dev.p;
    m.N = design->dev.N;
    m.T = T;
    m.sel = sel;
    m.sel_stride = sel_stride;
    m.n_per = n_per;
    m.n = n;
    m.nmax = nmax;
    m.theta0_per = d0_per;
    m.theta0 = d0;
    m.eta = g;
    m.tmin = mle->tmin;
    m.tmax = mle->tmax;
    m.maxit = mle->maxit;
    m.tol = mle->tol;
    m.theta_out = d_hat;
    m.iters = iters;
    m.status = status;
    r = lagp::mle_run(m, design->max_lds, s, &err);
    if (r) return fail(r == -1 ? LAGP_E_INVAL : LAGP_E_HIP, err);
    return LAGP_OK;
}

// ---------------------------------------------------------------- batches
int lagp_batch_create(const lagp_design* design, int64_t T, const lagp_params* prm, const int32_t* n_per,
                      const int32_t* ncand_per, uint32_t flags, lagp_batch** out)
{
    if (!out) return fail(LAGP_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!design || !prm) return fail(LAGP_E_INVAL, "design or params is NULL");
    if (T < 1) return fail(LAGP_E_INVAL, "T must be >= 1");
    if (prm->flags & LAGP_STRICT) return fail(LAGP_E_INVAL, "strict mode needs a host synchronisation; use lagp_predict");
    if (flags & ~(LAGP_BATCH_SEL | LAGP_BATCH_STATUS)) return fail(LAGP_E_INVAL, "unknown flag");
    int rc = check_device(design);
    if (rc) return rc;
    if ((n_per && is_device_ptr(n_per)) || (ncand_per && is_device_ptr(ncand_per)))
        return fail(LAGP_E_INVAL, "n_per and ncand_per must be host arrays");
    lagp_batch* b = new lagp_batch();
    b->design = const_cast<lagp_design*>(design);
    b->have_sel = flags & LAGP_BATCH_SEL;
    b->have_status = flags & LAGP_BATCH_STATUS;
    rc = build_plan(design, prm, T, n_per, ncand_per, b->have_sel, b->have_status, &b->plan);
    if (rc) { delete b; return rc; }
    const Plan& P = b->plan;
    const size_t sizes_b = lagp::align256((size_t)T * sizeof(int32_t));
    const size_t bytes = P.total + (n_per ? sizes_b : 0) + (ncand_per ? sizes_b : 0);
    hipError_t e = hipMalloc(&b->mem, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete b;
        return fail(LAGP_E_NOMEM, "batch workspace allocation of " + std::to_string(bytes) + " bytes failed");
    }
    char* q = b->mem + P.total;
    if (P.uneven) b->order = (int32_t*)(b->mem + P.knn_b + P.cand_b + P.design_b);
    if (n_per) { b->n_per = (int32_t*)q; q += sizes_b; }
    if (ncand_per) { b->ncand_per = (int32_t*)q; q += sizes_b; }
    e = hipSuccess;
    if (P.uneven) e = hipMemcpy(b->order, P.order.data(), T * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess && n_per) e = hipMemcpy(b->n_per, n_per, T * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess && ncand_per)
        e = hipMemcpy(b->ncand_per, ncand_per, T * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e != hipSuccess) { lagp_batch_destroy(b); return hip_fail("batch set-up", e); }
    rc = prepare_plan(design, P);
    if (rc) { lagp_batch_destroy(b); return rc; }
    *out = b;
    return LAGP_OK;
}

void lagp_batch_destroy(lagp_batch* b)
{
    if (!b) return;
    if (b->cap) (void)hipStreamSynchronize(b->cap);
    (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->mem) (void)hipFree(b->mem);
    delete b;
}

int lagp_batch_info(const lagp_batch* b, int32_t* buckets, size_t* workspace_bytes)
{
    if (!b) return fail(LAGP_E_INVAL, "batch is NULL");
    if (buckets) {
        int32_t n = 0;
        for (const Chunk& c : b->plan.chunks) n += (int32_t)c.buckets.size();
        *buckets = n;
    }
    if (workspace_bytes) *workspace_bytes = b->plan.total;
    return LAGP_OK;
}

static int batch_args(const lagp_batch* b, const double* XX, const Outputs& o)
{
    if (!b) return fail(LAGP_E_INVAL, "batch is NULL");
    if (!XX || !is_device_ptr(XX)) return fail(LAGP_E_INVAL, "XX must be a device pointer");
    if ((o.sel != nullptr) != b->have_sel) return fail(LAGP_E_INVAL, "sel must be given exactly when the batch was created with LAGP_BATCH_SEL");
    if ((o.status != nullptr) != b->have_status)
        return fail(LAGP_E_INVAL, "status must be given exactly when the batch was created with LAGP_BATCH_STATUS");
    int rc = check_device(b->design);
    if (rc) return rc;
    return check_outputs(o, b->plan.nmax);
}

int lagp_batch_enqueue(lagp_batch* b, const double* XX, double* mean, double* s2, int32_t* df, double* var,
                       int32_t* sel, int64_t sel_stride, int8_t* status, void* stream)
{
    const Outputs o = {mean, s2, df, var, sel, sel_stride, status};
    int rc = batch_args(b, XX, o);
    if (rc) return rc;
    return enqueue_plan(b->design, b->plan, b->mem, b->order, b->n_per, b->ncand_per, XX, o, (hipStream_t)stream,
                        true, false);
}

int lagp_batch_launch_graph(lagp_batch* b, const double* XX, double* mean, double* s2, int32_t* df, double* var,
                            int32_t* sel, int64_t sel_stride, int8_t* status, void* stream)
{
    const Outputs o = {mean, s2, df, var, sel, sel_stride, status};
    int rc = batch_args(b, XX, o);
    if (rc) return rc;
    const void* key[8] = {XX, mean, s2, df, var, sel, (const void*)(intptr_t)sel_stride, status};
    if (!b->exec || memcmp(key, b->key, sizeof key) != 0) {
        if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
        if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
        hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail("hipStreamBeginCapture", e);
        rc = enqueue_plan(b->design, b->plan, b->mem, b->order, b->n_per, b->ncand_per, XX, o, b->cap, true, false);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(b->cap, &g);
        if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
        if (e != hipSuccess) return hip_fail("hipStreamEndCapture", e);
        b->graph = g;
        e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) { b->exec = nullptr; return hip_fail("hipGraphInstantiate", e); }
        memcpy(b->key, key, sizeof key);
    }
    hipError_t e = hipGraphLaunch(b->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail("hipGraphLaunch", e);
    return LAGP_OK;
}

int lagp_design_set_variant(lagp_design* d, int32_t threads, int32_t coords)
{
    if (!d) return fail(LAGP_E_INVAL, "design is NULL");
    if (threads != 0 && threads != 256 && threads != 512) return fail(LAGP_E_INVAL, "threads must be 0, 256 or 512");
    if (coords < -1 || coords > 1) return fail(LAGP_E_INVAL, "coords must be -1, 0 or 1");
    d->force_threads = threads;
    d->force_coords = coords;
    d->force_lds_pct = -1;
    return LAGP_OK;
}

int lagp_design_set_variant_ex(lagp_design* d, int32_t threads, int32_t coords, int32_t lds_rows_pct)
{
    if (lds_rows_pct < -1 || lds_rows_pct > 100) return fail(LAGP_E_INVAL, "lds_rows_pct must be -1 or in [0, 100]");
    const int rc = lagp_design_set_variant(d, threads, coords);
    if (rc) return rc;
    d->force_lds_pct = lds_rows_pct;
    return LAGP_OK;
}

int lagp_predict_designs(const lagp_design* design, const double* XX, int64_t T, const int32_t* sel,
                         int64_t sel_stride, const int32_t* n_per, int32_t n, double dlen, const double* d_per,
                         double g, double* mean, double* s2, int32_t* df, double* var, int8_t* status, void* stream)
{
    if (!design) return fail(LAGP_E_INVAL, "design is NULL");
    if (T < 0) return fail(LAGP_E_INVAL, "T < 0");
    if (!d_per && (!(dlen > 0.0) || !isfinite(dlen)))
        return fail(LAGP_E_INVAL, "lengthscale d must be positive and finite");
    if (!(g >= 0.0) || !isfinite(g)) return fail(LAGP_E_INVAL, "nugget g must be >= 0 and finite");
    if (T == 0) return LAGP_OK;
    if (!XX || !sel || !mean || !s2) return fail(LAGP_E_INVAL, "XX, sel, mean and s2 are required");
    const void* devptrs[] = {XX, sel, mean, s2, df, var, status, n_per, d_per};
    for (const void* q : devptrs)
        if (q && !is_device_ptr(q)) return fail(LAGP_E_INVAL, "array arguments must be device pointers");
    int rc = check_device(design);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    int32_t nmax = n;
    if (n_per) {
        std::vector<int32_t> hn(T);
        hipError_t e = hipMemcpyAsync(hn.data(), n_per, T * sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail("per-location size copy", e);
        nmax = 0;
        for (int64_t t = 0; t < T; ++t) {
            if (hn[t] < 1) return fail(LAGP_E_INVAL, "every n must be >= 1");
            nmax = std::max(nmax, hn[t]);
        }
    }
    if (nmax < 1) return fail(LAGP_E_INVAL, "n must be >= 1");
    if (sel_stride < nmax) return fail(LAGP_E_INVAL, "sel_stride must be >= n");
    std::string err;
    int r = lagp::predict_prepare(nmax, design->max_lds, &err);
    if (r) return fail(r == -1 ? LAGP_E_INVAL : LAGP_E_HIP, err);
    r = lagp::predict_run(design->dev, XX, T, sel, sel_stride, n_per, nmax, dlen, d_per, g, mean, s2, df, var, status,
                          design->max_lds, s, &err);
    if (r) return fail(r == -1 ? LAGP_E_INVAL : LAGP_E_HIP, err);
    return LAGP_OK;
}

int lagp_timing_enable(lagp_design* d, int enable)
{
    if (!d) return fail(LAGP_E_INVAL, "design is NULL");
    d->timing = enable != 0;
    return LAGP_OK;
}

int lagp_phase_times(lagp_design* d, double* ms, int64_t* design_launches)
{
    if (!d) return fail(LAGP_E_INVAL, "design is NULL");
    double sum[LAGP_PHASES] = {};
    int64_t n = 0;
    int rc = LAGP_OK;
    if (!d->ev.empty()) {
        hipError_t e = hipEventSynchronize(d->ev.back());
        if (e != hipSuccess) rc = hip_fail("hipEventSynchronize", e);
    }
    for (size_t k = 1; rc == LAGP_OK && k < d->ev.size(); ++k) {
        const int ph = d->ev_phase[k];
        if (ph < 0) continue;
        float x = 0.f;
        if (hipEventElapsedTime(&x, d->ev[k - 1], d->ev[k]) != hipSuccess) {
            rc = fail(LAGP_E_HIP, "hipEventElapsedTime failed");
            break;
        }
        sum[ph] += x;
        n += d->ev_launches[k];
    }
    for (hipEvent_t e : d->ev) (void)hipEventDestroy(e);
    d->ev.clear();
    d->ev_phase.clear();
    d->ev_launches.clear();
    if (rc) return rc;
    if (ms)
        for (int k = 0; k < LAGP_PHASES; ++k) ms[k] = sum[k];
    if (design_launches) *design_launches = n;
    return LAGP_OK;
}

}  // extern "C"
