// lagp_api.cpp -- host runtime behind include/lagp.h: argument checks, the
// device-resident design, the workspace pool and the launch sequence
// (candidate sets, then greedy local designs with prediction) in chunks of
// locations.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "lagp.h"
#include "lagp_internal.h"

using lagp::DeviceDesign;

struct lagp_design {
    DeviceDesign dev;
    int device = 0;
    int num_cu = 0;
    size_t max_lds = 0;
    double* Xsoa = nullptr;
    double* Xaos = nullptr;
    double* y = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    bool timing = false;
    std::vector<hipEvent_t> ev;   // triples: before kNN, after kNN, after design
};

namespace {

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

__global__ void aos_to_soa_kernel(const double* __restrict__ aos, double* __restrict__ soa, int64_t N, int p)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= N * p) return;
    int64_t i = e / p;
    int k = (int)(e - i * p);
    soa[(int64_t)k * N + i] = aos[e];
}

// Rows idx[0..m-1] of src (row length w) into dst (m x w).
template <typename T>
__global__ void gather_rows_kernel(const T* __restrict__ src, int64_t w, const int64_t* __restrict__ idx, int64_t m,
                                   T* __restrict__ dst)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m * w) return;
    int64_t r = e / w, c = e - r * w;
    dst[e] = src[idx[r] * w + c];
}

// Rows of src (m x w) back to rows idx[r] of dst (row stride dstride >= w).
template <typename T>
__global__ void scatter_rows_kernel(const T* __restrict__ src, int64_t w, const int64_t* __restrict__ idx, int64_t m,
                                    T* __restrict__ dst, int64_t dstride)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m * w) return;
    int64_t r = e / w, c = e - r * w;
    dst[idx[r] * dstride + c] = src[e];
}

template <typename T>
void gather_rows(const T* src, int64_t w, const int64_t* idx, int64_t m, T* dst, hipStream_t s)
{
    if (m * w == 0) return;
    hipLaunchKernelGGL(gather_rows_kernel<T>, dim3((unsigned)((m * w + 255) / 256)), dim3(256), 0, s, src, w, idx, m,
                       dst);
}

template <typename T>
void scatter_rows(const T* src, int64_t w, const int64_t* idx, int64_t m, T* dst, int64_t dstride, hipStream_t s)
{
    if (m * w == 0 || !dst) return;
    hipLaunchKernelGGL(scatter_rows_kernel<T>, dim3((unsigned)((m * w + 255) / 256)), dim3(256), 0, s, src, w, idx,
                       m, dst, dstride);
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

const int64_t kChunk = (int64_t)1 << 17;   // locations per launch sequence
const int32_t kBucketMax = 512;

}  // namespace

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
    d->max_lds = prop.sharedMemPerBlock;
    const size_t bytes = (size_t)N * p * sizeof(double);
    if (hipMalloc(&d->Xaos, bytes) != hipSuccess || hipMalloc(&d->Xsoa, bytes) != hipSuccess ||
        hipMalloc(&d->y, (size_t)N * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        lagp_design_destroy(d);
        return fail(LAGP_E_NOMEM, "design allocation failed");
    }
    const hipMemcpyKind kind = host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    e = hipMemcpyAsync(d->Xaos, X, bytes, kind, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d->y, y, (size_t)N * sizeof(double), kind, s);
    if (e != hipSuccess) { lagp_design_destroy(d); return hip_fail("design copy", e); }
    const int64_t tot = N * p;
    hipLaunchKernelGGL(aos_to_soa_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, d->Xaos,
                       d->Xsoa, N, p);
    e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) { lagp_design_destroy(d); return hip_fail("design layout", e); }
    d->dev.Xaos = d->Xaos;
    d->dev.Xsoa = d->Xsoa;
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
    if (d->Xaos) (void)hipFree(d->Xaos);
    if (d->Xsoa) (void)hipFree(d->Xsoa);
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
        rc = ensure_ws(d, lagp::knn_workspace_bytes(tc, kBucketMax), s);
        if (rc) return rc;
        std::string err;
        int r = lagp::knn_run(d->dev, XX + t0 * d->dev.p, tc, M, nullptr, idx + t0 * idx_stride, idx_stride, true,
                              d->ws, d->ws_bytes, s, d->num_cu, d->max_lds, &err);
        if (r) return fail(r == -1 ? LAGP_E_INVAL : LAGP_E_HIP, err);
    }
    return LAGP_OK;
}

static int plan_for(const lagp_design* d, int32_t nmax, int32_t Mmax, const lagp_params* prm, int64_t tc,
                    lagp::DesignPlan* plan, size_t* knn_bytes, size_t* cand_bytes, size_t* design_bytes)
{
    std::string err;
    const char* thr = getenv("LAGP_DESIGN_THREADS");
    plan->threads = (thr && atoi(thr) == 512) ? 512 : 256;
    if (lagp::design_plan(d->dev, nmax, Mmax, prm->n0, prm->precision, d->num_cu, d->max_lds, plan, &err))
        return fail(LAGP_E_INVAL, err);
    *knn_bytes = lagp::align256(lagp::knn_workspace_bytes(tc, kBucketMax));
    *cand_bytes = lagp::align256((size_t)tc * Mmax * sizeof(int32_t));
    *design_bytes = lagp::align256(lagp::design_workspace_bytes(*plan));
    return LAGP_OK;
}

int lagp_workspace_bytes(const lagp_design* design, int64_t T, int32_t nmax, int32_t ncand_max, size_t* out)
{
    if (!design || !out) return fail(LAGP_E_INVAL, "NULL argument");
    if (T < 0 || nmax < 1 || ncand_max < nmax) return fail(LAGP_E_INVAL, "bad sizes");
    lagp_params prm = {1, nmax, ncand_max, 1.0, 0.0, 0, 0};
    lagp::DesignPlan plan;
    size_t a, b, c;
    int rc = plan_for(design, nmax, ncand_max, &prm, std::min(kChunk, std::max<int64_t>(T, 1)), &plan, &a, &b, &c);
    if (rc) return rc;
    *out = a + b + c;
    return LAGP_OK;
}

int lagp_predict(const lagp_design* design, const double* XX, int64_t T, const lagp_params* prm,
                 const int32_t* n_per, const int32_t* ncand_per, double* mean, double* s2, int32_t* df, double* var,
                 int32_t* sel, int64_t sel_stride, int8_t* status, void* stream);

// Re-run the locations `idx` in FP64 and scatter their outputs back.
static int redo_fp64(lagp_design* d, const double* XX, const lagp_params* prm, const int32_t* n_per,
                     const int32_t* ncand_per, const std::vector<int64_t>& idx, int32_t nmax, double* mean, double* s2,
                     int32_t* df, double* var, int32_t* sel, int64_t sel_stride, int8_t* status, hipStream_t s)
{
    const int64_t m = (int64_t)idx.size();
    const int p = d->dev.p;
    size_t bytes = lagp::align256(m * sizeof(int64_t)) + lagp::align256(m * p * sizeof(double)) +
                   2 * lagp::align256(m * sizeof(int32_t)) + 3 * lagp::align256(m * sizeof(double)) +
                   lagp::align256(m * sizeof(int32_t)) + lagp::align256(m * nmax * sizeof(int32_t)) +
                   lagp::align256(m);
    char* buf = nullptr;
    hipError_t e = hipMalloc(&buf, bytes);
    if (e != hipSuccess) { (void)hipGetLastError(); return fail(LAGP_E_NOMEM, "FP64 redo buffer allocation failed"); }
    char* q = buf;
    auto take = [&](size_t b) { char* r = q; q += lagp::align256(b); return r; };
    int64_t* di = (int64_t*)take(m * sizeof(int64_t));
    double* xx = (double*)take(m * p * sizeof(double));
    int32_t* np_ = (int32_t*)take(m * sizeof(int32_t));
    int32_t* mp_ = (int32_t*)take(m * sizeof(int32_t));
    double* me = (double*)take(m * sizeof(double));
    double* sc = (double*)take(m * sizeof(double));
    double* va = (double*)take(m * sizeof(double));
    int32_t* dfo = (int32_t*)take(m * sizeof(int32_t));
    int32_t* so = (int32_t*)take(m * nmax * sizeof(int32_t));
    int8_t* sto = (int8_t*)take(m);
    int rc = LAGP_OK;
    e = hipMemcpyAsync(di, idx.data(), m * sizeof(int64_t), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) { rc = hip_fail("redo index copy", e); goto done; }
    gather_rows<double>(XX, p, di, m, xx, s);
    if (n_per) gather_rows<int32_t>(n_per, 1, di, m, np_, s);
    if (ncand_per) gather_rows<int32_t>(ncand_per, 1, di, m, mp_, s);
    {
        lagp_params q64 = *prm;
        q64.precision = LAGP_PREC_FP64;
        q64.flags = 0;
        rc = lagp_predict(d, xx, m, &q64, n_per ? np_ : nullptr, ncand_per ? mp_ : nullptr, me, sc, dfo, va, so, nmax,
                          sto, s);
    }
    if (rc) goto done;
    scatter_rows<double>(me, 1, di, m, mean, 1, s);
    scatter_rows<double>(sc, 1, di, m, s2, 1, s);
    scatter_rows<double>(va, 1, di, m, var, 1, s);
    scatter_rows<int32_t>(dfo, 1, di, m, df, 1, s);
    scatter_rows<int8_t>(sto, 1, di, m, status, 1, s);
    scatter_rows<int32_t>(so, nmax, di, m, sel, sel_stride, s);
    e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) rc = hip_fail("FP64 redo", e);
done:
    (void)hipStreamSynchronize(s);
    (void)hipFree(buf);
    return rc;
}

int lagp_predict(const lagp_design* design, const double* XX, int64_t T, const lagp_params* prm,
                 const int32_t* n_per, const int32_t* ncand_per, double* mean, double* s2, int32_t* df, double* var,
                 int32_t* sel, int64_t sel_stride, int8_t* status, void* stream)
{
    if (!design || !prm) return fail(LAGP_E_INVAL, "design or params is NULL");
    if (T < 0) return fail(LAGP_E_INVAL, "T < 0");
    const int64_t N = design->dev.N;
    if (!(prm->d > 0.0) || !isfinite(prm->d)) return fail(LAGP_E_INVAL, "lengthscale d must be positive and finite");
    if (!(prm->g >= 0.0) || !isfinite(prm->g)) return fail(LAGP_E_INVAL, "nugget g must be >= 0 and finite");
    if (prm->precision != LAGP_PREC_FP64 && prm->precision != LAGP_PREC_SCORE_FP32)
        return fail(LAGP_E_INVAL, "unsupported precision mode");
    if (prm->flags & ~(uint32_t)LAGP_STRICT) return fail(LAGP_E_INVAL, "unknown flag");
    if (prm->n0 < 1) return fail(LAGP_E_INVAL, "n0 must be >= 1");
    if (!n_per && (prm->n < prm->n0)) return fail(LAGP_E_INVAL, "n must be >= n0");
    if (!ncand_per && (prm->ncand < 1 || prm->ncand > N)) return fail(LAGP_E_INVAL, "ncand must be in [1, N]");
    if (!n_per && !ncand_per && prm->ncand < prm->n) return fail(LAGP_E_INVAL, "ncand must be >= n");
    if (T == 0) return LAGP_OK;
    if (!XX || !mean || !s2) return fail(LAGP_E_INVAL, "XX, mean and s2 are required");
    int rc = check_device(design);
    if (rc) return rc;
    const void* devptrs[] = {XX, mean, s2, df, var, sel, status, n_per, ncand_per};
    for (const void* q : devptrs)
        if (q && !is_device_ptr(q)) return fail(LAGP_E_INVAL, "array arguments must be device pointers");
    hipStream_t s = (hipStream_t)stream;

    // Per-location sizes: validate on the host and take maxima.
    int32_t nmax = prm->n, Mmax = prm->ncand;
    if (n_per || ncand_per) {
        std::vector<int32_t> hn(n_per ? T : 0), hm(ncand_per ? T : 0);
        hipError_t e = hipSuccess;
        if (n_per) e = hipMemcpyAsync(hn.data(), n_per, T * sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess && ncand_per)
            e = hipMemcpyAsync(hm.data(), ncand_per, T * sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail("per-location size copy", e);
        nmax = 0;
        Mmax = 0;
        for (int64_t t = 0; t < T; ++t) {
            const int32_t nt = n_per ? hn[t] : prm->n;
            const int32_t mt = ncand_per ? hm[t] : prm->ncand;
            if (nt < prm->n0 || mt < nt || mt > N)
                return fail(LAGP_E_INVAL, "location " + std::to_string(t) + ": need n0 <= n <= ncand <= N");
            nmax = std::max(nmax, nt);
            Mmax = std::max(Mmax, mt);
        }
    }
    if (Mmax > 4096) return fail(LAGP_E_INVAL, "ncand above 4096 is not supported");
    if (nmax > 1024) return fail(LAGP_E_INVAL, "n above 1024 is not supported");
    if (sel && sel_stride < nmax) return fail(LAGP_E_INVAL, "sel_stride must be >= n");

    lagp_design* d = const_cast<lagp_design*>(design);
    const int64_t tc_max = std::min(kChunk, T);
    lagp::DesignPlan plan;
    size_t kb, cb, db;
    rc = plan_for(d, nmax, Mmax, prm, tc_max, &plan, &kb, &cb, &db);
    if (rc) return rc;
    const bool mix = prm->precision == LAGP_PREC_SCORE_FP32;
    if (mix && lagp::predict_lds_bytes(nmax) > d->max_lds)
        return fail(LAGP_E_INVAL, "n too large for the FP64 prediction kernel of the mixed mode");
    // The mixed mode needs the selections for its FP64 prediction pass.
    const size_t sb = (mix && !sel) ? lagp::align256((size_t)tc_max * nmax * sizeof(int32_t)) : 0;
    // ... and the per-location status to find locations to redo in FP64.
    const size_t stb = (mix && !status) ? lagp::align256((size_t)T) : 0;
    if (getenv("LAGP_VERBOSE"))
        fprintf(stderr,
                "[lagp] plan: n=%d ncand=%d p=%d threads=%d slots/thread=%d rows: reg=%d lds=%d global=%d "
                "coords_lds=%d lds=%zu B global_row_reads/loc=%lld workspace=%zu B\n",
                nmax, Mmax, d->dev.p, plan.threads, plan.cpt, plan.rreg, plan.rlds, plan.rglob,
                (int)plan.coords_lds, plan.lds_bytes, plan.global_row_reads, kb + cb + db + sb);
    rc = ensure_ws(d, kb + cb + db + sb + stb, s);
    if (rc) return rc;
    char* base = (char*)d->ws;
    void* knn_ws = base;
    int32_t* cand = (int32_t*)(base + kb);
    void* des_ws = base + kb + cb;
    int32_t* sel_ws = sb ? (int32_t*)(base + kb + cb + db) : nullptr;
    int8_t* st_all = status ? status : (stb ? (int8_t*)(base + kb + cb + db + sb) : nullptr);

    for (int64_t t0 = 0; t0 < T; t0 += kChunk) {
        const int64_t tc = std::min(kChunk, T - t0);
        std::string err;
        hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
        if (d->timing) {
            for (int k = 0; k < 3; ++k) {
                hipError_t e = hipEventCreate(&ev[k]);
                if (e != hipSuccess) return hip_fail("hipEventCreate", e);
                d->ev.push_back(ev[k]);
            }
            (void)hipEventRecord(ev[0], s);
        }
        int r = lagp::knn_run(d->dev, XX + t0 * d->dev.p, tc, Mmax, ncand_per ? ncand_per + t0 : nullptr, cand,
                              Mmax, false, knn_ws, kb, s, d->num_cu, d->max_lds, &err);
        if (r) return fail(r == -1 ? LAGP_E_INVAL : LAGP_E_HIP, err);
        if (d->timing) (void)hipEventRecord(ev[1], s);
        lagp::DesignLaunch L;
        L.XX = XX + t0 * d->dev.p;
        L.T = tc;
        L.cand = cand;
        L.cand_stride = Mmax;
        L.n_per = n_per ? n_per + t0 : nullptr;
        L.M_per = ncand_per ? ncand_per + t0 : nullptr;
        L.n0 = prm->n0;
        L.n = nmax;
        L.M = Mmax;
        L.theta = prm->d;
        L.eta = prm->g;
        L.precision = prm->precision;
        L.mean = mean + t0;
        L.s2 = s2 + t0;
        L.df = df ? df + t0 : nullptr;
        L.var = var ? var + t0 : nullptr;
        L.sel = sel ? sel + t0 * sel_stride : sel_ws;
        L.sel_stride = sel ? sel_stride : nmax;
        L.status = st_all ? st_all + t0 : nullptr;
        r = lagp::design_run(d->dev, L, plan, des_ws, db, s, &err);
        if (r) return fail(r == -1 ? LAGP_E_INVAL : LAGP_E_HIP, err);
        if (mix) {
            r = lagp::predict_run(d->dev, L.XX, tc, L.sel, L.sel_stride, L.n_per, nmax, prm->d, prm->g, L.mean, L.s2,
                                  L.df, L.var, L.status, d->max_lds, s, &err);
            if (r) return fail(r == -1 ? LAGP_E_INVAL : LAGP_E_HIP, err);
        }
        if (d->timing) (void)hipEventRecord(ev[2], s);
    }
    if (mix) {
        // FP32 ranking can lose positive definiteness where FP64 keeps it (tiny
        // nuggets, near-duplicate neighbours): redo those locations in FP64.
        std::vector<int8_t> hs(T);
        hipError_t e = hipMemcpyAsync(hs.data(), st_all, T, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail("status copy", e);
        std::vector<int64_t> redo;
        for (int64_t t = 0; t < T; ++t)
            if (hs[t] != LAGP_LOC_OK) redo.push_back(t);
        if (!redo.empty()) {
            rc = redo_fp64(d, XX, prm, n_per, ncand_per, redo, nmax, mean, s2, df, var, sel, sel_stride, status, s);
            if (rc) return rc;
        }
    }
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

int lagp_predict_designs(const lagp_design* design, const double* XX, int64_t T, const int32_t* sel,
                         int64_t sel_stride, const int32_t* n_per, int32_t n, double dlen, double g, double* mean,
                         double* s2, int32_t* df, double* var, int8_t* status, void* stream)
{
    if (!design) return fail(LAGP_E_INVAL, "design is NULL");
    if (T < 0) return fail(LAGP_E_INVAL, "T < 0");
    if (!(dlen > 0.0) || !isfinite(dlen)) return fail(LAGP_E_INVAL, "lengthscale d must be positive and finite");
    if (!(g >= 0.0) || !isfinite(g)) return fail(LAGP_E_INVAL, "nugget g must be >= 0 and finite");
    if (T == 0) return LAGP_OK;
    if (!XX || !sel || !mean || !s2) return fail(LAGP_E_INVAL, "XX, sel, mean and s2 are required");
    const void* devptrs[] = {XX, sel, mean, s2, df, var, status, n_per};
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
    int r = lagp::predict_run(design->dev, XX, T, sel, sel_stride, n_per, nmax, dlen, g, mean, s2, df, var, status,
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

int lagp_phase_times(lagp_design* d, double* knn_ms, double* design_ms, int64_t* launches)
{
    if (!d) return fail(LAGP_E_INVAL, "design is NULL");
    double a = 0.0, b = 0.0;
    int64_t n = 0;
    for (size_t k = 0; k + 2 < d->ev.size() + 0; k += 3) {
        hipError_t e = hipEventSynchronize(d->ev[k + 2]);
        if (e != hipSuccess) return hip_fail("hipEventSynchronize", e);
        float x = 0.f, y = 0.f;
        if (hipEventElapsedTime(&x, d->ev[k], d->ev[k + 1]) != hipSuccess ||
            hipEventElapsedTime(&y, d->ev[k + 1], d->ev[k + 2]) != hipSuccess)
            return fail(LAGP_E_HIP, "hipEventElapsedTime failed");
        a += x;
        b += y;
        ++n;
    }
    for (hipEvent_t e : d->ev) (void)hipEventDestroy(e);
    d->ev.clear();
    if (knn_ms) *knn_ms = a;
    if (design_ms) *design_ms = b;
    if (launches) *launches = n;
    return LAGP_OK;
}

}  // extern "C"
