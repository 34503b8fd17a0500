// lagp_internal.h -- declarations shared by the host runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

namespace lagp {

// Raise a kernel's dynamic-LDS limit to what the device allows next to the
// kernel's static LDS.  The limit is the device's rather than one launch's, so
// that every launch of the kernel (eager or in a captured graph) fits.
// With dyn_bytes > 0 it also checks that a launch with that much dynamic
// LDS fits next to the static part (a launch that does not fit aborts the
// queue).
inline bool set_lds_limit(const void* kernel, size_t max_lds, size_t dyn_bytes = 0)
{
    hipFuncAttributes fa;
    if (hipFuncGetAttributes(&fa, kernel) != hipSuccess) return false;
    if (fa.sharedSizeBytes >= max_lds) return false;
    if (fa.sharedSizeBytes + dyn_bytes > max_lds) return false;
    return hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(max_lds - fa.sharedSizeBytes)) == hipSuccess;
}

// Device-resident design: row-major coordinates (read a row at a time by the
// kNN scans and gathered by the other kernels), responses, and a strided
// row sample for the kNN's radius estimate.
struct DeviceDesign {
    const double* Xaos = nullptr;  // N x p
    const double* y = nullptr;     // N
    int64_t N = 0;
    int32_t p = 0;
    // Every KNN_SAMPLE_STRIDE-th design row, Ns x p row-major (the kNN
    // estimates each location's candidate radius on it); nullptr when not built.
    const double* Xaos_s = nullptr;
    int64_t Ns = 0;
};

constexpr int KNN_SAMPLE_STRIDE = 16;
// Keys a location's final kNN window may hold (sorted in LDS by one block).
constexpr int32_t KNN_BUCKET_MAX = 512;

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Dispatch a macro on the input dimension: compile-time 1..8, runtime otherwise.
#define LAGP_DISPATCH_P(pval, MACRO) \
    switch (pval) {                  \
    case 1: MACRO(1); break;         \
    case 2: MACRO(2); break;         \
    case 3: MACRO(3); break;         \
    case 4: MACRO(4); break;         \
    case 5: MACRO(5); break;         \
    case 6: MACRO(6); break;         \
    case 7: MACRO(7); break;         \
    case 8: MACRO(8); break;         \
    default: MACRO(0); break;        \
    }

// ---- nearest neighbours (knn.hip)
size_t knn_workspace_bytes(int64_t T, int32_t bucket_max);
// Returns 0, or <0 with *err set.  Row t of idx receives the M (or M_per[t])
// nearest design rows, unordered unless `sorted` (uniform M only).
int knn_run(const DeviceDesign& D, const double* XX, int64_t T, int32_t M, const int32_t* M_per,
            int32_t* idx, int64_t idx_stride, bool sorted, void* ws, size_t ws_bytes, hipStream_t stream,
            int num_cu, size_t max_lds, std::string* err, bool graph_safe = false);
// Host-side set-up of the kNN kernels for dimension p (dynamic LDS limits).
int knn_prepare(int p, size_t max_lds, std::string* err);
void fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);

// ---- greedy local design + prediction (design.hip)
struct DesignLaunch {
    // inputs
    const double* XX = nullptr;  // T x p
    int64_t T = 0;
    const int32_t* cand = nullptr;  // T x cand_stride (unordered candidate sets)
    int64_t cand_stride = 0;
    const int32_t* n_per = nullptr;
    const int32_t* M_per = nullptr;
    int32_t n0 = 0, n = 0, M = 0;  // uniform values (maxima when per-location arrays are given)
    double theta = 1.0, eta = 0.0;
    const double* theta_per = nullptr;  // nullable: per-location lengthscale (replaces theta)
    const int32_t* start = nullptr;     // nullable: saved starting designs (replace the n0 nearest)
    int64_t start_stride = 0;
    const int32_t* start_n = nullptr;   // nullable: per-location starting-design size (else n0)
    double vratio = 0.0;                // > 0: variance-ratio stopping threshold
    int32_t precision = 0;
    const int32_t* order = nullptr;   // work item -> location (nullable: identity over T)
    const uint32_t* count = nullptr;  // device-side item count (nullable: T items)
    // outputs
    double* mean = nullptr;
    double* s2 = nullptr;
    int32_t* df = nullptr;
    double* var = nullptr;
    int32_t* sel = nullptr;
    int64_t sel_stride = 0;
    int8_t* status = nullptr;
};

struct DesignPlan {
    int threads = 0;       // workgroup size (input: 256 or 512 preferred)
    int coords_pref = -1;  // input: -1 traffic model, 0 coordinates in global memory, 1 in LDS when they fit
    int lds_pct = 100;     // input: percent of the LDS left after the fixed part that holds tile rows
    int p = 0;
    int cpt = 0;           // candidate slots per thread
    int rreg = 0;          // register-resident tile rows
    int rlds = 0;          // LDS-resident tile rows
    int rglob = 0;         // global-resident tile rows
    bool coords_lds = false;
    bool y_lds = false;    // responses in LDS next to the coordinates
    int blocks = 0;        // persistent grid size
    size_t lds_bytes = 0;
    size_t lds_limit = 0;  // device LDS per workgroup
    size_t scratch_per_block = 0;  // bytes of global scratch per block
    size_t counter_bytes = 0;
    long long global_row_reads = 0;  // modelled candidate-row reads from global memory per location
    bool mix = false;                // FP32 or BF16 ranking tile with an exact re-score
    bool bf16 = false;               // BF16 tile storage
    bool trim = false;               // variant that skips empty slot columns
};

// Mmin: the smallest candidate-set size among the locations the plan will run.
int design_plan(const DeviceDesign& D, int32_t nmax, int32_t Mmax, int32_t Mmin, int32_t n0, int32_t precision,
                int num_cu, size_t max_lds, DesignPlan* plan, std::string* err);
size_t design_workspace_bytes(const DesignPlan& plan);
// Host-side set-up of the plan's kernel variant (dynamic LDS limit); call
// before design_run, outside any stream capture.
int design_prepare(const DesignPlan& plan, std::string* err);
// Enqueues the persistent design kernel (a fill kernel resets its work
// counter first); no allocation, no host synchronisation.
int design_run(const DeviceDesign& D, const DesignLaunch& L, const DesignPlan& plan, void* ws,
               size_t ws_bytes, hipStream_t stream, std::string* err);

// ---- prediction from given local designs (predict.hip)
size_t predict_lds_bytes(int nmax);
int predict_prepare(int32_t nmax, size_t max_lds, std::string* err);
// theta_per (nullable) gives each location its own lengthscale.
int predict_run(const DeviceDesign& D, const double* XX, int64_t T, const int32_t* sel, int64_t sel_stride,
                const int32_t* n_per, int32_t nmax, double theta, const double* theta_per, double eta, double* mean,
                double* s2, int32_t* df, double* var, int8_t* status, size_t max_lds, hipStream_t stream,
                std::string* err);

// ---- local maximum-likelihood lengthscale of given designs (mle.hip)
struct MleArgs {
    const double* Xaos = nullptr;   // design, N x p row-major
    const double* y = nullptr;
    int p = 0;
    int64_t N = 0;
    int64_t T = 0;                  // locations this launch processes (the grid)
    // nullable: the locations to process, T entries indexing the per-location
    // arrays below (else locations 0 .. T-1)
    const int32_t* order = nullptr;
    const int32_t* sel = nullptr;   // local design indices, sel_stride per location
    int64_t sel_stride = 0;
    const int32_t* n_per = nullptr; // nullable: per-location design size
    int n = 0;                      // uniform design size
    int nmax = 0;                   // largest design size of the processed locations (sizes LDS)
    const double* theta0_per = nullptr;   // nullable: per-location starting lengthscale
    double theta0 = 1.0;
    double eta = 0.0;
    double tmin = 0.0, tmax = 0.0;  // search interval
    int maxit = 0;
    double tol = 0.0;
    double* theta_out = nullptr;    // per location: the estimate (NaN where the design failed)
    int32_t* iters = nullptr;       // nullable: Newton iterates taken
    int8_t* status = nullptr;       // nullable: 0 OK, 1 failed
};
size_t mle_lds_bytes(int nmax, int p, int threads);

// ---- greedy MSPE local designs (mspe.hip)
struct MspeArgs {
    const double* Xaos = nullptr;
    const double* y = nullptr;
    int p = 0;
    const double* XX = nullptr;     // T x p
    int64_t T = 0;
    const int32_t* cand = nullptr;  // T x cand_stride candidate sets
    int64_t cand_stride = 0;
    const int32_t* n_per = nullptr; // nullable: per-location design size (else n)
    const int32_t* M_per = nullptr; // nullable: per-location candidate count (else M)
    int n0 = 0, n = 0, M = 0, nmax = 0;   // M: the largest candidate count (sizes the slab)
    double theta = 1.0, eta = 0.0;
    double* mean = nullptr;
    double* s2 = nullptr;
    int32_t* df = nullptr;
    double* var = nullptr;
    int32_t* sel = nullptr;
    int64_t sel_stride = 0;
    int8_t* status = nullptr;
    double* scratch = nullptr;      // blocks x scratch_stride doubles
    int64_t scratch_stride = 0;
    unsigned int* counter = nullptr;
    int lds_rows = 0;               // leading tile rows kept in LDS (set by mspe_run)
};
size_t mspe_lds_bytes(int nmax, int p);
size_t mspe_slab_bytes(int nmax, int Mmax, int p);
int mspe_prepare(int32_t nmax, int32_t Mmax, int p, size_t max_lds, std::string* err);
int mspe_run(const MspeArgs& a, int blocks, size_t max_lds, hipStream_t stream, std::string* err);
int mle_prepare(int32_t nmax, int p, size_t max_lds, std::string* err);
int mle_run(const MleArgs& a, size_t max_lds, hipStream_t stream, std::string* err);

}  // namespace lagp
