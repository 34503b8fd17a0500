// noalloc.hip -- lagp_predict_noalloc: lagp_predict with uniform sizes for
// callers that cannot allocate device memory.
//
// The workspace (candidate sets, kNN state, the design kernel's work counter
// and per-workgroup tile slabs, the mixed mode's own selection and status
// arrays) comes from one fixed device array defined here.  Each device gets
// its own copy of the array when the library's code object is loaded there;
// its device address is looked up once per device with hipGetSymbolAddress and
// kept, and only that address is handed to kernels.  Locations run in chunks
// small enough for the chunk's workspace to fit the array.  Nothing here
// allocates device memory: no hipMalloc, no hipFree, no allocating library
// call.  Every kernel initialises the workspace it reads (fill kernels for
// counters, init kernels for the kNN state), so contents left by an earlier
// call never matter; calls that overlap on one device share the array and
// race.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "lagp_runtime.h"

// Bytes of the static workspace (LAGP_NOALLOC_SCRATCH_BYTES in lagp.h).
constexpr size_t kScratchBytes = (size_t)256 << 20;

// In host code `scratch` names a host-side stand-in: only the address
// returned by hipGetSymbolAddress is valid on the device.
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch_dev[kMaxDevices] = {};

// The device address of this device's copy of `scratch`, looked up on the
// first call with that device current.
int scratch_address(int device, void** out)
{
    if (device < 0 || device >= kMaxDevices) return lagp_rt::fail(LAGP_E_NODEVICE, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_dev[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return lagp_rt::hip_fail("hipGetSymbolAddress(scratch)", e);
        }
        g_scratch_dev[device] = ptr;
    }
    *out = g_scratch_dev[device];
    return LAGP_OK;
}

}  // namespace

using namespace lagp_rt;

extern "C" {

size_t lagp_noalloc_scratch_bytes(void) { return kScratchBytes; }

int lagp_predict_noalloc(const lagp_design* design, const double* XX, int64_t T, const lagp_params* prm,
                         double* mean, double* s2, int32_t* df, double* var, int32_t* sel, int64_t sel_stride,
                         int8_t* status, void* stream)
{
    if (!design || !prm) return fail(LAGP_E_INVAL, "design or params is NULL");
    if (T < 0) return fail(LAGP_E_INVAL, "T < 0");
    if (prm->flags) return fail(LAGP_E_INVAL, "lagp_predict_noalloc takes no flags (strict mode needs a host wait)");
    if (T == 0) {
        Plan P;
        return build_plan(design, prm, 0, nullptr, nullptr, true, true, &P);
    }
    if (!XX || !mean || !s2) return fail(LAGP_E_INVAL, "XX, mean and s2 are required");
    int rc = check_device(design);
    if (rc) return rc;
    if (!is_device_ptr(XX)) return fail(LAGP_E_INVAL, "array arguments must be device pointers");
    const Outputs o = {mean, s2, df, var, sel, sel_stride, status};
    // The largest chunk whose workspace fits the array: halve from the
    // default until it does.
    Plan P;
    int64_t chunk = std::min<int64_t>(T, kChunk);
    for (;;) {
        P = Plan();
        rc = build_plan(design, prm, T, nullptr, nullptr, sel != nullptr, status != nullptr, &P, chunk);
        if (rc) return rc;
        if (P.total <= kScratchBytes) break;
        if (chunk == 1)
            return fail(LAGP_E_BUDGET, "one location needs " + std::to_string(P.total) +
                                           " bytes of workspace, more than the " + std::to_string(kScratchBytes) +
                                           "-byte static scratch of lagp_predict_noalloc");
        chunk = (chunk + 1) / 2;
    }
    rc = check_outputs(o, P.nmax);
    if (rc) return rc;
    lagp_design* d = const_cast<lagp_design*>(design);
    rc = prepare_plan(d, P);
    if (rc) return rc;
    void* ws = nullptr;
    rc = scratch_address(d->device, &ws);
    if (rc) return rc;
    // graph_safe: the kNN runs its fixed pass budget without host waits.
    return enqueue_plan(d, P, (char*)ws, nullptr, nullptr, nullptr, XX, o, (hipStream_t)stream, true, false, nullptr);
}

}  // extern "C"
