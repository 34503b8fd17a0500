// lagp_runtime.h -- internal host runtime shared by the entry points in
// lagp_api.cpp and the serving engine in server.cpp: the device-resident
// design, error reporting, and the batch planner (per-location size checks,
// size buckets, longest-first work lists, kernel-variant choice, workspace
// layout) with its capture-safe launch sequence.
#pragma once
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "lagp.h"
#include "lagp_internal.h"

struct lagp_design {
    lagp::DeviceDesign dev;
    int device = 0;
    int num_cu = 0;
    size_t max_lds = 0;
    double* Xaos_s = nullptr;   // strided sample of the design rows, row-major
    double* Xaos = nullptr;
    double* y = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    bool timing = false;
    // Phase timing: events on the launch stream; ev_phase[k] names the phase
    // of the interval that ends at ev[k] (LAGP_PHASE_*; -1 starts a chunk),
    // ev_launches[k] the design-kernel launches in it.
    std::vector<hipEvent_t> ev;
    std::vector<int> ev_phase;
    std::vector<int64_t> ev_launches;
    std::string arch;                   // e.g. "gfx950"
    int force_threads = 0;              // kernel-variant override (0: table or model)
    int force_coords = -1;
    int force_lds_pct = -1;             // -1: table (else all of the LDS left)
    // Streams and events that run the size buckets of an uneven plan in
    // concurrent lanes (lane 0 is the caller's stream); created outside
    // capture by prepare_plan, guarded by lane_mu while a plan forks.
    static constexpr int kLanes = 3;
    hipStream_t lane_stream[kLanes - 1] = {};
    hipEvent_t lane_fork = nullptr;
    hipEvent_t lane_join[kLanes - 1] = {};
    std::mutex lane_mu;
};

namespace lagp_rt {

const int64_t kChunk = (int64_t)1 << 17;   // locations per launch sequence

int fail(int code, const std::string& msg);
int hip_fail(const char* what, hipError_t e);
bool is_device_ptr(const void* p);
int check_device(const lagp_design* d);

struct Bucket {
    int32_t nmax = 0, Mmax = 0, Mmin = 1 << 30;
    int64_t first = 0, count = 0;   // range of the chunk's work list
    lagp::DesignPlan plan;
    int lane = 0;                   // concurrent lane (stream) the bucket runs in
};

struct Chunk {
    int64_t t0 = 0, T = 0;
    int32_t nmax = 0, Mmax = 0, Mmin = 1 << 30;
    std::vector<Bucket> buckets;
    int lanes = 1;                  // lanes in use (1: every bucket on the caller's stream)
    lagp::DesignPlan redo;   // FP64 plan for locations the mixed mode could not finish
};

struct Plan {
    lagp_params prm{};
    int64_t T = 0;
    int64_t chunk = kChunk;       // locations per launch sequence
    int32_t nmax = 0, Mmax = 0;
    int32_t nmin = 0;             // smallest design size
    bool uneven = false, mix = false, own_sel = false, own_status = false;
    bool alc2 = false;            // two-stage scheme with local lengthscale inference
    lagp_mle_params mle{};
    std::vector<Chunk> chunks;
    std::vector<int32_t> order;   // chunk-relative locations, chunk c at [t0, t0 + T)
    // workspace layout
    size_t knn_b = 0, cand_b = 0, design_b = 0, order_b = 0, sel_b = 0, status_b = 0, redo_b = 0;
    size_t lane_b = 0;            // design workspace per lane (design_b = lanes x lane_b)
    size_t sel1_b = 0, stage_b = 0;   // two-stage: first designs; stage outputs and lengthscales
    size_t total = 0;
};

// Optional inputs and outputs of the extended entry points.
struct ThetaIO {
    const double* d_per = nullptr;  // device T: per-location lengthscale (first design pass)
    double* d1 = nullptr;           // two-stage outputs, device T (nullable)
    double* d2 = nullptr;
    const int32_t* start = nullptr; // device T x start_stride: saved starting designs
    int64_t start_stride = 0;
    const int32_t* start_n = nullptr;   // device T: starting-design sizes (else params->n0)
    double vratio = 0.0;            // variance-ratio stopping threshold (0: off)
};

struct Outputs {
    double* mean;
    double* s2;
    int32_t* df;
    double* var;
    int32_t* sel;
    int64_t sel_stride;
    int8_t* status;
};

// Checks parameters and per-location sizes (host arrays, nullable) and builds
// the plan for T locations.
// `chunk` bounds the locations per launch sequence (and so the workspace).
// `lanes` bounds the concurrent lanes of an uneven plan's size buckets.
int build_plan(const lagp_design* d, const lagp_params* prm, int64_t T, const int32_t* hn, const int32_t* hm,
               bool have_sel, bool have_status, Plan* P, int64_t chunk = kChunk,
               int lanes = lagp_design::kLanes);
// Turns a plan into the two-stage scheme: checks the search controls and
// n >= 2, and adds the stage workspace.  have_sel: the caller passes sel.
int plan_alc2(const lagp_design* d, const lagp_mle_params* mle, bool have_sel, Plan* P);
// Host-side kernel set-up for every variant the plan launches (outside capture).
int prepare_plan(const lagp_design* d, const Plan& P);
// Enqueues the plan on stream s: kernel launches only.  ws holds P.total
// bytes; order_dev is the uploaded work list of an uneven plan; n_per and
// ncand_per are device arrays (nullable for uniform sizes).
// With `timing` the phases are bracketed by HIP events kept on the design.
int enqueue_plan(lagp_design* d, const Plan& P, char* ws, const int32_t* order_dev, const int32_t* n_per,
                 const int32_t* ncand_per, const double* XX, const Outputs& o, hipStream_t s, bool graph_safe,
                 bool timing, const ThetaIO* th = nullptr);
int check_mle_params(const lagp_mle_params* mle);
int check_outputs(const Outputs& o, int32_t nmax);

}  // namespace lagp_rt
