// design.hip -- plan and launch of the greedy-design kernel (the kernel
// itself is in design_kernel.h): tile-row placement across registers, LDS and
// global memory from a traffic model, workspace sizing, and dispatch to the
// compiled variant.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "design_kernel.h"

namespace lagp {

static int launch_any(const DesignArgs* a, const DesignPlan& plan, hipStream_t stream, std::string* err)
{
    if (plan.bf16) return plan.trim ? design_launch_bf16_trim(a, plan, stream, err) : design_launch_bf16(a, plan, stream, err);
    if (plan.mix) return plan.trim ? design_launch_mix_trim(a, plan, stream, err) : design_launch_mix(a, plan, stream, err);
    return plan.trim ? design_launch_f64_trim(a, plan, stream, err) : design_launch_f64(a, plan, stream, err);
}

// ------------------------------------------------------------------ plan
static size_t fixed_lds_bytes(int nmax, int p, int dt, bool mix)
{
    const int dw = dt / 64;
    const int nred = 2 * dw + (mix ? dw * (dw < 4 ? dw : 4) : 0);
    nmax = (nmax + 3) & ~3;
    size_t b = 0;
    b += (size_t)(3 * nmax + 2 * p + 1 + 4 + nred) * sizeof(double);
    b += (size_t)(2 * nred + nmax + 4) * sizeof(int);
    b = (b + 15) & ~(size_t)15;
    if (mix) {
        // exact factor (packed), delta, 1/delta, w_x, staged columns; slots, staged ids
        size_t m = (size_t)(packed_row(nmax) + 3 * nmax + dw * (nmax + 4)) * sizeof(double);
        m += (size_t)(nmax + 2 * dw) * sizeof(int);
        b += (m + 15) & ~(size_t)15;
    }
    return b;
}

// Global-memory row reads per location (in candidate rows) when rows
// [g0, nmax-2] live in global memory: row l is read at steps l+1 .. n-2.
static long long global_row_reads(int nmax, int g0)
{
    long long r = 0;
    for (int l = g0; l <= nmax - 2; ++l) r += (nmax - 2 - l);
    return r;
}

int design_plan(const DeviceDesign& D, int32_t nmax, int32_t Mmax, int32_t Mmin, int32_t n0, int32_t precision,
                int num_cu, size_t max_lds, DesignPlan* plan, std::string* err)
{
    (void)n0;
    const bool mix = precision != 0, bf16 = precision == 2;
    int dt = plan->threads == 512 ? 512 : 256;
    if (Mmax > 2048) dt = 512;   // at most 8 slots per thread
    int cpt = 1;
    while (cpt * dt < Mmax) cpt <<= 1;
    if (cpt * dt > 4096) { *err = "candidate-set size above 4096 is not supported"; return -1; }
    const int Mpad = cpt * dt;
    const int p = D.p;
    const int rows = nmax > 1 ? nmax - 1 : 0;  // W rows ever stored
    if (mix && nmax > 128) { *err = "the mixed precision mode supports n <= 128"; return -1; }
    const size_t fixed = fixed_lds_bytes(nmax, p, dt, mix);
    if (fixed > max_lds) { *err = "local design size too large for LDS"; return -1; }
    const size_t row_bytes = (size_t)Mpad * (bf16 ? 2 : mix ? sizeof(float) : sizeof(double));   // tile row
    const size_t crow_bytes = (size_t)Mpad * sizeof(double);                          // coordinate row
    const size_t avail = max_lds - fixed;
    // Option A: coordinates in LDS.  Option B: coordinates in global memory.
    // Cost: bytes read from global memory per location.  Either way a step
    // reads its one response from the design (LDS is worth more as tile rows).
    const int pcA = p, pc = p;
    // Trimmed variant when some location leaves a whole slot column empty.
    const bool trim = cpt > 1 && Mmin <= (cpt - 1) * dt;
    const int rregA = rreg_for(dt, cpt, true, mix, trim), rregB = rreg_for(dt, cpt, false, mix, trim);
    const int remA = rows > rregA ? rows - rregA : 0, remB = rows > rregB ? rows - rregB : 0;
    long long costA = -1, costB;
    int rldsA = 0;
    const int pct = std::max(0, std::min(100, plan->lds_pct));
    if (avail >= pcA * crow_bytes) {
        rldsA = std::min<long long>(remA, (avail - pcA * crow_bytes) / row_bytes * pct / 100);
        costA = global_row_reads(nmax, rregA + rldsA) * (long long)row_bytes;
    }
    const int rldsB = std::min<long long>(remB, avail / row_bytes * pct / 100);
    costB = (long long)pc * (nmax - 1) * (long long)crow_bytes + global_row_reads(nmax, rregB + rldsB) * (long long)row_bytes;
    bool cl = costA >= 0 && costA <= costB;
    if (plan->coords_pref == 0) cl = false;
    else if (plan->coords_pref == 1 && costA >= 0) cl = true;
    plan->cpt = cpt;
    plan->threads = dt;
    plan->p = p;
    plan->lds_limit = max_lds;
    plan->trim = trim;
    plan->mix = mix;
    plan->bf16 = bf16;
    plan->rreg = cl ? rregA : rregB;
    plan->rlds = cl ? rldsA : rldsB;
    plan->rglob = (cl ? remA : remB) - plan->rlds;
    plan->coords_lds = cl;
    plan->lds_bytes = fixed + (cl ? pcA * crow_bytes : 0) + (size_t)plan->rlds * row_bytes;
    plan->y_lds = false;
    plan->scratch_per_block = align256((cl ? 0 : pc * crow_bytes) + (size_t)plan->rglob * row_bytes);
    plan->blocks = num_cu;
    plan->counter_bytes = 256;
    plan->global_row_reads = (cl ? costA : costB) / (long long)row_bytes;
    return 0;
}

size_t design_workspace_bytes(const DesignPlan& plan)
{
    return plan.counter_bytes + plan.scratch_per_block * (size_t)plan.blocks;
}

int design_prepare(const DesignPlan& plan, std::string* err)
{
    return launch_any(nullptr, plan, nullptr, err);
}

int design_run(const DeviceDesign& D, const DesignLaunch& L, const DesignPlan& plan, void* ws,
               size_t ws_bytes, hipStream_t stream, std::string* err)
{
    if (L.T == 0) return 0;
    if (ws_bytes < design_workspace_bytes(plan)) { *err = "design workspace too small"; return -1; }
    DesignArgs a;
    a.Xaos = D.Xaos;
    a.y = D.y;
    a.p = D.p;
    a.XX = L.XX;
    a.T = L.T;
    a.cand = L.cand;
    a.cand_stride = L.cand_stride;
    a.n_per = L.n_per;
    a.M_per = L.M_per;
    a.n0 = L.n0;
    a.n = L.n;
    a.M = L.M;
    a.theta = L.theta;
    a.theta_per = L.theta_per;
    a.start = L.start;
    a.start_stride = L.start_stride;
    a.start_n = L.start_n;
    a.vratio = L.vratio;
    a.eta = L.eta;
    a.mean = L.mean;
    a.s2 = L.s2;
    a.df = L.df;
    a.var = L.var;
    a.sel = L.sel;
    a.sel_stride = L.sel_stride;
    a.status = L.status;
    a.counter = (unsigned int*)ws;
    a.scratch = (double*)((char*)ws + plan.counter_bytes);
    a.scratch_stride = (int64_t)(plan.scratch_per_block / sizeof(double));
    a.rlds = plan.rlds;
    a.coords_lds = plan.coords_lds ? 1 : 0;
    a.y_lds = plan.y_lds ? 1 : 0;
    a.nmax = L.n;
    a.order = L.order;
    a.count = L.count;
    fill_u32(a.counter, 1, 0u, stream);
    return launch_any(&a, plan, stream, err);
}

}  // namespace lagp
