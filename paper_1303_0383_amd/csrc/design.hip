// design.hip -- greedy ALC local design and local GP prediction on gfx950.
//
// One 256-thread workgroup owns one predictive location at a time and pulls
// the next location from a work counter (persistent kernel, Section 4.1's
// independent loop over locations).  Thread `tid` owns the candidate slots
// tid + k * 256, k < CPT.
//
// Algebra.  Write L_j for the Cholesky factor of K_j = K(X_j, X_j) + g I and
// keep the whitened tile W_j = L_j^{-1} K(X_j, C) over all candidates C, with
// w_x = L_j^{-1} k_j(x) and u = L_j^{-1} Y_j.  Then for every candidate c
//   v_j(c)     = 1 + g - ||W_j[:,c]||^2,
//   cov_j(x,c) = K(x,c) - w_x . W_j[:,c],
//   ALC_j(c)   = cov_j(x,c)^2 / v_j(c)            (eqs dxy / dxy2),
// and adding the chosen s appends one row to each of them:
//   delta = sqrt(v_j(s)),
//   r_c   = (K(s,c) - W_j[:,s] . W_j[:,c]) / delta  (row j of W),
//   r_x   = (K(s,x) - W_j[:,s] . w_x) / delta,  r_y = (y_s - W_j[:,s] . u) / delta,
//   v_{j+1}(c) = v_j(c) - r_c^2,  cov_{j+1}(x,c) = cov_j(x,c) - r_x r_c.
// This is the partitioned-inverse step of SM Section 1 written for the factor
// (the new last row of L_{j+1}^{-1} is [-(l/delta)' L_j^{-1}, 1/delta] with
// l = L_j^{-1} k_j(s)), carried to every candidate at once.  The chosen
// columns of W are the rows of L_n, so the final prediction
//   mean = w_x . u,  psi = u . u,  v_n(x) = 1 + g - w_x . w_x  (eqs predgp, preds2)
// needs no refactorisation.  Every dot product runs in ascending index
// order with separate multiply and subtract (the file is compiled with
// -ffp-contract=off), the same operation order as a row-by-row Cholesky
// factorisation and forward substitution.
//
// Storage of W (rows in selection order): the first RREG rows in registers
// (compile time), the next `rlds` rows in LDS, the rest in a per-workgroup
// global scratch slab.  Candidate coordinates live in LDS when they fit,
// else in the same slab.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "lagp_internal.h"

namespace lagp {

#define DT 256
#define DWAVES (DT / 64)

struct DesignArgs {
    const double* Xaos;
    const double* y;
    int p;
    const double* XX;
    int64_t T;
    const int32_t* cand;
    int64_t cand_stride;
    const int32_t* n_per;
    const int32_t* M_per;
    int n0, n, M;
    double theta, eta;
    double* mean;
    double* s2;
    int32_t* df;
    double* var;
    int32_t* sel;
    int64_t sel_stride;
    int8_t* status;
    double* scratch;
    int64_t scratch_stride;  // doubles per workgroup
    int rlds, coords_lds;
    int nmax;
    unsigned int* counter;
};

// Candidate ordering for the argmax: larger score first, then smaller index.
__device__ __forceinline__ bool better(double a, int ia, double b, int ib)
{
    return a > b || (a == b && ia < ib);
}
// Nearest-neighbour ordering: smaller squared distance first, then smaller index.
__device__ __forceinline__ bool nearer(double a, int ia, double b, int ib)
{
    return a < b || (a == b && ia < ib);
}

template <int P>
__device__ __forceinline__ double sqdist_lds(const double* __restrict__ a, const double* __restrict__ c,
                                             int cstride, int p)
{
    // a: uniform point (LDS/registers); c: candidate coordinates with stride cstride.
    double s = 0.0;
    if (P > 0) {
#pragma unroll
        for (int k = 0; k < P; ++k) {
            double t = a[k] - c[k * cstride];
            s += t * t;
        }
    } else {
        for (int k = 0; k < p; ++k) {
            double t = a[k] - c[k * cstride];
            s += t * t;
        }
    }
    return s;
}

template <int CPT, int RREG, int P>
__global__ void __launch_bounds__(DT, 1) design_kernel(const DesignArgs A)
{
    extern __shared__ double smem[];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int p = P > 0 ? P : A.p;
    const int nmax = A.nmax;
    const int Mpad = CPT * DT;
    const double theta = A.theta, eta = A.eta;
    const double one_eta = 1.0 + eta;

    // ---- LDS carve-up (doubles first, then ints)
    double* ws = smem;               // [nmax] column of the chosen candidate
    double* wx = ws + nmax;          // [nmax] L^{-1} k(x)
    double* uu = wx + nmax;          // [nmax] L^{-1} Y
    double* xl = uu + nmax;          // [p]    predictive location
    double* xsl = xl + p;            // [p]    chosen candidate
    double* misc = xsl + p;          // [4]    v_s, y_s
    double* redv = misc + 4;         // [2*DWAVES] per-wave best scores
    int* redi = (int*)(redv + 2 * DWAVES);  // [2*DWAVES] best design index
    int* reds = redi + 2 * DWAVES;          // [2*DWAVES] best slot
    int* forced = reds + 2 * DWAVES;        // [nmax] slots of the nearest neighbours
    int* ctl = forced + nmax;               // [4]  location, chosen index
    size_t off = (size_t)((char*)(ctl + 4) - (char*)smem);
    off = (off + 15) & ~(size_t)15;
    double* Xcl = (double*)((char*)smem + off);                // [p][Mpad] if coords in LDS
    double* Wl = Xcl + (A.coords_lds ? (size_t)p * Mpad : 0);  // [rlds][Mpad]

    double* Xcg = A.scratch + (int64_t)blockIdx.x * A.scratch_stride;
    double* Wg = Xcg + (A.coords_lds ? 0 : (int64_t)p * Mpad);
    double* Xc = A.coords_lds ? Xcl : Xcg;
    const int rlds = A.rlds;

    for (;;) {
        if (tid == 0) ctl[0] = (int)atomicAdd(A.counter, 1u);
        __syncthreads();
        const int64_t t = ctl[0];
        if (t >= A.T) break;
        const int n = A.n_per ? A.n_per[t] : A.n;
        const int M = A.M_per ? A.M_per[t] : A.M;
        const int n0 = A.n0;
        for (int k = tid; k < p; k += DT) xl[k] = A.XX[t * p + k];
        if (A.sel)
            for (int i = tid; i < n; i += DT) A.sel[t * A.sel_stride + i] = -1;
        __syncthreads();
        double xr[P > 0 ? P : 1];
        if (P > 0) {
#pragma unroll
            for (int k = 0; k < (P > 0 ? P : 1); ++k) xr[k] = xl[k];
        }
        const double* xp = P > 0 ? xr : xl;

        // ---- gather candidates; K(x,c), v_0(c) = 1 + g
        int ci[CPT];
        double yc[CPT], v[CPT], cov[CPT], d2[CPT];
        double Wr[RREG > 0 ? RREG : 1][CPT];
        uint32_t chosen = 0;   // bit k: slot retired (chosen or absent)
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int slot = tid + k * DT;
            if (slot < M) {
                const int c = A.cand[t * A.cand_stride + slot];
                ci[k] = c;
                yc[k] = A.y[c];
                const double* xc = A.Xaos + (int64_t)c * p;
                double s = 0.0;
                for (int kk = 0; kk < p; ++kk) {
                    const double ck = xc[kk];
                    Xc[(int64_t)kk * Mpad + slot] = ck;
                    const double tt = xp[kk] - ck;
                    s += tt * tt;
                }
                d2[k] = s;
                cov[k] = exp(-s / theta);
                v[k] = one_eta;
            } else {
                ci[k] = 0x7fffffff;
                yc[k] = 0.0;
                d2[k] = INFINITY;
                cov[k] = 0.0;
                v[k] = one_eta;
                chosen |= 1u << k;
                for (int kk = 0; kk < p; ++kk) Xc[(int64_t)kk * Mpad + slot] = 0.0;
            }
        }

        // ---- starting design: the n0 nearest candidates, by (distance, index)
        {
            uint32_t taken = chosen;
            for (int r = 0; r < n0; ++r) {
                double bd = INFINITY;
                int bi = 0x7fffffff, bs = -1;
#pragma unroll
                for (int k = 0; k < CPT; ++k) {
                    if (!((taken >> k) & 1u) && nearer(d2[k], ci[k], bd, bi)) {
                        bd = d2[k]; bi = ci[k]; bs = tid + k * DT;
                    }
                }
                for (int o = 32; o > 0; o >>= 1) {
                    double od = __shfl_xor(bd, o);
                    int oi = __shfl_xor(bi, o), os = __shfl_xor(bs, o);
                    if (nearer(od, oi, bd, bi)) { bd = od; bi = oi; bs = os; }
                }
                const int par = (r & 1) * DWAVES;
                if (lane == 0) { redv[par + wave] = bd; redi[par + wave] = bi; reds[par + wave] = bs; }
                __syncthreads();
                bd = redv[par]; bi = redi[par]; bs = reds[par];
                for (int w = 1; w < DWAVES; ++w)
                    if (nearer(redv[par + w], redi[par + w], bd, bi)) {
                        bd = redv[par + w]; bi = redi[par + w]; bs = reds[par + w];
                    }
                if (tid == 0) forced[r] = bs;
                if (bs >= 0 && (bs % DT) == tid) taken |= 1u << (bs / DT);
            }
        }
        __syncthreads();

        // ---- greedy steps
        int s_next = -1;
        int notpd = 0;
        for (int i = 0; i < n; ++i) {
            const int s = (i < n0) ? forced[i] : s_next;
            if (s < 0 || s >= M) { notpd = 1; break; }
            const int s_lane = s % DT;
            const int s_k = s / DT;
            // Owner publishes the register part of its column, v(s), y(s).
            if (tid == s_lane) {
                const int kk = __builtin_amdgcn_readfirstlane(s_k);
#pragma unroll
                for (int k = 0; k < CPT; ++k) {
                    if (k == kk) {
#pragma unroll
                        for (int l = 0; l < (RREG > 0 ? RREG : 0); ++l)
                            if (l < i) ws[l] = Wr[l][k];
                        misc[0] = v[k];
                        misc[1] = yc[k];
                        ctl[1] = ci[k];
                    }
                }
                chosen |= 1u << kk;
            }
            // Everyone copies the LDS / global part of the column.
            for (int l = RREG + tid; l < i; l += DT)
                ws[l] = (l < RREG + rlds) ? Wl[(int64_t)(l - RREG) * Mpad + s]
                                          : Wg[(int64_t)(l - RREG - rlds) * Mpad + s];
            for (int k = tid; k < p; k += DT) xsl[k] = Xc[(int64_t)k * Mpad + s];
            __syncthreads();

            const double vs = misc[0];
            const double ys = misc[1];
            const int cs = ctl[1];
            if (!(vs > 0.0)) { notpd = 1; break; }
            const double delta = sqrt(vs);
            double xs[P > 0 ? P : 1];
            if (P > 0) {
#pragma unroll
                for (int k = 0; k < (P > 0 ? P : 1); ++k) xs[k] = xsl[k];
            }
            const double* xsp = P > 0 ? xs : xsl;

            // New entries of w_x and u (every thread computes the same values).
            double ax = exp(-sqdist_lds<P>(xsp, xl, 1, p) / theta);
            double ay = ys;
            for (int l = 0; l < i; ++l) {
                const double w = ws[l];
                ax -= w * wx[l];
                ay -= w * uu[l];
            }
            const double rx = ax / delta;
            const double ry = ay / delta;
            if (tid == 0) {
                wx[i] = rx;
                uu[i] = ry;
                if (A.sel) A.sel[t * A.sel_stride + i] = cs;
            }
            if (i == n - 1) break;

            // Row i of W for every live candidate.
            double acc[CPT];
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
                const int slot = tid + k * DT;
                acc[k] = exp(-sqdist_lds<P>(xsp, Xc + slot, Mpad, p) / theta);
            }
#pragma unroll
            for (int l = 0; l < (RREG > 0 ? RREG : 0); ++l) {
                if (l < i) {
                    const double w = ws[l];
#pragma unroll
                    for (int k = 0; k < CPT; ++k) acc[k] -= w * Wr[l][k];
                }
            }
            {
                const int le = i < RREG + rlds ? i : RREG + rlds;
                for (int l = RREG; l < le; ++l) {
                    const double w = ws[l];
                    const double* row = Wl + (int64_t)(l - RREG) * Mpad + tid;
#pragma unroll
                    for (int k = 0; k < CPT; ++k) acc[k] -= w * row[k * DT];
                }
                for (int l = RREG + rlds; l < i; ++l) {
                    const double w = ws[l];
                    const double* row = Wg + (int64_t)(l - RREG - rlds) * Mpad + tid;
#pragma unroll
                    for (int k = 0; k < CPT; ++k) acc[k] -= w * row[k * DT];
                }
            }
            double r[CPT];
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
                r[k] = acc[k] / delta;
                v[k] -= r[k] * r[k];
                cov[k] -= rx * r[k];
            }
            if (i < RREG) {
#pragma unroll
                for (int l = 0; l < (RREG > 0 ? RREG : 0); ++l)
                    if (l == i) {
#pragma unroll
                        for (int k = 0; k < CPT; ++k) Wr[l][k] = r[k];
                    }
            } else if (i < RREG + rlds) {
                double* row = Wl + (int64_t)(i - RREG) * Mpad + tid;
#pragma unroll
                for (int k = 0; k < CPT; ++k) row[k * DT] = r[k];
            } else {
                double* row = Wg + (int64_t)(i - RREG - rlds) * Mpad + tid;
#pragma unroll
                for (int k = 0; k < CPT; ++k) row[k * DT] = r[k];
            }

            // Argmax of ALC_{i+1} over live candidates (needed from step n0 on).
            double bv = -INFINITY;
            int bi = 0x7fffffff, bs = -1;
            if (i + 1 >= n0) {
#pragma unroll
                for (int k = 0; k < CPT; ++k) {
                    if (!((chosen >> k) & 1u)) {
                        const double a = v[k] > 0.0 ? cov[k] * cov[k] / v[k] : -INFINITY;
                        if (bs < 0 || better(a, ci[k], bv, bi)) { bv = a; bi = ci[k]; bs = tid + k * DT; }
                    }
                }
                for (int o = 32; o > 0; o >>= 1) {
                    double ov = __shfl_xor(bv, o);
                    int oi = __shfl_xor(bi, o), os = __shfl_xor(bs, o);
                    if (os >= 0 && (bs < 0 || better(ov, oi, bv, bi))) { bv = ov; bi = oi; bs = os; }
                }
                if (lane == 0) { redv[wave] = bv; redi[wave] = bi; reds[wave] = bs; }
            }
            __syncthreads();
            if (i + 1 >= n0) {
                bv = redv[0]; bi = redi[0]; bs = reds[0];
                for (int w = 1; w < DWAVES; ++w)
                    if (reds[w] >= 0 && (bs < 0 || better(redv[w], redi[w], bv, bi))) {
                        bv = redv[w]; bi = redi[w]; bs = reds[w];
                    }
                if (bs < 0 || bv == -INFINITY) { notpd = 1; break; }
                s_next = bs;
            }
        }

        // ---- prediction (eqs predgp, preds2 with N -> n)
        __syncthreads();
        if (tid == 0) {
            double mean, s2v, var;
            if (notpd) {
                mean = s2v = var = NAN;
            } else {
                double m = 0.0, ps = 0.0, q = 0.0;
                for (int l = 0; l < n; ++l) {
                    m += wx[l] * uu[l];
                    ps += uu[l] * uu[l];
                    q += wx[l] * wx[l];
                }
                const double vxn = one_eta - q;
                mean = m;
                s2v = ps * vxn / n;
                var = n > 2 ? ps * vxn / (n - 2) : NAN;
            }
            A.mean[t] = mean;
            A.s2[t] = s2v;
            if (A.var) A.var[t] = var;
            if (A.df) A.df[t] = n;
            if (A.status) A.status[t] = notpd ? 1 : 0;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ plan
// Register-resident tile rows per candidate-slot count (about 180 VGPRs of tile).
template <int CPT> struct RregFor { static constexpr int value = CPT >= 16 ? 5 : CPT == 8 ? 11 : CPT == 4 ? 22 : CPT == 2 ? 44 : 64; };

static size_t fixed_lds_bytes(int nmax, int p)
{
    size_t b = 0;
    b += (size_t)(3 * nmax + 2 * p + 4 + 2 * DWAVES) * sizeof(double);
    b += (size_t)(4 * DWAVES + nmax + 4) * sizeof(int);
    return (b + 15) & ~(size_t)15;
}

static int rreg_of(int cpt)
{
    switch (cpt) {
    case 1: return RregFor<1>::value;
    case 2: return RregFor<2>::value;
    case 4: return RregFor<4>::value;
    case 8: return RregFor<8>::value;
    default: return RregFor<16>::value;
    }
}

int design_plan(const DeviceDesign& D, int32_t nmax, int32_t Mmax, int32_t n0, int32_t precision,
                int num_cu, size_t max_lds, DesignPlan* plan, std::string* err)
{
    (void)n0;
    (void)precision;
    int cpt = 1;
    while (cpt * DT < Mmax) cpt <<= 1;
    if (cpt > 16) { *err = "candidate-set size above 4096 is not supported"; return -1; }
    const int Mpad = cpt * DT;
    const int p = D.p;
    const int rows = nmax > 1 ? nmax - 1 : 0;  // W rows ever stored
    const int rreg = rreg_of(cpt);
    int rem = rows > rreg ? rows - rreg : 0;
    const size_t fixed = fixed_lds_bytes(nmax, p);
    if (fixed > max_lds) { *err = "local design size too large for LDS"; return -1; }
    size_t avail = max_lds - fixed;
    const size_t coord_bytes = (size_t)p * Mpad * sizeof(double);
    bool coords_lds = coord_bytes <= avail / 2 || coord_bytes + (size_t)rem * Mpad * 8 <= avail;
    if (coords_lds) avail -= coord_bytes;
    int rlds = (int)(avail / ((size_t)Mpad * sizeof(double)));
    if (rlds > rem) rlds = rem;
    const int rglob = rem - rlds;
    plan->cpt = cpt;
    plan->rreg = rreg;
    plan->rlds = rlds;
    plan->rglob = rglob;
    plan->coords_lds = coords_lds;
    plan->lds_bytes = fixed + (coords_lds ? coord_bytes : 0) + (size_t)rlds * Mpad * sizeof(double);
    plan->scratch_per_block =
        align256(((coords_lds ? 0 : (size_t)p * Mpad) + (size_t)rglob * Mpad) * sizeof(double));
    plan->blocks = num_cu;
    plan->counter_bytes = 256;
    return 0;
}

size_t design_workspace_bytes(const DesignPlan& plan)
{
    return plan.counter_bytes + plan.scratch_per_block * (size_t)plan.blocks;
}

template <int CPT, int P>
static int launch_design(const DesignArgs& a, const DesignPlan& plan, hipStream_t stream, std::string* err)
{
    constexpr int RREG = RregFor<CPT>::value;
    auto kern = design_kernel<CPT, RREG, P>;
    if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)plan.lds_bytes) != hipSuccess) {
        *err = "cannot reserve LDS for the design kernel";
        return -2;
    }
    hipLaunchKernelGGL(kern, dim3(plan.blocks), dim3(DT), plan.lds_bytes, stream, a);
    if (hipGetLastError() != hipSuccess) { *err = "design kernel launch failed"; return -2; }
    return 0;
}

template <int CPT>
static int launch_design_p(const DesignArgs& a, const DesignPlan& plan, hipStream_t stream, std::string* err)
{
    switch (a.p) {
    case 2: return launch_design<CPT, 2>(a, plan, stream, err);
    case 4: return launch_design<CPT, 4>(a, plan, stream, err);
    case 8: return launch_design<CPT, 8>(a, plan, stream, err);
    default: return launch_design<CPT, 0>(a, plan, stream, err);
    }
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
    a.nmax = L.n;
    if (hipMemsetAsync(a.counter, 0, sizeof(unsigned int), stream) != hipSuccess) {
        *err = "hipMemsetAsync failed";
        return -2;
    }
    switch (plan.cpt) {
    case 1: return launch_design_p<1>(a, plan, stream, err);
    case 2: return launch_design_p<2>(a, plan, stream, err);
    case 4: return launch_design_p<4>(a, plan, stream, err);
    case 8: return launch_design_p<8>(a, plan, stream, err);
    default: return launch_design_p<16>(a, plan, stream, err);
    }
}

}  // namespace lagp
