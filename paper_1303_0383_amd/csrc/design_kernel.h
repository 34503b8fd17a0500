// design_kernel.h -- greedy ALC local design and local GP prediction on gfx950.
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
#pragma once
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "lagp_internal.h"

#ifndef LAGP_RING_DEPTH
#define LAGP_RING_DEPTH 3
#endif

namespace lagp {


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
    const double* theta_per;  // nullable: per-location lengthscale (replaces theta)
    const int32_t* start;     // nullable: saved starting designs, T x start_stride (replace the n0 nearest)
    int64_t start_stride;
    const int32_t* start_n;   // nullable: per-location starting-design size (else n0)
    double vratio;            // > 0: stop once v_j(x) / v_{j+1}(x) falls below it
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
    int y_lds;               // the candidates' responses follow the coordinates in LDS (CL only)
    int nmax;
    unsigned int* counter;
    const int32_t* order;    // nullable: work item -> location (else identity)
    const uint32_t* count;   // nullable: number of work items, read on the device (else T)
};

// A block-uniform double held in scalar registers.
__device__ __forceinline__ double uniform_f64(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// ---- exact division helpers
// a / b correctly rounded from y = RN(1/b): q = RN(a*y), r = a - q*b (exact
// through the fused multiply-add), RN(q + r*y) = RN(a/b) (Markstein's
// correction; inputs here are normal and finite).
__device__ __forceinline__ double div_by(double a, double b, double y)
{
    const double q = a * y;
    const double r = __builtin_fma(-q, b, a);
    return __builtin_fma(r, y, q);
}

// ---- wave reductions with DPP (xor 1, xor 2 as quad permutes; rotations by
// 4 and 8 inside each 16-lane row), then cross-row shuffles.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ int dpp_i(int v)
{
    return __builtin_amdgcn_update_dpp(v, v, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp_d(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = dpp_i<CTRL, ROWS>((int)(b & 0xffffffffll));
    const int hi = dpp_i<CTRL, ROWS>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// A double from lane `l` of the wave (l uniform).
__device__ __forceinline__ double readlane_d(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Offset of row l of a packed lower triangle (row l holds l + 1 entries).
__host__ __device__ __forceinline__ int packed_row(int l) { return l * (l + 1) / 2; }

// Candidate ordering for the argmax: larger score first, then smaller index.
// (Bitwise & and | on the comparisons: no short-circuit branches.)
__device__ __forceinline__ bool better(double a, int ia, double b, int ib)
{
    return (a > b) | ((a == b) & (ia < ib));
}
// Nearest-neighbour ordering: smaller squared distance first, then smaller index.
__device__ __forceinline__ bool nearer(double a, int ia, double b, int ib)
{
    return (a < b) | ((a == b) & (ia < ib));
}

// Four consecutive LDS doubles (16-byte aligned start) as two 16-byte reads.
__device__ __forceinline__ void ld4(const double* p, double* o)
{
    const double2 a = *reinterpret_cast<const double2*>(p);
    const double2 b = *reinterpret_cast<const double2*>(p + 2);
    o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
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

// Rows of the whitened tile kept in registers for a workgroup size, slot
// count, coordinate placement, tile precision and trimming: the largest
// multiple of 4 that compiles without scratch spills for P = 8 (a compile
// sweep), capped at 64 (with one slot per thread LDS holds the rest).  With
// 256 threads (one wave per SIMD) a lane can hold 512 registers, the upper
// half as accumulation registers; with 512 threads a lane has 256.  The
// mixed mode's short list and re-score leave no room for register rows with
// 512 threads and 8 slots (with coordinates in LDS it spills a few values).
__host__ __device__ constexpr int rreg_for(int dt, int cpt, bool cl, bool mix = false, bool trim = false)
{
    if (dt == 256) {
        if (!mix) {
            switch (cpt) {
            case 1: return 64;
            case 2: return 64;
            case 4: return 40;
            default: return (cl || trim) ? 16 : 20;
            }
        }
        switch (cpt) {
        case 1: return 64;
        case 2: return 64;
        case 4: return 64;
        default: return cl ? 28 : 32;
        }
    }
    if (!mix) {
        switch (cpt) {
        case 1: return 64;
        case 2: return 32;
        case 4: return cl ? 8 : 12;
        default: return 0;
        }
    }
    switch (cpt) {
    case 1: return 64;
    case 2: return 48;
    case 4: return cl ? 12 : 16;
    default: return 0;
    }
}

// Global tile rows in the load ring per workgroup step (rows in flight + the
// one being consumed): about four rows of a 256-thread workgroup in flight
// cover the memory latency at full streaming rate.
__host__ __device__ constexpr int ring_depth(int cpt, bool mix)
{
    return (cpt * (mix ? 4 : 8)) >= 64 ? LAGP_RING_DEPTH : 5;
}

// Combine (value, design index, slot) with a partner lane's triple.
// MAX: larger value wins (argmax of ALC); otherwise smaller wins (nearest).
template <bool MAX>
__device__ __forceinline__ void pick(double& v, int& i, int& s, double ov, int oi, int os)
{
    const bool take = (os >= 0) & ((s < 0) | (MAX ? better(ov, oi, v, i) : nearer(ov, oi, v, i)));
    v = take ? ov : v;
    i = take ? oi : i;
    s = take ? os : s;
}

template <bool MAX>
__device__ __forceinline__ void wave_pick(double& v, int& i, int& s)
{
    pick<MAX>(v, i, s, dpp_d<0xB1>(v), dpp_i<0xB1>(i), dpp_i<0xB1>(s));     // xor 1
    pick<MAX>(v, i, s, dpp_d<0x4E>(v), dpp_i<0x4E>(i), dpp_i<0x4E>(s));     // xor 2
    pick<MAX>(v, i, s, dpp_d<0x124>(v), dpp_i<0x124>(i), dpp_i<0x124>(s));  // rotate 4 in row
    pick<MAX>(v, i, s, dpp_d<0x128>(v), dpp_i<0x128>(i), dpp_i<0x128>(s));  // rotate 8 in row
    pick<MAX>(v, i, s, __shfl_xor(v, 16), __shfl_xor(i, 16), __shfl_xor(s, 16));
    pick<MAX>(v, i, s, __shfl_xor(v, 32), __shfl_xor(i, 32), __shfl_xor(s, 32));
}

// Order-preserving 64-bit key of (score, design index) for short lists:
// larger score first, then smaller index.  The score is rounded to float, so
// scores within float rounding of each other rank by index; 0 marks no entry.
__device__ __forceinline__ uint64_t rank_key(double a, int idx)
{
    const uint32_t hi = a > 0.0 ? __float_as_uint((float)a) : 0u;
    return ((uint64_t)hi << 32) | (uint32_t)(0xffffffffu - (uint32_t)idx);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp_key(uint64_t k)
{
    const int lo = (int)(uint32_t)k, hi = (int)(uint32_t)(k >> 32);
    const int l2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWS, 0xF, false);
    const int h2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWS, 0xF, false);
    return ((uint64_t)(uint32_t)h2 << 32) | (uint32_t)l2;
}

// Largest key of the wave: row maxima by quad permutes and row rotations,
// then row broadcasts carry them into lane 63, which is read back.
__device__ __forceinline__ uint64_t wave_max_key(uint64_t k)
{
    uint64_t o;
    o = dpp_key<0xB1, 0xF>(k);  k = o > k ? o : k;   // xor 1
    o = dpp_key<0x4E, 0xF>(k);  k = o > k ? o : k;   // xor 2
    o = dpp_key<0x124, 0xF>(k); k = o > k ? o : k;   // rotate 4 in row
    o = dpp_key<0x128, 0xF>(k); k = o > k ? o : k;   // rotate 8 in row
    o = dpp_key<0x142, 0xA>(k); k = o > k ? o : k;   // lane 15 of rows 0, 2 into rows 1, 3
    o = dpp_key<0x143, 0xC>(k); k = o > k ? o : k;   // lane 31 into rows 2, 3
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)k, 63);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(k >> 32), 63);
    return ((uint64_t)hi << 32) | lo;
}

// The wave's best triple in lane 63: row reductions, then row broadcasts
// (lanes of rows outside a step's row mask compare with themselves).
template <bool MAX>
__device__ __forceinline__ void wave_pick63(double& v, int& i, int& s)
{
    pick<MAX>(v, i, s, dpp_d<0xB1>(v), dpp_i<0xB1>(i), dpp_i<0xB1>(s));     // xor 1
    pick<MAX>(v, i, s, dpp_d<0x4E>(v), dpp_i<0x4E>(i), dpp_i<0x4E>(s));     // xor 2
    pick<MAX>(v, i, s, dpp_d<0x124>(v), dpp_i<0x124>(i), dpp_i<0x124>(s));  // rotate 4 in row
    pick<MAX>(v, i, s, dpp_d<0x128>(v), dpp_i<0x128>(i), dpp_i<0x128>(s));  // rotate 8 in row
    pick<MAX>(v, i, s, dpp_d<0x142, 0xA>(v), dpp_i<0x142, 0xA>(i), dpp_i<0x142, 0xA>(s));  // lane 15 -> next row
    pick<MAX>(v, i, s, dpp_d<0x143, 0xC>(v), dpp_i<0x143, 0xC>(i), dpp_i<0x143, 0xC>(s));  // lane 31 -> rows 2, 3
}

// ---- the per-workgroup global slab through a buffer descriptor: one
// per-thread offset register and uniform (scalar) slot and row offsets, so no
// address registers per (slot, row) pair; accesses past the slab read 0 and
// are not written.
typedef unsigned int lagp_u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t slab_rsrc(const void* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ void bload(__amdgpu_buffer_rsrc_t r, int voff, int soff, double& v)
{
    v = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

__device__ __forceinline__ void bload(__amdgpu_buffer_rsrc_t r, int voff, int soff, float& v)
{
    v = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, int voff, int soff, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(lagp_u32x2, v), r, voff, soff, 0);
}

__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, int voff, int soff, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, voff, soff, 0);
}

// Tile storage: the FP64 and FP32 tiles keep rows in their compute type; the
// BF16 tile stores rows as bfloat16 (round to nearest even) and computes in
// FP32, so a row's register, LDS and global copies hold the same value.
template <int MIX>
struct TileTypes {
    using W = typename std::conditional<MIX != 0, float, double>::type;   // compute
    using S = typename std::conditional<MIX == 2, __bf16, W>::type;       // LDS and global rows
};

template <int MIX>
__device__ __forceinline__ typename TileTypes<MIX>::W tile_round(double r)
{
    if constexpr (MIX == 2) return (float)(__bf16)(float)r;
    else return (typename TileTypes<MIX>::W)r;
}

template <int MIX>
__device__ __forceinline__ void bload_tile(__amdgpu_buffer_rsrc_t r, int voff, int soff, typename TileTypes<MIX>::W& v)
{
    if constexpr (MIX == 2)
        v = (float)__builtin_bit_cast(__bf16, (unsigned short)__builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
    else
        bload(r, voff, soff, v);
}

template <int MIX>
__device__ __forceinline__ void bstore_tile(__amdgpu_buffer_rsrc_t r, int voff, int soff, typename TileTypes<MIX>::W v)
{
    if constexpr (MIX == 2)
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, (__bf16)v), r, voff, soff, 0);
    else
        bstore(r, voff, soff, v);
}

// Squared distance from the uniform point a to the candidate whose P
// coordinates sit in the slab at byte offsets soff + k * cstride (+ voff).
template <int P>
__device__ __forceinline__ double sqdist_slab(const double* __restrict__ a, __amdgpu_buffer_rsrc_t r, int voff,
                                              int soff, int cstride)
{
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < P; ++k) {
        double c;
        bload(r, voff, soff + k * cstride, c);
        const double t = a[k] - c;
        s += t * t;
    }
    return s;
}

// Four consecutive LDS floats (16-byte aligned start).
__device__ __forceinline__ void ld4(const float* p, float* o)
{
    const float4 a = *reinterpret_cast<const float4*>(p);
    o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w;
}

// DT threads per workgroup, CPT candidate slots per thread, RREG register
// rows, P compile-time dimension (0: runtime), CL candidate coordinates in LDS,
// MIX: the whitened tile stored and contracted in FP32 (ranking only), TRIM:
// locations may leave whole slot columns empty (candidate sets well below
// CPT * DT), whose global-memory traffic and exponentials are then skipped.
//
// Register economy decides how many tile rows stay on chip, so the step loop
// keeps few values alive besides the tile: the exponentials of a step are
// evaluated slot by slot (an empty asm with a memory clobber keeps the
// compiler from hoisting every slot's coordinate loads at once), LDS rows are
// consumed one at a time, and the global rows stream through a ring of three
// row buffers (two rows in flight while one is consumed).
template <int DT, int CPT, int RREG, int P, bool CL, int MIX, bool TRIM>
__global__ void __launch_bounds__(DT, 1) design_kernel(const DesignArgs A)
{
    using TW = typename TileTypes<MIX>::W;   // tile compute type
    using TS = typename TileTypes<MIX>::S;   // LDS and global tile rows
    constexpr int DWAVES = DT / 64;
    extern __shared__ double smem[];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int p = P > 0 ? P : A.p;
    const int nmax = (A.nmax + 3) & ~3;   // padded: 4-row blocks read up to 3 entries ahead
    const int Mpad = CPT * DT;
    const double eta = A.eta;
    const double one_eta = 1.0 + eta;

    // ---- LDS carve-up (doubles first, then ints)
    TW* ws = (TW*)smem;              // [nmax] column of the chosen candidate
    TW* wx = (TW*)(smem + nmax);     // [nmax] L^{-1} k(x)
    double* uu = smem + 2 * nmax;    // [nmax] L^{-1} Y
    double* xl = uu + nmax;          // [p]    predictive location
    double* xsl = xl + p;            // [p+1]  (spare)
    double* misc = xsl + p + 1;      // [4]    v_s, v_j(x)
    // per-wave best (score, design index, slot); the mixed mode adds each
    // wave's DWAVES best by the FP32-tile scores
    constexpr int NSHORT = DWAVES < 4 ? DWAVES : 4;   // mixed mode: candidates re-scored per step
    constexpr int NRED = 2 * DWAVES + (MIX ? DWAVES * NSHORT : 0);
    double* redv = misc + 4;         // [NRED]
    int* redi = (int*)(redv + NRED); // [NRED]
    int* reds = redi + NRED;         // [NRED]
    int* forced = reds + NRED;       // [nmax] slots of the starting design
    int* ctl = forced + nmax;               // [4]  location, chosen index, bad start, unset candidate
    size_t off = (size_t)((char*)(ctl + 4) - (char*)smem);
    off = (off + 15) & ~(size_t)15;
    // Mixed mode: the exact FP64 factor of the chosen points (packed rows of
    // L: row l holds W_l[0..l-1][s_l] and delta_l on the diagonal), delta_l and
    // 1/delta_l, the exact L^{-1}k(x) (u = L^{-1}Y is uu), the chosen slots,
    // and per wave one staged exact column with its v, cov(x, .), y-row and
    // score (then design index and slot).
    const int npk = packed_row(nmax);
    double* Lf = (double*)((char*)smem + off);   // [npk]
    double* dl = Lf + npk;                       // [nmax]
    double* rdl = dl + nmax;                     // [nmax]
    double* wx64 = rdl + nmax;                   // [nmax]
    double* stg = wx64 + nmax;                   // [DWAVES][nmax + 4]
    int* sslot = (int*)(stg + DWAVES * (nmax + 4));   // [nmax]
    int* mxi = sslot + nmax;                     // [2 * DWAVES]
    if (MIX) off = (((size_t)((char*)(mxi + 2 * DWAVES) - (char*)smem)) + 15) & ~(size_t)15;
    const int ylds = CL ? A.y_lds : 0;
    double* Xcl = (double*)((char*)smem + off);              // [p (+1)][Mpad] when CL: coordinates (y)
    TS* Wl = (TS*)(Xcl + (CL ? (size_t)(p + ylds) * Mpad : 0));  // [rlds][Mpad]

    double* Xcg = A.scratch + (int64_t)blockIdx.x * A.scratch_stride;
    TS* Wg = (TS*)(Xcg + (CL ? 0 : (int64_t)p * Mpad));
    double* Xc = CL ? Xcl : Xcg;
    const __amdgpu_buffer_rsrc_t slab = slab_rsrc(Xcg, (uint32_t)(A.scratch_stride * sizeof(double)));
    const int voff_c = tid * (int)sizeof(double);     // coordinate element of slot k = 0
    const int voff_w = tid * (int)sizeof(TS);         // tile-row element of slot k = 0
    const int wbase = CL ? 0 : p * Mpad * (int)sizeof(double);   // tile rows after the coordinates
    const int rowb = Mpad * (int)sizeof(TS);                      // bytes per global tile row
    const int rlds = A.rlds;
    const int G0 = RREG + rlds;   // first global row
    for (int e = tid; e < rlds * Mpad; e += DT) Wl[e] = (TS)0.0f;
    (void)xsl;

    for (;;) {
        if (tid == 0) {
            ctl[0] = (int)atomicAdd(A.counter, 1u);
            ctl[3] = 0;   // set when some candidate entry is unset
        }
        __syncthreads();
        const int64_t w = ctl[0];
        if (w >= (A.count ? (int64_t)*A.count : A.T)) break;
        const int64_t t = A.order ? A.order[w] : w;
        const int n = A.n_per ? A.n_per[t] : A.n;
        const int M = A.M_per ? A.M_per[t] : A.M;
        // A per-location lengthscale that is not a positive finite number
        // fails the location (no greedy step is taken).
        const double theta = A.theta_per ? uniform_f64(A.theta_per[t]) : A.theta;
        const double rtheta = 1.0 / theta;
        const bool theta_ok = theta > 0.0 && theta < INFINITY;
        // Slot columns k with k * DT >= M hold no candidate for any thread
        // (block-uniform).  When there are such columns, their global tile
        // rows are not written, their global reads are redirected to the last
        // live column (a cached line: no memory traffic; the values are
        // ignored) and their exponentials are skipped.
        const int kact = (M + DT - 1) / DT;
        const bool full = !TRIM || kact == CPT;
        const int n0 = (A.start && A.start_n) ? A.start_n[t] : A.n0;
        const int32_t* cand = A.cand + t * A.cand_stride;
        for (int k = tid; k < p; k += DT) xl[k] = A.XX[t * p + k];
        // ws, wx, uu are zero beyond the current step: padded terms subtract an exact 0.
        for (int l = tid; l < nmax; l += DT) { ws[l] = 0.0; wx[l] = 0.0; uu[l] = 0.0; }
        if (tid == 0) misc[1] = one_eta;   // v_j(x), tracked for the stopping rule
        if (A.sel)
            for (int i = tid; i < n; i += DT) A.sel[t * A.sel_stride + i] = -1;
        __syncthreads();

        // ---- gather candidates (coordinates and y into the coordinate block);
        //      K(x,c) and v_0(c) = 1 + g
        int ci[CPT];
        // FP64 tile: yc = y_c - sum_l u_l W[l][c] tracks each candidate's
        // whitened response the way cov tracks K(x,c) - sum_l w_x[l] W[l][c],
        // so the chosen point's entries of w_x and u come from its owner.
        double v[CPT], cov[CPT], d2[CPT], yc[CPT];
        TW Wr[RREG > 0 ? RREG : 1][CPT];
#pragma unroll
        for (int l = 0; l < (RREG > 0 ? RREG : 1); ++l)
#pragma unroll
            for (int k = 0; k < CPT; ++k) Wr[l][k] = 0.0;
        uint32_t chosen = 0;   // bit k: slot retired (chosen or absent)
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int slot = tid + k * DT;
            if (slot < M) {
                const int c0 = cand[slot];
                if (c0 < 0) ctl[3] = 1;
                const int c = c0 < 0 ? 0 : c0;
                ci[k] = c;
                if (CL && ylds) Xc[(int64_t)p * Mpad + slot] = A.y[c];
                const double* xc = A.Xaos + (int64_t)c * p;
                double sq = 0.0;
                for (int kk = 0; kk < p; ++kk) {
                    const double ck = xc[kk];
                    if (CL) Xc[(int64_t)kk * Mpad + slot] = ck;
                    else bstore(slab, voff_c, (kk * Mpad + k * DT) * (int)sizeof(double), ck);
                    const double tt = xl[kk] - ck;
                    sq += tt * tt;
                }
                d2[k] = sq;
                cov[k] = exp(-div_by(sq, theta, rtheta));
                yc[k] = MIX ? 0.0 : A.y[c];
            } else {
                ci[k] = 0x7fffffff;
                yc[k] = 0.0;
                if (CL && ylds) Xc[(int64_t)p * Mpad + slot] = 0.0;
                d2[k] = INFINITY;
                cov[k] = 0.0;
                chosen |= 1u << k;
                for (int kk = 0; kk < p; ++kk) {
                    if (CL) Xc[(int64_t)kk * Mpad + slot] = 0.0;
                    else bstore(slab, voff_c, (kk * Mpad + k * DT) * (int)sizeof(double), 0.0);
                }
            }
            v[k] = one_eta;
            asm volatile("" ::: "memory");
        }

        // ---- starting design: a saved design located among the candidates, or
        //      the n0 nearest candidates by (distance, index)
        if (A.start) {
            const int32_t* st = A.start + t * A.start_stride;
            for (int r = tid; r < n0; r += DT) forced[r] = -1;
            __syncthreads();
            uint32_t hit = 0;
            for (int r = 0; r < n0; ++r) {
                const int want = st[r];
#pragma unroll
                for (int k = 0; k < CPT; ++k)
                    if (tid + k * DT < M && ci[k] == want) {
                        forced[r] = ((hit >> k) & 1u) ? -2 : tid + k * DT;   // -2: repeated index
                        hit |= 1u << k;
                    }
            }
            __syncthreads();
            if (tid == 0) {
                int bad = 0;
                for (int r = 0; r < n0; ++r) bad |= forced[r] < 0;
                ctl[2] = bad;
            }
        } else {
            uint32_t taken = chosen;
            for (int r = 0; r < n0; ++r) {
                double bd = INFINITY;
                int bi = 0x7fffffff, bs = -1;
#pragma unroll
                for (int k = 0; k < CPT; ++k) {
                    const bool live = !((taken >> k) & 1u);
                    pick<false>(bd, bi, bs, live ? d2[k] : INFINITY, live ? ci[k] : 0x7fffffff, live ? tid + k * DT : -1);
                }
                wave_pick63<false>(bd, bi, bs);
                const int par = (r & 1) * DWAVES;
                if (lane == 63) { redv[par + wave] = bd; redi[par + wave] = bi; reds[par + wave] = bs; }
                __syncthreads();
                bd = redv[par]; bi = redi[par]; bs = reds[par];
                for (int w = 1; w < DWAVES; ++w) pick<false>(bd, bi, bs, redv[par + w], redi[par + w], reds[par + w]);
                if (tid == 0) forced[r] = bs;
                if (bs >= 0 && (bs % DT) == tid) taken |= 1u << (bs / DT);
            }
        }
        __syncthreads();
        const int nocand = ctl[3];   // a candidate entry the kNN marked as unset (-1)

        // ---- greedy steps
        const int badstart = A.start ? ctl[2] : 0;
        int s_next = -1;
        int notpd = (theta_ok && !badstart && !nocand) ? 0 : 1;
        int nuse = n;   // design size reached (the stopping rule may end the search early)
        double vxr = one_eta;   // exact v_j(x) (mixed mode), the same in every thread
        if constexpr (MIX) {
            // Row 0 of the exact factor: the first point's column is empty and
            // v_0(s_0) = 1 + g; its rows of w_x and u follow from K(s_0, x), y_s0.
            const int s0 = forced[0];
            if (!notpd && (s0 < 0 || s0 >= M)) notpd = 1;
            if (!notpd) {
                const double delta = sqrt(one_eta);
                const double rdelta = 1.0 / delta;
                double sq = 0.0;
                for (int kk = 0; kk < p; ++kk) {
                    const double tx = xl[kk] - Xc[(int64_t)kk * Mpad + s0];
                    sq += tx * tx;
                }
                const double rx = div_by(exp(-div_by(sq, theta, rtheta)), delta, rdelta);
                vxr -= rx * rx;
                if (tid == 0) {
                    Lf[0] = delta;
                    dl[0] = delta;
                    rdl[0] = rdelta;
                    wx64[0] = rx;
                    sslot[0] = s0;
                }
            }
        }
        // Full steps i = 0 .. n-2 append row i of W for every candidate and
        // choose the next point; the last chosen point is appended after the
        // loop (only its own column is needed there).
        for (int i = 0; i < n - 1 && !notpd && nuse == n; ++i) {
            const int s = (i < n0) ? forced[i] : s_next;
            if (s < 0 || s >= M) { notpd = 1; continue; }
            const int s_lane = s % DT;
            const int s_k = s / DT;
            // Phase A (before the barrier): the owner publishes the register
            // part of its column and v(s); everyone copies the LDS / global
            // part and evaluates K(s, .) for x and its own candidates.
            if (tid == s_lane) {
                const int kk = __builtin_amdgcn_readfirstlane(s_k);
#pragma unroll
                for (int k = 0; k < CPT; ++k) {
                    if (k == kk) {
#pragma unroll
                        for (int l = 0; l < (RREG > 0 ? RREG : 0); ++l)
                            if (l < i) ws[l] = Wr[l][k];
                        misc[0] = v[k];
                        if (!MIX) {
                            misc[2] = cov[k];
                            misc[3] = yc[k];
                        }
                        ctl[1] = ci[k];
                    }
                }
                chosen |= 1u << kk;
            }
            for (int l = RREG + tid; l < i; l += DT)
                ws[l] = (TW)((l < G0) ? Wl[(int64_t)(l - RREG) * Mpad + s] : Wg[(int64_t)(l - G0) * Mpad + s]);
            // K(x, s): the FP64 tile takes cov(s) from its owner after the
            // barrier; the mixed modes' ranking tile evaluates it here.
            double ax = 0.0, acc[CPT];
            if (P > 0) {
                double xs[P > 0 ? P : 1];
#pragma unroll
                for (int k = 0; k < (P > 0 ? P : 1); ++k) xs[k] = Xc[(int64_t)k * Mpad + s];
                if constexpr (MIX) ax = exp(-div_by(sqdist_lds<P>(xs, xl, 1, p), theta, rtheta));
                // K(s, c) in pairs of slots, coordinates from LDS or from the
                // slab.  A pair's two chains interleave (with one wave per
                // SIMD nothing else hides their latency); a runtime branch
                // per pair (kact == CPT for full candidate sets) keeps the
                // compiler from interleaving every slot's exponential, which
                // would cost tile rows.
                constexpr int KP = (CL && CPT >= 4) ? 4 : CPT >= 2 ? 2 : 1;
#pragma unroll
                for (int k0 = 0; k0 < CPT; k0 += KP) {
                    double sq[KP], e[KP];
#pragma unroll
                    for (int q = 0; q < KP; ++q) {
                        const int k = k0 + q;
                        if constexpr (CL) sq[q] = sqdist_lds<P>(xs, Xc + tid + k * DT, Mpad, p);
                        else sq[q] = sqdist_slab<(P > 0 ? P : 1)>(xs, slab, voff_c, k * DT * (int)sizeof(double),
                                                                  Mpad * (int)sizeof(double));
                        e[q] = 0.0;
                    }
                    if (k0 < kact) {
#pragma unroll
                        for (int q = 0; q < KP; ++q) {
                            const double eq = exp(-div_by(sq[q], theta, rtheta));
                            e[q] = k0 + q < kact ? eq : 0.0;
                        }
                    }
#pragma unroll
                    for (int q = 0; q < KP; ++q) acc[k0 + q] = e[q];
                    asm volatile("" ::: "memory");
                }
            } else {
                double sqx = 0.0, sq[CPT];
#pragma unroll
                for (int k = 0; k < CPT; ++k) sq[k] = 0.0;
                for (int kk = 0; kk < p; ++kk) {
                    const double a = Xc[(int64_t)kk * Mpad + s];
                    if constexpr (MIX) {
                        const double tx = a - xl[kk];
                        sqx += tx * tx;
                    }
#pragma unroll
                    for (int k = 0; k < CPT; ++k) {
                        const double tc = a - Xc[(int64_t)kk * Mpad + tid + k * DT];
                        sq[k] += tc * tc;
                    }
                }
                if constexpr (MIX) ax = exp(-div_by(sqx, theta, rtheta));
#pragma unroll
                for (int k = 0; k < CPT; ++k) {
                    acc[k] = exp(-div_by(sq[k], theta, rtheta));
                    asm volatile("" ::: "memory");
                }
            }

            // The first global rows are requested before the barrier.
            constexpr int DEPTH = ring_depth(CPT, MIX);
            TW bq[DEPTH][CPT];
            const int gcount = i > G0 ? i - G0 : 0;
            // Row loads are issued unconditionally (no branch between a load
            // and its use, so the compiler can count the loads in flight
            // instead of draining them): a row not yet written, or past the
            // slab, is read but never consumed (the descriptor returns zeros
            // past the slab).
            auto load_row = [&](int l, TW* b) {
                const int rb = wbase + (l - G0) * rowb;
#pragma unroll
                for (int k = 0; k < CPT; ++k)
                    bload_tile<MIX>(slab, voff_w, rb + (full ? k * DT : (k < kact ? k : kact - 1) * DT) * (int)sizeof(TS), b[k]);
            };
            if (gcount > 0) {
#pragma unroll
                for (int q = 0; q + 1 < DEPTH; ++q) load_row(G0 + q, bq[q]);
            }
            float dot[CPT], dotx = 0.0f;   // FP32 contraction (MIX)
#pragma unroll
            for (int k = 0; k < CPT; ++k) dot[k] = 0.0f;
            __syncthreads();   // B1: column of s, v(s) and its running sums published

            // The mixed mode's FP32 ranking stays self-consistent: its delta
            // is that of the tile's own v(s) (the exact one if that is not
            // positive); the exact factor is kept apart.
            const double vs = misc[0];
            if (!MIX && !(vs > 0.0)) { notpd = 1; continue; }
            const double delta = (MIX && !(vs > 0.0)) ? dl[i] : sqrt(vs);
            const double rdelta = 1.0 / delta;
            // FP64: the entries of w_x and u for s from its owner's running
            // sums (the same products in the same ascending order as a dot
            // product over the chosen column, so bitwise the same values).
            double ay = 0.0;
            if constexpr (!MIX) {
                ax = misc[2];
                ay = misc[3];
            }
            // Row i of W for every live candidate: acc = K(s,c) - sum_l ws[l] W[l][c].
            // Register rows, four per block; rows >= i within a block are zero.
#pragma unroll
            for (int l0 = 0; l0 < (RREG > 0 ? RREG : 0); l0 += 4) {
                if (l0 < i) {
                    TW wv[4], xv[4];
                    ld4(ws + l0, wv);
                    if constexpr (MIX) {
                        ld4(wx + l0, xv);
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
#pragma unroll
                            for (int k = 0; k < CPT; ++k) dot[k] = __builtin_fmaf(wv[r], Wr[l0 + r][k], dot[k]);
                            dotx = __builtin_fmaf(wv[r], xv[r], dotx);
                        }
                    } else {
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
#pragma unroll
                            for (int k = 0; k < CPT; ++k) acc[k] -= wv[r] * Wr[l0 + r][k];
                        }
                    }
                }
            }
            // LDS rows [RREG, min(i, G0)), one at a time.
            {
                const int le = i < G0 ? i : G0;
                for (int l = RREG; l < le; ++l) {
                    const TW wl = ws[l];
                    const TS* row = Wl + (int64_t)(l - RREG) * Mpad + tid;
                    if constexpr (MIX) {
#pragma unroll
                        for (int k = 0; k < CPT; ++k) dot[k] = __builtin_fmaf(wl, (float)row[k * DT], dot[k]);
                        dotx = __builtin_fmaf(wl, wx[l], dotx);
                    } else {
#pragma unroll
                        for (int k = 0; k < CPT; ++k) acc[k] -= wl * (TW)row[k * DT];
                    }
                }
            }
            // Global rows through the ring: row l is consumed while rows
            // l+1 .. l+DEPTH-1 are in flight.  Per-candidate order stays ascending.
            if (gcount > 0) {
                auto consume = [&](int l, const TW* b) {
                    const TW wl = ws[l];
                    if constexpr (MIX) {
#pragma unroll
                        for (int k = 0; k < CPT; ++k) dot[k] = __builtin_fmaf(wl, b[k], dot[k]);
                        dotx = __builtin_fmaf(wl, wx[l], dotx);
                    } else {
#pragma unroll
                        for (int k = 0; k < CPT; ++k) acc[k] -= wl * b[k];
                    }
                };
                // Whole blocks of DEPTH rows with no exit inside a block, then
                // the last rows, which are already in flight.
                int l = G0;
                for (int nb = gcount / DEPTH; nb > 0; --nb) {
#pragma unroll
                    for (int q = 0; q < DEPTH; ++q) {
                        load_row(l + DEPTH - 1, bq[(q + DEPTH - 1) % DEPTH]);
                        consume(l, bq[q]);
                        ++l;
                    }
                }
#pragma unroll
                for (int q = 0; q + 1 < DEPTH; ++q)
                    if (l + q < i) consume(l + q, bq[q]);
            }
            if constexpr (MIX) {
                ax -= (double)dotx;
#pragma unroll
                for (int k = 0; k < CPT; ++k) acc[k] -= (double)dot[k];
            }
            const double rx = MIX ? ax * rdelta : div_by(ax, delta, rdelta);
            const double ui = MIX ? 0.0 : div_by(ay, delta, rdelta);
            if (tid == 0) {
                wx[i] = rx;
                if (!MIX) {
                    uu[i] = ui;
                    misc[1] -= rx * rx;
                }
                if (A.sel) A.sel[t * A.sel_stride + i] = ctl[1];
            }
            double r[CPT];
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
                r[k] = MIX ? acc[k] * rdelta : div_by(acc[k], delta, rdelta);
                v[k] -= r[k] * r[k];
                cov[k] -= rx * r[k];
                if (!MIX) yc[k] -= ui * r[k];
            }
            if (i < RREG) {
#pragma unroll
                for (int l = 0; l < (RREG > 0 ? RREG : 0); ++l)
                    if (l == i) {
#pragma unroll
                        for (int k = 0; k < CPT; ++k) Wr[l][k] = tile_round<MIX>(r[k]);
                    }
            } else if (i < G0) {
                TS* row = Wl + (int64_t)(i - RREG) * Mpad + tid;
#pragma unroll
                for (int k = 0; k < CPT; ++k) row[k * DT] = (TS)tile_round<MIX>(r[k]);
            } else {
                const int rb = wbase + (i - G0) * rowb;
#pragma unroll
                for (int k = 0; k < CPT; ++k)
                    if (full || k < kact) bstore_tile<MIX>(slab, voff_w, rb + k * DT * (int)sizeof(TS), tile_round<MIX>(r[k]));
            }

            // Argmax of ALC_{i+1} over live candidates (needed from step n0 on).
            // The score only ranks candidates, so cov^2 / v uses a refined
            // reciprocal of v.
            double bv = -INFINITY;
            int bi = 0x7fffffff, bs = -1;
            if constexpr (!MIX) {
                if (i + 1 >= n0) {
                    // every slot's score, then the thread's best by a tree of
                    // picks (the order is total, so any bracketing agrees)
                    double av[CPT];
                    int ai[CPT], as[CPT];
#pragma unroll
                    for (int k = 0; k < CPT; ++k) {
                        // computed for every slot, kept where v > 0
                        double y = __builtin_amdgcn_rcp(v[k]);
                        y = __builtin_fma(__builtin_fma(-v[k], y, 1.0), y, y);
                        const double a = (v[k] > 0.0) ? (cov[k] * cov[k]) * y : -INFINITY;
                        const bool live = !((chosen >> k) & 1u);
                        av[k] = live ? a : -INFINITY;
                        ai[k] = live ? ci[k] : 0x7fffffff;
                        as[k] = live ? tid + k * DT : -1;
                    }
#pragma unroll
                    for (int h = 1; h < CPT; h *= 2)
#pragma unroll
                        for (int k = 0; k + h < CPT; k += 2 * h) pick<true>(av[k], ai[k], as[k], av[k + h], ai[k + h], as[k + h]);
                    bv = av[0];
                    bi = ai[0];
                    bs = as[0];
                    wave_pick63<true>(bv, bi, bs);
                    if (lane == 63) { redv[wave] = bv; redi[wave] = bi; reds[wave] = bs; }
                }
            } else {
                // Mixed mode: a short list of the DWAVES best candidates by the
                // FP32-tile scores (ties to the smaller design index, so the
                // list does not depend on where candidates sit), each wave
                // contributing its own DWAVES best.
                if (i + 1 >= n0) {
                    double sc[CPT];
#pragma unroll
                    for (int k = 0; k < CPT; ++k) {
                        double a = -INFINITY;
                        if (v[k] > 0.0) {
                            double y = __builtin_amdgcn_rcp(v[k]);
                            y = __builtin_fma(__builtin_fma(-v[k], y, 1.0), y, y);
                            a = (cov[k] * cov[k]) * y;
                        }
                        sc[k] = a;
                    }
                    // the wave's NSHORT best keys: each round takes the wave's
                    // largest key, and the thread holding it clears it and
                    // publishes its slot (keys are unique)
                    uint64_t key[CPT];
#pragma unroll
                    for (int k = 0; k < CPT; ++k) key[k] = ((chosen >> k) & 1u) ? 0ull : rank_key(sc[k], ci[k]);
#pragma unroll
                    for (int q = 0; q < NSHORT; ++q) {
                        uint64_t t = 0;
#pragma unroll
                        for (int k = 0; k < CPT; ++k) t = key[k] > t ? key[k] : t;
                        t = wave_max_key(t);
                        const int e = 2 * DWAVES + wave * NSHORT + q;
                        if (lane == 0) {
                            redv[e] = __longlong_as_double((long long)t);
                            if (t == 0) reds[e] = -1;
                        }
#pragma unroll
                        for (int k = 0; k < CPT; ++k)
                            if (t != 0 && key[k] == t) {
                                reds[e] = tid + k * DT;
                                key[k] = 0;
                            }
                    }
                }
            }
            __syncthreads();   // B2: partial maxima published; everyone is done with ws
            if constexpr (MIX) {
                // Each wave re-scores one short-listed candidate exactly in FP64
                // (its column of W by forward substitution against the exact
                // factor, in the order the FP64 kernel uses, so the score is the
                // FP64 kernel's) and stages it.  Before step n0 the next point
                // is the next starting point: wave 0 computes its column.
                int sa = -1, ia = 0x7fffffff;
                if (i + 1 >= n0 && wave < NSHORT) {
                    // the global list: wave w takes the entry of rank w among
                    // all waves' keys (rank = number of larger keys)
                    const int nl = DWAVES * NSHORT;
                    const uint64_t ke = lane < nl ? (uint64_t)__double_as_longlong(redv[2 * DWAVES + lane]) : 0ull;
                    // every key broadcast from its lane (no LDS round trip per key)
                    const uint32_t klo = (uint32_t)ke, khi = (uint32_t)(ke >> 32);
                    int rank = 0;
#pragma unroll
                    for (int j = 0; j < nl; ++j) {
                        const uint64_t kj = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)khi, j) << 32) |
                                            (uint32_t)__builtin_amdgcn_readlane((int)klo, j);
                        rank += kj > ke;
                    }
                    const uint64_t own = __ballot(lane < nl && ke != 0 && rank == wave);
                    if (own) {
                        const int el = __builtin_ctzll(own);
                        sa = reds[2 * DWAVES + el];
                        ia = (int)(0xffffffffu - (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)ke, el));
                    }
                } else if (wave == 0) {
                    sa = forced[i + 1];
                }
                const int jr = i + 1;   // rows of the exact column: design points 0..i
                double* rec = stg + wave * (nmax + 4);
                double bvw = -INFINITY;
                int biw = 0x7fffffff, bsw = -1;
                if (sa >= 0 && sa < M) {
                    // K(s_l, c) for the rows l = lane, lane + 64
                    auto kdist = [&](int sl, int sc) {
                        double sq = 0.0;
                        for (int kk = 0; kk < p; ++kk) {
                            const double tt = Xc[(int64_t)kk * Mpad + sl] - Xc[(int64_t)kk * Mpad + sc];
                            sq += tt * tt;
                        }
                        return exp(-div_by(sq, theta, rtheta));
                    };
                    double a0 = 0.0, a1 = 0.0;
                    if (lane < jr) a0 = kdist(sslot[lane], sa);
                    if (lane + 64 < jr) a1 = kdist(sslot[lane + 64], sa);
                    double sqx = 0.0;
                    for (int kk = 0; kk < p; ++kk) {
                        const double tt = xl[kk] - Xc[(int64_t)kk * Mpad + sa];
                        sqx += tt * tt;
                    }
                    double vA = one_eta, cA = exp(-div_by(sqx, theta, rtheta));
                    double w0 = 0.0, w1 = 0.0;
                    // Column-oriented forward substitution over rows l = lane
                    // (and lane + 64): row l subtracts L[l][m] W_m in ascending
                    // m, as the FP64 kernel does.  Rows at or above m and lanes
                    // past jr update too but are never read again, so no lane
                    // predicate is needed.  The factor entries L[l][m..m+3] and
                    // delta, 1/delta, w_x for m..m+3 are read as a block before
                    // the block's four dependent steps (one LDS latency per
                    // block).  Every read stays in LDS: a lane past jr reads
                    // from row 0, and row l's reads end at packed_row(l) + jr + 2
                    // <= packed_row(jr) + 2, inside the arrays that follow the
                    // factor.
                    auto solve = [&](auto two) {
                        constexpr bool TWO = decltype(two)::value;
                        constexpr int U = 4;
                        const int r0 = lane < jr ? packed_row(lane) : 0;
                        const int r1 = (TWO && lane + 64 < jr) ? packed_row(lane + 64) : 0;
                        for (int m0 = 0; m0 < jr; m0 += U) {
                            double g0[U], g1[U], dm[U], rm[U], xm[U];
#pragma unroll
                            for (int q = 0; q < U; ++q) {
                                g0[q] = Lf[r0 + m0 + q];
                                g1[q] = TWO ? Lf[r1 + m0 + q] : 0.0;
                                dm[q] = dl[m0 + q];
                                rm[q] = rdl[m0 + q];
                                xm[q] = wx64[m0 + q];
                            }
                            // No branch inside a block (so the block's steps
                            // interleave): a step past jr only updates rows
                            // that are no longer read, and its v and cov terms
                            // are dropped by selects.
#pragma unroll
                            for (int q = 0; q < U; ++q) {
                                const int m = m0 + q;
                                const double am =
                                    (!TWO || m < 64) ? readlane_d(a0, m & 63) : readlane_d(a1, m & 63);
                                const double W = div_by(am, dm[q], rm[q]);
                                a0 -= g0[q] * W;
                                if constexpr (TWO) a1 -= g1[q] * W;
                                const bool ok = m < jr;
                                const double vn = vA - W * W, cn = cA - xm[q] * W;
                                vA = ok ? vn : vA;
                                cA = ok ? cn : cA;
                                w0 = lane == m ? W : w0;
                                if constexpr (TWO) w1 = lane + 64 == m ? W : w1;
                            }
                        }
                    };
                    if (jr > 64) solve(std::integral_constant<bool, true>{});
                    else solve(std::integral_constant<bool, false>{});
                    if (lane < jr) rec[lane] = w0;
                    if (lane + 64 < jr) rec[lane + 64] = w1;
                    if (vA > 0.0) {
                        double y = __builtin_amdgcn_rcp(vA);
                        y = __builtin_fma(__builtin_fma(-vA, y, 1.0), y, y);
                        bvw = (cA * cA) * y;
                    }
                    biw = ia;
                    bsw = sa;
                    if (lane == 0) {
                        rec[nmax] = vA;
                        rec[nmax + 1] = cA;
                    }
                }
                if (lane == 0) { redv[wave] = bvw; redi[wave] = biw; reds[wave] = bsw; }
                __syncthreads();   // B3: exact scores staged
            }
            if (MIX || i + 1 >= n0) {
                bv = redv[0]; bi = redi[0]; bs = reds[0];
                int bw = 0;
                // (the mixed mode's entries past NSHORT are empty)
                for (int w = 1; w < (MIX ? NSHORT : DWAVES); ++w) {
                    const int before = bs;
                    pick<true>(bv, bi, bs, redv[w], redi[w], reds[w]);
                    if (bs != before) bw = w;
                }
                if (bs < 0 || (i + 1 >= n0 && bv == -INFINITY)) { notpd = 1; continue; }
                s_next = bs;
                double vx = misc[1];
                double dN = 0.0, rdN = 0.0, rxN = 0.0;
                const double* rec = stg + bw * (nmax + 4);
                if constexpr (MIX) {
                    // the chosen point's exact row of L, w_x and u
                    const double vN = rec[nmax];
                    if (!(vN > 0.0)) { notpd = 1; continue; }
                    dN = sqrt(vN);
                    rdN = 1.0 / dN;
                    rxN = div_by(rec[nmax + 1], dN, rdN);
                    vx = vxr;
                }
                // Stopping rule: the best candidate would shrink v(x) by less
                // than the factor vratio (v_{i+1}(x) was published before B2).
                if (A.vratio > 0.0 && i + 1 >= n0) {
                    const double vnext = vx - bv;
                    if (vnext > 0.0 && vx / vnext < A.vratio) nuse = i + 1;
                }
                if (MIX && nuse == n) {
                    vxr -= rxN * rxN;
                    const int ro = packed_row(i + 1);
                    for (int e = tid; e <= i; e += DT) Lf[ro + e] = rec[e];
                    if (tid == 0) {
                        Lf[ro + i + 1] = dN;
                        dl[i + 1] = dN;
                        rdl[i + 1] = rdN;
                        wx64[i + 1] = rxN;
                        sslot[i + 1] = bs;
                    }
                }
            }
        }

        // ---- the last point: its column of W, K(s, x) and y_s give row n-1
        //      of w_x and u (no candidate row is needed).  The mixed mode
        //      appended its exact row when the point was chosen.
        if (MIX && !notpd && nuse == n && n >= 1) {
            const int s = (n - 1 < n0) ? forced[n - 1] : s_next;
            if (s < 0 || s >= M) notpd = 1;
            else if (tid == 0 && A.sel) A.sel[t * A.sel_stride + n - 1] = cand[s];
        }
        if constexpr (MIX) {
            // u = L^{-1} Y_n for the design reached, by forward substitution
            // against the exact factor, each row in the order of the FP64
            // kernel's u chain (ascending, y_s first): lane l holds row l.
            __syncthreads();
            if (!notpd && wave == 0) {
                const int jn = nuse;
                const int r0 = packed_row(lane), r1 = packed_row(lane + 64);
                double a0 = lane < jn ? A.y[cand[sslot[lane]]] : 0.0;
                double a1 = lane + 64 < jn ? A.y[cand[sslot[lane + 64]]] : 0.0;
                for (int m = 0; m < jn; ++m) {
                    const bool lo = m < 64;
                    const double um = div_by(readlane_d(lo ? a0 : a1, m & 63), dl[m], rdl[m]);
                    if (lane == 0) uu[m] = um;
                    if (lane > m && lane < jn) a0 -= Lf[r0 + m] * um;
                    if (lane + 64 > m && lane + 64 < jn) a1 -= Lf[r1 + m] * um;
                }
            }
        }
        if (!MIX && !notpd && nuse == n && n >= 1) {
            const int i = n - 1;
            const int s = (i < n0) ? forced[i] : s_next;
            if (s < 0 || s >= M) {
                notpd = 1;
            } else {
                const int s_lane = s % DT;
                if (tid == s_lane) {
                    const int kk = __builtin_amdgcn_readfirstlane(s / DT);
#pragma unroll
                    for (int k = 0; k < CPT; ++k) {
                        if (k == kk) {
#pragma unroll
                            for (int l = 0; l < (RREG > 0 ? RREG : 0); ++l)
                                if (l < i) ws[l] = Wr[l][k];
                            misc[0] = v[k];
                            ctl[1] = ci[k];
                        }
                    }
                }
                for (int l = RREG + tid; l < i; l += DT)
                    ws[l] = (TW)((l < G0) ? Wl[(int64_t)(l - RREG) * Mpad + s] : Wg[(int64_t)(l - G0) * Mpad + s]);
                __syncthreads();
                const double vs = misc[0];
                if (!(vs > 0.0)) {
                    notpd = 1;
                } else if (tid == 0) {
                    const double delta = sqrt(vs);
                    const double rdelta = 1.0 / delta;
                    double sqx = 0.0;
                    for (int kk = 0; kk < p; ++kk) {
                        const double tx = Xc[(int64_t)kk * Mpad + s] - xl[kk];
                        sqx += tx * tx;
                    }
                    double ax = exp(-div_by(sqx, theta, rtheta));
                    double ay = (CL && ylds) ? Xc[(int64_t)p * Mpad + s] : A.y[cand[s]];
                    for (int l = 0; l < i; ++l) {
                        const double wl = ws[l];
                        ax -= wl * (double)wx[l];
                        ay -= wl * uu[l];
                    }
                    wx[i] = div_by(ax, delta, rdelta);
                    uu[i] = div_by(ay, delta, rdelta);
                    if (A.sel) A.sel[t * A.sel_stride + i] = ctl[1];
                }
            }
        }

        // ---- prediction (eqs predgp, preds2 with N -> n) from w_x and u; the
        //      mixed mode uses its exact FP64 rows.
        __syncthreads();
        if (tid == 0) {
            double mean, s2v, var;
            if (notpd) {
                mean = s2v = var = NAN;
            } else {
                double m = 0.0, ps = 0.0, q = 0.0;
                for (int l = 0; l < nuse; ++l) {
                    const double wl = MIX ? wx64[l] : (double)wx[l];
                    m += wl * uu[l];
                    ps += uu[l] * uu[l];
                    q += wl * wl;
                }
                const double vxn = one_eta - q;
                mean = m;
                s2v = ps * vxn / nuse;
                var = nuse > 2 ? ps * vxn / (nuse - 2) : NAN;
            }
            A.mean[t] = mean;
            A.s2[t] = s2v;
            if (A.var) A.var[t] = var;
            if (A.df) A.df[t] = nuse;
            if (A.status) A.status[t] = nocand ? 3 : badstart ? 2 : notpd ? 1 : 0;
        }
        __syncthreads();
    }
}

// With `a` null the kernel variant's dynamic-LDS limit is raised (host-side
// set-up, kept out of stream capture); otherwise the kernel is launched.
template <int DT, int CPT, int P, bool CL, int MIX, bool TRIM>
static int launch_design(const DesignArgs* a, const DesignPlan& plan, hipStream_t stream, std::string* err)
{
    constexpr int RREG = rreg_for(DT, CPT, CL, MIX, TRIM);
    auto kern = design_kernel<DT, CPT, RREG, P, CL, MIX, TRIM>;
    if (!a) {
        // Plans of one variant may differ in LDS size and a captured graph may
        // launch any of them: the limit is the device's.
        if (!set_lds_limit((const void*)kern, plan.lds_limit, plan.lds_bytes)) {
            *err = "cannot reserve LDS for the design kernel";
            return -2;
        }
        return 0;
    }
    hipLaunchKernelGGL(kern, dim3(plan.blocks), dim3(DT), plan.lds_bytes, stream, *a);
    if (hipGetLastError() != hipSuccess) { *err = "design kernel launch failed"; return -2; }
    return 0;
}

template <int DT, int CPT, bool CL, int MIX, bool TRIM>
static int launch_design_p(const DesignArgs* a, const DesignPlan& plan, hipStream_t stream, std::string* err)
{
    switch (plan.p) {
    case 2: return launch_design<DT, CPT, 2, CL, MIX, TRIM>(a, plan, stream, err);
    case 4: return launch_design<DT, CPT, 4, CL, MIX, TRIM>(a, plan, stream, err);
    case 8: return launch_design<DT, CPT, 8, CL, MIX, TRIM>(a, plan, stream, err);
    default: return launch_design<DT, CPT, 0, CL, MIX, TRIM>(a, plan, stream, err);
    }
}

template <int DT, int CPT, int MIX, bool TRIM>
static int launch_design_c(const DesignArgs* a, const DesignPlan& plan, hipStream_t stream, std::string* err)
{
    return plan.coords_lds ? launch_design_p<DT, CPT, true, MIX, TRIM>(a, plan, stream, err)
                           : launch_design_p<DT, CPT, false, MIX, TRIM>(a, plan, stream, err);
}

template <int DT, int MIX, bool TRIM>
static int launch_design_dt(const DesignArgs* a, const DesignPlan& plan, hipStream_t stream, std::string* err)
{
    switch (plan.cpt) {
    case 1: return launch_design_c<DT, 1, MIX, TRIM>(a, plan, stream, err);
    case 2: return launch_design_c<DT, 2, MIX, TRIM>(a, plan, stream, err);
    case 4: return launch_design_c<DT, 4, MIX, TRIM>(a, plan, stream, err);
    case 8: return launch_design_c<DT, 8, MIX, TRIM>(a, plan, stream, err);
    default: return launch_design_c<DT, 8, MIX, TRIM>(a, plan, stream, err);
    }
}

// One translation unit per (tile precision, TRIM) pair instantiates its variants.
template <int MIX, bool TRIM>
static int launch_variant(const DesignArgs* a, const DesignPlan& plan, hipStream_t stream, std::string* err)
{
    return plan.threads == 256 ? launch_design_dt<256, MIX, TRIM>(a, plan, stream, err)
                               : launch_design_dt<512, MIX, TRIM>(a, plan, stream, err);
}

int design_launch_f64(const DesignArgs* a, const DesignPlan& plan, hipStream_t stream, std::string* err);
int design_launch_f64_trim(const DesignArgs* a, const DesignPlan& plan, hipStream_t stream, std::string* err);
int design_launch_mix(const DesignArgs* a, const DesignPlan& plan, hipStream_t stream, std::string* err);
int design_launch_mix_trim(const DesignArgs* a, const DesignPlan& plan, hipStream_t stream, std::string* err);
int design_launch_bf16(const DesignArgs* a, const DesignPlan& plan, hipStream_t stream, std::string* err);
int design_launch_bf16_trim(const DesignArgs* a, const DesignPlan& plan, hipStream_t stream, std::string* err);

}  // namespace lagp
