// knn.hip -- exact brute-force nearest-neighbour candidate sets for gfx950.
//
// For every predictive location x_t the M design points with the smallest
// (squared distance, index) keys are selected (the nearest-neighbour
// sub-design of Section 3 and the N' nearest candidates of Section 6).
//
// Key: a 96-bit integer (bits of the non-negative FP64 squared distance) << 31
// | design index.  Non-negative doubles order like their bit patterns, so the
// integer order is exactly the (distance, index) order and every key is
// unique.  The M-th smallest key is found by radix refinement of a key window:
//
//   pass 0   64 bins over the binary exponent of d^2 (octaves 2^-51..2^11,
//            clamped at both ends);
//   pass k   64 equal bins over the current window;
// until the window holds at most BUCKET_MAX keys (or one key).  A collect
// pass then writes every key below the window straight to the output and the
// keys inside the window to a small per-location bucket, which a finalise
// kernel sorts to fill the remaining slots.
//
// Mapping: one thread per location, 256 locations per block.  Every lane of
// a wave tests the same design row at a time, so the rows (row-major copy)
// are read with wave-uniform addresses: scalar loads into SGPRs that feed the
// FP64 subtractions directly, with no LDS staging, no LDS broadcast traffic
// and no barriers in the scan.  Histograms are private per thread in LDS, so
// no thread shares a counter inside a block.  The design range is split over
// gridDim.y blocks to fill the chip; partial histograms then meet in global
// memory through atomics.
//
// Squared distances are summed over coordinates left to right with no fused
// multiply-add (this file is compiled with -ffp-contract=off).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "lagp_internal.h"

namespace lagp {

typedef unsigned __int128 u128;

#define KNN_THREADS 256
#define KNN_BINS 64
#define KNN_GRANULE 256 // rows: a design split is a multiple of this
#define KNN_MAX_PASSES 18
#define KNN_STAGE 16   // collected indices staged per thread before one slot reservation
#define KNN_KSTAGE 8   // window keys staged per thread before one bucket-slot reservation
#define KNN_COVER 32   // blocks per CU a split design aims for
#define KNN_MIN_CHUNK 8 // granules per split, at least
#define KNN_GROUP 4    // design rows whose distances are computed together

struct KnnState {
    uint64_t lo_hi, lo_lo;   // window lower bound (128-bit key)
    uint64_t hi_hi, hi_lo;   // window upper bound, exclusive
    uint32_t below;          // keys strictly below lo
    uint32_t bucket;         // keys inside the window (valid once settled)
    int32_t settled;         // 1: window final
    int32_t pass;            // passes run so far
    int32_t count_below;     // 1: the window was estimated, the next pass counts the keys below it
    int32_t misses;          // estimated windows that missed the M-th key
};

__device__ __forceinline__ u128 mk128(uint64_t h, uint64_t l) { return ((u128)h << 64) | l; }
__device__ __forceinline__ uint64_t hi64(u128 v) { return (uint64_t)(v >> 64); }
__device__ __forceinline__ uint64_t lo64(u128 v) { return (uint64_t)v; }

__device__ __forceinline__ int ceil_log2_128(u128 w)
{
    // smallest s with 2^s >= w (w >= 1)
    u128 v = w - 1;
    int s = 0;
    while (v) { v >>= 1; ++s; }
    return s;
}

// Squared distance of a design row to x, left to right.  P > 0 is the
// dimension known at compile time (x in registers); P == 0 reads a runtime
// dimension p with x kept in LDS.
template <int P>
__device__ __forceinline__ double row_d2(const double* __restrict__ pt, const double* x, int p)
{
    double s = 0.0;
    if (P > 0) {
#pragma unroll
        for (int k = 0; k < P; ++k) {
            double t = pt[k] - x[k];
            s += t * t;
        }
    } else {
        for (int k = 0; k < p; ++k) {
            double t = pt[k] - x[k * KNN_THREADS];
            s += t * t;
        }
    }
    return s;
}

// Visit design rows [i0, i1) of the row-major Xa in index order, calling
// f(d2, row) for each.  The row index is wave-uniform, so the row reads are
// scalar loads; distances are computed KNN_GROUP rows at a time before any
// of them is used, so the loads of a group are in flight together.
template <int P, class F>
__device__ __forceinline__ void scan_rows(const double* __restrict__ Xa, int64_t i0, int64_t i1,
                                          const double* x, int p, F& f)
{
    const int64_t pp = P > 0 ? P : p;
    int64_t i = i0;
    for (; i + KNN_GROUP <= i1; i += KNN_GROUP) {
        double d[KNN_GROUP];
#pragma unroll
        for (int u = 0; u < KNN_GROUP; ++u) d[u] = row_d2<P>(Xa + (i + u) * pp, x, p);
#pragma unroll
        for (int u = 0; u < KNN_GROUP; ++u) f(d[u], i + u);
    }
    for (; i < i1; ++i) f(row_d2<P>(Xa + i * pp, x, p), i);
}

// Pass 0 bin of a squared distance: its octave, clamped to [2^-51, 2^11).
__device__ __forceinline__ int exp_bin(uint64_t bits)
{
    int e = (int)(bits >> 52) - 971;
    return e < 0 ? 0 : (e > 63 ? 63 : e);
}

// Key window of pass 0 bin b.
__device__ __forceinline__ void exp_bin_window(int b, u128* lo, u128* hi)
{
    const u128 top = (u128)1 << 94;
    *lo = (b == 0) ? (u128)0 : ((u128)(uint64_t)(b + 971) << 83);
    *hi = (b == 63) ? top : ((u128)(uint64_t)(b + 972) << 83);
}

__global__ void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t v)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = v;
}

void fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
}

__global__ void knn_init_kernel(KnnState* st, uint32_t* hist, int64_t T)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    KnnState s;
    s.lo_hi = s.lo_lo = 0;
    s.hi_hi = (uint64_t)1 << 30;  // 2^94
    s.hi_lo = 0;
    s.below = 0;
    s.bucket = 0;
    s.settled = 0;
    s.pass = 0;
    s.count_below = 0;
    s.misses = 0;
    st[t] = s;
    for (int b = 0; b < KNN_BINS; ++b) hist[t * KNN_BINS + b] = 0;
}

// One histogram pass over design rows [i0, i1) for the 256 locations of this
// block.  Pass kind is taken per location from its state.
template <int P>
__global__ void __launch_bounds__(KNN_THREADS)
knn_hist_kernel(const double* __restrict__ Xa, int64_t N, int p, const double* __restrict__ XX,
                int64_t T, int32_t M, KnnState* __restrict__ st, uint32_t* __restrict__ hist,
                uint32_t* __restrict__ belowc, int64_t chunk)
{
    extern __shared__ double smem[];
    // Private histogram: two 16-bit counters per word (a split holds fewer
    // than 65536 design rows, so no count carries into its neighbour), bumped
    // with LDS atomic adds whose result is unused: no wait on an LDS read.
    uint32_t* hw = (uint32_t*)smem;                               // KNN_BINS / 2 * KNN_THREADS

    const int tid = threadIdx.x;
    const int64_t t = (int64_t)blockIdx.x * KNN_THREADS + tid;
    const int64_t i0 = (int64_t)blockIdx.y * chunk;
    const int64_t i1 = (i0 + chunk < N) ? i0 + chunk : N;

    bool active = false;
    int kind = 0;
    bool cbelow = false;
    uint32_t nbelow = 0;   // keys below an estimated window (count_below)
    u128 lo = 0, hi = 0;
    int shift = 0;
    double xr[P > 0 ? P : 1];
    double* xl = (double*)(hw + KNN_BINS / 2 * KNN_THREADS) + tid;  // P == 0: x in LDS
    const double* x = P > 0 ? xr : xl;
    if (t < T) {
        KnnState s = st[t];
        active = !s.settled;
        kind = s.pass == 0 ? 0 : 1;
        cbelow = s.count_below != 0;
        lo = mk128(s.lo_hi, s.lo_lo);
        hi = mk128(s.hi_hi, s.hi_lo);
        shift = ceil_log2_128(hi - lo) - 6;
        if (shift < 0) shift = 0;
        if (P > 0) {
#pragma unroll
            for (int k = 0; k < (P > 0 ? P : 1); ++k) xr[k] = XX[t * p + k];
        } else {
            for (int k = 0; k < p; ++k) xl[k * KNN_THREADS] = XX[t * p + k];
        }
    }
    if (!active) return;   // (no barriers below)

    for (int w = 0; w < KNN_BINS / 2; ++w) hw[w * KNN_THREADS + tid] = 0;
    auto bump = [&](int b) { atomicAdd(hw + (b >> 1) * KNN_THREADS + tid, 1u << ((b & 1) << 4)); };
    const uint64_t lo_d = (uint64_t)(lo >> 31);
    const uint64_t hi_d = (uint64_t)((hi - 1) >> 31);
    // Window bounds on whole squared-distance values (the index bits zero)
    // and bins at least one distance unit wide: bins follow from the
    // distance bits alone.
    const u128 low31 = ((u128)1 << 31) - 1;
    const bool aligned = ((lo & low31) == 0) && ((hi & low31) == 0) && shift >= 31;

    if (kind == 0) {
        auto bin = [&](double d2, int64_t) {
            bump(exp_bin((uint64_t)__double_as_longlong(d2)));
        };
        scan_rows<P>(Xa, i0, i1, x, p, bin);
    } else if (__all(aligned)) {
        // Every window of the wave (and so every bin) is bounded by whole
        // distance values: 64-bit arithmetic on the distance bits decides
        // each key, with no per-row choice between the two forms below.
        const int sh = shift - 31;
        auto bin = [&](double d2, int64_t) {
            uint64_t bits = (uint64_t)__double_as_longlong(d2);
            const bool under = bits < lo_d;
            nbelow += (under && cbelow) ? 1u : 0u;
            if (under || bits > hi_d) return;
            bump((int)((bits - lo_d) >> sh));
        };
        scan_rows<P>(Xa, i0, i1, x, p, bin);
    } else {
        auto bin = [&](double d2, int64_t gi) {
            uint64_t bits = (uint64_t)__double_as_longlong(d2);
            const bool under = bits < lo_d;
            nbelow += (under && cbelow) ? 1u : 0u;
            if (under || bits > hi_d) return;
            int b;
            if (aligned) {
                // the window and its bins are whole distance values: 64-bit arithmetic
                b = (int)((bits - lo_d) >> (shift - 31));
            } else {
                u128 key = ((u128)bits << 31) | (uint64_t)gi;
                if (key < lo) { nbelow += cbelow ? 1u : 0u; return; }
                if (key >= hi) return;
                b = (int)((key - lo) >> shift);
            }
            bump(b);
        };
        scan_rows<P>(Xa, i0, i1, x, p, bin);
    }
    if (cbelow && nbelow) {
        if (gridDim.y == 1) belowc[t] += nbelow;
        else atomicAdd(belowc + t, nbelow);
    }
    uint32_t* hg = hist + t * KNN_BINS;
    for (int b = 0; b < KNN_BINS; ++b) {
        uint32_t c = (hw[(b >> 1) * KNN_THREADS + tid] >> ((b & 1) << 4)) & 0xffffu;
        if (c) {
            if (gridDim.y == 1) hg[b] += c;
            else atomicAdd(hg + b, c);
        }
    }
}

// Choose the bin holding the M-th key; settle or narrow the window.
// Key window of squared distances [a, b] (both non-negative): keys whose
// distance bits lie in [bits(a), bits(b)]; the whole key range if empty.
__device__ __forceinline__ void d2_window(double a, double b, u128* lo, u128* hi)
{
    const u128 top = (u128)1 << 94;
    const uint64_t ab = (uint64_t)__double_as_longlong(a);
    const uint64_t bb = (uint64_t)__double_as_longlong(b);
    u128 nlo = (u128)ab << 31, nhi = (u128)(bb + 1) << 31;
    if (nhi > top) nhi = top;
    if (nlo >= nhi) { nlo = 0; nhi = top; }   // (non-finite distances) the whole key range
    *lo = nlo;
    *hi = nhi;
}

__device__ __forceinline__ double key_d2(u128 key)
{
    return __longlong_as_double((long long)(uint64_t)(key >> 31));
}

// On the design sample (mdiv = the sample stride) the target rank is
// ceil(M / mdiv); bucket_max = 0 there keeps refining.
__global__ void knn_decide_kernel(KnnState* st, uint32_t* hist, uint32_t* belowc, int64_t T, int32_t M_all,
                                  const int32_t* __restrict__ M_per, int32_t mdiv, int32_t bucket_max, double fac,
                                  uint32_t* unsettled)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    // Per-location sizes are clamped to the row length M_all (invalid sizes
    // are rejected before launch, or flagged by the design kernel).
    int32_t M = M_per ? (M_per[t] < M_all ? M_per[t] : M_all) : M_all;
    M = (M + mdiv - 1) / mdiv;
    KnnState s = st[t];
    if (s.settled) return;
    uint32_t* hg = hist + t * KNN_BINS;
    uint32_t cum = s.below;
    if (s.count_below) {
        // The window came from the sample: the pass counted the keys below it.
        s.count_below = 0;
        cum = belowc[t];
        belowc[t] = 0;
        uint32_t inwin = 0;
        for (int k = 0; k < KNN_BINS; ++k) inwin += hg[k];
        const u128 olo = mk128(s.lo_hi, s.lo_lo), ohi = mk128(s.hi_hi, s.hi_lo);
        if (cum >= (uint32_t)M || cum + inwin < (uint32_t)M) {
            const bool below = cum >= (uint32_t)M;
            u128 lo, hi;
            if (s.misses == 0) {
                // First miss: an estimated window again, on the missed side and
                // wider (squared distances by the factor 9^(2/p) = (3^(2/p))^2).
                const double f = fac * fac;
                if (below) d2_window(key_d2(olo) / f, key_d2(olo), &lo, &hi);
                else d2_window(key_d2(ohi), key_d2(ohi - 1) * f, &lo, &hi);
                if (below && hi > olo) hi = olo;
                if (!below && lo < ohi) lo = ohi;
                s.count_below = 1;
            } else {
                // Then the whole key range on the missed side, refined as usual:
                // [0, lo) holding `cum` keys, or [hi, 2^94) above cum + inwin keys.
                lo = below ? (u128)0 : ohi;
                hi = below ? olo : ((u128)1 << 94);
                s.below = below ? 0u : cum + inwin;
            }
            s.misses += 1;
            s.lo_hi = hi64(lo); s.lo_lo = lo64(lo);
            s.hi_hi = hi64(hi); s.hi_lo = lo64(hi);
            s.bucket = 0;
            s.pass += 1;
            s.settled = 0;
            st[t] = s;
            for (int k = 0; k < KNN_BINS; ++k) hg[k] = 0;
            atomicAdd(unsettled, 1u);
            return;
        }
    }
    int b = 0;
    for (; b < KNN_BINS - 1; ++b) {
        if (cum + hg[b] >= (uint32_t)M) break;
        cum += hg[b];
    }
    uint32_t inbin = hg[b];
    u128 lo, hi;
    if (s.pass == 0) {   // octave histogram
        exp_bin_window(b, &lo, &hi);
    } else {
        u128 olo = mk128(s.lo_hi, s.lo_lo), ohi = mk128(s.hi_hi, s.hi_lo);
        int shift = ceil_log2_128(ohi - olo) - 6;
        if (shift < 0) shift = 0;
        lo = olo + ((u128)(uint64_t)b << shift);
        hi = lo + ((u128)1 << shift);
        if (hi > ohi) hi = ohi;
    }
    s.lo_hi = hi64(lo); s.lo_lo = lo64(lo);
    s.hi_hi = hi64(hi); s.hi_lo = lo64(hi);
    s.below = cum;
    s.bucket = inbin;
    s.pass += 1;
    s.settled = (inbin <= (uint32_t)bucket_max) || (hi - lo <= 1);
    st[t] = s;
    for (int k = 0; k < KNN_BINS; ++k) hg[k] = 0;
    if (!s.settled) atomicAdd(unsettled, 1u);
}

// From the window that holds the sample's ceil(M / stride)-th key, estimate
// the full design's window: squared distances in [lo / fac, hi * fac] with
// fac = 3^(2/p), i.e. expected ranks from M/3 to 3M where the neighbour count
// grows like distance^p.  The next full pass counts the keys below it
// (count_below); the decide kernel handles an estimate that misses.
__global__ void knn_estimate_kernel(KnnState* st, int64_t T, double fac)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    KnnState s = st[t];
    const u128 lo = mk128(s.lo_hi, s.lo_lo), hi = mk128(s.hi_hi, s.hi_lo);
    u128 nlo, nhi;
    d2_window(key_d2(lo) / fac, key_d2(hi - 1) * fac, &nlo, &nhi);
    s.lo_hi = hi64(nlo); s.lo_lo = lo64(nlo);
    s.hi_hi = hi64(nhi); s.hi_lo = lo64(nhi);
    s.below = 0;
    s.bucket = 0;
    s.settled = 0;
    s.pass = 1;
    s.count_below = 1;
    st[t] = s;
}

// Collect: keys below the window go to idx[t][*]; keys inside the window go
// to the bucket with their full key.  When the design is split over several
// blocks (gridDim.y > 1) a location's output and bucket slots are reserved
// with atomics, KNN_STAGE indices or KNN_KSTAGE keys at a time from
// per-thread LDS stages, so no row waits on an atomic's result.
template <int P>
__global__ void __launch_bounds__(KNN_THREADS)
knn_collect_kernel(const double* __restrict__ Xa, int64_t N, int p, const double* __restrict__ XX,
                   int64_t T, const KnnState* __restrict__ st, uint32_t* __restrict__ counts,
                   int32_t* __restrict__ idx, int64_t idx_stride, uint64_t* __restrict__ bucket,
                   int32_t bucket_max, int64_t chunk)
{
    extern __shared__ double smem[];
    const int tid = threadIdx.x;
    const int64_t t = (int64_t)blockIdx.x * KNN_THREADS + tid;
    const int64_t i0 = (int64_t)blockIdx.y * chunk;
    const int64_t i1 = (i0 + chunk < N) ? i0 + chunk : N;
    const bool split = gridDim.y > 1;

    bool active = t < T;
    u128 lo = 0, hi = 0;
    double xr[P > 0 ? P : 1];
    double* xl = smem + tid;  // P == 0: x in LDS
    int32_t* stage = (int32_t*)(smem + (P > 0 ? 0 : (size_t)KNN_THREADS * p));
    uint64_t* kbits = (uint64_t*)(stage + KNN_STAGE * KNN_THREADS);   // staged window keys: distance bits
    uint32_t* kidx = (uint32_t*)(kbits + KNN_KSTAGE * KNN_THREADS);   // and design index
    int ns = 0;   // staged indices of this thread
    int nk = 0;   // staged window keys of this thread
    const double* x = P > 0 ? xr : xl;
    uint32_t nbelow = 0, nbkt = 0;
    if (active) {
        KnnState s = st[t];
        lo = mk128(s.lo_hi, s.lo_lo);
        hi = mk128(s.hi_hi, s.hi_lo);
        if (P > 0) {
#pragma unroll
            for (int k = 0; k < (P > 0 ? P : 1); ++k) xr[k] = XX[t * p + k];
        } else {
            for (int k = 0; k < p; ++k) xl[k * KNN_THREADS] = XX[t * p + k];
        }
    }
    const uint64_t lo_d = (uint64_t)(lo >> 31);
    const uint64_t hi_d = (uint64_t)((hi - 1) >> 31);
    if (!active) return;   // (no barriers below)
    int32_t* out = idx + t * idx_stride;
    uint64_t* bk = bucket + t * (int64_t)bucket_max * 2;
    auto put = [&](uint32_t slot, uint64_t bits, uint32_t gi) {
        if (slot < (uint32_t)bucket_max) {
            const u128 key = ((u128)bits << 31) | gi;
            bk[2 * slot] = hi64(key);
            bk[2 * slot + 1] = lo64(key);
        }
    };
    auto flush_keys = [&](int n) {
        const uint32_t b0 = atomicAdd(counts + 2 * t + 1, (uint32_t)n);
        for (int j = 0; j < n; ++j) put(b0 + j, kbits[j * KNN_THREADS + tid], kidx[j * KNN_THREADS + tid]);
    };
    // Windows bounded by whole distance values (the low 31 key bits zero at
    // both ends) are decided by the distance bits alone: key < lo exactly
    // when bits < lo_d, and key < hi exactly when bits <= hi_d.
    const u128 low31 = ((u128)1 << 31) - 1;
    const bool aligned = ((lo & low31) == 0) && ((hi & low31) == 0);
    const bool fast = __all(aligned);
    auto take = [&](double d2, int64_t gi) {
        uint64_t bits = (uint64_t)__double_as_longlong(d2);
        if (bits > hi_d) return;
        // the full key only at or above the window's first distance value
        const bool under = bits < lo_d;
        u128 key = 0;
        if (!under && !fast) key = ((u128)bits << 31) | (uint64_t)gi;
        if (under || (!fast && key < lo)) {
            if (!split) {
                out[nbelow++] = (int32_t)gi;
            } else {
                stage[ns * KNN_THREADS + tid] = (int32_t)gi;
                if (++ns == KNN_STAGE) {
                    const uint32_t b0 = atomicAdd(counts + 2 * t, (uint32_t)KNN_STAGE);
#pragma unroll
                    for (int j = 0; j < KNN_STAGE; ++j) out[b0 + j] = stage[j * KNN_THREADS + tid];
                    ns = 0;
                }
            }
        } else if (fast || key < hi) {
            if (!split) {
                put(nbkt++, bits, (uint32_t)gi);
            } else {
                kbits[nk * KNN_THREADS + tid] = bits;
                kidx[nk * KNN_THREADS + tid] = (uint32_t)gi;
                if (++nk == KNN_KSTAGE) {
                    flush_keys(KNN_KSTAGE);
                    nk = 0;
                }
            }
        }
    };
    scan_rows<P>(Xa, i0, i1, x, p, take);
    if (split && ns > 0) {
        const uint32_t b0 = atomicAdd(counts + 2 * t, (uint32_t)ns);
        for (int j = 0; j < ns; ++j) out[b0 + j] = stage[j * KNN_THREADS + tid];
    }
    if (split && nk > 0) flush_keys(nk);
    if (!split) {
        counts[2 * t] = nbelow;
        counts[2 * t + 1] = nbkt;
    }
}

// Sort each location's bucket (at most bucket_max keys, bucket_max a power of
// two <= 1024) and append its smallest M - below keys.  One block per location.
__global__ void __launch_bounds__(KNN_THREADS)
knn_finalize_kernel(int64_t T, int32_t M_all, const int32_t* __restrict__ M_per, const KnnState* __restrict__ st,
                    const uint32_t* __restrict__ counts, int32_t* __restrict__ idx,
                    int64_t idx_stride, const uint64_t* __restrict__ bucket, int32_t bucket_max,
                    int32_t* __restrict__ bad)
{
    __shared__ uint64_t kh[1024], kl[1024];
    const int64_t t = blockIdx.x;
    if (t >= T) return;
    const int32_t M = M_per ? (M_per[t] < M_all ? M_per[t] : M_all) : M_all;
    const KnnState s = st[t];
    const uint32_t nb = counts[2 * t], nk = counts[2 * t + 1];
    const int tid = threadIdx.x;
    if (!s.settled || nb != s.below || nk != s.bucket || nb + nk < (uint32_t)M || nk > (uint32_t)bucket_max) {
        // Cannot happen for finite inputs.  Mark the row (-1 entries: the
        // design kernel then fails the location with LAGP_LOC_NOCAND) and
        // report through the flag, which calls that wait on the host read.
        int32_t* row = idx + t * idx_stride;
        for (int e = tid; e < M; e += KNN_THREADS) row[e] = -1;
        if (tid == 0) atomicAdd(bad, 1);
        return;
    }
    const uint64_t* bk = bucket + t * (int64_t)bucket_max * 2;
    int P = 1;
    while (P < (int)nk) P <<= 1;
    for (int e = tid; e < P; e += KNN_THREADS) {
        if (e < (int)nk) { kh[e] = bk[2 * e]; kl[e] = bk[2 * e + 1]; }
        else { kh[e] = ~0ull; kl[e] = ~0ull; }
    }
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int e = tid; e < P; e += KNN_THREADS) {
                int partner = e ^ stride;
                if (partner > e) {
                    bool up = (e & size) == 0;
                    u128 a = mk128(kh[e], kl[e]), b = mk128(kh[partner], kl[partner]);
                    if ((a > b) == up) {
                        kh[e] = hi64(b); kl[e] = lo64(b);
                        kh[partner] = hi64(a); kl[partner] = lo64(a);
                    }
                }
            }
            __syncthreads();
        }
    }
    const int need = M - (int)nb;
    int32_t* out = idx + t * idx_stride + nb;
    for (int e = tid; e < need; e += KNN_THREADS)
        out[e] = (int32_t)(kl[e] & 0x7fffffffull);
}

// Sort a location's M indices by (squared distance, index): used only when a
// caller asks for ordered candidate lists.  One block per location, M <= 4096.
__global__ void __launch_bounds__(KNN_THREADS)
knn_sort_kernel(const double* __restrict__ Xaos, int p, const double* __restrict__ XX, int64_t T,
                int32_t M, int32_t* __restrict__ idx, int64_t idx_stride)
{
    __shared__ uint64_t kh[4096];
    __shared__ uint32_t ki[4096];
    const int64_t t = blockIdx.x;
    if (t >= T) return;
    const int tid = threadIdx.x;
    int32_t* row = idx + t * idx_stride;
    const double* x = XX + t * p;
    int P = 1;
    while (P < M) P <<= 1;
    for (int e = tid; e < P; e += KNN_THREADS) {
        if (e < M) {
            int32_t i = row[e];
            const double* xi = Xaos + (int64_t)i * p;
            double s = 0.0;
            for (int k = 0; k < p; ++k) {
                double d = xi[k] - x[k];
                s += d * d;
            }
            kh[e] = (uint64_t)__double_as_longlong(s);
            ki[e] = (uint32_t)i;
        } else {
            kh[e] = ~0ull;
            ki[e] = 0xffffffffu;
        }
    }
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int e = tid; e < P; e += KNN_THREADS) {
                int partner = e ^ stride;
                if (partner > e) {
                    bool up = (e & size) == 0;
                    bool gt = kh[e] > kh[partner] || (kh[e] == kh[partner] && ki[e] > ki[partner]);
                    if (gt == up) {
                        uint64_t th = kh[e]; kh[e] = kh[partner]; kh[partner] = th;
                        uint32_t ti = ki[e]; ki[e] = ki[partner]; ki[partner] = ti;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int e = tid; e < M; e += KNN_THREADS) row[e] = (int32_t)ki[e];
}

// ---------------------------------------------------------------- launcher
size_t knn_workspace_bytes(int64_t T, int32_t bucket_max)
{
    size_t b = 0;
    b += align256((size_t)T * sizeof(KnnState));
    b += align256((size_t)T * KNN_BINS * sizeof(uint32_t));
    b += align256((size_t)T * 2 * sizeof(uint32_t));
    b += align256((size_t)T * bucket_max * 2 * sizeof(uint64_t));
    b += align256((size_t)T * sizeof(uint32_t));   // keys below an estimated window
    b += align256(4 * sizeof(uint32_t));
    return b;
}

// Split a design of N rows over gridDim.y so that the grid covers the chip
// about KNN_COVER times over, keeping at least KNN_MIN_CHUNK granules per split and at most
// 65280 rows per split (16-bit private histogram counters).
static void knn_split(int64_t N, int64_t nblk, int num_cu, int64_t* chunk_out, int64_t* split_out)
{
    int64_t split = ((int64_t)KNN_COVER * num_cu + nblk - 1) / nblk;
    int64_t max_split = (N + KNN_MIN_CHUNK * KNN_GRANULE - 1) / (KNN_MIN_CHUNK * KNN_GRANULE);
    if (split > max_split) split = max_split;
    if (split < 1) split = 1;
    if (split > 65535) split = 65535;
    const int64_t max_chunk = 65280;
    if (split < (N + max_chunk - 1) / max_chunk) split = (N + max_chunk - 1) / max_chunk;
    int64_t chunk = (N + split - 1) / split;
    chunk = (chunk + KNN_GRANULE - 1) / KNN_GRANULE * KNN_GRANULE;
    *chunk_out = chunk;
    *split_out = (N + chunk - 1) / chunk;
}

static void knn_lds(int p, size_t* lds_hist, size_t* lds_coll)
{
    const size_t lds_x = p <= 8 ? 0 : (size_t)KNN_THREADS * p * sizeof(double);
    *lds_hist = (size_t)KNN_BINS * KNN_THREADS * 2 + lds_x;
    *lds_coll = lds_x + (size_t)KNN_STAGE * KNN_THREADS * sizeof(int32_t) +
                (size_t)KNN_KSTAGE * KNN_THREADS * (sizeof(uint64_t) + sizeof(uint32_t));
}

int knn_prepare(int p, size_t max_lds, std::string* err)
{
    size_t lds_hist, lds_coll;
    knn_lds(p, &lds_hist, &lds_coll);
    if (lds_hist > max_lds || lds_coll > max_lds) { *err = "input dimension too large for the kNN kernels"; return -1; }
#define LAGP_KNN_ATTR(PP)                                                                              \
    if (!set_lds_limit((const void*)knn_hist_kernel<PP>, max_lds) ||                                 \
        !set_lds_limit((const void*)knn_collect_kernel<PP>, max_lds)) {                               \
        *err = "cannot reserve LDS for the kNN kernels";                                              \
        return -2;                                                                                     \
    }
    LAGP_DISPATCH_P(p, LAGP_KNN_ATTR);
#undef LAGP_KNN_ATTR
    return 0;
}

int knn_run(const DeviceDesign& D, const double* XX, int64_t T, int32_t M, const int32_t* M_per,
            int32_t* idx, int64_t idx_stride, bool sorted, void* ws, size_t ws_bytes, hipStream_t stream,
            int num_cu, size_t max_lds, std::string* err, bool graph_safe)
{
    if (T == 0) return 0;
    const int32_t bucket_max = KNN_BUCKET_MAX;
    if (ws_bytes < knn_workspace_bytes(T, bucket_max)) { *err = "knn workspace too small"; return -1; }
    char* w = (char*)ws;
    KnnState* st = (KnnState*)w; w += align256((size_t)T * sizeof(KnnState));
    uint32_t* hist = (uint32_t*)w; w += align256((size_t)T * KNN_BINS * sizeof(uint32_t));
    uint32_t* counts = (uint32_t*)w; w += align256((size_t)T * 2 * sizeof(uint32_t));
    uint64_t* bucket = (uint64_t*)w; w += align256((size_t)T * bucket_max * 2 * sizeof(uint64_t));
    uint32_t* belowc = (uint32_t*)w; w += align256((size_t)T * sizeof(uint32_t));
    uint32_t* flags = (uint32_t*)w;  // [0] unsettled, [1] bad

    const int64_t nblk = (T + KNN_THREADS - 1) / KNN_THREADS;
    int64_t chunk, split, chunk_s = 0, split_s = 0;
    knn_split(D.N, nblk, num_cu, &chunk, &split);
    // Estimate each location's candidate radius on the design sample first
    // when the sample holds enough rows (two cheap passes replace the first
    // full octave pass).
    const bool use_sample = D.Xaos_s && D.Ns >= 2 * KNN_GRANULE && (int64_t)M * 8 <= D.N;
    const double fac = pow(3.0, 2.0 / D.p);   // 3^(2/p)
    if (use_sample) knn_split(D.Ns, nblk, num_cu, &chunk_s, &split_s);
    size_t lds_hist, lds_coll;
    knn_lds(D.p, &lds_hist, &lds_coll);
    if (lds_hist > max_lds || lds_coll > max_lds) { *err = "input dimension too large for the kNN kernels"; return -1; }
    if (!graph_safe && knn_prepare(D.p, max_lds, err)) return -2;

    hipLaunchKernelGGL(knn_init_kernel, dim3((unsigned)((T + 255) / 256)), dim3(256), 0, stream, st, hist, T);
    fill_u32(flags, 4, 0u, stream);
    fill_u32(belowc, T, 0u, stream);
    const dim3 grid((unsigned)nblk, (unsigned)split);
    const unsigned dgrid = (unsigned)((T + 255) / 256);
    if (use_sample) {
        // Octave pass and one refinement on the sample (never settling), then
        // the estimated window for the full design.
        const dim3 grid_s((unsigned)nblk, (unsigned)split_s);
        for (int pass = 0; pass < 2; ++pass) {
#define LAGP_KNN_HIST(PP) hipLaunchKernelGGL(knn_hist_kernel<PP>, grid_s, dim3(KNN_THREADS), lds_hist, stream, \
                                             D.Xaos_s, D.Ns, D.p, XX, T, M, st, hist, belowc, chunk_s)
            LAGP_DISPATCH_P(D.p, LAGP_KNN_HIST);
#undef LAGP_KNN_HIST
            hipLaunchKernelGGL(knn_decide_kernel, dim3(dgrid), dim3(256), 0, stream, st, hist, belowc, T, M, M_per,
                               (int32_t)KNN_SAMPLE_STRIDE, 0, fac, flags);
        }
        hipLaunchKernelGGL(knn_estimate_kernel, dim3(dgrid), dim3(256), 0, stream, st, T, fac);
    }
    // Without the sample the first pass leaves a key window at most 2^93
    // wide.  With it, the estimated window and one widened retry may miss,
    // leaving at most 2^94, which 16 refinements settle: 18 passes in all.
    // Each refinement divides the width by 64.
    // Without a host round trip (graph capture) all passes are launched;
    // blocks whose locations have settled return at once.
    for (int pass = 0; pass < KNN_MAX_PASSES; ++pass) {
#define LAGP_KNN_HIST(PP) hipLaunchKernelGGL(knn_hist_kernel<PP>, grid, dim3(KNN_THREADS), lds_hist, stream, \
                                             D.Xaos, D.N, D.p, XX, T, M, st, hist, belowc, chunk)
        LAGP_DISPATCH_P(D.p, LAGP_KNN_HIST);
#undef LAGP_KNN_HIST
        fill_u32(flags, 1, 0u, stream);
        hipLaunchKernelGGL(knn_decide_kernel, dim3(dgrid), dim3(256), 0, stream, st, hist, belowc, T, M, M_per, 1,
                           bucket_max, fac, flags);
        if (!graph_safe) {
            uint32_t unsettled = 0;
            if (hipMemcpyAsync(&unsettled, flags, 4, hipMemcpyDeviceToHost, stream) != hipSuccess ||
                hipStreamSynchronize(stream) != hipSuccess) {
                *err = "knn pass synchronisation failed";
                return -2;
            }
            if (unsettled == 0) break;
        }
    }
    fill_u32(counts, T * 2, 0u, stream);
#define LAGP_KNN_COLL(PP) hipLaunchKernelGGL(knn_collect_kernel<PP>, grid, dim3(KNN_THREADS), lds_coll, stream, \
                                             D.Xaos, D.N, D.p, XX, T, st, counts, idx, idx_stride, bucket, \
                                             bucket_max, chunk)
    LAGP_DISPATCH_P(D.p, LAGP_KNN_COLL);
#undef LAGP_KNN_COLL
    hipLaunchKernelGGL(knn_finalize_kernel, dim3((unsigned)T), dim3(KNN_THREADS), 0, stream, T, M, M_per, st, counts,
                       idx, idx_stride, bucket, bucket_max, (int32_t*)(flags + 1));
    if (sorted)
        hipLaunchKernelGGL(knn_sort_kernel, dim3((unsigned)T), dim3(KNN_THREADS), 0, stream, D.Xaos, D.p, XX,
                           T, M, idx, idx_stride);
    if (graph_safe) return hipGetLastError() == hipSuccess ? 0 : -2;
    uint32_t bad = 0;
    if (hipMemcpyAsync(&bad, flags + 1, 4, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess) {
        *err = "knn synchronisation failed";
        return -2;
    }
    if (bad) { *err = "knn selection inconsistent"; return -3; }
    if (hipGetLastError() != hipSuccess) { *err = "knn launch failed"; return -2; }
    return 0;
}

}  // namespace lagp
