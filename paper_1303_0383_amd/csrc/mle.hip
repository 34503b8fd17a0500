// mle.hip -- local maximum-likelihood lengthscale of given local designs.
//
// The concentrated log likelihood of a local design (eq gpk of Section 2;
// constants dropped)
//   l(theta) = -1/2 log|K| - n/2 log psi,   psi = Y'K^{-1}Y,
// and its first two derivatives (eqs dl, d2l of SM Section 2)
//   l'  = -1/2 tr(K^{-1} dK) + n/2 q / psi,                 q  = Y'K^{-1} dK K^{-1}Y,
//   l'' = -1/2 [tr(K^{-1} d2K) - tr((K^{-1} dK)^2)]
//         + n/2 (r - 2 sq) / psi + n/2 q^2 / psi^2,          r  = Y'K^{-1} d2K K^{-1}Y,
//                                                            sq = Y'K^{-1} dK K^{-1} dK K^{-1}Y.
// For the isotropic Gaussian kernel K(a,b) = exp(-d2/theta) the off-diagonal
// entries of dK and d2K are K d2/theta^2 and dK (d2/theta^2 - 2/theta); the
// diagonal (1 + g) does not depend on theta.  Section 3.2 finds the maximum
// once per location, after the design is complete, by a Newton-like search
// with these derivatives.
//
// One workgroup per location.  For each Newton iterate it
//   * builds K (packed lower triangle) and dK (packed strictly-lower
//     triangle) from the design coordinates held in LDS;
//   * factorises K right-looking in place, carrying u = L^{-1} Y, and keeps
//     the pivots L_kk -- for designs of up to 128 points by 16-column panels
//     (one wave factors a panel with its rows in registers, the trailing
//     blocks take the panel's rank-16 update on the FP64 matrix cores),
//     for larger ones one barrier per column, each column scaled during the
//     next column's phase;
//   * overwrites L with L^{-1} in place -- for designs of up to 128 points
//     by 16x16 blocks (each diagonal block inverted by one wave in
//     registers, then block row i of the inverse as -X_ii times the sum over
//     k < i of L_ik X_kj, both products on the FP64 matrix cores), for
//     larger ones by Gauss-Jordan elimination, one barrier per column (each
//     row scaled during the next phase, the next column of L copied aside
//     first);
//   * forms w = K^{-1} Y = L^{-T} u and k = dK w (each dot product split
//     over a few lanes of one wave), and from them
//     psi = u'u, q = w'k, sq = ||L^{-1} k||^2 and r = w' d2K w;
//   * forms tr(K^{-1} dK) and tr(K^{-1} d2K) with the entries of
//     K^{-1} = L^{-T} L^{-1} computed as they are used (for designs of up
//     to 128 points 16 x 16 tiles of them on the FP64 matrix cores, the
//     pairs' squared distances for d2K from tiles of x_a . x_b and the
//     points' norms), and
//     tr((K^{-1} dK)^2) = ||L^{-1} dK L^{-T}||_F^2 a panel of columns of
//     H = dK L^{-T} at a time: for designs of up to 128 points 16 columns on
//     the FP64 matrix cores, then the same columns of L^{-1} H (its tiles
//     on and below the diagonal: the product is symmetric), every product
//     stopping at its last nonzero term; larger designs PW columns on the
//     vector unit (one panel formed while the previous one is used);
//   * takes the safeguarded Newton step on l'(theta) = 0.
// The step rule: where l'' < 0 the step is -l'/l''; elsewhere it is theta in
// the direction of l'; a step leaving (tmin, tmax) goes half way to the
// bound instead; the search stops when a step moves theta by at most
// tol * theta, or after maxit iterates.
//
// A design with an index outside [0, N), fewer than 2 points, or a
// non-positive pivot at any iterate gives theta = NaN (and status NOTPD).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#include "lagp_internal.h"

namespace lagp {

namespace {

constexpr int PW = 8;   // panel width of the tr((K^{-1} dK)^2) product (designs above MF points)
constexpr int MF = 128; // designs of up to MF points take the panel products on the matrix cores

typedef double mf_d4 __attribute__((ext_vector_type(4)));

// The value v holds in lane l of the wave (l constant across the wave).
__device__ __forceinline__ double lane_value(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Doubles of the panel buffer: two PW-wide panels, or for designs of up to MF
// points one 16-column panel over the design padded to a multiple of 16.
__host__ __device__ inline size_t panel_doubles(int nm)
{
    const size_t a = 2 * (size_t)nm * PW;
    const size_t b = nm <= MF ? (size_t)((nm + 15) & ~15) * 16 : 0;
    return a > b ? a : b;
}
constexpr int NRED = 7; // sums reduced per iterate

// Packed indices.  Every index here is far below 2^24, so the products use
// the full-rate 24-bit multiply instead of the quarter-rate 32-bit one.
__device__ __forceinline__ int half_prod(int a, int b) { return (int)(__umul24((unsigned)a, (unsigned)b) >> 1); }
__device__ __forceinline__ int tri(int i, int k) { return half_prod(i, i + 1) + k; }   // lower, diagonal included
__device__ __forceinline__ int sl(int i, int k) { return half_prod(i, i - 1) + k; }    // strictly lower, i > k

// Row of packed-lower index e (a(a+1)/2 <= e < (a+1)(a+2)/2).  The float
// estimate is within one of the row for every index a design of up to a few
// hundred points has, so one branch-free correction each way suffices (a
// loop here compiles to far more instructions than the multiply-add it
// feeds).  The hardware square root (about 1 ulp) is used directly: the
// corrections absorb its error, and the correctly rounded sqrtf costs a
// dozen more instructions per call.
__device__ __forceinline__ int row_of(int e)
{
    int a = (int)((__builtin_amdgcn_sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
    a -= (half_prod(a, a + 1) > e) ? 1 : 0;
    a += (half_prod(a + 1, a + 2) <= e) ? 1 : 0;
    return a;
}

__device__ __forceinline__ double sqdist_rows(const double* xs, int a, int b, int p)
{
    double s = 0.0;
    for (int c = 0; c < p; ++c) {
        const double d = xs[a * p + c] - xs[b * p + c];
        s += d * d;
    }
    return s;
}

template <int MT>
__device__ __forceinline__ void block_sum(double (&v)[NRED], double* red, int tid)
{
#pragma unroll
    for (int k = 0; k < NRED; ++k)
        for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
    if ((tid & 63) == 0)
#pragma unroll
        for (int k = 0; k < NRED; ++k) red[k * (MT / 64) + (tid >> 6)] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NRED; ++k) {
        double s = red[k * (MT / 64)];
        for (int w = 1; w < MT / 64; ++w) s += red[k * (MT / 64) + w];
        v[k] = s;
    }
}

template <int MT>
__global__ void __launch_bounds__(MT) __attribute__((amdgpu_waves_per_eu(4))) mle_kernel(const MleArgs A)
{
    extern __shared__ double sm[];
    if ((int64_t)blockIdx.x >= A.T) return;
    const int64_t t = A.order ? (int64_t)A.order[blockIdx.x] : (int64_t)blockIdx.x;
    const int tid = threadIdx.x;
    const int p = A.p;
    const int n = A.n_per ? A.n_per[t] : A.n;
    const int32_t* D = A.sel + t * A.sel_stride;
    const int nm = A.nmax;
    // LDS carve-up (doubles), sized for nmax
    double* xs = sm;                              // [nmax][p] design coordinates
    double* Tm = xs + (size_t)nm * p;             // packed lower: K -> L -> L^{-1}
    double* Cd = Tm + (size_t)nm * (nm + 1) / 2;  // packed strictly lower: dK
    double* Hb = Cd + (size_t)nm * (nm - 1) / 2;  // panels of dK L^{-T} ([2][nmax][PW], or [16 ceil(n/16)][16])
    double* yv = Hb + panel_doubles(nm);          // Y
    double* u = yv + nm;                          // L^{-1} Y
    double* w = u + nm;                           // K^{-1} Y
    double* kw = w + nm;                          // dK K^{-1} Y
    double* col = kw + nm;                        // columns of L being eliminated (two buffers)
    double* col2 = col + nm;
    double* piv = col2 + nm;                      // pivots L_kk
    double* red = piv + nm;                       // [NRED][MT/64]
    __shared__ int bad, done;
    __shared__ double sh_theta;

    if (tid == 0) bad = (n < 2 || n > nm) ? 1 : 0;
    __syncthreads();
    if (!bad)
        for (int a = tid; a < n; a += MT)
            if (D[a] < 0 || D[a] >= A.N) bad = 1;
    __syncthreads();

    double theta = NAN;
    int it = 0;
    if (!bad) {
        for (int e = tid; e < n * p; e += MT) xs[e] = A.Xaos[(int64_t)D[e / p] * p + e % p];
        for (int a = tid; a < n; a += MT) yv[a] = A.y[D[a]];
        if (nm <= MF) {
            // squared norms of the design points (in the column buffers, which
            // only the Gauss-Jordan form of larger designs uses), for the
            // distances of the trace sums: |x_a - x_b|^2 = |x_a|^2 + |x_b|^2 - 2 x_a.x_b
            __syncthreads();
            for (int a = tid; a < n; a += MT) {
                double s = 0.0;
                for (int c = 0; c < p; ++c) s += xs[a * p + c] * xs[a * p + c];
                col[a] = s;
            }
        }
        const double th0 = A.theta0_per ? A.theta0_per[t] : A.theta0;
        theta = (th0 > A.tmin && th0 < A.tmax) ? th0 : sqrt(A.tmin * A.tmax);
        const int ntri = n * (n + 1) / 2;
        while (it < A.maxit) {
            __syncthreads();
            const double th2 = theta * theta;
            // ---- K and dK
            for (int e = tid; e < ntri; e += MT) {
                const int a = row_of(e), b = e - half_prod(a, a + 1);
                // the off-diagonal form is evaluated on the diagonal too and
                // discarded there (no divergent branch around the exponential)
                const double d2 = sqdist_rows(xs, a, b, p);
                const double k = exp(-(d2 / theta));
                Tm[e] = (a == b) ? 1.0 + A.eta : k;
                if (a != b) Cd[sl(a, b)] = k * d2 / th2;
            }
            for (int a = tid; a < n; a += MT) u[a] = yv[a];
            if (tid == 0) red[0] = 1.0 / Tm[0];   // thread 0 wrote Tm[0] (item 0) above
            __syncthreads();
            // ---- Cholesky, right-looking, one barrier per column: the pivot
            //      column m is used unscaled (products times the reciprocal of
            //      the unrooted pivot K^(m)_mm) and
            //      scaled in place during column m+1's phase, when nothing reads
            //      it; u = L^{-1} Y is carried the same way.
            // The reciprocal of each pivot is formed once, by thread 0, which
            // also updates the next pivot (trailing item 0), and passed on in
            // red[0..1] (free until the sums at the end of the iterate).
            int fail = 0;
            if (nm <= MF) {
                // Blocked by 16 columns: one wave factors a 16-column panel
                // (lanes over rows, no barrier: LDS operations of a wave
                // complete in issue order), scaling each column by its root
                // and carrying u = L^{-1} Y; then the trailing blocks take the
                // panel's rank-16 update as 16 x 16 x 16 products on the FP64
                // matrix cores (one 16 x 16 block per wave at a time).  The
                // diagonal keeps the unrooted pivots, the roots go to piv.
                const int lane = tid & 63, wave = tid >> 6;
                const int li = lane & 15, lk = lane >> 4;
                const int nb = (n + 15) >> 4;
                for (int kb = 0; kb < nb && !fail; ++kb) {
                    const int c0 = 16 * kb, c1 = (c0 + 16 < n) ? c0 + 16 : n;
                    if (wave == 0) {
                        // lane l holds the panel part of row c0 + l in registers for
                        // all 16 steps; row m of the panel is lane m - c0's row, read
                        // across lanes.  Rows c0 + 64 + l (designs above 64 points)
                        // follow in a second pass that reads the finished panel
                        // columns, roots and u back from LDS.
                        const int i0 = c0 + lane;
                        const bool h0 = i0 < n;
                        const int b0 = h0 ? tri(i0, 0) : 0;
                        double r0[16];
#pragma unroll
                        for (int q = 0; q < 16; ++q) {
                            const int k = c0 + q;
                            r0[q] = (h0 && k < c1 && k <= i0) ? Tm[b0 + k] : 0.0;
                        }
                        double u0 = h0 ? u[i0] : 0.0;
                        int f = 0;
#pragma unroll
                        for (int q = 0; q < 16; ++q) {
                            if (c0 + q < c1 && !f) {
                                const double pm = lane_value(r0[q], q);
                                if (!(pm > 0.0)) {
                                    f = 1;   // uniform: every lane read the same pivot
                                } else {
                                    // the update uses the column unscaled (times the
                                    // reciprocal of the unrooted pivot), so the root and
                                    // the scaling stay off the chain to the next pivot
                                    const double rpm = 1.0 / pm;
                                    const double t = r0[q] * rpm;
                                    const double uq = lane_value(u0, q);
                                    // every lane updates (no select): lanes above row
                                    // c0 + qq change only entries above the diagonal,
                                    // which are never read as pivots or stored
#pragma unroll
                                    for (int qq = q + 1; qq < 16; ++qq) {
                                        const double akm = lane_value(r0[q], qq);   // unscaled A_km, row k = c0 + qq
                                        r0[qq] -= t * akm;
                                    }
                                    if (lane > q) u0 -= t * uq;
                                    // L_kq = A_kq / sqrt(pm) = t sqrt(pm); u_q / sqrt(pm) = u_q sqrt(pm) / pm
                                    const double dp = sqrt(pm);
                                    if (lane == 0) piv[c0 + q] = dp;
                                    if (lane > q) r0[q] = t * dp;   // rows below the pivot
                                    if (lane == q) u0 = u0 * (dp * rpm);
                                }
                            }
                        }
#pragma unroll
                        for (int q = 0; q < 16; ++q) {
                            const int k = c0 + q;
                            if (h0 && k < c1 && k <= i0) Tm[b0 + k] = r0[q];
                        }
                        if (h0) u[i0] = u0;
                        if (!f && c0 + 64 < n) {
                            __builtin_amdgcn_wave_barrier();
                            const int i1 = c0 + 64 + lane;
                            const bool h1 = i1 < n;
                            const int b1 = h1 ? tri(i1, 0) : 0;
                            double r1[16];
#pragma unroll
                            for (int q = 0; q < 16; ++q) r1[q] = (h1 && c0 + q < c1) ? Tm[b1 + c0 + q] : 0.0;
                            double u1 = h1 ? u[i1] : 0.0;
#pragma unroll
                            for (int q = 0; q < 16; ++q) {
                                if (c0 + q < c1) {
                                    const int m = c0 + q;
                                    r1[q] = r1[q] / piv[m];
#pragma unroll
                                    for (int qq = q + 1; qq < 16; ++qq)
                                        if (c0 + qq < c1) r1[qq] -= r1[q] * Tm[tri(c0 + qq, m)];
                                    u1 -= r1[q] * u[m];
                                }
                            }
#pragma unroll
                            for (int q = 0; q < 16; ++q)
                                if (h1 && c0 + q < c1) Tm[b1 + c0 + q] = r1[q];
                            if (h1) u[i1] = u1;
                        }
                        if (lane == 0) red[0] = f ? 1.0 : 0.0;
                    }
                    __syncthreads();
                    if (red[0] != 0.0) { fail = 1; break; }   // uniform
                    // trailing blocks (ib, jb), kb < jb <= ib < nb: A_ib,jb -= L_ib,kb L_jb,kb^T
                    const int ntb = nb - kb - 1;
                    for (int tt = wave; tt < ntb * (ntb + 1) / 2; tt += MT / 64) {
                        int ib = kb + 1, rem = tt;
                        while (rem >= ib - kb) { rem -= ib - kb; ++ib; }
                        const int jb = kb + 1 + rem;
                        mf_d4 c;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int i = 16 * ib + 4 * r + lk, j = 16 * jb + li;
                            c[r] = (i < n && j <= i) ? Tm[tri(i, j)] : 0.0;
                        }
                        const int ia = 16 * ib + li, ja = 16 * jb + li;
#pragma unroll
                        for (int k0 = 0; k0 < 16; k0 += 4) {
                            const int kc = c0 + k0 + lk;
                            const double av = (ia < n && kc < c1) ? -Tm[tri(ia, kc)] : 0.0;
                            const double bv = (ja < n && kc < c1) ? Tm[tri(ja, kc)] : 0.0;
                            c = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, c, 0, 0, 0);
                        }
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int i = 16 * ib + 4 * r + lk, j = 16 * jb + li;
                            if (i < n && j <= i) Tm[tri(i, j)] = c[r];
                        }
                    }
                    __syncthreads();
                }
            } else {
            for (int m = 0; m < n; ++m) {
                const double pm = Tm[tri(m, m)];
                if (!(pm > 0.0)) { fail = 1; break; }   // uniform: every thread read the same pivot
                const double rpm = red[m & 1];
                if (m > 0) {
                    const double dp = piv[m - 1];
                    for (int i = m + tid; i < n; i += MT) Tm[tri(i, m - 1)] = Tm[tri(i, m - 1)] / dp;
                    if (tid == 0) u[m - 1] = u[m - 1] / dp;
                }
                if (tid == 0) piv[m] = sqrt(pm);
                // trailing triangle rows i > m, columns m < k <= i, folded into
                // a rectangle: trailing row r (r + 1 entries) and trailing row
                // tn - 1 - r (tn - r entries) share rectangle row r of tn + 1
                // columns, so every thread runs the same number of items with
                // no per-item row search; lanes 0..31 of a wave take rectangle
                // rows, the wave's two halves and the other waves interleave
                // its columns (thread 0 takes item (0, 0), the next pivot)
                const int tn = n - m - 1;
                for (int r = tid & 31; r < ((tn + 1) >> 1); r += 32) {
                    const int r2 = tn - 1 - r;   // >= r; equal for the middle row of an odd tn
                    const int b1 = tri(m + 1 + r, 0), b2 = tri(m + 1 + r2, 0);
                    const double l1 = Tm[b1 + m], l2 = Tm[b2 + m];
                    const int cmax = r2 > r ? tn : r;   // the middle row has no partner
                    for (int c = tid >> 5; c <= cmax; c += MT / 32) {
                        const bool lower = c <= r;
                        const int k = m + 1 + (lower ? c : c - r - 1);
                        const double li = lower ? l1 : l2;
                        const int o = (lower ? b1 : b2) + k;
                        Tm[o] -= (li * Tm[tri(k, m)]) * rpm;
                    }
                }
                const double um = u[m];
                for (int i = m + 1 + tid; i < n; i += MT) u[i] -= (Tm[tri(i, m)] * um) * rpm;
                if (tid == 0 && m + 1 < n) red[(m + 1) & 1] = 1.0 / Tm[tri(m + 1, m + 1)];
                __syncthreads();
            }
            if (!fail && tid == 0) u[n - 1] = u[n - 1] / piv[n - 1];   // column n-1 has no entries below its pivot
            }
            if (fail) {
                if (tid == 0) bad = 1;
                break;
            }
            if (nm <= MF) {
                // ---- L^{-1} in place by 16 x 16 blocks: each diagonal block
                //      X_ii = L_ii^{-1} by one wave (lane = row, the row kept in
                //      registers, earlier rows read across lanes), then block row
                //      by block row X_ij = -X_ii sum_{k=j}^{i-1} L_ik X_kj on the
                //      FP64 matrix cores (the sums staged in LDS first, since they
                //      read L blocks of the row that the products overwrite).
                const int lane = tid & 63, wave = tid >> 6;
                const int li = lane & 15, lk = lane >> 4;
                const int nb = (n + 15) >> 4;
                for (int kb = wave; kb < nb; kb += MT / 64) {
                    const int c0 = 16 * kb, i = c0 + li;
                    const bool hv = lane < 16 && i < n;
                    double xr[16];
#pragma unroll
                    for (int c = 0; c < 16; ++c) xr[c] = 0.0;   // sums of L_im X_mc over m < i
                    const double rd = hv ? 1.0 / piv[i] : 0.0;   // 1 / L_ii, formed by all rows at once
#pragma unroll
                    for (int m = 0; m < 16; ++m) {
                        if (c0 + m < n) {
                            // row m finishes: X_mc = -sum / L_mm (c < m), X_mm = 1 / L_mm
                            if (lane == m) {
#pragma unroll
                                for (int c = 0; c < 16; ++c)
                                    if (c < m) xr[c] = -xr[c] * rd;
                                xr[m] = rd;
                            }
                            const double lim = (hv && li > m) ? Tm[tri(i, c0 + m)] : 0.0;
                            // lim is zero on the rows at and above m (no select needed)
#pragma unroll
                            for (int c = 0; c <= m; ++c) {
                                const double xmc = lane_value(xr[c], m);
                                xr[c] += lim * xmc;
                            }
                        }
                    }
                    if (hv) {
#pragma unroll
                        for (int c = 0; c < 16; ++c)
                            if (c <= li) Tm[tri(i, c0 + c)] = xr[c];
                    }
                }
                __syncthreads();
                double* Ts = Hb;   // [nb - 1][16][16] sums of a block row
                for (int ib = 1; ib < nb; ++ib) {
                    // T_j = sum_{k=j}^{ib-1} L_ib,k X_k,j for every block j < ib
                    for (int jb = wave; jb < ib; jb += MT / 64) {
                        mf_d4 c = {0.0, 0.0, 0.0, 0.0};
                        const int ia = 16 * ib + li;
                        for (int kb = jb; kb < ib; ++kb) {
#pragma unroll
                            for (int k0 = 0; k0 < 16; k0 += 4) {
                                const int kc = 16 * kb + k0 + lk, jc = 16 * jb + li;
                                const double av = (ia < n && kc < n) ? Tm[tri(ia, kc)] : 0.0;
                                const double bv = (kc < n && jc <= kc) ? Tm[tri(kc, jc)] : 0.0;
                                c = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, c, 0, 0, 0);
                            }
                        }
#pragma unroll
                        for (int r = 0; r < 4; ++r) Ts[(jb * 16 + 4 * r + lk) * 16 + li] = c[r];
                    }
                    __syncthreads();
                    // X_ib,j = -X_ib,ib T_j (columns of X_ib,ib past n - 16 ib are zero)
                    const int kend = n - 16 * ib < 16 ? n - 16 * ib : 16;
                    for (int jb = wave; jb < ib; jb += MT / 64) {
                        mf_d4 c = {0.0, 0.0, 0.0, 0.0};
                        const int ia = 16 * ib + li;
#pragma unroll
                        for (int k0 = 0; k0 < 16; k0 += 4) {
                            if (k0 < kend) {   // uniform
                                const int kc = 16 * ib + k0 + lk;
                                const double av = (ia < n && kc <= ia) ? -Tm[tri(ia, kc)] : 0.0;
                                c = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Ts[(jb * 16 + k0 + lk) * 16 + li], c, 0, 0, 0);
                            }
                        }
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int ii = 16 * ib + 4 * r + lk, jj = 16 * jb + li;
                            if (ii < n) Tm[tri(ii, jj)] = c[r];
                        }
                    }
                    __syncthreads();
                }
            } else {
            // ---- L^{-1} in place, one barrier per column: row k of X = L^{-1} is
            //      used unscaled (times 1/L_kk on the fly) and scaled during the
            //      next phase; column k+1 of L is copied aside in phase k (two
            //      buffers), before phase k+1 overwrites it.
            double* rpv = w;   // 1 / L_kk (w is free until w = L^{-T} u)
            for (int i = 1 + tid; i < n; i += MT) col[i] = Tm[tri(i, 0)];
            for (int i = tid; i < n; i += MT) rpv[i] = 1.0 / piv[i];
            __syncthreads();
            for (int k = 0; k < n; ++k) {
                const double rk = rpv[k];
                const double* ck = (k & 1) ? col2 : col;
                double* cn = (k & 1) ? col : col2;
                if (k > 0) {
                    const double rp = rpv[k - 1];
                    for (int c = tid; c < k - 1; c += MT) Tm[tri(k - 1, c)] = Tm[tri(k - 1, c)] * rp;
                    if (tid == 0) Tm[tri(k - 1, k - 1)] = rp;
                }
                for (int i = k + 2 + tid; i < n; i += MT) cn[i] = Tm[tri(i, k + 1)];
                // rows i > k, columns c <= k: (i, c) advances by MT items without dividing per item
                const int w1 = k + 1, qi = MT / w1, qc = MT - qi * w1;
                int i = k + 1 + tid / w1, c = tid - (tid / w1) * w1;
                for (; i < n;) {
                    // both forms evaluated and one kept (no divergent branch)
                    const int o = tri(i, c);
                    const double upd = Tm[o] - ck[i] * (Tm[tri(k, c)] * rk);
                    Tm[o] = (c == k) ? -(ck[i] * rk) : upd;
                    i += qi;
                    c += qc;
                    if (c >= w1) { c -= w1; ++i; }
                }
                __syncthreads();
            }
            {
                const double rp = rpv[n - 1];
                for (int c = tid; c < n - 1; c += MT) Tm[tri(n - 1, c)] = Tm[tri(n - 1, c)] * rp;
                if (tid == 0) Tm[tri(n - 1, n - 1)] = rp;
            }
            __syncthreads();
            }
            // ---- w = L^{-T} u, then k = dK w, then z = L^{-1} k: each dot
            //      product taken by P lanes of one wave (P a power of two, as
            //      many as the workgroup's threads allow for the design, at most
            //      8), lane part pp summing the terms pp, pp + P, ..., the parts
            //      added across the P lanes (the same sum in every lane: the
            //      butterfly adds the same pairs in each)
            int lp = 0;
            while (lp < 3 && (2 << lp) * n <= MT) ++lp;
            const int P = 1 << lp, pp = tid & (P - 1), rstep = MT >> lp;
            for (int b = tid >> lp; b < n; b += rstep) {
                double s = 0.0;
                int o = tri(b + pp, b);            // (a, b), a = b + pp, b + pp + P, ...
                for (int a = b + pp; a < n; a += P) {
                    s += Tm[o] * u[a];
                    o += a * P + ((P * (P + 1)) >> 1);
                }
                for (int m = 1; m < P; m <<= 1) s += __shfl_xor(s, m);
                if (pp == 0) w[b] = s;
            }
            __syncthreads();
            for (int a = tid >> lp; a < n; a += rstep) {
                double s = 0.0;
                const double* ca = Cd + sl(a, 0);
                int b = pp;
                for (; b < a; b += P) s += ca[b] * w[b];
                if (b == a) b += P;                // dK_aa = 0
                for (; b < n; b += P) s += Cd[sl(b, a)] * w[b];
                for (int m = 1; m < P; m <<= 1) s += __shfl_xor(s, m);
                if (pp == 0) kw[a] = s;
            }
            __syncthreads();
            // sums: 0 psi, 1 q, 2 sq, 3 r, 4 t1, 5 t2, 6 t3
            double acc[NRED] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            for (int a = tid >> lp; a < n; a += rstep) {
                double z = 0.0;
                const double* la = Tm + tri(a, 0);
                for (int b = pp; b <= a; b += P) z += la[b] * kw[b];
                for (int m = 1; m < P; m <<= 1) z += __shfl_xor(z, m);
                if (pp == 0) {
                    acc[0] += u[a] * u[a];
                    acc[1] += w[a] * kw[a];
                    acc[2] += z * z;
                }
            }
            // off-diagonal pairs a > b: K^{-1}_ab = sum_{k >= a} Li_ka Li_kb
            const double r2t = 2.0 / theta;
            if (nm <= MF) {
                // 16 x 16 tiles (ta, tb), ta >= tb, of K^{-1} = L^{-T} L^{-1} on
                // the matrix cores (rows k from 16 ta on: Li_ka = 0 for k < a),
                // then each lane's entries with a > b
                const int np16 = (n + 15) & ~15, nt = np16 / 16, ntile = nt * (nt + 1) / 2;
                const int lane = tid & 63, wave = tid >> 6;
                const int li = lane & 15, lk = lane >> 4;
                for (int t = wave; t < ntile; t += MT / 64) {
                    int ta = 0;
                    while ((ta + 1) * (ta + 2) / 2 <= t) ++ta;
                    const int tb = t - ta * (ta + 1) / 2;
                    const int ai = 16 * ta + li, bj = 16 * tb + li;
                    mf_d4 c = {0.0, 0.0, 0.0, 0.0};
                    for (int k0 = 16 * ta; k0 < n; k0 += 4) {   // rows k >= n add zeros
                        const int k = k0 + lk;
                        const double av = (k < n && ai <= k) ? Tm[tri(k, ai)] : 0.0;   // A[i][kk] = Li_{k, a_i}
                        const double bv = (k < n && bj <= k) ? Tm[tri(k, bj)] : 0.0;   // B[kk][j] = Li_{k, b_j}
                        c = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, c, 0, 0, 0);
                    }
                    // the same tile of x_a . x_b, p coordinates at a time
                    mf_d4 g = {0.0, 0.0, 0.0, 0.0};
                    for (int k0 = 0; k0 < p; k0 += 4) {
                        const int k = k0 + lk;
                        const double xa = (ai < n && k < p) ? xs[ai * p + k] : 0.0;
                        const double xb = (bj < n && k < p) ? xs[bj * p + k] : 0.0;
                        g = __builtin_amdgcn_mfma_f64_16x16x4f64(xa, xb, g, 0, 0, 0);
                    }
                    const double nb = bj < n ? col[bj] : 0.0;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int a = 16 * ta + 4 * r + lk, b = bj;
                        if (a < n && b < a) {
                            const double ki = c[r];
                            const double kd = Cd[sl(a, b)];
                            const double d2 = (col[a] + nb) - 2.0 * g[r];
                            const double kdd = kd * (d2 / th2 - r2t);
                            acc[3] += 2.0 * (w[a] * w[b]) * kdd;
                            acc[4] += 2.0 * ki * kd;
                            acc[5] += 2.0 * ki * kdd;
                        }
                    }
                }
            } else {
            const int nsl = n * (n - 1) / 2;
            for (int e = tid; e < nsl; e += MT) {
                const int a = row_of(e) + 1, b = e - half_prod(a, a - 1);
                double ki = 0.0;
                int oa = tri(a, a), ob = tri(a, b);   // rows k = a, a + 1, ...: steps of k + 1
#pragma unroll 4
                for (int k = a; k < n; ++k) {
                    ki += Tm[oa] * Tm[ob];
                    oa += k + 1;
                    ob += k + 1;
                }
                const double kd = Cd[e];
                const double d2 = sqdist_rows(xs, a, b, p);
                const double kdd = kd * (d2 / th2 - r2t);
                acc[3] += 2.0 * (w[a] * w[b]) * kdd;
                acc[4] += 2.0 * ki * kd;
                acc[5] += 2.0 * ki * kdd;
            }
            }
            // ---- tr((K^{-1} dK)^2) = ||L^{-1} dK L^{-T}||_F^2
            if (nm <= MF) {
                // On the matrix cores (FP64, 16 x 16 x 4 per instruction), over
                // the design padded with zero rows and columns to np16 = 16
                // ceil(n/16): a 16-column panel of H = dK L^{-T} (one 16 x 16
                // tile per wave), staged in LDS, then the same columns of
                // M = L^{-1} H, whose squared entries sum to the trace (M is
                // symmetric: the tiles on and below the diagonal, those below
                // counted twice).  Operand layout of the
                // instruction: A[i][k] and B[k][j] come from lane i + 16 k and
                // j + 16 k, and lane l's result r is D[4 r + l / 16][l % 16].
                const int np16 = (n + 15) & ~15, nt = np16 / 16;
                const int lane = tid & 63, wave = tid >> 6;
                const int li = lane & 15, lk = lane >> 4;
                for (int q = 0; q < nt; ++q) {
                    const int j = 16 * q + li;   // this lane's column of H and M
                    for (int tw = wave; tw < nt; tw += MT / 64) {
                        const int a = 16 * tw + li;   // row of dK
                        mf_d4 c = {0.0, 0.0, 0.0, 0.0};
                        // b <= j < 16 q + 16 and b < n: later steps add zeros
                        const int kend = n < 16 * q + 16 ? n : 16 * q + 16;
                        for (int k0 = 0; k0 < kend; k0 += 4) {
                            const int b = k0 + lk;
                            double av = 0.0, bv = 0.0;
                            if (a < n && b < n && a != b) av = a > b ? Cd[sl(a, b)] : Cd[sl(b, a)];
                            if (j < n && b <= j) bv = Tm[tri(j, b)];   // L^{-T}[b][j] = Li_jb
                            c = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, c, 0, 0, 0);
                        }
#pragma unroll
                        for (int r = 0; r < 4; ++r) Hb[(16 * tw + 4 * r + lk) * 16 + li] = c[r];
                    }
                    __syncthreads();
                    for (int tw = wave; tw < nt; tw += MT / 64) {
                        if (tw < q) continue;   // M is symmetric: tiles above the diagonal mirror those below
                        const int i = 16 * tw + li;   // row of L^{-1} and M
                        mf_d4 c = {0.0, 0.0, 0.0, 0.0};
                        // a <= i < 16 tw + 16 and a < n: later steps add zeros
                        const int kend = n < 16 * tw + 16 ? n : 16 * tw + 16;
                        for (int k0 = 0; k0 < kend; k0 += 4) {
                            const int a = k0 + lk;
                            const double av = (i < n && a <= i) ? Tm[tri(i, a)] : 0.0;
                            c = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Hb[a * 16 + li], c, 0, 0, 0);
                        }
                        const double wt = tw == q ? 1.0 : 2.0;
#pragma unroll
                        for (int r = 0; r < 4; ++r) acc[6] += wt * (c[r] * c[r]);
                    }
                    __syncthreads();
                }
            } else {
            // PW columns at a time: phase ph forms panel ph of H = dK L^{-T}
            // and, from the other buffer, the entries M_ij (i >= j) of panel ph - 1
            const int np = (n + PW - 1) / PW;
            for (int ph = 0; ph <= np; ++ph) {
                if (ph < np) {
                    const int j0 = ph * PW, pw = (n - j0) < PW ? (n - j0) : PW;
                    double* H = Hb + (size_t)(ph & 1) * nm * PW;
                    // H[a][jj] = sum_{b <= j} dK_ab Li_jb, j = j0 + jj, in ascending
                    // b: row a of the strictly-lower dK for b < a, then column a
                    // (dK_aa = 0 adds nothing)
                    for (int e = tid; e < n * PW; e += MT) {
                        const int a = e / PW, jj = e % PW, j = j0 + jj;
                        if (jj >= pw) continue;
                        const double* lj = Tm + tri(j, 0);
                        const double* ca = Cd + sl(a, 0);
                        double s = 0.0;
                        const int b1 = a < j + 1 ? a : j + 1;
#pragma unroll 4
                        for (int b = 0; b < b1; ++b) s += ca[b] * lj[b];
                        int o = sl(a + 1, a);
#pragma unroll 4
                        for (int b = a + 1; b <= j; ++b) {
                            s += Cd[o] * lj[b];
                            o += b;
                        }
                        H[a * PW + jj] = s;
                    }
                }
                if (ph > 0) {
                    const int j0 = (ph - 1) * PW, pw = (n - j0) < PW ? (n - j0) : PW;
                    const double* H = Hb + (size_t)((ph - 1) & 1) * nm * PW;
                    // M_ij = sum_{a <= i} Li_ia H_aj for i >= j
                    for (int e = tid; e < n * PW; e += MT) {
                        const int i = e / PW, jj = e % PW, j = j0 + jj;
                        if (jj >= pw || i < j) continue;
                        double s = 0.0;
                        const double* li = Tm + tri(i, 0);
#pragma unroll 4
                        for (int a = 0; a <= i; ++a) s += li[a] * H[a * PW + jj];
                        acc[6] += (i == j ? 1.0 : 2.0) * (s * s);
                    }
                }
                __syncthreads();
            }
            }
            block_sum<MT>(acc, red, tid);
            if (tid == 0) {
                const double psi = acc[0], q = acc[1], sq = acc[2], r = acc[3], t1 = acc[4], t2 = acc[5], t3 = acc[6];
                const double nn = (double)n;
                const double l1 = -0.5 * t1 + 0.5 * nn * q / psi;
                const double l2 = -0.5 * (t2 - t3) + 0.5 * nn * (r - 2.0 * sq) / psi + 0.5 * nn * q * q / (psi * psi);
                const double step = (l2 < 0.0) ? -l1 / l2 : (l1 > 0.0 ? theta : -theta);
                double next = theta + step;
                if (!(next > A.tmin)) next = 0.5 * (theta + A.tmin);
                if (!(next < A.tmax)) next = 0.5 * (theta + A.tmax);
                done = fabs(next - theta) <= A.tol * theta;
                sh_theta = next;
            }
            __syncthreads();
            theta = sh_theta;
            ++it;
            if (done) break;
        }
    }
    __syncthreads();
    if (tid == 0) {
        A.theta_out[t] = bad ? NAN : theta;
        if (A.iters) A.iters[t] = it;
        if (A.status) A.status[t] = bad ? 1 : 0;
    }
}

template <int MT>
int launch(const MleArgs& a, size_t lds, hipStream_t stream)
{
    hipLaunchKernelGGL(mle_kernel<MT>, dim3((unsigned)a.T), dim3(MT), lds, stream, a);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

int threads_for(int nmax)
{
    if (const char* e = getenv("LAGP_MLE_THREADS")) {
        const int v = atoi(e);
        if (v == 64 || v == 128 || v == 256 || v == 512) return v;
    }
    return nmax <= 24 ? 128 : 256;
}

}  // namespace

size_t mle_lds_bytes(int nmax, int p, int threads)
{
    const size_t nm = (size_t)nmax;
    return (nm * p + nm * (nm + 1) / 2 + nm * (nm - 1) / 2 + panel_doubles(nmax) + 7 * nm + (size_t)NRED * (threads / 64)) *
           sizeof(double);
}

int mle_prepare(int32_t nmax, int p, size_t max_lds, std::string* err)
{
    if (mle_lds_bytes(nmax, p, 512) > max_lds) { *err = "local design too large for the likelihood kernel"; return -1; }
    const void* k[4] = {(const void*)mle_kernel<64>, (const void*)mle_kernel<128>, (const void*)mle_kernel<256>,
                        (const void*)mle_kernel<512>};
    for (const void* f : k)
        if (!set_lds_limit(f, max_lds)) { *err = "cannot reserve LDS for the likelihood kernel"; return -2; }
    return 0;
}

int mle_run(const MleArgs& a, size_t max_lds, hipStream_t stream, std::string* err)
{
    if (a.T == 0) return 0;
    const int mt = threads_for(a.nmax);
    const size_t lds = mle_lds_bytes(a.nmax, a.p, mt);
    if (lds > max_lds) { *err = "local design too large for the likelihood kernel"; return -1; }
    int rc = mt == 64    ? launch<64>(a, lds, stream)
             : mt == 128 ? launch<128>(a, lds, stream)
             : mt == 256 ? launch<256>(a, lds, stream)
                         : launch<512>(a, lds, stream);
    if (rc) { *err = "likelihood kernel launch failed"; return rc; }
    return 0;
}

}  // namespace lagp
