// mspe.hip -- greedy local designs by the MSPE criterion (Section 3.1,
// eq mspe), at a fixed lengthscale as Section 3.2 recommends.
//
// For a design of j >= 3 points and a candidate c the criterion is
//   J(c) = V_j(x|c) + (dmu_j(x)/dtheta)^2 / G_{j+1}(c),
//   V_j(x|c)   = psi/(j-2) (v_j(x) - cov_j(x,c)^2 / v_j(c)),
//   G_{j+1}(c) = F_j + dV_j(c)^2 / (2 V_j(c)^2) + dmu_j(c)^2 / V_j(c),
//   V_j(c)     = psi/(j-2) v_j(c),   F_j = -l''(theta) (eq d2l),
//   dmu_j(c)   = (kd_j(c) - dK K^{-1} k_j(c))' K^{-1} Y,
//   dV_j(c)    = [-q v_j(c) - psi (2 kd_j(c)'K^{-1}k_j(c) - k_j(c)'K^{-1} dK K^{-1} k_j(c))] / (j-2),
// with q = Y'K^{-1} dK K^{-1}Y = -dpsi/dtheta (the derivative of psi v/(j-2);
// the printed expression carries +q) and the next point minimises J.
//
// Everything is carried in the whitened basis of the greedy factor, as the
// ALC kernel does: L^{-1} (packed, one new row per step), the whitened tiles
// W = L^{-1} K(X_j, C) and Wd = L^{-1} dK(X_j, C) (one new row each per step,
// streamed from a per-workgroup slab), and the bordered matrices
// Hd = L^{-1} dK L^{-T} and Hdd = L^{-1} d2K L^{-T}, each extended by one
// column per step in O(j^2):
//   for the new point s with l = W[:,s], delta = sqrt(v_j(s)):
//   h[0..j) = (Wd[:,s] - Hd l) / delta,  h[j] = -(l.h[0..j)) / delta - (Wd[:,s].l) / delta^2,
// and likewise for Hdd with L^{-1} d2k_j(s) formed directly.  Per candidate
// the kernel keeps v(c), cov(x,c), a(c) = Wd[:,c].u, b(c) = Wd[:,c].W[:,c] and
// Q(c) = W[:,c]' Hd W[:,c], all updated in O(1) per step after four dot
// products over the candidate's tile columns (with l, z = Hd u and h over W,
// with l over Wd); then dmu(c) = a - W[:,c].z, k'K^{-1}kd = b and
// k'K^{-1}dK K^{-1}k = Q.  The location-level sums of l'' (tr Hdd, ||Hd||_F^2,
// u'Hdd u, u'Hd u, ||Hd u||^2) are bordered the same way.
//
// One workgroup per location (persistent over a work counter): 256 threads,
// or 512 above 1024 candidates, with up to 4 candidate slots per thread.  Arithmetic is FP64; the candidate
// tiles and coordinates live in a global slab, the factor and the bordered
// matrices in LDS.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "design_kernel.h"

namespace lagp {

namespace {

constexpr int MAXWAVES = 8;           // reduction slots (up to 512 threads)
constexpr int NSCAL = 16;             // location scalars in LDS

enum {
    S_PSI = 0, S_VX, S_T2, S_T3, S_Q, S_R, S_F, S_DMUX, S_VS, S_D2XS, S_UI, S_WXI, S_HI, S_ZI
};

__device__ __forceinline__ int tri(int i, int k) { return i * (i + 1) / 2 + k; }
// symmetric matrix stored as its packed lower triangle
__device__ __forceinline__ int sym(int i, int k) { return i >= k ? tri(i, k) : tri(k, i); }

// Bytes of the kernel's LDS arrays (the factor, the bordered matrices and the
// vectors below); LDS tile rows start at the next 8-byte boundary.
__host__ __device__ inline size_t lds_base_bytes(int nmax, int p)
{
    const size_t nm = (size_t)nmax;
    const size_t d = 3 * nm * (nm + 1) / 2 + nm * p + 14 * nm + 2 * (size_t)p + NSCAL + MAXWAVES;
    const size_t i = 2 * MAXWAVES + nm + 4;
    return d * sizeof(double) + i * sizeof(int);
}

// Sum over the 64 lanes of wave 0 (result in every lane of that wave).
__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// a . b over [0, len) by wave 0 (other waves must not call).
__device__ __forceinline__ double wdot(const double* a, const double* b, int len, int lane)
{
    double s = 0.0;
    for (int l = lane; l < len; l += 64) s += a[l] * b[l];
    return wave_sum(s);
}

template <int MT, int CPT>
__global__ void __launch_bounds__(MT, 1) mspe_kernel(const MspeArgs A)
{
    constexpr int MWAVES = MT / 64;
    extern __shared__ double smem[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int p = A.p;
    const int nm = A.nmax;
    const int ntri = nm * (nm + 1) / 2;
    const int Mpad = CPT * MT;
    const double theta = A.theta, eta = A.eta, one_eta = 1.0 + eta;
    const double th2 = theta * theta;

    double* Li = smem;                 // [ntri] L^{-1}, packed lower
    double* Hd = Li + ntri;            // [ntri] L^{-1} dK L^{-T}
    double* Hdd = Hd + ntri;           // [ntri] L^{-1} d2K L^{-T}
    double* XD = Hdd + ntri;           // [nm][p] design coordinates
    double* ws = XD + (size_t)nm * p;  // [nm] W[:,s]
    double* wds = ws + nm;             // [nm] Wd[:,s]
    double* wdds = wds + nm;           // [nm] L^{-1} d2k_j(s)
    double* kdd = wdds + nm;           // [nm] d2k_j(s)
    double* hdw = kdd + nm;            // [nm] Hd l
    double* hddw = hdw + nm;           // [nm] Hdd l
    double* h = hddw + nm;             // [nm] new column of Hd
    double* hh = h + nm;               // [nm] new column of Hdd
    double* u = hh + nm;               // [nm] L^{-1} Y
    double* wx = u + nm;               // [nm] L^{-1} k(x)
    double* wdx = wx + nm;             // [nm] L^{-1} dk(x)
    double* z = wdx + nm;              // [nm] Hd u
    double* lrow = z + nm;             // [nm] the new row of L^{-1}
    double* xl = lrow + nm;            // [p] location
    double* xs = xl + p;               // [p] the chosen point
    double* sc = xs + p;               // [NSCAL] location scalars
    double* redv = sc + NSCAL;           // [MAXWAVES]
    int* redi = (int*)(redv + MAXWAVES); // [MAXWAVES]
    int* reds = redi + MAXWAVES;         // [MAXWAVES]
    int* forced = reds + MAXWAVES;       // [nm]
    int* ctl = forced + nm;            // [4]

    double* Xc = A.scratch + (int64_t)blockIdx.x * A.scratch_stride;   // [p][Mpad] candidate coordinates
    double* Wt = Xc + (int64_t)p * Mpad;                                // [nm-1][Mpad] W rows
    double* Wdt = Wt + (int64_t)(nm - 1) * Mpad;                        // [nm-1][Mpad] Wd rows
    // The first RL rows of both tiles live in the LDS left over by the
    // arrays above (their slab rows stay unused); the rest stream from the slab.
    const int RL = A.lds_rows;
    double* Wl = smem + (lds_base_bytes(nm, p) + 7) / 8;   // [RL][Mpad] W rows
    double* Wdl = Wl + (size_t)RL * Mpad;                  // [RL][Mpad] Wd rows

    for (;;) {
        if (tid == 0) ctl[0] = (int)atomicAdd(A.counter, 1u);
        __syncthreads();
        const int64_t t = ctl[0];
        if (t >= A.T) break;
        const int n = A.n_per ? A.n_per[t] : A.n;
        const int M = A.M_per ? A.M_per[t] : A.M;
        const int n0 = A.n0;
        const int32_t* cand = A.cand + t * A.cand_stride;
        for (int k = tid; k < p; k += MT) xl[k] = A.XX[t * p + k];
        for (int e = tid; e < 3 * ntri; e += MT) Li[e] = 0.0;
        for (int l = tid; l < nm; l += MT) { u[l] = 0.0; wx[l] = 0.0; wdx[l] = 0.0; z[l] = 0.0; }
        if (tid < NSCAL) sc[tid] = 0.0;
        if (A.sel)
            for (int i = tid; i < n; i += MT) A.sel[t * A.sel_stride + i] = -1;
        __syncthreads();
        if (tid == 0) sc[S_VX] = one_eta;

        // ---- gather: coordinates into the slab; K(x,c); candidate state
        int ci[CPT];
        double d2x[CPT], v[CPT], cov[CPT], av[CPT], bv[CPT], Qv[CPT], zc[CPT];
        uint32_t chosen = 0;
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int slot = tid + k * MT;
            av[k] = bv[k] = Qv[k] = zc[k] = 0.0;
            v[k] = one_eta;
            if (slot < M) {
                const int c = cand[slot];
                ci[k] = c;
                double s = 0.0;
                for (int kk = 0; kk < p; ++kk) {
                    const double ck = A.Xaos[(int64_t)c * p + kk];
                    Xc[(int64_t)kk * Mpad + slot] = ck;
                    const double dd = xl[kk] - ck;
                    s += dd * dd;
                }
                d2x[k] = s;
                cov[k] = exp(-(s / theta));
            } else {
                ci[k] = 0x7fffffff;
                d2x[k] = INFINITY;
                cov[k] = 0.0;
                chosen |= 1u << k;
                for (int kk = 0; kk < p; ++kk) Xc[(int64_t)kk * Mpad + slot] = 0.0;
            }
        }
        // ---- starting design: the n0 nearest candidates
        {
            uint32_t taken = chosen;
            for (int r = 0; r < n0; ++r) {
                double bd = INFINITY;
                int bi = 0x7fffffff, bs = -1;
#pragma unroll
                for (int k = 0; k < CPT; ++k)
                    if (!((taken >> k) & 1u) && nearer(d2x[k], ci[k], bd, bi)) { bd = d2x[k]; bi = ci[k]; bs = tid + k * MT; }
                wave_pick<false>(bd, bi, bs);
                if (lane == 0) { redv[wave] = bd; redi[wave] = bi; reds[wave] = bs; }
                __syncthreads();
                bd = redv[0]; bi = redi[0]; bs = reds[0];
                for (int w2 = 1; w2 < MWAVES; ++w2) pick<false>(bd, bi, bs, redv[w2], redi[w2], reds[w2]);
                __syncthreads();
                if (tid == 0) forced[r] = bs;
                if (bs >= 0 && (bs % MT) == tid) taken |= 1u << (bs / MT);
            }
        }
        __syncthreads();

        int notpd = 0, s_next = -1;
        for (int i = 0; i < n; ++i) {
            const int s = (i < n0) ? forced[i] : s_next;
            if (s < 0 || s >= M) { notpd = 1; break; }
            // ---- phase A: the chosen column and point
            if (tid == s % MT) {
                const int kk = s / MT;
#pragma unroll
                for (int k = 0; k < CPT; ++k)
                    if (k == kk) {
                        sc[S_VS] = v[k];
                        sc[S_D2XS] = d2x[k];
                        ctl[1] = ci[k];
                    }
                chosen |= 1u << kk;
            }
            for (int l = tid; l < i; l += MT) {
                const bool on = l < RL;
                ws[l] = on ? Wl[(size_t)l * Mpad + s] : Wt[(int64_t)l * Mpad + s];
                wds[l] = on ? Wdl[(size_t)l * Mpad + s] : Wdt[(int64_t)l * Mpad + s];
            }
            for (int kk = tid; kk < p; kk += MT) {
                const double c = Xc[(int64_t)kk * Mpad + s];
                xs[kk] = c;
                XD[i * p + kk] = c;
            }
            __syncthreads();   // A1
            const double vs = sc[S_VS];
            if (!(vs > 0.0)) { notpd = 1; break; }
            const double delta = sqrt(vs);
            // ---- phase B: the location-level quantities of the new point
            //  second derivatives of K(x_l, s); L^{-1} row; Hd l; Hdd l
            for (int l = tid; l < i; l += MT) {
                double d2 = 0.0;
                for (int kk = 0; kk < p; ++kk) {
                    const double dd = XD[l * p + kk] - xs[kk];
                    d2 += dd * dd;
                }
                const double kv = exp(-(d2 / theta));
                kdd[l] = kv * (d2 * d2 / (th2 * th2) - 2.0 * d2 / (th2 * theta));
                double a1 = 0.0, a2 = 0.0;
                for (int m = 0; m < i; ++m) {
                    a1 += Hd[sym(l, m)] * ws[m];
                    a2 += Hdd[sym(l, m)] * ws[m];
                }
                hdw[l] = a1;
                hddw[l] = a2;
            }
            for (int m = tid; m < i; m += MT) {   // new row of L^{-1}: -(l' L^{-1})_m / delta
                double a = 0.0;
                for (int l = m; l < i; ++l) a += ws[l] * Li[tri(l, m)];
                lrow[m] = -a / delta;
            }
            __syncthreads();   // A2
            for (int l = tid; l < i; l += MT) {    // L^{-1} d2k_j(s), then the new columns
                double a = 0.0;
                for (int m = 0; m <= l; ++m) a += Li[tri(l, m)] * kdd[m];
                wdds[l] = a;
                h[l] = (wds[l] - hdw[l]) / delta;
                hh[l] = (a - hddw[l]) / delta;
            }
            for (int m = tid; m < i; m += MT) Li[tri(i, m)] = lrow[m];
            if (tid == 0) Li[tri(i, i)] = 1.0 / delta;
            __syncthreads();   // A3
            if (wave == 0) {
                const double wl_h = wdot(ws, h, i, lane);
                const double wl_hh = wdot(ws, hh, i, lane);
                const double wds_l = wdot(wds, ws, i, lane);
                const double wdds_l = wdot(wdds, ws, i, lane);
                const double h_u = wdot(h, u, i, lane);
                const double hh_u = wdot(hh, u, i, lane);
                const double h_h = wdot(h, h, i, lane);
                const double l_u = wdot(ws, u, i, lane);
                const double l_wx = wdot(ws, wx, i, lane);
                const double l_wdx = wdot(ws, wdx, i, lane);
                const double hi = -wl_h / delta - wds_l / (delta * delta);
                const double hhi = -wl_hh / delta - wdds_l / (delta * delta);
                const int c1 = ctl[1];
                const double d2xs = sc[S_D2XS];
                const double kxs = exp(-(d2xs / theta));
                const double ui = (A.y[c1] - l_u) / delta;
                const double wxi = (kxs - l_wx) / delta;
                const double wdxi = (kxs * d2xs / th2 - l_wdx) / delta;
                if (lane == 0) {
                    sc[S_Q] += 2.0 * ui * h_u + ui * ui * hi;
                    sc[S_R] += 2.0 * ui * hh_u + ui * ui * hhi;
                    sc[S_T2] += hhi;
                    sc[S_T3] += 2.0 * h_h + hi * hi;
                    sc[S_PSI] += ui * ui;
                    sc[S_VX] -= wxi * wxi;
                    sc[S_UI] = ui;
                    sc[S_WXI] = wxi;
                    sc[S_HI] = hi;
                    sc[S_ZI] = h_u + hi * ui;
                    h[i] = hi;
                    hh[i] = hhi;
                    u[i] = ui;
                    wx[i] = wxi;
                    wdx[i] = wdxi;
                    if (A.sel) A.sel[t * A.sel_stride + i] = c1;
                }
            }
            __syncthreads();   // A4
            const double ui = sc[S_UI];
            for (int m = tid; m <= i; m += MT) {   // border Hd and Hdd with row i
                Hd[tri(i, m)] = h[m];
                Hdd[tri(i, m)] = hh[m];
            }
            for (int l = tid; l < i; l += MT) z[l] += h[l] * ui;
            if (tid == 0) z[i] = sc[S_ZI];
            __syncthreads();   // A5
            const int j = i + 1;
            if (wave == 0 && j >= 3) {
                const double sq = wdot(z, z, j, lane);
                const double dmux = wdot(wdx, u, j, lane) - wdot(wx, z, j, lane);
                if (lane == 0) {
                    const double psi = sc[S_PSI], q = sc[S_Q], r = sc[S_R];
                    const double nn = (double)j;
                    sc[S_F] = 0.5 * (sc[S_T2] - sc[S_T3]) - 0.5 * nn * (r - 2.0 * sq) / psi - 0.5 * nn * q * q / (psi * psi);
                    sc[S_DMUX] = dmux;
                }
            }
            __syncthreads();   // A6: F and dmu(x) published
            if (i == n - 1) break;
            // ---- phase C: stream the candidate columns; new tile rows; O(1) updates
            const double wxi = sc[S_WXI], hi = sc[S_HI], zi = sc[S_ZI];
            double d1[CPT], dz[CPT], dh[CPT], d4[CPT];
#pragma unroll
            for (int k = 0; k < CPT; ++k) d1[k] = dz[k] = dh[k] = d4[k] = 0.0;
            // rows in LDS first, then the slab's rows stream with the next
            // row's loads in flight during this row's arithmetic (ascending
            // rows throughout)
            const int il = i < RL ? i : RL;
            for (int l = 0; l < il; ++l) {
                const double wl = ws[l], zl = z[l], hl = h[l];
#pragma unroll
                for (int k = 0; k < CPT; ++k) {
                    const double cw = Wl[(size_t)l * Mpad + tid + k * MT];
                    const double cwd = Wdl[(size_t)l * Mpad + tid + k * MT];
                    d1[k] += wl * cw;
                    dz[k] += zl * cw;
                    dh[k] += hl * cw;
                    d4[k] += wl * cwd;
                }
            }
            double nw[CPT], nwd[CPT];
            if (i > il) {
#pragma unroll
                for (int k = 0; k < CPT; ++k) {
                    nw[k] = Wt[(int64_t)il * Mpad + tid + k * MT];
                    nwd[k] = Wdt[(int64_t)il * Mpad + tid + k * MT];
                }
            }
            for (int l = il; l < i; ++l) {
                double cw[CPT], cwd[CPT];
#pragma unroll
                for (int k = 0; k < CPT; ++k) { cw[k] = nw[k]; cwd[k] = nwd[k]; }
                if (l + 1 < i) {
                    const double* wr = Wt + (int64_t)(l + 1) * Mpad + tid;
                    const double* wdr = Wdt + (int64_t)(l + 1) * Mpad + tid;
#pragma unroll
                    for (int k = 0; k < CPT; ++k) {
                        nw[k] = wr[k * MT];
                        nwd[k] = wdr[k * MT];
                    }
                }
                const double wl = ws[l], zl = z[l], hl = h[l];
#pragma unroll
                for (int k = 0; k < CPT; ++k) {
                    d1[k] += wl * cw[k];
                    dz[k] += zl * cw[k];
                    dh[k] += hl * cw[k];
                    d4[k] += wl * cwd[k];
                }
            }
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
                const int slot = tid + k * MT;
                double d2 = 0.0;
                for (int kk = 0; kk < p; ++kk) {
                    const double dd = xs[kk] - Xc[(int64_t)kk * Mpad + slot];
                    d2 += dd * dd;
                }
                const double ksc = exp(-(d2 / theta));
                const double r = (ksc - d1[k]) / delta;
                const double wdn = (ksc * d2 / th2 - d4[k]) / delta;
                double* wrow = i < RL ? Wl + (size_t)i * Mpad : Wt + (int64_t)i * Mpad;
                double* wdrow = i < RL ? Wdl + (size_t)i * Mpad : Wdt + (int64_t)i * Mpad;
                if (!((chosen >> k) & 1u)) {
                    wrow[slot] = r;
                    wdrow[slot] = wdn;
                    v[k] -= r * r;
                    cov[k] -= wxi * r;
                    av[k] += wdn * ui;
                    bv[k] += wdn * r;
                    Qv[k] += 2.0 * r * dh[k] + r * r * hi;
                    zc[k] = dz[k] + zi * r;
                } else {
                    wrow[slot] = 0.0;
                    wdrow[slot] = 0.0;
                }
            }
            // ---- argmin of J over live candidates (from step n0 on)
            if (j >= n0) {
                const double psi = sc[S_PSI], vx = sc[S_VX], q = sc[S_Q], F = sc[S_F], dmux = sc[S_DMUX];
                const double scl = psi / (j - 2);
                double bj = INFINITY;
                int bi = 0x7fffffff, bs = -1;
#pragma unroll
                for (int k = 0; k < CPT; ++k) {
                    if ((chosen >> k) & 1u) continue;
                    double J = INFINITY;
                    if (v[k] > 0.0) {
                        const double Vxc = scl * (vx - cov[k] * cov[k] / v[k]);
                        const double Vc = scl * v[k];
                        const double dmu = av[k] - zc[k];
                        const double dV = (-q * v[k] - psi * (2.0 * bv[k] - Qv[k])) / (j - 2);
                        const double G = F + dV * dV / (2.0 * Vc * Vc) + dmu * dmu / Vc;
                        J = Vxc + dmux * dmux / G;
                        if (!(J == J)) J = INFINITY;
                    }
                    if (bs < 0 || nearer(J, ci[k], bj, bi)) { bj = J; bi = ci[k]; bs = tid + k * MT; }
                }
                wave_pick<false>(bj, bi, bs);
                if (lane == 0) { redv[wave] = bj; redi[wave] = bi; reds[wave] = bs; }
                __syncthreads();   // B
                bj = redv[0]; bi = redi[0]; bs = reds[0];
                for (int w2 = 1; w2 < MWAVES; ++w2) pick<false>(bj, bi, bs, redv[w2], redi[w2], reds[w2]);
                if (bs < 0 || bj == INFINITY) { notpd = 1; break; }
                s_next = bs;
            }
            __syncthreads();   // everyone is done with this step's vectors
        }

        // ---- prediction (eqs predgp, preds2 with N -> n)
        __syncthreads();
        if (tid == 0) {
            double mean = NAN, s2v = NAN, var = NAN;
            if (!notpd) {
                double m = 0.0, ps = 0.0, qq = 0.0;
                for (int l = 0; l < n; ++l) {
                    m += wx[l] * u[l];
                    ps += u[l] * u[l];
                    qq += wx[l] * wx[l];
                }
                const double vxn = one_eta - qq;
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

template <int MT, int CPT>
int launch(const MspeArgs& a, size_t lds, int blocks, hipStream_t stream)
{
    hipLaunchKernelGGL((mspe_kernel<MT, CPT>), dim3(blocks), dim3(MT), lds, stream, a);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// 512 threads above 1024 candidates (at most 4 slots per thread), else 256.
int threads_for(int M) { return M > 1024 ? 512 : 256; }

int cpt_for(int M)
{
    const int mt = threads_for(M);
    int c = 1;
    while (c * mt < M) c <<= 1;
    return c;
}

}  // namespace

size_t mspe_lds_bytes(int nmax, int p) { return lds_base_bytes(nmax, p); }

size_t mspe_slab_bytes(int nmax, int Mmax, int p)
{
    const size_t Mpad = (size_t)cpt_for(Mmax) * threads_for(Mmax);
    return ((size_t)p + 2 * (size_t)(nmax > 1 ? nmax - 1 : 1)) * Mpad * sizeof(double);
}

int mspe_prepare(int32_t nmax, int32_t Mmax, int p, size_t max_lds, std::string* err)
{
    if (Mmax > 2048) { *err = "the MSPE kernel takes at most 2048 candidates"; return -1; }
    if (mspe_lds_bytes(nmax, p) > max_lds) { *err = "local design too large for the MSPE kernel"; return -1; }
    const void* k[6] = {(const void*)mspe_kernel<256, 1>, (const void*)mspe_kernel<256, 2>,
                        (const void*)mspe_kernel<256, 4>, (const void*)mspe_kernel<512, 1>,
                        (const void*)mspe_kernel<512, 2>, (const void*)mspe_kernel<512, 4>};
    for (const void* f : k)
        if (!set_lds_limit(f, max_lds)) { *err = "cannot reserve LDS for the MSPE kernel"; return -2; }
    return 0;
}

int mspe_run(const MspeArgs& args, int blocks, size_t max_lds, hipStream_t stream, std::string* err)
{
    if (args.T == 0) return 0;
    const size_t base = (lds_base_bytes(args.nmax, args.p) + 7) & ~(size_t)7;
    if (base > max_lds) { *err = "local design too large for the MSPE kernel"; return -1; }
    // as many leading tile rows (W and Wd) as the LDS left over holds
    MspeArgs a = args;
    const size_t pair = 2 * (size_t)cpt_for(a.M) * threads_for(a.M) * sizeof(double);
    const size_t fit = (max_lds - base) / pair;
    a.lds_rows = (int)std::min<size_t>(fit, (size_t)(a.nmax > 1 ? a.nmax - 1 : 0));
    const size_t lds = base + (size_t)a.lds_rows * pair;
    fill_u32(a.counter, 1, 0u, stream);
    const int c = cpt_for(a.M);
    int rc;
    if (threads_for(a.M) == 512)
        rc = c == 1 ? launch<512, 1>(a, lds, blocks, stream)
           : c == 2 ? launch<512, 2>(a, lds, blocks, stream)
                    : launch<512, 4>(a, lds, blocks, stream);
    else
        rc = c == 1 ? launch<256, 1>(a, lds, blocks, stream)
           : c == 2 ? launch<256, 2>(a, lds, blocks, stream)
                    : launch<256, 4>(a, lds, blocks, stream);
    if (rc) { *err = "MSPE kernel launch failed"; return rc; }
    return 0;
}

}  // namespace lagp
