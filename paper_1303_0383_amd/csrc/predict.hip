// predict.hip -- local GP prediction from given local designs (eqs predgp and
// preds2 of Section 2 with N -> n) through a fresh FP64 Cholesky
// factorisation of K_n = K(D, D) + g I.
//
// One 64-thread workgroup (a single wave) per location.  The lower triangle
// of K_n lives packed in LDS and is factorised right-looking: at column m the
// pivot is square-rooted, the column divided by it, and the trailing triangle
// and the two right-hand sides k_n(x) and Y_n are updated.  Every element is
// therefore reduced by its products in ascending column order, the same
// operation sequence as a row-by-row factorisation followed by forward
// substitution, and divisions are correctly rounded (3-FMA Markstein
// correction).  The file is compiled with -ffp-contract=off.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "lagp_internal.h"

namespace lagp {

namespace {

constexpr int PT = 64;   // threads per workgroup

__device__ __forceinline__ double qdiv(double a, double b, double y)
{
    const double q = a * y;
    const double r = __builtin_fma(-q, b, a);
    return __builtin_fma(r, y, q);
}

__device__ __forceinline__ int tri(int i, int k) { return i * (i + 1) / 2 + k; }

__global__ void __launch_bounds__(PT) local_predict_kernel(const double* __restrict__ Xaos,
                                                           const double* __restrict__ y, int p,
                                                           const double* __restrict__ XX, int64_t T,
                                                           int64_t N, const int32_t* __restrict__ sel, int64_t sel_stride,
                                                           const int32_t* __restrict__ n_per, int n_all,
                                                           double theta_all, const double* __restrict__ theta_per,
                                                           double eta, double* mean, double* s2, int32_t* df,
                                                           double* var, int8_t* status)
{
    extern __shared__ double sm[];
    const int64_t t = blockIdx.x;
    if (t >= T) return;
    const int tid = threadIdx.x;
    const int n = n_per ? n_per[t] : n_all;
    const int32_t* D = sel + t * sel_stride;
    double* A = sm;                       // packed lower triangle, n(n+1)/2
    double* b1 = A + n * (n + 1) / 2;     // k_n(x), then L^{-1} k_n(x)
    double* b2 = b1 + n;                  // Y_n, then L^{-1} Y_n
    __shared__ int bad;
    // A per-location lengthscale that is not a positive finite number fails the location.
    const double theta = theta_per ? theta_per[t] : theta_all;
    const double rtheta = 1.0 / theta;
    const double* x = XX + t * p;
    if (tid == 0) bad = (theta > 0.0 && theta < INFINITY) ? 0 : 1;
    __syncthreads();
    // A usable design has n valid indices (the design kernel marks failures with -1).
    for (int a = tid; a < n; a += PT)
        if (D[a] < 0 || D[a] >= N) bad = 1;
    __syncthreads();
    if (!bad) {
        for (int i = 0; i < n; ++i) {
            const double* xi = Xaos + (int64_t)D[i] * p;
            for (int k = tid; k <= i; k += PT) {
                double v;
                if (i == k) {
                    v = 1.0 + eta;
                } else {
                    const double* xk = Xaos + (int64_t)D[k] * p;
                    double s = 0.0;
                    for (int c = 0; c < p; ++c) {
                        const double d = xi[c] - xk[c];
                        s += d * d;
                    }
                    v = exp(-qdiv(s, theta, rtheta));
                }
                A[tri(i, k)] = v;
            }
        }
        for (int a = tid; a < n; a += PT) {
            const double* xa = Xaos + (int64_t)D[a] * p;
            double s = 0.0;
            for (int c = 0; c < p; ++c) {
                const double d = xa[c] - x[c];
                s += d * d;
            }
            b1[a] = exp(-qdiv(s, theta, rtheta));
            b2[a] = y[D[a]];
        }
        __syncthreads();
        for (int m = 0; m < n; ++m) {
            const double amm = A[tri(m, m)];
            if (!(amm > 0.0)) {   // uniform: every thread reads the same pivot
                if (tid == 0) bad = 1;
                break;
            }
            const double d = sqrt(amm);
            const double rd = 1.0 / d;
            __syncthreads();   // everyone has read the pivot before it is overwritten
            if (tid == 0) {
                A[tri(m, m)] = d;
                b1[m] = qdiv(b1[m], d, rd);
                b2[m] = qdiv(b2[m], d, rd);
            }
            for (int i = m + 1 + tid; i < n; i += PT) A[tri(i, m)] = qdiv(A[tri(i, m)], d, rd);
            __syncthreads();
            // Trailing update of rows i > m: columns m < k <= i, and both right-hand sides.
            for (int i = m + 1; i < n; ++i) {
                const double lim = A[tri(i, m)];
                for (int k = m + 1 + tid; k <= i; k += PT) A[tri(i, k)] -= lim * A[tri(k, m)];
            }
            for (int i = m + 1 + tid; i < n; i += PT) {
                const double lim = A[tri(i, m)];
                b1[i] -= lim * b1[m];
                b2[i] -= lim * b2[m];
            }
            __syncthreads();
        }
        __syncthreads();
    }
    if (tid == 0) {
        double mu = NAN, sc = NAN, vr = NAN;
        if (!bad) {
            double m = 0.0, ps = 0.0, q = 0.0;
            for (int l = 0; l < n; ++l) {
                m += b1[l] * b2[l];
                ps += b2[l] * b2[l];
                q += b1[l] * b1[l];
            }
            const double vx = (1.0 + eta) - q;
            mu = m;
            sc = ps * vx / n;
            vr = n > 2 ? ps * vx / (n - 2) : NAN;
        }
        mean[t] = mu;
        s2[t] = sc;
        if (var) var[t] = vr;
        if (df) df[t] = n;
        if (status) status[t] = bad ? 1 : 0;
    }
}

}  // namespace

size_t predict_lds_bytes(int nmax)
{
    return ((size_t)nmax * (nmax + 1) / 2 + 2 * (size_t)nmax) * sizeof(double);
}

int predict_prepare(int32_t nmax, size_t max_lds, std::string* err)
{
    const size_t lds = predict_lds_bytes(nmax);
    if (lds > max_lds) { *err = "local design too large for the prediction kernel"; return -1; }
    if (!set_lds_limit((const void*)local_predict_kernel, max_lds)) {
        *err = "cannot reserve LDS for the prediction kernel";
        return -2;
    }
    return 0;
}

int predict_run(const DeviceDesign& D, const double* XX, int64_t T, const int32_t* sel, int64_t sel_stride,
                const int32_t* n_per, int32_t nmax, double theta, const double* theta_per, double eta, double* mean,
                double* s2, int32_t* df, double* var, int8_t* status, size_t max_lds, hipStream_t stream,
                std::string* err)
{
    if (T == 0) return 0;
    const size_t lds = predict_lds_bytes(nmax);
    if (lds > max_lds) { *err = "local design too large for the prediction kernel"; return -1; }
    hipLaunchKernelGGL(local_predict_kernel, dim3((unsigned)T), dim3(PT), lds, stream, D.Xaos, D.y, D.p, XX, T, D.N, sel,
                       sel_stride, n_per, nmax, theta, theta_per, eta, mean, s2, df, var, status);
    if (hipGetLastError() != hipSuccess) { *err = "prediction kernel launch failed"; return -2; }
    return 0;
}

}  // namespace lagp
