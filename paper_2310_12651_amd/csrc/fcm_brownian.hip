// The pair part of Brownian velocities in fast FCM: y = C^(1/2) xi for the
// symmetric positive definite matrix C = M - M~ of the VF pair and self
// corrections (positive splitting, Sec. 3.3), by the Lanczos method the paper
// proposes for it (Sec. 7).  The product C v is the pair-correction pass with
// forces v and no torques; the recurrence runs on the host over device vectors
// (FP64), the small tridiagonal square root on the host.
#include <math.h>
#include <string.h>

#include "fcm_internal.h"

namespace fcm {

namespace {

constexpr int kRedBlocks = 256;
constexpr int kRedThreads = 256;
constexpr int kMaxLanczos = 64;

// partial[b] = sum over the elements block b visits of a[i] * b[i] (a fixed
// order per block: the host adds the partial sums in block order)
__global__ __launch_bounds__(kRedThreads) void k_dot(const double* __restrict__ a,
                                                     const double* __restrict__ b, int n,
                                                     double* __restrict__ partial) {
    __shared__ double sh[kRedThreads / 64];
    double s = 0.0;
    for (int i = blockIdx.x * kRedThreads + threadIdx.x; i < n; i += kRedBlocks * kRedThreads)
        s += a[i] * b[i];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kRedThreads / 64; ++w) t += sh[w];
        partial[blockIdx.x] = t;
    }
}

// y = alpha x + beta y (y is not read when beta = 0)
__global__ void k_axpby(double alpha, const double* __restrict__ x, double beta,
                        double* __restrict__ y, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = beta == 0.0 ? alpha * x[i] : alpha * x[i] + beta * y[i];
}

struct Coefs {
    double c[kMaxLanczos];
};

// y = sum_j c_j v_j over the m basis vectors v_j = basis + j * stride
__global__ void k_lincomb(const double* __restrict__ basis, size_t stride, Coefs c, int m,
                          double* __restrict__ y, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int j = 0; j < m; ++j) s += c.c[j] * basis[j * stride + i];
    y[i] = s;
}

int blocks(int n) { return (n + 255) / 256; }

hipError_t dot(const fcm_plan_impl* P, const double* a, const double* b, int n, hipStream_t st,
               double* out) {
    hipLaunchKernelGGL(k_dot, dim3(kRedBlocks), dim3(kRedThreads), 0, st, a, b, n, P->partial);
    double h[kRedBlocks];
    hipError_t e = hipMemcpyAsync(h, P->partial, sizeof(h), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    double s = 0.0;
    for (int k = 0; k < kRedBlocks; ++k) s += h[k];
    *out = s;
    return e;
}

// Eigen-decomposition of the symmetric m x m matrix A (row-major, destroyed):
// eigenvalues in w, eigenvectors in the columns of Q (cyclic Jacobi rotations).
void jacobi_eig(double* A, int m, double* w, double* Q) {
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) Q[i * m + j] = i == j ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < m; ++i) {
            diag += A[i * m + i] * A[i * m + i];
            for (int j = i + 1; j < m; ++j) off += A[i * m + j] * A[i * m + j];
        }
        if (off <= 1e-32 * diag) break;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) {
                const double apq = A[p * m + q];
                if (apq == 0.0) continue;
                const double theta = (A[q * m + q] - A[p * m + p]) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < m; ++k) {
                    const double akp = A[k * m + p], akq = A[k * m + q];
                    A[k * m + p] = c * akp - s * akq;
                    A[k * m + q] = s * akp + c * akq;
                }
                for (int k = 0; k < m; ++k) {
                    const double apk = A[p * m + k], aqk = A[q * m + k];
                    A[p * m + k] = c * apk - s * aqk;
                    A[q * m + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < m; ++k) {
                    const double qkp = Q[k * m + p], qkq = Q[k * m + q];
                    Q[k * m + p] = c * qkp - s * qkq;
                    Q[k * m + q] = s * qkp + c * qkq;
                }
            }
    }
    for (int i = 0; i < m; ++i) w[i] = A[i * m + i];
}

// c = beta0 T^(1/2) e1 for the m x m tridiagonal T (diagonal a, off-diagonal b)
void tridiag_sqrt_e1(const double* a, const double* b, int m, double beta0, double* c) {
    double T[kMaxLanczos * kMaxLanczos], Q[kMaxLanczos * kMaxLanczos], w[kMaxLanczos];
    memset(T, 0, sizeof(double) * m * m);
    for (int i = 0; i < m; ++i) {
        T[i * m + i] = a[i];
        if (i + 1 < m) T[i * m + i + 1] = T[(i + 1) * m + i] = b[i];
    }
    jacobi_eig(T, m, w, Q);
    for (int i = 0; i < m; ++i) {
        double s = 0.0;
        for (int k = 0; k < m; ++k) s += Q[i * m + k] * sqrt(fmax(w[k], 0.0)) * Q[0 * m + k];
        c[i] = beta0 * s;
    }
}

}  // namespace

hipError_t lanczos_sqrt_pair(fcm_plan_impl* P, const double* xi, double* y, double tol,
                             int* iters, hipStream_t st) {
    const int n = (int)(3 * P->N);
    const size_t stride = (size_t)3 * P->Ncap;
    double* V = P->krylov;           // basis v_1, v_2, ... (caller order, N x 3 each)
    double* w = P->corr + 3 * P->N;  // work vector
    const int cap = P->krylov_cap < kMaxLanczos ? P->krylov_cap : kMaxLanczos;
    double beta0 = 0.0;
    hipError_t e = dot(P, xi, xi, n, st, &beta0);
    beta0 = sqrt(beta0);
    *iters = 0;
    if (e != hipSuccess) return e;
    if (beta0 == 0.0) {
        hipLaunchKernelGGL(k_axpby, dim3(blocks(n)), dim3(256), 0, st, 0.0, xi, 0.0, y, n);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_axpby, dim3(blocks(n)), dim3(256), 0, st, 1.0 / beta0, xi, 0.0, V, n);
    double a[kMaxLanczos], b[kMaxLanczos], c[kMaxLanczos], cprev[kMaxLanczos];
    int m = 0;
    for (int j = 0; j < cap && e == hipSuccess; ++j) {
        double* vj = V + (size_t)j * stride;
        // w = C v_j: the pair pass with forces v_j and no torques (neighbours searched once)
        e = launch_refresh_forces(P, vj, nullptr, true, st);
        if (e == hipSuccess) e = launch_pair(P, w, nullptr, false, st, true, j == 0);
        if (e != hipSuccess) break;
        if (j > 0)
            hipLaunchKernelGGL(k_axpby, dim3(blocks(n)), dim3(256), 0, st, -b[j - 1],
                               V + (size_t)(j - 1) * stride, 1.0, w, n);
        e = dot(P, w, vj, n, st, &a[j]);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(k_axpby, dim3(blocks(n)), dim3(256), 0, st, -a[j], vj, 1.0, w, n);
        double bb = 0.0;
        e = dot(P, w, w, n, st, &bb);
        b[j] = sqrt(bb);
        m = j + 1;
        tridiag_sqrt_e1(a, b, m, beta0, c);
        double dn = 0.0, cn = 0.0;
        for (int i = 0; i < m; ++i) {
            const double d = c[i] - (i < m - 1 ? cprev[i] : 0.0);
            dn += d * d;
            cn += c[i] * c[i];
        }
        for (int i = 0; i < m; ++i) cprev[i] = c[i];
        if ((j > 0 && dn <= tol * tol * cn) || b[j] <= 1e-14 * beta0 || j + 1 == cap) break;
        hipLaunchKernelGGL(k_axpby, dim3(blocks(n)), dim3(256), 0, st, 1.0 / b[j], w, 0.0,
                           V + (size_t)(j + 1) * stride, n);
    }
    if (e != hipSuccess) return e;
    Coefs cf;
    for (int i = 0; i < kMaxLanczos; ++i) cf.c[i] = i < m ? c[i] : 0.0;
    hipLaunchKernelGGL(k_lincomb, dim3(blocks(n)), dim3(256), 0, st, V, stride, cf, m, y, n);
    *iters = m;
    return hipGetLastError();
}

hipError_t launch_axpby(double alpha, const double* x, double beta, double* y, int n,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_axpby, dim3(blocks(n)), dim3(256), 0, st, alpha, x, beta, y, n);
    return hipGetLastError();
}

}  // namespace fcm
