// Learned warm start: POD basis of MTF solutions and a small MLP (FP32), hand-written kernels.
//
// MLP: n_in -> width (tanh) -> width (tanh) -> n_out (linear), row-major activations
// [batch][features], weights W_l [out][in] row-major, parameters packed as
// (W1, b1, W2, b2, W3, b3).  Loss: mean squared error over all outputs of the batch.
#include "device.h"

#include <algorithm>

namespace mtf {

namespace {

// C[M][N] = sum_k opA(A)[m][k] opB(B)[k][n] (+ bias[n]) (+ tanh), FP32, 16 x 16 tiles.
// opA: ta = 0 -> A[m][k] at A[m*lda + k]; ta = 1 -> A[k][m] at A[k*lda + m].
// opB: tb = 0 -> B[k][n] at B[k*ldb + n]; tb = 1 -> B[n][k] at B[n*ldb + k].
// accumulate: C += result instead of C = result.
__global__ __launch_bounds__(256) void k_sgemm(int M, int N, int K, const float* __restrict__ A, int lda, int ta,
                                               const float* __restrict__ B, int ldb, int tb, const float* __restrict__ bias,
                                               int act_tanh, float* __restrict__ C, int ldc, int accumulate) {
    __shared__ float As[16][17];
    __shared__ float Bs[16][17];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int m = blockIdx.y * 16 + ty, n = blockIdx.x * 16 + tx;
    float acc = 0.f;
    for (int k0 = 0; k0 < K; k0 += 16) {
        const int ka = k0 + tx, kb = k0 + ty;
        const int am = blockIdx.y * 16 + ty;
        float a = 0.f, b = 0.f;
        if (am < M && ka < K) a = ta ? A[(int64_t)ka * lda + am] : A[(int64_t)am * lda + ka];
        const int bn = blockIdx.x * 16 + tx;
        if (bn < N && kb < K) b = tb ? B[(int64_t)bn * ldb + kb] : B[(int64_t)kb * ldb + bn];
        As[ty][tx] = a;
        Bs[ty][tx] = b;
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) acc += As[ty][kk] * Bs[kk][tx];
        __syncthreads();
    }
    if (m >= M || n >= N) return;
    if (bias) acc += bias[n];
    if (act_tanh) acc = tanhf(acc);
    float* c = C + (int64_t)m * ldc + n;
    *c = accumulate ? *c + acc : acc;
}

// dZ = dA * (1 - A^2) (tanh derivative), elementwise
__global__ void k_tanh_back(const float* __restrict__ A, const float* __restrict__ dA, float* __restrict__ dZ, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) dZ[e] = dA[e] * (1.f - A[e] * A[e]);
}

// dY = 2 (Y - T) / (rows * cols);  loss partials per block
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ Y, const float* __restrict__ T, float* __restrict__ dY,
                                             int64_t n, float scale, float* __restrict__ loss_part) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float l = 0.f;
    if (e < n) {
        const float d = Y[e] - T[e];
        dY[e] = 2.f * d * scale;
        l = d * d * scale;
    }
    __shared__ float red[256];
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// db[n] = sum_m dZ[m][n]
__global__ void k_colsum(const float* __restrict__ dZ, int M, int N, float* __restrict__ db) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int m = 0; m < M; ++m) s += dZ[(int64_t)m * N + n];
    db[n] = s;
}

// Adam (Kingma & Ba 2015) with bias correction folded into the step size.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m1, float* __restrict__ m2,
                       int64_t n, float lr_t, float b1, float b2, float eps) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float gi = g[e];
    const float a = b1 * m1[e] + (1.f - b1) * gi;
    const float b = b2 * m2[e] + (1.f - b2) * gi * gi;
    m1[e] = a;
    m2[e] = b;
    p[e] -= lr_t * a / (sqrtf(b) + eps);
}

// Gather rows idx[0..B) of X [n][cols] into Xb [B][cols]
__global__ void k_gather_rows(const float* __restrict__ X, const int* __restrict__ idx, int B, int cols, float* __restrict__ Xb) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)B * cols) return;
    const int r = (int)(e / cols), c = (int)(e % cols);
    Xb[e] = X[(int64_t)idx[r] * cols + c];
}

// ---------------------------------------------------------------------------
// complex64 helpers for the POD basis
// ---------------------------------------------------------------------------

// C (m x n) = A^H B with A (k x m), B (k x n), column-major, complex64.  64 x 64 tiles.
__global__ __launch_bounds__(256) void k_cgemm_hn(int m, int n, int k, const float* __restrict__ A, int64_t lda,
                                                  const float* __restrict__ B, int64_t ldb, float* __restrict__ C,
                                                  int64_t ldc) {
    __shared__ float2 As[8][64 + 1];
    __shared__ float2 Bs[8][64 + 1];
    const int tid = threadIdx.x;
    const int tr = tid & 15, tc = tid >> 4;
    const int row0 = blockIdx.x * 64, col0 = blockIdx.y * 64;
    float acc[4][4][2];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) acc[i][j][0] = acc[i][j][1] = 0.f;
    const float2* A2 = reinterpret_cast<const float2*>(A);
    const float2* B2 = reinterpret_cast<const float2*>(B);
    for (int k0 = 0; k0 < k; k0 += 8) {
        for (int e = tid; e < 512; e += 256) {
            const int kk = e & 7, r = e >> 3;
            const int gk = k0 + kk;
            const int gr = row0 + r;
            float2 a = (gr < m && gk < k) ? A2[gk + (int64_t)gr * lda] : make_float2(0.f, 0.f);
            As[kk][r] = make_float2(a.x, -a.y);     // conjugate
            const int gc = col0 + r;
            Bs[kk][r] = (gc < n && gk < k) ? B2[gk + (int64_t)gc * ldb] : make_float2(0.f, 0.f);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
            float2 a[4], b[4];
            for (int i = 0; i < 4; ++i) a[i] = As[kk][tr + 16 * i];
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tc + 16 * j];
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) {
                    acc[i][j][0] += a[i].x * b[j].x - a[i].y * b[j].y;
                    acc[i][j][1] += a[i].x * b[j].y + a[i].y * b[j].x;
                }
        }
        __syncthreads();
    }
    for (int i = 0; i < 4; ++i) {
        const int gr = row0 + tr + 16 * i;
        if (gr >= m) continue;
        for (int j = 0; j < 4; ++j) {
            const int gc = col0 + tc + 16 * j;
            if (gc >= n) continue;
            float* c = C + 2 * (gr + (int64_t)gc * ldc);
            c[0] = acc[i][j][0];
            c[1] = acc[i][j][1];
        }
    }
}

// complex128 [cols][ld] -> complex64 [cols][n]
// C = op(A) B in complex128 (column-major): op(A) = A (m x k, ld lda) when HERM is false, A^H (A
// stored k x m, ld lda) when true.  64 x 64 tile, k-tile 8, each thread 4 x 4 outputs; FP64 FMA.
template <bool HERM>
__global__ __launch_bounds__(256) void k_zgemm(int m, int n, int k, const double* __restrict__ A, int64_t lda,
                                               const double* __restrict__ B, int64_t ldb, double* __restrict__ C,
                                               int64_t ldc) {
    __shared__ double2 As[8][64 + 1];
    __shared__ double2 Bs[8][64 + 1];
    const int tid = threadIdx.x;
    const int tr = tid & 15, tc = tid >> 4;
    const int row0 = blockIdx.x * 64, col0 = blockIdx.y * 64;
    double acc[4][4][2];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) acc[i][j][0] = acc[i][j][1] = 0.0;
    const double2* A2 = reinterpret_cast<const double2*>(A);
    const double2* B2 = reinterpret_cast<const double2*>(B);
    for (int k0 = 0; k0 < k; k0 += 8) {
        for (int e = tid; e < 512; e += 256) {
            const int kk = e & 7, r = e >> 3;
            const int gk = k0 + kk;
            const int gr = row0 + r;
            double2 a = make_double2(0.0, 0.0);
            if (gr < m && gk < k) {
                if (HERM) {
                    a = A2[gk + (int64_t)gr * lda];
                    a.y = -a.y;                          // conjugate
                } else {
                    a = A2[gr + (int64_t)gk * lda];
                }
            }
            As[kk][r] = a;
            const int gc = col0 + r;
            Bs[kk][r] = (gc < n && gk < k) ? B2[gk + (int64_t)gc * ldb] : make_double2(0.0, 0.0);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
            double2 a[4], b[4];
            for (int i = 0; i < 4; ++i) a[i] = As[kk][tr + 16 * i];
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tc + 16 * j];
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) {
                    acc[i][j][0] = fma(a[i].x, b[j].x, fma(-a[i].y, b[j].y, acc[i][j][0]));
                    acc[i][j][1] = fma(a[i].x, b[j].y, fma(a[i].y, b[j].x, acc[i][j][1]));
                }
        }
        __syncthreads();
    }
    for (int i = 0; i < 4; ++i) {
        const int gr = row0 + tr + 16 * i;
        if (gr >= m) continue;
        for (int j = 0; j < 4; ++j) {
            const int gc = col0 + tc + 16 * j;
            if (gc >= n) continue;
            double* c = C + 2 * (gr + (int64_t)gc * ldc);
            c[0] = acc[i][j][0];
            c[1] = acc[i][j][1];
        }
    }
}

__global__ void k_c128_to_c64(const double* __restrict__ X, int64_t ld, int64_t n, int cols, float* __restrict__ Y) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (e >= n || c >= cols) return;
    Y[2 * ((int64_t)c * n + e)] = (float)X[2 * ((int64_t)c * ld + e)];
    Y[2 * ((int64_t)c * n + e) + 1] = (float)X[2 * ((int64_t)c * ld + e) + 1];
}

// complex64 [cols][n] -> complex128 [cols][ld]
__global__ void k_c64_to_c128(const float* __restrict__ X, int64_t n, int cols, double* __restrict__ Y, int64_t ld) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (e >= n || c >= cols) return;
    Y[2 * ((int64_t)c * ld + e)] = X[2 * ((int64_t)c * n + e)];
    Y[2 * ((int64_t)c * ld + e) + 1] = X[2 * ((int64_t)c * n + e) + 1];
}

inline unsigned gridn(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

void launch_sgemm(int M, int N, int K, const float* A, int lda, int ta, const float* B, int ldb, int tb, const float* bias,
                  int act_tanh, float* C, int ldc, int accumulate, hipStream_t s) {
    if (M <= 0 || N <= 0) return;
    hipLaunchKernelGGL(k_sgemm, dim3(gridn(N, 16), gridn(M, 16)), dim3(256), 0, s, M, N, K, A, lda, ta, B, ldb, tb, bias,
                       act_tanh, C, ldc, accumulate);
}

void launch_tanh_back(const float* A, const float* dA, float* dZ, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_tanh_back, dim3(gridn(n, 256)), dim3(256), 0, s, A, dA, dZ, n);
}

int launch_mse(const float* Y, const float* T, float* dY, int64_t n, float scale, float* loss_part, hipStream_t s) {
    const int nb = (int)gridn(n, 256);
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, s, Y, T, dY, n, scale, loss_part);
    return nb;
}

void launch_colsum(const float* dZ, int M, int N, float* db, hipStream_t s) {
    hipLaunchKernelGGL(k_colsum, dim3(gridn(N, 256)), dim3(256), 0, s, dZ, M, N, db);
}

void launch_adam(float* p, const float* g, float* m1, float* m2, int64_t n, float lr_t, float b1, float b2, float eps,
                 hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3(gridn(n, 256)), dim3(256), 0, s, p, g, m1, m2, n, lr_t, b1, b2, eps);
}

void launch_gather_rows(const float* X, const int* idx, int B, int cols, float* Xb, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_rows, dim3(gridn((int64_t)B * cols, 256)), dim3(256), 0, s, X, idx, B, cols, Xb);
}

void launch_cgemm_hn(int m, int n, int k, const float* A, int64_t lda, const float* B, int64_t ldb, float* C, int64_t ldc,
                     hipStream_t s) {
    if (m <= 0 || n <= 0) return;
    hipLaunchKernelGGL(k_cgemm_hn, dim3(gridn(m, 64), gridn(n, 64)), dim3(256), 0, s, m, n, k, A, lda, B, ldb, C, ldc);
}

void launch_zgemm(int m, int n, int k, bool herm_a, const double* A, int64_t lda, const double* B, int64_t ldb,
                  double* C, int64_t ldc, hipStream_t s) {
    if (m <= 0 || n <= 0) return;
    if (herm_a)
        hipLaunchKernelGGL(k_zgemm<true>, dim3(gridn(m, 64), gridn(n, 64)), dim3(256), 0, s, m, n, k, A, lda, B, ldb, C,
                           ldc);
    else
        hipLaunchKernelGGL(k_zgemm<false>, dim3(gridn(m, 64), gridn(n, 64)), dim3(256), 0, s, m, n, k, A, lda, B, ldb,
                           C, ldc);
}

void launch_c128_to_c64(const double* X, int64_t ld, int64_t n, int cols, float* Y, hipStream_t s) {
    hipLaunchKernelGGL(k_c128_to_c64, dim3(gridn(n, 256), (unsigned)cols), dim3(256), 0, s, X, ld, n, cols, Y);
}

void launch_c64_to_c128(const float* X, int64_t n, int cols, double* Y, int64_t ld, hipStream_t s) {
    hipLaunchKernelGGL(k_c64_to_c128, dim3(gridn(n, 256), (unsigned)cols), dim3(256), 0, s, X, n, cols, Y, ld);
}

}  // namespace mtf
