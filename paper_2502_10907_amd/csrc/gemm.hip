// Multi-right-hand-side block products on MFMA (gfx950).
//
// For many right-hand sides the diagonal blocks are applied as one GEMM per
// subdomain i:
//   [Y_iD | Y_iN] = [K_i | T_i] [[2 X_iD, 2 X_iN], [2/rho_i X_iN, -2 rho_i X_iD]]
// (M = E_i rows, K = 2 E_i, N = 2 nrhs), which is Problem 2's 2x2 Calderon block
// 2 A_i applied to all columns at once; the transmission part is added in the
// finishing kernel.  Complex64 operands are split into bfloat16 hi/lo planes
// (v = hi + lo + O(2^-17 |v|)) and every complex product is formed from three
// bf16 products per real product (hi*hi + hi*lo + lo*hi), twelve
// v_mfma_f32_32x32x16_bf16 per 32x32x16 complex tile, accumulated in FP32.
//
// Operand layouts (k-contiguous so MFMA fragments are single 16-byte LDS reads):
//   A planes: 4 x [Mp][Kp] row-major (re_hi, re_lo, im_hi, im_lo), zero padded;
//   B planes: 4 x [Np][Kp] (column n holds its Kp entries contiguously).
#include "device.h"

#include <algorithm>

namespace mtf {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int BM = 128, BN = 128, BK = 32, LDK = BK + 8;   // LDS row stride in bf16 (80 bytes)

__device__ inline uint16_t bf16_bits(float v) {
    __bf16 h = (__bf16)v;   // round to nearest even
    return __builtin_bit_cast(uint16_t, h);
}

__device__ inline float bf16_value(uint16_t b) { return (float)__builtin_bit_cast(__bf16, b); }

__device__ inline void split(float v, uint16_t& hi, uint16_t& lo) {
    hi = bf16_bits(v);
    lo = bf16_bits(v - bf16_value(hi));
}

__device__ inline bf16x8 negate(bf16x8 a) {
    uint4 u = __builtin_bit_cast(uint4, a);
    u.x ^= 0x80008000u; u.y ^= 0x80008000u; u.z ^= 0x80008000u; u.w ^= 0x80008000u;
    return __builtin_bit_cast(bf16x8, u);
}

__global__ __launch_bounds__(256) void k_gemm_bf16x3(const GemmDesc* __restrict__ descs, const int4* __restrict__ tiles,
                                                     const uint16_t* __restrict__ Abase,
                                                     const uint16_t* __restrict__ Bbase, float* __restrict__ Cbase) {
    __shared__ uint16_t As[4][BM][LDK];
    __shared__ uint16_t Bs[4][BN][LDK];
    const int4 tl = tiles[blockIdx.x];
    const GemmDesc g = descs[tl.x];
    const int64_t m0 = tl.y, n0 = tl.z;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const uint16_t* A = Abase + g.a_off;
    const uint16_t* B = Bbase + g.b_off;
    const int64_t pa = g.Mp * g.Kp, pb = g.Np * g.Kp;
    floatx16 accR[2][2], accI[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int e = 0; e < 16; ++e) { accR[i][j][e] = 0.f; accI[i][j][e] = 0.f; }
    for (int64_t k0 = 0; k0 < g.Kp; k0 += BK) {
        for (int c = tid; c < 2048; c += 256) {
            const int p = c >> 9, rem = c & 511, r = rem >> 2, q = rem & 3;
            *reinterpret_cast<uint4*>(&As[p][r][q * 8]) =
                *reinterpret_cast<const uint4*>(A + p * pa + (m0 + r) * g.Kp + k0 + q * 8);
            *reinterpret_cast<uint4*>(&Bs[p][r][q * 8]) =
                *reinterpret_cast<const uint4*>(B + p * pb + (n0 + r) * g.Kp + k0 + q * 8);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; kk += 16) {
            bf16x8 a[2][4], b[2][4], na[2][2];
            const int kl = kk + 8 * (lane >> 5);
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int r = wm * 64 + t * 32 + (lane & 31);
                const int cc = wn * 64 + t * 32 + (lane & 31);
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    a[t][p] = *reinterpret_cast<const bf16x8*>(&As[p][r][kl]);
                    b[t][p] = *reinterpret_cast<const bf16x8*>(&Bs[p][cc][kl]);
                }
                na[t][0] = negate(a[t][2]);
                na[t][1] = negate(a[t][3]);
            }
#pragma unroll
            for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                for (int tj = 0; tj < 2; ++tj) {
                    floatx16 r = accR[ti][tj], im = accI[ti][tj];
                    // re: Ar Br - Ai Bi
                    r = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[ti][0], b[tj][0], r, 0, 0, 0);
                    r = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[ti][0], b[tj][1], r, 0, 0, 0);
                    r = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[ti][1], b[tj][0], r, 0, 0, 0);
                    r = __builtin_amdgcn_mfma_f32_32x32x16_bf16(na[ti][0], b[tj][2], r, 0, 0, 0);
                    r = __builtin_amdgcn_mfma_f32_32x32x16_bf16(na[ti][0], b[tj][3], r, 0, 0, 0);
                    r = __builtin_amdgcn_mfma_f32_32x32x16_bf16(na[ti][1], b[tj][2], r, 0, 0, 0);
                    // im: Ar Bi + Ai Br
                    im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[ti][0], b[tj][2], im, 0, 0, 0);
                    im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[ti][0], b[tj][3], im, 0, 0, 0);
                    im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[ti][1], b[tj][2], im, 0, 0, 0);
                    im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[ti][2], b[tj][0], im, 0, 0, 0);
                    im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[ti][2], b[tj][1], im, 0, 0, 0);
                    im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[ti][3], b[tj][0], im, 0, 0, 0);
                    accR[ti][tj] = r;
                    accI[ti][tj] = im;
                }
        }
        __syncthreads();
    }
    float* C = Cbase + 2 * g.c_off;
    for (int ti = 0; ti < 2; ++ti)
        for (int tj = 0; tj < 2; ++tj)
            for (int e = 0; e < 16; ++e) {
                const int64_t row = m0 + wm * 64 + ti * 32 + (e >> 2) * 8 + (lane >> 5) * 4 + (e & 3);
                const int64_t col = n0 + wn * 64 + tj * 32 + (lane & 31);
                if (row < g.M && col < g.N) {
                    C[2 * (row + col * g.ldc)] = accR[ti][tj][e];
                    C[2 * (row + col * g.ldc) + 1] = accI[ti][tj][e];
                }
            }
}

// A planes of subdomain i.  mode 0 (operator): A[r][k] = K_i[r, k] (k < E), T_i[r, k - E]
// (E <= k < 2E); mode 1 (preconditioner): A[r][k] = (T_i^-1)[r, k] (k < E), passed as T.
// Zero in the padding.  64 x 64 tiles transposed through LDS: column-major reads and row-major
// writes both coalesced.
__global__ __launch_bounds__(256) void k_split_A(const GemmDesc* __restrict__ descs, const DomDesc* __restrict__ doms,
                                                 const int4* __restrict__ tiles, const float* __restrict__ T,
                                                 const float* __restrict__ K, uint16_t* __restrict__ Abase, int mode) {
    __shared__ float2 tile[64][65];
    const int4 tl = tiles[blockIdx.x];     // (dom, r0, k0)
    const GemmDesc g = descs[tl.x];
    const DomDesc dd = doms[tl.x];
    const int E = dd.E;
    const int r0 = tl.y, k0 = tl.z;
    const float2* T2 = reinterpret_cast<const float2*>(T) + dd.mat0;
    const float2* K2 = reinterpret_cast<const float2*>(K) + dd.mat0;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int rr = e & 63, kk = e >> 6;
        const int r = r0 + rr, k = k0 + kk;
        float2 v = make_float2(0.f, 0.f);
        if (mode == 0) {
            if (r < E && k < 2 * E) v = (k < E) ? K2[r + (int64_t)k * E] : T2[r + (int64_t)(k - E) * E];
        } else if (r < E && k < E) {
            v = T2[r + (int64_t)k * E];
        }
        tile[rr][kk] = v;
    }
    __syncthreads();
    uint16_t* A = Abase + g.a_off;
    const int64_t pa = g.Mp * g.Kp;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int kk = e & 63, rr = e >> 6;
        const int64_t r = r0 + rr, k = k0 + kk;
        if (r >= g.Mp || k >= g.Kp) continue;
        const float2 v = tile[rr][kk];
        uint16_t h, l;
        const int64_t idx = r * g.Kp + k;
        split(v.x, h, l);
        A[idx] = h;
        A[pa + idx] = l;
        split(v.y, h, l);
        A[2 * pa + idx] = h;
        A[3 * pa + idx] = l;
    }
}

// B planes of subdomain i for nrhs vectors x (complex128, column j at x + j*ld):
//   mode 0: column j : [2 x_iD ; 2/rho x_iN]    column nrhs + j : [2 x_iN ; -2 rho x_iD]
//   mode 1: column j : -x_iN / (2 rho)           column nrhs + j : rho/2 x_iD
__global__ __launch_bounds__(256) void k_split_B(const GemmDesc* __restrict__ descs, const DomDesc* __restrict__ doms,
                                                 int ndom, const double* __restrict__ x, int64_t ld, int nrhs,
                                                 uint16_t* __restrict__ Bbase, int mode) {
    const int dom = blockIdx.z;
    const GemmDesc g = descs[dom];
    const DomDesc dd = doms[dom];
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = blockIdx.y;
    if (k >= g.Kp || n >= g.Np) return;
    const int E = dd.E;
    double vr = 0.0, vi = 0.0;
    if (n < 2 * nrhs && k < (mode == 0 ? 2 * E : E)) {
        const int j = (int)(n % nrhs);
        const bool second = n >= nrhs;
        const double* xc = x + 2 * ((int64_t)j * ld + dd.off);
        double s;
        int64_t src;
        if (mode == 0) {
            if (!second) { if (k < E) { s = 2.0; src = k; } else { s = 2.0 / dd.rho; src = E + (k - E); } }
            else { if (k < E) { s = 2.0; src = E + k; } else { s = -2.0 * dd.rho; src = k - E; } }
        } else {
            if (!second) { s = -0.5 / dd.rho; src = E + k; }
            else { s = 0.5 * dd.rho; src = k; }
        }
        vr = s * xc[2 * src];
        vi = s * xc[2 * src + 1];
    }
    uint16_t* B = Bbase + g.b_off;
    const int64_t pb = g.Np * g.Kp;
    const int64_t idx = n * g.Kp + k;
    uint16_t h, l;
    split((float)vr, h, l);
    B[idx] = h;
    B[pb + idx] = l;
    split((float)vi, h, l);
    B[2 * pb + idx] = h;
    B[3 * pb + idx] = l;
}

// y = [C_D ; C_N] (+ transmission in mode 0), one thread per (dof, right-hand side).
__global__ __launch_bounds__(256) void k_gemm_finish(const DomDesc* __restrict__ doms, const GemmDesc* __restrict__ descs,
                                                     const int32_t* __restrict__ dof_dom, int64_t ndof,
                                                     const int32_t* __restrict__ dplus, const int32_t* __restrict__ dminus,
                                                     const double* __restrict__ gval, const int64_t* __restrict__ gcol,
                                                     const float* __restrict__ Cbase, const double* __restrict__ x,
                                                     double* __restrict__ y, int64_t ld, int nrhs, int mode) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (g >= ndof) return;
    const int dom = dof_dom[g];
    const DomDesc dd = doms[dom];
    const GemmDesc gd = descs[dom];
    const int64_t m = g - dd.dof0;
    const int E = dd.E;
    const float* C = Cbase + 2 * gd.c_off;
    double yD[2] = {C[2 * (m + (int64_t)j * gd.ldc)], C[2 * (m + (int64_t)j * gd.ldc) + 1]};
    double yN[2] = {C[2 * (m + (int64_t)(nrhs + j) * gd.ldc)], C[2 * (m + (int64_t)(nrhs + j) * gd.ldc) + 1]};
    const double* xj = x + 2 * (int64_t)j * ld;
    for (int side = 0; side < (mode == 0 ? 2 : 0); ++side) {
        const int32_t* pm = side == 0 ? dplus : dminus;
        const int64_t rec = dd.rec0 + pm[2 * g];
        const int a = pm[2 * g + 1];
        for (int c = 0; c < 3; ++c) {
            const double v = gval[9 * rec + 3 * a + c];
            const double* xd = xj + 2 * gcol[6 * rec + c];
            const double* xn = xj + 2 * gcol[6 * rec + 3 + c];
            yD[0] += v * xd[0]; yD[1] += v * xd[1];
            yN[0] += v * xn[0]; yN[1] += v * xn[1];
        }
    }
    double* yj = y + 2 * (int64_t)j * ld;
    yj[2 * (dd.off + m)] = yD[0];
    yj[2 * (dd.off + m) + 1] = yD[1];
    yj[2 * (dd.off + E + m)] = yN[0];
    yj[2 * (dd.off + E + m) + 1] = yN[1];
}

inline unsigned gridn(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

void launch_gemm_bf16x3(const GemmDesc* descs, const int4* tiles, int64_t ntiles, const uint16_t* A, const uint16_t* B,
                        float* C, hipStream_t s) {
    if (ntiles <= 0) return;
    hipLaunchKernelGGL(k_gemm_bf16x3, dim3((unsigned)ntiles), dim3(256), 0, s, descs, tiles, A, B, C);
}

void launch_split_A(const GemmDesc* descs, const DomDesc* doms, const int4* tiles, int64_t ntiles, const float* T,
                    const float* K, uint16_t* A, int mode, hipStream_t s) {
    if (ntiles <= 0) return;
    hipLaunchKernelGGL(k_split_A, dim3((unsigned)ntiles), dim3(256), 0, s, descs, doms, tiles, T, K, A, mode);
}

void launch_split_B(const GemmDesc* descs, const DomDesc* doms, int ndom, int64_t kp_max, int64_t np, const double* x,
                    int64_t ld, int nrhs, uint16_t* B, int mode, hipStream_t s) {
    hipLaunchKernelGGL(k_split_B, dim3(gridn(kp_max, 256), (unsigned)np, (unsigned)ndom), dim3(256), 0, s, descs, doms,
                       ndom, x, ld, nrhs, B, mode);
}

void launch_gemm_finish(const DomDesc* doms, const GemmDesc* descs, const int32_t* dof_dom, int64_t ndof,
                        const int32_t* dplus, const int32_t* dminus, const double* gval, const int64_t* gcol,
                        const float* C, const double* x, double* y, int64_t ld, int nrhs, int mode, hipStream_t s) {
    hipLaunchKernelGGL(k_gemm_finish, dim3(gridn(ndof, 256), (unsigned)nrhs), dim3(256), 0, s, doms, descs, dof_dom, ndof,
                       dplus, dminus, gval, gcol, C, x, y, ld, nrhs, mode);
}

}  // namespace mtf
