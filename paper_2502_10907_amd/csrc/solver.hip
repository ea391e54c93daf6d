// Solver kernels for gfx950: block MTF matvec, GMRES vector operations and the
// complex64 building blocks of the block T^-1 preconditioner.
//
// Block matvec (Problem 2, Section 3.2): for every subdomain i
//   y_iD =  2 K_i x_iD + 2/rho_i T_i x_iN + sum_j G^ij x_jD
//   y_iN = -2 rho_i T_i x_iD + 2 K_i x_iN + sum_j G^ij x_jN
// The dense part streams each T_i and K_i from HBM exactly once per product
// (coalesced columns, 64 consecutive rows per wavefront, 16-byte loads) and
// applies it to both x_iD and x_iN; column chunks give the grid enough
// workgroups, their partial sums are reduced in the finishing kernel that also
// applies the sparse transmission part (six terms per row).
#include "device.h"

#include <algorithm>

namespace mtf {

namespace {

constexpr int kChunk = 64;    // columns per dense-matvec workgroup (must match the host tiling)

template <typename RM>
struct C2 {
    RM re, im;
};

template <typename RM>
__global__ __launch_bounds__(256) void k_mv_dense(const DomDesc* __restrict__ doms, const int4* __restrict__ mtiles,
                                                  const RM* __restrict__ T, const RM* __restrict__ K,
                                                  const double* __restrict__ x, double* __restrict__ part) {
    const int4 t = mtiles[blockIdx.x];
    const DomDesc dd = doms[t.x];
    const int E = dd.E;
    const int c0 = t.z * kChunk;
    const int nc = min(kChunk, E - c0);
    __shared__ RM xs[kChunk][4];
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
        const double* xd = x + 2 * (dd.off + c0 + c);
        const double* xn = x + 2 * (dd.off + E + c0 + c);
        xs[c][0] = (RM)xd[0]; xs[c][1] = (RM)xd[1];
        xs[c][2] = (RM)xn[0]; xs[c][3] = (RM)xn[1];
    }
    __syncthreads();
    const int row = t.y + threadIdx.x;
    if (row >= E) return;
    RM tD[2] = {0, 0}, tN[2] = {0, 0}, kD[2] = {0, 0}, kN[2] = {0, 0};
    const C2<RM>* Tc = reinterpret_cast<const C2<RM>*>(T) + dd.mat0 + row + (int64_t)c0 * E;
    const C2<RM>* Kc = reinterpret_cast<const C2<RM>*>(K) + dd.mat0 + row + (int64_t)c0 * E;
#pragma unroll 4
    for (int c = 0; c < nc; ++c) {
        const C2<RM> a = Tc[(int64_t)c * E];
        const C2<RM> b = Kc[(int64_t)c * E];
        const RM xdr = xs[c][0], xdi = xs[c][1], xnr = xs[c][2], xni = xs[c][3];
        tD[0] += a.re * xdr - a.im * xdi; tD[1] += a.re * xdi + a.im * xdr;
        tN[0] += a.re * xnr - a.im * xni; tN[1] += a.re * xni + a.im * xnr;
        kD[0] += b.re * xdr - b.im * xdi; kD[1] += b.re * xdi + b.im * xdr;
        kN[0] += b.re * xnr - b.im * xni; kN[1] += b.re * xni + b.im * xnr;
    }
    const double rho = dd.rho;
    double* pD = part + 2 * (dd.part0 + (int64_t)(2 * t.z) * E + row);
    double* pN = part + 2 * (dd.part0 + (int64_t)(2 * t.z + 1) * E + row);
    pD[0] = 2.0 * (double)kD[0] + (2.0 / rho) * (double)tN[0];
    pD[1] = 2.0 * (double)kD[1] + (2.0 / rho) * (double)tN[1];
    pN[0] = -2.0 * rho * (double)tD[0] + 2.0 * (double)kN[0];
    pN[1] = -2.0 * rho * (double)tD[1] + 2.0 * (double)kN[1];
}

__global__ __launch_bounds__(256) void k_mv_finish(const DomDesc* __restrict__ doms, const int32_t* __restrict__ dof_dom,
                                                   int64_t ndof, const int32_t* __restrict__ dplus,
                                                   const int32_t* __restrict__ dminus, const double* __restrict__ gval,
                                                   const int64_t* __restrict__ gcol, const double* __restrict__ part,
                                                   const double* __restrict__ x, double* __restrict__ y) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ndof) return;
    const DomDesc dd = doms[dof_dom[g]];
    const int64_t m = g - dd.dof0;
    const int E = dd.E;
    double yD[2] = {0, 0}, yN[2] = {0, 0};
    for (int c = 0; c < dd.nchunk; ++c) {
        const double* pD = part + 2 * (dd.part0 + (int64_t)(2 * c) * E + m);
        const double* pN = part + 2 * (dd.part0 + (int64_t)(2 * c + 1) * E + m);
        yD[0] += pD[0]; yD[1] += pD[1];
        yN[0] += pN[0]; yN[1] += pN[1];
    }
    for (int side = 0; side < 2; ++side) {
        const int32_t* pm = side == 0 ? dplus : dminus;
        const int64_t rec = dd.rec0 + pm[2 * g];
        const int a = pm[2 * g + 1];
        for (int c = 0; c < 3; ++c) {
            const double v = gval[9 * rec + 3 * a + c];
            const double* xd = x + 2 * gcol[6 * rec + c];
            const double* xn = x + 2 * gcol[6 * rec + 3 + c];
            yD[0] += v * xd[0]; yD[1] += v * xd[1];
            yN[0] += v * xn[0]; yN[1] += v * xn[1];
        }
    }
    double* oD = y + 2 * (dd.off + m);
    double* oN = y + 2 * (dd.off + E + m);
    oD[0] = yD[0]; oD[1] = yD[1];
    oN[0] = yN[0]; oN[1] = yN[1];
}

// u = T^-1 x_N and v = T^-1 x_D per subdomain (complex64 matrix, FP32 accumulation).
__global__ __launch_bounds__(256) void k_pc_dense(const DomDesc* __restrict__ doms, const int4* __restrict__ mtiles,
                                                  const float* __restrict__ Ti, const double* __restrict__ x,
                                                  double* __restrict__ part) {
    const int4 t = mtiles[blockIdx.x];
    const DomDesc dd = doms[t.x];
    const int E = dd.E;
    const int c0 = t.z * kChunk;
    const int nc = min(kChunk, E - c0);
    __shared__ float xs[kChunk][4];
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
        const double* xd = x + 2 * (dd.off + c0 + c);
        const double* xn = x + 2 * (dd.off + E + c0 + c);
        xs[c][0] = (float)xd[0]; xs[c][1] = (float)xd[1];
        xs[c][2] = (float)xn[0]; xs[c][3] = (float)xn[1];
    }
    __syncthreads();
    const int row = t.y + threadIdx.x;
    if (row >= E) return;
    float aD[2] = {0, 0}, aN[2] = {0, 0};
    const C2<float>* Tc = reinterpret_cast<const C2<float>*>(Ti) + dd.mat0 + row + (int64_t)c0 * E;
#pragma unroll 4
    for (int c = 0; c < nc; ++c) {
        const C2<float> a = Tc[(int64_t)c * E];
        aD[0] += a.re * xs[c][0] - a.im * xs[c][1]; aD[1] += a.re * xs[c][1] + a.im * xs[c][0];
        aN[0] += a.re * xs[c][2] - a.im * xs[c][3]; aN[1] += a.re * xs[c][3] + a.im * xs[c][2];
    }
    double* pD = part + 2 * (dd.part0 + (int64_t)(2 * t.z) * E + row);
    double* pN = part + 2 * (dd.part0 + (int64_t)(2 * t.z + 1) * E + row);
    pD[0] = aD[0]; pD[1] = aD[1];
    pN[0] = aN[0]; pN[1] = aN[1];
}

// z_iD = -1/(2 rho) T^-1 x_iN,  z_iN = rho/2 T^-1 x_iD  (all dofs, or the dofs of `list`)
__global__ __launch_bounds__(256) void k_pc_finish(const DomDesc* __restrict__ doms, const int32_t* __restrict__ dof_dom,
                                                   int64_t ndof, const double* __restrict__ part, double* __restrict__ z,
                                                   const int32_t* __restrict__ list) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ndof) return;
    const int64_t g = list ? list[t] : t;
    const DomDesc dd = doms[dof_dom[g]];
    const int64_t m = g - dd.dof0;
    const int E = dd.E;
    double vD[2] = {0, 0}, vN[2] = {0, 0};
    for (int c = 0; c < dd.nchunk; ++c) {
        const double* pD = part + 2 * (dd.part0 + (int64_t)(2 * c) * E + m);
        const double* pN = part + 2 * (dd.part0 + (int64_t)(2 * c + 1) * E + m);
        vD[0] += pD[0]; vD[1] += pD[1];
        vN[0] += pN[0]; vN[1] += pN[1];
    }
    const double a = -0.5 / dd.rho, b = 0.5 * dd.rho;
    double* oD = z + 2 * (dd.off + m);
    double* oN = z + 2 * (dd.off + E + m);
    oD[0] = a * vN[0]; oD[1] = a * vN[1];
    oN[0] = b * vD[0]; oN[1] = b * vD[1];
}

// Block Gauss-Seidel stage input: w_i = v_i - sum_j G^ij z_j for the dofs of one stage (z holds
// the already computed stages, zero elsewhere).
__global__ __launch_bounds__(256) void k_gs_residual(const DomDesc* __restrict__ doms, const int32_t* __restrict__ dof_dom,
                                                     const int32_t* __restrict__ list, int64_t nlist,
                                                     const int32_t* __restrict__ dplus, const int32_t* __restrict__ dminus,
                                                     const double* __restrict__ gval, const int64_t* __restrict__ gcol,
                                                     const double* __restrict__ v, const double* __restrict__ z,
                                                     double* __restrict__ w) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nlist) return;
    const int64_t g = list[t];
    const DomDesc dd = doms[dof_dom[g]];
    const int64_t m = g - dd.dof0;
    const int64_t iD = dd.off + m, iN = dd.off + dd.E + m;
    double yD[2] = {v[2 * iD], v[2 * iD + 1]}, yN[2] = {v[2 * iN], v[2 * iN + 1]};
    for (int side = 0; side < 2; ++side) {
        const int32_t* pm = side == 0 ? dplus : dminus;
        const int64_t rec = dd.rec0 + pm[2 * g];
        const int a = pm[2 * g + 1];
        for (int c = 0; c < 3; ++c) {
            const double gv = gval[9 * rec + 3 * a + c];
            const double* zd = z + 2 * gcol[6 * rec + c];
            const double* zn = z + 2 * gcol[6 * rec + 3 + c];
            yD[0] -= gv * zd[0]; yD[1] -= gv * zd[1];
            yN[0] -= gv * zn[0]; yN[1] -= gv * zn[1];
        }
    }
    w[2 * iD] = yD[0]; w[2 * iD + 1] = yD[1];
    w[2 * iN] = yN[0]; w[2 * iN + 1] = yN[1];
}

// ---------------------------------------------------------------------------
// GMRES vector kernels (complex128)
// ---------------------------------------------------------------------------

__device__ inline double wsum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Batched Arnoldi kernels.  nb right-hand sides advance in lockstep: Krylov block j is an
// n x nb column-major slab at V + j*ldv (ldv = nb*n), column b of every slab belongs to
// right-hand side b (gridDim.z or blockIdx.z = b).  Per right-hand side b:
//   hpart[(b*(nvmax+1) + i) * nblk + blk]  partial dots,   h[b*(nvmax+1) + i]  reduced dots,
//   H + b*hstride + column j               Hessenberg column,   wn2[b], flag[b], npart[b*nblk + k].

// conj(V_i) . w for i < nv (and w . w in slot nv when `self`); skipped where flag[b] == 0.
__global__ __launch_bounds__(256) void k_multidot(const double* __restrict__ V, int64_t ldv, int nv, int nvmax,
                                                  const double* __restrict__ W, int64_t n, double* __restrict__ hpart,
                                                  int nblk, const int* __restrict__ flag) {
    const int b = blockIdx.z;
    if (flag && flag[b] == 0) return;
    const int i = blockIdx.y;
    const int blk = blockIdx.x;
    const int64_t chunk = (n + nblk - 1) / nblk;
    const int64_t lo = blk * chunk, hi = min(n, lo + chunk);
    const double* w = W + 2 * (int64_t)b * n;
    const double* v = (i == nv) ? w : V + 2 * ((int64_t)i * ldv + (int64_t)b * n);
    double re = 0, im = 0;
    for (int64_t e = lo + threadIdx.x; e < hi; e += blockDim.x) {
        const double vr = v[2 * e], vi = v[2 * e + 1], wr = w[2 * e], wi = w[2 * e + 1];
        re += vr * wr + vi * wi;
        im += vr * wi - vi * wr;
    }
    __shared__ double red[2][4];
    re = wsum(re);
    im = wsum(im);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) { red[0][wv] = re; red[1][wv] = im; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0, c = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) { a += red[0][k]; c += red[1][k]; }
        const int64_t slot = ((int64_t)b * (nvmax + 1) + i) * nblk + blk;
        hpart[2 * slot] = a;
        hpart[2 * slot + 1] = c;
    }
}

__global__ void k_reduce_h(const double* __restrict__ hpart, int nv, int nvmax, int nblk, double* __restrict__ h,
                           double* __restrict__ Hcol, int64_t hstride, double* __restrict__ wn2, int second,
                           const int* __restrict__ flag) {
    const int b = blockIdx.y;
    if (flag && flag[b] == 0) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int top = second ? nv : nv + 1;
    if (i >= top) return;
    double a = 0, c = 0;
    const int64_t base = ((int64_t)b * (nvmax + 1) + i) * nblk;
    for (int k = 0; k < nblk; ++k) { a += hpart[2 * (base + k)]; c += hpart[2 * (base + k) + 1]; }
    if (i == nv) { wn2[b] = a; return; }
    double* hb = h + 2 * ((int64_t)b * (nvmax + 1));
    double* Hb = Hcol + 2 * (int64_t)b * hstride;
    hb[2 * i] = a;
    hb[2 * i + 1] = c;
    if (second) { Hb[2 * i] += a; Hb[2 * i + 1] += c; }
    else { Hb[2 * i] = a; Hb[2 * i + 1] = c; }
}

// Second Gram-Schmidt pass only when the first lost too much: ||w'||^2 < ||w||^2 / 2 (DGKS test).
__global__ void k_reorth_flag(const double* __restrict__ wn2, const double* __restrict__ part, int nblk, int nb,
                              int* __restrict__ flag, int* __restrict__ count) {
    const int b = threadIdx.x;
    if (b >= nb) return;
    double s = 0;
    for (int k = 0; k < nblk; ++k) s += part[(int64_t)b * nblk + k];
    const int f = s < 0.5 * wn2[b] ? 1 : 0;
    flag[b] = f;
    count[b] += f;
}

// part[(b*nch + c)][e] = sum_{i in vector chunk c} V_i[e] h[i]   (64 vectors per chunk)
__global__ __launch_bounds__(256) void k_update_part(const double* __restrict__ V, int64_t ldv, int nv, int nvmax,
                                                     const double* __restrict__ h, double* __restrict__ part,
                                                     int64_t n, const int* __restrict__ flag) {
    const int b = blockIdx.z;
    if (flag && flag[b] == 0) return;
    __shared__ double hs[2 * 64];
    const int c = blockIdx.y;
    const int nch = gridDim.y;
    const int i0 = c * 64;
    const int cnt = min(64, nv - i0);
    const double* hb = h + 2 * ((int64_t)b * (nvmax + 1));
    if ((int)threadIdx.x < cnt) { hs[2 * threadIdx.x] = hb[2 * (i0 + threadIdx.x)]; hs[2 * threadIdx.x + 1] = hb[2 * (i0 + threadIdx.x) + 1]; }
    __syncthreads();
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    double re = 0, im = 0;
    const double* v = V + 2 * ((int64_t)i0 * ldv + (int64_t)b * n + e);
    int i = 0;
    for (; i + 8 <= cnt; i += 8) {
        double vr[8], vi[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) { vr[u] = v[2 * (int64_t)(i + u) * ldv]; vi[u] = v[2 * (int64_t)(i + u) * ldv + 1]; }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double hr = hs[2 * (i + u)], hi = hs[2 * (i + u) + 1];
            re += vr[u] * hr - vi[u] * hi;
            im += vr[u] * hi + vi[u] * hr;
        }
    }
    for (; i < cnt; ++i) {
        const double vr = v[2 * (int64_t)i * ldv], vi = v[2 * (int64_t)i * ldv + 1];
        const double hr = hs[2 * i], hi = hs[2 * i + 1];
        re += vr * hr - vi * hi;
        im += vr * hi + vi * hr;
    }
    const int64_t slot = ((int64_t)b * nch + c) * n + e;
    part[2 * slot] = re;
    part[2 * slot + 1] = im;
}

__global__ __launch_bounds__(256) void k_update_apply(const double* __restrict__ part, int nchunk, double* __restrict__ W,
                                                      int64_t n, const int* __restrict__ flag) {
    const int b = blockIdx.y;
    if (flag && flag[b] == 0) return;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    double re = 0, im = 0;
    for (int c = 0; c < nchunk; ++c) {
        const int64_t slot = ((int64_t)b * nchunk + c) * n + e;
        re += part[2 * slot];
        im += part[2 * slot + 1];
    }
    double* w = W + 2 * (int64_t)b * n;
    w[2 * e] -= re;
    w[2 * e + 1] -= im;
}

// x_b += V_b coef_b over the first cnt[b] vectors (column b of each slab)
__global__ __launch_bounds__(256) void k_combine(double* __restrict__ X, int64_t ldx, const double* __restrict__ V,
                                                 int64_t ldv, const int* __restrict__ cnt, int nvmax,
                                                 const double* __restrict__ coef, int64_t n) {
    const int b = blockIdx.y;
    __shared__ double hs[2 * 256];
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int nv = cnt[b];
    const double* cb = coef + 2 * ((int64_t)b * (nvmax + 1));
    double re = 0, im = 0;
    for (int i0 = 0; i0 < nv; i0 += 256) {
        const int m = min(256, nv - i0);
        __syncthreads();
        if ((int)threadIdx.x < m) { hs[2 * threadIdx.x] = cb[2 * (i0 + threadIdx.x)]; hs[2 * threadIdx.x + 1] = cb[2 * (i0 + threadIdx.x) + 1]; }
        __syncthreads();
        if (e < n) {
            for (int i = 0; i < m; ++i) {
                const double* v = V + 2 * ((int64_t)(i0 + i) * ldv + (int64_t)b * n + e);
                re += v[0] * hs[2 * i] - v[1] * hs[2 * i + 1];
                im += v[0] * hs[2 * i + 1] + v[1] * hs[2 * i];
            }
        }
    }
    if (e < n) { X[2 * ((int64_t)b * ldx + e)] += re; X[2 * ((int64_t)b * ldx + e) + 1] += im; }
}

// part[b*nblk + blk] = sum |w_b|^2 over chunk blk
__global__ __launch_bounds__(256) void k_norm2(const double* __restrict__ W, int64_t ldw, int64_t n, double* __restrict__ part,
                                               int nblk) {
    const int b = blockIdx.y;
    const double* w = W + 2 * (int64_t)b * ldw;
    const int64_t chunk = (n + nblk - 1) / nblk;
    const int64_t lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
    double s = 0;
    for (int64_t e = lo + threadIdx.x; e < hi; e += blockDim.x) s += w[2 * e] * w[2 * e] + w[2 * e + 1] * w[2 * e + 1];
    __shared__ double red[4];
    s = wsum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) a += red[k];
        part[(int64_t)b * nblk + blockIdx.x] = a;
    }
}

__global__ void k_axpby(double* __restrict__ y, const double* __restrict__ x, int64_t n, double ar, double ai, double b) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const double xr = x[2 * e], xi = x[2 * e + 1];
    y[2 * e] = b * y[2 * e] + ar * xr - ai * xi;
    y[2 * e + 1] = b * y[2 * e + 1] + ar * xi + ai * xr;
}

// y_b = x_b / ||x_b|| (norm from the partial sums; 0 stays 0); hsub + b*hstride receives the norm.
__global__ void k_scale_dev(double* __restrict__ Y, const double* __restrict__ X, int64_t ld, int64_t n,
                            const double* __restrict__ part, int nblk, double* __restrict__ hsub, int64_t hstride) {
    const int b = blockIdx.y;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0;
    for (int k = 0; k < nblk; ++k) s += part[(int64_t)b * nblk + k];
    const double nrm = sqrt(s);
    if (e == 0 && hsub) { hsub[2 * (int64_t)b * hstride] = nrm; hsub[2 * (int64_t)b * hstride + 1] = 0.0; }
    if (e >= n) return;
    const double inv = nrm > 0 ? 1.0 / nrm : 0.0;
    Y[2 * ((int64_t)b * ld + e)] = X[2 * ((int64_t)b * ld + e)] * inv;
    Y[2 * ((int64_t)b * ld + e) + 1] = X[2 * ((int64_t)b * ld + e) + 1] * inv;
}

// ---------------------------------------------------------------------------
// complex64 GEMM: D = alpha A B + beta C (column-major; C may alias D)
// 64 x 64 tile per workgroup, 4 x 4 complex outputs per thread, k-step 8.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_cgemm(int m, int n, int k, float ar, float ai, const float* __restrict__ A,
                                               int64_t lda, const float* __restrict__ B, int64_t ldb, float beta,
                                               const float* C, int64_t ldc, float* D, int64_t ldd) {
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
            const int r = e & 63, kk = e >> 6;
            const int gr = row0 + r, gk = k0 + kk;
            As[kk][r] = (gr < m && gk < k) ? A2[gr + (int64_t)gk * lda] : make_float2(0.f, 0.f);
            const int kb = e & 7, cc = e >> 3;
            const int gkb = k0 + kb, gc = col0 + cc;
            Bs[kb][cc] = (gkb < k && gc < n) ? B2[gkb + (int64_t)gc * ldb] : make_float2(0.f, 0.f);
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
            float re = ar * acc[i][j][0] - ai * acc[i][j][1];
            float im = ar * acc[i][j][1] + ai * acc[i][j][0];
            if (beta != 0.f) {
                const float* c = C + 2 * (gr + (int64_t)gc * ldc);
                re += beta * c[0];
                im += beta * c[1];
            }
            float* d = D + 2 * (gr + (int64_t)gc * ldd);
            d[0] = re;
            d[1] = im;
        }
    }
}

// In-place inverse of an n x n (n <= 64) complex64 block by Gauss-Jordan elimination
// with partial pivoting; one workgroup, the block held in LDS.
__global__ __launch_bounds__(256) void k_cinv_small(float* A, int64_t lda, int n, int* info) {
    __shared__ float2 M[64][65];
    __shared__ int piv[64];
    __shared__ float2 pvt;
    __shared__ float2 colk[64];
    const int tid = threadIdx.x;
    float2* A2 = reinterpret_cast<float2*>(A);
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int r = e % n, c = e / n;
        M[r][c] = A2[r + (int64_t)c * lda];
    }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        if (tid == 0) {
            int p = k;
            float best = -1.f;
            for (int i = k; i < n; ++i) {
                const float v = M[i][k].x * M[i][k].x + M[i][k].y * M[i][k].y;
                if (v > best) { best = v; p = i; }
            }
            piv[k] = p;
            if (!(best > 0.f)) info[0] = k + 1;
        }
        __syncthreads();
        const int p = piv[k];
        if (p != k) {
            for (int c = tid; c < n; c += blockDim.x) {
                const float2 t = M[k][c];
                M[k][c] = M[p][c];
                M[p][c] = t;
            }
        }
        __syncthreads();
        if (tid == 0) {
            const float2 a = M[k][k];
            const float den = a.x * a.x + a.y * a.y;
            pvt = make_float2(a.x / den, -a.y / den);   // 1 / a
            M[k][k] = make_float2(1.f, 0.f);
        }
        __syncthreads();
        for (int c = tid; c < n; c += blockDim.x) {
            const float2 v = M[k][c];
            M[k][c] = make_float2(v.x * pvt.x - v.y * pvt.y, v.x * pvt.y + v.y * pvt.x);
        }
        __syncthreads();
        for (int i = tid; i < n; i += blockDim.x) {
            colk[i] = M[i][k];
        }
        __syncthreads();
        for (int i = tid; i < n; i += blockDim.x) {
            if (i != k) M[i][k] = make_float2(0.f, 0.f);
        }
        __syncthreads();
        for (int e = tid; e < n * n; e += blockDim.x) {
            const int i = e % n, c = e / n;
            if (i == k) continue;
            const float2 f = colk[i];
            const float2 r = M[k][c];
            M[i][c].x -= f.x * r.x - f.y * r.y;
            M[i][c].y -= f.x * r.y + f.y * r.x;
        }
        __syncthreads();
    }
    // undo the row interchanges as column interchanges, last first
    for (int k = n - 1; k >= 0; --k) {
        const int p = piv[k];
        if (p != k) {
            for (int r = tid; r < n; r += blockDim.x) {
                const float2 t = M[r][k];
                M[r][k] = M[r][p];
                M[r][p] = t;
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int r = e % n, c = e / n;
        A2[r + (int64_t)c * lda] = M[r][c];
    }
}

__global__ void k_copy_d2f(const double* __restrict__ s, float* __restrict__ d, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) d[e] = (float)s[e];
}

__global__ void k_nonfinite(const float* __restrict__ a, int64_t n, int* flag) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n && !isfinite(a[e])) atomicOr(flag, 1);
}

inline unsigned gridn(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

void launch_matvec_dense_f64(const DomDesc* doms, const int4* mtiles, int64_t nmt, const double* T, const double* K,
                             const double* x, double* part, hipStream_t s) {
    hipLaunchKernelGGL(k_mv_dense<double>, dim3((unsigned)nmt), dim3(256), 0, s, doms, mtiles, T, K, x, part);
}

void launch_matvec_dense_f32(const DomDesc* doms, const int4* mtiles, int64_t nmt, const float* T, const float* K,
                             const double* x, double* part, hipStream_t s) {
    hipLaunchKernelGGL(k_mv_dense<float>, dim3((unsigned)nmt), dim3(256), 0, s, doms, mtiles, T, K, x, part);
}

void launch_matvec_finish(const DomDesc* doms, int /*ndom*/, const int32_t* dof_dom, int64_t ndof, const int32_t* dplus,
                          const int32_t* dminus, const double* gval, const int64_t* gcol, const double* part,
                          const double* x, double* y, hipStream_t s) {
    hipLaunchKernelGGL(k_mv_finish, dim3(gridn(ndof, 256)), dim3(256), 0, s, doms, dof_dom, ndof, dplus, dminus, gval,
                       gcol, part, x, y);
}

void launch_precond_apply(const DomDesc* doms, const int4* mtiles, int64_t nmt, const float* Tinv, const double* x,
                          double* part, hipStream_t s) {
    if (nmt <= 0) return;
    hipLaunchKernelGGL(k_pc_dense, dim3((unsigned)nmt), dim3(256), 0, s, doms, mtiles, Tinv, x, part);
}

void launch_precond_finish(const DomDesc* doms, int /*ndom*/, const int32_t* dof_dom, int64_t ndof, const double* part,
                           double* z, hipStream_t s, const int32_t* list) {
    if (ndof <= 0) return;
    hipLaunchKernelGGL(k_pc_finish, dim3(gridn(ndof, 256)), dim3(256), 0, s, doms, dof_dom, ndof, part, z, list);
}

void launch_gs_residual(const DomDesc* doms, const int32_t* dof_dom, const int32_t* list, int64_t nlist,
                        const int32_t* dplus, const int32_t* dminus, const double* gval, const int64_t* gcol,
                        const double* v, const double* z, double* w, hipStream_t s) {
    if (nlist <= 0) return;
    hipLaunchKernelGGL(k_gs_residual, dim3(gridn(nlist, 256)), dim3(256), 0, s, doms, dof_dom, list, nlist, dplus, dminus,
                       gval, gcol, v, z, w);
}

void launch_multidot(const double* V, int64_t ldv, int nv, int nvmax, const double* w, int64_t n, double* hpart,
                     int nblk, int self, const int* flag, int nb, hipStream_t s) {
    hipLaunchKernelGGL(k_multidot, dim3((unsigned)nblk, (unsigned)(nv + (self ? 1 : 0)), (unsigned)nb), dim3(256), 0, s,
                       V, ldv, nv, nvmax, w, n, hpart, nblk, flag);
}

void launch_reduce_h(const double* hpart, int nv, int nvmax, int nblk, double* h, double* Hcol, int64_t hstride,
                     double* wn2, int second, const int* flag, int nb, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_h, dim3(gridn(nv + 1, 128), (unsigned)nb), dim3(128), 0, s, hpart, nv, nvmax, nblk, h,
                       Hcol, hstride, wn2, second, flag);
}

void launch_reorth_flag(const double* wn2, const double* part, int nblk, int nb, int* flag, int* count, hipStream_t s) {
    hipLaunchKernelGGL(k_reorth_flag, dim3(1), dim3(256), 0, s, wn2, part, nblk, nb, flag, count);
}

void launch_update(const double* V, int64_t ldv, int nv, int nvmax, const double* h, double* w, int64_t n,
                   double* part, const int* flag, int nb, hipStream_t s) {
    const int nchunk = (nv + 63) / 64;
    hipLaunchKernelGGL(k_update_part, dim3(gridn(n, 256), (unsigned)nchunk, (unsigned)nb), dim3(256), 0, s, V, ldv, nv,
                       nvmax, h, part, n, flag);
    hipLaunchKernelGGL(k_update_apply, dim3(gridn(n, 256), (unsigned)nb), dim3(256), 0, s, part, nchunk, w, n, flag);
}

void launch_combine(double* x, int64_t ldx, const double* V, int64_t ldv, const int* cnt, int nvmax, const double* coef,
                    int64_t n, int nb, hipStream_t s) {
    hipLaunchKernelGGL(k_combine, dim3(gridn(n, 256), (unsigned)nb), dim3(256), 0, s, x, ldx, V, ldv, cnt, nvmax, coef, n);
}

void launch_norm2(const double* w, int64_t ldw, int64_t n, double* part, int nblk, int nb, hipStream_t s) {
    hipLaunchKernelGGL(k_norm2, dim3((unsigned)nblk, (unsigned)nb), dim3(256), 0, s, w, ldw, n, part, nblk);
}

void launch_axpby(double* y, const double* x, int64_t n, double ar, double ai, double b, hipStream_t s) {
    hipLaunchKernelGGL(k_axpby, dim3(gridn(n, 256)), dim3(256), 0, s, y, x, n, ar, ai, b);
}

void launch_scale_dev(double* y, const double* x, int64_t ld, int64_t n, const double* part, int nblk, double* hsub,
                      int64_t hstride, int nb, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_dev, dim3(gridn(n, 256), (unsigned)nb), dim3(256), 0, s, y, x, ld, n, part, nblk, hsub,
                       hstride);
}

void launch_copy_block_f64_to_f32(const double* src, float* dst, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_d2f, dim3(gridn(n, 256)), dim3(256), 0, s, src, dst, n);
}

void launch_cgemm_f32(int m, int n, int k, float ar, float ai, const float* A, int64_t lda, const float* B, int64_t ldb,
                      float beta, const float* C, int64_t ldc, float* D, int64_t ldd, hipStream_t s) {
    if (m <= 0 || n <= 0) return;
    hipLaunchKernelGGL(k_cgemm, dim3(gridn(m, 64), gridn(n, 64)), dim3(256), 0, s, m, n, k, ar, ai, A, lda, B, ldb,
                       beta, C, ldc, D, ldd);
}

int launch_cinv_small_f32(float* A, int64_t lda, int n, int* info, hipStream_t s) {
    if (n <= 0 || n > 64) return -1;
    hipLaunchKernelGGL(k_cinv_small, dim3(1), dim3(256), 0, s, A, lda, n, info);
    return 0;
}

void launch_nonfinite_check(const float* A, int64_t n, int* flag, hipStream_t s) {
    hipLaunchKernelGGL(k_nonfinite, dim3(gridn(n, 256)), dim3(256), 0, s, A, n, flag);
}

}  // namespace mtf
