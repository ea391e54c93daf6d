// Block Krylov kernels (gfx950): the dense FP64 contractions of block GMRES on the matrix cores.
//
// A block of p Krylov vectors against a basis of j vectors (complex128, each vector contiguous)
// is orthogonalised by classical Gram-Schmidt in block form:
//     H = V^H W          (j x p, one pass over the basis)           k_bdot + k_bdot_reduce
//     W <- W - V H       (N x p, one pass over the basis)           k_bupd + k_bupd_finish
// Both are GEMMs with one very long dimension (N) and p <= 32, so the basis is read once per pass
// and the arithmetic (8 p flops per complex basis entry) runs on v_mfma_f64_16x16x4f64; with p = 16
// the MFMA rate needed to keep pace with HBM is about half of the FP64 matrix peak.  The same
// update kernel forms linear combinations elsewhere (X += Z Y, V_{k+1} = W T).
//
// v_mfma_f64_16x16x4f64 lane layout (one wavefront, checked on the device): A[r][k] in lane
// r + 16 k, B[k][c] in lane c + 16 k, D[r][c] in lane c + 16 (r % 4), element r / 4 of the four
// accumulator doubles.
// The summation index only has to agree between A and B, so each lane feeds its k-slot with
// four consecutive unknowns (one 64-byte load per lane instead of four 16-byte ones).

#include "device.h"

namespace mtf {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// part[chunk][i][c] = sum over n in the chunk of conj(V_i[n]) W_c[n], i < j, c < p.
// One wavefront per (64 basis vectors, chunk of nc unknowns, 16 columns); nc is a multiple of 16.
__global__ __launch_bounds__(64) void k_bdot(const double2* __restrict__ V, int64_t ldv, int j,
                                             const double2* __restrict__ W, int64_t ldw, int p, int64_t n,
                                             int64_t nc, double2* __restrict__ part, int ppad) {
    const int lane = threadIdx.x;
    const int r = lane & 15, ks = lane >> 4;
    const int i0 = blockIdx.x * 64;
    const int col = blockIdx.z * 16 + r;
    const int64_t nb = (int64_t)blockIdx.y * nc;
    const int64_t ne = nb + nc < n ? nb + nc : n;
    const double2* vp[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int i = i0 + 16 * b + r;
        vp[b] = V + (int64_t)(i < j ? i : j - 1) * ldv;     // rows past j are computed, never stored
    }
    const double2* wp = W + (int64_t)(col < p ? col : p - 1) * ldw;
    d4 accr[4], acci[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        accr[b] = d4{0.0, 0.0, 0.0, 0.0};
        acci[b] = d4{0.0, 0.0, 0.0, 0.0};
    }
    for (int64_t n0 = nb; n0 < ne; n0 += 16) {
        const int64_t nn = n0 + 4 * ks;
        double2 w[4], v[4][4];
        if (nn + 4 <= ne) {
#pragma unroll
            for (int t = 0; t < 4; ++t) w[t] = wp[nn + t];
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int t = 0; t < 4; ++t) v[b][t] = vp[b][nn + t];
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const bool ok = nn + t < ne;
                w[t] = ok ? wp[nn + t] : make_double2(0.0, 0.0);
#pragma unroll
                for (int b = 0; b < 4; ++b) v[b][t] = ok ? vp[b][nn + t] : make_double2(0.0, 0.0);
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                // conj(v) w = (vr wr + vi wi) + i (vr wi - vi wr)
                accr[b] = mfma(v[b][t].x, w[t].x, accr[b]);
                accr[b] = mfma(v[b][t].y, w[t].y, accr[b]);
                acci[b] = mfma(v[b][t].x, w[t].y, acci[b]);
                acci[b] = mfma(-v[b][t].y, w[t].x, acci[b]);
            }
    }
    if (col >= p) return;
    double2* out = part + (int64_t)blockIdx.y * j * ppad;
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = i0 + 16 * b + 4 * q + ks;
            if (i < j) out[(int64_t)i * ppad + col] = make_double2(accr[b][q], acci[b][q]);
        }
}

// H[i * hld + c] = sum over chunks of part[chunk][i][c]  (i < j, c < p)
__global__ __launch_bounds__(256) void k_bdot_reduce(const double2* __restrict__ part, int nchunk, int j, int p,
                                                     int ppad, double2* __restrict__ H, int hld) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)j * ppad) return;
    const int c = (int)(e % ppad);
    if (c >= p) return;
    double sr = 0.0, si = 0.0;
    for (int k = 0; k < nchunk; ++k) {
        const double2 v = part[(int64_t)k * j * ppad + e];
        sr += v.x;
        si += v.y;
    }
    H[(e / ppad) * hld + c] = make_double2(sr, si);
}

// part[s][c][n] = sum over i in split s of V_i[n] H(i, c), H(i, c) at H[i * hs_i + c * hs_c].
// One wavefront per (64 unknowns, split of ks basis vectors, 16 columns); ks is a multiple of 4.
__global__ __launch_bounds__(64) void k_bupd(const double2* __restrict__ V, int64_t ldv, int j, int ksplit,
                                             const double2* __restrict__ H, int64_t hs_i, int64_t hs_c, int p,
                                             int64_t n, double2* __restrict__ part, int ppad) {
    const int lane = threadIdx.x;
    const int r = lane & 15, ks = lane >> 4;
    const int64_t n0 = (int64_t)blockIdx.x * 64;
    const int col = blockIdx.z * 16 + r;
    const int ib = blockIdx.y * ksplit;
    const int ie = ib + ksplit < j ? ib + ksplit : j;
    int64_t nrow[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int64_t nn = n0 + 16 * b + r;
        nrow[b] = nn < n ? nn : n - 1;                       // rows past n are computed, never stored
    }
    const int cc = col < p ? col : p - 1;
    d4 accr[4], acci[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        accr[b] = d4{0.0, 0.0, 0.0, 0.0};
        acci[b] = d4{0.0, 0.0, 0.0, 0.0};
    }
    for (int i = ib; i < ie; i += 4) {
        const int ii = i + ks;
        const bool ok = ii < ie && col < p;
        const int ic = ii < ie ? ii : ie - 1;
        double2 h = H[(int64_t)ic * hs_i + (int64_t)cc * hs_c];
        if (!ok) h = make_double2(0.0, 0.0);
        const double2* vrow = V + (int64_t)ic * ldv;
        double2 v[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) v[b] = vrow[nrow[b]];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            // v h = (vr hr - vi hi) + i (vr hi + vi hr)
            accr[b] = mfma(v[b].x, h.x, accr[b]);
            accr[b] = mfma(-v[b].y, h.y, accr[b]);
            acci[b] = mfma(v[b].x, h.y, acci[b]);
            acci[b] = mfma(v[b].y, h.x, acci[b]);
        }
    }
    if (col >= p) return;
    double2* out = part + ((int64_t)blockIdx.y * ppad + col) * n;
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t nn = n0 + 16 * b + 4 * q + ks;
            if (nn < n) out[nn] = make_double2(accr[b][q], acci[b][q]);
        }
}

// Y_c[n] = beta Yin_c[n] + alpha sum_s part[s][c][n]   (c < p, n < N; Y may alias Yin)
__global__ __launch_bounds__(256) void k_bupd_finish(const double2* __restrict__ part, int nsplit, int ppad, int p,
                                                     int64_t n, const double2* Yin, int64_t ldyin, double2* Y,
                                                     int64_t ldy, double alpha, double beta) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (e >= n || c >= p) return;
    double sr = 0.0, si = 0.0;
    for (int s = 0; s < nsplit; ++s) {
        const double2 v = part[((int64_t)s * ppad + c) * n + e];
        sr += v.x;
        si += v.y;
    }
    double2 y = make_double2(alpha * sr, alpha * si);
    if (beta != 0.0) {
        const double2 yi = Yin[(int64_t)c * ldyin + e];
        y.x += beta * yi.x;
        y.y += beta * yi.y;
    }
    Y[(int64_t)c * ldy + e] = y;
}

inline unsigned gridn(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

BlockDotPlan plan_bdot(int64_t n, int j, int p) {
    BlockDotPlan pl;
    pl.itiles = (j + 63) / 64;
    pl.ctiles = (p + 15) / 16;
    pl.ppad = 16 * pl.ctiles;
    int64_t want = (2048 + pl.itiles * pl.ctiles - 1) / (pl.itiles * pl.ctiles);
    const int64_t most = (n + 255) / 256;
    if (want > most) want = most;
    if (want < 1) want = 1;
    int64_t nc = (n + want - 1) / want;
    nc = ((nc + 15) / 16) * 16;
    pl.nc = nc;
    pl.nchunk = (int)((n + nc - 1) / nc);
    pl.part_elems = (int64_t)pl.nchunk * j * pl.ppad;
    return pl;
}

BlockUpdPlan plan_bupd(int64_t n, int j, int p) {
    BlockUpdPlan pl;
    pl.ntile = (n + 63) / 64;
    pl.ctiles = (p + 15) / 16;
    pl.ppad = 16 * pl.ctiles;
    const int64_t tiles = pl.ntile * pl.ctiles;
    int64_t want = (4096 + tiles - 1) / tiles;
    const int64_t most = (j + 63) / 64;
    if (want > most) want = most;
    if (want < 1) want = 1;
    int ks = (int)((j + want - 1) / want);
    ks = ((ks + 3) / 4) * 4;
    pl.ksplit = ks;
    pl.nsplit = (j + ks - 1) / ks;
    pl.part_elems = (int64_t)pl.nsplit * pl.ppad * n;
    return pl;
}

void launch_bdot(const BlockDotPlan& pl, const double* V, int64_t ldv, int j, const double* W, int64_t ldw, int p,
                 int64_t n, double* part, double* H, int hld, hipStream_t s) {
    if (j <= 0 || p <= 0 || n <= 0) return;
    hipLaunchKernelGGL(k_bdot, dim3((unsigned)pl.itiles, (unsigned)pl.nchunk, (unsigned)pl.ctiles), dim3(64), 0, s,
                       reinterpret_cast<const double2*>(V), ldv, j, reinterpret_cast<const double2*>(W), ldw, p, n,
                       pl.nc, reinterpret_cast<double2*>(part), pl.ppad);
    hipLaunchKernelGGL(k_bdot_reduce, dim3(gridn((int64_t)j * pl.ppad, 256)), dim3(256), 0, s,
                       reinterpret_cast<const double2*>(part), pl.nchunk, j, p, pl.ppad, reinterpret_cast<double2*>(H), hld);
}

void launch_bupd(const BlockUpdPlan& pl, const double* V, int64_t ldv, int j, const double* H, int64_t hs_i,
                 int64_t hs_c, int p, int64_t n, double* part, const double* Yin, int64_t ldyin, double* Y,
                 int64_t ldy, double alpha, double beta, hipStream_t s) {
    if (p <= 0 || n <= 0) return;
    if (j > 0)
        hipLaunchKernelGGL(k_bupd, dim3((unsigned)pl.ntile, (unsigned)pl.nsplit, (unsigned)pl.ctiles), dim3(64), 0, s,
                           reinterpret_cast<const double2*>(V), ldv, j, pl.ksplit, reinterpret_cast<const double2*>(H),
                           hs_i, hs_c, p, n, reinterpret_cast<double2*>(part), pl.ppad);
    hipLaunchKernelGGL(k_bupd_finish, dim3(gridn(n, 256), (unsigned)p), dim3(256), 0, s,
                       reinterpret_cast<const double2*>(part), j > 0 ? pl.nsplit : 0, pl.ppad, p, n,
                       reinterpret_cast<const double2*>(Yin), ldyin, reinterpret_cast<double2*>(Y), ldy, alpha, beta);
}

}  // namespace mtf
