// Block Krylov kernels (gfx950): the dense FP64 contractions of block GMRES on the matrix cores.
//
// A block of p Krylov vectors against a basis of j vectors (complex128, each vector contiguous)
// is orthogonalised by classical Gram-Schmidt in block form:
//     H = V^H W          (j x p, one pass over the basis)           k_bdot + k_bdot_reduce
//     W <- W - V H       (N x p, one pass over the basis)           k_bupd + k_bupd_finish
// Both are GEMMs with one very long dimension (N) and p <= 32, so each wavefront takes every column
// of its tile (up to two 16-column MFMA blocks) and the basis is read once per pass; the arithmetic
// (8 p flops per complex basis entry) runs on v_mfma_f64_16x16x4f64, which at p = 32 is the bound
// (16 flops per byte of basis against a ridge of 78.6 TFLOP/s / 8 TB/s, about 10).  The same
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

// part[chunk][i][c] = sum over n in the chunk of conj(V_i[n]) W_c[n], i < j, c < p <= 16 NCB.
// One wavefront per (64 basis vectors, chunk of nc unknowns) for all columns (NCB blocks of 16), so
// that each basis entry is read once; nc is a multiple of 16.
template <int NCB>
__global__ __launch_bounds__(64) void k_bdot(const double2* __restrict__ V, int64_t ldv, int j,
                                             const double2* __restrict__ W, int64_t ldw, int p, int64_t n,
                                             int64_t nc, double2* __restrict__ part, int ppad) {
    const int lane = threadIdx.x;
    const int r = lane & 15, ks = lane >> 4;
    const int i0 = blockIdx.x * 64;
    const int64_t nb = (int64_t)blockIdx.y * nc;
    const int64_t ne = nb + nc < n ? nb + nc : n;
    const double2* vp[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int i = i0 + 16 * b + r;
        vp[b] = V + (int64_t)(i < j ? i : j - 1) * ldv;     // rows past j are computed, never stored
    }
    const double2* wp[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
        const int col = 16 * cb + r;
        wp[cb] = W + (int64_t)(col < p ? col : p - 1) * ldw;
    }
    d4 accr[NCB][4], acci[NCB][4];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            accr[cb][b] = d4{0.0, 0.0, 0.0, 0.0};
            acci[cb][b] = d4{0.0, 0.0, 0.0, 0.0};
        }
    for (int64_t n0 = nb; n0 < ne; n0 += 16) {
        const int64_t nn = n0 + 4 * ks;
        double2 w[NCB][4], v[4][4];
        if (nn + 4 <= ne) {
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                for (int t = 0; t < 4; ++t) w[cb][t] = wp[cb][nn + t];
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int t = 0; t < 4; ++t) v[b][t] = vp[b][nn + t];
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const bool ok = nn + t < ne;
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) w[cb][t] = ok ? wp[cb][nn + t] : make_double2(0.0, 0.0);
#pragma unroll
                for (int b = 0; b < 4; ++b) v[b][t] = ok ? vp[b][nn + t] : make_double2(0.0, 0.0);
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    // conj(v) w = (vr wr + vi wi) + i (vr wi - vi wr)
                    accr[cb][b] = mfma(v[b][t].x, w[cb][t].x, accr[cb][b]);
                    accr[cb][b] = mfma(v[b][t].y, w[cb][t].y, accr[cb][b]);
                    acci[cb][b] = mfma(v[b][t].x, w[cb][t].y, acci[cb][b]);
                    acci[cb][b] = mfma(-v[b][t].y, w[cb][t].x, acci[cb][b]);
                }
    }
    double2* out = part + (int64_t)blockIdx.y * j * ppad;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
        const int col = 16 * cb + r;
        if (col >= p) continue;
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = i0 + 16 * b + 4 * q + ks;
                if (i < j) out[(int64_t)i * ppad + col] = make_double2(accr[cb][b][q], acci[cb][b][q]);
            }
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
// One wavefront per (64 unknowns, split of ks basis vectors) for all columns (NCB blocks of 16), so
// that each basis entry is read once; ks is a multiple of 4.
template <int NCB>
__global__ __launch_bounds__(64) void k_bupd(const double2* __restrict__ V, int64_t ldv, int j, int ksplit,
                                             const double2* __restrict__ H, int64_t hs_i, int64_t hs_c, int p,
                                             int64_t n, double2* __restrict__ part, int ppad) {
    const int lane = threadIdx.x;
    const int r = lane & 15, ks = lane >> 4;
    const int64_t n0 = (int64_t)blockIdx.x * 64;
    const int ib = blockIdx.y * ksplit;
    const int ie = ib + ksplit < j ? ib + ksplit : j;
    int64_t nrow[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int64_t nn = n0 + 16 * b + r;
        nrow[b] = nn < n ? nn : n - 1;                       // rows past n are computed, never stored
    }
    d4 accr[NCB][4], acci[NCB][4];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            accr[cb][b] = d4{0.0, 0.0, 0.0, 0.0};
            acci[cb][b] = d4{0.0, 0.0, 0.0, 0.0};
        }
    for (int i = ib; i < ie; i += 4) {
        const int ii = i + ks;
        const int ic = ii < ie ? ii : ie - 1;
        double2 h[NCB];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            const int col = 16 * cb + r;
            const int cc = col < p ? col : p - 1;
            h[cb] = H[(int64_t)ic * hs_i + (int64_t)cc * hs_c];
            if (!(ii < ie && col < p)) h[cb] = make_double2(0.0, 0.0);
        }
        const double2* vrow = V + (int64_t)ic * ldv;
        double2 v[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) v[b] = vrow[nrow[b]];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                // v h = (vr hr - vi hi) + i (vr hi + vi hr)
                accr[cb][b] = mfma(v[b].x, h[cb].x, accr[cb][b]);
                accr[cb][b] = mfma(-v[b].y, h[cb].y, accr[cb][b]);
                acci[cb][b] = mfma(v[b].x, h[cb].y, acci[cb][b]);
                acci[cb][b] = mfma(v[b].y, h[cb].x, acci[cb][b]);
            }
    }
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
        const int col = 16 * cb + r;
        if (col >= p) continue;
        double2* out = part + ((int64_t)blockIdx.y * ppad + col) * n;
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t nn = n0 + 16 * b + 4 * q + ks;
                if (nn < n) out[nn] = make_double2(accr[cb][b][q], acci[cb][b][q]);
            }
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


// Multi-right-hand-side FP64 product of the diagonal blocks (the 2 A_i part of M) for q vectors:
// one wavefront per (subdomain, 16 RB rows, k-range) for 16 NCB right-hand sides from it.z on.
// Launched with RB = 4, NCB = 1 (64 x 16 tiles, T_i and K_i read by two wavefronts for 32
// vectors): 32 x 32 tiles (read once) ran 7% slower (2.74 ms against 2.55 ms for 32 vectors on the
// 4x4x4 cube at h = 1/24) and 64 x 32 tiles (392 registers, one wavefront per SIMD) 86% slower:
//     yD += K (2 x_D) + T ((2 / rho) x_N),   yN += K (2 x_N) + T (-2 rho x_D)
// over its k-range of columns of T_i, K_i (complex128, column-major, read whole), written as
// partial sums per k-range; k_mmv_finish adds them up with the transmission terms.
template <int RB, int NCB>
__global__ __launch_bounds__(64) void k_mmv(const DomDesc* __restrict__ doms, const int4* __restrict__ items,
                                            const double2* __restrict__ T, const double2* __restrict__ K,
                                            const double2* __restrict__ x, int64_t ldx, int q,
                                            const int64_t* __restrict__ pbase, int kc, double2* __restrict__ part) {
    const int4 it = items[blockIdx.x];               // (dom, row0, rhs0, split)
    const DomDesc dd = doms[it.x];
    const int E = dd.E;
    const int lane = threadIdx.x;
    const int r = lane & 15, ks = lane >> 4;
    const int row0 = it.y;
    const int kb = it.w * kc;
    const int ke = kb + kc < E ? kb + kc : E;
    const double2* xd[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
        const int c = it.z + 16 * cb + r;
        xd[cb] = x + (int64_t)(c < q ? c : q - 1) * ldx + dd.off;
    }
    const double rho = dd.rho;
    const double2* Tb = T + dd.mat0;
    const double2* Kb = K + dd.mat0;
    int rowc[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b) {
        const int rr = row0 + 16 * b + r;
        rowc[b] = rr < E ? rr : E - 1;                  // rows past E are computed, never stored
    }
    d4 aDr[NCB][RB], aDi[NCB][RB], aNr[NCB][RB], aNi[NCB][RB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            aDr[cb][b] = d4{0.0, 0.0, 0.0, 0.0};
            aDi[cb][b] = aDr[cb][b];
            aNr[cb][b] = aDr[cb][b];
            aNi[cb][b] = aDr[cb][b];
        }
    for (int k0 = kb; k0 < ke; k0 += 16) {
        const int kk = k0 + 4 * ks;
        double2 vd[NCB][4], vn[NCB][4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const bool ok = kk + t < ke;
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                vd[cb][t] = ok ? xd[cb][kk + t] : make_double2(0.0, 0.0);
                vn[cb][t] = ok ? xd[cb][E + kk + t] : make_double2(0.0, 0.0);
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int col = kk + t < ke ? kk + t : ke - 1;     // its B values are zero past ke
            const double2* Kc = Kb + (int64_t)col * E;
            const double2* Tc = Tb + (int64_t)col * E;
            double2 kv[RB], tv[RB];
#pragma unroll
            for (int b = 0; b < RB; ++b) {
                kv[b] = Kc[rowc[b]];
                tv[b] = Tc[rowc[b]];
            }
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                // scaled right-hand operands: 2 x_D, 2 x_N, (2 / rho) x_N, -2 rho x_D
                const double dr = 2.0 * vd[cb][t].x, di = 2.0 * vd[cb][t].y;
                const double nr = 2.0 * vn[cb][t].x, ni = 2.0 * vn[cb][t].y;
                const double tnr = nr / rho, tni = ni / rho;
                const double tdr = -rho * dr, tdi = -rho * di;
#pragma unroll
                for (int b = 0; b < RB; ++b) {
                    // (a)(b) = (ar br - ai bi) + i (ar bi + ai br)
                    aDr[cb][b] = mfma(kv[b].x, dr, aDr[cb][b]);
                    aDr[cb][b] = mfma(-kv[b].y, di, aDr[cb][b]);
                    aDi[cb][b] = mfma(kv[b].x, di, aDi[cb][b]);
                    aDi[cb][b] = mfma(kv[b].y, dr, aDi[cb][b]);
                    aDr[cb][b] = mfma(tv[b].x, tnr, aDr[cb][b]);
                    aDr[cb][b] = mfma(-tv[b].y, tni, aDr[cb][b]);
                    aDi[cb][b] = mfma(tv[b].x, tni, aDi[cb][b]);
                    aDi[cb][b] = mfma(tv[b].y, tnr, aDi[cb][b]);
                    aNr[cb][b] = mfma(kv[b].x, nr, aNr[cb][b]);
                    aNr[cb][b] = mfma(-kv[b].y, ni, aNr[cb][b]);
                    aNi[cb][b] = mfma(kv[b].x, ni, aNi[cb][b]);
                    aNi[cb][b] = mfma(kv[b].y, nr, aNi[cb][b]);
                    aNr[cb][b] = mfma(tv[b].x, tdr, aNr[cb][b]);
                    aNr[cb][b] = mfma(-tv[b].y, tdi, aNr[cb][b]);
                    aNi[cb][b] = mfma(tv[b].x, tdi, aNi[cb][b]);
                    aNi[cb][b] = mfma(tv[b].y, tdr, aNi[cb][b]);
                }
            }
        }
    }
    // partial sums of split s: part[pbase[dom] + ((s q + rhs) 2 + side) E + row]
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
        const int c = it.z + 16 * cb + r;
        if (c >= q) continue;
        double2* outD = part + pbase[it.x] + ((int64_t)(it.w * q + c) * 2) * E;
        double2* outN = outD + E;
#pragma unroll
        for (int b = 0; b < RB; ++b)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int rr = row0 + 16 * b + 4 * e + ks;
                if (rr < E) {
                    outD[rr] = make_double2(aDr[cb][b][e], aDi[cb][b][e]);
                    outN[rr] = make_double2(aNr[cb][b][e], aNi[cb][b][e]);
                }
            }
    }
}

// y_j = sum over splits of the partial diagonal-block products + the transmission terms G x_j, for
// every dof of every subdomain and right-hand side j < q
__global__ __launch_bounds__(256) void k_mmv_finish(const DomDesc* __restrict__ doms, const int32_t* __restrict__ dof_dom,
                                                    int64_t ndof, const int32_t* __restrict__ dplus,
                                                    const int32_t* __restrict__ dminus, const double* __restrict__ gval,
                                                    const int64_t* __restrict__ gcol, const double2* __restrict__ part,
                                                    const int64_t* __restrict__ pbase, const int* __restrict__ nsplit,
                                                    int q, const double2* __restrict__ x, int64_t ldx,
                                                    double2* __restrict__ y, int64_t ldy) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (g >= ndof || j >= q) return;
    const int dom = dof_dom[g];
    const DomDesc dd = doms[dom];
    const int64_t m = g - dd.dof0;
    const int E = dd.E;
    double yD[2] = {0.0, 0.0}, yN[2] = {0.0, 0.0};
    const double2* pb = part + pbase[dom];
    for (int s = 0; s < nsplit[dom]; ++s) {
        const double2 a = pb[((int64_t)(s * q + j) * 2) * E + m];
        const double2 b = pb[((int64_t)(s * q + j) * 2 + 1) * E + m];
        yD[0] += a.x; yD[1] += a.y;
        yN[0] += b.x; yN[1] += b.y;
    }
    const double2* xj = x + (int64_t)j * ldx;
    for (int side = 0; side < 2; ++side) {
        const int32_t* pm = side == 0 ? dplus : dminus;
        const int64_t rec = dd.rec0 + pm[2 * g];
        const int a = pm[2 * g + 1];
        for (int c = 0; c < 3; ++c) {
            const double v = gval[9 * rec + 3 * a + c];
            const double2 xd = xj[gcol[6 * rec + c]];
            const double2 xn = xj[gcol[6 * rec + 3 + c]];
            yD[0] += v * xd.x; yD[1] += v * xd.y;
            yN[0] += v * xn.x; yN[1] += v * xn.y;
        }
    }
    double2* yj = y + (int64_t)j * ldy;
    yj[dd.off + m] = make_double2(yD[0], yD[1]);
    yj[dd.off + E + m] = make_double2(yN[0], yN[1]);
}


// Block preconditioner P_i = 1/2 [[0, -S_i^-1 / rho_i], [rho_i S_i^-1, 0]] on q vectors from the whole
// complex64 blocks (promoted to FP64 on the matrix cores), one wavefront per (subdomain, 16 RB rows,
// k-range) of one Gauss-Seidel stage for 16 NCB right-hand sides from it.z (as for k_mmv):
//     zD += S^-1 (-x_N / (2 rho)),   zN += S^-1 (rho x_D / 2)
// as partial sums per k-range (part layout as for k_mmv); k_pcmm_finish adds them up.
template <int RB, int NCB>
__global__ __launch_bounds__(64) void k_pcmm(const DomDesc* __restrict__ doms, const int4* __restrict__ items,
                                             const float2* __restrict__ S, const double2* __restrict__ x, int64_t ldx,
                                             int q, const int64_t* __restrict__ pbase, int kc,
                                             double2* __restrict__ part) {
    const int4 it = items[blockIdx.x];
    const DomDesc dd = doms[it.x];
    const int E = dd.E;
    const int lane = threadIdx.x;
    const int r = lane & 15, ks = lane >> 4;
    const int row0 = it.y;
    const int kb = it.w * kc;
    const int ke = kb + kc < E ? kb + kc : E;
    const double2* xd[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
        const int c = it.z + 16 * cb + r;
        xd[cb] = x + (int64_t)(c < q ? c : q - 1) * ldx + dd.off;
    }
    const double sD = 0.5 * dd.rho, sN = -0.5 / dd.rho;
    const float2* Sb = S + dd.mat0;
    int rowc[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b) {
        const int rr = row0 + 16 * b + r;
        rowc[b] = rr < E ? rr : E - 1;
    }
    d4 aDr[NCB][RB], aDi[NCB][RB], aNr[NCB][RB], aNi[NCB][RB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            aDr[cb][b] = d4{0.0, 0.0, 0.0, 0.0};
            aDi[cb][b] = aDr[cb][b];
            aNr[cb][b] = aDr[cb][b];
            aNi[cb][b] = aDr[cb][b];
        }
    for (int k0 = kb; k0 < ke; k0 += 16) {
        const int kk = k0 + 4 * ks;
        double2 vd[NCB][4], vn[NCB][4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const bool ok = kk + t < ke;
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                vd[cb][t] = ok ? xd[cb][kk + t] : make_double2(0.0, 0.0);
                vn[cb][t] = ok ? xd[cb][E + kk + t] : make_double2(0.0, 0.0);
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int col = kk + t < ke ? kk + t : ke - 1;
            const float2* Sc = Sb + (int64_t)col * E;
            double ar[RB], ai[RB];
#pragma unroll
            for (int b = 0; b < RB; ++b) {
                const float2 sv = Sc[rowc[b]];
                ar[b] = sv.x;
                ai[b] = sv.y;
            }
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                const double nr = sN * vn[cb][t].x, ni = sN * vn[cb][t].y;     // into zD
                const double dr = sD * vd[cb][t].x, di = sD * vd[cb][t].y;     // into zN
#pragma unroll
                for (int b = 0; b < RB; ++b) {
                    aDr[cb][b] = mfma(ar[b], nr, aDr[cb][b]);
                    aDr[cb][b] = mfma(-ai[b], ni, aDr[cb][b]);
                    aDi[cb][b] = mfma(ar[b], ni, aDi[cb][b]);
                    aDi[cb][b] = mfma(ai[b], nr, aDi[cb][b]);
                    aNr[cb][b] = mfma(ar[b], dr, aNr[cb][b]);
                    aNr[cb][b] = mfma(-ai[b], di, aNr[cb][b]);
                    aNi[cb][b] = mfma(ar[b], di, aNi[cb][b]);
                    aNi[cb][b] = mfma(ai[b], dr, aNi[cb][b]);
                }
            }
        }
    }
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
        const int c = it.z + 16 * cb + r;
        if (c >= q) continue;
        double2* outD = part + pbase[it.x] + ((int64_t)(it.w * q + c) * 2) * E;
        double2* outN = outD + E;
#pragma unroll
        for (int b = 0; b < RB; ++b)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int rr = row0 + 16 * b + 4 * e + ks;
                if (rr < E) {
                    outD[rr] = make_double2(aDr[cb][b][e], aDi[cb][b][e]);
                    outN[rr] = make_double2(aNr[cb][b][e], aNi[cb][b][e]);
                }
            }
    }
}

// z_j (rows of the listed dofs) = sum over splits of the partial block-preconditioner products
__global__ __launch_bounds__(256) void k_pcmm_finish(const DomDesc* __restrict__ doms, const int32_t* __restrict__ dof_dom,
                                                     const int32_t* __restrict__ list, int64_t nlist,
                                                     const double2* __restrict__ part, const int64_t* __restrict__ pbase,
                                                     const int* __restrict__ nsplit, int q, double2* __restrict__ z,
                                                     int64_t ldz) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (t >= nlist || j >= q) return;
    const int64_t g = list ? list[t] : t;
    const int dom = dof_dom[g];
    const DomDesc dd = doms[dom];
    const int64_t m = g - dd.dof0;
    const int E = dd.E;
    double zD[2] = {0.0, 0.0}, zN[2] = {0.0, 0.0};
    const double2* pb = part + pbase[dom];
    for (int s = 0; s < nsplit[dom]; ++s) {
        const double2 a = pb[((int64_t)(s * q + j) * 2) * E + m];
        const double2 b = pb[((int64_t)(s * q + j) * 2 + 1) * E + m];
        zD[0] += a.x; zD[1] += a.y;
        zN[0] += b.x; zN[1] += b.y;
    }
    double2* zj = z + (int64_t)j * ldz;
    zj[dd.off + m] = make_double2(zD[0], zD[1]);
    zj[dd.off + E + m] = make_double2(zN[0], zN[1]);
}

// Gauss-Seidel stage input for q vectors: w = v - (transmission from the subdomains of earlier
// stages) z, for the listed dofs (both traces)
__global__ __launch_bounds__(256) void k_gs_residual_q(const DomDesc* __restrict__ doms, const int32_t* __restrict__ dof_dom,
                                                       const int32_t* __restrict__ list, int64_t nlist,
                                                       const int32_t* __restrict__ dplus, const int32_t* __restrict__ dminus,
                                                       const double* __restrict__ gval, const int64_t* __restrict__ gcol,
                                                       const int32_t* __restrict__ other_dom,
                                                       const int32_t* __restrict__ dom_stage, int stage,
                                                       const double2* __restrict__ v, const double2* __restrict__ z,
                                                       double2* __restrict__ w, int64_t ld, int q) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (t >= nlist || j >= q) return;
    const int64_t g = list[t];
    const DomDesc dd = doms[dof_dom[g]];
    const int64_t m = g - dd.dof0;
    const int64_t iD = dd.off + m, iN = dd.off + dd.E + m;
    const double2* vj = v + (int64_t)j * ld;
    const double2* zj = z + (int64_t)j * ld;
    double2 yD = vj[iD], yN = vj[iN];
    for (int side = 0; side < 2; ++side) {
        const int32_t* pm = side == 0 ? dplus : dminus;
        const int64_t rec = dd.rec0 + pm[2 * g];
        if (dom_stage[other_dom[rec]] >= stage) continue;      // neighbour not swept yet
        const int a = pm[2 * g + 1];
        for (int c = 0; c < 3; ++c) {
            const double gv = gval[9 * rec + 3 * a + c];
            const double2 zd = zj[gcol[6 * rec + c]];
            const double2 zn = zj[gcol[6 * rec + 3 + c]];
            yD.x -= gv * zd.x; yD.y -= gv * zd.y;
            yN.x -= gv * zn.x; yN.y -= gv * zn.y;
        }
    }
    double2* wj = w + (int64_t)j * ld;
    wj[iD] = yD;
    wj[iN] = yN;
}

inline unsigned gridn(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

BlockDotPlan plan_bdot(int64_t n, int j, int p) {
    BlockDotPlan pl;
    pl.itiles = (j + 63) / 64;
    pl.ctiles = (p + 15) / 16;
    pl.ppad = 16 * pl.ctiles;
    int64_t want = (2048 + pl.itiles - 1) / pl.itiles;
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
    int64_t want = (4096 + pl.ntile - 1) / pl.ntile;
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
    const dim3 grid((unsigned)pl.itiles, (unsigned)pl.nchunk);
    if (pl.ctiles == 1)
        hipLaunchKernelGGL(k_bdot<1>, grid, dim3(64), 0, s, reinterpret_cast<const double2*>(V), ldv, j,
                           reinterpret_cast<const double2*>(W), ldw, p, n, pl.nc, reinterpret_cast<double2*>(part),
                           pl.ppad);
    else
        hipLaunchKernelGGL(k_bdot<2>, grid, dim3(64), 0, s, reinterpret_cast<const double2*>(V), ldv, j,
                           reinterpret_cast<const double2*>(W), ldw, p, n, pl.nc, reinterpret_cast<double2*>(part),
                           pl.ppad);
    hipLaunchKernelGGL(k_bdot_reduce, dim3(gridn((int64_t)j * pl.ppad, 256)), dim3(256), 0, s,
                       reinterpret_cast<const double2*>(part), pl.nchunk, j, p, pl.ppad, reinterpret_cast<double2*>(H), hld);
}

void launch_bupd(const BlockUpdPlan& pl, const double* V, int64_t ldv, int j, const double* H, int64_t hs_i,
                 int64_t hs_c, int p, int64_t n, double* part, const double* Yin, int64_t ldyin, double* Y,
                 int64_t ldy, double alpha, double beta, hipStream_t s) {
    if (p <= 0 || n <= 0) return;
    if (j > 0) {
        const dim3 grid((unsigned)pl.ntile, (unsigned)pl.nsplit);
        if (pl.ctiles == 1)
            hipLaunchKernelGGL(k_bupd<1>, grid, dim3(64), 0, s, reinterpret_cast<const double2*>(V), ldv, j, pl.ksplit,
                               reinterpret_cast<const double2*>(H), hs_i, hs_c, p, n, reinterpret_cast<double2*>(part),
                               pl.ppad);
        else
            hipLaunchKernelGGL(k_bupd<2>, grid, dim3(64), 0, s, reinterpret_cast<const double2*>(V), ldv, j, pl.ksplit,
                               reinterpret_cast<const double2*>(H), hs_i, hs_c, p, n, reinterpret_cast<double2*>(part),
                               pl.ppad);
    }
    hipLaunchKernelGGL(k_bupd_finish, dim3(gridn(n, 256), (unsigned)p), dim3(256), 0, s,
                       reinterpret_cast<const double2*>(part), j > 0 ? pl.nsplit : 0, pl.ppad, p, n,
                       reinterpret_cast<const double2*>(Yin), ldyin, reinterpret_cast<double2*>(Y), ldy, alpha, beta);
}

void launch_mmv(const DomDesc* doms, const int4* items, int64_t nitems, const double* T, const double* K, const double* x,
                int64_t ldx, int q, const int64_t* pbase, int kc, double* part, const int32_t* dof_dom, int64_t ndof,
                const int32_t* dplus, const int32_t* dminus, const double* gval, const int64_t* gcol,
                const int* nsplit, double* y, int64_t ldy, hipStream_t s) {
    if (q <= 0) return;
    if (nitems > 0) {
        auto* k = k_mmv<4, 1>;
        hipLaunchKernelGGL(k, dim3((unsigned)nitems), dim3(64), 0, s, doms, items,
                           reinterpret_cast<const double2*>(T), reinterpret_cast<const double2*>(K),
                           reinterpret_cast<const double2*>(x), ldx, q, pbase, kc, reinterpret_cast<double2*>(part));
    }
    hipLaunchKernelGGL(k_mmv_finish, dim3(gridn(ndof, 256), (unsigned)q), dim3(256), 0, s, doms, dof_dom, ndof, dplus,
                       dminus, gval, gcol, reinterpret_cast<const double2*>(part), pbase, nsplit, q,
                       reinterpret_cast<const double2*>(x), ldx, reinterpret_cast<double2*>(y), ldy);
}


void launch_pcmm(const DomDesc* doms, const int4* items, int64_t nitems, const float* S, const double* x, int64_t ldx,
                 int q, const int64_t* pbase, int kc, double* part, const int32_t* dof_dom, const int32_t* list,
                 int64_t nlist, const int* nsplit, double* z, int64_t ldz, hipStream_t s) {
    if (q <= 0 || nlist <= 0) return;
    if (nitems > 0) {
        auto* k = k_pcmm<4, 1>;
        hipLaunchKernelGGL(k, dim3((unsigned)nitems), dim3(64), 0, s, doms, items, reinterpret_cast<const float2*>(S),
                           reinterpret_cast<const double2*>(x), ldx, q, pbase, kc, reinterpret_cast<double2*>(part));
    }
    hipLaunchKernelGGL(k_pcmm_finish, dim3(gridn(nlist, 256), (unsigned)q), dim3(256), 0, s, doms, dof_dom, list, nlist,
                       reinterpret_cast<const double2*>(part), pbase, nsplit, q, reinterpret_cast<double2*>(z), ldz);
}

void launch_gs_residual_q(const DomDesc* doms, const int32_t* dof_dom, const int32_t* list, int64_t nlist,
                          const int32_t* dplus, const int32_t* dminus, const double* gval, const int64_t* gcol,
                          const int32_t* other_dom, const int32_t* dom_stage, int stage, const double* v,
                          const double* z, double* w, int64_t ld, int q, hipStream_t s) {
    if (q <= 0 || nlist <= 0) return;
    hipLaunchKernelGGL(k_gs_residual_q, dim3(gridn(nlist, 256), (unsigned)q), dim3(256), 0, s, doms, dof_dom, list, nlist,
                       dplus, dminus, gval, gcol, other_dom, dom_stage, stage, reinterpret_cast<const double2*>(v),
                       reinterpret_cast<const double2*>(z), reinterpret_cast<double2*>(w), ld, q);
}

}  // namespace mtf
