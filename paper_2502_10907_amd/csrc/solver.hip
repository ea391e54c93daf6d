// Solver kernels for gfx950: block MTF matvec, GMRES vector operations and the
// complex64 building blocks of the block T^-1 preconditioner.
//
// Block matvec (Problem 2, Section 3.2): for every subdomain i
//   y_iD =  2 K_i x_iD + 2/rho_i T_i x_iN + sum_j G^ij x_jD
//   y_iN = -2 rho_i T_i x_iD + 2 K_i x_iN + sum_j G^ij x_jN
// The dense part streams the upper-triangle tiles of each T_i and K_i from HBM
// once per product and applies every entry in both positions (the blocks are
// complex symmetric up to the touching-pair entries, which a sparse correction
// restores); per-tile partial sums are reduced in the finishing kernel that also
// applies the correction and the sparse transmission part (six terms per row).
#include "device.h"

#include <algorithm>
#include <type_traits>

namespace mtf {

namespace {

template <typename RM>
struct C2 {
    RM re, im;
};

// Cross-lane moves within rows of 16 lanes (DPP): quad_perm [1,0,3,2], quad_perm [2,3,0,1],
// row_half_mirror, row_mirror.  After the four steps of row16_sum every lane of a row holds the
// sum over its row.
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

template <int CTRL>
__device__ inline float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}

template <int CTRL>
__device__ inline double dpp_d(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

template <typename F>
__device__ inline F row16_sum(F v) {
    if constexpr (std::is_same<F, double>::value) {
        v += dpp_d<kDppXor1>(v);
        v += dpp_d<kDppXor2>(v);
        v += dpp_d<kDppHalfMirror>(v);
        v += dpp_d<kDppMirror>(v);
    } else {
        v += dpp_f<kDppXor1>(v);
        v += dpp_f<kDppXor2>(v);
        v += dpp_f<kDppHalfMirror>(v);
        v += dpp_f<kDppMirror>(v);
    }
    return v;
}

constexpr int kDppRor4 = 0x124, kDppRor8 = 0x128;     // row_ror:4, row_ror:8

template <int CTRL, typename F>
__device__ inline F dpp(F v) {
    if constexpr (std::is_same<F, double>::value) return dpp_d<CTRL>(v);
    else return dpp_f<CTRL>(v);
}

// Sums four values over the 16 lanes of a row with five cross-lane moves: the lanes of a pair
// trade half of their values, those of a quad half of the rest, and the four quads their one
// remaining value.  On return lane l holds the row sum of value q = 2 (l & 1) + ((l >> 1) & 1).
template <typename F>
__device__ inline F row16_sum4(const F (&v)[4], int rg) {
    const bool odd = rg & 1, hi = (rg >> 1) & 1;
    const F s0 = odd ? v[0] : v[2], s1 = odd ? v[1] : v[3];
    const F w0 = (odd ? v[2] : v[0]) + dpp<kDppXor1>(s0);
    const F w1 = (odd ? v[3] : v[1]) + dpp<kDppXor1>(s1);
    F u = (hi ? w1 : w0) + dpp<kDppXor2>(hi ? w0 : w1);
    u += dpp<kDppRor4>(u);
    u += dpp<kDppRor8>(u);
    return u;
}

// a * b + c in the precision of the operands
__device__ inline float fmat(float a, float b, float c) { return fmaf(a, b, c); }
__device__ inline double fmat(double a, double b, double c) { return fma(a, b, c); }

// acc += a * b for complex a = (ar, ai), b = (br, bi) as four FMAs
template <typename F>
__device__ inline void cfma(F& re, F& im, F ar, F ai, F br, F bi) {
    re = fmat(ar, br, re);
    re = fmat(-ai, bi, re);
    im = fmat(ar, bi, im);
    im = fmat(ai, br, im);
}

// Steps k + j (j < NS) of a register-slot ring, slot j, each issuing the load D groups ahead.
template <int NS, typename Step, int... j>
__device__ inline void ring_round(Step& step, int k, std::integer_sequence<int, j...>) {
    (step(k + j, std::integral_constant<int, j>{}, std::true_type{}), ...);
}

// The remaining steps K0 + j of a ring over KN groups: slot (K0 + j) % NS, a load issued only
// while group K0 + j + D exists.
template <int NS, int K0, int D, int KN, typename Step, int... j>
__device__ inline void ring_tail(Step& step, std::integer_sequence<int, j...>) {
    (step(K0 + j, std::integral_constant<int, (K0 + j) % NS>{}, std::bool_constant<(K0 + j + D < KN)>{}), ...);
}

// Symmetric-read block matvec.  The separated-pair part of T_i and K_i is complex symmetric (the
// quadrature of a separated pair is the same in both orders), so a wavefront reads only the tiles
// (I, J), I <= J, of 64 x 64 entries and applies each entry twice: as (row r, column c) and, off
// the diagonal, as (row c, column r).  In a diagonal tile the strict lower triangle is dropped and
// the diagonal entries are halved, so that both uses together apply each entry once.  The
// touching-pair entries differ between the two orders by the quadrature error of the singular
// rules; the exact lower entries are restored by the sparse correction applied in the finishing
// kernel.
// Lane (rg = l % 16, cg = l / 16) owns rows r0 + rg + 16 i (i < 4) and columns c0 + 4k + cg
// (k < 16): each load instruction reads 16 consecutive rows.  The tile and domain descriptors are
// wave-uniform (scalar loads); a column's eight loads share one 32-bit byte offset from the tile
// base.  Rows past E are not clamped: they read the next column (or at most 63 entries into the
// padding behind the blocks) and meet zero row values or unwritten outputs.  The loads of the
// next column group are issued before the arithmetic of the current one.  The wavefront's 64 column values of x are staged in
// LDS.  Direct sums stay in registers and are reduced over the four column phases at the end; the
// transposed sums of each column are reduced over the 16 row lanes at once (DPP).  Partial slots
// per row (nb = ceil(E/64) blocks): the direct part of tile (B, J) goes to slot J+1, the
// transposed part of tile (I, B) to slot I, so every row has nb + 1 slots, each written once.
template <typename RM>
__global__ __launch_bounds__(256, 2) void k_mv_sym(const DomDesc* __restrict__ doms, const int4* __restrict__ stiles,
                                                   int64_t ntiles, const RM* __restrict__ T, const RM* __restrict__ K,
                                                   const double* __restrict__ x, double* __restrict__ part) {
    using V2 = typename std::conditional<std::is_same<RM, double>::value, double2, float2>::type;
    using V4 = typename std::conditional<std::is_same<RM, double>::value, double4, float4>::type;
    __shared__ V4 xs[4][64];                            // per wavefront: x_D, x_N at column c0 + l
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t tix = (int64_t)blockIdx.x * 4 + wv;
    const bool live = tix < ntiles;
    const int4 t = stiles[live ? tix : ntiles - 1];
    const DomDesc dd = doms[t.x];
    const int E = dd.E;
    const int I = t.y, J = t.z;
    const int r0 = I * 64, c0 = J * 64;
    const int rg = lane & 15, cg = lane >> 4;
    const bool diag = I == J;
    const RM rho = (RM)dd.rho, irho = (RM)(1.0 / dd.rho);
    const double2* xD = reinterpret_cast<const double2*>(x) + dd.off;
    const double2* xN = xD + E;
    {
        const int c = c0 + lane;
        const bool ok = c < E;
        const int cs = ok ? c : E - 1;
        const double2 d = xD[cs], nn = xN[cs];
        xs[wv][lane] = V4{(RM)(ok ? d.x : 0.0), (RM)(ok ? d.y : 0.0), (RM)(ok ? nn.x : 0.0), (RM)(ok ? nn.y : 0.0)};
    }
    __syncthreads();
    if (!live) return;                                  // no workgroup barrier below
    // With A = 2 x_D, B = (2/rho) x_N = C / rho, C = 2 x_N and P = -rho A the 2x2 Calderon
    // block of a row is  y_D += K A + T B,  y_N += K C + T P.
    RM ra[4][2], rc[4][2];                              // A and C of this lane's rows (transposed part)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = r0 + rg + 16 * i;
        const bool ok = r < E;
        const int rs = ok ? r : E - 1;
        const double2 d = xD[rs], nn = xN[rs];
        ra[i][0] = (RM)(ok ? 2.0 * d.x : 0.0); ra[i][1] = (RM)(ok ? 2.0 * d.y : 0.0);
        rc[i][0] = (RM)(ok ? 2.0 * nn.x : 0.0); rc[i][1] = (RM)(ok ? 2.0 * nn.y : 0.0);
    }
    const int64_t tile0 = dd.mat0 + r0 + (int64_t)c0 * E;
    const char* Tt = reinterpret_cast<const char*>(reinterpret_cast<const V2*>(T) + tile0);
    const char* Kt = reinterpret_cast<const char*>(reinterpret_cast<const V2*>(K) + tile0);
    RM acc[4][4];                                       // per row: y_D (re, im), y_N (re, im)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[i][q] = 0;
    double* pbase = part + 2 * dd.part0;
    // ring of register slots: one column group ahead in FP64 (register bound), three in FP32
    constexpr int D = std::is_same<RM, double>::value ? 1 : 3, NS = D + 1;
    V2 tv[NS][4], kv[NS][4];
    // In a diagonal tile the lanes below the diagonal (row > column) issue no load: those entries
    // are dropped anyway, and the masked lanes' lines are not fetched.
    auto load = [&](int k, int slot) {
        const int c = c0 + 4 * k + cg;
        const int cs = c < E ? c : E - 1;
        const uint32_t boff = ((uint32_t)rg + (uint32_t)(cs - c0) * (uint32_t)E) * (uint32_t)sizeof(V2);
        const V2* tp = reinterpret_cast<const V2*>(Tt + boff);
        const V2* kp = reinterpret_cast<const V2*>(Kt + boff);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            V2 a{}, b{};
            if (!diag || rg + 16 * i <= 4 * k + cg) {
                a = tp[16 * i];
                b = kp[16 * i];
            }
            tv[slot][i] = a;
            kv[slot][i] = b;
        }
    };
    // column group k computes from slot k % 2 while group k + 1 is in flight (the slot and
    // whether a load is issued are compile-time, so no register set is kept alive across a branch)
    auto step = [&](int k, auto slot, auto issue) {
        constexpr int sl = decltype(slot)::value;
        if constexpr (decltype(issue)::value) load(k + D, (sl + D) % NS);
        const int c = c0 + 4 * k + cg;
        const V4 xv = xs[wv][4 * k + cg];
        const RM Ar = 2 * xv.x, Ai = 2 * xv.y, Cr = 2 * xv.z, Ci = 2 * xv.w;
        const RM Br = irho * Cr, Bi = irho * Ci, Pr = -rho * Ar, Pi = -rho * Ai;
        RM e[4][4];                                     // T re, T im, K re, K im
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            e[i][0] = tv[sl][i].x; e[i][1] = tv[sl][i].y;
            e[i][2] = kv[sl][i].x; e[i][3] = kv[sl][i].y;
        }
        if (diag) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = r0 + rg + 16 * i;
                const RM w = r < c ? RM(1) : (r == c ? RM(0.5) : RM(0));
#pragma unroll
                for (int q = 0; q < 4; ++q) e[i][q] *= w;
            }
        }
        RM vD[2] = {0, 0}, vN[2] = {0, 0}, tr[2] = {0, 0}, tp[2] = {0, 0};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const RM ar = e[i][0], ai = e[i][1], br = e[i][2], bi = e[i][3];
            // direct, row r
            cfma(acc[i][0], acc[i][1], br, bi, Ar, Ai);
            cfma(acc[i][0], acc[i][1], ar, ai, Br, Bi);
            cfma(acc[i][2], acc[i][3], br, bi, Cr, Ci);
            cfma(acc[i][2], acc[i][3], ar, ai, Pr, Pi);
            // transposed, row c: K A_r and K C_r directly, T C_r and T A_r scaled after the sum
            cfma(vD[0], vD[1], br, bi, ra[i][0], ra[i][1]);
            cfma(vN[0], vN[1], br, bi, rc[i][0], rc[i][1]);
            cfma(tr[0], tr[1], ar, ai, rc[i][0], rc[i][1]);
            cfma(tp[0], tp[1], ar, ai, ra[i][0], ra[i][1]);
        }
        const RM v[4] = {fmat(irho, tr[0], vD[0]), fmat(irho, tr[1], vD[1]), fmat(-rho, tp[0], vN[0]),
                         fmat(-rho, tp[1], vN[1])};
        // lanes rg = 0, 1, 2, 3 hold the sums of y_D re, y_N re, y_D im, y_N im of row c
        const RM u = row16_sum4(v, rg);
        if (rg < 4 && c < E) pbase[2 * ((int64_t)(2 * I + (rg & 1)) * E + c) + (rg >> 1)] = (double)u;
    };
#pragma unroll
    for (int k = 0; k < D; ++k) load(k, k);
    constexpr int kFull = ((16 - D) / NS) * NS;
#pragma unroll 1
    for (int k = 0; k < kFull; k += NS) ring_round<NS>(step, k, std::make_integer_sequence<int, NS>{});
    ring_tail<NS, kFull, D, 16>(step, std::make_integer_sequence<int, 16 - kFull>{});
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            acc[i][q] += __shfl_xor(acc[i][q], 16, 64);
            acc[i][q] += __shfl_xor(acc[i][q], 32, 64);
        }
    if (cg != 0) return;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = r0 + rg + 16 * i;
        if (r >= E) continue;
        double* pD = pbase + 2 * ((int64_t)(2 * (J + 1)) * E + r);
        double* pN = pbase + 2 * ((int64_t)(2 * (J + 1) + 1) * E + r);
        *reinterpret_cast<double2*>(pD) = make_double2((double)acc[i][0], (double)acc[i][1]);
        *reinterpret_cast<double2*>(pN) = make_double2((double)acc[i][2], (double)acc[i][3]);
    }
}

// Preconditioner product: v_D = S x_D, v_N = S x_N per subdomain with S the complex64 inverse of
// the symmetric part of T_i (symmetric up to the rounding of the inversion; only its tiles
// I <= J are read, each entry used as (r, c) and, off the diagonal, as (c, r); in a diagonal tile
// the strict lower triangle is dropped and the diagonal halved).  Tiles flagged in their fourth
// component belong to a subdomain whose block is the inverse of T_i itself: every tile (I, J) is
// listed and used directly only (the transposed slots of its rows are not summed).  Same
// lane layout within a column group, addressing and partial-slot layout as k_mv_sym; FP32
// arithmetic.  One workgroup per tile: wavefront w takes the four column groups of columns
// c0 + 16 w .. c0 + 16 w + 15 and issues all of its loads (8 KB) at once, so that a Gauss-Seidel
// stage with few tiles still has its whole block in flight; the row sums of the four wavefronts
// meet in LDS.
__global__ __launch_bounds__(256) void k_pc_sym(const DomDesc* __restrict__ doms, const int4* __restrict__ stiles,
                                                const float* __restrict__ Ti, const double* __restrict__ x,
                                                double* __restrict__ part) {
    __shared__ float4 xs[64];                           // x_D, x_N at column c0 + l
    __shared__ float4 xrs[64];                          // x_D, x_N at row r0 + l (0 past E)
    __shared__ float4 red[4][64];                       // per wavefront: direct sums of row r0 + l
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int4 t = stiles[blockIdx.x];
    const DomDesc dd = doms[t.x];
    const int E = dd.E;
    const int I = t.y, J = t.z;
    const int r0 = I * 64, c0 = J * 64;
    const int rg = lane & 15, cg = lane >> 4;
    const bool full = t.w != 0;                         // all tiles of the block, direct use only
    const bool diag = I == J && !full;
    const double2* xD = reinterpret_cast<const double2*>(x) + dd.off;
    const double2* xN = xD + E;
    if (wv < 2) {
        const int c = (wv == 0 ? c0 : r0) + lane;
        const bool ok = c < E;
        const int cs = ok ? c : E - 1;
        const double2 d = xD[cs], nn = xN[cs];
        const float4 v = ok ? make_float4((float)d.x, (float)d.y, (float)nn.x, (float)nn.y) : make_float4(0.f, 0.f, 0.f, 0.f);
        if (wv == 0) xs[lane] = v; else xrs[lane] = v;
    }
    const char* Tt = reinterpret_cast<const char*>(reinterpret_cast<const float2*>(Ti) + dd.mat0 + r0 + (int64_t)c0 * E);
    float2 a[4][4];                                     // [column group][row i]
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int c = c0 + 16 * wv + 4 * k + cg;
        const int cs = c < E ? c : E - 1;
        const uint32_t boff = ((uint32_t)rg + (uint32_t)(cs - c0) * (uint32_t)E) * (uint32_t)sizeof(float2);
        const float2* tp = reinterpret_cast<const float2*>(Tt + boff);
#pragma unroll
        for (int i = 0; i < 4; ++i) a[k][i] = tp[16 * i];
    }
    __syncthreads();
    float xr[4][4];                                     // x_D, x_N of this lane's rows
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float4 v = xrs[rg + 16 * i];
        xr[i][0] = v.x; xr[i][1] = v.y; xr[i][2] = v.z; xr[i][3] = v.w;
    }
    float acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[i][q] = 0.f;
    double* pbase = part + 2 * dd.part0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int cl = 16 * wv + 4 * k + cg;            // column within the tile
        const int c = c0 + cl;
        const float4 xv = xs[cl];
        float e[4][2];
#pragma unroll
        for (int i = 0; i < 4; ++i) { e[i][0] = a[k][i].x; e[i][1] = a[k][i].y; }
        if (diag) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = r0 + rg + 16 * i;
                const float w = r < c ? 1.f : (r == c ? 0.5f : 0.f);
                e[i][0] *= w;
                e[i][1] *= w;
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            cfma(acc[i][0], acc[i][1], e[i][0], e[i][1], xv.x, xv.y);
            cfma(acc[i][2], acc[i][3], e[i][0], e[i][1], xv.z, xv.w);
        }
        if (!full) {
            float v[4] = {0.f, 0.f, 0.f, 0.f};          // transposed: S x_D, S x_N of row c
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                cfma(v[0], v[1], e[i][0], e[i][1], xr[i][0], xr[i][1]);
                cfma(v[2], v[3], e[i][0], e[i][1], xr[i][2], xr[i][3]);
            }
            // lanes rg = 0, 1, 2, 3 hold the sums of v_D re, v_N re, v_D im, v_N im of row c
            const float u = row16_sum4(v, rg);
            if (rg < 4 && c < E) pbase[2 * ((int64_t)(2 * I + (rg & 1)) * E + c) + (rg >> 1)] = (double)u;
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            acc[i][q] += __shfl_xor(acc[i][q], 16, 64);
            acc[i][q] += __shfl_xor(acc[i][q], 32, 64);
        }
    if (cg == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) red[wv][rg + 16 * i] = make_float4(acc[i][0], acc[i][1], acc[i][2], acc[i][3]);
    }
    __syncthreads();
    // threads 0..63 write the D part of row r0 + l, threads 64..127 the N part
    if (wv >= 2) return;
    const int r = r0 + lane;
    if (r >= E) return;
    float sr = 0.f, si = 0.f;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const float4 v = red[w][lane];
        sr += wv == 0 ? v.x : v.z;
        si += wv == 0 ? v.y : v.w;
    }
    double* p = pbase + 2 * ((int64_t)(2 * (J + 1) + wv) * E + r);
    *reinterpret_cast<double2*>(p) = make_double2(sr, si);
}

// z_iD = -1/(2 rho) v_N, z_iN = rho/2 v_D from the slots of k_pc_sym that the row's tiles wrote
// (all dofs, or the dofs of `list`).  64 rows per workgroup, one per lane, so that every load of a
// slot reads the consecutive rows' entries at once; the four wavefronts take every fourth slot and
// meet in LDS.
__global__ __launch_bounds__(256) void k_pc_sym_finish(const DomDesc* __restrict__ doms,
                                                       const int32_t* __restrict__ dof_dom, int64_t ndof,
                                                       const double* __restrict__ part, const int2* __restrict__ slots,
                                                       double* __restrict__ z, const int32_t* __restrict__ list) {
    __shared__ double red[3][4][64];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t t = (int64_t)blockIdx.x * 64 + lane;
    const bool live = t < ndof;
    const int64_t ts = live ? t : ndof - 1;
    const int64_t g = list ? list[ts] : ts;
    const DomDesc dd = doms[dof_dom[g]];
    const int64_t m = g - dd.dof0;
    const int64_t E = dd.E;
    const int2 rng = slots[dd.chunk0 + (int)(m / 64)];
    const double2* pb = reinterpret_cast<const double2*>(part) + dd.part0 + m;
    double acc[4] = {0, 0, 0, 0};
#pragma unroll 4
    for (int c = rng.x + wv; c <= rng.y; c += 4) {
        const double2 d = pb[2 * c * E], n = pb[(2 * c + 1) * E];
        acc[0] += d.x; acc[1] += d.y;
        acc[2] += n.x; acc[3] += n.y;
    }
    if (wv > 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) red[wv - 1][q][lane] = acc[q];
    }
    __syncthreads();
    if (wv != 0 || !live) return;
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] += red[w][q][lane];
    const double a = -0.5 / dd.rho, b = 0.5 * dd.rho;
    double* oD = z + 2 * (dd.off + m);
    double* oN = z + 2 * (dd.off + E + m);
    *reinterpret_cast<double2*>(oD) = make_double2(a * acc[2], a * acc[3]);
    *reinterpret_cast<double2*>(oN) = make_double2(b * acc[0], b * acc[1]);
}

// A[r, c] <- 0 where the dofs r and c lie in different connected components (cid[r] != cid[c]) of the
// E x E complex64 block A (ld E)
__global__ void k_zero_offdiag_f32(float2* __restrict__ A, int E, const int32_t* __restrict__ cid) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)E * E) return;
    const int r = (int)(e % E), c = (int)(e / E);
    if (cid[r] != cid[c]) A[e] = make_float2(0.f, 0.f);
}

// A <- (A + A^T) / 2 for the n x n complex64 block A (ld n), in place
__global__ void k_symmetrize_f32(float* __restrict__ A, int n) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * n) return;
    const int r = (int)(e % n), c = (int)(e / n);
    if (r >= c) return;
    float2* A2 = reinterpret_cast<float2*>(A);
    const float2 u = A2[r + (int64_t)c * n], l = A2[c + (int64_t)r * n];
    const float2 m = make_float2(0.5f * (u.x + l.x), 0.5f * (u.y + l.y));
    A2[r + (int64_t)c * n] = m;
    A2[c + (int64_t)r * n] = m;
}

// Touching-pair corrections of the lower triangle: for each stored position (m, n), n < m, of the
// sparse pattern, D = A[m, n] - A[n, m] for A = T and K (complex, FP64), so that the symmetric-read
// product plus D x reproduces the stored blocks exactly.
template <typename RM>
__global__ void k_near_diff(const DomDesc* __restrict__ doms, const int32_t* __restrict__ dof_dom, int64_t ndof,
                            const int64_t* __restrict__ ptr, const int32_t* __restrict__ col, const RM* __restrict__ T,
                            const RM* __restrict__ K, double* __restrict__ out) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ndof) return;
    const DomDesc dd = doms[dof_dom[g]];
    const int64_t m = g - dd.dof0;
    const int64_t E = dd.E;
    const C2<RM>* Tb = reinterpret_cast<const C2<RM>*>(T) + dd.mat0;
    const C2<RM>* Kb = reinterpret_cast<const C2<RM>*>(K) + dd.mat0;
    for (int64_t q = ptr[g]; q < ptr[g + 1]; ++q) {
        const int64_t n = col[q];
        const C2<RM> a = Tb[m + n * E], at = Tb[n + m * E];
        const C2<RM> b = Kb[m + n * E], bt = Kb[n + m * E];
        double* o = out + 4 * q;
        o[0] = (double)a.re - (double)at.re;
        o[1] = (double)a.im - (double)at.im;
        o[2] = (double)b.re - (double)bt.re;
        o[3] = (double)b.im - (double)bt.im;
    }
}

// Finishing kernel of the symmetric-read product: nb + 1 partial slots per row, the touching-pair
// correction of the lower triangle and the transmission part.  64 rows per workgroup, one per lane,
// so that every load of a slot reads the consecutive rows' entries at once; the four wavefronts
// take every fourth slot, correction term and transmission term and meet in LDS.
__global__ __launch_bounds__(256) void k_mv_sym_finish(const DomDesc* __restrict__ doms,
                                                       const int32_t* __restrict__ dof_dom, int64_t ndof,
                                                       const int32_t* __restrict__ dplus,
                                                       const int32_t* __restrict__ dminus,
                                                       const double* __restrict__ gval, const int64_t* __restrict__ gcol,
                                                       const int64_t* __restrict__ nptr, const int32_t* __restrict__ ncol,
                                                       const double* __restrict__ nval, const double* __restrict__ part,
                                                       const double* __restrict__ x, double* __restrict__ y) {
    __shared__ double red[3][4][64];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t g = (int64_t)blockIdx.x * 64 + lane;
    const bool live = g < ndof;
    const int64_t gs = live ? g : ndof - 1;
    double acc[4] = {0, 0, 0, 0};     // yD re, im, yN re, im
    const DomDesc dd = doms[dof_dom[gs]];
    const int64_t m = gs - dd.dof0;
    const int64_t E = dd.E;
    const int nslot = dd.nchunk + 1;
    const double2* pb = reinterpret_cast<const double2*>(part) + dd.part0 + m;
#pragma unroll 4
    for (int c = wv; c < nslot; c += 4) {
        const double2 d = pb[2 * c * E], n = pb[(2 * c + 1) * E];
        acc[0] += d.x; acc[1] += d.y;
        acc[2] += n.x; acc[3] += n.y;
    }
    const double rho = dd.rho;
    const double* xD = x + 2 * dd.off;
    const double* xN = x + 2 * (dd.off + E);
    for (int64_t k = nptr[gs] + wv; k < nptr[gs + 1]; k += 4) {
        const int64_t n = ncol[k];
        const double* v = nval + 4 * k;
        const double tr = v[0], ti = v[1], kr = v[2], ki = v[3];
        const double dr = xD[2 * n], di = xD[2 * n + 1], nr = xN[2 * n], ni = xN[2 * n + 1];
        acc[0] += 2.0 * (kr * dr - ki * di) + (2.0 / rho) * (tr * nr - ti * ni);
        acc[1] += 2.0 * (kr * di + ki * dr) + (2.0 / rho) * (tr * ni + ti * nr);
        acc[2] += -2.0 * rho * (tr * dr - ti * di) + 2.0 * (kr * nr - ki * ni);
        acc[3] += -2.0 * rho * (tr * di + ti * dr) + 2.0 * (kr * ni + ki * nr);
    }
    for (int j = wv; j < 6; j += 4) {
        const int side = j / 3, c = j % 3;
        const int32_t* pm = side == 0 ? dplus : dminus;
        const int64_t rec = dd.rec0 + pm[2 * gs];
        const int a = pm[2 * gs + 1];
        const double v = gval[9 * rec + 3 * a + c];
        const double* xd = x + 2 * gcol[6 * rec + c];
        const double* xn = x + 2 * gcol[6 * rec + 3 + c];
        acc[0] += v * xd[0]; acc[1] += v * xd[1];
        acc[2] += v * xn[0]; acc[3] += v * xn[1];
    }
    if (wv > 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) red[wv - 1][q][lane] = acc[q];
    }
    __syncthreads();
    if (wv != 0 || !live) return;
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] += red[w][q][lane];
    double* oD = y + 2 * (dd.off + m);
    double* oN = y + 2 * (dd.off + E + m);
    *reinterpret_cast<double2*>(oD) = make_double2(acc[0], acc[1]);
    *reinterpret_cast<double2*>(oN) = make_double2(acc[2], acc[3]);
}

// Block Gauss-Seidel stage input: w_i = v_i - sum_j G^ij z_j for the dofs of one stage (z holds
// the already computed stages, zero elsewhere).
__global__ __launch_bounds__(256) void k_gs_residual(const DomDesc* __restrict__ doms, const int32_t* __restrict__ dof_dom,
                                                     const int32_t* __restrict__ list, int64_t nlist,
                                                     const int32_t* __restrict__ dplus, const int32_t* __restrict__ dminus,
                                                     const double* __restrict__ gval, const int64_t* __restrict__ gcol,
                                                     const int32_t* __restrict__ other_dom,
                                                     const int32_t* __restrict__ dom_stage, int stage,
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
        if (dom_stage[other_dom[rec]] >= stage) continue;      // neighbour not swept yet: its z is not set
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

// Batched Arnoldi with delayed classical Gram-Schmidt reorthogonalisation (DCGS2; Swirydowicz,
// Thomas, Yamazaki and others, 2020/2022).  At step j the slot V_j holds u, the candidate for
// q_j after ONE projection against Q_j = [q_0 .. q_{j-1}] (not yet normalised), and t = A u.  One
// pass over Q_j forms s = Q_j^H u, z = Q_j^H t, alpha = u^H u, gamma = u^H t; then
//   nu = sqrt(alpha - |s|^2),  q_j = (u - Q_j s) / nu,  c = (gamma - s^H z) / nu,
//   Hessenberg column j-1 (final) = its first-pass value + s, subdiagonal nu,
//   first-pass column j = ([z; c] - Hbar_j s) / nu   (A Q_j = Q_{j+1} Hbar_j),
//   next candidate u' = (t - Q_j z - q_j c) / nu,
// and a second pass over Q_j forms q_j and u' together: two reads of the basis per step instead
// of four.  nb right-hand sides advance in lockstep: Krylov slot j is an n x nb column-major slab
// at V + j*ldv (ldv = nb*n), column b belongs to right-hand side b (blockIdx.z or blockIdx.y).
// Per right-hand side b:  S, Z + b*(nvmax+1)  the coefficients (slot j holds alpha and gamma),
// H + b*hstride  the Hessenberg matrix (column-major, ld ldh),  scal + 4b  {nu, Re c, Im c}.
// The step index j is read from device memory (jdev[0]) by every kernel of a step, and the grids
// do not depend on it, so a captured sequence of steps can be replayed.

// Row chunks of the basis reductions at step j: about T work units (16 vectors x one chunk) per
// right-hand side, between cmin and kmax chunks.  Measured on the 27,648-row basis, about 1,300
// units in flight read fastest from the first step (512 chunks of 64 rows) to the last (32 chunks
// of 864 rows); fewer, longer chunks win once there are many vectors.  k_dot2 and k_reduce2 agree
// on it.
__device__ inline int dot_chunks(int nv, int T, int cmin, int kmax) {
    const int c = T / (nv / 16 + 1);
    return c < cmin ? cmin : min(c, kmax);
}

// One basis entry as complex128: the basis is stored in complex128 (double2) or complex64 (float2).
__device__ inline double2 basis_ld(const double2* p) { return *p; }
__device__ inline double2 basis_ld(const float2* p) {
    const float2 f = *p;
    return make_double2((double)f.x, (double)f.y);
}

// acc += {conj(x) u, conj(x) t}, stored as (re, im, re, im)
__device__ inline void dot2_acc(double (&a)[4], double2 x, double2 uu, double2 tt) {
    a[0] = fma(x.x, uu.x, fma(x.y, uu.y, a[0]));
    a[1] = fma(x.x, uu.y, fma(-x.y, uu.x, a[1]));
    a[2] = fma(x.x, tt.x, fma(x.y, tt.y, a[2]));
    a[3] = fma(x.x, tt.y, fma(-x.y, tt.x, a[3]));
}

// hpart[((b*(nvmax+1) + i)*kmax + blk)*4 + {0,1,2,3}] = partial {conj(v_i).u, conj(v_i).t} over row
// chunk blk, v_i = V_i for i < j and v_j = u = V_j; t = Tt (slab, ld n), or u itself when Tt is null.
// Complex128 basis.  Work unit k of a right-hand side is vector group k / nch, row chunk k % nch
// (nch = dot_chunks); the workgroups stride over the units.
__global__ __launch_bounds__(256) void k_dot2(const double2* __restrict__ V, int64_t ldv, const int* __restrict__ jdev,
                                              int nvmax, const double* __restrict__ Tt, int64_t n,
                                              double* __restrict__ hpart, int T, int cmin, int kmax) {
    // Row chunk of the basis against 16 vectors per work unit: lane (rg = l % 16, g = l / 16) of
    // wavefront w takes vector 16 vg + 4 w + g and rows lo + rg + 16 m, so that a load instruction
    // reads 16 consecutive rows of four vectors and the 16 row lanes of a vector meet in one
    // cross-lane reduction at the end of the chunk.
    const int nv = jdev[0];
    const int b = blockIdx.z;
    const int nch = dot_chunks(nv, T, cmin, kmax);
    const int64_t chunk = ((n + nch - 1) / nch + 15) / 16 * 16;
    const double2* u = V + ((int64_t)nv * ldv + (int64_t)b * n);
    const double2* t = Tt ? reinterpret_cast<const double2*>(Tt) + (int64_t)b * n : u;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int rg = lane & 15, g = lane >> 4;
    const int units = (nv / 16 + 1) * nch;
    for (int unit = blockIdx.x; unit < units; unit += gridDim.x) {
        const int vg = unit / nch, blk = unit - vg * nch;
        const int64_t lo = blk * chunk, hi = min(n, lo + chunk);
        const int i = vg * 16 + w * 4 + g;
        const int is = i <= nv ? i : nv;
        const double2* v = V + ((int64_t)is * ldv + (int64_t)b * n);
        double a[4] = {0, 0, 0, 0};                     // conj(v) u (re, im), conj(v) t (re, im)
#pragma unroll 8
        for (int64_t e = lo + rg; e < hi; e += 16) dot2_acc(a, v[e], u[e], t[e]);
        // lanes rg = 0, 1, 2, 3 hold the sums of a[0], a[2], a[1], a[3]
        const double sum = row16_sum4(a, rg);
        if (i <= nv && rg < 4)
            hpart[(((int64_t)b * (nvmax + 1) + i) * kmax + blk) * 4 + 2 * (rg & 1) + (rg >> 1)] = sum;
    }
}

// The same partial sums for a complex64 basis (slots i < j), with u read from its complex128 copy U
// (slab, ld n), so that alpha = u^H u and gamma = u^H t keep FP64 inputs.  A complex64 entry is half
// the bytes of the u and t entries it meets, so each lane takes four basis vectors per u, t load:
// lane (rg, g) of wavefront w takes vectors 16 vg + g + 4 k (k < 4) and rows lo + 64 m + 16 w + rg;
// the four wavefronts' sums of a vector meet in LDS.  (The layout of k_dot2 leaves the complex64
// pass no faster than the complex128 one; this one takes 38% less time at j = 760.)
__global__ __launch_bounds__(256) void k_dot2_c64(const float2* __restrict__ V, int64_t ldv,
                                                  const int* __restrict__ jdev, int nvmax,
                                                  const double* __restrict__ Tt, const double* __restrict__ U,
                                                  int64_t n, double* __restrict__ hpart, int T, int cmin, int kmax) {
    __shared__ double red[4][16][4];
    const int nv = jdev[0];
    const int b = blockIdx.z;
    const int nch = dot_chunks(nv, T, cmin, kmax);
    const int64_t chunk = ((n + nch - 1) / nch + 15) / 16 * 16;
    const double2* u = reinterpret_cast<const double2*>(U) + (int64_t)b * n;
    const double2* t = Tt ? reinterpret_cast<const double2*>(Tt) + (int64_t)b * n : u;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int rg = lane & 15, g = lane >> 4;
    const int units = (nv / 16 + 1) * nch;
    for (int unit = blockIdx.x; unit < units; unit += gridDim.x) {
        const int vg = unit / nch, blk = unit - vg * nch;
        const int64_t lo = blk * chunk, hi = min(n, lo + chunk);
        const float2* v[4];
        bool own[4];                                    // vector i >= j: u itself (only i == j is kept)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = vg * 16 + g + 4 * k;
            own[k] = i >= nv;
            v[k] = V + ((int64_t)(own[k] ? 0 : i) * ldv + (int64_t)b * n);
        }
        double a[4][4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int q = 0; q < 4; ++q) a[k][q] = 0.0;
        if (vg < nv / 16) {
#pragma unroll 2
            for (int64_t e = lo + 16 * w + rg; e < hi; e += 64) {
                const double2 uu = u[e], tt = t[e];
                double2 x[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) x[k] = basis_ld(v[k] + e);
#pragma unroll
                for (int k = 0; k < 4; ++k) dot2_acc(a[k], x[k], uu, tt);
            }
        } else {
            for (int64_t e = lo + 16 * w + rg; e < hi; e += 64) {
                const double2 uu = u[e], tt = t[e];
#pragma unroll
                for (int k = 0; k < 4; ++k) dot2_acc(a[k], own[k] ? uu : basis_ld(v[k] + e), uu, tt);
            }
        }
        // per vector k, lanes rg = 0, 1, 2, 3 hold the sums of a[k][0], a[k][2], a[k][1], a[k][3]
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double sum = row16_sum4(a[k], rg);
            if (rg < 4) red[w][g + 4 * k][2 * (rg & 1) + (rg >> 1)] = sum;
        }
        __syncthreads();
        if (threadIdx.x < 64) {
            const int vl = threadIdx.x >> 2, q = threadIdx.x & 3;
            const int i = vg * 16 + vl;
            if (i <= nv)
                hpart[(((int64_t)b * (nvmax + 1) + i) * kmax + blk) * 4 + q] =
                    red[0][vl][q] + red[1][vl][q] + red[2][vl][q] + red[3][vl][q];
        }
        __syncthreads();
    }
}

// S_i, Z_i from the partial sums, i <= j: one wavefront per vector
__global__ __launch_bounds__(256) void k_reduce2(const double* __restrict__ hpart, const int* __restrict__ jdev,
                                                 int nvmax, int T, int cmin, int kmax, double* __restrict__ S,
                                                 double* __restrict__ Z) {
    const int nv = jdev[0];
    const int b = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i > nv) return;
    const int nch = dot_chunks(nv, T, cmin, kmax);
    double a[4] = {0, 0, 0, 0};
    const double* p = hpart + ((int64_t)b * (nvmax + 1) + i) * kmax * 4;
    for (int k = lane; k < nch; k += 64) {
        const double4 q = *reinterpret_cast<const double4*>(p + 4 * k);
        a[0] += q.x; a[1] += q.y; a[2] += q.z; a[3] += q.w;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) a[q] = wsum(a[q]);
    if (lane != 0) return;
    const int64_t o = (int64_t)b * (nvmax + 1) + i;
    S[2 * o] = a[0]; S[2 * o + 1] = a[1];
    Z[2 * o] = a[2]; Z[2 * o + 1] = a[3];
}

// Partial products of the stored Hessenberg columns 0..j-1 with s: tile (row block rt of 64 rows,
// column block kc of 64 columns) -> hg[(b*nct + kc)*(nvmax+1) + i].  Only entries i <= k+1 count;
// row j of column j-1 is not final yet and is left out (k_dcgs_col adds its share).  Tiles with
// rt > kc + 1 lie below the band: they are neither written nor read.  blockIdx.x strides over the
// tiles of the (rt, kc) grid.
__device__ inline void hess_gemv_body(const double* __restrict__ H, int64_t ldh, int64_t hstride,
                                      const double* __restrict__ S, int nv, int nvmax, int nct,
                                      double* __restrict__ hg, int b, int tile0, int tstride) {
    if (nv < 1) return;
    const int nrt = (nv + 1 + 63) / 64, nkc = (nv + 63) / 64;
    const int r = threadIdx.x & 63, q = threadIdx.x >> 6;
    const double* Hb = H + 2 * (int64_t)b * hstride;
    const double* sb = S + 2 * (int64_t)b * (nvmax + 1);
    __shared__ double red[4][64][2];
    for (int tile = tile0; tile < nrt * nkc; tile += tstride) {
        const int rt = tile % nrt, kc = tile / nrt;
        if (rt > kc + 1) continue;
        const int i = rt * 64 + r;
        double re = 0, im = 0;
        const int k0 = kc * 64 + q * 16;
        if (i <= nv) {
#pragma unroll 4
            for (int kk = 0; kk < 16; ++kk) {
                const int k = k0 + kk;
                if (k >= nv || i > k + 1 || (k == nv - 1 && i == nv)) continue;
                const double hr = Hb[2 * ((int64_t)k * ldh + i)], hi = Hb[2 * ((int64_t)k * ldh + i) + 1];
                const double sr = sb[2 * k], si = sb[2 * k + 1];
                re += hr * sr - hi * si;
                im += hr * si + hi * sr;
            }
        }
        red[q][r][0] = re;
        red[q][r][1] = im;
        __syncthreads();
        if (q == 0 && i <= nv) {
            const double a = red[0][r][0] + red[1][r][0] + red[2][r][0] + red[3][r][0];
            const double c = red[0][r][1] + red[1][r][1] + red[2][r][1] + red[3][r][1];
            const int64_t o = ((int64_t)b * nct + kc) * (nvmax + 1) + i;
            hg[2 * o] = a;
            hg[2 * o + 1] = c;
        }
        __syncthreads();
    }
}

// nu = sqrt(alpha - |s|^2) and c = (gamma - s^H z) / nu of right-hand side b (alpha, gamma in
// slot j of S, Z).  Every workgroup of 256 threads that calls this sums in the same order, so all
// of them get the same values.
__device__ inline void dcgs_scalars(const double* __restrict__ sb, const double* __restrict__ zb, int nv,
                                    double& nu, double& cr, double& ci) {
    double ss = 0, pr = 0, pi = 0;
    for (int i = threadIdx.x; i < nv; i += 256) {
        const double sr = sb[2 * i], si = sb[2 * i + 1], zr = zb[2 * i], zi = zb[2 * i + 1];
        ss += sr * sr + si * si;
        pr += sr * zr + si * zi;
        pi += sr * zi - si * zr;
    }
    __shared__ double red[3][4];
    ss = wsum(ss); pr = wsum(pr); pi = wsum(pi);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) { red[0][wv] = ss; red[1][wv] = pr; red[2][wv] = pi; }
    __syncthreads();
    ss = pr = pi = 0;
    for (int k = 0; k < 4; ++k) { ss += red[0][k]; pr += red[1][k]; pi += red[2][k]; }
    const double alpha = sb[2 * nv];
    const double nu2 = alpha - ss;
    nu = nu2 > 0 ? sqrt(nu2) : 0.0;
    const double inv = nu > 0 ? 1.0 / nu : 0.0;
    cr = (zb[2 * nv] - pr) * inv;
    ci = (zb[2 * nv + 1] - pi) * inv;
}

// Finalise Hessenberg column j-1 and write the first-pass column j (skipped when `last`) for rows
// bx*256 .. bx*256+255.  When R is given, column j of the triangular factor U = Q R of the
// candidates is stored too: R[i, j] = s_i (i < j), R[j, j] = nu (per right-hand side at
// R + b*rstride, ld ldh).  When scal is given, {nu, Re c, Im c} go to scal + 4b.
__device__ inline void dcgs_col_body(double* __restrict__ H, int64_t ldh, int64_t hstride,
                                     const double* __restrict__ S, const double* __restrict__ Z,
                                     const double* __restrict__ hg, int nct, int nv, int nvmax,
                                     double* __restrict__ scal, int last, double* __restrict__ R, int64_t rstride,
                                     int b, int bx) {
    const double* sb = S + 2 * (int64_t)b * (nvmax + 1);
    const double* zb = Z + 2 * (int64_t)b * (nvmax + 1);
    double nu, cr, ci;
    dcgs_scalars(sb, zb, nv, nu, cr, ci);
    const double inv = nu > 0 ? 1.0 / nu : 0.0;
    if (scal && bx == 0 && threadIdx.x == 0) { scal[4 * b] = nu; scal[4 * b + 1] = cr; scal[4 * b + 2] = ci; }
    const int i = bx * 256 + threadIdx.x;
    if (i > nv) return;
    if (R) {
        double* Rc = R + 2 * ((int64_t)b * rstride + (int64_t)nv * ldh);
        Rc[2 * i] = i < nv ? sb[2 * i] : nu;
        Rc[2 * i + 1] = i < nv ? sb[2 * i + 1] : 0.0;
    }
    double* Hb = H + 2 * (int64_t)b * hstride;
    if (nv >= 1) {
        double* Hc = Hb + 2 * (int64_t)(nv - 1) * ldh;
        if (i < nv) { Hc[2 * i] += sb[2 * i]; Hc[2 * i + 1] += sb[2 * i + 1]; }
        else { Hc[2 * i] = nu; Hc[2 * i + 1] = 0.0; }
    }
    if (last) return;
    double hr = 0, hi = 0;
    if (nv >= 1) {
        const int kc0 = max(0, i / 64 - 1), kc1 = (nv + 63) / 64;    // the tiles this step wrote
        for (int kc = kc0; kc < kc1; ++kc) {
            const int64_t o = ((int64_t)b * nct + kc) * (nvmax + 1) + i;
            hr += hg[2 * o];
            hi += hg[2 * o + 1];
        }
        // column j-1 changed after the partial products: + (s_i or nu) * s_{j-1}
        const double lr = sb[2 * (nv - 1)], li = sb[2 * (nv - 1) + 1];
        const double fr = i < nv ? sb[2 * i] : nu, fi = i < nv ? sb[2 * i + 1] : 0.0;
        hr += fr * lr - fi * li;
        hi += fr * li + fi * lr;
    }
    const double zr = i < nv ? zb[2 * i] : cr, zi = i < nv ? zb[2 * i + 1] : ci;
    double* Hn = Hb + 2 * (int64_t)nv * ldh;
    Hn[2 * i] = (zr - hr) * inv;
    Hn[2 * i + 1] = (zi - hi) * inv;
}

// nu, c into scal; finalise Hessenberg column j-1; first-pass column j (skipped when `last`).
__global__ __launch_bounds__(256) void k_dcgs_col(double* __restrict__ H, int64_t ldh, int64_t hstride,
                                                  const double* __restrict__ S, const double* __restrict__ Z,
                                                  const double* __restrict__ hg, int nct, const int* __restrict__ jdev,
                                                  int nvmax, double* __restrict__ scal, int last, double* __restrict__ R,
                                                  int64_t rstride) {
    dcgs_col_body(H, ldh, hstride, S, Z, hg, nct, jdev[0], nvmax, scal, last, R, rstride, blockIdx.y, blockIdx.x);
}

// part[((b*ng + g)*n + e)*4 + {0..3}] = sum over the vectors i < j of group g of {V_i s_i, V_i z_i}
// (zero when a group has none).  The workgroups with
// blockIdx.x >= nxp instead form the partial products of the Hessenberg matrix with s
// (hess_gemv_body), which need nothing but S: the two independent parts of a step share a launch.
template <typename VT>
__global__ __launch_bounds__(256) void k_update2_part(const VT* __restrict__ V, int64_t ldv,
                                                      const int* __restrict__ jdev, int nvmax,
                                                      const double* __restrict__ S, const double* __restrict__ Z,
                                                      double* __restrict__ part, int64_t n, int nxp,
                                                      const double* __restrict__ H, int64_t ldh, int64_t hstride,
                                                      int nct, double* __restrict__ hg) {
    const int nv = jdev[0];
    const int b = blockIdx.z;
    if ((int)blockIdx.x >= nxp) {
        const int nhx = gridDim.x - nxp;
        hess_gemv_body(H, ldh, hstride, S, nv, nvmax, nct, hg, b, (blockIdx.x - nxp) + nhx * blockIdx.y,
                       nhx * gridDim.y);
        return;
    }
    __shared__ double cs[4 * 64];
    const int g = blockIdx.y, ng = gridDim.y;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t cb = (int64_t)b * (nvmax + 1);
    double ar = 0, ai = 0, br = 0, bi = 0;
    // group g takes vectors [g cv, (g + 1) cv), cv = ceil(j / ng) rounded up to 8, in LDS batches of 64
    const int cv = ((nv + ng - 1) / ng + 7) / 8 * 8;
    const int vend = min(nv, (g + 1) * cv);
    for (int i0 = g * cv; i0 < vend; i0 += 64) {
        const int cnt = min(64, vend - i0);
        __syncthreads();
        if ((int)threadIdx.x < cnt) {
            const int64_t o = cb + i0 + threadIdx.x;
            cs[4 * threadIdx.x] = S[2 * o]; cs[4 * threadIdx.x + 1] = S[2 * o + 1];
            cs[4 * threadIdx.x + 2] = Z[2 * o]; cs[4 * threadIdx.x + 3] = Z[2 * o + 1];
        }
        __syncthreads();
        if (e >= n) continue;
        const VT* v = V + ((int64_t)i0 * ldv + (int64_t)b * n + e);
        int i = 0;
        for (; i + 8 <= cnt; i += 8) {
            double vr[8], vi[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const double2 q = basis_ld(v + (int64_t)(i + k) * ldv);
                vr[k] = q.x;
                vi[k] = q.y;
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const double* q = cs + 4 * (i + k);
                ar += vr[k] * q[0] - vi[k] * q[1];
                ai += vr[k] * q[1] + vi[k] * q[0];
                br += vr[k] * q[2] - vi[k] * q[3];
                bi += vr[k] * q[3] + vi[k] * q[2];
            }
        }
        for (; i < cnt; ++i) {
            const double2 qv = basis_ld(v + (int64_t)i * ldv);
            const double vr = qv.x, vi = qv.y;
            const double* q = cs + 4 * i;
            ar += vr * q[0] - vi * q[1];
            ai += vr * q[1] + vi * q[0];
            br += vr * q[2] - vi * q[3];
            bi += vr * q[3] + vi * q[2];
        }
    }
    if (e >= n) return;
    double* o = part + (((int64_t)b * ng + g) * n + e) * 4;
    o[0] = ar; o[1] = ai; o[2] = br; o[3] = bi;
}

// q_j = (u - Q s)/nu into slot j, u' = (t - Q z - q_j c)/nu into slot j+1 and into Unext; when Zsrc
// is given it is also copied into slot j of Zdst (the preconditioned candidate of flexible GMRES).
// With a complex64 basis (VT = float2) u is read from Unext (its complex128 copy), q_j is rounded
// into slot j and u' goes to Unext only.
// Each workgroup forms nu and c itself from S and Z (dcgs_scalars).  The workgroups with
// blockIdx.x >= nxa finalise the Hessenberg columns instead (dcgs_col_body, rows 256 (blockIdx.x -
// nxa) onwards), which needs the partial products hg of the previous launch.
template <typename VT>
__global__ __launch_bounds__(256) void k_update2_apply(const double* __restrict__ part, int ng, VT* __restrict__ V,
                                                       int64_t ldv, const int* __restrict__ jdev, int* __restrict__ jnext,
                                                       const double* __restrict__ Tt, double* __restrict__ Unext,
                                                       int64_t n, const double* __restrict__ Zsrc,
                                                       double* __restrict__ Zdst, int nxa, int nvmax,
                                                       const double* __restrict__ S, const double* __restrict__ Z,
                                                       double* __restrict__ H, int64_t ldh, int64_t hstride,
                                                       const double* __restrict__ hg, int nct, double* __restrict__ R,
                                                       int64_t rstride) {
    const int nv = jdev[0];
    const int b = blockIdx.y;
    if ((int)blockIdx.x >= nxa) {
        dcgs_col_body(H, ldh, hstride, S, Z, hg, nct, nv, nvmax, nullptr, 0, R, rstride, b, blockIdx.x - nxa);
        return;
    }
    double nu, cr, ci;
    dcgs_scalars(S + 2 * (int64_t)b * (nvmax + 1), Z + 2 * (int64_t)b * (nvmax + 1), nv, nu, cr, ci);
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e == 0 && b == 0) jnext[0] = nv + 1;      // the other slot: read by the next step only
    if (e >= n) return;
    double ar = 0, ai = 0, br = 0, bi = 0;
    for (int g = 0; g < ng; ++g) {
        const double* p = part + (((int64_t)b * ng + g) * n + e) * 4;
        ar += p[0]; ai += p[1]; br += p[2]; bi += p[3];
    }
    const double inv = nu > 0 ? 1.0 / nu : 0.0;
    constexpr bool c64 = std::is_same<VT, float2>::value;
    VT* q = V + ((int64_t)nv * ldv + (int64_t)b * n + e);
    double2* uc = reinterpret_cast<double2*>(Unext) + (int64_t)b * n + e;
    const double2 u = c64 ? *uc : basis_ld(q);
    const double* t = Tt + 2 * ((int64_t)b * n + e);
    double qr = (u.x - ar) * inv, qi = (u.y - ai) * inv;
    if constexpr (c64) {
        // later steps see q_j rounded: u' is formed from the rounded value too, so that
        // t = Q z + q_j c + nu u' holds for the stored basis
        const float2 qf = make_float2((float)qr, (float)qi);
        *q = qf;
        qr = qf.x;
        qi = qf.y;
    }
    const double tr = (t[0] - br - (qr * cr - qi * ci)) * inv, ti = (t[1] - bi - (qr * ci + qi * cr)) * inv;
    if constexpr (!c64) {
        *q = make_double2(qr, qi);
        V[(int64_t)(nv + 1) * ldv + (int64_t)b * n + e] = make_double2(tr, ti);
    }
    *uc = make_double2(tr, ti);
    if (Zsrc) {
        const double* zs = Zsrc + 2 * ((int64_t)b * n + e);
        double* zd = Zdst + 2 * ((int64_t)nv * ldv + (int64_t)b * n + e);
        zd[0] = zs[0];
        zd[1] = zs[1];
    }
}

// p[0] = v
__global__ void k_set_int(int* p, int v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = v;
}

// Hst[(b*cnt + q)*ldh + i] = H column (jdev[0] - back + q) of right-hand side b, rows 0..ldh-1
__global__ void k_stage_cols(const double* __restrict__ H, int64_t ldh, int64_t hstride, const int* __restrict__ jdev,
                             int back, int cnt, double* __restrict__ Hst) {
    const int b = blockIdx.y;
    const int64_t c0 = jdev[0] - back;
    const int64_t tot = 2 * ldh * cnt;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x)
        Hst[(int64_t)b * tot + e] = H[2 * ((int64_t)b * hstride + c0 * ldh) + e];
}

// Back substitution y_b <- R_b^-1 y_b with the upper triangular cnt[b] x cnt[b] factor R_b
// (R + b*rstride, ld ldh), column by column; one workgroup per right-hand side.  A zero diagonal
// sets info[0] and leaves y_b unchanged from that column on.
__global__ __launch_bounds__(1024) void k_trsv_upper(const double* __restrict__ R, int64_t ldh, int64_t rstride,
                                                     const int* __restrict__ cnt, double* __restrict__ Y,
                                                     int64_t ystride, int* __restrict__ info) {
    const int b = blockIdx.x;
    const int it = cnt[b];
    const double* Rb = R + 2 * (int64_t)b * rstride;
    double* y = Y + 2 * (int64_t)b * ystride;
    __shared__ double wv[2];
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int i = it - 1; i >= 0; --i) {
        if (threadIdx.x == 0) {
            const double dr = Rb[2 * ((int64_t)i * ldh + i)], di = Rb[2 * ((int64_t)i * ldh + i) + 1];
            const double den = dr * dr + di * di;
            if (!(den > 0.0)) {
                bad = 1;
                info[0] = 1;
            } else {
                const double yr = y[2 * i], yi = y[2 * i + 1];
                wv[0] = (yr * dr + yi * di) / den;
                wv[1] = (yi * dr - yr * di) / den;
                y[2 * i] = wv[0];
                y[2 * i + 1] = wv[1];
            }
        }
        __syncthreads();
        if (bad) return;
        const double ar = wv[0], ai = wv[1];
        const double* col = Rb + 2 * (int64_t)i * ldh;
        for (int k = threadIdx.x; k < i; k += blockDim.x) {
            const double cr = col[2 * k], ci = col[2 * k + 1];
            y[2 * k] -= cr * ar - ci * ai;
            y[2 * k + 1] -= cr * ai + ci * ar;
        }
        __syncthreads();
    }
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

// complex64 GEMM on FP32 matrix cores (v_mfma_f32_32x32x2f32), batched over blockIdx.z, with
// optional skipped bands of rows and columns (see CGemm).  C may alias D: each output element is
// read and written by the same lane.
// Workgroup tile 128 x 64 complex, k-tile 16, four wavefronts in 2 x 2, each owning 64 x 32 as two
// 32 x 32 MFMA tiles.  Each complex product takes three real ones (Gauss's product, the 3M method):
// P1 = sum re*re, P2 = sum im*im, P3 = sum (re+im)*(re+im), then re = P1 - P2, im = P3 - P1 - P2;
// FP32 accumulation.  Its error bound is normwise (Higham, Accuracy and Stability, section 23.2.4),
// a little above the four-product form's and far below what a preconditioner's inverse needs.
// MFMA lane layout: first operand row l%32, k l/32; second operand k l/32, column l%32; result
// register i holds row (i/4)*8 + (l/32)*4 + i%4, column l%32.  Each tile is computed transposed
// (first operand B^T, second A^T), so that lane l holds matrix row l%32: the epilogue's loads and
// stores of C and D run down the columns (256 contiguous bytes per half-wavefront).
typedef float floatx16 __attribute__((ext_vector_type(16)));

__global__ __launch_bounds__(256, 3) void k_cgemm_mfma(const CGemm g) {
    constexpr int TM = 128, TN = 64, BK = 16;
    __shared__ float Ar[2][BK][TM], Ai[2][BK][TM];          // two k-tiles: one read, one filled
    __shared__ float Br[2][BK][TN + 1], Bi[2][BK][TN + 1];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wm = wv & 1, wn = wv >> 1;
    const int row0 = blockIdx.x * TM, col0 = blockIdx.y * TN;
    const int64_t z = blockIdx.z;
    const float2* A2 = reinterpret_cast<const float2*>(g.A) + z * g.sA;
    const float2* B2 = reinterpret_cast<const float2*>(g.B) + z * g.sB;
    const int m = g.m, n = g.n, k = g.k;
    floatx16 p10 = {}, p11 = {}, p20 = {}, p21 = {}, p30 = {}, p31 = {};
    const int ar_row = tid & 127, ar_k = (tid >> 7) * 8;     // A tile loader: one row, 8 k values
    const int bk = tid & 15, bc = tid >> 4;                   // B tile loader: one k, columns bc + 16q
    const int gr = row0 + ar_row;
    const int64_t pr = gr + (gr >= g.rg0 ? g.rgw : 0);
    int64_t pc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int gc = col0 + bc + 16 * q;
        pc[q] = gc + (gc >= g.cg0 ? g.cgw : 0);
    }
    // the next k-tile's global loads are issued before the matrix-core work on the current one
    float2 va[8], vb[4];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int gk = k0 + ar_k + q;
            va[q] = (gr < m && gk < k) ? A2[pr + (int64_t)gk * g.lda] : make_float2(0.f, 0.f);
        }
        const int gk = k0 + bk;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int gc = col0 + bc + 16 * q;
            vb[q] = (gc < n && gk < k) ? B2[gk + pc[q] * g.ldb] : make_float2(0.f, 0.f);
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            Ar[buf][ar_k + q][ar_row] = va[q].x;
            Ai[buf][ar_k + q][ar_row] = va[q].y;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            Br[buf][bk][bc + 16 * q] = vb[q].x;
            Bi[buf][bk][bc + 16 * q] = vb[q].y;
        }
    };
    fetch(0);
    stash(0);
    __syncthreads();
    // one barrier per k-tile: it orders the reads of buffer `cur` before its refill two tiles on,
    // and the refill of the other buffer before its reads in the next tile
    int cur = 0;
    for (int k0 = 0; k0 < k; k0 += BK) {
        const bool more = k0 + BK < k;
        if (more) fetch(k0 + BK);
#pragma unroll
        for (int kp = 0; kp < BK; kp += 2) {
            const int kk = kp + (lane >> 5);
            const int cc = wn * 32 + (lane & 31);
            const float b_r = Br[cur][kk][cc], b_i = Bi[cur][kk][cc];
            const int r0 = wm * 64 + (lane & 31);
            const float a0r = Ar[cur][kk][r0], a0i = Ai[cur][kk][r0];
            const float a1r = Ar[cur][kk][r0 + 32], a1i = Ai[cur][kk][r0 + 32];
            const float b_s = b_r + b_i, a0s = a0r + a0i, a1s = a1r + a1i;
            p10 = __builtin_amdgcn_mfma_f32_32x32x2f32(b_r, a0r, p10, 0, 0, 0);
            p11 = __builtin_amdgcn_mfma_f32_32x32x2f32(b_r, a1r, p11, 0, 0, 0);
            p20 = __builtin_amdgcn_mfma_f32_32x32x2f32(b_i, a0i, p20, 0, 0, 0);
            p21 = __builtin_amdgcn_mfma_f32_32x32x2f32(b_i, a1i, p21, 0, 0, 0);
            p30 = __builtin_amdgcn_mfma_f32_32x32x2f32(b_s, a0s, p30, 0, 0, 0);
            p31 = __builtin_amdgcn_mfma_f32_32x32x2f32(b_s, a1s, p31, 0, 0, 0);
        }
        if (more) stash(cur ^ 1);
        __syncthreads();
        cur ^= 1;
    }
    const float* Cz = g.C ? g.C + 2 * z * g.sC : nullptr;
    float* Dz = g.D + 2 * z * g.sD;
#pragma unroll
    for (int sub = 0; sub < 2; ++sub) {
        const floatx16& q1 = sub == 0 ? p10 : p11;
        const floatx16& q2 = sub == 0 ? p20 : p21;
        const floatx16& q3 = sub == 0 ? p30 : p31;
        const int row = row0 + wm * 64 + sub * 32 + (lane & 31);
        if (row >= m) continue;
        const int64_t prow = row + (g.band_cd && row >= g.rg0 ? g.rgw : 0);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int col = col0 + wn * 32 + (i / 4) * 8 + (lane >> 5) * 4 + (i % 4);
            if (col >= n) continue;
            const int64_t pcol = col + (g.band_cd && col >= g.cg0 ? g.cgw : 0);
            const float xr = q1[i] - q2[i], xi = q3[i] - q1[i] - q2[i];
            float re = g.ar * xr - g.ai * xi;
            float im = g.ar * xi + g.ai * xr;
            if (g.beta != 0.f) {
                const float* c = Cz + 2 * (prow + pcol * g.ldc);
                re += g.beta * c[0];
                im += g.beta * c[1];
            }
            float* d = Dz + 2 * (prow + pcol * g.ldd);
            d[0] = re;
            d[1] = im;
        }
    }
}

// (value, index) <- the better of its own and the DPP partner's: larger value, smaller index on ties
template <int CTRL>
__device__ inline void argmax_step(float& v, int& i) {
    const float ov = dpp_f<CTRL>(v);
    const int oi = __builtin_amdgcn_mov_dpp(i, CTRL, 0xF, 0xF, false);
    const bool better = (ov > v) | ((ov == v) & (oi < i));
    v = better ? ov : v;
    i = better ? oi : i;
}

// In-place inverse of n x n (n <= 64) complex64 blocks by Gauss-Jordan elimination with partial
// pivoting; one workgroup of 1024 threads per block (blockIdx.x), the block held in LDS.  Thread
// (lane c, wavefront w) owns column c of rows w, w+16, w+32, w+48.  Per elimination step k:
//  A. every wavefront reduces the 16 per-wavefront candidates for the pivot of column k (largest
//     modulus, smallest row on ties) across one row of lanes, and the scaled pivot row, the
//     multipliers (rows k and p exchanged) and the old row k are staged in LDS;
//  B. every thread updates its four entries (loads first, then stores); the owners of column k+1
//     leave their candidate for the next pivot.
// Two barriers per step.  The row exchanges become one column permutation, composed in registers
// and applied on the store.
__global__ __launch_bounds__(1024) void k_cinv_small(float* A, int64_t lda, int64_t stride, int n, int* info) {
    __shared__ float2 M[64][65];
    __shared__ float2 prow[64], pcol[64], oldk[64];
    __shared__ float cv[2][16];
    __shared__ int ci[2][16];
    __shared__ int piv[64], perm[64];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    float2* A2 = reinterpret_cast<float2*>(A) + stride * (int64_t)blockIdx.x;
    for (int c = wv; c < n; c += 16)
        if (lane < n) M[lane][c] = A2[lane + (int64_t)c * lda];
    __syncthreads();
    // candidates for the first pivot (column 0)
    if (lane == 0) {
        float best = -1.f;
        int bi = 0;
        for (int q = 0; q < 4; ++q) {
            const int i = wv + 16 * q;
            if (i < n) {
                const float v = M[i][0].x * M[i][0].x + M[i][0].y * M[i][0].y;
                if (v > best) { best = v; bi = i; }
            }
        }
        cv[0][wv] = best;
        ci[0][wv] = bi;
    }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        const int sl = k & 1;
        // lanes 0..15 of every wavefront take one candidate each and reduce them across the row of
        // 16 lanes (DPP); lane 0's result is the pivot
        float bv = lane < 16 ? cv[sl][lane] : -2.f;
        int bi = lane < 16 ? ci[sl][lane] : 0x7fffffff;
        argmax_step<kDppXor1>(bv, bi);
        argmax_step<kDppXor2>(bv, bi);
        argmax_step<kDppHalfMirror>(bv, bi);
        argmax_step<kDppMirror>(bv, bi);
        const float best = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(bv)));
        const int p = __builtin_amdgcn_readfirstlane(bi);
        if (tid == 0) {
            piv[k] = p;
            if (!(best > 0.f)) info[0] = k + 1;
        }
        {
            const float2 a = M[p][k];
            const float den = a.x * a.x + a.y * a.y;
            const float2 inv = make_float2(a.x / den, -a.y / den);
            if (tid < 64) {
                if (tid < n) {
                    const float2 v = M[p][tid];
                    prow[tid] = tid == k ? inv : make_float2(v.x * inv.x - v.y * inv.y, v.x * inv.y + v.y * inv.x);
                }
            } else if (tid < 128) {
                const int i = tid - 64;
                if (i < n) pcol[i] = M[i == k ? p : (i == p ? k : i)][k];
            } else if (tid < 192) {
                const int c = tid - 128;
                if (c < n) oldk[c] = M[k][c];
            }
        }
        __syncthreads();
        if (lane < n) {
            const int c = lane;
            const float2 r = prow[c];
            float2 v[4], f[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = wv + 16 * q;
                if (i < n) {
                    v[q] = i == p ? oldk[c] : M[i][c];
                    f[q] = pcol[i];
                }
            }
            float nb = -1.f;
            int ni = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = wv + 16 * q;
                if (i >= n) continue;
                float2 o;
                if (i == k) {
                    o = r;
                } else if (c == k) {
                    o = make_float2(-(f[q].x * r.x - f[q].y * r.y), -(f[q].x * r.y + f[q].y * r.x));
                } else {
                    o = make_float2(v[q].x - (f[q].x * r.x - f[q].y * r.y), v[q].y - (f[q].x * r.y + f[q].y * r.x));
                }
                M[i][c] = o;
                const float m2 = o.x * o.x + o.y * o.y;
                const bool better = (i > k) & (m2 > nb);
                nb = better ? m2 : nb;
                ni = better ? i : ni;
            }
            if (c == k + 1) {
                cv[sl ^ 1][wv] = nb;
                ci[sl ^ 1][wv] = ni;
            }
        }
        __syncthreads();
    }
    // undoing the row exchanges, last first, as column exchanges: out[:, j] = M[:, perm[j]]
    if (wv == 0) {
        int pj = lane;
        const int mypiv = lane < n ? piv[lane] : lane;
        for (int k = n - 1; k >= 0; --k) {
            const int pk = __shfl(mypiv, k, 64);
            const int vk = __shfl(pj, k, 64), vp = __shfl(pj, pk, 64);
            if (pk != k) {
                if (lane == k) pj = vp;
                if (lane == pk) pj = vk;
            }
        }
        perm[lane] = pj;
    }
    __syncthreads();
    for (int c = wv; c < n; c += 16)
        if (lane < n) A2[lane + (int64_t)c * lda] = M[lane][perm[c]];
}

__global__ void k_band_copy(const float2* __restrict__ src, int64_t lds, int64_t ss, float2* __restrict__ dst,
                            int64_t ldd, int64_t sd, int rows, int cols, int r0, int rw, int c0, int cw) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)rows * cols) return;
    const int r = (int)(e % rows), c = (int)(e / rows);
    const int64_t z = blockIdx.y;
    const int64_t pr = r + (r >= r0 ? rw : 0), pc = c + (c >= c0 ? cw : 0);
    dst[z * sd + pr + pc * ldd] = src[z * ss + r + (int64_t)c * lds];
}

// y = A x for batched n x n complex64 A (column-major, lda; matrix z at A + z sA, x at x + z sx):
// workgroup (row block, column chunk of 256) sums its chunk, then the chunks are added.
__global__ __launch_bounds__(256) void k_cgemv_part(const float2* __restrict__ A, int64_t lda, int64_t sA,
                                                    const float2* __restrict__ x, int64_t sx, int n,
                                                    float2* __restrict__ part, int64_t sp) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    const int c0 = blockIdx.y * 256, c1 = min(n, c0 + 256);
    const int64_t z = blockIdx.z;
    if (r >= n) return;
    const float2* Az = A + z * sA + r;
    const float2* xz = x + z * sx;
    float re = 0.f, im = 0.f;
    for (int k = c0; k < c1; ++k) {
        const float2 a = Az[(int64_t)k * lda], b = xz[k];
        re = fmaf(a.x, b.x, fmaf(-a.y, b.y, re));
        im = fmaf(a.x, b.y, fmaf(a.y, b.x, im));
    }
    part[z * sp + (int64_t)blockIdx.y * n + r] = make_float2(re, im);
}

// k_cgemv_part for a complex128 matrix (converted to FP32 on load), one matrix.
__global__ __launch_bounds__(256) void k_cgemv_part_f64src(const double2* __restrict__ A, int64_t lda,
                                                           const float2* __restrict__ x, int n,
                                                           float2* __restrict__ part) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    const int c0 = blockIdx.y * 256, c1 = min(n, c0 + 256);
    if (r >= n) return;
    const double2* Ar = A + r;
    float re = 0.f, im = 0.f;
    for (int k = c0; k < c1; ++k) {
        const double2 ad = Ar[(int64_t)k * lda];
        const float2 a = make_float2((float)ad.x, (float)ad.y), b = x[k];
        re = fmaf(a.x, b.x, fmaf(-a.y, b.y, re));
        im = fmaf(a.x, b.y, fmaf(a.y, b.x, im));
    }
    part[(int64_t)blockIdx.y * n + r] = make_float2(re, im);
}

// Padded gather of preconditioner blocks: workgroup (x, z) fills 256 consecutive entries (in
// column-major order) of slot z.  The transposed read of the symmetrisation is uncoalesced; the
// gather streams each block once and is small beside the inversion.
__global__ __launch_bounds__(256) void k_pad_gather(const PadBlock* __restrict__ blocks, int S, int sym,
                                                    float2* __restrict__ buf) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t SS = (int64_t)S * S;
    if (e >= SS) return;
    const int64_t z = blockIdx.y;
    const PadBlock b = blocks[z];
    const int r = (int)(e % S), c = (int)(e / S);
    float2 v = make_float2(r == c ? 1.f : 0.f, 0.f);
    if (r < b.n && c < b.n) {
        if (b.f64) {
            const double2* A = static_cast<const double2*>(b.src);
            double2 a = A[r + (int64_t)c * b.ld];
            if (sym) {
                const double2 t = A[c + (int64_t)r * b.ld];
                a = make_double2(0.5 * (a.x + t.x), 0.5 * (a.y + t.y));
            }
            v = make_float2((float)a.x, (float)a.y);
        } else {
            const float2* A = static_cast<const float2*>(b.src);
            v = A[r + (int64_t)c * b.ld];
            if (sym) {
                const float2 t = A[c + (int64_t)r * b.ld];
                v = make_float2(0.5f * (v.x + t.x), 0.5f * (v.y + t.y));
            }
        }
    }
    buf[z * SS + e] = v;
}

__global__ __launch_bounds__(256) void k_pad_scatter(const PadBlock* __restrict__ blocks, int S,
                                                     const float2* __restrict__ buf, int* __restrict__ flag) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t z = blockIdx.y;
    const PadBlock b = blocks[z];
    if (e >= (int64_t)b.n * b.n) return;
    const int r = (int)(e % b.n), c = (int)(e / b.n);
    const float2 v = buf[z * (int64_t)S * S + r + (int64_t)c * S];
    if (!isfinite(v.x) || !isfinite(v.y)) atomicOr(flag, 1);
    reinterpret_cast<float2*>(b.dst)[r + (int64_t)c * b.ld] = v;
}

// Single-trace operator for M = 1 through the MTF product: full = C x = [x; -Sigma x] (u_1 = -u_0)
// before it, y = R full_y = full_y[0:2E] - Sigma full_y[2E:4E] after it.
__global__ void k_stf_expand(const double2* __restrict__ x, const int8_t* __restrict__ sig, int64_t E,
                             double2* __restrict__ full) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 2 * E) return;
    const double2 v = x[e];
    const double sg = -(double)sig[e % E];
    full[e] = v;
    full[2 * E + e] = make_double2(sg * v.x, sg * v.y);
}

__global__ void k_stf_reduce(const double2* __restrict__ full, const int8_t* __restrict__ sig, int64_t E,
                             double2* __restrict__ y) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 2 * E) return;
    const double2 a = full[e], b = full[2 * E + e];
    const double sg = (double)sig[e % E];
    y[e] = make_double2(a.x - sg * b.x, a.y - sg * b.y);
}

__global__ void k_cgemv_sum(const float2* __restrict__ part, int n, int nch, int64_t sp, float2* __restrict__ y,
                            int64_t sy) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t z = blockIdx.y;
    if (r >= n) return;
    float re = 0.f, im = 0.f;
    for (int c = 0; c < nch; ++c) {
        const float2 v = part[z * sp + (int64_t)c * n + r];
        re += v.x;
        im += v.y;
    }
    y[z * sy + r] = make_float2(re, im);
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

void launch_matvec_sym_f64(const DomDesc* doms, const int4* stiles, int64_t ntiles, const double* T, const double* K,
                           const double* x, double* part, hipStream_t s) {
    hipLaunchKernelGGL(k_mv_sym<double>, dim3(gridn(ntiles, 4)), dim3(256), 0, s, doms, stiles, ntiles, T, K, x, part);
}

void launch_matvec_sym_f32(const DomDesc* doms, const int4* stiles, int64_t ntiles, const float* T, const float* K,
                           const double* x, double* part, hipStream_t s) {
    hipLaunchKernelGGL(k_mv_sym<float>, dim3(gridn(ntiles, 4)), dim3(256), 0, s, doms, stiles, ntiles, T, K, x, part);
}

void launch_near_diff_f64(const DomDesc* doms, const int32_t* dof_dom, int64_t ndof, const int64_t* ptr, const int32_t* col,
                          const double* T, const double* K, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_near_diff<double>, dim3(gridn(ndof, 256)), dim3(256), 0, s, doms, dof_dom, ndof, ptr, col, T, K,
                       out);
}

void launch_near_diff_f32(const DomDesc* doms, const int32_t* dof_dom, int64_t ndof, const int64_t* ptr, const int32_t* col,
                          const float* T, const float* K, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_near_diff<float>, dim3(gridn(ndof, 256)), dim3(256), 0, s, doms, dof_dom, ndof, ptr, col, T, K,
                       out);
}

void launch_matvec_sym_finish(const DomDesc* doms, const int32_t* dof_dom, int64_t ndof, const int32_t* dplus,
                              const int32_t* dminus, const double* gval, const int64_t* gcol, const int64_t* nptr,
                              const int32_t* ncol, const double* nval, const double* part, const double* x, double* y,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_mv_sym_finish, dim3(gridn(ndof, 64)), dim3(256), 0, s, doms, dof_dom, ndof, dplus, dminus, gval,
                       gcol, nptr, ncol, nval, part, x, y);
}

void launch_precond_sym(const DomDesc* doms, const int4* stiles, int64_t ntiles, const float* Tinv, const double* x,
                        double* part, hipStream_t s) {
    if (ntiles <= 0) return;
    hipLaunchKernelGGL(k_pc_sym, dim3((unsigned)ntiles), dim3(256), 0, s, doms, stiles, Tinv, x, part);
}

void launch_precond_sym_finish(const DomDesc* doms, const int32_t* dof_dom, int64_t ndof, const double* part,
                               const int2* slots, double* z, const int32_t* list, hipStream_t s) {
    if (ndof <= 0) return;
    hipLaunchKernelGGL(k_pc_sym_finish, dim3(gridn(ndof, 64)), dim3(256), 0, s, doms, dof_dom, ndof, part, slots, z, list);
}

void launch_zero_offdiag_f32(float* A, int E, const int32_t* cid, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_offdiag_f32, dim3(gridn((int64_t)E * E, 256)), dim3(256), 0, s, reinterpret_cast<float2*>(A),
                       E, cid);
}

void launch_symmetrize_f32(float* A, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_symmetrize_f32, dim3(gridn((int64_t)n * n, 256)), dim3(256), 0, s, A, n);
}

void launch_gs_residual(const DomDesc* doms, const int32_t* dof_dom, const int32_t* list, int64_t nlist,
                        const int32_t* dplus, const int32_t* dminus, const double* gval, const int64_t* gcol,
                        const int32_t* other_dom, const int32_t* dom_stage, int stage, const double* v, const double* z,
                        double* w, hipStream_t s) {
    if (nlist <= 0) return;
    hipLaunchKernelGGL(k_gs_residual, dim3(gridn(nlist, 256)), dim3(256), 0, s, doms, dof_dom, list, nlist, dplus, dminus,
                       gval, gcol, other_dom, dom_stage, stage, v, z, w);
}

void launch_dot2(const double* V, int64_t ldv, const int* jdev, int nvmax, const double* t, const double* U, int64_t n,
                 double* hpart, const DotPlan& d, bool c64, int nb, hipStream_t s) {
    const dim3 grid((unsigned)d.grid, 1, (unsigned)nb);
    if (c64)
        hipLaunchKernelGGL(k_dot2_c64, grid, dim3(256), 0, s, reinterpret_cast<const float2*>(V), ldv, jdev, nvmax, t, U,
                           n, hpart, d.units, d.cmin, d.kmax);
    else
        hipLaunchKernelGGL(k_dot2, grid, dim3(256), 0, s, reinterpret_cast<const double2*>(V), ldv, jdev, nvmax, t, n,
                           hpart, d.units, d.cmin, d.kmax);
}

void launch_reduce2(const double* hpart, const int* jdev, int nvmax, const DotPlan& d, double* S, double* Z, int nb,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_reduce2, dim3(gridn(nvmax + 1, 4), (unsigned)nb), dim3(256), 0, s, hpart, jdev, nvmax, d.units,
                       d.cmin, d.kmax, S, Z);
}

void launch_dcgs_col(double* H, int64_t ldh, int64_t hstride, const double* S, const double* Z, const double* hg, int nct,
                     const int* jdev, int nvmax, double* scal, int last, double* R, int64_t rstride, int nb, hipStream_t s) {
    hipLaunchKernelGGL(k_dcgs_col, dim3(gridn(nvmax + 1, 256), (unsigned)nb), dim3(256), 0, s, H, ldh, hstride, S, Z, hg,
                       nct, jdev, nvmax, scal, last, R, rstride);
}

void launch_update2(const double* V_, int64_t ldv, const int* jdev, int* jnext, int nvmax, const double* S,
                    const double* Z, const double* t, double* unext, int64_t n, double* part, int ng,
                    const double* zsrc, double* zdst, double* H, int64_t ldh, int64_t hstride, double* hg, int nct,
                    double* R, int64_t rstride, bool c64, int nb, hipStream_t s) {
    double* V = const_cast<double*>(V_);
    const int nxp = (int)gridn(n, 256);
    const int tiles = ((nvmax + 1 + 63) / 64) * ((nvmax + 63) / 64);
    const int nhx = std::max(1, (std::min(tiles, 256) + ng - 1) / ng);
    const dim3 gp((unsigned)(nxp + nhx), (unsigned)ng, (unsigned)nb);
    const int nxa = (int)gridn(n, 256);
    const int ncx = (int)gridn(nvmax + 1, 256);
    const dim3 ga((unsigned)(nxa + ncx), (unsigned)nb);
    if (c64) {
        float2* Vc = reinterpret_cast<float2*>(V);
        hipLaunchKernelGGL(k_update2_part<float2>, gp, dim3(256), 0, s, Vc, ldv, jdev, nvmax, S, Z, part, n, nxp, H, ldh,
                           hstride, nct, hg);
        hipLaunchKernelGGL(k_update2_apply<float2>, ga, dim3(256), 0, s, part, ng, Vc, ldv, jdev, jnext, t, unext, n,
                           zsrc, zdst, nxa, nvmax, S, Z, H, ldh, hstride, hg, nct, R, rstride);
    } else {
        double2* Vd = reinterpret_cast<double2*>(V);
        hipLaunchKernelGGL(k_update2_part<double2>, gp, dim3(256), 0, s, Vd, ldv, jdev, nvmax, S, Z, part, n, nxp, H,
                           ldh, hstride, nct, hg);
        hipLaunchKernelGGL(k_update2_apply<double2>, ga, dim3(256), 0, s, part, ng, Vd, ldv, jdev, jnext, t, unext, n,
                           zsrc, zdst, nxa, nvmax, S, Z, H, ldh, hstride, hg, nct, R, rstride);
    }
}

void launch_set_int(int* p, int v, hipStream_t s) { hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, p, v); }

void launch_stage_cols(const double* H, int64_t ldh, int64_t hstride, const int* jdev, int back, int cnt, double* Hst,
                       int nb, hipStream_t s) {
    hipLaunchKernelGGL(k_stage_cols, dim3(gridn(2 * ldh * cnt, 256), (unsigned)nb), dim3(256), 0, s, H, ldh, hstride, jdev,
                       back, cnt, Hst);
}


void launch_trsv_upper(const double* R, int64_t ldh, int64_t rstride, const int* cnt, double* y, int64_t ystride,
                       int* info, int nb, hipStream_t s) {
    hipLaunchKernelGGL(k_trsv_upper, dim3((unsigned)nb), dim3(1024), 0, s, R, ldh, rstride, cnt, y, ystride, info);
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

void launch_copy_block_f64_to_f32(const double* src, float* dst, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_d2f, dim3(gridn(n, 256)), dim3(256), 0, s, src, dst, n);
}

void launch_cgemm_f32(const CGemm& g, hipStream_t s) {
    if (g.m <= 0 || g.n <= 0 || g.batch <= 0) return;
    hipLaunchKernelGGL(k_cgemm_mfma, dim3(gridn(g.m, 128), gridn(g.n, 64), (unsigned)g.batch), dim3(256), 0, s, g);
}

void launch_band_copy_f32(const float* src, int64_t lds, int64_t ss, float* dst, int64_t ldd, int64_t sd, int rows,
                          int cols, int r0, int rw, int c0, int cw, int batch, hipStream_t s) {
    if (rows <= 0 || cols <= 0 || batch <= 0) return;
    hipLaunchKernelGGL(k_band_copy, dim3(gridn((int64_t)rows * cols, 256), (unsigned)batch), dim3(256), 0, s,
                       reinterpret_cast<const float2*>(src), lds, ss, reinterpret_cast<float2*>(dst), ldd, sd, rows,
                       cols, r0, rw, c0, cw);
}

void launch_cgemv_f32(const float* A, int64_t lda, int64_t sA, const float* x, int64_t sx, int n, int batch, float* part,
                      float* y, int64_t sy, hipStream_t s) {
    if (n <= 0 || batch <= 0) return;
    const int nch = (n + 255) / 256;
    const int64_t sp = (int64_t)nch * n;
    hipLaunchKernelGGL(k_cgemv_part, dim3((unsigned)nch, (unsigned)nch, (unsigned)batch), dim3(256), 0, s,
                       reinterpret_cast<const float2*>(A), lda, sA, reinterpret_cast<const float2*>(x), sx, n,
                       reinterpret_cast<float2*>(part), sp);
    hipLaunchKernelGGL(k_cgemv_sum, dim3(gridn(n, 256), (unsigned)batch), dim3(256), 0, s,
                       reinterpret_cast<const float2*>(part), n, nch, sp, reinterpret_cast<float2*>(y), sy);
}

int launch_cinv_small_f32(float* A, int64_t lda, int64_t stride, int n, int batch, int* info, hipStream_t s) {
    if (n <= 0 || n > 64 || batch <= 0) return -1;
    hipLaunchKernelGGL(k_cinv_small, dim3((unsigned)batch), dim3(1024), 0, s, A, lda, stride, n, info);
    return 0;
}

void launch_pad_gather(const PadBlock* blocks, int nblocks, int S, int sym, float* buf, hipStream_t s) {
    if (nblocks <= 0) return;
    hipLaunchKernelGGL(k_pad_gather, dim3(gridn((int64_t)S * S, 256), (unsigned)nblocks), dim3(256), 0, s, blocks, S,
                       sym, reinterpret_cast<float2*>(buf));
}

void launch_pad_scatter(const PadBlock* blocks, int nblocks, int S, const float* buf, int* flag, hipStream_t s) {
    if (nblocks <= 0) return;
    hipLaunchKernelGGL(k_pad_scatter, dim3(gridn((int64_t)S * S, 256), (unsigned)nblocks), dim3(256), 0, s, blocks, S,
                       reinterpret_cast<const float2*>(buf), flag);
}

void launch_cgemv_f64src(const double* A, int64_t lda, const float* x, int n, float* part, float* y, hipStream_t s) {
    if (n <= 0) return;
    const int nch = (n + 255) / 256;
    hipLaunchKernelGGL(k_cgemv_part_f64src, dim3((unsigned)nch, (unsigned)nch), dim3(256), 0, s,
                       reinterpret_cast<const double2*>(A), lda, reinterpret_cast<const float2*>(x), n,
                       reinterpret_cast<float2*>(part));
    hipLaunchKernelGGL(k_cgemv_sum, dim3(gridn(n, 256), 1u), dim3(256), 0, s, reinterpret_cast<const float2*>(part), n,
                       nch, (int64_t)nch * n, reinterpret_cast<float2*>(y), (int64_t)0);
}

void launch_stf_expand(const double* x, const int8_t* sig, int64_t E, double* full, hipStream_t s) {
    hipLaunchKernelGGL(k_stf_expand, dim3(gridn(2 * E, 256)), dim3(256), 0, s, reinterpret_cast<const double2*>(x), sig,
                       E, reinterpret_cast<double2*>(full));
}

void launch_stf_reduce(const double* full, const int8_t* sig, int64_t E, double* y, hipStream_t s) {
    hipLaunchKernelGGL(k_stf_reduce, dim3(gridn(2 * E, 256)), dim3(256), 0, s, reinterpret_cast<const double2*>(full),
                       sig, E, reinterpret_cast<double2*>(y));
}

void launch_nonfinite_check(const float* A, int64_t n, int* flag, hipStream_t s) {
    hipLaunchKernelGGL(k_nonfinite, dim3(gridn(n, 256)), dim3(256), 0, s, A, n, flag);
}

}  // namespace mtf
