// Galerkin assembly kernels for gfx950: EFIO T and MFIO K on RWG_i, transmission
// blocks, plane-wave right-hand sides and the far field.
//
// Weak forms (eq. boundary_operators tested in the twisted pairing of eq.
// self_duality_identity, integrated by parts on the closed Gamma_i):
//   T[m,n] = -i k  sum_q sum_r w_q w_r G(r_qr) [ phi_n(y_r).phi_m(x_q) - k^-2 div phi_n div phi_m ]
//   K[m,n] = -     sum_q sum_r w_q w_r grad_x G(x_q, y_r) . ( phi_n(y_r) x phi_m(x_q) )
// with G = exp(ikr)/(4 pi r) and grad_x G = (x - y) exp(ikr)(ikr - 1)/(4 pi r^3).
//
// Each triangle pair is reduced to 18 complex moments of the kernel in
// per-triangle local coordinates (x' = x - c_x, y' = y - c_y); RWG functions are
// affine, phi_a(x) = c_a (x' - p'_a), so the 3 x 3 local blocks of T and K follow
// exactly from the moments in an epilogue:
//   T_ab = -i k c_a c_b [ Mxy - q'_b.Mx - p'_a.My + (p'_a.q'_b - 4/k^2) M0 ]
//   K_ab = -c_a c_b [ -D.Nxy - p'_a.(D x Ny) - p'_a.Nxy - q'_b.(Nx x D) + q'_b.Nxy
//                     + (q'_b x p'_a).(D N0 + Nx - Ny) ]
// with D = c_x - c_y, M* the moments of w G and N* those of w g (grad_x G = g (x - y)):
//   M0 = sum wG, Mx = sum wG x', My = sum wG y', Mxy = sum wG x'.y',
//   N0 = sum wg, Nx = sum wg x', Ny = sum wg y', Nxy = sum wg x' x y'.
#include "device.h"

#include <algorithm>
#include <stdexcept>
#include <cmath>
#include <type_traits>

namespace mtf {

namespace {

constexpr double kInv4Pi = 0.07957747154594767;   // 1 / (4 pi)

template <typename R>
__device__ inline void atomic_add(R* p, R v) {
    unsafeAtomicAdd(p, v);
}

__global__ void k_fill(double* p, int64_t n, double v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

__global__ void k_fill_f(float* p, int64_t n, float v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

struct Rule6 {
    double bary[6][3];
    double w[6];
};

__global__ void k_tri_setup(const double* __restrict__ xyz, const int32_t* __restrict__ verts, int64_t nrec,
                            Rule6 rule, TriGeom* __restrict__ geom) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrec) return;
    double P[3][3];
    for (int a = 0; a < 3; ++a) {
        int32_t v = verts[3 * r + a];
        for (int k = 0; k < 3; ++k) P[a][k] = xyz[3 * (int64_t)v + k];
    }
    TriGeom g;
    for (int k = 0; k < 3; ++k) g.c[k] = (P[0][k] + P[1][k] + P[2][k]) * (1.0 / 3.0);
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 3; ++k) g.p[3 * a + k] = P[a][k] - g.c[k];
    double e1[3], e2[3];
    for (int k = 0; k < 3; ++k) { e1[k] = P[1][k] - P[0][k]; e2[k] = P[2][k] - P[0][k]; }
    double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    double twoA = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    g.area = 0.5 * twoA;
    for (int k = 0; k < 3; ++k) g.n[k] = cr[k] / twoA;
    for (int a = 0; a < 3; ++a) {
        const double* u = P[(a + 1) % 3];
        const double* v = P[(a + 2) % 3];
        double l = sqrt((v[0] - u[0]) * (v[0] - u[0]) + (v[1] - u[1]) * (v[1] - u[1]) + (v[2] - u[2]) * (v[2] - u[2]));
        g.coef[a] = l / twoA;
    }
    for (int q = 0; q < 6; ++q) {
        for (int k = 0; k < 3; ++k) {
            double x = rule.bary[q][0] * P[0][k] + rule.bary[q][1] * P[1][k] + rule.bary[q][2] * P[2][k];
            g.q[3 * q + k] = x - g.c[k];
        }
        g.w[q] = rule.w[q] * g.area;
    }
    g.pad = 0.0;
    geom[r] = g;
}

// ---------------------------------------------------------------------------
// separated pairs
// ---------------------------------------------------------------------------

template <typename R>
struct LRec {
    R p[9];
    R q[18];
    R w[6];
    R coef[3];
    double c[3];
    int32_t v[3];
    int32_t dof[3];
    int32_t sg[3];
};

// sin x and cos x in FP64 for the phases k r of the kernel: the reduction of Cody & Waite
// (Software Manual for the Elementary Functions, 1980), x = n pi/2 + t with pi/2 split into two
// 33-bit parts and a remainder (so n * part is exact for |n| < 2^20), then the Taylor series of
// sin t to t^15 and of cos t to t^16 on |t| <= pi/4, whose truncation error is below 7e-17 relative;
// quadrant n mod 4 picks and signs the two.  Valid for |x| < 2^20 pi/2 (about 1.6e6): the kernel
// phases k_i r stay below k_i times the mesh diameter, which mtf_set_materials limits to 1e6.  The
// parts of pi/2 are its 33-bit truncation, the next 33 bits, and the rounded rest.
__device__ inline void sincos_cw(double x, double* sp, double* cp) {
    constexpr double kTwoOverPi = 0.6366197723675814;
    constexpr double kP1 = 1.5707963267341256, kP2 = 6.077100506303966e-11, kP3 = 2.0222662487959506e-21;
    const double n = rint(x * kTwoOverPi);
    double t = fma(-n, kP1, x);
    t = fma(-n, kP2, t);
    t = fma(-n, kP3, t);
    const double t2 = t * t;
    double ps = -1.0 / 1307674368000.0;           // -1/15!
    ps = fma(ps, t2, 1.0 / 6227020800.0);         //  1/13!
    ps = fma(ps, t2, -1.0 / 39916800.0);          // -1/11!
    ps = fma(ps, t2, 1.0 / 362880.0);             //  1/9!
    ps = fma(ps, t2, -1.0 / 5040.0);              // -1/7!
    ps = fma(ps, t2, 1.0 / 120.0);                //  1/5!
    ps = fma(ps, t2, -1.0 / 6.0);                 // -1/3!
    const double sn = fma(ps * t2, t, t);
    double pc = 1.0 / 20922789888000.0;           //  1/16!
    pc = fma(pc, t2, -1.0 / 87178291200.0);       // -1/14!
    pc = fma(pc, t2, 1.0 / 479001600.0);          //  1/12!
    pc = fma(pc, t2, -1.0 / 3628800.0);           // -1/10!
    pc = fma(pc, t2, 1.0 / 40320.0);              //  1/8!
    pc = fma(pc, t2, -1.0 / 720.0);               // -1/6!
    pc = fma(pc, t2, 1.0 / 24.0);                 //  1/4!
    pc = fma(pc, t2, -0.5);                       // -1/2!
    const double cs = fma(pc, t2, 1.0);
    const int q = (int)n & 3;
    const double a = (q & 1) ? cs : sn, b = (q & 1) ? sn : cs;
    *sp = (q & 2) ? -a : a;
    *cp = ((q + 1) & 2) ? -b : b;
}

// 1/sqrt(x) in FP64 (x > 0): the hardware reciprocal square root estimate refined by two Newton
// steps y <- y + (y/2)(1 - x y^2), each doubling the number of correct bits.
__device__ inline double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-x * y, y, 1.0);
    return fma(0.5 * y, e, y);
}

template <typename R>
__device__ inline void kernel_values(R kr, R rinv, R wr, R& Gre, R& Gim, R& gre, R& gim);

template <>
__device__ inline void kernel_values<double>(double kr, double rinv, double wr, double& Gre, double& Gim,
                                             double& gre, double& gim) {
    double s, c;
    sincos_cw(kr, &s, &c);
    double a = wr * kInv4Pi * rinv;
    Gre = c * a;
    Gim = s * a;
    double b = a * rinv * rinv;
    gre = (-c - kr * s) * b;
    gim = (kr * c - s) * b;
}

template <>
__device__ inline void kernel_values<float>(float kr, float rinv, float wr, float& Gre, float& Gim,
                                            float& gre, float& gim) {
    float s, c;
    __sincosf(kr, &s, &c);
    float a = wr * (float)kInv4Pi * rinv;
    Gre = c * a;
    Gim = s * a;
    float b = a * rinv * rinv;
    gre = (-c - kr * s) * b;
    gim = (kr * c - s) * b;
}

template <typename R>
__device__ inline R rsqrt_r(R x);
template <>
__device__ inline double rsqrt_r<double>(double x) { return rsqrt_nr(x); }
template <>
__device__ inline float rsqrt_r<float>(float x) { return __frsqrt_rn(x); }

// Moments of one pair (complex values as re/im pairs).
template <typename R>
struct Moments {
    R M0[2], Mx[3][2], My[3][2], Mxy[2];
    R N0[2], Nx[3][2], Ny[3][2], Nxy[3][2];
};

template <typename R>
__device__ inline void zero_moments(Moments<R>& m) {
    m.M0[0] = m.M0[1] = m.Mxy[0] = m.Mxy[1] = m.N0[0] = m.N0[1] = R(0);
    for (int k = 0; k < 3; ++k)
        for (int c = 0; c < 2; ++c) m.Mx[k][c] = m.My[k][c] = m.Nx[k][c] = m.Ny[k][c] = m.Nxy[k][c] = R(0);
}

// Local blocks from the moments, with RWG signs, handed to sink(a, b, T re, T im, K re, K im).
template <typename R, typename Sink>
__device__ __attribute__((always_inline)) inline void epilogue(const Moments<R>& m, const R* pa_all, const R* qb_all,
                                                               const R* ca, const R* cb, const R* D, R k,
                                                               const int32_t* sgx, const int32_t* sgy, Sink sink) {
    const R four_over_k2 = R(4) / (k * k);
    for (int a = 0; a < 3; ++a) {
        const R* Pa = pa_all + 3 * a;
        // p'_a . My  and  p'_a . (D x Ny) + p'_a . Nxy  (independent of b)
        R pMy[2], pK[2];
        R DxNy[3][2];
        for (int c = 0; c < 2; ++c) {
            DxNy[0][c] = D[1] * m.Ny[2][c] - D[2] * m.Ny[1][c];
            DxNy[1][c] = D[2] * m.Ny[0][c] - D[0] * m.Ny[2][c];
            DxNy[2][c] = D[0] * m.Ny[1][c] - D[1] * m.Ny[0][c];
            pMy[c] = Pa[0] * m.My[0][c] + Pa[1] * m.My[1][c] + Pa[2] * m.My[2][c];
            pK[c] = Pa[0] * (DxNy[0][c] + m.Nxy[0][c]) + Pa[1] * (DxNy[1][c] + m.Nxy[1][c]) +
                    Pa[2] * (DxNy[2][c] + m.Nxy[2][c]);
        }
        for (int b = 0; b < 3; ++b) {
            const R* Qb = qb_all + 3 * b;
            const R pq = Pa[0] * Qb[0] + Pa[1] * Qb[1] + Pa[2] * Qb[2];
            R t[2], s[2];
            const R QxP[3] = {Qb[1] * Pa[2] - Qb[2] * Pa[1], Qb[2] * Pa[0] - Qb[0] * Pa[2], Qb[0] * Pa[1] - Qb[1] * Pa[0]};
            for (int c = 0; c < 2; ++c) {
                t[c] = m.Mxy[c] - (Qb[0] * m.Mx[0][c] + Qb[1] * m.Mx[1][c] + Qb[2] * m.Mx[2][c]) - pMy[c] +
                       (pq - four_over_k2) * m.M0[c];
                // Nx x D
                const R NxD0 = m.Nx[1][c] * D[2] - m.Nx[2][c] * D[1];
                const R NxD1 = m.Nx[2][c] * D[0] - m.Nx[0][c] * D[2];
                const R NxD2 = m.Nx[0][c] * D[1] - m.Nx[1][c] * D[0];
                const R DN = -(D[0] * m.Nxy[0][c] + D[1] * m.Nxy[1][c] + D[2] * m.Nxy[2][c]);
                const R qterm = Qb[0] * (m.Nxy[0][c] - NxD0) + Qb[1] * (m.Nxy[1][c] - NxD1) + Qb[2] * (m.Nxy[2][c] - NxD2);
                const R v0 = D[0] * m.N0[c] + m.Nx[0][c] - m.Ny[0][c];
                const R v1 = D[1] * m.N0[c] + m.Nx[1][c] - m.Ny[1][c];
                const R v2 = D[2] * m.N0[c] + m.Nx[2][c] - m.Ny[2][c];
                s[c] = DN - pK[c] + qterm + QxP[0] * v0 + QxP[1] * v1 + QxP[2] * v2;
            }
            const R f = ca[a] * cb[b] * R(sgx[a] * sgy[b]);
            // T = -i k f t ;  K = -f s
            const R Tre = k * f * t[1];
            const R Tim = -k * f * t[0];
            const R Kre = -f * s[0];
            const R Kim = -f * s[1];
            sink(a, b, Tre, Tim, Kre, Kim);
        }
    }
}

// Scatter of one pair's local blocks straight into T and K (global atomics).
template <typename RO>
struct GlobalSink {
    const int32_t* dofx;
    const int32_t* dofy;
    int64_t mat0;
    int32_t E;
    RO* T;
    RO* K;
    template <typename R>
    __device__ void operator()(int a, int b, R Tre, R Tim, R Kre, R Kim) const {
        const int64_t idx = 2 * (mat0 + (int64_t)dofx[a] + (int64_t)dofy[b] * E);
        atomic_add(T + idx, (RO)Tre);
        atomic_add(T + idx + 1, (RO)Tim);
        atomic_add(K + idx, (RO)Kre);
        atomic_add(K + idx + 1, (RO)Kim);
    }
};

// Local accumulator of a tile of separated pairs: slot 3 t + a is local dof a of tile
// triangle t (3 TX test and 3 TY trial slots); a dof that appears in several slots is kept in the first of them, so
// the tile's pairs add into LDS and only its distinct (test dof, trial dof) entries reach T and K.
// In FP64 it holds one operator at a time: the pairs add their T entries, the tile scatters them,
// then the same for K (the moments stay in registers in between); half the LDS of holding both
// lets three workgroups share a CU instead of one.  In FP32 both operators are held at once (the
// moments held across the extra barriers would cost more registers than the LDS saved).
template <typename R>
constexpr int kAccOps = std::is_same<R, double>::value ? 1 : 2;

// Shape of a tile of separated pairs: TX test triangles x TY trial triangles, one pair per
// thread, and the minimum number of resident waves per SIMD asked of the compiler (OCC; 1 leaves the
// register budget to the compiler).  The variants are the autotuner's choices (tile_variant()).
// SYM: the tile list holds each unordered pair of triangle groups once (test group <= trial group,
// TX == TY) and the tile evaluates the quadrature of each unordered triangle pair once, for both
// orders: the moments of the reversed pair (Y, X) are those of (X, Y) with Mx <-> My, Nx <-> Ny,
// Nxy -> -Nxy and D -> -D (the kernels depend on |x - y| only), so T(Y, X) = T(X, Y) (written to
// both positions) and K(Y, X) is a second epilogue on the relabelled moments.  In a tile on the
// diagonal only the pairs with test triangle < trial triangle are evaluated.
template <int TX_, int TY_, int OCC_, bool SYM_ = false>
struct TileShape {
    static constexpr int TX = TX_, TY = TY_, NT = TX_ * TY_, OCC = OCC_;
    static constexpr int SX = 3 * TX_, SY = 3 * TY_;     // accumulator slots per side
    static constexpr bool SYM = SYM_;
    static_assert(!SYM_ || TX_ == TY_, "a symmetric tile needs equal test and trial groups");
};

template <typename R, typename S>
struct TileAcc {
    R v[kAccOps<R>][S::SX][S::SY][2];    // [operator][test slot][trial slot][re, im]
    int first_x[S::SX], first_y[S::SY];  // first slot of the same dof, -1 when unused
    int order_x[S::SX], order_y[S::SY];  // the distinct slots of each side by increasing dof
    int nx, ny;                          // number of distinct test and trial dofs
};

// WHICH 0: T into v[0]; 1: K into v[0]; 2: T into v[0] and K into v[1]
template <typename R, typename S, int WHICH>
struct LdsSink {
    TileAcc<R, S>* acc;
    int sx, sy;                          // 3 * tile triangle of the pair, test and trial side
    __device__ void operator()(int a, int b, R Tre, R Tim, R Kre, R Kim) const {
        const int x = acc->first_x[sx + a], y = acc->first_y[sy + b];
        if constexpr (WHICH == 2) {
            atomicAdd(&acc->v[0][x][y][0], Tre);
            atomicAdd(&acc->v[0][x][y][1], Tim);
            atomicAdd(&acc->v[kAccOps<R> - 1][x][y][0], Kre);
            atomicAdd(&acc->v[kAccOps<R> - 1][x][y][1], Kim);
        } else {
            atomicAdd(&acc->v[0][x][y][0], WHICH == 0 ? Tre : Kre);
            atomicAdd(&acc->v[0][x][y][1], WHICH == 0 ? Tim : Kim);
        }
    }
};

// K of the reversed pair (test dof a on the trial-side triangle, trial dof b on the test-side one),
// added into v[0] at (test-side slot of b, trial-side slot of a); scattered to (row of a, column of b)
template <typename R, typename S>
struct LdsSinkRev {
    TileAcc<R, S>* acc;
    int sx, sy;
    __device__ void operator()(int a, int b, R, R, R Kre, R Kim) const {
        const int x = acc->first_x[sx + b], y = acc->first_y[sy + a];
        atomicAdd(&acc->v[0][x][y][0], Kre);
        atomicAdd(&acc->v[0][x][y][1], Kim);
    }
};

// One TX x TY tile of separated pairs (tile = (subdomain, first test triangle, first trial
// triangle)); all S::NT threads of the workgroup must call it (it holds workgroup barriers); pairs
// outside Gamma_i or touching are skipped by predication.  The pairs add into the tile's LDS
// accumulator, which is then scattered into T and K.
template <typename R, typename S>
__device__ __attribute__((always_inline)) inline void regular_tile(const int4 tile, const DomDesc* __restrict__ doms, const TriGeom* __restrict__ geom,
                                    const int32_t* __restrict__ verts, const int32_t* __restrict__ tdof,
                                    const int8_t* __restrict__ tsign, R* __restrict__ T, R* __restrict__ K,
                                    LRec<R>* rec, TileAcc<R, S>* acc) {
    constexpr int TX = S::TX, TY = S::TY, NT = S::NT, SX = S::SX, SY = S::SY;
    const DomDesc dd = doms[tile.x];
    const int tid = threadIdx.x;
    if (tid < TX + TY) {
        const int lt = (tid < TX) ? tile.y + tid : tile.z + (tid - TX);
        if (lt < dd.T) {
            const int64_t r = dd.rec0 + lt;
            const TriGeom& g = geom[r];
            LRec<R>& L = rec[tid];
            for (int i = 0; i < 9; ++i) L.p[i] = (R)g.p[i];
            for (int i = 0; i < 18; ++i) L.q[i] = (R)g.q[i];
            for (int i = 0; i < 6; ++i) L.w[i] = (R)g.w[i];
            for (int i = 0; i < 3; ++i) {
                L.coef[i] = (R)g.coef[i];
                L.c[i] = g.c[i];
                L.v[i] = verts[3 * r + i];
                L.dof[i] = tdof[3 * r + i];
                L.sg[i] = tsign[3 * r + i];
            }
        }
    }
    {
        R* z = &acc->v[0][0][0][0];
        for (int e = tid; e < kAccOps<R> * SX * SY * 2; e += NT) z[e] = R(0);
    }
    __syncthreads();
    for (int e = tid; e < SX + SY; e += NT) {
        // first slot holding the same dof (slots of triangles past the end of Gamma_i: -1)
        const int side = e < SX ? 0 : 1, sl = e < SX ? e : e - SX;
        const int t0 = side == 0 ? tile.y : tile.z, base = side == 0 ? 0 : TX;
        int f = -1;
        if (t0 + sl / 3 < dd.T) {
            const int d = rec[base + sl / 3].dof[sl % 3];
            f = sl;
            for (int q = 0; q < sl; ++q)
                if (rec[base + q / 3].dof[q % 3] == d) { f = q; break; }
        }
        if (side == 0) acc->first_x[sl] = f;
        else acc->first_y[sl] = f;
    }
    __syncthreads();
    // compact lists of the distinct slots for the scatter, the test dofs in increasing order: the
    // lanes of a wavefront then add into neighbouring rows of one column of T or K, and their
    // atomics share cache lines
    for (int e = tid; e < SX + SY; e += NT) {
        if (e < SX) {
            if (acc->first_x[e] != e) continue;
            const int d = rec[e / 3].dof[e % 3];
            int rank = 0;
            for (int q = 0; q < SX; ++q)
                if (acc->first_x[q] == q && rec[q / 3].dof[q % 3] < d) ++rank;
            acc->order_x[rank] = e;
        } else {
            const int sl = e - SX;
            if (acc->first_y[sl] != sl) continue;
            const int d = rec[TX + sl / 3].dof[sl % 3];
            int rank = 0;
            for (int q = 0; q < SY; ++q)
                if (acc->first_y[q] == q && rec[TX + q / 3].dof[q % 3] < d) ++rank;
            acc->order_y[rank] = sl;
        }
    }
    if (tid == 0) {
        int nx = 0, ny = 0;
        for (int q = 0; q < SX; ++q) nx += acc->first_x[q] == q;
        for (int q = 0; q < SY; ++q) ny += acc->first_y[q] == q;
        acc->nx = nx;
        acc->ny = ny;
    }
    __syncthreads();
    const int ix = tid / TY, iy = tid % TY;
    const int tx = tile.y + ix, ty = tile.z + iy;
    bool valid = tx < dd.T && ty < dd.T;
    if (S::SYM && tile.y == tile.z && ix >= iy) valid = false;     // the other order of a diagonal tile
    const LRec<R>& X = rec[ix];
    const LRec<R>& Y = rec[TX + iy];
    if (valid) {
        // touching pairs belong to the Sauter-Schwab path
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                if (X.v[a] == Y.v[b]) valid = false;
    }
    Moments<R> mom;
    zero_moments(mom);
    if (valid) {
        const R k = (R)dd.k;
        R D[3];
        for (int i = 0; i < 3; ++i) D[i] = (R)(X.c[i] - Y.c[i]);
        Moments<R>& m = mom;
        // FP64: one outer quadrature point at a time (the FP64 phase evaluations would otherwise spill);
        // at three resident waves per SIMD (168 VGPRs) also two inner points at a time, which costs
        // a few spilled registers outside the loop but hides more FP64 latency (64 clusters: 0.49 s
        // against 0.57 s at two waves with all six inner points unrolled)
        constexpr int kUnrollQ = std::is_same<R, double>::value ? 1 : 6;
        constexpr int kUnrollR = std::is_same<R, double>::value && S::OCC >= 3 ? 2 : 6;
#pragma unroll kUnrollQ
        for (int q = 0; q < 6; ++q) {
            const R x0 = X.q[3 * q], x1 = X.q[3 * q + 1], x2 = X.q[3 * q + 2];
            const R wq = X.w[q];
            const R dx0 = D[0] + x0, dx1 = D[1] + x1, dx2 = D[2] + x2;
            R s0[2] = {0, 0}, sy[3][2] = {{0, 0}, {0, 0}, {0, 0}};
            R t0[2] = {0, 0}, ty[3][2] = {{0, 0}, {0, 0}, {0, 0}};
#pragma unroll kUnrollR
            for (int r = 0; r < 6; ++r) {
                const R y0 = Y.q[3 * r], y1 = Y.q[3 * r + 1], y2 = Y.q[3 * r + 2];
                const R d0 = dx0 - y0, d1 = dx1 - y1, d2 = dx2 - y2;
                const R r2 = d0 * d0 + d1 * d1 + d2 * d2;
                const R rinv = rsqrt_r(r2);
                const R kr = k * (r2 * rinv);
                R Gre, Gim, gre, gim;
                kernel_values<R>(kr, rinv, Y.w[r], Gre, Gim, gre, gim);
                s0[0] += Gre; s0[1] += Gim;
                t0[0] += gre; t0[1] += gim;
                sy[0][0] += Gre * y0; sy[0][1] += Gim * y0;
                sy[1][0] += Gre * y1; sy[1][1] += Gim * y1;
                sy[2][0] += Gre * y2; sy[2][1] += Gim * y2;
                ty[0][0] += gre * y0; ty[0][1] += gim * y0;
                ty[1][0] += gre * y1; ty[1][1] += gim * y1;
                ty[2][0] += gre * y2; ty[2][1] += gim * y2;
            }
            const R xv[3] = {x0, x1, x2};
            for (int c = 0; c < 2; ++c) {
                m.M0[c] += wq * s0[c];
                m.N0[c] += wq * t0[c];
                m.Mxy[c] += wq * (x0 * sy[0][c] + x1 * sy[1][c] + x2 * sy[2][c]);
                for (int i = 0; i < 3; ++i) {
                    m.Mx[i][c] += wq * s0[c] * xv[i];
                    m.My[i][c] += wq * sy[i][c];
                    m.Nx[i][c] += wq * t0[c] * xv[i];
                    m.Ny[i][c] += wq * ty[i][c];
                }
                m.Nxy[0][c] += wq * (x1 * ty[2][c] - x2 * ty[1][c]);
                m.Nxy[1][c] += wq * (x2 * ty[0][c] - x0 * ty[2][c]);
                m.Nxy[2][c] += wq * (x0 * ty[1][c] - x1 * ty[0][c]);
            }
        }
        epilogue<R>(m, X.p, Y.p, X.coef, Y.coef, D, k, X.sg, Y.sg,
                    LdsSink<R, S, kAccOps<R> == 2 ? 2 : 0>{acc, 3 * ix, 3 * iy});
    }
    // distinct (test dof, trial dof) entries of the tile from accumulator `op` into `out`
    // distinct (test dof, trial dof) entries of accumulator `op` into `out`: at (test dof, trial
    // dof), or (`rev`) at (trial dof, test dof).  Neighbouring lanes take the real and imaginary
    // parts of one entry and walk the row side's dofs in increasing order, so one atomic
    // instruction covers a contiguous run of a column when those dofs are
    auto scatter = [&](int op, R* out, bool rev) {
        const int nx = acc->nx, ny = acc->ny;
        const int nr = rev ? ny : nx;
        for (int e = tid; e < nx * ny * 2; e += NT) {
            const int part = e & 1, xy = e >> 1;
            const int x = rev ? acc->order_x[xy / nr] : acc->order_x[xy % nr];
            const int y = rev ? acc->order_y[xy % nr] : acc->order_y[xy / nr];
            const R re = acc->v[op][x][y][0], im = acc->v[op][x][y][1];
            if (re == R(0) && im == R(0)) continue;
            const int64_t dx = rec[x / 3].dof[x % 3], dy = rec[TX + y / 3].dof[y % 3];
            const int64_t idx = 2 * (dd.mat0 + (rev ? dy + dx * dd.E : dx + dy * dd.E));
            atomic_add(out + idx + part, part ? im : re);
        }
    };
    auto clear = [&]() {
        R* z = &acc->v[0][0][0][0];
        for (int e = tid; e < SX * SY * 2; e += NT) z[e] = R(0);
    };
    __syncthreads();
    scatter(0, T, false);
    if (S::SYM) scatter(0, T, true);                 // T of the reversed pair: the same values, transposed
    if constexpr (kAccOps<R> == 2) {
        scatter(1, K, false);
    } else {
        __syncthreads();
        clear();
        __syncthreads();
        if (valid) {
            // the K pass repeats the epilogue from the moments still held in registers (only its K
            // half is computed)
            const R k = (R)dd.k;
            R D[3];
            for (int i = 0; i < 3; ++i) D[i] = (R)(X.c[i] - Y.c[i]);
            epilogue<R>(mom, X.p, Y.p, X.coef, Y.coef, D, k, X.sg, Y.sg, LdsSink<R, S, 1>{acc, 3 * ix, 3 * iy});
        }
        __syncthreads();
        scatter(0, K, false);
    }
    if constexpr (S::SYM) {
        // K of the reversed pair (Y, X) from the relabelled moments, transposed into place
        __syncthreads();
        clear();
        __syncthreads();
        if (valid) {
            const R k = (R)dd.k;
            R D[3];
            for (int i = 0; i < 3; ++i) D[i] = (R)(Y.c[i] - X.c[i]);
            for (int i = 0; i < 3; ++i)
                for (int c = 0; c < 2; ++c) {
                    const R mx = mom.Mx[i][c], nx = mom.Nx[i][c];
                    mom.Mx[i][c] = mom.My[i][c];
                    mom.My[i][c] = mx;
                    mom.Nx[i][c] = mom.Ny[i][c];
                    mom.Ny[i][c] = nx;
                    mom.Nxy[i][c] = -mom.Nxy[i][c];
                }
            epilogue<R>(mom, Y.p, X.p, Y.coef, X.coef, D, k, Y.sg, X.sg, LdsSinkRev<R, S>{acc, 3 * ix, 3 * iy});
        }
        __syncthreads();
        scatter(0, K, true);
    }
}

template <typename R, typename S>
__global__ __launch_bounds__(S::NT, S::OCC) void k_regular(const int4* __restrict__ tiles, const DomDesc* __restrict__ doms,
                                                           const TriGeom* __restrict__ geom, const int32_t* __restrict__ verts,
                                                           const int32_t* __restrict__ tdof, const int8_t* __restrict__ tsign,
                                                           R* __restrict__ T, R* __restrict__ K) {
    __shared__ LRec<R> rec[S::TX + S::TY];
    __shared__ TileAcc<R, S> acc;
    regular_tile<R, S>(tiles[blockIdx.x], doms, geom, verts, tdof, tsign, T, K, rec, &acc);
}

// ---------------------------------------------------------------------------
// touching pairs: Sauter-Schwab, FP64, one wavefront per pair
// ---------------------------------------------------------------------------

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One touching pair per wavefront (no workgroup barrier): Sauter-Schwab points split over the
// 64 lanes, moments reduced with shuffles, lane 0 scatters the local blocks.
__device__ __attribute__((always_inline)) inline void singular_pair(const SingPair sp, const DomDesc* __restrict__ doms, const TriGeom* __restrict__ geom,
                                     const int32_t* __restrict__ tdof, const int8_t* __restrict__ tsign,
                                     const double* __restrict__ ss_table, const int32_t* __restrict__ ss_off,
                                     const int32_t* __restrict__ ss_cnt, double* T64, double* K64, float* T32,
                                     float* K32, int lane) {
    const DomDesc dd = doms[sp.dom];
    const int64_t rx = dd.rec0 + sp.tx, ry = dd.rec0 + sp.ty;
    const TriGeom& gx = geom[rx];
    const TriGeom& gy = geom[ry];
    double X[3][3], Y[3][3];
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 3; ++k) {
            X[a][k] = gx.p[3 * sp.px[a] + k];
            Y[a][k] = gy.p[3 * sp.py[a] + k];
        }
    double D[3];
    for (int k = 0; k < 3; ++k) D[k] = gx.c[k] - gy.c[k];
    const double k = dd.k;
    const double jac = 4.0 * gx.area * gy.area;
    const double* tab = ss_table + 5 * (int64_t)ss_off[sp.kind];
    const int cnt = ss_cnt[sp.kind];
    Moments<double> m;
    zero_moments(m);
    for (int j = lane; j < cnt; j += 64) {
        const double* e = tab + 5 * j;
        const double sx = e[0], txp = e[1], sy = e[2], typ = e[3], w = e[4] * jac;
        double x[3], y[3], d[3];
        for (int i = 0; i < 3; ++i) {
            x[i] = X[0][i] + sx * (X[1][i] - X[0][i]) + txp * (X[2][i] - X[1][i]);
            y[i] = Y[0][i] + sy * (Y[1][i] - Y[0][i]) + typ * (Y[2][i] - Y[1][i]);
            d[i] = D[i] + x[i] - y[i];
        }
        const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        const double rinv = rsqrt_nr(r2);
        const double kr = k * r2 * rinv;
        double Gre, Gim, gre, gim;
        kernel_values<double>(kr, rinv, w, Gre, Gim, gre, gim);
        const double xy = x[0] * y[0] + x[1] * y[1] + x[2] * y[2];
        const double xc[3] = {x[1] * y[2] - x[2] * y[1], x[2] * y[0] - x[0] * y[2], x[0] * y[1] - x[1] * y[0]};
        m.M0[0] += Gre; m.M0[1] += Gim;
        m.N0[0] += gre; m.N0[1] += gim;
        m.Mxy[0] += Gre * xy; m.Mxy[1] += Gim * xy;
        for (int i = 0; i < 3; ++i) {
            m.Mx[i][0] += Gre * x[i]; m.Mx[i][1] += Gim * x[i];
            m.My[i][0] += Gre * y[i]; m.My[i][1] += Gim * y[i];
            m.Nx[i][0] += gre * x[i]; m.Nx[i][1] += gim * x[i];
            m.Ny[i][0] += gre * y[i]; m.Ny[i][1] += gim * y[i];
            m.Nxy[i][0] += gre * xc[i]; m.Nxy[i][1] += gim * xc[i];
        }
    }
    for (int c = 0; c < 2; ++c) {
        m.M0[c] = wave_sum(m.M0[c]);
        m.N0[c] = wave_sum(m.N0[c]);
        m.Mxy[c] = wave_sum(m.Mxy[c]);
        for (int i = 0; i < 3; ++i) {
            m.Mx[i][c] = wave_sum(m.Mx[i][c]);
            m.My[i][c] = wave_sum(m.My[i][c]);
            m.Nx[i][c] = wave_sum(m.Nx[i][c]);
            m.Ny[i][c] = wave_sum(m.Ny[i][c]);
            m.Nxy[i][c] = wave_sum(m.Nxy[i][c]);
        }
    }
    if (lane == 0) {
        int32_t dofx[3], dofy[3], sgx[3], sgy[3];
        for (int a = 0; a < 3; ++a) {
            dofx[a] = tdof[3 * rx + a];
            dofy[a] = tdof[3 * ry + a];
            sgx[a] = tsign[3 * rx + a];
            sgy[a] = tsign[3 * ry + a];
        }
        if (T64) epilogue<double>(m, gx.p, gy.p, gx.coef, gy.coef, D, k, sgx, sgy,
                                  GlobalSink<double>{dofx, dofy, dd.mat0, dd.E, T64, K64});
        if (T32) epilogue<double>(m, gx.p, gy.p, gx.coef, gy.coef, D, k, sgx, sgy,
                                  GlobalSink<float>{dofx, dofy, dd.mat0, dd.E, T32, K32});
    }
}

__global__ __launch_bounds__(256) void k_singular(const SingPair* __restrict__ pairs, int64_t npairs,
                                                  const DomDesc* __restrict__ doms, const TriGeom* __restrict__ geom,
                                                  const int32_t* __restrict__ tdof, const int8_t* __restrict__ tsign,
                                                  const double* __restrict__ ss_table, const int32_t* __restrict__ ss_off,
                                                  const int32_t* __restrict__ ss_cnt, double* T64, double* K64,
                                                  float* T32, float* K32) {
    const int64_t pid = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (pid >= npairs) return;   // uniform per wavefront; no workgroup barrier in singular_pair
    singular_pair(pairs[pid], doms, geom, tdof, tsign, ss_table, ss_off, ss_cnt, T64, K64, T32, K32, threadIdx.x & 63);
}

// ---------------------------------------------------------------------------
// persistent assembly of a batch of problems (one launch, dynamic work queue)
// ---------------------------------------------------------------------------
// Work item (int4): x = problem, y = subdomain, z = first test triangle, w = first trial triangle
// of a tile of separated pairs (shape S).  Each workgroup claims items through an atomic counter until
// the counter passes `nitems`; every wave then leaves the loop.  The touching pairs are not in the
// queue: their Sauter-Schwab path needs far more registers than a tile, and sharing one kernel
// would hold every tile to that register count (half the resident waves).
template <typename R, typename S>
__global__ __launch_bounds__(S::NT, S::OCC) void k_assemble_persistent(const int4* __restrict__ items, int64_t nitems,
                                                                       unsigned long long* counter,
                                                                       const BatchProb* __restrict__ probs) {
    __shared__ LRec<R> rec[S::TX + S::TY];
    __shared__ TileAcc<R, S> acc;
    __shared__ long long claimed;
    for (;;) {
        if (threadIdx.x == 0) claimed = (long long)atomicAdd(counter, 1ull);
        __syncthreads();
        const long long it = claimed;
        __syncthreads();
        if (it >= nitems) break;            // uniform across the workgroup
        const int4 w = items[it];
        const BatchProb bp = probs[w.x];
        regular_tile<R, S>(make_int4(w.y, w.z, w.w, 0), bp.doms, bp.geom, bp.verts, bp.tdof, bp.tsign,
                           static_cast<R*>(bp.T), static_cast<R*>(bp.K), rec, &acc);
        __syncthreads();                    // LDS records are reused by the next item
    }
}

// ---------------------------------------------------------------------------
// transmission blocks: signed local twisted-Gram values per triangle record
//   v[a][c] = s^i_a s^j_c int phi^j_c . (n_i x phi^i_a)
//           = s^i_a s^j_c c^i_a c^j_c A n_i . (p'^i_a x p'^j_c)   (exact: the integrand is linear)
// ---------------------------------------------------------------------------

__global__ void k_gram_local(const DomDesc* __restrict__ doms, int64_t nrec, const int32_t* __restrict__ rec_dom,
                             const TriGeom* __restrict__ geom, const int32_t* __restrict__ other_rec,
                             const int8_t* __restrict__ tsign, const int32_t* __restrict__ tdof,
                             const int32_t* __restrict__ other_dom, double* __restrict__ gval,
                             int64_t* __restrict__ gcol) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrec) return;
    const int64_t r2 = other_rec[r];
    const DomDesc dj = doms[other_dom[r]];
    const TriGeom& gi = geom[r];
    const TriGeom& gj = geom[r2];
    for (int a = 0; a < 3; ++a) {
        const double* pa = gi.p + 3 * a;
        for (int c = 0; c < 3; ++c) {
            const double* pc = gj.p + 3 * c;
            const double cx = pa[1] * pc[2] - pa[2] * pc[1];
            const double cy = pa[2] * pc[0] - pa[0] * pc[2];
            const double cz = pa[0] * pc[1] - pa[1] * pc[0];
            const double v = gi.coef[a] * gj.coef[c] * gi.area * (gi.n[0] * cx + gi.n[1] * cy + gi.n[2] * cz);
            gval[9 * r + 3 * a + c] = (double)(tsign[3 * r + a] * tsign[3 * r2 + c]) * v;
        }
    }
    for (int c = 0; c < 3; ++c) {
        const int64_t col = dj.off + tdof[3 * r2 + c];
        gcol[6 * r + c] = col;                // u_jD
        gcol[6 * r + 3 + c] = col + dj.E;     // u_jN
    }
}

// ---------------------------------------------------------------------------
// right-hand side: b_0D[m] = 2 int E_inc . phi_m,  b_0N[m] = 2 rho_0 int (d x p) e^{i k0 d.x} . phi_m
// ---------------------------------------------------------------------------

__global__ void k_rhs(const DomDesc d0, const TriGeom* __restrict__ geom, const int32_t* __restrict__ dplus,
                      const int32_t* __restrict__ dminus, int32_t E0, double k0, double rho0, int nrhs,
                      const double* __restrict__ dirs, const double* __restrict__ pol, double* __restrict__ b,
                      int64_t ldb) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t m = gid % E0;
    const int r = (int)(gid / E0);
    if (r >= nrhs) return;
    const double d[3] = {dirs[3 * r], dirs[3 * r + 1], dirs[3 * r + 2]};
    double pr[3], pi[3];
    for (int k = 0; k < 3; ++k) { pr[k] = pol[6 * r + 2 * k]; pi[k] = pol[6 * r + 2 * k + 1]; }
    // h = d x p
    const double hr[3] = {d[1] * pr[2] - d[2] * pr[1], d[2] * pr[0] - d[0] * pr[2], d[0] * pr[1] - d[1] * pr[0]};
    const double hi[3] = {d[1] * pi[2] - d[2] * pi[1], d[2] * pi[0] - d[0] * pi[2], d[0] * pi[1] - d[1] * pi[0]};
    double bD[2] = {0, 0}, bN[2] = {0, 0};
    for (int side = 0; side < 2; ++side) {
        const int32_t* pm = side == 0 ? dplus : dminus;
        const int64_t lt = pm[2 * (d0.dof0 + m)], a = pm[2 * (d0.dof0 + m) + 1];
        const double sgn = side == 0 ? 1.0 : -1.0;
        const TriGeom& g = geom[d0.rec0 + lt];
        for (int q = 0; q < 6; ++q) {
            double phi[3], x[3];
            for (int k = 0; k < 3; ++k) {
                phi[k] = g.coef[a] * (g.q[3 * q + k] - g.p[3 * a + k]);
                x[k] = g.c[k] + g.q[3 * q + k];
            }
            double s, c;
            sincos(k0 * (d[0] * x[0] + d[1] * x[1] + d[2] * x[2]), &s, &c);
            const double wq = sgn * g.w[q];
            const double pph_r = pr[0] * phi[0] + pr[1] * phi[1] + pr[2] * phi[2];
            const double pph_i = pi[0] * phi[0] + pi[1] * phi[1] + pi[2] * phi[2];
            const double hph_r = hr[0] * phi[0] + hr[1] * phi[1] + hr[2] * phi[2];
            const double hph_i = hi[0] * phi[0] + hi[1] * phi[1] + hi[2] * phi[2];
            bD[0] += wq * (pph_r * c - pph_i * s);
            bD[1] += wq * (pph_r * s + pph_i * c);
            bN[0] += wq * (hph_r * c - hph_i * s);
            bN[1] += wq * (hph_r * s + hph_i * c);
        }
    }
    double* col = b + 2 * ((int64_t)r * ldb + d0.off);
    col[2 * m] = 2.0 * bD[0];
    col[2 * m + 1] = 2.0 * bD[1];
    col[2 * (E0 + m)] = 2.0 * rho0 * bN[0];
    col[2 * (E0 + m) + 1] = 2.0 * rho0 * bN[1];
}

// ---------------------------------------------------------------------------
// far field: one workgroup per (rhs, direction)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_far_field(const DomDesc d0, const TriGeom* __restrict__ geom,
                                                   const int32_t* __restrict__ tdof, const int8_t* __restrict__ tsign,
                                                   int32_t T0, double k0, double rho0, const double* __restrict__ x,
                                                   int64_t ldx, const double* __restrict__ dirs, int ndir,
                                                   double* __restrict__ out) {
    const int dir = blockIdx.x % ndir;
    const int r = blockIdx.x / ndir;
    const double xh[3] = {dirs[3 * dir], dirs[3 * dir + 1], dirs[3 * dir + 2]};
    const double* xr = x + 2 * ((int64_t)r * ldx + d0.off);
    double acc[12];
    for (int i = 0; i < 12; ++i) acc[i] = 0.0;
    for (int64_t lt = threadIdx.x; lt < T0; lt += blockDim.x) {
        const int64_t rec = d0.rec0 + lt;
        const TriGeom& g = geom[rec];
        double cD[3][2], cN[3][2];
        for (int a = 0; a < 3; ++a) {
            const int64_t m = tdof[3 * rec + a];
            const double s = tsign[3 * rec + a] * g.coef[a];
            cD[a][0] = s * xr[2 * m]; cD[a][1] = s * xr[2 * m + 1];
            cN[a][0] = s * xr[2 * (d0.E + m)] / rho0; cN[a][1] = s * xr[2 * (d0.E + m) + 1] / rho0;
        }
        for (int q = 0; q < 6; ++q) {
            double xq[3];
            for (int k = 0; k < 3; ++k) xq[k] = g.c[k] + g.q[3 * q + k];
            double sn, cs;
            sincos(-k0 * (xh[0] * xq[0] + xh[1] * xq[1] + xh[2] * xq[2]), &sn, &cs);
            const double wq = g.w[q] * kInv4Pi;
            for (int k = 0; k < 3; ++k) {
                double vD[2] = {0, 0}, vN[2] = {0, 0};
                for (int a = 0; a < 3; ++a) {
                    const double ph = g.q[3 * q + k] - g.p[3 * a + k];
                    vD[0] += cD[a][0] * ph; vD[1] += cD[a][1] * ph;
                    vN[0] += cN[a][0] * ph; vN[1] += cN[a][1] * ph;
                }
                acc[2 * k] += wq * (vD[0] * cs - vD[1] * sn);
                acc[2 * k + 1] += wq * (vD[0] * sn + vD[1] * cs);
                acc[6 + 2 * k] += wq * (vN[0] * cs - vN[1] * sn);
                acc[6 + 2 * k + 1] += wq * (vN[0] * sn + vN[1] * cs);
            }
        }
    }
    __shared__ double red[12][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int i = 0; i < 12; ++i) {
        double v = wave_sum(acc[i]);
        if (lane == 0) red[i][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double F[2][3][2];
    for (int i = 0; i < 12; ++i) {
        double v = red[i][0] + red[i][1] + red[i][2] + red[i][3];
        F[i / 6][(i % 6) / 2][i % 2] = v;
    }
    // E_inf = i k0 [ xh x F_D - xh x (xh x F_N) ]
    double out3[3][2];
    for (int c = 0; c < 2; ++c) {
        const double* FD[3] = {&F[0][0][c], &F[0][1][c], &F[0][2][c]};
        const double* FN[3] = {&F[1][0][c], &F[1][1][c], &F[1][2][c]};
        double a[3] = {xh[1] * *FD[2] - xh[2] * *FD[1], xh[2] * *FD[0] - xh[0] * *FD[2], xh[0] * *FD[1] - xh[1] * *FD[0]};
        double t[3] = {xh[1] * *FN[2] - xh[2] * *FN[1], xh[2] * *FN[0] - xh[0] * *FN[2], xh[0] * *FN[1] - xh[1] * *FN[0]};
        double bb[3] = {xh[1] * t[2] - xh[2] * t[1], xh[2] * t[0] - xh[0] * t[2], xh[0] * t[1] - xh[1] * t[0]};
        for (int k = 0; k < 3; ++k) out3[k][c] = a[k] - bb[k];
    }
    double* o = out + 6 * ((int64_t)r * ndir + dir);
    for (int k = 0; k < 3; ++k) {
        // multiply by i k0
        o[2 * k] = -k0 * out3[k][1];
        o[2 * k + 1] = k0 * out3[k][0];
    }
}

inline unsigned grid_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

void launch_fill(double* p, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return;
    unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_fill, dim3(g), dim3(256), 0, s, p, n, v);
}

void launch_fill_f(float* p, int64_t n, float v, hipStream_t s) {
    if (n <= 0) return;
    unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_fill_f, dim3(g), dim3(256), 0, s, p, n, v);
}

// Tile variants the autotuner chooses from: (test x trial triangles, minimum waves per SIMD).
using TV0 = TileShape<16, 16, 2>;
using TV1 = TileShape<8, 32, 2>;
using TV2 = TileShape<32, 8, 2>;
using TV3 = TileShape<16, 8, 2>;
using TV4 = TileShape<16, 16, 3>;
using TV5 = TileShape<16, 16, 3, true>;
using TV6 = TileShape<16, 16, 2, true>;

template <typename F>
void with_variant(int v, F&& f) {
    switch (v) {
        case 0: f(TV0{}); break;
        case 1: f(TV1{}); break;
        case 2: f(TV2{}); break;
        case 3: f(TV3{}); break;
        case 4: f(TV4{}); break;
        case 5: f(TV5{}); break;
        case 6: f(TV6{}); break;
        default: throw std::invalid_argument("unknown tile variant");
    }
}

void tile_variant_shape(int v, int* tx, int* ty, int* occ) {
    with_variant(v, [&](auto sh) {
        using S = decltype(sh);
        *tx = S::TX;
        *ty = S::TY;
        *occ = S::OCC;
    });
}

bool tile_variant_sym(int v) {
    bool sym = false;
    with_variant(v, [&](auto sh) { sym = decltype(sh)::SYM; });
    return sym;
}

void launch_regular(int precision, int variant, const int4* tiles, int64_t ntiles, const DomDesc* doms,
                    const TriGeom* geom, const int32_t* verts, const int32_t* tdof, const int8_t* tsign, void* T,
                    void* K, hipStream_t s) {
    if (ntiles <= 0) return;
    with_variant(variant, [&](auto sh) {
        using S = decltype(sh);
        if (precision == 0)
            hipLaunchKernelGGL((k_regular<double, S>), dim3((unsigned)ntiles), dim3(S::NT), 0, s, tiles, doms, geom, verts,
                               tdof, tsign, static_cast<double*>(T), static_cast<double*>(K));
        else
            hipLaunchKernelGGL((k_regular<float, S>), dim3((unsigned)ntiles), dim3(S::NT), 0, s, tiles, doms, geom, verts,
                               tdof, tsign, static_cast<float*>(T), static_cast<float*>(K));
    });
}

void launch_singular(const SingPair* pairs, int64_t npairs, const DomDesc* doms, const TriGeom* geom,
                     const double* /*xyz*/, const int32_t* /*verts*/, const int32_t* tdof, const int8_t* tsign,
                     const double* ss_table, const int32_t* ss_off, const int32_t* ss_cnt, double* T64, double* K64,
                     float* T32, float* K32, hipStream_t s) {
    if (npairs <= 0) return;
    hipLaunchKernelGGL(k_singular, dim3(grid_for(npairs, 4)), dim3(256), 0, s, pairs, npairs, doms, geom, tdof, tsign,
                       ss_table, ss_off, ss_cnt, T64, K64, T32, K32);
}

void launch_gram_local(const DomDesc* doms, int /*ndom*/, int64_t nrec, const int32_t* rec_dom, const TriGeom* geom,
                       const int32_t* other_rec, const int8_t* tsign, const int32_t* tdof, const int32_t* other_dom,
                       double* gval, int64_t* gcol, hipStream_t s) {
    if (nrec <= 0) return;
    hipLaunchKernelGGL(k_gram_local, dim3(grid_for(nrec, 128)), dim3(128), 0, s, doms, nrec, rec_dom, geom, other_rec,
                       tsign, tdof, other_dom, gval, gcol);
}

void launch_rhs(const DomDesc* d0, const TriGeom* geom, const int32_t* dplus, const int32_t* dminus, int32_t E0,
                double k0, double rho0, int nrhs, const double* dirs, const double* pol, double* b, int64_t ldb,
                hipStream_t s) {
    int64_t n = (int64_t)E0 * nrhs;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_rhs, dim3(grid_for(n, 128)), dim3(128), 0, s, *d0, geom, dplus, dminus, E0, k0, rho0, nrhs,
                       dirs, pol, b, ldb);
}

void launch_far_field(const DomDesc* d0, const TriGeom* geom, const int32_t* tdof, const int8_t* tsign, int32_t T0,
                      double k0, double rho0, const double* x, int64_t ldx, int nrhs, const double* dirs, int ndir,
                      double* out, hipStream_t s) {
    if (nrhs <= 0 || ndir <= 0) return;
    hipLaunchKernelGGL(k_far_field, dim3((unsigned)(nrhs * ndir)), dim3(256), 0, s, *d0, geom, tdof, tsign, T0, k0,
                       rho0, x, ldx, dirs, ndir, out);
}

void launch_assemble_persistent(int precision, int variant, const int4* items, int64_t nitems,
                                unsigned long long* counter, const BatchProb* probs, int grid, hipStream_t s) {
    if (nitems <= 0) return;
    with_variant(variant, [&](auto sh) {
        using S = decltype(sh);
        if (precision == 0)
            hipLaunchKernelGGL((k_assemble_persistent<double, S>), dim3((unsigned)grid), dim3(S::NT), 0, s, items, nitems,
                               counter, probs);
        else
            hipLaunchKernelGGL((k_assemble_persistent<float, S>), dim3((unsigned)grid), dim3(S::NT), 0, s, items, nitems,
                               counter, probs);
    });
}

void launch_tri_setup_rule(const double* xyz, const int32_t* verts, int64_t nrec, const double* bary18,
                           const double* w6, TriGeom* geom, hipStream_t s) {
    if (nrec <= 0) return;
    Rule6 r;
    for (int q = 0; q < 6; ++q) {
        for (int k = 0; k < 3; ++k) r.bary[q][k] = bary18[3 * q + k];
        r.w[q] = w6[q];
    }
    hipLaunchKernelGGL(k_tri_setup, dim3(grid_for(nrec, 128)), dim3(128), 0, s, xyz, verts, nrec, r, geom);
}

}  // namespace mtf
