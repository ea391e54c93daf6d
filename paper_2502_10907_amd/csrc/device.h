// Device data structures and kernel launchers (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace mtf {

// Geometry of one triangle of one Gamma_i (Gamma_i orientation), FP64.
// Coordinates other than the centroid are relative to the centroid.
struct TriGeom {
    double c[3];      // centroid
    double p[9];      // vertices P_a - c
    double q[18];     // six quadrature points x_q - c
    double w[6];      // quadrature weights times area
    double coef[3];   // l_a / (2 A): RWG scale of the local function opposite vertex a
    double n[3];      // unit normal n_i
    double area;
    double pad;
};
static_assert(sizeof(TriGeom) == 44 * 8, "TriGeom layout");

struct DomDesc {
    int64_t rec0;     // first triangle record of the domain
    int64_t dof0;     // first dof record of the domain (concatenated dof tables)
    int64_t mat0;     // first entry of T_i / K_i in the concatenated matrix arrays
    int64_t off;      // first unknown of block i (u_iD), u_iN starts at off + E
    int64_t part0;    // first partial-sum slot of the domain in the matvec workspace
    int32_t T, E;
    int32_t nchunk;   // column chunks of the dense matvec
    int32_t chunk0;   // first entry of the domain's per-chunk tables (preconditioner slot ranges)
    double k, rho;
};

// One subdomain's multi-RHS GEMM (bf16-split planes; see gemm.hip).
struct GemmDesc {
    int64_t a_off;    // first element of the subdomain's A planes (4 planes of Mp x Kp bf16)
    int64_t b_off;    // first element of its B planes (4 planes of Np x Kp bf16)
    int64_t c_off;    // first complex64 of its output block (M x N, column-major, ld = ldc)
    int64_t Mp, Kp, Np;
    int64_t M, N, ldc;
};

struct SingPair {     // device copy of a touching pair
    int32_t dom, tx, ty, kind;
    int32_t px[3], py[3];
};

// Device pointers of one problem of a batch (persistent assembly).
struct BatchProb {
    const DomDesc* doms;
    const TriGeom* geom;
    const int32_t* verts;
    const int32_t* tdof;
    const int8_t* tsign;
    const SingPair* sing;
    void* T;          // double* or float* by precision
    void* K;
};

// ---- launchers (all asynchronous on `s`) ----
void launch_fill(double* p, int64_t n, double v, hipStream_t s);
void launch_fill_f(float* p, int64_t n, float v, hipStream_t s);

void launch_tri_setup_rule(const double* xyz, const int32_t* verts, int64_t nrec, const double* bary18,
                           const double* w6, TriGeom* geom, hipStream_t s);

// Separated-pair tiles: variant v (0..kTileVariants-1) is a tile of tx test x ty trial triangles
// (tx * ty threads) compiled for at least `occ` resident waves per SIMD; tiles: int4(subdomain,
// first test triangle, first trial triangle, 0) stepping by tx and ty.  precision 0 = FP64 blocks,
// 1 = FP32 (T, K point to double or float).
constexpr int kTileVariants = 7;
void tile_variant_shape(int v, int* tx, int* ty, int* occ);
// variant v lists each unordered pair of triangle groups once and evaluates both orders of a
// triangle pair from one quadrature (its tiles: test group <= trial group)
bool tile_variant_sym(int v);
void launch_regular(int precision, int variant, const int4* tiles, int64_t ntiles, const DomDesc* doms,
                    const TriGeom* geom, const int32_t* verts, const int32_t* tdof, const int8_t* tsign, void* T,
                    void* K, hipStream_t s);

// Touching pairs (Sauter-Schwab, FP64 arithmetic), results added to FP64 or FP32 blocks.
void launch_singular(const SingPair* pairs, int64_t npairs, const DomDesc* doms, const TriGeom* geom,
                     const double* xyz, const int32_t* verts, const int32_t* tdof, const int8_t* tsign,
                     const double* ss_table, const int32_t* ss_off, const int32_t* ss_cnt,
                     double* T64, double* K64, float* T32, float* K32, hipStream_t s);

// One persistent launch over the separated-pair tiles of a batch of problems (precision 0 = FP64,
// 1 = FP32; tile variant as for launch_regular; items: int4(problem, subdomain, first test triangle,
// first trial triangle)); `counter` must be zero; grid = number of persistent workgroups.
void launch_assemble_persistent(int precision, int variant, const int4* items, int64_t nitems,
                                unsigned long long* counter, const BatchProb* probs, int grid, hipStream_t s);

// Signed local transmission values and column indices per triangle record.
void launch_gram_local(const DomDesc* doms, int ndom, int64_t nrec, const int32_t* rec_dom,
                       const TriGeom* geom, const int32_t* other_rec, const int8_t* tsign,
                       const int32_t* tdof, const int32_t* other_dom, double* gval, int64_t* gcol,
                       hipStream_t s);

void launch_rhs(const DomDesc* d0, const TriGeom* geom, const int32_t* dplus, const int32_t* dminus,
                int32_t E0, double k0, double rho0, int nrhs, const double* dirs, const double* pol,
                double* b, int64_t ldb, hipStream_t s);

// Dense part of y = M x: partial sums of the 2x2 block products per column chunk.
// y = sum of partials + transmission; one thread per unknown pair (D, N) of a dof.

// GMRES vector kernels (complex128, length n), batched over nb right-hand sides in lockstep
// (Krylov slab j at V + j*ldv with ldv = nb*n; column b of each slab is right-hand side b).
// Kernels taking `flag` skip right-hand side b when flag[b] == 0.
// Arnoldi step with delayed reorthogonalisation (DCGS2), nb right-hand sides in lockstep; the
// step index j is read from jdev[0] on the device and the grids depend on nvmax only.
// Reductions over the basis at step j: `grid` workgroups per right-hand side; at step j each
// vector is split into clamp(units / (j / 16 + 1), cmin, kmax) row chunks, and hpart holds
// 4 * nb * (nvmax + 1) * kmax doubles.
struct DotPlan {
    int grid, units, cmin, kmax;
};
inline DotPlan dot_plan(int nb) {
    nb = nb < 1 ? 1 : nb;
    DotPlan d;
    d.grid = 2048 / nb < 32 ? 32 : 2048 / nb;
    d.units = 1280 / nb < 32 ? 32 : 1280 / nb;
    d.cmin = 32;
    d.kmax = d.units < 512 ? (d.units < 32 ? 32 : d.units) : 512;
    return d;
}
// V holds the basis in complex128 or, when c64, in complex64 (the same ldv, in entries); U is the
// complex128 copy of the candidate u (read instead of slot j when c64).
void launch_dot2(const double* V, int64_t ldv, const int* jdev, int nvmax, const double* t, const double* U, int64_t n,
                 double* hpart, const DotPlan& d, bool c64, int nb, hipStream_t s);  // partial Q^H [u t], u^H [u t] (t null: t = u)
void launch_reduce2(const double* hpart, const int* jdev, int nvmax, const DotPlan& d, double* S, double* Z, int nb,
                    hipStream_t s);
void launch_dcgs_col(double* H, int64_t ldh, int64_t hstride, const double* S, const double* Z, const double* hg, int nct,
                     const int* jdev, int nvmax, double* scal, int last, double* R, int64_t rstride, int nb, hipStream_t s);
// q_j, u_{j+1} (also unext); zsrc -> zdst slot j; *jnext = j+1.  The same two launches also form
// the partial products Hbar s (into hg), finalise Hessenberg column j-1, write the first-pass
// column j and, when R is given, column j of R.
void launch_update2(const double* V, int64_t ldv, const int* jdev, int* jnext, int nvmax, const double* S,
                    const double* Z, const double* t, double* unext, int64_t n, double* part, int ng,
                    const double* zsrc, double* zdst, double* H, int64_t ldh, int64_t hstride, double* hg, int nct,
                    double* R, int64_t rstride, bool c64, int nb, hipStream_t s);
void launch_set_int(int* p, int v, hipStream_t s);                         // p[0] = v
void launch_stage_cols(const double* H, int64_t ldh, int64_t hstride, const int* jdev, int back, int cnt, double* Hst,
                       int nb, hipStream_t s);                              // H columns j-back .. j-back+cnt-1
void launch_trsv_upper(const double* R, int64_t ldh, int64_t rstride, const int* cnt, double* y, int64_t ystride,
                       int* info, int nb, hipStream_t s);                  // y_b = R_b^-1 y_b (upper, cnt[b])
void launch_combine(double* x, int64_t ldx, const double* V, int64_t ldv, const int* cnt, int nvmax, const double* coef,
                    int64_t n, int nb, hipStream_t s);                       // x_b += V_b coef_b
void launch_norm2(const double* w, int64_t ldw, int64_t n, double* part, int nblk, int nb, hipStream_t s);
void launch_axpby(double* y, const double* x, int64_t n, double a_re, double a_im, double b,
                  hipStream_t s);       // y = b*y + a*x (a complex, b real)

void launch_far_field(const DomDesc* d0, const TriGeom* geom, const int32_t* tdof, const int8_t* tsign,
                      int32_t T0, double k0, double rho0, const double* x, int64_t ldx, int nrhs,
                      const double* dirs, int ndir, double* out, hipStream_t s);

// Complex64 helpers for the preconditioner.
void launch_copy_block_f64_to_f32(const double* src, float* dst, int64_t n, hipStream_t s);
// Batched complex64 GEMM on FP32 matrix cores, column-major: for z < batch,
//   D_z = alpha A_z B_z + beta C_z   (X_z = X + z * sX complex entries; C may alias D).
// Logical rows r of A, C, D map to physical rows r + (r >= rg0 ? rgw : 0) and logical columns c
// of B, C, D to c + (c >= cg0 ? cgw : 0): a band of rows/columns can be skipped.
struct CGemm {
    int m = 0, n = 0, k = 0, batch = 1;
    float ar = 1.f, ai = 0.f, beta = 0.f;
    const float* A = nullptr;
    int64_t lda = 0, sA = 0;
    const float* B = nullptr;
    int64_t ldb = 0, sB = 0;
    const float* C = nullptr;
    int64_t ldc = 0, sC = 0;
    float* D = nullptr;
    int64_t ldd = 0, sD = 0;
    int rg0 = 0x7fffffff, rgw = 0, cg0 = 0x7fffffff, cgw = 0;
    int band_cd = 1;     // 0: C and D are compact (the skipped bands apply to A's rows and B's columns only)
};
// dst[(r + (r >= r0 ? rw : 0)) + (c + (c >= c0 ? cw : 0)) * ldd] = src[r + c * lds] for a rows x cols
// complex64 block, batched (strides ss, sd)
void launch_band_copy_f32(const float* src, int64_t lds, int64_t ss, float* dst, int64_t ldd, int64_t sd, int rows,
                          int cols, int r0, int rw, int c0, int cw, int batch, hipStream_t s);
void launch_cgemm_f32(const CGemm& g, hipStream_t s);
// single product D = alpha A B + beta C (beta real)
inline void launch_cgemm_f32(int m, int n, int k, float alpha_re, float alpha_im, const float* A, int64_t lda,
                             const float* B, int64_t ldb, float beta_re, const float* C, int64_t ldc, float* D,
                             int64_t ldd, hipStream_t s) {
    CGemm g;
    g.m = m; g.n = n; g.k = k; g.ar = alpha_re; g.ai = alpha_im; g.beta = beta_re;
    g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc; g.D = D; g.ldd = ldd;
    launch_cgemm_f32(g, s);
}
// In-place inverse of the n x n (n <= 64) complex64 blocks A + z*stride (ld lda), z < batch;
// info[0] is set to a nonzero value on a zero pivot.
// y_z = A_z x_z for `batch` n x n complex64 matrices A_z = A + z sA (ld lda), x_z = x + z sx,
// y_z = y + z sy (strides in complex entries); part: batch * ceil(n / 256) * n complex scratch
void launch_cgemv_f32(const float* A, int64_t lda, int64_t sA, const float* x, int64_t sx, int n, int batch, float* part,
                      float* y, int64_t sy, hipStream_t s);
int  launch_cinv_small_f32(float* A, int64_t lda, int64_t stride, int n, int batch, int* info, hipStream_t s);
// Symmetric-read block matvec (tiles I <= J of 64 x 64; stiles: int4(domain, I, J, 0)), the
// touching-pair corrections of the lower triangle, and the finishing kernel.
void launch_matvec_sym_f64(const DomDesc* doms, const int4* stiles, int64_t ntiles, const double* T, const double* K,
                           const double* x, double* part, hipStream_t s);
void launch_matvec_sym_f32(const DomDesc* doms, const int4* stiles, int64_t ntiles, const float* T, const float* K,
                           const double* x, double* part, hipStream_t s);
void launch_near_diff_f64(const DomDesc* doms, const int32_t* dof_dom, int64_t ndof, const int64_t* ptr, const int32_t* col,
                          const double* T, const double* K, double* out, hipStream_t s);
void launch_near_diff_f32(const DomDesc* doms, const int32_t* dof_dom, int64_t ndof, const int64_t* ptr, const int32_t* col,
                          const float* T, const float* K, double* out, hipStream_t s);
void launch_matvec_sym_finish(const DomDesc* doms, const int32_t* dof_dom, int64_t ndof, const int32_t* dplus,
                              const int32_t* dminus, const double* gval, const int64_t* gcol, const int64_t* nptr,
                              const int32_t* ncol, const double* nval, const double* part, const double* x, double* y,
                              hipStream_t s);
// Symmetric-read preconditioner product (tiles I <= J of the complex64 inverse of the symmetric
// part of T_i), its finishing kernel, and the in-place symmetrisation A <- (A + A^T)/2.  The
// finishing kernel sums, for a row of chunk B of domain i, the partial slots
// slots[doms[i].chunk0 + B].x .. .y (inclusive): the slots its tiles wrote.
void launch_precond_sym(const DomDesc* doms, const int4* stiles, int64_t ntiles, const float* Tinv, const double* x,
                        double* part, hipStream_t s);
void launch_precond_sym_finish(const DomDesc* doms, const int32_t* dof_dom, int64_t ndof, const double* part,
                               const int2* slots, double* z, const int32_t* list, hipStream_t s);
void launch_zero_offdiag_f32(float* A, int E, const int32_t* cid, hipStream_t s);   // A[r,c] = 0 where cid[r] != cid[c]
void launch_symmetrize_f32(float* A, int n, hipStream_t s);
// w_i = v_i - sum_j G^ij z_j for the dofs in `list` (one block Gauss-Seidel stage)
void launch_gs_residual(const DomDesc* doms, const int32_t* dof_dom, const int32_t* list, int64_t nlist,
                        const int32_t* dplus, const int32_t* dminus, const double* gval, const int64_t* gcol,
                        const int32_t* other_dom, const int32_t* dom_stage, int stage, const double* v, const double* z,
                        double* w, hipStream_t s);
void launch_nonfinite_check(const float* A, int64_t n, int* flag, hipStream_t s);
// Single-trace formulation for M = 1 through the MTF product: full = [x; -Sigma x] (x = (u_D, u_N)
// on Gamma_0, 2E entries; sig[E] = +-1 with phi^1_m = sig_m phi^0_m), and y = full_y[0:2E] -
// Sigma full_y[2E:4E].
void launch_stf_expand(const double* x, const int8_t* sig, int64_t E, double* full, hipStream_t s);
void launch_stf_reduce(const double* full, const int8_t* sig, int64_t E, double* y, hipStream_t s);

// Preconditioner blocks of many problems inverted together: each n x n diagonal block (of T_i or
// of one connected component of Gamma_i) is copied into an S x S slot of a bucket of equal S >= n,
// with the identity in the padding (the inverse of diag(A, I) is diag(A^-1, I)), so that a bucket
// is one batched in-place inversion.
struct PadBlock {
    const void* src;     // first entry of the block (complex128 when f64, else complex64)
    float* dst;          // where the inverse goes (complex64, leading dimension ld)
    int64_t ld;          // leading dimension of src and dst (the E_i of the block's subdomain)
    int32_t n;           // order of the block
    int32_t f64;         // src is complex128
};
// buf + z S^2 (ld S) <- block z (symmetrised (A + A^T)/2 when sym), identity in the padding
void launch_pad_gather(const PadBlock* blocks, int nblocks, int S, int sym, float* buf, hipStream_t s);
// block z's destination <- the leading n x n part of buf + z S^2
// the leading n x n of every slot back to its block; *flag |= 1 when a copied entry is not finite
void launch_pad_scatter(const PadBlock* blocks, int nblocks, int S, const float* buf, int* flag, hipStream_t s);
// y = A x for one n x n complex128 block A (ld lda), complex64 x and y; part: ceil(n/256) * n
// complex64 scratch
void launch_cgemv_f64src(const double* A, int64_t lda, const float* x, int n, float* part, float* y, hipStream_t s);

// Multi-RHS block products (gemm.hip).
// mode 0: operator blocks [K_i | T_i]; mode 1: preconditioner blocks T_i^-1 (passed as T).
void launch_split_A(const GemmDesc* descs, const DomDesc* doms, const int4* tiles, int64_t ntiles, const float* T,
                    const float* K, uint16_t* A, int mode, hipStream_t s);
void launch_split_B(const GemmDesc* descs, const DomDesc* doms, int ndom, int64_t kp_max, int64_t np, const double* x,
                    int64_t ld, int nrhs, uint16_t* B, int mode, hipStream_t s);
void launch_gemm_bf16x3(const GemmDesc* descs, const int4* tiles, int64_t ntiles, const uint16_t* A, const uint16_t* B,
                        float* C, hipStream_t s);
void launch_gemm_finish(const DomDesc* doms, const GemmDesc* descs, const int32_t* dof_dom, int64_t ndof,
                        const int32_t* dplus, const int32_t* dminus, const double* gval, const int64_t* gcol,
                        const float* C, const double* x, double* y, int64_t ld, int nrhs, int mode, hipStream_t s);

}  // namespace mtf

namespace mtf {
// Learned warm start (learn.hip).
void launch_sgemm(int M, int N, int K, const float* A, int lda, int ta, const float* B, int ldb, int tb, const float* bias,
                  int act_tanh, float* C, int ldc, int accumulate, hipStream_t s);
void launch_tanh_back(const float* A, const float* dA, float* dZ, int64_t n, hipStream_t s);
int  launch_mse(const float* Y, const float* T, float* dY, int64_t n, float scale, float* loss_part, hipStream_t s);
void launch_colsum(const float* dZ, int M, int N, float* db, hipStream_t s);
void launch_adam(float* p, const float* g, float* m1, float* m2, int64_t n, float lr_t, float b1, float b2, float eps,
                 hipStream_t s);
void launch_gather_rows(const float* X, const int* idx, int B, int cols, float* Xb, hipStream_t s);
void launch_cgemm_hn(int m, int n, int k, const float* A, int64_t lda, const float* B, int64_t ldb, float* C, int64_t ldc,
                     hipStream_t s);
// C = op(A) B in complex128, op(A) = A (m x k) or A^H (A stored k x m) (POD of FP64 snapshots)
void launch_zgemm(int m, int n, int k, bool herm_a, const double* A, int64_t lda, const double* B, int64_t ldb,
                  double* C, int64_t ldc, hipStream_t s);
void launch_c128_to_c64(const double* X, int64_t ld, int64_t n, int cols, float* Y, hipStream_t s);
void launch_c64_to_c128(const float* X, int64_t n, int cols, double* Y, int64_t ld, hipStream_t s);
}  // namespace mtf

namespace mtf {
// Block Krylov contractions on the FP64 matrix cores (block.hip).  Vectors are complex128, each
// contiguous, vector i of a set at base + 2 i ld doubles.
struct BlockDotPlan {
    int itiles = 0, ctiles = 0, ppad = 0, nchunk = 0;
    int64_t nc = 0;
    int64_t part_elems = 0;   // complex partial sums the launch needs
};
struct BlockUpdPlan {
    int64_t ntile = 0;
    int ctiles = 0, ppad = 0, nsplit = 0, ksplit = 0;
    int64_t part_elems = 0;
};
BlockDotPlan plan_bdot(int64_t n, int j, int p);
BlockUpdPlan plan_bupd(int64_t n, int j, int p);
// H[i * hld + c] = V_i^H W_c for i < j, c < p (hld >= p); part: plan.part_elems complex
void launch_bdot(const BlockDotPlan& pl, const double* V, int64_t ldv, int j, const double* W, int64_t ldw, int p,
                 int64_t n, double* part, double* H, int hld, hipStream_t s);
// Y_c = beta Yin_c + alpha sum_{i < j} V_i H(i, c), H(i, c) at complex index i hs_i + c hs_c; Y may
// alias Yin (same ld); Yin is not read when beta is 0; part: plan.part_elems complex
void launch_bupd(const BlockUpdPlan& pl, const double* V, int64_t ldv, int j, const double* H, int64_t hs_i,
                 int64_t hs_c, int p, int64_t n, double* part, const double* Yin, int64_t ldyin, double* Y,
                 int64_t ldy, double alpha, double beta, hipStream_t s);
// y_j = M x_j for q vectors (complex128, ld ldx / ldy, q <= 32) from the whole FP64 blocks on the
// matrix cores: work items (dom, row0, rhs0, split) of mmv_rows(q) rows x mmv_rhs_step(q)
// right-hand sides x kc columns (kc a multiple of 16), partial sums of split s of subdomain d at
// part + pbase[d] (complex, nsplit[d] q 2 E_d of them), then the transmission terms.
inline int mmv_rows(int) { return 64; }
inline int mmv_rhs_step(int) { return 16; }
void launch_mmv(const DomDesc* doms, const int4* items, int64_t nitems, const double* T, const double* K, const double* x,
                int64_t ldx, int q, const int64_t* pbase, int kc, double* part, const int32_t* dof_dom, int64_t ndof,
                const int32_t* dplus, const int32_t* dminus, const double* gval, const int64_t* gcol,
                const int* nsplit, double* y, int64_t ldy, hipStream_t s);
// z = P x for q vectors on the dofs of one Gauss-Seidel stage (list: its dofs, or null for all nlist
// dofs), P_i from the whole complex64 blocks S (FP64 arithmetic on the matrix cores); work items
// and partial sums as for launch_mmv
void launch_pcmm(const DomDesc* doms, const int4* items, int64_t nitems, const float* S, const double* x, int64_t ldx,
                 int q, const int64_t* pbase, int kc, double* part, const int32_t* dof_dom, const int32_t* list,
                 int64_t nlist, const int* nsplit, double* z, int64_t ldz, hipStream_t s);
// w = v - (transmission from earlier stages) z for q vectors (ld), on the listed dofs of stage `stage`
void launch_gs_residual_q(const DomDesc* doms, const int32_t* dof_dom, const int32_t* list, int64_t nlist,
                          const int32_t* dplus, const int32_t* dminus, const double* gval, const int64_t* gcol,
                          const int32_t* other_dom, const int32_t* dom_stage, int stage, const double* v,
                          const double* z, double* w, int64_t ld, int q, hipStream_t s);
}  // namespace mtf
