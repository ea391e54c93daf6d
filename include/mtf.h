/*
 * mtf.h -- C ABI of the MI355X library for the local multiple traces
 * formulation (MTF) of heterogeneous Maxwell scattering.
 *
 * Problem statement followed by the calls (paper: "Local Multiple Traces
 * Formulation for Heterogeneous Electromagnetic Scattering: Implementation and
 * Preconditioning"):
 *   - geometry: a conforming skeleton mesh, every triangle labelled with the
 *     two subdomains it separates (Section 2.1, Section 3.2);
 *   - materials eps_r,i, mu_r,i and wavenumbers k_i = k0 sqrt(eps_r mu_r)
 *     (eq. relativeParameters);
 *   - incident plane waves E_inc = p exp(i k0 d.x) (eq. incidentNumexp);
 *   - the Galerkin system of Problem 2 (Section 3.2) on RWG_i spaces built by
 *     Algorithm 1 (Section 4.2).
 *
 * Conventions shared by every call
 *   Status codes: 0 = success; MTF_NOT_CONVERGED (1) = warning, outputs hold
 *   the best iterate; negative = error, nothing was written to outputs.
 *   mtf_last_error() returns a thread-local message for the last failing call.
 *   No C++ exception crosses the ABI.  Arguments are validated on the host
 *   before any device work, so invalid calls fail without touching the GPU.
 *
 *   Complex numbers are interleaved (re, im) pairs: complex128 = double[2],
 *   complex64 = float[2].  Matrices are column-major.
 *
 *   Unknown ordering (length N = 2 sum_i E_i):
 *       [u_0D, u_0N, u_1D, u_1N, ..., u_MD, u_MN]
 *   each block of length E_i = dim RWG_i in the dof order of
 *   mtf_get_dof_map.  u_iD holds the coefficients of gamma_D,i E, u_iN those
 *   of rho_i gamma_N,i E (eq. boundary_conditions_traces).
 *
 *   Pointers named *_dev are device pointers on the problem's device (for
 *   example torch CUDA/HIP tensor data); all other pointers are host memory.
 *   The caller owns every buffer it passes; the library copies what it keeps.
 *   Device work is ordered on the problem's stream; calls that return host
 *   data synchronise that stream.  A problem must not be used from two threads
 *   at once.
 */
#ifndef MTF_H
#define MTF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MTF_OK                 0
#define MTF_NOT_CONVERGED      1
#define MTF_ERR_ARG           -1
#define MTF_ERR_MESH          -2
#define MTF_ERR_NONFINITE     -3
#define MTF_ERR_HIP           -4
#define MTF_ERR_OOM           -5
#define MTF_ERR_STATE         -6
#define MTF_ERR_UNSUPPORTED   -7

#define MTF_FP64               0   /* complex128 quadrature, storage and matvec            */
#define MTF_FP32_MIXED         1   /* complex64 separated pairs, FP64 Sauter-Schwab pairs  */
#define MTF_BF16_SPLIT         2   /* products with many right-hand sides on MFMA: the complex64
                                      blocks split into bfloat16 hi/lo planes, three bf16
                                      products per real product, FP32 accumulation          */
#define MTF_FP64_MFMA          3   /* mtf_matvec only: FP64 products of up to 32 right-hand
                                      sides on the FP64 matrix cores from the whole FP64 blocks */

#define MTF_BLOCK_T            0
#define MTF_BLOCK_K            1

#define MTF_PREC_NONE          0
#define MTF_PREC_BLOCK_TINV    1   /* right block-Jacobi preconditioner from T_i^-1 (see mtf_solve) */
#define MTF_PREC_BLOCK_TINV_GS 2   /* one block Gauss-Seidel sweep with the same blocks (see mtf_solve) */

/* mtf_solve_opts.flags: by default the Arnoldi steps between two host reads of the Hessenberg
 * columns are captured once per GMRES cycle as a HIP graph and replayed; MTF_SOLVE_EAGER launches
 * the same kernels one by one instead (same results). */
#define MTF_SOLVE_EAGER 1
/* Build every block of the T_i^-1 preconditioners from T_i itself (read whole when applied)
 * instead of from its symmetric part; see mtf_solve.  Rebuilds the blocks when the last build
 * used the other kind. */
#define MTF_SOLVE_PC_FULL 2
/* Build every block of the T_i^-1 preconditioners as the inverse of T_i itself, per connected
 * component of Gamma_i (read whole when applied), at once: no symmetric-part attempt, no check
 * and no rebuilds.  The build then costs one inversion per block where the default costs a second
 * one for every block that fails its check, and a check product per block; each application reads
 * twice the entries of a symmetric-part block.  For batches of short solves (tens of steps), where
 * the build outweighs the applications.  Excludes MTF_SOLVE_PC_FULL.  Rebuilds the blocks when
 * the last build used another kind. */
#define MTF_SOLVE_PC_DIRECT 8
/* Store the Krylov basis in complex64 (compressed-basis GMRES: Aliaga, Anzt, Grutzmacher,
 * Quintana-Orti and Tomas): the Arnoldi arithmetic and the candidate vector stay complex128,
 * each orthonormal basis vector is rounded to complex64 when it is stored, which halves the bytes
 * of the two passes over the basis per step.  Needs a preconditioner (the flexible iteration,
 * whose correction uses the complex128 preconditioned vectors). */
#define MTF_SOLVE_BASIS_C64 4
/* Block GMRES over consecutive groups of p right-hand sides (1 <= p <= 32), each group sharing
 * one Krylov space (block flexible GMRES: Vital 1990; Gutknecht 2006): a block step applies the
 * preconditioner and the FP64 product to the p vectors of the newest basis block, orthogonalises
 * them against the whole basis by two passes of block classical Gram-Schmidt on the FP64 matrix
 * cores (one read of the basis per pass for all p vectors), and orthonormalises the block from
 * its Gram matrix with the columns scaled to unit norm (Cholesky QR, with diagonal pivoting so
 * that it reveals the rank; a second pass when the block is ill-conditioned), dropping directions
 * whose pivot is at most 1e-15 (noise of the Gram matrix), so that the block narrows when the
 * right-hand sides become dependent.  The products use MTF_FP64_MFMA and the preconditioner
 * MTF_PREC_MULTI for blocks of 3 or more vectors.  The block least-squares problem is reduced by Householder reflections on the
 * host; a group stops when every one of its residuals meets the target, restarts from the
 * corrected solution when the basis is full (opts.max_iters basis vectors, 0: from free device
 * memory, at most 24,000), and is checked with the FP64 residual as in the single-vector
 * iteration.  FP64 operator only (MTF_FP64, else MTF_ERR_UNSUPPORTED); any preconditioner; not
 * with MTF_SOLVE_BASIS_C64.  stats[i].iterations counts the block steps of i's group. */
#define MTF_SOLVE_BLOCK(p) ((((p) & 0xff)) << 8)

typedef struct mtf_problem_s* mtf_problem;

/* Message of the last failing call on this thread (never NULL). */
const char* mtf_last_error(void);

/* Library version. */
int mtf_version(int* major, int* minor);

/* Create a problem bound to HIP device `device` and HIP stream `stream`
 * (a hipStream_t; NULL = the default stream).  *out receives an opaque handle
 * owned by the library until mtf_problem_destroy. */
int mtf_problem_create(mtf_problem* out, int device, void* stream);

/* Free every device and host resource of the problem. NULL is accepted. */
int mtf_problem_destroy(mtf_problem p);

/* Skeleton mesh (Section 3.2 and the remark on meshing conventions).
 *   xyz   [nv][3]  vertex coordinates
 *   tri   [nt][3]  vertex ids in [0, nv); the right-hand normal
 *                  (v1-v0)x(v2-v0) points from label[t][0] to label[t][1]
 *   label [nt][2]  the two subdomains separated by the triangle, in [0, M],
 *                  distinct; 0 is the unbounded exterior Omega_0.  The paper's
 *                  convention is label[t][0] < label[t][1] (normal from min to
 *                  max); the opposite order is accepted per triangle.
 * Builds, on the host, Algorithm 1 for every subdomain (exterior normal n_i =
 * mesh normal when i == label[t][0], else its opposite), the RWG_i spaces and
 * the triangle-pair classes.  Fails with MTF_ERR_MESH when a Gamma_i is not a
 * closed, consistently oriented 2-manifold (every Gamma_i edge shared by exactly
 * two Gamma_i triangles traversing it in opposite directions), when a triangle
 * is degenerate, or when a subdomain has no triangle.  Arrays are copied.
 * The RWG_i dofs are the edges of Gamma_i ordered by their vertex ids (smaller
 * id, then larger), so a vertex numbering that keeps nearby vertices close keeps
 * nearby dofs close.  Each Gamma_i's triangles are stored in the order of their
 * sorted vertex ids (the dofs' order), which the assembly tiles follow; the
 * environment variable MTF_TRIANGLE_ORDER=morton orders them along a Morton curve
 * through their centroids instead, =input keeps the input order (any other value
 * fails with MTF_ERR_ARG).  Only the summation order of the blocks depends on it. */
int mtf_set_mesh(mtf_problem p, int64_t nv, const double* xyz, int64_t nt,
                 const int32_t* tri, const int32_t* label, int32_t M);

/* Materials (eq. relativeParameters): eps_r[M+1], mu_r[M+1] > 0, k0 > 0.
 * k_i = k0 sqrt(eps_r,i mu_r,i), rho_i = sqrt(eps_r,i / mu_r,i).  MTF_ERR_UNSUPPORTED when some
 * k_i times the diameter of the mesh's bounding box reaches 1e6 (over 1e5 wavelengths across: the
 * range of the FP64 phase reduction of the assembly kernels). */
int mtf_set_materials(mtf_problem p, double k0, const double* eps_r, const double* mu_r);

/* Sizes: N (total unknowns) and E[M+1] (dim RWG_i); either may be NULL. */
int mtf_get_sizes(mtf_problem p, int64_t* N, int64_t* E);

/* Dof map of RWG_i: for dof m, edge_vtx[2m..2m+1] = its edge's vertex ids
 * (a < b) and plus_tri[m] = the skeleton triangle tau+ (the Gamma_i triangle
 * whose oriented boundary runs from a to b; the RWG function is +l/(2A)(x-p) on
 * tau+ and -l/(2A)(x-p) on tau-).  Either output may be NULL. */
int mtf_get_dof_map(mtf_problem p, int32_t i, int32_t* edge_vtx, int32_t* plus_tri);

typedef struct {
    int32_t struct_size;     /* sizeof(mtf_assembly_opts)                            */
    int32_t precision;       /* MTF_FP64 or MTF_FP32_MIXED                             */
    int32_t singular_order;  /* Gauss-Legendre points per coordinate, 1..8 (default 4) */
    int32_t flags;           /* 0, or MTF_ASSEMBLE_ROUND_FP64                          */
} mtf_assembly_opts;

/* Launch configuration of the separated-pair assembly.  By default it is autotuned: on the first
 * assembly of a shape class (floor(log2) of the mean number of triangles per subdomain) in a
 * precision, each tile variant is timed once and the fastest kept for the process (and, for
 * mtf_batch_assemble, then the number of persistent workgroups per CU); with the environment
 * variable MTF_TUNE_CACHE naming a file the choices are also read from and appended to it.
 * flags |= MTF_ASSEMBLE_TILE(v) forces variant v instead (0 <= v < MTF_TILE_VARIANTS; see
 * mtf_tile_variant).  Every variant computes the same sums; only the order of the atomic
 * additions differs. */
#define MTF_TILE_VARIANTS 7
#define MTF_ASSEMBLE_TILE(v) ((((v) + 1) & 0xff) << 8)

/* With MTF_FP32_MIXED: the complex64 blocks are the FP64 blocks (assembled before) rounded to
 * complex64 instead of a new quadrature in FP32; rounding keeps them within one complex64 ulp of
 * the FP64 operator (relative difference about 2e-8 on the bench workload, against about 3e-7
 * for the FP32 quadrature).  mtf_assemble only. */
#define MTF_ASSEMBLE_ROUND_FP64 1

/* Galerkin assembly of T_i and K_i for every subdomain (eq. boundary_operators,
 * twisted pairing of eq. self_duality_identity) and of the transmission blocks
 * (eq. trick_transmission).  Separated triangle pairs use the symmetric
 * degree-4 six-point rule per triangle; pairs sharing a vertex, an edge or the
 * whole triangle use Sauter-Schwab rules in FP64.  MTF_FP64 also keeps the
 * FP64 blocks; MTF_FP32_MIXED assembles separated pairs in FP32 and stores
 * complex64 blocks (or rounds the FP64 blocks, MTF_ASSEMBLE_ROUND_FP64).  Both
 * precisions may be assembled on one problem (call twice).  Asynchronous on the
 * problem's stream.  MTF_ERR_STATE for MTF_ASSEMBLE_ROUND_FP64 without FP64 blocks. */
int mtf_assemble(mtf_problem p, const mtf_assembly_opts* opts);

/* Copy the dense E_i x E_i block `which` (MTF_BLOCK_T / MTF_BLOCK_K) of the
 * given precision to host memory dst (complex128 [E_i][E_i], column-major,
 * converted from complex64 for MTF_FP32_MIXED).  Synchronises. */
int mtf_copy_block(mtf_problem p, int32_t i, int32_t which, int32_t precision, double* dst);

/* Gather n entries (rows[k], cols[k]) of block `which` of subdomain i in the given
 * precision into out (complex128 [n], host); indices must lie in [0, E_i).  For sampled
 * checks of large blocks.  Synchronises. */
int mtf_get_entries(mtf_problem p, int32_t i, int32_t which, int32_t precision, int32_t n,
                    const int32_t* rows, const int32_t* cols, double* out);

/* Copy the transmission block G^ij (row block i, column block j, j in
 * Lambda_i; real, dense E_i x E_j column-major) to host memory.  Zero if
 * Gamma_ij is empty.  Synchronises. */
int mtf_copy_transmission(mtf_problem p, int32_t i, int32_t j, double* dst);

/* Right-hand sides for nrhs plane waves E_inc = p exp(i k0 d.x):
 *   d[nrhs][3] real unit directions, p_re/p_im [nrhs][3] polarisations;
 *   b_dev: complex128 [nrhs][ldb], ldb >= N (column r at b_dev + r*ldb).
 * Only the Gamma_0 rows are nonzero:
 *   b_0D[m] = 2 int E_inc . phi_m,  b_0N[m] = 2 rho_0 int (d x p) e^{i k0 d.x} . phi_m
 * (Proposition 1 read with the Stratton-Chu formula as printed:
 *  2 A_0 u_0 - u_0 = -2 u_inc, tested in the twisted pairing). */
int mtf_rhs_plane_waves(mtf_problem p, int32_t nrhs, const double* d, const double* p_re,
                        const double* p_im, void* b_dev, int64_t ldb);

/* y = M x for nrhs complex128 vectors (x_dev, y_dev: [nrhs][ld], ld >= N),
 * with M = 2A + X of Problem 2 applied from the stored blocks of `precision`.
 * MTF_BF16_SPLIT applies every subdomain's 2x2 Calderon block to all nrhs
 * columns as one GEMM, [Y_iD | Y_iN] = [K_i | T_i] [[2X_iD, 2X_iN], [2/rho X_iN,
 * -2 rho X_iD]], on MFMA (needs the MTF_FP32_MIXED blocks; relative error of the
 * product ~1e-5).  MTF_FP64_MFMA (nrhs <= 32, FP64 blocks) computes the same GEMM in FP64 on
 * v_mfma_f64_16x16x4f64, T_i and K_i read once for all nrhs vectors (block GMRES uses it for its
 * block products); the result equals the MTF_FP64 product up to summation order. */
int mtf_matvec(mtf_problem p, int32_t nrhs, const void* x_dev, void* y_dev, int64_t ld,
               int32_t precision);

/* The product of mtf_matvec (precision MTF_FP64 or MTF_FP32_MIXED only), for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  It calls no hipMalloc, hipFree or other allocating routine; the partial sums that
 * mtf_matvec keeps in a buffer of the problem go to a fixed 64 MiB array in device memory instead
 * (one per GPU, held until the process ends), so a problem whose product needs more than
 * 64 MiB of partial sums (16 bytes x sum_i 2 E_i (ceil(E_i/64) + 1); about 16 MB for N = 27,648)
 * is rejected with MTF_ERR_ARG before any device work.  Same kernels and results as mtf_matvec.
 * The array is shared by every call on that GPU and keeps the last call's contents (it needs no
 * clearing: every entry a call reads, that call wrote first): calls that overlap on one GPU, from
 * two streams or two threads, race and give wrong results.  The blocks of `precision` must have
 * been assembled (mtf_assemble allocates; this call does not). */
int mtf_matvec_noalloc(mtf_problem p, int32_t nrhs, const void* x_dev, void* y_dev, int64_t ld,
                       int32_t precision);

/* Measurement of the product above for one vector (x_dev, y_dev: complex128 [N] on the device,
 * precision MTF_FP64 or MTF_FP32_MIXED): `reps` products are launched on the problem's stream
 * with HIP events around each launch of the dense block kernel (every T_i, K_i entry streamed
 * once) and around each whole product (dense kernel + the kernel that sums the column-chunk
 * partials and applies the transmission blocks).  dense_s, total_s receive the mean seconds per
 * launch.  Synchronises; reps must be in [1, 10000]. */
int mtf_time_matvec(mtf_problem p, int32_t precision, int32_t reps, const void* x_dev, void* y_dev,
                    double* dense_s, double* total_s);

typedef struct {
    int32_t struct_size;      /* sizeof(mtf_solve_opts)                                     */
    int32_t precision;        /* operator used by the inner iteration: MTF_FP64 or MTF_FP32_MIXED */
    int32_t preconditioner;   /* MTF_PREC_NONE, MTF_PREC_BLOCK_TINV or MTF_PREC_BLOCK_TINV_GS */
    int32_t max_iters;        /* Arnoldi steps per GMRES cycle; 0: as many as half the free
                                 device memory holds, at most 8000 (2000 for lockstep batches) */
    int32_t max_refinements;  /* outer FP64 refinement steps (MTF_FP32_MIXED), 0 = 10        */
    int32_t flags;            /* 0, or MTF_SOLVE_EAGER, MTF_SOLVE_PC_FULL, MTF_SOLVE_PC_DIRECT, MTF_SOLVE_BASIS_C64, MTF_SOLVE_BLOCK(p) */
    double  rtol;             /* ||b - M x||_2 <= rtol ||b||_2 with the FP64 operator        */
    double  inner_rtol;       /* inner GMRES tolerance of a refinement step, 0 = 1e-3*... */
    const void* x0_dev;       /* complex128 initial guess [nrhs][ld] or NULL (zero)          */
} mtf_solve_opts;

typedef struct {
    int32_t iterations;       /* total Arnoldi steps                                   */
    int32_t refinements;      /* FP64 residual evaluations after the first             */
    int32_t converged;        /* 1 if rtol was met                                     */
    int32_t reorthogonalizations; /* Arnoldi steps with a second Gram-Schmidt pass (all kept steps) */
    double  rel_residual;     /* final ||b - M x|| / ||b|| with the FP64 operator       */
    double  t_precond_s;      /* time to build the preconditioner (first call only)    */
    double  t_solve_s;        /* wall time of the solve                                */
} mtf_solve_stats;

/* Solve M x = b by GMRES (full; FP64 Arnoldi by classical Gram-Schmidt with
 * delayed reorthogonalisation, two passes over the basis per step) for each of nrhs
 * right-hand sides (b_dev, x_dev: complex128 [nrhs][ld]).  A cycle ends when the
 * recurrence residual meets rtol; the FP64 residual is then recomputed and a new
 * cycle starts if it does not.  With MTF_PREC_BLOCK_TINV the iteration runs on M P, with P the
 * block-diagonal right preconditioner
 *     P_i = 1/2 [[0, -S_i^-1 / rho_i], [rho_i S_i^-1, 0]],  S_i = (T_i + T_i^T) / 2
 * (the inverse of the off-diagonal part of 2 A_i with T_i replaced by its symmetric
 * part, which differs from T_i only by the quadrature asymmetry of touching pairs; the
 * block shape of the block-OSRC preconditioner of Section 4.4), S_i^-1 computed once
 * per problem on the GPU in complex64 and applied reading its upper triangle only.  Where Gamma_i
 * has several connected components (the exterior of disjoint scatterers), S_i is taken block
 * diagonal over them, each component's block inverted on its own.
 * A block whose T_i is ill-conditioned enough that ||T_i S_i^-1 v - v|| > 1e-3 ||v|| on a
 * fixed vector v is rebuilt as T_i^-1 (per component) and read whole (every block at once with
 * MTF_SOLVE_PC_DIRECT; the whole T_i^-1, components or not, with MTF_SOLVE_PC_FULL).
 * MTF_PREC_BLOCK_TINV_GS applies one block Gauss-Seidel sweep instead: Omega_0
 * first, then the colour classes of the subdomain adjacency graph (subdomains
 * of one class share no interface and are done together), each block solving
 * with P_i after subtracting the transmission terms of the blocks already done.  Right
 * preconditioning leaves the residual that decides convergence, ||b - M x||, unchanged.  With either
 * preconditioner the iteration is flexible (the preconditioned vectors are kept),
 * so the FP32 application of P does not limit the attainable FP64 residual.
 * MTF_FP32_MIXED runs the inner GMRES with relaxed products (one right-hand side
 * at a time): the FP64 operator until the recurrence residual of the cycle has
 * fallen below 1% of tol / delta, the complex64 operator (FP32 arithmetic) after,
 * delta = ||(M_32 - M_64) r|| / ||M_64 r|| measured once on the first residual and
 * tol the cycle's relative target (half the outer one); late Krylov steps tolerate
 * larger product errors (Simoncini & Szyld 2003, Bouras & Fraysse 2005).  FP64
 * residuals correct the result (iterative refinement) until rtol holds for the
 * FP64 operator, which must have been assembled too.  stats[nrhs] may be NULL.
 * Returns MTF_NOT_CONVERGED if some right-hand side missed rtol. */
int mtf_solve(mtf_problem p, int32_t nrhs, const void* b_dev, void* x_dev, int64_t ld,
              const mtf_solve_opts* opts, mtf_solve_stats* stats);

/* Single-trace (PMCHWT) formulation for M = 1 (the remark on the PMCHWT in Section 3.2): adding
 * the two row blocks of Problem 2 with u_1 = -u_0 leaves one unknown pair u = u_0 = (u_0D, u_0N)
 * on Gamma_0 and the system 2 (A_0 - A_1) u = 2 u_inc, discretely
 *     M_STF = 2 A_0 + 2 Sigma A_1 Sigma,   phi^1_m = Sigma_mm phi^0_m (Sigma = -I on the reversed
 *     closed surface), A_i the Galerkin blocks [[K_i, T_i/rho_i], [-rho_i T_i, K_i]]
 * applied as R M C with the MTF product (C u = [u; -Sigma u], R y = y_0 - Sigma y_1; the
 * transmission blocks cancel).  Vectors are complex128 [nrhs][ld], ld >= 2 E_0, ordered (u_0D,
 * u_0N); the right-hand side is the first 2 E_0 entries of mtf_rhs_plane_waves.
 * mtf_stf_matvec: y = M_STF x.  mtf_solve_stf: GMRES (FP64 operator and Arnoldi, no
 * preconditioner; opts.precision MTF_FP64 and opts.preconditioner MTF_PREC_NONE, else
 * MTF_ERR_UNSUPPORTED) until ||b - M_STF x|| <= rtol ||b||.  MTF_ERR_UNSUPPORTED unless M = 1 with
 * Gamma_0 and Gamma_1 on the same edges.  The far field of u is that of the MTF vector [u, ...]
 * (mtf_far_field reads only its Gamma_0 entries). */
int mtf_stf_matvec(mtf_problem p, int32_t nrhs, const void* x_dev, void* y_dev, int64_t ld);
int mtf_solve_stf(mtf_problem p, int32_t nrhs, const void* b_dev, void* x_dev, int64_t ld,
                  const mtf_solve_opts* opts, mtf_solve_stats* stats);

/* z = P x for nrhs complex128 vectors (x_dev, z_dev: [nrhs][ld], ld >= N, no aliasing) with
 * the right preconditioner `preconditioner` (MTF_PREC_BLOCK_TINV or MTF_PREC_BLOCK_TINV_GS, as
 * defined for mtf_solve).  Builds S_i^-1 on first use (from the FP32 blocks if assembled, else
 * from the FP64 ones).  Stream-ordered.  With MTF_PREC_MULTI or'ed in (nrhs <= 32) all vectors are
 * preconditioned together: each complex64 block is read whole once for all of them and applied in
 * FP64 arithmetic on the FP64 matrix cores, one launch per Gauss-Seidel stage (block GMRES uses
 * this form; it synchronises). */
#define MTF_PREC_MULTI 0x100
int mtf_apply_preconditioner(mtf_problem p, int32_t preconditioner, int32_t nrhs, const void* x_dev,
                             void* z_dev, int64_t ld);

/* Far field E_inf(xhat) (E_sc ~ exp(i k0 |x|)/|x| E_inf) of nrhs solutions
 * x_dev [nrhs][ld] in ndir unit directions dir[ndir][3] (host), written to host
 * out: complex128 [nrhs][ndir][3].  From the Stratton-Chu formula in Omega_0:
 *   E_inf = i k0 [xhat x F(u_0D) - xhat x (xhat x F(u_0N / rho_0))],
 *   F(v) = 1/(4 pi) int_{Gamma_0} exp(-i k0 xhat.y) v(y) dy.  Synchronises. */
int mtf_far_field(mtf_problem p, int32_t nrhs, const void* x_dev, int64_t ld, int32_t ndir,
                  const double* dir, double* out);

/* Tile variant v: tiles of tx test x ty trial triangles (one pair per thread, tx * ty threads per
 * workgroup), compiled for at least `occupancy` resident waves per SIMD.  Variants 5 and 6 list each
 * unordered pair of triangle groups once and evaluate both orders of a triangle pair from one
 * quadrature (the kernels depend on the distance only: T of the reversed pair is the same value,
 * K a second epilogue on relabelled moments).  Any output may be NULL. */
int mtf_tile_variant(int32_t v, int32_t* tx, int32_t* ty, int32_t* occupancy);

/* Tile variant used by the last mtf_assemble of p (-1 before the first). */
int mtf_assembly_variant(mtf_problem p, int32_t* variant);

/* The autotuner's trials of this process, one line each (key, variant, workgroups per CU for batch
 * launches, seconds), as a NUL-terminated string truncated to cap bytes. */
int mtf_tuning_log(char* buf, int64_t cap);

/* Statistics of the last mtf_assemble: pair counts by class
 * (counts[0] separated, [1] vertex, [2] edge, [3] coincident, summed over
 * subdomains, ordered pairs) and the device time of the assembly kernels in
 * seconds (HIP events).  Synchronises. */
int mtf_assembly_stats(mtf_problem p, int64_t* counts, double* seconds);

/* ---------------------------------------------------------------------------
 * Batches of independent problems (many scatterers of uneven size).
 * ------------------------------------------------------------------------- */
typedef struct mtf_batch_s* mtf_batch;

/* A batch over n existing problems (each with mesh and materials set, all on one device
 * and stream, each at most once).  The problems stay owned by the caller and must outlive
 * the batch; the batch keeps its work list of the problems' current meshes. */
int mtf_batch_create(mtf_batch* out, int32_t n, const mtf_problem* problems);
int mtf_batch_destroy(mtf_batch b);

/* Assembles T_i and K_i of every problem of the batch: the separated triangle pairs of all
 * problems in ONE persistent launch (workgroups claim 16 x 16 tiles of separated pairs, across all
 * problems, largest problems first, from an atomic counter until the list is exhausted), then the
 * touching pairs (Sauter-Schwab, FP64) of each problem.  The launch is autotuned per shape class
 * and precision (see MTF_ASSEMBLE_TILE): every tile variant at 4 workgroups per CU, then 1, 2 and 8
 * workgroups per CU for the fastest, each timed on a persistent launch over every eighth tile
 * (grid_used, may be NULL, receives the workgroups launched); seconds (may be NULL) receives the
 * device time of the whole assembly.  Synchronises. */
int mtf_batch_assemble(mtf_batch b, const mtf_assembly_opts* opts, int32_t* grid_used, double* seconds);

/* Statistics of the last mtf_batch_assemble: ordered pair counts by class summed over the problems
 * (counts[4] as in mtf_assembly_stats; may be NULL), device times in seconds (seconds[2], may be
 * NULL): [0] the persistent launch over the separated pairs, [1] the touching pairs after it (HIP
 * events on the batch's stream), and the launch configuration (config[2], may be NULL): tile
 * variant and persistent workgroups.  Synchronises. */
int mtf_batch_assembly_stats(mtf_batch b, int64_t* counts, double* seconds, int32_t* config);

/* The T_i^-1 preconditioner blocks (as defined for mtf_solve) of every problem of the batch, built
 * together: every diagonal block (of each T_i, or of each connected component of Gamma_i) of every
 * problem is padded with the identity to an order rounded up to 128 and the blocks of equal padded
 * order are inverted as one batch (blocked Gauss-Jordan on FP32 matrix cores), instead of one
 * problem after another.  From the FP32 blocks where assembled, else from the FP64 ones.  flags:
 * 0, MTF_SOLVE_PC_FULL or MTF_SOLVE_PC_DIRECT.  The blocks stay with their problems (used by mtf_solve,
 * mtf_apply_preconditioner and mtf_batch_solve) until a new assembly of their source precision;
 * a later build reuses their storage.  The build's padded work buffers (the buckets and the
 * panel buffers of the inversion) stay with the batch for the next build, growing when a build
 * needs more, until mtf_batch_destroy.  Synchronises. */
int mtf_batch_build_preconditioner(mtf_batch b, int32_t flags);

/* mtf_solve of problem i on b_dev[i] -> x_dev[i] (one right-hand side each, ld = N_i) with
 * common options; stats[n] may be NULL.  The preconditioner blocks of the problems lacking them are
 * first built together (mtf_batch_build_preconditioner); stats[0] receives that build's time in
 * t_precond_s.  The problems are then solved on up to 4 streams at once (the environment variable
 * MTF_BATCH_LANES sets 1-8; 1 solves problem after problem on the problems' own streams), each
 * stream a host thread taking the next problem, largest first; with more than one, the call starts
 * with a device synchronisation and ends when every solve is complete, and each solve reads its
 * Hessenberg columns every 4 Arnoldi steps instead of 8 (the other streams keep the GPU busy
 * meanwhile, and fewer steps are spent past convergence).  A problem without FP64
 * blocks gets them assembled (default options) for its residual checks and released after its
 * solve; with opts.precision MTF_FP32_MIXED a problem without complex64 blocks gets them rounded
 * from its FP64 blocks (MTF_ASSEMBLE_ROUND_FP64) for its solve only, into buffers that each stream
 * keeps (grown to the largest problem it met, until mtf_batch_destroy) and lends to its solves.
 * Preconditioner blocks that a problem did not hold before the call are released after its solve
 * (also when the call fails).
 * A problem without GMRES work buffers of its own uses one of the batch's (one per stream,
 * allocated for the largest problem that stream met and kept until mtf_batch_destroy).  Device
 * memory needed beyond the assembled blocks: the preconditioner blocks of every problem (half the
 * bytes of the complex64 T_i, K_i), the build's padded work buffers (kept with the batch), per
 * stream one problem's temporary blocks (its complex64 blocks kept with the batch) and GMRES
 * buffers.  A caller that solves the same batch again after a new assembly builds the blocks with
 * mtf_batch_build_preconditioner first, so that they and their storage stay with the problems
 * instead of being allocated for every call.
 * max_iters 0 here means cycles of at most 1,000 Arnoldi steps (not the free-memory length of
 * mtf_solve): a batch is many small solves, whose Krylov storage would otherwise be sized from free
 * memory. */
int mtf_batch_solve(mtf_batch b, const void* const* b_dev, void* const* x_dev, const mtf_solve_opts* opts,
                    mtf_solve_stats* stats);

/* ---------------------------------------------------------------------------
 * Learned warm start: a POD basis of MTF solutions and a small MLP mapping
 * problem parameters to POD coefficients; GMRES then starts from x0 = Phi c.
 * (Not in the paper: an addition that changes only the initial guess; the FP64
 * residual of mtf_solve, relative to ||b||, still decides convergence.)
 * ------------------------------------------------------------------------- */

/* POD basis of nsnap solution snapshots U_dev (complex128 [nsnap][ldu], N rows
 * each): the r leading left singular vectors Phi_dev (complex128 [r][ldphi])
 * and singular values sv[r] (host), computed in complex128 from the snapshot
 * Gram matrix U^H U (FP64 GEMM on the device) by subspace iteration with
 * Rayleigh-Ritz, Phi = U Z Lambda^-1/2.  r <= nsnap, r <= 256.  Synchronises. */
int mtf_pod_build(mtf_problem p, int32_t nsnap, const void* U_dev, int64_t ldu, int32_t r,
                  void* Phi_dev, int64_t ldphi, double* sv);

/* C = Phi^H X for n vectors X_dev (complex128 [n][ldx]) -> C_dev (complex128 [n][r]); FP64. */
int mtf_pod_project(mtf_problem p, int32_t r, const void* Phi_dev, int64_t ldphi, int32_t n,
                    const void* X_dev, int64_t ldx, void* C_dev);

/* X = Phi C for n coefficient vectors C_dev (complex128 [n][r]) -> X_dev (complex128 [n][ldx]); FP64. */
int mtf_pod_expand(mtf_problem p, int32_t r, const void* Phi_dev, int64_t ldphi, int32_t n,
                   const void* C_dev, void* X_dev, int64_t ldx);

/* Multilayer perceptron n_in -> width (tanh) -> width (tanh) -> n_out (linear), FP32,
 * parameters packed (W1 [width][n_in], b1, W2 [width][width], b2, W3 [n_out][width], b3),
 * Glorot-uniform initialisation from a SplitMix64 stream seeded with `seed`, zero biases.
 * Activations are row-major [samples][features] float arrays on the device. */
typedef struct mtf_mlp_s* mtf_mlp;
int mtf_mlp_create(mtf_mlp* out, int device, void* stream, int32_t n_in, int32_t width,
                   int32_t n_out, uint64_t seed);
int mtf_mlp_destroy(mtf_mlp m);
int mtf_mlp_num_params(mtf_mlp m, int64_t* n);
int mtf_mlp_get_params(mtf_mlp m, float* host);           /* [num_params] */
int mtf_mlp_set_params(mtf_mlp m, const float* host);
/* Y_dev [n][n_out] = MLP(X_dev [n][n_in]). */
int mtf_mlp_forward(mtf_mlp m, int32_t n, const float* X_dev, float* Y_dev);
/* Mean squared error over all n x n_out outputs against targets T_dev and its gradient
 * with respect to the packed parameters (grad_host [num_params], may be NULL). */
int mtf_mlp_loss_grad(mtf_mlp m, int32_t n, const float* X_dev, const float* T_dev, float* loss,
                      float* grad_host);

typedef struct {
    int32_t struct_size;     /* sizeof(mtf_train_opts)                          */
    int32_t epochs;          /* passes over the data                            */
    int32_t batch;           /* minibatch size                                  */
    int32_t reserved;
    float   lr, beta1, beta2, eps;   /* Adam (Kingma & Ba 2015)                 */
    uint64_t seed;           /* SplitMix64 seed of the per-epoch shuffles       */
} mtf_train_opts;

/* Adam on the MSE loss with shuffled minibatches; loss_hist[epochs] (host, may be NULL)
 * receives the full-data loss after each epoch.  Synchronises at epoch ends. */
int mtf_mlp_train(mtf_mlp m, int32_t n, const float* X_dev, const float* T_dev,
                  const mtf_train_opts* opts, float* loss_hist);

#ifdef __cplusplus
}
#endif

#endif /* MTF_H */
