// C ABI of the MTF library: problem object, uploads, assembly and solver drivers.
#include "../../include/mtf.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <complex>
#include <cstring>
#include <exception>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "device.h"
#include "quadrature.h"
#include "runtime.h"
#include "skeleton.h"

namespace {

using namespace mtf;
using cd = std::complex<double>;

constexpr int kChunk = 64;    // columns per dense-matvec workgroup (matches solver.hip)
constexpr int kNblk = 32;     // partial sums of GMRES norms
constexpr int kGjPanel = 256; // block width of the Gauss-Jordan inversion (64-wide leaves inside)
constexpr double kPcSymTol = 1e-3;   // largest ||T_i S_i^-1 v - v|| / ||v|| of a symmetric-part block
constexpr int kSync = 8;      // Arnoldi steps between host reads of the Hessenberg columns (the most)
// ... of a problem solved on one of several batch lanes: the other lanes keep the GPU busy while
// one waits for its host read, and a shorter interval spends fewer steps past convergence
constexpr int kSyncLanes = 4;
constexpr int kMaxBatch = 64; // right-hand sides per lockstep GMRES batch (MFMA products)
constexpr int kMaxBlock = 32; // right-hand sides per block of block GMRES
// smallest kept pivot of the pivoted Cholesky factorisation of a block's scaled Gram matrix: the
// squared norm of what a unit column adds to the span of those kept before it.  Forming the Gram
// matrix rounds at 1e-16 relative, so smaller pivots are noise; a direction dropped below it leaves
// an error of at most 3e-8 of its column in the Arnoldi relation.
constexpr double kBlockKeep = 1e-15;
// blocks of at least this many vectors use the FP64 multi-RHS product (whole blocks, read once for
// the block); narrower ones the symmetric-read product per vector
constexpr int kMmvMin = 3;
constexpr int kUpdGroups = 8; // partial-sum groups of the basis update
constexpr int kBatchCycle = 1000;  // Arnoldi steps per cycle in mtf_batch_solve when max_iters is 0
constexpr int kEagerBatches = 2;   // Arnoldi batches of a cycle launched eagerly before a graph is captured
constexpr double kLookaheadFactor = 30.0;   // a second batch is queued while every residual exceeds this x target

struct GemmOp {
    DevBuf<uint16_t> A, B;
    DevBuf<float> C;
    DevBuf<GemmDesc> d;
    DevBuf<int4> tiles;
    int64_t ntiles = 0, kpmax = 0, np = 0;
    int nrhs = 0;
    bool haveA = false;
};

struct GmresWork {
    int64_t n = 0;
    int maxit = 0, nb = 0;
    DevBuf<double> V, Zt, Rf, tmp, tmp2, tmp3, r, hpart, S, Z, hg, scal, H, npart, upart, y;
    DevBuf<double> ufix, tfix, zfix, Hst;   // step-invariant candidate, product, preconditioned slabs; staged columns
    DevBuf<int> jdev;                // step index: step j reads slot j&1 and writes j+1 into the other slot
    int zslots = 0;                  // Krylov slots held by Zt (0: no preconditioned basis)
    DevBuf<int> cnt;                 // Arnoldi steps kept per right-hand side, then a zero-pivot flag
    double* host = nullptr;          // pinned: two areas of nb x kSync Hessenberg columns (the first also
                                     // takes the norm parts)
    hipEvent_t ev[2] = {nullptr, nullptr};   // completion of the copy into each area
    double* hosty = nullptr;         // pinned: nb x (maxit + 1) least-squares coefficients
    int* hostcnt = nullptr;          // pinned: nb step counts + flag
    int64_t cap_n = 0;               // unknowns the n-sized buffers were allocated for (n <= cap_n)
    ~GmresWork() { release(); }
    // frees every buffer; the next solve allocates again
    void release() {
        for (DevBuf<double>* b : {&V, &Zt, &Rf, &tmp, &tmp2, &tmp3, &r, &hpart, &S, &Z, &hg, &scal, &H, &npart, &upart,
                                  &y, &ufix, &tfix, &zfix, &Hst})
            b->reset();
        jdev.reset();
        cnt.reset();
        if (host) (void)hipHostFree(host);
        if (hosty) (void)hipHostFree(hosty);
        if (hostcnt) (void)hipHostFree(hostcnt);
        for (hipEvent_t& e : ev) {
            if (e) (void)hipEventDestroy(e);
            e = nullptr;
        }
        host = hosty = nullptr;
        hostcnt = nullptr;
        n = cap_n = 0;
        maxit = nb = zslots = 0;
    }
};

template <typename T>
void swap_buf(DevBuf<T>& a, DevBuf<T>& b) {
    std::swap(a.p, b.p);
    std::swap(a.n, b.n);
}

// Exchanges two workspaces (a batch lends its workspace to each problem's solve in turn).
void swap_work(GmresWork& a, GmresWork& b) {
    DevBuf<double>* da[] = {&a.V, &a.Zt, &a.Rf, &a.tmp, &a.tmp2, &a.tmp3, &a.r, &a.hpart, &a.S, &a.Z, &a.hg, &a.scal,
                            &a.H, &a.npart, &a.upart, &a.y, &a.ufix, &a.tfix, &a.zfix, &a.Hst};
    DevBuf<double>* db[] = {&b.V, &b.Zt, &b.Rf, &b.tmp, &b.tmp2, &b.tmp3, &b.r, &b.hpart, &b.S, &b.Z, &b.hg, &b.scal,
                            &b.H, &b.npart, &b.upart, &b.y, &b.ufix, &b.tfix, &b.zfix, &b.Hst};
    for (size_t k = 0; k < sizeof(da) / sizeof(da[0]); ++k) swap_buf(*da[k], *db[k]);
    swap_buf(a.jdev, b.jdev);
    swap_buf(a.cnt, b.cnt);
    std::swap(a.n, b.n);
    std::swap(a.cap_n, b.cap_n);
    std::swap(a.maxit, b.maxit);
    std::swap(a.nb, b.nb);
    std::swap(a.zslots, b.zslots);
    std::swap(a.host, b.host);
    std::swap(a.hosty, b.hosty);
    std::swap(a.hostcnt, b.hostcnt);
    std::swap(a.ev[0], b.ev[0]);
    std::swap(a.ev[1], b.ev[1]);
}

}  // namespace

// Work items and partial sums of the FP64 multi-right-hand-side product (launch_mmv) for q vectors.
struct MmvPlan {
    DevBuf<int4> items;
    DevBuf<int64_t> pbase;
    DevBuf<int> nsplit;
    DevBuf<double> part;
    int64_t nitems = 0;
    int q = 0;
};

// Work items of the block preconditioner (launch_pcmm) for q vectors: items of Gauss-Seidel stage st
// at [item0[st], item0[st + 1]) (one stage holding every subdomain for the block-Jacobi form).
struct PcmmPlan {
    DevBuf<int4> items;
    DevBuf<int64_t> pbase;
    DevBuf<int> nsplit;
    DevBuf<double> part;
    std::vector<int64_t> item0;
    int q = 0, pc = -1;
};

struct mtf_problem_s {
    int device = 0;
    hipStream_t stream = nullptr;

    bool has_mesh = false, has_mat = false;
    Skeleton sk;
    double k0 = 0;
    std::vector<double> eps, mu, kw, rho;

    std::vector<DomDesc> doms;
    int64_t nrec = 0, ndof = 0, mat_entries = 0, part_entries = 0;
    DevBuf<double> d_xyz;
    DevBuf<int32_t> d_verts, d_tdof, d_other_rec, d_other_dom, d_rec_dom, d_dplus, d_dminus, d_dof_dom;
    DevBuf<int8_t> d_tsign;
    DevBuf<TriGeom> d_geom;
    DevBuf<DomDesc> d_doms;
    DevBuf<double> d_gval;
    DevBuf<int64_t> d_gcol;
    DevBuf<int4> d_tiles, d_symtiles;
    int64_t ntiles = 0, nsymtiles = 0;
    int tile_variant = -1;           // tile variant of d_tiles (-1: not built)
    int last_variant = -1;           // tile variant of the last mtf_assemble
    DevBuf<int64_t> d_near_ptr;      // touching-pair lower-triangle pattern (CSR over dofs)
    DevBuf<int32_t> d_near_col;
    DevBuf<double> near64, near32;   // corrections A[m,n] - A[n,m] for T, K from the FP64 / FP32 blocks
    int64_t near_nnz = 0;
    DevBuf<SingPair> d_sing;
    DevBuf<double> d_ss;
    DevBuf<int32_t> d_ss_meta;   // off[4], cnt[4]
    int ss_order = 0;

    DevBuf<double> T64, K64;
    DevBuf<float> T32, K32, Tinv;
    bool have64 = false, have32 = false, have_tinv = false;
    int tinv_prec = MTF_FP64;        // blocks the T_i^-1 preconditioner was built from (MTF_FP64 / MTF_FP32_MIXED)
    GemmOp gm, gp;                   // multi-RHS MFMA products: operator blocks, preconditioner blocks
    MmvPlan mmv;                     // FP64 multi-RHS MFMA product
    PcmmPlan pcmm;                   // block preconditioner on the FP64 matrix cores
    // block Gauss-Seidel stages: stage 0 = {Omega_0}, then colour classes of the subdomain graph
    DevBuf<int4> d_stage_tiles, d_pctiles;    // preconditioner tiles per Gauss-Seidel stage, and all of them
    DevBuf<int2> d_pc_slots;                  // per row chunk (DomDesc::chunk0 + B): partial slots its tiles write
    int64_t npctiles = 0;
    std::vector<int> dom_colour;              // Gauss-Seidel stage of each subdomain (Omega_0: 0)
    std::vector<char> pc_full;                // 1: the block is T_i^-1 itself, read whole
    int pc_kind = 0;                          // how the blocks were built (PcKind)
    // host-side structure that depends on the mesh only, kept across builds (cleared by a new mesh):
    // the connected components of each Gamma_i, and what the uploaded tile lists were built for
    std::vector<std::vector<std::pair<int, int>>> comp_cache;
    bool comp_cached = false;
    int tiles_built_for = -1;                 // per_component flag of the uploaded lists (-1: none)
    std::vector<char> tiles_built_full;       // pc_full they were built with
    int gmres_sync = kSync;                   // Arnoldi steps between host reads of its GMRES cycles
    DevBuf<int32_t> d_stage_dofs, d_dom_stage;
    std::vector<int64_t> stage_tile0, stage_dof0;   // [nstage + 1] offsets
    double t_precond = 0;
    DevBuf<double> part;
    DevBuf<double> scratch_dirs;
    double t_assemble = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipStream_t capture = nullptr;   // private stream on which GMRES step graphs are captured (never run)
    // private streams of the preconditioner build (default priority, non-blocking): two lanes that
    // invert subdomain groups concurrently, each with a lookahead stream
    hipStream_t gj_lane[2] = {nullptr, nullptr}, gj_aux[2] = {nullptr, nullptr};
    hipEvent_t gj_fork[2] = {nullptr, nullptr}, gj_join[2] = {nullptr, nullptr};
    hipEvent_t gj_start = nullptr, gj_done[2] = {nullptr, nullptr};
    GmresWork gw;
    // single-trace (PMCHWT) operator mode for M = 1: GMRES vectors are (u_D, u_N) on Gamma_0
    bool stf = false;
    DevBuf<int8_t> stf_sign;         // phi^1_m = sign_m phi^0_m
    DevBuf<double> stf_x, stf_y;     // full-length MTF vectors around the product

    ~mtf_problem_s() {
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        for (int l = 0; l < 2; ++l) {
            if (gj_fork[l]) (void)hipEventDestroy(gj_fork[l]);
            if (gj_join[l]) (void)hipEventDestroy(gj_join[l]);
            if (gj_done[l]) (void)hipEventDestroy(gj_done[l]);
            if (gj_lane[l]) (void)hipStreamDestroy(gj_lane[l]);
            if (gj_aux[l]) (void)hipStreamDestroy(gj_aux[l]);
        }
        if (gj_start) (void)hipEventDestroy(gj_start);
        if (capture) (void)hipStreamDestroy(capture);
    }
};

namespace {

void sync(mtf_problem p) { HIPCHK(hipStreamSynchronize(p->stream)); }

// Largest accepted ||T_i S_i^-1 v - v|| / ||v|| of a symmetric-part preconditioner block: kPcSymTol,
// or the value of the environment variable MTF_PC_SYM_TOL when set (0 rebuilds every block from
// T_i itself; used to test that path).
double pc_sym_tol() {
    const char* e = std::getenv("MTF_PC_SYM_TOL");
    if (!e || !*e) return kPcSymTol;
    char* end = nullptr;
    const double v = std::strtod(e, &end);
    return (end && *end == 0 && v >= 0.0) ? v : kPcSymTol;
}

// How the T_i^-1 preconditioner blocks are built: from the symmetric part S_i (per connected
// component of Gamma_i), each block checked and rebuilt from T_i where S_i^-1 fails; from T_i
// directly (per component); or from the whole T_i.
enum PcKind { kPcSym = 0, kPcDirect = 1, kPcWhole = 2 };

int pc_kind_of(int flags) {
    const bool whole = (flags & MTF_SOLVE_PC_FULL) != 0, direct = (flags & MTF_SOLVE_PC_DIRECT) != 0;
    if (whole && direct) throw ArgError("MTF_SOLVE_PC_FULL and MTF_SOLVE_PC_DIRECT exclude each other");
    if (whole) return kPcWhole;
    // with the check threshold at 0 every symmetric-part block would be rebuilt
    if (direct || pc_sym_tol() <= 0.0) return kPcDirect;
    return kPcSym;
}

void upload_doms(mtf_problem p) {
    for (size_t i = 0; i < p->doms.size(); ++i) {
        p->doms[i].k = p->has_mat ? p->kw[i] : 0.0;
        p->doms[i].rho = p->has_mat ? p->rho[i] : 1.0;
    }
    p->d_doms.upload(p->doms, p->stream);
}

void set_mesh_impl(mtf_problem p, int64_t nv, const double* xyz, int64_t nt, const int32_t* tri, const int32_t* label,
                   int32_t M) {
    Skeleton sk = build_skeleton(nv, xyz, nt, tri, label, M);
    DeviceGuard g(p->device);
    hipStream_t s = p->stream;
    // record and dof tables concatenated over subdomains
    std::vector<DomDesc> doms(M + 1);
    int64_t rec = 0, dof = 0, mat = 0, part = 0;
    int32_t chunks = 0;
    for (int i = 0; i <= M; ++i) {
        const Domain& d = sk.dom[i];
        DomDesc& dd = doms[i];
        std::memset(&dd, 0, sizeof(dd));
        dd.rec0 = rec;
        dd.dof0 = dof;
        dd.mat0 = mat;
        dd.off = sk.offset[i];
        dd.part0 = part;
        dd.T = d.T;
        dd.E = d.E;
        dd.nchunk = (d.E + kChunk - 1) / kChunk;
        dd.chunk0 = chunks;
        dd.rho = 1.0;
        chunks += dd.nchunk;
        rec += d.T;
        dof += d.E;
        mat += (int64_t)d.E * d.E;
        part += (int64_t)(dd.nchunk + 1) * 2 * d.E;    // nchunk + 1 slots: symmetric-read product
    }
    std::vector<int32_t> verts(3 * rec), tdof(3 * rec), other_rec(rec), other_dom(rec), rec_dom(rec);
    std::vector<int8_t> tsign(3 * rec);
    std::vector<int32_t> dplus(2 * dof), dminus(2 * dof), dof_dom(dof);
    for (int i = 0; i <= M; ++i) {
        const Domain& d = sk.dom[i];
        const int64_t r0 = doms[i].rec0;
        for (int lt = 0; lt < d.T; ++lt) {
            for (int a = 0; a < 3; ++a) {
                verts[3 * (r0 + lt) + a] = d.verts[3 * lt + a];
                tdof[3 * (r0 + lt) + a] = d.tri_dof[3 * lt + a];
                tsign[3 * (r0 + lt) + a] = d.tri_sign[3 * lt + a];
            }
            other_dom[r0 + lt] = d.other[lt];
            other_rec[r0 + lt] = (int32_t)(doms[d.other[lt]].rec0 + d.other_lt[lt]);
            rec_dom[r0 + lt] = i;
        }
        const int64_t f0 = doms[i].dof0;
        for (int m = 0; m < d.E; ++m) {
            dplus[2 * (f0 + m)] = d.plus[2 * m];
            dplus[2 * (f0 + m) + 1] = d.plus[2 * m + 1];
            dminus[2 * (f0 + m)] = d.minus[2 * m];
            dminus[2 * (f0 + m) + 1] = d.minus[2 * m + 1];
            dof_dom[f0 + m] = i;
        }
    }
    std::vector<int4> symtiles;
    for (int i = 0; i <= M; ++i) {
        // column block by column block: the four tiles of a workgroup are vertically adjacent, so
        // their column segments are contiguous in memory
        for (int bj = 0; bj < doms[i].nchunk; ++bj)
            for (int bi = 0; bi <= bj; ++bi) symtiles.push_back(make_int4(i, bi, bj, 0));
    }
    // touching-pair pattern of the strictly lower triangle: (m, n), n < m, whose supports share a
    // vertex (CSR over the global dof index, local column n)
    std::vector<int64_t> nearptr(dof + 1, 0);
    std::vector<int32_t> nearcol;
    for (int i = 0; i <= M; ++i) {
        const Domain& d = sk.dom[i];
        std::unordered_map<int32_t, std::vector<int32_t>> vtri;        // global vertex -> local triangles
        for (int lt = 0; lt < d.T; ++lt)
            for (int a = 0; a < 3; ++a) vtri[d.verts[3 * lt + a]].push_back(lt);
        std::vector<int32_t> cols;
        for (int m = 0; m < d.E; ++m) {
            cols.clear();
            for (int side = 0; side < 2; ++side) {
                const int lt = side == 0 ? d.plus[2 * m] : d.minus[2 * m];
                for (int a = 0; a < 3; ++a)
                    for (int t2 : vtri[d.verts[3 * lt + a]])
                        for (int b = 0; b < 3; ++b) {
                            const int n = d.tri_dof[3 * t2 + b];
                            if (n < m) cols.push_back(n);
                        }
            }
            std::sort(cols.begin(), cols.end());
            cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
            nearcol.insert(nearcol.end(), cols.begin(), cols.end());
            nearptr[doms[i].dof0 + m + 1] = (int64_t)nearcol.size();
        }
    }
    // greedy colouring of subdomains 1..M (adjacent subdomains get different colours); stage 0 is Omega_0
    std::vector<int> colour(M + 1, -1);
    colour[0] = 0;
    int ncol = 0;
    for (int i = 1; i <= M; ++i) {
        std::vector<char> used(M + 2, 0);
        for (int lt = 0; lt < sk.dom[i].T; ++lt) {
            const int j = sk.dom[i].other[lt];
            if (j > 0 && colour[j] > 0) used[colour[j]] = 1;
        }
        int c = 1;
        while (used[c]) ++c;
        colour[i] = c;
        ncol = std::max(ncol, c);
    }
    std::vector<int32_t> sdofs;
    std::vector<int64_t> sd0{0};
    for (int c = 0; c <= ncol; ++c) {
        for (int i = 0; i <= M; ++i) {
            if (colour[i] != c) continue;
            const int E = sk.dom[i].E;
            for (int m = 0; m < E; ++m) sdofs.push_back((int32_t)(doms[i].dof0 + m));
        }
        sd0.push_back((int64_t)sdofs.size());
    }
    std::vector<SingPair> sing(sk.singular.size());
    for (size_t q = 0; q < sk.singular.size(); ++q) {
        const auto& a = sk.singular[q];
        SingPair& b = sing[q];
        b.dom = a.domain; b.tx = a.tx; b.ty = a.ty; b.kind = a.kind;
        for (int k = 0; k < 3; ++k) { b.px[k] = a.px[k]; b.py[k] = a.py[k]; }
    }

    p->d_xyz.upload(sk.xyz, s);
    p->d_verts.upload(verts, s);
    p->d_tdof.upload(tdof, s);
    p->d_tsign.upload(tsign, s);
    p->d_other_rec.upload(other_rec, s);
    p->d_other_dom.upload(other_dom, s);
    p->d_rec_dom.upload(rec_dom, s);
    p->d_dplus.upload(dplus, s);
    p->d_dminus.upload(dminus, s);
    p->d_dof_dom.upload(dof_dom, s);
    p->tile_variant = -1;                 // separated-pair tile lists are built per variant on demand
    p->d_symtiles.upload(symtiles, s);
    p->nsymtiles = (int64_t)symtiles.size();
    p->d_near_ptr.upload(nearptr, s);
    p->d_near_col.upload(nearcol, s);
    p->near_nnz = (int64_t)nearcol.size();
    p->near64.reset();
    p->near32.reset();
    p->d_sing.upload(sing, s);
    p->d_dom_stage.upload(colour, s);
    p->d_stage_dofs.upload(sdofs, s);
    p->dom_colour = colour;
    p->stage_dof0 = sd0;
    p->doms = doms;
    p->nrec = rec;
    p->ndof = dof;
    p->mat_entries = mat;
    p->part_entries = part;
    p->d_geom.alloc(rec);
    double bary[6][3], w[6];
    triangle_rule6(bary, w);
    launch_tri_setup_rule(p->d_xyz.p, p->d_verts.p, rec, &bary[0][0], w, p->d_geom.p, s);
    p->has_mat = false;
    upload_doms(p);
    p->d_gval.alloc(9 * rec);
    p->d_gcol.alloc(6 * rec);
    launch_gram_local(p->d_doms.p, M + 1, rec, p->d_rec_dom.p, p->d_geom.p, p->d_other_rec.p, p->d_tsign.p,
                      p->d_tdof.p, p->d_other_dom.p, p->d_gval.p, p->d_gcol.p, s);
    p->part.alloc(2 * part);
    HIPCHK(hipGetLastError());
    sync(p);   // host vectors above go out of scope
    p->sk = std::move(sk);
    p->comp_cache.clear();
    p->comp_cached = false;
    p->tiles_built_for = -1;
    p->has_mesh = true;
    p->have64 = p->have32 = p->have_tinv = false;
    p->T64.reset(); p->K64.reset(); p->T32.reset(); p->K32.reset(); p->Tinv.reset();
}

void ensure_ss(mtf_problem p, int order) {
    if (p->ss_order == order && p->d_ss.p) return;
    std::vector<double> tab;
    std::vector<int32_t> meta(8, 0);
    for (int kind = 1; kind <= 3; ++kind) {
        meta[kind] = (int32_t)(tab.size() / 5);
        sauter_schwab_rule(kind, order, tab);
        meta[4 + kind] = (int32_t)(tab.size() / 5) - meta[kind];
    }
    p->d_ss.upload(tab, p->stream);
    p->d_ss_meta.upload(meta, p->stream);
    sync(p);
    p->ss_order = order;
}

void parse_assembly_opts(const mtf_assembly_opts* o, int* prec, int* order, int* flags = nullptr, int* variant = nullptr) {
    *prec = MTF_FP64;
    *order = 4;
    int fl = 0;
    if (o) {
        if (o->struct_size < (int)sizeof(mtf_assembly_opts)) throw ArgError("mtf_assembly_opts.struct_size too small");
        *prec = o->precision;
        if (o->singular_order) *order = o->singular_order;
        fl = o->flags;
    }
    if (fl & ~(MTF_ASSEMBLE_ROUND_FP64 | 0xff00)) throw ArgError("unknown assembly flags");
    const int tv = ((fl >> 8) & 0xff) - 1;
    if (tv >= kTileVariants) throw ArgError("MTF_ASSEMBLE_TILE: variant out of range");
    if ((fl & MTF_ASSEMBLE_ROUND_FP64) && !flags) throw ArgError("MTF_ASSEMBLE_ROUND_FP64 applies to mtf_assemble only");
    if ((fl & MTF_ASSEMBLE_ROUND_FP64) && *prec != MTF_FP32_MIXED)
        throw ArgError("MTF_ASSEMBLE_ROUND_FP64 applies to MTF_FP32_MIXED");
    if (flags) *flags = fl & MTF_ASSEMBLE_ROUND_FP64;
    if (variant) *variant = tv;
    if (*prec != MTF_FP64 && *prec != MTF_FP32_MIXED) throw ArgError("unknown precision");
    if (*order < 1 || *order > 8) throw ArgError("singular_order must be in 1..8");
}

// Allocation of the T_i, K_i arrays (real numbers): the blocks and 64 complex entries of zero
// padding, which the symmetric-read product may read past the last block (masked rows).
int64_t mat_alloc_reals(mtf_problem p) { return 2 * (p->mat_entries + 64); }

// Allocates and zeroes the blocks of one precision and marks them current (kernels launched by the caller).
void assemble_prepare(mtf_problem p, int prec) {
    hipStream_t s = p->stream;
    const int64_t n2 = mat_alloc_reals(p);
    if (prec == MTF_FP64) {
        p->T64.alloc(n2); p->K64.alloc(n2);
        launch_fill(p->T64.p, n2, 0.0, s);
        launch_fill(p->K64.p, n2, 0.0, s);
        p->have64 = true;
    } else {
        p->T32.alloc(n2); p->K32.alloc(n2);
        launch_fill_f(p->T32.p, n2, 0.f, s);
        launch_fill_f(p->K32.p, n2, 0.f, s);
        p->have32 = true;
        p->gm.haveA = false;
    }
    if (p->tinv_prec == prec) p->have_tinv = false;     // its source blocks change
    p->gp.haveA = false;
}

// Touching-pair corrections of the lower triangle for the blocks of `prec` (after their assembly).
void near_corrections(mtf_problem p, int prec) {
    DevBuf<double>& out = prec == MTF_FP64 ? p->near64 : p->near32;
    const size_t need = 4 * (size_t)std::max<int64_t>(p->near_nnz, 1);
    if (out.n < need) out.alloc(need);        // a buffer lent by a batch lane may be larger
    if (prec == MTF_FP64)
        launch_near_diff_f64(p->d_doms.p, p->d_dof_dom.p, p->ndof, p->d_near_ptr.p, p->d_near_col.p, p->T64.p, p->K64.p,
                             out.p, p->stream);
    else
        launch_near_diff_f32(p->d_doms.p, p->d_dof_dom.p, p->ndof, p->d_near_ptr.p, p->d_near_col.p, p->T32.p, p->K32.p,
                             out.p, p->stream);
}

// ---------------------------------------------------------------------------
// autotuning of the separated-pair tiles
// ---------------------------------------------------------------------------
// The launch configuration (tile variant: tile shape, workgroup size and occupancy; and, for the
// persistent batch launch, workgroups per CU) is chosen by timing the candidates on the first
// assembly of a shape class and kept for the process, keyed by (GPU name, launch kind, precision,
// shape class); with the environment variable MTF_TUNE_CACHE naming a file, the choices are also
// read from and appended to it, so that later processes skip the trials.  The shape class is
// floor(log2) of the mean number of triangles per subdomain.
struct TuneChoice {
    int variant = 0, per_cu = 0;
    double seconds = 0.0;
};
std::mutex g_tune_mu;
std::map<std::string, TuneChoice> g_tune;
bool g_tune_loaded = false;
std::vector<std::string> g_tune_log;     // one line per trial of this process (variant, grid, seconds)

std::string tune_key(int device, const char* kind, int prec, int cls) {
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, device));
    std::string name = prop.gcnArchName;
    for (char& c : name)
        if (c == ' ' || c == '|') c = '_';
    return name + "|" + kind + "|" + (prec == MTF_FP64 ? "fp64" : "fp32") + "|" + std::to_string(cls);
}

bool tune_lookup(const std::string& key, TuneChoice* out) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_tune_loaded) {
        g_tune_loaded = true;
        if (const char* f = std::getenv("MTF_TUNE_CACHE")) {
            if (FILE* fp = std::fopen(f, "r")) {
                char k[256];
                TuneChoice c;
                while (std::fscanf(fp, "%255s %d %d %lf", k, &c.variant, &c.per_cu, &c.seconds) == 4)
                    if (c.variant >= 0 && c.variant < kTileVariants && c.per_cu >= 0) g_tune[k] = c;
                std::fclose(fp);
            }
        }
    }
    auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    *out = it->second;
    return true;
}

void tune_store(const std::string& key, const TuneChoice& c) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = c;
    if (const char* f = std::getenv("MTF_TUNE_CACHE")) {
        if (FILE* fp = std::fopen(f, "a")) {
            std::fprintf(fp, "%s %d %d %.9g\n", key.c_str(), c.variant, c.per_cu, c.seconds);
            std::fclose(fp);
        }
    }
}

static_assert(kTileVariants == MTF_TILE_VARIANTS, "the public tile-variant count must match the compiled variants");

int shape_class(double mean_tri) { return mean_tri <= 1.0 ? 0 : (int)std::floor(std::log2(mean_tri)); }

// Separated-pair tile list of the problem for tile variant v (subdomain, first test and trial
// triangle), rebuilt when the variant changes.
void ensure_tiles(mtf_problem p, int v) {
    if (p->tile_variant == v) return;
    int tx, ty, occ;
    tile_variant_shape(v, &tx, &ty, &occ);
    const bool sym = tile_variant_sym(v);
    std::vector<int4> tiles;
    for (int i = 0; i <= p->sk.M; ++i) {
        const int T = p->sk.dom[i].T;
        for (int x0 = 0; x0 < T; x0 += tx)
            for (int y0 = sym ? x0 : 0; y0 < T; y0 += ty) tiles.push_back(make_int4(i, x0, y0, 0));
    }
    p->d_tiles.upload(tiles, p->stream);
    p->ntiles = (int64_t)tiles.size();
    p->tile_variant = v;
    sync(p);
}

// Tile variant for assembling problem p in precision prec: the forced one, else the tuned one of its
// shape class (timing every variant's separated-pair launch once on this problem if none is known).
// The trial launches add into the blocks, which the caller clears afterwards.
int choose_variant(mtf_problem p, int prec, int forced, void* T, void* K) {
    if (forced >= 0) return forced;
    double mean = 0.0;
    for (int i = 0; i <= p->sk.M; ++i) mean += p->sk.dom[i].T;
    mean /= (p->sk.M + 1);
    const std::string key = tune_key(p->device, "single", prec, shape_class(mean));
    TuneChoice c;
    if (tune_lookup(key, &c)) return c.variant;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    TuneChoice best;
    best.seconds = 1e300;
    for (int v = 0; v < kTileVariants; ++v) {
        ensure_tiles(p, v);
        HIPCHK(hipEventRecord(e0, p->stream));
        launch_regular(prec == MTF_FP64 ? 0 : 1, v, p->d_tiles.p, p->ntiles, p->d_doms.p, p->d_geom.p, p->d_verts.p,
                       p->d_tdof.p, p->d_tsign.p, T, K, p->stream);
        HIPCHK(hipGetLastError());
        HIPCHK(hipEventRecord(e1, p->stream));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune_log.push_back(key + " variant " + std::to_string(v) + " " + std::to_string(ms * 1e-3) + " s");
        }
        if (ms * 1e-3 < best.seconds) { best.seconds = ms * 1e-3; best.variant = v; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    tune_store(key, best);
    return best.variant;
}

void assemble_impl(mtf_problem p, const mtf_assembly_opts* o) {
    if (!p->has_mesh || !p->has_mat) throw StateError("mtf_assemble needs mtf_set_mesh and mtf_set_materials first");
    int prec, order, flags, forced;
    parse_assembly_opts(o, &prec, &order, &flags, &forced);
    DeviceGuard g(p->device);
    hipStream_t s = p->stream;
    if (!p->ev0) { HIPCHK(hipEventCreate(&p->ev0)); HIPCHK(hipEventCreate(&p->ev1)); }
    const int64_t n2 = mat_alloc_reals(p);
    if (flags & MTF_ASSEMBLE_ROUND_FP64) {
        // complex64 blocks rounded from the FP64 ones (padding included)
        if (!p->have64) throw StateError("MTF_ASSEMBLE_ROUND_FP64 needs the FP64 blocks: assemble MTF_FP64 first");
        // (buffers lent by a batch lane may be larger than this problem's blocks)
        if (p->T32.n < (size_t)n2) p->T32.alloc(n2);
        if (p->K32.n < (size_t)n2) p->K32.alloc(n2);
        HIPCHK(hipEventRecord(p->ev0, s));
        launch_copy_block_f64_to_f32(p->T64.p, p->T32.p, n2, s);
        launch_copy_block_f64_to_f32(p->K64.p, p->K32.p, n2, s);
        near_corrections(p, MTF_FP32_MIXED);
        HIPCHK(hipGetLastError());
        HIPCHK(hipEventRecord(p->ev1, s));
        p->have32 = true;
        p->gm.haveA = false;
        if (p->tinv_prec == MTF_FP32_MIXED) p->have_tinv = false;
        p->gp.haveA = false;
        return;
    }
    ensure_ss(p, order);
    if (prec == MTF_FP64) { p->T64.alloc(n2); p->K64.alloc(n2); }
    else { p->T32.alloc(n2); p->K32.alloc(n2); }
    const int variant = choose_variant(p, prec, forced, prec == MTF_FP64 ? (void*)p->T64.p : (void*)p->T32.p,
                                       prec == MTF_FP64 ? (void*)p->K64.p : (void*)p->K32.p);
    ensure_tiles(p, variant);
    p->last_variant = variant;
    HIPCHK(hipEventRecord(p->ev0, s));
    const int32_t* meta = p->d_ss_meta.p;
    if (prec == MTF_FP64) {
        launch_fill(p->T64.p, n2, 0.0, s);
        launch_fill(p->K64.p, n2, 0.0, s);
        launch_regular(0, variant, p->d_tiles.p, p->ntiles, p->d_doms.p, p->d_geom.p, p->d_verts.p, p->d_tdof.p,
                       p->d_tsign.p, p->T64.p, p->K64.p, s);
        launch_singular(p->d_sing.p, (int64_t)p->d_sing.n, p->d_doms.p, p->d_geom.p, p->d_xyz.p, p->d_verts.p,
                        p->d_tdof.p, p->d_tsign.p, p->d_ss.p, meta, meta + 4, p->T64.p, p->K64.p, nullptr, nullptr, s);
    } else {
        launch_fill_f(p->T32.p, n2, 0.f, s);
        launch_fill_f(p->K32.p, n2, 0.f, s);
        launch_regular(1, variant, p->d_tiles.p, p->ntiles, p->d_doms.p, p->d_geom.p, p->d_verts.p, p->d_tdof.p,
                       p->d_tsign.p, p->T32.p, p->K32.p, s);
        launch_singular(p->d_sing.p, (int64_t)p->d_sing.n, p->d_doms.p, p->d_geom.p, p->d_xyz.p, p->d_verts.p,
                        p->d_tdof.p, p->d_tsign.p, p->d_ss.p, meta, meta + 4, nullptr, nullptr, p->T32.p, p->K32.p, s);
    }
    near_corrections(p, prec);
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(p->ev1, s));
    if (prec == MTF_FP64) p->have64 = true; else { p->have32 = true; p->gm.haveA = false; }
    if (p->tinv_prec == prec) p->have_tinv = false;      // its source blocks change
    p->gp.haveA = false;
}

void check_prec_available(mtf_problem p, int prec) {
    if (prec == MTF_FP64 && !p->have64) throw StateError("FP64 blocks not assembled");
    if ((prec == MTF_FP32_MIXED || prec == MTF_BF16_SPLIT) && !p->have32)
        throw StateError("FP32 blocks not assembled (MTF_FP32_MIXED)");
    if (prec != MTF_FP64 && prec != MTF_FP32_MIXED && prec != MTF_BF16_SPLIT) throw ArgError("unknown precision");
}

// GEMM descriptors, tiles and workspaces of one multi-RHS operator (mode 0: the diagonal
// blocks [K_i | T_i]; mode 1: the preconditioner blocks T_i^-1) for nrhs columns; the bf16
// A planes are rebuilt whenever their source blocks change.
void gemm_prepare(mtf_problem p, GemmOp& op, int mode, int nrhs) {
    if (op.haveA && op.nrhs == nrhs) return;
    hipStream_t s = p->stream;
    const int ndom = (int)p->doms.size();
    const int64_t Np = ((2 * (int64_t)nrhs + 127) / 128) * 128;
    std::vector<GemmDesc> gd(ndom);
    std::vector<int4> tiles;
    int64_t a = 0, b = 0, c = 0, kpmax = 0;
    for (int i = 0; i < ndom; ++i) {
        const int64_t E = p->doms[i].E;
        GemmDesc& g = gd[i];
        g.Mp = ((E + 127) / 128) * 128;
        g.Kp = (((mode == 0 ? 2 * E : E) + 31) / 32) * 32;
        g.Np = Np;
        g.M = E;
        g.N = 2 * nrhs;
        g.ldc = E;
        g.a_off = a;
        g.b_off = b;
        g.c_off = c;
        a += 4 * g.Mp * g.Kp;
        b += 4 * g.Np * g.Kp;
        c += E * 2 * nrhs;
        kpmax = std::max(kpmax, g.Kp);
        for (int64_t m0 = 0; m0 < g.Mp; m0 += 128)
            for (int64_t n0 = 0; n0 < Np; n0 += 128) tiles.push_back(make_int4(i, (int)m0, (int)n0, 0));
    }
    op.d.upload(gd, s);
    op.tiles.upload(tiles, s);
    op.ntiles = (int64_t)tiles.size();
    op.kpmax = kpmax;
    op.np = Np;
    op.B.alloc(b);
    op.C.alloc(2 * c);
    if (!op.haveA) {
        op.A.alloc(a);
        std::vector<int4> st;
        for (int i = 0; i < ndom; ++i)
            for (int64_t r0 = 0; r0 < gd[i].Mp; r0 += 64)
                for (int64_t k0 = 0; k0 < gd[i].Kp; k0 += 64) st.push_back(make_int4(i, (int)r0, (int)k0, 0));
        DevBuf<int4> dst;
        dst.upload(st, s);
        const float* T = mode == 0 ? p->T32.p : p->Tinv.p;
        const float* K = mode == 0 ? p->K32.p : p->Tinv.p;
        launch_split_A(op.d.p, p->d_doms.p, dst.p, (int64_t)st.size(), T, K, op.A.p, mode, s);
        HIPCHK(hipGetLastError());
        sync(p);
    }
    op.nrhs = nrhs;
    op.haveA = true;
}

// Y = M X (mode 0) or Z = P X (mode 1) for nrhs columns of ld with the MFMA block products.
void apply_gemm(mtf_problem p, int mode, int nrhs, const double* x, int64_t ld, double* y) {
    GemmOp& op = mode == 0 ? p->gm : p->gp;
    gemm_prepare(p, op, mode, nrhs);
    hipStream_t s = p->stream;
    launch_split_B(op.d.p, p->d_doms.p, (int)p->doms.size(), op.kpmax, op.np, x, ld, nrhs, op.B.p, mode, s);
    launch_gemm_bf16x3(op.d.p, op.tiles.p, op.ntiles, op.A.p, op.B.p, op.C.p, s);
    launch_gemm_finish(p->d_doms.p, op.d.p, p->d_dof_dom.p, p->ndof, p->d_dplus.p, p->d_dminus.p, p->d_gval.p,
                       p->d_gcol.p, op.C.p, x, y, ld, nrhs, mode, s);
}

void matvec_gemm(mtf_problem p, int nrhs, const double* x, int64_t ld, double* y) { apply_gemm(p, 0, nrhs, x, ld, y); }

// y = M x for one vector (device pointers, complex128 length N); the column-chunk partial sums go
// to `part` (the problem's own buffer unless given: 2 * part_entries doubles, every slot written
// before it is read, so it needs no clearing)
void matvec1(mtf_problem p, const double* x, double* y, int prec, double* part = nullptr) {
    hipStream_t s = p->stream;
    if (!part) part = p->part.p;
    if (prec == MTF_FP64)
        launch_matvec_sym_f64(p->d_doms.p, p->d_symtiles.p, p->nsymtiles, p->T64.p, p->K64.p, x, part, s);
    else
        launch_matvec_sym_f32(p->d_doms.p, p->d_symtiles.p, p->nsymtiles, p->T32.p, p->K32.p, x, part, s);
    launch_matvec_sym_finish(p->d_doms.p, p->d_dof_dom.p, p->ndof, p->d_dplus.p, p->d_dminus.p, p->d_gval.p,
                             p->d_gcol.p, p->d_near_ptr.p, p->d_near_col.p,
                             prec == MTF_FP64 ? p->near64.p : p->near32.p, part, x, y, s);
}

constexpr int kMmvCols = 1536;   // columns of T_i, K_i per work item of the FP64 multi-RHS product

// Y = M X for q <= 32 vectors (ld ldx, ldy) with the FP64 multi-RHS product on the matrix cores;
// the work items (largest column ranges first) and partial sums are kept per q.
void matvec_mmv(mtf_problem p, int q, const double* X, int64_t ldx, double* Y, int64_t ldy) {
    MmvPlan& mp = p->mmv;
    hipStream_t s = p->stream;
    if (mp.q != q) {
        std::vector<int4> items;
        std::vector<int64_t> pbase;
        std::vector<int> nsp;
        int64_t tot = 0;
        for (size_t d = 0; d < p->doms.size(); ++d) {
            const int E = p->doms[d].E;
            const int ns = (E + kMmvCols - 1) / kMmvCols;
            pbase.push_back(tot);
            nsp.push_back(ns);
            tot += (int64_t)ns * q * 2 * E;
            for (int sp = 0; sp < ns; ++sp)
                for (int r0 = 0; r0 < E; r0 += mmv_rows(q))
                    for (int c0 = 0; c0 < q; c0 += mmv_rhs_step(q)) items.push_back(make_int4((int)d, r0, c0, sp));
        }
        auto span = [&](const int4& it) { return std::min(kMmvCols, p->doms[it.x].E - it.w * kMmvCols); };
        std::stable_sort(items.begin(), items.end(), [&](const int4& a, const int4& b) { return span(a) > span(b); });
        mp.items.upload(items, s);
        mp.pbase.upload(pbase, s);
        mp.nsplit.upload(nsp, s);
        mp.part.alloc((size_t)2 * tot);
        mp.nitems = (int64_t)items.size();
        mp.q = q;
        sync(p);
    }
    launch_mmv(p->d_doms.p, mp.items.p, mp.nitems, p->T64.p, p->K64.p, X, ldx, q, mp.pbase.p, kMmvCols, mp.part.p,
               p->d_dof_dom.p, p->ndof, p->d_dplus.p, p->d_dminus.p, p->d_gval.p, p->d_gcol.p, mp.nsplit.p, Y, ldy, s);
}

// Z = P X for q <= 32 vectors (ld ld) with the block preconditioner read whole on the matrix cores:
// per Gauss-Seidel stage the stage input for all q vectors (into W, q x ld), then one launch over
// the stage's subdomains; for MTF_PREC_BLOCK_TINV one launch over every subdomain.
void precond_block(mtf_problem p, int pc, int q, const double* X, double* Z, double* W, int64_t ld) {
    PcmmPlan& pp = p->pcmm;
    hipStream_t s = p->stream;
    const int nd = (int)p->doms.size();
    const int nst = pc == MTF_PREC_BLOCK_TINV_GS ? (int)p->stage_tile0.size() - 1 : 1;
    if (pp.q != q || pp.pc != pc) {
        std::vector<int4> items;
        std::vector<int64_t> pbase(nd);
        std::vector<int> nsp(nd);
        int64_t tot = 0;
        for (int d = 0; d < nd; ++d) {
            const int E = p->doms[d].E;
            nsp[d] = (E + kMmvCols - 1) / kMmvCols;
            pbase[d] = tot;
            tot += (int64_t)nsp[d] * q * 2 * E;
        }
        pp.item0.assign(1, 0);
        auto span = [&](const int4& it) { return std::min(kMmvCols, p->doms[it.x].E - it.w * kMmvCols); };
        for (int st = 0; st < nst; ++st) {
            const size_t first = items.size();
            for (int d = 0; d < nd; ++d) {
                if (nst > 1 && p->dom_colour[d] != st) continue;
                const int E = p->doms[d].E;
                for (int sp = 0; sp < nsp[d]; ++sp)
                    for (int r0 = 0; r0 < E; r0 += mmv_rows(q))
                        for (int c0 = 0; c0 < q; c0 += mmv_rhs_step(q)) items.push_back(make_int4(d, r0, c0, sp));
            }
            std::stable_sort(items.begin() + first, items.end(),
                             [&](const int4& a, const int4& b) { return span(a) > span(b); });
            pp.item0.push_back((int64_t)items.size());
        }
        pp.items.upload(items, s);
        pp.pbase.upload(pbase, s);
        pp.nsplit.upload(nsp, s);
        pp.part.alloc((size_t)2 * tot);
        pp.q = q;
        pp.pc = pc;
        sync(p);
    }
    for (int st = 0; st < nst; ++st) {
        const int4* it = pp.items.p + pp.item0[st];
        const int64_t nit = pp.item0[st + 1] - pp.item0[st];
        if (nst == 1) {
            launch_pcmm(p->d_doms.p, it, nit, p->Tinv.p, X, ld, q, pp.pbase.p, kMmvCols, pp.part.p, p->d_dof_dom.p,
                        nullptr, p->ndof, pp.nsplit.p, Z, ld, s);
            continue;
        }
        const int32_t* dl = p->d_stage_dofs.p + p->stage_dof0[st];
        const int64_t ndl = p->stage_dof0[st + 1] - p->stage_dof0[st];
        const double* in = X;
        if (st > 0) {
            launch_gs_residual_q(p->d_doms.p, p->d_dof_dom.p, dl, ndl, p->d_dplus.p, p->d_dminus.p, p->d_gval.p,
                                 p->d_gcol.p, p->d_other_dom.p, p->d_dom_stage.p, st, X, Z, W, ld, q, s);
            in = W;
        }
        launch_pcmm(p->d_doms.p, it, nit, p->Tinv.p, in, ld, q, pp.pbase.p, kMmvCols, pp.part.p, p->d_dof_dom.p, dl, ndl,
                    pp.nsplit.p, Z, ld, s);
    }
}

// Partial sums of the allocation-free product (mtf_matvec_noalloc): a fixed array in device
// memory, one copy per GPU that the library runs on, held until the process ends.  Host code never
// passes `scratch` itself to a kernel (on the host that name is only a stand-in for the symbol):
// the device address of each GPU's copy is looked up once per device with hipGetSymbolAddress,
// with that device current, and that address is what the kernels receive.
constexpr int64_t kScratchReals = int64_t(8) << 20;     // 64 MiB of doubles = 4 Mi complex partial sums
static __device__ __align__(256) double scratch[kScratchReals];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (the device must be current).
double* scratch_on(int device) {
    if (device < 0 || device >= kMaxDevices) throw ArgError("device id out of range for the static scratch");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void* ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) throw HipError("hipGetSymbolAddress returned no address for the static scratch");
        g_scratch_dev[device] = static_cast<double*>(ptr);
    }
    return g_scratch_dev[device];
}

void precond1(mtf_problem p, const double* x, double* z) {
    launch_precond_sym(p->d_doms.p, p->d_pctiles.p, p->npctiles, p->Tinv.p, x, p->part.p, p->stream);
    launch_precond_sym_finish(p->d_doms.p, p->d_dof_dom.p, p->ndof, p->part.p, p->d_pc_slots.p, z, nullptr, p->stream);
}

// z = P_GS x: one block Gauss-Seidel sweep over the stages with the T_i^-1 block of each subdomain;
// within a stage the subdomains are not adjacent and are processed together.
void precond1_gs(mtf_problem p, const double* x, double* z, double* w) {
    hipStream_t s = p->stream;
    const int nst = (int)p->stage_tile0.size() - 1;
    for (int st = 0; st < nst; ++st) {
        const int4* tiles = p->d_stage_tiles.p + p->stage_tile0[st];
        const int64_t ntl = p->stage_tile0[st + 1] - p->stage_tile0[st];
        const int32_t* dl = p->d_stage_dofs.p + p->stage_dof0[st];
        const int64_t nd = p->stage_dof0[st + 1] - p->stage_dof0[st];
        const double* in = x;
        if (st > 0) {
            launch_gs_residual(p->d_doms.p, p->d_dof_dom.p, dl, nd, p->d_dplus.p, p->d_dminus.p, p->d_gval.p, p->d_gcol.p,
                               p->d_other_dom.p, p->d_dom_stage.p, st, x, z, w, s);
            in = w;
        }
        launch_precond_sym(p->d_doms.p, tiles, ntl, p->Tinv.p, in, p->part.p, s);
        launch_precond_sym_finish(p->d_doms.p, p->d_dof_dom.p, nd, p->part.p, p->d_pc_slots.p, z, dl, s);
    }
}

// Second stream and events for the lookahead of block_gj_inverse (default priority, like every
// stream here).
struct GjLookahead {
    hipStream_t s2 = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};

// In-place inverse of `batch` n x n complex64 matrices X + z*stride (leading dimension ld) by
// blocked Gauss-Jordan elimination over diagonal blocks P of width w <= W:
//   X_PP <- X_PP^-1;  X_Pj <- X_PP X_Pj;  X_ij <- X_ij - X_iP X_Pj;  X_iP <- -X_iP X_PP   (i, j not in P)
// The rank-w update is one batched matrix-core GEMM over the whole matrix minus the band P; it
// reads and writes the matrix once per block, so wider blocks cut the traffic.  X_PP is inverted
// by the same elimination with 64-wide blocks (pivoting within each 64 x 64 leaf).  A panel is
// updated in place when one workgroup tile spans its reduced dimension (128 rows, 64 columns);
// otherwise through `tmp` (W * n complex entries per matrix) and a copy back.
// With `la` (lookahead), the rank-w update first forms the next diagonal block X_P'P' (P' the block
// after P), which is then inverted on la->s2 while s carries on with the rest of the update and
// the column panel; s waits for it before the next row panel.  The leaf inversions, which occupy
// one CU each, then overlap the large update instead of following it.  P and P' are adjacent, so
// every piece of the update is a GEMM with one skipped band of rows and one of columns:
//   rows P', columns P' (first);  rows outside P u P', columns outside P;
//   rows P', columns outside P u P'.
void block_gj_inverse(float* X, int n, int64_t ld, int64_t stride, int batch, int* info, hipStream_t s, int W,
                      float* tmp, const GjLookahead* la = nullptr) {
    constexpr int kTileRows = 128, kTileCols = 64;
    const int64_t ts = (int64_t)W * n;                 // tmp stride per matrix (complex entries)
    auto invert_diag = [&](int q0, int w, hipStream_t st) {
        float* Xqq = X + 2 * (q0 + (int64_t)q0 * ld);
        if (w <= 64) launch_cinv_small_f32(Xqq, ld, stride, w, batch, info, st);
        else block_gj_inverse(Xqq, w, ld, stride, batch, info, st, 64, tmp);
    };
    // D(rows, cols) -= X(rows, P) X(P, cols): compact rows r -> r + (r >= rg0 ? rgw : 0), likewise cols
    auto update = [&](int p0, int w, int m, int rg0, int rgw, int nn, int cg0, int cgw) {
        if (m <= 0 || nn <= 0) return;
        CGemm t;
        t.m = m; t.n = nn; t.k = w; t.batch = batch; t.ar = -1.f; t.beta = 1.f;
        t.A = X + 2 * ((int64_t)p0 * ld); t.lda = ld; t.sA = stride;
        t.B = X + 2 * (int64_t)p0; t.ldb = ld; t.sB = stride;
        t.C = X; t.ldc = ld; t.sC = stride;
        t.D = X; t.ldd = ld; t.sD = stride;
        t.rg0 = rg0; t.rgw = rgw; t.cg0 = cg0; t.cgw = cgw;
        launch_cgemm_f32(t, s);
    };
    invert_diag(0, std::min(W, n), s);
    for (int p0 = 0; p0 < n; p0 += W) {
        const int w = std::min(W, n - p0);
        float* Xpp = X + 2 * (p0 + (int64_t)p0 * ld);
        float* Xrow = X + 2 * (int64_t)p0;            // row p0, column 0
        float* Xcol = X + 2 * ((int64_t)p0 * ld);     // row 0, column p0
        if (w == n) break;
        CGemm r;                                      // row panel
        r.m = w; r.n = n - w; r.k = w; r.batch = batch;
        r.A = Xpp; r.lda = ld; r.sA = stride;
        r.B = Xrow; r.ldb = ld; r.sB = stride;
        r.cg0 = p0; r.cgw = w;
        if (w <= kTileRows) {
            r.D = Xrow; r.ldd = ld; r.sD = stride;
            launch_cgemm_f32(r, s);
        } else {
            r.D = tmp; r.ldd = w; r.sD = ts; r.band_cd = 0;
            launch_cgemm_f32(r, s);
            launch_band_copy_f32(tmp, w, ts, Xrow, ld, stride, w, n - w, w, 0, p0, w, batch, s);
        }
        const int q0 = p0 + w, w2 = std::min(W, n - q0);   // the next block P' (w2 <= 0: none)
        if (la && w2 > 0) {
            update(p0, w, w2, 0, q0, w2, 0, q0);                          // rows P', columns P'
            HIPCHK(hipEventRecord(la->fork, s));
            HIPCHK(hipStreamWaitEvent(la->s2, la->fork, 0));
            invert_diag(q0, w2, la->s2);
            HIPCHK(hipEventRecord(la->join, la->s2));
            update(p0, w, n - w - w2, p0, w + w2, n - w, p0, w);          // rows outside P u P'
            update(p0, w, w2, 0, q0, n - w - w2, p0, w + w2);             // rows P', columns outside P u P'
        } else {
            update(p0, w, n - w, p0, w, n - w, p0, w);                    // everything outside P
        }
        CGemm c;                                      // column panel
        c.m = n - w; c.n = w; c.k = w; c.batch = batch; c.ar = -1.f;
        c.A = Xcol; c.lda = ld; c.sA = stride;
        c.B = Xpp; c.ldb = ld; c.sB = stride;
        c.rg0 = p0; c.rgw = w;
        if (w <= kTileCols) {
            c.D = Xcol; c.ldd = ld; c.sD = stride;
            launch_cgemm_f32(c, s);
        } else {
            c.D = tmp; c.ldd = n - w; c.sD = ts; c.band_cd = 0;
            launch_cgemm_f32(c, s);
            launch_band_copy_f32(tmp, n - w, ts, Xcol, ld, stride, n - w, w, p0, w, w, 0, batch, s);
        }
        if (w2 > 0) {
            if (la) HIPCHK(hipStreamWaitEvent(s, la->join, 0));
            else invert_diag(q0, w2, s);
        }
    }
}

std::vector<std::pair<int, int>> dof_components(const Domain& d);

// dof_components of every Gamma_i of the problem's mesh, computed on first use
const std::vector<std::pair<int, int>>& domain_components(mtf_problem p, int i) {
    if (!p->comp_cached) {
        p->comp_cache.assign(p->sk.dom.size(), {});
        for (size_t d = 0; d < p->sk.dom.size(); ++d)
            if (p->sk.dom[d].E > 0) p->comp_cache[d] = dof_components(p->sk.dom[d]);
        p->comp_cached = true;
    }
    return p->comp_cache[i];
}

// Preconditioner tile lists (all subdomains, and per Gauss-Seidel stage) and the partial slots each
// row chunk sums.  A block inverted over the connected components of Gamma_i (contiguous dof
// ranges, zero between components; `per_component`) lists only the 64 x 64 tiles that meet a
// component's diagonal block: with Imin(J) = lo(component holding dof 64 J) / 64, nondecreasing in
// J, tile (I, J), I <= J, meets one iff I >= Imin(J) (the component must reach from row chunk I
// to column chunk J).  A symmetric block lists those tiles (I <= J); the rows of chunk B then get
// transposed parts from tiles (I, B), I in [Imin(B), B], in slots I, and direct parts from tiles
// (B, J), J in [B, Jmax(B)], in slots J + 1, Jmax(B) the last J with Imin(J) <= B: slots
// [Imin(B), Jmax(B) + 1].  A whole-use block (the inverse of T_i itself) lists both orders and
// uses direct parts only: slots [Imin(B) + 1, Jmax(B) + 1].  A connected Gamma_i has Imin = 0.
void build_pc_tiles(mtf_problem p, bool per_component) {
    // the lists depend on the mesh, the component flag and pc_full only
    if (p->tiles_built_for == (per_component ? 1 : 0) && p->tiles_built_full == p->pc_full) return;
    const auto& D = p->doms;
    const int nd = (int)D.size();
    std::vector<std::vector<int>> imin(nd), jmax(nd);
    std::vector<int2> slots;
    for (int i = 0; i < nd; ++i) {
        const int nb = D[i].nchunk;
        std::vector<std::pair<int, int>> comps;
        if (per_component && D[i].E > 0) comps = domain_components(p, i);
        std::vector<int>& lo = imin[i];
        std::vector<int>& hi = jmax[i];
        lo.assign(nb, 0);
        hi.assign(nb, nb - 1);
        if (!comps.empty()) {
            size_t c = 0;
            for (int J = 0; J < nb; ++J) {
                while (comps[c].second <= J * kChunk) ++c;
                lo[J] = comps[c].first / kChunk;
            }
            int J = 0;
            for (int B = 0; B < nb; ++B) {
                while (J + 1 < nb && lo[J + 1] <= B) ++J;
                hi[B] = std::max(J, B);
            }
        }
        for (int B = 0; B < nb; ++B)
            slots.push_back(make_int2(p->pc_full[i] ? lo[B] + 1 : lo[B], hi[B] + 1));
    }
    auto tiles_of = [&](int i, std::vector<int4>& out) {
        const int nb = D[i].nchunk;
        const bool full = p->pc_full[i] != 0;
        for (int bj = 0; bj < nb; ++bj)
            for (int bi = 0; bi < nb; ++bi) {
                const bool meets = bi <= bj ? bi >= imin[i][bj] : (full && bj >= imin[i][bi]);
                if (meets) out.push_back(make_int4(i, bi, bj, full ? 1 : 0));
            }
    };
    std::vector<int4> all, st;
    std::vector<int64_t> st0{0};
    for (int i = 0; i < nd; ++i) tiles_of(i, all);
    const int ncol = *std::max_element(p->dom_colour.begin(), p->dom_colour.end());
    for (int c = 0; c <= ncol; ++c) {
        for (int i = 0; i < nd; ++i)
            if (p->dom_colour[i] == c) tiles_of(i, st);
        st0.push_back((int64_t)st.size());
    }
    p->d_pctiles.upload(all, p->stream);
    p->npctiles = (int64_t)all.size();
    p->d_stage_tiles.upload(st, p->stream);
    p->stage_tile0 = st0;
    p->d_pc_slots.upload(slots, p->stream);
    p->tiles_built_for = per_component ? 1 : 0;
    p->tiles_built_full = p->pc_full;
}

// Connected components of Gamma_i (its triangles joined through shared dofs) as dof ranges
// [lo, hi), in dof order.  Empty when Gamma_i is connected, or when a component's dofs do not form
// one contiguous range (then the block is treated whole).
std::vector<std::pair<int, int>> dof_components(const Domain& d) {
    const int E = d.E;
    std::vector<int> par(E);
    for (int m = 0; m < E; ++m) par[m] = m;
    auto root = [&](int m) {
        while (par[m] != m) m = par[m] = par[par[m]];
        return m;
    };
    for (int lt = 0; lt < d.T; ++lt) {
        const int a = root(d.tri_dof[3 * lt]);
        for (int q = 1; q < 3; ++q) {
            const int b = root(d.tri_dof[3 * lt + q]);
            if (a != b) par[b] = a;
        }
    }
    std::vector<std::pair<int, int>> runs;
    std::vector<char> seen(E, 0);
    for (int m = 0; m < E;) {
        const int r = root(m);
        if (seen[r]) return {};                        // the component comes back: not contiguous
        seen[r] = 1;
        int n = m + 1;
        while (n < E && root(n) == r) ++n;
        runs.emplace_back(m, n);
        m = n;
    }
    if (runs.size() < 2) return {};
    return runs;
}

void ensure_gj_streams(mtf_problem p);

// Blocks of the T_i^-1 preconditioner, complex64.  Each block is first the inverse of the
// symmetric part S_i = (T_i + T_i^T)/2, applied reading half of its entries.  Where Gamma_i has
// several connected components (the exterior of disjoint scatterers), S_i is replaced by its
// block diagonal over the components, each block inverted on its own: the cost of the inverse
// falls from the cube of the whole order to the sum of the components' cubes.  S_i differs from T_i
// by the two-order quadrature difference of touching pairs; where T_i is ill-conditioned that
// difference is amplified in the inverse.  So every block is checked on a fixed vector v: when
// ||T_i (S_i^-1 v) - v|| > kPcSymTol ||v||, the block is rebuilt as the inverse of T_i itself (per
// component) and read whole.  kind kPcDirect builds every block that way at once (no symmetric
// attempt, no check); kPcWhole inverts the whole T_i, components or not.
void build_tinv(mtf_problem p, int kind) {
    if (p->have_tinv && p->pc_kind == kind) return;
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = p->stream;
    const auto& D = p->doms;
    const int nd = (int)D.size();
    // 64 complex entries of padding: the symmetric-read apply may read up to 63 entries past the
    // last block (masked rows of its last column)
    p->Tinv.alloc(2 * (p->mat_entries + 64));
    HIPCHK(hipMemsetAsync(p->Tinv.p + 2 * p->mat_entries, 0, 2 * 64 * sizeof(float), s));
    DevBuf<int> info;
    info.alloc(2);
    HIPCHK(hipMemsetAsync(info.p, 0, 2 * sizeof(int), s));
    // streams of the inversions: non-blocking, so that they also overlap work on a caller's null
    // stream; ordered by events only
    ensure_gj_streams(p);
    GjLookahead la[2];
    for (int l = 0; l < 2; ++l) {
        la[l].s2 = p->gj_aux[l];
        la[l].fork = p->gj_fork[l];
        la[l].join = p->gj_join[l];
    }
    // T_i in complex64 (kept for the check and the rebuilt blocks)
    DevBuf<float> tcopy;
    const float* T32 = p->T32.p;
    if (!p->have32) {
        tcopy.alloc(2 * p->mat_entries);
        launch_copy_block_f64_to_f32(p->T64.p, tcopy.p, 2 * p->mat_entries, s);
        T32 = tcopy.p;
    }
    HIPCHK(hipMemcpyAsync(p->Tinv.p, T32, 2 * p->mat_entries * sizeof(float), hipMemcpyDeviceToDevice, s));
    p->pc_full.assign(nd, kind != kPcSym ? 1 : 0);
    for (int i = 0; i < nd; ++i)
        if (D[i].E > 0 && !p->pc_full[i]) launch_symmetrize_f32(p->Tinv.p + 2 * D[i].mat0, D[i].E, s);
    // several components: block diagonal over them (entries between components cleared)
    std::vector<std::vector<std::pair<int, int>>> comps(nd);
    std::vector<std::vector<int32_t>> cidh(nd);        // kept until the build synchronises
    std::vector<DevBuf<int32_t>> cids(nd);
    for (int i = 0; i < nd; ++i) {
        if (D[i].E == 0 || kind == kPcWhole) continue;
        comps[i] = domain_components(p, i);
        if (comps[i].empty()) continue;
        std::vector<int32_t>& cid = cidh[i];
        cid.resize(D[i].E);
        for (size_t q = 0; q < comps[i].size(); ++q)
            for (int m = comps[i][q].first; m < comps[i][q].second; ++m) cid[m] = (int32_t)q;
        cids[i].upload(cid, s);
        launch_zero_offdiag_f32(p->Tinv.p + 2 * D[i].mat0, D[i].E, cids[i].p, s);
    }
    // consecutive subdomains of equal size are stored back to back and inverted as one batch; the
    // groups are independent, so the one with the most work (the largest order) runs on lane 0 and
    // all others, one after another, on lane 1, each lane with its own scratch for the panels
    struct Group {
        int a, b;
        int64_t E;
    };
    std::vector<Group> groups;
    int64_t emax = 0;
    for (int a = 0; a < nd;) {
        int b = a + 1;
        const int64_t E = D[a].E;
        while (b < nd && D[b].E == E && D[b].mat0 == D[a].mat0 + (int64_t)(b - a) * E * E) ++b;
        if (E > 0) groups.push_back(Group{a, b, E});
        emax = std::max<int64_t>(emax, E);
        a = b;
    }
    size_t big = 0;
    for (size_t g = 1; g < groups.size(); ++g)
        if (groups[g].E > groups[big].E) big = g;
    int64_t tmp_entries[2] = {1, 1};                   // out-of-place panels: W * E per matrix of a batch
    for (size_t g = 0; g < groups.size(); ++g) {
        const int l = g == big ? 0 : 1;
        tmp_entries[l] = std::max(tmp_entries[l], (int64_t)(groups[g].b - groups[g].a) * kGjPanel * groups[g].E);
    }
    DevBuf<float> gjtmp[2];
    for (int l = 0; l < 2; ++l) gjtmp[l].alloc(2 * tmp_entries[l]);
    HIPCHK(hipEventRecord(p->gj_start, s));
    for (int l = 0; l < 2; ++l) HIPCHK(hipStreamWaitEvent(p->gj_lane[l], p->gj_start, 0));
    for (size_t g = 0; g < groups.size(); ++g) {
        const int l = g == big ? 0 : 1;
        const Group& q = groups[g];
        if (q.b - q.a == 1 && !comps[q.a].empty()) {
            for (const auto& c : comps[q.a]) {          // each component's diagonal block, in place
                const int64_t o = c.first + (int64_t)c.first * q.E;
                block_gj_inverse(p->Tinv.p + 2 * (D[q.a].mat0 + o), c.second - c.first, q.E, q.E * q.E, 1, info.p,
                                 p->gj_lane[l], kGjPanel, gjtmp[l].p, &la[l]);
            }
            continue;
        }
        block_gj_inverse(p->Tinv.p + 2 * D[q.a].mat0, (int)q.E, q.E, q.E * q.E, q.b - q.a, info.p, p->gj_lane[l],
                         kGjPanel, gjtmp[l].p, &la[l]);
    }
    for (int l = 0; l < 2; ++l) {
        HIPCHK(hipEventRecord(p->gj_done[l], p->gj_lane[l]));
        HIPCHK(hipStreamWaitEvent(s, p->gj_done[l], 0));
    }
    if (kind == kPcSym && emax > 0) {
        // check ||T_i (X_i v) - v|| / ||v|| with v_m = (cos m, sin 2m) per block
        std::vector<float> vh(2 * emax);
        for (int64_t m = 0; m < emax; ++m) { vh[2 * m] = (float)std::cos((double)m); vh[2 * m + 1] = (float)std::sin(2.0 * m); }
        std::vector<int64_t> uoff(nd + 1, 0);          // T_i X_i v of every block, back to back
        for (int i = 0; i < nd; ++i) uoff[i + 1] = uoff[i] + D[i].E;
        int64_t part_entries = 0;
        for (int a = 0; a < nd;) {                      // groups of equal size, as for the inversion
            int b = a + 1;
            while (b < nd && D[b].E == D[a].E && D[b].mat0 == D[a].mat0 + (int64_t)(b - a) * D[a].E * D[a].E) ++b;
            part_entries = std::max(part_entries, (int64_t)(b - a) * ((D[a].E + 255) / 256) * D[a].E);
            a = b;
        }
        DevBuf<float> v, w, u, part;
        v.alloc(2 * emax); w.alloc(2 * uoff[nd]); u.alloc(2 * uoff[nd]); part.alloc(2 * std::max<int64_t>(part_entries, 1));
        HIPCHK(hipMemcpyAsync(v.p, vh.data(), vh.size() * sizeof(float), hipMemcpyHostToDevice, s));
        for (int a = 0; a < nd;) {
            int b = a + 1;
            const int64_t E = D[a].E;
            while (b < nd && D[b].E == E && D[b].mat0 == D[a].mat0 + (int64_t)(b - a) * E * E) ++b;
            if (E > 0 && b - a == 1 && !comps[a].empty()) {
                // block diagonal over the components: each component's diagonal blocks of X_i and T_i
                for (const auto& c : comps[a]) {
                    const int64_t o = c.first + (int64_t)c.first * E;
                    const int nc = c.second - c.first;
                    launch_cgemv_f32(p->Tinv.p + 2 * (D[a].mat0 + o), E, E * E, v.p + 2 * c.first, 0, nc, 1, part.p,
                                     w.p + 2 * (uoff[a] + c.first), E, s);
                    launch_cgemv_f32(T32 + 2 * (D[a].mat0 + o), E, E * E, w.p + 2 * (uoff[a] + c.first), E, nc, 1,
                                     part.p, u.p + 2 * (uoff[a] + c.first), E, s);
                }
            } else if (E > 0) {
                // blocks a..b-1 are back to back (stride E^2), as are their slices of w and u (stride E)
                launch_cgemv_f32(p->Tinv.p + 2 * D[a].mat0, E, E * E, v.p, 0, (int)E, b - a, part.p, w.p + 2 * uoff[a], E, s);
                launch_cgemv_f32(T32 + 2 * D[a].mat0, E, E * E, w.p + 2 * uoff[a], E, (int)E, b - a, part.p,
                                 u.p + 2 * uoff[a], E, s);
            }
            a = b;
        }
        std::vector<float> uh(2 * uoff[nd]);
        HIPCHK(hipMemcpyAsync(uh.data(), u.p, uh.size() * sizeof(float), hipMemcpyDeviceToHost, s));
        sync(p);
        std::vector<int> redo;
        for (int i = 0; i < nd; ++i) {
            double num = 0, den = 0;
            for (int64_t m = 0; m < D[i].E; ++m) {
                const float* ui = uh.data() + 2 * (uoff[i] + m);
                const double dr = ui[0] - vh[2 * m], di = ui[1] - vh[2 * m + 1];
                num += dr * dr + di * di;
                den += (double)vh[2 * m] * vh[2 * m] + (double)vh[2 * m + 1] * vh[2 * m + 1];
            }
            if (D[i].E > 0 && !(std::sqrt(num / den) <= pc_sym_tol())) redo.push_back(i);
        }
        for (int i : redo) {
            const int64_t E = D[i].E;
            HIPCHK(hipMemcpyAsync(p->Tinv.p + 2 * D[i].mat0, T32 + 2 * D[i].mat0, 2 * E * E * sizeof(float),
                                  hipMemcpyDeviceToDevice, s));
            // lane 0's scratch holds W * E for the largest E, so it serves any single block
            if (!comps[i].empty()) {
                // several components: T_i's own component blocks, each inverted on its own
                launch_zero_offdiag_f32(p->Tinv.p + 2 * D[i].mat0, (int)E, cids[i].p, s);
                for (const auto& c : comps[i])
                    block_gj_inverse(p->Tinv.p + 2 * (D[i].mat0 + c.first + (int64_t)c.first * E), c.second - c.first,
                                     E, E * E, 1, info.p, s, kGjPanel, gjtmp[0].p, &la[0]);
            } else {
                block_gj_inverse(p->Tinv.p + 2 * D[i].mat0, (int)E, E, E * E, 1, info.p, s, kGjPanel, gjtmp[0].p,
                                 &la[0]);
            }
            p->pc_full[i] = 1;
        }
    }
    launch_nonfinite_check(p->Tinv.p, 2 * p->mat_entries, info.p + 1, s);
    HIPCHK(hipGetLastError());
    int h[2];
    HIPCHK(hipMemcpyAsync(h, info.p, sizeof(h), hipMemcpyDeviceToHost, s));
    sync(p);
    if (h[0] || h[1]) throw NonFiniteError("block preconditioner: singular pivot or non-finite inverse of T_i");
    build_pc_tiles(p, kind != kPcWhole);
    sync(p);
    p->have_tinv = true;
    p->tinv_prec = p->have32 ? MTF_FP32_MIXED : MTF_FP64;
    p->pc_kind = kind;
    p->gp.haveA = false;
    p->t_precond = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// Streams and events of the preconditioner build (created once per problem).
void ensure_gj_streams(mtf_problem p) {
    for (int l = 0; l < 2; ++l) {
        if (!p->gj_lane[l]) HIPCHK(hipStreamCreateWithFlags(&p->gj_lane[l], hipStreamNonBlocking));
        if (!p->gj_aux[l]) HIPCHK(hipStreamCreateWithFlags(&p->gj_aux[l], hipStreamNonBlocking));
        if (!p->gj_fork[l]) HIPCHK(hipEventCreateWithFlags(&p->gj_fork[l], hipEventDisableTiming));
        if (!p->gj_join[l]) HIPCHK(hipEventCreateWithFlags(&p->gj_join[l], hipEventDisableTiming));
        if (!p->gj_done[l]) HIPCHK(hipEventCreateWithFlags(&p->gj_done[l], hipEventDisableTiming));
    }
    if (!p->gj_start) HIPCHK(hipEventCreateWithFlags(&p->gj_start, hipEventDisableTiming));
}

// The T_i^-1 preconditioner blocks of every problem of a batch, built together (same blocks as
// build_tinv: the inverse of the symmetric part of each T_i, or of each connected component's
// diagonal block of it, checked on a fixed vector and rebuilt from T_i itself where the check
// fails; or as `kind` asks).  A batch of many small problems has hundreds of diagonal blocks of different orders;
// inverted one problem after another they are a long chain of small launches (the 64-wide leaf
// inversions occupy one CU each).  Here every block is copied into a slot of a bucket of equal
// padded order S (n rounded up to 128, the identity in the padding), and each bucket is one
// batched blocked Gauss-Jordan inversion, the buckets spread over two streams.  All problems
// share the stream s.  Returns the wall time of the build.
// Work buffers of batch_build_tinv: the padded buckets and the two lanes' panel buffers.  Kept by
// the caller from one build to the next (they only grow), so that a repeated build allocates and
// frees no device memory.
struct GjScratch {
    DevBuf<float> buf, tmp[2];
};

double batch_build_tinv(const std::vector<mtf_problem>& ps, int kind, hipStream_t s, GjScratch* keep = nullptr) {
    auto t0 = std::chrono::steady_clock::now();
    struct Blk {
        int prob, dom;
        PadBlock pb;
    };
    std::vector<Blk> blocks;
    int64_t emax = 0;
    for (size_t q = 0; q < ps.size(); ++q) {
        mtf_problem p = ps[q];
        const auto& D = p->doms;
        p->Tinv.alloc(2 * (p->mat_entries + 64));
        launch_fill_f(p->Tinv.p, 2 * (p->mat_entries + 64), 0.f, s);
        p->pc_full.assign(D.size(), kind != kPcSym ? 1 : 0);
        p->have_tinv = false;
        for (int i = 0; i < (int)D.size(); ++i) {
            const int64_t E = D[i].E;
            if (E == 0) continue;
            std::vector<std::pair<int, int>> comps;
            if (kind != kPcWhole) comps = domain_components(p, i);
            if (comps.empty()) comps.emplace_back(0, (int)E);
            for (const auto& c : comps) {
                const int64_t o = D[i].mat0 + c.first + (int64_t)c.first * E;
                PadBlock b;
                b.f64 = p->have32 ? 0 : 1;
                b.src = b.f64 ? static_cast<const void*>(p->T64.p + 2 * o) : static_cast<const void*>(p->T32.p + 2 * o);
                b.dst = p->Tinv.p + 2 * o;
                b.ld = E;
                b.n = c.second - c.first;
                blocks.push_back(Blk{(int)q, i, b});
            }
            emax = std::max(emax, E);
        }
    }
    if (blocks.empty()) return 0.0;
    mtf_problem p0 = ps[0];
    ensure_gj_streams(p0);
    GjLookahead la[2];
    for (int l = 0; l < 2; ++l) la[l] = GjLookahead{p0->gj_aux[l], p0->gj_fork[l], p0->gj_join[l]};
    DevBuf<int> info;
    info.alloc(2);
    HIPCHK(hipMemsetAsync(info.p, 0, 2 * sizeof(int), s));
    auto padded = [](int n) { return n <= 64 ? 64 : ((n + 127) / 128) * 128; };
    int smax = 64;
    for (const Blk& b : blocks) smax = std::max(smax, padded(b.pb.n));
    // the fixed check vector v_m = (cos m, sin 2m), long enough for every padded slot
    const int64_t vlen = std::max<int64_t>(emax, smax);
    std::vector<float> vh(2 * vlen);
    for (int64_t m = 0; m < vlen; ++m) { vh[2 * m] = (float)std::cos((double)m); vh[2 * m + 1] = (float)std::sin(2.0 * m); }
    DevBuf<float> v;
    v.alloc(2 * vlen);
    HIPCHK(hipMemcpyAsync(v.p, vh.data(), vh.size() * sizeof(float), hipMemcpyHostToDevice, s));

    // Inverts the listed blocks (symmetrised when sym) into their destinations; with `check`,
    // fills u[blocks] = T (X v) (X the new inverse), blocks back to back in list order.
    std::vector<float> uh;
    auto invert = [&](const std::vector<int>& idx, int sym, bool check) {
        std::map<int, std::vector<int>> bucket;
        for (int k : idx) bucket[padded(blocks[k].pb.n)].push_back(k);
        std::vector<PadBlock> hb;
        std::vector<int64_t> boff, bslot;              // per bucket: first PadBlock, first slot (complex entries)
        int64_t slots = 0, tmp_need[2] = {1, 1}, wlen = 0, part_need = 1;
        int lane = 0;
        std::vector<int> blane;
        for (auto& kv : bucket) {
            const int S = kv.first;
            boff.push_back((int64_t)hb.size());
            bslot.push_back(slots);
            for (int k : kv.second) hb.push_back(blocks[k].pb);
            slots += (int64_t)kv.second.size() * S * S;
            blane.push_back(lane);
            tmp_need[lane] = std::max<int64_t>(tmp_need[lane], (int64_t)kv.second.size() * kGjPanel * S);
            lane ^= 1;
            wlen += (int64_t)kv.second.size() * S;
            part_need = std::max<int64_t>(part_need, (int64_t)kv.second.size() * ((S + 255) / 256) * S);
        }
        DevBuf<PadBlock> dpb;
        dpb.upload(hb, s);
        GjScratch local;
        GjScratch& sc = keep ? *keep : local;
        auto grow = [](DevBuf<float>& d, int64_t count) {
            if (d.n < (size_t)count) d.alloc((size_t)count);
        };
        grow(sc.buf, 2 * slots);
        for (int l = 0; l < 2; ++l) grow(sc.tmp[l], 2 * tmp_need[l]);
        DevBuf<float>& buf = sc.buf;
        DevBuf<float>* tmp = sc.tmp;
        HIPCHK(hipEventRecord(p0->gj_start, s));
        for (int l = 0; l < 2; ++l) HIPCHK(hipStreamWaitEvent(p0->gj_lane[l], p0->gj_start, 0));
        size_t bi = 0;
        for (auto& kv : bucket) {
            const int S = kv.first, cnt = (int)kv.second.size(), l = blane[bi];
            hipStream_t ls = p0->gj_lane[l];
            float* bb = buf.p + 2 * bslot[bi];
            launch_pad_gather(dpb.p + boff[bi], cnt, S, sym, bb, ls);
            block_gj_inverse(bb, S, S, (int64_t)S * S, cnt, info.p, ls, kGjPanel, tmp[l].p, &la[l]);
            launch_pad_scatter(dpb.p + boff[bi], cnt, S, bb, info.p + 1, ls);   // checks every copied entry
            ++bi;
        }
        for (int l = 0; l < 2; ++l) {
            HIPCHK(hipEventRecord(p0->gj_done[l], p0->gj_lane[l]));
            HIPCHK(hipStreamWaitEvent(s, p0->gj_done[l], 0));
        }
        if (check) {
            // w = X v per slot (batched per bucket), then u = T_blk w[0:n] per block
            DevBuf<float> w, u, part;
            int64_t ulen = 0;
            for (int k : idx) ulen += blocks[k].pb.n;
            w.alloc(2 * wlen);
            u.alloc(2 * std::max<int64_t>(ulen, 1));
            int64_t pn = part_need;
            for (int k : idx) pn = std::max<int64_t>(pn, (int64_t)((blocks[k].pb.n + 255) / 256) * blocks[k].pb.n);
            part.alloc(2 * pn);
            bi = 0;
            int64_t wo = 0, uo = 0;
            for (auto& kv : bucket) {
                const int S = kv.first, cnt = (int)kv.second.size();
                launch_cgemv_f32(buf.p + 2 * bslot[bi], S, (int64_t)S * S, v.p, 0, S, cnt, part.p, w.p + 2 * wo, S, s);
                for (int j = 0; j < cnt; ++j) {
                    const PadBlock& b = blocks[kv.second[j]].pb;
                    float* wj = w.p + 2 * (wo + (int64_t)j * S);
                    if (b.f64)
                        launch_cgemv_f64src(static_cast<const double*>(b.src), b.ld, wj, b.n, part.p, u.p + 2 * uo, s);
                    else
                        launch_cgemv_f32(static_cast<const float*>(b.src), b.ld, 0, wj, 0, b.n, 1, part.p, u.p + 2 * uo, 0, s);
                    uo += b.n;
                }
                wo += (int64_t)cnt * S;
                ++bi;
            }
            uh.assign(2 * ulen, 0.f);
            HIPCHK(hipMemcpyAsync(uh.data(), u.p, uh.size() * sizeof(float), hipMemcpyDeviceToHost, s));
            // the check's order of blocks: bucket by bucket
            std::vector<int> order;
            for (auto& kv2 : bucket) order.insert(order.end(), kv2.second.begin(), kv2.second.end());
            HIPCHK(hipStreamSynchronize(s));
            return order;
        }
        HIPCHK(hipStreamSynchronize(s));
        return std::vector<int>();
    };

    std::vector<int> all(blocks.size());
    for (size_t k = 0; k < blocks.size(); ++k) all[k] = (int)k;
    const std::vector<int> order = invert(all, kind == kPcSym ? 1 : 0, kind == kPcSym);
    if (kind == kPcSym) {
        // ||T_i (X_i v) - v|| / ||v|| per subdomain (over its components); rebuild the failures
        std::map<std::pair<int, int>, std::pair<double, double>> err;
        int64_t uo = 0;
        for (int k : order) {
            const Blk& b = blocks[k];
            auto& e = err[{b.prob, b.dom}];
            for (int m = 0; m < b.pb.n; ++m) {
                const float* ui = uh.data() + 2 * (uo + m);
                const double dr = ui[0] - vh[2 * m], di = ui[1] - vh[2 * m + 1];
                e.first += dr * dr + di * di;
                e.second += (double)vh[2 * m] * vh[2 * m] + (double)vh[2 * m + 1] * vh[2 * m + 1];
            }
            uo += b.pb.n;
        }
        std::vector<int> redo;
        for (size_t k = 0; k < blocks.size(); ++k) {
            const auto& e = err[{blocks[k].prob, blocks[k].dom}];
            if (!(std::sqrt(e.first / e.second) <= pc_sym_tol())) {
                redo.push_back((int)k);
                ps[blocks[k].prob]->pc_full[blocks[k].dom] = 1;
            }
        }
        if (!redo.empty()) invert(redo, 0, false);
    }
    HIPCHK(hipGetLastError());
    int h[2];
    HIPCHK(hipMemcpyAsync(h, info.p, sizeof(h), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (h[0] || h[1]) throw NonFiniteError("block preconditioner: singular pivot or non-finite inverse of T_i");
    for (mtf_problem p : ps) {
        build_pc_tiles(p, kind != kPcWhole);
        p->have_tinv = true;
        p->tinv_prec = p->have32 ? MTF_FP32_MIXED : MTF_FP64;
        p->pc_kind = kind;
        p->gp.haveA = false;
    }
    HIPCHK(hipStreamSynchronize(s));
    const double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (mtf_problem p : ps) p->t_precond = t;
    return t;
}

void gmres_alloc(mtf_problem p, int maxit, int nb, bool flex) {
    GmresWork& w = p->gw;
    const int64_t n = p->stf ? 2 * (int64_t)p->sk.dom[0].E : p->sk.N;
    // a workspace allocated for at least n unknowns, maxit steps and nb columns serves as it is (the
    // buffers are laid out from w.n, w.maxit and w.nb)
    if (w.cap_n >= n && w.maxit >= maxit && w.nb >= nb) {
        w.n = n;
        if (flex && w.zslots < w.maxit) {
            w.Zt.alloc(2 * w.cap_n * (int64_t)w.nb * w.maxit);
            w.Rf.alloc(2 * (int64_t)(w.maxit + 1) * w.maxit * w.nb);
            w.zslots = w.maxit;
        }
        return;
    }
    w.n = n;
    w.cap_n = n;
    w.maxit = maxit;
    w.nb = nb;
    const int64_t ldh = maxit + 1;
    const int64_t nct = (maxit + 63) / 64;
    w.V.alloc(2 * n * (int64_t)nb * (maxit + 1));
    w.zslots = 0;
    w.Zt.reset();
    w.Rf.reset();
    if (flex) {
        w.Zt.alloc(2 * n * (int64_t)nb * maxit);
        w.Rf.alloc(2 * ldh * (int64_t)maxit * nb);
        w.zslots = maxit;
    }
    w.tmp.alloc(2 * n * nb);
    w.tmp2.alloc(2 * n * nb);
    w.tmp3.alloc(2 * n);
    w.r.alloc(2 * n * nb);
    w.hpart.alloc(4 * (int64_t)nb * (maxit + 1) * dot_plan(nb).kmax);
    w.S.alloc(2 * (int64_t)nb * (maxit + 1));
    w.Z.alloc(2 * (int64_t)nb * (maxit + 1));
    w.hg.alloc(2 * (int64_t)nb * nct * (maxit + 1));
    w.scal.alloc(4 * (int64_t)nb);
    w.H.alloc(2 * ldh * (int64_t)maxit * nb);
    w.npart.alloc((int64_t)nb * kNblk);
    w.upart.alloc(4 * n * (int64_t)nb * kUpdGroups);
    w.ufix.alloc(2 * n * nb);
    w.tfix.alloc(2 * n * nb);
    w.zfix.alloc(2 * n * nb);
    w.Hst.alloc(2 * ldh * (int64_t)kSync * nb);
    w.jdev.alloc(2);
    w.y.alloc(2 * (int64_t)nb * (maxit + 1));
    w.cnt.alloc(nb + 1);
    if (w.host) (void)hipHostFree(w.host);
    if (w.hosty) (void)hipHostFree(w.hosty);
    if (w.hostcnt) (void)hipHostFree(w.hostcnt);
    w.host = nullptr;
    w.hosty = nullptr;
    w.hostcnt = nullptr;
    HIPCHK(hipHostMalloc((void**)&w.host, ((size_t)4 * ldh * kSync * nb + (size_t)kNblk * nb) * sizeof(double),
                         hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&w.hosty, (size_t)2 * nb * ldh * sizeof(double), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&w.hostcnt, (size_t)(nb + 1) * sizeof(int), hipHostMallocDefault));
}

// column norms of nb vectors (stride ld)
std::vector<double> norms_dev(mtf_problem p, const double* v, int64_t ld, int nb) {
    GmresWork& w = p->gw;
    launch_norm2(v, ld, w.n, w.npart.p, kNblk, nb, p->stream);
    HIPCHK(hipMemcpyAsync(w.host, w.npart.p, (size_t)kNblk * nb * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    sync(p);
    std::vector<double> out(nb);
    for (int b = 0; b < nb; ++b) {
        double s = 0;
        for (int k = 0; k < kNblk; ++k) s += w.host[(size_t)b * kNblk + k];
        out[b] = std::sqrt(s);
    }
    return out;
}

// Inner operator A = M_prec P on the nb columns of slab src (ld n) into slab dst (ld n).
// z = P x for nb columns (ld n); pc: MTF_PREC_BLOCK_TINV (Jacobi) or MTF_PREC_BLOCK_TINV_GS.
void apply_pc(mtf_problem p, int pc, int prec, int nb, const double* x, double* z) {
    GmresWork& w = p->gw;
    const int64_t n = w.n;
    if (pc == MTF_PREC_BLOCK_TINV && prec == MTF_BF16_SPLIT) { apply_gemm(p, 1, nb, x, n, z); return; }
    for (int b = 0; b < nb; ++b) {
        if (pc == MTF_PREC_BLOCK_TINV_GS) precond1_gs(p, x + 2 * n * b, z + 2 * n * b, w.tmp3.p);
        else precond1(p, x + 2 * n * b, z + 2 * n * b);
    }
}

// ||(M_32 - M_64) v|| / ||M_64 v|| for one vector v (device, length N): the relative accuracy of
// the complex64 operator, which sets where a mixed solve may switch to it.
double operator_gap(mtf_problem p, const double* v) {
    GmresWork& w = p->gw;
    matvec1(p, v, w.tmp.p, MTF_FP64);
    matvec1(p, v, w.tmp2.p, MTF_FP32_MIXED);
    const double n64 = norms_dev(p, w.tmp.p, w.n, 1)[0];
    launch_axpby(w.tmp2.p, w.tmp.p, w.n, 1.0, 0.0, -1.0, p->stream);   // tmp2 = tmp - tmp2
    const double nd = norms_dev(p, w.tmp2.p, w.n, 1)[0];
    return n64 > 0.0 ? nd / n64 : 0.0;
}

// dst = M P src; the preconditioned slab P src goes to zout (or to scratch when zout is null)
void apply_inner(mtf_problem p, const double* src, double* dst, int nb, int prec, int pc, double* zout) {
    GmresWork& w = p->gw;
    const int64_t n = w.n;
    const double* in = src;
    if (pc != MTF_PREC_NONE) {
        double* z = zout ? zout : w.tmp.p;
        apply_pc(p, pc, prec, nb, src, z);
        in = z;
    }
    if (p->stf) {
        // single-trace operator R M C (M = 1), through the MTF product
        const int64_t E = p->sk.dom[0].E;
        for (int b = 0; b < nb; ++b) {
            launch_stf_expand(in + 2 * n * b, p->stf_sign.p, E, p->stf_x.p, p->stream);
            matvec1(p, p->stf_x.p, p->stf_y.p, prec);
            launch_stf_reduce(p->stf_y.p, p->stf_sign.p, E, dst + 2 * n * b, p->stream);
        }
        return;
    }
    if (prec == MTF_BF16_SPLIT) apply_gemm(p, 0, nb, in, n, dst);
    else
        for (int b = 0; b < nb; ++b) matvec1(p, in + 2 * n * b, dst + 2 * n * b, prec);
}

// Enters the single-trace mode for M = 1 (sign map and full-length vectors prepared); throws for
// other problems.
void stf_prepare(mtf_problem p) {
    if (p->sk.M != 1) throw UnsupportedError("the single-trace formulation needs M = 1");
    const Domain& d0 = p->sk.dom[0];
    const Domain& d1 = p->sk.dom[1];
    if (d0.E != d1.E || d0.edge_vtx != d1.edge_vtx)
        throw UnsupportedError("the single-trace formulation needs Gamma_0 and Gamma_1 on the same edges");
    if (!p->stf_sign.p) {
        std::vector<int8_t> sg(d0.E);
        for (int m = 0; m < d0.E; ++m)
            sg[m] = d0.tri[d0.plus[2 * m]] == d1.tri[d1.plus[2 * m]] ? int8_t(1) : int8_t(-1);
        p->stf_sign.upload(sg, p->stream);
    }
    p->stf_x.alloc(2 * p->sk.N);
    p->stf_y.alloc(2 * p->sk.N);
}

// y = M_STF x for nb vectors of length 2 E_0 (ld)
void stf_matvec(mtf_problem p, const double* x, double* y, int64_t ld, int nb) {
    const int64_t E = p->sk.dom[0].E;
    for (int b = 0; b < nb; ++b) {
        launch_stf_expand(x + 2 * ld * b, p->stf_sign.p, E, p->stf_x.p, p->stream);
        matvec1(p, p->stf_x.p, p->stf_y.p, MTF_FP64);
        launch_stf_reduce(p->stf_y.p, p->stf_sign.p, E, y + 2 * ld * b, p->stream);
    }
}

// One GMRES cycle for nb right-hand sides in lockstep: residual slab R (ld n), corrections added to
// the nb columns of X (ld ldx).  Arnoldi with delayed classical Gram-Schmidt reorthogonalisation:
// step j applies the operator to the once-projected candidate u_j, then one pass over the basis
// gives the coefficients and a second pass forms q_j and u_{j+1}; Hessenberg column j-1 becomes
// final at step j.  The Hessenberg matrix stays on the device; the host receives the final columns
// every kSync steps (p->gmres_sync, at most kSync) and applies the Givens rotations.  Each right-hand side stops at its own step.
// With a preconditioner the iteration is flexible: the preconditioned candidates zt_j = P u_j are
// kept, and since U = Q R (R upper triangular from the reorthogonalisation coefficients) the
// correction is Zt R^-1 y, so M times the correction matches the Arnoldi relation exactly even
// though P is applied in FP32.
// Every kernel of a step reads the step index from the device and works on step-invariant
// buffers, so the steps between two host reads (plus the staging of the final columns and
// their copy to pinned host memory) are captured once as a HIP graph and replayed (`graph`), or
// launched one by one; both run the same kernels.
// Returns the number of Arnoldi steps taken; it[b], est[b] (recurrence residual / ||r_b||) per column.
int gmres_cycle(mtf_problem p, const double* R, double* X, int64_t ldx, int nb, int prec, int pc,
                const std::vector<double>& tol, int maxit, std::vector<int>& itv, std::vector<double>& est,
                std::vector<int>& reorth, bool graph, double relax, bool c64) {
    GmresWork& w = p->gw;
    hipStream_t s = p->stream;
    // steps between host reads: even, since the replayed batch of steps alternates the two step-index
    // slots and must start on the same parity every time
    const int nsync = std::max(2, std::min(kSync, p->gmres_sync) & ~1);
    const int64_t n = w.n;
    const int64_t ldh = w.maxit + 1;
    const int64_t hstride = ldh * (int64_t)w.maxit;
    const int64_t ldv = n * nb;
    const int nvmax = w.maxit;
    const int nct = (w.maxit + 63) / 64;
    const bool flex = pc != MTF_PREC_NONE;
    if (flex && w.zslots < maxit) throw StateError("flexible GMRES basis not allocated");
    double* V = w.V.p;
    auto jslot = [&](int j) { return w.jdev.p + (j & 1); };
    auto Hc = [&](int j) { return w.H.p + 2 * ldh * (int64_t)j; };
    std::vector<double> beta = norms_dev(p, R, n, nb);
    // u_0 = r, step index 0
    if (c64 && !flex) throw ArgError("a complex64 basis needs the flexible (preconditioned) iteration");
    if (!c64) HIPCHK(hipMemcpyAsync(V, R, (size_t)2 * n * nb * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(w.ufix.p, R, (size_t)2 * n * nb * sizeof(double), hipMemcpyDeviceToDevice, s));
    launch_set_int(jslot(0), 0, s);
    // Relaxed products (complex64 operator only): the steps use the FP64 operator until every
    // live recurrence residual is at most relax times its initial value, the complex64 one after.
    int cur_prec = prec == MTF_FP32_MIXED && relax < 1.0 ? MTF_FP64 : prec;
    // one Arnoldi step with index jj (the kernels read jj from the device, so only its parity matters
    // to the launch sequence)
    auto step = [&](int jj) {
        const int* jr = jslot(jj);
        apply_inner(p, w.ufix.p, w.tfix.p, nb, cur_prec, pc, flex ? w.zfix.p : nullptr);
        launch_dot2(V, ldv, jr, nvmax, w.tfix.p, w.ufix.p, n, w.hpart.p, dot_plan(nb), c64, nb, s);
        launch_reduce2(w.hpart.p, jr, nvmax, dot_plan(nb), w.S.p, w.Z.p, nb, s);
        launch_update2(V, ldv, jr, jslot(jj + 1), nvmax, w.S.p, w.Z.p, w.tfix.p, w.ufix.p, n, w.upart.p, kUpdGroups,
                       flex ? w.zfix.p : nullptr, flex ? w.Zt.p : nullptr, w.H.p, ldh, hstride, w.hg.p, nct,
                       flex ? w.Rf.p : nullptr, hstride, c64, nb, s);
    };
    // nsync steps j0 .. j0+nsync-1 (j0 odd), then the final columns j0-1 .. j0+nsync-2 staged in Hst
    // (the caller copies them to one of the two host areas)
    const size_t stage_doubles = (size_t)2 * ldh * nsync * nb;
    const size_t stage_bytes = stage_doubles * sizeof(double);
    auto batch = [&](int j0) {
        for (int q = 0; q < nsync; ++q) step(j0 + q);
        launch_stage_cols(w.H.p, ldh, hstride, jslot(j0 + nsync), nsync + 1, nsync, w.Hst.p, nb, s);
    };
    for (hipEvent_t& e : w.ev)
        if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    hipGraphExec_t exec = nullptr;
    // On every exit (an exception included) the queued batches finish first: no replay of the
    // graph, and no copy into the pinned staging areas, may still be pending.
    struct ExecGuard {
        hipGraphExec_t& e;
        hipStream_t s;
        ~ExecGuard() {
            (void)hipStreamSynchronize(s);
            if (e) (void)hipGraphExecDestroy(e);
        }
    } exec_guard{exec, s};

    // host copies of the final Hessenberg columns after the rotations (column jj has jj+1 entries)
    std::vector<std::vector<std::vector<cd>>> H(nb);
    std::vector<std::vector<double>> cs(nb);
    std::vector<std::vector<cd>> sn(nb), gv(nb);
    std::vector<char> stop(nb, 0);
    std::vector<double> resid(beta);
    itv.assign(nb, 0);
    int live = 0;
    for (int b = 0; b < nb; ++b) {
        gv[b].push_back(beta[b]);
        if (beta[b] == 0.0) stop[b] = 1; else ++live;
    }
    std::vector<cd> col;
    // Givens rotations on final columns c0 .. c0+nc-1 held in hbuf ([b][q][ldh] complex)
    auto process = [&](int c0, int nc, const double* hbuf) {
        for (int b = 0; b < nb; ++b) {
            if (stop[b]) continue;
            const double* hb = hbuf + (size_t)2 * ldh * nc * b;
            for (int q = 0; q < nc && !stop[b]; ++q) {
                const int jj = c0 + q;
                col.assign(jj + 2, cd(0));
                for (int i = 0; i <= jj + 1; ++i) col[i] = cd(hb[2 * (ldh * q + i)], hb[2 * (ldh * q + i) + 1]);
                const double hn = col[jj + 1].real();
                for (int i = 0; i < jj; ++i) {
                    const cd tq = cs[b][i] * col[i] + sn[b][i] * col[i + 1];
                    col[i + 1] = -std::conj(sn[b][i]) * col[i] + cs[b][i] * col[i + 1];
                    col[i] = tq;
                }
                const cd a = col[jj];
                const double den = std::sqrt(std::norm(a) + hn * hn);
                double c;
                cd sj;
                if (std::abs(a) == 0.0) { c = 0.0; sj = 1.0; }
                else { c = std::abs(a) / den; sj = (a / std::abs(a)) * hn / den; }
                cs[b].push_back(c);
                sn[b].push_back(sj);
                col[jj] = c * a + sj * hn;
                col.resize(jj + 1);
                H[b].push_back(col);
                gv[b].push_back(-std::conj(sj) * gv[b][jj]);
                gv[b][jj] = c * gv[b][jj];
                itv[b] = jj + 1;
                resid[b] = std::abs(gv[b][jj + 1]);
                if (!std::isfinite(resid[b])) throw NonFiniteError("GMRES produced a non-finite residual");
                if (resid[b] <= tol[b] * beta[b] || hn == 0.0) { stop[b] = 1; --live; }
            }
        }
    };

    int j = 0, done_cols = 0;
    if (live > 0) {
        step(0);                           // step 0 (also makes every lazily allocated buffer exist)
        j = 1;
    }
    int batches = 0;
    // Batches launched and not yet processed (at most two): while the host applies the rotations to
    // one batch's columns, the next batch already runs.  Near convergence only one is launched at a
    // time, so that at most the steps of one batch are spent past the converging step.
    struct Pending {
        int c0, area;
    };
    Pending pend[2];
    int npend = 0, area = 0;
    auto launch_batch = [&](int j0) {
        // short cycles never pay for the capture: the first kEagerBatches batches run eagerly
        if (graph && batches++ >= kEagerBatches) {
            if (!exec) {
                // capture on the private stream (the caller's may be the null stream, which cannot be
                // captured); every launch in batch() goes to p->stream and s, redirected meanwhile
                if (!p->capture) HIPCHK(hipStreamCreate(&p->capture));
                const hipStream_t caller = p->stream;
                struct Restore {
                    mtf_problem p;
                    hipStream_t& s;
                    hipStream_t caller;
                    ~Restore() { p->stream = caller; s = caller; }
                } restore{p, s, caller};
                p->stream = s = p->capture;
                hipGraph_t g = nullptr;
                HIPCHK(hipStreamBeginCapture(p->capture, hipStreamCaptureModeThreadLocal));
                try {
                    batch(j0);
                } catch (...) {
                    (void)hipStreamEndCapture(p->capture, &g);
                    if (g) (void)hipGraphDestroy(g);
                    throw;
                }
                HIPCHK(hipStreamEndCapture(p->capture, &g));
                const hipError_t e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                HIPCHK(e);
            }
            HIPCHK(hipGraphLaunch(exec, s));
        } else {
            batch(j0);
        }
        HIPCHK(hipMemcpyAsync(w.host + area * stage_doubles, w.Hst.p, stage_bytes, hipMemcpyDeviceToHost, s));
        HIPCHK(hipEventRecord(w.ev[area], s));
        pend[npend++] = Pending{j0 - 1, area};
        area ^= 1;
    };
    auto finish_oldest = [&]() {
        const Pending q = pend[0];
        pend[0] = pend[1];
        --npend;
        HIPCHK(hipEventSynchronize(w.ev[q.area]));
        process(q.c0, nsync, w.host + q.area * stage_doubles);
        done_cols = q.c0 + nsync;
    };
    auto far = [&]() {
        for (int b = 0; b < nb; ++b)
            if (!stop[b] && !(resid[b] > kLookaheadFactor * tol[b] * beta[b])) return false;
        return true;
    };
    while (live > 0) {
        const int want = far() ? 2 : 1;
        while (npend < want && j + nsync <= maxit) {
            launch_batch(j);
            j += nsync;
        }
        if (npend > 0) {
            finish_oldest();
            if (cur_prec != prec) {
                bool below = true;
                for (int b = 0; b < nb; ++b)
                    if (!stop[b] && resid[b] > relax * beta[b]) below = false;
                if (below) {
                    while (npend > 0 && live > 0) finish_oldest();   // the queued batch used the FP64 product
                    npend = 0;
                    cur_prec = prec;                 // the captured batch holds the FP64 product
                    if (exec) {
                        sync(p);
                        HIPCHK(hipGraphExecDestroy(exec));
                        exec = nullptr;
                    }
                }
            }
            continue;
        }
        // tail: the remaining steps one by one, then the step that only finalises column maxit-1
        for (; j < maxit; ++j) step(j);
        launch_dot2(V, ldv, jslot(maxit), nvmax, nullptr, w.ufix.p, n, w.hpart.p, dot_plan(nb), c64, nb, s);
        launch_reduce2(w.hpart.p, jslot(maxit), nvmax, dot_plan(nb), w.S.p, w.Z.p, nb, s);
        launch_dcgs_col(w.H.p, ldh, hstride, w.S.p, w.Z.p, w.hg.p, nct, jslot(maxit), nvmax, w.scal.p, 1, nullptr,
                        hstride, nb, s);
        const int nc = maxit - done_cols;
        if (nc > 0) {
            HIPCHK(hipMemcpy2DAsync(w.host, (size_t)2 * ldh * nc * sizeof(double), Hc(done_cols),
                                    (size_t)2 * hstride * sizeof(double), (size_t)2 * ldh * nc * sizeof(double), nb,
                                    hipMemcpyDeviceToHost, s));
            sync(p);
            process(done_cols, nc, w.host);
        }
        done_cols = maxit;
        break;
    }
    const int steps = j;
    // back substitution per right-hand side; flexible: coefficients R^-1 y on the zt basis (device)
    double* yh = w.hosty;
    std::fill(yh, yh + (size_t)2 * nb * (nvmax + 1), 0.0);
    for (int b = 0; b < nb; ++b) {
        const int it = itv[b];
        std::vector<cd> yv(it);
        for (int i = it - 1; i >= 0; --i) {
            cd acc = gv[b][i];
            for (int k = i + 1; k < it; ++k) acc -= H[b][k][i] * yv[k];
            yv[i] = acc / H[b][i][i];
        }
        for (int i = 0; i < it; ++i) {
            yh[(size_t)2 * b * (nvmax + 1) + 2 * i] = yv[i].real();
            yh[(size_t)2 * b * (nvmax + 1) + 2 * i + 1] = yv[i].imag();
        }
    }
    for (int b = 0; b < nb; ++b) w.hostcnt[b] = itv[b];
    w.hostcnt[nb] = 0;
    HIPCHK(hipMemcpyAsync(w.y.p, yh, (size_t)2 * nb * (nvmax + 1) * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(w.cnt.p, w.hostcnt, (nb + 1) * sizeof(int), hipMemcpyHostToDevice, s));
    if (flex) launch_trsv_upper(w.Rf.p, ldh, hstride, w.cnt.p, w.y.p, nvmax + 1, w.cnt.p + nb, nb, s);
    launch_combine(X, ldx, flex ? w.Zt.p : V, ldv, w.cnt.p, nvmax, w.y.p, n, nb, s);   // X_b += basis_b coef_b
    HIPCHK(hipMemcpyAsync(w.hostcnt + nb, w.cnt.p + nb, sizeof(int), hipMemcpyDeviceToHost, s));
    sync(p);
    if (w.hostcnt[nb]) throw NonFiniteError("GMRES: zero pivot in the reorthogonalisation factor");
    est.assign(nb, 0.0);
    for (int b = 0; b < nb; ++b) {
        reorth[b] += itv[b];          // every kept step was reorthogonalised
        est[b] = beta[b] > 0 ? resid[b] / beta[b] : 0.0;
    }
    return steps;
}

// ---------------------------------------------------------------------------------------------
// Block flexible GMRES: q right-hand sides share one Krylov space (block Arnoldi with the FP64
// block Gram-Schmidt contractions of block.hip, a rank-revealing orthonormalisation of each new
// block, and the block least-squares problem reduced by Householder reflections on the host).

// Orthonormal basis of the span of n vectors W from their Gram matrix G = W^H W (column-major):
// Q = W T (n x k) and W ~= Q S (k x n).  The columns are scaled to unit norm, then the scaled Gram
// matrix is factored by Cholesky with diagonal pivoting (the largest remaining pivot first, as in
// LAPACK's pstrf), which stops once that pivot is at most `keep`: the factorisation reveals the
// rank, and the columns left over are expressed in the kept ones (their rows of S).  A column
// whose squared norm is at most 1e-26 ref2[c] counts as zero.  lmin: the smallest kept pivot.
struct Svqb {
    int k = 0;
    std::vector<cd> T, S;   // T: n x k, S: k x n, column-major
    double lmin = 1.0;
};
Svqb svqb(int n, const std::vector<cd>& G, const std::vector<double>& ref2, double keep) {
    std::vector<double> D(n, 0.0);
    for (int c = 0; c < n; ++c) {
        const double g = G[(size_t)c * n + c].real();
        if (g > 0.0 && g > 1e-26 * ref2[c]) D[c] = 1.0 / std::sqrt(g);
    }
    // A: scaled Gram matrix (row-major, Hermitian), updated in place to its Schur complements
    std::vector<cd> A((size_t)n * n);
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) A[(size_t)r * n + c] = D[r] * G[(size_t)c * n + r] * D[c];
    std::vector<cd> R((size_t)n * n, cd(0.0, 0.0));      // row-major, rows 0..k-1
    std::vector<int> perm(n);
    for (int i = 0; i < n; ++i) perm[i] = i;
    auto at = [&](int r, int c) -> cd& { return A[(size_t)r * n + c]; };
    int k = 0;
    double lmin = 1.0;
    for (; k < n; ++k) {
        int j = k;
        for (int i = k + 1; i < n; ++i)
            if (at(i, i).real() > at(j, j).real()) j = i;
        const double piv = at(j, j).real();
        if (!(piv > keep)) break;
        if (j != k) {                                     // symmetric swap of k and j
            for (int c = 0; c < n; ++c) std::swap(at(k, c), at(j, c));
            for (int r = 0; r < n; ++r) std::swap(at(r, k), at(r, j));
            for (int m = 0; m < k; ++m) std::swap(R[(size_t)m * n + k], R[(size_t)m * n + j]);
            std::swap(perm[k], perm[j]);
        }
        const double rkk = std::sqrt(piv);
        lmin = std::min(lmin, piv);
        R[(size_t)k * n + k] = rkk;
        for (int c = k + 1; c < n; ++c) R[(size_t)k * n + c] = at(k, c) / rkk;
        for (int r = k + 1; r < n; ++r) {
            const cd a = std::conj(R[(size_t)k * n + r]);
            const double ar = a.real(), ai = a.imag();
            for (int c = k + 1; c < n; ++c) {               // A(r, c) -= conj(R(k, r)) R(k, c)
                const cd b = R[(size_t)k * n + c];
                at(r, c) -= cd(ar * b.real() - ai * b.imag(), ar * b.imag() + ai * b.real());
            }
        }
    }
    Svqb o;
    o.k = k;
    o.lmin = k > 0 ? lmin : 0.0;
    // inverse of the leading k x k triangle R11 (upper triangular, column by column)
    std::vector<cd> Ri((size_t)k * k, cd(0.0, 0.0));   // row-major
    for (int c = 0; c < k; ++c) {
        Ri[(size_t)c * k + c] = 1.0 / R[(size_t)c * n + c];
        for (int r = c - 1; r >= 0; --r) {
            cd t = 0.0;
            for (int m = r + 1; m <= c; ++m) t += R[(size_t)r * n + m] * Ri[(size_t)m * k + c];
            Ri[(size_t)r * k + c] = -t / R[(size_t)r * n + r];
        }
    }
    // T = D P(:, 0:k) R11^-1;  S = [R11 R12] P^T D^-1
    o.T.assign((size_t)n * k, cd(0.0, 0.0));
    o.S.assign((size_t)k * n, cd(0.0, 0.0));
    for (int kk = 0; kk < k; ++kk)
        for (int m = 0; m <= kk; ++m) o.T[(size_t)kk * n + perm[m]] = D[perm[m]] * Ri[(size_t)m * k + kk];
    for (int m = 0; m < n; ++m) {
        const int c = perm[m];
        if (!(D[c] > 0.0)) continue;
        for (int r = 0; r < k && r <= m; ++r) o.S[(size_t)c * k + r] = R[(size_t)r * n + m] / D[c];
    }
    return o;
}

// Runs f(0..count-1) on up to 16 host threads (inline when the work is small).
template <typename F>
void host_parallel(int count, bool big, F&& f) {
    const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
    const int nt = big ? std::min<int>({count, 16, hw}) : 1;
    if (nt <= 1) {
        for (int i = 0; i < count; ++i) f(i);
        return;
    }
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&, t] {
            for (int i = t; i < count; i += nt) f(i);
        });
    for (std::thread& x : th) x.join();
}

// Householder reduction of the block Hessenberg matrix, column by column as Arnoldi delivers it,
// applied to the block right-hand side E_1 S_0 as well (one column per right-hand side): after a
// block step the rows below the triangular part hold each right-hand side's residual.
struct BlockLsq {
    int w2 = 0;                   // reflector capacity (twice the largest block)
    int q = 0;                    // right-hand sides
    int64_t gld = 0;              // rows of G
    std::vector<double> refl;     // reflector m: w2 complex at refl + 2 m w2 (rows m ..)
    std::vector<int> len;
    std::vector<double> tau;
    std::vector<double> G;        // gld x q complex, column-major
    void init(int cap_cols, int64_t rows, int pmax, int nq) {
        w2 = 2 * pmax;
        q = nq;
        gld = rows;
        refl.resize((size_t)2 * cap_cols * w2);
        len.resize(cap_cols);
        tau.resize(cap_cols);
        G.assign((size_t)2 * rows * nq, 0.0);     // reflectors are written before they are read
    }
    // y (complex, row 0 at y) <- H_m y
    void apply(int m, double* y) const {
        const double t = tau[m];
        if (t == 0.0) return;
        const double* v = refl.data() + (size_t)2 * m * w2;
        double* ym = y + 2 * (int64_t)m;
        const int L = len[m];
        double sr = 0.0, si = 0.0;
        for (int k = 0; k < L; ++k) {           // s = v^H y
            sr += v[2 * k] * ym[2 * k] + v[2 * k + 1] * ym[2 * k + 1];
            si += v[2 * k] * ym[2 * k + 1] - v[2 * k + 1] * ym[2 * k];
        }
        sr *= t;
        si *= t;
        for (int k = 0; k < L; ++k) {           // y -= v (tau s)
            ym[2 * k] -= v[2 * k] * sr - v[2 * k + 1] * si;
            ym[2 * k + 1] -= v[2 * k] * si + v[2 * k + 1] * sr;
        }
    }
    // reflector m from y[m .. m + L - 1], which becomes (alpha, 0, ..., 0)
    void make(int m, int L, double* y) {
        double* x = y + 2 * (int64_t)m;
        double nx2 = 0.0;
        for (int k = 0; k < L; ++k) nx2 += x[2 * k] * x[2 * k] + x[2 * k + 1] * x[2 * k + 1];
        double* v = refl.data() + (size_t)2 * m * w2;
        len[m] = L;
        if (!(nx2 > 0.0)) {
            tau[m] = 0.0;
            return;
        }
        const double nx = std::sqrt(nx2);
        const double ax0 = std::hypot(x[0], x[1]);
        const double pr = ax0 > 0.0 ? x[0] / ax0 : 1.0, pi = ax0 > 0.0 ? x[1] / ax0 : 0.0;
        const double ar = -pr * nx, ai = -pi * nx;                 // alpha = -e^{i arg x0} ||x||
        for (int k = 0; k < 2 * L; ++k) v[k] = x[k];
        v[0] -= ar;
        v[1] -= ai;
        tau[m] = 1.0 / (nx2 + nx * ax0);                           // 2 / ||v||^2
        x[0] = ar;
        x[1] = ai;
        for (int k = 1; k < L; ++k) x[2 * k] = x[2 * k + 1] = 0.0;
    }
};

struct BlockWork {
    DevBuf<double> V, Z, Wa, Wb, Wt, hd, pdot, pupd, R, Y, T, tmp, npart;
    DevBuf<int> cnt, info;
    double* hh[2] = {nullptr, nullptr};   // pinned: projections and Gram matrix of a block step (two steps in flight)
    double* hg = nullptr;                 // pinned: Gram matrix of an orthonormalisation pass
    double* ht = nullptr;                 // pinned: combination matrix T
    double* hc = nullptr;                 // pinned: new block column of the Hessenberg matrix (reduced in place)
    ~BlockWork() {
        for (double* q : {hh[0], hh[1], hg, ht, hc})
            if (q) (void)hipHostFree(q);
    }
};

double* pinned(size_t count) {
    double* q = nullptr;
    HIPCHK(hipHostMalloc((void**)&q, count * sizeof(double), hipHostMallocDefault));
    return q;
}

// Block flexible GMRES over groups of pb right-hand sides (FP64 operator and Arnoldi).  The host's
// reduction of a block column of the Hessenberg matrix overlaps the next block step on the GPU,
// which is launched as soon as the new basis block is formed (and discarded when the reduction
// shows convergence).
int block_solve(mtf_problem p, int32_t nrhs, const double* Bp, double* Xp, int64_t ld, const mtf_solve_opts& opts,
                int pb, int pc, mtf_solve_stats* stats, double t_pc) {
    const int64_t n = p->sk.N;
    hipStream_t s = p->stream;
    const bool use_pc = pc != MTF_PREC_NONE;
    const int maxref = opts.max_refinements ? opts.max_refinements : 10;
    const int pmax = std::min<int>(pb, nrhs);
    const int ppad = ((pmax + 15) / 16) * 16;
    // basis capacity (vectors in Z; V holds up to pmax more): opts.max_iters, else from memory
    int64_t dmax = opts.max_iters;
    if (dmax == 0) {
        size_t freeb = 0, totalb = 0;
        HIPCHK(hipMemGetInfo(&freeb, &totalb));
        const double budget = 0.5 * (double)freeb;
        const double a = 16.0, b = 16.0 * (use_pc ? 2.0 : 1.0) * (double)n;   // R (d^2) + V, Z (d n)
        dmax = (int64_t)((-b + std::sqrt(b * b + 4.0 * a * budget)) / (2.0 * a));
        dmax = std::min<int64_t>(dmax, 24000);
    }
    dmax = std::min<int64_t>(dmax, n);
    dmax = std::max<int64_t>(dmax, pmax);
    const int64_t vcap = dmax + pmax;
    BlockWork bw;
    bw.V.alloc((size_t)2 * vcap * n);
    if (use_pc) bw.Z.alloc((size_t)2 * dmax * n);
    bw.Wa.alloc((size_t)2 * pmax * n);
    bw.Wb.alloc((size_t)2 * pmax * n);
    if (pc == MTF_PREC_BLOCK_TINV_GS) bw.Wt.alloc((size_t)2 * pmax * n);
    bw.tmp.alloc((size_t)2 * n);
    bw.npart.alloc((size_t)kNblk * pmax);
    const size_t hcount = (size_t)2 * (2 * vcap * ppad + ppad * ppad);   // H1, H2, Gram (complex)
    bw.hd.alloc(hcount);
    bw.hh[0] = pinned(hcount);
    bw.hh[1] = pinned(hcount);
    bw.hg = pinned((size_t)2 * ppad * ppad);
    bw.ht = pinned((size_t)2 * pmax * pmax);
    bw.hc = pinned((size_t)2 * vcap * pmax);
    int64_t pd = 0, pu = 0;
    for (int pp = 1; pp <= pmax; ++pp)
        for (int64_t j = 1; j <= vcap; ++j) {
            pd = std::max(pd, plan_bdot(n, (int)j, pp).part_elems);
            pu = std::max(pu, plan_bupd(n, (int)j, pp).part_elems);
        }
    bw.pdot.alloc((size_t)2 * pd);
    bw.pupd.alloc((size_t)2 * pu);
    bw.R.alloc((size_t)2 * dmax * dmax);
    bw.Y.alloc((size_t)2 * dmax * pmax);
    bw.T.alloc((size_t)2 * pmax * pmax);
    bw.cnt.alloc(pmax);
    bw.info.alloc(1);
    double* H1 = bw.hd.p;
    double* H2 = bw.hd.p + (size_t)2 * vcap * ppad;
    double* Gd = bw.hd.p + (size_t)4 * vcap * ppad;
    double* zbase = use_pc ? bw.Z.p : bw.V.p;

    auto norms = [&](const double* v, int64_t ldv, int nb) {
        launch_norm2(v, ldv, n, bw.npart.p, kNblk, nb, s);
        std::vector<double> h((size_t)kNblk * nb);
        HIPCHK(hipMemcpyAsync(h.data(), bw.npart.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        sync(p);
        std::vector<double> out(nb);
        for (int b = 0; b < nb; ++b) {
            double t = 0.0;
            for (int k = 0; k < kNblk; ++k) t += h[(size_t)b * kNblk + k];
            out[b] = std::sqrt(t);
        }
        return out;
    };
    auto gram_of = [&](const double* g, int k) {      // host k x k column-major from the [i][c] staging
        std::vector<cd> G((size_t)k * k);
        for (int i = 0; i < k; ++i)
            for (int c = 0; c < k; ++c) G[(size_t)c * k + i] = cd(g[2 * (i * ppad + c)], g[2 * (i * ppad + c) + 1]);
        return G;
    };
    // Gram matrix of k vectors at W (synchronises)
    auto gram = [&](const double* W, int k) {
        launch_bdot(plan_bdot(n, k, k), W, n, k, W, n, k, n, bw.pdot.p, Gd, ppad, s);
        HIPCHK(hipMemcpyAsync(bw.hg, Gd, (size_t)2 * k * ppad * sizeof(double), hipMemcpyDeviceToHost, s));
        sync(p);
        return gram_of(bw.hg, k);
    };
    // dst (k' vectors) = src (k vectors) T for a host k x k' matrix T (column-major); stream-ordered
    // (the pinned staging of T is rewritten only after a later synchronisation)
    auto combine = [&](const double* src, int k, const std::vector<cd>& T, int kk, double* dst) {
        for (int c = 0; c < kk; ++c)
            for (int i = 0; i < k; ++i) {
                bw.ht[2 * ((size_t)i * kk + c)] = T[(size_t)c * k + i].real();     // [i][c] layout
                bw.ht[2 * ((size_t)i * kk + c) + 1] = T[(size_t)c * k + i].imag();
            }
        HIPCHK(hipMemcpyAsync(bw.T.p, bw.ht, (size_t)2 * k * kk * sizeof(double), hipMemcpyHostToDevice, s));
        launch_bupd(plan_bupd(n, k, kk), src, n, k, bw.T.p, kk, 1, kk, n, bw.pupd.p, nullptr, n, dst, n, 1.0, 0.0, s);
    };
    // the k vectors in Wa -> orthonormal Q at dst with Wa ~= Q S; a second pass when the first was
    // ill-conditioned
    auto orthonormalize = [&](int k, const std::vector<cd>& G, const std::vector<double>& ref2, double* dst,
                              std::vector<cd>& S) {
        Svqb a = svqb(k, G, ref2, kBlockKeep);
        if (a.k == 0) {
            S.clear();
            return 0;
        }
        if (a.lmin > 1e-8) {
            combine(bw.Wa.p, k, a.T, a.k, dst);
            S = a.S;
            return a.k;
        }
        combine(bw.Wa.p, k, a.T, a.k, bw.Wb.p);
        const std::vector<cd> G2 = gram(bw.Wb.p, a.k);
        Svqb b2 = svqb(a.k, G2, std::vector<double>(a.k, 1.0), kBlockKeep);
        combine(bw.Wb.p, a.k, b2.T, b2.k, dst);
        S.assign((size_t)b2.k * k, cd(0.0, 0.0));        // S = S2 S1
        for (int c = 0; c < k; ++c)
            for (int r = 0; r < b2.k; ++r) {
                cd t = 0.0;
                for (int m = 0; m < a.k; ++m) t += b2.S[(size_t)m * b2.k + r] * a.S[(size_t)c * a.k + m];
                S[(size_t)c * b2.k + r] = t;
            }
        return b2.k;
    };
    // one block step on the GPU: Z_k = P V_k, W = M Z_k, two block Gram-Schmidt passes against the
    // nrow basis vectors, the Gram matrix of W; projections and Gram matrix copied to hh[buf]
    auto launch_step = [&](int64_t ncol_, int64_t nrow_, int pk_, int buf) {
        const double* vk = bw.V.p + 2 * n * (nrow_ - pk_);
        double* zk = zbase + 2 * n * ncol_;
        if (use_pc && pk_ >= kMmvMin) precond_block(p, pc, pk_, vk, zk, bw.Wt.p, n);
        else if (use_pc)
            for (int c = 0; c < pk_; ++c) {
                if (pc == MTF_PREC_BLOCK_TINV_GS) precond1_gs(p, vk + 2 * n * c, zk + 2 * n * c, bw.tmp.p);
                else precond1(p, vk + 2 * n * c, zk + 2 * n * c);
            }
        if (pk_ >= kMmvMin) matvec_mmv(p, pk_, zk, n, bw.Wa.p, n);
        else
            for (int c = 0; c < pk_; ++c) matvec1(p, zk + 2 * n * c, bw.Wa.p + 2 * n * c, MTF_FP64);
        const int j = (int)nrow_;
        const BlockDotPlan pdp = plan_bdot(n, j, pk_);
        const BlockUpdPlan pup = plan_bupd(n, j, pk_);
        launch_bdot(pdp, bw.V.p, n, j, bw.Wa.p, n, pk_, n, bw.pdot.p, H1, ppad, s);
        launch_bupd(pup, bw.V.p, n, j, H1, ppad, 1, pk_, n, bw.pupd.p, bw.Wa.p, n, bw.Wa.p, n, -1.0, 1.0, s);
        launch_bdot(pdp, bw.V.p, n, j, bw.Wa.p, n, pk_, n, bw.pdot.p, H2, ppad, s);
        launch_bupd(pup, bw.V.p, n, j, H2, ppad, 1, pk_, n, bw.pupd.p, bw.Wa.p, n, bw.Wa.p, n, -1.0, 1.0, s);
        launch_bdot(plan_bdot(n, pk_, pk_), bw.Wa.p, n, pk_, bw.Wa.p, n, pk_, n, bw.pdot.p, Gd, ppad, s);
        const size_t hj = (size_t)2 * j * ppad * sizeof(double);
        double* hb = bw.hh[buf];
        HIPCHK(hipMemcpyAsync(hb, H1, hj, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(hb + (H2 - H1), H2, hj, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(hb + (Gd - H1), Gd, (size_t)2 * ppad * ppad * sizeof(double), hipMemcpyDeviceToHost, s));
    };

    int status = MTF_OK;
    BlockLsq ls;
    for (int g0 = 0; g0 < nrhs; g0 += pb) {
        const int q = std::min(pb, nrhs - g0);
        auto t0 = std::chrono::steady_clock::now();
        const double* B = Bp + 2 * ld * (int64_t)g0;
        double* X = Xp + 2 * ld * (int64_t)g0;
        for (int c = 0; c < q; ++c) {
            if (opts.x0_dev)
                HIPCHK(hipMemcpyAsync(X + 2 * ld * c, static_cast<const double*>(opts.x0_dev) + 2 * ld * (int64_t)(g0 + c),
                                      2 * n * sizeof(double), hipMemcpyDeviceToDevice, s));
            else launch_fill(X + 2 * ld * c, 2 * n, 0.0, s);
        }
        const std::vector<double> bn = norms(B, ld, q);
        std::vector<double> rel(q, 1.0);
        std::vector<char> conv(q, 0);
        std::vector<int> refin(q, 0);
        int steps_total = 0;
        for (int outer = 0; outer <= maxref; ++outer) {
            for (int c = 0; c < q; ++c) {                                // W = B - M X (FP64)
                double* wc = bw.Wa.p + 2 * n * c;
                matvec1(p, X + 2 * ld * c, wc, MTF_FP64);
                launch_axpby(wc, B + 2 * ld * c, n, 1.0, 0.0, -1.0, s);
            }
            const std::vector<double> rn = norms(bw.Wa.p, n, q);
            bool all = true;
            std::vector<double> ref2(q), tol(q);
            for (int c = 0; c < q; ++c) {
                rel[c] = bn[c] > 0.0 ? rn[c] / bn[c] : 0.0;
                if (outer > 0 && !conv[c]) ++refin[c];
                conv[c] = rel[c] <= opts.rtol;
                ref2[c] = conv[c] ? 0.0 : rn[c] * rn[c];                 // converged columns drop out
                tol[c] = 0.9 * opts.rtol * bn[c];
                if (!conv[c]) all = false;
            }
            if (all || outer == maxref) break;
            for (int c = 0; c < q; ++c)
                if (conv[c]) launch_fill(bw.Wa.p + 2 * n * c, 2 * n, 0.0, s);
            // V_1 S_0 = R (the residual block)
            std::vector<cd> S;
            int pk = orthonormalize(q, gram(bw.Wa.p, q), ref2, bw.V.p, S);
            ls.init((int)dmax, vcap, pmax, q);
            for (int c = 0; c < q; ++c)
                for (int r = 0; r < pk; ++r) {
                    ls.G[2 * ((size_t)c * vcap + r)] = S[(size_t)c * pk + r].real();
                    ls.G[2 * ((size_t)c * vcap + r) + 1] = S[(size_t)c * pk + r].imag();
                }
            int64_t ncol = 0, nrow = pk;     // columns of the Hessenberg matrix reduced; basis vectors
            int steps = 0, buf = 0;
            if (pk > 0 && pk <= dmax) launch_step(ncol, nrow, pk, buf);
            else pk = 0;
            while (pk > 0) {
                sync(p);                                                  // step data in hh[buf]
                const int j = (int)nrow;
                const double* h1 = bw.hh[buf];
                const double* h2 = h1 + (size_t)2 * vcap * ppad;
                const std::vector<cd> G = gram_of(h1 + (size_t)4 * vcap * ppad, pk);
                std::vector<double> r2(pk);
                for (int c = 0; c < pk; ++c) {
                    double t = G[(size_t)c * pk + c].real();
                    for (int i = 0; i < j; ++i) {
                        const size_t e = 2 * ((size_t)i * ppad + c);
                        t += std::norm(cd(h1[e] + h2[e], h1[e + 1] + h2[e + 1]));
                    }
                    r2[c] = t;                                           // ||M z_c||^2
                }
                std::vector<cd> Sn;
                const int pnew = orthonormalize(pk, G, r2, bw.V.p + 2 * n * nrow, Sn);
                const int64_t rows = nrow + pnew;
                const bool more = pnew > 0 && ncol + pk + pnew <= dmax;
                if (more) launch_step(ncol + pk, rows, pnew, buf ^ 1);   // overlaps the reduction below
                // new block column: rows 0..j-1 from the projections, then S
                double* hc = bw.hc;
                for (int c = 0; c < pk; ++c) {
                    double* y = hc + (size_t)2 * rows * c;
                    for (int i = 0; i < j; ++i) {
                        const size_t e = 2 * ((size_t)i * ppad + c);
                        y[2 * i] = h1[e] + h2[e];
                        y[2 * i + 1] = h1[e + 1] + h2[e + 1];
                    }
                    for (int r = 0; r < pnew; ++r) {
                        y[2 * (j + r)] = Sn[(size_t)c * pnew + r].real();
                        y[2 * (j + r) + 1] = Sn[(size_t)c * pnew + r].imag();
                    }
                }
                // earlier reflectors on the new columns (independent columns: host threads)
                host_parallel(pk, ncol * pk > 8192, [&](int c) {
                    double* y = hc + (size_t)2 * rows * c;
                    for (int64_t m = 0; m < ncol; ++m) ls.apply((int)m, y);
                });
                for (int c = 0; c < pk; ++c) {
                    const int64_t col = ncol + c;
                    double* y = hc + (size_t)2 * rows * c;
                    ls.make((int)col, (int)(rows - col), y);
                    for (int c2 = c + 1; c2 < pk; ++c2) ls.apply((int)col, hc + (size_t)2 * rows * c2);
                    for (int r = 0; r < q; ++r) ls.apply((int)col, ls.G.data() + (size_t)2 * vcap * r);
                }
                // R columns ncol .. ncol + pk - 1 (rows 0 .. ncol + pk - 1; zero below the diagonal)
                HIPCHK(hipMemcpy2DAsync(bw.R.p + (size_t)2 * ncol * dmax, (size_t)2 * dmax * sizeof(double), hc,
                                        (size_t)2 * rows * sizeof(double), (size_t)2 * (ncol + pk) * sizeof(double), pk,
                                        hipMemcpyHostToDevice, s));
                ncol += pk;
                nrow = rows;
                pk = pnew;
                ++steps;
                bool done = true;
                for (int c = 0; c < q; ++c) {
                    if (ref2[c] == 0.0) continue;
                    double t = 0.0;
                    for (int64_t r = ncol; r < nrow; ++r) {
                        const size_t e = 2 * ((size_t)c * vcap + r);
                        t += ls.G[e] * ls.G[e] + ls.G[e + 1] * ls.G[e + 1];
                    }
                    if (std::sqrt(t) > tol[c]) done = false;
                }
                if (done || !more) break;
                buf ^= 1;
            }
            steps_total += steps;
            if (ncol == 0) break;
            // X += Z Y, Y = R^-1 G(0:ncol, :)   (after a step launched past convergence, which
            // touches neither Z(0:ncol) nor R)
            std::vector<double> yh((size_t)2 * dmax * q, 0.0);
            for (int c = 0; c < q; ++c)
                std::memcpy(yh.data() + (size_t)2 * dmax * c, ls.G.data() + (size_t)2 * vcap * c,
                            (size_t)2 * ncol * sizeof(double));
            HIPCHK(hipMemcpyAsync(bw.Y.p, yh.data(), yh.size() * sizeof(double), hipMemcpyHostToDevice, s));
            std::vector<int> cn(q, (int)ncol);
            HIPCHK(hipMemcpyAsync(bw.cnt.p, cn.data(), q * sizeof(int), hipMemcpyHostToDevice, s));
            HIPCHK(hipMemsetAsync(bw.info.p, 0, sizeof(int), s));
            launch_trsv_upper(bw.R.p, dmax, 0, bw.cnt.p, bw.Y.p, dmax, bw.info.p, q, s);
            launch_bupd(plan_bupd(n, (int)ncol, q), zbase, n, (int)ncol, bw.Y.p, 1, dmax, q, n, bw.pupd.p, X, ld, X, ld,
                        1.0, 1.0, s);
            int info = 0;
            HIPCHK(hipMemcpyAsync(&info, bw.info.p, sizeof(int), hipMemcpyDeviceToHost, s));
            sync(p);
            if (info) throw NonFiniteError("block GMRES: zero pivot in the least-squares factor");
        }
        const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        for (int c = 0; c < q; ++c) {
            if (stats) {
                mtf_solve_stats& st = stats[g0 + c];
                st.iterations = steps_total;
                st.refinements = refin[c];
                st.converged = conv[c] ? 1 : 0;
                st.reorthogonalizations = steps_total;
                st.rel_residual = rel[c];
                st.t_precond_s = (g0 + c) == 0 ? t_pc : 0.0;
                st.t_solve_s = dt;
            }
            if (!conv[c]) status = MTF_NOT_CONVERGED;
        }
    }
    return status;
}

int solve_impl(mtf_problem p, int32_t nrhs, const void* b_dev, void* x_dev, int64_t ld, const mtf_solve_opts* o,
               mtf_solve_stats* stats) {
    if (!p->has_mesh || !p->has_mat) throw StateError("mtf_solve before mesh/materials");
    if (nrhs < 1 || !b_dev || !x_dev || ld < p->sk.N) throw ArgError("mtf_solve: bad nrhs, pointers or ld");
    mtf_solve_opts opts;
    std::memset(&opts, 0, sizeof(opts));
    opts.struct_size = sizeof(opts);
    opts.rtol = 1e-6;
    if (o) {
        if (o->struct_size < (int)sizeof(mtf_solve_opts)) throw ArgError("mtf_solve_opts.struct_size too small");
        opts = *o;
    }
    if (!(opts.rtol > 0.0) || !(opts.rtol < 1.0)) throw ArgError("rtol must be in (0, 1)");
    if (opts.max_iters < 0 || opts.max_refinements < 0) throw ArgError("negative iteration limits");
    int maxit = opts.max_iters;
    const int maxref = opts.max_refinements ? opts.max_refinements : 10;
    const int prec = opts.precision;
    check_prec_available(p, prec);
    if (!p->have64) throw StateError("mtf_solve checks residuals with the FP64 operator: assemble MTF_FP64 first");
    if (opts.preconditioner != MTF_PREC_NONE && opts.preconditioner != MTF_PREC_BLOCK_TINV &&
        opts.preconditioner != MTF_PREC_BLOCK_TINV_GS)
        throw ArgError("unknown preconditioner");
    DeviceGuard g(p->device);
    const int pc = opts.preconditioner;
    const bool use_pc = pc != MTF_PREC_NONE;
    if (opts.flags & ~(MTF_SOLVE_EAGER | MTF_SOLVE_PC_FULL | MTF_SOLVE_PC_DIRECT | MTF_SOLVE_BASIS_C64 | MTF_SOLVE_BLOCK(0xff)))
        throw ArgError("unknown solve flags");
    const bool basis_c64 = (opts.flags & MTF_SOLVE_BASIS_C64) != 0;
    const int block = (opts.flags >> 8) & 0xff;
    if (block > 0) {
        if (block > kMaxBlock) throw ArgError("block GMRES takes at most 32 right-hand sides per block");
        if (prec != MTF_FP64) throw UnsupportedError("block GMRES runs with the FP64 operator only");
        if (basis_c64) throw UnsupportedError("block GMRES keeps its basis in complex128");
    }
    if (basis_c64 && !use_pc) throw ArgError("MTF_SOLVE_BASIS_C64 needs a preconditioner (the flexible iteration)");
    const bool graph = (opts.flags & MTF_SOLVE_EAGER) == 0;
    const int pc_kind = pc_kind_of(opts.flags);
    double t_pc = 0;
    if (use_pc && (!p->have_tinv || p->pc_kind != pc_kind)) { build_tinv(p, pc_kind); t_pc = p->t_precond; }
    if (block > 0)
        return block_solve(p, nrhs, static_cast<const double*>(b_dev), static_cast<double*>(x_dev), ld, opts, block, pc,
                           stats, t_pc);
    // right-hand sides advance in lockstep batches when the products are GEMMs
    const int nbmax = prec == MTF_BF16_SPLIT ? std::min<int>(nrhs, kMaxBatch) : 1;
    if (maxit == 0) {
        // cycle length from memory: the Krylov slabs (basis, and the preconditioned candidates when
        // flexible: 16 N nb bytes per step each) and the Hessenberg matrix and triangular factor
        // (16 nb m^2 bytes each) may take half of the free device memory plus what this problem
        // already holds; at most 8000 steps for one right-hand side, 2000 for lockstep batches
        size_t freeb = 0, totalb = 0;
        HIPCHK(hipMemGetInfo(&freeb, &totalb));
        const GmresWork& w = p->gw;
        const double held = (double)(w.V.n + w.Zt.n + w.H.n + w.Rf.n) * sizeof(double);
        const double budget = 0.5 * ((double)freeb + held);
        const double f = use_pc ? 2.0 : 1.0;
        const double a = 16.0 * nbmax * f, bcoef = 16.0 * (double)p->sk.N * nbmax * f;
        const double m = (-bcoef + std::sqrt(bcoef * bcoef + 4.0 * a * budget)) / (2.0 * a);
        maxit = (int)std::min({nbmax > 1 ? 2000.0 : 8000.0, (double)p->sk.N, std::max(100.0, m)});
    }
    gmres_alloc(p, maxit, nbmax, use_pc);
    GmresWork& w = p->gw;
    hipStream_t s = p->stream;
    const int64_t n = p->sk.N;
    int status = MTF_OK;
    for (int r0 = 0; r0 < nrhs; r0 += nbmax) {
        const int nb = std::min(nbmax, nrhs - r0);
        auto t0 = std::chrono::steady_clock::now();
        const double* B = static_cast<const double*>(b_dev) + 2 * ld * (int64_t)r0;
        double* X = static_cast<double*>(x_dev) + 2 * ld * (int64_t)r0;
        for (int b = 0; b < nb; ++b) {
            if (opts.x0_dev)
                HIPCHK(hipMemcpyAsync(X + 2 * ld * b, static_cast<const double*>(opts.x0_dev) + 2 * ld * (int64_t)(r0 + b),
                                      2 * n * sizeof(double), hipMemcpyDeviceToDevice, s));
            else launch_fill(X + 2 * ld * b, 2 * n, 0.0, s);
        }
        const std::vector<double> bn = norms_dev(p, B, ld, nb);
        std::vector<int> iters(nb, 0), refin(nb, 0), reorth(nb, 0), itv;
        std::vector<double> rel(nb, 1.0), est;
        std::vector<char> conv(nb, 0);
        int total = 0;
        double delta = -1.0;
        for (int outer = 0; outer <= maxref; ++outer) {
            // true residuals with the FP64 operator (r = b itself from the zero initial guess)
            for (int b = 0; b < nb; ++b) {
                double* rb = w.r.p + 2 * n * b;
                if (outer == 0 && !opts.x0_dev) {
                    HIPCHK(hipMemcpyAsync(rb, B + 2 * ld * b, 2 * n * sizeof(double), hipMemcpyDeviceToDevice, s));
                    continue;
                }
                matvec1(p, X + 2 * ld * b, rb, MTF_FP64);
                launch_axpby(rb, B + 2 * ld * b, n, 1.0, 0.0, -1.0, s);   // r = b - M x
            }
            const std::vector<double> rn = norms_dev(p, w.r.p, n, nb);
            bool all = true;
            std::vector<double> tol(nb, 1.0);
            for (int b = 0; b < nb; ++b) {
                rel[b] = bn[b] > 0 ? rn[b] / bn[b] : 0.0;
                if (outer > 0 && !conv[b]) ++refin[b];
                conv[b] = rel[b] <= opts.rtol;
                if (conv[b]) { launch_fill(w.r.p + 2 * n * b, 2 * n, 0.0, s); continue; }
                all = false;
                double t = opts.rtol * bn[b] / rn[b];
                if (prec != MTF_FP64) t = std::max(t, opts.inner_rtol > 0 ? opts.inner_rtol : 1e-6);
                else if (opts.inner_rtol > 0) t = std::max(t, opts.inner_rtol);
                // the complex64 cycle leaves room for the gap its products open between the
                // recurrence and the FP64 residual
                tol[b] = (prec == MTF_FP32_MIXED ? 0.5 : 0.9) * t;
            }
            if (all || outer == maxref || total >= maxit * (maxref + 1)) break;
            double relax = 1.0;
            if (prec == MTF_FP32_MIXED && nb == 1) {
                // relative difference of the two operators on this residual; the complex64 products
                // are admitted once the recurrence residual has fallen to 1% of tol / delta
                if (delta < 0.0) delta = operator_gap(p, w.r.p);
                if (delta > 0.0) relax = std::min(1.0, 0.01 * tol[0] / delta);
            }
            total += gmres_cycle(p, w.r.p, X, ld, nb, prec, pc, tol, maxit, itv, est, reorth, graph, relax, basis_c64);
            for (int b = 0; b < nb; ++b) iters[b] += itv[b];
        }
        const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        for (int b = 0; b < nb; ++b) {
            if (stats) {
                mtf_solve_stats& st = stats[r0 + b];
                st.iterations = iters[b];
                st.refinements = refin[b];
                st.converged = conv[b] ? 1 : 0;
                st.reorthogonalizations = reorth[b];
                st.rel_residual = rel[b];
                st.t_precond_s = (r0 + b) == 0 ? t_pc : 0.0;
                st.t_solve_s = dt;
            }
            if (!conv[b]) status = MTF_NOT_CONVERGED;
        }
    }
    return status;
}

// GMRES on the single-trace system M_STF u = b (M = 1, FP64 operator, no preconditioner): cycles
// until the FP64 residual of the single-trace operator meets rtol.
int solve_stf_impl(mtf_problem p, int32_t nrhs, const void* b_dev, void* x_dev, int64_t ld, const mtf_solve_opts* o,
                   mtf_solve_stats* stats) {
    if (!p->has_mesh || !p->has_mat) throw StateError("mtf_solve_stf before mesh/materials");
    mtf_solve_opts opts;
    std::memset(&opts, 0, sizeof(opts));
    opts.struct_size = sizeof(opts);
    opts.rtol = 1e-6;
    if (o) {
        if (o->struct_size < (int)sizeof(mtf_solve_opts)) throw ArgError("mtf_solve_opts.struct_size too small");
        opts = *o;
    }
    const int64_t n = 2 * (int64_t)p->sk.dom[0].E;
    if (nrhs < 1 || !b_dev || !x_dev || ld < n) throw ArgError("mtf_solve_stf: bad nrhs, pointers or ld");
    if (!(opts.rtol > 0.0) || !(opts.rtol < 1.0)) throw ArgError("rtol must be in (0, 1)");
    if (opts.max_iters < 0 || opts.max_refinements < 0) throw ArgError("negative iteration limits");
    if (opts.precision != MTF_FP64) throw UnsupportedError("mtf_solve_stf runs the FP64 operator only");
    if (opts.preconditioner != MTF_PREC_NONE) throw UnsupportedError("mtf_solve_stf has no preconditioner");
    if (opts.flags & ~MTF_SOLVE_EAGER) throw ArgError("mtf_solve_stf accepts MTF_SOLVE_EAGER only");
    if (!p->have64) throw StateError("mtf_solve_stf needs the FP64 blocks");
    DeviceGuard g(p->device);
    stf_prepare(p);
    struct Mode {
        mtf_problem p;
        ~Mode() { p->stf = false; }
    } mode{p};
    p->stf = true;
    const int maxit = opts.max_iters ? opts.max_iters : (int)std::min<int64_t>(n, 4000);
    const int maxref = opts.max_refinements ? opts.max_refinements : 10;
    gmres_alloc(p, maxit, 1, false);
    GmresWork& w = p->gw;
    hipStream_t s = p->stream;
    int status = MTF_OK;
    for (int r = 0; r < nrhs; ++r) {
        auto t0 = std::chrono::steady_clock::now();
        const double* B = static_cast<const double*>(b_dev) + 2 * ld * (int64_t)r;
        double* X = static_cast<double*>(x_dev) + 2 * ld * (int64_t)r;
        if (opts.x0_dev)
            HIPCHK(hipMemcpyAsync(X, static_cast<const double*>(opts.x0_dev) + 2 * ld * (int64_t)r, 2 * n * sizeof(double),
                                  hipMemcpyDeviceToDevice, s));
        else launch_fill(X, 2 * n, 0.0, s);
        const double bn = norms_dev(p, B, n, 1)[0];
        int iters = 0, refin = 0;
        double rel = 1.0;
        bool conv = false;
        std::vector<int> itv, reorth(1, 0);
        std::vector<double> est;
        for (int outer = 0; outer <= maxref; ++outer) {
            stf_matvec(p, X, w.r.p, n, 1);
            launch_axpby(w.r.p, B, n, 1.0, 0.0, -1.0, s);           // r = b - M_STF x
            const double rn = norms_dev(p, w.r.p, n, 1)[0];
            rel = bn > 0 ? rn / bn : 0.0;
            if (outer > 0) ++refin;
            conv = rel <= opts.rtol;
            if (conv || outer == maxref) break;
            const std::vector<double> tol(1, 0.9 * opts.rtol * bn / rn);
            gmres_cycle(p, w.r.p, X, ld, 1, MTF_FP64, MTF_PREC_NONE, tol, maxit, itv, est, reorth,
                        (opts.flags & MTF_SOLVE_EAGER) == 0, 1.0, false);
            iters += itv[0];
        }
        if (stats) {
            mtf_solve_stats& st = stats[r];
            st.iterations = iters;
            st.refinements = refin;
            st.converged = conv ? 1 : 0;
            st.reorthogonalizations = reorth[0];
            st.rel_residual = rel;
            st.t_precond_s = 0.0;
            st.t_solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        }
        if (!conv) status = MTF_NOT_CONVERGED;
    }
    return status;
}

bool finite_all(const double* a, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

}  // namespace

namespace mtf {
thread_local std::string g_err = "no error";

void problem_info(mtf_problem p, int* device, hipStream_t* stream, int64_t* N) {
    if (!p) throw ArgError("problem is NULL");
    if (!p->has_mesh) throw StateError("no mesh");
    *device = p->device;
    *stream = p->stream;
    *N = p->sk.N;
}
}  // namespace mtf

extern "C" {

const char* mtf_last_error(void) { return g_err.c_str(); }

int mtf_version(int* major, int* minor) {
    if (major) *major = 0;
    if (minor) *minor = 1;
    return MTF_OK;
}

int mtf_problem_create(mtf_problem* out, int device, void* stream) {
    return guarded([&] {
        if (!out) throw ArgError("out is NULL");
        *out = nullptr;
        int n = 0;
        HIPCHK(hipGetDeviceCount(&n));
        if (device < 0 || device >= n) throw ArgError("device index out of range");
        auto p = std::make_unique<mtf_problem_s>();
        p->device = device;
        p->stream = static_cast<hipStream_t>(stream);
        *out = p.release();
        return MTF_OK;
    });
}

int mtf_problem_destroy(mtf_problem p) {
    if (!p) return MTF_OK;
    return guarded([&] {
        {
            DeviceGuard g(p->device);
            (void)hipStreamSynchronize(p->stream);
            delete p;
        }
        return MTF_OK;
    });
}

int mtf_set_mesh(mtf_problem p, int64_t nv, const double* xyz, int64_t nt, const int32_t* tri, const int32_t* label,
                 int32_t M) {
    return guarded([&] {
        if (!p) throw ArgError("problem is NULL");
        set_mesh_impl(p, nv, xyz, nt, tri, label, M);
        return MTF_OK;
    });
}

int mtf_set_materials(mtf_problem p, double k0, const double* eps_r, const double* mu_r) {
    return guarded([&] {
        if (!p) throw ArgError("problem is NULL");
        if (!p->has_mesh) throw StateError("mtf_set_materials before mtf_set_mesh");
        if (!eps_r || !mu_r) throw ArgError("eps_r / mu_r is NULL");
        if (!(k0 > 0.0) || !std::isfinite(k0)) throw ArgError("k0 must be positive and finite");
        const int M = p->sk.M;
        for (int i = 0; i <= M; ++i)
            if (!(eps_r[i] > 0.0) || !(mu_r[i] > 0.0) || !std::isfinite(eps_r[i]) || !std::isfinite(mu_r[i]))
                throw ArgError("eps_r and mu_r must be positive and finite");
        {
            // the FP64 kernel evaluation reduces phases k_i r exactly only below about 1.6e6
            double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
            for (int64_t v = 0; v < p->sk.nv; ++v)
                for (int c = 0; c < 3; ++c) {
                    lo[c] = std::min(lo[c], p->sk.xyz[3 * v + c]);
                    hi[c] = std::max(hi[c], p->sk.xyz[3 * v + c]);
                }
            const double diam = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                                          (hi[2] - lo[2]) * (hi[2] - lo[2]));
            for (int i = 0; i <= M; ++i)
                if (!(k0 * std::sqrt(eps_r[i] * mu_r[i]) * diam < 1e6))
                    throw UnsupportedError("k_i times the mesh diameter must be below 1e6");
        }
        DeviceGuard g(p->device);
        p->k0 = k0;
        p->eps.assign(eps_r, eps_r + M + 1);
        p->mu.assign(mu_r, mu_r + M + 1);
        p->kw.resize(M + 1);
        p->rho.resize(M + 1);
        for (int i = 0; i <= M; ++i) {
            p->kw[i] = k0 * std::sqrt(eps_r[i] * mu_r[i]);
            p->rho[i] = std::sqrt(eps_r[i] / mu_r[i]);
        }
        p->has_mat = true;
        upload_doms(p);
        sync(p);
        p->have64 = p->have32 = p->have_tinv = false;
        return MTF_OK;
    });
}

int mtf_get_sizes(mtf_problem p, int64_t* N, int64_t* E) {
    return guarded([&] {
        if (!p) throw ArgError("problem is NULL");
        if (!p->has_mesh) throw StateError("no mesh");
        if (N) *N = p->sk.N;
        if (E)
            for (int i = 0; i <= p->sk.M; ++i) E[i] = p->sk.dom[i].E;
        return MTF_OK;
    });
}

int mtf_get_dof_map(mtf_problem p, int32_t i, int32_t* edge_vtx, int32_t* plus_tri) {
    return guarded([&] {
        if (!p) throw ArgError("problem is NULL");
        if (!p->has_mesh) throw StateError("no mesh");
        if (i < 0 || i > p->sk.M) throw ArgError("subdomain index out of range");
        const Domain& d = p->sk.dom[i];
        if (edge_vtx) std::memcpy(edge_vtx, d.edge_vtx.data(), 2 * d.E * sizeof(int32_t));
        if (plus_tri)
            for (int m = 0; m < d.E; ++m) plus_tri[m] = d.tri[d.plus[2 * m]];
        return MTF_OK;
    });
}

int mtf_assemble(mtf_problem p, const mtf_assembly_opts* opts) {
    return guarded([&] {
        if (!p) throw ArgError("problem is NULL");
        assemble_impl(p, opts);
        return MTF_OK;
    });
}

int mtf_copy_block(mtf_problem p, int32_t i, int32_t which, int32_t precision, double* dst) {
    return guarded([&] {
        if (!p || !dst) throw ArgError("NULL argument");
        if (!p->has_mesh) throw StateError("no mesh");
        if (i < 0 || i > p->sk.M) throw ArgError("subdomain index out of range");
        if (which != MTF_BLOCK_T && which != MTF_BLOCK_K) throw ArgError("which must be MTF_BLOCK_T or MTF_BLOCK_K");
        check_prec_available(p, precision);
        DeviceGuard g(p->device);
        const DomDesc& d = p->doms[i];
        const int64_t ne = 2 * (int64_t)d.E * d.E;
        if (precision == MTF_FP64) {
            const double* src = (which == MTF_BLOCK_T ? p->T64.p : p->K64.p) + 2 * d.mat0;
            HIPCHK(hipMemcpyAsync(dst, src, ne * sizeof(double), hipMemcpyDeviceToHost, p->stream));
            sync(p);
        } else {
            std::vector<float> tmp(ne);
            const float* src = (which == MTF_BLOCK_T ? p->T32.p : p->K32.p) + 2 * d.mat0;
            HIPCHK(hipMemcpyAsync(tmp.data(), src, ne * sizeof(float), hipMemcpyDeviceToHost, p->stream));
            sync(p);
            for (int64_t e = 0; e < ne; ++e) dst[e] = tmp[e];
        }
        return MTF_OK;
    });
}

int mtf_get_entries(mtf_problem p, int32_t i, int32_t which, int32_t precision, int32_t n, const int32_t* rows,
                    const int32_t* cols, double* out) {
    return guarded([&] {
        if (!p || !rows || !cols || !out || n < 0) throw ArgError("bad arguments");
        if (!p->has_mesh) throw StateError("no mesh");
        if (i < 0 || i > p->sk.M) throw ArgError("subdomain index out of range");
        if (which != MTF_BLOCK_T && which != MTF_BLOCK_K) throw ArgError("which must be MTF_BLOCK_T or MTF_BLOCK_K");
        if (precision != MTF_FP64 && precision != MTF_FP32_MIXED) throw ArgError("precision must be MTF_FP64 or MTF_FP32_MIXED");
        check_prec_available(p, precision);
        const DomDesc& d = p->doms[i];
        for (int k = 0; k < n; ++k)
            if (rows[k] < 0 || rows[k] >= d.E || cols[k] < 0 || cols[k] >= d.E) throw ArgError("entry index out of range");
        DeviceGuard g(p->device);
        for (int k = 0; k < n; ++k) {
            const int64_t e = d.mat0 + rows[k] + (int64_t)cols[k] * d.E;
            if (precision == MTF_FP64) {
                const double* src = (which == MTF_BLOCK_T ? p->T64.p : p->K64.p) + 2 * e;
                HIPCHK(hipMemcpyAsync(out + 2 * k, src, 2 * sizeof(double), hipMemcpyDeviceToHost, p->stream));
            } else {
                float tmp[2];
                const float* src = (which == MTF_BLOCK_T ? p->T32.p : p->K32.p) + 2 * e;
                HIPCHK(hipMemcpyAsync(tmp, src, 2 * sizeof(float), hipMemcpyDeviceToHost, p->stream));
                sync(p);
                out[2 * k] = tmp[0];
                out[2 * k + 1] = tmp[1];
            }
        }
        sync(p);
        return MTF_OK;
    });
}

int mtf_copy_transmission(mtf_problem p, int32_t i, int32_t j, double* dst) {
    return guarded([&] {
        if (!p || !dst) throw ArgError("NULL argument");
        if (!p->has_mesh) throw StateError("no mesh");
        const int M = p->sk.M;
        if (i < 0 || i > M || j < 0 || j > M) throw ArgError("subdomain index out of range");
        DeviceGuard g(p->device);
        const DomDesc& di = p->doms[i];
        const DomDesc& dj = p->doms[j];
        std::vector<double> gval(9 * (size_t)di.T);
        std::vector<int64_t> gcol(6 * (size_t)di.T);
        HIPCHK(hipMemcpyAsync(gval.data(), p->d_gval.p + 9 * di.rec0, gval.size() * sizeof(double), hipMemcpyDeviceToHost, p->stream));
        HIPCHK(hipMemcpyAsync(gcol.data(), p->d_gcol.p + 6 * di.rec0, gcol.size() * sizeof(int64_t), hipMemcpyDeviceToHost, p->stream));
        sync(p);
        std::memset(dst, 0, sizeof(double) * (size_t)di.E * dj.E);
        const Domain& d = p->sk.dom[i];
        for (int lt = 0; lt < d.T; ++lt) {
            if (d.other[lt] != j) continue;
            for (int a = 0; a < 3; ++a) {
                const int m = d.tri_dof[3 * lt + a];
                for (int c = 0; c < 3; ++c) {
                    const int64_t col = gcol[6 * lt + c] - dj.off;
                    dst[m + col * di.E] += gval[9 * lt + 3 * a + c];
                }
            }
        }
        return MTF_OK;
    });
}

int mtf_rhs_plane_waves(mtf_problem p, int32_t nrhs, const double* d, const double* p_re, const double* p_im,
                        void* b_dev, int64_t ldb) {
    return guarded([&] {
        if (!p) throw ArgError("problem is NULL");
        if (!p->has_mesh || !p->has_mat) throw StateError("mtf_rhs_plane_waves before mesh/materials");
        if (nrhs < 1 || !d || !p_re || !p_im || !b_dev || ldb < p->sk.N) throw ArgError("bad arguments");
        if (!finite_all(d, 3 * nrhs) || !finite_all(p_re, 3 * nrhs) || !finite_all(p_im, 3 * nrhs))
            throw ArgError("non-finite direction or polarisation");
        for (int r = 0; r < nrhs; ++r) {
            const double nn = d[3 * r] * d[3 * r] + d[3 * r + 1] * d[3 * r + 1] + d[3 * r + 2] * d[3 * r + 2];
            if (std::fabs(nn - 1.0) > 1e-9) throw ArgError("directions must be unit vectors");
        }
        DeviceGuard g(p->device);
        std::vector<double> host(3 * nrhs + 6 * nrhs);
        std::memcpy(host.data(), d, 3 * nrhs * sizeof(double));
        for (int r = 0; r < nrhs; ++r)
            for (int k = 0; k < 3; ++k) {
                host[3 * nrhs + 6 * r + 2 * k] = p_re[3 * r + k];
                host[3 * nrhs + 6 * r + 2 * k + 1] = p_im[3 * r + k];
            }
        DevBuf<double> buf;
        buf.upload(host, p->stream);
        double* b = static_cast<double*>(b_dev);
        launch_fill(b, 2 * ldb * (int64_t)nrhs, 0.0, p->stream);
        launch_rhs(&p->doms[0], p->d_geom.p, p->d_dplus.p, p->d_dminus.p, p->doms[0].E, p->k0, p->rho[0], nrhs, buf.p,
                   buf.p + 3 * nrhs, b, ldb, p->stream);
        HIPCHK(hipGetLastError());
        sync(p);
        return MTF_OK;
    });
}

int mtf_matvec(mtf_problem p, int32_t nrhs, const void* x_dev, void* y_dev, int64_t ld, int32_t precision) {
    return guarded([&] {
        if (!p) throw ArgError("problem is NULL");
        if (!p->has_mesh || !p->has_mat) throw StateError("mtf_matvec before mesh/materials");
        if (nrhs < 1 || !x_dev || !y_dev || ld < p->sk.N) throw ArgError("bad arguments");
        if (x_dev == y_dev) throw ArgError("x and y must not alias");
        if (precision == MTF_FP64_MFMA) {
            if (nrhs > kMaxBlock) throw ArgError("MTF_FP64_MFMA takes at most 32 vectors");
            check_prec_available(p, MTF_FP64);
        } else {
            check_prec_available(p, precision);
        }
        DeviceGuard g(p->device);
        if (precision == MTF_FP64_MFMA) {
            matvec_mmv(p, nrhs, static_cast<const double*>(x_dev), ld, static_cast<double*>(y_dev), ld);
        } else if (precision == MTF_BF16_SPLIT) {
            matvec_gemm(p, nrhs, static_cast<const double*>(x_dev), ld, static_cast<double*>(y_dev));
        } else {
            for (int r = 0; r < nrhs; ++r)
                matvec1(p, static_cast<const double*>(x_dev) + 2 * ld * (int64_t)r,
                        static_cast<double*>(y_dev) + 2 * ld * (int64_t)r, precision);
        }
        HIPCHK(hipGetLastError());
        return MTF_OK;
    });
}

int mtf_matvec_noalloc(mtf_problem p, int32_t nrhs, const void* x_dev, void* y_dev, int64_t ld, int32_t precision) {
    return guarded([&] {
        if (!p) throw ArgError("problem is NULL");
        if (!p->has_mesh || !p->has_mat) throw StateError("mtf_matvec_noalloc before mesh/materials");
        if (nrhs < 1 || !x_dev || !y_dev || ld < p->sk.N) throw ArgError("bad arguments");
        if (x_dev == y_dev) throw ArgError("x and y must not alias");
        if (precision != MTF_FP64 && precision != MTF_FP32_MIXED)
            throw ArgError("mtf_matvec_noalloc: precision must be MTF_FP64 or MTF_FP32_MIXED");
        if (2 * p->part_entries > kScratchReals)
            throw ArgError("mtf_matvec_noalloc: the product needs " + std::to_string(16 * p->part_entries) +
                           " bytes of partial sums, more than the static scratch of " +
                           std::to_string(8 * kScratchReals) + " bytes");
        check_prec_available(p, precision);
        DeviceGuard g(p->device);
        double* ws = scratch_on(p->device);
        for (int r = 0; r < nrhs; ++r)
            matvec1(p, static_cast<const double*>(x_dev) + 2 * ld * (int64_t)r,
                    static_cast<double*>(y_dev) + 2 * ld * (int64_t)r, precision, ws);
        HIPCHK(hipGetLastError());
        return MTF_OK;
    });
}

int mtf_time_matvec(mtf_problem p, int32_t precision, int32_t reps, const void* x_dev, void* y_dev, double* dense_s,
                    double* total_s) {
    return guarded([&] {
        if (!p || !x_dev || !y_dev || !dense_s || !total_s) throw ArgError("bad arguments");
        if (!p->has_mesh || !p->has_mat) throw StateError("mtf_time_matvec before mesh/materials");
        if (reps < 1 || reps > 10000) throw ArgError("reps must be in [1, 10000]");
        if (x_dev == y_dev) throw ArgError("x and y must not alias");
        if (precision != MTF_FP64 && precision != MTF_FP32_MIXED) throw ArgError("precision must be MTF_FP64 or MTF_FP32_MIXED");
        check_prec_available(p, precision);
        DeviceGuard g(p->device);
        hipStream_t s = p->stream;
        const double* x = static_cast<const double*>(x_dev);
        double* y = static_cast<double*>(y_dev);
        std::vector<hipEvent_t> ev(3 * (size_t)reps, nullptr);
        struct Cleanup {
            std::vector<hipEvent_t>& e;
            ~Cleanup() { for (auto v : e) if (v) (void)hipEventDestroy(v); }
        } cleanup{ev};
        for (auto& e : ev) HIPCHK(hipEventCreate(&e));
        for (int r = 0; r < reps; ++r) {
            HIPCHK(hipEventRecord(ev[3 * r], s));
            if (precision == MTF_FP64)
                launch_matvec_sym_f64(p->d_doms.p, p->d_symtiles.p, p->nsymtiles, p->T64.p, p->K64.p, x, p->part.p, s);
            else
                launch_matvec_sym_f32(p->d_doms.p, p->d_symtiles.p, p->nsymtiles, p->T32.p, p->K32.p, x, p->part.p, s);
            HIPCHK(hipEventRecord(ev[3 * r + 1], s));
            launch_matvec_sym_finish(p->d_doms.p, p->d_dof_dom.p, p->ndof, p->d_dplus.p, p->d_dminus.p, p->d_gval.p,
                                     p->d_gcol.p, p->d_near_ptr.p, p->d_near_col.p,
                                     precision == MTF_FP64 ? p->near64.p : p->near32.p, p->part.p, x, y, s);
            HIPCHK(hipEventRecord(ev[3 * r + 2], s));
        }
        HIPCHK(hipGetLastError());
        sync(p);
        double td = 0, tt = 0;
        for (int r = 0; r < reps; ++r) {
            float a = 0, b = 0;
            HIPCHK(hipEventElapsedTime(&a, ev[3 * r], ev[3 * r + 1]));
            HIPCHK(hipEventElapsedTime(&b, ev[3 * r], ev[3 * r + 2]));
            td += a;
            tt += b;
        }
        *dense_s = td * 1e-3 / reps;
        *total_s = tt * 1e-3 / reps;
        return MTF_OK;
    });
}

int mtf_solve(mtf_problem p, int32_t nrhs, const void* b_dev, void* x_dev, int64_t ld, const mtf_solve_opts* opts,
              mtf_solve_stats* stats) {
    return guarded([&] {
        if (!p) throw ArgError("problem is NULL");
        return solve_impl(p, nrhs, b_dev, x_dev, ld, opts, stats);
    });
}

int mtf_solve_stf(mtf_problem p, int32_t nrhs, const void* b_dev, void* x_dev, int64_t ld, const mtf_solve_opts* opts,
                  mtf_solve_stats* stats) {
    return guarded([&] {
        if (!p) throw ArgError("problem is NULL");
        return solve_stf_impl(p, nrhs, b_dev, x_dev, ld, opts, stats);
    });
}

int mtf_stf_matvec(mtf_problem p, int32_t nrhs, const void* x_dev, void* y_dev, int64_t ld) {
    return guarded([&] {
        if (!p) throw ArgError("problem is NULL");
        if (!p->has_mesh || !p->has_mat) throw StateError("mtf_stf_matvec before mesh/materials");
        if (!p->have64) throw StateError("mtf_stf_matvec needs the FP64 blocks");
        if (nrhs < 1 || !x_dev || !y_dev || x_dev == y_dev) throw ArgError("bad arguments");
        DeviceGuard g(p->device);
        stf_prepare(p);
        if (ld < 2 * (int64_t)p->sk.dom[0].E) throw ArgError("ld < 2 E_0");
        stf_matvec(p, static_cast<const double*>(x_dev), static_cast<double*>(y_dev), ld, nrhs);
        HIPCHK(hipGetLastError());
        return MTF_OK;
    });
}

int mtf_apply_preconditioner(mtf_problem p, int32_t preconditioner, int32_t nrhs, const void* x_dev, void* z_dev,
                             int64_t ld) {
    return guarded([&] {
        if (!p) throw ArgError("problem is NULL");
        if (!p->has_mesh || !p->has_mat) throw StateError("mtf_apply_preconditioner before mesh/materials");
        if (nrhs < 1 || !x_dev || !z_dev || ld < p->sk.N) throw ArgError("bad arguments");
        if (x_dev == z_dev) throw ArgError("x and z must not alias");
        const bool multi = (preconditioner & MTF_PREC_MULTI) != 0;
        preconditioner &= ~MTF_PREC_MULTI;
        if (preconditioner != MTF_PREC_BLOCK_TINV && preconditioner != MTF_PREC_BLOCK_TINV_GS)
            throw ArgError("preconditioner must be MTF_PREC_BLOCK_TINV or MTF_PREC_BLOCK_TINV_GS");
        if (multi && nrhs > kMaxBlock) throw ArgError("MTF_PREC_MULTI takes at most 32 vectors");
        if (!p->have64 && !p->have32) throw StateError("mtf_apply_preconditioner before mtf_assemble");
        DeviceGuard g(p->device);
        if (!p->have_tinv) build_tinv(p, pc_kind_of(0));
        if (multi) {
            DevBuf<double> w;
            if (preconditioner == MTF_PREC_BLOCK_TINV_GS) w.alloc((size_t)2 * ld * nrhs);
            precond_block(p, preconditioner, nrhs, static_cast<const double*>(x_dev), static_cast<double*>(z_dev), w.p,
                          ld);
            HIPCHK(hipGetLastError());
            sync(p);                                                 // w is released on return
            return MTF_OK;
        }
        DevBuf<double> w;
        if (preconditioner == MTF_PREC_BLOCK_TINV_GS) w.alloc(2 * p->sk.N);
        for (int r = 0; r < nrhs; ++r) {
            const double* x = static_cast<const double*>(x_dev) + 2 * ld * (int64_t)r;
            double* z = static_cast<double*>(z_dev) + 2 * ld * (int64_t)r;
            if (preconditioner == MTF_PREC_BLOCK_TINV_GS) precond1_gs(p, x, z, w.p);
            else precond1(p, x, z);
        }
        HIPCHK(hipGetLastError());
        if (preconditioner == MTF_PREC_BLOCK_TINV_GS) sync(p);      // w is released on return
        return MTF_OK;
    });
}

int mtf_far_field(mtf_problem p, int32_t nrhs, const void* x_dev, int64_t ld, int32_t ndir, const double* dir,
                  double* out) {
    return guarded([&] {
        if (!p) throw ArgError("problem is NULL");
        if (!p->has_mesh || !p->has_mat) throw StateError("mtf_far_field before mesh/materials");
        if (nrhs < 1 || ndir < 1 || !x_dev || !dir || !out || ld < p->sk.N) throw ArgError("bad arguments");
        if (!finite_all(dir, 3 * ndir)) throw ArgError("non-finite direction");
        DeviceGuard g(p->device);
        std::vector<double> host(dir, dir + 3 * ndir);
        DevBuf<double> dd, o;
        dd.upload(host, p->stream);
        o.alloc(6 * (size_t)nrhs * ndir);
        launch_far_field(&p->doms[0], p->d_geom.p, p->d_tdof.p, p->d_tsign.p, p->doms[0].T, p->k0, p->rho[0],
                         static_cast<const double*>(x_dev), ld, nrhs, dd.p, ndir, o.p, p->stream);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(out, o.p, o.n * sizeof(double), hipMemcpyDeviceToHost, p->stream));
        sync(p);
        return MTF_OK;
    });
}

int mtf_tile_variant(int32_t v, int32_t* tx, int32_t* ty, int32_t* occupancy) {
    return guarded([&] {
        if (v < 0 || v >= kTileVariants) throw ArgError("tile variant out of range");
        int a, b, c;
        tile_variant_shape(v, &a, &b, &c);
        if (tx) *tx = a;
        if (ty) *ty = b;
        if (occupancy) *occupancy = c;
        return MTF_OK;
    });
}

int mtf_assembly_variant(mtf_problem p, int32_t* variant) {
    return guarded([&] {
        if (!p || !variant) throw ArgError("bad arguments");
        *variant = p->last_variant;
        return MTF_OK;
    });
}

int mtf_tuning_log(char* buf, int64_t cap) {
    return guarded([&] {
        if (!buf || cap < 1) throw ArgError("bad arguments");
        std::string all;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            for (const auto& l : g_tune_log) all += l + "\n";
        }
        const size_t n = std::min<size_t>(all.size(), (size_t)cap - 1);
        std::memcpy(buf, all.data(), n);
        buf[n] = 0;
        return MTF_OK;
    });
}

int mtf_assembly_stats(mtf_problem p, int64_t* counts, double* seconds) {
    return guarded([&] {
        if (!p) throw ArgError("problem is NULL");
        if (!p->has_mesh) throw StateError("no mesh");
        if (counts)
            for (int k = 0; k < 4; ++k) counts[k] = p->sk.pair_counts[k];
        if (seconds) {
            *seconds = 0;
            if (p->ev0 && (p->have64 || p->have32)) {
                DeviceGuard g(p->device);
                HIPCHK(hipEventSynchronize(p->ev1));
                float ms = 0;
                HIPCHK(hipEventElapsedTime(&ms, p->ev0, p->ev1));
                *seconds = ms * 1e-3;
            }
        }
        return MTF_OK;
    });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batches of independent problems: one persistent assembly launch
// ---------------------------------------------------------------------------

struct mtf_batch_s {
    std::vector<mtf_problem> probs;
    int device = 0;
    hipStream_t stream = nullptr;
    DevBuf<BatchProb> d_probs;
    DevBuf<int4> d_items, d_sample;
    DevBuf<unsigned long long> counter;
    int64_t nitems = 0, nsample = 0;
    int items_variant = -1;           // tile variant of d_items
    int last_variant = 0, last_grid = 0;
    static constexpr int kLanes = 8;
    GmresWork gw[kLanes];             // GMRES workspaces, each lent to the solves of one lane in turn
    hipStream_t lane[kLanes] = {};    // solve lanes (default priority, non-blocking), created on first use
    hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
    double last_tiles_s = 0.0;        // device time of the last persistent launch alone
    double last_total_s = 0.0;        // and of the whole last assembly (touching pairs included)
    GjScratch gj;                     // work buffers of the preconditioner build, kept between builds
    // complex64 blocks of a lane, lent to each problem the lane solves on the mixed path (rounded
    // from its FP64 blocks for that solve only), so that no solve allocates or frees them
    struct LaneC64 {
        DevBuf<float> T32, K32;
        DevBuf<double> near32;
    } c64[kLanes];
    ~mtf_batch_s() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (e2) (void)hipEventDestroy(e2);
        for (hipStream_t& l : lane)
            if (l) (void)hipStreamDestroy(l);
    }
};

namespace {

// Separated-pair tiles of every problem for tile variant v, problems by decreasing size.
void batch_items(mtf_batch b, int v) {
    if (b->items_variant == v) return;
    int tx, ty, occ;
    tile_variant_shape(v, &tx, &ty, &occ);
    std::vector<int> order(b->probs.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return b->probs[x]->mat_entries > b->probs[y]->mat_entries; });
    const bool sym = tile_variant_sym(v);
    std::vector<int4> items;
    for (int pi : order) {
        const mtf_problem p = b->probs[pi];
        for (int i = 0; i <= p->sk.M; ++i) {
            const int T = p->sk.dom[i].T;
            for (int x0 = 0; x0 < T; x0 += tx)
                for (int y0 = sym ? x0 : 0; y0 < T; y0 += ty) items.push_back(make_int4(pi, i, x0, y0));
        }
    }
    b->d_items.upload(items, b->stream);
    b->nitems = (int64_t)items.size();
    // every eighth item: the sample the autotuner times its candidates on
    std::vector<int4> sample;
    for (size_t k = 0; k < items.size(); k += 8) sample.push_back(items[k]);
    b->d_sample.upload(sample, b->stream);
    b->nsample = (int64_t)sample.size();
    b->items_variant = v;
    HIPCHK(hipStreamSynchronize(b->stream));
}

// Device time of one persistent launch over the autotuner's sample of tiles (tile variant v,
// `grid` workgroups); it adds into the blocks, which the real assembly clears.
double batch_trial(mtf_batch b, int prec, int v, int grid) {
    hipStream_t s = b->stream;
    batch_items(b, v);
    HIPCHK(hipMemsetAsync(b->counter.p, 0, sizeof(unsigned long long), s));
    HIPCHK(hipEventRecord(b->e0, s));
    launch_assemble_persistent(prec == MTF_FP64 ? 0 : 1, v, b->d_sample.p, b->nsample, b->counter.p, b->d_probs.p, grid, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(b->e1, s));
    HIPCHK(hipEventSynchronize(b->e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, b->e0, b->e1));
    return ms * 1e-3;
}

// Problem descriptors of the batch for precision prec (blocks allocated and cleared).
void batch_prepare(mtf_batch b, int prec) {
    std::vector<BatchProb> bp(b->probs.size());
    for (size_t i = 0; i < b->probs.size(); ++i) {
        mtf_problem p = b->probs[i];
        assemble_prepare(p, prec);
        BatchProb& q = bp[i];
        q.doms = p->d_doms.p;
        q.geom = p->d_geom.p;
        q.verts = p->d_verts.p;
        q.tdof = p->d_tdof.p;
        q.tsign = p->d_tsign.p;
        q.sing = p->d_sing.p;
        q.T = prec == MTF_FP64 ? (void*)p->T64.p : (void*)p->T32.p;
        q.K = prec == MTF_FP64 ? (void*)p->K64.p : (void*)p->K32.p;
    }
    b->d_probs.upload(bp, b->stream);
}

// one persistent launch over every problem; returns the device time in seconds
double batch_launch(mtf_batch b, int prec, int v, int grid) {
    hipStream_t s = b->stream;
    batch_items(b, v);
    batch_prepare(b, prec);
    HIPCHK(hipMemsetAsync(b->counter.p, 0, sizeof(unsigned long long), s));
    HIPCHK(hipEventRecord(b->e0, s));
    launch_assemble_persistent(prec == MTF_FP64 ? 0 : 1, v, b->d_items.p, b->nitems, b->counter.p, b->d_probs.p, grid, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(b->e1, s));
    // touching pairs (Sauter-Schwab, FP64 in both precisions), one launch per problem
    for (mtf_problem p : b->probs) {
        const int32_t* meta = p->d_ss_meta.p;
        launch_singular(p->d_sing.p, (int64_t)p->d_sing.n, p->d_doms.p, p->d_geom.p, p->d_xyz.p, p->d_verts.p,
                        p->d_tdof.p, p->d_tsign.p, p->d_ss.p, meta, meta + 4, prec == MTF_FP64 ? p->T64.p : nullptr,
                        prec == MTF_FP64 ? p->K64.p : nullptr, prec == MTF_FP64 ? nullptr : p->T32.p,
                        prec == MTF_FP64 ? nullptr : p->K32.p, s);
    }
    HIPCHK(hipEventRecord(b->e2, s));
    for (mtf_problem p : b->probs) near_corrections(p, prec);    // same stream, after the blocks
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    float ms = 0, ms2 = 0;
    HIPCHK(hipEventElapsedTime(&ms, b->e0, b->e1));
    HIPCHK(hipEventElapsedTime(&ms2, b->e0, b->e2));
    b->last_tiles_s = ms * 1e-3;
    b->last_total_s = ms2 * 1e-3;
    return ms2 * 1e-3;
}

}  // namespace

extern "C" {

int mtf_batch_create(mtf_batch* out, int32_t n, const mtf_problem* problems) {
    return guarded([&] {
        if (!out || !problems || n < 1) throw ArgError("bad arguments");
        *out = nullptr;
        auto b = std::make_unique<mtf_batch_s>();
        for (int i = 0; i < n; ++i) {
            mtf_problem p = problems[i];
            if (!p) throw ArgError("NULL problem in batch");
            if (!p->has_mesh || !p->has_mat) throw StateError("every problem of a batch needs mesh and materials");
            if (i > 0 && (p->device != problems[0]->device || p->stream != problems[0]->stream))
                throw ArgError("problems of a batch must share device and stream");
            for (int k = 0; k < i; ++k)
                if (problems[k] == p) throw ArgError("a problem appears twice in the batch");
            b->probs.push_back(p);
        }
        if (n >= (1 << 24)) throw ArgError("too many problems");
        b->device = problems[0]->device;
        b->stream = problems[0]->stream;
        DeviceGuard g(b->device);
        b->counter.alloc(1);
        HIPCHK(hipEventCreate(&b->e0));
        HIPCHK(hipEventCreate(&b->e1));
        HIPCHK(hipEventCreate(&b->e2));
        sync(problems[0]);
        *out = b.release();
        return MTF_OK;
    });
}

int mtf_batch_destroy(mtf_batch b) {
    if (!b) return MTF_OK;
    return guarded([&] {
        DeviceGuard g(b->device);
        (void)hipStreamSynchronize(b->stream);
        delete b;
        return MTF_OK;
    });
}

int mtf_batch_assemble(mtf_batch b, const mtf_assembly_opts* opts, int32_t* grid_used, double* seconds) {
    return guarded([&] {
        if (!b) throw ArgError("batch is NULL");
        int prec, order, forced;
        parse_assembly_opts(opts, &prec, &order, nullptr, &forced);
        DeviceGuard g(b->device);
        for (mtf_problem p : b->probs) {
            if (!p->has_mesh || !p->has_mat) throw StateError("problem lost its mesh or materials");
            ensure_ss(p, order);
        }
        hipDeviceProp_t prop;
        HIPCHK(hipGetDeviceProperties(&prop, b->device));
        const int cus = prop.multiProcessorCount;
        int v = forced, per = 0;
        if (v < 0) {
            double tri = 0, doms = 0;
            for (mtf_problem p : b->probs) {
                doms += p->sk.M + 1;
                for (int i = 0; i <= p->sk.M; ++i) tri += p->sk.dom[i].T;
            }
            const std::string key = tune_key(b->device, "persistent", prec, shape_class(tri / doms));
            TuneChoice c;
            if (tune_lookup(key, &c)) {
                v = c.variant;
                per = c.per_cu;
            } else {
                // autotuner: every tile variant at 4 workgroups per CU, then 1, 2, 4 and 8 workgroups
                // per CU for the fastest, each a persistent launch over every eighth tile
                batch_prepare(b, prec);
                TuneChoice best;
                best.seconds = 1e300;
                auto trial = [&](int tv, int tper) {
                    const double t = batch_trial(b, prec, tv, cus * tper);
                    {
                        std::lock_guard<std::mutex> lk(g_tune_mu);
                        g_tune_log.push_back(key + " variant " + std::to_string(tv) + " per_cu " + std::to_string(tper) +
                                             " " + std::to_string(t) + " s");
                    }
                    if (t < best.seconds) { best.seconds = t; best.variant = tv; best.per_cu = tper; }
                };
                for (int tv = 0; tv < kTileVariants; ++tv) trial(tv, 4);
                const int bv = best.variant;
                for (int tper : {1, 2, 8}) trial(bv, tper);
                tune_store(key, best);
                v = best.variant;
                per = best.per_cu;
            }
        }
        if (per == 0) per = 4;
        const double t = batch_launch(b, prec, v, cus * per);
        b->last_variant = v;
        b->last_grid = cus * per;
        if (grid_used) *grid_used = cus * per;
        if (seconds) *seconds = t;
        return MTF_OK;
    });
}

int mtf_batch_assembly_stats(mtf_batch b, int64_t* counts, double* seconds, int32_t* config) {
    return guarded([&] {
        if (!b) throw ArgError("batch is NULL");
        if (counts) {
            for (int c = 0; c < 4; ++c) counts[c] = 0;
            for (mtf_problem p : b->probs) {
                int64_t pc[4];
                const int r = mtf_assembly_stats(p, pc, nullptr);
                if (r < 0) throw StateError(g_err);
                for (int c = 0; c < 4; ++c) counts[c] += pc[c];
            }
        }
        if (seconds) {
            seconds[0] = b->last_tiles_s;
            seconds[1] = b->last_total_s - b->last_tiles_s;
        }
        if (config) {
            config[0] = b->last_variant;
            config[1] = b->last_grid;
        }
        return MTF_OK;
    });
}

int mtf_batch_build_preconditioner(mtf_batch b, int32_t flags) {
    return guarded([&] {
        if (!b) throw ArgError("batch is NULL");
        if (flags & ~(MTF_SOLVE_PC_FULL | MTF_SOLVE_PC_DIRECT))
            throw ArgError("flags: only MTF_SOLVE_PC_FULL or MTF_SOLVE_PC_DIRECT are accepted");
        const int kind = pc_kind_of(flags);
        DeviceGuard g(b->device);
        for (mtf_problem p : b->probs) {
            if (!p->has_mesh || !p->has_mat) throw StateError("problem lost its mesh or materials");
            if (!p->have32 && !p->have64) throw StateError("mtf_batch_build_preconditioner: assemble the batch first");
        }
        batch_build_tinv(b->probs, kind, b->stream, &b->gj);
        return MTF_OK;
    });
}

int mtf_batch_solve(mtf_batch b, const void* const* b_dev, void* const* x_dev, const mtf_solve_opts* opts,
                    mtf_solve_stats* stats) {
    return guarded([&] {
        if (!b || !b_dev || !x_dev) throw ArgError("bad arguments");
        const size_t np = b->probs.size();
        for (size_t i = 0; i < np; ++i)
            if (!b_dev[i] || !x_dev[i]) throw ArgError("NULL right-hand side or solution");
        // max_iters 0: cycles of at most kBatchCycle steps.  The Krylov storage of a cycle is
        // allocated per problem; sized from free memory it would be gigabytes per problem for
        // solves that take tens of steps, and allocating it would dominate the batch.
        mtf_solve_opts o{};
        o.struct_size = sizeof(o);
        o.rtol = 1e-6;
        if (opts) {
            if (opts->struct_size < (int)sizeof(mtf_solve_opts)) throw ArgError("mtf_solve_opts.struct_size too small");
            o = *opts;
        }
        if (o.max_iters == 0) o.max_iters = kBatchCycle;
        const int pc_kind = pc_kind_of(o.flags);
        DeviceGuard g(b->device);
        // what each problem held before the call; whatever the call creates beyond that is released
        // when the problem's solve ends, also when it ends with an error
        std::vector<char> tmpinv(np), tmpwork(np);
        for (size_t i = 0; i < np; ++i) {
            mtf_problem p = b->probs[i];
            if (!p->has_mesh || !p->has_mat) throw StateError("problem lost its mesh or materials");
            tmpinv[i] = !p->have_tinv;
            tmpwork[i] = p->gw.V.n == 0;
        }
        struct Release {
            mtf_problem p;
            bool tmp64 = false, tmpinv = false, tmpwork = false, tmp32 = false;
            mtf_batch_s::LaneC64* lend32 = nullptr;   // the complex64 blocks are the lane's: give them back
            ~Release() {
                if (!p) return;
                (void)hipStreamSynchronize(p->stream);
                if (tmp64) { p->T64.reset(); p->K64.reset(); p->near64.reset(); p->have64 = false; }
                if (tmp32) {
                    if (lend32) {
                        swap_buf(p->T32, lend32->T32);
                        swap_buf(p->K32, lend32->K32);
                        swap_buf(p->near32, lend32->near32);
                    } else {
                        p->T32.reset(); p->K32.reset(); p->near32.reset();
                    }
                    p->have32 = false;
                    p->gm.haveA = false;
                }
                if (tmpinv) { p->Tinv.reset(); p->have_tinv = false; p->gp.haveA = false; }
                if (tmpwork) p->gw.release();
            }
        };
        // the preconditioner blocks of every problem that lacks them, built together
        double t_pc = 0.0;
        if (o.preconditioner != MTF_PREC_NONE) {
            std::vector<mtf_problem> need;
            for (size_t i = 0; i < np; ++i) {
                mtf_problem p = b->probs[i];
                if (!p->have32 && !p->have64) throw StateError("mtf_batch_solve: assemble the batch first");
                if (!p->have_tinv || p->pc_kind != pc_kind) need.push_back(p);
            }
            if (!need.empty()) {
                try {
                    t_pc = batch_build_tinv(need, pc_kind, b->stream, &b->gj);
                } catch (...) {
                    for (size_t i = 0; i < np; ++i)
                        if (tmpinv[i]) { b->probs[i]->Tinv.reset(); b->probs[i]->have_tinv = false; }
                    throw;
                }
            }
        }
        // The problems are solved on `lanes` streams at once, each lane a host thread taking the next
        // problem (largest first) with a workspace of its own: the GMRES steps of small problems are
        // latency-bound, and independent problems overlap.  MTF_BATCH_LANES sets the count (1-8,
        // default 4; 1 solves one after another on the problems' own streams).
        int lanes = 4;
        if (const char* e = std::getenv("MTF_BATCH_LANES")) lanes = std::atoi(e);
        lanes = std::max(1, std::min<int>(lanes, std::min<size_t>(mtf_batch_s::kLanes, np)));
        std::vector<size_t> order(np);
        for (size_t i = 0; i < np; ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return b->probs[x]->sk.N > b->probs[y]->sk.N; });
        std::vector<char> done(np, 0);
        std::atomic<size_t> counter{0};
        std::atomic<bool> abort{false};
        std::mutex mu;
        std::exception_ptr err;
        int status = MTF_OK;
        auto solve_one = [&](size_t i, GmresWork& lw, mtf_batch_s::LaneC64& lc) {
            mtf_problem p = b->probs[i];
            Release rel{p, !p->have64, (bool)tmpinv[i], false};
            // a problem without a workspace of its own borrows the lane's (allocated once, for the
            // largest problem the lane met), so the Krylov buffers are not allocated per problem
            struct Lend {
                GmresWork& a;
                GmresWork& b;
                bool on;
                ~Lend() {
                    if (on) swap_work(a, b);
                }
            } lend{p->gw, lw, (bool)tmpwork[i]};
            if (lend.on) swap_work(p->gw, lw);
            if (rel.tmp64) {
                mtf_assembly_opts ao{};
                ao.struct_size = sizeof(ao);
                ao.precision = MTF_FP64;
                ao.singular_order = 4;
                ao.flags = MTF_ASSEMBLE_TILE(b->last_variant);   // the batch's tuned tiles, no new trials
                assemble_impl(p, &ao);       // the preconditioner stays: it was built from the FP32 blocks
            }
            if (o.precision == MTF_FP32_MIXED && !p->have32) {
                // complex64 blocks rounded from the FP64 ones for this solve only (no second quadrature)
                mtf_assembly_opts ao{};
                ao.struct_size = sizeof(ao);
                ao.precision = MTF_FP32_MIXED;
                ao.singular_order = 4;
                ao.flags = MTF_ASSEMBLE_ROUND_FP64;
                swap_buf(p->T32, lc.T32);    // the lane's buffers, grown to the largest problem it met
                swap_buf(p->K32, lc.K32);
                swap_buf(p->near32, lc.near32);
                rel.lend32 = &lc;
                rel.tmp32 = true;
                assemble_impl(p, &ao);       // the preconditioner stays: it was built from the FP64 blocks
            }
            const int r = solve_impl(p, 1, b_dev[i], x_dev[i], p->sk.N, &o, stats ? stats + i : nullptr);
            if (stats) stats[i].t_precond_s = i == 0 ? t_pc : 0.0;
            return r;
        };
        if (lanes == 1) {
            for (size_t k = 0; k < np; ++k) {
                const size_t i = order[k];
                try {
                    const int r = solve_one(i, b->gw[0], b->c64[0]);
                    if (r != MTF_OK) status = r;
                    done[i] = 1;
                } catch (...) {
                    for (size_t j = 0; j < np; ++j)
                        if (!done[j] && j != i && tmpinv[j]) { b->probs[j]->Tinv.reset(); b->probs[j]->have_tinv = false; b->probs[j]->gp.haveA = false; }
                    throw;
                }
            }
            return status;
        }
        for (int l = 0; l < lanes; ++l)
            if (!b->lane[l]) HIPCHK(hipStreamCreateWithFlags(&b->lane[l], hipStreamNonBlocking));
        HIPCHK(hipDeviceSynchronize());          // inputs and preconditioner blocks complete
        auto lane_fn = [&](int l) {
            try {
                DeviceGuard dg(b->device);
                for (;;) {
                    if (abort.load()) return;
                    const size_t k = counter.fetch_add(1);
                    if (k >= np) return;
                    const size_t i = order[k];
                    mtf_problem p = b->probs[i];
                    struct OnLane {
                        mtf_problem p;
                        hipStream_t own;
                        ~OnLane() {
                            (void)hipStreamSynchronize(p->stream);
                            p->stream = own;
                        }
                    } on{p, p->stream};
                    p->stream = b->lane[l];
                    struct SyncSteps {
                        mtf_problem p;
                        ~SyncSteps() { p->gmres_sync = kSync; }
                    } sync_steps{p};
                    p->gmres_sync = kSyncLanes;
                    const int r = solve_one(i, b->gw[l], b->c64[l]);
                    std::lock_guard<std::mutex> lk(mu);
                    if (r != MTF_OK) status = r;
                    done[i] = 1;
                }
            } catch (...) {
                std::lock_guard<std::mutex> lk(mu);
                if (!err) err = std::current_exception();
                abort = true;
            }
        };
        std::vector<std::thread> th;
        for (int l = 0; l < lanes; ++l) th.emplace_back(lane_fn, l);
        for (std::thread& t : th) t.join();
        if (err) {
            // problems not solved: release the preconditioner blocks built above
            for (size_t j = 0; j < np; ++j)
                if (!done[j] && tmpinv[j]) { b->probs[j]->Tinv.reset(); b->probs[j]->have_tinv = false; b->probs[j]->gp.haveA = false; }
            std::rethrow_exception(err);
        }
        return status;
    });
}

}  // extern "C"
