// Skeleton bookkeeping (Section 4.2): Algorithm 1, RWG_i tables, pair classes.
#include "skeleton.h"

#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <unordered_map>

namespace mtf {

namespace {

inline uint64_t edge_key(int32_t a, int32_t b) {
    uint32_t lo = (uint32_t)std::min(a, b), hi = (uint32_t)std::max(a, b);
    return ((uint64_t)lo << 32) | hi;
}

}  // namespace

Skeleton build_skeleton(int64_t nv, const double* xyz, int64_t nt, const int32_t* tri,
                        const int32_t* label, int32_t M) {
    if (nv < 3 || nt < 1 || M < 1) throw ArgError("mesh needs nv >= 3, nt >= 1, M >= 1");
    if (nv > INT32_MAX || nt > INT32_MAX) throw ArgError("mesh too large for 32-bit ids");
    if (!xyz || !tri || !label) throw ArgError("null mesh array");
    Skeleton sk;
    sk.M = M;
    sk.nv = nv;
    sk.nt = nt;
    sk.xyz.assign(xyz, xyz + 3 * nv);
    for (int64_t v = 0; v < 3 * nv; ++v)
        if (!std::isfinite(xyz[v])) throw ArgError("non-finite vertex coordinate");

    // Per-triangle validation.
    for (int64_t t = 0; t < nt; ++t) {
        const int32_t* v = tri + 3 * t;
        const int32_t* l = label + 2 * t;
        for (int a = 0; a < 3; ++a)
            if (v[a] < 0 || v[a] >= nv) throw MeshError("triangle " + std::to_string(t) + ": vertex id out of range");
        if (v[0] == v[1] || v[1] == v[2] || v[0] == v[2])
            throw MeshError("triangle " + std::to_string(t) + ": repeated vertex");
        if (l[0] < 0 || l[0] > M || l[1] < 0 || l[1] > M || l[0] == l[1])
            throw MeshError("triangle " + std::to_string(t) + ": labels must be distinct and in [0, M]");
        const double* p0 = xyz + 3 * v[0];
        const double* p1 = xyz + 3 * v[1];
        const double* p2 = xyz + 3 * v[2];
        double e1[3], e2[3];
        for (int k = 0; k < 3; ++k) { e1[k] = p1[k] - p0[k]; e2[k] = p2[k] - p0[k]; }
        double cx = e1[1] * e2[2] - e1[2] * e2[1];
        double cy = e1[2] * e2[0] - e1[0] * e2[2];
        double cz = e1[0] * e2[1] - e1[1] * e2[0];
        double a2 = std::sqrt(cx * cx + cy * cy + cz * cz);
        double l2 = std::max({e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2], e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]});
        if (!(a2 > 1e-12 * l2)) throw MeshError("triangle " + std::to_string(t) + ": degenerate (zero area)");
    }

    // Algorithm 1: for every subdomain i and every j in Lambda_i, append the triangles of
    // Gamma_ij with multiplier swap = +1 when the mesh normal is the exterior normal n_i
    // (i == label[0]; with the min->max convention this is sign(j - i)), else -1.
    sk.dom.resize(M + 1);
    std::vector<std::vector<int32_t>> tris_of(M + 1);
    for (int64_t t = 0; t < nt; ++t) {
        tris_of[label[2 * t]].push_back((int32_t)t);
        tris_of[label[2 * t + 1]].push_back((int32_t)t);
    }
    // Each Gamma_i's triangles are put in an order in which TX consecutive ones form a compact
    // patch, so that an assembly tile shares dofs between its triangles and scatters fewer
    // distinct entries.  Default: by their vertex ids (smallest, middle, largest), the order the
    // RWG dofs follow (edges are numbered by their vertex ids), so a tile's test dofs also lie close
    // together and the atomics of its scatter share cache lines.  MTF_TRIANGLE_ORDER=morton orders
    // them along a Morton (Z-order) curve through their centroids instead (compact patches whatever
    // the vertex numbering), =input keeps the input order.  Only summation order depends on it.
    const char* ord = std::getenv("MTF_TRIANGLE_ORDER");
    const std::string order = ord ? std::string(ord) : std::string("vertex");
    if (order != "vertex" && order != "morton" && order != "input")
        throw ArgError("MTF_TRIANGLE_ORDER must be vertex, morton or input");
    if (order == "vertex") {
        auto sorted3 = [&](int32_t t, int32_t* v) {
            for (int a = 0; a < 3; ++a) v[a] = tri[3 * t + a];
            std::sort(v, v + 3);
        };
        for (auto& l : tris_of)
            std::stable_sort(l.begin(), l.end(), [&](int32_t x, int32_t y) {
                int32_t a[3], b[3];
                sorted3(x, a);
                sorted3(y, b);
                return std::lexicographical_compare(a, a + 3, b, b + 3);
            });
    } else if (order == "morton") {
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int64_t v = 0; v < nv; ++v)
            for (int k = 0; k < 3; ++k) {
                lo[k] = std::min(lo[k], xyz[3 * v + k]);
                hi[k] = std::max(hi[k], xyz[3 * v + k]);
            }
        auto spread = [](uint64_t x) {          // 20 bits -> every third bit of 60
            x &= 0xFFFFFull;
            x = (x | (x << 32)) & 0x1F00000000FFFFull;
            x = (x | (x << 16)) & 0x1F0000FF0000FFull;
            x = (x | (x << 8)) & 0x100F00F00F00F00Full;
            x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
            x = (x | (x << 2)) & 0x1249249249249249ull;
            return x;
        };
        std::vector<uint64_t> key(nt);
        for (int64_t t = 0; t < nt; ++t) {
            uint64_t k = 0;
            for (int a = 0; a < 3; ++a) {
                double c = 0.0;
                for (int q = 0; q < 3; ++q) c += xyz[3 * tri[3 * t + q] + a];
                c /= 3.0;
                const double span = hi[a] - lo[a];
                const double f = span > 0 ? (c - lo[a]) / span : 0.0;
                const uint64_t qv = (uint64_t)std::min(1048575.0, std::max(0.0, f * 1048575.0));
                k |= spread(qv) << a;
            }
            key[t] = k;
        }
        for (auto& l : tris_of)
            std::stable_sort(l.begin(), l.end(), [&](int32_t x, int32_t y) { return key[x] < key[y]; });
    }
    // position of each skeleton triangle in the two domains it belongs to
    std::vector<int32_t> pos_lo(nt), pos_hi(nt);
    for (int i = 0; i <= M; ++i) {
        Domain& d = sk.dom[i];
        d.id = i;
        d.T = (int)tris_of[i].size();
        if (d.T == 0) throw MeshError("subdomain " + std::to_string(i) + " has no boundary triangle");
        d.tri = tris_of[i];
        d.verts.resize(3 * d.T);
        d.other.resize(d.T);
        for (int lt = 0; lt < d.T; ++lt) {
            int32_t t = d.tri[lt];
            const int32_t* v = tri + 3 * t;
            bool exterior = label[2 * t] == i;     // swap = +1
            d.verts[3 * lt + 0] = v[0];
            d.verts[3 * lt + 1] = exterior ? v[1] : v[2];
            d.verts[3 * lt + 2] = exterior ? v[2] : v[1];
            d.other[lt] = exterior ? label[2 * t + 1] : label[2 * t];
            (exterior ? pos_lo : pos_hi)[t] = lt;
        }
    }
    for (int i = 0; i <= M; ++i) {
        Domain& d = sk.dom[i];
        d.other_lt.resize(d.T);
        for (int lt = 0; lt < d.T; ++lt) {
            int32_t t = d.tri[lt];
            bool exterior = label[2 * t] == i;
            d.other_lt[lt] = exterior ? pos_hi[t] : pos_lo[t];
        }
    }

    // RWG_i: one dof per Gamma_i edge; tau+ traverses the edge (a < b) from a to b.
    for (int i = 0; i <= M; ++i) {
        Domain& d = sk.dom[i];
        struct Occ { int32_t lt, a; bool fwd; int n; int32_t lt2, a2; bool fwd2; };
        std::unordered_map<uint64_t, Occ> occ;
        occ.reserve(3 * d.T);
        for (int lt = 0; lt < d.T; ++lt) {
            for (int a = 0; a < 3; ++a) {
                int32_t u = d.verts[3 * lt + (a + 1) % 3], w = d.verts[3 * lt + (a + 2) % 3];
                uint64_t key = edge_key(u, w);
                auto it = occ.find(key);
                if (it == occ.end()) {
                    occ.emplace(key, Occ{lt, a, u < w, 1, -1, -1, false});
                } else {
                    Occ& o = it->second;
                    if (o.n >= 2)
                        throw MeshError("Gamma_" + std::to_string(i) + ": an edge is shared by more than two of its triangles");
                    o.lt2 = lt; o.a2 = a; o.fwd2 = u < w; o.n = 2;
                }
            }
        }
        std::vector<uint64_t> keys;
        keys.reserve(occ.size());
        for (auto& kv : occ) keys.push_back(kv.first);
        std::sort(keys.begin(), keys.end());
        d.E = (int)keys.size();
        d.edge_vtx.resize(2 * d.E);
        d.plus.resize(2 * d.E);
        d.minus.resize(2 * d.E);
        d.tri_dof.assign(3 * d.T, -1);
        d.tri_sign.assign(3 * d.T, 0);
        for (int m = 0; m < d.E; ++m) {
            const Occ& o = occ[keys[m]];
            if (o.n != 2 || o.fwd == o.fwd2)
                throw MeshError("Gamma_" + std::to_string(i) + " is not a closed, consistently oriented surface");
            d.edge_vtx[2 * m] = (int32_t)(keys[m] >> 32);
            d.edge_vtx[2 * m + 1] = (int32_t)(keys[m] & 0xffffffffu);
            int32_t ltp = o.fwd ? o.lt : o.lt2, ap = o.fwd ? o.a : o.a2;
            int32_t ltm = o.fwd ? o.lt2 : o.lt, am = o.fwd ? o.a2 : o.a;
            d.plus[2 * m] = ltp; d.plus[2 * m + 1] = ap;
            d.minus[2 * m] = ltm; d.minus[2 * m + 1] = am;
            d.tri_dof[3 * ltp + ap] = m; d.tri_sign[3 * ltp + ap] = 1;
            d.tri_dof[3 * ltm + am] = m; d.tri_sign[3 * ltm + am] = -1;
        }
    }

    // Touching pairs of every Gamma_i by shared global vertex ids (the mesh is conforming).
    for (int i = 0; i <= M; ++i) {
        Domain& d = sk.dom[i];
        std::unordered_map<int32_t, std::vector<int32_t>> v2t;
        for (int lt = 0; lt < d.T; ++lt)
            for (int a = 0; a < 3; ++a) v2t[d.verts[3 * lt + a]].push_back(lt);
        std::vector<int32_t> nb;
        int64_t touching = 0;
        for (int lt = 0; lt < d.T; ++lt) {
            nb.clear();
            for (int a = 0; a < 3; ++a)
                for (int32_t o : v2t[d.verts[3 * lt + a]]) nb.push_back(o);
            std::sort(nb.begin(), nb.end());
            nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
            for (int32_t ly : nb) {
                SingularPair sp;
                sp.domain = i; sp.tx = lt; sp.ty = ly;
                const int32_t* vx = &d.verts[3 * lt];
                const int32_t* vy = &d.verts[3 * ly];
                int nsh = 0;
                int8_t ox[3], oy[3];
                bool usedx[3] = {false, false, false}, usedy[3] = {false, false, false};
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b)
                        if (vx[a] == vy[b]) { ox[nsh] = (int8_t)a; oy[nsh] = (int8_t)b; usedx[a] = usedy[b] = true; ++nsh; }
                if (nsh == 3) {
                    for (int a = 0; a < 3; ++a) { ox[a] = (int8_t)a; }
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b)
                            if (vy[b] == vx[a]) oy[a] = (int8_t)b;
                } else {
                    int kx = nsh, ky = nsh;
                    for (int a = 0; a < 3; ++a) if (!usedx[a]) ox[kx++] = (int8_t)a;
                    for (int b = 0; b < 3; ++b) if (!usedy[b]) oy[ky++] = (int8_t)b;
                }
                for (int a = 0; a < 3; ++a) { sp.px[a] = ox[a]; sp.py[a] = oy[a]; }
                sp.kind = nsh;
                sk.singular.push_back(sp);
                sk.pair_counts[nsh] += 1;
                ++touching;
            }
        }
        sk.pair_counts[0] += (int64_t)d.T * d.T - touching;
    }

    sk.offset.resize(M + 2);
    sk.offset[0] = 0;
    for (int i = 0; i <= M; ++i) sk.offset[i + 1] = sk.offset[i] + 2 * (int64_t)sk.dom[i].E;
    sk.N = sk.offset[M + 1];
    return sk;
}

}  // namespace mtf
