// Host-side skeleton bookkeeping: Algorithm 1 (normal swaps per subdomain),
// RWG_i dof tables and triangle-pair classes (Section 4.2 of the paper).
// Integer work only; runs once per mesh.
#pragma once

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace mtf {

struct MeshError : std::runtime_error {
    explicit MeshError(const std::string& s) : std::runtime_error(s) {}
};
struct ArgError : std::runtime_error {
    explicit ArgError(const std::string& s) : std::runtime_error(s) {}
};

// Gamma_i with its RWG_i space.
struct Domain {
    int id = 0;
    int T = 0;                       // triangles of Gamma_i
    int E = 0;                       // dim RWG_i
    std::vector<int32_t> tri;        // [T]   skeleton triangle id
    std::vector<int32_t> verts;      // [T*3] vertex ids in Gamma_i orientation (n_i = right-hand normal)
    std::vector<int32_t> other;      // [T]   the other subdomain j of the triangle (Gamma_ij)
    std::vector<int32_t> other_lt;   // [T]   local index of the same triangle in Gamma_j
    std::vector<int32_t> edge_vtx;   // [E*2] edge vertex ids (a < b)
    std::vector<int32_t> plus;       // [E*2] (local triangle, local vertex opposite the edge) of tau+
    std::vector<int32_t> minus;      // [E*2] same for tau-
    std::vector<int32_t> tri_dof;    // [T*3] dof of the edge opposite local vertex a
    std::vector<int8_t>  tri_sign;   // [T*3] +1 on tau+, -1 on tau-
};

// A pair of touching triangles of one Gamma_i (ordered: x test, y trial).
struct SingularPair {
    int32_t domain;
    int32_t tx, ty;                  // local triangle ids
    int32_t kind;                    // 3 coincident, 2 edge, 1 vertex (shared vertex count)
    int8_t  px[3], py[3];            // local vertex order of each parametrisation: shared vertices
                                     // first, in the same order on both triangles
};

struct Skeleton {
    int M = 0;
    int64_t nv = 0, nt = 0;
    std::vector<double> xyz;         // [nv*3]
    std::vector<Domain> dom;         // [M+1]
    std::vector<SingularPair> singular;
    int64_t pair_counts[4] = {0, 0, 0, 0};   // ordered pairs by shared-vertex count (0 = separated)
    int64_t N = 0;                   // 2 sum E_i
    std::vector<int64_t> offset;     // [M+2] start of block i in the unknown vector
};

// Validates the mesh and builds every table; throws MeshError / ArgError.
Skeleton build_skeleton(int64_t nv, const double* xyz, int64_t nt, const int32_t* tri,
                        const int32_t* label, int32_t M);

}  // namespace mtf
