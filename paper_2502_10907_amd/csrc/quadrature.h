// Quadrature tables built on the host and uploaded once.
#pragma once

#include <vector>

namespace mtf {

// Symmetric degree-4 rule on a triangle, 6 points (Dunavant 1985):
// barycentric coordinates [6][3] and weights [6] summing to one.
void triangle_rule6(double bary[6][3], double w[6]);

// n-point Gauss-Legendre rule on [0, 1] (Newton iteration on P_n).
void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w);

// Sauter-Schwab relative-coordinate rule on T x T, T = {0 <= t <= s <= 1}, mapped to a
// physical triangle by chi(s, t) = P0 + s (P1 - P0) + t (P2 - P1) (Sauter & Schwab,
// Boundary Element Methods, Section 5.2).  kind: 3 coincident (6 regions), 2 edge-adjacent
// with the shared edge P0P1 (5 regions), 1 vertex-adjacent with the shared vertex P0
// (2 regions); n Gauss-Legendre points per coordinate of [0,1]^4.
// Appends points as (s_x, t_x, s_y, t_y, weight) to `out`; weights integrate over T x T.
void sauter_schwab_rule(int kind, int n, std::vector<double>& out);

}  // namespace mtf
