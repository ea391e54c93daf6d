#include "quadrature.h"

#include <cmath>
#include <stdexcept>

namespace mtf {

void triangle_rule6(double bary[6][3], double w[6]) {
    // Two orbits of (a, a, 1-2a); published constants of the degree-4 rule.
    const double a[2] = {0.445948490915965, 0.091576213509771};
    const double wt[2] = {0.223381589678011, 0.109951743655322};
    int q = 0;
    for (int o = 0; o < 2; ++o) {
        double b = 1.0 - 2.0 * a[o];
        double pts[3][3] = {{a[o], a[o], b}, {a[o], b, a[o]}, {b, a[o], a[o]}};
        for (int p = 0; p < 3; ++p, ++q) {
            for (int k = 0; k < 3; ++k) bary[q][k] = pts[p][k];
            w[q] = wt[o];
        }
    }
}

void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w) {
    if (n < 1 || n > 64) throw std::invalid_argument("Gauss-Legendre order out of range");
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        double z = std::cos(pi * (i + 0.75) / (n + 0.5));   // Tricomi initial guess
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;                         // three-term recurrence for P_n(z)
            for (int k = 2; k <= n; ++k) {
                double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            double pn = (n == 1) ? z : p1;
            double pnm1 = (n == 1) ? 1.0 : p0;
            dp = n * (z * pn - pnm1) / (z * z - 1.0);
            double dz = pn / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        // recompute derivative at the converged node
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = pk;
        }
        double pn = (n == 1) ? z : p1;
        double pnm1 = (n == 1) ? 1.0 : p0;
        dp = n * (z * pn - pnm1) / (z * z - 1.0);
        x[i] = 0.5 * (1.0 - z);
        w[i] = 1.0 / ((1.0 - z * z) * dp * dp);              // (2/((1-z^2)P'^2)) / 2
    }
}

void sauter_schwab_rule(int kind, int n, std::vector<double>& out) {
    std::vector<double> g, gw;
    gauss_legendre01(n, g, gw);
    auto emit = [&](double xs, double xt, double ys, double yt, double wgt) {
        out.push_back(xs); out.push_back(xt); out.push_back(ys); out.push_back(yt); out.push_back(wgt);
    };
    for (int i0 = 0; i0 < n; ++i0)
    for (int i1 = 0; i1 < n; ++i1)
    for (int i2 = 0; i2 < n; ++i2)
    for (int i3 = 0; i3 < n; ++i3) {
        const double xi = g[i0], a = g[i1], b = g[i2], c = g[i3];
        const double w = gw[i0] * gw[i1] * gw[i2] * gw[i3];
        if (kind == 3) {
            // identical panels: six regions, Jacobian xi^3 a^2 b
            const double J = w * xi * xi * xi * a * a * b;
            emit(xi, xi * (1 - a + a * b), xi * (1 - a * b * c), xi * (1 - a), J);
            emit(xi * (1 - a * b * c), xi * (1 - a), xi, xi * (1 - a + a * b), J);
            emit(xi, xi * a * (1 - b + b * c), xi * (1 - a * b), xi * a * (1 - b), J);
            emit(xi * (1 - a * b), xi * a * (1 - b), xi, xi * a * (1 - b + b * c), J);
            emit(xi * (1 - a * b * c), xi * a * (1 - b * c), xi, xi * a * (1 - b), J);
            emit(xi, xi * a * (1 - b), xi * (1 - a * b * c), xi * a * (1 - b * c), J);
        } else if (kind == 2) {
            // common edge: five regions
            const double J1 = w * xi * xi * xi * a * a;
            const double J = J1 * b;
            emit(xi, xi * a * c, xi * (1 - a * b), xi * a * (1 - b), J1);
            emit(xi, xi * a, xi * (1 - a * b * c), xi * a * b * (1 - c), J);
            emit(xi * (1 - a * b), xi * a * (1 - b), xi, xi * a * b * c, J);
            emit(xi * (1 - a * b * c), xi * a * b * (1 - c), xi, xi * a, J);
            emit(xi * (1 - a * b * c), xi * a * (1 - b * c), xi, xi * a * b, J);
        } else if (kind == 1) {
            // common vertex: two regions, Jacobian xi^3 b
            const double J = w * xi * xi * xi * b;
            emit(xi, xi * a, xi * b, xi * b * c, J);
            emit(xi * b, xi * b * c, xi, xi * a, J);
        } else {
            throw std::invalid_argument("Sauter-Schwab kind must be 1, 2 or 3");
        }
    }
}

}  // namespace mtf
