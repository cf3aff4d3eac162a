// Compile-time 1D reference-element data of degree K on [0,1] (Sec. 5 set-up):
// Gauss-Lobatto-Legendre nodes, the (K+1)-point Gauss rule, the element mass
// and stiffness matrices  M[a][b] = int l_a l_b,  A[a][b] = int l_a' l_b'
// (exact with K+1 Gauss points), and the prolongation from one cell to its two
// halves  P[f][c] = l_c(x_f)  with fine nodes x/2 and 1/2 + x/2.  For the
// cell-based (deformed-mesh) operator also the basis values at the Gauss
// points  gB[q][a] = l_a(g_q)  and the collocation derivative on the Gauss
// points  gD[q][p] = L_p'(g_q)  (L_p the Lagrange polynomials on the Gauss
// points), which maps values at the points to derivatives at the points.
//
// Everything is evaluated by the compiler in double (constexpr), so the device
// kernels see the matrix entries as literal constants.  The host set-up uses
// the same tables.
#pragma once

namespace rk {
namespace elem {

constexpr double cabs(double x) { return x < 0 ? -x : x; }

// cos by its Taylor series after reduction to [-pi, pi] (initial guesses only)
constexpr double ccos(double x) {
    constexpr double pi = 3.14159265358979323846;
    while (x > pi) x -= 2 * pi;
    while (x < -pi) x += 2 * pi;
    double term = 1, sum = 1;
    for (int n = 1; n < 30; ++n) {
        term *= -x * x / ((2 * n - 1) * (2 * n));
        sum += term;
    }
    return sum;
}

// P_m(s), P_m'(s), P_m''(s) by the three-term recurrence
struct Leg {
    double p, dp, d2p;
};
constexpr Leg legendre(int m, double s) {
    double p0 = 1, p1 = s, dp0 = 0, dp1 = 1, d0 = 0, d1 = 0;
    if (m == 0) return {1, 0, 0};
    for (int j = 1; j < m; ++j) {
        const double p2 = ((2 * j + 1) * s * p1 - j * p0) / (j + 1);
        const double dp2 = ((2 * j + 1) * (p1 + s * dp1) - j * dp0) / (j + 1);
        const double d2 = ((2 * j + 1) * (2 * dp1 + s * d1) - j * d0) / (j + 1);
        p0 = p1; p1 = p2; dp0 = dp1; dp1 = dp2; d0 = d1; d1 = d2;
    }
    return {p1, dp1, d1};
}

template <int K>
struct Data {
    double x[K + 1];                 // GLL nodes on [0,1]
    double gx[K + 1], gw[K + 1];     // Gauss points and weights on [0,1]
    double M[K + 1][K + 1];          // element mass matrix (unit cell)
    double A[K + 1][K + 1];          // element stiffness matrix (unit cell)
    double P[2 * K + 1][K + 1];      // cell-to-halves prolongation
    double gB[K + 1][K + 1];         // GLL basis at the Gauss points, [q][a]
    double gD[K + 1][K + 1];         // collocation derivative on the Gauss points, [q][p]
    double gBd[K + 1][K + 1];        // GLL basis derivatives at the Gauss points, [q][a]
};

template <int K>
constexpr Data<K> make() {
    constexpr double pi = 3.14159265358979323846;
    Data<K> d{};
    // GLL nodes: end points and the roots of P_K' (Newton with P_K'').
    d.x[0] = 0;
    d.x[K] = 1;
    for (int i = 1; i < K; ++i) {
        double s = -ccos(pi * i / K);
        for (int it = 0; it < 60; ++it) {
            const Leg l = legendre(K, s);
            const double ds = l.dp / l.d2p;
            s -= ds;
            if (cabs(ds) < 1e-17) break;
        }
        d.x[i] = (s + 1) / 2;
    }
    for (int i = 0; i <= K / 2; ++i) {           // exact symmetry about 1/2
        const double m = (d.x[i] + (1 - d.x[K - i])) / 2;
        d.x[i] = m;
        d.x[K - i] = 1 - m;
    }
    if (K % 2 == 0) d.x[K / 2] = 0.5;
    // Gauss-Legendre rule with K+1 points (Newton on P_{K+1}).
    const int n = K + 1;
    for (int i = 0; i < n; ++i) {
        double s = -ccos(pi * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 60; ++it) {
            const Leg l = legendre(n, s);
            const double ds = l.p / l.dp;
            s -= ds;
            if (cabs(ds) < 1e-17) break;
        }
        const Leg l = legendre(n, s);
        d.gx[i] = (s + 1) / 2;
        d.gw[i] = 1.0 / ((1 - s * s) * l.dp * l.dp);
    }
    // Lagrange values and derivatives at the Gauss points.
    double B[K + 1][K + 1] = {}, D[K + 1][K + 1] = {};
    for (int q = 0; q < n; ++q)
        for (int a = 0; a <= K; ++a) {
            double v = 1, dv = 0;
            for (int m = 0; m <= K; ++m) {
                if (m == a) continue;
                const double f = (d.gx[q] - d.x[m]) / (d.x[a] - d.x[m]);
                dv = dv * f + v / (d.x[a] - d.x[m]);
                v *= f;
            }
            B[q][a] = v;
            D[q][a] = dv;
            d.gB[q][a] = v;
            d.gBd[q][a] = dv;
        }
    for (int q = 0; q < n; ++q)
        for (int p = 0; p < n; ++p) {
            double v = 1, dv = 0;
            for (int m = 0; m < n; ++m) {
                if (m == p) continue;
                const double f = (d.gx[q] - d.gx[m]) / (d.gx[p] - d.gx[m]);
                dv = dv * f + v / (d.gx[p] - d.gx[m]);
                v *= f;
            }
            d.gD[q][p] = dv;
        }
    for (int a = 0; a <= K; ++a)
        for (int b = 0; b <= K; ++b) {
            double m = 0, s = 0;
            for (int q = 0; q < n; ++q) {
                m += d.gw[q] * B[q][a] * B[q][b];
                s += d.gw[q] * D[q][a] * D[q][b];
            }
            d.M[a][b] = m;
            d.A[a][b] = s;
        }
    for (int f = 0; f <= 2 * K; ++f) {
        const double xf = f <= K ? d.x[f] / 2 : 0.5 + d.x[f - K] / 2;
        for (int c = 0; c <= K; ++c) {
            double v = 1;
            for (int m = 0; m <= K; ++m)
                if (m != c) v *= (xf - d.x[m]) / (d.x[c] - d.x[m]);
            d.P[f][c] = v;
        }
    }
    return d;
}

template <int K>
struct Table {
    static constexpr Data<K> d = make<K>();
};

}  // namespace elem
}  // namespace rk
