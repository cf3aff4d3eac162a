// Host-side set-up mathematics: the Radau IIA tableau, the Crout factor of
// A^-1 and its eigen-decomposition (Sec. 2, eq. irk:P), the direct complex
// diagonalisation of A^-1 (eq. irk:Ainv) in long double, and the 1D Q_k
// element data (Sec. 5 set-up) from the compile-time tables.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <string>

#include "element_data.h"
#include "rk_internal.h"

namespace rk {
namespace {

using ld = long double;

// P_m(s) and its first two derivatives by the three-term recurrence.
void legendre(int m, ld s, ld& p, ld& dp, ld& d2p) {
    ld p0 = 1, p1 = s, dp0 = 0, dp1 = 1, d2p0 = 0, d2p1 = 0;
    if (m == 0) { p = 1; dp = 0; d2p = 0; return; }
    for (int j = 1; j < m; ++j) {
        ld p2 = ((2 * j + 1) * s * p1 - j * p0) / (j + 1);
        ld dp2 = ((2 * j + 1) * (p1 + s * dp1) - j * dp0) / (j + 1);
        ld d2p2 = ((2 * j + 1) * (2 * dp1 + s * d2p1) - j * d2p0) / (j + 1);
        p0 = p1; p1 = p2; dp0 = dp1; dp1 = dp2; d2p0 = d2p1; d2p1 = d2p2;
    }
    p = p1; dp = dp1; d2p = d2p1;
}

// n-point Gauss-Legendre rule on [0,1] by Newton on P_n.
void gauss(int n, ld* x, ld* w) {
    const ld pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < n; ++i) {
        ld s = -std::cos(pi * (i + 0.75L) / (n + 0.5L));
        ld p, dp, d2p;
        for (int it = 0; it < 100; ++it) {
            legendre(n, s, p, dp, d2p);
            ld ds = p / dp;
            s -= ds;
            if (std::fabs(ds) < 1e-19L) break;
        }
        legendre(n, s, p, dp, d2p);
        x[i] = (s + 1) / 2;
        w[i] = 1.0L / ((1 - s * s) * dp * dp);   // = (2/((1-s^2)P'^2)) / 2
    }
}

// Integral over [0, up] of the j-th Lagrange polynomial on nodes c[0..q).
ld lagrange_integral(const ld* c, int q, int j, ld up) {
    ld gx[16], gw[16];
    int ng = q / 2 + 2;
    gauss(ng, gx, gw);
    ld sum = 0;
    for (int g = 0; g < ng; ++g) {
        ld x = up * gx[g], v = 1;
        for (int m = 0; m < q; ++m)
            if (m != j) v *= (x - c[m]) / (c[j] - c[m]);
        sum += gw[g] * v;
    }
    return sum * up;
}

// Gauss-Jordan inverse with partial pivoting (n <= 9).
bool invert(int n, const ld* a, ld* inv) {
    ld m[RK_MAX_Q][2 * RK_MAX_Q];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < 2 * n; ++j) m[i][j] = j < n ? a[i * n + j] : (j - n == i ? 1 : 0);
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(m[r][c]) > std::fabs(m[piv][c])) piv = r;
        if (m[piv][c] == 0) return false;
        if (piv != c)
            for (int j = 0; j < 2 * n; ++j) std::swap(m[piv][j], m[c][j]);
        ld d = m[c][c];
        for (int j = 0; j < 2 * n; ++j) m[c][j] /= d;
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            ld f = m[r][c];
            if (f != 0)
                for (int j = 0; j < 2 * n; ++j) m[r][j] -= f * m[c][j];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) inv[i * n + j] = m[i][j + n];
    return true;
}

using cld = std::complex<ld>;

// Solves (a - shift I) x = rhs in place (x <- rhs) by Gaussian elimination
// with partial pivoting; returns the determinant of (a - shift I).  A zero
// pivot is replaced by a tiny one (inverse iteration at an exact eigenvalue).
cld shifted_solve(int n, const ld* a, cld shift, cld* x) {
    cld m[RK_MAX_Q][RK_MAX_Q];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) m[i][j] = cld(a[i * n + j]) - (i == j ? shift : cld(0));
    cld det = 1;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::abs(m[r][c]) > std::abs(m[piv][c])) piv = r;
        if (piv != c) {
            for (int j = 0; j < n; ++j) std::swap(m[piv][j], m[c][j]);
            if (x) std::swap(x[piv], x[c]);
            det = -det;
        }
        if (m[c][c] == cld(0)) m[c][c] = cld(1e-30L);
        det *= m[c][c];
        for (int r = c + 1; r < n; ++r) {
            const cld f = m[r][c] / m[c][c];
            for (int j = c; j < n; ++j) m[r][j] -= f * m[c][j];
            if (x) x[r] -= f * x[c];
        }
    }
    if (x)
        for (int i = n - 1; i >= 0; --i) {
            cld acc = x[i];
            for (int j = i + 1; j < n; ++j) acc -= m[i][j] * x[j];
            x[i] = acc / m[i][i];
        }
    return det;
}

// Eigenvalues of a (n x n) as the roots of the monic p(z) = det(z I - a),
// evaluated by elimination, with the Weierstrass (Durand-Kerner) iteration
// z_i <- z_i - p(z_i) / prod_{j != i} (z_i - z_j).
bool eigenvalues(int n, const ld* a, cld* z) {
    ld rad = 0;   // infinity norm bounds every eigenvalue
    for (int i = 0; i < n; ++i) {
        ld row = 0;
        for (int j = 0; j < n; ++j) row += std::fabs(a[i * n + j]);
        rad = std::max(rad, row);
    }
    const cld seed(0.4L, 0.9L);
    cld p = 1;
    for (int i = 0; i < n; ++i) { z[i] = rad * p; p *= seed; }
    ld change = 0;
    for (int it = 0; it < 2000; ++it) {
        change = 0;
        for (int i = 0; i < n; ++i) {
            // det(z I - a) = (-1)^n det(a - z I)
            cld pz = shifted_solve(n, a, z[i], nullptr);
            if (n % 2) pz = -pz;
            cld den = 1;
            for (int j = 0; j < n; ++j)
                if (j != i) den *= z[i] - z[j];
            if (den == cld(0)) den = cld(1e-30L);
            const cld dz = pz / den;
            z[i] -= dz;
            change = std::max(change, std::abs(dz) / std::max(std::abs(z[i]), (ld)1e-30L));
        }
        if (change < 1e-17L) return true;
    }
    // the determinant's rounding error stalls the last digits for larger n
    return change < 1e-13L;
}

// Right eigenvector for the eigenvalue lam by three steps of inverse
// iteration, scaled so that its largest component is 1.
void eigenvector(int n, const ld* a, cld lam, cld* v) {
    for (int i = 0; i < n; ++i) v[i] = cld(1.0L + 0.1L * i, 0.05L * i);
    for (int it = 0; it < 3; ++it) {
        shifted_solve(n, a, lam, v);
        int im = 0;
        for (int i = 1; i < n; ++i)
            if (std::abs(v[i]) > std::abs(v[im])) im = i;
        const cld s = v[im];
        for (int i = 0; i < n; ++i) v[i] /= s;
    }
}

// The real slot form of the direct diagonalisation of Ai = A^-1.
bool build_complex(int Q, const ld* Ai, Tableau& t, std::string& err) {
    cld z[RK_MAX_Q];
    if (!eigenvalues(Q, Ai, z)) { err = "eigenvalues of A^-1 did not converge"; return false; }
    ld scale = 0;
    for (int i = 0; i < Q; ++i) scale = std::max(scale, std::abs(z[i]));
    cld pairs[RK_MAX_Q];
    int np = 0, nr = 0;
    cld real = 0;
    for (int i = 0; i < Q; ++i) {
        if (std::fabs(z[i].imag()) <= 1e-12L * scale) { real = cld(z[i].real(), 0); ++nr; }
        else if (z[i].imag() > 0) pairs[np++] = z[i];
    }
    if (nr != Q % 2 || 2 * np + nr != Q) { err = "unexpected spectrum of A^-1"; return false; }
    std::sort(pairs, pairs + np, [](const cld& x, const cld& y) { return x.real() < y.real(); });
    const int nb = np + nr;
    ld U[RK_MAX_Q * RK_MAX_Q] = {0}, T[RK_MAX_Q * RK_MAX_Q];
    cld v[RK_MAX_Q];
    for (int j = 0; j < np; ++j) {
        eigenvector(Q, Ai, pairs[j], v);
        for (int r = 0; r < Q; ++r) {
            U[r * Q + j] = 2 * v[r].real();
            U[r * Q + nb + j] = -2 * v[r].imag();
        }
    }
    if (nr) {
        eigenvector(Q, Ai, real, v);
        for (int r = 0; r < Q; ++r) U[r * Q + np] = v[r].real();
    }
    if (!invert(Q, U, T)) { err = "eigenvector matrix of A^-1 singular"; return false; }
    ld L[RK_MAX_Q * RK_MAX_Q] = {0};
    for (int j = 0; j < np; ++j) {
        const ld a = pairs[j].real(), b = pairs[j].imag();
        L[j * Q + j] = a; L[j * Q + nb + j] = -b;
        L[(nb + j) * Q + j] = b; L[(nb + j) * Q + nb + j] = a;
    }
    if (nr) L[np * Q + np] = real.real();
    // check T A^-1 U = Lam_r
    ld dev = 0;
    for (int i = 0; i < Q; ++i)
        for (int j = 0; j < Q; ++j) {
            ld acc = 0;
            for (int l = 0; l < Q; ++l)
                for (int m = 0; m < Q; ++m) acc += T[i * Q + l] * Ai[l * Q + m] * U[m * Q + j];
            dev = std::max(dev, std::fabs(acc - L[i * Q + j]));
        }
    if (!(dev <= 1e-10L * scale)) { err = "direct diagonalisation of A^-1 inaccurate"; return false; }
    t.nb = nb;
    t.npair = np;
    for (int j = 0; j < RK_MAX_Q; ++j) { t.clam_re[j] = 0; t.clam_im[j] = 0; t.hshift[j] = 0; }
    for (int j = 0; j < np; ++j) {
        t.clam_re[j] = (double)pairs[j].real();
        t.clam_im[j] = (double)pairs[j].imag();
        t.hshift[j] = t.hshift[nb + j] = (double)(pairs[j].real() + pairs[j].imag());
    }
    if (nr) { t.clam_re[np] = (double)real.real(); t.hshift[np] = (double)real.real(); }
    for (int i = 0; i < Q * Q; ++i) {
        t.CT[i] = (double)T[i]; t.CU[i] = (double)U[i]; t.CLam[i] = (double)L[i];
    }
    return true;
}

}  // namespace

bool build_tableau(int Q, Tableau& t, std::string& err) {
    if (Q < 1 || Q > RK_MAX_Q) { err = "Q out of range"; return false; }
    t.Q = Q;
    // Radau IIA nodes: roots of f(x) = P_Q(2x-1) - P_{Q-1}(2x-1) on (0,1],
    // bracketed on a fine grid and refined by bisection; c_Q = 1 exactly.
    ld c[RK_MAX_Q];
    auto f = [&](ld x) {
        ld p, dp, d2p, q, dq, d2q;
        legendre(Q, 2 * x - 1, p, dp, d2p);
        legendre(Q - 1, 2 * x - 1, q, dq, d2q);
        return p - q;
    };
    int found = 0;
    const int G = 20000;
    ld xa = 0, fa = f(xa);
    for (int i = 1; i < G && found < Q - 1; ++i) {
        ld xb = (ld)i / G, fb = f(xb);
        if (fa == 0) { c[found++] = xa; }
        else if ((fa < 0) != (fb < 0)) {
            ld lo = xa, hi = xb, flo = fa;
            for (int it = 0; it < 200; ++it) {
                ld mid = (lo + hi) / 2, fm = f(mid);
                if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else hi = mid;
            }
            c[found++] = (lo + hi) / 2;
        }
        xa = xb; fa = fb;
    }
    if (found != Q - 1) { err = "Radau node search failed"; return false; }
    c[Q - 1] = 1;
    ld A[RK_MAX_Q * RK_MAX_Q], Ai[RK_MAX_Q * RK_MAX_Q];
    for (int i = 0; i < Q; ++i) {
        for (int j = 0; j < Q; ++j) A[i * Q + j] = lagrange_integral(c, Q, j, c[i]);
        t.b[i] = (double)lagrange_integral(c, Q, i, 1);
        t.c[i] = (double)c[i];
    }
    if (!invert(Q, A, Ai)) { err = "A_Q singular"; return false; }
    // Crout: A^-1 = L U, U unit upper triangular, no pivoting.
    ld L[RK_MAX_Q * RK_MAX_Q] = {0}, U[RK_MAX_Q * RK_MAX_Q] = {0};
    for (int i = 0; i < Q; ++i) U[i * Q + i] = 1;
    for (int j = 0; j < Q; ++j) {
        for (int i = j; i < Q; ++i) {
            ld s = Ai[i * Q + j];
            for (int m = 0; m < j; ++m) s -= L[i * Q + m] * U[m * Q + j];
            L[i * Q + j] = s;
        }
        if (L[j * Q + j] == 0) { err = "Crout factorisation of A^-1 breaks down"; return false; }
        for (int i = j + 1; i < Q; ++i) {
            ld s = Ai[j * Q + i];
            for (int m = 0; m < j; ++m) s -= L[j * Q + m] * U[m * Q + i];
            U[j * Q + i] = s / L[j * Q + j];
        }
    }
    // L = S Lam S^-1: eigenvalues diag(L); eigenvector i is zero above row i,
    // one at row i, and follows from (L - lam_i I) s = 0 below.
    ld S[RK_MAX_Q * RK_MAX_Q] = {0}, Si[RK_MAX_Q * RK_MAX_Q];
    for (int i = 0; i < Q; ++i) {
        S[i * Q + i] = 1;
        for (int m = i + 1; m < Q; ++m) {
            ld acc = 0;
            for (int r = i; r < m; ++r) acc += L[m * Q + r] * S[r * Q + i];
            ld den = L[i * Q + i] - L[m * Q + m];
            if (den == 0) { err = "L has a repeated eigenvalue"; return false; }
            S[m * Q + i] = acc / den;
        }
    }
    if (!invert(Q, S, Si)) { err = "S singular"; return false; }
    for (int i = 0; i < Q * Q; ++i) {
        t.A[i] = (double)A[i]; t.Ainv[i] = (double)Ai[i];
        t.L[i] = (double)L[i]; t.U[i] = (double)U[i];
        t.S[i] = (double)S[i]; t.Sinv[i] = (double)Si[i];
    }
    for (int i = 0; i < Q; ++i) t.lam[i] = (double)L[i * Q + i];
    return build_complex(Q, Ai, t, err);
}

namespace {
template <int K>
void copy_element(Element1D& e) {
    constexpr auto d = elem::make<K>();
    const int n1 = K + 1;
    for (int i = 0; i < n1; ++i) e.nodes[i] = d.x[i];
    for (int a = 0; a < n1; ++a)
        for (int b = 0; b < n1; ++b) {
            e.mass[a * n1 + b] = d.M[a][b];
            e.stiff[a * n1 + b] = d.A[a][b];
        }
    for (int f = 0; f <= 2 * K; ++f)
        for (int c = 0; c < n1; ++c) e.prol[f * n1 + c] = d.P[f][c];
}
}  // namespace

// 1D element data: the compile-time tables that the kernels use.
void build_element(int k, Element1D& e) {
    e.k = k;
    switch (k) {
        case 1: copy_element<1>(e); break;
        case 2: copy_element<2>(e); break;
        case 3: copy_element<3>(e); break;
        case 4: copy_element<4>(e); break;
        case 5: copy_element<5>(e); break;
        default: copy_element<6>(e); break;
    }
}

}  // namespace rk
