// Host construction of the Runge-Kutta tableaux and of the real eigenbasis
// of A0^{-1} (paper Sections 1.1, 3.1 and 5).  Pure host code, long double.
//
// * Nodes: roots of the shifted Legendre polynomial P_s(2x-1) (Gauss) or of
//   P_s(2x-1) - P_{s-1}(2x-1) (Radau IIA, c_s = 1), found by bracketing on a
//   fine grid and Newton polishing.
// * A, b: collocation integrals a_ij = int_0^{c_i} l_j, b_j = int_0^1 l_j of
//   the Lagrange basis on the nodes.
// * Eigenbasis: characteristic polynomial of A0^{-1} (Faddeev-LeVerrier),
//   roots by the Aberth-Ehrlich iteration, eigenvectors as null vectors of
//   (A0^{-1} - lambda I) by complex elimination with full pivoting.  Complex
//   pairs eta +- i beta give the real 2x2 block [[eta, beta], [-beta, eta]]
//   with the columns (Re v, Im v) of the eigenvector of eta + i beta, phased so
//   that Re v is orthogonal to Im v (the form [[eta, phi], [-beta^2/phi, eta]]
//   of Section 3.1 with phi = beta).
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "irk_internal.h"

namespace irk {

typedef long double ld;
typedef std::complex<long double> cld;

static ld binom(int n, int k) {
    ld r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

// A polynomial of degree < IRK_MAX_STAGES + 2 (ascending coefficients) or a
// short list of nodes, in a fixed-size array: the tableau construction works
// without heap memory.
struct Poly {
    ld c[IRK_MAX_STAGES + 2];
    int n = 0;                          // number of coefficients (entries)
    void push(ld v) { c[n++] = v; }
};

// ascending coefficients of P_n(2x - 1) = sum_k (-1)^(n+k) C(n,k) C(n+k,k) x^k
static Poly shifted_legendre(int n) {
    Poly c;
    for (int k = 0; k <= n; ++k)
        c.push((((n + k) % 2) ? -1.0L : 1.0L) * binom(n, k) * binom(n + k, k));
    return c;
}

static ld horner(const Poly &c, ld x, ld *deriv) {
    ld p = 0, dp = 0;
    for (int k = c.n - 1; k >= 0; --k) {
        dp = dp * x + p;
        p = p * x + c.c[k];
    }
    if (deriv) *deriv = dp;
    return p;
}

// real roots of c in [0, 1] (all simple), ascending
static Poly roots_unit_interval(const Poly &c, int expect) {
    Poly r;
    const int G = 20000;
    ld xa = 0, fa = horner(c, 0, nullptr);
    for (int g = 1; g <= G && r.n < expect; ++g) {
        ld xb = (ld)g / G, fb = horner(c, xb, nullptr);
        if (fb == 0) { r.push(xb); xa = xb; fa = fb; continue; }
        if ((fa < 0) != (fb < 0) && fa != 0) {
            ld lo = xa, hi = xb, flo = fa;
            for (int it = 0; it < 200; ++it) {          // bisection
                ld mid = 0.5L * (lo + hi), fm = horner(c, mid, nullptr);
                if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else hi = mid;
            }
            ld x = 0.5L * (lo + hi);
            for (int it = 0; it < 5; ++it) {             // Newton polish
                ld d, f = horner(c, x, &d);
                if (d != 0) x -= f / d;
            }
            r.push(x);
        }
        xa = xb; fa = fb;
    }
    return r;
}

// Lagrange basis polynomial l_j on the nodes c
static Poly lagrange(const Poly &c, int j) {
    Poly p;
    p.push(1.0L);
    ld den = 1;
    for (int m = 0; m < c.n; ++m) {
        if (m == j) continue;
        Poly q;
        q.n = p.n + 1;
        for (int k = 0; k < q.n; ++k) q.c[k] = 0.0L;
        for (int k = 0; k < p.n; ++k) { q.c[k] -= p.c[k] * c.c[m]; q.c[k + 1] += p.c[k]; }
        p = q;
        den *= (c.c[j] - c.c[m]);
    }
    for (int k = 0; k < p.n; ++k) p.c[k] /= den;
    return p;
}

static ld integrate0(const Poly &p, ld x) {
    ld s = 0, xp = x;
    for (int k = 0; k < p.n; ++k) { s += p.c[k] * xp / (ld)(k + 1); xp *= x; }
    return s;
}

// Published L-stable SDIRK methods (lower triangular A with constant
// diagonal gamma, stiffly accurate: b = last row, c = row sums).
static bool sdirk_tableau(int s, ld *A, ld *b, ld *c) {
    for (int i = 0; i < s * s; ++i) A[i] = 0;
    if (s == 1) {
        A[0] = 1;                                   // backward Euler
    } else if (s == 2) {                            // Alexander, order 2
        const ld g = 1.0L - 1.0L / sqrtl(2.0L);
        A[0] = g;
        A[2] = 1.0L - g; A[3] = g;
    } else if (s == 3) {                            // Alexander, order 3
        // gamma: root of x^3 - 3x^2 + 3x/2 - 1/6 in (1/3, 1/2), by Newton
        ld g = 0.4358665L;
        for (int it = 0; it < 20; ++it)
            g -= (g * g * g - 3 * g * g + 1.5L * g - 1.0L / 6) / (3 * g * g - 6 * g + 1.5L);
        const ld t2 = 0.5L * (1 + g);
        const ld b1 = -(6 * g * g - 16 * g + 1) / 4, b2 = (6 * g * g - 20 * g + 5) / 4;
        A[0] = g;
        A[3] = t2 - g; A[4] = g;
        A[6] = b1; A[7] = b2; A[8] = g;
    } else if (s == 5) {                            // Hairer-Wanner, order 4
        const ld r[5][5] = {{1.0L / 4, 0, 0, 0, 0},
                            {1.0L / 2, 1.0L / 4, 0, 0, 0},
                            {17.0L / 50, -1.0L / 25, 1.0L / 4, 0, 0},
                            {371.0L / 1360, -137.0L / 2720, 15.0L / 544, 1.0L / 4, 0},
                            {25.0L / 24, -49.0L / 48, 125.0L / 16, -85.0L / 12, 1.0L / 4}};
        for (int i = 0; i < 5; ++i)
            for (int j = 0; j < 5; ++j) A[i * 5 + j] = r[i][j];
    } else {
        return false;
    }
    for (int i = 0; i < s; ++i) {
        ld sum = 0;
        for (int j = 0; j < s; ++j) sum += A[i * s + j];
        c[i] = sum;
        b[i] = A[(s - 1) * s + i];
    }
    return true;
}

bool build_tableau_ld(int family, int s, ld *A, ld *b, ld *c) {
    if (s < 1 || s > IRK_MAX_STAGES) return false;
    if (family == IRK_SDIRK) return sdirk_tableau(s, A, b, c);
    Poly nodes;
    if (family == IRK_GAUSS) {
        nodes = roots_unit_interval(shifted_legendre(s), s);
    } else if (family == IRK_RADAU_IIA) {
        if (s == 1) {
            nodes.push(1.0L);
        } else {
            Poly p = shifted_legendre(s), q = shifted_legendre(s - 1);
            for (int k = 0; k < q.n; ++k) p.c[k] -= q.c[k];
            // deflate the root at x = 1: divide by (x - 1) (synthetic division)
            const int deg = s;
            Poly d;
            d.n = deg;
            ld carry = p.c[deg];
            for (int k = deg - 1; k >= 0; --k) { d.c[k] = carry; carry = p.c[k] + carry; }
            nodes = roots_unit_interval(d, s - 1);
            nodes.push(1.0L);
        }
    } else if (family == IRK_LOBATTO_IIIC) {
        // nodes 0, the roots of d/dx P_{s-1}(2x-1), 1
        if (s < 2) return false;
        nodes.push(0.0L);
        if (s > 2) {
            Poly q = shifted_legendre(s - 1), dq;
            dq.n = s - 1;
            for (int k = 1; k < s; ++k) dq.c[k - 1] = k * q.c[k];
            const Poly r = roots_unit_interval(dq, s - 2);
            for (int k = 0; k < r.n; ++k) nodes.push(r.c[k]);
        }
        nodes.push(1.0L);
    } else {
        return false;
    }
    if (nodes.n != s) return false;
    std::sort(nodes.c, nodes.c + nodes.n);
    for (int j = 0; j < s; ++j) {
        const Poly l = lagrange(nodes, j);
        for (int i = 0; i < s; ++i) A[i * s + j] = integrate0(l, nodes.c[i]);
        b[j] = integrate0(l, 1.0L);
    }
    if (family == IRK_LOBATTO_IIIC) {
        // a_i1 = b_1 and the simplifying conditions C(s-1) for the other
        // entries of each row: sum_{j>=2} a_ij c_j^{k-1} = c_i^k/k - b_1 [k=1]
        const int m = s - 1;
        for (int i = 0; i < s; ++i) {
            ld M[IRK_MAX_STAGES][IRK_MAX_STAGES + 1];
            for (int k = 1; k <= m; ++k) {
                for (int j = 1; j < s; ++j) M[k - 1][j - 1] = powl(nodes.c[j], (ld)(k - 1));
                M[k - 1][m] = powl(nodes.c[i], (ld)k) / k - (k == 1 ? b[0] : 0.0L);
            }
            for (int col = 0; col < m; ++col) {             // Gaussian elimination, partial pivoting
                int piv = col;
                for (int r = col + 1; r < m; ++r)
                    if (fabsl(M[r][col]) > fabsl(M[piv][col])) piv = r;
                for (int q = 0; q <= m; ++q) std::swap(M[col][q], M[piv][q]);
                if (M[col][col] == 0) return false;
                for (int r = 0; r < m; ++r) {
                    if (r == col) continue;
                    const ld f = M[r][col] / M[col][col];
                    for (int q = col; q <= m; ++q) M[r][q] -= f * M[col][q];
                }
            }
            A[i * s] = b[0];
            for (int j = 1; j < s; ++j) A[i * s + j] = M[j - 1][m] / M[j - 1][j - 1];
        }
    }
    for (int i = 0; i < s; ++i) c[i] = nodes.c[i];
    return true;
}

// Gauss-Jordan inverse with partial pivoting (n <= 5)
static bool invert_ld(int n, const ld *M, ld *Minv) {
    ld a[IRK_MAX_STAGES][2 * IRK_MAX_STAGES];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < 2 * n; ++j)
            a[i][j] = j < n ? M[i * n + j] : (j - n == i ? 1.0L : 0.0L);
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabsl(a[r][col]) > fabsl(a[piv][col])) piv = r;
        if (a[piv][col] == 0) return false;
        for (int j = 0; j < 2 * n; ++j) std::swap(a[col][j], a[piv][j]);
        ld inv = 1.0L / a[col][col];
        for (int j = 0; j < 2 * n; ++j) a[col][j] *= inv;
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            ld f = a[r][col];
            if (f == 0) continue;
            for (int j = 0; j < 2 * n; ++j) a[r][j] -= f * a[col][j];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Minv[i * n + j] = a[i][n + j];
    return true;
}

// characteristic polynomial coefficients (ascending, monic) by Faddeev-LeVerrier
static std::vector<ld> charpoly(int n, const ld *M) {
    std::vector<ld> cp(n + 1, 0.0L);
    cp[n] = 1.0L;
    std::vector<ld> Mk(n * n, 0.0L), AMk(n * n);
    for (int k = 1; k <= n; ++k) {
        // Mk = M * M_{k-1} + c_{n-k+1} I
        std::vector<ld> T(n * n, 0.0L);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                ld sacc = 0;
                for (int q = 0; q < n; ++q) sacc += M[i * n + q] * Mk[q * n + j];
                T[i * n + j] = sacc + (i == j ? cp[n - k + 1] : 0.0L);
            }
        Mk = T;
        ld tr = 0;
        for (int i = 0; i < n; ++i) {
            ld sacc = 0;
            for (int q = 0; q < n; ++q) sacc += M[i * n + q] * Mk[q * n + i];
            tr += sacc;
        }
        cp[n - k] = -tr / (ld)k;
    }
    return cp;
}

static std::vector<cld> aberth(const std::vector<ld> &cp) {
    int n = (int)cp.size() - 1;
    std::vector<cld> z(n);
    // initial guesses on a circle of the Cauchy bound radius
    ld rad = 0;
    for (int k = 0; k < n; ++k) rad = std::max(rad, fabsl(cp[k]));
    rad = 1 + rad;
    for (int k = 0; k < n; ++k) z[k] = std::polar(rad * 0.5L, (ld)(2 * M_PI * (k + 0.25) / n));
    auto evalp = [&](cld x, cld *d) {
        cld p = 0, dp = 0;
        for (int k = n; k >= 0; --k) { dp = dp * x + p; p = p * x + cp[k]; }
        *d = dp;
        return p;
    };
    for (int it = 0; it < 500; ++it) {
        ld maxstep = 0;
        for (int k = 0; k < n; ++k) {
            cld d, p = evalp(z[k], &d);
            if (std::abs(p) == 0) continue;
            cld ratio = p / d, sum = 0;
            for (int j = 0; j < n; ++j)
                if (j != k) sum += 1.0L / (z[k] - z[j]);
            cld w = ratio / (1.0L - ratio * sum);
            z[k] -= w;
            maxstep = std::max(maxstep, std::abs(w) / std::max((ld)1, std::abs(z[k])));
        }
        if (maxstep < 1e-30L) break;
    }
    for (int k = 0; k < n; ++k) {                          // Newton polish
        for (int it = 0; it < 3; ++it) {
            cld d, p = evalp(z[k], &d);
            if (std::abs(d) > 0) z[k] -= p / d;
        }
    }
    return z;
}

// null vector of (M - lam I) by complex elimination with full pivoting
static std::vector<cld> null_vector(int n, const ld *M, cld lam) {
    cld a[IRK_MAX_STAGES][IRK_MAX_STAGES];
    int colperm[IRK_MAX_STAGES];
    for (int i = 0; i < n; ++i) {
        colperm[i] = i;
        for (int j = 0; j < n; ++j) a[i][j] = cld(M[i * n + j]) - (i == j ? lam : cld(0));
    }
    for (int k = 0; k < n - 1; ++k) {
        int pr = k, pc = k;
        ld best = -1;
        for (int i = k; i < n; ++i)
            for (int j = k; j < n; ++j)
                if (std::abs(a[i][j]) > best) { best = std::abs(a[i][j]); pr = i; pc = j; }
        for (int j = 0; j < n; ++j) std::swap(a[k][j], a[pr][j]);
        for (int i = 0; i < n; ++i) std::swap(a[i][k], a[i][pc]);
        std::swap(colperm[k], colperm[pc]);
        for (int i = k + 1; i < n; ++i) {
            cld f = a[i][k] / a[k][k];
            for (int j = k; j < n; ++j) a[i][j] -= f * a[k][j];
        }
    }
    // the last pivot is ~0: set the last permuted unknown to 1, back-substitute
    std::vector<cld> y(n);
    y[n - 1] = 1;
    for (int k = n - 2; k >= 0; --k) {
        cld sacc = 0;
        for (int j = k + 1; j < n; ++j) sacc += a[k][j] * y[j];
        y[k] = -sacc / a[k][k];
    }
    std::vector<cld> v(n);
    for (int k = 0; k < n; ++k) v[colperm[k]] = y[k];
    return v;
}

// Real Schur basis of A0^{-1} (Section 3.1): A0^{-1} = Q0 R0 Q0^T with Q0
// orthogonal and R0 block upper triangular.  Built from the real eigenbasis
// T (blocks in its order: real eigenvalues, then pairs by decreasing beta):
// T = Q R (Gram-Schmidt), so Q^T A0^{-1} Q = R Lambda R^{-1} is block upper
// triangular; each 2x2 diagonal block is then rotated to equal diagonal
// entries [[eta, phi], [-beta^2/phi, eta]], with a quarter turn if needed so
// that |phi| <= beta (the standardized form), and every column's sign is
// fixed so that its largest entry is positive.
bool build_schur_blocks(int family, int s, EigenBlocks *eb) {
    EigenBlocks e;
    if (!build_eigen_blocks(family, s, &e)) return false;
    ld Q[IRK_MAX_STAGES * IRK_MAX_STAGES];
    for (int i = 0; i < s * s; ++i) Q[i] = e.T[i];
    // modified Gram-Schmidt on the columns, twice (long double)
    for (int pass = 0; pass < 2; ++pass)
        for (int j = 0; j < s; ++j) {
            for (int q = 0; q < j; ++q) {
                ld dot = 0;
                for (int i = 0; i < s; ++i) dot += Q[i * s + q] * Q[i * s + j];
                for (int i = 0; i < s; ++i) Q[i * s + j] -= dot * Q[i * s + q];
            }
            ld nrm = 0;
            for (int i = 0; i < s; ++i) nrm += Q[i * s + j] * Q[i * s + j];
            nrm = sqrtl(nrm);
            if (!(nrm > 0)) return false;
            for (int i = 0; i < s; ++i) Q[i * s + j] /= nrm;
        }
    ld Ai[IRK_MAX_STAGES * IRK_MAX_STAGES], R[IRK_MAX_STAGES * IRK_MAX_STAGES];
    for (int i = 0; i < s * s; ++i) Ai[i] = e.Ainv[i];
    {   // a long double A0^{-1} (the float64 copy costs digits)
        ld A[IRK_MAX_STAGES * IRK_MAX_STAGES], b[IRK_MAX_STAGES], c[IRK_MAX_STAGES];
        if (!build_tableau_ld(family, s, A, b, c) || !invert_ld(s, A, Ai)) return false;
    }
    auto rform = [&]() {                   // R = Q^T A0^{-1} Q
        for (int i = 0; i < s; ++i)
            for (int j = 0; j < s; ++j) {
                ld acc = 0;
                for (int k = 0; k < s; ++k) {
                    ld t = 0;
                    for (int l = 0; l < s; ++l) t += Ai[k * s + l] * Q[l * s + j];
                    acc += Q[k * s + i] * t;
                }
                R[i * s + j] = acc;
            }
    };
    auto rotate = [&](int r, ld cs, ld sn) {    // Q <- Q G on columns r, r+1
        for (int i = 0; i < s; ++i) {
            const ld a = Q[i * s + r], b = Q[i * s + r + 1];
            Q[i * s + r] = cs * a + sn * b;
            Q[i * s + r + 1] = -sn * a + cs * b;
        }
    };
    rform();
    for (int k = 0; k < e.nblocks; ++k) {
        if (e.width[k] != 2) continue;
        const int r = e.first[k];
        const ld p = R[r * s + r], q = R[r * s + r + 1], u = R[(r + 1) * s + r], t = R[(r + 1) * s + r + 1];
        // G = [[cos, -sin], [sin, cos]]: a' - d' = (p - t) cos 2th + (q + u) sin 2th = 0
        const ld th = 0.5L * atan2l(-(p - t), q + u);
        rotate(r, cosl(th), sinl(th));
        rform();
        if (fabsl(R[r * s + r + 1]) > fabsl(R[(r + 1) * s + r])) {     // quarter turn
            rotate(r, 0.0L, 1.0L);
            rform();
        }
    }
    for (int j = 0; j < s; ++j) {          // sign: largest entry of each column positive
        int ib = 0;
        ld big = 0;
        for (int i = 0; i < s; ++i)
            if (fabsl(Q[i * s + j]) > big) { big = fabsl(Q[i * s + j]); ib = i; }
        if (Q[ib * s + j] < 0)
            for (int i = 0; i < s; ++i) Q[i * s + j] = -Q[i * s + j];
    }
    rform();
    *eb = e;
    eb->schur = true;
    for (int k = 0; k < e.nblocks; ++k) {
        const int r = e.first[k];
        if (e.width[k] == 2) {
            eb->eta[k] = (double)(0.5L * (R[r * s + r] + R[(r + 1) * s + r + 1]));
            eb->c12[k] = (double)R[r * s + r + 1];
            eb->c21[k] = (double)R[(r + 1) * s + r];
            eb->beta[k] = (double)sqrtl(fmaxl(-R[r * s + r + 1] * R[(r + 1) * s + r], 0.0L));
        } else {
            eb->eta[k] = (double)R[r * s + r];
            eb->c12[k] = eb->c21[k] = 0.0;
            eb->beta[k] = 0.0;
        }
        eb->gamma_star[k] = eb->eta[k] + eb->beta[k] * eb->beta[k] / eb->eta[k];
    }
    // R0 with its entries below the block diagonal (rounding level) dropped
    for (int i = 0; i < s; ++i)
        for (int j = 0; j < s; ++j) {
            int bi = 0, bj = 0;
            for (int k = 0; k < e.nblocks; ++k) {
                if (i >= e.first[k] && i < e.first[k] + e.width[k]) bi = k;
                if (j >= e.first[k] && j < e.first[k] + e.width[k]) bj = k;
            }
            eb->R[i * s + j] = bj < bi ? 0.0 : (double)R[i * s + j];
        }
    for (int i = 0; i < s; ++i)
        for (int j = 0; j < s; ++j) {
            ld tl = 0;
            for (int q = 0; q < s; ++q) tl += Q[i * s + q] * (ld)eb->R[q * s + j];
            eb->TLam[i * s + j] = (double)tl;
            eb->T[i * s + j] = (double)Q[i * s + j];
            eb->Tinv[i * s + j] = (double)Q[j * s + i];
        }
    for (int k = 0; k < s; ++k) {              // Newton-like (1) stage of each row
        ld dk[IRK_MAX_STAGES], big = 0;
        for (int i = 0; i < s; ++i) {
            dk[i] = Q[i * s + k] * Q[i * s + k];
            if (dk[i] > big) big = dk[i];
        }
        int best = 0;
        while (best + 1 < s && dk[best] < big * (1.0L - 1e-12L)) ++best;
        eb->argmax_stage[k] = best;
    }
    return true;
}

// One SDIRK stage as a 1-stage method: A = [gamma], b = [1], c = [c_i];
// one real block, eta = 1/gamma.
void build_sdirk_stage_block(double gamma, double ci, EigenBlocks *eb) {
    *eb = EigenBlocks();
    eb->s = 1;
    eb->nblocks = 1;
    eb->A[0] = gamma;
    eb->Ainv[0] = 1.0 / gamma;
    eb->b[0] = 1.0;
    eb->c[0] = ci;
    eb->T[0] = eb->Tinv[0] = 1.0;
    eb->TLam[0] = 1.0 / gamma;
    eb->width[0] = 1;
    eb->first[0] = 0;
    eb->eta[0] = 1.0 / gamma;
    eb->beta[0] = 0.0;
    eb->gamma_star[0] = 1.0 / gamma;
    eb->c12[0] = eb->c21[0] = 0.0;
    eb->R[0] = 1.0 / gamma;
    eb->argmax_stage[0] = 0;
}

bool build_eigen_blocks(int family, int s, EigenBlocks *eb) {
    if (family == IRK_SDIRK) return false;         // stages are sequential, no eigenbasis
    ld A[IRK_MAX_STAGES * IRK_MAX_STAGES], b[IRK_MAX_STAGES], c[IRK_MAX_STAGES];
    if (!build_tableau_ld(family, s, A, b, c)) return false;
    ld Ai[IRK_MAX_STAGES * IRK_MAX_STAGES];
    if (!invert_ld(s, A, Ai)) return false;
    for (int i = 0; i < s * s; ++i) { eb->A[i] = (double)A[i]; eb->Ainv[i] = (double)Ai[i]; }
    for (int i = 0; i < s; ++i) { eb->b[i] = (double)b[i]; eb->c[i] = (double)c[i]; }
    eb->s = s;

    std::vector<cld> lam = s == 1 ? std::vector<cld>{cld(Ai[0])} : aberth(charpoly(s, Ai));
    std::vector<ld> reals;
    std::vector<cld> ups;                                   // eigenvalues with Im > 0
    for (auto &l : lam) {
        if (fabsl(l.imag()) < 1e-12L * std::max((ld)1, std::abs(l))) reals.push_back(l.real());
        else if (l.imag() > 0) ups.push_back(l);
    }
    std::sort(reals.begin(), reals.end());
    std::sort(ups.begin(), ups.end(), [](const cld &x, const cld &y) { return x.imag() > y.imag(); });
    if ((int)(reals.size() + 2 * ups.size()) != s) return false;

    ld T[IRK_MAX_STAGES * IRK_MAX_STAGES] = {0};
    int row = 0, nb = 0;
    for (ld lr : reals) {
        std::vector<cld> v = null_vector(s, Ai, cld(lr));
        ld nrm = 0, big = 0;
        int ib = 0;
        for (int i = 0; i < s; ++i) { nrm += std::norm(v[i]); if (fabsl(v[i].real()) > big) { big = fabsl(v[i].real()); ib = i; } }
        ld sg = v[ib].real() < 0 ? -1.0L : 1.0L;
        for (int i = 0; i < s; ++i) T[i * s + row] = sg * v[i].real() / sqrtl(nrm);
        eb->width[nb] = 1; eb->eta[nb] = (double)lr; eb->beta[nb] = 0.0; eb->first[nb] = row;
        ++nb; ++row;
    }
    for (cld l : ups) {
        std::vector<cld> v = null_vector(s, Ai, l);
        ld nrm = 0;
        for (int i = 0; i < s; ++i) nrm += std::norm(v[i]);
        for (int i = 0; i < s; ++i) v[i] /= sqrtl(nrm);
        // phase: Re v orthogonal to Im v, |Re v| >= |Im v|
        ld aa = 0, bb = 0, ab = 0;
        for (int i = 0; i < s; ++i) { aa += v[i].real() * v[i].real(); bb += v[i].imag() * v[i].imag(); ab += v[i].real() * v[i].imag(); }
        ld th = 0.5L * atan2l(-2.0L * ab, aa - bb);
        cld rot = std::polar((ld)1, th);
        for (int i = 0; i < s; ++i) v[i] *= rot;
        aa = bb = 0;
        for (int i = 0; i < s; ++i) { aa += v[i].real() * v[i].real(); bb += v[i].imag() * v[i].imag(); }
        if (bb > aa) for (int i = 0; i < s; ++i) v[i] *= cld(0, 1);   // quarter turn
        int ib = 0;
        ld big = 0;
        for (int i = 0; i < s; ++i) if (fabsl(v[i].real()) > big) { big = fabsl(v[i].real()); ib = i; }
        if (v[ib].real() < 0) for (int i = 0; i < s; ++i) v[i] = -v[i];
        for (int i = 0; i < s; ++i) { T[i * s + row] = v[i].real(); T[i * s + row + 1] = v[i].imag(); }
        eb->width[nb] = 2; eb->eta[nb] = (double)l.real(); eb->beta[nb] = (double)l.imag(); eb->first[nb] = row;
        ++nb; row += 2;
    }
    eb->nblocks = nb;
    ld Ti[IRK_MAX_STAGES * IRK_MAX_STAGES];
    if (!invert_ld(s, T, Ti)) return false;
    // Lambda (block diagonal) and T Lambda, used for the stage update
    ld Lam[IRK_MAX_STAGES * IRK_MAX_STAGES] = {0};
    for (int k = 0; k < nb; ++k) {
        int r = eb->first[k];
        ld e = eb->eta[k], bt = eb->beta[k];
        Lam[r * s + r] = e;
        if (eb->width[k] == 2) {
            Lam[r * s + r + 1] = bt; Lam[(r + 1) * s + r] = -bt; Lam[(r + 1) * s + r + 1] = e;
        }
        eb->c12[k] = (double)bt;
        eb->c21[k] = (double)-bt;
        eb->gamma_star[k] = (double)(e + bt * bt / e);
    }
    for (int i = 0; i < s * s; ++i) eb->R[i] = (double)Lam[i];
    for (int i = 0; i < s; ++i)
        for (int j = 0; j < s; ++j) {
            ld tl = 0;
            for (int q = 0; q < s; ++q) tl += T[i * s + q] * Lam[q * s + j];
            eb->TLam[i * s + j] = (double)tl;
            eb->T[i * s + j] = (double)T[i * s + j];
            eb->Tinv[i * s + j] = (double)Ti[i * s + j];
        }
    // d weights d[k][l][i] = Tinv[k][i] T[i][l] (equation (Q0approx)), and the
    // stage Newton-like (1) lumps each diagonal weight vector to: the lowest
    // stage index whose |d_kk,i| is within a relative 1e-12 of the largest.
    // The real eigenvalue's row of Gauss (odd s) and of 3-stage Lobatto IIIC
    // has its two largest weights equal (d_kk,i = d_kk,s-1-i), so a plain
    // argmax would pick the stage by rounding.
    for (int k = 0; k < s; ++k) {
        ld dk[IRK_MAX_STAGES], big = 0;
        for (int i = 0; i < s; ++i) {
            dk[i] = fabsl(Ti[k * s + i] * T[i * s + k]);
            if (dk[i] > big) big = dk[i];
        }
        int best = 0;
        while (best + 1 < s && dk[best] < big * (1.0L - 1e-12L)) ++best;
        eb->argmax_stage[k] = best;
    }
    return true;
}

}  // namespace irk

extern "C" irk_status irk_tableau(irk_family family, int s, double *A, double *b, double *c) {
    if (!A || !b || !c || s < 1 || s > IRK_MAX_STAGES) return IRK_E_ARG;
    long double Al[IRK_MAX_STAGES * IRK_MAX_STAGES], bl[IRK_MAX_STAGES], cl[IRK_MAX_STAGES];
    if (!irk::build_tableau_ld(family, s, Al, bl, cl)) return IRK_E_ARG;
    for (int i = 0; i < s * s; ++i) A[i] = (double)Al[i];
    for (int i = 0; i < s; ++i) { b[i] = (double)bl[i]; c[i] = (double)cl[i]; }
    return IRK_OK;
}

extern "C" irk_status irk_eigen_blocks(irk_family family, int s, double *T, double *Tinv,
                                       int *nblocks, int *width, double *eta, double *beta,
                                       double *gamma_star, int *first_row) {
    if (!T || !Tinv || !nblocks || !width || !eta || !beta || !gamma_star || !first_row) return IRK_E_ARG;
    irk::EigenBlocks eb;
    if (!irk::build_eigen_blocks(family, s, &eb)) return IRK_E_ARG;
    std::memcpy(T, eb.T, sizeof(double) * s * s);
    std::memcpy(Tinv, eb.Tinv, sizeof(double) * s * s);
    *nblocks = eb.nblocks;
    for (int k = 0; k < eb.nblocks; ++k) {
        width[k] = eb.width[k]; eta[k] = eb.eta[k]; beta[k] = eb.beta[k];
        gamma_star[k] = eb.gamma_star[k]; first_row[k] = eb.first[k];
    }
    return IRK_OK;
}

extern "C" irk_status irk_schur_blocks(irk_family family, int s, double *Q0, double *R0) {
    if (!Q0 || !R0 || s < 1 || s > IRK_MAX_STAGES) return IRK_E_ARG;
    irk::EigenBlocks eb;
    if (!irk::build_schur_blocks(family, s, &eb)) return IRK_E_ARG;
    std::memcpy(Q0, eb.T, sizeof(double) * s * s);
    std::memcpy(R0, eb.R, sizeof(double) * s * s);
    return IRK_OK;
}
