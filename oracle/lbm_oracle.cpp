/*
 * lbm_oracle.cpp -- plain FP64 CPU reference of the thermal lattice Boltzmann method with
 * characteristic (LODI / CBC) non-reflecting boundaries of Klass, Gabbana & Bartel,
 * "Characteristic Boundary Condition for Thermal Lattice Boltzmann Methods" (arXiv 2307.16766).
 *
 * TEST INFRASTRUCTURE.  This is the oracle that the GPU library is checked against.  Only the
 * test-suite, the package smoke check and the CPU-baseline leg of the benchmark may load it.
 * It shares no source, header, table or constant generator with the GPU library: it derives
 * its own lattice constants (isotropy solve), builds the Hermite equilibrium from its tensor
 * definition, and builds the characteristic matrices explicitly.
 *
 * Every step is a separate, unfused pass over plain std::vector storage, in the order of the
 * paper's LBM flowchart (Sec. 2, Fig. "flowchart-lbm-algo") and the CBC flowchart
 * (Sec. 3.3, Fig. "flowchart-cbc-lbm"):
 *     stream -> macroscopic fields -> collide -> characteristic boundary solve (RK4)
 *     -> mesoscopic Dirichlet reconstruction.
 * The state kept between steps is the post-collision population field, the macroscopic field
 * (boundary nodes hold the boundary solver's values), and the pre-collision populations of
 * the last step (needed for the viscous terms, which are frozen at the old time level).
 *
 * The solver is a template over the scalar type: `double` for values and `Dual` (value plus
 * NTAN forward-mode tangents) for directional derivatives used to check the GPU adjoint.
 *
 * Readings of the paper that this file adopts (each also listed in the design notes):
 *  - 4th-order equilibrium: the Hermite expansion of the Maxwellian in the scaled variables
 *    xi = c/cs, u/cs, theta = T (dimensionless, T0 = 1); the printed (c^2-4) factor of the
 *    (u.c)^2 (T-1) term of eq. feq-4 is (xi^2-6) in this expansion.
 *  - Lattice constants: the D2Q37 weights are solved from the isotropy conditions up to
 *    degree 9 (Appendix B table is given to 14 digits only), the D2Q17 weights up to degree 7
 *    (they equal the closed forms of Tab. d2q17; the caption's expression is 1/cs).  D2Q17 uses
 *    the 3rd-order equilibrium of eq. feq-3, D2Q37 the 4th-order one of eq. feq-4.
 *  - Matrix S (Sec. 3.1): entry S_41 carries cs^2, not cs (S S^-1 = I only then).
 *  - Non-equilibrium part f^neq = f - f^eq (eq. NEEP); viscous stress
 *    Pi' = -(1 - 1/(2 tau)) sum c c f^neq (eq. LaplaceU); physical heat flux
 *    q = (1 - 1/(2 tau)) 1/2 sum f |c-u|^2 (c-u) (eq. LaplaceT with the same factor).
 *  - Where the mesoscopic viscous terms are evaluated (Sec. 3.3, "Evaluation of viscous terms"):
 *    at x_f - M, the first bulk node whose pre-collision populations all streamed from bulk
 *    nodes, with the one-sided difference over x_f - M, x_f - M - 1, x_f - M - 2 and central
 *    differences along the side; the result serves every layer of the row.  At x_f itself (the
 *    paper's wording) the populations streamed in from the equilibrium layers carry no
 *    non-equilibrium part, and the one-sided difference across that deficit feeds back on the
 *    layers' state: CBC-RELAX with the equilibrium BC then grows without bound.
 *  - Relaxation (eq. LODI-Relax / CBC-Relax, Z = P, transverse target 0) acts on the incoming
 *    acoustic amplitude only: -alpha T_x,i + K (P - P_inf) / (4 rho cs^2) (thermal) or
 *    -alpha T_x,i + K (P - P_inf) (isothermal), K = sigma (1 - Ma^2) c_inf / L.  Incoming
 *    entropy and shear waves keep the annihilation value of their scheme.
 *  - Viscous terms of the -FD variant (Sec. 4.2, "Treatment of viscous terms"): nu lap(u) and
 *    (nu c_p / (Pr cs^2)) lap(T~) by second differences of the macroscopic values of each layer
 *    (backward four-point formula at the outermost layer, central elsewhere and along the side),
 *    plus the viscous heating of eq. NSF-CHAR from first differences; unlike the mesoscopic
 *    terms they are evaluated from the stage values at every RK4 stage.
 *  - RK4 (Sec. 3.3 "Time integration"): wave directions and viscous terms frozen at time t,
 *    bulk values linearly interpolated in time, all layers and rows of a side advanced as
 *    one coupled system.
 *  - Corners (Sec. 3.3 "corner treatment"): one LODI analysis along the outward diagonal at
 *    the innermost corner node, one-sided second-order difference through the two inward
 *    diagonal bulk nodes; the result is copied to the M x M corner block; corners are
 *    advanced before the straight sides, which see corner values interpolated in time.
 *  - Equilibrium Dirichlet reconstruction replaces all q populations on all M layers.
 *
 * Pins of the boundary solve (tests/test_oracle_boundary_solve.py, test_oracle_characteristic.py):
 * the RK4 step of a side and of a corner equals the degree-4 Taylor polynomial of the exact
 * solution of the linearised layer system with linearly interpolated bulk values; the transverse
 * terms equal the tangential flux Jacobian times the tangential derivatives; the end rows of a
 * side see the corner block's value as their neighbour beyond the end (at t and t + dt
 * interpolated like bulk values); the diagonal corner analysis and the M x M block copy directly.
 */
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------- forward-mode dual number
constexpr int NTAN = 3;

struct Dual {
    double v;
    double d[NTAN];
    Dual() : v(0.0) { for (double& x : d) x = 0.0; }
    Dual(double a) : v(a) { for (double& x : d) x = 0.0; }  // NOLINT: implicit on purpose
};
inline Dual operator+(Dual a, const Dual& b) { a.v += b.v; for (int k = 0; k < NTAN; ++k) a.d[k] += b.d[k]; return a; }
inline Dual operator-(Dual a, const Dual& b) { a.v -= b.v; for (int k = 0; k < NTAN; ++k) a.d[k] -= b.d[k]; return a; }
inline Dual operator-(Dual a) { a.v = -a.v; for (int k = 0; k < NTAN; ++k) a.d[k] = -a.d[k]; return a; }
inline Dual operator*(const Dual& a, const Dual& b) {
    Dual r; r.v = a.v * b.v;
    for (int k = 0; k < NTAN; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
    return r;
}
inline Dual operator/(const Dual& a, const Dual& b) {
    Dual r; r.v = a.v / b.v;
    for (int k = 0; k < NTAN; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v);
    return r;
}
inline Dual& operator+=(Dual& a, const Dual& b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, const Dual& b) { a = a - b; return a; }
inline Dual& operator*=(Dual& a, const Dual& b) { a = a * b; return a; }
inline Dual operator+(double a, const Dual& b) { return Dual(a) + b; }
inline Dual operator-(double a, const Dual& b) { return Dual(a) - b; }
inline Dual operator*(double a, const Dual& b) { return Dual(a) * b; }
inline Dual operator/(double a, const Dual& b) { return Dual(a) / b; }
inline Dual operator+(const Dual& a, double b) { return a + Dual(b); }
inline Dual operator-(const Dual& a, double b) { return a - Dual(b); }
inline Dual operator*(const Dual& a, double b) { return a * Dual(b); }
inline Dual operator/(const Dual& a, double b) { return a / Dual(b); }
inline Dual sqrt(const Dual& a) {
    Dual r; r.v = std::sqrt(a.v);
    for (int k = 0; k < NTAN; ++k) r.d[k] = a.d[k] / (2.0 * r.v);
    return r;
}
inline double value(double x) { return x; }
inline double value(const Dual& x) { return x.v; }
using std::sqrt;

// ---------------------------------------------------------------- lattice (Appendix B)
struct Lattice {
    int stencil = 0, q = 0, M = 0;
    bool thermal = false;
    int order = 0;          // order of the Hermite expansion of the equilibrium
    double cs2 = 0, cs = 0;
    std::vector<int> cx, cy;
    std::vector<double> w;
    // Hermite tensor polynomials of xi = c / cs, flattened row-major, per population.
    std::vector<double> h1, h2, h3, h4;
};

// All members of a fully symmetric velocity group (Appendix B notation: (a,b) stands for every
// sign and axis permutation of the pair).
static std::vector<std::pair<int, int>> group_members(int a, int b) {
    std::vector<std::pair<int, int>> out;
    const int base[2][2] = {{a, b}, {b, a}};
    for (auto& pq : base)
        for (int sp : {1, -1})
            for (int sq : {1, -1}) {
                std::pair<int, int> m(sp * pq[0], sq * pq[1]);
                if (std::find(out.begin(), out.end(), m) == out.end()) out.push_back(m);
            }
    std::sort(out.begin(), out.end());
    return out;
}

static long double dfact(int n) { long double r = 1; while (n > 1) { r *= n; n -= 2; } return r; }

// Gauss-Hermite isotropy condition: sum_i w_i c_x^(2a) c_y^(2b) = (2a-1)!! (2b-1)!! cs^(2(a+b)).
// `lin` pairs are solved as a linear system for the group weights at a given cs^2; the `chk`
// pair is the remaining condition, whose root fixes cs^2 (Sec. 2: quadrature of the given order).
struct IsoProblem {
    std::vector<std::pair<int, int>> groups, lin;
    std::pair<int, int> chk;
};

static long double group_moment(const std::pair<int, int>& g, int a, int b) {
    long double s = 0;
    for (auto& m : group_members(g.first, g.second)) {
        long double t = 1;
        for (int k = 0; k < 2 * a; ++k) t *= m.first;
        for (int k = 0; k < 2 * b; ++k) t *= m.second;
        s += t;
    }
    return s;
}

static std::vector<long double> solve_weights(const IsoProblem& P, long double s) {
    const int n = (int)P.groups.size();
    std::vector<long double> A(n * (n + 1));
    for (int r = 0; r < n; ++r) {
        const int a = P.lin[r].first, b = P.lin[r].second;
        for (int c = 0; c < n; ++c) A[r * (n + 1) + c] = group_moment(P.groups[c], a, b);
        A[r * (n + 1) + n] = dfact(2 * a - 1) * dfact(2 * b - 1) * std::pow(s, (long double)(a + b));
    }
    for (int c = 0; c < n; ++c) {  // Gaussian elimination, partial pivoting
        int p = c;
        for (int r = c + 1; r < n; ++r) if (std::fabs(A[r * (n + 1) + c]) > std::fabs(A[p * (n + 1) + c])) p = r;
        for (int k = 0; k <= n; ++k) std::swap(A[c * (n + 1) + k], A[p * (n + 1) + k]);
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            long double f = A[r * (n + 1) + c] / A[c * (n + 1) + c];
            for (int k = c; k <= n; ++k) A[r * (n + 1) + k] -= f * A[c * (n + 1) + k];
        }
    }
    std::vector<long double> wg(n);
    for (int r = 0; r < n; ++r) wg[r] = A[r * (n + 1) + n] / A[r * (n + 1) + r];
    return wg;
}

static long double iso_residual(const IsoProblem& P, long double s) {
    auto wg = solve_weights(P, s);
    long double m = 0;
    for (size_t g = 0; g < P.groups.size(); ++g) m += wg[g] * group_moment(P.groups[g], P.chk.first, P.chk.second);
    const int a = P.chk.first, b = P.chk.second;
    return m - dfact(2 * a - 1) * dfact(2 * b - 1) * std::pow(s, (long double)(a + b));
}

static Lattice make_lattice(int stencil) {
    Lattice L;
    IsoProblem P;
    long double lo, hi;
    if (stencil == 9) {  // Tab. d2q9: single-speed, isothermal, 2nd-order equilibrium
        P.groups = {{0, 0}, {1, 0}, {1, 1}};
        P.lin = {{0, 0}, {1, 0}, {1, 1}};
        P.chk = {2, 0};
        lo = 0.2L; hi = 0.5L;
        L.M = 1; L.thermal = false; L.order = 2;
    } else if (stencil == 37) {  // Tab. d2q37: 9th-order quadrature, 4th-order equilibrium
        P.groups = {{0, 0}, {1, 0}, {1, 1}, {2, 0}, {2, 1}, {2, 2}, {3, 0}, {3, 1}};
        P.lin = {{0, 0}, {1, 0}, {2, 0}, {1, 1}, {3, 0}, {2, 1}, {3, 1}, {2, 2}};
        P.chk = {4, 0};
        lo = 0.65L; hi = 0.75L;
        L.M = 3; L.thermal = true; L.order = 4;
    } else if (stencil == 17) {  // Tab. d2q17: 7th-order quadrature, 3rd-order equilibrium
        P.groups = {{0, 0}, {1, 0}, {1, 1}, {2, 2}, {3, 0}};
        P.lin = {{0, 0}, {1, 0}, {2, 0}, {1, 1}, {3, 0}};
        P.chk = {2, 1};
        lo = 0.3L; hi = 0.45L;
        L.M = 3; L.thermal = true; L.order = 3;
    } else {
        return L;
    }
    // bisection on the remaining isotropy condition
    long double flo = iso_residual(P, lo);
    for (int it = 0; it < 200; ++it) {
        long double mid = 0.5L * (lo + hi);
        long double fm = iso_residual(P, mid);
        if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else { hi = mid; }
        if (hi - lo < 1e-21L) break;
    }
    const long double s = 0.5L * (lo + hi);
    auto wg = solve_weights(P, s);
    L.stencil = stencil;
    L.cs2 = (double)s;
    L.cs = (double)std::sqrt(s);
    for (size_t g = 0; g < P.groups.size(); ++g)
        for (auto& m : group_members(P.groups[g].first, P.groups[g].second)) {
            L.cx.push_back(m.first);
            L.cy.push_back(m.second);
            L.w.push_back((double)wg[g]);
        }
    L.q = (int)L.w.size();
    // Hermite tensor polynomials H^(n)(xi) (probabilists' convention, unit variance)
    auto del = [](int a, int b) { return a == b ? 1.0 : 0.0; };
    for (int i = 0; i < L.q; ++i) {
        const double xi[2] = {L.cx[i] / L.cs, L.cy[i] / L.cs};
        for (int a = 0; a < 2; ++a) L.h1.push_back(xi[a]);
        for (int a = 0; a < 2; ++a) for (int b = 0; b < 2; ++b) L.h2.push_back(xi[a] * xi[b] - del(a, b));
        for (int a = 0; a < 2; ++a) for (int b = 0; b < 2; ++b) for (int c = 0; c < 2; ++c)
            L.h3.push_back(xi[a] * xi[b] * xi[c] - (xi[a] * del(b, c) + xi[b] * del(a, c) + xi[c] * del(a, b)));
        for (int a = 0; a < 2; ++a) for (int b = 0; b < 2; ++b) for (int c = 0; c < 2; ++c) for (int e = 0; e < 2; ++e)
            L.h4.push_back(xi[a] * xi[b] * xi[c] * xi[e]
                           - (xi[a] * xi[b] * del(c, e) + xi[a] * xi[c] * del(b, e) + xi[a] * xi[e] * del(b, c)
                              + xi[b] * xi[c] * del(a, e) + xi[b] * xi[e] * del(a, c) + xi[c] * xi[e] * del(a, b))
                           + (del(a, b) * del(c, e) + del(a, c) * del(b, e) + del(a, e) * del(b, c)));
    }
    return L;
}

static const Lattice& lattice(int stencil) {
    static const Lattice L9 = make_lattice(9);
    static const Lattice L17 = make_lattice(17);
    static const Lattice L37 = make_lattice(37);
    return stencil == 9 ? L9 : (stencil == 17 ? L17 : L37);
}

// ---------------------------------------------------------------- equilibrium (eq. feq-3/feq-4)
// Hermite expansion of the Maxwellian: f_i^eq = w_i rho sum_n a^(n) : H^(n)(xi_i) / n!, with the
// coefficients a^(1) = u, a^(2) = uu + th d, a^(3) = uuu + th (d u)_sym,
// a^(4) = uuuu + th (d uu)_sym + th^2 (d d)_sym, u in units of cs and th = T - 1.
template <class S>
static void equilibrium(const Lattice& L, const S& rho, const S& ux, const S& uy, const S& T, S* out) {
    const S u[2] = {ux / L.cs, uy / L.cs};
    const S th = L.thermal ? T - 1.0 : S(0.0);
    auto del = [](int a, int b) { return a == b ? 1.0 : 0.0; };
    S a2[4], a3[8], a4[16];
    for (int a = 0; a < 2; ++a) for (int b = 0; b < 2; ++b) a2[a * 2 + b] = u[a] * u[b] + th * del(a, b);
    for (int a = 0; a < 2; ++a) for (int b = 0; b < 2; ++b) for (int c = 0; c < 2; ++c)
        a3[(a * 2 + b) * 2 + c] = u[a] * u[b] * u[c] + th * (u[a] * del(b, c) + u[b] * del(a, c) + u[c] * del(a, b));
    for (int a = 0; a < 2; ++a) for (int b = 0; b < 2; ++b) for (int c = 0; c < 2; ++c) for (int e = 0; e < 2; ++e)
        a4[((a * 2 + b) * 2 + c) * 2 + e] =
            u[a] * u[b] * u[c] * u[e]
            + th * (u[a] * u[b] * del(c, e) + u[a] * u[c] * del(b, e) + u[a] * u[e] * del(b, c)
                    + u[b] * u[c] * del(a, e) + u[b] * u[e] * del(a, c) + u[c] * u[e] * del(a, b))
            + th * th * (del(a, b) * del(c, e) + del(a, c) * del(b, e) + del(a, e) * del(b, c));
    for (int i = 0; i < L.q; ++i) {
        S s1 = u[0] * L.h1[2 * i] + u[1] * L.h1[2 * i + 1];
        S s2 = 0.0, s3 = 0.0, s4 = 0.0;
        for (int k = 0; k < 4; ++k) s2 += a2[k] * L.h2[4 * i + k];
        if (L.order >= 3) for (int k = 0; k < 8; ++k) s3 += a3[k] * L.h3[8 * i + k];
        if (L.order >= 4) for (int k = 0; k < 16; ++k) s4 += a4[k] * L.h4[16 * i + k];
        out[i] = L.w[i] * rho * (1.0 + s1 + s2 / 2.0 + s3 / 6.0 + s4 / 24.0);
    }
}

// Macroscopic moments (eq. macro): rho = sum f, rho u = sum f c, 2 rho e = sum f |c-u|^2 with
// e = (d/2) T~ = cs^2 T in d = 2 (T dimensionless).  Single-speed D2Q9 is isothermal: T = 1.
template <class S>
static void moments(const Lattice& L, const S* f, S& rho, S& ux, S& uy, S& T) {
    S r = 0.0, jx = 0.0, jy = 0.0;
    for (int i = 0; i < L.q; ++i) { r += f[i]; jx += f[i] * (double)L.cx[i]; jy += f[i] * (double)L.cy[i]; }
    rho = r; ux = jx / r; uy = jy / r;
    if (L.thermal) {
        S e = 0.0;
        for (int i = 0; i < L.q; ++i) {
            S dx = (double)L.cx[i] - ux, dy = (double)L.cy[i] - uy;
            e += f[i] * (dx * dx + dy * dy);
        }
        T = e / (2.0 * r * L.cs2);
    } else {
        T = 1.0;
    }
}

// ---------------------------------------------------------------- characteristic system (Sec. 3.1)
// Local frame: U = (rho, u_n, u_t, T) (thermal, n = 4) or (rho, u_n, u_t) (isothermal, n = 3),
// n the outward normal.  Wave order (thermal): entropy (u_n), shear (u_n), acoustic (u_n - s),
// acoustic (u_n + s), s = sqrt(2 cs^2 T).  Isothermal: shear (u_n), acoustic (u_n - cs),
// acoustic (u_n + cs).
template <class S>
struct CharSys {
    int n;
    S A[16], Sm[16], Si[16], lam[4];
};

template <class S>
static CharSys<S> char_system(const Lattice& L, const S* U) {
    CharSys<S> c;
    for (int k = 0; k < 16; ++k) { c.A[k] = 0.0; c.Sm[k] = 0.0; c.Si[k] = 0.0; }
    const double cs2 = L.cs2;
    const S rho = U[0], un = U[1];
    if (L.thermal) {
        c.n = 4;
        const S T = U[3];
        const S Tt = cs2 * T;          // lattice temperature T~ = cs^2 T
        const S s = sqrt(2.0 * Tt);    // adiabatic sound speed, gamma = cp / cv = 2
        auto a = [&](int r, int k) -> S& { return c.A[r * 4 + k]; };
        auto m = [&](int r, int k) -> S& { return c.Sm[r * 4 + k]; };
        auto mi = [&](int r, int k) -> S& { return c.Si[r * 4 + k]; };
        a(0, 0) = un; a(0, 1) = rho;
        a(1, 0) = Tt / rho; a(1, 1) = un; a(1, 3) = cs2;
        a(2, 2) = un;
        a(3, 1) = Tt / cs2; a(3, 3) = un;
        const S r8 = sqrt(Tt / (8.0 * cs2 * cs2));
        m(0, 0) = -Tt / (2.0 * rho * cs2); m(0, 3) = 0.5;
        m(1, 2) = 1.0;
        m(2, 0) = Tt / (4.0 * rho * cs2); m(2, 1) = -r8; m(2, 3) = 0.25;
        m(3, 0) = Tt / (4.0 * rho * cs2); m(3, 1) = r8; m(3, 3) = 0.25;
        const S r2 = sqrt(2.0 * cs2 * cs2 / Tt);
        mi(0, 0) = -rho * cs2 / Tt; mi(0, 2) = rho * cs2 / Tt; mi(0, 3) = rho * cs2 / Tt;
        mi(1, 2) = -r2; mi(1, 3) = r2;
        mi(2, 1) = 1.0;
        mi(3, 0) = 1.0; mi(3, 2) = 1.0; mi(3, 3) = 1.0;
        c.lam[0] = un; c.lam[1] = un; c.lam[2] = un - s; c.lam[3] = un + s;
    } else {
        c.n = 3;
        const double cs = L.cs;
        auto a = [&](int r, int k) -> S& { return c.A[r * 3 + k]; };
        auto m = [&](int r, int k) -> S& { return c.Sm[r * 3 + k]; };
        auto mi = [&](int r, int k) -> S& { return c.Si[r * 3 + k]; };
        a(0, 0) = un; a(0, 1) = rho;
        a(1, 0) = cs2 / rho; a(1, 1) = un;
        a(2, 2) = un;
        m(0, 2) = 1.0;
        m(1, 0) = cs2; m(1, 1) = -rho * cs;
        m(2, 0) = cs2; m(2, 1) = rho * cs;
        mi(0, 1) = 1.0 / (2.0 * cs2); mi(0, 2) = 1.0 / (2.0 * cs2);
        mi(1, 1) = -1.0 / (2.0 * rho * cs); mi(1, 2) = 1.0 / (2.0 * rho * cs);
        mi(2, 0) = 1.0;
        c.lam[0] = un; c.lam[1] = un - cs; c.lam[2] = un + cs;
    }
    return c;
}

template <class S>
static void matvec(int n, const S* M, const S* x, S* y) {
    for (int r = 0; r < n; ++r) { S s = 0.0; for (int k = 0; k < n; ++k) s += M[r * n + k] * x[k]; y[r] = s; }
}

// ---------------------------------------------------------------- simulation
enum { BC_PERIODIC = 0, BC_LODI = 1, BC_LODI_RELAX = 2, BC_CBC = 3, BC_CBC_RELAX = 4, BC_ZG = 5, BC_DIRICHLET = 6 };
inline bool is_char(int b) { return b >= BC_LODI && b <= BC_CBC_RELAX; }
inline bool is_relax(int b) { return b == BC_LODI_RELAX || b == BC_CBC_RELAX; }
inline bool is_full_cbc(int b) { return b == BC_CBC || b == BC_CBC_RELAX; }

std::string g_err;

template <class S>
struct Relax {
    S sigma = 0.0, alpha = 0.0;
    double rho_inf = 1.0, T_inf = 1.0, mach = 0.0, length = 0.0;
};

// Geometry of one straight side in its local frame: k is the outward index (k = 0 is the
// adjacent bulk node x_f, k = j = 1..M the boundary layers x_{b,j}), r the row along the side.
struct SideGeo {
    int side = 0, nax = 0, sn = 1, Nn = 0, Nt = 0, r0 = 0, len = 0, xf = 0;
    bool tper = false;
};

template <class S>
struct Sim {
    const Lattice& L;
    int nx, ny, q, M;
    double tau;
    int bc[4];
    bool xper, yper;
    SideGeo geo[4];
    Relax<S> rp[4];
    std::vector<S> inlet[4];   // Dirichlet profiles [len][4]
    int meso[4] = {0, 0, 0, 0};   // mesoscopic BC of a characteristic side: 0 equilibrium, 1 NEEP
    int vfd[4] = {0, 0, 0, 0};    // viscous terms of a CBC side: 0 mesoscopic moments, 1 differences
    std::vector<S> f, fpre, U;  // f, fpre: [q][ny][nx]; U: [4][ny][nx]
    long steps = 0;

    Sim(const Lattice& lat, int nx_, int ny_, double tau_, const int* bc_)
        : L(lat), nx(nx_), ny(ny_), q(lat.q), M(lat.M), tau(tau_) {
        for (int s = 0; s < 4; ++s) bc[s] = bc_[s];
        xper = bc[0] == BC_PERIODIC;
        yper = bc[2] == BC_PERIODIC;
        for (int s = 0; s < 4; ++s) {
            SideGeo& g = geo[s];
            g.side = s;
            g.nax = s < 2 ? 0 : 1;
            g.sn = (s % 2 == 0) ? -1 : 1;
            g.Nn = g.nax == 0 ? nx : ny;
            g.Nt = g.nax == 0 ? ny : nx;
            g.tper = g.nax == 0 ? yper : xper;
            g.r0 = g.tper ? 0 : M;
            g.len = g.tper ? g.Nt : g.Nt - 2 * M;
            g.xf = g.sn > 0 ? g.Nn - 1 - M : M;
        }
        f.assign((size_t)q * nx * ny, S(0.0));
        fpre = f;
        U.assign((size_t)4 * nx * ny, S(0.0));
        for (int s = 0; s < 4; ++s) inlet[s].assign((size_t)geo[s].len * 4, S(0.0));
    }

    size_t id(int x, int y) const { return (size_t)y * nx + x; }
    size_t plane() const { return (size_t)nx * ny; }
    bool is_bulk(int x, int y) const {
        return (xper || (x >= M && x <= nx - 1 - M)) && (yper || (y >= M && y <= ny - 1 - M));
    }
    void node(const SideGeo& g, int k, int r, int& x, int& y) const {
        int nc = g.xf + g.sn * k;
        int tc = g.r0 + r;
        if (g.tper) tc = ((tc % g.Nt) + g.Nt) % g.Nt;
        if (g.nax == 0) { x = nc; y = tc; } else { x = tc; y = nc; }
    }
    void getU(const std::vector<S>& F, int x, int y, S* u4) const {
        for (int c = 0; c < 4; ++c) u4[c] = F[c * plane() + id(x, y)];
    }
    void setU(std::vector<S>& F, int x, int y, const S* u4) const {
        for (int c = 0; c < 4; ++c) F[c * plane() + id(x, y)] = u4[c];
    }
    void node_feq(std::vector<S>& F, int x, int y, const S* u4) const {
        std::vector<S> fe(q);
        equilibrium(L, u4[0], u4[1], u4[2], u4[3], fe.data());
        for (int i = 0; i < q; ++i) F[i * plane() + id(x, y)] = fe[i];
    }
    void node_moments(const std::vector<S>& F, int x, int y, S* u4) const {
        std::vector<S> fl(q);
        for (int i = 0; i < q; ++i) fl[i] = F[i * plane() + id(x, y)];
        moments(L, fl.data(), u4[0], u4[1], u4[2], u4[3]);
    }

    // initial state: f = f^eq(fields) at every node (Sec. 2, "Initialize")
    // dT: seeded temperature [ny][nx]; dF: seeded (rho, ux, uy, T) [4][ny][nx] (either or none)
    void init(const double* rho, const double* ux, const double* uy, const double* T, const std::vector<S>* dT,
              const std::vector<S>* dF = nullptr) {
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                S u4[4] = {rho[id(x, y)], ux[id(x, y)], uy[id(x, y)], L.thermal ? S(T[id(x, y)]) : S(1.0)};
                if (dT && L.thermal) u4[3] = (*dT)[id(x, y)];
                if (dF)
                    for (int c = 0; c < (L.thermal ? 4 : 3); ++c) u4[c] = (*dF)[c * plane() + id(x, y)];
                setU(U, x, y, u4);
                node_feq(f, x, y, u4);
            }
        // Dirichlet sides: the default profile is the initial state of the first layer, and a
        // profile takes effect when it is set: every layer of the row holds its equilibrium from
        // time 0 on (as with an explicit profile, oracle_set_inlet)
        for (int s = 0; s < 4; ++s) {
            if (bc[s] != BC_DIRICHLET) continue;
            const SideGeo& g = geo[s];
            for (int r = 0; r < g.len; ++r) {
                int x, y; node(g, 1, r, x, y);
                S u4[4]; getU(U, x, y, u4);
                for (int c = 0; c < 4; ++c) inlet[s][r * 4 + c] = u4[c];
                for (int j = 2; j <= M; ++j) {
                    int xj, yj; node(g, j, r, xj, yj);
                    setU(U, xj, yj, u4);
                    node_feq(f, xj, yj, u4);
                }
            }
        }
        fpre = f;
        steps = 0;
    }

    // -------------------------------------------------- viscous data (Sec. 3.3, eq. LaplaceU/LaplaceT)
    // Pi' (nn, nt, tt), q (n, t) and rho at a node, in side-local components, from the
    // pre-collision populations of the current time level.  Boundary nodes hold equilibria, whose
    // non-equilibrium moments vanish: zero is returned for them.
    void visc_node(const SideGeo& g, int x, int y, S* out6) const {
        for (int c = 0; c < 6; ++c) out6[c] = 0.0;
        if (!is_bulk(x, y)) return;
        std::vector<S> fl(q), fe(q);
        for (int i = 0; i < q; ++i) fl[i] = fpre[i * plane() + id(x, y)];
        S rho, ux, uy, T;
        moments(L, fl.data(), rho, ux, uy, T);
        equilibrium(L, rho, ux, uy, T, fe.data());
        const double fac = 1.0 - 1.0 / (2.0 * tau);
        S P[2][2] = {{0.0, 0.0}, {0.0, 0.0}}, Q[2] = {0.0, 0.0};
        for (int i = 0; i < q; ++i) {
            const double c[2] = {(double)L.cx[i], (double)L.cy[i]};
            S fn = fl[i] - fe[i];
            for (int a = 0; a < 2; ++a) for (int b = 0; b < 2; ++b) P[a][b] -= fac * c[a] * c[b] * fn;
            if (L.thermal) {
                S d0 = c[0] - ux, d1 = c[1] - uy;
                S e = fl[i] * (d0 * d0 + d1 * d1) * 0.5 * fac;
                Q[0] += e * d0; Q[1] += e * d1;
            }
        }
        const int a = g.nax, b = 1 - g.nax;
        out6[0] = rho;
        out6[1] = P[a][a];
        out6[2] = (double)g.sn * P[a][b];
        out6[3] = P[b][b];
        out6[4] = (double)g.sn * Q[a];
        out6[5] = Q[b];
    }

    // V (local components, eq. NSF-CHAR) at row r of a side, frozen at the old time level: the
    // divergence of Pi' and q at the bulk node kof nodes inward of x_f, one-sided along the normal
    // (eq. FD-dx-bw over that node and the next two inward) and central along the side
    // (eq. FD-dx-center), plus the viscous heating Pi':grad u = Pi':Pi' / mu.  The side solve
    // takes kof = M: x_f - M is the first node none of whose populations streamed from the
    // layers (with the equilibrium BC those carry no non-equilibrium part).
    void visc_row(const SideGeo& g, int r, S* V4, int kof) const {
        const double nu = (tau - 0.5) * L.cs2;
        S d[3][6], up[6], dn[6];
        for (int k = 0; k < 3; ++k) { int x, y; node(g, -kof - k, r, x, y); visc_node(g, x, y, d[k]); }
        int x, y;
        if (g.tper || r + 1 < g.len) { node(g, -kof, r + 1, x, y); visc_node(g, x, y, up); }
        else { for (auto& v : up) v = 0.0; }
        if (g.tper || r - 1 >= 0) { node(g, -kof, r - 1, x, y); visc_node(g, x, y, dn); }
        else { for (auto& v : dn) v = 0.0; }
        auto dn_ = [&](int c) { return 0.5 * (3.0 * d[0][c] - 4.0 * d[1][c] + d[2][c]); };
        auto dt_ = [&](int c) { return 0.5 * (up[c] - dn[c]); };
        const S rho = d[0][0];
        V4[0] = 0.0;
        V4[1] = (dn_(1) + dt_(2)) / rho;
        V4[2] = (dn_(2) + dt_(3)) / rho;
        V4[3] = 0.0;
        if (L.thermal) {
            const S heat = (0.5 * (d[0][1] * d[0][1] + d[0][3] * d[0][3]) + d[0][2] * d[0][2]) / (rho * rho * nu * L.cs2);
            V4[3] = -(dn_(4) + dt_(5)) / (rho * L.cs2) + heat;
        }
    }

    void visc_terms(const SideGeo& g, std::vector<S>& V) const {
        V.assign((size_t)g.len * 4, S(0.0));
        for (int r = 0; r < g.len; ++r) visc_row(g, r, &V[(size_t)r * 4], M);
    }

    // -------------------------------------------------- frames
    void to_local(int nax, int sn, const S* u4, S* l) const {
        l[0] = u4[0];
        l[1] = (double)sn * u4[1 + nax];
        l[2] = u4[2 - nax];
        l[3] = u4[3];
    }
    void from_local_rate(int nax, int sn, const S* l, S* u4) const {
        u4[0] = l[0];
        u4[1 + nax] = (double)sn * l[1];
        u4[2 - nax] = l[2];
        u4[3] = L.thermal ? l[3] : S(0.0);
    }

    S relax_K(int s) const {
        const Relax<S>& p = rp[s];
        const double cinf = L.thermal ? std::sqrt(2.0 * L.cs2 * p.T_inf) : L.cs;
        const double Lg = p.length > 0 ? p.length : (double)geo[s].Nn;
        return p.sigma * ((1.0 - p.mach * p.mach) * cinf / Lg);
    }
    double P_inf(int s) const { return rp[s].rho_inf * L.cs2 * (L.thermal ? rp[s].T_inf : 1.0); }

    // amplitude that relaxes pressure toward P_inf when placed in an incoming acoustic wave
    S pressure_term(const S* loc, const S& K, double Pinf) const {
        if (L.thermal) {
            const S P = loc[0] * L.cs2 * loc[3];
            return K * (P - Pinf) / (4.0 * loc[0] * L.cs2);
        }
        const S P = loc[0] * L.cs2;
        return K * (P - Pinf);
    }
    bool acoustic(int i) const { return L.thermal ? (i >= 2) : (i >= 1); }

    // -------------------------------------------------- corners (Sec. 3.3, corner treatment)
    struct Corner { int sx, sy; bool active, zg; };
    Corner corner(int cidx) const {  // cidx: 0 = (x0,y0), 1 = (x1,y0), 2 = (x0,y1), 3 = (x1,y1)
        Corner c;
        c.sx = cidx & 1; c.sy = 2 + (cidx >> 1);
        c.active = !xper && !yper;
        c.zg = c.active && bc[c.sx] == BC_ZG;
        return c;
    }
    void corner_node(const Corner& c, int& x, int& y) const {
        x = geo[c.sx].xf + geo[c.sx].sn;
        y = geo[c.sy].xf + geo[c.sy].sn;
    }
    // corner LODI right-hand side along the outward diagonal
    void corner_rhs(const Corner& c, const S* Uc, const S* Ucn, const S* B1, const S* B2, S* dU) const {
        const double ndx = geo[c.sx].sn / std::sqrt(2.0), ndy = geo[c.sy].sn / std::sqrt(2.0);
        const double tdx = -ndy, tdy = ndx;
        auto loc = [&](const S* u, S* l) {
            l[0] = u[0]; l[1] = u[1] * ndx + u[2] * ndy; l[2] = u[1] * tdx + u[2] * tdy; l[3] = u[3];
        };
        S l0[4], l1[4], l2[4], ln[4];
        loc(Uc, l0); loc(B1, l1); loc(B2, l2); loc(Ucn, ln);
        const int n = L.thermal ? 4 : 3;
        S dU_n[4];
        for (int k = 0; k < 4; ++k) dU_n[k] = (3.0 * l0[k] - 4.0 * l1[k] + l2[k]) / (2.0 * std::sqrt(2.0));
        S vec[4];
        pack(l0, vec); S dv[4]; pack(dU_n, dv);
        CharSys<S> cs = char_system(L, vec);
        S vecn[4]; pack(ln, vecn);
        CharSys<S> csn = char_system(L, vecn);
        S Sd[4]; matvec(n, cs.Sm, dv, Sd);
        S Lb[4];
        const bool relax = is_relax(bc[c.sx]);
        const S K = relax ? relax_K(c.sx) : S(0.0);
        for (int i = 0; i < n; ++i) {
            if (value(csn.lam[i]) >= 0.0) Lb[i] = cs.lam[i] * Sd[i];
            else Lb[i] = (relax && acoustic(i)) ? pressure_term(l0, K, P_inf(c.sx)) : S(0.0);
        }
        S r[4]; matvec(n, cs.Si, Lb, r);
        S rl[4] = {0.0, 0.0, 0.0, 0.0};
        unpack_neg(r, rl);
        dU[0] = rl[0];
        dU[1] = rl[1] * ndx + rl[2] * tdx;
        dU[2] = rl[1] * ndy + rl[2] * tdy;
        dU[3] = L.thermal ? rl[3] : S(0.0);
    }
    // local (rho, un, ut, T) <-> state vector of the characteristic system
    void pack(const S* l, S* v) const { v[0] = l[0]; v[1] = l[1]; v[2] = l[2]; if (L.thermal) v[3] = l[3]; else v[3] = 0.0; }
    void unpack_neg(const S* v, S* l) const { l[0] = -v[0]; l[1] = -v[1]; l[2] = -v[2]; l[3] = L.thermal ? -v[3] : S(0.0); }

    // -------------------------------------------------- one straight side: coupled RK4
    struct SideCtx {
        const SideGeo* g;
        int s;
        const std::vector<S>* Y;    // stage values [M][len][4], layer j at index j-1
        const std::vector<S>* Y0;   // values at time t
        const std::vector<S>* Un;   // macroscopic field at t + dt (bulk filled)
        const std::vector<S>* V;    // viscous terms [len][4]
        const S* corner_lo[2];      // corner values (t, t + dt) at r = -1
        const S* corner_hi[2];      // corner values (t, t + dt) at r = len
        double theta;
    };

    void side_value(const SideCtx& c, int k, int r, S* u4) const {
        const SideGeo& g = *c.g;
        if (k >= 1) {
            if (r >= 0 && r < g.len) { for (int m = 0; m < 4; ++m) u4[m] = (*c.Y)[((size_t)(k - 1) * g.len + r) * 4 + m]; return; }
            if (g.tper) {
                int rr = ((r % g.len) + g.len) % g.len;
                for (int m = 0; m < 4; ++m) u4[m] = (*c.Y)[((size_t)(k - 1) * g.len + rr) * 4 + m];
                return;
            }
            const S* const* cv = r < 0 ? c.corner_lo : c.corner_hi;
            for (int m = 0; m < 4; ++m) u4[m] = (1.0 - c.theta) * cv[0][m] + c.theta * cv[1][m];
            return;
        }
        int x, y; node(g, k, r, x, y);
        S a[4], b[4];
        getU(U, x, y, a); getU(*c.Un, x, y, b);
        for (int m = 0; m < 4; ++m) u4[m] = (1.0 - c.theta) * a[m] + c.theta * b[m];
    }

    // V of the -FD variant (Sec. 4.2, treatment of viscous terms) at layer j, row r, from the
    // stage values: the Laplacians of eq. NSF-CHAR by second differences -- the backward
    // four-point formula at the outermost layer, the central one at inner layers and along the
    // side -- and the heating term from the first differences that the amplitudes use.
    void visc_fd(const SideCtx& c, int j, int r, S* Vv) const {
        const SideGeo& g = *c.g;
        auto lv = [&](int k, int rr, S* l) { S u4[4]; side_value(c, k, rr, u4); to_local(g.nax, g.sn, u4, l); };
        S l0[4], up[4], dw[4], dn[4], d2n[4], d2t[4], dtv[4];
        lv(j, r, l0); lv(j, r + 1, up); lv(j, r - 1, dw);
        if (j == M) {
            S a[4], bb[4], cc[4], dd[4]; lv(M - 1, r, bb); lv(M - 2, r, cc); lv(M - 3, r, dd);
            for (int m = 0; m < 4; ++m) a[m] = l0[m];
            for (int m = 0; m < 4; ++m) {
                d2n[m] = 2.0 * a[m] - 5.0 * bb[m] + 4.0 * cc[m] - dd[m];
                dn[m] = 0.5 * (3.0 * a[m] - 4.0 * bb[m] + cc[m]);
            }
        } else {
            S a[4], cc[4]; lv(j + 1, r, a); lv(j - 1, r, cc);
            for (int m = 0; m < 4; ++m) { d2n[m] = a[m] - 2.0 * l0[m] + cc[m]; dn[m] = 0.5 * (a[m] - cc[m]); }
        }
        for (int m = 0; m < 4; ++m) { d2t[m] = up[m] - 2.0 * l0[m] + dw[m]; dtv[m] = 0.5 * (up[m] - dw[m]); }
        const double nu = (tau - 0.5) * L.cs2;
        const double cp = 2.0, Pr = 1.0;   // c_p = d/2 + 1 in d = 2; BGK fixes Pr = 1
        Vv[0] = 0.0;
        Vv[1] = nu * (d2n[1] + d2t[1]);
        Vv[2] = nu * (d2n[2] + d2t[2]);
        Vv[3] = 0.0;
        if (L.thermal) {
            const S sa = dn[1] - dtv[2], sb = dtv[1] + dn[2];
            Vv[3] = (nu * cp / Pr) * (d2n[3] + d2t[3]) + (nu / L.cs2) * (sa * sa + sb * sb);
        }
    }

    // V of the -FD variant at time t for layer j (1..M), row r of side s, away from the ends
    // of a side with non-periodic rows
    void visc_fd_probe(int s, int j, int r, S* V4) {
        const SideGeo& g = geo[s];
        std::vector<S> Y0((size_t)M * g.len * 4);
        for (int jj = 1; jj <= M; ++jj)
            for (int rr = 0; rr < g.len; ++rr) {
                int x, y; node(g, jj, rr, x, y);
                getU(U, x, y, &Y0[((size_t)(jj - 1) * g.len + rr) * 4]);
            }
        SideCtx c;
        c.g = &g; c.s = s; c.Y = &Y0; c.Y0 = &Y0; c.Un = &U; c.V = nullptr;
        c.corner_lo[0] = c.corner_lo[1] = c.corner_hi[0] = c.corner_hi[1] = nullptr;
        c.theta = 0.0;
        visc_fd(c, j, r, V4);
    }

    // transverse terms T of eq. NSF-CHAR (local components) at layer j, row r: the tangential
    // flux derivatives, by central differences along the side (eq. FD-dx-center); at the end rows
    // of a side with non-periodic rows the neighbour beyond the end is the corner block's value
    void transverse(const SideCtx& c, int j, int r, S* Tv) const {
        const SideGeo& g = *c.g;
        auto lv = [&](int k, int rr, S* l) { S u4[4]; side_value(c, k, rr, u4); to_local(g.nax, g.sn, u4, l); };
        S l0[4], up[4], dw[4];
        lv(j, r, l0); lv(j, r + 1, up); lv(j, r - 1, dw);
        auto dt = [&](S vu, S vd) { return 0.5 * (vu - vd); };
        Tv[0] = -dt(up[0] * up[2], dw[0] * dw[2]);
        Tv[1] = -l0[2] * dt(up[1], dw[1]);
        if (L.thermal) {
            Tv[2] = -(L.cs2 / l0[0]) * dt(up[0] * up[3], dw[0] * dw[3]) - l0[2] * dt(up[2], dw[2]);
            Tv[3] = -dt(up[3] * up[2], dw[3] * dw[2]);
        } else {
            Tv[2] = -(L.cs2 / l0[0]) * dt(up[0], dw[0]) - l0[2] * dt(up[2], dw[2]);
            Tv[3] = 0.0;
        }
    }

    void side_rhs(const SideCtx& c, int j, int r, S* dU) const {
        const SideGeo& g = *c.g;
        const int n = L.thermal ? 4 : 3;
        const int b = bc[c.s];
        auto lv = [&](int k, int rr, S* l) { S u4[4]; side_value(c, k, rr, u4); to_local(g.nax, g.sn, u4, l); };
        S l0[4]; lv(j, r, l0);
        S dn[4];
        if (j == M) {  // eq. FD-dx-bw (outermost layer)
            S a[4], bb[4], cc[4]; lv(M, r, a); lv(M - 1, r, bb); lv(M - 2, r, cc);
            for (int m = 0; m < 4; ++m) dn[m] = 0.5 * (3.0 * a[m] - 4.0 * bb[m] + cc[m]);
        } else {        // eq. FD-dx-center (inner layers)
            S a[4], cc[4]; lv(j + 1, r, a); lv(j - 1, r, cc);
            for (int m = 0; m < 4; ++m) dn[m] = 0.5 * (a[m] - cc[m]);
        }
        S Tv[4];
        transverse(c, j, r, Tv);
        S Vv[4];
        if (is_full_cbc(b) && vfd[c.s]) {
            visc_fd(c, j, r, Vv);
        } else {
            for (int m = 0; m < 4; ++m) Vv[m] = (*c.V)[(size_t)r * 4 + m];
        }
        // characteristic analysis at the stage value; wave directions from time t
        S vec[4], dv[4], tv[4], vv[4];
        pack(l0, vec); pack(dn, dv);
        tv[0] = Tv[0]; tv[1] = Tv[1]; tv[2] = Tv[2]; tv[3] = Tv[3];
        vv[0] = Vv[0]; vv[1] = Vv[1]; vv[2] = Vv[2]; vv[3] = Vv[3];
        if (!L.thermal) { tv[3] = 0.0; vv[3] = 0.0; }
        CharSys<S> cs = char_system(L, vec);
        S u0g[4], l00[4];
        for (int m = 0; m < 4; ++m) u0g[m] = (*c.Y0)[((size_t)(j - 1) * g.len + r) * 4 + m];
        to_local(g.nax, g.sn, u0g, l00);
        S vec0[4]; pack(l00, vec0);
        CharSys<S> cs0 = char_system(L, vec0);
        S Sd[4], ST[4], SV[4];
        matvec(n, cs.Sm, dv, Sd);    // S dU/dn
        matvec(n, cs.Sm, tv, ST);    // transverse amplitudes  T_x = S T
        matvec(n, cs.Sm, vv, SV);    // viscous amplitudes     V_x = S V
        const S K = is_relax(b) ? relax_K(c.s) : S(0.0);
        const S alpha = is_relax(b) ? rp[c.s].alpha : S(0.0);
        S Lb[4];
        for (int i = 0; i < n; ++i) {
            if (value(cs0.lam[i]) >= 0.0) { Lb[i] = cs.lam[i] * Sd[i]; continue; }  // outgoing
            // incoming: annihilation (eq. PNR / eq. CBC-PNR); the relaxation of eq. LODI-Relax /
            // eq. CBC-Relax (transverse target 0, pressure target P_inf) acts on the incoming
            // acoustic wave only
            S in = is_full_cbc(b) ? ST[i] + SV[i] : S(0.0);
            if (is_relax(b) && acoustic(i)) in = in - alpha * ST[i] + pressure_term(l0, K, P_inf(c.s));
            Lb[i] = in;
        }
        S r4[4]; matvec(n, cs.Si, Lb, r4);
        S rl[4]; unpack_neg(r4, rl);                 // -S^-1 Lbar  (eq. thermal_LODI_macro_evo)
        if (is_full_cbc(b))                          // + T + V     (eq. thermal_CBC_macro_evo)
            for (int m = 0; m < n; ++m) rl[m] = rl[m] + tv[m] + vv[m];
        from_local_rate(g.nax, g.sn, rl, dU);
    }

    // corner ids at the low-row and high-row ends of side s
    void side_corners(int s, int& clo, int& chi) const {
        if (geo[s].nax == 0) { clo = (s & 1) | 0; chi = (s & 1) | 2; }
        else { clo = ((s - 2) << 1) | 0; chi = ((s - 2) << 1) | 1; }
    }

    void side_solve(int s, std::vector<S>& Un, const S corner_vals[4][2][4]) {
        const SideGeo& g = geo[s];
        const size_t nY = (size_t)M * g.len * 4;
        std::vector<S> Y0(nY), Ys(nY), K(nY), acc(nY), V;
        for (int j = 1; j <= M; ++j)
            for (int r = 0; r < g.len; ++r) {
                int x, y; node(g, j, r, x, y);
                getU(U, x, y, &Y0[((size_t)(j - 1) * g.len + r) * 4]);
            }
        if (is_full_cbc(bc[s]) && !vfd[s]) visc_terms(g, V); else V.assign((size_t)g.len * 4, S(0.0));
        SideCtx c;
        c.g = &g; c.s = s; c.Y0 = &Y0; c.Un = &Un; c.V = &V;
        int clo, chi;
        side_corners(s, clo, chi);
        c.corner_lo[0] = corner_vals[clo][0]; c.corner_lo[1] = corner_vals[clo][1];
        c.corner_hi[0] = corner_vals[chi][0]; c.corner_hi[1] = corner_vals[chi][1];
        const double a_st[4] = {0.0, 0.5, 0.5, 1.0};   // classic RK4 stage offsets
        const double b_st[4] = {1.0, 2.0, 2.0, 1.0};
        acc = Y0;
        for (int st = 0; st < 4; ++st) {
            for (size_t k = 0; k < nY; ++k) Ys[k] = st == 0 ? Y0[k] : Y0[k] + a_st[st] * K[k];
            c.Y = &Ys; c.theta = a_st[st];
            std::vector<S> Kn(nY);
            for (int j = 1; j <= M; ++j)
                for (int r = 0; r < g.len; ++r) side_rhs(c, j, r, &Kn[((size_t)(j - 1) * g.len + r) * 4]);
            K = Kn;
            for (size_t k = 0; k < nY; ++k) acc[k] = acc[k] + (b_st[st] / 6.0) * K[k];
        }
        for (int j = 1; j <= M; ++j)
            for (int r = 0; r < g.len; ++r) {
                int x, y; node(g, j, r, x, y);
                setU(Un, x, y, &acc[((size_t)(j - 1) * g.len + r) * 4]);
            }
    }

    // One RK4 step of the corner's LODI analysis (Sec. 3.3, corner treatment and "Time
    // integration"): Ut holds the time-t field, Un the bulk values at t + dt; returns the corner
    // node's value at t (U0) and at t + dt (acc).  The two inward diagonal bulk nodes are
    // interpolated linearly in time at the stages; wave directions are those at t.
    void corner_step(const Corner& c, const std::vector<S>& Ut, const std::vector<S>& Un, S* U0, S* acc) const {
        int x, y; corner_node(c, x, y);
        const int vx = -geo[c.sx].sn, vy = -geo[c.sy].sn;
        getU(Ut, x, y, U0);
        S b1n[4], b1p[4], b2n[4], b2p[4];
        getU(Ut, x + vx, y + vy, b1n); getU(Un, x + vx, y + vy, b1p);
        getU(Ut, x + 2 * vx, y + 2 * vy, b2n); getU(Un, x + 2 * vx, y + 2 * vy, b2p);
        const double a_st[4] = {0.0, 0.5, 0.5, 1.0}, b_st[4] = {1.0, 2.0, 2.0, 1.0};
        S Kc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int m = 0; m < 4; ++m) acc[m] = U0[m];
        for (int st = 0; st < 4; ++st) {
            const double th = a_st[st];
            S Ys[4], B1[4], B2[4];
            for (int m = 0; m < 4; ++m) {
                Ys[m] = U0[m] + a_st[st] * Kc[m];
                B1[m] = (1.0 - th) * b1n[m] + th * b1p[m];
                B2[m] = (1.0 - th) * b2n[m] + th * b2p[m];
            }
            corner_rhs(c, Ys, U0, B1, B2, Kc);
            for (int m = 0; m < 4; ++m) acc[m] = acc[m] + (b_st[st] / 6.0) * Kc[m];
        }
    }

    // -------------------------------------------------- probes of the boundary solve
    // (exposed through the C API so that the tests can pin the time integration, the transverse
    // terms and the corner coupling against closed forms)
    void layers_of(int s, const std::vector<S>& F, std::vector<S>& Y) const {
        const SideGeo& g = geo[s];
        Y.assign((size_t)M * g.len * 4, S(0.0));
        for (int j = 1; j <= M; ++j)
            for (int r = 0; r < g.len; ++r) {
                int x, y; node(g, j, r, x, y);
                getU(F, x, y, &Y[((size_t)(j - 1) * g.len + r) * 4]);
            }
    }
    void corner_values_of(const std::vector<S>& F, S cv[4][4]) const {
        for (int ci = 0; ci < 4; ++ci) {
            for (int m = 0; m < 4; ++m) cv[ci][m] = 0.0;
            Corner c = corner(ci);
            if (!c.active) continue;
            int x, y; corner_node(c, x, y);
            getU(F, x, y, cv[ci]);
        }
    }
    // right-hand side of side s at stage values Y [M][len][4] with the wave directions of the
    // layer values in Uv; the bulk and corner values are read from Uv as they are (no time
    // interpolation); V (CBC, mesoscopic) from the current pre-collision populations
    void side_rhs_probe(int s, const std::vector<S>& Uv, const std::vector<S>& Y, std::vector<S>& K) {
        const SideGeo& g = geo[s];
        std::vector<S> Y0, V;
        layers_of(s, Uv, Y0);
        if (is_full_cbc(bc[s]) && !vfd[s]) visc_terms(g, V); else V.assign((size_t)g.len * 4, S(0.0));
        S cv[4][4];
        corner_values_of(Uv, cv);
        int clo, chi;
        side_corners(s, clo, chi);
        SideCtx c;
        c.g = &g; c.s = s; c.Y = &Y; c.Y0 = &Y0; c.Un = &Uv; c.V = &V; c.theta = 0.0;
        c.corner_lo[0] = c.corner_lo[1] = cv[clo];
        c.corner_hi[0] = c.corner_hi[1] = cv[chi];
        std::vector<S> keep;
        keep.swap(U);
        U = Uv;
        K.assign(Y.size(), S(0.0));
        for (int j = 1; j <= M; ++j)
            for (int r = 0; r < g.len; ++r) side_rhs(c, j, r, &K[((size_t)(j - 1) * g.len + r) * 4]);
        U.swap(keep);
    }
    // one boundary step of side s from the time-t field Ut to t + dt, bulk and corner values at
    // t + dt taken from Unp1; returns the layers' new values Y1 [M][len][4]
    void side_step_probe(int s, const std::vector<S>& Ut, const std::vector<S>& Unp1, std::vector<S>& Y1) {
        S c0[4][4], c1[4][4], cv[4][2][4];
        corner_values_of(Ut, c0);
        corner_values_of(Unp1, c1);
        for (int ci = 0; ci < 4; ++ci)
            for (int m = 0; m < 4; ++m) { cv[ci][0][m] = c0[ci][m]; cv[ci][1][m] = c1[ci][m]; }
        std::vector<S> keep, Un = Unp1;
        keep.swap(U);
        U = Ut;
        side_solve(s, Un, cv);
        U.swap(keep);
        layers_of(s, Un, Y1);
    }
    // transverse terms at layer j, row r of side s from the current macroscopic field
    void transverse_probe(int s, int j, int r, S* Tv) const {
        const SideGeo& g = geo[s];
        std::vector<S> Y0;
        layers_of(s, U, Y0);
        S cv[4][4];
        corner_values_of(U, cv);
        int clo, chi;
        side_corners(s, clo, chi);
        SideCtx c;
        c.g = &g; c.s = s; c.Y = &Y0; c.Y0 = &Y0; c.Un = &U; c.V = nullptr; c.theta = 0.0;
        c.corner_lo[0] = c.corner_lo[1] = cv[clo];
        c.corner_hi[0] = c.corner_hi[1] = cv[chi];
        transverse(c, j, r, Tv);
    }

    // -------------------------------------------------- one time step
    void step() {
        const size_t P = plane();
        std::vector<S> fs(f.size(), S(0.0)), fc(f.size(), S(0.0)), Un(U.size(), S(0.0));
        // 1. streaming (eq. lbe, left-hand side) on bulk nodes
#pragma omp parallel for schedule(static)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                if (!is_bulk(x, y)) continue;
                for (int i = 0; i < q; ++i) {
                    int xs = x - L.cx[i], ys = y - L.cy[i];
                    if (xper) xs = (xs + nx) % nx;
                    if (yper) ys = (ys + ny) % ny;
                    fs[i * P + id(x, y)] = f[i * P + id(xs, ys)];
                }
            }
        // 2. macroscopic fields (eq. macro) and 3. BGK collision (eq. bgk) on bulk nodes
#pragma omp parallel for schedule(static)
        for (int y = 0; y < ny; ++y) {
            std::vector<S> fl(q), fe(q);
            for (int x = 0; x < nx; ++x) {
                if (!is_bulk(x, y)) continue;
                for (int i = 0; i < q; ++i) fl[i] = fs[i * P + id(x, y)];
                S u4[4];
                moments(L, fl.data(), u4[0], u4[1], u4[2], u4[3]);
                setU(Un, x, y, u4);
                equilibrium(L, u4[0], u4[1], u4[2], u4[3], fe.data());
                for (int i = 0; i < q; ++i) fc[i * P + id(x, y)] = fl[i] - (fl[i] - fe[i]) / tau;
            }
        }
        // 4. macroscopic boundary solver: corners first, then straight sides
        S cv[4][2][4];
        for (int ci = 0; ci < 4; ++ci)
            for (int t = 0; t < 2; ++t) for (int m = 0; m < 4; ++m) cv[ci][t][m] = 0.0;
        for (int ci = 0; ci < 4; ++ci) {
            Corner c = corner(ci);
            if (!c.active || c.zg) continue;
            corner_step(c, U, Un, cv[ci][0], cv[ci][1]);
            for (int jx = 1; jx <= M; ++jx)
                for (int jy = 1; jy <= M; ++jy) {
                    int xx = geo[c.sx].xf + geo[c.sx].sn * jx, yy = geo[c.sy].xf + geo[c.sy].sn * jy;
                    setU(Un, xx, yy, cv[ci][1]);
                }
        }
        for (int s = 0; s < 4; ++s)
            if (is_char(bc[s])) side_solve(s, Un, cv);
        // 5. mesoscopic Dirichlet reconstruction (Sec. 3.3 "Mesoscopic BC"; eq. zg-bc for ZG)
        for (int s = 0; s < 4; ++s) {
            const SideGeo& g = geo[s];
            if (bc[s] == BC_PERIODIC) continue;
            for (int r = 0; r < g.len; ++r)
                for (int j = 1; j <= M; ++j) {
                    int x, y; node(g, j, r, x, y);
                    if (bc[s] == BC_DIRICHLET) {
                        setU(Un, x, y, &inlet[s][(size_t)r * 4]);
                        node_feq(fc, x, y, &inlet[s][(size_t)r * 4]);
                    } else if (bc[s] == BC_ZG) {
                        int xf, yf; node(g, 0, r, xf, yf);
                        for (int i = 0; i < q; ++i) fc[i * P + id(x, y)] = fc[i * P + id(xf, yf)];
                        S u4[4]; node_moments(fc, x, y, u4); setU(Un, x, y, u4);
                    } else {
                        S u4[4]; getU(Un, x, y, u4); node_feq(fc, x, y, u4);
                        if (meso[s] == 1) {
                            // eq. NEEP: add the non-equilibrium part of the adjacent bulk node x_f
                            // (post-collision populations, so the layer holds the post-collision
                            // state that the same NEEP populations would reach in the collision)
                            int xf, yf; node(g, 0, r, xf, yf);
                            S uf[4]; getU(Un, xf, yf, uf);
                            std::vector<S> fe(q);
                            equilibrium(L, uf[0], uf[1], uf[2], uf[3], fe.data());
                            for (int i = 0; i < q; ++i)
                                fc[i * P + id(x, y)] = fc[i * P + id(x, y)] + (fc[i * P + id(xf, yf)] - fe[i]);
                        }
                    }
                }
        }
        for (int ci = 0; ci < 4; ++ci) {
            Corner c = corner(ci);
            if (!c.active) continue;
            int xc, yc; corner_node(c, xc, yc);
            const int vx = -geo[c.sx].sn, vy = -geo[c.sy].sn;
            for (int jx = 1; jx <= M; ++jx)
                for (int jy = 1; jy <= M; ++jy) {
                    int x = geo[c.sx].xf + geo[c.sx].sn * jx, y = geo[c.sy].xf + geo[c.sy].sn * jy;
                    if (c.zg) {
                        for (int i = 0; i < q; ++i) fc[i * P + id(x, y)] = fc[i * P + id(xc + vx, yc + vy)];
                        S u4[4]; node_moments(fc, x, y, u4); setU(Un, x, y, u4);
                    } else {
                        S u4[4]; getU(Un, x, y, u4); node_feq(fc, x, y, u4);
                    }
                }
        }
        // pre-collision populations of the new time level (used for the viscous terms)
        for (size_t k = 0; k < fs.size(); ++k) {
            const size_t node_id = k % P;
            const int x = (int)(node_id % nx), y = (int)(node_id / nx);
            fpre[k] = is_bulk(x, y) ? fs[k] : fc[k];
        }
        f.swap(fc);
        U.swap(Un);
        ++steps;
    }

    // diagnostics: mass, momentum x/y, energy (1/2 sum f |c|^2), loss, max |u|, non-finite count
    void diagnostics(double* out) const {
        double m = 0, jx = 0, jy = 0, e = 0, loss = 0, umax = 0, bad = 0;
        const double Pinf = L.cs2;
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                double r = 0, ax = 0, ay = 0, en = 0;
                for (int i = 0; i < q; ++i) {
                    double fi = value(f[i * plane() + id(x, y)]);
                    if (!std::isfinite(fi)) bad += 1;
                    r += fi; ax += fi * L.cx[i]; ay += fi * L.cy[i];
                    en += 0.5 * fi * (L.cx[i] * L.cx[i] + L.cy[i] * L.cy[i]);
                }
                m += r; jx += ax; jy += ay; e += en;
                const double ux = ax / r, uy = ay / r;
                umax = std::max(umax, std::sqrt(ux * ux + uy * uy));
                if (is_interior(x, y)) {
                    const double p = L.cs2 * value(U[id(x, y)]) * value(U[3 * plane() + id(x, y)]);
                    loss += (p - Pinf) * (p - Pinf);
                }
            }
        out[0] = m; out[1] = jx; out[2] = jy; out[3] = e; out[4] = loss; out[5] = umax; out[6] = bad; out[7] = (double)steps;
    }
    bool is_interior(int x, int y) const { return is_bulk(x, y); }

    S loss() const {
        S acc = 0.0;
        const double Pinf = L.cs2;
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                if (!is_interior(x, y)) continue;
                S u4[4]; getU(U, x, y, u4);
                S p = L.cs2 * u4[0] * u4[3];
                acc += (p - Pinf) * (p - Pinf);
            }
        return acc;
    }
};

int validate(int stencil, int nx, int ny, double tau, const int* bc) {
    if (stencil != 9 && stencil != 17 && stencil != 37) { g_err = "stencil must be 9, 17 or 37"; return -1; }
    const int M = stencil == 9 ? 1 : 3;
    if (!(tau > 0.5)) { g_err = "tau must exceed 1/2"; return -1; }
    for (int s = 0; s < 4; ++s) if (bc[s] < 0 || bc[s] > 6) { g_err = "bad boundary type"; return -1; }
    if ((bc[0] == BC_PERIODIC) != (bc[1] == BC_PERIODIC) || (bc[2] == BC_PERIODIC) != (bc[3] == BC_PERIODIC)) {
        g_err = "periodic sides must come in pairs"; return -1;
    }
    const bool xp = bc[0] == BC_PERIODIC, yp = bc[2] == BC_PERIODIC;
    if (nx < (xp ? M + 1 : 2 * M + 3) || ny < (yp ? M + 1 : 2 * M + 3)) { g_err = "grid too small"; return -1; }
    // the viscous terms of a CBC side are evaluated at x_f - M .. x_f - M - 2 (bulk nodes)
    if (((is_full_cbc(bc[0]) || is_full_cbc(bc[1])) && nx < 3 * M + 3) ||
        ((is_full_cbc(bc[2]) || is_full_cbc(bc[3])) && ny < 3 * M + 3)) {
        g_err = "CBC sides need at least 3M + 3 nodes along their normal"; return -1;
    }
    if (!xp && !yp) {
        for (int cx = 0; cx < 2; ++cx)
            for (int cy = 2; cy < 4; ++cy) {
                const bool ok = (is_char(bc[cx]) && is_char(bc[cy])) || (bc[cx] == BC_ZG && bc[cy] == BC_ZG);
                if (!ok) { g_err = "corner between these boundary types is not supported"; return -1; }
            }
    }
    if (stencil == 9)
        for (int s = 0; s < 4; ++s)
            if (is_full_cbc(bc[s])) { g_err = "CBC with viscous terms needs the heat-flux moment (thermal stencils)"; return -1; }
    return 0;
}

}  // namespace

// ===================================================================== C API (ctypes)
extern "C" {

const char* oracle_error(void) { return g_err.c_str(); }

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

// Threads for the OpenMP loops from now on (timing of the CPU baseline on one core).
void oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_lattice(int stencil, int* q, int* M, double* cs2, double* w, int* cx, int* cy) {
    if (stencil != 9 && stencil != 17 && stencil != 37) return -1;
    const Lattice& L = lattice(stencil);
    *q = L.q; *M = L.M; *cs2 = L.cs2;
    for (int i = 0; i < L.q; ++i) { if (w) w[i] = L.w[i]; if (cx) cx[i] = L.cx[i]; if (cy) cy[i] = L.cy[i]; }
    return 0;
}

int oracle_feq(int stencil, double rho, double ux, double uy, double T, double* out) {
    if (stencil != 9 && stencil != 17 && stencil != 37) return -1;
    equilibrium(lattice(stencil), rho, ux, uy, T, out);
    return 0;
}

int oracle_moments(int stencil, const double* f, double* u4) {
    if (stencil != 9 && stencil != 17 && stencil != 37) return -1;
    moments(lattice(stencil), f, u4[0], u4[1], u4[2], u4[3]);
    return 0;
}

// characteristic matrices at a local-frame state (rho, u_n, u_t, T); n x n row-major
int oracle_char_matrices(int stencil, const double* U, double* A, double* S, double* Si, double* lam) {
    if (stencil != 9 && stencil != 17 && stencil != 37) return -1;
    auto c = char_system<double>(lattice(stencil), U);
    for (int k = 0; k < c.n * c.n; ++k) { A[k] = c.A[k]; S[k] = c.Sm[k]; Si[k] = c.Si[k]; }
    for (int k = 0; k < c.n; ++k) lam[k] = c.lam[k];
    return c.n;
}

void* oracle_create(int stencil, int nx, int ny, double tau, const int* bc) {
    if (validate(stencil, nx, ny, tau, bc) != 0) return nullptr;
    return new Sim<double>(lattice(stencil), nx, ny, tau, bc);
}

void oracle_destroy(void* h) { delete static_cast<Sim<double>*>(h); }

int oracle_side_len(void* h, int side) { return static_cast<Sim<double>*>(h)->geo[side].len; }

// p = {sigma, alpha, rho_inf, T_inf, mach, length}
int oracle_set_relax(void* h, int side, const double* p) {
    auto* s = static_cast<Sim<double>*>(h);
    if (side < 0 || side > 3) return -1;
    s->rp[side].sigma = p[0]; s->rp[side].alpha = p[1]; s->rp[side].rho_inf = p[2];
    s->rp[side].T_inf = p[3]; s->rp[side].mach = p[4]; s->rp[side].length = p[5];
    return 0;
}

// Mesoscopic BC of a characteristic side (Sec. 3.3 "Mesoscopic BC"): 0 equilibrium, 1 NEEP.
int oracle_set_recon(void* h, int side, int mode) {
    auto* s = static_cast<Sim<double>*>(h);
    if (side < 0 || side > 3 || mode < 0 || mode > 1) return -1;
    if (mode == 1 && !(s->bc[side] >= BC_LODI && s->bc[side] <= BC_CBC_RELAX)) return -1;
    s->meso[side] = mode;
    return 0;
}

// Viscous terms of a CBC side: 0 from the mesoscopic moments (eq. LaplaceU / LaplaceT), 1 by
// finite differences of the macroscopic values (the -FD variant of Sec. 4.2).
int oracle_visc_fd_probe(void* h, int side, int j, int r, double* out) {
    auto* s = static_cast<Sim<double>*>(h);
    if (side < 0 || side > 3 || s->bc[side] == BC_PERIODIC || j < 1 || j > s->M) return -1;
    const auto& g = s->geo[side];
    if (!(g.tper || (r >= 1 && r + 1 < g.len))) return -1;
    s->visc_fd_probe(side, j, r, out);
    return 0;
}

int oracle_set_viscous(void* h, int side, int mode) {
    auto* s = static_cast<Sim<double>*>(h);
    if (side < 0 || side > 3 || mode < 0 || mode > 1) return -1;
    if (mode == 1 && !is_full_cbc(s->bc[side])) return -1;
    s->vfd[side] = mode;
    return 0;
}

// Fixed profile of a Dirichlet side [len][4]; it takes effect at once: the boundary layers get
// the equilibrium populations of the profile.
int oracle_set_inlet(void* h, int side, const double* Uin) {
    auto* s = static_cast<Sim<double>*>(h);
    if (side < 0 || side > 3 || s->bc[side] != BC_DIRICHLET) return -1;
    for (size_t k = 0; k < s->inlet[side].size(); ++k) s->inlet[side][k] = Uin[k];
    const SideGeo& g = s->geo[side];
    for (int r = 0; r < g.len; ++r)
        for (int j = 1; j <= s->M; ++j) {
            int x, y; s->node(g, j, r, x, y);
            const double* u4 = &s->inlet[side][(size_t)r * 4];
            s->setU(s->U, x, y, u4);
            s->node_feq(s->f, x, y, u4);
            s->node_feq(s->fpre, x, y, u4);
        }
    return 0;
}

int oracle_init(void* h, const double* rho, const double* ux, const double* uy, const double* T) {
    static_cast<Sim<double>*>(h)->init(rho, ux, uy, T, nullptr);
    return 0;
}

int oracle_step(void* h, int n) {
    auto* s = static_cast<Sim<double>*>(h);
    for (int k = 0; k < n; ++k) s->step();
    return 0;
}

int oracle_macro(void* h, double* rho, double* ux, double* uy, double* T) {
    auto* s = static_cast<Sim<double>*>(h);
    const size_t P = s->plane();
    for (size_t k = 0; k < P; ++k) { rho[k] = s->U[k]; ux[k] = s->U[P + k]; uy[k] = s->U[2 * P + k]; T[k] = s->U[3 * P + k]; }
    return 0;
}

int oracle_pops(void* h, double* f) {
    auto* s = static_cast<Sim<double>*>(h);
    std::memcpy(f, s->f.data(), s->f.size() * sizeof(double));
    return 0;
}

int oracle_diag(void* h, double* out) {
    static_cast<Sim<double>*>(h)->diagnostics(out);
    return 0;
}

// Forward-mode run: tangents of the loss (sum over interior nodes of (P - P_inf)^2 at the final
// step, P = rho cs^2 T, P_inf = cs^2) along NTAN directions.  Direction k perturbs sigma by
// dsigma[k] and alpha by dalpha[k] on every characteristic side, and the initial temperature by
// dT[k][ny][nx].  relax: [4][6] as in oracle_set_relax.  out: loss, then NTAN derivatives.
int oracle_tangent_run(int stencil, int nx, int ny, double tau, const int* bc, const double* relax,
                       const double* dsigma, const double* dalpha, const double* rho, const double* ux,
                       const double* uy, const double* T, const double* dT, int nsteps, double* out) {
    if (validate(stencil, nx, ny, tau, bc) != 0) return -1;
    Sim<Dual> s(lattice(stencil), nx, ny, tau, bc);
    for (int side = 0; side < 4; ++side) {
        const double* p = relax + 6 * side;
        Dual sg(p[0]), al(p[1]);
        for (int k = 0; k < NTAN; ++k) { sg.d[k] = dsigma[k]; al.d[k] = dalpha[k]; }
        s.rp[side].sigma = sg; s.rp[side].alpha = al;
        s.rp[side].rho_inf = p[2]; s.rp[side].T_inf = p[3]; s.rp[side].mach = p[4]; s.rp[side].length = p[5];
    }
    std::vector<Dual> Td((size_t)nx * ny);
    for (size_t n = 0; n < Td.size(); ++n) {
        Td[n] = Dual(T[n]);
        for (int k = 0; k < NTAN; ++k) Td[n].d[k] = dT[(size_t)k * nx * ny + n];
    }
    s.init(rho, ux, uy, T, &Td);
    for (int k = 0; k < nsteps; ++k) s.step();
    Dual l = s.loss();
    out[0] = l.v;
    for (int k = 0; k < NTAN; ++k) out[1 + k] = l.d[k];
    return 0;
}

// Forward-mode run with tangents on all four initial fields: direction k perturbs sigma and
// alpha as above and (rho0, ux0, uy0, T0) by dF[k][4][ny][nx].  The loss is the pressure loss
// above, or with wlin != NULL the linear functional sum over all nodes of
// wlin[c][y][x] * (rho, ux, uy, T)_c at the final step.  out: loss, then NTAN derivatives.
// visc: NULL, or the viscous-term mode per side (0 mesoscopic, 1 finite differences; CBC sides);
// recon: NULL, or the mesoscopic BC per side (0 equilibrium, 1 NEEP; characteristic sides)
int oracle_tangent_run_fields_ex(int stencil, int nx, int ny, double tau, const int* bc, const double* relax,
                                 const double* dsigma, const double* dalpha, const double* rho, const double* ux,
                                 const double* uy, const double* T, const double* dF, const double* wlin,
                                 const int* visc, const int* recon, int nsteps, double* out) {
    if (validate(stencil, nx, ny, tau, bc) != 0) return -1;
    Sim<Dual> s(lattice(stencil), nx, ny, tau, bc);
    for (int side = 0; side < 4; ++side) {
        if (visc) {
            if (visc[side] != 0 && !is_full_cbc(bc[side])) { g_err = "finite-difference viscous terms need a CBC side"; return -1; }
            s.vfd[side] = visc[side];
        }
        if (recon) {
            if (recon[side] != 0 && !(bc[side] >= BC_LODI && bc[side] <= BC_CBC_RELAX)) { g_err = "NEEP needs a characteristic side"; return -1; }
            s.meso[side] = recon[side];
        }
    }
    for (int side = 0; side < 4; ++side) {
        const double* p = relax + 6 * side;
        Dual sg(p[0]), al(p[1]);
        for (int k = 0; k < NTAN; ++k) { sg.d[k] = dsigma[k]; al.d[k] = dalpha[k]; }
        s.rp[side].sigma = sg; s.rp[side].alpha = al;
        s.rp[side].rho_inf = p[2]; s.rp[side].T_inf = p[3]; s.rp[side].mach = p[4]; s.rp[side].length = p[5];
    }
    const size_t n = (size_t)nx * ny;
    const double* base[4] = {rho, ux, uy, T};
    std::vector<Dual> F(4 * n);
    for (int c = 0; c < 4; ++c)
        for (size_t e = 0; e < n; ++e) {
            F[c * n + e] = Dual(base[c] ? base[c][e] : 1.0);
            for (int k = 0; k < NTAN; ++k) F[c * n + e].d[k] = dF[((size_t)k * 4 + c) * n + e];
        }
    s.init(rho, ux, uy, T, nullptr, &F);
    for (int k = 0; k < nsteps; ++k) s.step();
    Dual l = 0.0;
    if (wlin) {
        for (int c = 0; c < 4; ++c)
            for (size_t e = 0; e < n; ++e) l = l + Dual(wlin[c * n + e]) * s.U[c * n + e];
    } else {
        l = s.loss();
    }
    out[0] = l.v;
    for (int k = 0; k < NTAN; ++k) out[1 + k] = l.d[k];
    return 0;
}

int oracle_tangent_run_fields(int stencil, int nx, int ny, double tau, const int* bc, const double* relax,
                              const double* dsigma, const double* dalpha, const double* rho, const double* ux,
                              const double* uy, const double* T, const double* dF, const double* wlin, int nsteps,
                              double* out) {
    return oracle_tangent_run_fields_ex(stencil, nx, ny, tau, bc, relax, dsigma, dalpha, rho, ux, uy, T, dF, wlin,
                                        nullptr, nullptr, nsteps, out);
}

// Right-hand side of the corner LODI analysis (Sec. 3.3, corner treatment) of corner cidx
// (0 = (x0, y0), 1 = (x1, y0), 2 = (x0, y1), 3 = (x1, y1)) for given states (global components
// rho, ux, uy, T): Uc at the innermost corner node, Ucn the state fixing the wave directions, B1
// and B2 at the two inward diagonal nodes.  Exposed to pin the diagonal analysis.
int oracle_corner_rhs_probe(void* h, int cidx, const double* Uc, const double* Ucn, const double* B1,
                            const double* B2, double* out) {
    auto* s = static_cast<Sim<double>*>(h);
    if (cidx < 0 || cidx > 3) return -1;
    const auto c = s->corner(cidx);
    if (!c.active || c.zg) return -1;
    s->corner_rhs(c, Uc, Ucn, B1, B2, out);
    return 0;
}

// Viscous terms V = (0, V_n, V_t, V_T) (local frame) at bulk node (x, y) of a domain whose
// direction along the side is periodic, as if a boundary with outward normal along axis nax
// (0 = x, 1 = y) and sign sn sat just beyond (x, y).  Exposed to pin eq. LaplaceU/LaplaceT.
int oracle_visc_probe(void* h, int nax, int sn, int x, int y, double* out) {
    auto* s = static_cast<Sim<double>*>(h);
    SideGeo g;
    g.nax = nax; g.sn = sn;
    g.Nn = nax == 0 ? s->nx : s->ny;
    g.Nt = nax == 0 ? s->ny : s->nx;
    g.tper = true; g.r0 = 0; g.len = g.Nt;
    g.xf = nax == 0 ? x : y;
    const int r = nax == 0 ? y : x;
    if (g.xf - 2 * sn < 0 || g.xf - 2 * sn >= g.Nn) return -1;
    s->visc_row(g, r, out, 0);
    return 0;
}

// Probes of the boundary solve.  Fields are [4][ny][nx] (rho, ux, uy, T), layer values
// [M][len][4] (global components) with layer j at index j - 1 and rows as in oracle_side_len.
static bool probe_side_ok(Sim<double>* s, int side) {
    return side >= 0 && side <= 3 && is_char(s->bc[side]);
}

// Right-hand side of the layers' evolution (eq. thermal_LODI_macro_evo / thermal_CBC_macro_evo)
// of a characteristic side at stage values Y, everything else (bulk nodes, corner blocks, the
// wave directions from the layers) read from the field Uv without time interpolation.
int oracle_side_rhs_probe(void* h, int side, const double* Uv, const double* Y, double* K) {
    auto* s = static_cast<Sim<double>*>(h);
    if (!probe_side_ok(s, side)) return -1;
    const size_t nF = 4 * s->plane(), nY = (size_t)s->M * s->geo[side].len * 4;
    std::vector<double> F(Uv, Uv + nF), Yv(Y, Y + nY), Kv;
    s->side_rhs_probe(side, F, Yv, Kv);
    std::memcpy(K, Kv.data(), nY * sizeof(double));
    return 0;
}

// One RK4 step (Sec. 3.3, "Time integration") of a characteristic side from the field Ut at time
// t, with the bulk and corner values at t + dt from Unp1; writes the layers' values at t + dt.
int oracle_side_step_probe(void* h, int side, const double* Ut, const double* Unp1, double* Y1) {
    auto* s = static_cast<Sim<double>*>(h);
    if (!probe_side_ok(s, side)) return -1;
    const size_t nF = 4 * s->plane(), nY = (size_t)s->M * s->geo[side].len * 4;
    std::vector<double> A(Ut, Ut + nF), B(Unp1, Unp1 + nF), Yv;
    s->side_step_probe(side, A, B, Yv);
    std::memcpy(Y1, Yv.data(), nY * sizeof(double));
    return 0;
}

// One RK4 step of corner cidx's diagonal LODI analysis from the field Ut at time t, with the two
// inward diagonal bulk nodes at t + dt from Unp1; writes the corner value at t + dt.
int oracle_corner_step_probe(void* h, int cidx, const double* Ut, const double* Unp1, double* out4) {
    auto* s = static_cast<Sim<double>*>(h);
    if (cidx < 0 || cidx > 3) return -1;
    const auto c = s->corner(cidx);
    if (!c.active || c.zg) return -1;
    const size_t nF = 4 * s->plane();
    std::vector<double> A(Ut, Ut + nF), B(Unp1, Unp1 + nF);
    double U0[4];
    s->corner_step(c, A, B, U0, out4);
    return 0;
}

// Transverse terms T (eq. NSF-CHAR, local components (rho, u_n, u_t, T)) at layer j (1..M), row r
// of a characteristic side, from the current macroscopic field.
int oracle_transverse_probe(void* h, int side, int j, int r, double* out4) {
    auto* s = static_cast<Sim<double>*>(h);
    if (!probe_side_ok(s, side) || j < 1 || j > s->M || r < 0 || r >= s->geo[side].len) return -1;
    s->transverse_probe(side, j, r, out4);
    return 0;
}

// Plain loss of the current state (same definition as in oracle_tangent_run).
double oracle_loss(void* h) { return static_cast<Sim<double>*>(h)->loss(); }

}  // extern "C"
