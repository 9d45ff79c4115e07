/*
 * lbm3d_oracle.cpp -- plain FP64 CPU reference of the three-dimensional extension of the
 * characteristic boundary conditions of Klass, Gabbana & Bartel (arXiv 2307.16766, Appendix A):
 * thermal BGK lattice Boltzmann on the D3Q39 stencil with LODI / CBC boundaries on the two faces
 * normal to one axis (x, y or z) of a box that is periodic along the other two.
 *
 * TEST INFRASTRUCTURE.  Like the two-dimensional oracle, this file is what the GPU library is
 * checked against; only the test-suite, the package smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no source, header, table or constant generator with the GPU
 * library: the lattice comes from its own isotropy solve, the equilibrium from the Hermite tensor
 * definition, the characteristic matrices from the formulas of Appendix A.
 *
 * Steps (one time step, unfused, in the order of the paper's flowcharts):
 *     stream -> macroscopic fields -> collide -> characteristic solve on each face (RK4)
 *     -> mesoscopic Dirichlet reconstruction (equilibrium or eq. NEEP) / zero gradient.
 *
 * Readings (each also listed in the design notes):
 *  - Stencil: the paper points to the D3Q39 and D3Q103 rules without data.  D3Q39 is the rule on
 *    the velocity groups (0,0,0), (1,0,0), (1,1,1), (2,0,0), (2,2,0), (3,0,0) that integrates
 *    Gaussian moments up to degree 7; its weights and cs^2 are solved here from the isotropy
 *    conditions.  Degree 7 carries the 3rd-order equilibrium of eq. feq-3 (as D2Q17 in 2D).
 *  - d = 3: c_v = 3/2, c_p = 5/2, gamma = 5/3 (Appendix A); T = sum f |c-u|^2 / (3 rho cs^2).
 *  - Characteristic system: A, S, S^-1 and Lambda of Appendix A in the local frame
 *    U = (rho, u_n, u_t1, u_t2, T), waves ordered entropy, shear t1, shear t2, acoustic -/+.
 *    The transverse terms are those of Appendix A, with central differences along the two
 *    tangential axes (t1, t2) = the axes that follow the normal cyclically (y, z for x-faces;
 *    z, x for y-faces; x, y for z-faces): Appendix A written for a face normal to x, rotated.
 *  - Viscous terms of the CBC schemes from the mesoscopic moments at x_f - M .. x_f - M - 2 (as
 *    in 2D): V_u = div(Pi') / rho, V_T = (-div q + Pi':Pi' / (2 rho nu)) / (rho c_v cs^2), with
 *    Pi' = -(1 - 1/(2 tau)) sum c c (f - f^eq) and q = (1 - 1/(2 tau)) 1/2 sum f |c-u|^2 (c-u).
 *  - Relaxation: the incoming acoustic amplitude gets -alpha T_x,i + K (P - P_inf) / (5 rho cs^2),
 *    the pressure coefficient of the acoustic rows of S (1/5 in 3D, 1/4 in 2D), with
 *    K = sigma (1 - Ma^2) c_inf / L and c_inf = sqrt(gamma cs^2 T_inf).
 *  - Faces: the two faces normal to one axis carry boundaries; the other two axes are periodic
 *    (the paper gives no edge or corner treatment in 3D).
 */
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

std::string g_err3;

// ---------------------------------------------------------------- lattice
struct Lattice3 {
    int q = 0, M = 0, order = 0;
    double cs2 = 0, cs = 0;
    std::vector<int> cx, cy, cz;
    std::vector<double> w;
    std::vector<double> h1, h2, h3;   // Hermite tensor polynomials of xi = c / cs, row-major
};

using Triple = std::array<int, 3>;

// every sign and axis permutation of a group (a, b, c)
static std::vector<Triple> members3(int a, int b, int c) {
    std::vector<Triple> out;
    int p[3] = {a, b, c};
    std::sort(p, p + 3);
    do {
        for (int s = 0; s < 8; ++s) {
            Triple m = {(s & 1) ? -p[0] : p[0], (s & 2) ? -p[1] : p[1], (s & 4) ? -p[2] : p[2]};
            if (std::find(out.begin(), out.end(), m) == out.end()) out.push_back(m);
        }
    } while (std::next_permutation(p, p + 3));
    std::sort(out.begin(), out.end());
    return out;
}

static long double dfact3(int n) { long double r = 1; while (n > 1) { r *= n; n -= 2; } return r; }

static long double group_moment3(const Triple& g, const Triple& e) {
    long double s = 0;
    for (auto& m : members3(g[0], g[1], g[2])) {
        long double t = 1;
        for (int d = 0; d < 3; ++d) for (int k = 0; k < 2 * e[d]; ++k) t *= m[d];
        s += t;
    }
    return s;
}

static long double gauss3(const Triple& e, long double s) {
    return dfact3(2 * e[0] - 1) * dfact3(2 * e[1] - 1) * dfact3(2 * e[2] - 1) * std::pow(s, (long double)(e[0] + e[1] + e[2]));
}

// group weights from the linear isotropy conditions at a given cs^2 (Gaussian elimination)
static std::vector<long double> solve_weights3(const std::vector<Triple>& groups, const std::vector<Triple>& lin, long double s) {
    const int n = (int)groups.size();
    std::vector<long double> A(n * (n + 1));
    for (int r = 0; r < n; ++r) {
        for (int c = 0; c < n; ++c) A[r * (n + 1) + c] = group_moment3(groups[c], lin[r]);
        A[r * (n + 1) + n] = gauss3(lin[r], s);
    }
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r) if (std::fabs(A[r * (n + 1) + c]) > std::fabs(A[p * (n + 1) + c])) p = r;
        for (int k = 0; k <= n; ++k) std::swap(A[c * (n + 1) + k], A[p * (n + 1) + k]);
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const long double f = A[r * (n + 1) + c] / A[c * (n + 1) + c];
            for (int k = c; k <= n; ++k) A[r * (n + 1) + k] -= f * A[c * (n + 1) + k];
        }
    }
    std::vector<long double> wg(n);
    for (int r = 0; r < n; ++r) wg[r] = A[r * (n + 1) + n] / A[r * (n + 1) + r];
    return wg;
}

static Lattice3 make_lattice3(int stencil) {
    Lattice3 L;
    if (stencil != 39) return L;
    // D3Q39: degree-7 rule; the six group weights from six isotropy conditions, cs^2 from the
    // seventh, (1,1,1), by bisection (its only root in the bracket)
    const std::vector<Triple> groups = {{0, 0, 0}, {1, 0, 0}, {1, 1, 1}, {2, 0, 0}, {2, 2, 0}, {3, 0, 0}};
    const std::vector<Triple> lin = {{0, 0, 0}, {1, 0, 0}, {2, 0, 0}, {1, 1, 0}, {3, 0, 0}, {2, 1, 0}};
    const Triple chk = {1, 1, 1};
    auto resid = [&](long double s) {
        auto wg = solve_weights3(groups, lin, s);
        long double m = 0;
        for (size_t g = 0; g < groups.size(); ++g) m += wg[g] * group_moment3(groups[g], chk);
        return m - gauss3(chk, s);
    };
    long double lo = 0.6L, hi = 0.7L, flo = resid(lo);
    for (int it = 0; it < 200 && hi - lo > 1e-21L; ++it) {
        const long double mid = 0.5L * (lo + hi), fm = resid(mid);
        if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else { hi = mid; }
    }
    const long double s = 0.5L * (lo + hi);
    auto wg = solve_weights3(groups, lin, s);
    L.cs2 = (double)s;
    L.cs = (double)std::sqrt(s);
    L.M = 3;
    L.order = 3;
    for (size_t g = 0; g < groups.size(); ++g)
        for (auto& m : members3(groups[g][0], groups[g][1], groups[g][2])) {
            L.cx.push_back(m[0]); L.cy.push_back(m[1]); L.cz.push_back(m[2]);
            L.w.push_back((double)wg[g]);
        }
    L.q = (int)L.w.size();
    auto del = [](int a, int b) { return a == b ? 1.0 : 0.0; };
    for (int i = 0; i < L.q; ++i) {
        const double xi[3] = {L.cx[i] / L.cs, L.cy[i] / L.cs, L.cz[i] / L.cs};
        for (int a = 0; a < 3; ++a) L.h1.push_back(xi[a]);
        for (int a = 0; a < 3; ++a) for (int b = 0; b < 3; ++b) L.h2.push_back(xi[a] * xi[b] - del(a, b));
        for (int a = 0; a < 3; ++a) for (int b = 0; b < 3; ++b) for (int c = 0; c < 3; ++c)
            L.h3.push_back(xi[a] * xi[b] * xi[c] - (xi[a] * del(b, c) + xi[b] * del(a, c) + xi[c] * del(a, b)));
    }
    return L;
}

static const Lattice3& lattice3(int stencil) {
    static const Lattice3 L39 = make_lattice3(39);
    static const Lattice3 none;
    return stencil == 39 ? L39 : none;
}

// ---------------------------------------------------------------- equilibrium (eq. feq-3 in 3D)
// f^eq = w rho (1 + a1 . H1 + a2 : H2 / 2 + a3 : H3 / 6) with a1 = u, a2 = uu + th d,
// a3 = uuu + th (d u)_sym; u in units of cs, th = T - 1.
static void equilibrium3(const Lattice3& L, double rho, double ux, double uy, double uz, double T, double* out) {
    const double u[3] = {ux / L.cs, uy / L.cs, uz / L.cs};
    const double th = T - 1.0;
    auto del = [](int a, int b) { return a == b ? 1.0 : 0.0; };
    double a2[9], a3[27];
    for (int a = 0; a < 3; ++a) for (int b = 0; b < 3; ++b) a2[a * 3 + b] = u[a] * u[b] + th * del(a, b);
    for (int a = 0; a < 3; ++a) for (int b = 0; b < 3; ++b) for (int c = 0; c < 3; ++c)
        a3[(a * 3 + b) * 3 + c] = u[a] * u[b] * u[c] + th * (u[a] * del(b, c) + u[b] * del(a, c) + u[c] * del(a, b));
    for (int i = 0; i < L.q; ++i) {
        double s1 = 0.0, s2 = 0.0, s3 = 0.0;
        for (int k = 0; k < 3; ++k) s1 += u[k] * L.h1[3 * i + k];
        for (int k = 0; k < 9; ++k) s2 += a2[k] * L.h2[9 * i + k];
        for (int k = 0; k < 27; ++k) s3 += a3[k] * L.h3[27 * i + k];
        out[i] = L.w[i] * rho * (1.0 + s1 + s2 / 2.0 + s3 / 6.0);
    }
}

// rho = sum f, rho u = sum f c, 2 rho e = sum f |c-u|^2 with e = (d/2) cs^2 T, d = 3
static void moments3(const Lattice3& L, const double* f, double* u5) {
    double r = 0, jx = 0, jy = 0, jz = 0;
    for (int i = 0; i < L.q; ++i) { r += f[i]; jx += f[i] * L.cx[i]; jy += f[i] * L.cy[i]; jz += f[i] * L.cz[i]; }
    const double ux = jx / r, uy = jy / r, uz = jz / r;
    double e = 0;
    for (int i = 0; i < L.q; ++i) {
        const double dx = L.cx[i] - ux, dy = L.cy[i] - uy, dz = L.cz[i] - uz;
        e += f[i] * (dx * dx + dy * dy + dz * dz);
    }
    u5[0] = r; u5[1] = ux; u5[2] = uy; u5[3] = uz; u5[4] = e / (3.0 * r * L.cs2);
}

// ---------------------------------------------------------------- characteristic system (Appendix A)
constexpr double CV3 = 1.5, CP3 = 2.5, GAMMA3 = CP3 / CV3;

struct Char5 {
    double A[25], Sm[25], Si[25], lam[5];
};

// local frame U = (rho, u_n, u_t1, u_t2, T); waves: entropy, shear t1, shear t2, acoustic -, +
static Char5 char_system3(double cs2, const double* U) {
    Char5 c;
    for (int k = 0; k < 25; ++k) { c.A[k] = 0.0; c.Sm[k] = 0.0; c.Si[k] = 0.0; }
    const double rho = U[0], un = U[1], Tt = cs2 * U[4];
    const double s = std::sqrt(GAMMA3 * Tt);
    auto a = [&](int r, int k) -> double& { return c.A[r * 5 + k]; };
    auto m = [&](int r, int k) -> double& { return c.Sm[r * 5 + k]; };
    auto mi = [&](int r, int k) -> double& { return c.Si[r * 5 + k]; };
    a(0, 0) = un; a(0, 1) = rho;
    a(1, 0) = Tt / rho; a(1, 1) = un; a(1, 4) = cs2;
    a(2, 2) = un;
    a(3, 3) = un;
    a(4, 1) = Tt / (cs2 * CV3); a(4, 4) = un;
    const double r15 = std::sqrt(Tt / (15.0 * cs2 * cs2));
    m(0, 0) = -2.0 * Tt / (5.0 * rho * cs2); m(0, 4) = 0.6;
    m(1, 2) = 1.0;
    m(2, 3) = 1.0;
    m(3, 0) = Tt / (5.0 * rho * cs2); m(3, 1) = -r15; m(3, 4) = 0.2;
    m(4, 0) = Tt / (5.0 * rho * cs2); m(4, 1) = r15; m(4, 4) = 0.2;
    const double q15 = std::sqrt(15.0 * cs2 * cs2 / (4.0 * Tt));
    mi(0, 0) = -rho * cs2 / Tt; mi(0, 3) = 1.5 * rho * cs2 / Tt; mi(0, 4) = 1.5 * rho * cs2 / Tt;
    mi(1, 3) = -q15; mi(1, 4) = q15;
    mi(2, 1) = 1.0;
    mi(3, 2) = 1.0;
    mi(4, 0) = 1.0; mi(4, 3) = 1.0; mi(4, 4) = 1.0;
    c.lam[0] = un; c.lam[1] = un; c.lam[2] = un; c.lam[3] = un - s; c.lam[4] = un + s;
    return c;
}

static void matvec5(const double* M, const double* x, double* y) {
    for (int r = 0; r < 5; ++r) { double s = 0.0; for (int k = 0; k < 5; ++k) s += M[r * 5 + k] * x[k]; y[r] = s; }
}

// ---------------------------------------------------------------- simulation
enum { B3_PERIODIC = 0, B3_LODI = 1, B3_LODI_RELAX = 2, B3_CBC = 3, B3_CBC_RELAX = 4, B3_ZG = 5 };
inline bool char3(int b) { return b >= B3_LODI && b <= B3_CBC_RELAX; }
inline bool relax3(int b) { return b == B3_LODI_RELAX || b == B3_CBC_RELAX; }
inline bool full3(int b) { return b == B3_CBC || b == B3_CBC_RELAX; }

struct Relax3 {
    double sigma = 0.0, alpha = 0.0, rho_inf = 1.0, T_inf = 1.0, mach = 0.0, length = 0.0;
};

struct Sim3 {
    const Lattice3& L;
    int nx, ny, nz, q, M;
    int ax;              // axis normal to the two faces: 0 = x, 1 = y, 2 = z
    int dim[3];          // nx, ny, nz
    double tau;
    int bc[2];           // faces at the low and the high end of axis ax; the other axes are periodic
    bool fper;           // faces periodic (no boundaries)
    Relax3 rp[2];
    int meso[2] = {0, 0};
    std::vector<double> f, fpre, U;   // f, fpre: [q][nz][ny][nx]; U: [5][nz][ny][nx]
    long steps = 0;

    Sim3(const Lattice3& lat, int nx_, int ny_, int nz_, double tau_, const int* bc_, int ax_)
        : L(lat), nx(nx_), ny(ny_), nz(nz_), q(lat.q), M(lat.M), ax(ax_), tau(tau_) {
        dim[0] = nx; dim[1] = ny; dim[2] = nz;
        bc[0] = bc_[0]; bc[1] = bc_[1];
        fper = bc[0] == B3_PERIODIC;
        f.assign((size_t)q * plane(), 0.0);
        fpre = f;
        U.assign((size_t)5 * plane(), 0.0);
    }

    // face frame: the normal axis ax and the tangential axes a1 = ax + 1, a2 = ax + 2 (mod 3); a
    // node of a face's row is (kn, t1, t2) with kn along the normal; rows r = t2 * n1 + t1
    int a1() const { return (ax + 1) % 3; }
    int a2() const { return (ax + 2) % 3; }
    int nn() const { return dim[ax]; }
    int n1() const { return dim[a1()]; }
    int n2() const { return dim[a2()]; }
    size_t plane() const { return (size_t)nx * ny * nz; }
    size_t id(int x, int y, int z) const { return ((size_t)z * ny + y) * nx + x; }
    size_t fid(int kn, int t1, int t2) const {
        int c[3];
        c[ax] = kn; c[a1()] = t1; c[a2()] = t2;
        return id(c[0], c[1], c[2]);
    }
    bool is_bulk_n(int kn) const { return fper || (kn >= M && kn <= nn() - 1 - M); }
    bool is_bulk(int x, int y, int z) const { const int c[3] = {x, y, z}; return is_bulk_n(c[ax]); }
    int sn(int s) const { return s == 0 ? -1 : 1; }
    int xf(int s) const { return s == 0 ? M : nn() - 1 - M; }
    int xk(int s, int k) const { return xf(s) + sn(s) * k; }   // k = 0: x_f; k = j: layer j
    int w1(int t) const { return ((t % n1()) + n1()) % n1(); }
    int w2(int t) const { return ((t % n2()) + n2()) % n2(); }
    void getU(const std::vector<double>& F, size_t k, double* u5) const {
        for (int c = 0; c < 5; ++c) u5[c] = F[c * plane() + k];
    }
    void setU(std::vector<double>& F, size_t k, const double* u5) const {
        for (int c = 0; c < 5; ++c) F[c * plane() + k] = u5[c];
    }
    void node_feq(std::vector<double>& F, size_t k, const double* u5) const {
        std::vector<double> fe(q);
        equilibrium3(L, u5[0], u5[1], u5[2], u5[3], u5[4], fe.data());
        for (int i = 0; i < q; ++i) F[i * plane() + k] = fe[i];
    }
    void node_moments(const std::vector<double>& F, size_t k, double* u5) const {
        std::vector<double> fl(q);
        for (int i = 0; i < q; ++i) fl[i] = F[i * plane() + k];
        moments3(L, fl.data(), u5);
    }
    // local frame of face s: (rho, u_n, u_t1, u_t2, T), u_n = sn u_ax
    void to_local(int s, const double* g, double* l) const {
        l[0] = g[0]; l[1] = sn(s) * g[1 + ax]; l[2] = g[1 + a1()]; l[3] = g[1 + a2()]; l[4] = g[4];
    }
    void rate_to_global(int s, const double* l, double* g) const {
        g[0] = l[0]; g[1 + ax] = sn(s) * l[1]; g[1 + a1()] = l[2]; g[1 + a2()] = l[3]; g[4] = l[4];
    }

    void init(const double* rho, const double* ux, const double* uy, const double* uz, const double* T) {
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    const size_t k = id(x, y, z);
                    const double u5[5] = {rho[k], ux[k], uy[k], uz[k], T[k]};
                    setU(U, k, u5);
                    node_feq(f, k, u5);
                }
        fpre = f;
        steps = 0;
    }

    double relax_K(int s) const {
        const Relax3& p = rp[s];
        const double cinf = std::sqrt(GAMMA3 * L.cs2 * p.T_inf);
        const double Lg = p.length > 0 ? p.length : (double)nn();
        return p.sigma * (1.0 - p.mach * p.mach) * cinf / Lg;
    }

    // Pi' (nn, n1, n2, 11, 12, 22), q (n, 1, 2) in the local frame of outward normal g e_ax and
    // rho at node (kn, t1, t2), from the pre-collision populations of the current time level; zero
    // on boundary layers (equilibria)
    void visc_node(int g, int kn, int t1, int t2, double* o10) const {
        for (int c = 0; c < 10; ++c) o10[c] = 0.0;
        if (!is_bulk_n(kn)) return;
        const size_t k = fid(kn, t1, t2);
        std::vector<double> fl(q), fe(q);
        for (int i = 0; i < q; ++i) fl[i] = fpre[i * plane() + k];
        double u5[5];
        moments3(L, fl.data(), u5);
        equilibrium3(L, u5[0], u5[1], u5[2], u5[3], u5[4], fe.data());
        const double fac = 1.0 - 1.0 / (2.0 * tau);
        double P[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, Qv[3] = {0, 0, 0};
        for (int i = 0; i < q; ++i) {
            const double c[3] = {(double)L.cx[i], (double)L.cy[i], (double)L.cz[i]};
            const double fn = fl[i] - fe[i];
            for (int a = 0; a < 3; ++a) for (int b = 0; b < 3; ++b) P[a][b] -= fac * c[a] * c[b] * fn;
            const double d[3] = {c[0] - u5[1], c[1] - u5[2], c[2] - u5[3]};
            const double e = fl[i] * (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) * 0.5 * fac;
            for (int a = 0; a < 3; ++a) Qv[a] += e * d[a];
        }
        const int n = ax, b1 = a1(), b2 = a2();
        o10[0] = u5[0];
        o10[1] = P[n][n]; o10[2] = g * P[n][b1]; o10[3] = g * P[n][b2];
        o10[4] = P[b1][b1]; o10[5] = P[b1][b2]; o10[6] = P[b2][b2];
        o10[7] = g * Qv[n]; o10[8] = Qv[b1]; o10[9] = Qv[b2];
    }

    // V (local frame of outward normal g e_ax) at bulk node (kn0, t1, t2), frozen at time t:
    // div Pi' / rho and the temperature term, normal derivatives one-sided over kn0, kn0 - g,
    // kn0 - 2 g (eq. FD-dx-bw), tangential derivatives central along t1 and t2 (eq.
    // FD-dx-center).  On a face, kn0 = x_f - sn M (the first node none of whose populations
    // streamed from the layers) and g = sn.
    void visc_row(int g, int kn0, int t1, int t2, double* V5) const {
        const double nu = (tau - 0.5) * L.cs2;
        double d[3][10], yp[10], ym[10], zp[10], zm[10];
        for (int k = 0; k < 3; ++k) visc_node(g, kn0 - g * k, t1, t2, d[k]);
        visc_node(g, kn0, w1(t1 + 1), t2, yp); visc_node(g, kn0, w1(t1 - 1), t2, ym);
        visc_node(g, kn0, t1, w2(t2 + 1), zp); visc_node(g, kn0, t1, w2(t2 - 1), zm);
        auto dn = [&](int c) { return 0.5 * (3.0 * d[0][c] - 4.0 * d[1][c] + d[2][c]); };
        auto d1 = [&](int c) { return 0.5 * (yp[c] - ym[c]); };
        auto d2 = [&](int c) { return 0.5 * (zp[c] - zm[c]); };
        const double rho = d[0][0];
        const double* p = d[0];
        const double pp = p[1] * p[1] + p[4] * p[4] + p[6] * p[6] + 2.0 * (p[2] * p[2] + p[3] * p[3] + p[5] * p[5]);
        V5[0] = 0.0;
        V5[1] = (dn(1) + d1(2) + d2(3)) / rho;
        V5[2] = (dn(2) + d1(4) + d2(5)) / rho;
        V5[3] = (dn(3) + d1(5) + d2(6)) / rho;
        V5[4] = (-(dn(7) + d1(8) + d2(9)) + pp / (2.0 * rho * nu)) / (rho * CV3 * L.cs2);
    }

    struct FaceCtx {
        int s;
        const std::vector<double>* Y;    // stage values [M][n1*n2][5]
        const std::vector<double>* Y0;   // values at time t
        const std::vector<double>* Un;   // macroscopic field at t + dt (bulk filled)
        const std::vector<double>* V;    // viscous terms [n1*n2][5]
        double theta;
    };

    // value (global components) at outward index k of row (t1, t2): layers from the stage
    // values, bulk nodes interpolated in time
    void face_value(const FaceCtx& c, int k, int t1, int t2, double* u5) const {
        t1 = w1(t1); t2 = w2(t2);
        const size_t r = (size_t)t2 * n1() + t1;
        if (k >= 1) {
            for (int m = 0; m < 5; ++m) u5[m] = (*c.Y)[((size_t)(k - 1) * n1() * n2() + r) * 5 + m];
            return;
        }
        const size_t node = fid(xk(c.s, k), t1, t2);
        double a[5], b[5];
        getU(U, node, a); getU(*c.Un, node, b);
        for (int m = 0; m < 5; ++m) u5[m] = (1.0 - c.theta) * a[m] + c.theta * b[m];
    }

    // transverse terms of Appendix A (local frame) at layer j of row (t1, t2), central
    // differences of the stage values along t1 and t2
    void transverse(const FaceCtx& c, int j, int t1, int t2, double* Tv) const {
        auto lv = [&](int k, int u1, int u2, double* l) { double g[5]; face_value(c, k, u1, u2, g); to_local(c.s, g, l); };
        double l0[5], yp[5], ym[5], zp[5], zm[5];
        lv(j, t1, t2, l0);
        lv(j, t1 + 1, t2, yp); lv(j, t1 - 1, t2, ym); lv(j, t1, t2 + 1, zp); lv(j, t1, t2 - 1, zm);
        auto dy = [&](double u, double d) { return 0.5 * (u - d); };
        const double cs2 = L.cs2;
        const double rho = l0[0], v = l0[2], w = l0[3], T = l0[4];
        Tv[0] = -dy(yp[0] * yp[2], ym[0] * ym[2]) - dy(zp[0] * zp[3], zm[0] * zm[3]);
        Tv[1] = -(v * dy(yp[1], ym[1]) + w * dy(zp[1], zm[1]));
        Tv[2] = -(cs2 / rho) * dy(yp[0] * yp[4], ym[0] * ym[4]) - (v * dy(yp[2], ym[2]) + w * dy(zp[2], zm[2]));
        Tv[3] = -(cs2 / rho) * dy(zp[0] * zp[4], zm[0] * zm[4]) - (v * dy(yp[3], ym[3]) + w * dy(zp[3], zm[3]));
        Tv[4] = -(T / CV3) * (dy(yp[2], ym[2]) + dy(zp[3], zm[3])) - (v * dy(yp[4], ym[4]) + w * dy(zp[4], zm[4]));
    }

    void layers_of(int s, const std::vector<double>& F, std::vector<double>& Y) const {
        const size_t R = (size_t)n1() * n2();
        Y.assign((size_t)M * R * 5, 0.0);
        for (int j = 1; j <= M; ++j)
            for (int t2 = 0; t2 < n2(); ++t2)
                for (int t1 = 0; t1 < n1(); ++t1)
                    getU(F, fid(xk(s, j), t1, t2), &Y[((size_t)(j - 1) * R + (size_t)t2 * n1() + t1) * 5]);
    }

    // the transverse terms at layer j of row (t1, t2) of face s from the current state
    void transverse_probe(int s, int j, int t1, int t2, double* Tv) const {
        std::vector<double> Y0;
        layers_of(s, U, Y0);
        FaceCtx c;
        c.s = s; c.Y = &Y0; c.Y0 = &Y0; c.Un = &U; c.V = nullptr; c.theta = 0.0;
        transverse(c, j, t1, t2, Tv);
    }

    void face_rhs(const FaceCtx& c, int j, int t1, int t2, double* dU) const {
        const int s = c.s, b = bc[s];
        auto lv = [&](int k, int u1, int u2, double* l) { double g[5]; face_value(c, k, u1, u2, g); to_local(s, g, l); };
        double l0[5], dn[5];
        lv(j, t1, t2, l0);
        if (j == M) {
            double a[5], bb[5], cc[5]; lv(M, t1, t2, a); lv(M - 1, t1, t2, bb); lv(M - 2, t1, t2, cc);
            for (int m = 0; m < 5; ++m) dn[m] = 0.5 * (3.0 * a[m] - 4.0 * bb[m] + cc[m]);
        } else {
            double a[5], cc[5]; lv(j + 1, t1, t2, a); lv(j - 1, t1, t2, cc);
            for (int m = 0; m < 5; ++m) dn[m] = 0.5 * (a[m] - cc[m]);
        }
        const double cs2 = L.cs2;
        const double rho = l0[0], T = l0[4];
        double Tv[5];
        transverse(c, j, t1, t2, Tv);
        const size_t r = (size_t)w2(t2) * n1() + w1(t1);
        double Vv[5] = {0, 0, 0, 0, 0};
        if (full3(b)) for (int m = 0; m < 5; ++m) Vv[m] = (*c.V)[r * 5 + m];
        Char5 cs = char_system3(cs2, l0);
        double u0g[5], l00[5];
        for (int m = 0; m < 5; ++m) u0g[m] = (*c.Y0)[((size_t)(j - 1) * n1() * n2() + r) * 5 + m];
        to_local(s, u0g, l00);
        Char5 cs0 = char_system3(cs2, l00);
        double Sd[5], ST[5], SV[5];
        matvec5(cs.Sm, dn, Sd);
        matvec5(cs.Sm, Tv, ST);
        matvec5(cs.Sm, Vv, SV);
        const double K = relax3(b) ? relax_K(s) : 0.0;
        const double alpha = relax3(b) ? rp[s].alpha : 0.0;
        const double Pinf = rp[s].rho_inf * cs2 * rp[s].T_inf;
        double Lb[5];
        for (int i = 0; i < 5; ++i) {
            if (cs0.lam[i] >= 0.0) { Lb[i] = cs.lam[i] * Sd[i]; continue; }
            double in = full3(b) ? ST[i] + SV[i] : 0.0;
            if (relax3(b) && i >= 3) in = in - alpha * ST[i] + K * (rho * cs2 * T - Pinf) / (5.0 * rho * cs2);
            Lb[i] = in;
        }
        double r5[5], rl[5];
        matvec5(cs.Si, Lb, r5);
        for (int m = 0; m < 5; ++m) rl[m] = -r5[m];
        if (full3(b)) for (int m = 0; m < 5; ++m) rl[m] += Tv[m] + Vv[m];
        rate_to_global(s, rl, dU);
    }

    void face_solve(int s, std::vector<double>& Un) {
        const size_t R = (size_t)n1() * n2(), nY = (size_t)M * R * 5;
        std::vector<double> Y0, Ys(nY), Kk(nY, 0.0), acc(nY), V((size_t)R * 5, 0.0);
        layers_of(s, U, Y0);
        if (full3(bc[s]))
            for (int t2 = 0; t2 < n2(); ++t2)
                for (int t1 = 0; t1 < n1(); ++t1) visc_row(sn(s), xf(s) - sn(s) * M, t1, t2, &V[((size_t)t2 * n1() + t1) * 5]);
        FaceCtx c;
        c.s = s; c.Y0 = &Y0; c.Un = &Un; c.V = &V;
        const double a_st[4] = {0.0, 0.5, 0.5, 1.0}, b_st[4] = {1.0, 2.0, 2.0, 1.0};
        acc = Y0;
        for (int st = 0; st < 4; ++st) {
            for (size_t k = 0; k < nY; ++k) Ys[k] = st == 0 ? Y0[k] : Y0[k] + a_st[st] * Kk[k];
            c.Y = &Ys; c.theta = a_st[st];
            std::vector<double> Kn(nY);
            for (int j = 1; j <= M; ++j)
                for (int t2 = 0; t2 < n2(); ++t2)
                    for (int t1 = 0; t1 < n1(); ++t1)
                        face_rhs(c, j, t1, t2, &Kn[((size_t)(j - 1) * R + (size_t)t2 * n1() + t1) * 5]);
            Kk = Kn;
            for (size_t k = 0; k < nY; ++k) acc[k] += (b_st[st] / 6.0) * Kk[k];
        }
        for (int j = 1; j <= M; ++j)
            for (int t2 = 0; t2 < n2(); ++t2)
                for (int t1 = 0; t1 < n1(); ++t1)
                    setU(Un, fid(xk(s, j), t1, t2), &acc[((size_t)(j - 1) * R + (size_t)t2 * n1() + t1) * 5]);
    }

    void step() {
        const size_t P = plane();
        std::vector<double> fs(f.size(), 0.0), fc(f.size(), 0.0), Un(U.size(), 0.0);
        bool per[3] = {true, true, true};
        per[ax] = fper;
        // 1. streaming on bulk nodes (periodic along the tangential axes and, without faces, along
        // the normal one)
#pragma omp parallel for schedule(static)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    if (!is_bulk(x, y, z)) continue;
                    for (int i = 0; i < q; ++i) {
                        int src[3] = {x - L.cx[i], y - L.cy[i], z - L.cz[i]};
                        for (int d = 0; d < 3; ++d)
                            if (per[d]) src[d] = ((src[d] % dim[d]) + dim[d]) % dim[d];
                        fs[i * P + id(x, y, z)] = f[i * P + id(src[0], src[1], src[2])];
                    }
                }
        // 2./3. moments and BGK collision on bulk nodes
#pragma omp parallel
        {
            std::vector<double> fl(q), fe(q);
#pragma omp for schedule(static)
            for (int z = 0; z < nz; ++z)
                for (int y = 0; y < ny; ++y)
                    for (int x = 0; x < nx; ++x) {
                        if (!is_bulk(x, y, z)) continue;
                        const size_t k = id(x, y, z);
                        for (int i = 0; i < q; ++i) fl[i] = fs[i * P + k];
                        double u5[5];
                        moments3(L, fl.data(), u5);
                        setU(Un, k, u5);
                        equilibrium3(L, u5[0], u5[1], u5[2], u5[3], u5[4], fe.data());
                        for (int i = 0; i < q; ++i) fc[i * P + k] = fl[i] - (fl[i] - fe[i]) / tau;
                    }
        }
        // 4. characteristic solve on each face
        for (int s = 0; s < 2; ++s)
            if (char3(bc[s])) face_solve(s, Un);
        // 5. reconstruction of the layers
        for (int s = 0; s < 2; ++s) {
            if (bc[s] == B3_PERIODIC) continue;
            for (int t2 = 0; t2 < n2(); ++t2)
                for (int t1 = 0; t1 < n1(); ++t1)
                    for (int j = 1; j <= M; ++j) {
                        const size_t k = fid(xk(s, j), t1, t2), kf = fid(xf(s), t1, t2);
                        if (bc[s] == B3_ZG) {
                            for (int i = 0; i < q; ++i) fc[i * P + k] = fc[i * P + kf];
                            double u5[5]; node_moments(fc, k, u5); setU(Un, k, u5);
                            continue;
                        }
                        double u5[5]; getU(Un, k, u5); node_feq(fc, k, u5);
                        if (meso[s] == 1) {   // eq. NEEP, post-collision non-equilibrium part of x_f
                            double uf[5]; getU(Un, kf, uf);
                            std::vector<double> fe(q);
                            equilibrium3(L, uf[0], uf[1], uf[2], uf[3], uf[4], fe.data());
                            for (int i = 0; i < q; ++i) fc[i * P + k] += fc[i * P + kf] - fe[i];
                        }
                    }
        }
        // pre-collision populations of the new time level (viscous terms of the next step)
        for (size_t k = 0; k < fs.size(); ++k) {
            const size_t nd = k % P;
            const int x = (int)(nd % nx), y = (int)((nd / nx) % ny), z = (int)(nd / ((size_t)nx * ny));
            fpre[k] = is_bulk(x, y, z) ? fs[k] : fc[k];
        }
        f.swap(fc);
        U.swap(Un);
        ++steps;
    }

    // mass, momentum x/y/z, energy (1/2 sum f |c|^2), loss (interior sum (P - P_inf)^2),
    // max |u|, non-finite count
    void diagnostics(double* out) const {
        double m = 0, jx = 0, jy = 0, jz = 0, e = 0, loss = 0, umax = 0, bad = 0;
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    double r = 0, ax_ = 0, ay = 0, az = 0, en = 0;
                    for (int i = 0; i < q; ++i) {
                        const double fi = f[i * plane() + id(x, y, z)];
                        if (!std::isfinite(fi)) bad += 1;
                        r += fi; ax_ += fi * L.cx[i]; ay += fi * L.cy[i]; az += fi * L.cz[i];
                        en += 0.5 * fi * (L.cx[i] * L.cx[i] + L.cy[i] * L.cy[i] + L.cz[i] * L.cz[i]);
                    }
                    m += r; jx += ax_; jy += ay; jz += az; e += en;
                    umax = std::max(umax, std::sqrt(ax_ * ax_ + ay * ay + az * az) / r);
                    if (is_bulk(x, y, z)) {
                        const double p = L.cs2 * U[id(x, y, z)] * U[4 * plane() + id(x, y, z)] - L.cs2;
                        loss += p * p;
                    }
                }
        out[0] = m; out[1] = jx; out[2] = jy; out[3] = jz; out[4] = e; out[5] = loss; out[6] = umax; out[7] = bad;
    }
};

}  // namespace

// ====================================================================== C interface
extern "C" {

const char* oracle3d_last_error() { return g_err3.c_str(); }

int oracle3d_lattice(int stencil, int* q, int* M, double* cs2, double* w, int* cx, int* cy, int* cz) {
    const Lattice3& L = lattice3(stencil);
    if (L.q == 0) { g_err3 = "stencil must be 39"; return -1; }
    *q = L.q; *M = L.M; *cs2 = L.cs2;
    for (int i = 0; i < L.q; ++i) {
        if (w) w[i] = L.w[i];
        if (cx) cx[i] = L.cx[i];
        if (cy) cy[i] = L.cy[i];
        if (cz) cz[i] = L.cz[i];
    }
    return 0;
}

int oracle3d_feq(int stencil, double rho, double ux, double uy, double uz, double T, double* out) {
    const Lattice3& L = lattice3(stencil);
    if (L.q == 0) return -1;
    equilibrium3(L, rho, ux, uy, uz, T, out);
    return 0;
}

int oracle3d_moments(int stencil, const double* f, double* u5) {
    const Lattice3& L = lattice3(stencil);
    if (L.q == 0) return -1;
    moments3(L, f, u5);
    return 0;
}

// A, S, S^-1 (row-major 5 x 5) and Lambda at a local state U = (rho, u_n, u_t1, u_t2, T)
int oracle3d_char_matrices(int stencil, const double* U, double* A, double* S, double* Si, double* lam) {
    const Lattice3& L = lattice3(stencil);
    if (L.q == 0) return -1;
    Char5 c = char_system3(L.cs2, U);
    for (int k = 0; k < 25; ++k) { A[k] = c.A[k]; S[k] = c.Sm[k]; Si[k] = c.Si[k]; }
    for (int k = 0; k < 5; ++k) lam[k] = c.lam[k];
    return 0;
}

// Faces normal to axis `axis` (0 = x, 1 = y, 2 = z) at its two ends; the other two axes periodic.
void* oracle3d_create_axis(int stencil, int nx, int ny, int nz, double tau, const int* bc, int axis) {
    const Lattice3& L = lattice3(stencil);
    if (L.q == 0) { g_err3 = "stencil must be 39"; return nullptr; }
    if (!(tau > 0.5)) { g_err3 = "tau must exceed 1/2"; return nullptr; }
    if (axis < 0 || axis > 2) { g_err3 = "axis must be 0, 1 or 2"; return nullptr; }
    for (int s = 0; s < 2; ++s)
        if (bc[s] < B3_PERIODIC || bc[s] > B3_ZG) { g_err3 = "unknown boundary type"; return nullptr; }
    if ((bc[0] == B3_PERIODIC) != (bc[1] == B3_PERIODIC)) { g_err3 = "periodic faces come in pairs"; return nullptr; }
    const bool fp = bc[0] == B3_PERIODIC;
    const int d[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a) {
        const int need = (a == axis && !fp) ? 2 * L.M + 3 : L.M + 1;
        if (d[a] < need) { g_err3 = "grid too small"; return nullptr; }
    }
    // the viscous terms of a CBC face are evaluated at x_f - M .. x_f - M - 2 (bulk nodes)
    if ((full3(bc[0]) || full3(bc[1])) && d[axis] < 3 * L.M + 3) { g_err3 = "CBC faces need 3M + 3 nodes across"; return nullptr; }
    return new Sim3(L, nx, ny, nz, tau, bc, axis);
}

void* oracle3d_create(int stencil, int nx, int ny, int nz, double tau, const int* bc) {
    return oracle3d_create_axis(stencil, nx, ny, nz, tau, bc, 0);
}

void oracle3d_destroy(void* h) { delete static_cast<Sim3*>(h); }

int oracle3d_set_relax(void* h, int side, double sigma, double alpha, double rho_inf, double T_inf, double mach,
                       double length) {
    auto* s = static_cast<Sim3*>(h);
    for (int k = 0; k < 2; ++k) {
        if (side >= 0 && k != side) continue;
        s->rp[k].sigma = sigma; s->rp[k].alpha = alpha; s->rp[k].rho_inf = rho_inf;
        s->rp[k].T_inf = T_inf; s->rp[k].mach = mach; s->rp[k].length = length;
    }
    return 0;
}

int oracle3d_set_recon(void* h, int side, int mode) {
    auto* s = static_cast<Sim3*>(h);
    if (side < 0 || side > 1 || mode < 0 || mode > 1) return -1;
    if (mode == 1 && !char3(s->bc[side])) return -1;
    s->meso[side] = mode;
    return 0;
}

int oracle3d_init(void* h, const double* rho, const double* ux, const double* uy, const double* uz, const double* T) {
    static_cast<Sim3*>(h)->init(rho, ux, uy, uz, T);
    return 0;
}

int oracle3d_step(void* h, int n) {
    auto* s = static_cast<Sim3*>(h);
    for (int k = 0; k < n; ++k) s->step();
    return 0;
}

// macroscopic fields [5][nz][ny][nx] = (rho, ux, uy, uz, T)
int oracle3d_macro(void* h, double* out) {
    auto* s = static_cast<Sim3*>(h);
    std::memcpy(out, s->U.data(), s->U.size() * sizeof(double));
    return 0;
}

int oracle3d_pops(void* h, double* out) {
    auto* s = static_cast<Sim3*>(h);
    std::memcpy(out, s->f.data(), s->f.size() * sizeof(double));
    return 0;
}

int oracle3d_diag(void* h, double* out8) {
    static_cast<Sim3*>(h)->diagnostics(out8);
    return 0;
}

// transverse terms (local components) at layer j (1..M) of row (t1, t2) of face `side` (t1, t2:
// coordinates along the axes following the normal, e.g. y and z for x-faces)
int oracle3d_transverse_probe(void* h, int side, int j, int t1, int t2, double* out5) {
    auto* s = static_cast<Sim3*>(h);
    if (side < 0 || side > 1 || s->bc[side] == B3_PERIODIC || j < 1 || j > s->M) return -1;
    if (t1 < 0 || t1 >= s->n1() || t2 < 0 || t2 >= s->n2()) return -1;
    s->transverse_probe(side, j, t1, t2, out5);
    return 0;
}

// V (local frame of outward normal g e_axis, g = +-1) at bulk node (kn, t1, t2) at the current
// time, as a face evaluates it at x_f - sn M; kn, kn - g, kn - 2 g must be bulk nodes
int oracle3d_visc_probe(void* h, int g, int kn, int t1, int t2, double* out5) {
    auto* s = static_cast<Sim3*>(h);
    if ((g != 1 && g != -1) || t1 < 0 || t1 >= s->n1() || t2 < 0 || t2 >= s->n2()) return -1;
    for (int k = 0; k < 3; ++k) {
        const int kk = kn - g * k;
        if (kk < 0 || kk >= s->nn() || !s->is_bulk_n(kk)) return -1;
    }
    s->visc_row(g, kn, t1, t2, out5);
    return 0;
}

}  // extern "C"
