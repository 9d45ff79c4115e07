// lattice3.h -- the D3Q39 stencil and per-node physics of the three-dimensional GPU path.
//
// The paper (Appendix A) points to D3Q39 / D3Q103 for d = 3 without their data.  D3Q39 is the
// degree-7 Gauss-Hermite rule on the velocity groups (0,0,0), (1,0,0), (1,1,1), (2,0,0), (2,2,0),
// (3,0,0) with cs^2 = 2/3 and the rational group weights 1/12, 1/12, 1/27, 2/135, 1/432, 1/1620
// (the solution of the isotropy conditions up to degree 7); it carries the 3rd-order equilibrium
// of eq. feq-3, with d = 3 in its Hermite polynomials.  Maximum displacement M = 3.
//
// Library order as in two dimensions: index 0 is the rest velocity, 1..NP one member of every
// opposite pair, NP+1..2NP their opposites; the equilibrium is evaluated per pair.
#pragma once

#include <hip/hip_runtime.h>

namespace lbm3 {

struct D3Q39 {
    static constexpr int Q = 39, NP = 19, M = 3, NG = 6;
    static constexpr double cs2 = 2.0 / 3.0;
    static constexpr double cs = 0.81649658092772603273242802490196379;
    __host__ __device__ static constexpr int pcx(int p) {
        constexpr int t[20] = {0, 1, 0, 0, 1, -1, 1, 1, 2, 0, 0, 2, -2, 2, -2, 0, 0, 3, 0, 0};
        return t[p];
    }
    __host__ __device__ static constexpr int pcy(int p) {
        constexpr int t[20] = {0, 0, 1, 0, 1, 1, -1, 1, 0, 2, 0, 2, 2, 0, 0, 2, -2, 0, 3, 0};
        return t[p];
    }
    __host__ __device__ static constexpr int pcz(int p) {
        constexpr int t[20] = {0, 0, 0, 1, 1, 1, 1, -1, 0, 0, 2, 0, 0, 2, 2, 2, 2, 0, 0, 3};
        return t[p];
    }
    // symmetry group: 0 (0,0,0), 1 (1,0,0), 2 (1,1,1), 3 (2,0,0), 4 (2,2,0), 5 (3,0,0)
    __host__ __device__ static constexpr int grp(int p) {
        constexpr int t[20] = {0, 1, 1, 1, 2, 2, 2, 2, 3, 3, 3, 4, 4, 4, 4, 4, 4, 5, 5, 5};
        return t[p];
    }
    __host__ __device__ static constexpr double wg(int g) {
        constexpr double t[6] = {1.0 / 12.0, 1.0 / 12.0, 1.0 / 27.0, 2.0 / 135.0, 1.0 / 432.0, 1.0 / 1620.0};
        return t[g];
    }
    __host__ __device__ static constexpr int c2g(int g) { constexpr int t[6] = {0, 1, 3, 4, 8, 9}; return t[g]; }
};

using L3 = D3Q39;

__host__ __device__ constexpr int cx3(int i) { return i == 0 ? 0 : (i <= L3::NP ? L3::pcx(i) : -L3::pcx(i - L3::NP)); }
__host__ __device__ constexpr int cy3(int i) { return i == 0 ? 0 : (i <= L3::NP ? L3::pcy(i) : -L3::pcy(i - L3::NP)); }
__host__ __device__ constexpr int cz3(int i) { return i == 0 ? 0 : (i <= L3::NP ? L3::pcz(i) : -L3::pcz(i - L3::NP)); }
__host__ __device__ constexpr double wt3(int i) { return L3::wg(i == 0 ? 0 : L3::grp(i <= L3::NP ? i : i - L3::NP)); }
__host__ __device__ constexpr int c2_3(int i) { return cx3(i) * cx3(i) + cy3(i) * cy3(i) + cz3(i) * cz3(i); }

// Moments from deviations d_i = f_i - w_i (eq. macro, d = 3): rm1 = rho - 1, u, and
// th = T - 1 from 3 rho cs^2 T = sum f |c|^2 - |j|^2 / rho with sum w |c|^2 = 3 cs^2.
template <typename R>
__device__ __forceinline__ void moments3_dev(const R* d, R& rm1, R& ux, R& uy, R& uz, R& th) {
    R s0 = d[0], jx = 0, jy = 0, jz = 0, e = 0;
#pragma unroll
    for (int p = 1; p <= L3::NP; ++p) {
        const R a = d[p], b = d[p + L3::NP];
        const R sp = a + b, dp = a - b;
        s0 += sp;
        if (cx3(p) != 0) jx += R(cx3(p)) * dp;
        if (cy3(p) != 0) jy += R(cy3(p)) * dp;
        if (cz3(p) != 0) jz += R(cz3(p)) * dp;
        e += R(c2_3(p)) * sp;
    }
    rm1 = s0;
    const R ir = R(1) / (R(1) + s0);
    ux = jx * ir;
    uy = jy * ir;
    uz = jz * ir;
    th = (e - R(3.0 * L3::cs2) * s0 - (jx * jx + jy * jy + jz * jz) * ir) * ir * R(1.0 / (3.0 * L3::cs2));
}

// Equilibrium deviations fe_i - w_i = w_i [(rho - 1) + rho (H_i - 1)] of eq. feq-3 in d = 3, in
// the scaled variables xi = c/cs, u/cs:  H - 1 = a + (a^2 - u^2 + th (xi^2 - 3)) / 2
// + a (a^2 - 3 u^2 + 3 th (xi^2 - 5)) / 6 with a = xi.u; per opposite pair
//   E = C0 + a^2 / 2,  O = a (D0 + a^2 / 6),  C0 = (th (xi^2 - 3) - u^2) / 2,
//   D0 = 1 + (th (xi^2 - 5) - u^2) / 2.
template <typename R>
__device__ __forceinline__ void feq3_dev(R rm1, R ux, R uy, R uz, R th, R* fe) {
    const R rho = R(1) + rm1;
    const R ics = R(1.0 / L3::cs);
    const R vx = ux * ics, vy = uy * ics, vz = uz * ics;
    const R u2 = vx * vx + vy * vy + vz * vz;
    R C0[L3::NG], D0[L3::NG];
#pragma unroll
    for (int g = 0; g < L3::NG; ++g) {
        const R xi2 = R(L3::c2g(g) / L3::cs2);
        C0[g] = R(0.5) * (th * (xi2 - R(3)) - u2);
        D0[g] = R(1) + R(0.5) * (th * (xi2 - R(5)) - u2);
    }
    fe[0] = R(L3::wg(0)) * (rm1 + rho * C0[0]);
#pragma unroll
    for (int p = 1; p <= L3::NP; ++p) {
        const int g = L3::grp(p);
        R a = R(0);
        if (L3::pcx(p) != 0) a += R(L3::pcx(p)) * vx;
        if (L3::pcy(p) != 0) a += R(L3::pcy(p)) * vy;
        if (L3::pcz(p) != 0) a += R(L3::pcz(p)) * vz;
        a *= ics;
        const R a2 = a * a;
        const R E = C0[g] + R(0.5) * a2;
        const R O = a * (D0[g] + a2 * R(1.0 / 6.0));
        const R w = R(L3::wg(g));
        fe[p] = w * (rm1 + rho * (E + O));
        fe[p + L3::NP] = w * (rm1 + rho * (E - O));
    }
}

// BGK collision in deviation form (eq. bgk).  In float the increment's residual in the collision
// invariants is projected off with the degree <= 2 Hermite basis w_i (a0 + a.c + a4 (|c|^2 -
// 3 cs^2)), coefficients from sum w = 1, sum w c c = cs^2 I, sum w (|c|^2 - 3 cs^2)^2 = 6 cs^4
// (zero in exact arithmetic), as in two dimensions.
template <typename R>
__device__ __forceinline__ void collide3_dev(R* d, R omega) {
    R rm1, ux, uy, uz, th;
    moments3_dev<R>(d, rm1, ux, uy, uz, th);
    R fe[L3::Q];
    feq3_dev<R>(rm1, ux, uy, uz, th, fe);
    if (sizeof(R) == 8) {
#pragma unroll
        for (int i = 0; i < L3::Q; ++i) d[i] = d[i] + omega * (fe[i] - d[i]);
        return;
    }
    R m0 = 0, mx = 0, my = 0, mz = 0, me = 0;
#pragma unroll
    for (int i = 0; i < L3::Q; ++i) {
        fe[i] = omega * (fe[i] - d[i]);
        m0 += fe[i];
        if (cx3(i) != 0) mx += R(cx3(i)) * fe[i];
        if (cy3(i) != 0) my += R(cy3(i)) * fe[i];
        if (cz3(i) != 0) mz += R(cz3(i)) * fe[i];
        me += R(c2_3(i)) * fe[i];
    }
    const R ics2 = R(1.0 / L3::cs2);
    const R a0 = m0, a1 = mx * ics2, a2 = my * ics2, a3 = mz * ics2;
    const R a4 = (me - R(3.0 * L3::cs2) * m0) * R(1.0 / (6.0 * L3::cs2 * L3::cs2));
#pragma unroll
    for (int i = 0; i < L3::Q; ++i) {
        R b = a0 + a4 * R(c2_3(i) - 3.0 * L3::cs2);
        if (cx3(i) != 0) b += a1 * R(cx3(i));
        if (cy3(i) != 0) b += a2 * R(cy3(i));
        if (cz3(i) != 0) b += a3 * R(cz3(i));
        d[i] = d[i] + (fe[i] - R(wt3(i)) * b);
    }
}

}  // namespace lbm3
