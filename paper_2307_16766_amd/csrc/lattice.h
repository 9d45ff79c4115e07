// lattice.h -- velocity stencils, weights and per-node physics of the GPU path (gfx950).
//
// Stencils (Appendix B of Klass, Gabbana & Bartel, arXiv 2307.16766):
//   D2Q9  : single speed, cs^2 = 1/3, 2nd-order isothermal equilibrium.
//   D2Q17 : 7th-order Gauss-Hermite rule, max displacement 3, 3rd-order equilibrium (eq. feq-3);
//           the weights are the closed forms in sqrt(193) of Tab. d2q17, cs^2 = 72 / (5 (25 +
//           sqrt 193)) (the caption's expression is 1 / cs).
//   D2Q37 : 9th-order Gauss-Hermite rule, max displacement 3, 4th-order equilibrium (eq. feq-4).
// The D2Q37 weights are the full-precision solution of the isotropy conditions (the table of
// Appendix B prints 14 digits, which leaks mass at the 1e-13 level per step); cs^2 is the real
// root of 35 s^3 - 70 s^2 + 49 s - 12 = 0.
//
// Library order: index 0 is the rest velocity, 1..NP a set of velocities no two of which are
// opposite, NP+1..2NP their opposites (c_{p+NP} = -c_p).  The equilibrium is evaluated per
// opposite pair from its even and odd parts in a = xi.u (one polynomial for both members).
#pragma once

#include <hip/hip_runtime.h>

namespace lbm {

template <int Q> struct Lat;

template <> struct Lat<9> {
    static constexpr int Q = 9, NP = 4, M = 1, NG = 3, order = 2;
    static constexpr bool thermal = false;
    static constexpr double cs2 = 1.0 / 3.0;
    static constexpr double cs = 0.57735026918962576451;
    __host__ __device__ static constexpr int pcx(int p) { constexpr int t[5] = {0, 1, 0, 1, -1}; return t[p]; }
    __host__ __device__ static constexpr int pcy(int p) { constexpr int t[5] = {0, 0, 1, 1, 1}; return t[p]; }
    __host__ __device__ static constexpr int grp(int p) { constexpr int t[5] = {0, 1, 1, 2, 2}; return t[p]; }
    __host__ __device__ static constexpr double wg(int g) {
        constexpr double t[3] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 36.0};
        return t[g];
    }
    __host__ __device__ static constexpr int c2g(int g) { constexpr int t[3] = {0, 1, 2}; return t[g]; }
};

template <> struct Lat<17> {
    static constexpr int Q = 17, NP = 8, M = 3, NG = 5, order = 3;
    static constexpr bool thermal = true;
    static constexpr double cs2 = 0.37025186701833984971891509863238152;
    static constexpr double cs = 0.60848325122252941903029945215239698;
    __host__ __device__ static constexpr int pcx(int p) { constexpr int t[9] = {0, 1, 0, 1, -1, 2, -2, 3, 0}; return t[p]; }
    __host__ __device__ static constexpr int pcy(int p) { constexpr int t[9] = {0, 0, 1, 1, 1, 2, 2, 0, 3}; return t[p]; }
    // symmetry group: 0 (0,0), 1 (1,0), 2 (1,1), 3 (2,2), 4 (3,0)
    __host__ __device__ static constexpr int grp(int p) { constexpr int t[9] = {0, 1, 1, 2, 2, 3, 3, 4, 4}; return t[p]; }
    __host__ __device__ static constexpr double wg(int g) {
        constexpr double t[5] = {0.40200514690911262594166439245907543, 0.11615486649778154387403545662591120,
                                 0.033006353622986913949753825914721682, 7.9078602165918131237133240548163573e-05,
                                 0.00025841454978746755955748610405009878};
        return t[g];
    }
    __host__ __device__ static constexpr int c2g(int g) { constexpr int t[5] = {0, 1, 2, 8, 9}; return t[g]; }
};

template <> struct Lat<37> {
    static constexpr int Q = 37, NP = 18, M = 3, NG = 8, order = 4;
    static constexpr bool thermal = true;
    static constexpr double cs2 = 0.69795332201968308823840905538932529;
    static constexpr double cs = 0.83543600713620375307803652819861195;
    __host__ __device__ static constexpr int pcx(int p) {
        constexpr int t[19] = {0, 1, 0, 1, -1, 2, 0, 2, 1, -1, -2, 2, -2, 3, 0, 3, 1, -1, -3};
        return t[p];
    }
    __host__ __device__ static constexpr int pcy(int p) {
        constexpr int t[19] = {0, 0, 1, 1, 1, 0, 2, 1, 2, 2, 1, 2, 2, 0, 3, 1, 3, 3, 1};
        return t[p];
    }
    // symmetry group: 0 (0,0), 1 (1,0), 2 (1,1), 3 (2,0), 4 (2,1), 5 (2,2), 6 (3,0), 7 (3,1)
    __host__ __device__ static constexpr int grp(int p) {
        constexpr int t[19] = {0, 1, 1, 2, 2, 3, 3, 4, 4, 4, 4, 5, 5, 6, 6, 7, 7, 7, 7};
        return t[p];
    }
    __host__ __device__ static constexpr double wg(int g) {
        constexpr double t[8] = {0.23315066913235250228650670, 0.10730609154221900241246430,
                                 0.057667859888794882030069220, 0.014208216158450750264698940,
                                 0.0053530490005137752327315020, 0.0010119375926735754754109090,
                                 0.00024530102775771734546591660, 0.00028341425299419821740052530};
        return t[g];
    }
    __host__ __device__ static constexpr int c2g(int g) { constexpr int t[8] = {0, 1, 2, 4, 5, 8, 9, 10}; return t[g]; }
};

// full-index accessors (0..Q-1)
template <int Q> __host__ __device__ constexpr int cx(int i) {
    using L = Lat<Q>;
    return i == 0 ? 0 : (i <= L::NP ? L::pcx(i) : -L::pcx(i - L::NP));
}
template <int Q> __host__ __device__ constexpr int cy(int i) {
    using L = Lat<Q>;
    return i == 0 ? 0 : (i <= L::NP ? L::pcy(i) : -L::pcy(i - L::NP));
}
template <int Q> __host__ __device__ constexpr double wt(int i) {
    using L = Lat<Q>;
    return L::wg(i == 0 ? 0 : L::grp(i <= L::NP ? i : i - L::NP));
}
template <int Q> __host__ __device__ constexpr int c2(int i) { return cx<Q>(i) * cx<Q>(i) + cy<Q>(i) * cy<Q>(i); }

// ------------------------------------------------------------------ per-node physics
// Moments from deviations d_i = f_i - w_i (eq. macro): rm1 = rho - 1 = sum d, j, and
// theta = T - 1 from 2 rho cs^2 T = sum f |c|^2 - |j|^2 / rho with sum w |c|^2 = 2 cs^2.
// rho - 1 is kept as its own variable: forming 1 + rm1 and subtracting 1 again would round
// the deviation to the precision of an O(1) number.
template <int Q, typename R>
__device__ __forceinline__ void moments_dev(const R* d, R& rm1, R& ux, R& uy, R& th) {
    R s0 = d[0], jx = 0, jy = 0, e = 0;
#pragma unroll
    for (int p = 1; p <= Lat<Q>::NP; ++p) {
        const R a = d[p], b = d[p + Lat<Q>::NP];
        const R sp = a + b, dp = a - b;
        s0 += sp;
        if (cx<Q>(p) != 0) jx += R(cx<Q>(p)) * dp;
        if (cy<Q>(p) != 0) jy += R(cy<Q>(p)) * dp;
        e += R(c2<Q>(p)) * sp;
    }
    rm1 = s0;
    const R ir = R(1) / (R(1) + s0);
    ux = jx * ir;
    uy = jy * ir;
    if (Lat<Q>::thermal) {
        th = (e - R(2.0 * Lat<Q>::cs2) * s0 - (jx * jx + jy * jy) * ir) * ir * R(0.5 / Lat<Q>::cs2);
    } else {
        th = R(0);
    }
}

// Equilibrium deviations fe_i - w_i = w_i [(rho - 1) + rho (H_i - 1)], with H the bracket of
// eq. feq-3 / feq-4 in the scaled variables xi = c/cs, u/cs (the printed (c^2 - 4) of the
// (u.c)^2 (T-1) term reads (xi^2 - 6) there).  Split per opposite pair into
//   H - 1 = E(a^2) + a O(a^2),  a = xi.u/cs,
//   E = C0 + a^2 (C1 + a^2/24),  O = D0 + a^2/6   (D2Q37, 4th order)
//   E = C0 + a^2 / 2,            O = D0 + a^2/6   (D2Q17, 3rd order: no 4th-order terms)
//   E = (a^2 - u^2)/2,  O = 1                    (D2Q9)
template <int Q, typename R>
__device__ __forceinline__ void feq_dev(R rm1, R ux, R uy, R th, R* fe) {
    using L = Lat<Q>;
    const R rho = R(1) + rm1;
    const R ics = R(1.0 / L::cs);
    const R vx = ux * ics, vy = uy * ics;
    const R u2 = vx * vx + vy * vy;
    R C0[L::NG], C1[L::NG], D0[L::NG];
#pragma unroll
    for (int g = 0; g < L::NG; ++g) {
        if (L::order == 4) {
            const R xi2 = R(L::c2g(g) / L::cs2);
            C0[g] = R(0.5) * (th * (xi2 - R(2)) - u2)
                    + R(0.125) * u2 * u2 + R(0.25) * th * u2 * (R(4) - xi2)
                    + R(0.125) * th * th * (xi2 * xi2 - R(8) * xi2 + R(8));
            C1[g] = R(0.5) + R(0.25) * (th * (xi2 - R(6)) - u2);
            D0[g] = R(1) + R(0.5) * (th * (xi2 - R(4)) - u2);
        } else if (L::order == 3) {
            const R xi2 = R(L::c2g(g) / L::cs2);
            C0[g] = R(0.5) * (th * (xi2 - R(2)) - u2);
            C1[g] = R(0.5);
            D0[g] = R(1) + R(0.5) * (th * (xi2 - R(4)) - u2);
        } else {
            C0[g] = R(-0.5) * u2;
            C1[g] = R(0.5);
            D0[g] = R(1);
        }
    }
    fe[0] = R(L::wg(0)) * (rm1 + rho * C0[0]);
#pragma unroll
    for (int p = 1; p <= L::NP; ++p) {
        const int g = L::grp(p);
        const R a = (R(L::pcx(p)) * vx + R(L::pcy(p)) * vy) * ics;
        const R a2 = a * a;
        R E, O;
        if (L::order == 4) {
            E = C0[g] + a2 * (C1[g] + a2 * R(1.0 / 24.0));
            O = a * (D0[g] + a2 * R(1.0 / 6.0));
        } else if (L::order == 3) {
            E = C0[g] + a2 * C1[g];
            O = a * (D0[g] + a2 * R(1.0 / 6.0));
        } else {
            E = C0[g] + C1[g] * a2;
            O = a;
        }
        const R w = R(L::wg(g));
        fe[p] = w * (rm1 + rho * (E + O));
        fe[p + L::NP] = w * (rm1 + rho * (E - O));
    }
}

// BGK collision (eq. bgk) in deviation form: d* = d + omega (de - d), omega = 1/tau.
// In float the increment D = omega (de - d) carries a rounding residual in the collision
// invariants (mass, momentum, and energy for the thermal stencil) that does not average out:
// the weights rounded to float make sum_i w_i (H_i - 1) differ from zero with a sign fixed by
// the flow.  The residual is removed by subtracting its projection on the degree <= 2 Hermite
// basis, w_i (a0 + a1 c_x + a2 c_y + a3 (|c|^2 - 2 cs^2)), whose coefficients follow from the
// quadrature identities sum w = 1, sum w c_a c_b = cs^2 delta_ab and
// sum w (|c|^2 - 2 cs^2)^2 = 4 cs^4.  In exact arithmetic the projection is zero.
template <int Q, typename R>
__device__ __forceinline__ void collide_dev(R* d, R omega) {
    R rm1, ux, uy, th;
    moments_dev<Q, R>(d, rm1, ux, uy, th);
    R fe[Q];
    feq_dev<Q, R>(rm1, ux, uy, th, fe);
    if (sizeof(R) == 8) {
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] = d[i] + omega * (fe[i] - d[i]);
        return;
    }
    using L = Lat<Q>;
    R m0 = 0, mx = 0, my = 0, me = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        fe[i] = omega * (fe[i] - d[i]);   // the increment
        m0 += fe[i];
        if (cx<Q>(i) != 0) mx += R(cx<Q>(i)) * fe[i];
        if (cy<Q>(i) != 0) my += R(cy<Q>(i)) * fe[i];
        if (L::thermal) me += R(c2<Q>(i)) * fe[i];
    }
    const R a0 = m0, a1 = mx * R(1.0 / L::cs2), a2 = my * R(1.0 / L::cs2);
    const R a3 = L::thermal ? (me - R(2.0 * L::cs2) * m0) * R(0.25 / (L::cs2 * L::cs2)) : R(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        R b = a0 + a1 * R(cx<Q>(i)) + a2 * R(cy<Q>(i));
        if (L::thermal) b += a3 * R(c2<Q>(i) - 2.0 * L::cs2);
        d[i] = d[i] + (fe[i] - R(wt<Q>(i)) * b);
    }
}

}  // namespace lbm
