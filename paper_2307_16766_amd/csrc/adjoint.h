// adjoint.h -- discrete adjoint of the time step of kernels.h (gfx950, FP64 adjoint state).
//
// The paper has no adjoint; this differentiates the discrete map that the GPU path computes.
// State of step n: post-collision populations f^n (all nodes), the boundary layer states U_b^n
// of every characteristic side and the corner states U_c^n.  With g^{n+1}(x) = pull of f^n at x,
//   bulk x          : f^{n+1}(x) = C(g^{n+1}(x))                     (eq. lbe, eq. bgk)
//   strip, diagonal : X^{n+1} = m(g^{n+1}(x_f)), D^{n+1} = m(g^{n+1}(c + v), g^{n+1}(c + 2v))
//   corners         : U_c^{n+1} = RK4_c(U_c^n; D^n, D^{n+1})
//   sides           : U_b^{n+1} = RK4_s(U_b^n; X^n, X^{n+1}, U_c^n, U_c^{n+1})
//   layers, blocks  : f^{n+1} = f^eq(U_b^{n+1}), f^eq(U_c^{n+1})
// with m = (rho, u_x, u_y, T) the moments (eq. macro).  Because the collision conserves the
// moments, m(C(g)) = m(g) identically, so X^n = m(g^n(x_f)) as a function.
//
// Adjoint variables (all FP64):
//   V(x) : nu = dL/dg at bulk nodes (adjoint of the pulled, pre-collision populations);
//          lambda = dL/df at boundary-layer and corner-block nodes;
//   adjoint region (same offsets as the forward region): direct adjoints of U_b^n, of the
//          strip X^n and corner diagonal D^n as time-n inputs, and of U_c^n.
// One reverse step n+1 -> n is two launches (three when the corners read the sides' terms):
//   k_adj_side   : per chunk of side rows, fold lambda^{n+1} of the layers into the adjoint of
//                  U_b^{n+1} (J_feq^T), reverse the four RK4 stages (stage inputs stored by the
//                  recomputation) with a hand-written VJP of the characteristic rate, emit the
//                  adjoints of U_b^n and X^n, add the adjoint of X^{n+1} to nu^{n+1}(x_f) through
//                  J_m^T, and accumulate the adjoints of K and alpha; further blocks reverse the
//                  corners (fold of the M x M block, reverse corner RK4), or k_adj_corner does
//                  after the sides when transverse relaxation couples the sides to the corners;
//   k_adj_bulk   : lambda^n(y, i) = nu^{n+1}(y + c_i, i) (reverse pull, bulk sources only, plus
//                  the corner diagonal nodes' corrections), nu^n = J_C^T lambda^n at bulk nodes:
//                  nu_i = (1 - omega) lambda_i + omega (G_0 + c_ix G_1 + c_iy G_2 + |c_i|^2 G_3),
//                  G = (dm/dM)^T (df^eq/dm)^T lambda, M the linear moments (sum f, sum f c,
//                  sum f |c|^2); at n = 0 it gives dL/d(rho0, ux0, uy0, T0) = (df^eq/dm)^T lambda^0.
// Supported boundaries: all of them.  CBC sides with the mesoscopic viscous terms add their VJP
// at the nodes x_f - M .. x_f - M - 2, NEEP and zero-gradient sides add terms of nu^{n+1}(x_f); the layers
// of a Dirichlet side are constants of the given profile, or, with the default profile (the
// initial state of the first layer), collect the adjoint of that profile (k_adj_dir_collect).
#pragma once

#include "kernels.h"

namespace lbm {

// ------------------------------------------------------------------ per-node adjoint pieces
// G = (d f^eq / d(rho, ux, uy, T))^T lam, from the pair form of feq_dev: per opposite pair
// H - 1 = E(a) +- O(a), so sum_pm lam w H = w (S (1 + E) + D O) with S, D the sum and
// difference of the pair's lam.
template <int Q>
__device__ __forceinline__ void feq_vjp(const double* m, const double* lam, double* G) {
    using L = Lat<Q>;
    const double rho = m[0];
    const double th = L::thermal ? m[3] - 1.0 : 0.0;
    const double ics = 1.0 / L::cs;
    const double vx = m[1] * ics, vy = m[2] * ics;
    const double u2 = vx * vx + vy * vy;
    double C0[L::NG], C1[L::NG], D0[L::NG], C0t[L::NG], C0u[L::NG], C1t[L::NG], D0t[L::NG];
#pragma unroll
    for (int g = 0; g < L::NG; ++g) {
        if (L::order == 3) {
            const double xi2 = L::c2g(g) / L::cs2;
            C0[g] = 0.5 * (th * (xi2 - 2.0) - u2);
            C1[g] = 0.5;
            D0[g] = 1.0 + 0.5 * (th * (xi2 - 4.0) - u2);
            C0t[g] = 0.5 * (xi2 - 2.0);
            C0u[g] = -0.5;
            C1t[g] = 0.0;
            D0t[g] = 0.5 * (xi2 - 4.0);
        } else if (L::thermal) {
            const double xi2 = L::c2g(g) / L::cs2;
            const double x4 = xi2 * xi2 - 8.0 * xi2 + 8.0;
            C0[g] = 0.5 * (th * (xi2 - 2.0) - u2) + 0.125 * u2 * u2 + 0.25 * th * u2 * (4.0 - xi2) + 0.125 * th * th * x4;
            C1[g] = 0.5 + 0.25 * (th * (xi2 - 6.0) - u2);
            D0[g] = 1.0 + 0.5 * (th * (xi2 - 4.0) - u2);
            C0t[g] = 0.5 * (xi2 - 2.0) + 0.25 * u2 * (4.0 - xi2) + 0.25 * th * x4;
            C0u[g] = -0.5 + 0.25 * u2 + 0.25 * th * (4.0 - xi2);
            C1t[g] = 0.25 * (xi2 - 6.0);
            D0t[g] = 0.5 * (xi2 - 4.0);
        } else {
            C0[g] = -0.5 * u2; C1[g] = 0.5; D0[g] = 1.0;
            C0t[g] = 0.0; C0u[g] = -0.5; C1t[g] = 0.0; D0t[g] = 0.0;
        }
    }
    double gr = L::wg(0) * lam[0] * (1.0 + C0[0]);
    double gth = L::wg(0) * lam[0] * C0t[0];
    double gu2 = L::wg(0) * lam[0] * C0u[0];
    double gvx = 0.0, gvy = 0.0;
#pragma unroll
    for (int p = 1; p <= L::NP; ++p) {
        const int g = L::grp(p);
        const double w = L::wg(g);
        const double a = (L::pcx(p) * vx + L::pcy(p) * vy) * ics;
        const double a2 = a * a;
        const double S = lam[p] + lam[p + L::NP], D = lam[p] - lam[p + L::NP];
        double E, O, Et, Ot, Eu, Ou, Ea, Oa;
        if (L::order == 3) {
            E = C0[g] + a2 * C1[g];
            O = a * (D0[g] + a2 * (1.0 / 6.0));
            Et = C0t[g];
            Ot = a * D0t[g];
            Eu = C0u[g];
            Ou = -0.5 * a;
            Ea = 2.0 * a * C1[g];
            Oa = D0[g] + 0.5 * a2;
        } else if (L::thermal) {
            E = C0[g] + a2 * (C1[g] + a2 * (1.0 / 24.0));
            O = a * (D0[g] + a2 * (1.0 / 6.0));
            Et = C0t[g] + a2 * C1t[g];
            Ot = a * D0t[g];
            Eu = C0u[g] - 0.25 * a2;
            Ou = -0.5 * a;
            Ea = 2.0 * a * C1[g] + a2 * a * (1.0 / 6.0);
            Oa = D0[g] + 0.5 * a2;
        } else {
            E = C0[g] + C1[g] * a2;
            O = a;
            Et = 0.0; Ot = 0.0;
            Eu = -0.5; Ou = 0.0;
            Ea = a; Oa = 1.0;
        }
        gr += w * (S * (1.0 + E) + D * O);
        gth += w * (S * Et + D * Ot);
        gu2 += w * (S * Eu + D * Ou);
        const double ga = w * (S * Ea + D * Oa);
        if (L::pcx(p) != 0) gvx += L::pcx(p) * ga;
        if (L::pcy(p) != 0) gvy += L::pcy(p) * ga;
    }
    // f^eq = w rho (1 + E +- O): every term but the first carries the factor rho
    G[0] = gr;
    G[1] = rho * (gvx * ics + 2.0 * vx * gu2) * ics;
    G[2] = rho * (gvy * ics + 2.0 * vy * gu2) * ics;
    G[3] = L::thermal ? rho * gth : 0.0;
}

// GM = (dm/dM)^T G for m = (rho, ux, uy, T) as functions of M = (sum f, sum f c_x, sum f c_y,
// sum f |c|^2): rho = M0, u = (M1, M2)/rho, T = (M3 - |j|^2/rho) / (2 rho cs^2).
template <int Q>
__device__ __forceinline__ void mom_vjp(const double* m, const double* G, double* GM) {
    const double ir = 1.0 / m[0];
    const double ux = m[1], uy = m[2];
    if (Lat<Q>::thermal) {
        const double k = 0.5 * ir / Lat<Q>::cs2;
        GM[0] = G[0] - (ux * G[1] + uy * G[2]) * ir + (ux * ux + uy * uy - 2.0 * Lat<Q>::cs2 * m[3]) * k * G[3];
        GM[1] = G[1] * ir - 2.0 * k * ux * G[3];
        GM[2] = G[2] * ir - 2.0 * k * uy * G[3];
        GM[3] = k * G[3];
    } else {
        GM[0] = G[0] - (ux * G[1] + uy * G[2]) * ir;
        GM[1] = G[1] * ir;
        GM[2] = G[2] * ir;
        GM[3] = 0.0;
    }
}

template <int Q>
__device__ __forceinline__ double phi_dot(int i, const double* GM) {
    double v = GM[0];
    if (cx<Q>(i) != 0) v += cx<Q>(i) * GM[1];
    if (cy<Q>(i) != 0) v += cy<Q>(i) * GM[2];
    if (Lat<Q>::thermal) v += c2<Q>(i) * GM[3];
    return v;
}

// VJP of char_rate for the four schemes of Tab. CBCs.  Viscous terms of the CBC variants: with
// vfd, those of the -FD variant (Sec. 4.2), evaluated from the stage values as in the forward step:
// V = (0, nu lap u_n, nu lap u_t, 2 nu lap T + (nu / cs^2)(sa^2 + sb^2)), lap = d2n + up - 2 U +
// dw, sa = dn u_n - d_t u_t, sb = d_t u_n + dn u_t, differentiated through the stage values;
// without vfd, the mesoscopic terms Vin (frozen over the stages, an input), whose adjoint is
// returned in Vb.  Inputs as char_rate plus the second normal difference d2n; rb = adjoint of
// the rate; outputs the adjoints of U, dn, d2n, up, dw (side-local components), of V and of K
// and alpha.  The wave directions are frozen at time t (no derivative).
template <int Q, bool CBC>
__device__ __forceinline__ void char_rate_vjp(const double* U, const double* dn, const double* d2n, const double* up,
                                              const double* dw, const double* Vin, const double* U0, int scheme,
                                              int vfd, double nu, double K, double alpha, double Pinf, const double* rb,
                                              double* Ub, double* dnb, double* d2nb, double* upb, double* dwb,
                                              double* Vb, double& Kb, double& alb) {
    constexpr bool THERMAL = Lat<Q>::thermal;
    constexpr double cs2 = Lat<Q>::cs2;
    constexpr double cs = Lat<Q>::cs;
    const bool full = CBC && THERMAL && (scheme == BC_CBC || scheme == BC_CBC_RELAX);
    const bool relax = scheme == BC_LODI_RELAX || (CBC && scheme == BC_CBC_RELAX);
    const double rho = U[0], u = U[1], v = U[2], T = U[3];
    const double ir = 1.0 / rho;
    const double T1 = -0.5 * (up[0] * up[2] - dw[0] * dw[2]);
    const double T2 = -v * 0.5 * (up[1] - dw[1]);
    // T3 enters the rate and in2 linearly: only its adjoint T3b is needed
    const double T4 = THERMAL ? -0.5 * (up[3] * up[2] - dw[3] * dw[2]) : 0.0;
    const double u0 = U0[1];
    double rhob = 0.0, ub = 0.0, vb = 0.0, Tb = 0.0, T1b = 0.0, T2b = 0.0, T3b = 0.0, T4b = 0.0;
    for (int m = 0; m < 4; ++m) { dnb[m] = 0.0; d2nb[m] = 0.0; upb[m] = 0.0; dwb[m] = 0.0; Vb[m] = 0.0; }
    Kb = 0.0;
    alb = 0.0;
    if (THERMAL) {
        // viscous terms (zero for the LODI schemes)
        double lap[4] = {0.0, 0.0, 0.0, 0.0}, V1 = 0.0, V3 = 0.0, sa = 0.0, sh = 0.0;   // V2 enters the rate only
        if (full && vfd) {
            for (int m = 1; m < 4; ++m) lap[m] = d2n[m] + up[m] - 2.0 * U[m] + dw[m];
            sa = dn[1] - 0.5 * (up[2] - dw[2]);
            sh = 0.5 * (up[1] - dw[1]) + dn[2];
            V1 = nu * lap[1];
            V3 = 2.0 * nu * lap[3] + nu * (1.0 / cs2) * (sa * sa + sh * sh);
        } else if (full) {
            V1 = Vin[1];
            V3 = Vin[3];
        }
        const double s = sqrt(2.0 * cs2 * T);
        const double s0 = sqrt(2.0 * cs2 * U0[3]);
        // reciprocals taken once (each division is a long dependent sequence on the stage's chain)
        const double iT = 1.0 / T, is = 1.0 / s;
        const double a = 0.25 * T * ir, b = s * (0.25 / cs2);
        const double W3 = a * dn[0] - b * dn[1] + 0.25 * dn[3];
        const double W4 = a * dn[0] + b * dn[1] + 0.25 * dn[3];
        const double L1 = u * (-2.0 * a * dn[0] + 0.5 * dn[3]);
        const double L3 = (u - s) * W3, L4 = (u + s) * W4;
        const double ST1 = -2.0 * a * T1 + 0.5 * T4;
        const double ST3 = a * T1 - b * T2 + 0.25 * T4, ST4 = a * T1 + b * T2 + 0.25 * T4;
        double in1 = 0.0, in3 = 0.0, in4 = 0.0;
        if (full) {
            in1 = ST1 + 0.5 * V3;
            in3 = ST3 - b * V1 + 0.25 * V3;
            in4 = ST4 + b * V1 + 0.25 * V3;
        }
        const double pr = relax ? K * (rho * cs2 * T - Pinf) * ir * (0.25 / cs2) : 0.0;
        if (relax) {
            in3 += pr - alpha * ST3;
            in4 += pr - alpha * ST4;
        }
        const bool o1 = u0 >= 0.0, o3 = u0 - s0 >= 0.0, o4 = u0 + s0 >= 0.0;
        const double B1 = o1 ? L1 : in1, B3 = o3 ? L3 : in3, B4 = o4 ? L4 : in4;
        const double rhoT = rho * iT, q = 2.0 * cs2 * is;
        const double Bb1 = rb[0] * rhoT - rb[3];
        const double Bb2 = -rb[2];
        const double Bb3 = -rb[0] * rhoT + rb[1] * q - rb[3];
        const double Bb4 = -rb[0] * rhoT - rb[1] * q - rb[3];
        const double Bs = B1 - B3 - B4;
        rhob += rb[0] * Bs * iT;
        Tb += -rb[0] * rho * Bs * iT * iT;
        double sb = -rb[1] * q * (B3 - B4) * is;
        const double L1b = o1 ? Bb1 : 0.0, L2b = o1 ? Bb2 : 0.0, L3b = o3 ? Bb3 : 0.0, L4b = o4 ? Bb4 : 0.0;
        const double in1b = o1 ? 0.0 : Bb1, in2b = o1 ? 0.0 : Bb2;
        const double in3b = o3 ? 0.0 : Bb3, in4b = o4 ? 0.0 : Bb4;
        double ab = 0.0, bb = 0.0, ST1b = 0.0, ST3b = 0.0, ST4b = 0.0, V1b = 0.0, V2b = 0.0, V3b = 0.0;
        if (relax) {
            const double prb = in3b + in4b;
            alb = -(in3b * ST3 + in4b * ST4);
            ST3b -= alpha * in3b;
            ST4b -= alpha * in4b;
            Kb = prb * (rho * cs2 * T - Pinf) * ir * (0.25 / cs2);
            // pr = K (T / 4 - Pinf / (4 cs^2 rho))
            Tb += prb * K * 0.25;
            rhob += prb * K * 0.25 * Pinf * ir * ir * (1.0 / cs2);
        }
        if (full) {
            // incoming amplitudes S (T + V) (in2 = T3 + V2) and the direct T + V of the rate
            ST1b += in1b;
            V3b += 0.5 * in1b + 0.25 * (in3b + in4b) + rb[3];
            T3b += in2b + rb[2];
            V2b += in2b + rb[2];
            ST3b += in3b;
            ST4b += in4b;
            bb += V1 * (in4b - in3b);
            V1b += b * (in4b - in3b) + rb[1];
            T1b += rb[0];
            T2b += rb[1];
            T4b += rb[3];
        }
        ab += -2.0 * T1 * ST1b;
        T1b += -2.0 * a * ST1b;
        T4b += 0.5 * ST1b;
        ab += T1 * (ST3b + ST4b);
        T1b += a * (ST3b + ST4b);
        bb += T2 * (ST4b - ST3b);
        T2b += b * (ST4b - ST3b);
        T4b += 0.25 * (ST3b + ST4b);
        // amplitudes
        ub += (-2.0 * a * dn[0] + 0.5 * dn[3]) * L1b;
        ab += -2.0 * u * dn[0] * L1b;
        dnb[0] += -2.0 * a * u * L1b;
        dnb[3] += 0.5 * u * L1b;
        ub += dn[2] * L2b;
        dnb[2] += u * L2b;
        ub += W3 * L3b + W4 * L4b;
        sb += -W3 * L3b + W4 * L4b;
        const double W3b = (u - s) * L3b, W4b = (u + s) * L4b;
        ab += dn[0] * (W3b + W4b);
        dnb[0] += a * (W3b + W4b);
        bb += dn[1] * (W4b - W3b);
        dnb[1] += b * (W4b - W3b);
        dnb[3] += 0.25 * (W3b + W4b);
        // b = s / (4 cs^2), a = T / (4 rho), s = sqrt(2 cs^2 T)
        sb += bb * (0.25 / cs2);
        Tb += ab * 0.25 * ir;
        rhob += -ab * 0.25 * T * ir * ir;
        Tb += sb * cs2 * is;
        if (full && !vfd) {
            Vb[1] = V1b;
            Vb[2] = V2b;
            Vb[3] = V3b;
        }
        if (full && vfd) {
            // viscous terms: lap = d2n + up - 2 U + dw; heating from sa and sh
            const double lb[4] = {0.0, nu * V1b, nu * V2b, 2.0 * nu * V3b};
            const double sab = 2.0 * nu * (1.0 / cs2) * sa * V3b, shb = 2.0 * nu * (1.0 / cs2) * sh * V3b;
            for (int m = 1; m < 4; ++m) {
                d2nb[m] += lb[m];
                upb[m] += lb[m];
                dwb[m] += lb[m];
            }
            ub += -2.0 * lb[1];
            vb += -2.0 * lb[2];
            Tb += -2.0 * lb[3];
            dnb[1] += sab;
            upb[2] += -0.5 * sab;
            dwb[2] += 0.5 * sab;
            upb[1] += 0.5 * shb;
            dwb[1] += -0.5 * shb;
            dnb[2] += shb;
        }
        if (full) {
            // T3 = -cs^2 / rho * (d_t (rho T)) - v d_t u_t (central differences)
            rhob += cs2 * ir * ir * 0.5 * (up[0] * up[3] - dw[0] * dw[3]) * T3b;
            upb[0] += -cs2 * ir * 0.5 * up[3] * T3b;
            upb[3] += -cs2 * ir * 0.5 * up[0] * T3b;
            dwb[0] += cs2 * ir * 0.5 * dw[3] * T3b;
            dwb[3] += cs2 * ir * 0.5 * dw[0] * T3b;
            vb += -0.5 * (up[2] - dw[2]) * T3b;
            upb[2] += -0.5 * v * T3b;
            dwb[2] += 0.5 * v * T3b;
        }
    } else {
        const double c = cs;
        const double Wm = cs2 * dn[0] - rho * c * dn[1], Wp = cs2 * dn[0] + rho * c * dn[1];
        const double Lm = (u - c) * Wm, Lp = (u + c) * Wp;
        const double pr = relax ? K * (cs2 * rho - Pinf) : 0.0;
        const double inm = relax ? pr - alpha * (cs2 * T1 - rho * c * T2) : 0.0;
        const double inp = relax ? pr - alpha * (cs2 * T1 + rho * c * T2) : 0.0;
        const bool o0 = u0 >= 0.0, om = u0 - c >= 0.0, op = u0 + c >= 0.0;
        const double Bm = om ? Lm : inm, Bp = op ? Lp : inp;
        const double Bmb = -rb[0] * (0.5 / cs2) + rb[1] * (0.5 / c) * ir;
        const double Bpb = -rb[0] * (0.5 / cs2) - rb[1] * (0.5 / c) * ir;
        const double B0b = -rb[2];
        rhob += -rb[1] * (Bm - Bp) * (0.5 / c) * ir * ir;
        const double L0b = o0 ? B0b : 0.0, Lmb = om ? Bmb : 0.0, Lpb = op ? Bpb : 0.0;
        const double inmb = om ? 0.0 : Bmb, inpb = op ? 0.0 : Bpb;
        ub += dn[2] * L0b;
        dnb[2] += u * L0b;
        ub += Wm * Lmb + Wp * Lpb;
        const double Wmb = (u - c) * Lmb, Wpb = (u + c) * Lpb;
        dnb[0] += cs2 * (Wmb + Wpb);
        dnb[1] += rho * c * (Wpb - Wmb);
        rhob += c * dn[1] * (Wpb - Wmb);
        if (relax) {
            const double prb = inmb + inpb;
            Kb = prb * (cs2 * rho - Pinf);
            rhob += prb * K * cs2;
            alb = -(inmb * (cs2 * T1 - rho * c * T2) + inpb * (cs2 * T1 + rho * c * T2));
            T1b += -alpha * cs2 * (inmb + inpb);
            T2b += alpha * rho * c * (inmb - inpb);
            rhob += alpha * c * T2 * (inmb - inpb);
        }
    }
    // transverse terms T1, T2, T4 (eq. NSF-CHAR, central differences)
    upb[0] += -0.5 * up[2] * T1b;
    upb[2] += -0.5 * up[0] * T1b;
    dwb[0] += 0.5 * dw[2] * T1b;
    dwb[2] += 0.5 * dw[0] * T1b;
    vb += -0.5 * (up[1] - dw[1]) * T2b;
    upb[1] += -0.5 * v * T2b;
    dwb[1] += 0.5 * v * T2b;
    if (THERMAL) {
        upb[3] += -0.5 * up[2] * T4b;
        upb[2] += -0.5 * up[3] * T4b;
        dwb[3] += 0.5 * dw[2] * T4b;
        dwb[2] += 0.5 * dw[3] * T4b;
    }
    Ub[0] = rhob; Ub[1] = ub; Ub[2] = vb; Ub[3] = THERMAL ? Tb : 0.0;
}

// VJP of corner_rate: adjoints of Uc, U1, U2 (global components) and of K
template <int Q>
__device__ __forceinline__ void corner_rate_vjp(const CornerDev& c, const double* Uc, const double* U1, const double* U2,
                                                const double* Un, const double* rb, double* Ucb, double* U1b,
                                                double* U2b, double& Kb) {
    const double tdx = -c.ndy, tdy = c.ndx;
    double l0[4], l1[4], l2[4], ln[4];
    auto loc = [&](const double* g, double* l) {
        l[0] = g[0]; l[1] = g[1] * c.ndx + g[2] * c.ndy; l[2] = g[1] * tdx + g[2] * tdy; l[3] = g[3];
    };
    auto loc_t = [&](const double* l, double* g) {   // transpose of loc
        g[0] = l[0]; g[1] = l[1] * c.ndx + l[2] * tdx; g[2] = l[1] * c.ndy + l[2] * tdy; g[3] = l[3];
    };
    loc(Uc, l0); loc(U1, l1); loc(U2, l2); loc(Un, ln);
    constexpr double inv = 0.35355339059327376220;
    double dn[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) dn[k] = (3.0 * l0[k] - 4.0 * l1[k] + l2[k]) * inv;
    double rl[4];
    rl[0] = rb[0];
    rl[1] = rb[1] * c.ndx + rb[2] * c.ndy;
    rl[2] = rb[1] * tdx + rb[2] * tdy;
    rl[3] = rb[3];
    double Ub[4], dnb[4], d2nb[4], upb[4], dwb[4], Vb[4], alb;
    const double zero4[4] = {0.0, 0.0, 0.0, 0.0};
    char_rate_vjp<Q, false>(l0, dn, zero4, l0, l0, zero4, ln, c.relax ? BC_LODI_RELAX : BC_LODI, 0, 0.0, c.K, 0.0, c.Pinf, rl,
                     Ub, dnb, d2nb, upb, dwb, Vb, Kb, alb);
    double a0[4], a1[4], a2[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        a0[k] = Ub[k] + upb[k] + dwb[k] + 3.0 * inv * dnb[k];
        a1[k] = -4.0 * inv * dnb[k];
        a2[k] = inv * dnb[k];
    }
    loc_t(a0, Ucb); loc_t(a1, U1b); loc_t(a2, U2b);
}

// ------------------------------------------------------------------ kernel arguments
struct AdjArgs {
    BndArgs b;               // geometry and relaxation; reg_cur = forward region of time n, reg_next = n+1
    char* adj_cur;           // adjoint region of time n (written)
    const char* adj_next;    // adjoint region of time n+1 (read)
    double* ccon;            // [corner][side axis][n, n+1][4]: side contributions to the corner adjoints
    double* gm;              // corrections of nu^{n+1} at the corner diagonal nodes, (dm/dM)^T Xbar:
                             // [side][row 0, row len-1][4] (end rows of the strips, = c + v), then
                             // [corner][c + v, c + 2v][4] (the corner's own)
    double* acc;             // [side blocks][2] (dK, dalpha), then [corner] (dK)
    double* V1;              // nu / lambda of time n+1
    double* V0;              // nu / lambda of time n (written by k_adj_bulk)
    const double* mom;       // moments of time n, planes [4][ny][pitch]
    const double* mom1;      // moments of time n + 1 (bulk nodes), same layout
    double* grad;            // n = 0: dL/d(rho0, ux0, uy0, T0), [4][ny][nx]
    int ablk0[4], anblk[4];  // side blocks of k_adj_side
    int arows[4];            // owned rows per side block, per side
    int nadj;                // total side blocks
    int cside[4][2];         // per corner: adjacent side of each axis (-1 if none)
    int crow[4][2];          // per corner: that side's row next to the corner
    int coupled;             // corners read the sides' contributions (transverse relaxation alpha != 0)
    int vism;                // some CBC side uses the mesoscopic viscous terms
    int neep_any;            // some characteristic side uses NEEP (eq. NEEP)
    double* neep[4];         // per NEEP or zero-gradient side, row r: the terms a_i [Q] and GM [4] that
                             // nu^{n+1}(x_f) gets as a_i - phi_i . GM; NULL for other sides
    double* zgc;             // per zero-gradient corner: the same terms for nu^{n+1}(c + v), [4][Q + 4]
    int zgc_any;
    double* dacc[4];         // per Dirichlet side with the default profile: [M][len][4] adjoint of the
                             // row's profile collected per layer node; NULL for other sides
    const double* dprof[4];  // that side's profile [len][4] (rho, ux, uy, T)
    int dir_any;
};

// ------------------------------------------------------------------ reverse of a side chunk
// LDS row lr <-> side row r = r0 - 8 + lr.  Owned rows [r0, r1).  Reverse dependencies: the
// adjoint of U_b^n on owned rows needs stage s's VJP within s + 1 rows of them, which needs the
// stage inputs within s + 2 rows (stored by the recomputation of the step, k_step with HIST).
template <int Q, bool CBC>
__device__ void adj_chunk(const AdjArgs& g, const SideDev& sd, int side, int blk, int chunk) {
    constexpr int M = Lat<Q>::M, NR = 256 / M, MS = (M == 1) ? 2 : 1, H = 8, NN = NR * M;
    __shared__ double sY[4][NN * 4];            // stage inputs Y_0 = U_b^n, Y_1, Y_2, Y_3 (global components)
    // per node and stage (double-buffered: one barrier per reverse stage): adjoints of dn, up, dw
    // and of d2n (-FD viscous terms)
    __shared__ double sGn[2][NN * 4], sGu[2][NN * 4], sGd[2][NN * 4];
    __shared__ double sG2[2][(M == 3 ? NN : 1) * 4];
    __shared__ double sVr[NR * 4];                             // per row: mesoscopic viscous terms of time n
    __shared__ double sXn[NR * MS * 4], sXp[NR * MS * 4];       // strip values at n, n+1
    __shared__ double sXbn[NR * MS * 4], sXbp[NR * MS * 4];     // strip adjoints (owned rows)
    __shared__ double sC[2][2][4];
    __shared__ double sCb[2][2][M][4];
    __shared__ double sRed[2][4];
    const BndArgs& a = g.b;
    const int tid = threadIdx.x;
    const int len = sd.len, tper = sd.tper;
    const int r0 = chunk * g.arows[side];
    const int r1 = min(r0 + g.arows[side], len);
    const int nlr = min(NR, r1 - r0 + 2 * H);   // LDS rows in use
    const double* ubn = (const double*)(a.reg_cur + sd.off_ub);
    const double* ubp = (const double*)(a.reg_next + sd.off_ub);
    const double* stn = (const double*)(a.reg_cur + sd.off_strip);
    const double* stp = (const double*)(a.reg_next + sd.off_strip);
    const double* mub1 = (const double*)(g.adj_next + sd.off_ub);
    double* mub0 = (double*)(g.adj_cur + sd.off_ub);
    double* xbo = (double*)(g.adj_cur + sd.off_strip);
    const double* xbp = (const double*)(g.adj_next + sd.off_strip);
    auto valid = [&](int r) { return tper || (r >= 0 && r < len); };
    auto phys = [&](int r) { return tper ? ((r % len) + len) % len : r; };
    auto within = [&](int r, int h) { return r >= r0 - h && r < r1 + h; };

    // ---- phase A: time-n and time-(n+1) values, fold of lambda^{n+1} on the layers ----------
    const int t = tid;
    const int lr = t / M, jj = t % M, j = jj + 1, r = r0 - H + lr;
    const bool node = t < NN && lr < nlr && valid(r);
    double yb1[4] = {0.0, 0.0, 0.0, 0.0};   // adjoint of this node's U_b^{n+1}
    // every load of this phase is issued before the first use of any, so that their latencies
    // overlap (a store to LDS waits for its value, and waits on loads go in issue order)
    const bool fold = node && within(r, 4);
    const int rp = node ? phys(r) : 0;
    double y0v[4], yv[3][4], u4[4], mb[4], lam[Q];
    if (node) {
        // stage inputs Y_0 = U_b^n and Y_1..Y_3 (stored by the recomputation of this step)
        const double* ys = (const double*)(a.reg_next + sd.off_stage);
        for (int m = 0; m < 4; ++m) y0v[m] = ubn[((size_t)jj * len + rp) * 4 + m];
        for (int st = 1; st <= 3; ++st)
            for (int m = 0; m < 4; ++m) yv[st - 1][m] = ys[(((size_t)(st - 1) * M + jj) * len + rp) * 4 + m];
    }
    if (fold) {   // lambda^{n+1} of this layer node, folded into the adjoint of U_b^{n+1} below
        for (int m = 0; m < 4; ++m) u4[m] = ubp[((size_t)jj * len + rp) * 4 + m];
        for (int m = 0; m < 4; ++m) mb[m] = mub1[((size_t)jj * len + rp) * 4 + m];
        int x, y; side_node(sd, j, rp, x, y);
#pragma unroll
        for (int i = 0; i < Q; ++i) lam[i] = g.V1[pix<Q>(a.pitch, i, x, y)];
    }
    double cval = 0.0;
    // this work-group's running sums of the parameter adjoints, added to at the end
    const double acc0 = tid < 2 ? g.acc[blk * 2 + tid] : 0.0;
    if (!tper && tid < 16) {
        // the two corners' offsets read with uniform indices (see uniform_corner)
        const unsigned long long oLo = uni(a.c[sd.corner_lo < 0 ? 0 : sd.corner_lo].off_cu);
        const unsigned long long oHi = uni(a.c[sd.corner_hi < 0 ? 0 : sd.corner_hi].off_cu);
        const int e = tid / 8, w = (tid / 4) % 2, m = tid % 4;
        const char* reg = w == 0 ? a.reg_cur : a.reg_next;
        cval = ((const double*)(reg + (e == 0 ? oLo : oHi)))[m];
    }
    for (int e = tid; e < nlr * MS; e += blockDim.x) {
        const int l2 = e / MS, k = e % MS, rr = r0 - H + l2;
        for (int m = 0; m < 4; ++m) { sXbn[e * 4 + m] = 0.0; sXbp[e * 4 + m] = 0.0; }
        if (!valid(rr)) continue;
        double xn[4], xp[4];
        for (int m = 0; m < 4; ++m) {
            xn[m] = stn[((size_t)k * len + phys(rr)) * 4 + m];
            xp[m] = stp[((size_t)k * len + phys(rr)) * 4 + m];
        }
        for (int m = 0; m < 4; ++m) { sXn[e * 4 + m] = xn[m]; sXp[e * 4 + m] = xp[m]; }
    }
    if (!tper && tid < 16) (&sC[0][0][0])[tid] = cval;   // [e][w][m] = tid / 8, (tid / 4) % 2, tid % 4
    if (node) {
        for (int m = 0; m < 4; ++m) sY[0][t * 4 + m] = y0v[m];
        for (int st = 1; st <= 3; ++st)
            for (int m = 0; m < 4; ++m) sY[st][t * 4 + m] = yv[st - 1][m];
    }
    if (fold) {
        double G[4];
        feq_vjp<Q>(u4, lam, G);
        for (int m = 0; m < 4; ++m) yb1[m] = mb[m] + G[m];
    }
    if (tid < 2 * 2 * M * 4) (&sCb[0][0][0][0])[tid] = 0.0;
    // mesoscopic viscous terms of time n (CBC sides without -FD), as in the forward step
    const bool meso_v = CBC && (sd.scheme == BC_CBC || sd.scheme == BC_CBC_RELAX) && !sd.vfd;
    const bool fd_v = CBC && (sd.scheme == BC_CBC || sd.scheme == BC_CBC_RELAX) && sd.vfd;   // second differences enter
    const double nu = (a.tau - 0.5) * Lat<Q>::cs2;
    const double* visn = meso_v ? (const double*)(a.reg_cur + sd.off_vis) : nullptr;
    for (int l2 = tid; l2 < nlr; l2 += blockDim.x) {
        const int rr = r0 - H + l2;
        for (int m = 0; m < 4; ++m) sVr[l2 * 4 + m] = 0.0;
        if (meso_v && valid(rr))
            visc_terms_row<Q>(visn, len, phys(rr), valid(rr + 1) ? phys(rr + 1) : -1, valid(rr - 1) ? phys(rr - 1) : -1,
                              nu, &sVr[l2 * 4]);
    }
    __syncthreads();
    // NEEP (eq. NEEP): the layers of row r hold f^eq(U_b) + (1 - omega)(g - f^eq(m(g))) with g
    // pulled at x_f, so the adjoint of that g gets (1 - omega)(Lambda - phi . GM), Lambda = the sum
    // of lambda^{n+1} over the layers, GM = (dm/dM)^T (df^eq/dm)^T Lambda at the strip's moments;
    // k_adj_bulk adds it where it pulls from x_f (owned rows; the layers are read-only here)
    if (sd.meso == 1 && g.neep[side]) {
        const double cn = 1.0 - a.omega;
        double* nb = g.neep[side];
        for (int e = tid; e < r1 - r0; e += blockDim.x) {
            const int rr = r0 + e, l2 = H + e;
            double lam[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) lam[i] = 0.0;
            for (int q = 1; q <= M; ++q) {
                int x, y; side_node(sd, q, rr, x, y);
#pragma unroll
                for (int i = 0; i < Q; ++i) lam[i] += g.V1[pix<Q>(a.pitch, i, x, y)];
            }
            double G[4], GM[4];
            feq_vjp<Q>(&sXp[(l2 * MS) * 4], lam, G);
            mom_vjp<Q>(&sXp[(l2 * MS) * 4], G, GM);
            double* o = nb + (size_t)rr * (Q + 4);
#pragma unroll
            for (int i = 0; i < Q; ++i) o[i] = cn * lam[i];
            for (int m = 0; m < 4; ++m) o[Q + m] = cn * GM[m];
        }
    }

    const double ast[4] = {0.0, 0.5, 0.5, 1.0}, bst[4] = {1.0, 2.0, 2.0, 1.0};
    // side-local stage-st inputs of this thread's node
    // The stage inputs of this node, side-local.  Every LDS read is issued unconditionally (indices
    // clamped into the arrays, the alternatives chosen by value afterwards), so that a stage waits
    // for the LDS once instead of once per branch: dn = cU U + cA Y(kA) + cB Y(kB) with the
    // one-sided (j = M, eq. FD-dx-bw) or central (eq. FD-dx-center) coefficients, Y(k) of layer
    // k >= 1 from the stored stage input, of k <= 0 from the strip interpolated in time.
    const int nax = sd.nax;
    const double snv = sd.sn;
    auto loc = [&](const double* gv, double* l) {   // to_local
        l[0] = gv[0];
        l[1] = snv * (nax == 0 ? gv[1] : gv[2]);
        l[2] = nax == 0 ? gv[2] : gv[1];
        l[3] = gv[3];
    };
    const bool one = j == M;
    const int kA = one ? M - 1 : j + 1, kB = one ? M - 2 : j - 1, kC = M - 3;
    const double cU = one ? 1.5 : 0.0, cA = one ? -2.0 : 0.5, cB = one ? 0.5 : -0.5;
    const int lrc = min(max(lr, 1), NR - 2);   // clamped row (the reads of non-node threads stay in the arrays)
    auto inputs = [&](int st, double* U, double* dn, double* d2n, double* up, double* dw, double* U0) {
        const double th = ast[st];
        const double* Ys = sY[st];
        auto rd = [&](int k, double* gv) {   // Y(k), global components
            const double* y = &Ys[(lrc * M + max(k, 1) - 1) * 4];
            const double* bn = &sXn[(lrc * MS + min(max(-k, 0), MS - 1)) * 4];
            const double* bp = &sXp[(lrc * MS + min(max(-k, 0), MS - 1)) * 4];
            double yv[4], sv[4];
            for (int m = 0; m < 4; ++m) { yv[m] = y[m]; sv[m] = (1.0 - th) * bn[m] + th * bp[m]; }
            for (int m = 0; m < 4; ++m) gv[m] = k >= 1 ? yv[m] : sv[m];
        };
        double gU[4], gA[4], gB[4], gC[4] = {0.0, 0.0, 0.0, 0.0}, gu[4], gd[4], cu[4], cd[4], g0[4];
        rd(j, gU);
        rd(kA, gA);
        rd(kB, gB);
        if (M == 3 && fd_v) rd(kC, gC);
        const double* yu = &Ys[(min(lrc + 1, NR - 1) * M + jj) * 4];
        const double* yd = &Ys[(max(lrc - 1, 0) * M + jj) * 4];
        for (int m = 0; m < 4; ++m) {
            gu[m] = yu[m];
            gd[m] = yd[m];
            cu[m] = (1.0 - th) * sC[1][0][m] + th * sC[1][1][m];   // row len: the high corner
            cd[m] = (1.0 - th) * sC[0][0][m] + th * sC[0][1][m];   // row -1: the low corner
            g0[m] = sY[0][t * 4 + m];
        }
        const bool cor_u = !tper && r + 1 >= len, cor_d = !tper && r - 1 < 0;
        for (int m = 0; m < 4; ++m) {
            gu[m] = cor_u ? cu[m] : gu[m];
            gd[m] = cor_d ? cd[m] : gd[m];
        }
        double a[4], b[4], c[4];
        loc(gU, U);
        loc(gA, a);
        loc(gB, b);
        loc(gu, up);
        loc(gd, dw);
        loc(g0, U0);
        for (int m = 0; m < 4; ++m) dn[m] = cU * U[m] + cA * a[m] + cB * b[m];
        for (int m = 0; m < 4; ++m) d2n[m] = 0.0;
        if (fd_v) {   // second differences of the -FD viscous terms (Sec. 4.2): backward at j = M
            loc(gC, c);
            for (int m = 0; m < 4; ++m)
                d2n[m] = one ? (M == 3 ? 2.0 * U[m] - 5.0 * a[m] + 4.0 * b[m] - c[m] : 0.0) : a[m] - 2.0 * U[m] + b[m];
        }
    };

    // ---- phase C: reverse stages 3..0 (stage inputs loaded in phase A) ------------------------
    const bool owned = node && r >= r0 && r < r1;
    double ybn[4];   // adjoint of U_b^n (owned rows)
    for (int m = 0; m < 4; ++m) ybn[m] = owned ? yb1[m] : 0.0;
    double aK = 0.0, aA = 0.0;
    double vacc[4] = {0.0, 0.0, 0.0, 0.0};   // adjoint of this node's mesoscopic V, summed over the stages
    double gnext[4] = {0.0, 0.0, 0.0, 0.0};  // adjoint of this node's input of the later stage
    for (int st = 3; st >= 0; --st) {
        const double th = ast[st];
        double* bGn = sGn[st & 1];
        double* bGu = sGu[st & 1];
        double* bGd = sGd[st & 1];
        double* bG2 = sG2[st & 1];
        double gself[4] = {0, 0, 0, 0};
        if (node && within(r, st + 1)) {
            double kb[4], rb[4];
            for (int m = 0; m < 4; ++m)
                kb[m] = bst[st] * (1.0 / 6.0) * yb1[m] + (st < 3 ? ast[st + 1] * gnext[m] : 0.0);
            to_local(sd, kb, rb);
            double U[4], dn[4], d2n[4], up[4], dw[4], U0[4];
            inputs(st, U, dn, d2n, up, dw, U0);
            double Ubl[4], dnbl[4], d2nbl[4], upbl[4], dwbl[4], Vbl[4], Kb, alb;
            char_rate_vjp<Q, CBC>(U, dn, d2n, up, dw, &sVr[lr * 4], U0, sd.scheme, sd.vfd, nu, sd.K, sd.alpha, sd.Pinf, rb,
                             Ubl, dnbl, d2nbl, upbl, dwbl, Vbl, Kb, alb);
            if (meso_v)
                for (int m = 0; m < 4; ++m) vacc[m] += Vbl[m];
            double Ubg[4], dnbg[4], d2nbg[4], upbg[4], dwbg[4];
            rate_to_global(sd, Ubl, Ubg);
            rate_to_global(sd, dnbl, dnbg);
            rate_to_global(sd, d2nbl, d2nbg);
            rate_to_global(sd, upbl, upbg);
            rate_to_global(sd, dwbl, dwbg);
            for (int m = 0; m < 4; ++m) {
                gself[m] = Ubg[m] + (j == M ? 1.5 * dnbg[m] : 0.0);
                bGn[t * 4 + m] = dnbg[m];
                bGu[t * 4 + m] = upbg[m];
                bGd[t * 4 + m] = dwbg[m];
            }
            if constexpr (M == 3)
                if (fd_v)
                    for (int m = 0; m < 4; ++m) {
                        gself[m] += (j == M ? 2.0 : -2.0) * d2nbg[m];
                        bG2[t * 4 + m] = d2nbg[m];
                    }
            if (owned) {
                aK += Kb;
                aA += alb;
                if (jj == 0) {   // the strip enters the normal difference of layer 1
                    double xb[MS][4];
                    for (int m = 0; m < 4; ++m) {
                        if (M == 1) { xb[0][m] = -2.0 * dnbg[m]; xb[MS - 1][m] = 0.5 * dnbg[m]; }
                        else xb[0][m] = -0.5 * dnbg[m];
                    }
                    for (int k = 0; k < MS; ++k)
                        for (int m = 0; m < 4; ++m) {
                            sXbn[(lr * MS + k) * 4 + m] += (1.0 - th) * xb[k][m];
                            sXbp[(lr * MS + k) * 4 + m] += th * xb[k][m];
                        }
                }
                if (!tper && r == 0)
                    for (int m = 0; m < 4; ++m) { sCb[0][0][jj][m] += (1.0 - th) * dwbg[m]; sCb[0][1][jj][m] += th * dwbg[m]; }
                if (!tper && r == len - 1)
                    for (int m = 0; m < 4; ++m) { sCb[1][0][jj][m] += (1.0 - th) * upbg[m]; sCb[1][1][jj][m] += th * upbg[m]; }
            }
        }
        __syncthreads();
        // gather the adjoint of this stage's input on rows within st of the owned range
        if (node && within(r, st)) {
            // every read first (clamped indices), the terms chosen by value: one LDS wait
            double vq[M][4], vu[4], vd[4];
            for (int q = 1; q <= M; ++q)
                for (int m = 0; m < 4; ++m) vq[q - 1][m] = bGn[((lrc * M) + q - 1) * 4 + m];
            for (int m = 0; m < 4; ++m) {
                vu[m] = bGu[(max(lrc - 1, 0) * M + jj) * 4 + m];
                vd[m] = bGd[(min(lrc + 1, NR - 1) * M + jj) * 4 + m];
            }
            double yb[4];
            for (int m = 0; m < 4; ++m) yb[m] = gself[m];
            for (int q = 1; q <= M; ++q) {   // normal differences of the other layers of this row (cf = 0 at q = j)
                const double cf = q == M ? ((j == M - 1) ? -2.0 : (j == M - 2 ? 0.5 : 0.0))
                                         : ((j == q + 1) ? 0.5 : (j == q - 1 ? -0.5 : 0.0));
                for (int m = 0; m < 4; ++m) yb[m] += cf != 0.0 ? cf * vq[q - 1][m] : 0.0;
            }
            if constexpr (M == 3) if (fd_v) {   // second differences: backward (2, -5, 4, -1) at q = M, central below
                double v2[M][4];
                for (int q = 1; q <= M; ++q)
                    for (int m = 0; m < 4; ++m) v2[q - 1][m] = bG2[((lrc * M) + q - 1) * 4 + m];
                for (int q = 1; q <= M; ++q) {
                    if (q == j) continue;
                    const double c2 = q == M ? (j == M - 1 ? -5.0 : (j == M - 2 ? 4.0 : 0.0))
                                             : ((j == q + 1 || j == q - 1) ? 1.0 : 0.0);
                    for (int m = 0; m < 4; ++m) yb[m] += c2 != 0.0 ? c2 * v2[q - 1][m] : 0.0;
                }
            }
            if constexpr (M == 3) if (fd_v) {
                // the strip x_f is layer 0 of the second differences: +1 in layer 1's central one,
                // -1 in layer M's backward one (owned rows, as the first differences' strip terms)
                if (owned && jj == 0)
                    for (int m = 0; m < 4; ++m) {
                        const double xb = bG2[(lr * M) * 4 + m] - bG2[(lr * M + M - 1) * 4 + m];
                        sXbn[(lr * MS) * 4 + m] += (1.0 - th) * xb;
                        sXbp[(lr * MS) * 4 + m] += th * xb;
                    }
            }
            const bool vm1 = valid(r - 1), vp1 = valid(r + 1);
            for (int m = 0; m < 4; ++m) yb[m] += vm1 ? vu[m] : 0.0;
            for (int m = 0; m < 4; ++m) yb[m] += vp1 ? vd[m] : 0.0;
            for (int m = 0; m < 4; ++m) gnext[m] = yb[m];
            if (owned) for (int m = 0; m < 4; ++m) ybn[m] += yb[m];
        }
        // (no second barrier: the next stage writes the other buffers; a thread reaches its
        // writes to these only after the next stage's barrier, which every gather here precedes)
    }
    __syncthreads();   // the strip adjoints and buffers of the last stage, read below

    // ---- phase D: outputs ----------------------------------------------------------------------
    if (owned) {
        const int rp = phys(r);
        for (int m = 0; m < 4; ++m) mub0[((size_t)jj * len + rp) * 4 + m] = ybn[m];
    }
    if (meso_v) {
        // adjoint of the viscous moments of time n at x_f - M .. x_f - M - 2 of the owned rows, from
        // the adjoints of V of rows r - 1, r, r + 1 (complete on rows within one of the owned
        // range); k_adj_bulk adds it to nu^n through the moments' derivatives
        if (t < NN)
            for (int m = 0; m < 4; ++m) sGn[1][t * 4 + m] = node ? vacc[m] : 0.0;
        __syncthreads();
        constexpr double cs2 = Lat<Q>::cs2;
        double* visb = (double*)(g.adj_cur + sd.off_vis);
        for (int e = tid; e < r1 - r0; e += blockDim.x) {
            const int rr = r0 + e, l2 = H + e, rp = phys(rr);
            auto vsum = [&](int l, double* o) {
                for (int m = 0; m < 4; ++m) {
                    o[m] = 0.0;
                    for (int q = 0; q < M; ++q) o[m] += sGn[1][(l * M + q) * 4 + m];
                }
            };
            const bool hm = valid(rr - 1), hp = valid(rr + 1);
            double Vb0[4], Vbm[4] = {0.0, 0.0, 0.0, 0.0}, Vbp[4] = {0.0, 0.0, 0.0, 0.0};
            vsum(l2, Vb0);
            if (hm) vsum(l2 - 1, Vbm);
            if (hp) vsum(l2 + 1, Vbp);
            const double* w0 = &visn[((size_t)0 * len + rp) * 6];
            const double* w1 = &visn[((size_t)1 * len + rp) * 6];
            const double* w2 = &visn[((size_t)2 * len + rp) * 6];
            double upv[6] = {0, 0, 0, 0, 0, 0}, dwv[6] = {0, 0, 0, 0, 0, 0};
            if (hp) for (int m = 0; m < 6; ++m) upv[m] = visn[((size_t)0 * len + phys(rr + 1)) * 6 + m];
            if (hm) for (int m = 0; m < 6; ++m) dwv[m] = visn[((size_t)0 * len + phys(rr - 1)) * 6 + m];
            auto dn_ = [&](int m) { return 0.5 * (3.0 * w0[m] - 4.0 * w1[m] + w2[m]); };
            auto dt_ = [&](int m) { return 0.5 * (upv[m] - dwv[m]); };
            const double ir = 1.0 / w0[0];
            const double X1 = dn_(1) + dt_(2), X2 = dn_(2) + dt_(3), X3 = dn_(4) + dt_(5);
            const double heat = (0.5 * (w0[1] * w0[1] + w0[3] * w0[3]) + w0[2] * w0[2]) * ir * ir / (nu * cs2);
            // V_n = X1 / rho, V_t = X2 / rho, V_T = -X3 / (rho cs^2) + heat, heat ~ 1 / rho^2
            const double A1 = Vb0[1] * ir, A2 = Vb0[2] * ir, A3 = -Vb0[3] * ir / cs2;
            const double ck[3] = {1.5, -2.0, 0.5};
            double vb[3][6];
            for (int k = 0; k < 3; ++k) {
                for (int m = 0; m < 6; ++m) vb[k][m] = 0.0;
                vb[k][1] = ck[k] * A1;
                vb[k][2] = ck[k] * A2;
                vb[k][4] = ck[k] * A3;
            }
            vb[0][0] = -(Vb0[1] * X1 + Vb0[2] * X2) * ir * ir + Vb0[3] * (X3 * ir * ir / cs2 - 2.0 * heat * ir);
            const double hh = Vb0[3] * ir * ir / (nu * cs2);
            vb[0][1] += hh * w0[1];
            vb[0][2] += 2.0 * hh * w0[2];
            vb[0][3] += hh * w0[3];
            // rows r - 1 and r + 1 take this row's x_f moments in their differences along the side
            if (hm) {
                const double irm = 1.0 / dwv[0];
                vb[0][2] += 0.5 * Vbm[1] * irm;
                vb[0][3] += 0.5 * Vbm[2] * irm;
                vb[0][5] += -0.5 * Vbm[3] * irm / cs2;
            }
            if (hp) {
                const double irp = 1.0 / upv[0];
                vb[0][2] -= 0.5 * Vbp[1] * irp;
                vb[0][3] -= 0.5 * Vbp[2] * irp;
                vb[0][5] -= -0.5 * Vbp[3] * irp / cs2;
            }
            for (int k = 0; k < 3; ++k)
                for (int m = 0; m < 6; ++m) visb[((size_t)k * len + rp) * 6 + m] = vb[k][m];
        }
    }
    // strips: adjoint of X^n (a time-n input) for the next reverse step; the adjoint of X^{n+1}
    // (this step's new value plus the previous reverse step's time-(n+1) input) is added to
    // nu^{n+1}(x_f) as phi . (dm/dM)^T Xbar, except at the end rows next to corners (the corner
    // diagonal node c + v, shared with the other side and the corner), whose term goes to gm
    for (int e = tid; e < NR * MS; e += blockDim.x) {
        const int l2 = e / MS, k = e % MS, rr = r0 - H + l2;
        if (rr < r0 || rr >= r1 || !valid(rr)) continue;
        const int rp = phys(rr);
        const size_t o = ((size_t)k * len + rp) * 4;
        const bool end_row = !tper && k == 0 && (rp == 0 || rp == len - 1);   // len >= 3: the two ends differ
        int x, y; side_node(sd, -k, rp, x, y);
        double* v1 = g.V1 + pix<Q>(a.pitch, 0, x, y);
        // every load before the first store (one round trip)
        double Z[4], v[Q];
        for (int m = 0; m < 4; ++m) Z[m] = xbp[o + m];
        if (!end_row) {
#pragma unroll
            for (int i = 0; i < Q; ++i) v[i] = v1[(unsigned long long)i * a.pitch];
        }
        double GM[4];
        for (int m = 0; m < 4; ++m) {
            xbo[o + m] = sXbn[e * 4 + m];
            Z[m] += sXbp[e * 4 + m];
        }
        mom_vjp<Q>(&sXp[e * 4], Z, GM);
        if (end_row) {
            for (int m = 0; m < 4; ++m) g.gm[(side * 2 + (rp == 0 ? 0 : 1)) * 4 + m] = GM[m];
            continue;
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) v1[(unsigned long long)i * a.pitch] = v[i] + phi_dot<Q>(i, GM);
    }
    if (!tper && tid < 16) {
        const int e = tid / 8, w = (tid / 4) % 2, m = tid % 4;
        const bool mine = e == 0 ? (r0 == 0) : (r1 == len);
        if (mine) {
            double v = 0.0;
            for (int q = 0; q < M; ++q) v += sCb[e][w][q][m];
            const int ci = e == 0 ? sd.corner_lo : sd.corner_hi;
            g.ccon[((ci * 2 + sd.nax) * 2 + w) * 4 + m] = v;
        }
    }
    // parameter adjoints: fixed-order block reduction
    const double wk = wave_sum(aK), wa = wave_sum(aA);
    if ((tid & 63) == 0) { sRed[0][tid >> 6] = wk; sRed[1][tid >> 6] = wa; }
    __syncthreads();
    if (tid < 2) {
        const double v = sRed[tid][0] + sRed[tid][1] + sRed[tid][2] + sRed[tid][3];
        g.acc[blk * 2 + tid] = acc0 + v;
    }
}

// ------------------------------------------------------------------ reverse of a corner
// One work-group per corner: fold of the M x M block (J_feq^T of lambda^{n+1}), transposed
// Jacobians of the four stage rates with unit cotangents (16 threads; the stage inputs were
// stored by the recomputation), then the reverse RK4 sweep on one thread.  Writes the adjoints
// of U_c^n and D^n (time-n inputs) and the corner's terms of the corrections of nu^{n+1} at
// c + v and c + 2v.  The sides' contributions (ccon) are read only when the sides' transverse
// terms reach the corner values (coupled).
template <int Q>
__device__ void corner_adj(const AdjArgs& g, int ci) {
    constexpr int M = Lat<Q>::M;
    const BndArgs& a = g.b;
    const int tid = threadIdx.x;
    const CornerDev& c = a.c[ci];
    if (!c.active || c.zg) return;
    __shared__ double sF[M * M][4];
    // U_c^n, U_c^{n+1}, D^n, D^{n+1}, adjoint of U_c^{n+1}, adjoint of D^{n+1} as a time-(n+1)
    // input, side contributions [axis][n, n+1]
    __shared__ double sIn[52];
    __shared__ double sJT[4][4][13];   // [stage][m][Yc (4), D1 (4), D2 (4), K]
    enum { I_UN = 0, I_UP = 4, I_DN = 8, I_DP = 16, I_MU = 24, I_DB = 28, I_CC = 36 };
    if (tid < 52) {
        const int t = tid;
        double v;
        if (t < I_UP) v = ((const double*)(a.reg_cur + c.off_cu))[t - I_UN];
        else if (t < I_DN) v = ((const double*)(a.reg_next + c.off_cu))[t - I_UP];
        else if (t < I_DP) v = ((const double*)(a.reg_cur + c.off_cd))[t - I_DN];
        else if (t < I_MU) v = ((const double*)(a.reg_next + c.off_cd))[t - I_DP];
        else if (t < I_DB) v = ((const double*)(g.adj_next + c.off_cu))[t - I_MU];
        else if (t < I_CC) v = ((const double*)(g.adj_next + c.off_cd))[t - I_DB];
        else v = g.coupled ? g.ccon[ci * 16 + (t - I_CC)] : 0.0;
        sIn[t] = v;
    }
    if (tid >= 64 && tid < 64 + M * M) {
        const int q = tid - 64, jx = q / M, jy = q % M;
        const int x = c.x0 + c.sxn * jx, y = c.y0 + c.syn * jy;
        const double* cup = (const double*)(a.reg_next + c.off_cu);
        double lam[Q], u4[4], G[4];
#pragma unroll
        for (int i = 0; i < Q; ++i) lam[i] = g.V1[pix<Q>(a.pitch, i, x, y)];
        for (int m = 0; m < 4; ++m) u4[m] = cup[m];
        feq_vjp<Q>(u4, lam, G);
        for (int m = 0; m < 4; ++m) sF[q][m] = G[m];
    }
    __syncthreads();
    const double ast[4] = {0.0, 0.5, 0.5, 1.0}, bst[4] = {1.0, 2.0, 2.0, 1.0};
    {
        const int u = tid - 128;
        if (u >= 0 && u < 16) {
            const int st = u / 4, m = u % 4;
            const double th = ast[st];
            const double* Un = &sIn[I_UN];
            const double* ycs = (const double*)(a.reg_next + c.off_cs);
            double Y[4], B1[4], B2[4], e[4] = {0, 0, 0, 0}, Ycb[4], B1b[4], B2b[4], Kb;
            e[m] = 1.0;
            for (int k = 0; k < 4; ++k) {
                Y[k] = st == 0 ? Un[k] : ycs[(st - 1) * 4 + k];
                B1[k] = (1.0 - th) * sIn[I_DN + k] + th * sIn[I_DP + k];
                B2[k] = (1.0 - th) * sIn[I_DN + 4 + k] + th * sIn[I_DP + 4 + k];
            }
            corner_rate_vjp<Q>(c, Y, B1, B2, Un, e, Ycb, B1b, B2b, Kb);
            for (int k = 0; k < 4; ++k) {
                sJT[st][m][k] = Ycb[k];
                sJT[st][m][4 + k] = B1b[k];
                sJT[st][m][8 + k] = B2b[k];
            }
            sJT[st][m][12] = Kb;
        }
    }
    __syncthreads();
    if (tid != 0) return;
    const double* cc = &sIn[I_CC];   // [axis][n, n+1][4]
    double ub[4];
    for (int m = 0; m < 4; ++m) {
        ub[m] = sIn[I_MU + m];
        for (int q = 0; q < M * M; ++q) ub[m] += sF[q][m];
        for (int ax = 0; ax < 2; ++ax) ub[m] += cc[(ax * 2 + 1) * 4 + m];
    }
    double ybn[4], yb[4] = {0, 0, 0, 0}, Dbn[8] = {0, 0, 0, 0, 0, 0, 0, 0}, Dbp[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double Kacc = 0.0;
    for (int m = 0; m < 4; ++m) ybn[m] = ub[m];
    for (int st = 3; st >= 0; --st) {
        const double th = ast[st];
        double kb[4], v[13];
        for (int m = 0; m < 4; ++m) kb[m] = bst[st] * (1.0 / 6.0) * ub[m] + (st < 3 ? ast[st + 1] * yb[m] : 0.0);
        for (int k = 0; k < 13; ++k)
            v[k] = kb[0] * sJT[st][0][k] + kb[1] * sJT[st][1][k] + kb[2] * sJT[st][2][k] + kb[3] * sJT[st][3][k];
        Kacc += v[12];
        for (int m = 0; m < 4; ++m) {
            yb[m] = v[m];
            ybn[m] += v[m];
            Dbn[m] += (1.0 - th) * v[4 + m]; Dbn[4 + m] += (1.0 - th) * v[8 + m];
            Dbp[m] += th * v[4 + m]; Dbp[4 + m] += th * v[8 + m];
        }
    }
    double* mucn = (double*)(g.adj_cur + c.off_cu);
    double* dbn = (double*)(g.adj_cur + c.off_cd);
    for (int m = 0; m < 4; ++m) {
        mucn[m] = ybn[m] + cc[(0 * 2 + 0) * 4 + m] + cc[(1 * 2 + 0) * 4 + m];
        dbn[m] = Dbn[m];
        dbn[4 + m] = Dbn[4 + m];
    }
    g.acc[2 * g.nadj + ci] += Kacc;
    // the corner's terms of the corrections at c + v and c + 2v (time n+1)
    double Z1[4], Z2[4], GM[4];
    for (int m = 0; m < 4; ++m) {
        Z1[m] = Dbp[m] + sIn[I_DB + m];
        Z2[m] = Dbp[4 + m] + sIn[I_DB + 4 + m];
    }
    mom_vjp<Q>(&sIn[I_DP], Z1, GM);
    for (int m = 0; m < 4; ++m) g.gm[(8 + ci * 2 + 0) * 4 + m] = GM[m];
    mom_vjp<Q>(&sIn[I_DP + 4], Z2, GM);
    for (int m = 0; m < 4; ++m) g.gm[(8 + ci * 2 + 1) * 4 + m] = GM[m];
}

// ------------------------------------------------------------------ reverse of a zero-gradient side
// The layers of row r hold the post-collision populations C(g) of x_f (eq. zg-bc), the corner
// blocks those of the inward diagonal node c + v: the adjoint of that g gets C^T Lambda =
// (1 - omega) Lambda + omega phi . GM, Lambda = the sum of lambda^{n+1} over the copies, GM =
// (dm/dM)^T (df^eq/dm)^T Lambda at g's moments (time n + 1).  Written as (a, -GM') with a =
// (1 - omega) Lambda, GM' = omega GM for k_adj_bulk, which adds a_i - phi_i . GM' where it pulls
// from these nodes.  One thread per row; the corners on the first thread of the owning side.
template <int Q>
__device__ void zg_adj_chunk(const AdjArgs& g, const SideDev& sd, int side, int chunk) {
    constexpr int M = Lat<Q>::M;
    const BndArgs& a = g.b;
    const double om = a.omega;
    const unsigned long long plane = (unsigned long long)a.ny * a.pitch;
    auto emit = [&](int x, int y, const double* lam, double* o) {
        const unsigned long long id = (unsigned long long)y * a.pitch + x;
        const double m[4] = {g.mom1[id], g.mom1[plane + id], g.mom1[2 * plane + id],
                             Lat<Q>::thermal ? g.mom1[3 * plane + id] : 1.0};
        double G[4], GM[4];
        feq_vjp<Q>(m, lam, G);
        mom_vjp<Q>(m, G, GM);
#pragma unroll
        for (int i = 0; i < Q; ++i) o[i] = (1.0 - om) * lam[i];
        for (int k = 0; k < 4; ++k) o[Q + k] = -om * GM[k];
    };
    const int r = chunk * 256 + (int)threadIdx.x;
    if (r < sd.len) {
        double lam[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) lam[i] = 0.0;
        for (int j = 1; j <= M; ++j) {
            int x, y; side_node(sd, j, r, x, y);
#pragma unroll
            for (int i = 0; i < Q; ++i) lam[i] += g.V1[pix<Q>(a.pitch, i, x, y)];
        }
        int xf, yf; side_node(sd, 0, r, xf, yf);
        emit(xf, yf, lam, g.neep[side] + (size_t)r * (Q + 4));
    }
    if (!sd.tper && sd.owns_corners && threadIdx.x == 0) {
        for (int e = 0; e < 2; ++e) {
            const int ci = e == 0 ? sd.corner_lo : sd.corner_hi;
            const bool mine = e == 0 ? (chunk == 0) : ((chunk + 1) * 256 >= sd.len);
            if (ci < 0 || !mine || !a.c[ci].active || !a.c[ci].zg) continue;
            const CornerDev& c = a.c[ci];
            double lam[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) lam[i] = 0.0;
            for (int jx = 0; jx < M; ++jx)
                for (int jy = 0; jy < M; ++jy) {
#pragma unroll
                    for (int i = 0; i < Q; ++i) lam[i] += g.V1[pix<Q>(a.pitch, i, c.x0 + c.sxn * jx, c.y0 + c.syn * jy)];
                }
            emit(c.xc + c.vx, c.yc + c.vy, lam, g.zgc + (size_t)ci * (Q + 4));
        }
    }
}

// side chunks; when the corners do not read the sides' contributions, the corners too (the
// blocks after the side chunks).  CBC: compiled with the CBC variants' terms (some side is CBC
// or CBC-RELAX); without them the LODI schemes run a leaner kernel.
template <int Q, bool CBC>
__device__ __forceinline__ void adj_side_block(const AdjArgs& g, int b) {
    if (b >= g.nadj) {
        corner_adj<Q>(g, b - g.nadj);
        return;
    }
    int s = 0;
    while (s < 4 && !(g.anblk[s] > 0 && b >= g.ablk0[s] && b < g.ablk0[s] + g.anblk[s])) ++s;
    if (s == 4) return;
    if (g.b.s[s].kind == KIND_ZG) zg_adj_chunk<Q>(g, g.b.s[s], s, b - g.ablk0[s]);
    else adj_chunk<Q, CBC>(g, g.b.s[s], s, b, b - g.ablk0[s]);
}

template <int Q, bool CBC>
__global__ __launch_bounds__(256) void k_adj_side(AdjArgs g) {
    adj_side_block<Q, CBC>(g, (int)blockIdx.x);
}

// corners after the side chunks (coupled case)
template <int Q>
__global__ __launch_bounds__(256) void k_adj_corner(AdjArgs g) {
    corner_adj<Q>(g, blockIdx.x);
}

// Layer node (x, y) of a Dirichlet side with the default profile: its slot of the side's
// accumulator and its row's profile, or NULL.  Such a side has a periodic transverse axis, so its
// rows are all the nodes along it (r0 = 0).
template <int Q>
__device__ __forceinline__ double* dir_slot(const AdjArgs& g, int x, int y, const double*& prof) {
    constexpr int M = Lat<Q>::M;
#pragma unroll
    for (int sd = 0; sd < 4; ++sd) {
        double* acc = g.dacc[sd];
        if (!acc) continue;
        const SideDev& S = g.b.s[sd];
        const int j = ((S.nax == 0 ? x : y) - S.xf) * S.sn;
        if (j < 1 || j > M) continue;
        const int r = (S.nax == 0 ? y : x) - S.r0;
        prof = g.dprof[sd] + (size_t)r * 4;
        return acc + ((size_t)(j - 1) * S.len + r) * 4;
    }
    return nullptr;
}

// a += (d f^eq / d(rho, ux, uy, T))^T lam at the profile values u
template <int Q>
__device__ __forceinline__ void dir_fold(const double* u, const double* lam, double* a) {
    const double m[4] = {u[0], u[1], u[2], Lat<Q>::thermal ? u[3] : 1.0};
    double G[4];
    feq_vjp<Q>(m, lam, G);
    for (int c = 0; c < 4; ++c) a[c] += G[c];
}

// Per row of a Dirichlet side with the default profile: the profile is the initial state of the
// first layer node, so its collected adjoint is dL/d(rho0, ux0, uy0, T0) there (after the INIT
// pass, which leaves the gradient of every layer node of such a side at zero).
template <int Q>
__global__ __launch_bounds__(256) void k_adj_dir_collect(AdjArgs g, int s, int nx, int ny) {
    constexpr int M = Lat<Q>::M;
    const SideDev& S = g.b.s[s];
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= S.len) return;
    int x, y;
    side_node(S, 1, r, x, y);
    const size_t n = (size_t)nx * ny, id = (size_t)y * nx + x;
    for (int c = 0; c < 4; ++c) {
        double v = 0.0;
        for (int j = 0; j < M; ++j) v += g.dacc[s][((size_t)j * S.len + r) * 4 + c];
        g.grad[c * n + id] = v;
    }
}

// ------------------------------------------------------------------ bulk reverse
// One thread per node (all nodes; 256-node tiles of one row).  INIT: the reverse of the
// initialisation f^0 = f^eq(fields) at every node; the fields are read back as the moments of
// f^0 (mom of time 0), which the equilibrium reproduces exactly.
template <int Q, bool PX, bool PY, bool INIT>
__global__ __launch_bounds__(256) void k_adj_bulk(AdjArgs g, BulkArgs k, int bpr) {
    const int x = (blockIdx.x % bpr) * 256 + threadIdx.x, y = blockIdx.x / bpr;
    if (x >= k.nx) return;
    const unsigned long long pitch = k.pitch;
    // this node's moments of time n, loaded with the pull (every node has them)
    const unsigned long long plane = (unsigned long long)k.ny * pitch, o = (unsigned long long)y * pitch + x;
    const double m[4] = {g.mom[o], g.mom[plane + o], g.mom[2 * plane + o], Lat<Q>::thermal ? g.mom[3 * plane + o] : 1.0};
    double lam[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int xs = x + cx<Q>(i), ys = y + cy<Q>(i);
        if (PX) xs = wrapi(xs, k.nx);
        if (PY) ys = wrapi(ys, k.ny);
        const bool src = xs >= k.x0 && xs <= k.x1 && ys >= k.y0 && ys <= k.y1;
        const double v = g.V1[src ? pix<Q>(pitch, i, xs, ys) : 0ull];   // in bounds either way
        lam[i] = src ? v : 0.0;
    }
    if (g.neep_any) {
        // NEEP terms of nu^{n+1} at the x_f nodes of NEEP sides (written by the side chunks)
#pragma unroll
        for (int sd = 0; sd < 4; ++sd) {
            const double* nb = g.neep[sd];
            if (!nb) continue;
            const SideDev& S = g.b.s[sd];
            const bool xn = S.nax == 0;
            const int own = xn ? x : y;
            if (own < S.xf - 3 || own > S.xf + 3) continue;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                int xs = x + cx<Q>(i), ys = y + cy<Q>(i);
                if (PX) xs = wrapi(xs, k.nx);
                if (PY) ys = wrapi(ys, k.ny);
                const int nc = xn ? xs : ys, r = (xn ? ys : xs) - S.r0;
                if (nc != S.xf || r < 0 || r >= S.len) continue;
                const double* o = nb + (size_t)r * (Q + 4);
                lam[i] += o[i] - phi_dot<Q>(i, o + Q);
            }
        }
    }
    if (g.zgc_any) {
        // zero-gradient corner blocks: terms of nu^{n+1} at the inward diagonal node c + v
        for (int ci = 0; ci < 4; ++ci) {
            const CornerDev& c = g.b.c[ci];
            if (!c.active || !c.zg) continue;
            const int dx = c.xc + c.vx - x, dy = c.yc + c.vy - y;
            if (dx < -3 || dx > 3 || dy < -3 || dy > 3) continue;
            const double* o = g.zgc + (size_t)ci * (Q + 4);
#pragma unroll
            for (int i = 0; i < Q; ++i)
                if (cx<Q>(i) == dx && cy<Q>(i) == dy) lam[i] += o[i] - phi_dot<Q>(i, o + Q);
        }
    }
    // corrections of nu^{n+1} at the corner diagonal nodes c + v (the corner's term and both
    // adjacent strips' end rows) and c + 2v, for the nodes that pull from them
    constexpr int M = Lat<Q>::M;
    const bool corner_rows = y <= 3 * M + 1 || y >= k.ny - 2 - 3 * M;   // uniform per work-group
    if (corner_rows) {
        // the four corners' descriptors through uniform copies (scalar loads, see uniform_corner),
        // the corrections loaded only by the threads next to a diagonal node
        for (int ci = 0; ci < 4; ++ci) {
            const CornerDev c = uniform_corner(g.b.c[ci]);
            if (!c.active || c.zg) continue;
            int gi[2];
            for (int ax = 0; ax < 2; ++ax) gi[ax] = uni(g.cside[ci][ax] * 2 + (g.crow[ci][ax] == 0 ? 0 : 1));
            for (int e = 0; e < 2; ++e) {
                const int dx = c.xc + (e + 1) * c.vx - x, dy = c.yc + (e + 1) * c.vy - y;
                if (dx < -M || dx > M || dy < -M || dy > M) continue;
                double GM[4];
                for (int m = 0; m < 4; ++m) {
                    GM[m] = g.gm[(8 + ci * 2 + e) * 4 + m];
                    if (e == 0)
                        for (int ax = 0; ax < 2; ++ax) GM[m] += g.gm[gi[ax] * 4 + m];
                }
#pragma unroll
                for (int i = 0; i < Q; ++i)
                    if (cx<Q>(i) == dx && cy<Q>(i) == dy) lam[i] += phi_dot<Q>(i, GM);
            }
        }
    }
    if (INIT) {
        const int id = y * k.nx + x;
        if (g.dir_any) {
            // lambda^1 and lambda^0 of a default-profile layer node go to its row's profile
            const double* prof;
            double* a = dir_slot<Q>(g, x, y, prof);
            if (a) {
#pragma unroll
                for (int i = 0; i < Q; ++i) lam[i] += g.V1[pix<Q>(pitch, i, x, y)];
                dir_fold<Q>(prof, lam, a);
            }
        }
        double G[4];
        feq_vjp<Q>(m, lam, G);
        // the layers of a Dirichlet side hold the equilibrium of the profile, not of the initial
        // fields there
        for (int sd = 0; sd < 4; ++sd) {
            const SideDev& S = g.b.s[sd];
            if (S.kind != KIND_DIRICHLET) continue;
            const int j = ((S.nax == 0 ? x : y) - S.xf) * S.sn;
            if (j >= 1 && j <= M)
                for (int a = 0; a < 4; ++a) G[a] = 0.0;
        }
        const size_t n = (size_t)k.nx * k.ny;
        for (int a = 0; a < 4; ++a) g.grad[a * n + id] = G[a];
        return;
    }
    const bool bulk = x >= k.x0 && x <= k.x1 && y >= k.y0 && y <= k.y1;
    double* out = g.V0 + pix<Q>(pitch, 0, x, y);
    if (!bulk) {
#pragma unroll
        for (int i = 0; i < Q; ++i) out[(unsigned long long)i * pitch] = lam[i];
        if (g.dir_any) {
            // lambda^{n+1} of a default-profile layer node goes to its row's profile (lambda^n is
            // taken by the next reverse step, lambda^0 by the INIT pass)
            const double* prof;
            double* a = dir_slot<Q>(g, x, y, prof);
            if (a) {
#pragma unroll
                for (int i = 0; i < Q; ++i) lam[i] = g.V1[pix<Q>(pitch, i, x, y)];
                dir_fold<Q>(prof, lam, a);
            }
        }
        return;
    }
    double G[4], GM[4];
    feq_vjp<Q>(m, lam, G);
    mom_vjp<Q>(m, G, GM);
    const double om = k.omega_d;
#pragma unroll
    for (int i = 0; i < Q; ++i) out[(unsigned long long)i * pitch] = (1.0 - om) * lam[i] + om * phi_dot<Q>(i, GM);
    if (Lat<Q>::thermal && g.vism) {
        // nodes x_f - M, x_f - M - 1, x_f - M - 2 of a CBC side with the mesoscopic viscous terms: the moments
        // Pi' and q of eq. LaplaceU / LaplaceT taken from g^n there (time-n inputs of the next
        // step's V); with d = c_i - u, f = 1 - 1/(2 tau):
        //   d Pi'_ab / d g_i = -f (d_a d_b - |d|^2 delta_ab / 2),
        //   d q_a / d g_i = f (|d|^2 / 2 - 2 cs^2 T) d_a + Pi'_ab d_b / rho,  d rho / d g_i = 1
#pragma unroll
        for (int sd = 0; sd < 4; ++sd) {
            const SideDev& S = g.b.s[sd];
            if (S.kind != KIND_CHAR || !(S.scheme == BC_CBC || S.scheme == BC_CBC_RELAX) || S.vfd) continue;
            const bool xn = S.nax == 0;
            const int nc = xn ? x : y, tc = xn ? y : x;
            const int kk = (S.xf - nc) * S.sn - M, rr = tc - S.r0;   // nodes x_f - M - kk
            if (kk < 0 || kk > 2 || rr < 0 || rr >= S.len) continue;
            const size_t o6 = ((size_t)kk * S.len + rr) * 6;
            const double* vb = (const double*)(g.adj_cur + S.off_vis) + o6;
            const double* w = (const double*)(g.b.reg_cur + S.off_vis) + o6;
            // side-local (n, t) components to global (x, y)
            const double sn = S.sn;
            const double Pbxx = xn ? vb[1] : vb[3], Pbyy = xn ? vb[3] : vb[1], Pbxy = sn * vb[2];
            const double Qbx = xn ? sn * vb[4] : vb[5], Qby = xn ? vb[5] : sn * vb[4];
            const double Pxx = xn ? w[1] : w[3], Pyy = xn ? w[3] : w[1], Pxy = sn * w[2];
            const double Rb = vb[0];
            const double fac = 1.0 - 0.5 / g.b.tau, ir = 1.0 / m[0], ct = 2.0 * Lat<Q>::cs2 * m[3];
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const double d0 = cx<Q>(i) - m[1], d1 = cy<Q>(i) - m[2], h = 0.5 * (d0 * d0 + d1 * d1);
                double v = Rb - fac * (Pbxx * (d0 * d0 - h) + Pbyy * (d1 * d1 - h) + Pbxy * d0 * d1);
                v += Qbx * (fac * (h - ct) * d0 + (Pxx * d0 + Pxy * d1) * ir);
                v += Qby * (fac * (h - ct) * d1 + (Pxy * d0 + Pyy * d1) * ir);
                out[(unsigned long long)i * pitch] += v;
            }
        }
    }
}

// ------------------------------------------------------------------ seed at the final step
// V^N = J_m^T dL/dm at every node (nu at bulk nodes, lambda at layer and block nodes).  seed:
// dL/d(rho, ux, uy, T) [4][ny][nx], or NULL for the pressure loss sum over the bulk nodes of
// (P - cs^2)^2, P = cs^2 rho T.
template <int Q, typename T>
__global__ __launch_bounds__(256) void k_adj_seed(const T* __restrict__ F, const double* __restrict__ seed, double* V,
                                                  BulkArgs k, int bpr) {
    const int x = (blockIdx.x % bpr) * 256 + threadIdx.x, y = blockIdx.x / bpr;
    if (x >= k.nx) return;
    double d[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) d[i] = (double)F[pix<Q>(k.pitch, i, x, y)];
    double rm1, u, v, th;
    moments_dev<Q, double>(d, rm1, u, v, th);
    const double m[4] = {1.0 + rm1, u, v, 1.0 + th};
    double s[4] = {0, 0, 0, 0};
    if (seed) {
        const size_t n = (size_t)k.nx * k.ny, id = (size_t)y * k.nx + x;
        for (int a = 0; a < 4; ++a) s[a] = seed[a * n + id];
    } else if (x >= k.x0 && x <= k.x1 && y >= k.y0 && y <= k.y1) {
        const double cs2 = Lat<Q>::cs2;
        const double p = cs2 * (rm1 + th + rm1 * th);   // P - cs^2
        s[0] = 2.0 * p * cs2 * m[3];
        s[3] = Lat<Q>::thermal ? 2.0 * p * cs2 * m[0] : 0.0;
    }
    double GM[4];
    mom_vjp<Q>(m, s, GM);
#pragma unroll
    for (int i = 0; i < Q; ++i) V[pix<Q>(k.pitch, i, x, y)] = phi_dot<Q>(i, GM);
}

// moments of a population buffer into (rho, ux, uy, T) planes (start of a recomputed segment)
template <int Q, typename T>
__global__ __launch_bounds__(256) void k_adj_moments(const T* __restrict__ F, double* __restrict__ mom, BulkArgs k, int bpr) {
    const int x = (blockIdx.x % bpr) * 256 + threadIdx.x, y = blockIdx.x / bpr;
    if (x >= k.nx) return;
    double d[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) d[i] = (double)F[pix<Q>(k.pitch, i, x, y)];
    double rm1, u, v, th;
    moments_dev<Q, double>(d, rm1, u, v, th);
    const unsigned long long plane = (unsigned long long)k.ny * k.pitch, o = (unsigned long long)y * k.pitch + x;
    mom[o] = 1.0 + rm1; mom[plane + o] = u; mom[2 * plane + o] = v; mom[3 * plane + o] = 1.0 + th;
}

// ------------------------------------------------------------------ boundary terms of the initial fields
// U_b^0, the strip X^0, U_c^0 and D^0 are the initial fields at their nodes.  One work-group,
// one source at a time (sides in order, then corners), so nodes shared by two sources are
// updated in a fixed order.
template <int Q>
__global__ __launch_bounds__(256) void k_adj_final(AdjArgs g) {
    constexpr int M = Lat<Q>::M, MS = (M == 1) ? 2 : 1;
    const BndArgs& a = g.b;
    const size_t n = (size_t)a.nx * a.ny;
    const char* adj = g.adj_cur;   // adjoint region of time 0
    for (int s = 0; s < 4; ++s) {
        const SideDev& sd = a.s[s];
        if (sd.kind == KIND_CHAR) {
            const double* mub = (const double*)(adj + sd.off_ub);
            const double* xb = (const double*)(adj + sd.off_strip);
            for (int e = threadIdx.x; e < sd.len * (M + MS); e += blockDim.x) {
                const int k = e / sd.len, r = e % sd.len;   // k < M: layer k+1; else strip k-M
                int x, y;
                const double* src;
                if (k < M) { side_node(sd, k + 1, r, x, y); src = &mub[((size_t)k * sd.len + r) * 4]; }
                else { side_node(sd, -(k - M), r, x, y); src = &xb[((size_t)(k - M) * sd.len + r) * 4]; }
                const size_t id = (size_t)y * a.nx + x;
                for (int c = 0; c < 4; ++c) g.grad[c * n + id] += src[c];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) {
        for (int ci = 0; ci < 4; ++ci) {
            const CornerDev& c = a.c[ci];
            if (!c.active || c.zg) continue;
            const double* mu = (const double*)(adj + c.off_cu);
            const double* db = (const double*)(adj + c.off_cd);
            const int m = threadIdx.x;
            g.grad[m * n + (size_t)c.yc * a.nx + c.xc] += mu[m];
            g.grad[m * n + (size_t)(c.yc + c.vy) * a.nx + c.xc + c.vx] += db[m];
            g.grad[m * n + (size_t)(c.yc + 2 * c.vy) * a.nx + c.xc + 2 * c.vx] += db[4 + m];
        }
    }
}

}  // namespace lbm
