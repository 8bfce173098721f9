// lb_collide.h -- the collision of one fluid cell and its store.
//
// Eq. (cgoperator): Omega = Omega3 [Omega1 + Omega2].  Every population is
// regularised (Eq. (reg)) before the BGK relaxation (Eq. (modbgk)) with the
// mixture tau of Eq. (tauinter); the force (substrate drag and body force)
// enters Omega1 by the exact-difference method; the perturbation Omega2
// (Eq. (pertopform)) is applied once to the colour-blind total; Omega3
// recolours with the rest-frame equilibria.  Because the regularised
// populations depend on the moments only, the colour-blind post-collision
// total is
//   f*_i = sum_k rho_k phi_i^k + rho w_i E_i(u + F/rho)
//          + (1 - 1/tau) w_i / (2 c_s^4) Q_i : Pi^neq + Omega2_i,
// E_i(v) = c_i.v / c_s^2 + (c_i.v)^2 / (2 c_s^4) - v^2 / (2 c_s^2), and
//   f^Y_i = (rho_Y / rho) f*_i
//           + beta rho_Y rho_B / rho^2 cos(phi_i) sum_k rho_k phi_i^k.
#pragma once

#include "lb_device.h"

namespace lbk {

// Colour gradients, Eq. (lattgrad), already divided by c_s^2:
// g[0..2] = grad rho^N, g[3..5] = grad(rho_Y/rho), g[6..8] = grad(rho_B/rho).
template <typename R>
struct Grad {
    R g[9];
};

template <typename R, int I>
__device__ __forceinline__ void store_one(const DevParams &P, R rY, R rB, R drho, R rho, R vx, R vy, R vz, R vv,
                                          R om, const R (&Pi)[6], R trPi, R pA, R invFF, bool pert, R Fx, R Fy, R Fz,
                                          R gx, R gy, R gz, double fracY, R rec, R *__restrict__ dT, R *__restrict__ dY,
                                          long long cell, long long N)
{
    constexpr int X = lbq::cx(I), Yc = lbq::cy(I), Z = lbq::cz(I);
    constexpr int SH = lbq::shell(I);
    const R wi = R(lbq::w(I));
    // c.v, c.Pi.c
    R cv = R(0);
    if (X) cv += X > 0 ? vx : -vx;
    if (Yc) cv += Yc > 0 ? vy : -vy;
    if (Z) cv += Z > 0 ? vz : -vz;
    R cPc = R(0);
    if (X) cPc += Pi[0];
    if (Yc) cPc += Pi[1];
    if (Z) cPc += Pi[2];
    if (X && Yc) cPc += (X * Yc > 0 ? R(2) : R(-2)) * Pi[3];
    if (X && Z) cPc += (X * Z > 0 ? R(2) : R(-2)) * Pi[4];
    if (Yc && Z) cPc += (Yc * Z > 0 ? R(2) : R(-2)) * Pi[5];
    const R E = wi * (R(3) * cv + R(4.5) * cv * cv - R(1.5) * vv);
    const R neq = om * wi * R(4.5) * (cPc - R(1.0 / 3.0) * trPi);
    R om2 = R(0);
    if (I > 0) {
        R Fc = R(0);
        if (X) Fc += X > 0 ? Fx : -Fx;
        if (Yc) Fc += Yc > 0 ? Fy : -Fy;
        if (Z) Fc += Z > 0 ? Fz : -Fz;
        om2 = pert ? pA * (wi * Fc * Fc * invFF - R(lbq::B_of_shell(SH))) : R(0);
    } else {
        om2 = pert ? -pA * R(lbq::B_of_shell(0)) : R(0);
    }
    const R phiY = R(P.phi[0][SH]), phiB = R(P.phi[1][SH]);
    const R Tst = rY * R(P.phid[0][SH]) + rB * R(P.phid[1][SH]) + drho * wi + rho * E + neq + om2;
    // the ink's share of f*, formed in FP64 so that sum_i f^Y_i = rho_Y holds
    // to the final rounding of each stored value
    const double fst = lbq::w(I) * P.rho_ref + (double)Tst;
    double Yst = fracY * fst;
    if (I > 0) {
        R cg = R(0);
        if (X) cg += X > 0 ? gx : -gx;
        if (Yc) cg += Yc > 0 ? gy : -gy;
        if (Z) cg += Z > 0 ? gz : -gz;
        Yst += (double)(rec * R(lbq::inv_len(I)) * cg * (rY * phiY + rB * phiB));
    }
    dT[I * N + cell] = Tst;
    dY[I * N + cell] = R(Yst);
}

template <typename R, int I = 0>
__device__ __forceinline__ void store_all(const DevParams &P, R rY, R rB, R drho, R rho, R vx, R vy, R vz, R vv,
                                          R om, const R (&Pi)[6], R trPi, R pA, R invFF, bool pert, R Fx, R Fy, R Fz,
                                          R gx, R gy, R gz, double fracY, R rec, R *__restrict__ dT, R *__restrict__ dY,
                                          long long cell, long long N)
{
    if constexpr (I < lbq::Q) {
        store_one<R, I>(P, rY, rB, drho, rho, vx, vy, vz, vv, om, Pi, trPi, pA, invFF, pert, Fx, Fy, Fz, gx, gy, gz,
                        fracY, rec, dT, dY, cell, N);
        store_all<R, I + 1>(P, rY, rB, drho, rho, vx, vy, vz, vv, om, Pi, trPi, pA, invFF, pert, Fx, Fy, Fz, gx, gy,
                            gz, fracY, rec, dT, dY, cell, N);
    }
}

// Collide one fluid cell from its moment set and colour gradients; store the
// 38 post-collision values at the cell (the next step pulls them) and return
// rho_Y, rho_B and the bare velocity for the boundary rules of the next pull.
template <typename R>
__device__ __forceinline__ void collide_store(const DevParams &P, const Mom<R> &M, const Grad<R> &G, int z,
                                              R *__restrict__ dT, R *__restrict__ dY, long long cell, long long N,
                                              R &out_rY, R &out_rB, R (&out_u)[3])
{
    const R cs2 = R(1.0 / 3.0);
    const double rho_d = P.rho_ref + M.dm[0];
    const double fracY_d = M.dm[1] / rho_d;
    const R drho = R(M.dm[0]), rY = R(M.dm[1]);
    const R rho = R(rho_d);
    const R rB = R(rho_d - M.dm[1]);
    const R irho = R(1) / rho;
    const R ux = M.m[2] * irho, uy = M.m[3] * irho, uz = M.m[4] * irho;

    // force: body force and the substrate drag (exact-difference method)
    R Fx = rho * R(P.g[0]), Fy = rho * R(P.g[1]), Fz = rho * R(P.g[2]);
    if (P.drag_gamma != 0.0 && P.face_lo == FACE_WALL && (double)z + 0.5 < P.drag_range) {
        const R gam = R(P.drag_gamma) * rY;
        Fx -= gam * (ux - R(P.u_lo[0]));
        Fy -= gam * (uy - R(P.u_lo[1]));
        Fz -= gam * (uz - R(P.u_lo[2]));
    }
    const R vx = ux + Fx * irho, vy = uy + Fy * irho, vz = uz + Fz * irho;
    const R vv = vx * vx + vy * vy + vz * vz;

    // non-equilibrium stresses: total (collision) and ink (strain rate)
    const R iso = rY * R(P.dcs2[0]) + rB * R(P.dcs2[1]) + drho * cs2;
    R Pi[6];
    Pi[0] = M.m[5] - iso - rho * ux * ux;
    Pi[1] = M.m[6] - iso - rho * uy * uy;
    Pi[2] = M.m[7] - iso - rho * uz * uz;
    Pi[3] = M.m[8] - rho * ux * uy;
    Pi[4] = M.m[9] - rho * ux * uz;
    Pi[5] = M.m[10] - rho * uy * uz;
    const R trPi = Pi[0] + Pi[1] + Pi[2];
    const R cY2 = cs2 + R(P.dcs2[0]);
    const R Yxx = M.m[11] - rY * (cY2 + ux * ux);
    const R Yyy = M.m[12] - rY * (cY2 + uy * uy);
    const R Yzz = M.m[13] - rY * (cY2 + uz * uz);
    const R Yxy = M.m[14] - rY * ux * uy;
    const R Yxz = M.m[15] - rY * ux * uz;
    const R Yyz = M.m[16] - rY * uy * uz;
    const R S = sqrt(Yxx * Yxx + Yyy * Yyy + Yzz * Yzz + R(2) * (Yxy * Yxy + Yxz * Yxz + Yyz * Yyz));

    // local relaxation time: ink from its strain rate, air Newtonian, mixed
    // harmonically in the viscosity (Eq. (tauinter))
    const R tauY = tau_ink<R>(P, S, rY);
    const R nuY = cs2 * (tauY - R(0.5)), nuB = cs2 * (R(P.tau_b) - R(0.5));
    const R inv_nu = (rY * irho) / nuY + (rB * irho) / nuB;
    const R tau = R(0.5) + R(3) / inv_nu;
    const R om = R(1) - R(1) / tau;

    // colour-gradient force F_cg = (rho_B/rho) grad(rho_Y/rho) - (rho_Y/rho) grad(rho_B/rho)
    const R fracY = R(fracY_d), fracB = rB * irho;
    R Fcx = fracB * G.g[3] - fracY * G.g[6];
    R Fcy = fracB * G.g[4] - fracY * G.g[7];
    R Fcz = fracB * G.g[5] - fracY * G.g[8];
    // only the direction of F_cg enters Omega2: scale by its largest
    // component so |F|^2 neither underflows nor overflows; below 1e-30 the
    // operator (proportional to |grad rho^N| ~ |F_cg|) is negligible
    const R Fmax = fmax(fabs(Fcx), fmax(fabs(Fcy), fabs(Fcz)));
    const bool pert = Fmax > R(1e-30);
    const R iF = pert ? R(1) / Fmax : R(0);
    Fcx *= iF;
    Fcy *= iF;
    Fcz *= iF;
    const R invFF = pert ? R(1) / (Fcx * Fcx + Fcy * Fcy + Fcz * Fcz) : R(0);
    const R gn2 = G.g[0] * G.g[0] + G.g[1] * G.g[1] + G.g[2] * G.g[2];
    const R gn = sqrt(gn2);
    const R pA = R(0.5) * R(P.A) * gn;
    const R geps2 = gn2 + R(P.eps2);
    const R inv_geps = geps2 > R(0) ? R(1) / sqrt(geps2) : R(0);
    const R rec = R(P.beta) * fracY * fracB * inv_geps;

    store_all<R>(P, rY, rB, drho, rho, vx, vy, vz, vv, om, Pi, trPi, pA, invFF, pert, Fcx, Fcy, Fcz, G.g[0], G.g[1],
                 G.g[2], fracY_d, rec, dT, dY, cell, N);
    out_rY = rY;
    out_rB = rB;
    out_u[0] = ux;
    out_u[1] = uy;
    out_u[2] = uz;
}

}  // namespace lbk
