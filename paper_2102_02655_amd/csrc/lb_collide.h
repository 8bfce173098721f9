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

#include <utility>

#include "lb_device.h"

namespace lbk {

// Colour gradients, Eq. (lattgrad), already divided by c_s^2:
// g[0..2] = grad rho^N, g[3..5] = grad(rho_Y/rho), g[6..8] = grad(rho_B/rho).
template <typename R>
struct Grad {
    R g[9];
};

// Per-cell coefficients of the post-collision total.  On D3Q19 every term of
// f*_i is a quadratic form in c_i times w_i, plus a rest-link correction:
//   f*_i - w_i rho_ref = w_i [ k1 + a.c_i + c_i.Bm.c_i ]                (i > 0)
//   f*_0 - w_0 rho_ref = t0                                             (i = 0)
// with, for u' = u + F/rho (exact-difference method), omega = 1 - 1/tau,
// the unit colour-gradient direction n and p = (A/2) |grad rho^N|:
//   a  = 3 rho u'
//   Bm = 4.5 rho u'u' + 4.5 omega Pi^neq + p (n n - I)
//   a0 = -1.5 rho u'^2 - 1.5 omega tr Pi^neq + (2/3) p
//   k1 = a0 + drho + sum_k rho_k (phi_i^k - w_i) / w_i
//   t0 = w_0 (a0 + drho) + sum_k rho_k (phi_0^k - w_0)
// which is the regularised BGK of Eq. (reg)/(modbgk) with the equilibrium's
// rest-frame weights, plus Omega2 of Eq. (pertopform) with
// B_i = w_i (|c_i|^2 - 2/3).  The ink share is
//   f^Y_i = (rho_Y/rho) f*_i + w_i (beta rho_Y rho_B / rho^2) e (c_i.n_eps)/|c_i|
// with sum_k rho_k phi_i^k = w_i e on the moving links.
template <typename R>
struct OutCoef {
    R k1, t0, ax, ay, az, bxx, byy, bzz, bxy, bxz, byz;
    R rx, ry, rz;  // w-free recolouring vector: rec * e * grad rho^N
    double fracY;
};

// The quadratic form of OutCoef grouped by lattice axis and plane, formed
// once per cell: every moving link's bracket is then one addition,
//   axis link  +-e_a        : s_a +- a_a,              s_a = k1 + B_aa
//   plane link (sa, sb) in ab: (s_ab + sa sb B_ab) + sa (a_a + sa sb a_b),
// s_ab = k1 + B_aa + B_bb, and the recolouring sum c_i.r likewise.
template <typename R>
struct LinkSums {
    R t0;
    R s[3], a[3], r[3];
    R p[3], m[3];    // s_ab + B_ab, s_ab - B_ab  (ab = xy, xz, yz)
    R ap[3], am[3];  // a_a + a_b, a_a - a_b
    R rp[3], rm[3];  // r_a + r_b, r_a - r_b
    double fracY;
};

template <typename R>
__device__ __forceinline__ LinkSums<R> link_sums(const OutCoef<R> &K)
{
    LinkSums<R> L;
    L.t0 = K.t0;
    const R b[3] = {K.bxx, K.byy, K.bzz}, a[3] = {K.ax, K.ay, K.az}, r[3] = {K.rx, K.ry, K.rz};
    const R bo[3] = {K.bxy, K.bxz, K.byz};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        L.s[d] = K.k1 + b[d];
        L.a[d] = a[d];
        L.r[d] = r[d];
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const int da = q < 2 ? 0 : 1, db = q == 0 ? 1 : 2;
        const R sab = L.s[da] + b[db];
        L.p[q] = sab + bo[q];
        L.m[q] = sab - bo[q];
        L.ap[q] = a[da] + a[db];
        L.am[q] = a[da] - a[db];
        L.rp[q] = r[da] + r[db];
        L.rm[q] = r[da] - r[db];
    }
    L.fracY = K.fracY;
    return L;
}

// Post-collision T value of link I and its recolouring term w_i c_i.r/|c_i|.
template <typename R, int I>
__device__ __forceinline__ void link_value(const LinkSums<R> &L, R &Tst, R &cgw)
{
    constexpr int X = lbq::cx(I), Yc = lbq::cy(I), Z = lbq::cz(I);
    constexpr int nz = (X != 0) + (Yc != 0) + (Z != 0);
    if constexpr (I == 0) {
        Tst = L.t0;
        cgw = R(0);
    } else {
        const R wi = R(lbq::w(I));
        R q, cg;
        if constexpr (nz == 1) {
            constexpr int d = X ? 0 : (Yc ? 1 : 2);
            constexpr int sg = X + Yc + Z;
            q = L.s[d] + (sg > 0 ? L.a[d] : -L.a[d]);
            cg = sg > 0 ? L.r[d] : -L.r[d];
        } else {
            // plane ab with components (sa, sb)
            constexpr int q_ = Z == 0 ? 0 : (Yc == 0 ? 1 : 2);
            constexpr int sa = q_ == 2 ? Yc : X, sb = Z == 0 ? Yc : Z;
            const R base = sa * sb > 0 ? L.p[q_] : L.m[q_];
            const R av = sa * sb > 0 ? L.ap[q_] : L.am[q_];
            const R rv = sa * sb > 0 ? L.rp[q_] : L.rm[q_];
            q = base + (sa > 0 ? av : -av);
            cg = sa > 0 ? rv : -rv;
        }
        Tst = wi * q;
        cgw = (wi * R(lbq::inv_len(I))) * cg;
    }
}

// Store of link I into the population planes pT (set T) and pY (set Y) at
// byte offset cellb.  The next step reads these once, a full sweep later, so
// the stores are non-temporal.
template <typename R, int I>
__device__ __forceinline__ void store_one(const DevParams &P, const LinkSums<R> &L, gchar *pT, gchar *pY,
                                          unsigned cellb)
{
    typedef __attribute__((address_space(1))) R gR;
    R Tst, cgw;
    link_value<R, I>(L, Tst, cgw);
    // the ink's share fracY (w_i rho_ref + T_i) + recolouring, formed in FP64
    // so that sum_i f^Y_i = rho_Y holds to the final rounding of each stored
    // value (an FP32 fracY, or any FP32 rounding of fracY T_i, would bias
    // every cell of a uniform region alike)
    const R Yst = R(__builtin_fma(L.fracY, lbq::w(I) * P.rho_ref + (double)Tst, (double)cgw));
    __builtin_nontemporal_store(Tst, reinterpret_cast<gR *>(pT + cellb));
    __builtin_nontemporal_store(Yst, reinterpret_cast<gR *>(pY + cellb));
}

// The 38 stores; base: population plane 0 of the destination set, pstride:
// bytes per population plane.
template <typename R>
__device__ __forceinline__ void store_all(const DevParams &P, const OutCoef<R> &K, gchar *base,
                                          unsigned long long pstride, unsigned cellb)
{
    const LinkSums<R> L = link_sums(K);
    gchar *pT = base;
    gchar *pY = base + (unsigned long long)lbq::Q * pstride;
    [&]<int... I>(std::integer_sequence<int, I...>) {
        ((store_one<R, I>(P, L, pT + (unsigned long long)I * pstride, pY + (unsigned long long)I * pstride, cellb)),
         ...);
    }(std::make_integer_sequence<int, lbq::Q>{});
}

// Reduced storage: link I's deviation from the equilibrium of this cell's
// post-collision moments (rho_Y, rho_B, u'), 16-bit (the deviation is the
// non-equilibrium, perturbation and recolouring part of the compact form).
template <int ST, int I>
__device__ __forceinline__ void store_one_dev(const DevParams &P, const LinkSums<float> &L, const EqCell &ec,
                                              gchar *pw, unsigned cellb)
{
    typedef __attribute__((address_space(1))) unsigned gU;
    float Tst, cgw;
    link_value<float, I>(L, Tst, cgw);
    const float Yst = float(__builtin_fma(L.fracY, lbq::w(I) * P.rho_ref + (double)Tst, (double)cgw));
    float fT, fY;
    feq_TY_cell<I>(P, ec, fT, fY);
    constexpr float s = eq_scale<I>();  // exact: the deviations are f* - s fT, f* - s fY
    const unsigned wd = encode_pair<ST, I>(__builtin_fmaf(-s, fT, Tst), __builtin_fmaf(-s, fY, Yst));
    __builtin_nontemporal_store(wd, reinterpret_cast<gU *>(pw + cellb));
}

template <int ST>
__device__ __forceinline__ void store_all_dev(const DevParams &P, const OutCoef<float> &K, float rY, float rB,
                                              float vx, float vy, float vz, gchar *base, unsigned long long pstride,
                                              unsigned cellb)
{
    const EqCell ec = eq_cell(P, rY, rB, vx, vy, vz);
    const LinkSums<float> L = link_sums(K);
    // an opaque 32-bit offset: every store then takes the scalar-base form
    // (no 64-bit address arithmetic per store)
    asm volatile("" : "+v"(cellb));
    [&]<int... I>(std::integer_sequence<int, I...>) {
        ((store_one_dev<ST, I>(P, L, ec, base + (unsigned long long)I * pstride, cellb)), ...);
    }(std::make_integer_sequence<int, lbq::Q>{});
}

// What the collision needs of a cell, derived from its moment set: the two
// masses (FP64), momentum, the total non-equilibrium stress and the BGK
// factor 1 - 1/tau of the local mixture relaxation time.
template <typename R>
struct CellState {
    double drho, rY;
    R j[3];
    R Pi[6];
    R om;
};

template <typename R>
__device__ __forceinline__ CellState<R> cell_state(const DevParams &P, const Mom<R> &M)
{
    CellState<R> C;
    const R cs2 = R(1.0 / 3.0);
    C.drho = M.dm[0];
    C.rY = M.dm[1];
    const double rho_d = P.rho_ref + M.dm[0];
    const R drho = R(M.dm[0]), rY = R(M.dm[1]);
    const R rho = R(rho_d);
    const R rB = R(rho_d - M.dm[1]);
    const R irho = rcp_of(rho);
    const R ux = M.m[2] * irho, uy = M.m[3] * irho, uz = M.m[4] * irho;
    C.j[0] = M.m[2];
    C.j[1] = M.m[3];
    C.j[2] = M.m[4];
    // non-equilibrium stresses: total (collision) and ink (strain rate)
    // isotropic part of the equilibrium stress, formed from the FP64 masses:
    // at unequal alpha its terms are O(rho) and cancel to O(drho)
    const R iso = R(M.dm[1] * P.dcs2[0] + (rho_d - M.dm[1]) * P.dcs2[1] + M.dm[0] * (1.0 / 3.0));
    C.Pi[0] = M.m[5] - iso - rho * ux * ux;
    C.Pi[1] = M.m[6] - iso - rho * uy * uy;
    C.Pi[2] = M.m[7] - iso - rho * uz * uz;
    C.Pi[3] = M.m[8] - rho * ux * uy;
    C.Pi[4] = M.m[9] - rho * ux * uz;
    C.Pi[5] = M.m[10] - rho * uy * uz;
    const R pY = R(M.dm[1] * (1.0 / 3.0 + P.dcs2[0]));  // the ink's isotropic stress, from the FP64 mass
    const R Yxx = M.m[11] - pY - rY * ux * ux;
    const R Yyy = M.m[12] - pY - rY * uy * uy;
    const R Yzz = M.m[13] - pY - rY * uz * uz;
    const R Yxy = M.m[14] - rY * ux * uy;
    const R Yxz = M.m[15] - rY * ux * uz;
    const R Yyz = M.m[16] - rY * uy * uz;
    const R S = sqrt_of(Yxx * Yxx + Yyy * Yyy + Yzz * Yzz + R(2) * (Yxy * Yxy + Yxz * Yxz + Yyz * Yyz));
    // local relaxation time: ink from its strain rate, air Newtonian, mixed
    // harmonically in the viscosity (Eq. (tauinter))
    const R tauY = tau_ink<R>(P, S, rY);
    const R nuY = cs2 * (tauY - R(0.5)), nuB = cs2 * (R(P.tau_b) - R(0.5));
    const R inv_nu = (rY * irho) * rcp_of(nuY) + (rB * irho) * rcp_of(nuB);
    const R tau = R(0.5) + R(3) * rcp_of(inv_nu);
    C.om = R(1) - rcp_of(tau);
    return C;
}

// Collide one fluid cell from its state and colour gradients; store the 38
// post-collision values at the cell (the next step pulls them) and return
// rho_Y, rho_B and the bare velocity for the boundary rules of the next pull.
template <typename R, int ST = ST_PLAIN>
__device__ __forceinline__ void collide_state(const DevParams &P, const CellState<R> &C, const Grad<R> &G, int z,
                                              char *__restrict__ dst, unsigned long long pstride, unsigned cellb,
                                              R &out_rY, R &out_rB, R (&out_u)[3], float *__restrict__ mo_dst = nullptr,
                                              long long cell = 0)
{
    const double rho_d = P.rho_ref + C.drho;
    const double fracY_d = C.rY / rho_d;
    const R drho = R(C.drho), rY = R(C.rY);
    const R rho = R(rho_d);
    const R rB = R(rho_d - C.rY);
    const R irho = rcp_of(rho);
    const R ux = C.j[0] * irho, uy = C.j[1] * irho, uz = C.j[2] * irho;

    // force: body force and the substrate drag (exact-difference method)
    R Fx = rho * R(P.g[0]), Fy = rho * R(P.g[1]), Fz = rho * R(P.g[2]);
    if (P.drag_gamma != 0.0 && P.face_lo == FACE_WALL && (double)z + 0.5 < P.drag_range) {
        const R gam = R(P.drag_gamma) * rY;
        Fx -= gam * (ux - R(P.u_lo[0]));
        Fy -= gam * (uy - R(P.u_lo[1]));
        Fz -= gam * (uz - R(P.u_lo[2]));
    }
    const R vx = ux + Fx * irho, vy = uy + Fy * irho, vz = uz + Fz * irho;
    const R trPi = C.Pi[0] + C.Pi[1] + C.Pi[2];
    const R om = C.om;

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
    const R iF = pert ? rcp_of(Fmax) : R(0);
    Fcx *= iF;
    Fcy *= iF;
    Fcz *= iF;
    const R invFF = pert ? rcp_of(Fcx * Fcx + Fcy * Fcy + Fcz * Fcz) : R(0);
    const R gn2 = G.g[0] * G.g[0] + G.g[1] * G.g[1] + G.g[2] * G.g[2];
    const R pA = pert ? R(0.5) * R(P.A) * sqrt_of(gn2) : R(0);
    const R geps2 = gn2 + R(P.eps2);
    const R inv_geps = geps2 > R(0) ? rsqrt_of(geps2) : R(0);
    const R pn = pA * invFF;

    OutCoef<R> K;
    const R h = R(4.5);
    K.ax = R(3) * rho * vx;
    K.ay = R(3) * rho * vy;
    K.az = R(3) * rho * vz;
    K.bxx = h * (rho * vx * vx + om * C.Pi[0]) + pn * Fcx * Fcx - pA;
    K.byy = h * (rho * vy * vy + om * C.Pi[1]) + pn * Fcy * Fcy - pA;
    K.bzz = h * (rho * vz * vz + om * C.Pi[2]) + pn * Fcz * Fcz - pA;
    K.bxy = R(2) * (h * (rho * vx * vy + om * C.Pi[3]) + pn * Fcx * Fcy);
    K.bxz = R(2) * (h * (rho * vx * vz + om * C.Pi[4]) + pn * Fcx * Fcz);
    K.byz = R(2) * (h * (rho * vy * vz + om * C.Pi[5]) + pn * Fcy * Fcz);
    const R a0 = R(-1.5) * (rho * (vx * vx + vy * vy + vz * vz) + om * trPi) + R(2.0 / 3.0) * pA;
    // rest-frame weights relative to w: phi_i^k - w_i = w_i kappa_k (i > 0)
    // (the equilibrium shifts are formed from the FP64 masses: at unequal
    // alpha the terms are O(rho) and cancel to O(drho) on the moving links)
    const double rB_d = rho_d - C.rY;
    const double k1_eq = C.drho + C.rY * (P.phid[0][1] / lbq::w(1)) + rB_d * (P.phid[1][1] / lbq::w(1));
    const double t0_eq = lbq::w(0) * C.drho + C.rY * P.phid[0][0] + rB_d * P.phid[1][0];
    K.k1 = a0 + R(k1_eq);
    K.t0 = R(lbq::w(0)) * a0 + R(t0_eq);
    // recolouring: beta rho_Y rho_B / rho^2 * e / |grad rho^N|_eps * grad rho^N,
    // e = sum_k rho_k (1 - alpha_k) / (1 - w_0)
    const R e = rY * R(P.phi[0][1] / lbq::w(1)) + rB * R(P.phi[1][1] / lbq::w(1));
    const R rec = R(P.beta) * fracY * fracB * inv_geps * e;
    K.rx = rec * G.g[0];
    K.ry = rec * G.g[1];
    K.rz = rec * G.g[2];
    K.fracY = fracY_d;
    if constexpr (ST == ST_PLAIN) {
        store_all<R>(P, K, fresh_global(dst), fresh_uniform(pstride), cellb);
    } else {
        store_all_dev<ST>(P, K, rY, rB, vx, vy, vz, fresh_global(dst), fresh_uniform(pstride), cellb);
        const long long NM = P.NM;
        const auto md = as_global(mo_dst);
        md[cell] = rY;
        md[NM + cell] = rB;
        md[2 * NM + cell] = vx;
        md[3 * NM + cell] = vy;
        md[4 * NM + cell] = vz;
    }
    out_rY = rY;
    out_rB = rB;
    out_u[0] = ux;
    out_u[1] = uy;
    out_u[2] = uz;
}

}  // namespace lbk
