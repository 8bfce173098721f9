// lb_device.h -- per-cell device functions of the colour-gradient step.
//
// Population storage (both FP64 and FP32 forms): two structure-of-arrays
// sets, x fastest,
//   set 0: T_i = f^Y_i + f^B_i - w_i rho_ref   (the total, shifted by the
//          reference rest state so that bulk values are small deviations)
//   set 1: Y_i = f^Y_i                          (the ink)
// which is a change of basis of the paper's (f^Y, f^B): f^B_i = T_i + w_i
// rho_ref - Y_i.  Every formula below is the paper's, rewritten for this
// basis; the shift keeps the total density, momentum and stress accurate in
// FP32.
//
// The per-cell moment set carried from the pull to the collision (the
// regularised collision needs no more than these, Eq. (reg)):
//   dm[0] drho = sum T_i       (rho = rho_ref + drho)        FP64
//   dm[1] rhoY = sum Y_i                                     FP64
//   m[2..4]   j = sum T_i c_i  (total momentum)
//   m[5..10]  PT = sum T_i c c (xx, yy, zz, xy, xz, yz)
//   m[11..16] PY = sum Y_i c c
// The two masses are summed and carried in FP64 whatever the storage: in a
// uniform region every cell rounds alike, so FP32 rounding of a colour's mass
// (or of rho_Y / rho in the recolouring) would not average out but drift.
#pragma once

#include <utility>

#include <hip/hip_runtime.h>

#include "d3q19.h"

namespace lbk {

constexpr int NMOM = 17;   // indices of m[]; m[0], m[1] are unused (see dm)
constexpr int NMOMR = 15;  // moments stored in the storage type: m[2..16]
constexpr int NCHI = 3;   // rho^N, rho_Y/rho, rho_B/rho
constexpr int NMAC = 5;   // rho_Y, rho_B, u (bare) for the next pull's boundary rules

enum Rheo { RHEO_NEWTON = 0, RHEO_POWER = 1, RHEO_CROSS = 2 };
enum Face { FACE_PERIODIC = 0, FACE_WALL = 1, FACE_PRESSURE = 2 };
enum Col { COL_OUT = 0, COL_BORE = 1, COL_SHELL = 2 };
enum Site { ST_FLUID = 0, ST_NOZ, ST_WALL_LO, ST_WALL_HI, ST_OPEN_LO, ST_OPEN_HI, ST_LID };

// Everything a kernel needs about one simulation; passed by value.
struct DevParams {
    int nx, ny, nz;
    int periodic_z;
    int face_lo, face_hi;
    long long N;
    long long NP;              // population plane stride, in stored elements (N plus padding)
    long long NM;              // source-moment plane stride of the reduced forms (floats)
    double rho_ref;            // shift of set 0 (air reference density)
    double rho0[2];            // phase-field normalisation
    double phi[2][3];          // phi_i^k per shell
    double phid[2][3];         // phi_i^k - w_i per shell
    double dcs2[2];            // c_{s,k}^2 - c_s^2 (second moment of phi^k minus that of w)
    double A, beta, eps2;
    double tau_b;
    int rheology;
    double tau_y;
    double Kp, n;              // power law: nu / c_s^2 = Kp gdot^(n-1)
    double nu0p, nuinfp, lambda, m;  // Cross: nu / c_s^2 = nuinfp + (nu0p - nuinfp) / (1 + (lambda gdot)^m)
    double tau_min, tau_max;
    double s_lo, s_hi;         // shear-thinning clamp thresholds of s = S / (c_s^2 rho_Y)
    double lg_lo, lg_hi;       // log2 of the strain rates at the clamps
    double rho_eps;
    double zeta_wall[2], zeta_noz[2];
    double drag_gamma, drag_range;
    double g[3];
    double u_lo[3], u_hi[3];
    double rho_lo[2], rho_hi[2];
    int has_nozzle;
    double ri2, ro2, rout, tip_z;
    double vnoz[2];
    double x0noz[2];           // head axis (x, y) at t = 0
    double u_in[3];            // u_ink + v_nozzle, Eq. (movnozzle)
    double lid_rho;
    // Boundary-only arrays (moment sets and colour fields of the prepared
    // cells, macro fields for the next step's boundary rules): component
    // stride NA.  aux = 0: one slot per cell of the box (NA = N).  aux = 1:
    // compact slots (aidx) for the az_lo / az_hi layers at the z faces and
    // the head region -- planes ah_z0 .. nz - az_hi - 1, columns taken
    // modulo (aw, ah) from a_head0 on; slot NA - 1 is a sink for cells
    // outside both (never used by a correct step).
    int aux, az_lo, az_hi, ah_z0, aw, ah;
    int amx, amy;  // column masks of the window: aw - 1 (a power of two) or all ones (aw = nx)
    long long NA, a_head0;
    // equilibrium coefficients of the reduced storage forms (see EqCell):
    // phi_1^Y, phi_1^B, w_1 rho_ref, g_Y, g_Y - g_B, g_B
    float eqf[6];
};

// The same pointer in the global address space: global instructions count
// only against the vector-memory counter, where flat ones count against the
// LDS counter as well (a wait for an LDS read would also wait for them).
// Every array of the kernels lives in global memory.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *as_global(T *p)
{
    return (__attribute__((address_space(1))) T *)p;
}

// Head axis of the previous and the current step, wrapped into the box.
struct HeadPos {
    double hx_p, hy_p, hx_c, hy_c;
};

__device__ __forceinline__ int wrap(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// Slot of cell (x, y, z) (inside the box) in the boundary-only arrays.  The
// head region's window (aw x ah columns, each a power of two dividing the
// box extent, or the extent itself) is wider than every set of cells a step
// or two consecutive steps touch around the head axis (the head box, its
// neighbours, the macro fields written for the next step), so no two cells
// in use at once share a slot.  Straight-line code: it is inlined at every
// boundary rule's neighbour reads.
__host__ __device__ inline long long aidx(const DevParams &P, int x, int y, int z)
{
    const long long pl = (long long)P.nx * P.ny;
    if (!P.aux) return (long long)z * pl + (long long)y * P.nx + x;
    if (z < P.az_lo) return (long long)z * pl + (long long)y * P.nx + x;
    if (z >= P.nz - P.az_hi) return (long long)(P.az_lo + z - (P.nz - P.az_hi)) * pl + (long long)y * P.nx + x;
    if (z < P.ah_z0) return P.NA - 1;
    return P.a_head0 + ((long long)(z - P.ah_z0) * P.ah + (y & P.amy)) * P.aw + (x & P.amx);
}

// ---------------------------------------------------------------- geometry
// Decided in FP64 with every operation rounded as written (no FMA
// contraction), so that the rasterised template is identical on every
// implementation that evaluates the same expressions.

__device__ __forceinline__ int column_class(const DevParams &P, double hx, double hy, int x, int y)
{
#pragma clang fp contract(off)
    double dx = (double)x - hx;
    double dy = (double)y - hy;
    if (dx >= 0.5 * P.nx) dx -= P.nx;
    if (dx < -0.5 * P.nx) dx += P.nx;
    if (dy >= 0.5 * P.ny) dy -= P.ny;
    if (dy < -0.5 * P.ny) dy += P.ny;
    double r2 = dx * dx + dy * dy;
    if (r2 < P.ri2) return COL_BORE;
    if (r2 < P.ro2) return COL_SHELL;
    return COL_OUT;
}

// True when no column within one lattice link of (x, y) can touch the shell:
// lets bulk cells skip the FP64 geometry entirely (conservative).
__device__ __forceinline__ bool far_from_head(const DevParams &P, double hx, double hy, int x, int y)
{
    if (!P.has_nozzle) return true;
    double dx = fabs((double)x - hx), dy = fabs((double)y - hy);
    dx = fmin(dx, (double)P.nx - dx);
    dy = fmin(dy, (double)P.ny - dy);
    double lim = P.rout + 3.0;
    return dx > lim || dy > lim;
}

__device__ __forceinline__ bool is_solid(const DevParams &P, double hx, double hy, int x, int y, int z)
{
    if (!P.has_nozzle) return false;
    if ((double)z < P.tip_z) return false;
    return column_class(P, hx, hy, x, y) == COL_SHELL;
}

// Site type of (x, y, z) (x, y already wrapped); z is wrapped in place when
// the z faces are periodic.  Above the top face the head's columns override
// the face: bore = inlet lid, shell = nozzle solid.
__device__ __forceinline__ int classify(const DevParams &P, double hx, double hy, int x, int y, int &z, bool near)
{
    if (z < 0 || z >= P.nz) {
        if (P.periodic_z) {
            z = wrap(z, P.nz);
        } else {
            bool lo = z < 0;
            if (!lo && near) {
                int cc = column_class(P, hx, hy, x, y);
                if (cc == COL_BORE) return ST_LID;
                if (cc == COL_SHELL) return ST_NOZ;
            }
            int face = lo ? P.face_lo : P.face_hi;
            if (face == FACE_WALL) return lo ? ST_WALL_LO : ST_WALL_HI;
            return lo ? ST_OPEN_LO : ST_OPEN_HI;
        }
    }
    if (near && is_solid(P, hx, hy, x, y, z)) return ST_NOZ;
    return ST_FLUID;
}

// classify() for a site whose column class at the previous head position is
// already known (cc): the same decision without the geometry.
__device__ __forceinline__ int classify_cc(const DevParams &P, int cc, int &z, bool near)
{
    if (z < 0 || z >= P.nz) {
        if (P.periodic_z) {
            z = wrap(z, P.nz);
        } else {
            bool lo = z < 0;
            if (!lo && near) {
                if (cc == COL_BORE) return ST_LID;
                if (cc == COL_SHELL) return ST_NOZ;
            }
            int face = lo ? P.face_lo : P.face_hi;
            if (face == FACE_WALL) return lo ? ST_WALL_LO : ST_WALL_HI;
            return lo ? ST_OPEN_LO : ST_OPEN_HI;
        }
    }
    if (near && P.has_nozzle && (double)z >= P.tip_z && cc == COL_SHELL) return ST_NOZ;
    return ST_FLUID;
}

// Column classes of the 3 x 3 columns around (x, y) at the previous head
// position (cc[1 + dx][1 + dy]); only near the head, where they matter.
__device__ __forceinline__ void column_classes(const DevParams &P, const HeadPos &H, int x, int y, bool near,
                                               int (&cc)[3][3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            cc[a][b] = near ? column_class(P, H.hx_p, H.hy_p, wrap(x + a - 1, P.nx), wrap(y + b - 1, P.ny)) : COL_OUT;
}

__device__ __forceinline__ long long cidx(const DevParams &P, int x, int y, int z)
{
    return ((long long)z * P.ny + y) * P.nx + x;
}

// --------------------------------------------------------------- moments

template <typename R>
struct Mom {
    double dm[2];
    R m[NMOM];
};

// Sums start at -0, the identity of IEEE addition (+0 is not: -0 + 0 = +0),
// so the first term costs no addition.
template <typename R>
__device__ __forceinline__ void mom_zero(Mom<R> &M)
{
    M.dm[0] = M.dm[1] = -0.0;
#pragma unroll
    for (int q = 0; q < NMOM; ++q) M.m[q] = R(-0.0);
}

// Accumulate one pulled population pair.  FULL = false keeps only the two
// masses (cells whose density feeds a neighbour's colour gradient).
template <typename R, int I, bool FULL = true>
__device__ __forceinline__ void mom_add(Mom<R> &M, R T, R Y)
{
    constexpr int X = lbq::cx(I), Yc = lbq::cy(I), Z = lbq::cz(I);
    M.dm[0] += (double)T;
    M.dm[1] += (double)Y;
    if constexpr (!FULL) return;
    if (X) M.m[2] += X > 0 ? T : -T;
    if (Yc) M.m[3] += Yc > 0 ? T : -T;
    if (Z) M.m[4] += Z > 0 ? T : -T;
    if (X) M.m[5] += T;
    if (Yc) M.m[6] += T;
    if (Z) M.m[7] += T;
    if (X && Yc) M.m[8] += X * Yc > 0 ? T : -T;
    if (X && Z) M.m[9] += X * Z > 0 ? T : -T;
    if (Yc && Z) M.m[10] += Yc * Z > 0 ? T : -T;
    if (X) M.m[11] += Y;
    if (Yc) M.m[12] += Y;
    if (Z) M.m[13] += Y;
    if (X && Yc) M.m[14] += X * Yc > 0 ? Y : -Y;
    if (X && Z) M.m[15] += X * Z > 0 ? Y : -Y;
    if (Yc && Z) M.m[16] += Yc * Z > 0 ? Y : -Y;
}

// Accumulate link I (odd) and its opposite I + 1 together: the odd moments
// take the pair's difference and the even ones its sum, one addition each
// instead of two; the masses stay per link (FP64).
template <typename R, int I, bool FULL = true>
__device__ __forceinline__ void mom_add_pair(Mom<R> &M, R Ta, R Ya, R Tb, R Yb)
{
    static_assert((I & 1) == 1 && lbq::opp(I) == I + 1, "a link and its opposite");
    constexpr int X = lbq::cx(I), Yc = lbq::cy(I), Z = lbq::cz(I);
    M.dm[0] += (double)Ta;
    M.dm[1] += (double)Ya;
    M.dm[0] += (double)Tb;
    M.dm[1] += (double)Yb;
    if constexpr (!FULL) return;
    const R dT = Ta - Tb, sT = Ta + Tb, sY = Ya + Yb;
    if (X) M.m[2] += X > 0 ? dT : -dT;
    if (Yc) M.m[3] += Yc > 0 ? dT : -dT;
    if (Z) M.m[4] += Z > 0 ? dT : -dT;
    if (X) M.m[5] += sT;
    if (Yc) M.m[6] += sT;
    if (Z) M.m[7] += sT;
    if (X && Yc) M.m[8] += X * Yc > 0 ? sT : -sT;
    if (X && Z) M.m[9] += X * Z > 0 ? sT : -sT;
    if (Yc && Z) M.m[10] += Yc * Z > 0 ? sT : -sT;
    if (X) M.m[11] += sY;
    if (Yc) M.m[12] += sY;
    if (Z) M.m[13] += sY;
    if (X && Yc) M.m[14] += X * Yc > 0 ? sY : -sY;
    if (X && Z) M.m[15] += X * Z > 0 ? sY : -sY;
    if (Yc && Z) M.m[16] += Yc * Z > 0 ? sY : -sY;
}

// Boundary-flux accumulators of one pull (FP64): bounce-back family (Y, B),
// anti-bounce-back (Y, B).
struct Flux {
    double wallY, wallB, openY, openB;
};

// ------------------------------------------------------ population storage
// ST 0: populations stored in the arithmetic type R (set T: f - w rho_ref,
// set Y: f^Y).  ST 1 / 2 (reduced storage, R = float): the deviation of each
// post-collision population from the equilibrium of its source cell's
// moments (rho_Y, rho_B, u'), as BF16 (ST 1) or as FP16 of delta / w_i
// (ST 2), with the moments stored in FP32 beside them.  The two deviations
// of link i (set T in the low half, set Y in the high half) share one 32-bit
// word: 19 planes of words, one memory instruction per link.  Encoder and decoder
// evaluate the equilibrium with the same function (no contraction), so the
// only loss is the 16-bit rounding of the deviation.
enum { ST_PLAIN = 0, ST_BF16 = 1, ST_F16 = 2 };
constexpr int NMO = 5;  // stored source moments: rho_Y, rho_B, u'_x, u'_y, u'_z

__device__ __forceinline__ float dec_bf16(unsigned short h) { return __uint_as_float((unsigned)h << 16); }
__device__ __forceinline__ float dec_f16(unsigned short h) { return (float)__builtin_bit_cast(_Float16, h); }

// The stored word of link I: the deviations of set T (low half) and set Y
// (high half), rounded to nearest even by one packed conversion.
template <int ST, int I>
__device__ __forceinline__ unsigned encode_pair(float dT, float dY)
{
    typedef float f2v __attribute__((ext_vector_type(2)));
    if constexpr (ST == ST_BF16) {
        typedef __bf16 h2v __attribute__((ext_vector_type(2)));
        return __builtin_bit_cast(unsigned, __builtin_convertvector((f2v{dT, dY}), h2v));
    } else {
        typedef _Float16 h2v __attribute__((ext_vector_type(2)));
        constexpr float k = float(1.0 / lbq::w(I));
        return __builtin_bit_cast(unsigned, __builtin_convertvector((f2v{dT * k, dY * k}), h2v));
    }
}

template <int ST, int I>
__device__ __forceinline__ float decode_dev(unsigned short h)
{
    if constexpr (ST == ST_BF16)
        return dec_bf16(h);
    else
        return dec_f16(h) * float(lbq::w(I));
}

// Equilibrium of link I for moments (rho_Y, rho_B, u), in the stored bases:
// T = f^eq - w_I rho_ref (both colours), Y = f^{Y,eq}.  For a moving link
// phi_I^k = w_I (1 - alpha_k) / (1 - w_0) (Sec. II.A), so both are w_I / w_1
// (w_1: the weight of an axis link) times an affine function of
// q_I = 3 c_I.u + 9/2 (c_I.u)^2 whose coefficients belong to the cell:
//   T = s_I (t_rho q_I + a_T),   Y = s_I (t_Y q_I + a_Y),   s_I = w_I / w_1,
//   t_rho = w_1 rho,  t_Y = w_1 rho_Y,  k = 3/2 u.u,
//   a_T = phi_1^Y rho_Y + phi_1^B rho_B - w_1 (rho_ref + rho k),
//   a_Y = rho_Y (phi_1^Y - w_1 k).
// s_I is 1 or 1/2, so the scaling is exact.  The rest link follows from the
// same coefficients: Y_0 = g_Y t_Y + (w_0 / w_1) a_Y and
// T_0 = (g_Y - g_B) t_Y + g_B t_rho + (w_0 / w_1) a_T, with
// g_k = (alpha_k - w_0 phi_1^k / w_1) / w_1 (DevParams::eqf).  A cell's
// coefficients (EqCell) are formed once; a link then costs a few operations.
// Explicit fused multiply-adds make the result the same instructions
// wherever it is inlined (encoder and decoders agree bit for bit).
struct EqCell {
    float tr, ty, aT, aY, ux3, uy3, uz3;  // t_rho, t_Y, a_T, a_Y, 3u
};

__device__ __forceinline__ EqCell eq_cell(const DevParams &P, float rY, float rB, float ux, float uy, float uz)
{
#pragma clang fp contract(off)
    constexpr float w1 = float(lbq::w_of_shell(1));
    EqCell c;
    const float k = 1.5f * __builtin_fmaf(ux, ux, __builtin_fmaf(uy, uy, uz * uz));
    c.tr = w1 * (rY + rB);
    c.ty = w1 * rY;
    c.aT = __builtin_fmaf(-c.tr, k, __builtin_fmaf(rY, P.eqf[0], __builtin_fmaf(rB, P.eqf[1], -P.eqf[2])));
    c.aY = __builtin_fmaf(-c.ty, k, rY * P.eqf[0]);
    c.ux3 = 3.f * ux;
    c.uy3 = 3.f * uy;
    c.uz3 = 3.f * uz;
    return c;
}

// s_I of the scaling above
template <int I>
constexpr float eq_scale()
{
    return I == 0 ? 1.f : float(lbq::w(I) / lbq::w_of_shell(1));
}

// Link I's equilibrium before the scaling: T = s_I fT, Y = s_I fY.
template <int I>
__device__ __forceinline__ void feq_TY_cell(const DevParams &P, const EqCell &c, float &fT, float &fY)
{
#pragma clang fp contract(off)
    constexpr int X = lbq::cx(I), Yc = lbq::cy(I), Z = lbq::cz(I);
    if constexpr (I == 0) {
        constexpr float r0 = float(lbq::w_of_shell(0) / lbq::w_of_shell(1));
        fY = __builtin_fmaf(c.ty, P.eqf[3], r0 * c.aY);
        fT = __builtin_fmaf(c.ty, P.eqf[4], __builtin_fmaf(c.tr, P.eqf[5], r0 * c.aT));
    } else {
        // c_I . 3u over the nonzero components only (an added 0 would stay:
        // it is not an identity for -0)
        const float ax = X > 0 ? c.ux3 : -c.ux3, ay = Yc > 0 ? c.uy3 : -c.uy3, az = Z > 0 ? c.uz3 : -c.uz3;
        static_assert((X != 0) + (Yc != 0) + (Z != 0) <= 2, "D3Q19 links have at most two components");
        float cu;
        if constexpr (X != 0)
            cu = Yc != 0 ? ax + ay : (Z != 0 ? ax + az : ax);
        else
            cu = Yc != 0 ? (Z != 0 ? ay + az : ay) : az;
        const float q = cu * __builtin_fmaf(0.5f, cu, 1.f);
        fT = __builtin_fmaf(c.tr, q, c.aT);
        fY = __builtin_fmaf(c.ty, q, c.aY);
    }
}

// Link I of a cell from its stored word (16-bit deviations: T in the low
// half, Y in the high half) and its source cell's coefficients.
template <int ST, int I>
__device__ __forceinline__ void dec_link(const DevParams &P, const EqCell &c, unsigned w, float &T, float &Y)
{
    float fT, fY;
    feq_TY_cell<I>(P, c, fT, fY);
    constexpr float s = eq_scale<I>();
    T = __builtin_fmaf(s, fT, decode_dev<ST, I>((unsigned short)(w & 0xFFFFu)));
    Y = __builtin_fmaf(s, fY, decode_dev<ST, I>((unsigned short)(w >> 16)));
}

// Read access to the post-collision populations of step t-1: the reduced
// storage forms (R = float) in the primary template, plain storage below.
template <typename R, int ST>
struct PopSrc {
    static_assert(sizeof(R) == 4, "reduced storage computes in FP32");
    const unsigned *s;
    const float *mo;      // NMO planes of source moments
    long long N, NP, NM;  // cells; population and moment plane strides
    // what a link needs from memory: the packed word of population plane
    // `plane` at `cell` and that cell's moments; decoded for link I
    struct Raw {
        unsigned w;
        float m[NMO];
    };
    __device__ __forceinline__ Raw load_raw(int plane, long long cell) const
    {
        Raw r;
        r.w = as_global(s)[plane * NP + cell];
#pragma unroll
        for (int k = 0; k < NMO; ++k) r.m[k] = as_global(mo)[k * NM + cell];
        return r;
    }
    template <int I>
    __device__ __forceinline__ void finish(const DevParams &P, const Raw &r, float &T, float &Y) const
    {
        dec_link<ST, I>(P, eq_cell(P, r.m[0], r.m[1], r.m[2], r.m[3], r.m[4]), r.w, T, Y);
    }
    template <int I>
    __device__ __forceinline__ void get(const DevParams &P, long long cell, float &T, float &Y) const
    {
        finish<I>(P, load_raw(I, cell), T, Y);
    }
};

template <typename R>
struct PopSrc<R, ST_PLAIN> {
    const R *s;
    long long N, NP;  // cells; population plane stride
    struct Raw {
        R T, Y;
    };
    __device__ __forceinline__ Raw load_raw(int plane, long long cell) const
    {
        return Raw{as_global(s)[plane * NP + cell], as_global(s)[(lbq::Q + plane) * NP + cell]};
    }
    template <int I>
    __device__ __forceinline__ void finish(const DevParams &, const Raw &r, R &T, R &Y) const
    {
        T = r.T;
        Y = r.Y;
    }
    template <int I>
    __device__ __forceinline__ void get(const DevParams &, long long cell, R &T, R &Y) const
    {
        T = as_global(s)[I * NP + cell];
        Y = as_global(s)[(lbq::Q + I) * NP + cell];
    }
};

// Boundary rule of link I (Eq. (lbm) as a pull): f_i(x, t) comes from x - c_i
// at t-1 unless that site is not fluid at t-1; then from the rule applied to
// x's own post-collision population of the opposite link, (Tout, Yout)
// (Sec. II.B: halfway bounce-back, Eq. (movwall) with the wall density
// extrapolated inward, Eq. (movnozzle) on the lid, anti-bounce-back on
// pressure faces).  st: the class of x - c_i.
template <typename R, int I, bool FULL = true>
__device__ __forceinline__ void pull_rule(const DevParams &P, const HeadPos &H, const R *__restrict__ mac, int x,
                                          int y, int z, long long acell, bool near, const int (&cc)[3][3], int st,
                                          R Tout, R Yout, Mom<R> &M, Flux &fl)
{
    constexpr int X = lbq::cx(I), Yc = lbq::cy(I), Z = lbq::cz(I);
    const long long N = P.NA;  // mac: boundary-only arrays, cell = this cell's slot
    const R wi = R(lbq::w(I));
    R T, Yv;
    if (st == ST_OPEN_LO || st == ST_OPEN_HI) {
        const bool lo = st == ST_OPEN_LO;
        const double rw0 = lo ? P.rho_lo[0] : P.rho_hi[0], rw1 = lo ? P.rho_lo[1] : P.rho_hi[1];
        // u_w = (3 u(x) - u(x + c_i)) / 2 at t-1 when x + c_i was fluid
        R ux = as_global(mac)[2 * N + acell], uy = as_global(mac)[3 * N + acell], uz = as_global(mac)[4 * N + acell];
        int x1 = X ? wrap(x + X, P.nx) : x, y1 = Yc ? wrap(y + Yc, P.ny) : y, z1 = z + Z;
        int s1 = classify_cc(P, cc[1 + X][1 + Yc], z1, near);
        if (s1 == ST_FLUID) {
            const long long c1 = aidx(P, x1, y1, z1);
            ux = (R(3) * ux - as_global(mac)[2 * N + c1]) * R(0.5);
            uy = (R(3) * uy - as_global(mac)[3 * N + c1]) * R(0.5);
            uz = (R(3) * uz - as_global(mac)[4 * N + c1]) * R(0.5);
        }
        R cu = R(X) * ux + R(Yc) * uy + R(Z) * uz;
        R uu = ux * ux + uy * uy + uz * uz;
        R E = wi * (cu * cu * R(4.5) - uu * R(1.5));
        R phiY = R(P.phi[0][lbq::shell(I)]), phiB = R(P.phi[1][lbq::shell(I)]);
        R rY = R(rw0), rB = R(rw1);
        Yv = -Yout + R(2) * rY * (phiY + E);
        T = -Tout - R(2) * wi * R(P.rho_ref) + R(2) * (rY * phiY + rB * phiB) + R(2) * (rY + rB) * E;
    } else {
        double U0, U1, U2;
        R rwY, rwB;
        if (st == ST_LID) {
            U0 = P.u_in[0];
            U1 = P.u_in[1];
            U2 = P.u_in[2];
            rwY = R(P.lid_rho);
            rwB = R(0);
        } else {
            if (st == ST_NOZ) {
                U0 = P.vnoz[0];
                U1 = P.vnoz[1];
                U2 = 0.0;
            } else {
                const bool lo = st == ST_WALL_LO;
                U0 = lo ? P.u_lo[0] : P.u_hi[0];
                U1 = lo ? P.u_lo[1] : P.u_hi[1];
                U2 = lo ? P.u_lo[2] : P.u_hi[2];
            }
            rwY = R(0);
            rwB = R(0);
            if (U0 * X + U1 * Yc + U2 * Z != 0.0) {
                // rho_w by quadratic extrapolation to the link midpoint from
                // x, x + c_i, x + 2 c_i (the inward direction), at t-1
                R r0Y = as_global(mac)[0 * N + acell], r0B = as_global(mac)[1 * N + acell];
                int x1 = X ? wrap(x + X, P.nx) : x, y1 = Yc ? wrap(y + Yc, P.ny) : y, z1 = z + Z;
                int s1 = classify_cc(P, cc[1 + X][1 + Yc], z1, near);
                if (s1 == ST_FLUID) {
                    const long long c1 = aidx(P, x1, y1, z1);
                    R r1Y = as_global(mac)[0 * N + c1], r1B = as_global(mac)[1 * N + c1];
                    int x2 = X ? wrap(x1 + X, P.nx) : x1, y2 = Yc ? wrap(y1 + Yc, P.ny) : y1, z2 = z1 + Z;
                    int s2 = classify(P, H.hx_p, H.hy_p, x2, y2, z2, near);
                    if (s2 == ST_FLUID) {
                        const long long c2 = aidx(P, x2, y2, z2);
                        R r2Y = as_global(mac)[0 * N + c2], r2B = as_global(mac)[1 * N + c2];
                        rwY = (R(15) * r0Y - R(10) * r1Y + R(3) * r2Y) * R(0.125);
                        rwB = (R(15) * r0B - R(10) * r1B + R(3) * r2B) * R(0.125);
                    } else {
                        rwY = (R(3) * r0Y - r1Y) * R(0.5);
                        rwB = (R(3) * r0B - r1B) * R(0.5);
                    }
                } else {
                    rwY = r0Y;
                    rwB = r0B;
                }
                rwY = rwY > R(0) ? rwY : R(0);
                rwB = rwB > R(0) ? rwB : R(0);
            }
        }
        // f_i(x, t) = f*_ibar(x, t-1) + 2 w_i rho_w (U . c_i) / c_s^2
        R Uc = R(U0 * X + U1 * Yc + U2 * Z);
        R k = R(6) * wi * Uc;
        Yv = Yout + k * rwY;
        T = Tout + k * (rwY + rwB);
    }
    // mass this link's rule adds, per colour (selects, not branches, so the
    // accumulators stay in registers)
    const bool open = st == ST_OPEN_LO || st == ST_OPEN_HI;
    const double dY = (double)(Yv - Yout), dB = (double)(T - Tout) - dY;
    fl.openY += open ? dY : 0.0;
    fl.openB += open ? dB : 0.0;
    fl.wallY += open ? 0.0 : dY;
    fl.wallB += open ? 0.0 : dB;
    mom_add<R, I, FULL>(M, T, Yv);
}

// Pull of all links of one cell with the boundary rules.  Every link is
// classified first and its population read (from x - c_i, or x's own
// opposite link at a boundary) before any rule is applied, so the reads are
// in flight together; then the rules and the moments, link by link in order.
template <typename R, bool FULL = true, typename PS>
__device__ __forceinline__ void pull_all(const DevParams &P, const HeadPos &H, const PS &src,
                                         const R *__restrict__ mac, int x, int y, int z, long long cell, bool near,
                                         bool first, Mom<R> &M, Flux &fl)
{
    typename PS::Raw raw[lbq::Q];
    int st[lbq::Q];
    int cc[3][3];
    column_classes(P, H, x, y, near && !first, cc);
    const long long acell = aidx(P, x, y, z);  // slot in the macro fields
    [&]<int... I>(std::integer_sequence<int, I...>) {
        (
            [&] {
                constexpr int X = lbq::cx(I), Yc = lbq::cy(I), Z = lbq::cz(I);
                int s_ = ST_FLUID, plane = I;
                long long sc = cell;
                if (!first) {
                    const int xs = X ? wrap(x - X, P.nx) : x;
                    const int ys = Yc ? wrap(y - Yc, P.ny) : y;
                    int zs = z - Z;  // classify wraps it when z is periodic
                    s_ = (Z == 0 && !near) ? ST_FLUID : classify_cc(P, cc[1 - X][1 - Yc], zs, near);
                    const long long scf = ((long long)zs * P.ny + ys) * P.nx + xs;
                    sc = s_ == ST_FLUID ? scf : cell;
                    plane = s_ == ST_FLUID ? I : lbq::opp(I);
                }
                st[I] = s_;
                raw[I] = src.load_raw(plane, sc);
            }(),
            ...);
    }(std::make_integer_sequence<int, lbq::Q>{});
    [&]<int... I>(std::integer_sequence<int, I...>) {
        (
            [&] {
                R T, Y;
                if (st[I] == ST_FLUID) {
                    src.template finish<I>(P, raw[I], T, Y);
                    mom_add<R, I, FULL>(M, T, Y);
                } else {
                    src.template finish<lbq::opp(I)>(P, raw[I], T, Y);
                    pull_rule<R, I, FULL>(P, H, mac, x, y, z, acell, near, cc, st[I], T, Y, M, fl);
                }
            }(),
            ...);
    }(std::make_integer_sequence<int, lbq::Q>{});
}

// A uniform (scalar) value the optimiser must treat as new at this point:
// derived addresses are then formed where they are used instead of being
// hoisted out of a loop and kept (and spilled) for its whole length.
template <typename T>
__device__ __forceinline__ T fresh_uniform(T v)
{
    asm volatile("" : "+s"(v));
    return v;
}

// Global-memory pointers (address space 1): loads and stores through them are
// global (not flat) instructions with a scalar base.
typedef __attribute__((address_space(1))) char gchar;
typedef __attribute__((address_space(1))) const char gcchar;

template <typename P>
__device__ __forceinline__ gchar *fresh_global(P *p)
{
    return (gchar *)fresh_uniform((unsigned long long)p);
}

template <typename P>
__device__ __forceinline__ gcchar *fresh_global_c(const P *p)
{
    return (gcchar *)fresh_uniform((unsigned long long)p);
}

// Pull of a cell none of whose links touches a boundary (all 18 sources are
// fluid at t-1): plain shifted loads, x and y periodic, z periodic or inside.
// Addresses are a scalar plane base plus a 32-bit byte offset (one address
// register per load, no 64-bit vector arithmetic); a population plane is
// below 4 GiB (checked at creation).
struct BulkIdx {
    unsigned xo[3], yo[3], zo[3];  // byte offsets of x-1..x+1, rows y-1..y+1, planes z-1..z+1
};

template <typename R>
__device__ __forceinline__ BulkIdx bulk_index(const DevParams &P, int x, int y, int z)
{
    BulkIdx b;
    const unsigned s = sizeof(R), row = (unsigned)P.nx * s, plane = (unsigned)P.nx * (unsigned)P.ny * s;
#pragma unroll
    for (int d = -1; d <= 1; ++d) {
        b.xo[d + 1] = (unsigned)wrap(x + d, P.nx) * s;
        b.yo[d + 1] = (unsigned)wrap(y + d, P.ny) * row;
        b.zo[d + 1] = (unsigned)wrap(z + d, P.nz) * plane;
    }
    return b;
}

// mom_add over all links of loaded values: the rest link, then one opposite
// pair at a time (the barrier keeps the scheduler from converting every
// loaded value to FP64 up front, 76 registers, before the mass sums consume
// them).
template <typename R, bool FULL, int I = 0>
__device__ __forceinline__ void mom_add_all(Mom<R> &M, const R (&vT)[lbq::Q], const R (&vY)[lbq::Q])
{
    if constexpr (I == 0) {
        mom_add<R, 0, FULL>(M, vT[0], vY[0]);
        __builtin_amdgcn_sched_barrier(0);
        mom_add_all<R, FULL, 1>(M, vT, vY);
    } else if constexpr (I < lbq::Q) {
        mom_add_pair<R, I, FULL>(M, vT[I], vY[I], vT[I + 1], vY[I + 1]);
        __builtin_amdgcn_sched_barrier(0);
        mom_add_all<R, FULL, I + 2>(M, vT, vY);
    }
}

// The 38 loads of a bulk pull (issued together, used later: the march keeps
// them in flight across another plane's collision).  base: population plane
// 0 of the source set; pstride: bytes per population plane; cellb: the
// cell's own byte offset (the first step reads the cell's own slots: the
// initial state is an equilibrium).
template <typename R, bool FIRST>
__device__ __forceinline__ void pull_bulk_issue(gcchar *base, unsigned long long pstride, const BulkIdx &B,
                                                unsigned cellb, R (&vT)[lbq::Q], R (&vY)[lbq::Q])
{
    typedef __attribute__((address_space(1))) const R gR;
    gcchar *pT = base;
    gcchar *pY = base + (unsigned long long)lbq::Q * pstride;
#pragma unroll
    for (int I = 0; I < lbq::Q; ++I) {
        const unsigned off = FIRST ? cellb : B.zo[1 - lbq::cz(I)] + B.yo[1 - lbq::cy(I)] + B.xo[1 - lbq::cx(I)];
        vT[I] = *reinterpret_cast<gR *>(pT + off);
        vY[I] = *reinterpret_cast<gR *>(pY + off);
        pT += pstride;
        pY += pstride;
    }
}

// The 19 word loads of a bulk pull in the reduced storage forms.
template <bool FIRST>
__device__ __forceinline__ void pull_bulk_issue_words(gcchar *base, unsigned long long pstride, const BulkIdx &B,
                                                      unsigned cellb, unsigned (&v)[lbq::Q])
{
    typedef __attribute__((address_space(1))) const unsigned gU;
    gcchar *p = base;
#pragma unroll
    for (int I = 0; I < lbq::Q; ++I) {
        const unsigned off = FIRST ? cellb : B.zo[1 - lbq::cz(I)] + B.yo[1 - lbq::cy(I)] + B.xo[1 - lbq::cx(I)];
        v[I] = *reinterpret_cast<gU *>(p + off);
        p += pstride;
    }
}


// Reciprocal and square roots.  FP32 takes the hardware approximations
// (v_rcp_f32, v_sqrt_f32, v_rsq_f32: about 1 ulp, flushed denormal
// results) where IEEE division would cost a ten-instruction sequence; the
// operands here are O(1) or clamped away from the denormal range.  FP64 keeps
// the correctly rounded forms.
template <typename R>
__device__ __forceinline__ R rcp_of(R v)
{
    return R(1) / v;
}
template <>
__device__ __forceinline__ float rcp_of<float>(float v)
{
    return __builtin_amdgcn_rcpf(v);
}
template <typename R>
__device__ __forceinline__ R sqrt_of(R v)
{
    return sqrt(v);
}
template <>
__device__ __forceinline__ float sqrt_of<float>(float v)
{
    return __builtin_amdgcn_sqrtf(v);
}
template <typename R>
__device__ __forceinline__ R rsqrt_of(R v)
{
    return R(1) / sqrt(v);
}
template <>
__device__ __forceinline__ float rsqrt_of<float>(float v)
{
    // a denormal argument is raised to the smallest normal float, so that a
    // flushed input cannot turn into an infinite result
    return __builtin_amdgcn_rsqf(fmaxf(v, 1.17549435e-38f));
}

// Colour fields of a site from its densities: rho^N (the standard phase field
// (rho_Y/rho_Y^0 - rho_B/rho_B^0) / (rho_Y/rho_Y^0 + rho_B/rho_B^0)) and the
// colour fractions.  Zero where the densities vanish.
template <typename R>
__device__ __forceinline__ void chi_of(const DevParams &P, R rY, R rB, R &cN, R &cY, R &cB)
{
    R a = rY * R(1.0 / P.rho0[0]), b = rB * R(1.0 / P.rho0[1]);
    R s = a + b, t = rY + rB;
    const R is = s != R(0) ? rcp_of(s) : R(0);
    const R it = t != R(0) ? rcp_of(t) : R(0);
    cN = (a - b) * is;
    cY = rY * it;
    cB = rB * it;
}

// ----------------------------------------------------------- rheology

// Ink relaxation time from the strain rate, Eqs. (stressvsstrain) and
// (tauofgammadot): gdot tau_Y(gdot) = s with s = |Pi^Y| / (c_s^2 rho_Y) and
// gdot = 2|Gamma|.  The unclamped law gdot tau(gdot) is increasing, so the
// clamped solution is clamp(tau(root of the unclamped equation)).  Power law:
// precomputed thresholds give the clamped ends exactly; inside, Newton on
// log2(gdot) from the right of the root (the log-sum-exp is convex, so the
// iterates decrease monotonically), 4 steps.  Cross: Newton with a bracket.
template <typename R>
__device__ __forceinline__ R lg2(R v);
template <>
__device__ __forceinline__ float lg2<float>(float v) { return __log2f(v); }
template <>
__device__ __forceinline__ double lg2<double>(double v) { return log2(v); }
template <typename R>
__device__ __forceinline__ R ex2(R v);
template <>
__device__ __forceinline__ float ex2<float>(float v) { return __builtin_amdgcn_exp2f(v); }
template <>
__device__ __forceinline__ double ex2<double>(double v) { return exp2(v); }

template <typename R>
__device__ __forceinline__ R tau_ink(const DevParams &P, R S, R rY)
{
    if (P.rheology == RHEO_NEWTON) return R(P.tau_y);
    R r = rY > R(P.rho_eps) ? rY : R(P.rho_eps);
    R s = S * R(3) * rcp_of(r);
    const R tmin = R(P.tau_min), tmax = R(P.tau_max);
    if (P.rheology == RHEO_POWER) {
        if (!(s > R(P.s_lo))) return tmax;
        if (s >= R(P.s_hi)) return tmin;
        const R n = R(P.n), Kp = R(P.Kp);
        const R ls = lg2<R>(s);
        // start: the smaller of the inertial and the viscous limits, clipped
        R x = fmin(ls + R(1), (ls - lg2<R>(Kp)) * rcp_of(n));
        x = fmin(fmax(x, R(P.lg_lo)), R(P.lg_hi));
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            R a = R(0.5) * ex2<R>(x);
            R b = Kp * ex2<R>(n * x);
            R G = a + b;
            R h = lg2<R>(G) - ls;
            x -= h * G * rcp_of(a + n * b);
        }
        R tau = R(0.5) + Kp * ex2<R>((n - R(1)) * x);
        return fmin(fmax(tau, tmin), tmax);
    }
    // Cross law
    const R m = R(P.m), lam = R(P.lambda), nuinf = R(P.nuinfp), dnu = R(P.nu0p - P.nuinfp);
    const R t0 = R(0.5) + R(P.nu0p), tinf = R(0.5) + R(P.nuinfp);
    if (!(s > R(0))) return fmin(fmax(t0, tmin), tmax);
    R lo = lg2<R>(s / fmax(t0, tinf)), hi = lg2<R>(s / fmin(t0, tinf));
    R x = hi;
    const R ls = lg2<R>(s);
    const R llam = lg2<R>(lam > R(0) ? lam : R(1));
#pragma unroll 1
    for (int it = 0; it < 12; ++it) {
        R q = lam > R(0) ? ex2<R>(m * (llam + x)) : R(0);
        const R iq = rcp_of(R(1) + q);
        R nu = nuinf + dnu * iq;
        R tau = R(0.5) + nu;
        R h = x + lg2<R>(tau) - ls;
        if (h > R(0)) hi = x; else lo = x;
        R dnudx = -dnu * m * q * (iq * iq);  // d nu / d log2(gdot) * ln 2 folded below
        R hp = R(1) + dnudx * rcp_of(tau);
        R xn = x - h * rcp_of(hp);
        // the closed bracket: a converged iterate (h = 0 sets lo = x, and
        // the step is zero) stays where it is
        x = (xn >= lo && xn <= hi) ? xn : R(0.5) * (lo + hi);
    }
    R q = lam > R(0) ? ex2<R>(m * (llam + x)) : R(0);
    R tau = R(0.5) + nuinf + dnu * rcp_of(R(1) + q);
    return fmin(fmax(tau, tmin), tmax);
}

}  // namespace lbk
