// lb_d2q9.h -- the paper's own lattice on the GPU: D2Q9 in the x-z plane of a
// box one cell deep in y (Sec. II.A: w = 4/9, 1/9, 1/36; the phi table
// alpha, (1-alpha)/5, (1-alpha)/20; B_i = -4/27, 2/27, 5/108; c_s^2 = 1/3).
//
// The step is four per-cell kernels (a 2-D box of the paper's size has a
// few hundred thousand cells, so no plane march is needed):
//   k2_pull     the step's geometry from the device step counter; every
//               cell pulls its 9 populations with the boundary rules of
//               Sec. II.B (halfway and moving-wall bounce-back with the
//               extrapolated wall density, the inlet lid, anti-bounce-back)
//               and reduces them to its moment set and colour fields; the
//               mass each rule adds and the mass of nodes the head covers
//               go to FP64 per-block sums
//   k2_create   nodes the head releases: f^eq(rho_bar, v_nozzle)
//   k2_wall     fictitious densities of the head's solid nodes (Eq. (wet))
//               and the colour fields of the rows beyond the z faces
//   k2_collide  colour gradient (Eq. (lattgrad)), the ink's relaxation time
//               from its strain rate, regularised BGK with exact-difference
//               forcing, perturbation and recolouring; stores the 18
//               post-collision values and the macro fields the next pull's
//               boundary rules read; advances the step counter
// Storage, moment and auxiliary layouts are those of the D3Q19 path with
// every y component zero (set 0 holds T_i = f^Y_i + f^B_i - w_i rho_ref, set
// 1 holds f^Y_i; nine planes each), so the read-out's output and reduction
// kernels serve both lattices.
#pragma once

#include "lb_device.h"
#include "lb_fused.h"

namespace lbk2 {

using namespace lbk;

constexpr int Q = 9;

// velocities (c_x, c_z): rest; +x, -x, +z, -z; (1, 1), (-1, -1), (1, -1),
// (-1, 1) -- opposite links adjacent, as in the D3Q19 table
__host__ __device__ constexpr int cx(int i)
{
    constexpr int v[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
    return v[i];
}
__host__ __device__ constexpr int cz(int i)
{
    constexpr int v[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
    return v[i];
}
__host__ __device__ constexpr int shell(int i) { return i == 0 ? 0 : (i <= 4 ? 1 : 2); }
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
__host__ __device__ constexpr double w_of_shell(int s) { return s == 0 ? 4.0 / 9.0 : (s == 1 ? 1.0 / 9.0 : 1.0 / 36.0); }
__host__ __device__ constexpr double w(int i) { return w_of_shell(shell(i)); }
__host__ __device__ constexpr double inv_len(int i) { return shell(i) == 1 ? 1.0 : 0.70710678118654752440; }

// The moment set of a pulled cell: FP64 masses, momentum and the second
// moments of the total and of the ink (xx, zz, xz).
template <typename R>
struct Mom2 {
    double dm[2];
    R j[2];
    R PT[3], PY[3];
};

template <typename R, int I>
__device__ __forceinline__ void mom2_add(Mom2<R> &M, R T, R Y)
{
    constexpr int X = cx(I), Z = cz(I);
    M.dm[0] += (double)T;
    M.dm[1] += (double)Y;
    if (X) M.j[0] += X > 0 ? T : -T;
    if (Z) M.j[1] += Z > 0 ? T : -T;
    if (X) M.PT[0] += T;
    if (Z) M.PT[1] += T;
    if (X && Z) M.PT[2] += X * Z > 0 ? T : -T;
    if (X) M.PY[0] += Y;
    if (Z) M.PY[1] += Y;
    if (X && Z) M.PY[2] += X * Z > 0 ? Y : -Y;
}

// site class of (x, z) with the head at (hx, hy); z is wrapped in place when
// periodic (the box's single y row is y = 0)
__device__ __forceinline__ int site2(const DevParams &P, double hx, double hy, int x, int &z)
{
    return classify(P, hx, hy, x, 0, z, P.has_nozzle != 0);
}

__device__ __forceinline__ long long c2(const DevParams &P, int x, int z) { return (long long)z * P.nx + x; }

// Link I of cell (x, z) whose source x - c_I is not fluid at t-1: the rule of
// that site applied to the cell's own post-collision population of the
// opposite link (Tout, Yout), Sec. II.B; the mass it adds per colour goes to
// the flux accumulators.
template <typename R, int I>
__device__ __forceinline__ void pull_rule2(const DevParams &P, const HeadPos &H, const R *__restrict__ mac, int x,
                                           int z, long long cell, int st, R Tout, R Yout, R &T, R &Yv, Flux &fl)
{
    constexpr int X = cx(I), Z = cz(I);
    const long long N = P.N;
    const R wi = R(w(I));
    if (st == ST_OPEN_LO || st == ST_OPEN_HI) {
        const bool lo = st == ST_OPEN_LO;
        const double rw0 = lo ? P.rho_lo[0] : P.rho_hi[0], rw1 = lo ? P.rho_lo[1] : P.rho_hi[1];
        // u_w = (3 u(x) - u(x + c_i)) / 2 at t-1 when x + c_i was fluid
        R ux = mac[2 * N + cell], uz = mac[4 * N + cell];
        const int x1 = X ? wrap(x + X, P.nx) : x;
        int z1 = z + Z;
        if (site2(P, H.hx_p, H.hy_p, x1, z1) == ST_FLUID) {
            const long long k1 = c2(P, x1, z1);
            ux = (R(3) * ux - mac[2 * N + k1]) * R(0.5);
            uz = (R(3) * uz - mac[4 * N + k1]) * R(0.5);
        }
        const R cu = R(X) * ux + R(Z) * uz;
        const R uu = ux * ux + uz * uz;
        const R E = wi * (cu * cu * R(4.5) - uu * R(1.5));
        const R phiY = R(P.phi[0][shell(I)]), phiB = R(P.phi[1][shell(I)]);
        const R rY = R(rw0), rB = R(rw1);
        Yv = -Yout + R(2) * rY * (phiY + E);
        T = -Tout - R(2) * wi * R(P.rho_ref) + R(2) * (rY * phiY + rB * phiB) + R(2) * (rY + rB) * E;
    } else {
        double U0, U2;
        R rwY, rwB;
        if (st == ST_LID) {
            U0 = P.u_in[0];
            U2 = P.u_in[2];
            rwY = R(P.lid_rho);
            rwB = R(0);
        } else {
            if (st == ST_NOZ) {
                U0 = P.vnoz[0];
                U2 = 0.0;
            } else {
                const bool lo = st == ST_WALL_LO;
                U0 = lo ? P.u_lo[0] : P.u_hi[0];
                U2 = lo ? P.u_lo[2] : P.u_hi[2];
            }
            rwY = R(0);
            rwB = R(0);
            if (U0 * X + U2 * Z != 0.0) {
                // rho_w by quadratic extrapolation to the link midpoint from
                // x, x + c_i, x + 2 c_i (inward), at t-1
                const R r0Y = mac[cell], r0B = mac[N + cell];
                const int x1 = X ? wrap(x + X, P.nx) : x;
                int z1 = z + Z;
                if (site2(P, H.hx_p, H.hy_p, x1, z1) == ST_FLUID) {
                    const long long k1 = c2(P, x1, z1);
                    const R r1Y = mac[k1], r1B = mac[N + k1];
                    const int x2 = X ? wrap(x1 + X, P.nx) : x1;
                    int z2 = z1 + Z;
                    if (site2(P, H.hx_p, H.hy_p, x2, z2) == ST_FLUID) {
                        const long long k2 = c2(P, x2, z2);
                        const R r2Y = mac[k2], r2B = mac[N + k2];
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
        const R k = R(6) * wi * R(U0 * X + U2 * Z);
        Yv = Yout + k * rwY;
        T = Tout + k * (rwY + rwB);
    }
    const bool open = st == ST_OPEN_LO || st == ST_OPEN_HI;
    const double dY = (double)(Yv - Yout), dB = (double)(T - Tout) - dY;
    fl.openY += open ? dY : 0.0;
    fl.openB += open ? dB : 0.0;
    fl.wallY += open ? 0.0 : dY;
    fl.wallB += open ? 0.0 : dB;
}

// The pull of one cell at step t (t = 0 on the first step: the stored state
// is then the initial equilibrium, read in place).
template <typename R>
__device__ __forceinline__ void pull2(const DevParams &P, const HeadPos &H, const R *__restrict__ src,
                                      const R *__restrict__ mac, int x, int z, long long cell, bool first,
                                      Mom2<R> &M, Flux &fl)
{
    const long long NP = P.NP;
    [&]<int... I>(std::integer_sequence<int, I...>) {
        (
            [&] {
                constexpr int X = cx(I), Z = cz(I);
                R T, Y;
                int st = ST_FLUID;
                long long sc = cell;
                if (!first) {
                    const int xs = X ? wrap(x - X, P.nx) : x;
                    int zs = z - Z;
                    st = site2(P, H.hx_p, H.hy_p, xs, zs);
                    sc = c2(P, xs, zs);
                }
                if (st == ST_FLUID) {
                    T = src[I * NP + sc];
                    Y = src[(Q + I) * NP + sc];
                } else {
                    pull_rule2<R, I>(P, H, mac, x, z, cell, st, src[opp(I) * NP + cell],
                                     src[(Q + opp(I)) * NP + cell], T, Y, fl);
                }
                mom2_add<R, I>(M, T, Y);
            }(),
            ...);
    }(std::make_integer_sequence<int, Q>{});
}

// Initial state: f^k = f^{k,eq}(rho^k, u) at the fluid cells of step 0.
template <typename R>
__global__ __launch_bounds__(256) void k2_init(DevParams P, const StepGeom *__restrict__ G,
                                               const double *__restrict__ rho_y, const double *__restrict__ rho_b,
                                               const double *__restrict__ u, int has_u, R *__restrict__ dst)
{
    const HeadPos H = G->H;
    const long long cell = (long long)blockIdx.x * 256 + threadIdx.x;
    if (cell >= P.N) return;
    const int z = (int)(cell / P.nx), x = (int)(cell - (long long)z * P.nx);
    const bool solid = is_solid(P, H.hx_c, H.hy_c, x, 0, z);
    const double rY = rho_y[cell], rB = rho_b[cell];
    const double ux = has_u ? u[3 * cell] : 0.0, uz = has_u ? u[3 * cell + 2] : 0.0;
    const double uu = ux * ux + uz * uz;
    for (int i = 0; i < Q; ++i) {
        double T = 0.0, fY = 0.0;
        if (!solid) {
            const int sh = shell(i);
            const double wi = w(i);
            const double cu = cx(i) * ux + cz(i) * uz;
            const double E = wi * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
            fY = rY * (P.phi[0][sh] + E);
            T = rY * P.phid[0][sh] + rB * P.phid[1][sh] + (rY + rB - P.rho_ref) * wi + (rY + rB) * E;
        }
        dst[i * P.NP + cell] = R(T);
        dst[(Q + i) * P.NP + cell] = R(fY);
    }
}

// moment set -> the D3Q19 path's auxiliary layout (y components zero)
template <typename R>
__device__ __forceinline__ void store_mom2(const DevParams &P, const Mom2<R> &M, double *__restrict__ momd,
                                           R *__restrict__ mom, long long cell)
{
    const long long N = P.N;
    momd[cell] = M.dm[0];
    momd[N + cell] = M.dm[1];
    const R m[NMOMR] = {M.j[0], R(0), M.j[1], M.PT[0], R(0), M.PT[1], R(0), M.PT[2], R(0),
                        M.PY[0], R(0), M.PY[1], R(0), M.PY[2], R(0)};
#pragma unroll
    for (int q = 0; q < NMOMR; ++q) mom[q * N + cell] = m[q];
}

// The pull of every cell at step t (grid-stride).  Step mode: the step's
// geometry is computed by every block from the device step counter and kept
// by block 0; boundary fluxes and deleted mass are added to the block's
// cumulative slot.  Read-out mode (readout != 0): the geometry is already in
// G; the block's slot is written (pending values, nothing committed).
template <typename R>
__global__ __launch_bounds__(256) void k2_pull(DevParams P, StepGeom *__restrict__ G, const R *__restrict__ src,
                                               const R *__restrict__ mac, double *__restrict__ momd,
                                               R *__restrict__ mom, R *__restrict__ chi,
                                               double *__restrict__ slots, int first, int readout)
{
    __shared__ StepGeom sg;
    if (threadIdx.x == 0) make_geom(P, G->t, G->first, sg);
    __syncthreads();
    if (!readout && blockIdx.x == 0 && threadIdx.x == 0) *G = sg;
    const HeadPos H = sg.H;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (long long cell = (long long)blockIdx.x * 256 + threadIdx.x; cell < P.N; cell += (long long)gridDim.x * 256) {
        const int z = (int)(cell / P.nx), x = (int)(cell - (long long)z * P.nx);
        if (is_solid(P, H.hx_p, H.hy_p, x, 0, z)) continue;  // no populations (created below if released)
        Mom2<R> M = {{0.0, 0.0}, {R(0), R(0)}, {R(0), R(0), R(0)}, {R(0), R(0), R(0)}};
        Flux fl = {0.0, 0.0, 0.0, 0.0};
        pull2<R>(P, H, src, mac, x, z, cell, first != 0, M, fl);
        if (!is_solid(P, H.hx_c, H.hy_c, x, 0, z)) {
            store_mom2<R>(P, M, momd, mom, cell);
            double cN, cY, cB;
            chi_of<double>(P, M.dm[1], P.rho_ref + M.dm[0] - M.dm[1], cN, cY, cB);
            chi[cell] = R(cN);
            chi[P.N + cell] = R(cY);
            chi[2 * P.N + cell] = R(cB);
        } else {  // covered by the head at t: deleted, its mass recorded
            acc[4] += M.dm[1];
            acc[5] += P.rho_ref + M.dm[0] - M.dm[1];
        }
        acc[0] += fl.wallY;
        acc[1] += fl.wallB;
        acc[2] += fl.openY;
        acc[3] += fl.openB;
    }
    block_sum<6>(acc, slots + (long long)blockIdx.x * 6, readout == 0);
}

// Nodes released by the head (solid at t-1, fluid at t): the moments of
// f^{k,eq}(rho_bar^k, v_nozzle), rho_bar^k the mean over the D2Q9 neighbours
// fluid at both steps (pure air rho_B^0 if there is none).
template <typename R>
__global__ __launch_bounds__(256) void k2_create(DevParams P, const StepGeom *__restrict__ G,
                                                 double *__restrict__ momd, R *__restrict__ mom, R *__restrict__ chi,
                                                 double *__restrict__ slots, int commit)
{
    const HeadPos H = G->H;
    const Box3 hb = G->hb;
    double acc[2] = {0.0, 0.0};
    const long long total = (long long)hb.w * hb.d;
    for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < total; k += (long long)gridDim.x * 256) {
        const int x = wrap_any(hb.x0 + (int)(k % hb.w), P.nx), z = hb.z0 + (int)(k / hb.w);
        if (z < 0 || z >= P.nz) continue;
        if (!is_solid(P, H.hx_p, H.hy_p, x, 0, z) || is_solid(P, H.hx_c, H.hy_c, x, 0, z)) continue;
        double sY = 0.0, sB = 0.0;
        int cnt = 0;
        for (int i = 1; i < Q; ++i) {
            int zz = z + cz(i);
            if (P.periodic_z) zz = wrap(zz, P.nz);
            if (zz < 0 || zz >= P.nz) continue;
            const int xx = wrap(x + cx(i), P.nx);
            if (is_solid(P, H.hx_p, H.hy_p, xx, 0, zz) || is_solid(P, H.hx_c, H.hy_c, xx, 0, zz)) continue;
            const long long nb = c2(P, xx, zz);
            const double rY = momd[P.N + nb];
            sY += rY;
            sB += P.rho_ref + momd[nb] - rY;
            ++cnt;
        }
        const double rY = cnt ? sY / cnt : 0.0, rB = cnt ? sB / cnt : P.rho0[1];
        const double vx = P.vnoz[0], rho = rY + rB, cs2 = 1.0 / 3.0;
        const double iso = rY * P.dcs2[0] + rB * P.dcs2[1] + (rho - P.rho_ref) * cs2;
        const double cY2 = cs2 + P.dcs2[0];
        Mom2<R> M;
        M.dm[0] = rho - P.rho_ref;
        M.dm[1] = rY;
        M.j[0] = R(rho * vx);
        M.j[1] = R(0);
        M.PT[0] = R(iso + rho * vx * vx);
        M.PT[1] = R(iso);
        M.PT[2] = R(0);
        M.PY[0] = R(rY * (cY2 + vx * vx));
        M.PY[1] = R(rY * cY2);
        M.PY[2] = R(0);
        const long long cell = c2(P, x, z);
        store_mom2<R>(P, M, momd, mom, cell);
        double cN, cYf, cBf;
        chi_of<double>(P, rY, rB, cN, cYf, cBf);
        chi[cell] = R(cN);
        chi[P.N + cell] = R(cYf);
        chi[2 * P.N + cell] = R(cBf);
        acc[0] += rY;
        acc[1] += rB;
    }
    block_sum<2>(acc, slots + (long long)blockIdx.x * 2, commit != 0);
}

// Colour fields the collision's stencil reads at non-fluid sites: the head's
// solid nodes (Eq. (wet) with the nozzle's affinity, from their D2Q9 fluid
// neighbours) and the rows z = -1 and z = nz (walls from the adjacent fluid
// row with the walls' affinity, pressure faces their imposed densities, the
// inlet lid pure ink, the shell above the top the nozzle's fictitious
// densities).  Threads 0 .. 2 nx - 1 of the grid take the rows, the rest the
// head box.
template <typename R>
__global__ __launch_bounds__(256) void k2_wall(DevParams P, const StepGeom *__restrict__ G,
                                               const double *__restrict__ momd, R *__restrict__ chi,
                                               R *__restrict__ ghost)
{
    const HeadPos H = G->H;
    const Box3 hb = G->hb;
    const long long rows = P.periodic_z ? 0 : 2LL * P.nx;
    const long long total = rows + (P.has_nozzle ? (long long)hb.w * hb.d : 0);
    for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < total; k += (long long)gridDim.x * 256) {
        int x, z;
        bool row = k < rows;
        if (row) {
            const int face = (int)(k / P.nx);
            x = (int)(k - (long long)face * P.nx);
            z = face == 0 ? -1 : P.nz;
        } else {
            const long long h = k - rows;
            x = wrap_any(hb.x0 + (int)(h % hb.w), P.nx);
            z = hb.z0 + (int)(h / hb.w);
            if (z < 0 || z >= P.nz || !is_solid(P, H.hx_c, H.hy_c, x, 0, z)) continue;
        }
        // the site's class at t (above the top, the head's columns override the face)
        int zc = z;
        const int st = row ? site2(P, H.hx_c, H.hy_c, x, zc) : ST_NOZ;
        double rY, rB;
        if (st == ST_LID) {
            rY = P.lid_rho;
            rB = 0.0;
        } else if (st == ST_OPEN_LO || st == ST_OPEN_HI) {
            const bool lo = st == ST_OPEN_LO;
            rY = lo ? P.rho_lo[0] : P.rho_hi[0];
            rB = lo ? P.rho_lo[1] : P.rho_hi[1];
        } else {
            const double zY = st == ST_NOZ ? P.zeta_noz[0] : P.zeta_wall[0];
            const double zB = st == ST_NOZ ? P.zeta_noz[1] : P.zeta_wall[1];
            double nY = 0.0, nB = 0.0, den = 0.0;
            for (int i = 1; i < Q; ++i) {
                const int xx = wrap(x + cx(i), P.nx);
                int zz = z + cz(i);
                if (site2(P, H.hx_c, H.hy_c, xx, zz) != ST_FLUID) continue;
                const long long nb = c2(P, xx, zz);
                const double wi = w(i), ry = momd[P.N + nb];
                nY += wi * ry;
                nB += wi * (P.rho_ref + momd[nb] - ry);
                den += wi;
            }
            rY = den > 0.0 ? zY * nY / den : 0.0;
            rB = den > 0.0 ? zB * nB / den : 0.0;
        }
        double cN, cY, cB;
        chi_of<double>(P, rY, rB, cN, cY, cB);
        if (row) {
            const int face = z < 0 ? 0 : 1;
            ghost[(face * 3 + 0) * P.nx + x] = R(cN);
            ghost[(face * 3 + 1) * P.nx + x] = R(cY);
            ghost[(face * 3 + 2) * P.nx + x] = R(cB);
        } else {
            const long long cell = c2(P, x, z);
            chi[cell] = R(cN);
            chi[P.N + cell] = R(cY);
            chi[2 * P.N + cell] = R(cB);
        }
    }
}

// Collision of every fluid cell from its moment set and the colour stencil;
// the compact form of the D3Q19 path in two dimensions:
//   f*_i - w_i rho_ref = w_i [k1 + a.c_i + c_i.Bm.c_i] (i > 0), t0 (i = 0),
// with Omega2's isotropic part (D - 1)/3 = 1/3 of p (B_i = w_i (|c_i|^2 -
// 1/3) on D2Q9), and f^Y_i = (rho_Y/rho)(w_i rho_ref + T_i) + w_i (c_i.r)/|c_i|.
template <typename R>
__global__ __launch_bounds__(256) void k2_collide(DevParams P, StepGeom *__restrict__ G,
                                                  const double *__restrict__ momd, const R *__restrict__ mom,
                                                  const R *__restrict__ chi, const R *__restrict__ ghost,
                                                  R *__restrict__ dst, R *__restrict__ mac_next)
{
    const HeadPos H = G->H;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        G->t += 1;
        G->first = 0;
    }
    const long long cell = (long long)blockIdx.x * 256 + threadIdx.x;
    if (cell >= P.N) return;
    const long long N = P.N;
    const int z = (int)(cell / P.nx), x = (int)(cell - (long long)z * P.nx);
    if (is_solid(P, H.hx_c, H.hy_c, x, 0, z)) {
        for (int i = 0; i < Q; ++i) {
            dst[i * P.NP + cell] = R(0);
            dst[(Q + i) * P.NP + cell] = R(0);
        }
        return;
    }
    // state: masses, momentum, non-equilibrium stresses, local tau
    const double drho_d = momd[cell], rY_d = momd[N + cell];
    const double rho_d = P.rho_ref + drho_d, rB_d = rho_d - rY_d;
    const R rY = R(rY_d), rB = R(rB_d), rho = R(rho_d);
    const R irho = rcp_of(rho);
    const R jx = mom[cell], jz = mom[2 * N + cell];
    const R ux = jx * irho, uz = jz * irho;
    const R iso = R(rY_d * P.dcs2[0] + rB_d * P.dcs2[1] + drho_d * (1.0 / 3.0));
    const R Pxx = mom[3 * N + cell] - iso - rho * ux * ux;
    const R Pzz = mom[5 * N + cell] - iso - rho * uz * uz;
    const R Pxz = mom[7 * N + cell] - rho * ux * uz;
    const R pY = R(rY_d * (1.0 / 3.0 + P.dcs2[0]));
    const R Yxx = mom[9 * N + cell] - pY - rY * ux * ux;
    const R Yzz = mom[11 * N + cell] - pY - rY * uz * uz;
    const R Yxz = mom[13 * N + cell] - rY * ux * uz;
    const R S = sqrt_of(Yxx * Yxx + Yzz * Yzz + R(2) * Yxz * Yxz);
    const R tauY = tau_ink<R>(P, S, rY);
    const R cs2 = R(1.0 / 3.0);
    const R nuY = cs2 * (tauY - R(0.5)), nuB = cs2 * (R(P.tau_b) - R(0.5));
    const R inv_nu = (rY * irho) * rcp_of(nuY) + (rB * irho) * rcp_of(nuB);
    const R tau = R(0.5) + R(3) * rcp_of(inv_nu);
    const R om = R(1) - rcp_of(tau);
    // colour gradients, Eq. (lattgrad): rho^N, rho_Y/rho, rho_B/rho
    R g[3][2] = {{R(0), R(0)}, {R(0), R(0)}, {R(0), R(0)}};
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const int xx = wrap(x + cx(i), P.nx);
        int zz = z + cz(i);
        if (P.periodic_z) zz = wrap(zz, P.nz);
        R c[3];
        if (zz < 0 || zz >= P.nz) {
            const int face = zz < 0 ? 0 : 1;
#pragma unroll
            for (int f = 0; f < 3; ++f) c[f] = ghost[(face * 3 + f) * P.nx + xx];
        } else {
            const long long nb = c2(P, xx, zz);
#pragma unroll
            for (int f = 0; f < 3; ++f) c[f] = chi[f * N + nb];
        }
        const R kk = R(3.0 * w(i));
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            if (cx(i)) g[f][0] += R(cx(i)) * kk * c[f];
            if (cz(i)) g[f][1] += R(cz(i)) * kk * c[f];
        }
    }
    // force: body force and the substrate drag (exact-difference method)
    R Fx = rho * R(P.g[0]), Fz = rho * R(P.g[2]);
    if (P.drag_gamma != 0.0 && P.face_lo == FACE_WALL && (double)z + 0.5 < P.drag_range) {
        const R gam = R(P.drag_gamma) * rY;
        Fx -= gam * (ux - R(P.u_lo[0]));
        Fz -= gam * (uz - R(P.u_lo[2]));
    }
    const R vx = ux + Fx * irho, vz = uz + Fz * irho;
    const double fracY_d = rY_d / rho_d;
    const R fracY = R(fracY_d), fracB = rB * irho;
    R Fcx = fracB * g[1][0] - fracY * g[2][0];
    R Fcz = fracB * g[1][1] - fracY * g[2][1];
    const R Fmax = fmax(fabs(Fcx), fabs(Fcz));
    const bool pert = Fmax > R(1e-30);
    const R iF = pert ? rcp_of(Fmax) : R(0);
    Fcx *= iF;
    Fcz *= iF;
    const R invFF = pert ? rcp_of(Fcx * Fcx + Fcz * Fcz) : R(0);
    const R gn2 = g[0][0] * g[0][0] + g[0][1] * g[0][1];
    const R pA = pert ? R(0.5) * R(P.A) * sqrt_of(gn2) : R(0);
    const R geps2 = gn2 + R(P.eps2);
    const R inv_geps = geps2 > R(0) ? rsqrt_of(geps2) : R(0);
    const R pn = pA * invFF;
    const R h = R(4.5);
    const R ax = R(3) * rho * vx, az = R(3) * rho * vz;
    const R bxx = h * (rho * vx * vx + om * Pxx) + pn * Fcx * Fcx - pA;
    const R bzz = h * (rho * vz * vz + om * Pzz) + pn * Fcz * Fcz - pA;
    const R bxz = R(2) * (h * (rho * vx * vz + om * Pxz) + pn * Fcx * Fcz);
    const R a0 = R(-1.5) * (rho * (vx * vx + vz * vz) + om * (Pxx + Pzz)) + R(1.0 / 3.0) * pA;
    const double k1_eq = drho_d + rY_d * (P.phid[0][1] / w(1)) + rB_d * (P.phid[1][1] / w(1));
    const double t0_eq = w(0) * drho_d + rY_d * P.phid[0][0] + rB_d * P.phid[1][0];
    const R k1 = a0 + R(k1_eq);
    const R t0 = R(w(0)) * a0 + R(t0_eq);
    const R e = rY * R(P.phi[0][1] / w(1)) + rB * R(P.phi[1][1] / w(1));
    const R rec = R(P.beta) * fracY * fracB * inv_geps * e;
    const R rx = rec * g[0][0], rz = rec * g[0][1];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int X = cx(i), Z = cz(i);
        R Tst, cgw;
        if (i == 0) {
            Tst = t0;
            cgw = R(0);
        } else {
            const R q = k1 + R(X) * ax + R(Z) * az + R(X * X) * bxx + R(Z * Z) * bzz + R(X * Z) * bxz;
            Tst = R(w(i)) * q;
            cgw = R(w(i) * inv_len(i)) * (R(X) * rx + R(Z) * rz);
        }
        const R Yst = R(__builtin_fma(fracY_d, w(i) * P.rho_ref + (double)Tst, (double)cgw));
        dst[i * P.NP + cell] = Tst;
        dst[(Q + i) * P.NP + cell] = Yst;
    }
    mac_next[cell] = rY;
    mac_next[N + cell] = rB;
    mac_next[2 * N + cell] = ux;
    mac_next[3 * N + cell] = R(0);
    mac_next[4 * N + cell] = uz;
}

}  // namespace lbk2
