// lbprint.hip -- gfx950 kernels and the C ABI (include/lbprint.h) of the
// colour-gradient lattice Boltzmann printing step (arXiv:2102.02655).
//
// One time step t-1 -> t on the caller's stream:
//   k_pre      the step's geometry (head position, boundary boxes) from the
//              device step counter; pulls the cells whose links touch a
//              boundary with the rules of Sec. II.B (z faces, the head's
//              box), their moments and colour fields; deleted nodes' mass
//              and boundary fluxes into FP64 per-block sums
//   k_create   nodes released by the moving head: f^eq(rho_bar, v_nozzle)
//   k_wall     the head's fictitious wall densities, Eq. (wet)
//   k_ghost    colour fields of the ghost layers beyond the z faces
//   k_fused_pc every other cell (lb_fused.h): pull, moments, colour stencil
//              (Eq. (lattgrad)), rheology, regularised collision,
//              perturbation, recolouring, store; advances the step counter
// The stored state between steps is the post-collision population pair.
// Read-out (k_moments, k_create, k_output, k_reduce) pulls the whole box
// without committing anything.  Batched stepping runs the same kernel bodies
// for many simulations per launch (kb_*, over a device slot table).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>
#include <mutex>
#include <algorithm>
#include <cstddef>
#include <limits>
#include <memory>

#include "../../include/lbprint.h"
#include "lb_collide.h"
#include "lb_device.h"
#include "lb_fused.h"

using namespace lbk;

namespace {

constexpr int TPB = 256;       // threads per block of the per-cell kernels
constexpr int NB_SPARSE = 256;  // fixed grid of the head-box kernels (deterministic slots)
constexpr int NB_PRE = 2048;    // most blocks of the boundary preparation kernel (slots of its sums)
constexpr int NSLOT = 6;       // per-block FP64 sums: wall Y, wall B, open Y, open B, deleted Y, deleted B
constexpr int NPART = 6;       // per-block FP64 sums of the output: mass Y, B, momentum xyz, unstable

// ------------------------------------------------------------ reductions

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Deterministic block sum of NV doubles (fixed shuffle and wave order);
// thread 0 adds (accumulate) or writes the result to slot[0..NV).
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *slot, bool accumulate)
{
    __shared__ double red[NV][TPB / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double s = wave_sum(v[q]);
        if (lane == 0) red[q][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double s = 0.0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[q][w];
            slot[q] = accumulate ? slot[q] + s : s;
        }
    }
}

__device__ __forceinline__ void cell_xyz(const DevParams &P, long long cell, int &x, int &y, int &z)
{
    long long plane = (long long)P.nx * P.ny;
    z = (int)(cell / plane);
    long long r = cell - (long long)z * plane;
    y = (int)(r / P.nx);
    x = (int)(r - (long long)y * P.nx);
}

// colour fields at slot `cell` of arrays with component stride `st`
template <typename R>
__device__ __forceinline__ void write_chi(const DevParams &P, R *chi, long long cell, long long st, double rY,
                                          double rB)
{
    double cN, cY, cB;
    chi_of<double>(P, rY, rB, cN, cY, cB);
    as_global(chi)[cell] = R(cN);
    as_global(chi)[st + cell] = R(cY);
    as_global(chi)[2 * st + cell] = R(cB);
}

// densities of a fluid cell from its FP64 masses (slot c, component stride st)
__device__ __forceinline__ void dens(const DevParams &P, const double *__restrict__ momd, long long c, long long st,
                                    double &rY, double &rB)
{
    rY = as_global(momd)[st + c];
    rB = P.rho_ref + as_global(momd)[c] - rY;
}

// ------------------------------------------------------------------ kernels

// Initial state: f^k = f^{k,eq}(rho^k, u) at the fluid cells of step 0.
// Reduced storage: zero deviations and the cell's moments (the decoded
// populations are then the equilibrium).
template <typename R, int ST>
__global__ __launch_bounds__(TPB) void k_init(DevParams P, const StepGeom *__restrict__ G,
                                              const double *__restrict__ rho_y, const double *__restrict__ rho_b,
                                              const double *__restrict__ u, int has_u, void *__restrict__ dst_v,
                                              float *__restrict__ mo)
{
    const HeadPos H = G->H;
    long long cell = (long long)blockIdx.x * TPB + threadIdx.x;
    if (cell >= P.N) return;
    int x, y, z;
    cell_xyz(P, cell, x, y, z);
    bool solid = !far_from_head(P, H.hx_c, H.hy_c, x, y) && is_solid(P, H.hx_c, H.hy_c, x, y, z);
    double rY = rho_y[cell], rB = rho_b[cell];
    double ux = has_u ? u[3 * cell] : 0.0, uy = has_u ? u[3 * cell + 1] : 0.0, uz = has_u ? u[3 * cell + 2] : 0.0;
    if constexpr (ST != ST_PLAIN) {
        unsigned *d = reinterpret_cast<unsigned *>(dst_v);
        for (int i = 0; i < lbq::Q; ++i) d[i * P.NP + cell] = 0;
        const double m[NMO] = {rY, rB, ux, uy, uz};
        for (int k = 0; k < NMO; ++k) mo[k * P.NM + cell] = solid ? 0.f : float(m[k]);
        return;
    }
    R *dT = reinterpret_cast<R *>(dst_v), *dY = dT + (long long)lbq::Q * P.NP;
    double uu = ux * ux + uy * uy + uz * uz;
    for (int i = 0; i < lbq::Q; ++i) {
        if (solid) {
            dT[i * P.NP + cell] = R(0);
            dY[i * P.NP + cell] = R(0);
            continue;
        }
        int sh = lbq::shell(i);
        double wi = lbq::w(i);
        double cu = lbq::cx(i) * ux + lbq::cy(i) * uy + lbq::cz(i) * uz;
        double E = wi * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
        double fY = rY * (P.phi[0][sh] + E);
        double T = rY * P.phid[0][sh] + rB * P.phid[1][sh] + (rY + rB - P.rho_ref) * wi + (rY + rB) * E;
        dT[i * P.NP + cell] = R(T);
        dY[i * P.NP + cell] = R(fY);
    }
}

// Pull + moments of one cell at step t: moment set, colour fields, and into
// acc the boundary fluxes of its pull (when fluxes) and, for a node the head
// covers at t, its deleted mass.
// RO (read-out): masses and momentum into full-box arrays at the cell's
// index; else (boundary preparation) the whole moment set and the colour
// fields into the boundary-only arrays at the cell's slot.
template <typename R, bool RO, typename PS>
__device__ __forceinline__ void moments_cell(const DevParams &P, const HeadPos &H, const PS &src,
                                             const R *__restrict__ mac, double *__restrict__ momd,
                                             R *__restrict__ mom, R *__restrict__ chi, long long cell, int x, int y,
                                             int z, bool first, bool fluxes, double (&acc)[NSLOT], int &any)
{
    bool near = !far_from_head(P, H.hx_p, H.hy_p, x, y) || !far_from_head(P, H.hx_c, H.hy_c, x, y);
    bool sp = near && is_solid(P, H.hx_p, H.hy_p, x, y, z);
    bool sc = near && is_solid(P, H.hx_c, H.hy_c, x, y, z);
    if (sp) return;
    Mom<R> M;
    mom_zero(M);
    Flux fl = {0.0, 0.0, 0.0, 0.0};
    pull_all<R, true>(P, H, src, mac, x, y, z, cell, near, first, M, fl);
    if (!sc) {
        if constexpr (RO) {
            as_global(momd)[cell] = M.dm[0];
            as_global(momd)[P.N + cell] = M.dm[1];
#pragma unroll
            for (int q = 2; q < 5; ++q) as_global(mom)[(q - 2) * P.N + cell] = M.m[q];
        } else {
            const long long a = aidx(P, x, y, z), NA = P.NA;
            as_global(momd)[a] = M.dm[0];
            as_global(momd)[NA + a] = M.dm[1];
#pragma unroll
            for (int q = 2; q < NMOM; ++q) as_global(mom)[(q - 2) * NA + a] = M.m[q];
            write_chi<R>(P, chi, a, NA, M.dm[1], P.rho_ref + M.dm[0] - M.dm[1]);
        }
    } else {
        acc[4] += M.dm[1];
        acc[5] += P.rho_ref + M.dm[0] - M.dm[1];
        any = 1;
    }
    if (fluxes) {
        acc[0] += fl.wallY;
        acc[1] += fl.wallB;
        acc[2] += fl.openY;
        acc[3] += fl.openB;
        any |= (fl.wallY != 0.0) | (fl.wallB != 0.0) | (fl.openY != 0.0) | (fl.openB != 0.0);
    }
}

// Whole-box pull + moments (read-out path): writes this step's pending
// boundary fluxes and deleted mass per block, touching no cumulative state.
template <typename R, int ST>
__global__ __launch_bounds__(TPB) void k_moments(DevParams P, const StepGeom *__restrict__ G,
                                                 PopSrc<R, ST> src, const R *__restrict__ mac,
                                                 double *__restrict__ momd, R *__restrict__ mom, R *__restrict__ chi,
                                                 double *__restrict__ slots, int first)
{
    const HeadPos H = G->H;
    double acc[NSLOT] = {0, 0, 0, 0, 0, 0};
    int any = 0;
    // grid-stride: with one block per 256 cells each thread takes one cell
    for (long long cell = (long long)blockIdx.x * TPB + threadIdx.x; cell < P.N;
         cell += (long long)gridDim.x * TPB) {
        int x, y, z;
        cell_xyz(P, cell, x, y, z);
        moments_cell<R, true>(P, H, src, mac, momd, mom, chi, cell, x, y, z, first != 0, true, acc, any);
    }
    block_sum<NSLOT>(acc, slots + (long long)blockIdx.x * NSLOT, false);
}

// Boundary preparation of a time step: the cells whose pull touches a
// boundary (the z faces' layers, the head's box) are pulled here with the
// boundary rules of Sec. II.B; their moment sets and colour fields feed the
// fused kernel, the wall densities and the created nodes.  The mass each
// boundary rule adds and the mass of nodes the head covers are added to the
// block's cumulative slot.  Boxes 1 and 2 skip cells of box 0 (the head box)
// so that no cell is counted twice.
// (body for block bid of nblk; the standalone kernel below and the batched
// kernel call it)
template <typename R, int ST>
__device__ __forceinline__ void pre_body(const DevParams &P, StepGeom *__restrict__ G, const PopSrc<R, ST> &src,
                                         const R *__restrict__ mac, double *__restrict__ momd, R *__restrict__ mom,
                                         R *__restrict__ chi, double *__restrict__ slots, int first, int bid, int nblk)
{
    // the step's geometry from the device step counter (every block), kept
    // in memory by block 0 for the step's later kernels
    __shared__ StepGeom sg;
    if (threadIdx.x == 0) make_geom(P, G->t, G->first, sg);
    __syncthreads();
    if (bid == 0 && threadIdx.x == 0) *G = sg;
    const HeadPos H = sg.H;
    const Box3 b0 = sg.bx[0], b1 = sg.bx[1], b2 = sg.bx[2];
    const int nbox = sg.nbox;
    double acc[NSLOT] = {0, 0, 0, 0, 0, 0};
    int any = 0;
    for (int bi = 0; bi < nbox; ++bi) {
        const Box3 B = bi == 0 ? b0 : (bi == 1 ? b1 : b2);
        const long long total = (long long)B.w * B.h * B.d;
        for (long long k = (long long)bid * TPB + threadIdx.x; k < total; k += (long long)nblk * TPB) {
            int ix = (int)(k % B.w), iy = (int)((k / B.w) % B.h), iz = (int)(k / ((long long)B.w * B.h));
            int x = ((B.x0 + ix) % P.nx + P.nx) % P.nx, y = ((B.y0 + iy) % P.ny + P.ny) % P.ny, z = B.z0 + iz;
            if (z < 0 || z >= P.nz) continue;
            if (bi > 0 && in_box(P, b0, x, y, z)) continue;
            moments_cell<R, false>(P, H, src, mac, momd, mom, chi, cidx(P, x, y, z), x, y, z, first != 0, true, acc,
                                   any);
        }
    }
    if (!__syncthreads_or(any)) return;
    block_sum<NSLOT>(acc, slots + (long long)bid * NSLOT, true);
}

template <typename R, int ST>
__global__ __launch_bounds__(TPB) void k_pre(DevParams P, StepGeom *__restrict__ G, PopSrc<R, ST> src,
                                             const R *__restrict__ mac, double *__restrict__ momd,
                                             R *__restrict__ mom, R *__restrict__ chi, double *__restrict__ slots,
                                             int first)
{
    pre_body<R, ST>(P, G, src, mac, momd, mom, chi, slots, first, blockIdx.x, gridDim.x);
}

// Sec. II.B: nodes released by the head (solid at t-1, fluid at t) start at
// f^{k,eq}(rho_bar^k, v_nozzle), rho_bar^k the mean over the lattice
// neighbours fluid at both steps (pure air rho_B^0 if there is none).  Only
// the moment set and the colour fields are needed downstream.
template <typename R>
__device__ __forceinline__ void create_body(const DevParams &P, const StepGeom *__restrict__ G,
                                            double *__restrict__ momd, R *__restrict__ mom, R *__restrict__ chi,
                                            double *__restrict__ slots, int commit, int bid, int nblk)
{
    const HeadPos H = G->H;
    const int bx0 = G->hb.x0, by0 = G->hb.y0, bz0 = G->hb.z0, bw = G->hb.w, bh = G->hb.h, bd = G->hb.d;
    // the read-out (commit = 0) keeps full-box arrays of masses and momentum;
    // the step the boundary-only arrays
    const bool ro = commit == 0;
    const long long st = ro ? P.N : P.NA;
    double acc[2] = {0.0, 0.0};
    const long long total = (long long)bw * bh * bd;
    for (long long k = (long long)bid * TPB + threadIdx.x; k < total; k += (long long)nblk * TPB) {
        int ix = (int)(k % bw), iy = (int)((k / bw) % bh), iz = (int)(k / ((long long)bw * bh));
        int x = ((bx0 + ix) % P.nx + P.nx) % P.nx, y = ((by0 + iy) % P.ny + P.ny) % P.ny, z = bz0 + iz;
        if (z < 0 || z >= P.nz) continue;
        if (!is_solid(P, H.hx_p, H.hy_p, x, y, z) || is_solid(P, H.hx_c, H.hy_c, x, y, z)) continue;
        // the neighbours fluid at both steps, all classified before any read
        // (the reads are in flight together); others add an exact zero
        long long nc[lbq::Q];
        bool use[lbq::Q];
#pragma unroll
        for (int i = 1; i < lbq::Q; ++i) {
            int zz = z + lbq::cz(i);
            if (P.periodic_z) zz = wrap(zz, P.nz);
            const bool in = zz >= 0 && zz < P.nz;
            int xx = wrap(x + lbq::cx(i), P.nx), yy = wrap(y + lbq::cy(i), P.ny);
            use[i] = in && !is_solid(P, H.hx_p, H.hy_p, xx, yy, zz) && !is_solid(P, H.hx_c, H.hy_c, xx, yy, zz);
            nc[i] = use[i] ? (ro ? cidx(P, xx, yy, zz) : aidx(P, xx, yy, zz)) : (ro ? cidx(P, x, y, z) : aidx(P, x, y, z));
        }
        double nd[lbq::Q][2];
#pragma unroll
        for (int i = 1; i < lbq::Q; ++i) dens(P, momd, nc[i], st, nd[i][0], nd[i][1]);
        double sY = 0.0, sB = 0.0;
        int cnt = 0;
#pragma unroll
        for (int i = 1; i < lbq::Q; ++i) {
            sY += use[i] ? nd[i][0] : 0.0;
            sB += use[i] ? nd[i][1] : 0.0;
            cnt += use[i] ? 1 : 0;
        }
        double rY = cnt ? sY / cnt : 0.0, rB = cnt ? sB / cnt : P.rho0[1];
        const long long cell = ro ? cidx(P, x, y, z) : aidx(P, x, y, z);
        // moments of f^eq(rho_bar, v): drho, rho_Y, j = rho v, second moments
        double vx = P.vnoz[0], vy = P.vnoz[1];
        double rho = rY + rB;
        double cs2 = 1.0 / 3.0;
        double iso = rY * P.dcs2[0] + rB * P.dcs2[1] + (rho - P.rho_ref) * cs2;
        double cY2 = cs2 + P.dcs2[0];
        double m[NMOM] = {rho - P.rho_ref, rY, rho * vx, rho * vy, 0.0,
                          iso + rho * vx * vx, iso + rho * vy * vy, iso, rho * vx * vy, 0.0, 0.0,
                          rY * (cY2 + vx * vx), rY * (cY2 + vy * vy), rY * cY2, rY * vx * vy, 0.0, 0.0};
        as_global(momd)[cell] = m[0];
        as_global(momd)[st + cell] = m[1];
        for (int q = 2; q < (ro ? 5 : NMOM); ++q) as_global(mom)[(q - 2) * st + cell] = R(m[q]);
        if (!ro) write_chi<R>(P, chi, cell, st, rY, rB);
        acc[0] += rY;
        acc[1] += rB;
    }
    block_sum<2>(acc, slots + (long long)bid * 2, commit != 0);
}

template <typename R>
__global__ __launch_bounds__(TPB) void k_create(DevParams P, const StepGeom *__restrict__ G,
                                                double *__restrict__ momd, R *__restrict__ mom, R *__restrict__ chi,
                                                double *__restrict__ slots, int commit)
{
    create_body<R>(P, G, momd, mom, chi, slots, commit, blockIdx.x, gridDim.x);
}

// Fictitious densities of the head's solid cells that touch fluid, Eq. (wet):
// rho_s^k = zeta^k sum_i w_i s_i rho^k(x + c_i) / sum_i w_i s_i.
template <typename R>
__device__ __forceinline__ void wall_body(const DevParams &P, const StepGeom *__restrict__ G,
                                          const double *__restrict__ momd, R *__restrict__ chi, int bid, int nblk)
{
    const HeadPos H = G->H;
    const int bx0 = G->hb.x0, by0 = G->hb.y0, bz0 = G->hb.z0, bw = G->hb.w, bh = G->hb.h, bd = G->hb.d;
    const long long total = (long long)bw * bh * bd;
    for (long long k = (long long)bid * TPB + threadIdx.x; k < total; k += (long long)nblk * TPB) {
        int ix = (int)(k % bw), iy = (int)((k / bw) % bh), iz = (int)(k / ((long long)bw * bh));
        int x = ((bx0 + ix) % P.nx + P.nx) % P.nx, y = ((by0 + iy) % P.ny + P.ny) % P.ny, z = bz0 + iz;
        if (z < 0 || z >= P.nz) continue;
        if (!is_solid(P, H.hx_c, H.hy_c, x, y, z)) continue;
        // the fluid neighbours, all classified before any read (the reads
        // are in flight together); others add an exact zero
        long long nc[lbq::Q];
        bool use[lbq::Q];
#pragma unroll
        for (int i = 1; i < lbq::Q; ++i) {
            int zz = z + lbq::cz(i);
            if (P.periodic_z) zz = wrap(zz, P.nz);
            const bool in = zz >= 0 && zz < P.nz;
            int xx = wrap(x + lbq::cx(i), P.nx), yy = wrap(y + lbq::cy(i), P.ny);
            use[i] = in && !is_solid(P, H.hx_c, H.hy_c, xx, yy, zz);
            nc[i] = use[i] ? aidx(P, xx, yy, zz) : aidx(P, x, y, z);
        }
        double nd[lbq::Q][2];
#pragma unroll
        for (int i = 1; i < lbq::Q; ++i) dens(P, momd, nc[i], P.NA, nd[i][0], nd[i][1]);
        double nY = 0.0, nB = 0.0, den = 0.0;
#pragma unroll
        for (int i = 1; i < lbq::Q; ++i) {
            const double wi = lbq::w(i);
            nY += use[i] ? wi * nd[i][0] : 0.0;
            nB += use[i] ? wi * nd[i][1] : 0.0;
            den += use[i] ? wi : 0.0;
        }
        const long long cell = aidx(P, x, y, z);
        double sY = den > 0.0 ? P.zeta_noz[0] * nY / den : 0.0;
        double sB = den > 0.0 ? P.zeta_noz[1] * nB / den : 0.0;
        write_chi<R>(P, chi, cell, P.NA, sY, sB);
    }
}

template <typename R>
__global__ __launch_bounds__(TPB) void k_wall(DevParams P, const StepGeom *__restrict__ G,
                                              const double *__restrict__ momd, R *__restrict__ chi)
{
    wall_body<R>(P, G, momd, chi, blockIdx.x, gridDim.x);
}

// Colour fields of the ghost layers below (face 0) and above (face 1) the
// box: walls carry Eq. (wet)'s fictitious densities from the adjacent fluid
// layer, pressure faces their imposed densities, the inlet lid pure ink, the
// head's shell columns above the top the nozzle's fictitious densities.
template <typename R>
__device__ __forceinline__ void ghost_body(const DevParams &P, const StepGeom *__restrict__ G,
                                           const double *__restrict__ momd, R *__restrict__ ghost, int bid)
{
    const HeadPos H = G->H;
    long long plane = (long long)P.nx * P.ny;
    long long k = (long long)bid * TPB + threadIdx.x;
    if (k >= 2 * plane) return;
    int face = (int)(k / plane);
    long long c = k - face * plane;
    int y = (int)(c / P.nx), x = (int)(c - (long long)y * P.nx);
    int zg = face == 0 ? -1 : P.nz;
    int zin = face == 0 ? 0 : P.nz - 1;
    double rY, rB;
    int kind;  // 0 = wall-like (zeta), 1 = fixed
    double z0 = P.zeta_wall[0], z1 = P.zeta_wall[1];
    if (face == 1 && P.has_nozzle && column_class(P, H.hx_c, H.hy_c, x, y) != COL_OUT) {
        if (column_class(P, H.hx_c, H.hy_c, x, y) == COL_BORE) {
            kind = 1;
            rY = P.lid_rho;
            rB = 0.0;
        } else {
            kind = 0;
            z0 = P.zeta_noz[0];
            z1 = P.zeta_noz[1];
        }
    } else {
        int f = face == 0 ? P.face_lo : P.face_hi;
        if (f == FACE_WALL) {
            kind = 0;
        } else {
            kind = 1;
            rY = face == 0 ? P.rho_lo[0] : P.rho_hi[0];
            rB = face == 0 ? P.rho_lo[1] : P.rho_hi[1];
        }
    }
    if (kind == 0) {
        double nY = 0.0, nB = 0.0, den = 0.0;
        for (int i = 1; i < lbq::Q; ++i) {
            if (zg + lbq::cz(i) != zin) continue;
            int xx = wrap(x + lbq::cx(i), P.nx), yy = wrap(y + lbq::cy(i), P.ny);
            if (is_solid(P, H.hx_c, H.hy_c, xx, yy, zin)) continue;
            double wi = lbq::w(i);
            double nrY, nrB;
            dens(P, momd, aidx(P, xx, yy, zin), P.NA, nrY, nrB);
            nY += wi * nrY;
            nB += wi * nrB;
            den += wi;
        }
        rY = den > 0.0 ? z0 * nY / den : 0.0;
        rB = den > 0.0 ? z1 * nB / den : 0.0;
    }
    double cN, cY, cB;
    chi_of<double>(P, rY, rB, cN, cY, cB);
    as_global(ghost)[(face * 3 + 0) * plane + c] = R(cN);
    as_global(ghost)[(face * 3 + 1) * plane + c] = R(cY);
    as_global(ghost)[(face * 3 + 2) * plane + c] = R(cB);
}

template <typename R>
__global__ __launch_bounds__(TPB) void k_ghost(DevParams P, const StepGeom *__restrict__ G,
                                               const double *__restrict__ momd, R *__restrict__ ghost)
{
    ghost_body<R>(P, G, momd, ghost, blockIdx.x);
}

// Fields for lb_moments: rho_Y, rho_B, physical velocity (j + F/2)/rho; block
// sums of mass and momentum; instability flag.
template <typename R, typename O>
__global__ __launch_bounds__(TPB) void k_output(DevParams P, const StepGeom *__restrict__ G,
                                                const double *__restrict__ momd, const R *__restrict__ mom,
                                                O *__restrict__ ory, O *__restrict__ orb, O *__restrict__ ou,
                                                double *__restrict__ part)
{
    const HeadPos H = G->H;
    double acc[NPART] = {0, 0, 0, 0, 0, 0};
    // grid-stride: with one block per 256 cells each thread takes one cell
    for (long long cell = (long long)blockIdx.x * TPB + threadIdx.x; cell < P.N;
         cell += (long long)gridDim.x * TPB) {
        int x, y, z;
        cell_xyz(P, cell, x, y, z);
        bool solid = !far_from_head(P, H.hx_c, H.hy_c, x, y) && is_solid(P, H.hx_c, H.hy_c, x, y, z);
        double rY = 0.0, rB = 0.0, U[3] = {0.0, 0.0, 0.0};
        if (!solid) {
            dens(P, momd, cell, P.N, rY, rB);
            double r = rY + rB;
            double j[3] = {(double)mom[cell], (double)mom[P.N + cell], (double)mom[2 * P.N + cell]};
            double F[3];
            for (int a = 0; a < 3; ++a) F[a] = r * P.g[a];
            if (P.drag_gamma != 0.0 && P.face_lo == FACE_WALL && (double)z + 0.5 < P.drag_range)
                for (int a = 0; a < 3; ++a) F[a] -= P.drag_gamma * rY * (j[a] / r - P.u_lo[a]);
            for (int a = 0; a < 3; ++a) U[a] = (j[a] + 0.5 * F[a]) / r;
            acc[0] += rY;
            acc[1] += rB;
            acc[2] += j[0];
            acc[3] += j[1];
            acc[4] += j[2];
            double uu = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
            bool bad = !(r > 0.0) || !(uu <= 0.09) || rY != rY || rB != rB;
            acc[5] = bad ? 1.0 : acc[5];
        }
        if (ory) ory[cell] = O(rY);
        if (orb) orb[cell] = O(rB);
        if (ou) {
            ou[3 * cell] = O(U[0]);
            ou[3 * cell + 1] = O(U[1]);
            ou[3 * cell + 2] = O(U[2]);
        }
    }
    block_sum<NPART>(acc, part + (long long)blockIdx.x * NPART, false);
}

// ------------------------------------------------------------ observables
// Printing observables of one x-z section (Sec. IV): thread cells (ink below
// z_hi in the window of columns), their highest z and column span, the
// largest pressure deviation of the section's ink and the ink cells touching
// the substrate.  Per-block values, then one block; every operation is a sum
// of integers or a maximum, so the result does not depend on the grid.
constexpr int NOBS = 6;  // count, max z, max(-s), max s, max (p - p0), substrate count

__device__ __forceinline__ double obs_op(int q, double a, double b)
{
    return (q == 0 || q == 5) ? a + b : fmax(a, b);
}

__device__ __forceinline__ void block_obs(double (&v)[NOBS], double *slot)
{
    __shared__ double red[NOBS][TPB / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NOBS; ++q) {
        double a = v[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) a = obs_op(q, a, __shfl_xor(a, o, 64));
        if (lane == 0) red[q][wid] = a;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int q = 0; q < NOBS; ++q) {
            double a = red[q][0];
            for (int w = 1; w < (int)(blockDim.x >> 6); ++w) a = obs_op(q, a, red[q][w]);
            slot[q] = a;
        }
}

__device__ __forceinline__ void obs_init(double (&v)[NOBS])
{
    v[0] = 0.0;
    v[1] = -1.0;
    v[2] = v[3] = v[4] = -1e300;
    v[5] = 0.0;
}

__global__ __launch_bounds__(TPB) void k_observe(DevParams P, const StepGeom *__restrict__ G,
                                                 const double *__restrict__ momd, int x_lo, int x_len, int z_hi,
                                                 int ysec, double *__restrict__ part)
{
    const HeadPos H = G->H;
    const double cY2 = P.dcs2[0] + 1.0 / 3.0, cB2 = P.dcs2[1] + 1.0 / 3.0;
    const double p0 = P.rho0[1] * cB2;
    double v[NOBS];
    obs_init(v);
    const long long area = (long long)P.nx * P.nz;
    for (long long k = (long long)blockIdx.x * TPB + threadIdx.x; k < area; k += (long long)gridDim.x * TPB) {
        const int z = (int)(k / P.nx), x = (int)(k - (long long)z * P.nx);
        if (is_solid(P, H.hx_c, H.hy_c, x, ysec, z)) continue;
        double rY, rB;
        dens(P, momd, cidx(P, x, ysec, z), P.N, rY, rB);
        if (!(rY * P.rho0[1] > rB * P.rho0[0])) continue;  // rho^N > 0
        v[4] = fmax(v[4], rY * cY2 + rB * cB2 - p0);
        v[5] += z == 0 ? 1.0 : 0.0;
        int s = x - x_lo;
        if (s < 0) s += P.nx;
        if (s < x_len && z < z_hi) {
            v[0] += 1.0;
            v[1] = fmax(v[1], (double)z);
            v[2] = fmax(v[2], -(double)s);
            v[3] = fmax(v[3], (double)s);
        }
    }
    block_obs(v, part + (long long)blockIdx.x * NOBS);
}

__global__ __launch_bounds__(TPB) void k_observe_final(const double *__restrict__ part, int nb,
                                                       double *__restrict__ out)
{
    double v[NOBS];
    obs_init(v);
    for (int b = threadIdx.x; b < nb; b += TPB)
        for (int q = 0; q < NOBS; ++q) v[q] = obs_op(q, v[q], part[(long long)b * NOBS + q]);
    block_obs(v, out);
}

// Deterministic final sums for lb_moments (one block):
// out = mass[2], mom[3], wall[2], open[2], created[2], deleted[2], unstable.
// Committed boundary fluxes live in the fused kernel's block slots, committed
// deleted / created mass in the boundary kernels' slots; pend / pendc hold
// the read-out's not-yet-committed values of the current step.
// The step's geometry from the device step counter (one thread).
__global__ void k_clock(DevParams P, StepGeom *__restrict__ G)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        StepGeom g;
        make_geom(P, G->t, G->first, g);
        *G = g;
    }
}

__global__ __launch_bounds__(TPB) void k_reduce(const double *__restrict__ part, const double *__restrict__ pend,
                                                long long nbm, const double *__restrict__ cumpre, int nbp,
                                                const double *__restrict__ cumc, const double *__restrict__ pendc,
                                                int nbs, int nbsp, double *__restrict__ out)
{
    double v[14] = {0};
    for (long long b = threadIdx.x; b < nbm; b += TPB) {
        const double *p = part + b * NPART;
        for (int q = 0; q < 5; ++q) v[q] += p[q];
        v[13] = fmax(v[13], p[5]);
        const double *d = pend + b * NSLOT;
        v[5] += d[0];
        v[6] += d[1];
        v[7] += d[2];
        v[8] += d[3];
        v[11] += d[4];
        v[12] += d[5];
    }
    for (int b = threadIdx.x; b < nbp; b += TPB) {
        const double *c = cumpre + (long long)b * NSLOT;
        v[5] += c[0];
        v[6] += c[1];
        v[7] += c[2];
        v[8] += c[3];
        v[11] += c[4];
        v[12] += c[5];
    }
    for (int b = threadIdx.x; b < nbs; b += TPB) {
        v[9] += cumc[2 * b] + (b < nbsp ? pendc[2 * b] : 0.0);
        v[10] += cumc[2 * b + 1] + (b < nbsp ? pendc[2 * b + 1] : 0.0);
    }
    __shared__ double red[14][TPB];
    for (int q = 0; q < 14; ++q) red[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int st = TPB / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int q = 0; q < 14; ++q)
                red[q][threadIdx.x] = q == 13 ? fmax(red[q][threadIdx.x], red[q][threadIdx.x + st])
                                              : red[q][threadIdx.x] + red[q][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 14; ++q) out[q] = red[q][0];
}

}  // namespace

// the D2Q9 kernels (they use the block sums above)
#include "lb_d2q9.h"

// ====================================================================== host

namespace {

thread_local std::string g_err;

constexpr size_t ALIGN = 256;
size_t al(size_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

struct Layout {
    size_t pops, dmo, momd, mom, chi, ghost, mac, pend, part, cumpre, cumc, pendc, red, geo, tab, total;
    long long NA;    // slots of the boundary-only arrays (momd, mom, chi, mac)
    size_t ro;       // read-out arrays (masses, momentum) inside the spare population buffer
    long long nbm;   // blocks of the whole-box read-out kernels
    FusedGrid fg;    // tiling of the fused step kernel
    long long nbf;   // its block count
    int ty;          // its tile height
    unsigned nb_wall;  // blocks of the wall-density kernel (grid-stride over the head box)
    unsigned nb_pre;   // blocks of the boundary preparation kernel (its largest cell count, at most NB_PRE)
    unsigned nb_create;  // blocks of the node-creation kernel (the head box, at most NB_SPARSE)
};

size_t real_size(int storage) { return storage == LB_F64 ? 8 : 4; }                    // arithmetic type
size_t pop_size(int storage) { return storage == LB_F64 ? 8 : (storage == LB_F32 ? 4 : 2); }  // stored population
bool reduced(int storage) { return storage == LB_BF16_DEV || storage == LB_F16_DEV; }

// Population planes: 2 x 19 of one value per cell, or 19 words packing both
// colours (reduced forms).  A plane whose byte size is a multiple of a large
// power of two would put the same cell of all planes -- the 38 streams one
// wave reads or writes together -- on the same memory channels; planes of
// 16 MiB and more are therefore spaced by one MiB and 256 B of padding
// (measured: about 4% less time per step on the 512 x 256 x 128 print bed).
// The reduced forms' five source-moment planes are spaced the same way.
long long plane_stride(long long N, int storage)
{
    const long long esz = reduced(storage) ? 4 : (long long)pop_size(storage);
    const long long b = N * esz;
    const long long pad = b >= (16LL << 20) ? (1LL << 20) + 256 : 256;
    return (b + pad) / esz;
}
bool is_d2(const lb_params &p) { return p.lattice == 9; }
int lattice_q(const lb_params &p) { return is_d2(p) ? lbk2::Q : lbq::Q; }
size_t pop_set_bytes(long long N, int storage, int q)
{
    const size_t esz = reduced(storage) ? 4 : pop_size(storage);
    const size_t planes = reduced(storage) ? q : 2 * q;
    return planes * (size_t)plane_stride(N, storage) * esz;
}

// Fused kernel tile height per storage type (TY + 3 waves).  LDS: colour ring
// 4 x 3 x 66 (TY + 2) values, state ring 2 x 64 TY x (2 FP64 + 10 values).
constexpr int TY_F32 = 4;
constexpr int TY_F64 = 5;
// the producer/consumer step kernel: tile height and tile rows per collider
// wave, per storage form (FP32 plain; reduced storage, whose moment ring
// needs LDS)
constexpr int PC_TY_PLAIN = 4, PC_CR_PLAIN = 1;
constexpr int PC_TY_DEV = 4, PC_CR_DEV = 1;

// ------------------------------------------------------ batched stepping
//
// One launch per kernel of a step advances every member of a batch: the
// device slot table holds each member's parameters, buffers (for both step
// parities of the batch) and the range of blocks it owns in each kernel's
// grid.  A block finds its member by binary search over the members' block
// offsets and runs the member's kernel body with its block index within the
// member's share, which is the grid the member would use alone; members with
// fewer steps to go than the launch's step index leave at once.
constexpr int BATCH_MAX = 64;
enum { BK_PRE = 0, BK_CREATE, BK_WALL, BK_GHOST, BK_FUSED, BK_N };

struct BatchSlot {
    DevParams P;
    FusedGrid fg;
    StepGeom *G;
    const void *src[2];       // population copy read at batch steps of parity q (q = j & 1)
    void *dst[2];
    const void *mac_prev[2];  // macro fields written by the previous step
    void *mac_next[2];
    const float *mo_src[2];   // source moments (reduced storage forms)
    float *mo_dst[2];
    double *momd;
    void *mom, *chi, *ghost;
    double *cumpre, *cumc;
    int nsteps;               // batch steps this member takes (launch j runs iff j < nsteps)
    unsigned nb[BK_N];        // the member's blocks in each kernel
    unsigned off[BK_N];       // its first block in each kernel's grid
};

struct BatchTable {
    int n;
    unsigned total[BK_N];
    BatchSlot slot[BATCH_MAX];
};

// The member owning block b of kernel `kind`, or -1 (blocks past the total,
// or in the padding that aligns a member's first block).  Offsets are
// non-decreasing in member order; a member without blocks in a kernel
// shares its offset with the next member.
__device__ __forceinline__ int batch_member(const BatchTable *__restrict__ T, int kind, unsigned b)
{
    if (b >= T->total[kind]) return -1;
    int lo = 0, hi = T->n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (T->slot[mid].off[kind] <= b) lo = mid;
        else hi = mid;
    }
    const BatchSlot &S = T->slot[lo];
    return (b >= S.off[kind] && b - S.off[kind] < S.nb[kind]) ? lo : -1;
}

template <typename R, int ST>
__device__ __forceinline__ PopSrc<R, ST> batch_src(const BatchSlot &S, int q)
{
    PopSrc<R, ST> s;
    if constexpr (ST == ST_PLAIN) {
        s.s = static_cast<const R *>(S.src[q]);
    } else {
        s.s = static_cast<const unsigned *>(S.src[q]);
        s.mo = static_cast<const float *>(S.mo_src[q]);
        s.NM = S.P.NM;
    }
    s.N = S.P.N;
    s.NP = S.P.NP;
    return s;
}

template <typename R, int ST>
__global__ __launch_bounds__(TPB) void kb_pre(const BatchTable *__restrict__ T, int j)
{
    const int m = batch_member(T, BK_PRE, blockIdx.x);
    if (m < 0) return;
    const BatchSlot &S = T->slot[m];
    if (j >= S.nsteps) return;
    const int q = j & 1;
    const DevParams &P = S.P;  // fields read from the table on demand (scalar loads)
    pre_body<R, ST>(P, S.G, batch_src<R, ST>(S, q), static_cast<const R *>(S.mac_prev[q]), S.momd,
                    static_cast<R *>(S.mom), static_cast<R *>(S.chi), S.cumpre, 0, blockIdx.x - S.off[BK_PRE], S.nb[BK_PRE]);
}

template <typename R>
__global__ __launch_bounds__(TPB) void kb_create(const BatchTable *__restrict__ T, int j)
{
    const int m = batch_member(T, BK_CREATE, blockIdx.x);
    if (m < 0) return;
    const BatchSlot &S = T->slot[m];
    if (j >= S.nsteps) return;
    const DevParams &P = S.P;  // fields read from the table on demand (scalar loads)
    create_body<R>(P, S.G, S.momd, static_cast<R *>(S.mom), static_cast<R *>(S.chi), S.cumc, 1,
                   blockIdx.x - S.off[BK_CREATE], S.nb[BK_CREATE]);
}

template <typename R>
__global__ __launch_bounds__(TPB) void kb_wall(const BatchTable *__restrict__ T, int j)
{
    const int m = batch_member(T, BK_WALL, blockIdx.x);
    if (m < 0) return;
    const BatchSlot &S = T->slot[m];
    if (j >= S.nsteps) return;
    const DevParams &P = S.P;  // fields read from the table on demand (scalar loads)
    wall_body<R>(P, S.G, S.momd, static_cast<R *>(S.chi), blockIdx.x - S.off[BK_WALL], S.nb[BK_WALL]);
}

template <typename R>
__global__ __launch_bounds__(TPB) void kb_ghost(const BatchTable *__restrict__ T, int j)
{
    const int m = batch_member(T, BK_GHOST, blockIdx.x);
    if (m < 0) return;
    const BatchSlot &S = T->slot[m];
    if (j >= S.nsteps) return;
    const DevParams &P = S.P;  // fields read from the table on demand (scalar loads)
    ghost_body<R>(P, S.G, S.momd, static_cast<R *>(S.ghost), blockIdx.x - S.off[BK_GHOST]);
}

template <typename R, int TY, int ST, int CR>
__global__ __launch_bounds__((TY + 3 + TY / CR) * 64, 1) void kb_fused_pc(const BatchTable *__restrict__ T, int j)
{
    const int m = batch_member(T, BK_FUSED, blockIdx.x);
    if (m < 0) return;
    const BatchSlot &S = T->slot[m];
    if (j >= S.nsteps) return;
    const int q = j & 1;
    // the member's parameters as a local copy (loaded once, like kernel
    // arguments), not a reference into the table
    const DevParams P = S.P;
    const FusedGrid fg = S.fg;
    fused_pc_body<R, TY, false, ST, CR>(P, S.G, fg, static_cast<const char *>(S.src[q]), static_cast<char *>(S.dst[q]),
                                        S.momd, static_cast<const R *>(S.mom), static_cast<const R *>(S.chi),
                                        static_cast<const R *>(S.ghost), static_cast<R *>(S.mac_next[q]), S.mo_src[q],
                                        S.mo_dst[q], blockIdx.x - S.off[BK_FUSED], S.nb[BK_FUSED]);
}

template <int TY>
__global__ __launch_bounds__((TY + 3) * 64, 2) void kb_fused64(const BatchTable *__restrict__ T, int j)
{
    const int m = batch_member(T, BK_FUSED, blockIdx.x);
    if (m < 0) return;
    const BatchSlot &S = T->slot[m];
    if (j >= S.nsteps) return;
    const int q = j & 1;
    const DevParams P = S.P;
    const FusedGrid fg = S.fg;
    fused_body<double, TY, false>(P, S.G, fg, static_cast<const double *>(S.src[q]), static_cast<double *>(S.dst[q]),
                                  S.momd, static_cast<const double *>(S.mom), static_cast<const double *>(S.chi),
                                  static_cast<const double *>(S.ghost), static_cast<double *>(S.mac_next[q]),
                                  blockIdx.x - S.off[BK_FUSED], S.nb[BK_FUSED]);
}

// Tiling of the step kernel: full-width 64 x ty tiles, the height split into
// z chunks so that the launch has about `want` blocks.  The result of a cell
// does not depend on the chunking (every chunk re-pulls its halo planes
// identically), so a batch may chunk a member differently from a lone run.
FusedGrid fused_grid(const lb_params &p, int ty, long long want_blocks = 512)
{
    FusedGrid g;
    g.ntx = (p.nx + 63) / 64;
    g.nty = (p.ny + ty - 1) / ty;
    long long tiles = (long long)g.ntx * g.nty;
    // one resident block per CU: about two rounds of blocks on 256 CUs, z
    // chunks of at least 8 planes (long chunks spend fewer halo planes)
    long long want = (want_blocks + tiles - 1) / tiles;
    long long maxc = std::max(1, p.nz / 8);
    g.nzc = (int)std::max(1LL, std::min(want, maxc));
    if (const char *e = std::getenv("LBPRINT_ZLEN")) {
        int z = std::atoi(e);
        if (z > 0) g.nzc = (p.nz + z - 1) / z;
    }
    g.zlen = (p.nz + g.nzc - 1) / g.nzc;
    g.nzc = (p.nz + g.zlen - 1) / g.zlen;
    return g;
}

// Boundary-only arrays (moment sets and colour fields of the prepared cells,
// macro fields for the next step's boundary rules).  Only the cells next to
// the z faces and around the head use them, so a D3Q19 box with walls keeps
// them compact (DevParams::aux): three layers at each z face (the prepared
// face planes and the two planes whose macro fields the face rules
// extrapolate from), and the head region from four planes below the tip up,
// its columns taken modulo a window.  A step touches the head box (r_out + 2
// around the axis at the step's two positions, rounded out), one more cell
// for neighbour reads, two for the extrapolation, and the macro fields
// within r_out + 4 of the axis for the next step, which reads them around
// the next position: at most 2 ceil(r_out) + 12 consecutive columns over two
// steps of a head moving at most half a cell per step.  The window is the
// smallest power of two dividing the box's extent that is at least
// 2 ceil(r_out) + 16 (the extent itself if there is none), so that columns
// sharing a slot are a whole number of windows apart also across the
// periodic boundary, and a column's place in it is a mask.  Periodic boxes,
// faster heads and boxes the compact form would not shrink keep one slot per
// cell.
int window_of(int extent, int need)
{
    for (int d = 1; d < extent; d *= 2)
        if (d >= need && extent % d == 0) return d;
    return extent;
}

struct AuxPlan {
    int aux, az_lo, az_hi, ah_z0, aw, ah;
    long long NA, a_head0;
};

AuxPlan aux_plan(const lb_params &p)
{
    AuxPlan a;
    std::memset(&a, 0, sizeof(a));
    const long long N = (long long)p.nx * p.ny * p.nz, pl = (long long)p.nx * p.ny;
    a.NA = N;
    const int az = 3;
    if (is_d2(p) || p.face_zlo == LB_FACE_PERIODIC || p.nz <= 2 * az + 1) return a;
    long long head = 0;
    int z0 = p.nz - az, aw = 0, ah = 0;
    if (p.has_nozzle) {
        if (std::fabs(p.noz_v[0]) > 0.5 || std::fabs(p.noz_v[1]) > 0.5) return a;
        const int win = 2 * (int)std::ceil(p.noz_r_in + p.noz_wall) + 16;
        aw = window_of(p.nx, win);
        ah = window_of(p.ny, win);
        z0 = std::max(az, (int)std::floor(p.noz_tip_z) - 4);
        z0 = std::min(z0, p.nz - az);
        head = (long long)(p.nz - az - z0) * aw * ah;
    }
    const long long NA = 2LL * az * pl + head + 1;  // + the sink slot
    if (NA >= N) return a;
    a.aux = 1;
    a.az_lo = a.az_hi = az;
    a.ah_z0 = z0;
    a.aw = aw;
    a.ah = ah;
    a.NA = NA;
    a.a_head0 = 2LL * az * pl;
    return a;
}

Layout layout_of(const lb_params &p)
{
    Layout L;
    long long N = (long long)p.nx * p.ny * p.nz;
    size_t rs = real_size(p.storage);
    L.nbm = (N + TPB - 1) / TPB;
    L.ty = p.storage == LB_F64 ? TY_F64 : (reduced(p.storage) ? PC_TY_DEV : PC_TY_PLAIN);
    L.fg = fused_grid(p, L.ty);
    {
        // the head box spans at most 2 (r_out + 2) + 4 columns each way
        long long wmax = p.has_nozzle ? 2 * (long long)std::ceil(p.noz_r_in + p.noz_wall + 2.0) + 4 : 0;
        long long bw = std::min<long long>(wmax, p.nx), bh = std::min<long long>(wmax, p.ny);
        long long tot = bw * bh * p.nz;
        L.nb_wall = (unsigned)std::max<long long>(1, std::min<long long>((tot + TPB - 1) / TPB, 4096));
        // sized to the work, so that the preparation of a small box leaves
        // the GPU to other simulations' kernels
        const long long faces = p.face_zlo == LB_FACE_PERIODIC ? 0 : 2LL * p.nx * p.ny;
        L.nb_pre = (unsigned)std::max<long long>(1, std::min<long long>((tot + faces + TPB - 1) / TPB, NB_PRE));
        L.nb_create = (unsigned)std::max<long long>(1, std::min<long long>((tot + TPB - 1) / TPB, NB_SPARSE));
        if (is_d2(p)) {
            // D2Q9: the pull is one grid-stride kernel over the box whose
            // blocks keep the step's sums (at most NB_PRE slots); the wall
            // kernel takes the two ghost rows and the head box
            const long long area = bw * p.nz;
            L.nb_pre = (unsigned)std::max<long long>(1, std::min<long long>(L.nbm, NB_PRE));
            L.nb_create = (unsigned)std::max<long long>(1, std::min<long long>((area + TPB - 1) / TPB, NB_SPARSE));
            L.nb_wall = (unsigned)std::max<long long>(1, std::min<long long>((area + 2LL * p.nx + TPB - 1) / TPB, 4096));
        }
    }
    L.nbf = (long long)L.fg.ntx * L.fg.nty * L.fg.nzc;
    size_t off = 0;
    L.pops = off;
    off += 2 * al(pop_set_bytes(N, p.storage, lattice_q(p)));
    L.dmo = off;  // source moments of the reduced storage forms (two copies)
    if (reduced(p.storage)) off += 2 * al(NMO * (size_t)plane_stride(N, LB_F32) * 4);
    const long long NA = aux_plan(p).NA;
    L.NA = NA;
    L.momd = off;
    off += al(2 * (size_t)NA * 8);
    L.mom = off;
    off += al(NMOMR * (size_t)NA * rs);
    L.chi = off;
    off += al(NCHI * (size_t)NA * rs);
    L.ghost = off;
    off += al(2 * NCHI * (size_t)p.nx * p.ny * rs);
    L.mac = off;
    off += 2 * al(NMAC * (size_t)NA * rs);
    // the read-out's masses (FP64) and momentum, after the largest staged
    // output (five FP64 fields) in the spare population buffer; D2Q9's
    // read-out writes the boundary-only arrays, which are full-box there
    L.ro = al(5 * (size_t)N * 8);
    L.pend = off;
    off += al((size_t)L.nbm * NSLOT * 8);
    L.part = off;
    off += al((size_t)L.nbm * NPART * 8);
    L.cumpre = off;
    off += al((size_t)NB_PRE * NSLOT * 8);
    L.cumc = off;
    off += al(NB_SPARSE * 2 * 8);
    L.pendc = off;
    off += al(NB_SPARSE * 2 * 8);
    L.red = off;
    off += al(16 * 8);
    L.geo = off;
    off += al(sizeof(StepGeom));
    L.tab = off;  // the handle's one-member slot table (its steps after the first)
    off += al(offsetof(BatchTable, slot) + sizeof(BatchSlot));
    L.total = off;
    return L;
}

const char *validate(const lb_params &p)
{
    if (p.nx < 1 || p.ny < 1 || p.nz < 1) return "box dimensions must be positive";
    if ((long long)p.nx * p.ny * p.nz > (1LL << 34)) return "box too large";
    if ((long long)p.nx * p.ny * p.nz * (long long)real_size(p.storage) >= (1LL << 32))
        return "box too large: one population plane must stay below 4 GiB";
    if (p.storage < LB_F64 || p.storage > LB_F16_DEV) return "unknown storage form";
    if (!(p.tau_b > 0.5)) return "tau_b must exceed 1/2";
    if (p.rheology < 0 || p.rheology > 2) return "unknown rheology";
    if (p.rheology == LB_NEWTONIAN && !(p.tau_y > 0.5)) return "tau_y must exceed 1/2";
    if (p.rheology != LB_NEWTONIAN && !(p.tau_min > 0.5 && p.tau_max >= p.tau_min)) return "need 1/2 < tau_min <= tau_max";
    if (p.rheology == LB_POWER_LAW && !(p.K > 0.0 && p.n > 0.0 && p.n <= 1.0)) return "power law needs K > 0, 0 < n <= 1";
    if (p.rheology == LB_CROSS && !(p.nu0 > 0.0 && p.nu_inf > 0.0 && p.lambda >= 0.0 && p.m > 0.0 && p.m < 1.0))
        return "Cross law needs nu0, nu_inf > 0, lambda >= 0, 0 < m < 1";
    if (!(p.rho0[0] > 0.0 && p.rho0[1] > 0.0)) return "rho0 must be positive";
    if (p.face_zlo < 0 || p.face_zlo > 2 || p.face_zhi < 0 || p.face_zhi > 2) return "unknown face type";
    if ((p.face_zlo == LB_FACE_PERIODIC) != (p.face_zhi == LB_FACE_PERIODIC)) return "z faces must be both periodic or neither";
    if (p.has_nozzle) {
        if (p.face_zhi == LB_FACE_PERIODIC) return "a nozzle needs a non-periodic top face";
        if (!(p.noz_tip_z >= 0.0 && p.noz_tip_z <= p.nz - 1)) return "nozzle tip outside the box";
        if (!(p.noz_r_in > 0.0 && p.noz_wall > 0.0)) return "nozzle radii must be positive";
        if (!(std::fabs(p.noz_v[0]) < 1.0 && std::fabs(p.noz_v[1]) < 1.0)) return "head speed must be below one cell per step";
    }
    if (p.eps_g < 0.0 || p.rho_eps <= 0.0) return "eps_g >= 0 and rho_eps > 0 required";
    if (p.lattice != 0 && p.lattice != 9 && p.lattice != 19) return "lattice must be 0 or 19 (D3Q19) or 9 (D2Q9)";
    if (is_d2(p)) {
        if (p.ny != 1) return "D2Q9 lives in the x-z plane: ny must be 1";
        if (p.storage != LB_F64 && p.storage != LB_F32) return "D2Q9 runs with LB_F64 or LB_F32 storage";
        if (p.body_g[1] != 0.0 || p.u_zlo[1] != 0.0 || p.u_zhi[1] != 0.0)
            return "D2Q9: y components of the body force and wall velocities must be 0";
        if (p.has_nozzle && (p.u_ink[1] != 0.0 || p.noz_v[1] != 0.0 || p.noz_x0[1] != 0.0))
            return "D2Q9: the head moves in x only, centred on y = 0";
    }
    return nullptr;
}

DevParams make_dev(const lb_params &p)
{
#pragma clang fp contract(off)
    DevParams P;
    std::memset(&P, 0, sizeof(P));
    P.nx = p.nx;
    P.ny = p.ny;
    P.nz = p.nz;
    P.N = (long long)p.nx * p.ny * p.nz;
    P.NP = plane_stride(P.N, p.storage);
    P.NM = plane_stride(P.N, LB_F32);
    P.periodic_z = p.face_zlo == LB_FACE_PERIODIC;
    P.face_lo = p.face_zlo;
    P.face_hi = p.face_zhi;
    P.rho_ref = p.rho0[1];
    P.rho0[0] = p.rho0[0];
    P.rho0[1] = p.rho0[1];
    const bool d2 = is_d2(p);
    const double cs2 = 1.0 / 3.0, w0 = d2 ? lbk2::w_of_shell(0) : lbq::w_of_shell(0);
    for (int k = 0; k < 2; ++k) {
        double a = p.alpha[k];
        for (int s = 0; s < 3; ++s) {
            double ws = d2 ? lbk2::w_of_shell(s) : lbq::w_of_shell(s);
            P.phi[k][s] = s == 0 ? a : (1.0 - a) * ws / (1.0 - w0);
            P.phid[k][s] = P.phi[k][s] - ws;
        }
        P.dcs2[k] = (1.0 - a) * cs2 / (1.0 - w0) - cs2;
    }
    {
        // coefficients of the reduced forms' equilibrium (D3Q19 weights)
        const double v0 = lbq::w_of_shell(0), v1 = lbq::w_of_shell(1);
        double g[2];
        for (int k = 0; k < 2; ++k) g[k] = (p.alpha[k] - v0 * (1.0 - p.alpha[k]) / (1.0 - v0)) / v1;
        P.eqf[0] = float((1.0 - p.alpha[0]) * v1 / (1.0 - v0));
        P.eqf[1] = float((1.0 - p.alpha[1]) * v1 / (1.0 - v0));
        P.eqf[2] = float(v1 * P.rho_ref);
        P.eqf[3] = float(g[0]);
        P.eqf[4] = float(g[0] - g[1]);
        P.eqf[5] = float(g[1]);
    }
    P.A = p.A;
    P.beta = p.beta;
    P.eps2 = p.eps_g * p.eps_g;
    P.tau_b = p.tau_b;
    P.rheology = p.rheology;
    P.tau_y = p.tau_y;
    P.tau_min = p.tau_min;
    P.tau_max = p.tau_max;
    P.rho_eps = p.rho_eps;
    if (p.rheology == LB_POWER_LAW) {
        P.Kp = p.K / cs2;
        P.n = p.n;
        if (p.n == 1.0) {  // Newtonian in disguise
            P.rheology = RHEO_NEWTON;
            double t = 0.5 + P.Kp;
            P.tau_y = t < p.tau_min ? p.tau_min : (t > p.tau_max ? p.tau_max : t);
        } else {
            double g1 = std::pow((p.tau_max - 0.5) / P.Kp, 1.0 / (p.n - 1.0));
            double g2 = std::pow((p.tau_min - 0.5) / P.Kp, 1.0 / (p.n - 1.0));
            P.s_lo = g1 * p.tau_max;
            P.s_hi = g2 * p.tau_min;
            P.lg_lo = std::log2(g1);
            P.lg_hi = std::log2(g2);
        }
    } else if (p.rheology == LB_CROSS) {
        P.nu0p = p.nu0 / cs2;
        P.nuinfp = p.nu_inf / cs2;
        P.lambda = p.lambda;
        P.m = p.m;
    }
    for (int k = 0; k < 2; ++k) {
        P.zeta_wall[k] = p.zeta_wall[k];
        P.zeta_noz[k] = p.zeta_noz[k];
        P.rho_lo[k] = p.rho_zlo[k];
        P.rho_hi[k] = p.rho_zhi[k];
    }
    P.drag_gamma = p.drag_gamma;
    P.drag_range = p.drag_range;
    for (int a = 0; a < 3; ++a) {
        P.g[a] = p.body_g[a];
        P.u_lo[a] = p.u_zlo[a];
        P.u_hi[a] = p.u_zhi[a];
    }
    P.has_nozzle = p.has_nozzle;
    if (p.has_nozzle) {
        P.ri2 = p.noz_r_in * p.noz_r_in;
        double ro = p.noz_r_in + p.noz_wall;
        P.ro2 = ro * ro;
        P.rout = ro;
        P.tip_z = p.noz_tip_z;
        P.vnoz[0] = p.noz_v[0];
        P.vnoz[1] = p.noz_v[1];
        P.x0noz[0] = p.noz_x0[0];
        P.x0noz[1] = p.noz_x0[1];
        P.u_in[0] = p.u_ink[0] + p.noz_v[0];
        P.u_in[1] = p.u_ink[1] + p.noz_v[1];
        P.u_in[2] = p.u_ink[2];
        P.lid_rho = p.lid_rho_y;
    }
    const AuxPlan a = aux_plan(p);
    P.aux = a.aux;
    P.az_lo = a.az_lo;
    P.az_hi = a.az_hi;
    P.ah_z0 = a.ah_z0;
    P.aw = a.aw;
    P.ah = a.ah;
    P.amx = a.aw == p.nx ? -1 : a.aw - 1;
    P.amy = a.ah == p.ny ? -1 : a.ah - 1;
    P.NA = a.NA;
    P.a_head0 = a.a_head0;
    return P;
}

}  // namespace

struct lb_handle {
    lb_params p;
    DevParams P;
    Layout L;
    hipStream_t stream;
    char *ws;
    int cur;
    long t;
    int first;
    int unstable;
    std::string err;
    // lb_moments_noalloc: this device's copy of the static scratch array
    // (null with scratch_err set if its address could not be taken)
    double *scratch = nullptr;
    std::string scratch_err;
    // kernel timing (lb_timing): three events per timed step
    int timing = 0;
    std::vector<hipEvent_t> ev;
    size_t nev = 0;
    double acc_step = 0.0, acc_prep = 0.0;
    long acc_n = 0;
    // batched stepping (lb_step_batch): instantiated k-step chains of this
    // handle, keyed by (k, population buffer, step parity), captured on a
    // private stream
    struct Chain {
        int k, cur, parity;
        hipGraphExec_t exec;
    };
    std::vector<Chain> chains;
    hipStream_t cap = nullptr;
    // batched stepping (lb_batch_step): orders the batch stream after this
    // handle's stream
    hipEvent_t bev = nullptr;
    // blocks of each step kernel over the handle's own slot table
    unsigned lone_nb[BK_N] = {0, 0, 0, 0, 0};
    ~lb_handle()
    {
        if (bev) (void)hipEventDestroy(bev);
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        for (Chain &c : chains) (void)hipGraphExecDestroy(c.exec);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

namespace {

lb_status fail(lb_handle *h, lb_status s, const std::string &msg)
{
    if (h) h->err = msg;
    g_err = msg;
    return s;
}

lb_status check_launch(lb_handle *h, const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(h, LB_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    return LB_OK;
}

template <typename R>
R *as(lb_handle *h, size_t off)
{
    return reinterpret_cast<R *>(h->ws + off);
}

// population copy `which` (0 / 1) and, for the reduced storage forms, the
// source moments stored with it
char *pops_at(lb_handle *h, int which)
{
    return h->ws + h->L.pops + which * al(pop_set_bytes(h->P.N, h->p.storage, lattice_q(h->p)));
}

// The read-out's full-box masses (2N doubles) and momentum (3N values) at
// cell indices: in the spare population buffer after the staged outputs
// (D3Q19; its size, 2 x 19 values or 19 words per cell, exceeds the 68 bytes
// per cell this takes at most), or the boundary-only arrays themselves
// (D2Q9, full-box there).
double *ro_momd(lb_handle *h)
{
    if (is_d2(h->p)) return as<double>(h, h->L.momd);
    return reinterpret_cast<double *>(pops_at(h, 1 - h->cur) + h->L.ro);
}

template <typename R>
R *ro_mom(lb_handle *h)
{
    if (is_d2(h->p)) return as<R>(h, h->L.mom);
    return reinterpret_cast<R *>(pops_at(h, 1 - h->cur) + h->L.ro + al(2 * (size_t)h->P.N * 8));
}

float *mo_at(lb_handle *h, int which)
{
    if (!reduced(h->p.storage)) return nullptr;
    return as<float>(h, h->L.dmo + which * al(NMO * (size_t)h->P.NM * 4));
}

template <typename R, int ST>
PopSrc<R, ST> pop_src(lb_handle *h, int which)
{
    PopSrc<R, ST> s;
    if constexpr (ST == ST_PLAIN) {
        s.s = reinterpret_cast<const R *>(pops_at(h, which));
    } else {
        s.s = reinterpret_cast<const unsigned *>(pops_at(h, which));
        s.mo = mo_at(h, which);
        s.NM = h->P.NM;
    }
    s.N = h->P.N;
    s.NP = h->P.NP;
    return s;
}

StepGeom *geo(lb_handle *h) { return as<StepGeom>(h, h->L.geo); }

// The step's geometry from the device step counter.
lb_status launch_clock(lb_handle *h)
{
    hipLaunchKernelGGL(k_clock, dim3(1), dim3(64), 0, h->stream, h->P, geo(h));
    return check_launch(h, "k_clock");
}

// macro buffer written at step t is t & 1; the pull of step t reads (t - 1) & 1
template <typename R>
R *mac_at(lb_handle *h, long t)
{
    return as<R>(h, h->L.mac + (t & 1) * al(NMAC * (size_t)h->P.NA * sizeof(R)));
}

// Where one read-out keeps its per-call partial sums: the pending boundary
// fluxes and deletions of the pull (nb blocks x NSLOT), the fields' sums
// (nb blocks x NPART), the pending created mass (NB_SPARSE x 2) and the 14
// final values.  lb_moments uses slots in the handle's workspace and one
// block per 256 cells; lb_moments_noalloc the library's static device array
// and a fixed grid.
struct ReadSlots {
    double *pend, *part, *pendc, *red;
    unsigned nb;          // blocks of the whole-box read-out kernels
    bool zero_pendc;      // clear pendc when no creation is pending (else count no slot)
};

// Read-out pull: moments of the whole box at the current step, pending
// fluxes / deletions / creations (nothing committed).  Returns the number of
// pending-creation slots written (k_reduce reads that many).
template <typename R, int ST>
lb_status run_readout(lb_handle *h, const ReadSlots &S, int &nbsp)
{
    const Layout &L = h->L;
    const bool d2 = is_d2(h->p);
    if (lb_status s = launch_clock(h)) return s;
    if (d2)
        hipLaunchKernelGGL(lbk2::k2_pull<R>, dim3(S.nb), dim3(TPB), 0, h->stream, h->P, geo(h),
                           reinterpret_cast<const R *>(pops_at(h, h->cur)), mac_at<R>(h, h->t - 1),
                           as<double>(h, L.momd), as<R>(h, L.mom), as<R>(h, L.chi), S.pend, h->first, 1);
    else
        hipLaunchKernelGGL((k_moments<R, ST>), dim3(S.nb), dim3(TPB), 0, h->stream, h->P, geo(h),
                           pop_src<R, ST>(h, h->cur), mac_at<R>(h, h->t - 1), ro_momd(h), ro_mom<R>(h),
                           as<R>(h, L.chi), S.pend, h->first);
    if (lb_status s = check_launch(h, "k_moments")) return s;
    if (h->p.has_nozzle && !h->first) {
        if (d2)
            hipLaunchKernelGGL(lbk2::k2_create<R>, dim3(L.nb_create), dim3(TPB), 0, h->stream, h->P, geo(h),
                               as<double>(h, L.momd), as<R>(h, L.mom), as<R>(h, L.chi), S.pendc, 0);
        else
            hipLaunchKernelGGL(k_create<R>, dim3(L.nb_create), dim3(TPB), 0, h->stream, h->P, geo(h), ro_momd(h),
                               ro_mom<R>(h), as<R>(h, L.chi), S.pendc, 0);
        if (lb_status s = check_launch(h, "k_create")) return s;
        nbsp = S.zero_pendc ? NB_SPARSE : (int)L.nb_create;
    } else if (S.zero_pendc) {
        if (hipMemsetAsync(S.pendc, 0, NB_SPARSE * 2 * 8, h->stream) != hipSuccess)
            return fail(h, LB_EDEVICE, "hipMemsetAsync");
        nbsp = NB_SPARSE;
    } else {
        nbsp = 0;
    }
    return LB_OK;
}

// Fold the recorded events into the running sums (waits for them).
lb_status timing_fold(lb_handle *h)
{
    for (size_t k = 0; k + 2 < h->nev; k += 3) {
        float a = 0.f, b = 0.f;
        hipError_t e = hipEventSynchronize(h->ev[k + 2]);
        if (e == hipSuccess) e = hipEventElapsedTime(&a, h->ev[k], h->ev[k + 1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&b, h->ev[k + 1], h->ev[k + 2]);
        if (e != hipSuccess) {
            h->nev = 0;
            return fail(h, LB_EDEVICE, std::string("timing events: ") + hipGetErrorString(e));
        }
        h->acc_prep += a;
        h->acc_step += b;
        h->acc_n += 1;
    }
    h->nev = 0;
    return LB_OK;
}

constexpr size_t MAX_TIMED_EVENTS = 3 * 1024;

// Record timing event k (0: step start, 1: before the fused kernel, 2: after).
lb_status timing_mark(lb_handle *h, int k)
{
    if (!h->timing) return LB_OK;
    if (k == 0) h->nev -= h->nev % 3;  // drop the marks of a step that failed part-way
    if (k == 0 && h->nev + 3 > MAX_TIMED_EVENTS)
        if (lb_status s = timing_fold(h)) return s;
    if (h->nev >= h->ev.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return fail(h, LB_EDEVICE, "hipEventCreate");
        h->ev.push_back(e);
    }
    if (hipEventRecord(h->ev[h->nev], h->stream) != hipSuccess) return fail(h, LB_EDEVICE, "hipEventRecord");
    h->nev += 1;
    return LB_OK;
}

template <typename R, int ST>
lb_status launch_fused(lb_handle *h)
{
    constexpr int TY = sizeof(R) == 8 ? TY_F64 : (ST == ST_PLAIN ? PC_TY_PLAIN : PC_TY_DEV);
    constexpr int CR = ST == ST_PLAIN ? PC_CR_PLAIN : PC_CR_DEV;
    const Layout &L = h->L;
    void *src = pops_at(h, h->cur), *dst = pops_at(h, 1 - h->cur);
    if constexpr (sizeof(R) == 4) {
        const dim3 block((TY + 3 + TY / CR) * 64);
        if (h->first)
            hipLaunchKernelGGL((k_fused_pc<R, TY, true, ST, CR>), dim3((unsigned)L.nbf), block, 0, h->stream, h->P,
                               geo(h), L.fg, src, dst, as<double>(h, L.momd), as<R>(h, L.mom), as<R>(h, L.chi),
                               as<R>(h, L.ghost), mac_at<R>(h, h->t), mo_at(h, h->cur), mo_at(h, 1 - h->cur));
        else
            hipLaunchKernelGGL((k_fused_pc<R, TY, false, ST, CR>), dim3((unsigned)L.nbf), block, 0, h->stream, h->P,
                               geo(h), L.fg, src, dst, as<double>(h, L.momd), as<R>(h, L.mom), as<R>(h, L.chi),
                               as<R>(h, L.ghost), mac_at<R>(h, h->t), mo_at(h, h->cur), mo_at(h, 1 - h->cur));
    } else {
        static_assert(ST == ST_PLAIN, "FP64 storage is plain");
        const R *s64 = reinterpret_cast<const R *>(src);
        R *d64 = reinterpret_cast<R *>(dst);
        if (h->first)
            hipLaunchKernelGGL((k_fused<R, TY, true>), dim3((unsigned)L.nbf), dim3((TY + 3) * 64), 0, h->stream, h->P,
                               geo(h), L.fg, s64, d64, as<double>(h, L.momd), as<R>(h, L.mom), as<R>(h, L.chi),
                               as<R>(h, L.ghost), mac_at<R>(h, h->t));
        else
            hipLaunchKernelGGL((k_fused<R, TY, false>), dim3((unsigned)L.nbf), dim3((TY + 3) * 64), 0, h->stream,
                               h->P, geo(h), L.fg, s64, d64, as<double>(h, L.momd), as<R>(h, L.mom),
                               as<R>(h, L.chi), as<R>(h, L.ghost), mac_at<R>(h, h->t));
    }
    return check_launch(h, "k_fused");
}

// One time step: the step's geometry, boundary preparation (pulls of the
// cells next to the z faces and the head, node creation, wall densities,
// ghost layers), the fused step kernel over the whole box, the step counter.
// Every launch argument is the same at every step of one parity (the
// population and macro buffers alternate), so an even number of steps can be
// captured once and replayed.
// Steps after the first run the batched kernels over the handle's own
// one-member table (the same compiled code as a batch, so a simulation
// gives the same bits alone and in a batch); the table's buffers are indexed
// by the step's parity, which equals the population buffer index.
template <typename R, int ST>
lb_status run_step_table(lb_handle *h)
{
    const BatchTable *T = as<BatchTable>(h, h->L.tab);
    const unsigned *nb = h->lone_nb;
    const int j = (int)(h->t & 1);
    if (lb_status s = timing_mark(h, 0)) return s;
    hipLaunchKernelGGL((kb_pre<R, ST>), dim3(nb[BK_PRE]), dim3(TPB), 0, h->stream, T, j);
    if (nb[BK_CREATE]) hipLaunchKernelGGL(kb_create<R>, dim3(nb[BK_CREATE]), dim3(TPB), 0, h->stream, T, j);
    if (nb[BK_WALL]) hipLaunchKernelGGL(kb_wall<R>, dim3(nb[BK_WALL]), dim3(TPB), 0, h->stream, T, j);
    if (nb[BK_GHOST]) hipLaunchKernelGGL(kb_ghost<R>, dim3(nb[BK_GHOST]), dim3(TPB), 0, h->stream, T, j);
    if (lb_status s = check_launch(h, "boundary kernels")) return s;
    if (lb_status s = timing_mark(h, 1)) return s;
    if constexpr (sizeof(R) == 4) {
        constexpr int TY = ST == ST_PLAIN ? PC_TY_PLAIN : PC_TY_DEV;
        constexpr int CR = ST == ST_PLAIN ? PC_CR_PLAIN : PC_CR_DEV;
        hipLaunchKernelGGL((kb_fused_pc<R, TY, ST, CR>), dim3(nb[BK_FUSED]), dim3((TY + 3 + TY / CR) * 64), 0,
                           h->stream, T, j);
    } else {
        hipLaunchKernelGGL(kb_fused64<TY_F64>, dim3(nb[BK_FUSED]), dim3((TY_F64 + 3) * 64), 0, h->stream, T, j);
    }
    if (lb_status s = check_launch(h, "step kernel")) return s;
    if (lb_status s = timing_mark(h, 2)) return s;
    h->cur = 1 - h->cur;
    h->t += 1;
    return LB_OK;
}

// One D2Q9 step: the pull with the step's geometry and boundary sums, node
// creation, the colour fields of the head's solid nodes and the ghost rows,
// the collision.  As for D3Q19 the launch arguments depend on the step's
// parity only.
template <typename R>
lb_status run_step2(lb_handle *h)
{
    const Layout &L = h->L;
    if (lb_status s = timing_mark(h, 0)) return s;
    hipLaunchKernelGGL(lbk2::k2_pull<R>, dim3(L.nb_pre), dim3(TPB), 0, h->stream, h->P, geo(h),
                       reinterpret_cast<const R *>(pops_at(h, h->cur)), mac_at<R>(h, h->t - 1), as<double>(h, L.momd),
                       as<R>(h, L.mom), as<R>(h, L.chi), as<double>(h, L.cumpre), h->first, 0);
    if (h->p.has_nozzle && !h->first)
        hipLaunchKernelGGL(lbk2::k2_create<R>, dim3(L.nb_create), dim3(TPB), 0, h->stream, h->P, geo(h),
                           as<double>(h, L.momd), as<R>(h, L.mom), as<R>(h, L.chi), as<double>(h, L.cumc), 1);
    if (h->p.has_nozzle || !h->P.periodic_z)
        hipLaunchKernelGGL(lbk2::k2_wall<R>, dim3(L.nb_wall), dim3(TPB), 0, h->stream, h->P, geo(h),
                           as<double>(h, L.momd), as<R>(h, L.chi), as<R>(h, L.ghost));
    if (lb_status s = check_launch(h, "D2Q9 pull / boundary kernels")) return s;
    if (lb_status s = timing_mark(h, 1)) return s;
    hipLaunchKernelGGL(lbk2::k2_collide<R>, dim3((unsigned)L.nbm), dim3(TPB), 0, h->stream, h->P, geo(h),
                       as<double>(h, L.momd), as<R>(h, L.mom), as<R>(h, L.chi), as<R>(h, L.ghost),
                       reinterpret_cast<R *>(pops_at(h, 1 - h->cur)), mac_at<R>(h, h->t));
    if (lb_status s = check_launch(h, "k2_collide")) return s;
    if (lb_status s = timing_mark(h, 2)) return s;
    h->cur = 1 - h->cur;
    h->t += 1;
    h->first = 0;
    return LB_OK;
}

template <typename R, int ST>
lb_status run_step(lb_handle *h)
{
    if (is_d2(h->p)) return run_step2<R>(h);
    if (!h->first) return run_step_table<R, ST>(h);
    const Layout &L = h->L;
    if (lb_status s = timing_mark(h, 0)) return s;
    if (!h->p.has_nozzle && h->P.periodic_z)
        if (lb_status s = launch_clock(h)) return s;  // otherwise k_pre computes the geometry
    if (h->p.has_nozzle || !h->P.periodic_z) {
        hipLaunchKernelGGL((k_pre<R, ST>), dim3(L.nb_pre), dim3(TPB), 0, h->stream, h->P, geo(h), pop_src<R, ST>(h, h->cur),
                           mac_at<R>(h, h->t - 1), as<double>(h, L.momd), as<R>(h, L.mom), as<R>(h, L.chi),
                           as<double>(h, L.cumpre), h->first);
        if (lb_status s = check_launch(h, "k_pre")) return s;
    }
    if (h->p.has_nozzle) {
        if (!h->first) {
            hipLaunchKernelGGL(k_create<R>, dim3(L.nb_create), dim3(TPB), 0, h->stream, h->P, geo(h),
                               as<double>(h, L.momd), as<R>(h, L.mom), as<R>(h, L.chi), as<double>(h, L.cumc), 1);
            if (lb_status s = check_launch(h, "k_create")) return s;
        }
        hipLaunchKernelGGL(k_wall<R>, dim3(L.nb_wall), dim3(TPB), 0, h->stream, h->P, geo(h), as<double>(h, L.momd),
                           as<R>(h, L.chi));
        if (lb_status s = check_launch(h, "k_wall")) return s;
    }
    if (!h->P.periodic_z) {
        long long n = 2LL * h->p.nx * h->p.ny;
        hipLaunchKernelGGL(k_ghost<R>, dim3((unsigned)((n + TPB - 1) / TPB)), dim3(TPB), 0, h->stream, h->P, geo(h),
                           as<double>(h, L.momd), as<R>(h, L.ghost));
        if (lb_status s = check_launch(h, "k_ghost")) return s;
    }
    if (lb_status s = timing_mark(h, 1)) return s;
    if (lb_status s = launch_fused<R, ST>(h)) return s;
    if (lb_status s = timing_mark(h, 2)) return s;
    h->cur = 1 - h->cur;
    h->t += 1;
    h->first = 0;
    return LB_OK;
}

template <typename R, typename O>
lb_status run_output(lb_handle *h, const ReadSlots &S, O *ry, O *rb, O *u)
{
    hipLaunchKernelGGL((k_output<R, O>), dim3(S.nb), dim3(TPB), 0, h->stream, h->P, geo(h),
                       ro_momd(h), ro_mom<R>(h), ry, rb, u, S.part);
    return check_launch(h, "k_output");
}

ReadSlots workspace_slots(lb_handle *h)
{
    const Layout &L = h->L;
    return ReadSlots{as<double>(h, L.pend), as<double>(h, L.part), as<double>(h, L.pendc), as<double>(h, L.red),
                     (unsigned)L.nbm, true};
}

template <typename R, int ST>
lb_status moments_impl(lb_handle *h, void *ry, void *rb, void *u, int dst_dev, int dtype, lb_conserved *cons,
                       const ReadSlots &S)
{
    const Layout &L = h->L;
    const long long N = h->P.N;
    int nbsp = 0;
    if (lb_status s = run_readout<R, ST>(h, S, nbsp)) return s;
    // outputs: direct to device pointers, or staged in the spare population buffer
    char *stage = pops_at(h, 1 - h->cur);
    size_t osz = dtype == 0 ? 8 : 4;
    void *dry = ry, *drb = rb, *du = u;
    if (!dst_dev) {
        dry = ry ? stage : nullptr;
        drb = rb ? stage + N * osz : nullptr;
        du = u ? stage + 2 * N * osz : nullptr;
    }
    lb_status s = dtype == 0 ? run_output<R, double>(h, S, (double *)dry, (double *)drb, (double *)du)
                             : run_output<R, float>(h, S, (float *)dry, (float *)drb, (float *)du);
    if (s) return s;
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(TPB), 0, h->stream, S.part, S.pend, (long long)S.nb,
                       as<double>(h, L.cumpre), NB_PRE, as<double>(h, L.cumc), S.pendc, NB_SPARSE, nbsp, S.red);
    if ((s = check_launch(h, "k_reduce"))) return s;
    double red[16];
    hipError_t e = hipMemcpyAsync(red, S.red, 14 * 8, hipMemcpyDeviceToHost, h->stream);
    if (!dst_dev && e == hipSuccess) {
        if (ry) e = hipMemcpyAsync(ry, dry, N * osz, hipMemcpyDeviceToHost, h->stream);
        if (rb && e == hipSuccess) e = hipMemcpyAsync(rb, drb, N * osz, hipMemcpyDeviceToHost, h->stream);
        if (u && e == hipSuccess) e = hipMemcpyAsync(u, du, 3 * N * osz, hipMemcpyDeviceToHost, h->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail(h, LB_EDEVICE, std::string("lb_moments copy: ") + hipGetErrorString(e));
    if (cons) {
        cons->mass[0] = red[0];
        cons->mass[1] = red[1];
        for (int a = 0; a < 3; ++a) cons->mom[a] = red[2 + a];
        cons->mass_wall[0] = red[5];
        cons->mass_wall[1] = red[6];
        cons->mass_open[0] = red[7];
        cons->mass_open[1] = red[8];
        cons->mass_created[0] = red[9];
        cons->mass_created[1] = red[10];
        cons->mass_deleted[0] = red[11];
        cons->mass_deleted[1] = red[12];
    }
    if (red[13] != 0.0) {
        h->unstable = 1;
        return fail(h, LB_EUNSTABLE, "unstable state: NaN, non-positive density or |u| > 0.3");
    }
    return LB_OK;
}

// Call f.operator()<R, ST>() for the handle's storage form: R the arithmetic
// type, ST the stored representation.
template <typename F>
lb_status with_storage(lb_handle *h, F &&f)
{
    switch (h->p.storage) {
    case LB_F64: return f.template operator()<double, ST_PLAIN>();
    case LB_F32: return f.template operator()<float, ST_PLAIN>();
    case LB_BF16_DEV: return f.template operator()<float, ST_BF16>();
    default: return f.template operator()<float, ST_F16>();
    }
}

lb_status step_one(lb_handle *h)
{
    return with_storage(h, [&]<typename R, int ST>() { return run_step<R, ST>(h); });
}

lb_status moments_any(lb_handle *h, void *ry, void *rb, void *u, int dst_dev, int dtype, lb_conserved *cons)
{
    const ReadSlots S = workspace_slots(h);
    return with_storage(h, [&]<typename R, int ST>() {
        return moments_impl<R, ST>(h, ry, rb, u, dst_dev, dtype, cons, S);
    });
}

// ------------------------------------------------ read-out without scratch
//
// lb_moments_noalloc keeps the read-out's per-call partial sums in `scratch`,
// a file-scope device array of NA_TOTAL doubles (102.5 KB), instead of the
// handle's workspace, with a fixed grid of at most NB_NA blocks (grid-stride
// kernels), so its size does not depend on the box.  Each GPU the library
// runs on holds its own copy until the process ends.  In host code the
// array's name is not a device address: the kernels get each device's copy
// through the pointer hipGetSymbolAddress returned for that device
// (scratch_dev), taken once per device at lb_create.  Every call on one GPU
// shares the array; the kernels write every slot they read, so nothing has
// to be cleared, and calls that overlap on one GPU race.
constexpr int NB_NA = 1024;
constexpr size_t NA_PEND = 0;
constexpr size_t NA_PART = NA_PEND + (size_t)NB_NA * NSLOT;
constexpr size_t NA_PENDC = NA_PART + (size_t)NB_NA * NPART;
constexpr size_t NA_RED = NA_PENDC + (size_t)NB_SPARSE * 2;
constexpr size_t NA_TOTAL = NA_RED + 16;

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_dev[MAX_DEVICES] = {};

}  // namespace

static __device__ __align__(256) double scratch[NA_TOTAL];

namespace {

// The device address of `scratch` on device `dev` (looked up once per
// device, with that device current).
lb_status scratch_dev(int dev, double **out, std::string &err)
{
    if (dev < 0 || dev >= MAX_DEVICES) {
        err = "device index out of range";
        return LB_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess) {
            err = "hipGetDevice failed";
            return LB_EDEVICE;
        }
        if (cur != dev && hipSetDevice(dev) != hipSuccess) {
            err = "hipSetDevice failed";
            return LB_EDEVICE;
        }
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p) {
            err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return LB_EDEVICE;
        }
        g_scratch_dev[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_dev[dev];
    return LB_OK;
}

lb_status moments_noalloc_any(lb_handle *h, void *ry, void *rb, void *u, int dst_dev, int dtype,
                              lb_conserved *cons)
{
    if (!h->scratch) return fail(h, LB_EDEVICE, "lb_moments_noalloc: no device scratch: " + h->scratch_err);
    const long long nb = std::min<long long>(h->L.nbm, NB_NA);
    if (nb > NB_NA || (long long)h->L.nb_create > NB_SPARSE)
        return fail(h, LB_EINVAL, "lb_moments_noalloc: the read-out needs more slots than the device scratch holds");
    double *sc = h->scratch;
    const ReadSlots S{sc + NA_PEND, sc + NA_PART, sc + NA_PENDC, sc + NA_RED, (unsigned)nb, false};
    return with_storage(h, [&]<typename R, int ST>() {
        return moments_impl<R, ST>(h, ry, rb, u, dst_dev, dtype, cons, S);
    });
}

// ---------------------------------------------------------------- batching

constexpr size_t MAX_CHAINS = 4;

// The instantiated graph of k steps of one handle (k even: the buffers a
// step uses depend on the step's parity only, so the chain replays correctly
// while the handle's parity and population buffer match the key).  Captured
// on the handle's private stream; the host-side state is restored afterwards
// (capturing runs nothing).
lb_status chain_exec(lb_handle *h, int k, hipGraphExec_t *out)
{
    const int parity = (int)(h->t & 1);
    for (const lb_handle::Chain &c : h->chains)
        if (c.k == k && c.cur == h->cur && c.parity == parity) {
            *out = c.exec;
            return LB_OK;
        }
    if (!h->cap && hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking) != hipSuccess)
        return fail(h, LB_EDEVICE, "hipStreamCreate (capture stream)");
    const hipStream_t saved = h->stream;
    const int cur = h->cur, first = h->first, timing = h->timing;
    const long t = h->t;
    if (hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(h, LB_EDEVICE, "hipStreamBeginCapture");
    h->timing = 0;
    h->stream = h->cap;
    lb_status st = LB_OK;
    for (int j = 0; j < k && st == LB_OK; ++j)
        st = step_one(h);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(h->cap, &g);
    h->stream = saved;
    h->cur = cur;
    h->first = first;
    h->t = t;
    h->timing = timing;
    if (st != LB_OK || e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        if (st != LB_OK) return st;
        return fail(h, LB_EDEVICE, std::string("stream capture: ") + hipGetErrorString(e));
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return fail(h, LB_EDEVICE, "hipGraphInstantiate");
    if (h->chains.size() >= MAX_CHAINS) {
        // an evicted chain may still be running on the handle's stream
        if (hipStreamSynchronize(h->stream) != hipSuccess) return fail(h, LB_EDEVICE, "hipStreamSynchronize");
        (void)hipGraphExecDestroy(h->chains.front().exec);
        h->chains.erase(h->chains.begin());
    }
    h->chains.push_back(lb_handle::Chain{k, cur, parity, exec});
    *out = exec;
    return LB_OK;
}

lb_status step_eager(lb_handle *h, int n)
{
    for (int j = 0; j < n; ++j) {
        lb_status s = step_one(h);
        if (s) return s;
    }
    return LB_OK;
}

}  // namespace

// ---------------------------------------------------------------- batches

struct lb_batch {
    int storage = 0;
    hipStream_t stream = nullptr;
    BatchTable *dtab = nullptr;                 // device slot table (the caller's workspace)
    BatchTable *htab[2] = {nullptr, nullptr};   // pinned host staging, used in turn
    hipEvent_t hev[2] = {nullptr, nullptr};     // the upload from htab[i] has run
    bool hev_used[2] = {false, false};
    int hcur = 0;
    hipStream_t cap = nullptr;                  // private capture stream
    hipGraphExec_t exec = nullptr;              // gk steps of the batched kernels
    int gk = 0;
    unsigned gcap[BK_N] = {0, 0, 0, 0, 0};      // grid of each batched kernel in the graph
    hipEvent_t done = nullptr;                  // the last launch has run
    std::string err;
    ~lb_batch()
    {
        if (exec) {
            (void)hipStreamSynchronize(stream);
            (void)hipGraphExecDestroy(exec);
        }
        for (int i = 0; i < 2; ++i) {
            if (hev[i]) (void)hipEventDestroy(hev[i]);
            if (htab[i]) (void)hipHostFree(htab[i]);
        }
        if (done) (void)hipEventDestroy(done);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

namespace {

lb_status bfail(lb_batch *b, lb_status s, const std::string &msg)
{
    if (b) b->err = msg;
    g_err = msg;
    return s;
}

size_t batch_table_bytes() { return al(sizeof(BatchTable)); }

template <typename F>
lb_status with_form(int storage, F &&f)
{
    switch (storage) {
    case LB_F64: return f.template operator()<double, ST_PLAIN>();
    case LB_F32: return f.template operator()<float, ST_PLAIN>();
    case LB_BF16_DEV: return f.template operator()<float, ST_BF16>();
    default: return f.template operator()<float, ST_F16>();
    }
}

// The batched kernels of batch step j, in the order of a lone step.
template <typename R, int ST>
lb_status batch_launch_step(lb_batch *b, hipStream_t st, int j)
{
    const BatchTable *T = b->dtab;
    const unsigned *c = b->gcap;
    if (c[BK_PRE]) hipLaunchKernelGGL((kb_pre<R, ST>), dim3(c[BK_PRE]), dim3(TPB), 0, st, T, j);
    if (c[BK_CREATE]) hipLaunchKernelGGL(kb_create<R>, dim3(c[BK_CREATE]), dim3(TPB), 0, st, T, j);
    if (c[BK_WALL]) hipLaunchKernelGGL(kb_wall<R>, dim3(c[BK_WALL]), dim3(TPB), 0, st, T, j);
    if (c[BK_GHOST]) hipLaunchKernelGGL(kb_ghost<R>, dim3(c[BK_GHOST]), dim3(TPB), 0, st, T, j);
    if (c[BK_FUSED]) {
        if constexpr (sizeof(R) == 4) {
            constexpr int TY = ST == ST_PLAIN ? PC_TY_PLAIN : PC_TY_DEV;
            constexpr int CR = ST == ST_PLAIN ? PC_CR_PLAIN : PC_CR_DEV;
            hipLaunchKernelGGL((kb_fused_pc<R, TY, ST, CR>), dim3(c[BK_FUSED]), dim3((TY + 3 + TY / CR) * 64), 0, st,
                               T, j);
        } else {
            hipLaunchKernelGGL(kb_fused64<TY_F64>, dim3(c[BK_FUSED]), dim3((TY_F64 + 3) * 64), 0, st, T, j);
        }
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return bfail(b, LB_EDEVICE, std::string("batched launch: ") + hipGetErrorString(e));
    return LB_OK;
}

// Capture k batch steps (grids b->gcap) once on the private stream and
// instantiate them; the previous graph is released after the batch stream
// has run it.
lb_status batch_capture(lb_batch *b, int k)
{
    if (!b->cap && hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess)
        return bfail(b, LB_EDEVICE, "hipStreamCreate (batch capture stream)");
    if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return bfail(b, LB_EDEVICE, "hipStreamBeginCapture (batch)");
    lb_status st = LB_OK;
    for (int j = 0; j < k && st == LB_OK; ++j)
        st = with_form(b->storage, [&]<typename R, int ST>() { return batch_launch_step<R, ST>(b, b->cap, j); });
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (st != LB_OK || e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        if (st != LB_OK) return st;
        return bfail(b, LB_EDEVICE, std::string("batch stream capture: ") + hipGetErrorString(e));
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return bfail(b, LB_EDEVICE, "hipGraphInstantiate (batch)");
    if (b->exec) {
        if (hipStreamSynchronize(b->stream) != hipSuccess) return bfail(b, LB_EDEVICE, "hipStreamSynchronize (batch)");
        (void)hipGraphExecDestroy(b->exec);
    }
    b->exec = exec;
    b->gk = k;
    return LB_OK;
}

void *mac_ptr(lb_handle *h, long t)
{
    return h->ws + h->L.mac + (t & 1) * al(NMAC * (size_t)h->P.NA * real_size(h->p.storage));
}

// A handle's slot: its buffers for the steps of parity q = 0, 1 counted from
// a step t0 at which its population buffer is cur0, the tiling fg of its
// step kernel, and the blocks each step kernel gives it (the boundary
// kernels' grids are the handle's own: their per-block sums depend on them).
void fill_slot(lb_handle *h, BatchSlot &S, int cur0, long t0, const FusedGrid &fg, int nsteps)
{
    const Layout &L = h->L;
    S.P = h->P;
    S.fg = fg;
    S.G = geo(h);
    for (int q = 0; q < 2; ++q) {
        const int cq = cur0 ^ q;
        S.src[q] = pops_at(h, cq);
        S.dst[q] = pops_at(h, 1 - cq);
        S.mac_prev[q] = mac_ptr(h, t0 + q - 1);
        S.mac_next[q] = mac_ptr(h, t0 + q);
        S.mo_src[q] = mo_at(h, cq);
        S.mo_dst[q] = mo_at(h, 1 - cq);
    }
    S.momd = as<double>(h, L.momd);
    S.mom = h->ws + L.mom;
    S.chi = h->ws + L.chi;
    S.ghost = h->ws + L.ghost;
    S.cumpre = as<double>(h, L.cumpre);
    S.cumc = as<double>(h, L.cumc);
    S.nsteps = nsteps;
    const bool noz = h->p.has_nozzle != 0, per = h->P.periodic_z != 0;
    // a handle without boundary work still gets one preparation block,
    // which computes its step geometry
    S.nb[BK_PRE] = (noz || !per) ? L.nb_pre : 1;
    S.nb[BK_CREATE] = noz ? L.nb_create : 0;
    S.nb[BK_WALL] = noz ? L.nb_wall : 0;
    S.nb[BK_GHOST] = per ? 0 : (unsigned)((2LL * h->p.nx * h->p.ny + TPB - 1) / TPB);
    S.nb[BK_FUSED] = (unsigned)((long long)fg.ntx * fg.nty * fg.nzc);
    for (int kind = 0; kind < BK_N; ++kind) S.off[kind] = 0;
}

unsigned next_pow2(unsigned v)
{
    unsigned p = 64;
    while (p < v) p <<= 1;
    return p;
}

}  // namespace

extern "C" {

lb_status lb_footprint(const lb_params *p, size_t *bytes)
{
    if (!p || !bytes) return fail(nullptr, LB_EINVAL, "null argument");
    if (const char *m = validate(*p)) return fail(nullptr, LB_EINVAL, m);
    *bytes = layout_of(*p).total;
    return LB_OK;
}

lb_status lb_create(const lb_params *p, const double *rho_y, const double *rho_b, const double *u,
                    void *dev_workspace, size_t ws_bytes, void *hip_stream, lb_handle **out)
{
    if (out) *out = nullptr;
    if (!p || !rho_y || !rho_b || !dev_workspace || !out) return fail(nullptr, LB_EINVAL, "null argument");
    if (const char *m = validate(*p)) return fail(nullptr, LB_EINVAL, m);
    if (reinterpret_cast<uintptr_t>(dev_workspace) % ALIGN) return fail(nullptr, LB_EINVAL, "workspace not 256-byte aligned");
    Layout L = layout_of(*p);
    if (ws_bytes < L.total) return fail(nullptr, LB_ENOMEM, "workspace smaller than lb_footprint()");
    lb_handle *h = new lb_handle();
    h->p = *p;
    h->P = make_dev(*p);
    h->L = L;
    h->stream = reinterpret_cast<hipStream_t>(hip_stream);
    h->ws = reinterpret_cast<char *>(dev_workspace);
    h->cur = 0;
    h->t = 0;
    h->first = 1;
    h->unstable = 0;
    {
        // the device of the workspace: where lb_moments_noalloc's scratch lives
        hipPointerAttribute_t attr;
        int dev = -1;
        if (hipPointerGetAttributes(&attr, dev_workspace) == hipSuccess) dev = attr.device;
        else (void)hipGetLastError();
        if (dev < 0) (void)hipGetDevice(&dev);
        if (scratch_dev(dev, &h->scratch, h->scratch_err) != LB_OK) h->scratch = nullptr;
    }
    const long long N = h->P.N;
    // stage the initial fields in the second population buffer (at least
    // 72 B per cell, the fields need 40)
    char *stage = pops_at(h, 1);
    double *dry = reinterpret_cast<double *>(stage);
    double *drb = dry + N;
    double *du = drb + N;
    hipError_t e = hipMemcpyAsync(dry, rho_y, N * 8, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(drb, rho_b, N * 8, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess && u) e = hipMemcpyAsync(du, u, 3 * N * 8, hipMemcpyHostToDevice, h->stream);
    // cumulative and pending per-block sums start at zero (kernels sized to a
    // box's work leave the slots past their grid untouched)
    if (e == hipSuccess) e = hipMemsetAsync(h->ws + L.cumpre, 0, L.red - L.cumpre, h->stream);
    // device step counter: t = 0, no step taken (the stream is synchronised
    // below, before g0 goes out of scope)
    StepGeom g0;
    std::memset(&g0, 0, sizeof(g0));
    g0.first = 1;
    if (e == hipSuccess) e = hipMemcpyAsync(geo(h), &g0, sizeof(g0), hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) {
        std::string m = std::string("lb_create: ") + hipGetErrorString(e);
        delete h;
        return fail(nullptr, LB_EDEVICE, m);
    }
    // the handle's one-member slot table for its steps after the first
    // (staged on the heap until the stream synchronisation below)
    std::unique_ptr<BatchTable> lone(new BatchTable());
    lone->n = 1;
    fill_slot(h, lone->slot[0], 0, 0, L.fg, std::numeric_limits<int>::max());
    for (int kind = 0; kind < BK_N; ++kind) {
        lone->total[kind] = lone->slot[0].nb[kind];
        h->lone_nb[kind] = lone->slot[0].nb[kind];
    }
    if (!is_d2(*p))
        e = hipMemcpyAsync(as<BatchTable>(h, L.tab), lone.get(), offsetof(BatchTable, slot) + sizeof(BatchSlot),
                           hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) {
        std::string m = std::string("lb_create: ") + hipGetErrorString(e);
        delete h;
        return fail(nullptr, LB_EDEVICE, m);
    }
    dim3 grid((unsigned)L.nbm);
    hipLaunchKernelGGL(k_clock, dim3(1), dim3(64), 0, h->stream, h->P, geo(h));
    with_storage(h, [&]<typename R, int ST>() {
        if (is_d2(*p))
            hipLaunchKernelGGL(lbk2::k2_init<R>, grid, dim3(TPB), 0, h->stream, h->P, geo(h), dry, drb, du, u ? 1 : 0,
                               reinterpret_cast<R *>(pops_at(h, 0)));
        else
            hipLaunchKernelGGL((k_init<R, ST>), grid, dim3(TPB), 0, h->stream, h->P, geo(h), dry, drb, du,
                               u ? 1 : 0, (void *)pops_at(h, 0), mo_at(h, 0));
        return LB_OK;
    });
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        std::string m = std::string("lb_create init: ") + hipGetErrorString(e);
        delete h;
        return fail(nullptr, LB_EDEVICE, m);
    }
    *out = h;
    return LB_OK;
}

lb_status lb_step(lb_handle *h, int nsteps)
{
    if (!h || nsteps < 0) return fail(h, LB_EINVAL, "bad handle or step count");
    if (h->unstable) return fail(h, LB_ESTATE, "handle is unstable; only lb_moments and lb_destroy are allowed");
    for (int n = 0; n < nsteps; ++n) {
        lb_status s = step_one(h);
        if (s) return s;
        if (h->p.check_interval > 0 && h->t % h->p.check_interval == 0) {
            lb_conserved c;
            s = moments_any(h, nullptr, nullptr, nullptr, 1, 0, &c);
            if (s) return s;
        }
    }
    return LB_OK;
}

lb_status lb_moments(lb_handle *h, void *rho_y, void *rho_b, void *u, int dst_is_device, int dtype, lb_conserved *cons)
{
    if (!h || (dtype != 0 && dtype != 1)) return fail(h, LB_EINVAL, "bad handle or dtype");
    return moments_any(h, rho_y, rho_b, u, dst_is_device, dtype, cons);
}

lb_status lb_moments_noalloc(lb_handle *h, void *rho_y, void *rho_b, void *u, int dst_is_device, int dtype,
                             lb_conserved *cons)
{
    if (!h || (dtype != 0 && dtype != 1)) return fail(h, LB_EINVAL, "bad handle or dtype");
    return moments_noalloc_any(h, rho_y, rho_b, u, dst_is_device, dtype, cons);
}

lb_status lb_observe(lb_handle *h, const lb_window *w, lb_observables *out)
{
    if (!h || !w || !out) return fail(h, LB_EINVAL, "null argument");
    const int nx = h->p.nx, nz = h->p.nz;
    if (w->x_len < 1 || w->x_len > nx || w->y < 0 || w->y >= h->p.ny)
        return fail(h, LB_EINVAL, "lb_observe: window needs 1 <= x_len <= nx and 0 <= y < ny");
    const int x_lo = ((w->x_lo % nx) + nx) % nx;
    const ReadSlots S = workspace_slots(h);
    int nbsp = 0;
    if (lb_status s = with_storage(h, [&]<typename R, int ST>() { return run_readout<R, ST>(h, S, nbsp); }))
        return s;
    // the section's cells, at most one block per 256 (the read-out's part
    // slots hold one entry per 256 cells of the box)
    const int nb = (int)std::min<long long>(((long long)nx * nz + TPB - 1) / TPB, 1024);
    hipLaunchKernelGGL(k_observe, dim3(nb), dim3(TPB), 0, h->stream, h->P, geo(h), ro_momd(h), x_lo,
                       w->x_len, w->z_hi, w->y, S.part);
    hipLaunchKernelGGL(k_observe_final, dim3(1), dim3(TPB), 0, h->stream, S.part, nb, S.red);
    if (lb_status s = check_launch(h, "k_observe")) return s;
    double v[NOBS];
    hipError_t e = hipMemcpyAsync(v, S.red, sizeof(v), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail(h, LB_EDEVICE, std::string("lb_observe: ") + hipGetErrorString(e));
    const bool thread = v[0] > 0.0;
    out->ink_area = v[0];
    out->height = thread ? v[1] + 1.0 : 0.0;
    out->width = thread ? v[3] + v[2] + 1.0 : 0.0;
    out->coverage = thread ? v[0] / (out->height * out->width) : 0.0;
    out->p0 = h->P.rho0[1] * (h->P.dcs2[1] + 1.0 / 3.0);
    out->dp_max = v[4] > -1e299 ? v[4] : 0.0;
    out->substrate_ink = v[5];
    return LB_OK;
}

long lb_time(const lb_handle *h) { return h ? h->t : -1; }

lb_status lb_timing(lb_handle *h, int enable)
{
    if (!h) return fail(nullptr, LB_EINVAL, "null handle");
    h->timing = enable != 0;
    return LB_OK;
}

lb_status lb_timing_read(lb_handle *h, double *step_ms, double *prep_ms, long *steps)
{
    if (!h) return fail(nullptr, LB_EINVAL, "null handle");
    if (lb_status s = timing_fold(h)) return s;
    if (step_ms) *step_ms = h->acc_step;
    if (prep_ms) *prep_ms = h->acc_prep;
    if (steps) *steps = h->acc_n;
    h->acc_step = h->acc_prep = 0.0;
    h->acc_n = 0;
    return LB_OK;
}

lb_status lb_step_batch(lb_handle *const *hs, const int *nsteps, int n)
{
    if (!hs || !nsteps || n < 1) return fail(nullptr, LB_EINVAL, "lb_step_batch: null argument or n < 1");
    for (int i = 0; i < n; ++i) {
        if (!hs[i] || nsteps[i] < 0) return fail(nullptr, LB_EINVAL, "lb_step_batch: bad handle or step count");
        for (int j = 0; j < i; ++j)
            if (hs[j] == hs[i]) return fail(hs[i], LB_EINVAL, "lb_step_batch: a handle appears twice");
        if (hs[i]->unstable) return fail(hs[i], LB_ESTATE, "handle is unstable; only lb_moments and lb_destroy");
        if (hs[i]->p.check_interval > 0)
            return fail(hs[i], LB_EINVAL, "lb_step_batch: handles with check_interval > 0 step with lb_step");
    }
    // per handle: its first step and an odd remainder as ordinary launches,
    // the even part as one launch of its instantiated chain
    for (int i = 0; i < n; ++i) {
        lb_handle *h = hs[i];
        int k = nsteps[i];
        if (k > 0 && h->first) {
            if (lb_status s = step_eager(h, 1)) return s;
            --k;
        }
        const int g = k & ~1;
        if (g > 0) {
            hipGraphExec_t exec;
            if (lb_status s = chain_exec(h, g, &exec)) return s;
            if (hipGraphLaunch(exec, h->stream) != hipSuccess) return fail(h, LB_EDEVICE, "hipGraphLaunch");
            h->t += g;
            h->first = 0;
        }
        if (k & 1)
            if (lb_status s = step_eager(h, 1)) return s;
    }
    return LB_OK;
}

lb_status lb_destroy(lb_handle *h)
{
    if (!h) return LB_EINVAL;
    // the handle's chains may still run on its stream
    if (!h->chains.empty()) (void)hipStreamSynchronize(h->stream);
    delete h;
    return LB_OK;
}

lb_status lb_batch_footprint(size_t *bytes)
{
    if (!bytes) return fail(nullptr, LB_EINVAL, "null argument");
    *bytes = batch_table_bytes();
    return LB_OK;
}

lb_status lb_batch_create(int storage, void *dev_workspace, size_t ws_bytes, void *hip_stream, lb_batch **out)
{
    if (out) *out = nullptr;
    if (!dev_workspace || !out) return fail(nullptr, LB_EINVAL, "null argument");
    if (storage < LB_F64 || storage > LB_F16_DEV) return fail(nullptr, LB_EINVAL, "unknown storage form");
    if (reinterpret_cast<uintptr_t>(dev_workspace) % ALIGN)
        return fail(nullptr, LB_EINVAL, "workspace not 256-byte aligned");
    if (ws_bytes < batch_table_bytes()) return fail(nullptr, LB_ENOMEM, "workspace smaller than lb_batch_footprint()");
    lb_batch *b = new lb_batch();
    b->storage = storage;
    b->stream = reinterpret_cast<hipStream_t>(hip_stream);
    b->dtab = reinterpret_cast<BatchTable *>(dev_workspace);
    hipError_t e = hipSuccess;
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        e = hipHostMalloc((void **)&b->htab[i], sizeof(BatchTable), hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->hev[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
    if (e != hipSuccess) {
        std::string m = std::string("lb_batch_create: ") + hipGetErrorString(e);
        delete b;
        return fail(nullptr, LB_EDEVICE, m);
    }
    *out = b;
    return LB_OK;
}

lb_status lb_batch_step(lb_batch *b, lb_handle *const *hs, const int *nsteps, int n)
{
    if (!b) return fail(nullptr, LB_EINVAL, "null batch");
    if (n < 0 || n > BATCH_MAX || (n > 0 && (!hs || !nsteps)))
        return bfail(b, LB_EINVAL, "lb_batch_step: bad member list (at most 64 members)");
    for (int i = 0; i < n; ++i) {
        if (!hs[i] || nsteps[i] < 0) return bfail(b, LB_EINVAL, "lb_batch_step: bad handle or step count");
        for (int j = 0; j < i; ++j)
            if (hs[j] == hs[i]) return bfail(b, LB_EINVAL, "lb_batch_step: a handle appears twice");
        if (hs[i]->p.storage != b->storage) return bfail(b, LB_EINVAL, "lb_batch_step: storage form differs from the batch's");
        if (is_d2(hs[i]->p)) return bfail(b, LB_EINVAL, "lb_batch_step: a batch steps D3Q19 simulations");
        if (hs[i]->unstable) return bfail(b, LB_ESTATE, "lb_batch_step: a member is unstable");
        if (hs[i]->p.check_interval > 0)
            return bfail(b, LB_EINVAL, "lb_batch_step: handles with check_interval > 0 step with lb_step");
    }
    // the batch stream runs after each member's earlier work
    for (int i = 0; i < n; ++i) {
        lb_handle *h = hs[i];
        if (h->stream == b->stream || nsteps[i] == 0) continue;
        if (!h->bev && hipEventCreateWithFlags(&h->bev, hipEventDisableTiming) != hipSuccess)
            return bfail(b, LB_EDEVICE, "hipEventCreate (member)");
        if (hipEventRecord(h->bev, h->stream) != hipSuccess || hipStreamWaitEvent(b->stream, h->bev, 0) != hipSuccess)
            return bfail(b, LB_EDEVICE, "member stream ordering");
    }
    // a member's first step (it reads its own initial slots) runs alone, on
    // the batch stream
    int k[BATCH_MAX];
    for (int i = 0; i < n; ++i) {
        lb_handle *h = hs[i];
        k[i] = nsteps[i];
        if (k[i] > 0 && h->first) {
            const hipStream_t saved = h->stream;
            const int timing = h->timing;
            h->stream = b->stream;
            h->timing = 0;
            const lb_status s = step_one(h);
            h->stream = saved;
            h->timing = timing;
            if (s) return bfail(b, s, h->err);
            k[i] -= 1;
        }
    }
    // the slot table, staged in pinned host memory and uploaded in stream order
    const int slot_buf = b->hcur;
    if (b->hev_used[slot_buf] && hipEventSynchronize(b->hev[slot_buf]) != hipSuccess)
        return bfail(b, LB_EDEVICE, "hipEventSynchronize (table staging)");
    BatchTable &T = *b->htab[slot_buf];
    T.n = 0;
    for (int kind = 0; kind < BK_N; ++kind) T.total[kind] = 0;
    int active = 0, kmax = 0;
    for (int i = 0; i < n; ++i) active += k[i] > 0;
    // z chunks: the batch as a whole fills the GPU, so members chunk less
    const long long want = active ? std::max(64, 1024 / active) : 512;
    for (int i = 0; i < n; ++i) {
        if (k[i] <= 0) continue;
        lb_handle *h = hs[i];
        BatchSlot &S = T.slot[T.n++];
        fill_slot(h, S, h->cur, h->t, fused_grid(h->p, h->L.ty, want), k[i]);
        for (int kind = 0; kind < BK_N; ++kind) {
            unsigned off = T.total[kind];
            if (kind == BK_FUSED) off = (off + 7u) & ~7u;  // keep the member's XCD-aware order
            S.off[kind] = off;
            T.total[kind] = off + S.nb[kind];
        }
        kmax = std::max(kmax, k[i]);
    }
    if (T.n > 0) {
        const size_t bytes = offsetof(BatchTable, slot) + (size_t)T.n * sizeof(BatchSlot);
        if (hipMemcpyAsync(b->dtab, &T, bytes, hipMemcpyHostToDevice, b->stream) != hipSuccess ||
            hipEventRecord(b->hev[slot_buf], b->stream) != hipSuccess)
            return bfail(b, LB_EDEVICE, "slot table upload");
        b->hev_used[slot_buf] = true;
        b->hcur ^= 1;
        // one graph of kmax steps, captured again only when the step count
        // or a kernel's block count outgrows it
        bool again = !b->exec || kmax > b->gk || kmax * 2 < b->gk;
        unsigned cap[BK_N];
        for (int kind = 0; kind < BK_N; ++kind) {
            cap[kind] = b->gcap[kind];
            if (T.total[kind] > cap[kind]) {
                cap[kind] = next_pow2(T.total[kind] + T.total[kind] / 4);
                again = true;
            }
        }
        if (again) {
            for (int kind = 0; kind < BK_N; ++kind) b->gcap[kind] = cap[kind];
            if (lb_status s = batch_capture(b, kmax)) return s;
        }
        if (hipGraphLaunch(b->exec, b->stream) != hipSuccess) return bfail(b, LB_EDEVICE, "hipGraphLaunch (batch)");
    }
    // each member's later work runs after the batch
    if (hipEventRecord(b->done, b->stream) != hipSuccess) return bfail(b, LB_EDEVICE, "hipEventRecord (batch)");
    for (int i = 0; i < n; ++i) {
        lb_handle *h = hs[i];
        if (h->stream != b->stream && nsteps[i] > 0 && hipStreamWaitEvent(h->stream, b->done, 0) != hipSuccess)
            return bfail(b, LB_EDEVICE, "member stream ordering");
        h->t += k[i];
        h->cur ^= (k[i] & 1);
        if (nsteps[i] > 0) h->first = 0;
    }
    return LB_OK;
}

lb_status lb_batch_destroy(lb_batch *b)
{
    if (!b) return LB_EINVAL;
    delete b;
    return LB_OK;
}

const char *lb_batch_last_error(const lb_batch *b) { return b ? b->err.c_str() : g_err.c_str(); }

const char *lb_strerror(lb_status s)
{
    switch (s) {
    case LB_OK: return "ok";
    case LB_EINVAL: return "invalid argument";
    case LB_ENOMEM: return "workspace too small";
    case LB_EDEVICE: return "device error";
    case LB_EUNSTABLE: return "unstable simulation";
    case LB_ESTATE: return "call not allowed in this state";
    }
    return "unknown status";
}

const char *lb_last_error(const lb_handle *h) { return h ? h->err.c_str() : g_err.c_str(); }

}  // extern "C"
