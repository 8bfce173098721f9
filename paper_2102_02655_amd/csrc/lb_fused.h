// lb_fused.h -- the single-pass time step: pull, moments, colour stencil,
// collision and store in one kernel.
//
// The colour gradient of a cell (Eq. (lattgrad)) needs the post-stream
// densities of its 18 neighbours at the same time level, i.e. the pulled
// populations of the neighbours.  A workgroup therefore owns a 64 x TY tile of
// columns and marches up a chunk of z planes, one thread per column of the
// tile or of its one-cell ring.  Iteration p:
//   1. issue the 38 loads that pull the thread's cell of plane p;
//   2. collide the tile cell of plane p - 2 from its parked state and the LDS
//      colour stencil (planes p - 3 .. p - 1), store its 38 values
//      (this arithmetic covers the latency of the loads of step 1);
//   3. reduce the loaded populations: colour fields into a 4-plane LDS ring,
//      and for tile cells the state the collision needs (masses, momentum,
//      the non-equilibrium stress, the BGK factor of the local relaxation
//      time -- the regularised collision needs nothing else, Eq. (reg)) into
//      a 2-plane LDS ring;
//   4. barrier.
// Each population is read from HBM by its owning tile; ring and z-halo
// re-reads are shared with neighbouring workgroups, which the XCD-aware
// block order keeps on the same L2.
//
// Waves: TY tile-row waves, 2 ring-row waves, 1 wave for the two ring
// columns.  LDS plane layout: (TY + 2) rows x 66 columns, column 0 = x0 - 1.
#pragma once

#include "lb_collide.h"
#include "lb_device.h"

namespace lbk {

struct FusedGrid {
    int ntx, nty, nzc, zlen;
};

struct Box3 {
    int x0, y0, z0, w, h, d;
};

// Geometry of one time step (from step t to t + 1), a function of t alone:
// the head axis at t - 1 and t (Sec. II.B, x_h(t) = x_h(0) + v t), the head's
// box (cells its template can touch between the two positions, two cells of
// margin, from the tip plane up) and the boxes of cells whose pull touches a
// boundary.  It lives in device memory, written by a one-thread kernel at the
// start of every step from a device step counter, so that the launches of a
// step have the same arguments at every step (a captured multi-step graph
// replays correctly).
struct StepGeom {
    long long t;  // steps completed
    int first;    // no step taken yet
    int nbox;     // boundary-preparation boxes in use
    HeadPos H;
    Box3 hb;      // head box
    Box3 bx[3];   // boundary-preparation boxes: head box one plane deeper, z = 0, z = nz - 1
};

// Head axis at step t, wrapped into [0, n); also the unwrapped position.
// Rounded as written (no contraction), identical on host and device.
__host__ __device__ inline void head_axis(const DevParams &P, long long t, double &hx, double &hy, double &ux,
                                          double &uy)
{
#pragma clang fp contract(off)
    const double x = P.x0noz[0] + P.vnoz[0] * (double)t;
    const double y = P.x0noz[1] + P.vnoz[1] * (double)t;
    ux = x;
    uy = y;
    hx = x - (double)P.nx * floor(x / (double)P.nx);
    hy = y - (double)P.ny * floor(y / (double)P.ny);
}

__host__ __device__ inline void make_geom(const DevParams &P, long long t, int first, StepGeom &g)
{
#pragma clang fp contract(off)
    g.t = t;
    g.first = first;
    double uxc = 0, uyc = 0, uxp = 0, uyp = 0;
    g.H.hx_c = g.H.hy_c = g.H.hx_p = g.H.hy_p = 0.0;
    if (P.has_nozzle) {
        head_axis(P, t, g.H.hx_c, g.H.hy_c, uxc, uyc);
        if (first) {
            g.H.hx_p = g.H.hx_c;
            g.H.hy_p = g.H.hy_c;
            uxp = uxc;
            uyp = uyc;
        } else {
            head_axis(P, t - 1, g.H.hx_p, g.H.hy_p, uxp, uyp);
        }
    }
    g.hb = Box3{0, 0, 0, 0, 0, 0};
    g.nbox = 1;
    g.bx[0] = g.bx[1] = g.bx[2] = Box3{0, 0, 0, 0, 0, 0};
    if (P.has_nozzle) {
        const double r = P.rout + 2.0;
        const double xl = fmin(uxp, uxc), xh = fmax(uxp, uxc), yl = fmin(uyp, uyc), yh = fmax(uyp, uyc);
        Box3 b;
        b.x0 = (int)floor(xl - r);
        b.y0 = (int)floor(yl - r);
        b.w = (int)ceil(xh + r) - b.x0 + 1;
        b.h = (int)ceil(yh + r) - b.y0 + 1;
        if (b.w > P.nx) {
            b.w = P.nx;
            b.x0 = 0;
        }
        if (b.h > P.ny) {
            b.h = P.ny;
            b.y0 = 0;
        }
        b.z0 = (int)floor(P.tip_z);
        if (b.z0 < 0) b.z0 = 0;
        b.d = P.nz - b.z0;
        g.hb = b;
        const int z0 = b.z0 - 1 > 0 ? b.z0 - 1 : 0;
        g.bx[0] = Box3{b.x0, b.y0, z0, b.w, b.h, P.nz - z0};
    }
    if (!P.periodic_z) {
        g.bx[g.nbox++] = Box3{0, 0, 0, P.nx, P.ny, 1};
        if (P.nz > 1) g.bx[g.nbox++] = Box3{0, 0, P.nz - 1, P.nx, P.ny, 1};
    }
}

// Cells whose pull touches a boundary (a z face or the head) are pulled with
// the boundary rules by the preparation kernel; every other cell has only
// fluid sources.
__device__ __forceinline__ bool in_box(const DevParams &P, const Box3 &B, int x, int y, int z)
{
    if (B.w <= 0) return false;
    int dx = x - B.x0, dy = y - B.y0;
    dx = ((dx % P.nx) + P.nx) % P.nx;
    dy = ((dy % P.ny) + P.ny) % P.ny;
    return dx < B.w && dy < B.h && z >= B.z0 && z < B.z0 + B.d;
}

__device__ __forceinline__ int wrap_any(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

// The next step's pull reads the bare moments of this step near boundaries
// only (wall density extrapolation, the pressure faces' velocity).
__device__ __forceinline__ bool macro_needed(const DevParams &P, const HeadPos &H, int x, int y, int z)
{
    if (!P.periodic_z && (z <= 2 || z >= P.nz - 3)) return true;
    if (!P.has_nozzle || (double)z < P.tip_z - 3.0) return false;
    double dx = fabs((double)x - H.hx_c), dy = fabs((double)y - H.hy_c);
    dx = fmin(dx, (double)P.nx - dx);
    dy = fmin(dy, (double)P.ny - dy);
    double lim = P.rout + 4.0;
    return dx <= lim && dy <= lim;
}

// Body of the single-role step kernel for block `bid` of `nblk` (the
// standalone kernel passes its own block index; the batched kernel the
// block's index within its simulation's share of the grid).
template <typename R, int TY, bool FIRST>
__device__ __forceinline__ void fused_body(const DevParams &P, StepGeom *__restrict__ G, const FusedGrid &FG,
                                           const R *__restrict__ src, R *__restrict__ dst,
                                           const double *__restrict__ momd_p, const R *__restrict__ mom_p,
                                           const R *__restrict__ chi_p, const R *__restrict__ ghost_p,
                                           R *__restrict__ mac_next_p, int bid, int nblk)
{
    // every array through global (not flat) instructions
    const auto momd = as_global(momd_p);
    const auto mom = as_global(mom_p);
    const auto chi = as_global(chi_p);
    const auto ghost = as_global(ghost_p);
    const auto mac_next = as_global(mac_next_p);
    constexpr int W = 66, HH = TY + 2, PL = W * HH, NI = TY * 64;
    const HeadPos H = G->H;
    const Box3 head = G->bx[0];
    // the last kernel of the step advances the device step counter (the
    // fields read above are not written by it)
    if (bid == 0 && threadIdx.x == 0) {
        G->t += 1;
        G->first = 0;
    }
    __shared__ R chi_l[4][3][PL];
    __shared__ double st_d[2][2][NI];
    __shared__ R st_r[2][10][NI];

    // XCD-aware order: consecutive blocks go round-robin over the 8 XCDs, so
    // block b handles tile (b % 8) * (nb / 8) + b / 8 and each XCD works on a
    // contiguous band of tiles.
    const int nb = nblk;
    const int b = bid;
    const int t = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
    const int tx = t % FG.ntx, ty = (t / FG.ntx) % FG.nty, tz = t / (FG.ntx * FG.nty);
    const int x0 = tx * 64, y0 = ty * TY, z0 = tz * FG.zlen;
    const int z1 = min(z0 + FG.zlen, P.nz);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;

    int cx, cy, row, col;
    bool active = true;
    if (wave < TY) {
        cx = x0 + lane;
        cy = y0 + wave;
        row = wave + 1;
        col = lane + 1;
    } else if (wave == TY) {
        cx = x0 + lane;
        cy = y0 - 1;
        row = 0;
        col = lane + 1;
    } else if (wave == TY + 1) {
        cx = x0 + lane;
        cy = y0 + TY;
        row = TY + 1;
        col = lane + 1;
    } else {
        if (lane < HH) {
            cx = x0 - 1;
            cy = y0 - 1 + lane;
            row = lane;
            col = 0;
        } else if (lane < 2 * HH) {
            cx = x0 + 64;
            cy = y0 - 1 + lane - HH;
            row = lane - HH;
            col = 65;
        } else {
            cx = x0;
            cy = y0;
            row = 0;
            col = 0;
            active = false;
        }
    }
    // tile cells outside the box are ring duty for the wrapped column
    const bool tile = active && wave < TY && cx < P.nx && cy < P.ny;
    const int xw = wrap_any(cx, P.nx), yw = wrap_any(cy, P.ny);
    const int lidx = row * W + col;
    const int ii = wave * 64 + lane;  // tile threads' state index
    const bool shell_c = active && !far_from_head(P, H.hx_c, H.hy_c, xw, yw) &&
                         column_class(P, H.hx_c, H.hy_c, xw, yw) == COL_SHELL;
    // the column's part of the "prepared" test (fixed for the march)
    const bool head_col = active && in_box(P, Box3{head.x0, head.y0, 0, head.w, head.h, P.nz}, xw, yw, 0);
    const long long col_off = (long long)yw * P.nx + xw;
    const long long plane_sz = (long long)P.nx * P.ny;
    const unsigned long long pstride = (unsigned long long)P.NP * sizeof(R);  // bytes per population plane
    bool ok1 = false, ok2 = false;  // plane p-1 / p-2 of this tile cell is fluid

    for (int p = z0 - 1; p <= z1 + 1; ++p) {
        // ---- 1. issue the bulk loads of plane p
        const bool load = active && p <= z1;
        int zp = p;
        bool ghost_plane = false;
        if (zp < 0 || zp >= P.nz) {
            if (P.periodic_z)
                zp = wrap_any(zp, P.nz);
            else
                ghost_plane = true;
        }
        const bool own = tile && p >= z0 && p < z1;
        const bool zface = !P.periodic_z && (zp == 0 || zp == P.nz - 1);
        const bool prep = load && !ghost_plane && (zface || (head_col && zp >= head.z0 && zp < head.z0 + head.d));
        const bool bulk = load && !ghost_plane && !prep;
        const long long cell = ghost_plane ? 0 : col_off + (long long)zp * plane_sz;
        R vT[lbq::Q], vY[lbq::Q];
        if (bulk)
            pull_bulk_issue<R, FIRST>(fresh_global_c(src), fresh_uniform(pstride),
                                      bulk_index<R>(P, xw, yw, zp), (unsigned)(cell * (long long)sizeof(R)), vT, vY);
        __builtin_amdgcn_sched_barrier(0);

        // ---- 2. collide plane c = p - 2 (stencil planes p - 3 .. p - 1)
        const int c = p - 2;
        if (ok2) {
            const int ss = c & 1;
            const int sm = (c + 3) & 3, s0 = c & 3, sp1 = (c + 1) & 3;
            Grad<R> G;
#pragma unroll
            for (int m = 0; m < 9; ++m) G.g[m] = R(0);
#pragma unroll
            for (int i = 1; i < lbq::Q; i += 2) {
                const int X = lbq::cx(i), Yc = lbq::cy(i), Z = lbq::cz(i);
                const int sa = Z > 0 ? sp1 : (Z < 0 ? sm : s0);
                const int sb = Z > 0 ? sm : (Z < 0 ? sp1 : s0);
                const int la = (row + Yc) * W + col + X, lb = (row - Yc) * W + col - X;
                const R kk = R(3.0 * lbq::w(i));
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    const R d = kk * (chi_l[sa][f][la] - chi_l[sb][f][lb]);
                    if (X) G.g[3 * f + 0] += X > 0 ? d : -d;
                    if (Yc) G.g[3 * f + 1] += Yc > 0 ? d : -d;
                    if (Z) G.g[3 * f + 2] += Z > 0 ? d : -d;
                }
            }
            CellState<R> C;
            C.drho = st_d[ss][0][ii];
            C.rY = st_d[ss][1][ii];
#pragma unroll
            for (int a = 0; a < 3; ++a) C.j[a] = st_r[ss][a][ii];
#pragma unroll
            for (int a = 0; a < 6; ++a) C.Pi[a] = st_r[ss][3 + a][ii];
            C.om = st_r[ss][9][ii];
            const long long ccell = col_off + (long long)c * plane_sz;
            R rY, rB, u[3];
            collide_state<R>(P, C, G, c, reinterpret_cast<char *>(dst), pstride,
                             (unsigned)(ccell * (long long)sizeof(R)), rY, rB, u);
            if (macro_needed(P, H, xw, yw, c)) {
                const long long a = aidx(P, xw, yw, c), NA = P.NA;
                mac_next[a] = rY;
                mac_next[NA + a] = rB;
                mac_next[2 * NA + a] = u[0];
                mac_next[3 * NA + a] = u[1];
                mac_next[4 * NA + a] = u[2];
            }
        }
        __builtin_amdgcn_sched_barrier(0);

        // ---- 3. reduce plane p: colour fields and the tile cell's state
        bool cur_ok = false;
        if (load) {
            R cN, cY, cB;
            if (ghost_plane) {
                const long long plane = (long long)P.nx * P.ny;
                const int face = zp < 0 ? 0 : 1;
                const long long gc = (long long)yw * P.nx + xw;
                cN = ghost[(face * 3 + 0) * plane + gc];
                cY = ghost[(face * 3 + 1) * plane + gc];
                cB = ghost[(face * 3 + 2) * plane + gc];
            } else {
                Mom<R> M;
                mom_zero(M);
                bool fluid = true;
                if (prep) {
                    // boundary cell (pulled with the boundary rules), head
                    // solid (wall densities) or node just created
                    const long long a = aidx(P, xw, yw, zp), NA = P.NA;
                    cN = chi[a];
                    cY = chi[NA + a];
                    cB = chi[2 * NA + a];
                    fluid = !(shell_c && (double)zp >= P.tip_z);
                    if (own && fluid) {
                        M.dm[0] = momd[a];
                        M.dm[1] = momd[NA + a];
#pragma unroll
                        for (int m = 2; m < NMOM; ++m) M.m[m] = mom[(m - 2) * NA + a];
                    }
                } else {
                    if (own)
                        mom_add_all<R, true>(M, vT, vY);
                    else
                        mom_add_all<R, false>(M, vT, vY);
                    chi_of<R>(P, R(M.dm[1]), R(P.rho_ref + M.dm[0] - M.dm[1]), cN, cY, cB);
                }
                if (own && fluid) {
                    const CellState<R> C = cell_state<R>(P, M);
                    const int ss = p & 1;
                    st_d[ss][0][ii] = C.drho;
                    st_d[ss][1][ii] = C.rY;
#pragma unroll
                    for (int a = 0; a < 3; ++a) st_r[ss][a][ii] = C.j[a];
#pragma unroll
                    for (int a = 0; a < 6; ++a) st_r[ss][3 + a][ii] = C.Pi[a];
                    st_r[ss][9][ii] = C.om;
                    cur_ok = true;
                }
            }
            const int cs = p & 3;
            chi_l[cs][0][lidx] = cN;
            chi_l[cs][1][lidx] = cY;
            chi_l[cs][2][lidx] = cB;
        }
        ok2 = ok1;
        ok1 = cur_ok;
        __syncthreads();
    }
}

template <typename R, int TY, bool FIRST>
__global__ __launch_bounds__((TY + 3) * 64, 2) void k_fused(DevParams P, StepGeom *__restrict__ G,
                                                            FusedGrid FG, const R *__restrict__ src,
                                                            R *__restrict__ dst,
                                                            const double *__restrict__ momd,
                                                            const R *__restrict__ mom, const R *__restrict__ chi,
                                                            const R *__restrict__ ghost, R *__restrict__ mac_next)
{
    fused_body<R, TY, FIRST>(P, G, FG, src, dst, momd, mom, chi, ghost, mac_next, blockIdx.x, gridDim.x);
}

// Producer/consumer form of the march.  Waves 0 .. TY + 2 are loaders (the
// tile rows, the two ring rows, the two ring columns as above): they pull and
// reduce plane p, keeping the loads of plane p + 1 in flight meanwhile (FP32),
// and write the colour fields and the tile cells' raw moments to LDS.
// The following TY / CR waves are colliders, CR tile rows each: in the same
// iteration they take plane p - 2 (stencil planes p - 3 .. p - 1, all reduced
// in earlier iterations) from its moments to its 38 stored values, the local
// relaxation time included.  One barrier per
// plane.  Loads and stores are issued by different waves, so neither waits
// behind the other in a wave's queue of outstanding memory operations.
template <typename R, int TY, bool FIRST, int ST = ST_PLAIN, int CR = 1>
__device__ __forceinline__ void fused_pc_body(const DevParams &P, StepGeom *__restrict__ G, const FusedGrid &FG,
                                              const void *__restrict__ src, void *__restrict__ dst,
                                              const double *__restrict__ momd_p, const R *__restrict__ mom_p,
                                              const R *__restrict__ chi_p, const R *__restrict__ ghost_p,
                                              R *__restrict__ mac_next_p, const float *__restrict__ mo_src_p,
                                              float *__restrict__ mo_dst, int bid, int nblk)
{
    // every array through global (not flat) instructions
    const auto momd = as_global(momd_p);
    const auto mom = as_global(mom_p);
    const auto chi = as_global(chi_p);
    const auto ghost = as_global(ghost_p);
    const auto mac_next = as_global(mac_next_p);
    const auto mo_src = as_global(mo_src_p);
    // E: stored element type; reduced storage keeps 16-bit deviations and
    // decodes them with the source cells' moments (an LDS ring of planes, the
    // tile with a two-cell halo: the ring cells' sources included)
    typedef typename std::conditional<ST == ST_PLAIN, R, unsigned>::type E;
    constexpr int W = 66, HH = TY + 2, PL = W * HH, NI = TY * 64;
    constexpr int MW = 68, MH = TY + 4, MR = MW * MH;  // moment region: x0-2 .. x0+65, y0-2 .. y0+TY+1
    constexpr bool DEEP = sizeof(R) == 4;
    // the ring keeps each source cell's equilibrium coefficients (EqCell:
    // t_rho, t_Y, a_T, a_Y, 3u), formed once per cell as it is written
    constexpr int NEQ = 7;
    __shared__ float mring[ST == ST_PLAIN ? 1 : 4][NEQ][ST == ST_PLAIN ? 1 : MR];
    const HeadPos H = G->H;
    const Box3 head = G->bx[0];
    // the last kernel of the step advances the device step counter (the
    // fields read above are not written by it)
    if (bid == 0 && threadIdx.x == 0) {
        G->t += 1;
        G->first = 0;
    }
    __shared__ R chi_l[4][3][PL];
    __shared__ double mo_d[4][2][NI];      // masses delta rho, rho_Y (FP64)
    __shared__ R mo_r[4][NMOMR][NI];       // the other raw moments m[2..16]
    __shared__ unsigned char st_ok[4][NI];

    const int nb = nblk;
    const int b = bid;
    const int t = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
    const int tx = t % FG.ntx, ty = (t / FG.ntx) % FG.nty, tz = t / (FG.ntx * FG.nty);
    const int x0 = tx * 64, y0 = ty * TY, z0 = tz * FG.zlen;
    const int z1 = min(z0 + FG.zlen, P.nz);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long plane_sz = (long long)P.nx * P.ny;
    const unsigned long long pstride = (unsigned long long)P.NP * sizeof(E);

    if (wave >= TY + 3) {
        // ---------------- collider: tile rows r0, r0 + TY / CR, ... (CR rows)
        const int r0 = wave - (TY + 3);
        // every wave of the block passes the same barriers: one after the
        // loaders' prologue, then one per plane
        __syncthreads();
        for (int p = z0 - 1; p <= z1 + 1; ++p) {
            const int c = p - 2;
#pragma unroll 1
            for (int k = 0; k < CR; ++k) {
            const int r = r0 + k * (TY / CR);
            const int cx = x0 + lane, cy = y0 + r;
            const bool tile = cx < P.nx && cy < P.ny;
            const int xw = wrap_any(cx, P.nx), yw = wrap_any(cy, P.ny);
            const int row = r + 1, col = lane + 1;
            const int ii = r * 64 + lane;
            const long long col_off = (long long)yw * P.nx + xw;
            if (tile && c >= z0 && st_ok[c & 3][ii]) {
                const int ss = c & 3;
                const int sm = (c + 3) & 3, s0 = c & 3, sp1 = (c + 1) & 3;
                // the local relaxation time first, then the colour stencil:
                // the solve's temporaries and the stencil's reads do not
                // overlap (register pressure)
                CellState<R> C;
                {
                    Mom<R> M;
                    M.dm[0] = mo_d[ss][0][ii];
                    M.dm[1] = mo_d[ss][1][ii];
#pragma unroll
                    for (int m = 2; m < NMOM; ++m) M.m[m] = mo_r[ss][m - 2][ii];
                    C = cell_state<R>(P, M);
                }
                __builtin_amdgcn_sched_barrier(0);
                Grad<R> G;
#pragma unroll
                for (int m = 0; m < 9; ++m) G.g[m] = R(0);
#pragma unroll
                for (int i = 1; i < lbq::Q; i += 2) {
                    const int X = lbq::cx(i), Yc = lbq::cy(i), Z = lbq::cz(i);
                    const int sa = Z > 0 ? sp1 : (Z < 0 ? sm : s0);
                    const int sb = Z > 0 ? sm : (Z < 0 ? sp1 : s0);
                    const int la = (row + Yc) * W + col + X, lb = (row - Yc) * W + col - X;
                    const R kk = R(3.0 * lbq::w(i));
#pragma unroll
                    for (int f = 0; f < 3; ++f) {
                        const R d = kk * (chi_l[sa][f][la] - chi_l[sb][f][lb]);
                        if (X) G.g[3 * f + 0] += X > 0 ? d : -d;
                        if (Yc) G.g[3 * f + 1] += Yc > 0 ? d : -d;
                        if (Z) G.g[3 * f + 2] += Z > 0 ? d : -d;
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
                const long long ccell = col_off + (long long)c * plane_sz;
                R rY, rB, u[3];
                collide_state<R, ST>(P, C, G, c, reinterpret_cast<char *>(dst), pstride,
                                     (unsigned)(ccell * (long long)sizeof(E)), rY, rB, u, mo_dst, ccell);
                if (macro_needed(P, H, xw, yw, c)) {
                    const long long a = aidx(P, xw, yw, c), NA = P.NA;
                    mac_next[a] = rY;
                    mac_next[NA + a] = rB;
                    mac_next[2 * NA + a] = u[0];
                    mac_next[3 * NA + a] = u[1];
                    mac_next[4 * NA + a] = u[2];
                }
            }
            }
            __syncthreads();
        }
        return;
    }

    // ---------------- loader: tile row, ring row or ring columns
    int cx, cy, row, col;
    bool active = true;
    if (wave < TY) {
        cx = x0 + lane;
        cy = y0 + wave;
        row = wave + 1;
        col = lane + 1;
    } else if (wave == TY) {
        cx = x0 + lane;
        cy = y0 - 1;
        row = 0;
        col = lane + 1;
    } else if (wave == TY + 1) {
        cx = x0 + lane;
        cy = y0 + TY;
        row = TY + 1;
        col = lane + 1;
    } else {
        if (lane < HH) {
            cx = x0 - 1;
            cy = y0 - 1 + lane;
            row = lane;
            col = 0;
        } else if (lane < 2 * HH) {
            cx = x0 + 64;
            cy = y0 - 1 + lane - HH;
            row = lane - HH;
            col = 65;
        } else {
            cx = x0;
            cy = y0;
            row = 0;
            col = 0;
            active = false;
        }
    }
    const bool tile = active && wave < TY && cx < P.nx && cy < P.ny;
    const int xw = wrap_any(cx, P.nx), yw = wrap_any(cy, P.ny);
    const int lidx = row * W + col;
    const int ii = wave * 64 + lane;
    const bool shell_c = active && !far_from_head(P, H.hx_c, H.hy_c, xw, yw) &&
                         column_class(P, H.hx_c, H.hy_c, xw, yw) == COL_SHELL;
    const bool head_col = active && in_box(P, Box3{head.x0, head.y0, 0, head.w, head.h, P.nz}, xw, yw, 0);
    const long long col_off = (long long)yw * P.nx + xw;

    struct PlaneJob {
        bool load, ghost, prep, bulk, own;
        int zp;
        long long cell;
    };
    auto job = [&](int p) {
        PlaneJob J;
        J.load = active && p <= z1;
        J.zp = p;
        J.ghost = false;
        if (p < 0 || p >= P.nz) {
            if (P.periodic_z)
                J.zp = wrap_any(p, P.nz);
            else
                J.ghost = true;
        }
        J.own = tile && p >= z0 && p < z1;
        const bool zface = !P.periodic_z && (J.zp == 0 || J.zp == P.nz - 1);
        J.prep = J.load && !J.ghost && (zface || (head_col && J.zp >= head.z0 && J.zp < head.z0 + head.d));
        J.bulk = J.load && !J.ghost && !J.prep;
        J.cell = J.ghost ? 0 : col_off + (long long)J.zp * plane_sz;
        return J;
    };
    auto issue = [&](int p, E(&vT)[lbq::Q], E(&vY)[lbq::Q]) {
        const PlaneJob J = job(p);
        if (J.bulk) {
            if constexpr (ST == ST_PLAIN)
                pull_bulk_issue<E, FIRST>(fresh_global_c(reinterpret_cast<const E *>(src)), fresh_uniform(pstride),
                                          bulk_index<E>(P, xw, yw, J.zp), (unsigned)(J.cell * (long long)sizeof(E)),
                                          vT, vY);
            else
                pull_bulk_issue_words<FIRST>(fresh_global_c(reinterpret_cast<const E *>(src)), fresh_uniform(pstride),
                                             bulk_index<E>(P, xw, yw, J.zp), (unsigned)(J.cell * (long long)sizeof(E)),
                                             vT);
        }
    };

    // moment ring (reduced storage): this thread's share of the region, two
    // cells at most, loaded one iteration before they are written to LDS
    const int lx = cx - x0, ly = cy - y0;  // tile-relative position (ring: -1 / 64, -1 / TY)
    float mreg[2][NMO];
    auto m_issue = [&](int q) {
        if constexpr (ST != ST_PLAIN) {
            int zq = q;
            const bool ok = P.periodic_z || (q >= 0 && q < P.nz);
            if (P.periodic_z) zq = wrap_any(q, P.nz);
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int k = threadIdx.x + r * (TY + 3) * 64;
                if (ok && k < MR) {
                    const int mx = wrap_any(x0 - 2 + k % MW, P.nx), my = wrap_any(y0 - 2 + k / MW, P.ny);
                    const long long mc = (long long)zq * plane_sz + (long long)my * P.nx + mx;
#pragma unroll
                    for (int m = 0; m < NMO; ++m) mreg[r][m] = mo_src[m * P.NM + mc];
                }
            }
        }
    };
    auto m_write = [&](int q) {
        if constexpr (ST != ST_PLAIN) {
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int k = threadIdx.x + r * (TY + 3) * 64;
                if (k < MR) {
                    const EqCell ec = eq_cell(P, mreg[r][0], mreg[r][1], mreg[r][2], mreg[r][3], mreg[r][4]);
                    mring[q & 3][0][k] = ec.tr;
                    mring[q & 3][1][k] = ec.ty;
                    mring[q & 3][2][k] = ec.aT;
                    mring[q & 3][3][k] = ec.aY;
                    mring[q & 3][4][k] = ec.ux3;
                    mring[q & 3][5][k] = ec.uy3;
                    mring[q & 3][6][k] = ec.uz3;
                }
            }
        }
    };
    // decode of link I of the pulled cell at plane p (reduced storage)
    // coefficients of link I's source cell for the pulled cell at plane p
    // (reduced storage)
    auto coef = [&]<int I>(int p) {
        constexpr int X = lbq::cx(I), Yc = lbq::cy(I), Z = lbq::cz(I);
        const int sl = FIRST ? (p & 3) : ((p - Z) & 3);
        const int k = FIRST ? (ly + 2) * MW + lx + 2 : (ly + 2 - Yc) * MW + lx + 2 - X;
        return EqCell{mring[sl][0][k], mring[sl][1][k], mring[sl][2][k], mring[sl][3][k],
                      mring[sl][4][k], mring[sl][5][k], mring[sl][6][k]};
    };

    auto reduce = [&](int p, const E(&vT)[lbq::Q], const E(&vY)[lbq::Q]) {
        const PlaneJob J = job(p);
        if (!J.load) return;
        R cN, cY, cB;
        bool cur_ok = false;
        if (J.ghost) {
            const int face = p < 0 ? 0 : 1;
            const long long gc = (long long)yw * P.nx + xw;
            cN = ghost[(face * 3 + 0) * plane_sz + gc];
            cY = ghost[(face * 3 + 1) * plane_sz + gc];
            cB = ghost[(face * 3 + 2) * plane_sz + gc];
        } else {
            Mom<R> M;
            mom_zero(M);
            bool fluid = true;
            if (J.prep) {
                const long long a = aidx(P, xw, yw, J.zp), NA = P.NA;
                cN = chi[a];
                cY = chi[NA + a];
                cB = chi[2 * NA + a];
                fluid = !(shell_c && (double)J.zp >= P.tip_z);
                if (J.own && fluid) {
                    M.dm[0] = momd[a];
                    M.dm[1] = momd[NA + a];
#pragma unroll
                    for (int m = 2; m < NMOM; ++m) M.m[m] = mom[(m - 2) * NA + a];
                }
            } else {
                // one code path for tile and ring cells (a branch here lets
                // the compiler hoist all 38 FP64 conversions above it)
                if constexpr (ST == ST_PLAIN) {
                    mom_add_all<R, true>(M, vT, vY);
                } else {
                    // the rest link, then one opposite pair at a time; the
                    // LDS reads of the next pair's coefficients are issued
                    // before the current pair is decoded, so their latency
                    // overlaps that arithmetic.  Ring cells need only the two
                    // masses (their colour fields); the branch is uniform per
                    // wave.
                    auto decode_all = [&]<bool FULL>() {
                        EqCell nA = coef.template operator()<1>(p), nB = coef.template operator()<2>(p);
                        {
                            R T, Y;
                            dec_link<ST, 0>(P, coef.template operator()<0>(p), vT[0], T, Y);
                            mom_add<R, 0, FULL>(M, T, Y);
                            __builtin_amdgcn_sched_barrier(0);
                        }
                        [&]<int... K>(std::integer_sequence<int, K...>) {
                            (
                                [&] {
                                    constexpr int I = 2 * K + 1;
                                    const EqCell cA = nA, cB = nB;
                                    if constexpr (I + 2 < lbq::Q) {
                                        nA = coef.template operator()<I + 2>(p);
                                        nB = coef.template operator()<I + 3>(p);
                                    }
                                    R Ta, Ya, Tb, Yb;
                                    dec_link<ST, I>(P, cA, vT[I], Ta, Ya);
                                    dec_link<ST, I + 1>(P, cB, vT[I + 1], Tb, Yb);
                                    mom_add_pair<R, I, FULL>(M, Ta, Ya, Tb, Yb);
                                    __builtin_amdgcn_sched_barrier(0);
                                }(),
                                ...);
                        }(std::make_integer_sequence<int, (lbq::Q - 1) / 2>{});
                    };
                    if (wave < TY)
                        decode_all.template operator()<true>();
                    else
                        decode_all.template operator()<false>();
                }
                chi_of<R>(P, R(M.dm[1]), R(P.rho_ref + M.dm[0] - M.dm[1]), cN, cY, cB);
            }
            if (J.own && fluid) {
                const int ss = p & 3;
                mo_d[ss][0][ii] = M.dm[0];
                mo_d[ss][1][ii] = M.dm[1];
#pragma unroll
                for (int m = 2; m < NMOM; ++m) mo_r[ss][m - 2][ii] = M.m[m];
                cur_ok = true;
            }
        }
        const int cs = p & 3;
        chi_l[cs][0][lidx] = cN;
        chi_l[cs][1][lidx] = cY;
        chi_l[cs][2][lidx] = cB;
        if (wave < TY) st_ok[p & 3][ii] = cur_ok ? 1 : 0;
    };

    E aT[lbq::Q], aY[lbq::Q];
    if constexpr (!DEEP) {
        __syncthreads();
        for (int p = z0 - 1; p <= z1 + 1; ++p) {
            issue(p, aT, aY);
            __builtin_amdgcn_sched_barrier(0);
            reduce(p, aT, aY);
            __syncthreads();
        }
        return;
    }
    E bT[lbq::Q], bY[lbq::Q];
    if constexpr (ST != ST_PLAIN) {
        // moments of planes z0 - 2 .. z0 in LDS, z0 + 1 in registers
        for (int q = z0 - 2; q <= z0; ++q) {
            m_issue(q);
            m_write(q);
        }
        m_issue(z0 + 1);
    }
    issue(z0 - 1, aT, aY);
    __syncthreads();
    for (int p = z0 - 1; p <= z1 + 1; p += 2) {
        m_write(p + 2);
        m_issue(p + 3);
        issue(p + 1, bT, bY);
        __builtin_amdgcn_sched_barrier(0);
        reduce(p, aT, aY);
        __syncthreads();
        if (p + 1 > z1 + 1) break;
        m_write(p + 3);
        m_issue(p + 4);
        issue(p + 2, aT, aY);
        __builtin_amdgcn_sched_barrier(0);
        reduce(p + 1, bT, bY);
        __syncthreads();
    }
}

template <typename R, int TY, bool FIRST, int ST = ST_PLAIN, int CR = 1>
__global__ __launch_bounds__((TY + 3 + TY / CR) * 64, 1) void k_fused_pc(DevParams P, StepGeom *__restrict__ G,
                                                                  FusedGrid FG, const void *__restrict__ src,
                                                                  void *__restrict__ dst,
                                                                  const double *__restrict__ momd,
                                                                  const R *__restrict__ mom,
                                                                  const R *__restrict__ chi,
                                                                  const R *__restrict__ ghost,
                                                                  R *__restrict__ mac_next,
                                                                  const float *__restrict__ mo_src,
                                                                  float *__restrict__ mo_dst)
{
    fused_pc_body<R, TY, FIRST, ST, CR>(P, G, FG, src, dst, momd, mom, chi, ghost, mac_next, mo_src, mo_dst,
                                        blockIdx.x, gridDim.x);
}

}  // namespace lbk
