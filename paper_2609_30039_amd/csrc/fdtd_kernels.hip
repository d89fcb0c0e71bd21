// fdtd_kernels.hip -- HIP kernels of libfdtd for gfx950 (MI355X).
//
// The Yee step is memory bound (~1 flop per byte against a machine balance of
// ~20 flop/B), so there is no matrix-core work: kernels are built around
// coalesced x-fastest rows, z-marching columns that keep the previous plane in
// registers, XCD-aware block placement and state sets that a step reads and
// writes separately.
//
// Two kernel families compute bitwise-identical results (same per-node
// functions, no implicit contraction):
//   split  one launch for the E update and one for the H update (their
//          transposes for the adjoint); the simple reference path;
//   fused  a single pass per step: a block of 4 waves covers 64 x-columns by
//          4R rows, marches z, computes E^{n+1} on its tile plus a one-cell
//          halo and H^{n+3/2} on the 62 x (4R-2) interior it owns; x
//          neighbours travel by lane shuffles, y neighbours across waves by a
//          double-buffered LDS row, z neighbours stay in registers.
#include <hip/hip_runtime.h>
#include <float.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "fdtd_dev.h"
#include "fdtd_launch.h"

namespace fdtd {

// ------------------------------------------------------------ block mapping
// Workgroups are dispatched round-robin over the 8 XCDs; remap so that each
// XCD receives a contiguous run of logical tiles (neighbouring tiles then
// share that XCD's L2).
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int X = 8;
    int x = b % X, idx = b / X;
    int q = nb / X, r = nb % X;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + idx;
}

__device__ __forceinline__ int find_domain(const int* __restrict__ bs, int ndom, int b) {
    int lo = 0, hi = ndom;   // bs[lo] <= b < bs[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (bs[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

struct Col {
    int i, j, k0, k1, x0, y0;
    bool ok;
};

// split kernels: 256 threads = W (x) by 256 / W (y) columns, z chunk of length
// kz.  Column blocks are numbered domain by domain, x fastest, then rows,
// then z chunks; xr[0..7] / xr[8..15] are the start and length of the run of
// them that XCD x takes (the dispatcher sends workgroup b to XCD b % 8), cut
// by the host into runs of equal estimated cost.  braw: the workgroup among
// the column blocks (blockIdx.x when negative); beyond its run's end it idles.
template <typename T, int W>
__device__ __forceinline__ Col column(const DomDev<T>* doms, const int* bs, int ndom, int kz, const DomDev<T>*& dp,
                                      const int* __restrict__ xr, int braw = -1) {
    constexpr int NR = 256 / W;
    Col c;
    const int raw = braw < 0 ? (int)blockIdx.x : braw, xcd = raw & 7, m = raw >> 3;
    if (m >= xr[8 + xcd]) {
        dp = doms;
        c.ok = false;
        return c;
    }
    int b = xr[xcd] + m;
    int dom = find_domain(bs, ndom, b);
    dp = doms + dom;
    const DomDev<T>& d = *dp;
    int lb = b - bs[dom];
    int nbx = (d.n[0] + W - 1) / W, nby = (d.n[1] + NR - 1) / NR;
    int bx = lb % nbx;
    int r = lb / nbx;
    int by = r % nby, bz = r / nby;
    c.x0 = bx * W;
    c.y0 = by * NR;
    c.i = c.x0 + (int)(threadIdx.x % W);
    c.j = c.y0 + (int)(threadIdx.x / W);
    c.k0 = bz * kz;
    c.k1 = min(c.k0 + kz, d.n[2]);
    c.ok = c.i < d.n[0] && c.j < d.n[1];
    return c;
}

// Tile-table columns of the split adjoint.  A tile is (domain | class << 24,
// x0 | xlen << 24, y0, k0) and covers W x-columns by 256 / W rows: W = 32 (8 rows, two rows
// per wave) inside, W = 16 (16 rows) for the narrow x-slab zones.  Columns
// at or beyond x0 + xlen are idle.
template <int W>
struct TileCol {
    int i, j, k0, k1, x0, y0;
    bool ok;
};

template <typename T, int W>
__device__ __forceinline__ TileCol<W> tile_column(const DomDev<T>* doms, const int4 e, int kz, const DomDev<T>*& dp) {
    TileCol<W> c;
    dp = doms + (e.x & 0xFFFFFF);
    const DomDev<T>& d = *dp;
    const int xlen = e.y >> 24, lx = (int)(threadIdx.x % W);
    c.x0 = e.y & 0xFFFFFF;
    c.y0 = e.z;
    c.i = c.x0 + lx;
    c.j = e.z + (int)(threadIdx.x / W);
    c.k0 = e.w;
    c.k1 = min(e.w + kz, d.n[2]);
    c.ok = lx < xlen && c.j < d.n[1];
    return c;
}

// ------------------------------------------------------------ per-axis views
// Absorber coefficients of one index along an axis, eps^-1 over a block, and
// absorber memories fetched ahead: shared by the split and the plain tile
// kernels, whose node arithmetic is that of e_update / h_update.
template <typename T>
struct EpsView {
    int mode;                   // 0 background everywhere, 1 inside the eps box, 2 partial
    int diag;
    const FDTD_GLOBAL T* p[3];
    int lo[3], hi[3], ex, ey;   // ex: the stored row length, ey: the box's rows per plane
    int exa;                    // x of a stored row's first element
    T bg;
};

template <typename T>
__device__ __forceinline__ EpsView<T> eps_view(const DomDev<T>& d, int X0, int Y0, int NR, int klo, int khi) {
    EpsView<T> v;
    v.diag = d.eps_diag;
    v.bg = d.epsinv_bg;
    for (int c = 0; c < 3; ++c) v.p[c] = gp(d.epsinv[c]);
    for (int a = 0; a < 3; ++a) {
        v.lo[a] = d.elo[a];
        v.hi[a] = d.ehi[a];
    }
    v.ex = d.exs;
    v.exa = d.exa;
    v.ey = d.ehi[1] - d.elo[1];
    int lo[3] = {X0, Y0, klo}, hi[3] = {X0 + 63, Y0 + NR - 1, khi};
    bool inside = true, outside = false;
    for (int a = 0; a < 3; ++a) {
        if (lo[a] < d.elo[a] || hi[a] >= d.ehi[a]) inside = false;
        if (hi[a] < d.elo[a] || lo[a] >= d.ehi[a]) outside = true;
    }
    v.mode = outside ? 0 : (inside ? 1 : 2);
    return v;
}

// eps^-1 of the three components at (i, j, k)
template <typename T>
__device__ __forceinline__ void eps_at(const EpsView<T>& v, int i, int j, int k, T out[3]) {
    bool in = v.mode == 1 || (v.mode == 2 && i >= v.lo[0] && i < v.hi[0] && j >= v.lo[1] && j < v.hi[1] &&
                              k >= v.lo[2] && k < v.hi[2]);
    if (!in) {
        out[0] = out[1] = out[2] = v.bg;
        return;
    }
    int q = ((k - v.lo[2]) * v.ey + (j - v.lo[1])) * v.ex + (i - v.exa);
    out[0] = v.p[0][q];
    if (v.diag) {
        out[1] = v.p[1][q];
        out[2] = v.p[2][q];
    } else {
        out[1] = out[2] = out[0];
    }
}

template <typename T>
struct Cpml1 {
    int side;                  // -1 outside the slabs
    int idx;                   // index along the axis
    T bE, cE, kE, bH, cH, kH;
};

template <typename T>
__device__ __forceinline__ Cpml1<T> cpml_at(const DomDev<T>& d, int a, int x) {
    Cpml1<T> c;
    c.idx = x;
    c.side = (x >= 0 && x < d.n[a]) ? slab_side(d, a, x) : -1;
    c.bE = c.cE = c.kE = c.bH = c.cH = c.kH = T(0);
    if (c.side >= 0) {
        const FDTD_GLOBAL T* tb = gp(d.tab[a]);
        int n = d.n[a];
        c.bE = tb[x];
        c.cE = tb[n + x];
        c.kE = tb[2 * n + x];
        c.bH = tb[3 * n + x];
        c.cH = tb[4 * n + x];
        c.kH = tb[5 * n + x];
    }
    return c;
}

// psi slab offset of node (i,j,k) on axis a, side s (32-bit)
template <typename T>
__device__ __forceinline__ int poff(const DomDev<T>& d, int a, int s, int i, int j, int k) {
    int L = d.L[a][s];
    if (a == 0) return (k * d.n[1] + j) * L + (s ? i - (d.n[0] - L) : i);
    if (a == 1) return (k * L + (s ? j - (d.n[1] - L) : j)) * d.n[0] + i;
    return ((s ? k - (d.n[2] - L) : k) * d.n[1] + j) * d.n[0] + i;
}

// one stretched term: psi_new = b psi + c D; D/kappa + psi_new (as stretch())
template <typename T>
__device__ __forceinline__ T st_term(T* base, long long rso, long long wso, bool own, T b, T c, T ki, T D) {
    FDTD_GLOBAL T* g = gp(base);
    T pn = fma(b, g[rso], c * D);
    if (own) g[wso] = pn;
    return fma(ki, D, pn);
}

// psi memories of the six terms of one node, slots ordered
// 0: y-slab term of Ex (E) / Hx (H), 1: y-slab term of Ez / Hz,
// 2: z-slab term of Ey / Hy, 3: z-slab term of Ex / Hx,
// 4: x-slab term of Ez / Hz, 5: x-slab term of Ey / Hy.
// (E side: Ex t0, Ez t1, Ey t0, Ex t1, Ez t0, Ey t1; H side: Hx t0, Hz t1,
// Hy t0, Hx t1, Hz t0, Hy t1.)
template <typename T>
__device__ __forceinline__ void psi_load(const DomDev<T>& d, T* const (&psi)[3][2][2], long long so, bool v,
                                         const Cpml1<T>& cx, const Cpml1<T>& cy, const Cpml1<T>& cz, int i, int j, int k,
                                         T out[6]) {
    for (int q = 0; q < 6; ++q) out[q] = T(0);
    if (!v) return;
    if (cy.side >= 0) {
        int o = poff(d, 1, cy.side, i, j, k);
        out[0] = gp(psi[1][cy.side][0] + so)[o];
        out[1] = gp(psi[1][cy.side][1] + so)[o];
    }
    if (cz.side >= 0) {
        int o = poff(d, 2, cz.side, i, j, k);
        out[2] = gp(psi[2][cz.side][0] + so)[o];
        out[3] = gp(psi[2][cz.side][1] + so)[o];
    }
    if (cx.side >= 0) {
        int o = poff(d, 0, cx.side, i, j, k);
        out[4] = gp(psi[0][cx.side][0] + so)[o];
        out[5] = gp(psi[0][cx.side][1] + so)[o];
    }
}

// stretched term from a prefetched memory: psi_new = b psi + c D (stored by
// the owner), returns D/kappa + psi_new (the arithmetic of stretch())
template <typename T>
__device__ __forceinline__ T st_pref(T* base, long long wso, int off, bool own, T b, T c, T ki, T psi, T D) {
    T pn = fma(b, psi, c * D);
    if (own) gp(base + wso)[off] = pn;
    return fma(ki, D, pn);
}

// ============================================================ forward, split
// One thread per (i, j) column marching its z chunk, one launch for E and one
// for H.  Absorber coefficients are loaded once per column (x, y) and per
// plane (z, block-uniform); the next plane's operands, absorber memories
// included, are fetched before the current plane is computed and stored, so
// a wave keeps a plane of loads in flight while it works (the compiler cannot
// hoist loads above the stores: it cannot tell the state arrays apart).
// Blocks that touch no absorber slab skip the memories; Lorentz cells take
// the general e_update_v.  With rs == ws the kernels update in place: every
// value a thread writes is read only by that thread.
struct BlkFlags {
    bool cp, lor;
};

// A block of the single-pass family: its cells, their +x, +y, +z neighbours
// (whose E^{n+1} its H updates read, recomputed in the block) and their
// -x, -y, -z neighbours (whose H its E updates read) lie off every absorbing
// slab, wall node and dispersive box, so every update there is the plain
// Yee one.  The split kernels skip exactly these blocks in that family.
template <typename T>
__device__ __forceinline__ bool blk_interior(const DomDev<T>& d, int x0, int y0, int k0, int k1, int w, int nr) {
    if (!d.onep) return false;
    const int lo[3] = {x0, y0, k0}, hi[3] = {x0 + w, y0 + nr, k1};   // hi: the +1 neighbours, inclusive
    bool lor = d.has_lor;
    for (int a = 0; a < 3; ++a) {
        if (lo[a] < max(1, d.L[a][0]) || hi[a] >= d.n[a] - d.L[a][1]) return false;
        if (hi[a] < d.llo[a] || lo[a] >= d.lhi[a]) lor = false;
    }
    return !lor;
}

template <typename T>
__device__ __forceinline__ BlkFlags blk_flags(const DomDev<T>& d, int x0, int y0, int k0, int k1, int w = 64,
                                              int nr = 4) {
    int lo[3] = {x0, y0, k0}, hi[3] = {min(x0 + w - 1, d.n[0] - 1), min(y0 + nr - 1, d.n[1] - 1), k1 - 1};
    BlkFlags f;
    f.cp = false;
    for (int a = 0; a < 3; ++a)
        if (lo[a] < d.L[a][0] || hi[a] >= d.n[a] - d.L[a][1]) f.cp = true;
    f.lor = d.has_lor;
    for (int a = 0; a < 3; ++a)
        if (hi[a] < d.llo[a] || lo[a] >= d.lhi[a]) f.lor = false;
    return f;
}

template <typename T>
struct ColE {
    T hx, hy, hz, hy_xm, hz_xm, hx_ym, hz_ym;   // H^{n+1/2} at the node and one step back along x and y
    T e[3], ei[3];                               // E^n and eps^-1 at the node
    T ps[6];                                     // E-side absorber memories (psi_load order)
};

template <typename T>
__device__ __forceinline__ void cole_fetch(const DomDev<T>& d, ColE<T>& p, const FDTD_GLOBAL T* const (&h)[3],
                                           const FDTD_GLOBAL T* const (&e)[3], long long f, const EpsView<T>& ev,
                                           bool cp, const Cpml1<T>& cx, const Cpml1<T>& cy, long long so, int i,
                                           int j, int k) {
    p.hx = h[0][f];
    p.hy = h[1][f];
    p.hz = h[2][f];
    p.hy_xm = nb_back(d, h[1], f, 0, i);
    p.hz_xm = nb_back(d, h[2], f, 0, i);
    p.hx_ym = nb_back(d, h[0], f, 1, j);
    p.hz_ym = nb_back(d, h[2], f, 1, j);
    p.e[0] = e[0][f];
    p.e[1] = e[1][f];
    p.e[2] = e[2][f];
    eps_at(ev, i, j, k, p.ei);
    if (cp) psi_load(d, d.psiE, so, true, cx, cy, cpml_at(d, 2, k), i, j, k, p.ps);
}

// E update of the Lorentz boxes (one thread per box cell, x fastest): the
// general per-node path with the auxiliary-differential-equation history.
template <typename T>
__device__ __forceinline__ void e_lor_block(const DomDev<T>* __restrict__ doms, const int* __restrict__ lbs, int ndom,
                                           int b, int rs, int ws, int t, const int* __restrict__ tdev) {
    if (b >= lbs[ndom]) return;
    int dom = find_domain(lbs, ndom, b);
    const DomDev<T>& d = doms[dom];
    const int bx = d.lhi[0] - d.llo[0], by = d.lhi[1] - d.llo[1], bzn = d.lhi[2] - d.llo[2];
    long long q = (long long)(b - lbs[dom]) * 256 + threadIdx.x;
    if (!d.has_lor || q >= (long long)bx * by * bzn) return;
    if (tdev) t += *tdev;
    const int i = d.llo[0] + (int)(q % bx), j = d.llo[1] + (int)((q / bx) % by), k = d.llo[2] + (int)(q / ((long long)bx * by));
    const long long so = (long long)rs * d.fs, wo = (long long)ws * d.fs, pl = d.plane;
    const long long f = (long long)k * pl + (long long)j * d.pitch + i;
    const FDTD_GLOBAL T* Hx = gp(d.H[0] + so);
    const FDTD_GLOBAL T* Hy = gp(d.H[1] + so);
    const FDTD_GLOBAL T* Hz = gp(d.H[2] + so);
    T hx = Hx[f], hy = Hy[f], hz = Hz[f];
    T hy_xm = nb_back(d, Hy, f, 0, i), hz_xm = nb_back(d, Hz, f, 0, i);
    T hx_ym = nb_back(d, Hx, f, 1, j), hz_ym = nb_back(d, Hz, f, 1, j);
    T hxm = k > 0 ? Hx[f - pl] : T(0), hym = k > 0 ? Hy[f - pl] : T(0);
    // Ex: d-_y Hz - d-_z Hy ; Ey: d-_z Hx - d-_x Hz ; Ez: d-_x Hy - d-_y Hx
    T ex = e_update(d, 0, i, j, k, f, hz, hz_ym, hy, hym, rs, ws, true, t);
    T ey = e_update(d, 1, i, j, k, f, hx, hxm, hz, hz_xm, rs, ws, true, t);
    T ez = e_update(d, 2, i, j, k, f, hy, hy_xm, hx, hx_ym, rs, ws, true, t);
    gp(d.E[0] + wo)[f] = ex;
    gp(d.E[1] + wo)[f] = ey;
    gp(d.E[2] + wo)[f] = ez;
}

// Blocks [0, nlb) update the Lorentz boxes (e_lor_block; nlb is a multiple
// of 8 so that the column blocks keep their XCD placement), the rest the
// columns.  TENS = false serves the domains with a scalar or diagonal
// permittivity; TENS = true the tensor domains, whose E update takes two
// passes: this one writes the stretched curl of every edge (absorber memories
// updated, zero on walls) into d.curl, k_tens_e applies the node assembly.
template <typename T, int W, bool TENS>
__global__ void __launch_bounds__(256) k_fwd_e(const DomDev<T>* __restrict__ doms, const int* __restrict__ bs,
                                               const int* __restrict__ xr, const int* __restrict__ lbs, int nlb,
                                               int ndom, int kz, int rs, int ws, int t, const int* __restrict__ tdev,
                                               int skip_interior) {
    if ((int)blockIdx.x < nlb) {
        e_lor_block(doms, lbs, ndom, xcd_remap(blockIdx.x, nlb), rs, ws, t, tdev);
        return;
    }
    const DomDev<T>* dp;
    Col c = column<T, W>(doms, bs, ndom, kz, dp, xr, (int)blockIdx.x - nlb);
    if (!c.ok || dp->tens != (int)TENS) return;
    if (skip_interior && blk_interior(*dp, c.x0, c.y0, c.k0, c.k1, W, 256 / W)) return;   // the single pass takes it
    if (tdev) t += *tdev;   // graph replays: step index held on the device
    const DomDev<T>& d = *dp;
    const int i = c.i, j = c.j;
    const long long so = (long long)rs * d.fs, wo = (long long)ws * d.fs, pl = d.plane;
    const FDTD_GLOBAL T* h[3] = {gp(d.H[0] + so), gp(d.H[1] + so), gp(d.H[2] + so)};
    const FDTD_GLOBAL T* e[3] = {gp(d.E[0] + so), gp(d.E[1] + so), gp(d.E[2] + so)};
    FDTD_GLOBAL T* ew[3] = {gp(d.E[0] + wo), gp(d.E[1] + wo), gp(d.E[2] + wo)};
    const BlkFlags bf = blk_flags(d, c.x0, c.y0, c.k0, c.k1, W, 256 / W);
    EpsView<T> ev = eps_view(d, c.x0, c.y0, 256 / W, c.k0, c.k1 - 1);
    if (TENS) ev.mode = 0;   // eps^-1 is applied by the assembly pass
    const Cpml1<T> cx = cpml_at(d, 0, i), cy = cpml_at(d, 1, j);
    const T S = d.S;
    long long f = (long long)c.k0 * pl + (long long)j * d.pitch + i;
    T hxm = 0, hym = 0;   // Hx, Hy one plane below
    if (c.k0 > 0) {
        hxm = h[0][f - pl];
        hym = h[1][f - pl];
    }
    ColE<T> cu, nx;
    cole_fetch(d, cu, h, e, f, ev, bf.cp, cx, cy, so, i, j, c.k0);
    for (int k = c.k0; k < c.k1; ++k, f += pl) {
        if (k + 1 < c.k1) cole_fetch(d, nx, h, e, f + pl, ev, bf.cp, cx, cy, so, i, j, k + 1);
        if (!(bf.lor && in_lor(d, i, j, k))) {   // Lorentz cells: e_lor_block
            T ex, ey, ez;
            T Dx0 = cu.hz - cu.hz_ym, Dx1 = cu.hy - hym;    // Ex: Hz along y, Hy along z
            T Dy0 = cu.hx - hxm, Dy1 = cu.hz - cu.hz_xm;    // Ey: Hx along z, Hz along x
            T Dz0 = cu.hy - cu.hy_xm, Dz1 = cu.hx - cu.hx_ym;   // Ez: Hy along x, Hx along y
            // unmasked nodes (E tangential to a wall is held at 0; periodic axes have none)
            const bool fx = !e_masked_d(d, 0, i, j, k), fy = !e_masked_d(d, 1, i, j, k),
                       fz = !e_masked_d(d, 2, i, j, k);
            if (bf.cp) {
                const Cpml1<T> cz = cpml_at(d, 2, k);
                const T* pe = cu.ps;
                if (cy.side >= 0) {
                    int q = poff(d, 1, cy.side, i, j, k);
                    Dx0 = st_pref(d.psiE[1][cy.side][0], wo, q, fx, cy.bE, cy.cE, cy.kE, pe[0], Dx0);
                    Dz1 = st_pref(d.psiE[1][cy.side][1], wo, q, fz, cy.bE, cy.cE, cy.kE, pe[1], Dz1);
                }
                if (cz.side >= 0) {
                    int q = poff(d, 2, cz.side, i, j, k);
                    Dy0 = st_pref(d.psiE[2][cz.side][0], wo, q, fy, cz.bE, cz.cE, cz.kE, pe[2], Dy0);
                    Dx1 = st_pref(d.psiE[2][cz.side][1], wo, q, fx, cz.bE, cz.cE, cz.kE, pe[3], Dx1);
                }
                if (cx.side >= 0) {
                    int q = poff(d, 0, cx.side, i, j, k);
                    Dz0 = st_pref(d.psiE[0][cx.side][0], wo, q, fz, cx.bE, cx.cE, cx.kE, pe[4], Dz0);
                    Dy1 = st_pref(d.psiE[0][cx.side][1], wo, q, fy, cx.bE, cx.cE, cx.kE, pe[5], Dy1);
                }
            }
            if constexpr (TENS) {
                gp(d.curl[0])[f] = fx ? Dx0 - Dx1 : T(0);
                gp(d.curl[1])[f] = fy ? Dy0 - Dy1 : T(0);
                gp(d.curl[2])[f] = fz ? Dz0 - Dz1 : T(0);
                hxm = cu.hx;
                hym = cu.hy;
                cu = nx;
                continue;
            }
            ex = fma(S * cu.ei[0], Dx0 - Dx1, cu.e[0]);
            ey = fma(S * cu.ei[1], Dy0 - Dy1, cu.e[1]);
            ez = fma(S * cu.ei[2], Dz0 - Dz1, cu.e[2]);
            for (int q = 0; q < d.nsrc; ++q) {
                const SrcDev<T>& sr = d.src[q];
                if (t < sr.nwave && k == sr.k && (sr.kind == 1 || (i == sr.i && j == sr.j))) {
                    T v = gp(sr.wave)[t];
                    if (sr.comp == 0) ex += v;
                    else if (sr.comp == 1) ey += v;
                    else ez += v;
                }
            }
            // PEC: E_c is zero where the index along c+1 or c+2 is 0 (not on a periodic axis)
            if (!fx) ex = T(0);
            if (!fy) ey = T(0);
            if (!fz) ez = T(0);
            ew[0][f] = ex;
            ew[1][f] = ey;
            ew[2][f] = ez;
        }
        hxm = cu.hx;
        hym = cu.hy;
        cu = nx;
    }
}


// ============================================================ forward, single pass
// Interior blocks (blk_interior) advance E and H in one launch, z-marching a
// column per thread like the split kernels, into the other state set.  At
// plane k a thread computes E^{n+1} of its own column at plane k+1 and of
// its +x and +y neighbour columns at plane k (the components its H update
// reads: Ez, Ey at i+1; Ez, Ex at j+1), then H^{n+3/2} at plane k.  The
// neighbours' E^{n+1} are recomputed rather than exchanged, so the block
// needs no LDS and no barrier; their operands are the neighbours' own loads,
// served by the caches.  Every update is the split kernels' arithmetic on
// the same operands, so the result is bitwise the split family's.
template <typename T>
struct OneOwn {   // own column, plane p: H, H one back along x and y, E^n, eps^-1
    T h[3], hy_xm, hz_xm, hx_ym, hz_ym, e[3], ep[3];
};

template <typename T>
struct OneNb {    // the +x and +y columns' E-update operands at plane p
    T hx_xp, hy_xp, hz_xp, hx_xpym, ey_xp, ez_xp, epy_xp, epz_xp;
    T hx_yp, hy_yp, hz_yp, hy_xmyp, ex_yp, ez_yp, epx_yp, epz_yp;
};

// eps^-1 of component c at (i,j,k) from a view whose mode covers the cell
template <typename T>
__device__ __forceinline__ T eps1(const EpsView<T>& v, int c, int i, int j, int k) {
    const bool in = v.mode == 1 || (v.mode == 2 && i >= v.lo[0] && i < v.hi[0] && j >= v.lo[1] && j < v.hi[1] &&
                                    k >= v.lo[2] && k < v.hi[2]);
    if (!in) return v.bg;
    const int q = ((k - v.lo[2]) * v.ey + (j - v.lo[1])) * v.ex + (i - v.exa);
    return v.p[v.diag ? c : 0][q];
}

template <typename T>
__device__ __forceinline__ void one_own(const FDTD_GLOBAL T* const (&h)[3], const FDTD_GLOBAL T* const (&e)[3],
                                        const EpsView<T>& ev, OneOwn<T>& o, long long f, long long P, int i, int j,
                                        int k) {
    o.h[0] = h[0][f];
    o.h[1] = h[1][f];
    o.h[2] = h[2][f];
    o.hy_xm = h[1][f - 1];
    o.hz_xm = h[2][f - 1];
    o.hx_ym = h[0][f - P];
    o.hz_ym = h[2][f - P];
    o.e[0] = e[0][f];
    o.e[1] = e[1][f];
    o.e[2] = e[2][f];
    eps_at(ev, i, j, k, o.ep);
}

template <typename T>
__device__ __forceinline__ void one_nb(const FDTD_GLOBAL T* const (&h)[3], const FDTD_GLOBAL T* const (&e)[3],
                                       const EpsView<T>& ev, OneNb<T>& n, long long f, long long P, int i, int j,
                                       int k) {
    n.hx_xp = h[0][f + 1];
    n.hy_xp = h[1][f + 1];
    n.hz_xp = h[2][f + 1];
    n.hx_xpym = h[0][f + 1 - P];
    n.ey_xp = e[1][f + 1];
    n.ez_xp = e[2][f + 1];
    n.epy_xp = eps1(ev, 1, i + 1, j, k);
    n.epz_xp = eps1(ev, 2, i + 1, j, k);
    n.hx_yp = h[0][f + P];
    n.hy_yp = h[1][f + P];
    n.hz_yp = h[2][f + P];
    n.hy_xmyp = h[1][f - 1 + P];
    n.ex_yp = e[0][f + P];
    n.ez_yp = e[2][f + P];
    n.epx_yp = eps1(ev, 0, i, j + 1, k);
    n.epz_yp = eps1(ev, 2, i, j + 1, k);
}

// the sources of E_c at (i, j, k) for step t, added in the split kernel's order
template <typename T>
__device__ __forceinline__ T add_src(const DomDev<T>& d, int c, int i, int j, int k, int t, T v) {
    for (int q = 0; q < d.nsrc; ++q) {
        const SrcDev<T>& sr = d.src[q];
        if (sr.comp == c && t < sr.nwave && k == sr.k && (sr.kind == 1 || (i == sr.i && j == sr.j)))
            v += gp(sr.wave)[t];
    }
    return v;
}

template <typename T, int W>
__global__ void __launch_bounds__(256) k_fwd_one(const DomDev<T>* __restrict__ doms, const int* __restrict__ bs,
                                                 const int* __restrict__ xr, int ndom, int kz, int rs, int ws, int t,
                                                 const int* __restrict__ tdev, int slot) {
    constexpr int NR = 256 / W;
    const DomDev<T>* dp;
    Col c = column<T, W>(doms, bs, ndom, kz, dp, xr);
    if (!c.ok || !blk_interior(*dp, c.x0, c.y0, c.k0, c.k1, W, NR)) return;
    if (tdev) t += *tdev;
    const DomDev<T>& d = *dp;
    const int i = c.i, j = c.j, k0 = c.k0, k1 = c.k1;
    const long long so = (long long)rs * d.fs, wo = (long long)ws * d.fs, pl = d.plane, P = d.pitch;
    const FDTD_GLOBAL T* h[3] = {gp(d.H[0] + so), gp(d.H[1] + so), gp(d.H[2] + so)};
    const FDTD_GLOBAL T* e[3] = {gp(d.E[0] + so), gp(d.E[1] + so), gp(d.E[2] + so)};
    FDTD_GLOBAL T* ew[3] = {gp(d.E[0] + wo), gp(d.E[1] + wo), gp(d.E[2] + wo)};
    FDTD_GLOBAL T* hw[3] = {gp(d.H[0] + wo), gp(d.H[1] + wo), gp(d.H[2] + wo)};
    // the block's cells and their +1 neighbours, planes k0 .. k1
    EpsView<T> ev = eps_view(d, c.x0, c.y0, NR + 1, k0, k1);
    {
        bool inside = true, outside = false;
        const int lo[3] = {c.x0, c.y0, k0}, hi[3] = {c.x0 + W, c.y0 + NR, k1};
        for (int a = 0; a < 3; ++a) {
            if (lo[a] < d.elo[a] || hi[a] >= d.ehi[a]) inside = false;
            if (hi[a] < d.elo[a] || lo[a] >= d.ehi[a]) outside = true;
        }
        ev.mode = outside ? 0 : (inside ? 1 : 2);
    }
    const T S = d.S;
    long long f = (long long)k0 * pl + (long long)j * P + i;
    // own E^{n+1} at plane k0, from H at k0 and k0 - 1
    T hxm = h[0][f - pl], hym = h[1][f - pl];
    T hx_xp_m = h[0][f - pl + 1], hy_yp_m = h[1][f - pl + P];   // the +x column's Hx, the +y column's Hy at k0 - 1
    OneOwn<T> cu, no;
    one_own(h, e, ev, cu, f, P, i, j, k0);
    T ex = fma(S * cu.ep[0], (cu.h[2] - cu.hz_ym) - (cu.h[1] - hym), cu.e[0]);
    T ey = fma(S * cu.ep[1], (cu.h[0] - hxm) - (cu.h[2] - cu.hz_xm), cu.e[1]);
    T ez = fma(S * cu.ep[2], (cu.h[1] - cu.hy_xm) - (cu.h[0] - cu.hx_ym), cu.e[2]);
    ex = add_src(d, 0, i, j, k0, t, ex);
    ey = add_src(d, 1, i, j, k0, t, ey);
    ez = add_src(d, 2, i, j, k0, t, ez);
    T hc[3] = {cu.h[0], cu.h[1], cu.h[2]};   // own H^{n+1/2} at plane k
    OneNb<T> nb;
    one_own(h, e, ev, no, f + pl, P, i, j, k0 + 1);
    one_nb(h, e, ev, nb, f, P, i, j, k0);
    for (int k = k0; k < k1; ++k, f += pl) {
        OneOwn<T> no2 = no;
        OneNb<T> nn = nb;
        if (k + 1 < k1) {   // fetch ahead: own plane k + 2, neighbour plane k + 1
            one_own(h, e, ev, no2, f + 2 * pl, P, i, j, k + 2);
            one_nb(h, e, ev, nn, f + pl, P, i, j, k + 1);
        }
        // own E^{n+1} at plane k + 1
        T ex1 = fma(S * no.ep[0], (no.h[2] - no.hz_ym) - (no.h[1] - hc[1]), no.e[0]);
        T ey1 = fma(S * no.ep[1], (no.h[0] - hc[0]) - (no.h[2] - no.hz_xm), no.e[1]);
        T ez1 = fma(S * no.ep[2], (no.h[1] - no.hy_xm) - (no.h[0] - no.hx_ym), no.e[2]);
        ex1 = add_src(d, 0, i, j, k + 1, t, ex1);
        ey1 = add_src(d, 1, i, j, k + 1, t, ey1);
        ez1 = add_src(d, 2, i, j, k + 1, t, ez1);
        // the +x column's Ez, Ey and the +y column's Ez, Ex at plane k
        T ez_xp = fma(S * nb.epz_xp, (nb.hy_xp - hc[1]) - (nb.hx_xp - nb.hx_xpym), nb.ez_xp);
        T ey_xp = fma(S * nb.epy_xp, (nb.hx_xp - hx_xp_m) - (nb.hz_xp - hc[2]), nb.ey_xp);
        T ez_yp = fma(S * nb.epz_yp, (nb.hy_yp - nb.hy_xmyp) - (nb.hx_yp - hc[0]), nb.ez_yp);
        T ex_yp = fma(S * nb.epx_yp, (nb.hz_yp - hc[2]) - (nb.hy_yp - hy_yp_m), nb.ex_yp);
        ez_xp = add_src(d, 2, i + 1, j, k, t, ez_xp);
        ey_xp = add_src(d, 1, i + 1, j, k, t, ey_xp);
        ez_yp = add_src(d, 2, i, j + 1, k, t, ez_yp);
        ex_yp = add_src(d, 0, i, j + 1, k, t, ex_yp);
        // H^{n+3/2} at plane k
        const T hx = fma(-S, (ez_yp - ez) - (ey1 - ey), hc[0]);
        const T hy = fma(-S, (ex1 - ex) - (ez_xp - ez), hc[1]);
        const T hz = fma(-S, (ey_xp - ey) - (ex_yp - ex), hc[2]);
        ew[0][f] = ex;
        ew[1][f] = ey;
        ew[2][f] = ez;
        hw[0][f] = hx;
        hw[1][f] = hy;
        hw[2][f] = hz;
        if (slot >= 0) sample_node(d, slot, i, j, k, ex, ey, ez, hx, hy, hz);
        hx_xp_m = nb.hx_xp;
        hy_yp_m = nb.hy_yp;
        hc[0] = no.h[0];
        hc[1] = no.h[1];
        hc[2] = no.h[2];
        ex = ex1;
        ey = ey1;
        ez = ez1;
        no = no2;
        nb = nn;
    }
}

// ------------------------------------------------ tensor media, assembly pass
// Operands of plane k of the assembly pass that are not carried over from
// plane k-1 (c: curl, a: node eps^-1; suffixes name the offset from (i,j,k))
template <typename T>
struct TensPlane {
    T cz, cz_xp, cz_yp;                 // Cz at (i,j,k), (i+1,j,k), (i,j+1,k)
    T cy_xp, cy_xpym;                   // Cy at (i+1,j,k), (i+1,j-1,k)
    T cx_yp, cx_xmyp;                   // Cx at (i,j+1,k), (i-1,j+1,k)
    T cx_zp, cx_xmzp, cy_zp, cy_ymzp;   // plane k+1: Cx at (i,j,k+1), (i-1,j,k+1); Cy at (i,j,k+1), (i,j-1,k+1)
    T a_xx, a_yy, a_xy;                 // node (i,j,k)
    T axp_xx, axp_xy, axp_xz;           // node (i+1,j,k)
    T ayp_yy, ayp_xy, ayp_yz;           // node (i,j+1,k)
    T azp_zz, azp_xz, azp_yz;           // node (i,j,k+1)
    T e[3];
};

// Per-column addressing of the assembly pass: curl and node-tensor offsets
// of (i,j) with the in-grid and in-box tests of the x and y neighbours
// evaluated once per column; the per-plane tests are on k alone.  Across a
// periodic seam a neighbour column is the one at the other end: its edges
// carry the real Bloch factor, its node tensors repeat unchanged.
template <typename T>
struct TensCol {
    const FDTD_GLOBAL T* c[3];           // curl arrays
    const FDTD_GLOBAL T* a[6];           // node eps^-1 arrays over the box
    long long fc;                        // field offset of (i, j, 0)
    long long qc;                        // box offset of (i, j, elo_z) (valid when the column is in the box)
    long long pl, bpl;                   // field plane, box plane
    long long oxm, oxp, oym, oyp;        // field offsets of the columns i-1, i+1, j-1, j+1 from (i, j)
    long long qxp, qyp;                  // box offsets of the node columns i+1 and j+1 from (i, j)
    T fxm, fxp, fym, fyp;                // their edges' Bloch factors (1 inside the grid)
    int pitch, bx;
    bool xm, xp, ym, yp;                 // the neighbour column exists (inside the grid or across a seam)
    bool bxy, bxpy, bxyp;                // (i,j), (i+1,j), (i,j+1) inside the box's x-y extent
    int nz, ez0, ez1;
    T bg;
};

template <typename T>
__device__ __forceinline__ T tc(const TensCol<T>& m, int b, long long off, bool ok) {
    return ok ? m.c[b][m.fc + off] : T(0);
}

// component q (xx yy zz xy xz yz) of the node tensor at column offset off
// (in-box flag inb) and plane k; outside the box (the nodes on the high walls
// included) the background eps^-1 times the identity
template <typename T>
__device__ __forceinline__ T ta(const TensCol<T>& m, int q, long long off, bool inb, int k) {
    return (inb && k >= m.ez0 && k < m.ez1) ? m.a[q][m.qc + (long long)(k - m.ez0) * m.bpl + off]
                                            : (q < 3 ? m.bg : T(0));
}

// PER: the domain has a periodic axis (neighbour offsets and Bloch factors
// from the column's table); else the neighbours are the fixed offsets
template <typename T, bool PER>
__device__ __forceinline__ void tens_fetch(const TensCol<T>& m, TensPlane<T>& p, const FDTD_GLOBAL T* const (&e)[3],
                                           int k, long long f) {
    const long long o = (long long)k * m.pl;
    const bool up = k + 1 < m.nz;
    p.cz = tc(m, 2, o, true);
    if constexpr (PER) {
        p.cz_xp = m.fxp * tc(m, 2, o + m.oxp, m.xp);
        p.cz_yp = m.fyp * tc(m, 2, o + m.oyp, m.yp);
        p.cy_xp = m.fxp * tc(m, 1, o + m.oxp, m.xp);
        p.cy_xpym = (m.fxp * m.fym) * tc(m, 1, o + m.oxp + m.oym, m.xp && m.ym);
        p.cx_yp = m.fyp * tc(m, 0, o + m.oyp, m.yp);
        p.cx_xmyp = (m.fxm * m.fyp) * tc(m, 0, o + m.oxm + m.oyp, m.xm && m.yp);
        p.cx_xmzp = m.fxm * tc(m, 0, o + m.pl + m.oxm, up && m.xm);
        p.cy_ymzp = m.fym * tc(m, 1, o + m.pl + m.oym, up && m.ym);
    } else {
        const long long P = m.pitch;
        p.cz_xp = tc(m, 2, o + 1, m.xp);
        p.cz_yp = tc(m, 2, o + P, m.yp);
        p.cy_xp = tc(m, 1, o + 1, m.xp);
        p.cy_xpym = tc(m, 1, o + 1 - P, m.xp && m.ym);
        p.cx_yp = tc(m, 0, o + P, m.yp);
        p.cx_xmyp = tc(m, 0, o - 1 + P, m.xm && m.yp);
        p.cx_xmzp = tc(m, 0, o + m.pl - 1, up && m.xm);
        p.cy_ymzp = tc(m, 1, o + m.pl - P, up && m.ym);
    }
    p.cx_zp = tc(m, 0, o + m.pl, up);
    p.cy_zp = tc(m, 1, o + m.pl, up);
    const long long qx = PER ? m.qxp : 1, qy = PER ? m.qyp : (long long)m.bx;
    p.a_xx = ta(m, 0, 0, m.bxy, k);
    p.a_yy = ta(m, 1, 0, m.bxy, k);
    p.a_xy = ta(m, 3, 0, m.bxy, k);
    p.axp_xx = ta(m, 0, qx, m.bxpy, k);
    p.axp_xy = ta(m, 3, qx, m.bxpy, k);
    p.axp_xz = ta(m, 4, qx, m.bxpy, k);
    p.ayp_yy = ta(m, 1, qy, m.bxyp, k);
    p.ayp_xy = ta(m, 3, qy, m.bxyp, k);
    p.ayp_yz = ta(m, 5, qy, m.bxyp, k);
    p.azp_zz = ta(m, 2, 0, m.bxy, k + 1);
    p.azp_xz = ta(m, 4, 0, m.bxy, k + 1);
    p.azp_yz = ta(m, 5, 0, m.bxy, k + 1);
    p.e[0] = e[0][f];
    p.e[1] = e[1][f];
    p.e[2] = e[2][f];
}

// E^{n+1} = E^n + S (node assembly of eps^-1) curl, plus the sources, for the
// tensor domains, one thread per (i, j) column of a z chunk.  The edge of
// component c from node v0 to v1 = v0 + e_c takes, at each end v,
// eps^-1_cc(v)/2 times its own curl and eps^-1_cb(v)/4 times the sum of the
// curls of the two b edges meeting at v (leaving and arriving), b != c.
// Edges tangential to a wall keep E = 0; on a periodic axis the edges and
// nodes past the seam are those at the other end (Section 2.2), the edges
// times the real Bloch factor.  Reads and writes only its own E
// nodes, so it runs in place like the other split kernels.  Along z the
// column keeps what plane k+1 shares with plane k (the Cz below, the Cx and
// Cy above, the node above) in registers, and fetches plane k+1's other
// operands before it computes and stores plane k.  PER = true serves the
// tensor domains with a periodic axis, false the others.
template <typename T, int W, bool PER>
__global__ void __launch_bounds__(256) k_tens_e(const DomDev<T>* __restrict__ doms, const int* __restrict__ bs,
                                                const int* __restrict__ xr, int ndom, int kz, int rs, int ws, int t,
                                                const int* __restrict__ tdev) {
    const DomDev<T>* dp;
    Col c = column<T, W>(doms, bs, ndom, kz, dp, xr);
    if (!c.ok || !dp->tens || (dp->per[0] || dp->per[1]) != PER) return;
    if (tdev) t += *tdev;
    const DomDev<T>& d = *dp;
    const int i = c.i, j = c.j;
    const long long so = (long long)rs * d.fs, wo = (long long)ws * d.fs;
    const FDTD_GLOBAL T* e[3] = {gp(d.E[0] + so), gp(d.E[1] + so), gp(d.E[2] + so)};
    FDTD_GLOBAL T* ew[3] = {gp(d.E[0] + wo), gp(d.E[1] + wo), gp(d.E[2] + wo)};
    const T S = d.S, h = T(0.5), q4 = T(0.25);
    const int k0 = c.k0;
    TensCol<T> m;
    for (int b = 0; b < 3; ++b) m.c[b] = gp((const T*)d.curl[b]);
    for (int q = 0; q < 6; ++q) m.a[q] = gp(d.tinv[q]);
    m.pitch = d.pitch;
    m.pl = d.plane;
    m.fc = (long long)j * d.pitch + i;
    m.bx = d.exs;
    m.bpl = (long long)m.bx * (d.ehi[1] - d.elo[1]);
    m.qc = (long long)(j - d.elo[1]) * m.bx + (i - d.exa);
    // neighbour columns: inside the grid, else across a periodic seam (the
    // column at the other end, the Bloch factor on its edges), else none
    const long long P = d.pitch;
    const int nx1 = d.n[0] - 1, ny1 = d.n[1] - 1;
    m.xm = i > 0 || d.per[0];
    m.xp = i < nx1 || d.per[0];
    m.ym = j > 0 || d.per[1];
    m.yp = j < ny1 || d.per[1];
    m.oxm = i > 0 ? -1 : nx1;
    m.oxp = i < nx1 ? 1 : -nx1;
    m.oym = j > 0 ? -P : ny1 * P;
    m.oyp = j < ny1 ? P : -ny1 * P;
    m.fxm = i > 0 ? T(1) : d.bsign[0];
    m.fxp = i < nx1 ? T(1) : d.bsign[0];
    m.fym = j > 0 ? T(1) : d.bsign[1];
    m.fyp = j < ny1 ? T(1) : d.bsign[1];
    // the node columns i+1 and j+1 (the first ones past a seam; past a wall
    // outside every box)
    const int i1 = i < nx1 || !d.per[0] ? i + 1 : 0, j1 = j < ny1 || !d.per[1] ? j + 1 : 0;
    m.qxp = i1 - i;
    m.qyp = (long long)(j1 - j) * m.bx;
    const bool inx = i >= d.elo[0] && i < d.ehi[0], inx1 = i1 >= d.elo[0] && i1 < d.ehi[0];
    const bool iny = j >= d.elo[1] && j < d.ehi[1], iny1 = j1 >= d.elo[1] && j1 < d.ehi[1];
    m.bxy = inx && iny;
    m.bxpy = inx1 && iny;
    m.bxyp = inx && iny1;
    m.nz = d.n[2];
    m.ez0 = d.elo[2];
    m.ez1 = d.ehi[2];
    m.bg = d.epsinv_bg;
    // carried into plane k0: Cz below it, Cx and Cy on it, the z-related node entries
    const long long o0 = (long long)k0 * m.pl;
    T czm = tc(m, 2, o0 - m.pl, k0 > 0), cx = tc(m, 0, o0, true), cy = tc(m, 1, o0, true);
    T czm_xp, czm_yp, cx_xm, cy_ym;
    if constexpr (PER) {
        czm_xp = m.fxp * tc(m, 2, o0 - m.pl + m.oxp, k0 > 0 && m.xp);
        czm_yp = m.fyp * tc(m, 2, o0 - m.pl + m.oyp, k0 > 0 && m.yp);
        cx_xm = m.fxm * tc(m, 0, o0 + m.oxm, m.xm);
        cy_ym = m.fym * tc(m, 1, o0 + m.oym, m.ym);
    } else {
        czm_xp = tc(m, 2, o0 - m.pl + 1, k0 > 0 && m.xp);
        czm_yp = tc(m, 2, o0 - m.pl + m.pitch, k0 > 0 && m.yp);
        cx_xm = tc(m, 0, o0 - 1, m.xm);
        cy_ym = tc(m, 1, o0 - m.pitch, m.ym);
    }
    T a_zz = ta(m, 2, 0, m.bxy, k0), a_xz = ta(m, 4, 0, m.bxy, k0), a_yz = ta(m, 5, 0, m.bxy, k0);
    long long f = fidx(d, i, j, k0);
    TensPlane<T> cu, nx;
    tens_fetch<T, PER>(m, cu, e, k0, f);
    for (int k = k0; k < c.k1; ++k, f += d.plane) {
        if (k + 1 < c.k1) tens_fetch<T, PER>(m, nx, e, k + 1, f + d.plane);
        const T sx = cx + cx_xm, sy = cy + cy_ym, sz = cu.cz + czm;   // the two edges of each axis at v0
        T mx = h * (cu.a_xx + cu.axp_xx) * cx;
        mx += q4 * (cu.a_xy * sy + cu.axp_xy * (cu.cy_xp + cu.cy_xpym));
        mx += q4 * (a_xz * sz + cu.axp_xz * (cu.cz_xp + czm_xp));
        T my = h * (cu.a_yy + cu.ayp_yy) * cy;
        my += q4 * (cu.a_xy * sx + cu.ayp_xy * (cu.cx_yp + cu.cx_xmyp));
        my += q4 * (a_yz * sz + cu.ayp_yz * (cu.cz_yp + czm_yp));
        T mz = h * (a_zz + cu.azp_zz) * cu.cz;
        mz += q4 * (a_xz * sx + cu.azp_xz * (cu.cx_zp + cu.cx_xmzp));
        mz += q4 * (a_yz * sy + cu.azp_yz * (cu.cy_zp + cu.cy_ymzp));
        T ex = fma(S, mx, cu.e[0]);
        T ey = fma(S, my, cu.e[1]);
        T ez = fma(S, mz, cu.e[2]);
        for (int q = 0; q < d.nsrc; ++q) {
            const SrcDev<T>& sr = d.src[q];
            if (t < sr.nwave && k == sr.k && (sr.kind == 1 || (i == sr.i && j == sr.j))) {
                T v = gp(sr.wave)[t];
                if (sr.comp == 0) ex += v;
                else if (sr.comp == 1) ey += v;
                else ez += v;
            }
        }
        if (e_masked_d(d, 0, i, j, k)) ex = T(0);
        if (e_masked_d(d, 1, i, j, k)) ey = T(0);
        if (e_masked_d(d, 2, i, j, k)) ez = T(0);
        ew[0][f] = ex;
        ew[1][f] = ey;
        ew[2][f] = ez;
        // plane k+1 inherits
        czm = cu.cz;
        czm_xp = cu.cz_xp;
        czm_yp = cu.cz_yp;
        cx = cu.cx_zp;
        cx_xm = cu.cx_xmzp;
        cy = cu.cy_zp;
        cy_ym = cu.cy_ymzp;
        a_zz = cu.azp_zz;
        a_xz = cu.azp_xz;
        a_yz = cu.azp_yz;
        cu = nx;
    }
}

// reads E^{n+1} from set ws (written by k_fwd_e), H^{n+1/2} from set rs
template <typename T>
struct ColH {
    T e1[3];                          // E^{n+1} one plane up
    T ey_xp, ez_xp, ex_yp, ez_yp;     // E^{n+1} one step forward along x and y
    T h[3];                           // H^{n+1/2} at the node
    T ps[6];                          // H-side absorber memories (psi_load order)
};

template <typename T>
__device__ __forceinline__ void colh_fetch(const DomDev<T>& d, ColH<T>& p, const FDTD_GLOBAL T* const (&e)[3],
                                           const FDTD_GLOBAL T* const (&h)[3], long long f, bool cp,
                                           const Cpml1<T>& cx, const Cpml1<T>& cy, long long so, int i, int j,
                                           int k) {
    const bool up = k + 1 < d.n[2];
    const long long pl = d.plane;
    p.e1[0] = up ? e[0][f + pl] : T(0);
    p.e1[1] = up ? e[1][f + pl] : T(0);
    p.e1[2] = up ? e[2][f + pl] : T(0);
    p.ey_xp = nb_fwd(d, e[1], f, 0, i);
    p.ez_xp = nb_fwd(d, e[2], f, 0, i);
    p.ex_yp = nb_fwd(d, e[0], f, 1, j);
    p.ez_yp = nb_fwd(d, e[2], f, 1, j);
    p.h[0] = h[0][f];
    p.h[1] = h[1][f];
    p.h[2] = h[2][f];
    if (cp) psi_load(d, d.psiH, so, true, cx, cy, cpml_at(d, 2, k), i, j, k, p.ps);
}

// In-kernel sampling (slot >= 0): a thread whose column lies in a plane
// monitor's rectangle writes, on the monitor plane, E^{n+1} and the new H,
// and on the plane below (flux) the new Hx, Hy, into the ring slot.
template <typename T>
__device__ __forceinline__ void sample_node(const DomDev<T>& d, int slot, int i, int j, int k, T ex, T ey, T ez,
                                            T hx, T hy, T hz) {
    for (int q = 0; q < d.nsmp; ++q) {
        const SmpDev& m = d.smp[q];
        if (i < m.i0 || i >= m.i1 || j < m.j0 || j >= m.j1) continue;
        const bool on = k == m.k, below = m.kind == 1 && k + 1 == m.k;
        if (!on && !below) continue;
        const long long np = m.npts;
        FDTD_GLOBAL T* buf = gp((T*)m.ring) + (long long)slot * m.rcomp * np + (j - m.j0) * (m.i1 - m.i0) + (i - m.i0);
        if (m.kind == 1) {
            if (on) {
                buf[0] = ex;
                buf[np] = ey;
                buf[2 * np] = hx;
                buf[4 * np] = hy;
                if (k == 0) buf[3 * np] = buf[5 * np] = T(0);   // no plane below
            } else {
                buf[3 * np] = hx;
                buf[5 * np] = hy;
            }
        } else {
            const int c = m.comp;
            buf[0] = c == 0 ? ex : c == 1 ? ey : c == 2 ? ez : c == 3 ? hx : c == 4 ? hy : hz;
        }
    }
}

template <typename T, int W>
__global__ void __launch_bounds__(256) k_fwd_h(const DomDev<T>* __restrict__ doms, const int* __restrict__ bs,
                                               const int* __restrict__ xr, int ndom, int kz, int rs, int ws, int slot,
                                               int skip_interior) {
    const DomDev<T>* dp;
    Col c = column<T, W>(doms, bs, ndom, kz, dp, xr);
    if (!c.ok) return;
    if (skip_interior && blk_interior(*dp, c.x0, c.y0, c.k0, c.k1, W, 256 / W)) return;
    const DomDev<T>& d = *dp;
    const int i = c.i, j = c.j;
    const long long so = (long long)rs * d.fs, wo = (long long)ws * d.fs, pl = d.plane;
    const FDTD_GLOBAL T* e[3] = {gp(d.E[0] + wo), gp(d.E[1] + wo), gp(d.E[2] + wo)};
    const FDTD_GLOBAL T* h[3] = {gp(d.H[0] + so), gp(d.H[1] + so), gp(d.H[2] + so)};
    FDTD_GLOBAL T* hw[3] = {gp(d.H[0] + wo), gp(d.H[1] + wo), gp(d.H[2] + wo)};
    const BlkFlags bf = blk_flags(d, c.x0, c.y0, c.k0, c.k1, W, 256 / W);
    const Cpml1<T> cx = cpml_at(d, 0, i), cy = cpml_at(d, 1, j);
    const T S = d.S;
    long long f = (long long)c.k0 * pl + (long long)j * d.pitch + i;
    T ex = e[0][f], ey = e[1][f], ez = e[2][f];
    ColH<T> cu, nx;
    colh_fetch(d, cu, e, h, f, bf.cp, cx, cy, so, i, j, c.k0);
    for (int k = c.k0; k < c.k1; ++k, f += pl) {
        if (k + 1 < c.k1) colh_fetch(d, nx, e, h, f + pl, bf.cp, cx, cy, so, i, j, k + 1);
        // Hx: d+_y Ez - d+_z Ey ; Hy: d+_z Ex - d+_x Ez ; Hz: d+_x Ey - d+_y Ex
        T Dx0 = cu.ez_yp - ez, Dx1 = cu.e1[1] - ey;
        T Dy0 = cu.e1[0] - ex, Dy1 = cu.ez_xp - ez;
        T Dz0 = cu.ey_xp - ey, Dz1 = cu.ex_yp - ex;
        if (bf.cp) {
            const Cpml1<T> cz = cpml_at(d, 2, k);
            const T* ph = cu.ps;
            if (cy.side >= 0) {
                int q = poff(d, 1, cy.side, i, j, k);
                Dx0 = st_pref(d.psiH[1][cy.side][0], wo, q, true, cy.bH, cy.cH, cy.kH, ph[0], Dx0);
                Dz1 = st_pref(d.psiH[1][cy.side][1], wo, q, true, cy.bH, cy.cH, cy.kH, ph[1], Dz1);
            }
            if (cz.side >= 0) {
                int q = poff(d, 2, cz.side, i, j, k);
                Dy0 = st_pref(d.psiH[2][cz.side][0], wo, q, true, cz.bH, cz.cH, cz.kH, ph[2], Dy0);
                Dx1 = st_pref(d.psiH[2][cz.side][1], wo, q, true, cz.bH, cz.cH, cz.kH, ph[3], Dx1);
            }
            if (cx.side >= 0) {
                int q = poff(d, 0, cx.side, i, j, k);
                Dz0 = st_pref(d.psiH[0][cx.side][0], wo, q, true, cx.bH, cx.cH, cx.kH, ph[4], Dz0);
                Dy1 = st_pref(d.psiH[0][cx.side][1], wo, q, true, cx.bH, cx.cH, cx.kH, ph[5], Dy1);
            }
        }
        const T hx = fma(-S, Dx0 - Dx1, cu.h[0]);
        const T hy = fma(-S, Dy0 - Dy1, cu.h[1]);
        const T hz = fma(-S, Dz0 - Dz1, cu.h[2]);
        hw[0][f] = hx;
        hw[1][f] = hy;
        hw[2][f] = hz;
        if (slot >= 0) sample_node(d, slot, i, j, k, ex, ey, ez, hx, hy, hz);
        ex = cu.e1[0];
        ey = cu.e1[1];
        ez = cu.e1[2];
        cu = nx;
    }
}

// ============================================================ adjoint, split
// Two launches per adjoint step, shaped like the forward pair:
//   k_adj_ht  at E nodes (gathers Hbar from the node and one step back, like
//             the E update): cotangent of E^{n+1} after the H transpose, the
//             E-update transpose with the Lorentz history, the new Ebar^n
//             (set ws), the scaled cotangent U = S coef Ebar_pre (into the
//             scratch Et), the E-side absorber memory cotangents (set ws) and
//             dJ/deps from the forward state (set fsr);
//   k_adj_et  at H nodes (gathers U from the node and one step forward, like
//             the H update): Hbar^n (set ws) and the H-side absorber memory
//             cotangents (set ws).
// Every node's E-side work is done once; the raw-difference cotangent of an
// E term at a neighbour is rebuilt from its U and its old memory cotangent.

// cotangent of E^{n+1}_e after the H transpose, from Ebar (given) and Hbar
// (set rs): term 1 of H_{e+1} along e+2 (+), term 2 of H_{e+2} along e+1 (-)
template <typename T>
__device__ __forceinline__ T ht_update_v(const DomDev<T>& d, int e, int i, int j, int k, T acc, T hb1, T hb1m,
                                         T hb2, T hb2m, int rs) {
    if (e_masked(e, i, j, k)) return T(0);
    const int a1 = (e + 2) % 3, a2 = (e + 1) % 3;
    T t1 = hT_dbar(d, a1, 0, T(1), i, j, k, hb1, rs, rs, false);
    T t1m = coord(a1, i, j, k) > 0
                ? hT_dbar(d, a1, 0, T(1), i - (a1 == 0), j - (a1 == 1), k - (a1 == 2), hb1m, rs, rs, false)
                : T(0);
    T t2 = hT_dbar(d, a2, 1, T(-1), i, j, k, hb2, rs, rs, false);
    T t2m = coord(a2, i, j, k) > 0
                ? hT_dbar(d, a2, 1, T(-1), i - (a2 == 0), j - (a2 == 1), k - (a2 == 2), hb2m, rs, rs, false)
                : T(0);
    acc += t1m - t1;
    acc += t2m - t2;
    return acc;
}

// Transposed absorber term with hoisted coefficients: ybar through
// mem = psibar + ybar, returns ki ybar + c mem (stretch_T, read only).
template <typename T>
__device__ __forceinline__ T tr_term(bool slab, T ki, T c, T psi, T ybar) {
    return slab ? fma(ki, ybar, c * (psi + ybar)) : ybar;
}

// Variant masks of the adjoint passes: bit 0, 1, 2 = the block (or the
// neighbour one step back / forward that it reads) meets the x, y, z absorber
// slabs, so those memory cotangents are handled; bit 3 (E-node pass) = the
// block holds Lorentz cells or gradient cells inside a slab, which take the
// general per-node path.  The host sorts blocks into classes; each class is
// a kernel of its own with only the registers it needs.
constexpr int kAdjFull = 15;

// the two memory slots (psi_load order) of axis a at node (i,j,k), if the
// node lies in that axis' slab
template <typename T>
__device__ __forceinline__ void psi_axis(const DomDev<T>& d, T* const (&psi)[3][2][2], long long so, int a,
                                         const Cpml1<T>& ca, int i, int j, int k, T& p0, T& p1) {
    p0 = p1 = T(0);
    if (ca.side < 0) return;
    int o = poff(d, a, ca.side, i, j, k);
    p0 = gp(psi[a][ca.side][0] + so)[o];
    p1 = gp(psi[a][ca.side][1] + so)[o];
}

template <typename T>
struct AdjColE {
    T hx, hy, hz, hy_xm, hz_xm, hx_ym, hz_ym;   // Hbar at the node and one step back along x and y
    T eb[3], ei[3];                              // Ebar and eps^-1 at the node
    T ph[6];                                     // H-side memory cotangents at the node (psi_load order)
    T phx[2], phy[2];                            // at (i-1): x-slab slots 4, 5; at (j-1): y-slab slots 0, 1
    T pe[6];                                     // E-side memory cotangents at the node
};

template <typename T, int V>
__device__ __forceinline__ void adje_fetch(const DomDev<T>& d, AdjColE<T>& p, const FDTD_GLOBAL T* const (&h)[3],
                                           const FDTD_GLOBAL T* const (&e)[3], long long f, const EpsView<T>& ev,
                                           const Cpml1<T>& cx, const Cpml1<T>& cy, const Cpml1<T>& cxm,
                                           const Cpml1<T>& cym, long long ro, int i, int j, int k) {
    p.hx = h[0][f];
    p.hy = h[1][f];
    p.hz = h[2][f];
    p.hy_xm = i > 0 ? h[1][f - 1] : T(0);
    p.hz_xm = i > 0 ? h[2][f - 1] : T(0);
    p.hx_ym = j > 0 ? h[0][f - d.pitch] : T(0);
    p.hz_ym = j > 0 ? h[2][f - d.pitch] : T(0);
    p.eb[0] = e[0][f];
    p.eb[1] = e[1][f];
    p.eb[2] = e[2][f];
    eps_at(ev, i, j, k, p.ei);
    if (V & 1) {
        psi_axis(d, d.psiHa, ro, 0, cx, i, j, k, p.ph[4], p.ph[5]);
        psi_axis(d, d.psiEa, ro, 0, cx, i, j, k, p.pe[4], p.pe[5]);
        psi_axis(d, d.psiHa, ro, 0, cxm, i - 1, j, k, p.phx[0], p.phx[1]);
    }
    if (V & 2) {
        psi_axis(d, d.psiHa, ro, 1, cy, i, j, k, p.ph[0], p.ph[1]);
        psi_axis(d, d.psiEa, ro, 1, cy, i, j, k, p.pe[0], p.pe[1]);
        psi_axis(d, d.psiHa, ro, 1, cym, i, j - 1, k, p.phy[0], p.phy[1]);
    }
    if (V & 4) {
        const Cpml1<T> cz = cpml_at(d, 2, k);
        psi_axis(d, d.psiHa, ro, 2, cz, i, j, k, p.ph[2], p.ph[3]);
        psi_axis(d, d.psiEa, ro, 2, cz, i, j, k, p.pe[2], p.pe[3]);
    }
}

template <typename T, int V, int W>
__device__ __forceinline__ void adj_ht_tile(const DomDev<T>* __restrict__ doms, const int4 tile, int kz, int rs,
                                            int ws, int fsr) {
    const DomDev<T>* dp;
    const TileCol<W> c = tile_column<T, W>(doms, tile, kz, dp);
    if (!c.ok) return;
    const DomDev<T>& d = *dp;
    if (!d.grad) return;
    const int i = c.i, j = c.j;
    const long long ro = (long long)rs * d.as, wo = (long long)ws * d.as, pl = d.plane;
    const FDTD_GLOBAL T* h[3] = {gp(d.Ha[0] + ro), gp(d.Ha[1] + ro), gp(d.Ha[2] + ro)};
    const FDTD_GLOBAL T* e[3] = {gp(d.Ea[0] + ro), gp(d.Ea[1] + ro), gp(d.Ea[2] + ro)};
    FDTD_GLOBAL T* ew[3] = {gp(d.Ea[0] + wo), gp(d.Ea[1] + wo), gp(d.Ea[2] + wo)};
    FDTD_GLOBAL T* uw[3] = {gp(d.Et[0]), gp(d.Et[1]), gp(d.Et[2])};
    constexpr bool CX = V & 1, CY = V & 2, CZ = V & 4, FULL = V & 8;
    constexpr int NR = 256 / W;   // rows per block
    const EpsView<T> ev = eps_view(d, c.x0, c.y0, NR, c.k0, c.k1 - 1);
    const Cpml1<T> cx = cpml_at(d, 0, i), cy = cpml_at(d, 1, j), cxm = cpml_at(d, 0, i - 1), cym = cpml_at(d, 1, j - 1);
    const T S = d.S, mS = -d.S;
    long long f = (long long)c.k0 * pl + (long long)j * d.pitch + i;
    T hxm = 0, hym = 0;      // Hbar x, y one plane below
    T pzm2 = 0, pzm3 = 0;    // H-side z-slab memory cotangents one plane below (slots 2, 3)
    if (c.k0 > 0) {
        hxm = h[0][f - pl];
        hym = h[1][f - pl];
        if (CZ) psi_axis(d, d.psiHa, ro, 2, cpml_at(d, 2, c.k0 - 1), i, j, c.k0 - 1, pzm2, pzm3);
    }
    AdjColE<T> cu, nx;
    adje_fetch<T, V>(d, cu, h, e, f, ev, cx, cy, cxm, cym, ro, i, j, c.k0);
    for (int k = c.k0; k < c.k1; ++k, f += pl) {
        if (k + 1 < c.k1) adje_fetch<T, V>(d, nx, h, e, f + pl, ev, cx, cy, cxm, cym, ro, i, j, k + 1);
        const Cpml1<T> cz = cpml_at(d, 2, k), czm = cpml_at(d, 2, k - 1);
        const bool sx = CX && cx.side >= 0, sy = CY && cy.side >= 0, sz = CZ && cz.side >= 0;
        const bool sxm = CX && cxm.side >= 0, sym = CY && cym.side >= 0, szm = CZ && czm.side >= 0;
        // H transposes (hT_dbar): ybar = -S sign Hbar; term 1 (+), term 2 (-)
        T et[3];
        {   // Ex: Hy term 0 along z (slot 2), Hz term 1 along y (slot 1)
            T t1 = tr_term(sz, cz.kH, cz.cH, cu.ph[2], mS * cu.hy);
            T t1m = k > 0 ? tr_term(szm, czm.kH, czm.cH, pzm2, mS * hym) : T(0);
            T t2 = tr_term(sy, cy.kH, cy.cH, cu.ph[1], S * cu.hz);
            T t2m = j > 0 ? tr_term(sym, cym.kH, cym.cH, cu.phy[1], S * cu.hz_ym) : T(0);
            T acc = cu.eb[0];
            acc += t1m - t1;
            acc += t2m - t2;
            et[0] = (j == 0 || k == 0) ? T(0) : acc;
        }
        {   // Ey: Hz term 0 along x (slot 4), Hx term 1 along z (slot 3)
            T t1 = tr_term(sx, cx.kH, cx.cH, cu.ph[4], mS * cu.hz);
            T t1m = i > 0 ? tr_term(sxm, cxm.kH, cxm.cH, cu.phx[0], mS * cu.hz_xm) : T(0);
            T t2 = tr_term(sz, cz.kH, cz.cH, cu.ph[3], S * cu.hx);
            T t2m = k > 0 ? tr_term(szm, czm.kH, czm.cH, pzm3, S * hxm) : T(0);
            T acc = cu.eb[1];
            acc += t1m - t1;
            acc += t2m - t2;
            et[1] = (i == 0 || k == 0) ? T(0) : acc;
        }
        {   // Ez: Hx term 0 along y (slot 0), Hy term 1 along x (slot 5)
            T t1 = tr_term(sy, cy.kH, cy.cH, cu.ph[0], mS * cu.hx);
            T t1m = j > 0 ? tr_term(sym, cym.kH, cym.cH, cu.phy[0], mS * cu.hx_ym) : T(0);
            T t2 = tr_term(sx, cx.kH, cx.cH, cu.ph[5], S * cu.hy);
            T t2m = i > 0 ? tr_term(sxm, cxm.kH, cxm.cH, cu.phx[1], S * cu.hy_xm) : T(0);
            T acc = cu.eb[2];
            acc += t1m - t1;
            acc += t2m - t2;
            et[2] = (i == 0 || j == 0) ? T(0) : acc;
        }
        // E-update transposes at the node
        T u[3], en[3], epre[3];
        if (FULL && in_lor(d, i, j, k)) {
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                AdjE<T> r = et_node(d, cc, i, j, k, et[cc], rs, ws, true);
                en[cc] = r.en;
                epre[cc] = r.epre;
                u[cc] = e_masked(cc, i, j, k) ? T(0) : S * r.coef * r.epre;
            }
        } else {
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                en[cc] = et[cc];
                epre[cc] = et[cc];
                u[cc] = e_masked(cc, i, j, k) ? T(0) : S * cu.ei[cc] * et[cc];
            }
        }
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            ew[cc][f] = en[cc];
            uw[cc][f] = u[cc];
        }
        // E-side memory cotangents (owner): psibar <- b (psibar + ybar), ybar = +u (term 0), -u (term 1)
        if (sy) {
            int q = poff(d, 1, cy.side, i, j, k);
            if (j > 0 && k > 0) gp(d.psiEa[1][cy.side][0] + wo)[q] = cy.bE * (cu.pe[0] + u[0]);    // Ex t0
            if (i > 0 && j > 0) gp(d.psiEa[1][cy.side][1] + wo)[q] = cy.bE * (cu.pe[1] + -u[2]);   // Ez t1
        }
        if (sz) {
            int q = poff(d, 2, cz.side, i, j, k);
            if (i > 0 && k > 0) gp(d.psiEa[2][cz.side][0] + wo)[q] = cz.bE * (cu.pe[2] + u[1]);    // Ey t0
            if (j > 0 && k > 0) gp(d.psiEa[2][cz.side][1] + wo)[q] = cz.bE * (cu.pe[3] + -u[0]);   // Ex t1
        }
        if (sx) {
            int q = poff(d, 0, cx.side, i, j, k);
            if (i > 0 && j > 0) gp(d.psiEa[0][cx.side][0] + wo)[q] = cx.bE * (cu.pe[4] + u[2]);    // Ez t0
            if (i > 0 && k > 0) gp(d.psiEa[0][cx.side][1] + wo)[q] = cx.bE * (cu.pe[5] + -u[1]);   // Ey t1
        }
        // dJ/deps from the forward state
        if (!FULL && in_gbox(d, i, j, k)) {
            // no absorber or Lorentz cell here: -S eps^-2 Ebar_pre curl with the plain curl
            const long long fo = (long long)fsr * d.fs;
            const FDTD_GLOBAL T* hf[3] = {gp(d.H[0] + fo), gp(d.H[1] + fo), gp(d.H[2] + fo)};
            const T fx = hf[0][f], fy = hf[1][f], fz = hf[2][f];
            const T fz_ym = j > 0 ? hf[2][f - d.pitch] : T(0), fx_ym = j > 0 ? hf[0][f - d.pitch] : T(0);
            const T fz_xm = i > 0 ? hf[2][f - 1] : T(0), fy_xm = i > 0 ? hf[1][f - 1] : T(0);
            const T fy_zm = k > 0 ? hf[1][f - pl] : T(0), fx_zm = k > 0 ? hf[0][f - pl] : T(0);
            const T curl[3] = {(fz - fz_ym) - (fy - fy_zm), (fx - fx_zm) - (fz - fz_xm), (fy - fy_xm) - (fx - fx_ym)};
            double g[3] = {0, 0, 0};
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
                if (!e_masked(cc, i, j, k))
                    g[cc] = -(double)epre[cc] * (double)(S * cu.ei[cc] * cu.ei[cc] * curl[cc]);
            grad_store(d, i, j, k, g);
        } else if (FULL && in_gbox(d, i, j, k)) {
            const long long fo = (long long)fsr * d.fs;
            T H[3], Hm[3][3];
            for (int q = 0; q < 3; ++q) H[q] = gp(d.H[q])[f + fo];
            for (int q = 0; q < 3; ++q) {
                Hm[0][q] = i > 0 ? gp(d.H[q])[f + fo - 1] : T(0);
                Hm[1][q] = j > 0 ? gp(d.H[q])[f + fo - d.pitch] : T(0);
                Hm[2][q] = k > 0 ? gp(d.H[q])[f + fo - pl] : T(0);
            }
            double g[3] = {0, 0, 0};
            for (int cc = 0; cc < 3; ++cc) {
                if (e_masked(cc, i, j, k)) continue;
                const int a0 = (cc + 1) % 3, a1 = (cc + 2) % 3, h0 = (cc + 2) % 3, h1 = (cc + 1) % 3;
                g[cc] = grad_term(d, cc, i, j, k, f, epre[cc], H[h0], Hm[a0][h0], H[h1], Hm[a1][h1], fsr);
            }
            grad_store(d, i, j, k, g);
        }
        hxm = cu.hx;
        hym = cu.hy;
        if (CZ) {
            pzm2 = cu.ph[2];
            pzm3 = cu.ph[3];
        }
        cu = nx;
    }
}

// Raw-difference cotangents of the six curl terms at one E node.
template <typename T>
struct Dbar6 {
    T x0, x1, y0, y1, z0, z1;   // component (x,y,z), term 0 (along c+1, +) or 1 (along c+2, -)
};

// Owner work at E node (i,j,k) from the cotangents etot[3]: E-update
// transposes, new cotangents of E^n (returned in en[3]), the six
// raw-difference cotangents, and dJ/deps from the forward state (set fsr).
template <typename T>
__device__ __forceinline__ Dbar6<T> et_cell(const DomDev<T>& d, int i, int j, int k, const T etot[3], int rs, int ws,
                                            bool own, int fsr, T en[3]) {
    long long f = fidx(d, i, j, k);
    Dbar6<T> o;
    T* dd[3][2] = {{&o.x0, &o.x1}, {&o.y0, &o.y1}, {&o.z0, &o.z1}};
    bool ing = own && in_gbox(d, i, j, k);
    T H[3] = {0, 0, 0}, Hm[3][3];   // forward H at the node and one step back along x, y, z
    if (ing) {
        const long long fo = fsr * d.fs;
        for (int q = 0; q < 3; ++q) H[q] = gp(d.H[q])[f + fo];
        for (int q = 0; q < 3; ++q) {
            Hm[0][q] = i > 0 ? gp(d.H[q])[f + fo - 1] : T(0);
            Hm[1][q] = j > 0 ? gp(d.H[q])[f + fo - d.pitch] : T(0);
            Hm[2][q] = k > 0 ? gp(d.H[q])[f + fo - d.plane] : T(0);
        }
    }
    double g[3] = {0, 0, 0};
    for (int cc = 0; cc < 3; ++cc) {
        AdjE<T> r = et_node(d, cc, i, j, k, etot[cc], rs, ws, own);
        en[cc] = r.en;
        const int a0 = (cc + 1) % 3, a1 = (cc + 2) % 3;
        if (e_masked(cc, i, j, k)) {
            *dd[cc][0] = T(0);
            *dd[cc][1] = T(0);
            continue;
        }
        *dd[cc][0] = et_dbar(d, a0, 0, T(1), i, j, k, r.epre, r.coef, rs, ws, own);
        *dd[cc][1] = et_dbar(d, a1, 1, T(-1), i, j, k, r.epre, r.coef, rs, ws, own);
        if (ing) {
            const int h0 = (cc + 2) % 3, h1 = (cc + 1) % 3;
            g[cc] = grad_term(d, cc, i, j, k, f, r.epre, H[h0], Hm[a0][h0], H[h1], Hm[a1][h1], fsr);
        }
    }
    if (ing) grad_store(d, i, j, k, g);
    return o;
}

// Raw-difference cotangent of term r of E_c at node (i,j,k) from its scaled
// cotangent u and the memory cotangent of set rs (read only): ybar = +u
// (term 0) or -u (term 1) through the transposed absorber recursion.
template <typename T>
__device__ __forceinline__ T u_dbar(const DomDev<T>& d, int c, int r, int i, int j, int k, T u, int rs) {
    if (e_masked(c, i, j, k)) return T(0);
    const int a = r == 0 ? (c + 1) % 3 : (c + 2) % 3;
    return stretch_T(d, d.psiEa, rs, rs, false, a, r, 0, i, j, k, r == 0 ? u : -u);
}

template <typename T>
struct AdjColH {
    T u1[3];                          // U one plane up
    T uy_xp, uz_xp, ux_yp, uz_yp;     // U one step forward along x and y
    T hb[3];                          // Hbar at the node (set rs)
    T ph[6];                          // H-side memory cotangents at the node (psi_load order)
    T pe1[6];                         // E-side memory cotangents one plane up
    T pex[2], pey[2];                 // at (i+1): x-slab slots 4, 5; at (j+1): y-slab slots 0, 1
};

template <typename T, int V>
__device__ __forceinline__ void adjh_fetch(const DomDev<T>& d, AdjColH<T>& p, const FDTD_GLOBAL T* const (&u)[3],
                                           const FDTD_GLOBAL T* const (&h)[3], long long f, const Cpml1<T>& cx,
                                           const Cpml1<T>& cy, const Cpml1<T>& cxp, const Cpml1<T>& cyp, long long ro,
                                           int i, int j, int k) {
    const bool up = k + 1 < d.n[2];
    const long long pl = d.plane;
    p.u1[0] = up ? u[0][f + pl] : T(0);
    p.u1[1] = up ? u[1][f + pl] : T(0);
    p.u1[2] = up ? u[2][f + pl] : T(0);
    p.uy_xp = i + 1 < d.n[0] ? u[1][f + 1] : T(0);
    p.uz_xp = i + 1 < d.n[0] ? u[2][f + 1] : T(0);
    p.ux_yp = j + 1 < d.n[1] ? u[0][f + d.pitch] : T(0);
    p.uz_yp = j + 1 < d.n[1] ? u[2][f + d.pitch] : T(0);
    p.hb[0] = h[0][f];
    p.hb[1] = h[1][f];
    p.hb[2] = h[2][f];
    if (V & 1) {
        psi_axis(d, d.psiHa, ro, 0, cx, i, j, k, p.ph[4], p.ph[5]);
        p.pe1[4] = p.pe1[5] = T(0);
        if (up) psi_axis(d, d.psiEa, ro, 0, cx, i, j, k + 1, p.pe1[4], p.pe1[5]);
        psi_axis(d, d.psiEa, ro, 0, cxp, i + 1, j, k, p.pex[0], p.pex[1]);
    }
    if (V & 2) {
        psi_axis(d, d.psiHa, ro, 1, cy, i, j, k, p.ph[0], p.ph[1]);
        p.pe1[0] = p.pe1[1] = T(0);
        if (up) psi_axis(d, d.psiEa, ro, 1, cy, i, j, k + 1, p.pe1[0], p.pe1[1]);
        psi_axis(d, d.psiEa, ro, 1, cyp, i, j + 1, k, p.pey[0], p.pey[1]);
    }
    if (V & 4) {
        psi_axis(d, d.psiHa, ro, 2, cpml_at(d, 2, k), i, j, k, p.ph[2], p.ph[3]);
        p.pe1[2] = p.pe1[3] = T(0);
        if (up) psi_axis(d, d.psiEa, ro, 2, cpml_at(d, 2, k + 1), i, j, k + 1, p.pe1[2], p.pe1[3]);
    }
}

// the six raw-difference cotangents of the E node (i,j,k) from its U and its
// E-side memory cotangents pe (psi_load order); masked components give zero
template <typename T>
__device__ __forceinline__ Dbar6<T> dbar6(int i, int j, int k, T ux, T uy, T uz, const T pe[6], bool sx, bool sy,
                                          bool sz, const Cpml1<T>& cx, const Cpml1<T>& cy, const Cpml1<T>& cz) {
    Dbar6<T> o;
    const bool mx = j == 0 || k == 0, my = i == 0 || k == 0, mz = i == 0 || j == 0;
    o.x0 = mx ? T(0) : tr_term(sy, cy.kE, cy.cE, pe[0], ux);     // Ex term 0 along y
    o.x1 = mx ? T(0) : tr_term(sz, cz.kE, cz.cE, pe[3], -ux);    // Ex term 1 along z
    o.y0 = my ? T(0) : tr_term(sz, cz.kE, cz.cE, pe[2], uy);     // Ey term 0 along z
    o.y1 = my ? T(0) : tr_term(sx, cx.kE, cx.cE, pe[5], -uy);    // Ey term 1 along x
    o.z0 = mz ? T(0) : tr_term(sx, cx.kE, cx.cE, pe[4], uz);     // Ez term 0 along x
    o.z1 = mz ? T(0) : tr_term(sy, cy.kE, cy.cE, pe[1], -uz);    // Ez term 1 along y
    return o;
}

template <typename T, int V, int W>
__device__ __forceinline__ void adj_et_tile(const DomDev<T>* __restrict__ doms, const int4 tile, int kz, int rs,
                                            int ws) {
    const DomDev<T>* dp;
    const TileCol<W> c = tile_column<T, W>(doms, tile, kz, dp);
    if (!c.ok) return;
    const DomDev<T>& d = *dp;
    if (!d.grad) return;
    const int i = c.i, j = c.j, nx = d.n[0], ny = d.n[1], nz = d.n[2];
    const long long ro = (long long)rs * d.as, wo = (long long)ws * d.as, pl = d.plane;
    const FDTD_GLOBAL T* u[3] = {gp(d.Et[0]), gp(d.Et[1]), gp(d.Et[2])};
    const FDTD_GLOBAL T* h[3] = {gp(d.Ha[0] + ro), gp(d.Ha[1] + ro), gp(d.Ha[2] + ro)};
    FDTD_GLOBAL T* hw[3] = {gp(d.Ha[0] + wo), gp(d.Ha[1] + wo), gp(d.Ha[2] + wo)};
    constexpr bool CX = V & 1, CY = V & 2, CZ = V & 4;
    const Cpml1<T> cx = cpml_at(d, 0, i), cy = cpml_at(d, 1, j), cxp = cpml_at(d, 0, i + 1), cyp = cpml_at(d, 1, j + 1);
    const T S = d.S, mS = -d.S;
    long long f = (long long)c.k0 * pl + (long long)j * d.pitch + i;
    Dbar6<T> cur;
    {
        T pe[6] = {0, 0, 0, 0, 0, 0};
        const Cpml1<T> cz = cpml_at(d, 2, c.k0);
        if (CX) psi_axis(d, d.psiEa, ro, 0, cx, i, j, c.k0, pe[4], pe[5]);
        if (CY) psi_axis(d, d.psiEa, ro, 1, cy, i, j, c.k0, pe[0], pe[1]);
        if (CZ) psi_axis(d, d.psiEa, ro, 2, cz, i, j, c.k0, pe[2], pe[3]);
        cur = dbar6(i, j, c.k0, u[0][f], u[1][f], u[2][f], pe, CX && cx.side >= 0, CY && cy.side >= 0,
                    CZ && cz.side >= 0, cx, cy, cz);
    }
    AdjColH<T> cu, nx_;
    adjh_fetch<T, V>(d, cu, u, h, f, cx, cy, cxp, cyp, ro, i, j, c.k0);
    for (int k = c.k0; k < c.k1; ++k, f += pl) {
        if (k + 1 < c.k1) adjh_fetch<T, V>(d, nx_, u, h, f + pl, cx, cy, cxp, cyp, ro, i, j, k + 1);
        const Cpml1<T> cz = cpml_at(d, 2, k), czp = cpml_at(d, 2, k + 1);
        const bool sx = CX && cx.side >= 0, sy = CY && cy.side >= 0, sz = CZ && cz.side >= 0;
        // E terms of the plane above (all six: they are the next plane's own terms)
        Dbar6<T> up{};
        if (k + 1 < nz)
            up = dbar6(i, j, k + 1, cu.u1[0], cu.u1[1], cu.u1[2], cu.pe1, sx, sy, CZ && czp.side >= 0, cx, cy, czp);
        // x neighbour: Ez term 0 and Ey term 1 (along x); y neighbour: Ez term 1 and Ex term 0 (along y)
        T xp_z0 = 0, xp_y1 = 0, yp_z1 = 0, yp_x0 = 0;
        if (i + 1 < nx) {
            const bool s = CX && cxp.side >= 0;
            if (j > 0) xp_z0 = tr_term(s, cxp.kE, cxp.cE, cu.pex[0], cu.uz_xp);
            if (k > 0) xp_y1 = tr_term(s, cxp.kE, cxp.cE, cu.pex[1], -cu.uy_xp);
        }
        if (j + 1 < ny) {
            const bool s = CY && cyp.side >= 0;
            if (i > 0) yp_z1 = tr_term(s, cyp.kE, cyp.cE, cu.pey[1], -cu.uz_yp);
            if (k > 0) yp_x0 = tr_term(s, cyp.kE, cyp.cE, cu.pey[0], cu.ux_yp);
        }
        T hbx = cu.hb[0], hby = cu.hb[1], hbz = cu.hb[2];
        // H-side memory cotangents of this node (owner): psibar <- b (psibar + ybar), ybar = -S sign Hbar
        if (sy) {
            int q = poff(d, 1, cy.side, i, j, k);
            gp(d.psiHa[1][cy.side][0] + wo)[q] = cy.bH * (cu.ph[0] + mS * hbx);   // Hx term 0 along y
            gp(d.psiHa[1][cy.side][1] + wo)[q] = cy.bH * (cu.ph[1] + S * hbz);    // Hz term 1 along y
        }
        if (sz) {
            int q = poff(d, 2, cz.side, i, j, k);
            gp(d.psiHa[2][cz.side][0] + wo)[q] = cz.bH * (cu.ph[2] + mS * hby);   // Hy term 0 along z
            gp(d.psiHa[2][cz.side][1] + wo)[q] = cz.bH * (cu.ph[3] + S * hbx);    // Hx term 1 along z
        }
        if (sx) {
            int q = poff(d, 0, cx.side, i, j, k);
            gp(d.psiHa[0][cx.side][0] + wo)[q] = cx.bH * (cu.ph[4] + mS * hbz);   // Hz term 0 along x
            gp(d.psiHa[0][cx.side][1] + wo)[q] = cx.bH * (cu.ph[5] + S * hby);    // Hy term 1 along x
        }
        hbx += (cur.y0 - up.y0) + (cur.z1 - yp_z1);
        hby += (cur.z0 - xp_z0) + (cur.x1 - up.x1);
        hbz += (cur.x0 - yp_x0) + (cur.y1 - xp_y1);
        hw[0][f] = hbx;
        hw[1][f] = hby;
        hw[2][f] = hbz;
        cur = up;
        cu = nx_;
    }
}

// One launch per adjoint pass over every tile class: the class of a tile
// selects the variant.  The host lays the table out so that the tiles each
// XCD receives form a contiguous spatial run of balanced cost (tiles of value
// (domain, xlen 0) are padding and return at once).
// The general class (Lorentz cells, gradient cells in a slab; rare) has a
// launch of its own, which keeps its registers out of the others.  In FP32
// both passes are held to 4 waves per SIMD (128 VGPRs, a few spills in the
// slab variants): measured faster than 3 waves without spills.  FP64 needs
// about twice the registers: at 4 waves it spilled over 300 VGPRs per lane;
// 3 waves (168 VGPRs, about 90 spills) measured fastest over the 212^3 and
// 536^3 workloads, 2 waves (no spills) gained less at 536^3.
template <typename T> constexpr int kAdjHtWaves = sizeof(T) == 8 ? 3 : 4;
template <typename T> constexpr int kAdjEtWaves = sizeof(T) == 8 ? 3 : 4;

template <typename T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kAdjHtWaves<T>, 8))) k_adj_ht(const DomDev<T>* __restrict__ doms, const int4* __restrict__ tiles,
                                                int kz, int rs, int ws, int fsr) {
    const int4 e = tiles[blockIdx.x];
    static_assert(kAdjClasses1 == 7, "one case per class");
    switch (e.x >> 24) {
    case 0: adj_ht_tile<T, 0, 32>(doms, e, kz, rs, ws, fsr); break;
    case 1: adj_ht_tile<T, 6, 32>(doms, e, kz, rs, ws, fsr); break;
    case 3: adj_ht_tile<T, 1, 16>(doms, e, kz, rs, ws, fsr); break;
    case 4: adj_ht_tile<T, 7, 16>(doms, e, kz, rs, ws, fsr); break;
    case 6: adj_ht_tile<T, 6, 16>(doms, e, kz, rs, ws, fsr); break;
    default: break;   // general classes 2 and 5: k_adj_ht_full
    }
}

// The general class in FP32 just exceeds 128 VGPRs with the loop over poles;
// held to 4 waves (2 spills) it measured 269 us against 318 us at 3 waves on
// the 536^3 workload's dispersive box.
template <typename T> constexpr int kAdjFullWaves = sizeof(T) == 8 ? 2 : 4;

template <typename T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kAdjFullWaves<T>, 8))) k_adj_ht_full(const DomDev<T>* __restrict__ doms,
                                                     const int4* __restrict__ tiles, int kz, int rs, int ws, int fsr) {
    const int4 e = tiles[blockIdx.x];
    if ((e.x >> 24) == 2) adj_ht_tile<T, kAdjFull, 32>(doms, e, kz, rs, ws, fsr);
    else adj_ht_tile<T, kAdjFull, 16>(doms, e, kz, rs, ws, fsr);
}

template <typename T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kAdjEtWaves<T>, 8)))
k_adj_et(const DomDev<T>* __restrict__ doms, const int4* __restrict__ tiles, int kz, int rs, int ws) {
    const int4 e = tiles[blockIdx.x];
    static_assert(kAdjClasses2 == 6, "one case per class");
    switch (e.x >> 24) {
    case 0: adj_et_tile<T, 0, 32>(doms, e, kz, rs, ws); break;
    case 1: adj_et_tile<T, 6, 32>(doms, e, kz, rs, ws); break;
    case 2: adj_et_tile<T, 7, 32>(doms, e, kz, rs, ws); break;
    case 3: adj_et_tile<T, 1, 16>(doms, e, kz, rs, ws); break;
    case 4: adj_et_tile<T, 7, 16>(doms, e, kz, rs, ws); break;
    default: adj_et_tile<T, 6, 16>(doms, e, kz, rs, ws); break;
    }
}

// ============================================================ fused tiles
constexpr int kWaves = 4;

struct Tile {
    int X0, Y0, k0, k1, lane, w;
    bool gen;   // tile touches absorbers, PEC faces, the Lorentz box or a source
};

// Tile-table entry: (domain, X0, Y0, k0); the block covers x in [X0, X0+64),
// rows [Y0, Y0 + 4R) and planes [k0, k1) (+ one halo plane on each side).
template <typename T, int R>
__device__ __forceinline__ Tile fused_tile(const DomDev<T>& d, int4 e, int kz) {
    Tile tl;
    tl.X0 = e.y;
    tl.Y0 = e.z;
    tl.k0 = e.w;
    tl.k1 = min(tl.k0 + kz, d.n[2]);
    tl.lane = threadIdx.x & 63;
    tl.w = threadIdx.x >> 6;
    // block-uniform classification
    int xlo = tl.X0, xhi = tl.X0 + 63, ylo = tl.Y0, yhi = tl.Y0 + kWaves * R - 1, zlo = tl.k0 - 1, zhi = tl.k1;
    bool g = xlo <= 0 || ylo <= 0 || zlo <= 0;
    int lo[3] = {xlo, ylo, zlo}, hi[3] = {xhi, yhi, zhi};
    for (int a = 0; a < 3; ++a) {
        if (d.L[a][0] > 0 && lo[a] < d.L[a][0]) g = true;
        if (d.L[a][1] > 0 && hi[a] >= d.n[a] - d.L[a][1]) g = true;
    }
    if (d.has_lor && hi[0] >= d.llo[0] && lo[0] < d.lhi[0] && hi[1] >= d.llo[1] && lo[1] < d.lhi[1] &&
        hi[2] >= d.llo[2] && lo[2] < d.lhi[2])
        g = true;
    for (int s = 0; s < d.nsrc; ++s) {
        const SrcDev<T>& sr = d.src[s];
        if (sr.k >= lo[2] && sr.k <= hi[2] &&
            (sr.kind == 1 || (sr.i >= lo[0] && sr.i <= hi[0] && sr.j >= lo[1] && sr.j <= hi[1])))
            g = true;
    }
    tl.gen = g;
    return tl;
}

// ============================================================ forward, fused
template <typename T, int R, bool GEN>
__device__ __forceinline__ void fwd_fused_body(const DomDev<T>& d, const Tile& tl, int rs, int ws, int t) {
    __shared__ T sH[2][kWaves][2][64];   // row R-1 of each wave: Hx, Hz of the newest H plane
    __shared__ T sE[2][kWaves][2][64];   // row 0 of each wave: Ex, Ez of the newest E^{n+1} plane
    const int nx = d.n[0], ny = d.n[1], nz = d.n[2];
    const int lane = tl.lane, w = tl.w;
    const int i = tl.X0 + lane;
    const bool ix = i >= 0 && i < nx;
    const long long ro = rs * d.fs, wo = ws * d.fs;
    int jr[R];
    bool vr[R], ecomp[R], own[R];
    for (int r = 0; r < R; ++r) {
        int row = w * R + r;
        jr[r] = tl.Y0 + row;
        vr[r] = ix && jr[r] >= 0 && jr[r] < ny;
        ecomp[r] = vr[r] && lane >= 1 && row >= 1;
        own[r] = vr[r] && lane >= 1 && lane <= 62 && row >= 1 && row <= kWaves * R - 2;
    }
    T Hk[R][3], Ek[R][3];     // H^{n+1/2} and E^{n+1} at plane k
    for (int r = 0; r < R; ++r)
        for (int q = 0; q < 3; ++q) {
            Hk[r][q] = T(0);
            Ek[r][q] = T(0);
        }
    if (tl.k0 > 0)
        for (int r = 0; r < R; ++r)
            if (vr[r]) {
                long long f = fidx(d, i, jr[r], tl.k0 - 1) + ro;
                Hk[r][0] = gp(d.H[0])[f];
                Hk[r][1] = gp(d.H[1])[f];
            }
    for (int k = tl.k0 - 1; k < tl.k1; ++k) {
        const int kn = k + 1;             // plane of the E update
        const bool have_n = kn < nz;
        T Hn[R][3], En[R][3];
        for (int r = 0; r < R; ++r) {
            Hn[r][0] = Hn[r][1] = Hn[r][2] = T(0);
            if (vr[r] && have_n) {
                long long f = fidx(d, i, jr[r], kn) + ro;
                Hn[r][0] = gp(d.H[0])[f];
                Hn[r][1] = gp(d.H[1])[f];
                Hn[r][2] = gp(d.H[2])[f];
            }
        }
        const int pb = kn & 1;
        sH[pb][w][0][lane] = Hn[R - 1][0];
        sH[pb][w][1][lane] = Hn[R - 1][2];
        __syncthreads();
        T hx_ym0 = w > 0 ? sH[pb][w - 1][0][lane] : T(0);
        T hz_ym0 = w > 0 ? sH[pb][w - 1][1][lane] : T(0);
        // ---- E^{n+1} at plane kn
        for (int r = 0; r < R; ++r) {
            T hy_xm = __shfl_up(Hn[r][1], 1);
            T hz_xm = __shfl_up(Hn[r][2], 1);
            T hx_ym = r > 0 ? Hn[r - 1][0] : hx_ym0;
            T hz_ym = r > 0 ? Hn[r - 1][2] : hz_ym0;
            En[r][0] = En[r][1] = En[r][2] = T(0);
            if (ecomp[r] && have_n) {
                const int j = jr[r];
                long long f = fidx(d, i, j, kn);
                bool o = own[r] && kn >= tl.k0 && kn < tl.k1;
                if (GEN) {
                    En[r][0] = e_update(d, 0, i, j, kn, f, Hn[r][2], hz_ym, Hn[r][1], Hk[r][1], rs, ws, o, t);
                    En[r][1] = e_update(d, 1, i, j, kn, f, Hn[r][0], Hk[r][0], Hn[r][2], hz_xm, rs, ws, o, t);
                    En[r][2] = e_update(d, 2, i, j, kn, f, Hn[r][1], hy_xm, Hn[r][0], hx_ym, rs, ws, o, t);
                } else {
                    En[r][0] = e_bulk(d, 0, i, j, kn, f, Hn[r][2], hz_ym, Hn[r][1], Hk[r][1], rs);
                    En[r][1] = e_bulk(d, 1, i, j, kn, f, Hn[r][0], Hk[r][0], Hn[r][2], hz_xm, rs);
                    En[r][2] = e_bulk(d, 2, i, j, kn, f, Hn[r][1], hy_xm, Hn[r][0], hx_ym, rs);
                }
                if (o) {
                    gp(d.E[0])[f + wo] = En[r][0];
                    gp(d.E[1])[f + wo] = En[r][1];
                    gp(d.E[2])[f + wo] = En[r][2];
                }
            }
        }
        // ---- H^{n+3/2} at plane k (uses E^{n+1} at k from the previous pass)
        if (k >= tl.k0) {
            const int pk = k & 1;
            T ex_yp3 = w + 1 < kWaves ? sE[pk][w + 1][0][lane] : T(0);
            T ez_yp3 = w + 1 < kWaves ? sE[pk][w + 1][1][lane] : T(0);
            for (int r = 0; r < R; ++r) {
                T ey_xp = __shfl_down(Ek[r][1], 1);
                T ez_xp = __shfl_down(Ek[r][2], 1);
                T ex_yp = r + 1 < R ? Ek[r + 1][0] : ex_yp3;
                T ez_yp = r + 1 < R ? Ek[r + 1][2] : ez_yp3;
                if (own[r]) {
                    const int j = jr[r];
                    long long f = fidx(d, i, j, k);
                    T hx, hy, hz;
                    if (GEN) {
                        hx = h_update(d, 0, i, j, k, Hk[r][0], ez_yp, Ek[r][2], En[r][1], Ek[r][1], rs, ws, true);
                        hy = h_update(d, 1, i, j, k, Hk[r][1], En[r][0], Ek[r][0], ez_xp, Ek[r][2], rs, ws, true);
                        hz = h_update(d, 2, i, j, k, Hk[r][2], ey_xp, Ek[r][1], ex_yp, Ek[r][0], rs, ws, true);
                    } else {
                        hx = h_bulk(d, Hk[r][0], ez_yp, Ek[r][2], En[r][1], Ek[r][1]);
                        hy = h_bulk(d, Hk[r][1], En[r][0], Ek[r][0], ez_xp, Ek[r][2]);
                        hz = h_bulk(d, Hk[r][2], ey_xp, Ek[r][1], ex_yp, Ek[r][0]);
                    }
                    gp(d.H[0])[f + wo] = hx;
                    gp(d.H[1])[f + wo] = hy;
                    gp(d.H[2])[f + wo] = hz;
                }
            }
        }
        sE[pb][w][0][lane] = En[0][0];
        sE[pb][w][1][lane] = En[0][2];
        for (int r = 0; r < R; ++r)
            for (int q = 0; q < 3; ++q) {
                Hk[r][q] = Hn[r][q];
                Ek[r][q] = En[r][q];
            }
    }
}

template <typename T, int R>
__global__ void __launch_bounds__(256) k_fwd_fused(const DomDev<T>* __restrict__ doms, const int4* __restrict__ tiles,
                                                   int kz, int rs, int ws, int t) {
    const int4 e = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const DomDev<T>& d = doms[e.x];
    Tile tl = fused_tile<T, R>(d, e, kz);
    fwd_fused_body<T, R, true>(d, tl, rs, ws, t);
}

// ============================================================ adjoint, fused
// Same tiling; the E-like pass forms the cotangent of E^{n+1} (H transpose)
// and applies the E-update transpose at E nodes, the H-like pass applies the
// transposed backward differences to Hbar.  Exchanged between nodes are the
// raw-difference cotangents (absorber transpose already applied at their
// source node).
template <typename T, int R>
__device__ __forceinline__ void adj_fused_body(const DomDev<T>& d, const Tile& tl, int rs, int ws, int fsr) {
    __shared__ T sH[2][kWaves][2][64];   // row R-1: Hz term 1 (along y), Hx term 0 (along y)
    __shared__ T sE[2][kWaves][2][64];   // row 0: Ez term 1 (along y), Ex term 0 (along y)
    const int nx = d.n[0], ny = d.n[1], nz = d.n[2];
    const int lane = tl.lane, w = tl.w;
    const int i = tl.X0 + lane;
    const bool ix = i >= 0 && i < nx;
    const long long ro = rs * d.as, wo = ws * d.as;
    int jr[R];
    bool vr[R], ecomp[R], own[R];
    for (int r = 0; r < R; ++r) {
        int row = w * R + r;
        jr[r] = tl.Y0 + row;
        vr[r] = ix && jr[r] >= 0 && jr[r] < ny;
        ecomp[r] = vr[r] && lane >= 1 && row >= 1;
        own[r] = vr[r] && lane >= 1 && lane <= 62 && row >= 1 && row <= kWaves * R - 2;
    }
    // plane-k registers: Hbar input, H-term cotangents along z, E-term cotangents
    T Hbk[R][3], dHyz_k[R], dHxz_k[R];
    Dbar6<T> Dk[R];
    for (int r = 0; r < R; ++r) {
        Hbk[r][0] = Hbk[r][1] = Hbk[r][2] = T(0);
        dHyz_k[r] = dHxz_k[r] = T(0);
        Dk[r] = Dbar6<T>{};
    }
    if (tl.k0 > 0)
        for (int r = 0; r < R; ++r)
            if (vr[r]) {
                const int kk = tl.k0 - 1;
                long long f = fidx(d, i, jr[r], kk) + ro;
                dHyz_k[r] = hT_dbar(d, 2, 0, T(1), i, jr[r], kk, gp(d.Ha[1])[f], rs, rs, false);
                dHxz_k[r] = hT_dbar(d, 2, 1, T(-1), i, jr[r], kk, gp(d.Ha[0])[f], rs, rs, false);
            }
    for (int k = tl.k0 - 1; k < tl.k1; ++k) {
        const int kn = k + 1;
        const bool have_n = kn < nz;
        const bool hown_n = kn >= tl.k0 && kn < tl.k1;   // H nodes of plane kn belong to this chunk
        T Hbn[R][3];
        T dHxy[R], dHxz[R], dHyz[R], dHyx[R], dHzx[R], dHzy[R];
        for (int r = 0; r < R; ++r) {
            Hbn[r][0] = Hbn[r][1] = Hbn[r][2] = T(0);
            dHxy[r] = dHxz[r] = dHyz[r] = dHyx[r] = dHzx[r] = dHzy[r] = T(0);
            if (vr[r] && have_n) {
                const int j = jr[r];
                long long f = fidx(d, i, j, kn) + ro;
                Hbn[r][0] = gp(d.Ha[0])[f];
                Hbn[r][1] = gp(d.Ha[1])[f];
                Hbn[r][2] = gp(d.Ha[2])[f];
                bool o = own[r] && hown_n;
                dHxy[r] = hT_dbar(d, 1, 0, T(1), i, j, kn, Hbn[r][0], rs, ws, o);
                dHxz[r] = hT_dbar(d, 2, 1, T(-1), i, j, kn, Hbn[r][0], rs, ws, o);
                dHyz[r] = hT_dbar(d, 2, 0, T(1), i, j, kn, Hbn[r][1], rs, ws, o);
                dHyx[r] = hT_dbar(d, 0, 1, T(-1), i, j, kn, Hbn[r][1], rs, ws, o);
                dHzx[r] = hT_dbar(d, 0, 0, T(1), i, j, kn, Hbn[r][2], rs, ws, o);
                dHzy[r] = hT_dbar(d, 1, 1, T(-1), i, j, kn, Hbn[r][2], rs, ws, o);
            }
        }
        const int pb = kn & 1;
        sH[pb][w][0][lane] = dHzy[R - 1];
        sH[pb][w][1][lane] = dHxy[R - 1];
        __syncthreads();
        T dHzy_m0 = w > 0 ? sH[pb][w - 1][0][lane] : T(0);
        T dHxy_m0 = w > 0 ? sH[pb][w - 1][1][lane] : T(0);
        // ---- E-like pass at plane kn
        Dbar6<T> Dn[R];
        for (int r = 0; r < R; ++r) {
            T dHzx_m = __shfl_up(dHzx[r], 1);
            T dHyx_m = __shfl_up(dHyx[r], 1);
            T dHzy_m = r > 0 ? dHzy[r - 1] : dHzy_m0;
            T dHxy_m = r > 0 ? dHxy[r - 1] : dHxy_m0;
            Dn[r] = Dbar6<T>{};
            if (ecomp[r] && have_n) {
                const int j = jr[r];
                long long f = fidx(d, i, j, kn);
                bool o = own[r] && kn >= tl.k0 && kn < tl.k1;
                T et[3];
                // Ebar_e += [t1(p - e_a1) - t1(p)] + [t2(p - e_a2) - t2(p)]
                // Ex: t1 = Hy along z, t2 = Hz along y; Ey: t1 = Hz along x, t2 = Hx along z;
                // Ez: t1 = Hx along y, t2 = Hy along x
                T t1[3] = {dHyz[r], dHzx[r], dHxy[r]}, t1m[3] = {dHyz_k[r], dHzx_m, dHxy_m};
                T t2[3] = {dHzy[r], dHxz[r], dHyx[r]}, t2m[3] = {dHzy_m, dHxz_k[r], dHyx_m};
                for (int e = 0; e < 3; ++e) {
                    if (e_masked(e, i, j, kn)) {
                        et[e] = T(0);
                        continue;
                    }
                    T acc = gp(d.Ea[e])[f + ro];
                    acc += t1m[e] - t1[e];
                    acc += t2m[e] - t2[e];
                    et[e] = acc;
                }
                T en[3];
                Dn[r] = et_cell(d, i, j, kn, et, rs, ws, o, fsr, en);
                if (o) {
                    gp(d.Ea[0])[f + wo] = en[0];
                    gp(d.Ea[1])[f + wo] = en[1];
                    gp(d.Ea[2])[f + wo] = en[2];
                }
            }
        }
        // ---- H-like pass at plane k
        if (k >= tl.k0) {
            const int pk = k & 1;
            T z1_yp3 = w + 1 < kWaves ? sE[pk][w + 1][0][lane] : T(0);
            T x0_yp3 = w + 1 < kWaves ? sE[pk][w + 1][1][lane] : T(0);
            for (int r = 0; r < R; ++r) {
                T z0_xp = __shfl_down(Dk[r].z0, 1);
                T y1_xp = __shfl_down(Dk[r].y1, 1);
                T z1_yp = r + 1 < R ? Dk[r + 1].z1 : z1_yp3;
                T x0_yp = r + 1 < R ? Dk[r + 1].x0 : x0_yp3;
                if (own[r]) {
                    long long f = fidx(d, i, jr[r], k);
                    T hbx = Hbk[r][0], hby = Hbk[r][1], hbz = Hbk[r][2];
                    hbx += (Dk[r].y0 - Dn[r].y0) + (Dk[r].z1 - z1_yp);
                    hby += (Dk[r].z0 - z0_xp) + (Dk[r].x1 - Dn[r].x1);
                    hbz += (Dk[r].x0 - x0_yp) + (Dk[r].y1 - y1_xp);
                    gp(d.Ha[0])[f + wo] = hbx;
                    gp(d.Ha[1])[f + wo] = hby;
                    gp(d.Ha[2])[f + wo] = hbz;
                }
            }
        }
        sE[pb][w][0][lane] = Dn[0].z1;
        sE[pb][w][1][lane] = Dn[0].x0;
        for (int r = 0; r < R; ++r) {
            Hbk[r][0] = Hbn[r][0];
            Hbk[r][1] = Hbn[r][1];
            Hbk[r][2] = Hbn[r][2];
            dHyz_k[r] = dHyz[r];
            dHxz_k[r] = dHxz[r];
            Dk[r] = Dn[r];
        }
    }
}

template <typename T, int R>
__global__ void __launch_bounds__(256) k_adj_fused(const DomDev<T>* __restrict__ doms, const int4* __restrict__ tiles,
                                                   int kz, int rs, int ws, int fsr) {
    const int4 e = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const DomDev<T>& d = doms[e.x];
    if (!d.grad) return;
    Tile tl = fused_tile<T, R>(d, e, kz);
    adj_fused_body<T, R>(d, tl, rs, ws, fsr);
}

// ============================================================ plain tiles
// Every tile without Lorentz cells: ghost lanes and rows (outside the domain)
// read zero and write nothing, PEC nodes stay zero, soft sources are added,
// and with CP the absorber recursion is applied per term.  Absorber
// coefficients are loaded once per lane (x), per row (y) and per plane (z).
// The arithmetic of every node is that of e_update / h_update.

template <typename T, int R, bool CP>
__device__ __forceinline__ void fwd_plain_body(const DomDev<T>& d, int X0, int Y0, int k0, int k1, int rs, int ws,
                                               int t) {
    __shared__ T sH[2][kWaves][2][64];
    __shared__ T sE[2][kWaves][2][64];
    const int nx = d.n[0], ny = d.n[1], nz = d.n[2];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = X0 + lane;
    const bool ix = i >= 0 && i < nx;
    const int pitch = d.pitch, plane = (int)d.plane;
    const T S = d.S;
    const long long fso = (long long)rs * d.fs, fwo = (long long)ws * d.fs;
    const FDTD_GLOBAL T* __restrict__ rH0 = gp(d.H[0] + fso);
    const FDTD_GLOBAL T* __restrict__ rH1 = gp(d.H[1] + fso);
    const FDTD_GLOBAL T* __restrict__ rH2 = gp(d.H[2] + fso);
    const FDTD_GLOBAL T* __restrict__ rE0 = gp(d.E[0] + fso);
    const FDTD_GLOBAL T* __restrict__ rE1 = gp(d.E[1] + fso);
    const FDTD_GLOBAL T* __restrict__ rE2 = gp(d.E[2] + fso);
    FDTD_GLOBAL T* __restrict__ wH0 = gp(d.H[0] + fwo);
    FDTD_GLOBAL T* __restrict__ wH1 = gp(d.H[1] + fwo);
    FDTD_GLOBAL T* __restrict__ wH2 = gp(d.H[2] + fwo);
    FDTD_GLOBAL T* __restrict__ wE0 = gp(d.E[0] + fwo);
    FDTD_GLOBAL T* __restrict__ wE1 = gp(d.E[1] + fwo);
    FDTD_GLOBAL T* __restrict__ wE2 = gp(d.E[2] + fwo);
    const EpsView<T> ev = eps_view(d, X0, Y0, kWaves * R, k0 - 1, k1);
    int jr[R], ro[R];
    bool vr[R], own[R], ecomp[R];
    Cpml1<T> cy[R];
    for (int r = 0; r < R; ++r) {
        int row = w * R + r;
        jr[r] = Y0 + row;
        vr[r] = ix && jr[r] >= 0 && jr[r] < ny;
        ro[r] = vr[r] ? jr[r] * pitch + i : 0;
        ecomp[r] = vr[r] && lane >= 1 && row >= 1;
        own[r] = vr[r] && lane >= 1 && lane <= 62 && row >= 1 && row <= kWaves * R - 2;
        if (CP) cy[r] = cpml_at(d, 1, jr[r]);
    }
    Cpml1<T> cx;
    if (CP) cx = cpml_at(d, 0, i);
    T Hk[R][3], Ek[R][3], Hp[R][3], Ep[R][3];
    T pEp[CP ? R : 1][6], pHp[CP ? R : 1][6];   // prefetched memories: E side at kn, H side at k
    for (int r = 0; r < R; ++r)
        for (int q = 0; q < 3; ++q) {
            Hk[r][q] = Ek[r][q] = Hp[r][q] = Ep[r][q] = T(0);
        }
    if (CP) {
        Cpml1<T> cz0 = cpml_at(d, 2, k0);
        for (int r = 0; r < R; ++r) psi_load(d, d.psiE, fso, vr[r], cx, cy[r], cz0, i, jr[r], k0, pEp[CP ? r : 0]);
        for (int r = 0; r < R; ++r)
            for (int q = 0; q < 6; ++q) pHp[CP ? r : 0][q] = T(0);
    }
    for (int r = 0; r < R; ++r) {
        if (!vr[r]) continue;
        if (k0 > 0) {
            int f = (k0 - 1) * plane + ro[r];
            Hk[r][0] = rH0[f];
            Hk[r][1] = rH1[f];
        }
        int f = k0 * plane + ro[r];
        Hp[r][0] = rH0[f];
        Hp[r][1] = rH1[f];
        Hp[r][2] = rH2[f];
        Ep[r][0] = rE0[f];
        Ep[r][1] = rE1[f];
        Ep[r][2] = rE2[f];
    }
    for (int k = k0 - 1; k < k1; ++k) {
        const int kn = k + 1;
        const bool have_n = kn < nz;
        T Hn[R][3], Eo[R][3];
        T pE[CP ? R : 1][6], pH[CP ? R : 1][6];
        for (int r = 0; r < R; ++r)
            for (int q = 0; q < 3; ++q) {
                Hn[r][q] = Hp[r][q];
                Eo[r][q] = Ep[r][q];
            }
        if (CP)
            for (int r = 0; r < R; ++r)
                for (int q = 0; q < 6; ++q) {
                    pE[CP ? r : 0][q] = pEp[CP ? r : 0][q];
                    pH[CP ? r : 0][q] = pHp[CP ? r : 0][q];
                }
        const bool pf = kn < k1 && kn + 1 < nz;
        if (pf) {
            for (int r = 0; r < R; ++r) {
                if (!vr[r]) continue;
                int f = (kn + 1) * plane + ro[r];
                Hp[r][0] = rH0[f];
                Hp[r][1] = rH1[f];
                Hp[r][2] = rH2[f];
                Ep[r][0] = rE0[f];
                Ep[r][1] = rE1[f];
                Ep[r][2] = rE2[f];
            }
        } else {
            for (int r = 0; r < R; ++r)
                for (int q = 0; q < 3; ++q) Hp[r][q] = Ep[r][q] = T(0);
        }
        if (CP) {
            // memories of the next E pass (plane kn+1) and of the next H pass (plane kn)
            Cpml1<T> czp = cpml_at(d, 2, kn + 1), czh = cpml_at(d, 2, kn);
            for (int r = 0; r < R; ++r) {
                psi_load(d, d.psiE, fso, vr[r] && pf, cx, cy[r], czp, i, jr[r], kn + 1, pEp[CP ? r : 0]);
                psi_load(d, d.psiH, fso, vr[r] && kn < k1, cx, cy[r], czh, i, jr[r], kn, pHp[CP ? r : 0]);
            }
        }
        const int pb = kn & 1;
        sH[pb][w][0][lane] = Hn[R - 1][0];
        sH[pb][w][1][lane] = Hn[R - 1][2];
        __syncthreads();
        T hx_ym0 = w > 0 ? sH[pb][w - 1][0][lane] : T(0);
        T hz_ym0 = w > 0 ? sH[pb][w - 1][1][lane] : T(0);
        const bool kin = kn >= k0 && kn < k1;
        Cpml1<T> czn;
        if (CP) czn = cpml_at(d, 2, kn);
        T En[R][3];
        for (int r = 0; r < R; ++r) {
            T hy_xm = __shfl_up(Hn[r][1], 1);
            T hz_xm = __shfl_up(Hn[r][2], 1);
            T hx_ym = r > 0 ? Hn[r - 1][0] : hx_ym0;
            T hz_ym = r > 0 ? Hn[r - 1][2] : hz_ym0;
            En[r][0] = En[r][1] = En[r][2] = T(0);
            if (ecomp[r] && have_n) {
                const int j = jr[r];
                const bool o = own[r] && kin;
                T ei[3];
                eps_at(ev, i, j, kn, ei);
                // raw differences of the six terms
                T Dx0 = Hn[r][2] - hz_ym, Dx1 = Hn[r][1] - Hk[r][1];   // Ex: Hz along y, Hy along z
                T Dy0 = Hn[r][0] - Hk[r][0], Dy1 = Hn[r][2] - hz_xm;   // Ey: Hx along z, Hz along x
                T Dz0 = Hn[r][1] - hy_xm, Dz1 = Hn[r][0] - hx_ym;      // Ez: Hy along x, Hx along y
                if (CP) {
                    const T* pe = pE[CP ? r : 0];
                    if (cy[r].side >= 0) {
                        int q = poff(d, 1, cy[r].side, i, j, kn);
                        Dx0 = st_pref(d.psiE[1][cy[r].side][0], fwo, q, o && j > 0 && kn > 0, cy[r].bE, cy[r].cE,
                                      cy[r].kE, pe[0], Dx0);
                        Dz1 = st_pref(d.psiE[1][cy[r].side][1], fwo, q, o && i > 0 && j > 0, cy[r].bE, cy[r].cE,
                                      cy[r].kE, pe[1], Dz1);
                    }
                    if (czn.side >= 0) {
                        int q = poff(d, 2, czn.side, i, j, kn);
                        Dy0 = st_pref(d.psiE[2][czn.side][0], fwo, q, o && i > 0 && kn > 0, czn.bE, czn.cE, czn.kE,
                                      pe[2], Dy0);
                        Dx1 = st_pref(d.psiE[2][czn.side][1], fwo, q, o && j > 0 && kn > 0, czn.bE, czn.cE, czn.kE,
                                      pe[3], Dx1);
                    }
                    if (cx.side >= 0) {
                        int q = poff(d, 0, cx.side, i, j, kn);
                        Dz0 = st_pref(d.psiE[0][cx.side][0], fwo, q, o && i > 0 && j > 0, cx.bE, cx.cE, cx.kE,
                                      pe[4], Dz0);
                        Dy1 = st_pref(d.psiE[0][cx.side][1], fwo, q, o && i > 0 && kn > 0, cx.bE, cx.cE, cx.kE,
                                      pe[5], Dy1);
                    }
                }
                T ex = fma(S * ei[0], Dx0 - Dx1, Eo[r][0]);
                T ey = fma(S * ei[1], Dy0 - Dy1, Eo[r][1]);
                T ez = fma(S * ei[2], Dz0 - Dz1, Eo[r][2]);
                for (int q = 0; q < d.nsrc; ++q) {
                    const SrcDev<T>& sr = d.src[q];
                    if (t < sr.nwave && kn == sr.k && (sr.kind == 1 || (i == sr.i && j == sr.j))) {
                        T v = gp(sr.wave)[t];
                        if (sr.comp == 0) ex += v;
                        else if (sr.comp == 1) ey += v;
                        else ez += v;
                    }
                }
                // PEC: E_c is zero where the index along c+1 or c+2 is 0
                if (j == 0 || kn == 0) ex = T(0);
                if (i == 0 || kn == 0) ey = T(0);
                if (i == 0 || j == 0) ez = T(0);
                En[r][0] = ex;
                En[r][1] = ey;
                En[r][2] = ez;
                if (o) {
                    int f = kn * plane + ro[r];
                    wE0[f] = ex;
                    wE1[f] = ey;
                    wE2[f] = ez;
                }
            }
        }
        if (k >= k0) {
            const int pk = k & 1;
            Cpml1<T> czk;
            if (CP) czk = cpml_at(d, 2, k);
            T ex_yp3 = w + 1 < kWaves ? sE[pk][w + 1][0][lane] : T(0);
            T ez_yp3 = w + 1 < kWaves ? sE[pk][w + 1][1][lane] : T(0);
            for (int r = 0; r < R; ++r) {
                T ey_xp = __shfl_down(Ek[r][1], 1);
                T ez_xp = __shfl_down(Ek[r][2], 1);
                T ex_yp = r + 1 < R ? Ek[r + 1][0] : ex_yp3;
                T ez_yp = r + 1 < R ? Ek[r + 1][2] : ez_yp3;
                if (own[r]) {
                    const int j = jr[r];
                    T Ax0 = ez_yp - Ek[r][2], Ax1 = En[r][1] - Ek[r][1];   // Hx: Ez along y, Ey along z
                    T Ay0 = En[r][0] - Ek[r][0], Ay1 = ez_xp - Ek[r][2];   // Hy: Ex along z, Ez along x
                    T Az0 = ey_xp - Ek[r][1], Az1 = ex_yp - Ek[r][0];      // Hz: Ey along x, Ex along y
                    if (CP) {
                        const T* ph = pH[CP ? r : 0];
                        if (cy[r].side >= 0) {
                            int q = poff(d, 1, cy[r].side, i, j, k);
                            Ax0 = st_pref(d.psiH[1][cy[r].side][0], fwo, q, true, cy[r].bH, cy[r].cH, cy[r].kH, ph[0],
                                          Ax0);
                            Az1 = st_pref(d.psiH[1][cy[r].side][1], fwo, q, true, cy[r].bH, cy[r].cH, cy[r].kH, ph[1],
                                          Az1);
                        }
                        if (czk.side >= 0) {
                            int q = poff(d, 2, czk.side, i, j, k);
                            Ay0 = st_pref(d.psiH[2][czk.side][0], fwo, q, true, czk.bH, czk.cH, czk.kH, ph[2], Ay0);
                            Ax1 = st_pref(d.psiH[2][czk.side][1], fwo, q, true, czk.bH, czk.cH, czk.kH, ph[3], Ax1);
                        }
                        if (cx.side >= 0) {
                            int q = poff(d, 0, cx.side, i, j, k);
                            Az0 = st_pref(d.psiH[0][cx.side][0], fwo, q, true, cx.bH, cx.cH, cx.kH, ph[4], Az0);
                            Ay1 = st_pref(d.psiH[0][cx.side][1], fwo, q, true, cx.bH, cx.cH, cx.kH, ph[5], Ay1);
                        }
                    }
                    int f = k * plane + ro[r];
                    wH0[f] = fma(-S, Ax0 - Ax1, Hk[r][0]);
                    wH1[f] = fma(-S, Ay0 - Ay1, Hk[r][1]);
                    wH2[f] = fma(-S, Az0 - Az1, Hk[r][2]);
                }
            }
        }
        sE[pb][w][0][lane] = En[0][0];
        sE[pb][w][1][lane] = En[0][2];
        for (int r = 0; r < R; ++r)
            for (int q = 0; q < 3; ++q) {
                Hk[r][q] = Hn[r][q];
                Ek[r][q] = En[r][q];
            }
    }
}

// ============================================================ adjoint, bulk tiles
// Tiles that lie inside the domain (no ghost nodes, no PEC nodes) and touch
// no absorber, Lorentz cell or source: plain transposed Yee arithmetic,
// 32-bit offsets, the next plane's loads issued before the current plane is
// processed.  Results equal the general path bitwise.
//
// Adjoint of a bulk tile.  Hbar and Ebar (set rs) -> set ws; dJ/deps inside
// the gradient box from the forward H (set fsr).  GRAD: the tile meets the
// gradient box.
template <typename T, int R, bool GRAD>
__device__ __forceinline__ void adj_bulk_body(const DomDev<T>& d, int X0, int Y0, int k0, int k1, int rs, int ws,
                                              int fsr) {
    __shared__ T sH[2][kWaves][4][64];   // row R-1: Hbar z, Hbar x, forward Hx, forward Hz
    __shared__ T sE[2][kWaves][2][64];   // row 0: Ez term 1, Ex term 0
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = X0 + lane;
    const int pitch = d.pitch, plane = (int)d.plane;
    const T S = d.S, mS = -d.S;          // -S*sgn for sgn = +1 and sgn = -1 (exact)
    const FDTD_GLOBAL T* __restrict__ rH0 = gp(d.Ha[0] + rs * d.as);
    const FDTD_GLOBAL T* __restrict__ rH1 = gp(d.Ha[1] + rs * d.as);
    const FDTD_GLOBAL T* __restrict__ rH2 = gp(d.Ha[2] + rs * d.as);
    const FDTD_GLOBAL T* __restrict__ rE0 = gp(d.Ea[0] + rs * d.as);
    const FDTD_GLOBAL T* __restrict__ rE1 = gp(d.Ea[1] + rs * d.as);
    const FDTD_GLOBAL T* __restrict__ rE2 = gp(d.Ea[2] + rs * d.as);
    FDTD_GLOBAL T* __restrict__ wH0 = gp(d.Ha[0] + ws * d.as);
    FDTD_GLOBAL T* __restrict__ wH1 = gp(d.Ha[1] + ws * d.as);
    FDTD_GLOBAL T* __restrict__ wH2 = gp(d.Ha[2] + ws * d.as);
    FDTD_GLOBAL T* __restrict__ wE0 = gp(d.Ea[0] + ws * d.as);
    FDTD_GLOBAL T* __restrict__ wE1 = gp(d.Ea[1] + ws * d.as);
    FDTD_GLOBAL T* __restrict__ wE2 = gp(d.Ea[2] + ws * d.as);
    const FDTD_GLOBAL T* __restrict__ fH0 = gp(d.H[0] + fsr * d.fs);
    const FDTD_GLOBAL T* __restrict__ fH1 = gp(d.H[1] + fsr * d.fs);
    const FDTD_GLOBAL T* __restrict__ fH2 = gp(d.H[2] + fsr * d.fs);
    const EpsView<T> ev = eps_view(d, X0, Y0, kWaves * R, k0 - 1, k1);
    int ro[R], jr[R];
    bool own[R], ecomp[R];
    for (int r = 0; r < R; ++r) {
        int row = w * R + r;
        jr[r] = Y0 + row;
        ro[r] = jr[r] * pitch + i;
        ecomp[r] = lane >= 1 && row >= 1;
        own[r] = lane >= 1 && lane <= 62 && row >= 1 && row <= kWaves * R - 2;
    }
    // plane-k registers: Hbar at k; forward Hx, Hy at k (gradient z-differences)
    T Hb[R][3], Fk[R][2];
    Dbar6<T> Dk[R];
    T Hbp[R][3], Ebp[R][3], Fp[R][3];   // prefetched plane
    for (int r = 0; r < R; ++r) {
        int f = (k0 - 1) * plane + ro[r];
        Hb[r][0] = rH0[f];
        Hb[r][1] = rH1[f];
        Hb[r][2] = T(0);
        Fk[r][0] = GRAD ? fH0[f] : T(0);
        Fk[r][1] = GRAD ? fH1[f] : T(0);
        Dk[r] = Dbar6<T>{};
        f += plane;
        Hbp[r][0] = rH0[f];
        Hbp[r][1] = rH1[f];
        Hbp[r][2] = rH2[f];
        Ebp[r][0] = rE0[f];
        Ebp[r][1] = rE1[f];
        Ebp[r][2] = rE2[f];
        if (GRAD) {
            Fp[r][0] = fH0[f];
            Fp[r][1] = fH1[f];
            Fp[r][2] = fH2[f];
        } else {
            Fp[r][0] = Fp[r][1] = Fp[r][2] = T(0);
        }
    }
    for (int k = k0 - 1; k < k1; ++k) {
        const int kn = k + 1;
        T Hn[R][3], Eo[R][3], Fn[R][3];
        for (int r = 0; r < R; ++r)
            for (int q = 0; q < 3; ++q) {
                Hn[r][q] = Hbp[r][q];
                Eo[r][q] = Ebp[r][q];
                Fn[r][q] = Fp[r][q];
            }
        if (kn < k1) {
            for (int r = 0; r < R; ++r) {
                int f = (kn + 1) * plane + ro[r];
                Hbp[r][0] = rH0[f];
                Hbp[r][1] = rH1[f];
                Hbp[r][2] = rH2[f];
                Ebp[r][0] = rE0[f];
                Ebp[r][1] = rE1[f];
                Ebp[r][2] = rE2[f];
                if (GRAD) {
                    Fp[r][0] = fH0[f];
                    Fp[r][1] = fH1[f];
                    Fp[r][2] = fH2[f];
                }
            }
        }
        const int pb = kn & 1;
        sH[pb][w][0][lane] = Hn[R - 1][2];
        sH[pb][w][1][lane] = Hn[R - 1][0];
        if (GRAD) {
            sH[pb][w][2][lane] = Fn[R - 1][0];
            sH[pb][w][3][lane] = Fn[R - 1][2];
        }
        __syncthreads();
        T hz_m0 = w > 0 ? sH[pb][w - 1][0][lane] : T(0);
        T hx_m0 = w > 0 ? sH[pb][w - 1][1][lane] : T(0);
        T fx_m0 = (GRAD && w > 0) ? sH[pb][w - 1][2][lane] : T(0);
        T fz_m0 = (GRAD && w > 0) ? sH[pb][w - 1][3][lane] : T(0);
        const bool kin = kn >= k0 && kn < k1;
        Dbar6<T> Dn[R];
        for (int r = 0; r < R; ++r) {
            // raw-difference cotangents of the H terms at the node: -S sgn Hbar
            T dHxy = mS * Hn[r][0], dHxz = S * Hn[r][0];
            T dHyz = mS * Hn[r][1], dHyx = S * Hn[r][1];
            T dHzx = mS * Hn[r][2], dHzy = S * Hn[r][2];
            T hz_xm = __shfl_up(Hn[r][2], 1), hy_xm = __shfl_up(Hn[r][1], 1);
            T dHzx_m = mS * hz_xm, dHyx_m = S * hy_xm;
            T dHzy_m = S * (r > 0 ? Hn[r - 1][2] : hz_m0);
            T dHxy_m = mS * (r > 0 ? Hn[r - 1][0] : hx_m0);
            T dHyz_k = mS * Hb[r][1], dHxz_k = S * Hb[r][0];
            T fy_xm = GRAD ? __shfl_up(Fn[r][1], 1) : T(0), fz_xm = GRAD ? __shfl_up(Fn[r][2], 1) : T(0);
            Dn[r] = Dbar6<T>{};
            if (ecomp[r]) {
                const int j = jr[r];
                T et0 = Eo[r][0], et1 = Eo[r][1], et2 = Eo[r][2];
                et0 += dHyz_k - dHyz;
                et0 += dHzy_m - dHzy;
                et1 += dHzx_m - dHzx;
                et1 += dHxz_k - dHxz;
                et2 += dHxy_m - dHxy;
                et2 += dHyx_m - dHyx;
                T ei[3];
                eps_at(ev, i, j, kn, ei);
                T c0 = S * ei[0], c1 = S * ei[1], c2 = S * ei[2];
                Dn[r].x0 = c0 * et0;
                Dn[r].x1 = -c0 * et0;
                Dn[r].y0 = c1 * et1;
                Dn[r].y1 = -c1 * et1;
                Dn[r].z0 = c2 * et2;
                Dn[r].z1 = -c2 * et2;
                if (own[r] && kin) {
                    int f = kn * plane + ro[r];
                    st_nt(wE0, f, et0);
                    st_nt(wE1, f, et1);
                    st_nt(wE2, f, et2);
                    if (GRAD && in_gbox(d, i, j, kn)) {
                        T fx_ym = r > 0 ? Fn[r - 1][0] : fx_m0, fz_ym = r > 0 ? Fn[r - 1][2] : fz_m0;
                        // forward curls: Ex (Hz along y, Hy along z), Ey (Hx along z, Hz along x), Ez (Hy along x, Hx along y)
                        T cx = (Fn[r][2] - fz_ym) - (Fn[r][1] - Fk[r][1]);
                        T cy = (Fn[r][0] - Fk[r][0]) - (Fn[r][2] - fz_xm);
                        T cz = (Fn[r][1] - fy_xm) - (Fn[r][0] - fx_ym);
                        double g[3];
                        g[0] = -(double)et0 * (double)(S * ei[0] * ei[0] * cx);
                        g[1] = -(double)et1 * (double)(S * ei[1] * ei[1] * cy);
                        g[2] = -(double)et2 * (double)(S * ei[2] * ei[2] * cz);
                        grad_store(d, i, j, kn, g);
                    }
                }
            }
        }
        if (k >= k0) {
            const int pk = k & 1;
            T z1_yp3 = w + 1 < kWaves ? sE[pk][w + 1][0][lane] : T(0);
            T x0_yp3 = w + 1 < kWaves ? sE[pk][w + 1][1][lane] : T(0);
            for (int r = 0; r < R; ++r) {
                T z0_xp = __shfl_down(Dk[r].z0, 1);
                T y1_xp = __shfl_down(Dk[r].y1, 1);
                T z1_yp = r + 1 < R ? Dk[r + 1].z1 : z1_yp3;
                T x0_yp = r + 1 < R ? Dk[r + 1].x0 : x0_yp3;
                if (own[r]) {
                    int f = k * plane + ro[r];
                    T hbx = Hb[r][0], hby = Hb[r][1], hbz = Hb[r][2];
                    hbx += (Dk[r].y0 - Dn[r].y0) + (Dk[r].z1 - z1_yp);
                    hby += (Dk[r].z0 - z0_xp) + (Dk[r].x1 - Dn[r].x1);
                    hbz += (Dk[r].x0 - x0_yp) + (Dk[r].y1 - y1_xp);
                    st_nt(wH0, f, hbx);
                    st_nt(wH1, f, hby);
                    st_nt(wH2, f, hbz);
                }
            }
        }
        sE[pb][w][0][lane] = Dn[0].z1;
        sE[pb][w][1][lane] = Dn[0].x0;
        for (int r = 0; r < R; ++r) {
            Hb[r][0] = Hn[r][0];
            Hb[r][1] = Hn[r][1];
            Hb[r][2] = Hn[r][2];
            Fk[r][0] = Fn[r][0];
            Fk[r][1] = Fn[r][1];
            Dk[r] = Dn[r];
        }
    }
}

template <typename T, int R>
__global__ void __launch_bounds__(256) k_adj_bulk(const DomDev<T>* __restrict__ doms, const int4* __restrict__ tiles,
                                                  int kz, int rs, int ws, int fsr) {
    const int4 e = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const DomDev<T>& d = doms[e.x];
    if (!d.grad) return;
    const int k1 = min(e.w + kz, d.n[2]);
    bool g = d.grad && e.y + 63 >= d.glo[0] && e.y < d.ghi[0] && e.z + kWaves * R - 1 >= d.glo[1] &&
             e.z < d.ghi[1] && k1 - 1 >= d.glo[2] && e.w < d.ghi[2];
    if (g) adj_bulk_body<T, R, true>(d, e.y, e.z, e.w, k1, rs, ws, fsr);
    else adj_bulk_body<T, R, false>(d, e.y, e.z, e.w, k1, rs, ws, fsr);
}

// ============================================================ monitors
// Sample one plane monitor (state set cs) into slot `slot` of its ring buffer
// [block][rcomp][npts] (E at time n, H at n + 1/2; flux: H at planes k and
// k-1, averaged by the spectrum update).  The split H kernel writes the same
// layout when it samples in-kernel.
template <typename T>
__global__ void k_sample(const DomDev<T>* __restrict__ doms, MonDev m, int cs, int slot) {
    const DomDev<T>& d = doms[m.dom];
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    int ni = m.i1 - m.i0, npts = ni * (m.j1 - m.j0);
    if (q >= npts) return;
    int i = m.i0 + q % ni, j = m.j0 + q / ni, k = m.k;
    long long f = fidx(d, i, j, k) + cs * d.fs;
    FDTD_GLOBAL T* buf = gp((T*)m.samples) + (long long)slot * m.rcomp * npts;
    const FDTD_GLOBAL T* Hx = gp(d.H[0]);
    const FDTD_GLOBAL T* Hy = gp(d.H[1]);
    if (m.kind == 1) {
        buf[q] = gp(d.E[0])[f];
        buf[npts + q] = gp(d.E[1])[f];
        buf[2 * npts + q] = Hx[f];
        buf[3 * npts + q] = k > 0 ? Hx[f - d.plane] : T(0);
        buf[4 * npts + q] = Hy[f];
        buf[5 * npts + q] = k > 0 ? Hy[f - d.plane] : T(0);
    } else {
        buf[q] = m.comp < 3 ? gp(d.E[m.comp])[f] : gp(d.H[m.comp - 3])[f];
    }
}

// Accumulate `count` buffered samples taken at steps n0 .. n0+count-1 into the
// FP64 spectra acc[f][comp][pt] += x * exp(-i w t), t = n (E) or n + 1/2 (H).
// grid.y = frequency; the block's twiddles sit in LDS.
template <typename T>
__global__ void k_dft(MonDev m, int n0, int count, const int* __restrict__ tdev) {
    __shared__ double tw[2][2][kMaxDftBlock];   // [E|H][cos|sin][sample]
    if (tdev) n0 += *tdev;
    int f = blockIdx.y;
    double w = m.omega[f];
    for (int s = threadIdx.x; s < count; s += blockDim.x) {
        double te = (double)(n0 + s), th = te + 0.5;
        double sn, cs;
        sincos(w * te, &sn, &cs);
        tw[0][0][s] = cs;
        tw[0][1][s] = sn;
        sincos(w * th, &sn, &cs);
        tw[1][0][s] = cs;
        tw[1][1][s] = sn;
    }
    __syncthreads();
    int npts = (m.i1 - m.i0) * (m.j1 - m.j0);
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npts) return;
    const T* buf = (const T*)m.samples;
    for (int cq = 0; cq < m.ncomp; ++cq) {
        int ish = (m.kind == 1) ? (cq >= 2) : (m.comp >= 3);
        // ring component(s) of spectrum component cq: flux <Hx>, <Hy> average planes k and k-1
        const int r0 = (m.kind == 1 && cq >= 2) ? 2 * cq - 2 : cq;
        double re = 0, im = 0;
        for (int s = 0; s < count; ++s) {
            const T* b = buf + (long long)s * m.rcomp * npts + q;
            const T v = (m.kind == 1 && cq >= 2) ? T(0.5) * (b[r0 * npts] + b[(r0 + 1) * npts]) : b[r0 * npts];
            double x = (double)v;
            re = fma(x, tw[ish][0][s], re);
            im = fma(-x, tw[ish][1][s], im);
        }
        double* a = m.acc + (((long long)f * m.ncomp + cq) * npts + q) * 2;
        a[0] += re;
        a[1] += im;
    }
}

template <typename T>
__global__ void k_probe(const DomDev<T>* __restrict__ doms, MonDev m, int cs, int n, const int* __restrict__ tdev) {
    const DomDev<T>& d = doms[m.dom];
    if (tdev) n += *tdev;
    if (n < 0 || n >= m.ntrace) return;
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        long long f = fidx(d, m.pi, m.pj, m.k) + cs * d.fs;
        m.trace[n] = (double)(m.comp < 3 ? d.E[m.comp][f] : d.H[m.comp - 3][f]);
    }
}

// Seeds dJ/du^n of one plane monitor into the cotangent state (set as_):
// Re sum_f G_f exp(+i w t), t = n (E) or n + 1/2 (H).
template <typename T>
__global__ void k_seed(const DomDev<T>* __restrict__ doms, MonDev m, int as_, int n) {
    const DomDev<T>& d = doms[m.dom];
    int npts = (m.i1 - m.i0) * (m.j1 - m.j0);
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npts) return;
    int ni = m.i1 - m.i0;
    int i = m.i0 + q % ni, j = m.j0 + q / ni, k = m.k;
    long long f = fidx(d, i, j, k) + as_ * d.as;
    for (int cq = 0; cq < m.ncomp; ++cq) {
        int comp = m.kind == 1 ? (cq < 2 ? cq : cq + 1) : m.comp;   // flux: Ex, Ey, Hx, Hy
        int ish = comp >= 3;
        double t = (double)n + (ish ? 0.5 : 0.0);
        double s = 0;
        for (int fr = 0; fr < m.nf; ++fr) {
            const double* g = m.cot + (((long long)fr * m.ncomp + cq) * npts + q) * 2;
            double sn, cs;
            sincos(m.omega[fr] * t, &sn, &cs);
            s += g[0] * cs - g[1] * sn;
        }
        if (m.kind == 1 && ish) {
            T* H = d.Ha[comp - 3];
            H[f] += (T)(0.5 * s);
            if (k > 0) H[f - d.plane] += (T)(0.5 * s);
        } else if (ish) {
            d.Ha[comp - 3][f] += (T)s;
        } else {
            d.Ea[comp][f] += (T)s;
        }
    }
}

template <typename T>
__global__ void k_probe_seed(const DomDev<T>* __restrict__ doms, MonDev m, int as_, int n) {
    const DomDev<T>& d = doms[m.dom];
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        long long f = fidx(d, m.pi, m.pj, m.k) + as_ * d.as;
        double g = m.cot[n - 1];
        if (m.comp < 3) d.Ea[m.comp][f] += (T)g;
        else d.Ha[m.comp - 3][f] += (T)g;
    }
}

// ============================================================ utilities
// device-resident step index of graph replays: set, or advance by the steps
// a replay has taken
__global__ void k_step_counter(int* __restrict__ c, int value, int add) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *c = add ? *c + value : value;
}

__global__ void __launch_bounds__(256) k_add_f64(double* __restrict__ y, const double* __restrict__ x, long long n) {
    for (long long q = (long long)blockIdx.x * 256 + threadIdx.x; q < n; q += (long long)gridDim.x * 256) y[q] += x[q];
}

__global__ void k_fill_zero(uint32_t* __restrict__ p, long long n_words) {
    long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; q < n_words; q += stride) p[q] = 0u;
}

__global__ void k_copy_words(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst, long long n_words) {
    long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; q < n_words; q += stride) dst[q] = src[q];
}

// ---- Reversible mode (Section 3.2): the forward fields of the lossless box R
// are rebuilt by stepping Eq. 1 backward, H first (from E^{m}), then E (from
// the rebuilt H^{m-1/2}); the values just outside R come from the per-step
// record of the interface.  Every cell of R runs the transposed order of its
// forward update with the opposite sign: H^{m-1/2} = H^{m+1/2} + S C^+ E^m,
// E^{m-1} = (E^m - s^m) - S eps^-1 C^- H^{m-1/2}.  Cells outside R are left
// stale: the adjoint reads the forward state only inside the gradient box.

// face f of domain d: axis a = f % 3, high = f >= 3; cell q -> (u, v) along
// the two other axes b = a+1, c = a+2 (u fastest)
template <typename T>
__device__ __forceinline__ void rev_face_cell(const DomDev<T>& d, int f, long long q, int& i, int& j, int& k) {
    const int a = f % 3, b = (a + 1) % 3, c = (a + 2) % 3;
    const int nb = d.rhi[b] - d.rlo[b];
    int x[3];
    x[a] = f >= 3 ? d.rhi[a] : d.rlo[a] - 1;
    x[b] = d.rlo[b] + (int)(q % nb);
    x[c] = d.rlo[c] + (int)(q / nb);
    i = x[0];
    j = x[1];
    k = x[2];
}

// copy the interface of the current state (set cs) into record slot `slot`:
// low faces H_{a+1}, H_{a+2} at index rlo_a - 1, high faces E_{a+1}, E_{a+2}
// at index rhi_a; grid y = domain
template <typename T>
__global__ void __launch_bounds__(256) k_rev_record(const DomDev<T>* __restrict__ doms, int cs, int slot) {
    const DomDev<T>& d = doms[blockIdx.y];
    if (!d.rev) return;
    const long long so = (long long)cs * d.fs;
    T* rec = d.rec + (long long)slot * d.rec_stride;
    for (int f = 0; f < 6; ++f) {
        if (d.rface[f] < 0) continue;
        const int a = f % 3;
        const long long cnt = d.rfcnt[a];
        for (long long q = (long long)blockIdx.x * 256 + threadIdx.x; q < cnt; q += (long long)gridDim.x * 256) {
            int i, j, k;
            rev_face_cell(d, f, q, i, j, k);
            const long long fi = fidx(d, i, j, k) + so;
            T* const* src = f >= 3 ? d.E : d.H;
            gp(rec)[d.rface[f] + q] = gp(src[(a + 1) % 3])[fi];
            gp(rec)[d.rface[f] + cnt + q] = gp(src[(a + 2) % 3])[fi];
        }
    }
}

// a recorded value: component r (0 -> a+1, 1 -> a+2) of face f at (i, j, k)
template <typename T>
__device__ __forceinline__ T rev_rec(const DomDev<T>& d, const T* rec, int f, int r, int i, int j, int k) {
    if (d.rface[f] < 0) return T(0);    // no absorbing slab there: the ghost zero
    const int a = f % 3, b = (a + 1) % 3;
    const int x[3] = {i, j, k};
    const long long q = (long long)(x[(a + 2) % 3] - d.rlo[(a + 2) % 3]) * (d.rhi[b] - d.rlo[b]) + (x[b] - d.rlo[b]);
    return gp(rec)[d.rface[f] + r * d.rfcnt[a] + q];
}

// E^m one step forward along axis a from a node of R: inside R from the field,
// on R's high face from the record (component c of E)
template <typename T>
__device__ __forceinline__ T rev_e_up(const DomDev<T>& d, const T* rec, const FDTD_GLOBAL T* e, long long f, int c,
                                      int a, int i, int j, int k) {
    const int x[3] = {i, j, k};
    if (x[a] + 1 < d.rhi[a]) return e[f + (a == 0 ? 1 : (a == 1 ? (long long)d.pitch : d.plane))];
    if (x[a] + 1 >= d.n[a]) return T(0);   // ghost
    int y[3] = {i, j, k};
    y[a] += 1;
    return rev_rec(d, rec, 3 + a, c == (a + 1) % 3 ? 0 : 1, y[0], y[1], y[2]);
}

template <typename T>
__device__ __forceinline__ T rev_h_down(const DomDev<T>& d, const T* rec, const FDTD_GLOBAL T* h, long long f, int c,
                                        int a, int i, int j, int k) {
    const int x[3] = {i, j, k};
    if (x[a] - 1 >= d.rlo[a]) return h[f - (a == 0 ? 1 : (a == 1 ? (long long)d.pitch : d.plane))];
    if (x[a] == 0) return T(0);             // ghost
    int y[3] = {i, j, k};
    y[a] -= 1;
    return rev_rec(d, rec, a, c == (a + 1) % 3 ? 0 : 1, y[0], y[1], y[2]);
}

// H^{m-1/2} over R from E^m (set rs) and H^{m+1/2} (set rs) into set ws,
// with the interface E^m of record slot m; grid y = domain, x over R's cells
template <typename T>
__global__ void __launch_bounds__(256) k_rev_h(const DomDev<T>* __restrict__ doms, int rs, int ws, int slot) {
    const DomDev<T>& d = doms[blockIdx.y];
    if (!d.rev) return;
    const int rx = d.rhi[0] - d.rlo[0], ry = d.rhi[1] - d.rlo[1], rz = d.rhi[2] - d.rlo[2];
    const long long ncell = (long long)rx * ry * rz;
    const T* rec = d.rec + (long long)slot * d.rec_stride;
    const long long so = (long long)rs * d.fs, wo = (long long)ws * d.fs;
    const FDTD_GLOBAL T* e[3] = {gp(d.E[0] + so), gp(d.E[1] + so), gp(d.E[2] + so)};
    const T S = d.S;
    for (long long q = (long long)blockIdx.x * 256 + threadIdx.x; q < ncell; q += (long long)gridDim.x * 256) {
        const int i = d.rlo[0] + (int)(q % rx), j = d.rlo[1] + (int)((q / rx) % ry), k = d.rlo[2] + (int)(q / ((long long)rx * ry));
        const long long f = fidx(d, i, j, k);
        const T ex = e[0][f], ey = e[1][f], ez = e[2][f];
        // Hx: d+_y Ez - d+_z Ey ; Hy: d+_z Ex - d+_x Ez ; Hz: d+_x Ey - d+_y Ex
        const T Dx0 = rev_e_up(d, rec, e[2], f, 2, 1, i, j, k) - ez, Dx1 = rev_e_up(d, rec, e[1], f, 1, 2, i, j, k) - ey;
        const T Dy0 = rev_e_up(d, rec, e[0], f, 0, 2, i, j, k) - ex, Dy1 = rev_e_up(d, rec, e[2], f, 2, 0, i, j, k) - ez;
        const T Dz0 = rev_e_up(d, rec, e[1], f, 1, 0, i, j, k) - ey, Dz1 = rev_e_up(d, rec, e[0], f, 0, 1, i, j, k) - ex;
        gp(d.H[0] + wo)[f] = fma(S, Dx0 - Dx1, gp(d.H[0] + so)[f]);
        gp(d.H[1] + wo)[f] = fma(S, Dy0 - Dy1, gp(d.H[1] + so)[f]);
        gp(d.H[2] + wo)[f] = fma(S, Dz0 - Dz1, gp(d.H[2] + so)[f]);
    }
}

// E^{m-1} over R from E^m (set rs) and H^{m-1/2} (set ws, written by k_rev_h)
// into set ws, with the interface H^{m-1/2} of record slot m - 1; the source
// value of forward step t = m - 1 is taken off before the curl term
template <typename T>
__global__ void __launch_bounds__(256) k_rev_e(const DomDev<T>* __restrict__ doms, int rs, int ws, int slot, int t) {
    const DomDev<T>& d = doms[blockIdx.y];
    if (!d.rev) return;
    const int rx = d.rhi[0] - d.rlo[0], ry = d.rhi[1] - d.rlo[1], rz = d.rhi[2] - d.rlo[2];
    const long long ncell = (long long)rx * ry * rz;
    const T* rec = d.rec + (long long)slot * d.rec_stride;
    const long long so = (long long)rs * d.fs, wo = (long long)ws * d.fs;
    const FDTD_GLOBAL T* h[3] = {gp(d.H[0] + wo), gp(d.H[1] + wo), gp(d.H[2] + wo)};
    const T S = d.S;
    for (long long q = (long long)blockIdx.x * 256 + threadIdx.x; q < ncell; q += (long long)gridDim.x * 256) {
        const int i = d.rlo[0] + (int)(q % rx), j = d.rlo[1] + (int)((q / rx) % ry), k = d.rlo[2] + (int)(q / ((long long)rx * ry));
        const long long f = fidx(d, i, j, k);
        const T hx = h[0][f], hy = h[1][f], hz = h[2][f];
        // Ex: d-_y Hz - d-_z Hy ; Ey: d-_z Hx - d-_x Hz ; Ez: d-_x Hy - d-_y Hx
        const T Dx0 = hz - rev_h_down(d, rec, h[2], f, 2, 1, i, j, k), Dx1 = hy - rev_h_down(d, rec, h[1], f, 1, 2, i, j, k);
        const T Dy0 = hx - rev_h_down(d, rec, h[0], f, 0, 2, i, j, k), Dy1 = hz - rev_h_down(d, rec, h[2], f, 2, 0, i, j, k);
        const T Dz0 = hy - rev_h_down(d, rec, h[1], f, 1, 0, i, j, k), Dz1 = hx - rev_h_down(d, rec, h[0], f, 0, 1, i, j, k);
        const T D[3] = {Dx0 - Dx1, Dy0 - Dy1, Dz0 - Dz1};
        for (int c = 0; c < 3; ++c) {
            if (e_masked(c, i, j, k)) {
                gp(d.E[c] + wo)[f] = T(0);
                continue;
            }
            T v = gp(d.E[c] + so)[f];
            for (int q2 = 0; q2 < d.nsrc; ++q2) {
                const SrcDev<T>& sr = d.src[q2];
                if (sr.comp == c && t < sr.nwave && k == sr.k && (sr.kind == 1 || (i == sr.i && j == sr.j)))
                    v -= gp(sr.wave)[t];
            }
            gp(d.E[c] + wo)[f] = fma(-S * epsinv_at(d, c, i, j, k), D[c], v);
        }
    }
}

// ---- Poynting flux of a plane spectrum (Section 2.4):
//   F(w_f) = Re sum_p (Ex Hy* - Ey Hx*),  spectra [nf][4][np] complex128.
// Two launches, no atomics, a fixed summation order: block (b, f) sums its
// contiguous run of points (each thread a strided subset), reduces across
// its wave with xor shuffles and across its 4 waves through LDS, and writes
// one partial; the second launch reduces the nblk partials of frequency f
// the same way.  The result depends only on (nf, np), never on timing.
__device__ __forceinline__ double block_sum(double s) {
    __shared__ double red[4];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void __launch_bounds__(256) k_flux_partial(const double2* __restrict__ sp, long long np, int nblk,
                                                      double* __restrict__ part) {
    const int f = blockIdx.y, b = blockIdx.x;
    const double2* a = sp + (long long)f * 4 * np;
    const long long chunk = (np + nblk - 1) / nblk, p0 = (long long)b * chunk, p1 = min(np, p0 + chunk);
    double s = 0.0;
    for (long long q = p0 + threadIdx.x; q < p1; q += 256) {
        const double2 ex = a[q], ey = a[np + q], hx = a[2 * np + q], hy = a[3 * np + q];
        s += (ex.x * hy.x + ex.y * hy.y) - (ey.x * hx.x + ey.y * hx.y);
    }
    s = block_sum(s);
    if (threadIdx.x == 0) part[(long long)f * nblk + b] = s;
}

__global__ void __launch_bounds__(256) k_flux_final(const double* __restrict__ part, int nblk,
                                                    double* __restrict__ out) {
    const int f = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) s += part[(long long)f * nblk + b];
    s = block_sum(s);
    if (threadIdx.x == 0) out[f] = s;
}

// Field energy of one domain (the watchdog's reduction): the sum of squares
// of its six fields over the grid (row padding skipped), FP64, as kEnergyBlocks
// partial sums over contiguous runs of elements, then one block reduces them;
// a fixed order, and a NaN or infinity anywhere makes the result non-finite.
template <typename T>
__global__ void __launch_bounds__(256) k_energy_partial(const DomDev<T>* __restrict__ doms, int dom, int cs,
                                                        double* __restrict__ part) {
    const DomDev<T>& d = doms[dom];
    const long long nx = d.n[0], n = nx * d.n[1] * d.n[2];
    const long long chunk = (n + kEnergyBlocks - 1) / kEnergyBlocks, q0 = (long long)blockIdx.x * chunk,
                    q1 = min(n, q0 + chunk);
    double s = 0.0;
    for (int c = 0; c < 6; ++c) {
        const FDTD_GLOBAL T* F = gp((c < 3 ? d.E[c] : d.H[c - 3]) + (long long)cs * d.fs);
        for (long long q = q0 + threadIdx.x; q < q1; q += 256) {
            const double v = (double)F[(q / nx) * d.pitch + q % nx];
            s = fma(v, v, s);
        }
    }
    s = block_sum(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// max |x| of an FP32 array into *out (as ordered bits; out pre-zeroed)
// ---- BF16 checkpoint slots.  The forward state arrays of all domains are
// listed in one table (BfArr); every array is cut into chunks of kBfChunk
// elements and each block takes one chunk, so a save is three launches
// (partial maxima, per-array scale, pack) and a restore one, whatever the
// number of arrays.  Array starts and slot offsets are 256-byte aligned, so a
// thread moves 8 elements as two float4 loads and one 16-byte bf16 store.

// array whose chunk block b belongs to (largest q with blk0 <= b)
__device__ inline int bf_array(const BfArr* __restrict__ a, int narr, int b) {
    int lo = 0, hi = narr - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a[mid].blk0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ inline float block_max(float m) {
    __shared__ float red[4];
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_down(m, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    return fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

// part[b] = max |x| over chunk b (no atomics; deterministic)
__global__ void __launch_bounds__(256) k_bf16_partmax(const BfArr* __restrict__ arr, int narr, long long shift,
                                                      float* __restrict__ part) {
    const int q = bf_array(arr, narr, blockIdx.x);
    const BfArr& A = arr[q];
    const float* x = (const float*)((const char*)A.p + shift);
    const long long e0 = (long long)(blockIdx.x - A.blk0) * kBfChunk;
    const long long e1 = min(e0 + kBfChunk, A.n);
    const long long v1 = e0 + ((e1 - e0) & ~7LL);
    float m = 0.f;
    for (long long v = e0 + 8 * threadIdx.x; v < v1; v += 8 * 256) {
        const float4 u = *(const float4*)(x + v);
        const float4 w = *(const float4*)(x + v + 4);
        m = fmaxf(m, fmaxf(fmaxf(fabsf(u.x), fabsf(u.y)), fmaxf(fabsf(u.z), fabsf(u.w))));
        m = fmaxf(m, fmaxf(fmaxf(fabsf(w.x), fabsf(w.y)), fmaxf(fabsf(w.z), fabsf(w.w))));
    }
    if (v1 + threadIdx.x < e1) m = fmaxf(m, fabsf(x[v1 + threadIdx.x]));
    m = block_max(m);
    if (threadIdx.x == 0) part[blockIdx.x] = m;
}

// scale[q] = max over the chunks of array q (one block per array)
__global__ void __launch_bounds__(256) k_bf16_scale(const BfArr* __restrict__ arr, const float* __restrict__ part,
                                                    unsigned int* __restrict__ scale) {
    const BfArr& A = arr[blockIdx.x];
    float m = 0.f;
    for (int b = threadIdx.x; b < A.nblk; b += 256) m = fmaxf(m, part[A.blk0 + b]);
    m = block_max(m);
    if (threadIdx.x == 0) scale[blockIdx.x] = __float_as_uint(m);
}

// x / scale rounded to bfloat16 (round to nearest even).  An array whose
// largest magnitude is below the smallest normal float (a slab the wave has not
// reached yet) is stored as zeros: 1/scale would overflow and 0 * inf is NaN.
__device__ inline uint32_t bf16_bits(float v) {
    const uint32_t u = __float_as_uint(v);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

__global__ void __launch_bounds__(256) k_bf16_pack(const BfArr* __restrict__ arr, int narr, long long shift,
                                                   const unsigned int* __restrict__ scale, char* __restrict__ slot) {
    const int q = bf_array(arr, narr, blockIdx.x);
    const BfArr& A = arr[q];
    const float* x = (const float*)((const char*)A.p + shift);
    uint16_t* y = (uint16_t*)(slot + A.boff);
    const float s = __uint_as_float(scale[q]);
    const float inv = s >= FLT_MIN ? 1.f / s : 0.f;
    const long long e0 = (long long)(blockIdx.x - A.blk0) * kBfChunk;
    const long long e1 = min(e0 + kBfChunk, A.n);
    const long long v1 = e0 + ((e1 - e0) & ~7LL);
    for (long long v = e0 + 8 * threadIdx.x; v < v1; v += 8 * 256) {
        const float4 u = *(const float4*)(x + v);
        const float4 w = *(const float4*)(x + v + 4);
        uint4 o;
        o.x = bf16_bits(u.x * inv) | (bf16_bits(u.y * inv) << 16);
        o.y = bf16_bits(u.z * inv) | (bf16_bits(u.w * inv) << 16);
        o.z = bf16_bits(w.x * inv) | (bf16_bits(w.y * inv) << 16);
        o.w = bf16_bits(w.z * inv) | (bf16_bits(w.w * inv) << 16);
        *(uint4*)(y + v) = o;
    }
    if (v1 + threadIdx.x < e1) y[v1 + threadIdx.x] = (uint16_t)bf16_bits(x[v1 + threadIdx.x] * inv);
}

__device__ inline float bf16_float(uint32_t h) { return __uint_as_float(h << 16); }

__global__ void __launch_bounds__(256) k_bf16_unpack(const BfArr* __restrict__ arr, int narr, long long shift,
                                                     const unsigned int* __restrict__ scale,
                                                     const char* __restrict__ slot) {
    const int q = bf_array(arr, narr, blockIdx.x);
    const BfArr& A = arr[q];
    float* x = (float*)((char*)A.p + shift);
    const uint16_t* y = (const uint16_t*)(slot + A.boff);
    float s = __uint_as_float(scale[q]);
    if (!(s >= FLT_MIN)) s = 0.f;
    const long long e0 = (long long)(blockIdx.x - A.blk0) * kBfChunk;
    const long long e1 = min(e0 + kBfChunk, A.n);
    const long long v1 = e0 + ((e1 - e0) & ~7LL);
    for (long long v = e0 + 8 * threadIdx.x; v < v1; v += 8 * 256) {
        const uint4 h = *(const uint4*)(y + v);
        *(float4*)(x + v) = make_float4(bf16_float(h.x & 0xffffu) * s, bf16_float(h.x >> 16) * s,
                                        bf16_float(h.y & 0xffffu) * s, bf16_float(h.y >> 16) * s);
        *(float4*)(x + v + 4) = make_float4(bf16_float(h.z & 0xffffu) * s, bf16_float(h.z >> 16) * s,
                                            bf16_float(h.w & 0xffffu) * s, bf16_float(h.w >> 16) * s);
    }
    if (v1 + threadIdx.x < e1) x[v1 + threadIdx.x] = bf16_float(y[v1 + threadIdx.x]) * s;
}

// 64-bit wrap-around weighted sum of 32-bit words (slot checksum)
__global__ void k_checksum(const uint32_t* __restrict__ w, long long n, unsigned long long* out) {
    unsigned long long s = 0;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x)
        s += (unsigned long long)w[q] * (unsigned long long)(1 + (q & 1023));
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off);
    if ((threadIdx.x & 63) == 0) atomicAdd(out, s);
}

// ============================================================ launchers
static inline int blocks_1d(long long n, int bs, int cap = 65536) {
    long long b = (n + bs - 1) / bs;
    return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

template <typename T, int R>
__global__ void __launch_bounds__(256) k_fwd_plain_cp(const DomDev<T>* __restrict__ doms,
                                                      const int4* __restrict__ tiles, int kz, int rs, int ws, int t) {
    const int4 e = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const DomDev<T>& d = doms[e.x];
    fwd_plain_body<T, R, true>(d, e.y, e.z, e.w, min(e.w + kz, d.n[2]), rs, ws, t);
}

template <typename T, int R>
__global__ void __launch_bounds__(256) k_fwd_plain_nc(const DomDev<T>* __restrict__ doms,
                                                      const int4* __restrict__ tiles, int kz, int rs, int ws, int t) {
    const int4 e = tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const DomDev<T>& d = doms[e.x];
    fwd_plain_body<T, R, false>(d, e.y, e.z, e.w, min(e.w + kz, d.n[2]), rs, ws, t);
}

#define FDTD_ROWS_SWITCH(KER, R, ...)                                                              \
    switch (R) {                                                                                  \
        case 2: hipLaunchKernelGGL((KER<T, 2>), __VA_ARGS__); break;                              \
        case 8: hipLaunchKernelGGL((KER<T, 8>), __VA_ARGS__); break;                              \
        default: hipLaunchKernelGGL((KER<T, 4>), __VA_ARGS__); break;                             \
    }

template <typename T>
void launch_fwd(const LaunchCfg& c, const void* doms, int rs, int ws, int t, hipStream_t s, const int* tdev,
                int slot) {
    const DomDev<T>* dd = (const DomDev<T>*)doms;
    if (c.kernel == 1) {
        // one launch per pass over all blocks: a second launch for the
        // interior blocks costs more in its drain than its leaner registers win
        const int nlb = (c.nlor + 7) / 8 * 8;
        const int sk = c.onepass;
        if (c.ntens < c.ndom) {
            if (c.sw == 32)
                hipLaunchKernelGGL((k_fwd_e<T, 32, false>), dim3(nlb + c.ngrid), dim3(256), 0, s, dd, c.bs, c.xr,
                                   c.lbs, nlb, c.ndom, c.kz, rs, ws, t, tdev, sk);
            else
                hipLaunchKernelGGL((k_fwd_e<T, 64, false>), dim3(nlb + c.ngrid), dim3(256), 0, s, dd, c.bs, c.xr,
                                   c.lbs, nlb, c.ndom, c.kz, rs, ws, t, tdev, sk);
        }
        if (c.ntens) {   // tensor domains: curl pass, then the assembly pass
            if (c.sw == 32) {
                hipLaunchKernelGGL((k_fwd_e<T, 32, true>), dim3(c.ngrid), dim3(256), 0, s, dd, c.bs, c.xr, c.lbs, 0,
                                   c.ndom, c.kz, rs, ws, t, tdev, 0);
                if (c.ntens > c.ntper)
                    hipLaunchKernelGGL((k_tens_e<T, 32, false>), dim3(c.ngrid), dim3(256), 0, s, dd, c.bs, c.xr,
                                       c.ndom, c.kz, rs, ws, t, tdev);
                if (c.ntper)
                    hipLaunchKernelGGL((k_tens_e<T, 32, true>), dim3(c.ngrid), dim3(256), 0, s, dd, c.bs, c.xr,
                                       c.ndom, c.kz, rs, ws, t, tdev);
            } else {
                hipLaunchKernelGGL((k_fwd_e<T, 64, true>), dim3(c.ngrid), dim3(256), 0, s, dd, c.bs, c.xr, c.lbs, 0,
                                   c.ndom, c.kz, rs, ws, t, tdev, 0);
                if (c.ntens > c.ntper)
                    hipLaunchKernelGGL((k_tens_e<T, 64, false>), dim3(c.ngrid), dim3(256), 0, s, dd, c.bs, c.xr,
                                       c.ndom, c.kz, rs, ws, t, tdev);
                if (c.ntper)
                    hipLaunchKernelGGL((k_tens_e<T, 64, true>), dim3(c.ngrid), dim3(256), 0, s, dd, c.bs, c.xr,
                                       c.ndom, c.kz, rs, ws, t, tdev);
            }
        }
        if (sk) {   // interior blocks: one pass (reads set rs only, so it may run after the E pass)
            if (c.sw == 32)
                hipLaunchKernelGGL((k_fwd_one<T, 32>), dim3(c.ngrid), dim3(256), 0, s, dd, c.bs, c.xr, c.ndom, c.kz,
                                   rs, ws, t, tdev, slot);
            else
                hipLaunchKernelGGL((k_fwd_one<T, 64>), dim3(c.ngrid), dim3(256), 0, s, dd, c.bs, c.xr, c.ndom, c.kz,
                                   rs, ws, t, tdev, slot);
        }
        if (c.sw == 32)
            hipLaunchKernelGGL((k_fwd_h<T, 32>), dim3(c.ngrid), dim3(256), 0, s, dd, c.bs, c.xr, c.ndom, c.kz, rs, ws,
                               slot, sk);
        else
            hipLaunchKernelGGL((k_fwd_h<T, 64>), dim3(c.ngrid), dim3(256), 0, s, dd, c.bs, c.xr, c.ndom, c.kz, rs, ws,
                               slot, sk);
        return;
    }
    if (c.nfgen) FDTD_ROWS_SWITCH(k_fwd_fused, c.rows, dim3(c.nfgen), dim3(256), 0, s, dd, c.tfgen, c.kz, rs, ws, t)
    if (c.nfcp) FDTD_ROWS_SWITCH(k_fwd_plain_cp, c.rows, dim3(c.nfcp), dim3(256), 0, s, dd, c.tfcp, c.kz, rs, ws, t)
    if (c.nfplain)
        FDTD_ROWS_SWITCH(k_fwd_plain_nc, c.rows, dim3(c.nfplain), dim3(256), 0, s, dd, c.tfplain, c.kz, rs, ws, t)
}

template <typename T>
void launch_adj(const LaunchCfg& c, const void* doms, int rs, int ws, int fsr, hipStream_t s, int pass,
                const hipStream_t* cs) {
    const DomDev<T>* dd = (const DomDev<T>*)doms;
    if (c.kernel == 1) {
        // ta1: [general tiles (na1g)][the other classes]
        if (pass == 0 && c.na1g)
            hipLaunchKernelGGL(k_adj_ht_full<T>, dim3(c.na1g), dim3(256), 0, s, dd, c.ta1, c.kz, rs, ws, fsr);
        if (pass == 0 && c.na1 > c.na1g)
            hipLaunchKernelGGL(k_adj_ht<T>, dim3(c.na1 - c.na1g), dim3(256), 0, s, dd, c.ta1 + c.na1g, c.kz, rs, ws,
                               fsr);
        if (pass == 1 && c.na2) hipLaunchKernelGGL(k_adj_et<T>, dim3(c.na2), dim3(256), 0, s, dd, c.ta2, c.kz, rs, ws);
        return;
    }
    if (pass != 0) return;
    if (c.ngen) FDTD_ROWS_SWITCH(k_adj_fused, c.rows, dim3(c.ngen), dim3(256), 0, s, dd, c.tgen, c.kz, rs, ws, fsr)
    if (c.nbulk) FDTD_ROWS_SWITCH(k_adj_bulk, c.rows, dim3(c.nbulk), dim3(256), 0, s, dd, c.tbulk, c.kz, rs, ws, fsr)
}

template <typename T>
void launch_sample(const void* doms, const MonDev& m, int cs, int slot, hipStream_t s) {
    int npts = (m.i1 - m.i0) * (m.j1 - m.j0);
    hipLaunchKernelGGL(k_sample<T>, dim3((npts + 255) / 256), dim3(256), 0, s, (const DomDev<T>*)doms, m, cs, slot);
}

template <typename T>
void launch_dft(const MonDev& m, int n0, int count, hipStream_t s, const int* tdev) {
    int npts = (m.i1 - m.i0) * (m.j1 - m.j0);
    hipLaunchKernelGGL(k_dft<T>, dim3((npts + 255) / 256, m.nf), dim3(256), 0, s, m, n0, count, tdev);
}

template <typename T>
void launch_probe(const void* doms, const MonDev& m, int cs, int n, hipStream_t s, const int* tdev) {
    hipLaunchKernelGGL(k_probe<T>, dim3(1), dim3(64), 0, s, (const DomDev<T>*)doms, m, cs, n, tdev);
}

template <typename T>
void launch_seed(const void* doms, const MonDev& m, int as_, int n, hipStream_t s) {
    if (m.kind == 0) {
        hipLaunchKernelGGL(k_probe_seed<T>, dim3(1), dim3(64), 0, s, (const DomDev<T>*)doms, m, as_, n);
        return;
    }
    int npts = (m.i1 - m.i0) * (m.j1 - m.j0);
    hipLaunchKernelGGL(k_seed<T>, dim3((npts + 255) / 256), dim3(256), 0, s, (const DomDev<T>*)doms, m, as_, n);
}

void launch_step_counter(int* c, int value, bool add, hipStream_t s) {
    hipLaunchKernelGGL(k_step_counter, dim3(1), dim3(64), 0, s, c, value, add ? 1 : 0);
}

void launch_zero(void* p, size_t bytes, hipStream_t s) {
    long long nw = (long long)(bytes / 4);
    if (nw == 0) return;
    hipLaunchKernelGGL(k_fill_zero, dim3(blocks_1d(nw, 256, 8192)), dim3(256), 0, s, (uint32_t*)p, nw);
}

void launch_add_f64(double* y, const double* x, size_t n, hipStream_t s) {
    if (!n) return;
    hipLaunchKernelGGL(k_add_f64, dim3(blocks_1d((long long)n, 256, 4096)), dim3(256), 0, s, y, x, (long long)n);
}

void launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
    long long nw = (long long)(bytes / 4);
    if (nw == 0) return;
    hipLaunchKernelGGL(k_copy_words, dim3(blocks_1d(nw, 256, 8192)), dim3(256), 0, s, (const uint32_t*)src,
                       (uint32_t*)dst, nw);
}

void launch_bf16_save(const BfArr* arr, int narr, int nblk, long long shift, float* part, unsigned int* scale,
                      char* slot, hipStream_t s) {
    if (narr == 0 || nblk == 0) return;
    hipLaunchKernelGGL(k_bf16_partmax, dim3(nblk), dim3(256), 0, s, arr, narr, shift, part);
    hipLaunchKernelGGL(k_bf16_scale, dim3(narr), dim3(256), 0, s, arr, (const float*)part, scale);
    hipLaunchKernelGGL(k_bf16_pack, dim3(nblk), dim3(256), 0, s, arr, narr, shift, (const unsigned int*)scale, slot);
}

void launch_bf16_restore(const BfArr* arr, int narr, int nblk, long long shift, const unsigned int* scale,
                         const char* slot, hipStream_t s) {
    if (narr == 0 || nblk == 0) return;
    hipLaunchKernelGGL(k_bf16_unpack, dim3(nblk), dim3(256), 0, s, arr, narr, shift, scale, slot);
}

// Partial sums of the allocation-free flux entry point.  Every GPU the
// library runs on holds its own copy until the process ends; calls on one GPU
// share it (each call rewrites every partial it reads, so nothing has to be
// cleared between calls; calls that overlap on one GPU race).  Host code
// never passes this name to a kernel: it is a host-side stand-in, and the
// device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) double scratch[kFluxScratchBytes / 8];

namespace {
constexpr int kMaxDevices = 64;
std::once_flag g_scratch_once[kMaxDevices];
double* g_scratch_ptr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];
}  // namespace

int flux_scratch(double** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return -1;
    std::call_once(g_scratch_once[dev], [dev] {   // with that device current
        void* p = nullptr;
        g_scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch_ptr[dev] = (double*)p;
    });
    if (g_scratch_err[dev] != hipSuccess || !g_scratch_ptr[dev]) return -1;
    *out = g_scratch_ptr[dev];
    return 0;
}

template <typename T>
void launch_rev_record(const void* doms, int ndom, int cs, int slot, int maxcnt, hipStream_t s) {
    k_rev_record<T><<<dim3(blocks_1d(maxcnt, 256, 4096), ndom), 256, 0, s>>>((const DomDev<T>*)doms, cs, slot);
}

template <typename T>
void launch_rev_step(const void* doms, int ndom, int rs, int ws, int m, long long maxcells, hipStream_t s) {
    const dim3 g(blocks_1d(maxcells, 256, 16384), ndom);
    k_rev_h<T><<<g, 256, 0, s>>>((const DomDev<T>*)doms, rs, ws, m);
    k_rev_e<T><<<g, 256, 0, s>>>((const DomDev<T>*)doms, rs, ws, m - 1, m - 1);
}

int flux_blocks(long long npts) {
    const long long b = (npts + kFluxPoints - 1) / kFluxPoints;
    return (int)std::max(1LL, std::min((long long)kFluxMaxBlocks, b));
}

void launch_flux(const double* spectra, int nf, long long npts, double* part, double* out, hipStream_t s) {
    const int nblk = flux_blocks(npts);
    k_flux_partial<<<dim3(nblk, nf), 256, 0, s>>>((const double2*)spectra, npts, nblk, part);
    k_flux_final<<<nf, 256, 0, s>>>(part, nblk, out);
}

template <typename T>
void launch_energy(const void* doms, int dom, int cs, double* part, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_energy_partial<T>, dim3(kEnergyBlocks), dim3(256), 0, s, (const DomDev<T>*)doms, dom, cs,
                       part);
    hipLaunchKernelGGL(k_flux_final, dim3(1), dim3(256), 0, s, (const double*)part, kEnergyBlocks, out);
}

void launch_checksum(const void* p, size_t bytes, unsigned long long* out, hipStream_t s) {
    long long nw = (long long)(bytes / 4);
    if (nw == 0) return;
    hipLaunchKernelGGL(k_checksum, dim3(blocks_1d(nw, 256, 4096)), dim3(256), 0, s, (const uint32_t*)p, nw, out);
}

int split_blocks(int nx, int ny, int nz, int kz, int w) {
    const int nr = 256 / w;
    return ((nx + w - 1) / w) * ((ny + nr - 1) / nr) * ((nz + kz - 1) / kz);
}

#define FDTD_INSTANTIATE(T)                                                                   \
    template void launch_fwd<T>(const LaunchCfg&, const void*, int, int, int, hipStream_t, const int*, int); \
    template void launch_adj<T>(const LaunchCfg&, const void*, int, int, int, hipStream_t, int, const hipStream_t*); \
    template void launch_sample<T>(const void*, const MonDev&, int, int, hipStream_t);        \
    template void launch_dft<T>(const MonDev&, int, int, hipStream_t, const int*);            \
    template void launch_probe<T>(const void*, const MonDev&, int, int, hipStream_t, const int*); \
    template void launch_seed<T>(const void*, const MonDev&, int, int, hipStream_t);            \
    template void launch_rev_record<T>(const void*, int, int, int, int, hipStream_t);          \
    template void launch_rev_step<T>(const void*, int, int, int, int, long long, hipStream_t);        \
    template void launch_energy<T>(const void*, int, int, double*, double*, hipStream_t);
FDTD_INSTANTIATE(float)
FDTD_INSTANTIATE(double)

}  // namespace fdtd
