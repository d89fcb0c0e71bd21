// fdtd_node_adj.h -- pieces shared by the per-node adjoint passes of tensor
// media and Bloch-periodic domains (internal).
//
// These passes give each thread one (i, j) column of kNodeKz planes of a
// domain, 64 x-columns by 4 rows per 256-thread block, and march it in z:
// the z neighbour a node reads is the previous (or next) plane of the same
// thread, carried in registers, so a plane's operands are fetched once.
#pragma once
#include "fdtd_dev.h"

namespace fdtd {

constexpr int kNodeTx = 64, kNodeTy = 4, kNodeKz = 8;

// the node one step back along a from x, across a periodic seam when x[a] = 0
// (fac: the Bloch factor there, else 1); false past a wall
template <typename T>
__device__ __forceinline__ bool back_node(const DomDev<T>& d, int a, const int x[3], int y[3], T& fac) {
    y[0] = x[0];
    y[1] = x[1];
    y[2] = x[2];
    fac = T(1);
    if (x[a] > 0) {
        y[a] -= 1;
        return true;
    }
    if (!d.per[a]) return false;
    y[a] = d.n[a] - 1;
    fac = d.bsign[a];
    return true;
}

// the node one step forward along a, across a periodic seam when x[a] = n - 1
template <typename T>
__device__ __forceinline__ bool fwd_node(const DomDev<T>& d, int a, const int x[3], int y[3], T& fac) {
    y[0] = x[0];
    y[1] = x[1];
    y[2] = x[2];
    fac = T(1);
    if (x[a] + 1 < d.n[a]) {
        y[a] += 1;
        return true;
    }
    if (!d.per[a]) return false;
    y[a] = 0;
    fac = d.bsign[a];
    return true;
}

// Operands of one plane of HtGather: Hbar (set rs) at the node and at its back
// neighbours along x and y, Ebar^{n+1} (set rs) at the node.
template <typename T>
struct HtPlane {
    T hx, hy, hz;          // Hbar at (i, j, k)
    T hz_ym, hx_ym;        // Hbar_z, Hbar_x at the back node along y
    T hz_xm, hy_xm;        // Hbar_z, Hbar_y at the back node along x
    T ex, ey, ez;          // Ebar^{n+1} at (i, j, k)
};

// The H-update transpose gathered onto the E nodes of one column.  H_c's term
// t (t = 0: difference along c+1 of E_{c+2}, sign +; t = 1: along c+2 of
// E_{c+1}, sign -) has raw-difference cotangent Dbar_ct(p) (the transposed
// absorber recursion of ybar = -S sign Hbar_c(p), memories of set rs read
// only).  With D(p) = E(p + a) - E(p), E_e(x) collects Dbar(back node) - Dbar(x)
// from (c, t) = (e+1, 0) along e+2 and (e+2, 1) along e+1.  Along z (no seam)
// the back node's terms are the previous plane's own ones, carried.  The back
// nodes along x and y (across a seam, or none past a wall) are fixed per
// column; fetch() loads a plane's operands so that a caller can issue plane
// k+1's loads before it computes and stores plane k.
template <typename T>
struct HtGather {
    const DomDev<T>& d;
    int i, j, rs, ws;
    long long ro;
    T dz_y0, dz_x1;        // own z-terms of the plane below: Dbar of (Hy, t=0) and (Hx, t=1)
    bool okx, oky;         // the back node along x / y exists
    int bx[3], by[3];      // its (i, j) (k of the plane)
    T fx, fy;              // its Bloch factor
    long long ox, oy;      // its flat offset from (i, j)

    __device__ __forceinline__ HtGather(const DomDev<T>& d_, int i_, int j_, int k0, int rs_, int ws_)
        : d(d_), i(i_), j(j_), rs(rs_), ws(ws_), ro((long long)rs_ * d_.as), dz_y0(0), dz_x1(0) {
        const int x[3] = {i, j, 0};
        okx = back_node(d, 0, x, bx, fx);
        oky = back_node(d, 1, x, by, fy);
        ox = (long long)(bx[0] - i);
        oy = (long long)(by[1] - j) * d.pitch;
        if (k0 > 0) {
            const long long f = fidx(d, i, j, k0 - 1) + ro;
            dz_y0 = hT_dbar(d, 2, 0, T(1), i, j, k0 - 1, gp(d.Ha[1])[f], rs, ws, false);
            dz_x1 = hT_dbar(d, 2, 1, T(-1), i, j, k0 - 1, gp(d.Ha[0])[f], rs, ws, false);
        }
    }

    // the operands of the plane at flat index f
    __device__ __forceinline__ HtPlane<T> fetch(long long f) const {
        const long long fr = f + ro;
        HtPlane<T> p;
        p.hx = gp(d.Ha[0])[fr];
        p.hy = gp(d.Ha[1])[fr];
        p.hz = gp(d.Ha[2])[fr];
        p.hz_ym = oky ? gp(d.Ha[2])[fr + oy] : T(0);
        p.hx_ym = oky ? gp(d.Ha[0])[fr + oy] : T(0);
        p.hz_xm = okx ? gp(d.Ha[2])[fr + ox] : T(0);
        p.hy_xm = okx ? gp(d.Ha[1])[fr + ox] : T(0);
        p.ex = gp(d.Ea[0])[fr];
        p.ey = gp(d.Ea[1])[fr];
        p.ez = gp(d.Ea[2])[fr];
        return p;
    }

    // et[e]: Ebar^{n+1} of set rs plus the gathered terms at plane k from its
    // fetched operands (zero on a node a wall holds)
    __device__ __forceinline__ void gather(int k, const HtPlane<T>& p, T et[3]) {
        // own terms: (Hx,0) along y, (Hx,1) along z, (Hy,0) along z, (Hy,1) along x, (Hz,0) along x, (Hz,1) along y
        const T ox0 = hT_dbar(d, 1, 0, T(1), i, j, k, p.hx, rs, ws, false);
        const T ox1 = hT_dbar(d, 2, 1, T(-1), i, j, k, p.hx, rs, ws, false);
        const T oy0 = hT_dbar(d, 2, 0, T(1), i, j, k, p.hy, rs, ws, false);
        const T oy1 = hT_dbar(d, 0, 1, T(-1), i, j, k, p.hy, rs, ws, false);
        const T oz0 = hT_dbar(d, 0, 0, T(1), i, j, k, p.hz, rs, ws, false);
        const T oz1 = hT_dbar(d, 1, 1, T(-1), i, j, k, p.hz, rs, ws, false);
        // the back nodes' terms: (Hz,1) and (Hx,0) along y, (Hz,0) and (Hy,1) along x
        const T bz1 = oky ? fy * hT_dbar(d, 1, 1, T(-1), by[0], by[1], k, p.hz_ym, rs, ws, false) : T(0);
        const T bx0 = oky ? fy * hT_dbar(d, 1, 0, T(1), by[0], by[1], k, p.hx_ym, rs, ws, false) : T(0);
        const T bz0 = okx ? fx * hT_dbar(d, 0, 0, T(1), bx[0], bx[1], k, p.hz_xm, rs, ws, false) : T(0);
        const T by1 = okx ? fx * hT_dbar(d, 0, 1, T(-1), bx[0], bx[1], k, p.hy_xm, rs, ws, false) : T(0);
        // Ex: (Hy,0) along z, (Hz,1) along y; Ey: (Hz,0) along x, (Hx,1) along z; Ez: (Hx,0) along y, (Hy,1) along x
        et[0] = e_masked_d(d, 0, i, j, k) ? T(0) : p.ex + (dz_y0 - oy0) + (bz1 - oz1);
        et[1] = e_masked_d(d, 1, i, j, k) ? T(0) : p.ey + (bz0 - oz0) + (dz_x1 - ox1);
        et[2] = e_masked_d(d, 2, i, j, k) ? T(0) : p.ez + (bx0 - ox0) + (by1 - oy1);
        dz_y0 = oy0;
        dz_x1 = ox1;
    }
};

// E-update transpose at E node c of a domain that may have periodic axes
// (the walls' masks from e_masked_d): from etot, the cotangent of E^{n+1}
// after the H transpose, the cotangent of E^{n+1} before the source (epre),
// the curl's coefficient (eps^-1, or 1/den in a dispersive cell) and, with
// the pole histories' transposes stored into set ws, the new cotangent of
// E^n.  The same recursion as the walled domains' et_node.
template <typename T>
__device__ __forceinline__ AdjE<T> et_node_d(const DomDev<T>& d, int c, int i, int j, int k, T etot, int rs, int ws) {
    AdjE<T> r;
    r.epre = T(0);
    r.coef = T(0);
    r.en = T(0);
    const long long as = d.as;
    if (e_masked_d(d, c, i, j, k)) {
        if (in_lor(d, i, j, k)) {
            const long long q = lidx(d, i, j, k) + ws * as;
            gp(d.lora[0][c])[q] = T(0);
            for (int p = 0; p < d.npole; ++p) {
                gp(d.lora[1][c])[q + p * d.lbox] = T(0);
                gp(d.lora[2][c])[q + p * d.lbox] = T(0);
            }
        }
        return r;
    }
    const T einv = epsinv_at(d, c, i, j, k);
    if (!in_lor(d, i, j, k)) {
        r.epre = etot;
        r.coef = einv;
        r.en = etot;
        return r;
    }
    // each pole's roll W^{n+1} = al W^n + xi W^{n-1} + g/2 (E^{n+1} - E^{n-1}) feeds E^{n+1};
    // E^{n+1}_pre = [einf E^n + gsum/4 E^{n-1} + S curl - sum ((1 + al) W^n + xi W^{n-1}) / 2] / den
    const long long q = lidx(d, i, j, k);
    const T einf = T(1) / einv;
    const T invden = T(1) / (einf + T(0.25) * d.lgs);
    T ep = etot;
    for (int p = 0; p < d.npole; ++p) ep = fma(T(0.5) * d.lg[p], gp(d.lora[1][c])[q + p * d.lbox + rs * as], ep);
    r.epre = ep;
    r.coef = invden;
    const T s = ep * invden;
    r.en = fma(einf, s, gp(d.lora[0][c])[q + rs * as]);
    T enm1 = T(0);
    for (int p = 0; p < d.npole; ++p) {
        const long long o = q + p * d.lbox;
        const T wb = gp(d.lora[1][c])[o + rs * as], wob = gp(d.lora[2][c])[o + rs * as];
        T wn = fma(d.lal[p], wb, wob);
        T wnm1 = d.lxi[p] * wb;
        enm1 = p == 0 ? -T(0.5) * d.lg[0] * wb : fma(-T(0.5) * d.lg[p], wb, enm1);
        wn = fma(-T(0.5) * (T(1) + d.lal[p]), s, wn);
        wnm1 = fma(-T(0.5) * d.lxi[p], s, wnm1);
        gp(d.lora[1][c])[o + ws * as] = wn;
        gp(d.lora[2][c])[o + ws * as] = wnm1;
    }
    enm1 = fma(T(0.25) * d.lgs, s, enm1);
    gp(d.lora[0][c])[q + ws * as] = enm1;
    return r;
}

}  // namespace fdtd
