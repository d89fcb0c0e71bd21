// fdtd_per_adj.hip -- adjoint step of Bloch-periodic domains for gfx950.
//
// On a periodic axis (x or y, Section 2.2) the forward differences take the
// node past the last one as the first times the real Bloch factor, and the
// node before the first as the last times the factor.  The transpose
// (Section 3.1) scatters across the seam with the conjugate factor, which
// for the real factors +1 and -1 is the factor itself; the E nodes on a
// periodic axis's first plane have no wall.  Two launches per step, the
// split adjoint's two passes written per node with the seam in their
// neighbour gathers:
//   k_padj_e  per E node: the H-update transpose gathered onto the node, the
//             E-update transpose (the identity on E^n, or in a dispersive
//             cell the pole histories' transposes) into the new Ebar, the
//             scaled cotangent u = S coef Ebar_pre into the scratch Et, the
//             E-side memory cotangents (absorbing faces on the other axes)
//             and dJ/deps from the forward state;
//   k_padj_h  per H node: u through the transposed absorber recursion and
//             the curl into the new Hbar, and the H-side memory cotangents.
// Each thread marches one (i, j) column of kNodeKz planes (fdtd_node_adj.h),
// carrying the z neighbours' terms.  Set rs of the adjoint state is read,
// set ws written.
#include <hip/hip_runtime.h>

#include "fdtd_dev.h"
#include "fdtd_launch.h"
#include "fdtd_node_adj.h"

namespace fdtd {
namespace {

// k_padj_e's wave target per SIMD: FP32 at 8 (62 VGPRs, no spills; the
// compiler alone takes 68 and 7 waves), 2.04 against 2.34 ms on the 512 x 512 x
// 536 Bloch cell.  FP64 keeps its 5.  (One wave more cost k_tadj_ht and
// k_tens_e their spills: 1.63 -> 2.43 and 2.08 -> 3.06 ms.)
template <typename T> constexpr int kPadjEWaves = sizeof(T) == 8 ? 5 : 8;

template <typename T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kPadjEWaves<T>, 8)))
k_padj_e(const DomDev<T>* __restrict__ dp, int rs, int ws, int fsr) {
    const DomDev<T>& d = *dp;
    const int i = blockIdx.x * kNodeTx + threadIdx.x % kNodeTx, j = blockIdx.y * kNodeTy + threadIdx.x / kNodeTx;
    const int k0 = blockIdx.z * kNodeKz, k1 = min(k0 + kNodeKz, d.n[2]);
    if (i >= d.n[0] || j >= d.n[1]) return;
    const long long wo = (long long)ws * d.as, fo = (long long)fsr * d.fs;
    const T S = d.S;
    HtGather<T> hg(d, i, j, k0, rs, ws);
    HtPlane<T> cu = hg.fetch(fidx(d, i, j, k0)), nx;
    for (int k = k0; k < k1; ++k) {
        const long long f = fidx(d, i, j, k);
        const int x[3] = {i, j, k};
        if (k + 1 < k1) nx = hg.fetch(f + d.plane);   // plane k+1's loads ahead of plane k's stores
        T et[3], u[3], epre[3];
        hg.gather(k, cu, et);
        cu = nx;
        for (int e = 0; e < 3; ++e) {
            const AdjE<T> r = et_node_d(d, e, i, j, k, et[e], rs, ws);
            epre[e] = r.epre;
            u[e] = e_masked_d(d, e, i, j, k) ? T(0) : S * r.coef * r.epre;
            gp(d.Ea[e])[f + wo] = r.en;
            gp(d.Et[e])[f] = u[e];
        }
        // E-side memory cotangents (owner): ybar = +u (term 0), -u (term 1)
        if (slab_side(d, 0, i) >= 0 || slab_side(d, 1, j) >= 0 || slab_side(d, 2, k) >= 0)
            for (int c = 0; c < 3; ++c) {
                if (e_masked_d(d, c, i, j, k)) continue;
                for (int t = 0; t < 2; ++t)
                    (void)stretch_T(d, d.psiEa, rs, ws, true, (c + 1 + t) % 3, t, 0, i, j, k, t == 0 ? u[c] : -u[c]);
            }
        if (!in_gbox(d, i, j, k)) continue;
        // dJ/deps_c = -S eps^-2 Ebar curl with the forward stretched curl of u^n,
        // its backward differences taken across the seam
        double g[3] = {0, 0, 0};
        for (int c = 0; c < 3; ++c) {
            if (e_masked_d(d, c, i, j, k)) continue;
            const int a0 = (c + 1) % 3, a1 = (c + 2) % 3;
            const FDTD_GLOBAL T* H0 = gp(d.H[(c + 2) % 3]) + fo;
            const FDTD_GLOBAL T* H1 = gp(d.H[(c + 1) % 3]) + fo;
            int y[3];
            T fac;
            const T h0m = back_node(d, a0, x, y, fac) ? fac * H0[fidx(d, y[0], y[1], y[2])] : T(0);
            const T h1m = back_node(d, a1, x, y, fac) ? fac * H1[fidx(d, y[0], y[1], y[2])] : T(0);
            g[c] = grad_term(d, c, i, j, k, f, epre[c], H0[f], h0m, H1[f], h1m, fsr);
        }
        grad_store(d, i, j, k, g);
    }
}

// raw-difference cotangent of E_c's term t (along a = c+1+t, ybar = sign u_c)
// at node (i,j,k), zero on a node a wall holds; memories of set rs read only
template <typename T>
__device__ __forceinline__ T e_dbar(const DomDev<T>& d, int c, int t, int i, int j, int k, T uc, int rs, int ws) {
    if (e_masked_d(d, c, i, j, k)) return T(0);
    return stretch_T(d, d.psiEa, rs, ws, false, (c + 1 + t) % 3, t, 0, i, j, k, t == 0 ? uc : -uc);
}

// Operands of one plane of k_padj_h: u (the scratch Et) at the node and at its
// forward neighbours along y and x, Hbar (set rs) at the node
template <typename T>
struct HnPlane {
    T ux, uy, uz;
    T uz_yp, ux_yp;     // u_z, u_x at the forward node along y
    T uz_xp, uy_xp;     // u_z, u_y at the forward node along x
    T hbx, hby, hbz;
};

template <typename T>
__device__ __forceinline__ HnPlane<T> hn_fetch(const FDTD_GLOBAL T* const (&u)[3], const DomDev<T>& d, long long f,
                                               long long ro, bool okx, long long oxp, bool oky, long long oyp) {
    HnPlane<T> p;
    p.ux = u[0][f];
    p.uy = u[1][f];
    p.uz = u[2][f];
    p.uz_yp = oky ? u[2][f + oyp] : T(0);
    p.ux_yp = oky ? u[0][f + oyp] : T(0);
    p.uz_xp = okx ? u[2][f + oxp] : T(0);
    p.uy_xp = okx ? u[1][f + oxp] : T(0);
    p.hbx = gp(d.Ha[0])[f + ro];
    p.hby = gp(d.Ha[1])[f + ro];
    p.hbz = gp(d.Ha[2])[f + ro];
    return p;
}

template <typename T>
__global__ void __launch_bounds__(256) k_padj_h(const DomDev<T>* __restrict__ dp, int rs, int ws) {
    const DomDev<T>& d = *dp;
    const int i = blockIdx.x * kNodeTx + threadIdx.x % kNodeTx, j = blockIdx.y * kNodeTy + threadIdx.x / kNodeTx;
    const int k0 = blockIdx.z * kNodeKz, k1 = min(k0 + kNodeKz, d.n[2]);
    if (i >= d.n[0] || j >= d.n[1]) return;
    const long long ro = (long long)rs * d.as, wo = (long long)ws * d.as, pl = d.plane;
    const FDTD_GLOBAL T* u[3] = {gp(d.Et[0]), gp(d.Et[1]), gp(d.Et[2])};
    const T S = d.S;
    // the forward nodes along x and y (across a seam; none past a wall), fixed per column
    const int x0[3] = {i, j, 0};
    int nxn[3], nyn[3];
    T fxp, fyp;
    const bool okx = fwd_node(d, 0, x0, nxn, fxp), oky = fwd_node(d, 1, x0, nyn, fyp);
    const long long oxp = nxn[0] - i, oyp = (long long)(nyn[1] - j) * d.pitch;
    long long f = fidx(d, i, j, k0);
    HnPlane<T> cu = hn_fetch(u, d, f, ro, okx, oxp, oky, oyp);
    // own z-terms of the current plane: (Ex, 1) and (Ey, 0), both along z
    T ex1 = e_dbar(d, 0, 1, i, j, k0, cu.ux, rs, ws), ey0 = e_dbar(d, 1, 0, i, j, k0, cu.uy, rs, ws);
    for (int k = k0; k < k1; ++k, f += pl) {
        const bool up = k + 1 < d.n[2];
        // plane k+1's loads ahead of plane k's stores (past the chunk, only the z neighbours)
        HnPlane<T> nx;
        if (k + 1 < k1) {
            nx = hn_fetch(u, d, f + pl, ro, okx, oxp, oky, oyp);
        } else {
            nx.ux = up ? u[0][f + pl] : T(0);
            nx.uy = up ? u[1][f + pl] : T(0);
        }
        const T ex1u = up ? e_dbar(d, 0, 1, i, j, k + 1, nx.ux, rs, ws) : T(0);
        const T ey0u = up ? e_dbar(d, 1, 0, i, j, k + 1, nx.uy, rs, ws) : T(0);
        const T ex0 = e_dbar(d, 0, 0, i, j, k, cu.ux, rs, ws), ey1 = e_dbar(d, 1, 1, i, j, k, cu.uy, rs, ws);
        const T ez0 = e_dbar(d, 2, 0, i, j, k, cu.uz, rs, ws), ez1 = e_dbar(d, 2, 1, i, j, k, cu.uz, rs, ws);
        // Dbar of E_c's term t at the forward node along x or y, zero past a wall
        const T fz1 = oky ? fyp * e_dbar(d, 2, 1, nyn[0], nyn[1], k, cu.uz_yp, rs, ws) : T(0);
        const T fx0 = oky ? fyp * e_dbar(d, 0, 0, nyn[0], nyn[1], k, cu.ux_yp, rs, ws) : T(0);
        const T fz0 = okx ? fxp * e_dbar(d, 2, 0, nxn[0], nxn[1], k, cu.uz_xp, rs, ws) : T(0);
        const T fy1 = okx ? fxp * e_dbar(d, 1, 1, nxn[0], nxn[1], k, cu.uy_xp, rs, ws) : T(0);
        // H_h(x) collects Dbar(x) - Dbar(forward node) from the terms it enters:
        // Hx: (Ey,0) along z, (Ez,1) along y; Hy: (Ez,0) along x, (Ex,1) along z;
        // Hz: (Ex,0) along y, (Ey,1) along x
        gp(d.Ha[0])[f + wo] = cu.hbx + (ey0 - ey0u) + (ez1 - fz1);
        gp(d.Ha[1])[f + wo] = cu.hby + (ez0 - fz0) + (ex1 - ex1u);
        gp(d.Ha[2])[f + wo] = cu.hbz + (ex0 - fx0) + (ey1 - fy1);
        // H-side memory cotangents (owner): ybar = -S sign Hbar
        if (slab_side(d, 0, i) >= 0 || slab_side(d, 1, j) >= 0 || slab_side(d, 2, k) >= 0) {
            const T hb[3] = {cu.hbx, cu.hby, cu.hbz};
            for (int c = 0; c < 3; ++c)
                for (int t = 0; t < 2; ++t)
                    (void)stretch_T(d, d.psiHa, rs, ws, true, (c + 1 + t) % 3, t, 3, i, j, k,
                                    -S * (t == 0 ? T(1) : T(-1)) * hb[c]);
        }
        ex1 = ex1u;
        ey0 = ey0u;
        cu = nx;
    }
}

}  // namespace

template <typename T>
void launch_per_adj(const void* doms, int dom, const int n[3], int rs, int ws, int fsr, hipStream_t s) {
    const DomDev<T>* dp = (const DomDev<T>*)doms + dom;
    const dim3 grid((n[0] + kNodeTx - 1) / kNodeTx, (n[1] + kNodeTy - 1) / kNodeTy, (n[2] + kNodeKz - 1) / kNodeKz);
    hipLaunchKernelGGL(k_padj_e<T>, grid, dim3(256), 0, s, dp, rs, ws, fsr);
    hipLaunchKernelGGL(k_padj_h<T>, grid, dim3(256), 0, s, dp, rs, ws);
}

template <typename T>
void launch_per_adj_h(const void* doms, int dom, const int n[3], int rs, int ws, hipStream_t s) {
    const DomDev<T>* dp = (const DomDev<T>*)doms + dom;
    const dim3 grid((n[0] + kNodeTx - 1) / kNodeTx, (n[1] + kNodeTy - 1) / kNodeTy, (n[2] + kNodeKz - 1) / kNodeKz);
    hipLaunchKernelGGL(k_padj_h<T>, grid, dim3(256), 0, s, dp, rs, ws);
}

template void launch_per_adj<float>(const void*, int, const int*, int, int, int, hipStream_t);
template void launch_per_adj<double>(const void*, int, const int*, int, int, int, hipStream_t);
template void launch_per_adj_h<float>(const void*, int, const int*, int, int, hipStream_t);
template void launch_per_adj_h<double>(const void*, int, const int*, int, int, hipStream_t);

}  // namespace fdtd
