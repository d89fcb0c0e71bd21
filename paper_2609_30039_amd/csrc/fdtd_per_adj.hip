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

template <typename T>
__global__ void __launch_bounds__(256) k_padj_e(const DomDev<T>* __restrict__ dp, int rs, int ws, int fsr) {
    const DomDev<T>& d = *dp;
    const int i = blockIdx.x * kNodeTx + threadIdx.x % kNodeTx, j = blockIdx.y * kNodeTy + threadIdx.x / kNodeTx;
    const int k0 = blockIdx.z * kNodeKz, k1 = min(k0 + kNodeKz, d.n[2]);
    if (i >= d.n[0] || j >= d.n[1]) return;
    const long long wo = (long long)ws * d.as, fo = (long long)fsr * d.fs;
    const T S = d.S;
    HtGather<T> hg(d, i, j, k0, rs, ws);
    for (int k = k0; k < k1; ++k) {
        const long long f = fidx(d, i, j, k);
        const int x[3] = {i, j, k};
        T et[3], u[3], epre[3];
        hg.plane(k, f, et);
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

template <typename T>
__global__ void __launch_bounds__(256) k_padj_h(const DomDev<T>* __restrict__ dp, int rs, int ws) {
    const DomDev<T>& d = *dp;
    const int i = blockIdx.x * kNodeTx + threadIdx.x % kNodeTx, j = blockIdx.y * kNodeTy + threadIdx.x / kNodeTx;
    const int k0 = blockIdx.z * kNodeKz, k1 = min(k0 + kNodeKz, d.n[2]);
    if (i >= d.n[0] || j >= d.n[1]) return;
    const long long ro = (long long)rs * d.as, wo = (long long)ws * d.as, pl = d.plane;
    const FDTD_GLOBAL T* u[3] = {gp(d.Et[0]), gp(d.Et[1]), gp(d.Et[2])};
    const T S = d.S;
    // Dbar of E_c's term t at the forward node along a (x, y: across a seam), zero past a wall
    auto fwd_term = [&](int c, int t, int a, int k) -> T {
        const int x[3] = {i, j, k};
        int y[3];
        T fac;
        if (!fwd_node(d, a, x, y, fac)) return T(0);
        return fac * e_dbar(d, c, t, y[0], y[1], y[2], u[c][fidx(d, y[0], y[1], y[2])], rs, ws);
    };
    long long f = fidx(d, i, j, k0);
    T ux = u[0][f], uy = u[1][f], uz = u[2][f];
    // own z-terms of the current plane: (Ex, 1) and (Ey, 0), both along z
    T ex1 = e_dbar(d, 0, 1, i, j, k0, ux, rs, ws), ey0 = e_dbar(d, 1, 0, i, j, k0, uy, rs, ws);
    for (int k = k0; k < k1; ++k, f += pl) {
        const bool up = k + 1 < d.n[2];
        const T uxu = up ? u[0][f + pl] : T(0), uyu = up ? u[1][f + pl] : T(0), uzu = up ? u[2][f + pl] : T(0);
        const T ex1u = up ? e_dbar(d, 0, 1, i, j, k + 1, uxu, rs, ws) : T(0);
        const T ey0u = up ? e_dbar(d, 1, 0, i, j, k + 1, uyu, rs, ws) : T(0);
        const T ex0 = e_dbar(d, 0, 0, i, j, k, ux, rs, ws), ey1 = e_dbar(d, 1, 1, i, j, k, uy, rs, ws);
        const T ez0 = e_dbar(d, 2, 0, i, j, k, uz, rs, ws), ez1 = e_dbar(d, 2, 1, i, j, k, uz, rs, ws);
        // H_h(x) collects Dbar(x) - Dbar(forward node) from the terms it enters:
        // Hx: (Ey,0) along z, (Ez,1) along y; Hy: (Ez,0) along x, (Ex,1) along z;
        // Hz: (Ex,0) along y, (Ey,1) along x
        const T hbx = gp(d.Ha[0])[f + ro], hby = gp(d.Ha[1])[f + ro], hbz = gp(d.Ha[2])[f + ro];
        gp(d.Ha[0])[f + wo] = hbx + (ey0 - ey0u) + (ez1 - fwd_term(2, 1, 1, k));
        gp(d.Ha[1])[f + wo] = hby + (ez0 - fwd_term(2, 0, 0, k)) + (ex1 - ex1u);
        gp(d.Ha[2])[f + wo] = hbz + (ex0 - fwd_term(0, 0, 1, k)) + (ey1 - fwd_term(1, 1, 0, k));
        // H-side memory cotangents (owner): ybar = -S sign Hbar
        if (slab_side(d, 0, i) >= 0 || slab_side(d, 1, j) >= 0 || slab_side(d, 2, k) >= 0) {
            const T hb[3] = {hbx, hby, hbz};
            for (int c = 0; c < 3; ++c)
                for (int t = 0; t < 2; ++t)
                    (void)stretch_T(d, d.psiHa, rs, ws, true, (c + 1 + t) % 3, t, 3, i, j, k,
                                    -S * (t == 0 ? T(1) : T(-1)) * hb[c]);
        }
        ux = uxu;
        uy = uyu;
        uz = uzu;
        ex1 = ex1u;
        ey0 = ey0u;
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
