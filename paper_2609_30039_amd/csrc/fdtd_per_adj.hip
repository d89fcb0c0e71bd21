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
//             new Ebar (no dispersion in a periodic domain with a gradient,
//             so the E-update transpose is the identity on E^n), the scaled
//             cotangent u = S eps^-1 Ebar into the scratch Et, the E-side
//             memory cotangents (absorbing faces on the other axes) and
//             dJ/deps from the forward state;
//   k_padj_h  per H node: u through the transposed absorber recursion and
//             the curl into the new Hbar, and the H-side memory cotangents.
// One thread per node, 64 x-nodes by 4 rows per block, one plane per grid
// row (a z-stride loop beyond the grid's z extent).  Set rs of the adjoint
// state is read, set ws written.
#include <hip/hip_runtime.h>

#include "fdtd_dev.h"
#include "fdtd_launch.h"

namespace fdtd {
namespace {

constexpr int kTx = 64, kTy = 4, kMaxGridZ = 65535;

// the node one step back along a from x, across a periodic seam when x[a] = 0:
// returns false past a wall; fac is the Bloch factor taken at the seam, else 1
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

template <typename T>
__global__ void __launch_bounds__(256) k_padj_e(const DomDev<T>* __restrict__ dp, int rs, int ws, int fsr) {
    const DomDev<T>& d = *dp;
    const int i = blockIdx.x * kTx + threadIdx.x % kTx, j = blockIdx.y * kTy + threadIdx.x / kTx;
    if (i >= d.n[0] || j >= d.n[1]) return;
    const long long ro = (long long)rs * d.as, wo = (long long)ws * d.as, fo = (long long)fsr * d.fs;
    const T S = d.S;
    for (int k = blockIdx.z; k < d.n[2]; k += gridDim.z) {
        const long long f = fidx(d, i, j, k);
        const int x[3] = {i, j, k};
        T et[3], u[3];
        for (int e = 0; e < 3; ++e) {
            et[e] = T(0);
            u[e] = T(0);
            if (e_masked_d(d, e, i, j, k)) continue;
            T acc = gp(d.Ea[e])[f + ro];
            // E_e enters H_c's term t, differenced forward along a (t = 0: c = e+1,
            // a = e+2, sign +; t = 1: c = e+2, a = e+1, sign -): Ebar_e(x) gets
            // fac Dbar(back node) - Dbar(x)
            for (int t = 0; t < 2; ++t) {
                const int c = t == 0 ? (e + 1) % 3 : (e + 2) % 3;
                const int a = t == 0 ? (e + 2) % 3 : (e + 1) % 3;
                const T sgn = t == 0 ? T(1) : T(-1);
                const FDTD_GLOBAL T* hb = gp(d.Ha[c]) + ro;
                acc -= hT_dbar(d, a, t, sgn, i, j, k, hb[f], rs, ws, false);
                int y[3];
                T fac;
                if (back_node(d, a, x, y, fac))
                    acc += fac * hT_dbar(d, a, t, sgn, y[0], y[1], y[2], hb[fidx(d, y[0], y[1], y[2])], rs, ws, false);
            }
            et[e] = acc;
            u[e] = S * epsinv_at(d, e, i, j, k) * acc;
        }
        for (int e = 0; e < 3; ++e) {
            gp(d.Ea[e])[f + wo] = et[e];
            gp(d.Et[e])[f] = u[e];
        }
        // E-side memory cotangents (owner): ybar = +u (term 0), -u (term 1)
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
            g[c] = grad_term(d, c, i, j, k, f, et[c], H0[f], h0m, H1[f], h1m, fsr);
        }
        grad_store(d, i, j, k, g);
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_padj_h(const DomDev<T>* __restrict__ dp, int rs, int ws) {
    const DomDev<T>& d = *dp;
    const int i = blockIdx.x * kTx + threadIdx.x % kTx, j = blockIdx.y * kTy + threadIdx.x / kTx;
    if (i >= d.n[0] || j >= d.n[1]) return;
    const long long ro = (long long)rs * d.as, wo = (long long)ws * d.as;
    const T S = d.S;
    for (int k = blockIdx.z; k < d.n[2]; k += gridDim.z) {
        const long long f = fidx(d, i, j, k);
        const int x[3] = {i, j, k};
        T hb[3];
        for (int h = 0; h < 3; ++h) hb[h] = gp(d.Ha[h])[f + ro];
        for (int h = 0; h < 3; ++h) {
            T acc = hb[h];
            // H_h enters E_c's term t, differenced backward along a (t = 0: c = h+1,
            // a = h+2, sign +; t = 1: c = h+2, a = h+1, sign -), ybar = sign u_c:
            // Hbar_h(x) gets Dbar(x) - fac Dbar(forward node)
            for (int t = 0; t < 2; ++t) {
                const int c = t == 0 ? (h + 1) % 3 : (h + 2) % 3;
                const int a = t == 0 ? (h + 2) % 3 : (h + 1) % 3;
                const T sgn = t == 0 ? T(1) : T(-1);
                const FDTD_GLOBAL T* uc = gp(d.Et[c]);
                if (!e_masked_d(d, c, i, j, k))
                    acc += stretch_T(d, d.psiEa, rs, ws, false, a, t, 0, i, j, k, sgn * uc[f]);
                int y[3];
                T fac;
                if (fwd_node(d, a, x, y, fac) && !e_masked_d(d, c, y[0], y[1], y[2]))
                    acc -= fac * stretch_T(d, d.psiEa, rs, ws, false, a, t, 0, y[0], y[1], y[2],
                                           sgn * uc[fidx(d, y[0], y[1], y[2])]);
            }
            gp(d.Ha[h])[f + wo] = acc;
        }
        // H-side memory cotangents (owner): ybar = -S sign Hbar
        for (int c = 0; c < 3; ++c)
            for (int t = 0; t < 2; ++t)
                (void)stretch_T(d, d.psiHa, rs, ws, true, (c + 1 + t) % 3, t, 3, i, j, k,
                                -S * (t == 0 ? T(1) : T(-1)) * hb[c]);
    }
}

}  // namespace

template <typename T>
void launch_per_adj(const void* doms, int dom, const int n[3], int rs, int ws, int fsr, hipStream_t s) {
    const DomDev<T>* dp = (const DomDev<T>*)doms + dom;
    const dim3 grid((n[0] + kTx - 1) / kTx, (n[1] + kTy - 1) / kTy, std::min(n[2], kMaxGridZ));
    hipLaunchKernelGGL(k_padj_e<T>, grid, dim3(256), 0, s, dp, rs, ws, fsr);
    hipLaunchKernelGGL(k_padj_h<T>, grid, dim3(256), 0, s, dp, rs, ws);
}

template void launch_per_adj<float>(const void*, int, const int*, int, int, int, hipStream_t);
template void launch_per_adj<double>(const void*, int, const int*, int, int, int, hipStream_t);

}  // namespace fdtd
